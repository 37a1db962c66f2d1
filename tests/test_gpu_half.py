"""GPU parity of the FP16 storage format (SAP_F16: spinor components as half2 scaled by a
per-site FP32 norm, links as half2, FP16 products summed in FP32) against the FP64 oracle, and of
mixed-precision solves whose inner Krylov iterations run on FP16 fields inside the FP64
defect correction (Sec. 3).

Tolerances follow from the format. A component of a site with norm m (its largest
component magnitude) is stored as a half in [-1, 1], so packing and unpacking is exact
up to half a unit in the last place of [0.5, 1): |err| <= 2^-12 m (the FP32 scaling adds
a few 2^-24 m). For the hop, each of the 8 terms of eq. 2 sees a projected half spinor
of at most 2 max|psi| per component times a link whose entries carry 2^-12 errors, and
a link times the projected input error; the projected half spinor is itself rounded to
FP16 once (at most 2^-11 of its neighbour's norm per component, since it is below 2 in
norm units) before the FP16 x FP16 products summed in FP32, which adds at most
8 * sqrt(6) * 2^-11 (about 39 * 2^-12) of the largest input component to a hop sum in
the worst case. These rounding errors point in unrelated directions, so with
kappa <= 0.16 and the output itself rounded once the error of M stays well below
16 * 2^-12 of the largest input component (F16_TOL below), and that of D_eo below
F16_TOL / 0.16; on 24^3 x 48 the measured errors are about 1.7 * 2^-12 (M) and
7 * 2^-12 (D_eo).
Solves are checked by their FP64 residual, as for FP32 inner solves."""
import numpy as np
import pytest

import synth
from oracle import dirac, lattice, solvers

pytestmark = pytest.mark.gpu

SHAPES = [  # (L, l0, l0_sub, kappa)
    ((4, 4, 4, 4), 2, 0, 0.155),
    ((6, 2, 4, 6), 3, 0, 0.16),            # V/2 = 144: one partial workgroup
    ((8, 6, 2, 10), 2, 0, 0.13),           # V/2 = 480: ragged tail
    ((16, 4, 6, 4), 4, 2, 0.1575),         # level-2 blocks
]
HALF_ULP = 2.0 ** -12
F16_TOL = 16 * HALF_ULP


@pytest.fixture(scope="module")
def gu():
    import gpu_util
    return gpu_util


def _err_vs_input(got, ref, psi):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(psi)))


@pytest.mark.parametrize("L,l0,l0_sub,k", SHAPES)
def test_pack_unpack_roundtrip_within_half_ulp(gu, L, l0, l0_sub, k):
    import paper_0710_0066_amd as sap
    print(f"f16 pack/unpack L={L}", flush=True)
    U = synth.gauge_field(L, 0.5, 1101)
    psi = synth.gaussian_spinor(L, 2101, nrhs=3)
    psi[0, 0, 0, 0, 0] = 0.0                            # an all-zero site: norm 0
    psi[1, 1, 0, 0, 0] *= 1e-20                          # a tiny site: the norm rescales it
    ctx = gu.make_ctx(L, l0, k, U, l0_sub, max_rhs=3)
    f = gu.to_sap(ctx, psi, 3, sap.SAP_F16)
    assert f.numel() * 4 == ctx.field_bytes(3, sap.SAP_F16) == 3 * 26 * 4 * ctx.field_bytes(1, sap.SAP_F64) // (24 * 16)
    got = gu.from_sap(ctx, f, 3, psi.shape, sap.SAP_F16)
    m = np.max(np.maximum(np.abs(psi.real), np.abs(psi.imag)), axis=(-2, -1), keepdims=True)
    err = np.maximum(np.abs(got.real - psi.real), np.abs(got.imag - psi.imag))
    assert np.all(err <= 1.01 * HALF_ULP * m)
    assert np.all(got[0, 0, 0, 0, 0] == 0)
    assert np.any(got[1, 1, 0, 0, 0] != 0)


@pytest.mark.parametrize("L,l0,l0_sub,k", SHAPES)
@pytest.mark.parametrize("nrhs", [1, 3])
def test_apply_M_f16_matches_oracle(gu, L, l0, l0_sub, k, nrhs):
    import paper_0710_0066_amd as sap
    print(f"f16 apply_M L={L} nrhs={nrhs}", flush=True)
    U = synth.gauge_field(L, 0.5, 1103)
    psi = synth.gaussian_spinor(L, 2103, nrhs=nrhs)
    ref = dirac.apply_M(U, psi, k)
    ctx = gu.make_ctx(L, l0, k, U, l0_sub, max_rhs=nrhs)
    fin = gu.to_sap(ctx, psi, nrhs, sap.SAP_F16)
    fout = ctx.new_field(nrhs, sap.SAP_F16)
    sap.apply_M(ctx, fout, fin, nrhs, sap.SAP_F16)
    got = gu.from_sap(ctx, fout, nrhs, psi.shape, sap.SAP_F16)
    err = _err_vs_input(got, ref, psi)
    assert err <= F16_TOL, err
    # the format is not FP32 in disguise: the error is at the FP16 level
    assert err >= 1e-5, err


@pytest.mark.parametrize("L,l0,l0_sub,k", SHAPES)
def test_apply_W_f16_matches_oracle(gu, L, l0, l0_sub, k):
    import paper_0710_0066_amd as sap
    print(f"f16 apply_W1_block L={L}", flush=True)
    U = synth.gauge_field(L, 0.5, 1105)
    psi = synth.gaussian_spinor(L, 2105, nrhs=2)
    ctx = gu.make_ctx(L, l0, k, U, l0_sub, max_rhs=2)
    levels = [(1, l0)] + ([(2, l0_sub)] if l0_sub else [])
    fin = gu.to_sap(ctx, psi, 2, sap.SAP_F16)
    for level, lb in levels:
        ref_all = dirac.apply_W(U, psi, k, lb)
        nb = L[0] // lb
        for block, color, cname in [(-1, sap.SAP_ALL, "all"), (-1, sap.SAP_BLACK, "black"),
                                    (-1, sap.SAP_WHITE, "white"), (nb - 1, sap.SAP_ALL, None)]:
            m = lattice.single_block_mask(L, lb, block) if block >= 0 else lattice.colour_x0_mask(L, lb, cname)
            ref = ref_all * lattice.site_mask(L, m)
            fout = ctx.new_field(2, sap.SAP_F16)
            fout.fill_(7.0)                              # every site must be written
            sap.apply_W1_block(ctx, fout, fin, 2, level, block, color, sap.SAP_F16)
            got = gu.from_sap(ctx, fout, 2, psi.shape, sap.SAP_F16)
            off = ~np.broadcast_to(lattice.site_mask(L, m) != 0, got.shape)
            assert np.all(got[off] == 0), (level, block, color)
            assert _err_vs_input(got, ref, psi) <= F16_TOL, (level, block, color)


@pytest.mark.parametrize("L,l0,l0_sub,k", SHAPES[:3])
@pytest.mark.parametrize("nrhs", [1, 5])
def test_apply_Dslash_eo_f16_matches_oracle(gu, L, l0, l0_sub, k, nrhs):
    import paper_0710_0066_amd as sap
    print(f"f16 apply_Dslash_eo L={L} nrhs={nrhs}", flush=True)
    U = synth.gauge_field(L, 0.5, 1107)
    psi = synth.gaussian_spinor(L, 2107, nrhs=nrhs)
    par = lattice.parity(L)
    ctx = gu.make_ctx(L, l0, k, U, l0_sub, max_rhs=nrhs)
    for parity in (0, 1):
        m_out = lattice.site_mask(L, par == parity)
        ref = dirac.hop(U, psi * lattice.site_mask(L, par != parity)) * m_out
        fin = gu.to_sap(ctx, psi, nrhs, sap.SAP_F16)
        fout = gu.to_sap(ctx, psi, nrhs, sap.SAP_F16)   # the other parity must stay as it was
        sap.apply_Dslash_eo(ctx, fout, fin, nrhs, parity, sap.SAP_F16)
        got = gu.from_sap(ctx, fout, nrhs, psi.shape, sap.SAP_F16)
        keep = np.broadcast_to(~(m_out != 0), got.shape)
        assert np.array_equal(got[keep], gu.from_sap(ctx, fin, nrhs, psi.shape, sap.SAP_F16)[keep])
        # the bare hop has no unit term: 8 hops of kappa = 1
        assert _err_vs_input(got * m_out, ref, psi) <= F16_TOL / 0.16, parity


def _relres(U, x, b, k, lb=None, mask=None):
    r = b - dirac.apply_op(U, x, k, lb)
    if mask is not None:
        r = r * mask
        b = b * mask
    ax = tuple(range(r.ndim - 6, r.ndim))
    return np.sqrt(np.sum(np.abs(r) ** 2, axis=ax) / np.sum(np.abs(b) ** 2, axis=ax))


def _opts(sap, method, tol=1e-10):
    m = {"cg": sap.SAP_CG, "bicgstab": sap.SAP_BICGSTAB, "geom": sap.SAP_GEOM,
         "sap_bicgstab": sap.SAP_SAP_BICGSTAB}[method]
    return sap.solve_opts(tol=tol, max_iter=200000, inner_prec=sap.SAP_F16, inner_tol=1e-2, max_outer=80,
                          method=m, sap_ncy=2)


@pytest.mark.parametrize("method", ["cg", "bicgstab", "geom", "sap_bicgstab"])
def test_solve_full_f16_inner_matches_dense_solution(gu, method):
    import paper_0710_0066_amd as sap
    L, l0, k = (4, 4, 4, 4), 2, 0.12
    print(f"f16 solve_full {method}", flush=True)
    U = synth.gauge_field(L, 0.5, 1109)
    b = synth.gaussian_spinor(L, 2109, nrhs=2)
    A = dirac.dense_matrix(U, k)
    x_lu = np.linalg.solve(A, b.reshape(2, -1).T).T.reshape(b.shape)
    ctx = gu.make_ctx(L, l0, k, U, max_rhs=2)
    fx = ctx.new_field(2)
    info = sap.solve_full(ctx, fx, gu.to_sap(ctx, b, 2), 2, _opts(sap, method))
    x = gu.from_sap(ctx, fx, 2, b.shape)
    res = _relres(U, x, b, k)
    assert np.all(res <= 1e-10), res
    for i in range(2):
        assert abs(info[i].true_rel_res - res[i]) <= 1e-12 and info[i].iters > 0
    assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) <= np.linalg.cond(A) * 1e-10


@pytest.mark.parametrize("method", ["cg", "bicgstab"])
@pytest.mark.parametrize("level,color", [(1, "all"), (1, "black"), (2, "white")])
def test_solve_blocks_f16_inner_matches_oracle(gu, method, level, color):
    import paper_0710_0066_amd as sap
    L, l0, l0s, k = (16, 4, 2, 4), 4, 2, 0.15
    print(f"f16 solve_blocks {method} level={level} color={color}", flush=True)
    U = synth.gauge_field(L, 0.5, 1111)
    b = synth.gaussian_spinor(L, 2111, nrhs=3)
    lb = l0 if level == 1 else l0s
    m = lattice.site_mask(L, lattice.colour_x0_mask(L, lb, color))
    x_ref, _, _ = solvers.solve_eo(U, b * m, k, lb, tol=1e-13)
    ctx = gu.make_ctx(L, l0, k, U, l0s, max_rhs=3)
    fx = ctx.new_field(3)
    fx.fill_(3.0)
    cmap = {"all": sap.SAP_ALL, "black": sap.SAP_BLACK, "white": sap.SAP_WHITE}
    info = sap.solve_blocks(ctx, fx, gu.to_sap(ctx, b, 3), 3, level, cmap[color], _opts(sap, method))
    x = gu.from_sap(ctx, fx, 3, b.shape)
    assert np.all(x[~np.broadcast_to(m != 0, x.shape)] == 0)
    assert np.all(_relres(U, x, b, k, lb, m) <= 1e-10)
    assert np.max(np.abs(x - x_ref)) / np.max(np.abs(x_ref)) <= 1e-7
    assert max(i.outer for i in info) >= 2          # FP16 inner solves need several corrections


def test_f16_links_follow_gauge_updates(gu):
    """The reduced link copies follow the links when they change. After set_gauge, FP16
    apply_M tracks the oracle on the new field. After the HMC link update (which writes
    the copies itself) and after a translation in x0 (the copy kernel), the even-odd hop
    matches the oracle on the links read back in FP64: in FP16 with the LDS-staged mapping
    (which reads the three-row FP16 copy) and with march2 (the two-row copy), in FP32 and
    in FP64."""
    import torch
    import paper_0710_0066_amd as sap
    L, l0, k = (8, 4, 4, 4), 4, 0.15
    U0 = synth.gauge_field(L, 0.5, 1113)
    U1 = synth.gauge_field(L, 0.5, 1114)
    psi = synth.gaussian_spinor(L, 2113)
    ctx = gu.make_ctx(L, l0, k, U0, max_rhs=2)
    ctx.set_gauge(gu.dev(U1))
    fout = ctx.new_field(1, sap.SAP_F16)
    sap.apply_M(ctx, fout, gu.to_sap(ctx, psi, 1, sap.SAP_F16), 1, sap.SAP_F16)
    got = gu.from_sap(ctx, fout, 1, psi.shape, sap.SAP_F16)
    assert _err_vs_input(got, dirac.apply_M(U1, psi, k), psi) <= F16_TOL

    par = lattice.parity(L)
    psi2 = synth.gaussian_spinor(L, 2114, nrhs=2)
    cases = [(sap.SAP_F16, 20, F16_TOL / 0.16), (sap.SAP_F16, 12, F16_TOL / 0.16),
             (sap.SAP_F32, 20, F32_TOL / 0.16), (sap.SAP_F64, 12, 1e-12)]

    def check_hops(step):
        Uo = torch.zeros(U1.size, dtype=torch.complex128, device="cuda")
        ctx.get_gauge(Uo)
        U = Uo.cpu().numpy().reshape(U1.shape)
        for prec, hop_map, tol in cases:
            sap.sap_set_hop_map(ctx, 0, prec, 2, hop_map)
            fin = gu.to_sap(ctx, psi2, 2, prec)
            fo = ctx.new_field(2, prec)
            for parity in (0, 1):
                m_out = lattice.site_mask(L, par == parity)
                ref = dirac.hop(U, psi2 * lattice.site_mask(L, par != parity)) * m_out
                sap.apply_Dslash_eo(ctx, fo, fin, 2, parity, prec)
                got = gu.from_sap(ctx, fo, 2, psi2.shape, prec) * m_out
                assert _err_vs_input(got, ref, psi2) <= tol, (step, prec, hop_map, parity)

    P = ctx.new_momenta()
    g = torch.Generator(device="cpu").manual_seed(1115)
    P.copy_(0.3 * torch.randn(P.numel(), generator=g, dtype=torch.float64))
    sap.sap_update_links(ctx, P, 0.7)
    check_hops("update")
    sap.sap_shift_gauge(ctx, 1)
    check_hops("shift")


F32_TOL = 64 * 2.0 ** -24      # the same bound with FP32 rounding, plus FP32 accumulation


@pytest.mark.parametrize("prec_name", ["f32", "f16"])
def test_precision_16x16x16x32_operator_error_and_solves(gu, prec_name):
    """The 16^3x32 workload (kappa = 0.1575) in FP32 and FP16 storage: apply_M and apply_W1
    against the FP64 oracle on every element, and full and block solves whose inner
    iterations run at that storage precision, to a 1e-10 residual recomputed by the
    oracle; the reduced-precision solution is compared with the FP64-inner one. The errors
    are printed."""
    import paper_0710_0066_amd as sap
    prec = {"f32": sap.SAP_F32, "f16": sap.SAP_F16}[prec_name]
    tol = {"f32": F32_TOL, "f16": F16_TOL}[prec_name]
    itol = {"f32": 1e-5, "f16": 1e-2}[prec_name]
    cfg = synth.CONFIGS["precision_16x16x16x32"]
    L, k, l0 = cfg["L"], cfg["kappa"], cfg["l0"]
    print(f"{prec_name} 16^3x32", flush=True)
    U = synth.gauge_field(L, cfg["eps"], cfg["seed_gauge"])
    psi = synth.gaussian_spinor(L, cfg["seed_src"])
    ctx = gu.make_ctx(L, l0, k, U, cfg["l0_sub"], max_rhs=1)
    fin = gu.to_sap(ctx, psi, 1, prec)
    fout = ctx.new_field(1, prec)
    sap.apply_M(ctx, fout, fin, 1, prec)
    eM = _err_vs_input(gu.from_sap(ctx, fout, 1, psi.shape, prec), dirac.apply_M(U, psi, k), psi)
    sap.apply_W1_block(ctx, fout, fin, 1, 1, -1, sap.SAP_ALL, prec)
    eW = _err_vs_input(gu.from_sap(ctx, fout, 1, psi.shape, prec), dirac.apply_W(U, psi, k, l0), psi)
    print(f"  apply_M {prec_name} max error / max|psi| = {eM:.2e}, apply_W1 {eW:.2e}", flush=True)
    assert eM <= tol and eW <= tol
    fb = gu.to_sap(ctx, psi, 1)
    x = {}
    for name, p, it in (("f64", sap.SAP_F64, 0.0), (prec_name, prec, itol)):
        fx = ctx.new_field(1)
        o = sap.solve_opts(tol=1e-10, max_iter=500000, inner_prec=p, inner_tol=it, max_outer=200)
        info = sap.solve_full(ctx, fx, fb, 1, o)
        x[name] = gu.from_sap(ctx, fx, 1, psi.shape)
        res = float(_relres(U, x[name], psi, k))
        print(f"  solve_full inner={name}: iters={info[0].iters} outer={info[0].outer} res={res:.2e}", flush=True)
        assert res <= 1e-10
    d = float(np.linalg.norm(x[prec_name] - x["f64"]) / np.linalg.norm(x["f64"]))
    print(f"  |x_{prec_name} - x_f64| / |x_f64| = {d:.2e}", flush=True)
    assert d <= 1e-7
    fx = ctx.new_field(1)
    o = sap.solve_opts(tol=1e-10, max_iter=500000, inner_prec=prec, inner_tol=itol, max_outer=80)
    info = sap.solve_blocks(ctx, fx, fb, 1, 1, sap.SAP_ALL, o)
    xb = gu.from_sap(ctx, fx, 1, psi.shape)
    res = float(np.max(_relres(U, xb, psi, k, l0)))
    print(f"  solve_blocks inner={prec_name}: max iters={max(i.iters for i in info)} "
          f"outer={max(i.outer for i in info)} res={res:.2e}", flush=True)
    assert res <= 1e-10


@pytest.mark.parametrize("hop_map", [0, 11, 12, 13, 14, 20])
@pytest.mark.parametrize("L,l0,l0_sub,k", [SHAPES[1], SHAPES[3], ((32, 4, 4, 6), 4, 2, 0.15),
                                          ((16, 10, 10, 12), 4, 2, 0.14)])
def test_every_f16_hop_mapping_matches_oracle(gu, hop_map, L, l0, l0_sub, k):
    """The FP16 hop with each of its work-item mappings (site, x0-marching with 1 / 2 / 4
    rhs per work-item, walk1 running as march1, and the LDS-staged slab kernel) gives the
    oracle's D_eo and M with 1 and 5 right-hand sides, and the block solves that use the
    gamma_5-folded, block-restricted and colour-selected forms reach a 1e-10 residual. On
    the 16 x 10^2 x 12 lattice the slab tile (5 x 5 x 6 sites) has halos in x1 and x2."""
    import paper_0710_0066_amd as sap
    print(f"f16 hop map {hop_map} L={L}", flush=True)
    U = synth.gauge_field(L, 0.5, 1121)
    par = lattice.parity(L)
    for nrhs in (1, 5):
        psi = synth.gaussian_spinor(L, 2121 + nrhs, nrhs=nrhs)
        ctx = gu.make_ctx(L, l0, k, U, l0_sub, max_rhs=nrhs)
        sap.sap_set_hop_map(ctx, 0, sap.SAP_F16, nrhs, hop_map)
        sap.sap_set_hop_map(ctx, 1, sap.SAP_F16, nrhs, hop_map)
        fin = gu.to_sap(ctx, psi, nrhs, sap.SAP_F16)
        fout = ctx.new_field(nrhs, sap.SAP_F16)
        for parity in (0, 1):
            m_out = lattice.site_mask(L, par == parity)
            ref = dirac.hop(U, psi * lattice.site_mask(L, par != parity)) * m_out
            sap.apply_Dslash_eo(ctx, fout, fin, nrhs, parity, sap.SAP_F16)
            got = gu.from_sap(ctx, fout, nrhs, psi.shape, sap.SAP_F16) * m_out
            assert _err_vs_input(got, ref, psi) <= F16_TOL / 0.16, (nrhs, parity)
        sap.apply_M(ctx, fout, fin, nrhs, sap.SAP_F16)
        got = gu.from_sap(ctx, fout, nrhs, psi.shape, sap.SAP_F16)
        assert _err_vs_input(got, dirac.apply_M(U, psi, k), psi) <= F16_TOL, nrhs
        fb = gu.to_sap(ctx, psi, nrhs)
        fx = ctx.new_field(nrhs)
        opts = sap.solve_opts(tol=1e-10, inner_prec=sap.SAP_F16, inner_tol=1e-2, max_outer=80)
        cases = [(1, l0, sap.SAP_BLACK, "black")] + ([(2, l0_sub, sap.SAP_ALL, "all")] if l0_sub else [])
        for level, lb, colour, cname in cases:
            sap.solve_blocks(ctx, fx, fb, nrhs, level, colour, opts)
            x = gu.from_sap(ctx, fx, nrhs, psi.shape)
            msk = lattice.site_mask(L, lattice.colour_x0_mask(L, lb, cname))
            assert np.all(_relres(U, x, psi, k, lb, msk) <= 1e-10), (nrhs, level)
