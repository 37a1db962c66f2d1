"""GPU parity of apply_M and apply_W1_block (FP64 and FP32) against the FP64 oracle on
the same seeded inputs, element by element, on lattices that span several workgroups and
have ragged tails, on the 16^3x32 workload, and on the 24^3x48 workload."""
import numpy as np
import pytest

import synth
from oracle import dirac, lattice

pytestmark = pytest.mark.gpu

SHAPES = [  # (L, l0, l0_sub, kappa)
    ((4, 4, 4, 4), 2, 0, 0.155),
    ((6, 2, 4, 6), 3, 0, 0.16),            # V/2 = 144: one partial workgroup
    ((8, 6, 2, 10), 2, 0, 0.13),           # V/2 = 480: ragged tail
    ((16, 4, 6, 4), 4, 2, 0.1575),         # level-2 blocks
]
F64_TOL = 1e-13
F32_TOL = 2e-6


@pytest.fixture(scope="module")
def gu():
    import gpu_util
    return gpu_util


@pytest.mark.parametrize("L,l0,l0_sub,k", SHAPES)
@pytest.mark.parametrize("nrhs", [1, 3])
def test_apply_M_matches_oracle(gu, L, l0, l0_sub, k, nrhs):
    import paper_0710_0066_amd as sap
    print(f"apply_M L={L} nrhs={nrhs}", flush=True)
    U = synth.gauge_field(L, 0.5, 1001)
    psi = synth.gaussian_spinor(L, 2001, nrhs=nrhs)
    ref = dirac.apply_M(U, psi, k)
    ctx = gu.make_ctx(L, l0, k, U, l0_sub, max_rhs=nrhs)
    for prec, tol in [(sap.SAP_F64, F64_TOL), (sap.SAP_F32, F32_TOL)]:
        fin = gu.to_sap(ctx, psi, nrhs, prec)
        fout = ctx.new_field(nrhs, prec)
        sap.apply_M(ctx, fout, fin, nrhs, prec)
        got = gu.from_sap(ctx, fout, nrhs, psi.shape, prec)
        assert gu.rel_err(got, ref) <= tol, (prec, gu.rel_err(got, ref))


@pytest.mark.parametrize("L,l0,l0_sub,k", SHAPES)
def test_apply_W_matches_oracle(gu, L, l0, l0_sub, k):
    import paper_0710_0066_amd as sap
    print(f"apply_W1_block L={L}", flush=True)
    U = synth.gauge_field(L, 0.5, 1003)
    psi = synth.gaussian_spinor(L, 2003, nrhs=2)
    ctx = gu.make_ctx(L, l0, k, U, l0_sub, max_rhs=2)
    levels = [(1, l0)] + ([(2, l0_sub)] if l0_sub else [])
    for level, lb in levels:
        ref_all = dirac.apply_W(U, psi, k, lb)
        nb = L[0] // lb
        cases = [(-1, sap.SAP_ALL, "all"), (-1, sap.SAP_BLACK, "black"), (-1, sap.SAP_WHITE, "white"),
                 (nb - 1, sap.SAP_ALL, None), (0, sap.SAP_BLACK, None)]
        for block, color, cname in cases:
            if block >= 0:
                m = lattice.single_block_mask(L, lb, block)
            else:
                m = lattice.colour_x0_mask(L, lb, cname)
            ref = ref_all * lattice.site_mask(L, m)
            for prec, tol in [(sap.SAP_F64, F64_TOL), (sap.SAP_F32, F32_TOL)]:
                fin = gu.to_sap(ctx, psi, 2, prec)
                fout = ctx.new_field(2, prec)
                fout.fill_(7.0)        # every site must be written
                sap.apply_W1_block(ctx, fout, fin, 2, level, block, color, prec)
                got = gu.from_sap(ctx, fout, 2, psi.shape, prec)
                err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref_all)))
                assert err <= tol, (level, block, color, prec, err)


@pytest.mark.parametrize("L,l0,l0_sub,k", SHAPES[:3])
@pytest.mark.parametrize("nrhs", [1, 5])
def test_apply_Dslash_eo_matches_oracle(gu, L, l0, l0_sub, k, nrhs):
    """D_eo / D_oe: the hop of eq. 2 restricted to one output parity, reading the other."""
    import paper_0710_0066_amd as sap
    print(f"apply_Dslash_eo L={L} nrhs={nrhs}", flush=True)
    U = synth.gauge_field(L, 0.5, 1011)
    psi = synth.gaussian_spinor(L, 2011, nrhs=nrhs)
    par = lattice.parity(L)
    ctx = gu.make_ctx(L, l0, k, U, l0_sub, max_rhs=nrhs)
    for parity in (0, 1):
        m_out = lattice.site_mask(L, par == parity)
        ref = dirac.hop(U, psi * lattice.site_mask(L, par != parity)) * m_out
        for prec, tol in [(sap.SAP_F64, F64_TOL), (sap.SAP_F32, F32_TOL)]:
            fin = gu.to_sap(ctx, psi, nrhs, prec)
            fout = gu.to_sap(ctx, psi, nrhs, prec)      # the other parity must stay as it was
            sap.apply_Dslash_eo(ctx, fout, fin, nrhs, parity, prec)
            got = gu.from_sap(ctx, fout, nrhs, psi.shape, prec)
            keep = np.broadcast_to(~m_out, got.shape)
            assert np.array_equal(got[keep], gu.from_sap(ctx, fin, nrhs, psi.shape, prec)[keep])
            assert gu.rel_err(got * m_out, ref) <= tol, (parity, prec)


@pytest.mark.parametrize("hop_map", list(range(21)))
@pytest.mark.parametrize("L,l0,l0_sub,k", [SHAPES[1], SHAPES[3], ((32, 4, 4, 6), 4, 2, 0.15),
                                          ((16, 10, 10, 12), 4, 2, 0.14)])
def test_every_hop_mapping_matches_oracle(gu, hop_map, L, l0, l0_sub, k):
    """Each work-item mapping of the hop kernel (site, lane4, wave4, their rhs-slowest
    orders, register-blocked 2 / 4 rhs, x0-marching per XCD and, for the even-odd hop, the
    x0-streaming kernel with LDS staging, the x0-walking kernels with time neighbours
    carried in registers, the x0-band kernel with one band of slices per XCD and the slab
    kernels with LDS-staged spatial tiles) gives the oracle's D_eo, M and W, with 1 and 5
    right-hand sides, including the gamma_5-folded and block-restricted forms the solvers
    use (through solve_blocks with CG and BiCGstab, which with the LDS-staged FP32 mapping
    also take their norms and dot products from the hop). On the 16 x 10^2 x 12 lattice
    the slab tiles (5 x 5 x 12 sites in FP32, 2 x 5 x 12 in FP64) leave halos in both x1
    and x2 and every XCD walks a band of two slices."""
    import paper_0710_0066_amd as sap
    print(f"hop map {hop_map} L={L}", flush=True)
    U = synth.gauge_field(L, 0.5, 1021)
    par = lattice.parity(L)
    for nrhs in (1, 5):
        psi = synth.gaussian_spinor(L, 2021 + nrhs, nrhs=nrhs)
        ctx = gu.make_ctx(L, l0, k, U, l0_sub, max_rhs=nrhs)
        for prec, tol in [(sap.SAP_F64, F64_TOL), (sap.SAP_F32, F32_TOL)]:
            sap.sap_set_hop_map(ctx, 0, prec, nrhs, hop_map)
            if hop_map != 3:
                sap.sap_set_hop_map(ctx, 1, prec, nrhs, hop_map)   # full operator too
            fin = gu.to_sap(ctx, psi, nrhs, prec)
            fout = ctx.new_field(nrhs, prec)
            for parity in (0, 1):
                m_out = lattice.site_mask(L, par == parity)
                ref = dirac.hop(U, psi * lattice.site_mask(L, par != parity)) * m_out
                sap.apply_Dslash_eo(ctx, fout, fin, nrhs, parity, prec)
                got = gu.from_sap(ctx, fout, nrhs, psi.shape, prec) * m_out
                assert gu.rel_err(got, ref) <= tol, (nrhs, prec, parity)
            sap.apply_M(ctx, fout, fin, nrhs, prec)
            assert gu.rel_err(gu.from_sap(ctx, fout, nrhs, psi.shape, prec), dirac.apply_M(U, psi, k)) <= tol
        # the solvers' even-odd block hops (gamma_5 folding, block drop, colour selection)
        b = psi
        fb = gu.to_sap(ctx, b, nrhs)
        fx = ctx.new_field(nrhs)
        cases = [(1, l0, sap.SAP_BLACK, "black", sap.SAP_CG)]
        if l0_sub:
            cases += [(2, l0_sub, sap.SAP_ALL, "all", sap.SAP_CG), (2, l0_sub, sap.SAP_ALL, "all", sap.SAP_BICGSTAB)]
        for level, lb, colour, cname, method in cases:
            opts = sap.solve_opts(tol=1e-10, inner_prec=sap.SAP_F32, inner_tol=1e-5, method=method)
            sap.solve_blocks(ctx, fx, fb, nrhs, level, colour, opts)
            x = gu.from_sap(ctx, fx, nrhs, b.shape)
            msk = lattice.site_mask(L, lattice.colour_x0_mask(L, lb, cname))
            r = (b - dirac.apply_W(U, x, k, lb)) * msk
            ax = tuple(range(r.ndim - 6, r.ndim))
            res = np.sqrt(np.sum(np.abs(r) ** 2, axis=ax) / np.sum(np.abs(b * msk) ** 2, axis=ax))
            assert np.all(res <= 1e-10), (level, method, res)


@pytest.mark.parametrize("name", ["plain_16x16x16x32", "batched_24x24x24x48"])
def test_apply_M_and_W_full_size(gu, name):
    """Full-size workloads in the launch configuration the benchmark times: every
    element compared with the oracle (FP64 <= 1e-13, FP32 error bounded)."""
    import paper_0710_0066_amd as sap
    cfg = synth.CONFIGS[name]
    L, k, l0 = cfg["L"], cfg["kappa"], cfg["l0"]
    print(f"full size {name}", flush=True)
    U = synth.gauge_field(L, cfg["eps"], cfg["seed_gauge"])
    psi = synth.gaussian_spinor(L, cfg["seed_src"])
    ctx = gu.make_ctx(L, l0, k, U, cfg["l0_sub"], max_rhs=1)
    refM = dirac.apply_M(U, psi, k)
    refW = dirac.apply_W(U, psi, k, l0)
    for prec, tol in [(sap.SAP_F64, F64_TOL), (sap.SAP_F32, F32_TOL)]:
        fin = gu.to_sap(ctx, psi, 1, prec)
        fout = ctx.new_field(1, prec)
        sap.apply_M(ctx, fout, fin, 1, prec)
        assert gu.rel_err(gu.from_sap(ctx, fout, 1, psi.shape, prec), refM) <= tol
        sap.apply_W1_block(ctx, fout, fin, 1, 1, -1, sap.SAP_ALL, prec)
        assert gu.rel_err(gu.from_sap(ctx, fout, 1, psi.shape, prec), refW) <= tol


def test_benchmark_launch_24x24x24x48_12rhs(gu):
    """The benchmark's own launches: the even-odd hop on all 12 right-hand sides of the
    24^3x48 workload with the mappings bench.py times (bench.HEADLINE_MAPS) in FP64, FP32 and
    FP16 storage, both output parities, every rhs compared with the oracle's hop on every
    site; then the tuner's choices, three rhs checked."""
    import paper_0710_0066_amd as sap
    from bench import HEADLINE_MAPS, hop_map_id
    cfg = synth.CONFIGS["batched_24x24x24x48"]
    L, k, l0, nrhs = cfg["L"], cfg["kappa"], cfg["l0"], cfg["nrhs"]
    print(f"benchmark launch 24^3x48, 12 rhs, maps {HEADLINE_MAPS}", flush=True)
    U = synth.gauge_field(L, cfg["eps"], cfg["seed_gauge"])
    psi = synth.gaussian_spinor(L, cfg["seed_src"], nrhs=nrhs)
    ctx = gu.make_ctx(L, l0, k, U, cfg["l0_sub"], max_rhs=nrhs)
    ref = [dirac.hop(U, psi[r]) for r in range(nrhs)]
    f16_tol = 16 * 2.0 ** -12 / 0.16
    precs = {"f64": (sap.SAP_F64, F64_TOL), "f32": (sap.SAP_F32, F32_TOL), "f16": (sap.SAP_F16, f16_tol)}

    def run(prec, tol, rhs):
        fin = gu.to_sap(ctx, psi, nrhs, prec)
        fout = ctx.new_field(nrhs, prec)
        fout.fill_(3.0)
        for parity in (0, 1):
            sap.apply_Dslash_eo(ctx, fout, fin, nrhs, parity, prec)
        got = gu.from_sap(ctx, fout, nrhs, psi.shape, prec)
        for r in rhs:
            scale = np.max(np.abs(psi[r] if prec == sap.SAP_F16 else ref[r]))
            err = float(np.max(np.abs(got[r] - ref[r])) / scale)
            assert err <= tol, (prec, r, err)

    for name, (prec, tol) in precs.items():
        print(f"  {name} map {HEADLINE_MAPS[name]}", flush=True)
        sap.sap_set_hop_map(ctx, 0, prec, nrhs, hop_map_id(sap, HEADLINE_MAPS[name]))
        run(prec, tol, range(nrhs))
    tuned = sap.sap_tune(ctx, nrhs)
    print(f"  tuned even-odd maps: f32 {min(tuned['eo_f32'], key=tuned['eo_f32'].get)}, "
          f"f64 {min(tuned['eo_f64'], key=tuned['eo_f64'].get)}, f16 {min(tuned['eo_f16'], key=tuned['eo_f16'].get)}",
          flush=True)
    for name, (prec, tol) in precs.items():
        run(prec, tol, (0, 5, nrhs - 1))


def test_pack_unpack_roundtrip(gu):
    import paper_0710_0066_amd as sap
    L = (6, 2, 4, 6)
    U = synth.gauge_field(L, 0.5, 5)
    psi = synth.gaussian_spinor(L, 6, nrhs=2)
    ctx = gu.make_ctx(L, 3, 0.1, U, max_rhs=2)
    f = gu.to_sap(ctx, psi, 2)
    assert np.array_equal(gu.from_sap(ctx, f, 2, psi.shape), psi)
    import torch
    Uo = torch.zeros(U.size, dtype=torch.complex128, device="cuda")
    ctx.get_gauge(Uo)
    assert np.array_equal(Uo.cpu().numpy().reshape(U.shape), U)
    p = synth.gaussian_momenta(L, 7)
    fp = ctx.new_momenta()
    ctx.pack_momenta(fp, gu.dev(p))
    back = torch.zeros(p.size, dtype=torch.float64, device="cuda")
    ctx.unpack_momenta(back, fp)
    assert np.array_equal(back.cpu().numpy().reshape(p.shape), p)


def test_many_rhs_every_mapping_and_invalid_arguments(gu):
    """21 right-hand sides (odd, more groups than any workgroup or set holds) through every
    hop mapping in FP32 and FP16, three rhs checked against the oracle on every site; and
    the host-side argument checks: nrhs 0 or above max_rhs, an unknown precision, aliasing
    input and output."""
    import paper_0710_0066_amd as sap
    L, l0, k, nrhs = (8, 4, 2, 6), 2, 0.15, 21
    print("21 rhs, every mapping", flush=True)
    U = synth.gauge_field(L, 0.5, 1051)
    psi = synth.gaussian_spinor(L, 2051, nrhs=nrhs)
    ctx = gu.make_ctx(L, l0, k, U, max_rhs=nrhs)
    check = (0, 10, nrhs - 1)
    ref = {r: dirac.hop(U, psi[r]) for r in check}
    for prec, tol in [(sap.SAP_F32, F32_TOL), (sap.SAP_F16, 16 * 2.0 ** -12 / 0.16)]:
        fin = gu.to_sap(ctx, psi, nrhs, prec)
        fout = ctx.new_field(nrhs, prec)
        for hop_map in range(sap.HOP_NMAP):
            sap.sap_set_hop_map(ctx, 0, prec, nrhs, hop_map)
            fout.fill_(5.0)
            for parity in (0, 1):
                sap.apply_Dslash_eo(ctx, fout, fin, nrhs, parity, prec)
            got = gu.from_sap(ctx, fout, nrhs, psi.shape, prec)
            for r in check:
                scale = np.max(np.abs(psi[r] if prec == sap.SAP_F16 else ref[r]))
                err = float(np.max(np.abs(got[r] - ref[r])) / scale)
                assert err <= tol, (prec, hop_map, r, err)
        sap.sap_set_hop_map(ctx, 0, prec, nrhs, -1)
    f = ctx.new_field(1)
    g = ctx.new_field(1)
    for call in (lambda: sap.apply_M(ctx, f, g, 0, sap.SAP_F64),
                 lambda: sap.apply_M(ctx, f, g, nrhs + 1, sap.SAP_F64),
                 lambda: sap.apply_M(ctx, f, g, 1, 7),
                 lambda: sap.apply_Dslash_eo(ctx, f, g, 1, 2, sap.SAP_F64),
                 lambda: sap.solve_blocks(ctx, f, g, 0, 1, sap.SAP_ALL, sap.solve_opts()),
                 lambda: sap.solve_full(ctx, f, f, 1, sap.solve_opts())):
        with pytest.raises(sap.SapError) as e:
            call()
        assert e.value.code == sap.SAP_E_ARG
