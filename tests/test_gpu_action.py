"""GPU parity of the paper's four-part pseudo-fermion action (Sec. 1, end) and its
five-level trajectory (Sec. 2) against the oracle: the even-odd mass-preconditioned parts
S1, S2 and the level-2 Schwarz term S3 (heat bath, action, force), a whole trajectory on
a small lattice, and a 16^3x32 trajectory with Table 1's parameters for that lattice."""
import numpy as np
import pytest
import torch

import synth
from oracle import action, forces, hmc, schwarz

pytestmark = pytest.mark.gpu

L, L01, L02, K, RHO = (8, 4, 2, 4), 4, 2, 0.15, 0.2


@pytest.fixture(scope="module")
def gu():
    import gpu_util
    return gpu_util


def _opts(sap, tol=1e-13, inner=None):
    inner = sap.SAP_F64 if inner is None else inner
    return sap.solve_opts(tol=tol, max_iter=500000, inner_prec=inner, inner_tol=1e-6, max_outer=80)


def _mom_from_sap(ctx, f, Lat):
    out = torch.zeros(int(np.prod(Lat)) * 32, dtype=torch.float64, device="cuda")
    ctx.unpack_momenta(out, f)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(tuple(Lat) + (4, 8))


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_eo_pf_terms_match_oracle(gu):
    """S1 = ||W3eo^-1 phi||^2 and S2 = ||phi + rho W2eo^-1 phi||^2: heat bath, action (equal
    to ||P_e xi||^2 at the heat bath) and force, FP64, FP32 and FP16 inner solves (the
    shifted even-odd solves of W3eo = W2eo + rho run on FP16 fields in the last case)."""
    import paper_0710_0066_amd as sap
    print("eo pseudo-fermion terms", flush=True)
    U = synth.gauge_field(L, 0.5, 101)
    A = action.FourPart(U, K, L01, L02, RHO, tol=1e-13)
    ctx = gu.make_ctx(L, L01, K, U, L02)
    for kind in (1, 2):
        xi = synth.noise_spinor(L, 102 + kind)
        phi_ref = A.heat_bath1(A.e * xi) if kind == 1 else A.heat_bath2(A.e * xi)
        fphi = ctx.new_field(1)
        sap.eo_pf_heat_bath(ctx, fphi, gu.to_sap(ctx, xi, 1), kind, RHO, _opts(sap))
        assert _rel(gu.from_sap(ctx, fphi, 1, xi.shape), phi_ref) <= 1e-10
        S_ref = A.S1(phi_ref) if kind == 1 else A.S2(phi_ref)
        F_ref = A.F1(phi_ref) if kind == 1 else A.F2(phi_ref)
        assert abs(S_ref - float(np.sum(np.abs(A.e * xi) ** 2))) <= 1e-10 * S_ref
        for inner, ftol in ((sap.SAP_F64, 1e-9), (sap.SAP_F32, 1e-7), (sap.SAP_F16, 1e-7)):
            o = _opts(sap, tol=1e-13 if inner == sap.SAP_F64 else 1e-11, inner=inner)
            if inner == sap.SAP_F16:
                o.inner_tol = 2e-3
            F = ctx.new_momenta()
            S = sap.eo_pf_force(ctx, F, 1.0, fphi, kind, RHO, o)
            assert abs(S - S_ref) <= 1e-9 * S_ref, (kind, inner)
            assert _rel(_mom_from_sap(ctx, F, L), F_ref) <= ftol, (kind, inner)
        assert abs(sap.eo_pf_force(ctx, None, 0.0, fphi, kind, RHO, _opts(sap)) - S_ref) <= 1e-9 * S_ref
    with pytest.raises(sap.SapError):
        sap.eo_pf_force(ctx, F, 1.0, fphi, 3, RHO, _opts(sap))


def test_level2_schwarz_term_matches_oracle(gu):
    """S3: the Schwarz term of W1 over the level-2 blocks (heat bath, action = ||Pi_2 g||^2,
    force); a field outside the range of Pi_2 is rejected."""
    import paper_0710_0066_amd as sap
    print("level-2 schwarz term", flush=True)
    U = synth.gauge_field(L, 0.5, 111)
    A = action.FourPart(U, K, L01, L02, RHO, tol=1e-13)
    ctx = gu.make_ctx(L, L01, K, U, L02)
    g = synth.noise_spinor(L, 112)
    chi_ref = A.heat_bath3(g)
    fchi = ctx.new_field(1)
    sap.schwarz2_heat_bath(ctx, fchi, gu.to_sap(ctx, g, 1), _opts(sap))
    assert _rel(gu.from_sap(ctx, fchi, 1, g.shape), chi_ref) <= 1e-10
    F = ctx.new_momenta()
    S = sap.schwarz2_force(ctx, F, 1.0, fchi, _opts(sap))
    p3 = float(np.sum(np.abs(schwarz.Pi(g, L, L02, L01)) ** 2))
    assert abs(S - p3) <= 1e-9 * p3
    assert _rel(_mom_from_sap(ctx, F, L), A.F3(chi_ref)) <= 1e-9
    # the level-1 boundary field is not in the range of Pi_2
    f4 = ctx.new_field(1)
    sap.schwarz_heat_bath(ctx, f4, gu.to_sap(ctx, g, 1), _opts(sap))
    with pytest.raises(sap.SapError) as e:
        sap.schwarz2_force(ctx, F, 1.0, f4, _opts(sap))
    assert e.value.code == sap.SAP_E_ARG


def _inputs(Lat, seed):
    return (synth.gaussian_momenta(Lat, seed),) + tuple(synth.noise_spinor(Lat, seed + i) for i in (1, 2, 3, 4))


def test_hmc_4pf_trajectory_matches_oracle(gu):
    """A tau = 0.3 trajectory of the five-level scheme (gauge and S1 Sexton-Weingarten, S2,
    S3, S4 leap-frog, n = (2, 2, 1, 1, 2)) with the same momenta and noise on both sides."""
    import paper_0710_0066_amd as sap
    Lat, beta, tau, n = (8, 2, 2, 4), 5.6, 0.3, (2, 2, 1, 1, 2)
    print("four-part hmc vs oracle", flush=True)
    U = synth.gauge_field(Lat, 0.4, 121)
    p0, xi1, xi2, g3, g4 = _inputs(Lat, 122)
    A = action.FourPart(U, K, L01, L02, RHO, tol=1e-13)
    fields = (A.heat_bath1(A.e * xi1), A.heat_bath2(A.e * xi2), A.heat_bath3(g3), A.heat_bath4(g4))
    make = lambda V: action.FourPart(V, K, L01, L02, RHO, tol=1e-13)
    lev = action.five_level(fields, K, beta, L01, L02, RHO, n, make)
    U_ref, acc_ref, dH_ref, H0_ref, H1_ref = hmc.trajectory(lev, U, p0, tau, u_metropolis=0.0)
    ctx = gu.make_ctx(Lat, L01, K, U, L02)
    fU = gu.dev(U).clone()
    fp = ctx.new_momenta()
    ctx.pack_momenta(fp, gu.dev(p0))
    o = _opts(sap)
    prm = sap.hmc4_params(beta, tau, RHO, n, fp, gu.dev(xi1), gu.dev(xi2), gu.dev(g3), gu.dev(g4), 0.0, o, o)
    info = sap.hmc_trajectory_4pf(ctx, fU, prm)
    print(f"  dH gpu {info.dH:.12e} oracle {dH_ref:.12e}", flush=True)
    assert info.accepted == 1 and acc_ref
    assert abs(info.H0 - H0_ref) <= 1e-9 * abs(H0_ref)
    assert abs(info.dH - dH_ref) <= 1e-7 * max(1.0, abs(dH_ref))
    assert np.max(np.abs(fU.cpu().numpy().reshape(U.shape) - U_ref)) <= 1e-9


def test_hmc_4pf_16x16x16x32(gu):
    """One tau = 1 trajectory on 16^3x32 with Table 1's parameters for L0 = 32, L = 16,
    kappa = 0.1575 (scheme B, rho = 0.2, n4..n0 = 4, 1, 3, 2, 4), level-1 blocks of L0/2
    and level-2 blocks of L0/4 (Sec. 1), beta = 5.6, mixed-precision solves. Checks the
    heat-bath identities (each S_j equals its noise norm at the start) and reports dH."""
    import time
    import paper_0710_0066_amd as sap
    cfg = synth.CONFIGS["hmc_16x16x16x32"]
    Lat, k, beta = cfg["L"], cfg["kappa"], cfg["beta"]
    l01, l02, rho, n = Lat[0] // 2, Lat[0] // 4, 0.2, (4, 2, 3, 1, 4)
    print("four-part hmc 16^3x32", flush=True)
    U = synth.gauge_field(Lat, cfg["eps"], cfg["seed_gauge"])
    p0, xi1, xi2, g3, g4 = _inputs(Lat, cfg["seed_mom"])
    ctx = gu.make_ctx(Lat, l01, k, U, l02)
    fU = gu.dev(U).clone()
    fp = ctx.new_momenta()
    ctx.pack_momenta(fp, gu.dev(p0))
    fo = _opts(sap, tol=1e-10, inner=sap.SAP_F32)
    ao = _opts(sap, tol=1e-12, inner=sap.SAP_F32)
    scale = hmc.step_profile("B", Lat[0])
    prm = sap.hmc4_params(beta, 1.0, rho, n, fp, gu.dev(xi1), gu.dev(xi2), gu.dev(g3), gu.dev(g4), 0.5, fo, ao,
                          step_scale=scale)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = sap.hmc_trajectory_4pf(ctx, fU, prm)
    dt = time.perf_counter() - t0
    print(f"  dH {info.dH:.6e} accepted {info.accepted} S0 {list(info.S0)} iters {info.solver_iters} "
          f"{dt:.2f}s", flush=True)
    e = np.array([1.0, 0.0])[np.indices(Lat).sum(axis=0) % 2][..., None, None]
    n2 = lambda f: float(np.sum(np.abs(f) ** 2))
    assert abs(info.S0[1] - n2(e * xi1)) <= 1e-8 * info.S0[1]
    assert abs(info.S0[2] - n2(e * xi2)) <= 1e-8 * info.S0[2]
    assert abs(info.S0[3] - n2(schwarz.Pi(g3, Lat, l02, l01))) <= 1e-8 * info.S0[3]
    assert abs(info.S0[4] - n2(schwarz.Pi(g4, Lat, l01))) <= 1e-8 * info.S0[4]
    assert np.isfinite(info.dH) and info.accepted == (0.5 < np.exp(-info.dH))


def test_eo_pf_terms_with_geometric_series_match_oracle(gu):
    """S1 and S2 with the solver Sec. 3 uses for them, the geometric series of the
    even-site systems (W3eo = W2eo + rho: every term carries 1 / (1 + rho)), in FP64 and
    with FP32 inner terms: heat bath, action and force against the oracle's CGLS-based
    values (the solutions are unique, so only the solver tolerance separates them)."""
    import paper_0710_0066_amd as sap
    print("eo pseudo-fermion terms, geometric series", flush=True)
    U = synth.gauge_field(L, 0.5, 141)
    A = action.FourPart(U, K, L01, L02, RHO, tol=1e-13)
    ctx = gu.make_ctx(L, L01, K, U, L02)
    for kind in (1, 2):
        xi = synth.noise_spinor(L, 142 + kind)
        phi_ref = A.heat_bath1(A.e * xi) if kind == 1 else A.heat_bath2(A.e * xi)
        S_ref = A.S1(phi_ref) if kind == 1 else A.S2(phi_ref)
        F_ref = A.F1(phi_ref) if kind == 1 else A.F2(phi_ref)
        for inner, tol, ftol in ((sap.SAP_F64, 1e-13, 1e-9), (sap.SAP_F32, 1e-11, 1e-7)):
            o = _opts(sap, tol=tol, inner=inner)
            o.method = sap.SAP_GEOM
            fphi = ctx.new_field(1)
            sap.eo_pf_heat_bath(ctx, fphi, gu.to_sap(ctx, xi, 1), kind, RHO, o)
            assert _rel(gu.from_sap(ctx, fphi, 1, xi.shape), phi_ref) <= 1e-9, (kind, inner)
            F = ctx.new_momenta()
            S = sap.eo_pf_force(ctx, F, 1.0, fphi, kind, RHO, o)
            assert abs(S - S_ref) <= 1e-9 * S_ref, (kind, inner, S, S_ref)
            assert _rel(_mom_from_sap(ctx, F, L), F_ref) <= ftol, (kind, inner)


def test_hmc_4pf_trajectory_with_the_papers_solvers_matches_oracle(gu):
    """The five-level trajectory with Sec. 3's solver assignment through part_solve: the
    geometric series for S1, S2 and S3 (even-site series with the 1 / (1 + rho) factor for
    S1 and S2; level-1 and level-2 block series for S3) and BiCGstab on M right-preconditioned
    by a Schwarz cycle with 8-term series block solves for S4 (its heat bath runs even-odd
    BiCGstab on the blocks), against the oracle's trajectory with CGLS solves: same dH and
    links to the solver tolerance."""
    import paper_0710_0066_amd as sap
    Lat, k, beta, tau, n = (8, 2, 2, 4), 0.13, 5.6, 0.3, (2, 2, 1, 1, 2)
    print("four-part hmc, paper's solvers, vs oracle", flush=True)
    U = synth.gauge_field(Lat, 0.4, 151)
    p0, xi1, xi2, g3, g4 = _inputs(Lat, 152)
    A = action.FourPart(U, k, L01, L02, RHO, tol=1e-13)
    fields = (A.heat_bath1(A.e * xi1), A.heat_bath2(A.e * xi2), A.heat_bath3(g3), A.heat_bath4(g4))
    make = lambda V: action.FourPart(V, k, L01, L02, RHO, tol=1e-13)
    lev = action.five_level(fields, k, beta, L01, L02, RHO, n, make)
    U_ref, acc_ref, dH_ref, H0_ref, H1_ref = hmc.trajectory(lev, U, p0, tau, u_metropolis=0.0)
    ctx = gu.make_ctx(Lat, L01, k, U, L02)
    fU = gu.dev(U).clone()
    fp = ctx.new_momenta()
    ctx.pack_momenta(fp, gu.dev(p0))
    geom = _opts(sap)
    geom.method = sap.SAP_GEOM
    sapb = _opts(sap)
    sapb.method, sapb.sap_ncy, sapb.sap_block_terms, sapb.max_iter = sap.SAP_SAP_BICGSTAB, 1, 8, 2000
    parts = [geom, geom, geom, sapb] * 2
    o = _opts(sap)
    prm = sap.hmc4_params(beta, tau, RHO, n, fp, gu.dev(xi1), gu.dev(xi2), gu.dev(g3), gu.dev(g4), 0.0, o, o,
                          part_solve=parts)
    info = sap.hmc_trajectory_4pf(ctx, fU, prm)
    print(f"  dH gpu {info.dH:.12e} oracle {dH_ref:.12e} iters {info.solver_iters}", flush=True)
    assert info.accepted == 1 and acc_ref
    assert abs(info.H0 - H0_ref) <= 1e-9 * abs(H0_ref)
    assert abs(info.dH - dH_ref) <= 1e-7 * max(1.0, abs(dH_ref))
    assert np.max(np.abs(fU.cpu().numpy().reshape(U.shape) - U_ref)) <= 1e-9
    with pytest.raises(sap.SapError) as e:
        sap.hmc4_params(beta, tau, RHO, n, fp, gu.dev(xi1), gu.dev(xi2), gu.dev(g3), gu.dev(g4), 0.0, o, o,
                        part_solve=parts[:4])
    assert e.value.code == sap.SAP_E_ARG
