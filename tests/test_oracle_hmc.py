"""Pins of the oracle's molecular dynamics: the link exponential against scipy's expm,
unitarity and det 1, reversibility of a two-level Sexton-Weingarten trajectory, and the
second-order scaling dH ~ h^2 of both integrators (Sec. 2)."""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import forces, hmc, schwarz, solvers


def test_exp_iP_matches_expm_and_is_special_unitary():
    p = synth.gaussian_momenta((2, 2, 2, 2), 61)
    E = hmc.exp_iP(p, 0.37)
    P = hmc.su3_algebra(p)
    for idx in [(0, 0, 0, 0, 0), (1, 0, 1, 1, 3), (1, 1, 1, 1, 2)]:
        np.testing.assert_allclose(E[idx], scipy.linalg.expm(0.37j * P[idx]), atol=1e-14)
    eye = np.broadcast_to(np.eye(3), E.shape)
    np.testing.assert_allclose(E @ np.swapaxes(E.conj(), -1, -2), eye, atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(E), 1.0, atol=1e-14)
    # T^a are orthonormal: Tr(T^a T^b) = delta_ab / 2, so 1/2 sum p^2 = Tr P^2
    np.testing.assert_allclose(np.trace(P @ P, axis1=-2, axis2=-1).real,
                               0.5 * np.sum(p * p, axis=-1), atol=1e-13)


def _levels(L, U, k, l0, n_outer, n_inner, tol=1e-13):
    phi = synth.gaussian_spinor(L, 62)
    mk = lambda V: schwarz.Solvers(V, k, l0, tol=tol)
    chi = schwarz.heat_bath(U, synth.noise_spinor(L, 63), k, l0, mk(U))
    return hmc.schwarz_two_level(phi, chi, k, 5.6, l0, n_outer, n_inner, mk)


def test_reversibility_two_level_sw():
    L, l0, k = (8, 2, 2, 2), 2, 0.15
    U = synth.gauge_field(L, 0.4, 64)
    p = synth.gaussian_momenta(L, 65)
    lev = _levels(L, U, k, l0, n_outer=3, n_inner=2)
    U1, p1 = hmc.integrate(lev, U, p, 0.5)
    U2, p2 = hmc.integrate(lev, U1, -p1, 0.5)
    assert np.max(np.abs(U2 - U)) <= 1e-10
    assert np.max(np.abs(p2 + p)) <= 1e-9


@pytest.mark.parametrize("scheme", ["SW", "LF"])
def test_dH_scales_as_h_squared(scheme):
    L, l0, k = (8, 2, 2, 2), 2, 0.15
    U = synth.gauge_field(L, 0.4, 66)
    p = synth.gaussian_momenta(L, 67)
    dH = []
    for n in (4, 8):
        lev = _levels(L, U, k, l0, n_outer=n, n_inner=2)
        for lv in lev:
            lv.scheme = scheme
        H0 = hmc.hamiltonian(lev, U, p)
        U1, p1 = hmc.integrate(lev, U, p, 0.1)
        dH.append(hmc.hamiltonian(lev, U1, p1) - H0)
    ratio = dH[0] / dH[1]
    assert 3.6 < ratio < 4.4, (dH, ratio)


def test_pure_gauge_trajectory_metropolis():
    """kappa = 0 limit: only S_G; dH small and decisions follow min(1, exp(-dH))."""
    L = (4, 4, 4, 4)
    U = synth.gauge_field(L, 0.3, 68)
    p = synth.gaussian_momenta(L, 69)
    lev = [hmc.Level(lambda V: forces.gauge_force(V, 5.6), lambda V: forces.gauge_action(V, 5.6),
                     "SW", 20)]
    Uo, acc, dH, H0, H1 = hmc.trajectory(lev, U, p, 1.0, u_metropolis=0.0)
    assert acc and abs(dH) < 0.5
    Uo2, acc2, *_ = hmc.trajectory(lev, U, p, 1.0, u_metropolis=np.nextafter(np.exp(-dH), 2))
    assert (not acc2) and np.array_equal(Uo2, U)


def test_step_size_schemes_match_the_paper():
    """Sec. 2 schemes A/B/C: the tables as printed (golden fixture), the stated averages over
    all links (A: 0.525, B and C: about 0.59), links with s = 0 stay fixed."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "step_size_schemes.json")))
    for name in "ABC":
        sp, tm = hmc.STEP_SCHEMES[name]
        spec = g[name]
        assert list(tm) == spec["time"]
        assert list(sp) == spec.get("spatial_read", spec.get("spatial"))
        prof = hmc.step_profile(name, spec["L0"])
        avg = prof.mean()
        if name == "A":
            assert abs(avg - 0.525) < 1e-15
            printed = np.array(spec["spatial_printed"])
            assert abs((3 * printed.mean() + np.mean(tm)) / 4 - 0.75) < 1e-15   # the misprint
        else:
            assert abs(avg - 0.59) < 0.015
    assert hmc.step_profile("B", 32).mean() == 19 / 32
    assert hmc.step_profile("C", 32).mean() == 37 / 64
    # active links of scheme B: 23 of 32 per period -> about 72 %
    assert np.mean(hmc.step_profile("B", 32) > 0) == 23 / 32


def test_step_profile_md_is_reversible_and_keeps_inactive_links():
    L, l0, k = (8, 2, 2, 2), 2, 0.15
    U = synth.gauge_field(L, 0.4, 80)
    p = synth.gaussian_momenta(L, 81)
    sc = np.tile(np.array([[0.0, 0.5, 1.0, 1.0], [0.5, 1.0, 0.25, 0.0]]), (4, 1))   # [L0, 4]
    lev = _levels(L, U, k, l0, n_outer=2, n_inner=2)
    U1, p1 = hmc.integrate(lev, U, p, 0.3, sc)
    U2, p2 = hmc.integrate(lev, U1, -p1, 0.3, sc)
    assert np.max(np.abs(U2 - U)) <= 1e-10
    frozen = sc == 0
    for x0, mu in zip(*np.nonzero(frozen)):
        assert np.array_equal(U1[x0, :, :, :, mu], U[x0, :, :, :, mu])


def test_time_shift_preserves_the_action():
    L, l0, k = (8, 2, 2, 2), 2, 0.15
    U = synth.gauge_field(L, 0.4, 82)
    Ut = hmc.time_shift(U, 3)
    assert abs(forces.gauge_action(Ut, 5.6) - forces.gauge_action(U, 5.6)) < 1e-10
    # det M is translation invariant: |M^{-1} phi|^2 for a translated phi agrees
    phi = synth.gaussian_spinor(L, 83)
    S1 = forces.pf_action(U, phi, k, None, W_inv=solvers.lu_solver(U, k, None))
    phit = np.roll(phi, -3, axis=0)
    phit[-3:] *= -1.0                       # the antiperiodic wrap moves with the field
    S2 = forces.pf_action(Ut, phit, k, None, W_inv=solvers.lu_solver(Ut, k, None))
    assert abs(S1 - S2) < 1e-9 * S1
