"""Pins of the Y_e-coupled oracle (electron-fraction equation, eq. a62a; coupled block system,
eqs. a62ac-a62ae; temperature update, eqs. a62b and a62d) against what the physics and the
mathematics fix: total lepton-number and energy conservation, the decoupled limit, central
differences of the Jacobian, and a dense solve of the assembled system."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from oracle import ye_coupled as yc


def _ray(zones=16, groups=6, outer_bc=1, terms=7, ray=3):
    w = synth.make(1, rays=[ray], zones=zones, groups=groups, species=4)
    ye = synth.ye_inputs(w, 1, rays=[ray])
    wn = w.numpy()
    wn["outer_bc"] = outer_bc
    wn["terms"] = terms
    cs = yc.coupled_systems(wn, ye.numpy())[0]
    u_n = yc.pack(wn["psi_n"][0, 0], wn["psi_n"][1, 0], cs.ye_n)
    return wn, ye.numpy(), cs, u_n


def _perturbed(cs, u_n, seed=5):
    rng = np.random.default_rng(seed)
    u = u_n.copy()
    N = cs.N
    u[:, :2 * N] *= 1.0 + 0.05 * rng.standard_normal(u[:, :2 * N].shape)
    u[:, 2 * N] += 0.01 * rng.standard_normal(cs.I)
    return u


def test_pack_and_species_rows_at_fixed_ye():
    """At Y_e = Y_e^n the species rows are exactly the single-species residuals."""
    wn, _, cs, u_n = _ray()
    u = _perturbed(cs, u_n)
    N = cs.N
    u[:, 2 * N] = cs.ye_n
    G = yc.residual(cs, u_n, u)
    np.testing.assert_array_equal(G[:, :N], oracle.residual(cs.nue, u_n[:, :N], u[:, :N]))
    np.testing.assert_array_equal(G[:, N:2 * N], oracle.residual(cs.nuebar, u_n[:, N:2 * N], u[:, N:2 * N]))


def test_species_rows_use_opacities_at_the_new_ye():
    """Without diffusion (whose mean free path stays at Y_e^n), the species rows at any Y_e are the
    single-species residuals with kappa_a and eta evaluated at that Y_e."""
    wn, _, cs, u_n = _ray(terms=synth.TERM_EMABS | synth.TERM_NES)
    u = _perturbed(cs, u_n, seed=11)
    N = cs.N
    dy = u[:, 2 * N] - cs.ye_n
    G = yc.residual(cs, u_n, u)
    for q, sy in enumerate((cs.nue, cs.nuebar)):
        at_y = dataclasses.replace(sy, kappa_a=sy.kappa_a + dy[:, None] * cs.dka_dye[q],
                                   eta=sy.eta + dy[:, None] * cs.deta_dye[q])
        ref = oracle.residual(at_y, u_n[:, q * N:(q + 1) * N], u[:, q * N:(q + 1) * N])
        np.testing.assert_allclose(G[:, q * N:(q + 1) * N], ref, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("terms", [7, 3])
def test_coupled_jacobian_matches_central_differences(terms):
    """The analytic (2N+1)-block Jacobian, Y_e row and column included, against central differences."""
    _, _, cs, u_n = _ray(zones=5, groups=4, terms=terms)
    # occupations away from zero and from each other: central differences must not cross the
    # limiter's floor or the |Delta psi| kink
    rng = np.random.default_rng(7)
    u = u_n.copy()
    N = cs.N
    u[:, :2 * N] = rng.uniform(0.05, 0.9, size=u[:, :2 * N].shape)
    u[:, 2 * N] += 0.01 * rng.standard_normal(cs.I)
    J = yc.dense_jacobian(cs, u)
    x = u.ravel()
    Jfd = np.zeros_like(J)
    for j in range(x.size):
        h = 1e-5 * max(abs(x[j]), 1e-3)
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        Gp = yc.residual(cs, u_n, xp.reshape(u.shape)).ravel()
        Gm = yc.residual(cs, u_n, xm.reshape(u.shape)).ravel()
        Jfd[:, j] = (Gp - Gm) / (2 * h)
    # a central difference at this step carries ~1e-10 of the row's largest entry in rounding
    # and truncation noise; the Y_e row and column reach 0.4-1 of their rows in the inner zones,
    # so a dropped or mis-signed coupling term exceeds this bound by orders of magnitude
    rowmax = np.abs(J).max(axis=1, keepdims=True)
    assert np.all(np.abs(J - Jfd) <= 1e-6 * np.abs(J) + 1e-9 * rowmax)


def test_coupled_block_thomas_matches_dense_solve():
    """Block-Thomas on the (2N+1)-block system equals a dense LAPACK solve of the assembled matrix."""
    _, _, cs, u_n = _ray(zones=12, groups=5)
    u = _perturbed(cs, u_n, seed=9)
    A, bm, bp = yc.jacobian_blocks(cs, u)
    rhs = np.random.default_rng(3).standard_normal(u.shape)
    x = oracle.block_thomas_solve(A, bm, bp, rhs)
    xd = np.linalg.solve(yc.dense_jacobian(cs, u), rhs.ravel()).reshape(u.shape)
    assert np.max(np.abs(x - xd)) < 1e-12 * np.max(np.abs(xd))


def test_total_lepton_number_is_conserved():
    """Zero-flux boundaries, diffusion + emission/absorption + NES: the converged step conserves
    electrons plus (nu_e - anti-nu_e) over the ray (eqs. a51-a55 with eq. a62a), while each of the
    two parts changes."""
    _, _, cs, u_n = _ray(zones=20, groups=6, outer_bc=0)
    res = yc.newton(cs, u_n, max_iter=30, rtol=1e-13)
    assert res.converged
    L0, L1 = yc.lepton_number(cs, u_n), yc.lepton_number(cs, res.psi)
    _, V, _, _ = oracle.geometry(cs.nue.r_edge)
    electrons = lambda u: float(np.sum(V * cs.rho * u[:, -1] / yc.M_B_G))      # noqa: E731
    moved = abs(electrons(res.psi) - electrons(u_n))
    assert moved > 1e3 * abs(L1 - L0)
    assert abs(L1 - L0) <= 1e-12 * abs(electrons(u_n))


def test_lepton_pin_catches_a_wrong_coupling_constant(monkeypatch):
    """A planted mistake (twice the Y_e rate) breaks lepton conservation."""
    _, _, cs, u_n = _ray(zones=12, groups=5, outer_bc=0)
    good = yc.zeta
    monkeypatch.setattr(yc, "zeta", lambda c: 2.0 * good(c))
    res = yc.newton(cs, u_n, max_iter=30, rtol=1e-13)
    _, V, _, _ = oracle.geometry(cs.nue.r_edge)
    electrons = float(np.sum(V * cs.rho * u_n[:, -1] / yc.M_B_G))
    assert abs(yc.lepton_number(cs, res.psi) - yc.lepton_number(cs, u_n)) > 1e-9 * electrons


def test_decoupled_limit_equals_single_species_steps():
    """Without Y_e dependence of the opacities the species rows decouple: psi equals the single-species
    oracle's steps, and Y_e is the explicit eq. a62a update at the converged psi."""
    _, _, cs, u_n = _ray(zones=16, groups=6)
    cs = dataclasses.replace(cs, dka_dye=np.zeros_like(cs.dka_dye), deta_dye=np.zeros_like(cs.deta_dye))
    # a fixed number of full updates on both sides (the residual-based stopping rule would stop the
    # joint and the separate iterations at different counts, which moves only cells far below the
    # residual's scale)
    res = yc.newton(cs, u_n, max_iter=6, rtol=0.0)
    N = cs.N
    pe = oracle.newton(cs.nue, u_n[:, :N], max_iter=6, rtol=0.0).psi
    pa = oracle.newton(cs.nuebar, u_n[:, N:2 * N], max_iter=6, rtol=0.0).psi
    # LAPACK factors the (2N+1) and the N blocks in different orders, so agreement is to rounding
    # at each zone's scale (its largest occupation), not relative to cells 30 decades below it
    for joint, alone in ((res.psi[:, :N], pe), (res.psi[:, N:2 * N], pa)):
        zone_scale = np.max(np.abs(alone), axis=1, keepdims=True)
        assert np.max(np.abs(joint - alone) / zone_scale) < 1e-13
    _, W = oracle.group_energies(cs.nue.e_edge)
    s = lambda sy, p: sy.eta * (1.0 - p) - sy.kappa_a * p      # noqa: E731
    y = cs.ye_n - cs.nue.c_dt * yc.zeta(cs) * ((s(cs.nue, pe) - s(cs.nuebar, pa)) @ W)
    np.testing.assert_allclose(res.psi[:, 2 * N], y, rtol=0, atol=1e-14)


def test_coupled_newton_converges_quadratically():
    _, _, cs, u_n = _ray(zones=24, groups=8, ray=11)
    res = yc.newton(cs, u_n, max_iter=30, rtol=1e-13)
    h = res.history
    assert res.converged and res.iters <= 5
    for a, b in zip(h[1:-1], h[2:]):
        if b > 1e-14:
            assert b < 10.0 * a * a / h[0] + 1e-15


def test_temperature_update_conserves_total_energy():
    """Zero-flux boundaries, all four species (statistical weights 1, 1, 2, 2): the matter energy
    change of eq. a62b balances the neutrino energy change, and eq. a62d turns it into dT."""
    wn, ye, cs, u_n = _ray(zones=16, groups=6, outer_bc=0)
    res = yc.newton(cs, u_n, max_iter=30, rtol=1e-14)
    sy = oracle.systems_from_workload(wn)
    others = [sy[2][0], sy[3][0]]
    p_others = [oracle.newton(s, wn["psi_n"][q, 0], max_iter=30, rtol=1e-14).psi for q, s in zip((2, 3), others)]
    weights = (1.0, 1.0, 2.0, 2.0)
    de, T1 = yc.temperature_update(cs, others, res.psi, p_others, weights, wn["temp"][0], ye["de_dT"][0],
                                   ye["de_dye"][0])
    _, V, _, _ = oracle.geometry(cs.nue.r_edge)
    matter = float(np.sum(V * cs.rho / yc.M_B_G * de))
    N = cs.N
    new = [res.psi[:, :N], res.psi[:, N:2 * N]] + p_others
    old = [u_n[:, :N], u_n[:, N:2 * N], wn["psi_n"][2, 0], wn["psi_n"][3, 0]]
    systems = [cs.nue, cs.nuebar] + others
    nu = sum(w * (yc.neutrino_energy(s, a) - yc.neutrino_energy(s, b)) for w, s, a, b in zip(weights, systems, new, old))
    assert abs(matter) > 0
    assert abs(matter + nu) <= 1e-10 * abs(matter)
    dy = res.psi[:, 2 * N] - cs.ye_n
    # T^{n+1} - T^n cancels to ~1e-12 of T in the outer zones: compare at the scale of T de/dT
    atol = 1e-14 * float(np.max(wn["temp"][0] * ye["de_dT"][0]))
    np.testing.assert_allclose((T1 - wn["temp"][0]) * ye["de_dT"][0] + dy * ye["de_dye"][0], de, rtol=1e-12, atol=atol)


# ------------------------------------------------------------------ the lapse (eq. a58 with a != 1)

def _lapsed(cs, R0=5.0e5):
    """The coupled system with the lapse a(R) = sqrt(1 - R0/R) on both species (0.71 at 10 km)."""
    re = cs.nue.r_edge
    rc = 0.5 * (re[1:] + re[:-1])
    a, ae = np.sqrt(1.0 - R0 / rc), np.sqrt(1.0 - R0 / re)
    return dataclasses.replace(cs, nue=dataclasses.replace(cs.nue, lapse=a, lapse_edge=ae),
                               nuebar=dataclasses.replace(cs.nuebar, lapse=a, lapse_edge=ae))


def test_total_lepton_number_is_conserved_with_a_lapse():
    """With a lapse the neutrinos of zone i number (V_i/a_i^3) sum_k W_k psi; zero-flux boundaries, all
    terms: the converged coupled step conserves electrons plus that (nu_e - anti-nu_e) number."""
    _, _, cs, u_n = _ray(zones=20, groups=6, outer_bc=0)
    cs = _lapsed(cs)
    assert np.ptp(cs.nue.lapse) > 0.2
    res = yc.newton(cs, u_n, max_iter=30, rtol=1e-13)
    assert res.converged
    L0, L1 = yc.lepton_number(cs, u_n), yc.lepton_number(cs, res.psi)
    _, V, _, _ = oracle.geometry(cs.nue.r_edge)
    electrons = lambda u: float(np.sum(V * cs.rho * u[:, -1] / yc.M_B_G))      # noqa: E731
    assert abs(electrons(res.psi) - electrons(u_n)) > 1e3 * abs(L1 - L0)
    assert abs(L1 - L0) <= 1e-12 * abs(electrons(u_n))


def test_lapse_lepton_pin_catches_a_missing_phase_space_factor(monkeypatch):
    """A planted Y_e rate without the lapse's a^-2 (the a = 1 form) breaks the lapsed lepton sum."""
    _, _, cs, u_n = _ray(zones=12, groups=5, outer_bc=0)
    cs = _lapsed(cs)
    good = yc.zeta
    monkeypatch.setattr(yc, "zeta", lambda c: good(c) * yc.lapse(c) ** 2)
    res = yc.newton(cs, u_n, max_iter=30, rtol=1e-13)
    _, V, _, _ = oracle.geometry(cs.nue.r_edge)
    electrons = float(np.sum(V * cs.rho * u_n[:, -1] / yc.M_B_G))
    monkeypatch.setattr(yc, "zeta", good)
    assert abs(yc.lepton_number(cs, res.psi) - yc.lepton_number(cs, u_n)) > 1e-9 * electrons


@pytest.mark.parametrize("terms", [7, 3])
def test_coupled_jacobian_with_lapse_matches_central_differences(terms):
    _, _, cs, u_n = _ray(zones=5, groups=4, terms=terms)
    cs = _lapsed(cs)
    rng = np.random.default_rng(8)
    u = u_n.copy()
    N = cs.N
    u[:, :2 * N] = rng.uniform(0.05, 0.9, size=u[:, :2 * N].shape)
    u[:, 2 * N] += 0.01 * rng.standard_normal(cs.I)
    J = yc.dense_jacobian(cs, u)
    x = u.ravel()
    Jfd = np.zeros_like(J)
    for j in range(x.size):
        h = 1e-5 * max(abs(x[j]), 1e-3)
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        Jfd[:, j] = (yc.residual(cs, u_n, xp.reshape(u.shape)).ravel()
                     - yc.residual(cs, u_n, xm.reshape(u.shape)).ravel()) / (2 * h)
    rowmax = np.abs(J).max(axis=1, keepdims=True)
    assert np.all(np.abs(J - Jfd) <= 1e-6 * np.abs(J) + 1e-9 * rowmax)
