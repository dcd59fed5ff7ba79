"""Pins of the oracle's conservation sums, luminosity and stopping level (CPU).

* n_tot and e_tot (eqs. a60-a62 with the phase-space weights of eq. a01b) against the number and
  energy integrals of a Fermi-Dirac spectrum, computed by adaptive quadrature;
* the absolute scale of the number luminosity L_N (the number through the outer surface, eq. a62)
  against the net emission rate of the source (eq. a54) in a steady state, where the two must agree;
* the rounding level of the stopping rule against the residual of the exact discrete solution:
  the exact solution is found in extended precision (np.longdouble residuals, iterative refinement),
  rounded to float64, and its float64 residual must lie well below the level (the target can be
  reached), while every state the rule accepts must equal that solution to the float64 bar (the rule
  does not stop early).  The same for the Y_e-coupled system.
"""
import dataclasses

import numpy as np
import pytest
import scipy.integrate

import synth
from oracle import transport as tr
from oracle import ye_coupled as yc


def fd(E, T, mu):
    x = (E - mu) / T
    return np.where(x > 0, np.exp(-np.abs(x)) / (1.0 + np.exp(-np.abs(x))), 1.0 / (1.0 + np.exp(-np.abs(x))))


def one_zone_system(N, e_lo=2.0, e_hi=300.0, I=3, **kw):
    e = np.geomspace(e_lo, e_hi, N + 1)
    r = np.array([1.0e6 * 1.3 ** j for j in range(I + 1)])
    z = np.zeros((I, N))
    base = dict(r_edge=r, e_edge=e, temp=np.full(I, 5.0), kappa_a=z + 1e-4, eta=z + 1e-4, kappa_s=z + 1e-4,
                nes_amp=np.zeros(I), nes_g=np.eye(N), c_dt=3e4, terms=tr.TERM_EMABS)
    base.update(kw)
    return tr.System(**base)


@pytest.mark.parametrize("T,mu", [(4.0, 8.0), (10.0, -5.0), (25.0, 50.0)])
def test_number_and_energy_sums_are_fermi_dirac_integrals(T, mu):
    """With psi = f_FD(eps_k) in every zone of a fine grid, sum_k W_k psi and sum_k W_k eps_k psi tend to
    the integrals of E^2 f and E^3 f over the grid's range (W_k = eps_k^2 d eps_k, eq. a01b); the
    volumes sum to the shell volume (R_out^3 - R_in^3)/3."""
    N = 4000
    sysm = one_zone_system(N)
    eps, _ = tr.group_energies(sysm.e_edge)
    psi = np.tile(fd(eps, T, mu), (sysm.I, 1))
    st = tr.step_stats(sysm, psi, psi)
    vol = (sysm.r_edge[-1] ** 3 - sysm.r_edge[0] ** 3) / 3.0
    lo, hi = sysm.e_edge[0], sysm.e_edge[-1]
    n_ref = scipy.integrate.quad(lambda E: E * E * fd(E, T, mu), lo, hi, epsabs=0, epsrel=1e-12, limit=400)[0]
    e_ref = scipy.integrate.quad(lambda E: E ** 3 * fd(E, T, mu), lo, hi, epsabs=0, epsrel=1e-12, limit=400)[0]
    assert abs(st["n_tot"] / (vol * n_ref) - 1.0) < 1e-5
    assert abs(st["e_tot"] / (vol * e_ref) - 1.0) < 1e-5


def test_energy_sum_pin_catches_a_wrong_weight(monkeypatch):
    """A planted mistake in the energy weight (eps_k^2 in place of eps_k) fails the pin above."""
    real = tr.group_energies
    monkeypatch.setattr(tr, "group_energies", lambda e: (real(e)[0] ** 2, real(e)[1]))
    with pytest.raises(AssertionError):
        test_number_and_energy_sums_are_fermi_dirac_integrals(4.0, 8.0)


def _steady_state_single_zone(N):
    """One zone, zero inner flux, free-streaming outer boundary, emission/absorption only: the steady state
    psi* of G(psi; psi^n = psi) = 0, c dt [A H / V - eta (1 - psi) + kappa_a psi] = 0 with H = psi at the
    outer edge, is psi* = eta / (A/V + eta + kappa_a) per group."""
    rng = np.random.default_rng(5)
    e = np.geomspace(3.0, 80.0, N + 1)
    r = np.array([2.0e6, 3.5e6])
    ka = rng.uniform(1e-7, 1e-6, (1, N))
    et = rng.uniform(1e-7, 1e-6, (1, N))
    sysm = tr.System(r_edge=r, e_edge=e, temp=np.array([5.0]), kappa_a=ka, eta=et, kappa_s=ka.copy(),
                     nes_amp=np.zeros(1), nes_g=np.eye(N), c_dt=3e4,
                     terms=tr.TERM_DIFFUSION | tr.TERM_EMABS, outer_bc=1)
    _, V, A, _ = tr.geometry(r)
    return sysm, et / (A[1] / V[0] + et + ka), V[0]


def test_luminosity_equals_net_emission_rate_in_a_steady_state():
    """In a steady state the number leaving through the outer surface per unit time equals the number
    created per unit time by the source: emission minus absorption, c (eta (1 - psi) - kappa_a psi) per
    state and unit volume (eq. a54; eta and kappa_a are inverse mean free paths), summed with the volume
    V and the phase-space weights W_k, with the same constant factors dropped as in L_N."""
    sysm, psi, V = _steady_state_single_zone(6)
    G = tr.residual(sysm, psi, psi)
    assert np.max(np.abs(G)) < 1e-15                     # it is the steady state
    _, W = tr.group_energies(sysm.e_edge)
    rate = tr.C_LIGHT * V * np.sum(W * (sysm.eta[0] * (1.0 - psi[0]) - sysm.kappa_a[0] * psi[0]))
    st = tr.step_stats(sysm, psi, psi)
    assert abs(st["lum_n"] / rate - 1.0) < 1e-13
    assert abs(tr.luminosity(sysm, psi) / rate - 1.0) < 1e-13
    # per time step: the boundary term of the budget is L_N dt, with c dt the step's light travel length
    assert abs(st["b_n"] / (rate * sysm.c_dt / tr.C_LIGHT) - 1.0) < 1e-13


def test_luminosity_pin_catches_a_dropped_speed_of_light(monkeypatch):
    monkeypatch.setattr(tr, "C_LIGHT", 1.0)
    sysm, psi, V = _steady_state_single_zone(6)
    _, W = tr.group_energies(sysm.e_edge)
    rate = 2.99792458e10 * V * np.sum(W * (sysm.eta[0] * (1.0 - psi[0]) - sysm.kappa_a[0] * psi[0]))
    assert abs(tr.luminosity(sysm, psi) / rate - 1.0) > 0.5


# ---------------------------------------------------------------- the rounding level of the stopping rule

def _ld(x):
    if isinstance(x, np.ndarray):
        return x.astype(np.longdouble)
    if dataclasses.is_dataclass(x):
        return dataclasses.replace(x, **{f.name: _ld(getattr(x, f.name)) for f in dataclasses.fields(x)})
    return x


def _exact_solution(res_fn, jac_solve, u_n, u0, sweeps=6):
    """The discrete solution in extended precision: long-double residuals, float64 Newton corrections
    (iterative refinement), from a float64 starting point."""
    u = u0.astype(np.longdouble)
    for _ in range(sweeps):
        u = u + jac_solve(u.astype(np.float64), -res_fn(u))
    return u


def rel_err(a, ref, tau=1e-30):
    return float(np.max(np.abs(a - ref) / np.maximum(np.abs(ref), tau)))


@pytest.mark.parametrize("shape,lapse", [(dict(S=2, R=2, I=40, N=12), False), (dict(S=1, R=2, I=24, N=20), True)])
def test_rounding_level_brackets_the_exact_solution(shape, lapse):
    """(a) The float64 residual of the exact solution rounded to float64 is at least 32x below the level,
    so the target max(rtol res0, level) can be reached; (b) every state the oracle's Newton iteration
    accepts under the rule equals the exact solution to 1e-13 (tau-relative), so the rule does not stop
    before psi is resolved to the float64 bar."""
    w = synth.make_custom(**shape).numpy()
    syss = tr.systems_from_workload(w)
    for s in range(w["S"]):
        for r in range(w["R"]):
            sysm = syss[s][r]
            if lapse:
                a_e = np.sqrt(1.0 - 2.0e5 / sysm.r_edge)
                rc = 0.5 * (sysm.r_edge[1:] + sysm.r_edge[:-1])
                sysm = dataclasses.replace(sysm, lapse=np.sqrt(1.0 - 2.0e5 / rc), lapse_edge=a_e)
            pn = w["psi_n"][s, r]
            res = tr.newton(sysm, pn, max_iter=40, rtol=1e-12)
            assert res.converged
            sl, pnl = _ld(sysm), pn.astype(np.longdouble)

            def jsolve(u, rhs):
                A, bm, bp = tr.jacobian_blocks(sysm, u)
                return tr.block_thomas_solve(A, bm, bp, rhs.astype(np.float64))

            exact = _exact_solution(lambda u: tr.residual(sl, pnl, u), jsolve, pn, res.psi)
            assert np.max(np.abs(tr.residual(sl, pnl, exact))) < 1e-17
            rounded = exact.astype(np.float64)
            lev = tr.residual_rounding_level(sysm, pn, rounded)
            assert np.max(np.abs(tr.residual(sysm, pn, rounded))) <= lev / 32.0
            assert rel_err(res.psi, rounded) < 1e-13


def test_coupled_rounding_level_brackets_the_exact_solution():
    """The same two properties for the Y_e-coupled system (psi of both species and Y_e)."""
    w = synth.make_custom(S=2, R=2, I=20, N=8)
    y = synth.ye_inputs(w, 0, R_full=2)
    wn, yn = w.numpy(), y.numpy()
    for r, cs in enumerate(yc.coupled_systems(wn, yn)):
        u_n = yc.pack(wn["psi_n"][0, r], wn["psi_n"][1, r], cs.ye_n)
        res = yc.newton(cs, u_n, max_iter=40, rtol=1e-12)
        assert res.converged
        csl, unl = _ld(cs), u_n.astype(np.longdouble)

        def jsolve(u, rhs):
            A, bm, bp = yc.jacobian_blocks(cs, u)
            return yc.block_thomas_solve(A, bm, bp, rhs.astype(np.float64))

        exact = _exact_solution(lambda u: yc.residual(csl, unl, u), jsolve, u_n, res.psi)
        rounded = exact.astype(np.float64)
        lev = yc.rounding_level(cs, u_n, rounded)
        assert np.max(np.abs(yc.residual(cs, u_n, rounded))) <= lev / 32.0
        N = cs.N
        # psi relative to the largest occupation of its zone and species, Y_e relative to itself
        for q in range(2):
            got, ref = res.psi[:, q * N:(q + 1) * N], rounded[:, q * N:(q + 1) * N]
            scale = np.maximum(np.max(np.abs(ref), axis=-1, keepdims=True), 1e-30)
            assert float(np.max(np.abs(got - ref) / scale)) < 1e-13
        assert rel_err(res.psi[:, 2 * N], rounded[:, 2 * N]) < 1e-13


def test_rounding_level_pin_catches_a_loose_level(monkeypatch):
    """A level 1e7 times larger (about 1e-9 of the largest term) lets the iteration stop an update early,
    and pin (b) fails."""
    real = tr.residual_rounding_level
    monkeypatch.setattr(tr, "residual_rounding_level", lambda *a: 1e7 * real(*a))
    with pytest.raises(AssertionError):
        test_rounding_level_brackets_the_exact_solution(dict(S=1, R=2, I=40, N=12), False)
