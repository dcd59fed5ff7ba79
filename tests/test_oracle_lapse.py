"""Pins of the oracle's lapse terms (eq. a58 with a != 1; eqs. a8a, t1-t7), CPU only.

* the conservative form of eq. a58 (multiplied by c V_i dt / a_i^2): with zero-flux boundaries the
  number sum_i V_i / a_i^3 sum_k W_k psi is unchanged at every Newton iterate;
* the static gravitational-redshift test: in a source-free, transparent medium around an emitting core
  the steady state carries a constant flux at infinity A H / a^2 in every group (eq. t3), so the local
  luminosity goes as a^-2 (eq. t4) and the mean local energy of the emerging neutrinos as a^-1
  (eq. t7, here in its flux-weighted form, which the discrete steady state satisfies exactly);
* Fermi-Dirac at the local energies E / a is a fixed point of emission/absorption and NES;
* the analytic Jacobian equals central differences of the residual.
"""
import numpy as np
import pytest

from oracle import transport as tr

R0 = 5.0e5      # cm: a(R) = sqrt(1 - R0 / R), a(10 km) = 0.71 (the paper uses 2.04 km; a larger R0 gives a
                # larger redshift on the same grid)


def lapse_of(r_edge):
    rc = 0.5 * (r_edge[1:] + r_edge[:-1])
    return np.sqrt(1.0 - R0 / rc), np.sqrt(1.0 - R0 / r_edge)


def make_system(I=24, N=10, terms=7, seed=0, c_dt=3e4, outer_bc=1, transparent_from=None, r_span=100.0):
    r = np.random.default_rng(seed)
    r_edge = 1e6 * r_span ** (np.arange(I + 1) / I)
    e_edge = 2.0 * 150.0 ** (np.arange(N + 1) / N)
    eps, _ = tr.group_energies(e_edge)
    T = 8.0 * (r_edge[:-1] / 1e6) ** -0.3
    a, ae = lapse_of(r_edge)
    loc = eps[None, :] / a[:, None]                             # local energies E / a
    ka = 1e-5 * (loc / 10.0) ** 2 * (1.0 + 0.1 * r.standard_normal((I, N)))
    mu = 2.0 * T
    eta = ka * np.exp(-(loc - mu[:, None]) / T[:, None])
    ks = 2.0 * ka
    if transparent_from is not None:
        ka[transparent_from:] = 0.0
        eta[transparent_from:] = 0.0
        ks[transparent_from:] = 1e-14
    G = np.exp(-(np.log(eps)[:, None] - np.log(eps)[None, :]) ** 2 / (2 * 0.3 ** 2))
    return tr.System(r_edge=r_edge, e_edge=e_edge, temp=T, kappa_a=ka, eta=eta, kappa_s=ks,
                     nes_amp=1e-6 * np.ones(I), nes_g=G, c_dt=c_dt, outer_bc=outer_bc, terms=terms,
                     lapse=a, lapse_edge=ae)


def test_number_at_infinity_is_conserved_with_zero_flux_boundaries():
    sys = make_system(terms=tr.TERM_DIFFUSION, outer_bc=0, c_dt=3e8, r_span=4.0)
    a = sys.lapse
    _, V, _, _ = tr.geometry(sys.r_edge)
    _, W = tr.group_energies(sys.e_edge)
    r = np.random.default_rng(3)
    psi_n = r.uniform(0.0, 0.8, (sys.I, sys.N))
    weight = (V / a ** 3)[:, None] * W[None, :]
    n0 = np.sum(weight * psi_n)
    for iters in (1, 2, 6):
        psi = tr.newton(sys, psi_n, max_iter=iters, rtol=0.0).psi
        assert np.max(np.abs(psi - psi_n)) > 0.05                 # transport moves the neutrinos
        assert abs(np.sum(weight * psi) - n0) <= 1e-13 * n0
    # the same sum without the a^3 is not conserved: the pin sees the lapse factor
    plain = V[:, None] * W[None, :]
    assert abs(np.sum(plain * psi) - np.sum(plain * psi_n)) > 1e-4 * np.sum(plain * psi_n)


def steady_state():
    """An emitting core (zones 0-3) inside a transparent medium, advanced to its steady state with a
    time step far beyond every transport time (backward Euler then solves the stationary equations)."""
    sys = make_system(I=40, N=8, terms=tr.TERM_DIFFUSION | tr.TERM_EMABS, transparent_from=4, c_dt=1e22)
    psi0 = np.zeros((sys.I, sys.N))
    res = tr.newton(sys, psi0, max_iter=80, rtol=1e-15)
    return sys, res.psi


def test_static_redshift_luminosity_and_mean_energy():
    sys, psi = steady_state()
    H = tr._edge_fluxes(sys, psi)[0]                 # [I+1][N]
    _, _, A, _ = tr.geometry(sys.r_edge)
    ae = sys.lapse_edge
    eps, W = tr.group_energies(sys.e_edge)
    edges = np.arange(6, sys.I)                      # interior edges of the transparent region
    phi = A[edges, None] * H[edges] / ae[edges, None] ** 2          # flux at infinity per group (eq. t3)
    assert np.all(phi > 0.0)
    assert np.allclose(phi, phi[0][None, :], rtol=1e-9, atol=0)
    # local luminosity: sum over groups of local energy x local phase space x flux, times the area
    lum = A[edges] * np.sum((W / ae[edges, None] ** 3) * (eps / ae[edges, None]) * H[edges], axis=1)
    assert np.allclose(lum * ae[edges] ** 2, (lum * ae[edges] ** 2)[0], rtol=1e-9, atol=0)     # eq. t4
    mean_e = np.sum(W * (eps / ae[edges, None]) * H[edges], axis=1) / np.sum(W * H[edges], axis=1)
    assert np.allclose(mean_e * ae[edges], (mean_e * ae[edges])[0], rtol=1e-9, atol=0)          # eq. t7
    # the redshift is visible: L changes by (a_out / a_in)^-2 across the region
    assert lum[-1] / lum[0] == pytest.approx((ae[edges[0]] / ae[edges[-1]]) ** 2, rel=1e-9)
    assert (ae[edges[0]] / ae[edges[-1]]) ** 2 < 0.8


def test_redshift_pin_catches_a_missing_edge_lapse(monkeypatch):
    """Edge areas without the 1/a^2 of eq. a58: the steady flux A H is then constant instead, and the
    luminosity no longer goes as a^-2."""
    real = tr._weights

    def no_edge_lapse(sys):
        vf, Aw, a = real(sys)
        return vf, Aw * sys.lapse_edge ** 2, a
    monkeypatch.setattr(tr, "_weights", no_edge_lapse)
    sys, psi = steady_state()
    H = tr._edge_fluxes(sys, psi)[0]
    _, _, A, _ = tr.geometry(sys.r_edge)
    edges = np.arange(6, sys.I)
    phi = A[edges, None] * H[edges] / sys.lapse_edge[edges, None] ** 2
    assert not np.allclose(phi, phi[0][None, :], rtol=1e-3, atol=0)


def test_fermi_dirac_at_local_energies_is_a_fixed_point():
    sys = make_system(terms=tr.TERM_EMABS | tr.TERM_NES)
    eps, _ = tr.group_energies(sys.e_edge)
    loc = eps[None, :] / sys.lapse[:, None]
    f = 1.0 / (np.exp((loc - 2.0 * sys.temp[:, None]) / sys.temp[:, None]) + 1.0)
    G = tr.residual(sys, f, f)
    scale = sys.c_dt * sys.lapse[:, None] * (sys.kappa_a * f + sys.eta * (1.0 - f))
    assert np.max(np.abs(G) / scale) < 1e-12
    # at the energies at infinity instead (no lapse in the NES kernels) it is not
    sys.lapse, sys.lapse_edge = None, None
    f_inf = 1.0 / (np.exp((eps[None, :] - 2.0 * sys.temp[:, None]) / sys.temp[:, None]) + 1.0)
    assert np.max(np.abs(tr.residual(sys, f_inf, f_inf))) > 1e-3 * np.max(np.abs(scale))


@pytest.mark.parametrize("terms", [7, tr.TERM_DIFFUSION, tr.TERM_NES | tr.TERM_EMABS])
def test_jacobian_with_lapse_matches_central_differences(terms):
    sys = make_system(I=6, N=5, terms=terms, seed=4)
    r = np.random.default_rng(5)
    psi = r.uniform(0.05, 0.9, (sys.I, sys.N))
    J = tr.dense_jacobian(sys, psi)
    h = 1e-6
    Jfd = np.zeros_like(J)
    for m in range(psi.size):
        d = np.zeros(psi.size)
        d[m] = h * max(abs(psi.ravel()[m]), 1e-3)
        gp = tr.residual(sys, psi, psi + d.reshape(psi.shape)).ravel()
        gm = tr.residual(sys, psi, psi - d.reshape(psi.shape)).ravel()
        Jfd[:, m] = (gp - gm) / (2 * d[m])
    assert np.allclose(J, Jfd, rtol=1e-6, atol=1e-8 * np.abs(J).max())


def _lapse_gradient_mismatch(sys, psin, names=("kappa_a", "eta", "kappa_s", "nes_amp", "psi_n"), seed=9):
    """Largest |adjoint - central difference| of dL/dtheta along random relative directions, relative to
    the adjoint value (plus a floor of 1e-9 L)."""
    import dataclasses

    def solve(sy, pn):
        return tr.newton(sy, pn, max_iter=40, rtol=1e-15).psi

    psi = solve(sys, psin)
    mu = tr.adjoint(sys, psi, tr.luminosity_seed(sys, psi.shape))
    g = tr.param_vjp(sys, psi, mu)
    L0 = tr.luminosity(sys, psi)
    r = np.random.default_rng(seed)
    h = 1e-6
    worst = 0.0
    for name in names:
        for _ in range(2):
            base = psin if name == "psi_n" else getattr(sys, name)
            d = r.standard_normal(base.shape) * base

            def L(sign):
                if name == "psi_n":
                    return tr.luminosity(sys, solve(sys, psin + sign * h * d))
                sy = dataclasses.replace(sys, **{name: base + sign * h * d})
                return tr.luminosity(sy, solve(sy, psin))

            fd = (L(+1) - L(-1)) / (2 * h)
            an = float(np.sum(g[name] * d))
            worst = max(worst, abs(fd - an) / (abs(an) + 1e-9 * abs(L0) / 1e-5))
    return worst


def _lapse_gradient_case():
    sys = make_system(I=10, N=6, seed=6, c_dt=3e4, r_span=20.0)
    import dataclasses
    sys = dataclasses.replace(sys, kappa_a=sys.kappa_a * 3e3, eta=sys.eta * 3e3, kappa_s=sys.kappa_s * 3e3,
                              nes_amp=sys.nes_amp * 3e5)
    r = np.random.default_rng(7)
    psin = r.uniform(0.05, 0.6, (sys.I, sys.N))
    return sys, psin


def test_luminosity_gradient_with_lapse_matches_central_differences():
    """dL/dtheta of the lapsed luminosity L = c A_{I+1/2}/a_{I+1/2}^2 sum_k W_k H (eq. a62 with eq. a58's
    lapse) from the adjoint, J^T mu = dL/dpsi and g = -mu^T dG/dtheta, equals central differences of
    L(psi^{n+1}(theta)) for kappa_a, eta, kappa_s, the NES amplitude and psi^n."""
    sys, psin = _lapse_gradient_case()
    assert np.ptp(sys.lapse) > 0.1                               # the lapse varies across the grid
    assert _lapse_gradient_mismatch(sys, psin) < 1e-5


def test_lapse_gradient_pin_catches_a_missing_source_lapse(monkeypatch):
    """Plant the parameter VJP without the lapse on the emission/absorption and NES terms (the a = 1
    form): the central-difference pin must fail."""
    orig = tr._weights

    def no_source_lapse(sys):
        vf, Aw, a = orig(sys)
        return vf, Aw, np.ones_like(a)

    sys, psin = _lapse_gradient_case()
    real_vjp = tr.param_vjp

    def planted(sy, psi, mu):
        monkeypatch.setattr(tr, "_weights", no_source_lapse)
        try:
            return real_vjp(sy, psi, mu)
        finally:
            monkeypatch.setattr(tr, "_weights", orig)

    monkeypatch.setattr(tr, "param_vjp", planted)
    assert _lapse_gradient_mismatch(sys, psin, names=("kappa_a", "nes_amp")) > 1e-3
