"""Pins of the oracle's geometric flux limiter and geometric outer boundary (CPU only).

The geometric piece of the limiter (eqs. a23-a26a) and the constant-luminosity outer boundary
(eq. a62af, with the neutrinosphere radius squared) are checked against what the paper fixes: the
relation psi^(1) = (1 + mu_nu) psi^(0) / 2 it imposes (eq. a26b), its limits (free streaming far
outside, half the occupation at the neutrinosphere, no effect inside it), F = min(F_intrp, F_geom),
the ghost-zone relation and its constant-luminosity origin, the budget identity and the Jacobian by
central differences.  Planted mistakes (a wrong sign of mu, a dropped square root, the unsquared
R_nu) are caught.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import oracle.transport as ot
import synth


def _system(I=14, N=6, limiter=ot.LIMITER_GEOM, outer_bc=ot.BC_GEOMETRIC, **kw):
    w = synth.make_custom(S=1, R=1, I=I, N=N).numpy()
    w.update(limiter=limiter, outer_bc=outer_bc)
    sysm = oracle.systems_from_workload(w)[0][0]
    return dataclasses.replace(sysm, **kw), w["psi_n"][0, 0]


def test_limb_factor_limits_eqs_a24_a25():
    """(1 + mu_nu)/2: 1/2 at the neutrinosphere (mu_nu = 0), 1 far outside (mu_nu -> 1, free streaming),
    and the closed form at R = 2 R_nu, where mu_nu = sqrt(3)/2; undefined (no limit) inside."""
    r_nu = np.array([1e6, 2e6, 5e6])
    np.testing.assert_allclose(ot.limb_factor(1e6 * (1 + 1e-12), r_nu[:1]), [0.5], atol=1e-5)
    np.testing.assert_allclose(ot.limb_factor(1e16, r_nu), 1.0, rtol=1e-12)
    np.testing.assert_allclose(ot.limb_factor(4e6, np.array([2e6])), [(1 + np.sqrt(3) / 2) / 2], rtol=1e-15)
    assert np.isnan(ot.limb_factor(3e6, np.array([5e6]))[0])


@pytest.mark.parametrize("limb", [0.5, 0.8, 0.999])
def test_free_streaming_regime_gives_the_geometric_relation_eq_a26b(limb):
    """Where the mean free path is huge, F_intrp -> 0 only like 1/lam, while F_geom imposes
    psi^(1) = limb psi^(0) exactly: H = limb m for an outward gradient (eq. a26b), independent of lam."""
    u = np.array([0.3, 1e-3, 2e-9])
    v = 0.25 * u
    for lam in (1e20, 1e30):
        H, du, dv, dl = ot.edge_flux(u, v, lam, 1e5, 1e-300, 2, limb)
        m = 0.5 * (u + v)
        np.testing.assert_allclose(H, limb * m, rtol=1e-14)
        np.testing.assert_allclose(du, 0.5 * limb, rtol=1e-14)
        np.testing.assert_allclose(dv, 0.5 * limb, rtol=1e-14)
        assert np.all(dl == 0.0)
    # an inward gradient reverses the sign
    H, *_ = ot.edge_flux(v, u, 1e30, 1e5, 1e-300, 2, limb)
    np.testing.assert_allclose(H, -limb * 0.5 * (u + v), rtol=1e-14)


def test_inside_the_neutrinosphere_the_limiter_is_f_intrp():
    """F_geom = 1 for R <= R_nu, so min(F_intrp, F_geom) = F_intrp (F_intrp <= 1): identical fluxes."""
    rng = np.random.default_rng(3)
    u, v = rng.uniform(0, 1, 50), rng.uniform(0, 1, 50)
    lam = 10 ** rng.uniform(2, 8, 50)
    a = ot.edge_flux(u, v, lam, 1e5, 1e-300, 1)
    b = ot.edge_flux(u, v, lam, 1e5, 1e-300, 2, np.full(50, np.nan))
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_limiter_is_the_minimum_eq_a26a():
    """|H| = (lam/3) F |dpsi/dR| with F = min(F_intrp, F_geom): never above the F_intrp flux nor above
    limb m, equal to one of them, and of the sign of -dpsi/dR."""
    rng = np.random.default_rng(5)
    n = 400
    u, v = rng.uniform(0, 1, n), rng.uniform(0, 1, n)
    lam = 10 ** rng.uniform(3, 9, n)
    limb = rng.uniform(0.5, 1.0, n)
    D = 1e5
    H2 = ot.edge_flux(u, v, lam, D, 1e-300, 2, limb)[0]
    H1 = ot.edge_flux(u, v, lam, D, 1e-300, 1)[0]
    Hg = limb * 0.5 * (u + v)
    assert np.all(np.abs(H2) <= np.abs(H1) * (1 + 1e-15))
    assert np.all(np.abs(H2) <= Hg * (1 + 1e-15))
    assert np.all(np.isclose(np.abs(H2), np.abs(H1), rtol=1e-14) | np.isclose(np.abs(H2), Hg, rtol=1e-14))
    assert np.all(np.sign(H2) == -np.sign(v - u))
    # both regimes occur in this sample
    assert np.any(np.abs(H2) < np.abs(H1) * (1 - 1e-3)) and np.any(np.abs(H2) < Hg * (1 - 1e-3))


def test_edge_flux_derivatives_match_central_differences():
    """dH/du, dH/dv, dH/dlam of the geometric limiter (both branches, away from the switch)."""
    rng = np.random.default_rng(8)
    n = 200
    u, v = rng.uniform(0.1, 1, n), rng.uniform(0.1, 1, n)
    lam = 10 ** rng.uniform(3, 9, n)
    limb = rng.uniform(0.5, 1.0, n)
    D = 1e5
    H, du, dv, dl = ot.edge_flux(u, v, lam, D, 1e-300, 2, limb)
    h = 1e-7

    def f(uu, vv, ll):
        return ot.edge_flux(uu, vv, ll, D, 1e-300, 2, limb)[0]

    ok = np.abs(np.abs(H) / (limb * 0.5 * (u + v)) - 1) > 1e-3     # away from the switch
    for d_an, fp, fm, scale in [(du, f(u + h, v, lam), f(u - h, v, lam), h),
                                (dv, f(u, v + h, lam), f(u, v - h, lam), h),
                                (dl, f(u, v, lam * (1 + h)), f(u, v, lam * (1 - h)), h * lam)]:
        fd = (fp - fm) / (2 * scale)
        np.testing.assert_allclose(d_an[ok], fd[ok], rtol=1e-5, atol=1e-12 * np.max(np.abs(fd)))


def test_ghost_zone_relation_eq_a62af():
    """(R_{I+1}^2 - R_nu^2/4) psi_{I+1} = (R_I^2 - R_nu^2/4) psi_I; pure inverse square without a
    neutrinosphere; and to first order in (R_nu/R)^2 the constant luminosity (1 + mu) R^2 psi / 2 the
    condition comes from (the mismatch is of order (R_nu/R)^4)."""
    sysm, _ = _system()
    Rc = oracle.geometry(sysm.r_edge)[0]
    R_g, ratio, D = ot.outer_ghost(sysm)
    R_I = Rc[-1]
    np.testing.assert_allclose(R_g - sysm.r_edge[-1], sysm.r_edge[-1] - R_I, rtol=1e-14)
    q = 0.25 * sysm.r_nu ** 2
    np.testing.assert_allclose((R_g ** 2 - q) * ratio, R_I ** 2 - q, rtol=1e-14)
    s0 = dataclasses.replace(sysm, r_nu=np.zeros_like(sysm.r_nu))
    np.testing.assert_allclose(ot.outer_ghost(s0)[1], (R_I / R_g) ** 2, rtol=1e-14)
    for scale in (2.0, 20.0):                       # a surface a few neutrinosphere radii out
        r_nu = R_I / scale * np.ones(3)
        sx = dataclasses.replace(sysm, r_nu=r_nu)
        rt = ot.outer_ghost(sx)[1]
        mu = lambda R: np.sqrt(1 - (r_nu / R) ** 2)
        lum = 0.5 * (1 + mu(R_g)) * R_g ** 2 * rt / (0.5 * (1 + mu(R_I)) * R_I ** 2)
        assert np.all(np.abs(lum - 1) < 0.2 * (1 / scale) ** 4 + 1e-15)


@pytest.mark.parametrize("limiter,outer_bc", [(2, 2), (2, 1), (1, 2)])
def test_budget_identity_and_luminosity_with_geometric_options(limiter, outer_bc):
    """n - n^n + B_N - Q_N - NES_N = sum V W G with the outer flux of the chosen boundary; L_N is that
    flux times c A; the free-streaming flux bounds the geometric boundary's from above."""
    sysm, psin = _system(limiter=limiter, outer_bc=outer_bc)
    res = oracle.newton(sysm, psin, max_iter=40, rtol=1e-13)
    psi = res.psi
    st = oracle.step_stats(sysm, psin, psi)
    G = oracle.residual(sysm, psin, psi)
    vf, _, _ = ot._weights(sysm)
    _, W = oracle.group_energies(sysm.e_edge)
    np.testing.assert_allclose(st["budget"], float(np.sum((1 / vf)[:, None] * W[None, :] * G)),
                               atol=1e-12 * st["n_tot"])
    assert st["lum_n"] == pytest.approx(oracle.luminosity(sysm, psi), rel=1e-14)
    if outer_bc == 2:
        assert 0 < st["lum_n"] < ot.C_LIGHT * sysm.r_edge[-1] ** 2 * np.sum(W * psi[-1])


@pytest.mark.parametrize("limiter,outer_bc", [(2, 2), (2, 1), (1, 2)])
def test_jacobian_with_geometric_options_matches_central_differences(limiter, outer_bc):
    """Block-tridiagonal Jacobian (both boundaries, both limiters) against central differences of G."""
    sysm, psin = _system(I=10, N=5, limiter=limiter, outer_bc=outer_bc)
    # optically thin outer zones so that the geometric branch is taken at some edges
    sysm = dataclasses.replace(sysm, kappa_a=sysm.kappa_a * 1e-3, eta=sysm.eta * 1e-3, kappa_s=sysm.kappa_s * 1e-3)
    # occupations of moderate range (so that central differences resolve every entry), falling outward
    psi = np.random.default_rng(4).uniform(0.3, 0.6, psin.shape) * np.linspace(1.0, 0.05, sysm.I)[:, None]
    J = oracle.dense_jacobian(sysm, psi)
    n = psi.size
    h = 1e-7
    Jfd = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = h * max(abs(psi.ravel()[j]), 1e-30)
        Jfd[:, j] = (oracle.residual(sysm, psin, psi + e.reshape(psi.shape)).ravel()
                     - oracle.residual(sysm, psin, psi - e.reshape(psi.shape)).ravel()) / (2 * e[j])
    np.testing.assert_allclose(J, Jfd, rtol=2e-5, atol=1e-8 * np.max(np.abs(J)))
    if limiter == 2:
        H1 = ot._edge_fluxes(dataclasses.replace(sysm, limiter=1), psi)[0]
        H2 = ot._edge_fluxes(sysm, psi)[0]
        assert np.any(np.abs(H2[1:-1]) < np.abs(H1[1:-1]) * (1 - 1e-6))     # the geometric branch is taken


def test_luminosity_seed_of_the_geometric_boundary_matches_central_differences():
    sysm, psin = _system()
    psi = np.random.default_rng(2).uniform(0.2, 0.5, psin.shape)      # every group resolved by the differences
    seed = oracle.luminosity_seed(sysm, psi.shape, psi)
    h = 1e-3          # the outer flux is homogeneous of degree one in psi_I, so a large step stays exact
    for k in range(sysm.N):
        d = np.zeros_like(psi)
        d[-1, k] = h * psi[-1, k]
        fd = (oracle.luminosity(sysm, psi + d) - oracle.luminosity(sysm, psi - d)) / (2 * d[-1, k])
        assert seed[-1, k] == pytest.approx(fd, rel=1e-6)
    assert np.all(seed[:-1] == 0)


def test_pins_catch_a_wrong_sign_of_mu(monkeypatch):
    real = ot.limb_factor
    monkeypatch.setattr(ot, "limb_factor", lambda R, r_nu: 1.0 - real(R, r_nu) + 0.5)
    with pytest.raises(AssertionError):
        test_limb_factor_limits_eqs_a24_a25()


def test_pins_catch_a_dropped_square_root(monkeypatch):
    def bad(R, r_nu):
        r_nu = np.asarray(r_nu, dtype=np.float64)
        out = np.full(r_nu.shape, np.nan)
        o = R > r_nu
        out[o] = 0.5 * (1.0 + (1.0 - (r_nu[o] / R) ** 2))
        return out
    monkeypatch.setattr(ot, "limb_factor", bad)
    with pytest.raises(AssertionError):
        test_limb_factor_limits_eqs_a24_a25()


def test_pins_catch_the_unsquared_neutrinosphere_radius(monkeypatch):
    real = ot.outer_ghost

    def bad(sysm):
        R_g, _, D = real(sysm)
        R_I = oracle.geometry(sysm.r_edge)[0][-1]
        q = 0.25 * sysm.r_nu
        return R_g, np.clip((R_I ** 2 - q) / (R_g ** 2 - q), 0, 1), D
    monkeypatch.setattr(ot, "outer_ghost", bad)
    with pytest.raises(AssertionError):
        test_ghost_zone_relation_eq_a62af()
