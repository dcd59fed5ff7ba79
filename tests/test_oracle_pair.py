"""Pins of the oracle's neutrino-antineutrino pair processes (eqs. d11-d22) in the coupled nu_e /
anti-nu_e / Y_e step (CPU only).

The angular factors are checked against direct numerical integration of the ratios that define them
(eqs. d16, d19) and against their printed limits (eq. d20, eq. d22); the pair sources against the
symmetry that makes pairs conserve nu - anti-nu number, against Fermi-Dirac equilibrium with opposite
chemical potentials (detailed balance of eq. d12) and the sign of the departure from it; the coupled
step against total lepton-number and energy conservation and its Jacobian against central
differences.  Planted mistakes (a wrong sign in the creation factor, the ray-wise transposed chi, a
weight of the wrong species) are caught.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth
from oracle import ye_coupled as yc


def _ray(zones=16, groups=6, outer_bc=1, terms=7, ray=3):
    w = synth.make(1, rays=[ray], zones=zones, groups=groups, species=4)
    ye = synth.ye_inputs(w, 1, rays=[ray], pairs=True)
    wn = w.numpy()
    wn["outer_bc"] = outer_bc
    wn["terms"] = terms
    cs = yc.coupled_systems(wn, ye.numpy())[0]
    u_n = yc.pack(wn["psi_n"][0, 0], wn["psi_n"][1, 0], cs.ye_n)
    return wn, ye.numpy(), cs, u_n


def _sphere_pairs(n=48):
    """Gauss-Legendre nodes in mu and a uniform grid in the azimuth difference: quadrature of
    (4 pi)^-2 int dOmega int dOmega' F(mu, mu', n.n')."""
    x, wx = np.polynomial.legendre.leggauss(n)
    ph = (np.arange(2 * n) + 0.5) * np.pi / n
    return x, wx, ph


def _angular_average(fnu, fnubar, lo=(-1.0, -1.0)):
    """(4 pi)^-2 int int f(mu) fbar(mu') (1 - n.n')^2 over mu in [lo0, 1], mu' in [lo1, 1]."""
    x, wx, ph = _sphere_pairs()
    m1 = lo[0] + (x + 1) * (1 - lo[0]) / 2
    w1 = wx * (1 - lo[0]) / 2
    m2 = lo[1] + (x + 1) * (1 - lo[1]) / 2
    w2 = wx * (1 - lo[1]) / 2
    a, b, p = np.meshgrid(m1, m2, ph, indexing="ij")
    wa, wb = np.meshgrid(w1, w2, indexing="ij")
    ndot = a * b + np.sqrt(1 - a * a) * np.sqrt(1 - b * b) * np.cos(p)
    integrand = fnu(a) * fnubar(b) * (1 - ndot) ** 2
    # azimuth of one direction integrates to 2 pi, the difference is averaged over [0, 2 pi)
    return float(np.sum(wa[:, :, None] * wb[:, :, None] * integrand) * (2 * np.pi) * (2 * np.pi / ph.size)
                 / (4 * np.pi) ** 2)


@pytest.mark.parametrize("p0,p1,q0,q1", [(0.3, 0.05, 0.2, 0.06), (0.8, 0.2, 0.1, -0.01), (1e-3, 3e-4, 0.5, 0.1)])
def test_chi1_is_the_ratio_of_eq_d16(p0, p1, q0, q1):
    num = _angular_average(lambda m: p0 + 3 * m * p1, lambda m: q0 + 3 * m * q1)
    den = _angular_average(lambda m: p0 + 0 * m, lambda m: q0 + 0 * m)
    assert yc.chi1(p1 / p0, q1 / q0) == pytest.approx(num / den, rel=1e-10)


@pytest.mark.parametrize("mu,mub", [(0.3, 0.6), (-0.5, 0.9), (0.95, 0.99), (0.0, -0.2)])
def test_chi2_is_the_ratio_of_eq_d19(mu, mub):
    """Distributions constant inside the cones mu >= mu_i (mu' >= mu_i'), normalised to the same zeroth
    moments (eqs. d17, d18), against the isotropic ones."""
    num = _angular_average(lambda m: 2 / (1 - mu) + 0 * m, lambda m: 2 / (1 - mub) + 0 * m, lo=(mu, mub))
    den = _angular_average(lambda m: 1 + 0 * m, lambda m: 1 + 0 * m)
    assert yc.chi2(mu, mub) == pytest.approx(num / den, rel=1e-8)


def test_chi2_limits_and_eq_d20():
    assert yc.chi2(-1.0, -1.0) == 1.0                        # isotropic: no correction
    assert yc.chi2(1.0, 1.0) == 0.0                          # collinear beams do not annihilate
    mu = np.linspace(-1, 1, 41)
    np.testing.assert_allclose(yc.chi2(mu, mu), (1 - mu) ** 2 * (mu * mu + 4 * mu + 5) / 8, rtol=1e-14, atol=1e-15)


def test_limb_cosine_eq_d22():
    x = np.array([0.0, 0.6, 1.0, 1.0 + 1e-8, 1.2, 3.0])
    mu = yc.limb_cosine(x)
    np.testing.assert_allclose(mu[:3], [1.0, 0.8, 0.0], atol=1e-15)
    assert -1e-3 < mu[3] < 0                                  # just inside: small and negative
    np.testing.assert_allclose(mu[4], -np.sqrt(1.2 ** 2 - 1), rtol=1e-14)
    assert mu[5] == -1.0                                      # clipped deep inside
    # deep inside chi_2 -> 1, so chi = min(chi_1, chi_2) is governed by chi_1 (the text after eq. d22)
    assert yc.chi2(mu[5], mu[5]) == 1.0


def test_pairs_conserve_nu_minus_antinu_number():
    """Each pair event creates or destroys one nu_e and one anti-nu_e: sum_k W_k S_nu = sum_k W_k S_nubar
    in every zone, for any occupations (eq. d11 with its creation and annihilation kernels)."""
    _, _, cs, _ = _ray(zones=10, groups=7)
    rng = np.random.default_rng(4)
    # species with different neutrinospheres and flux factors, so that chi is not symmetric in (k, k')
    eta = cs.pair_eta1.copy()
    eta[1] = rng.uniform(0, 1, eta[1].shape)
    cs = dataclasses.replace(cs, pair_eta1=eta, nuebar=dataclasses.replace(cs.nuebar, r_nu=1.7 * cs.nuebar.r_nu))
    pe, pa = rng.uniform(0, 1, (cs.I, cs.N)), rng.uniform(0, 1, (cs.I, cs.N))
    s_e, s_a = yc.pair_sources(cs, pe, pa)
    _, W = oracle.group_energies(cs.nue.e_edge)
    np.testing.assert_allclose(s_e @ W, s_a @ W, rtol=1e-12)
    assert np.all(np.abs(s_e @ W) > 0)


def _isotropic(cs):
    """No anisotropy: flux factors 0 (chi_1 = 1) and neutrinospheres outside the grid (chi_2 = 1)."""
    big = 1e12 * np.ones(cs.N)
    return dataclasses.replace(cs, pair_eta1=np.zeros_like(cs.pair_eta1),
                               nue=dataclasses.replace(cs.nue, r_nu=big), nuebar=dataclasses.replace(cs.nuebar, r_nu=big))


@pytest.mark.parametrize("dmu", [0.0, 3.0, -3.0])
def test_fermi_dirac_pairs_with_opposite_chemical_potentials_are_in_equilibrium(dmu):
    """Detailed balance (eq. d12): creation balances annihilation for Fermi-Dirac occupations with
    mu_nu + mu_nubar = 0; with mu_nu + mu_nubar > 0 the excess annihilates (S < 0), below it pairs are
    created (S > 0)."""
    _, _, cs, _ = _ray(zones=8, groups=8)
    cs = _isotropic(cs)
    eps, W = oracle.group_energies(cs.nue.e_edge)
    T = cs.nue.temp[:, None]
    mu = 5.0
    fd = lambda m: 0.5 * (1.0 - np.tanh(0.5 * (eps[None, :] - m) / T))   # noqa: E731  Fermi-Dirac, no overflow
    s_e, s_a = yc.pair_sources(cs, fd(mu + dmu), fd(-mu))
    scale = np.max(np.abs(yc.pair_kernels(cs)[0]))
    if dmu == 0.0:
        assert np.max(np.abs(s_e)) < 1e-14 * scale and np.max(np.abs(s_a)) < 1e-14 * scale
    else:
        assert np.all(np.sign(s_e @ W) == -np.sign(dmu)) and np.all(np.sign(s_a @ W) == -np.sign(dmu))


def test_coupled_jacobian_with_pairs_matches_central_differences():
    _, _, cs, u_n = _ray(zones=5, groups=4)
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
        Jfd[:, j] = (yc.residual(cs, u_n, xp.reshape(u.shape)).ravel()
                     - yc.residual(cs, u_n, xm.reshape(u.shape)).ravel()) / (2 * h)
    rowmax = np.abs(J).max(axis=1, keepdims=True)
    assert np.all(np.abs(J - Jfd) <= 1e-6 * np.abs(J) + 1e-9 * rowmax)
    # the cross-species blocks are populated by the pairs
    A, _, _ = yc.jacobian_blocks(cs, u)
    assert np.min(np.abs(A[:, :N, N:2 * N])) > 0


def test_total_lepton_number_is_conserved_with_pairs():
    _, _, cs, u_n = _ray(zones=20, groups=6, outer_bc=0)
    res = yc.newton(cs, u_n, max_iter=30, rtol=1e-13)
    assert res.converged
    L0, L1 = yc.lepton_number(cs, u_n), yc.lepton_number(cs, res.psi)
    _, V, _, _ = oracle.geometry(cs.nue.r_edge)
    electrons = float(np.sum(V * cs.rho * u_n[:, -1] / yc.M_B_G))
    assert abs(L1 - L0) <= 1e-12 * abs(electrons)
    # the pairs change the step: without them psi differs
    res0 = yc.newton(dataclasses.replace(cs, pair_amp=None), u_n, max_iter=30, rtol=1e-13)
    assert np.max(np.abs(res.psi[:, :2 * cs.N] - res0.psi[:, :2 * cs.N]) / np.max(np.abs(res0.psi[:, :2 * cs.N]))) > 1e-6


def test_temperature_update_conserves_total_energy_with_pairs():
    wn, ye, cs, u_n = _ray(zones=16, groups=6, outer_bc=0)
    res = yc.newton(cs, u_n, max_iter=30, rtol=1e-14)
    sy = oracle.systems_from_workload(wn)
    others = [sy[2][0], sy[3][0]]
    p_others = [oracle.newton(s, wn["psi_n"][q, 0], max_iter=30, rtol=1e-14).psi for q, s in zip((2, 3), others)]
    weights = (1.0, 1.0, 2.0, 2.0)
    de, _ = yc.temperature_update(cs, others, res.psi, p_others, weights, wn["temp"][0], ye["de_dT"][0],
                                  ye["de_dye"][0])
    _, V, _, _ = oracle.geometry(cs.nue.r_edge)
    matter = float(np.sum(V * cs.rho / yc.M_B_G * de))
    N = cs.N
    new = [res.psi[:, :N], res.psi[:, N:2 * N]] + p_others
    old = [u_n[:, :N], u_n[:, N:2 * N], wn["psi_n"][2, 0], wn["psi_n"][3, 0]]
    systems = [cs.nue, cs.nuebar] + others
    nu = sum(w * (yc.neutrino_energy(s, a) - yc.neutrino_energy(s, b)) for w, s, a, b in zip(weights, systems, new, old))
    assert abs(matter + nu) <= 1e-10 * abs(matter)


def test_pins_catch_a_wrong_sign_in_the_creation_factor(monkeypatch):
    real = yc.pair_kernels

    def bad(cs):
        qa, qp, qba, qbp = real(cs)
        eps, _ = oracle.group_energies(cs.nue.e_edge)
        with np.errstate(over="ignore", invalid="ignore"):
            flip = np.exp(2 * (eps[:, None] + eps[None, :])[None] / cs.nue.temp[:, None, None])
            return qa, qp * flip, qba, qbp * np.transpose(flip, (0, 2, 1))
    monkeypatch.setattr(yc, "pair_kernels", bad)
    with pytest.raises(AssertionError):
        test_fermi_dirac_pairs_with_opposite_chemical_potentials_are_in_equilibrium(0.0)


def test_pins_catch_the_printed_closed_form_of_chi1(monkeypatch):
    """The closed form printed with eq. d16 (1/6 in place of 3/2) is not the ratio that defines it."""
    monkeypatch.setattr(yc, "chi1", lambda a, b: 1.0 - np.asarray(a) * np.asarray(b) / 6.0)
    with pytest.raises(AssertionError):
        test_chi1_is_the_ratio_of_eq_d16(0.3, 0.05, 0.2, 0.06)


def test_pins_catch_an_untransposed_angular_factor(monkeypatch):
    """The anti-neutrino rows must see chi with its groups exchanged; using chi as it stands breaks the
    nu - anti-nu balance."""
    real = yc.pair_sources

    def bad(cs, pe, pa):
        s_e, _ = real(cs, pe, pa)
        _, _, qba, qbp = yc.pair_kernels(cs)
        chi = yc.pair_chi(cs)
        s_a = (1.0 - pa) * np.einsum("ikl,il->ik", qbp, 1.0 - pe) - pa * np.einsum("ikl,il->ik", qba * chi, pe)
        return s_e, s_a
    monkeypatch.setattr(yc, "pair_sources", bad)
    with pytest.raises(AssertionError):
        test_pairs_conserve_nu_minus_antinu_number()


def test_pins_catch_a_weight_of_the_wrong_species(monkeypatch):
    real = yc.pair_kernels

    def bad(cs):
        qa, qp, qba, qbp = real(cs)
        _, W = oracle.group_energies(cs.nue.e_edge)
        fix = (W[None, :] / W[:, None])[None]          # Qbar with W_k' (its own group) instead of W_k
        return qa, qp, qba / fix.transpose(0, 2, 1), qbp / fix.transpose(0, 2, 1)
    monkeypatch.setattr(yc, "pair_kernels", bad)
    with pytest.raises(AssertionError):
        test_pairs_conserve_nu_minus_antinu_number()
