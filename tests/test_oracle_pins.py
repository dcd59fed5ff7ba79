"""Pins of the CPU oracle against what the paper and the mathematics fix (CPU only).

Each test names the passage it follows.  None of them retypes the oracle's
formula: they use closed forms, conservation invariants, limits, symmetries,
brute-force dense solves and finite differences, so that a dropped term, a wrong
sign or index or a transposed operand in the oracle fails at least one of them.
The last group plants such mistakes in the oracle (monkeypatched, CPU only) and
checks that the pins catch them.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import oracle.transport as ot
import synth

D1, EA, NES = synth.TERM_DIFFUSION, synth.TERM_EMABS, synth.TERM_NES


def _system(S=1, R=1, I=12, N=6, s=0, r=0, **kw):
    w = synth.make_custom(S=S, R=R, I=I, N=N).numpy()
    w.update(kw)
    return oracle.systems_from_workload(w)[s][r], w["psi_n"][s, r]


def _uniform_system(I, N, T, mu, rho=3e13, terms=synth.TERMS_ALL):
    """A spatially uniform medium (all zones identical) with zero-flux boundaries."""
    sysm, _ = _system(I=I, N=N, outer_bc=synth.BC_ZERO_FLUX, terms=terms)
    eps, W = oracle.group_energies(sysm.e_edge)
    ka = np.tile(1e-6 * (rho / 1e14) * (eps / 10.0) ** 2, (I, 1))
    x = (eps - mu) / T
    f_fd = 1.0 / (1.0 + np.exp(x))
    sysm = dataclasses.replace(
        sysm, temp=np.full(I, T), kappa_a=ka, eta=ka * np.exp(-x)[None, :], kappa_s=2 * ka,
        nes_amp=np.full(I, 1e-7 * rho / 1e14 * 50.0))          # a strong NES kernel
    return sysm, np.tile(f_fd, (I, 1))


# ------------------------------------------------------------------ grids

def test_group_weight_identity_eq_a01b():
    """eq. a01b: eps_k^2 (e_{k+1/2} - e_{k-1/2}) = (e_{k+1/2}^3 - e_{k-1/2}^3)/3, which holds
    only with the square restored on the left of eq. a01."""
    e = 2.0 * 150.0 ** (np.arange(21) / 20.0)
    eps, W = oracle.group_energies(e)
    np.testing.assert_allclose(eps ** 2 * np.diff(e), W, rtol=1e-14)
    assert np.all((eps > e[:-1]) & (eps < e[1:]))


def test_geometry_volumes_and_areas():
    """Zone volumes are r^2 dr integrals (4 pi dropped) and telescope to the ball shell."""
    r = np.sort(np.random.default_rng(1).uniform(1e6, 1e9, 40))
    Rc, V, A, D = oracle.geometry(r)
    for i in range(len(V)):
        xs = np.linspace(r[i], r[i + 1], 2001)
        np.testing.assert_allclose(V[i], np.trapezoid(xs ** 2, xs), rtol=1e-6)
    np.testing.assert_allclose(V.sum(), (r[-1] ** 3 - r[0] ** 3) / 3, rtol=1e-13)
    np.testing.assert_allclose(A, r ** 2, rtol=0)
    assert np.all(D > 0) and np.all((Rc > r[:-1]) & (Rc < r[1:]))


# ------------------------------------------------------------------ P1: e/a closed form

@pytest.mark.parametrize("terms", [EA, EA | D1])
def test_single_zone_emission_absorption_closed_form(terms):
    """Single zone, zero flux on both sides, NES off: backward Euler of eq. a58 with the
    eq. a54 source is linear, so one Newton step gives
    psi = (psi^n + c dt j) / (1 + c dt (j + kappa_a)) exactly."""
    rng = np.random.default_rng(2)
    for trial in range(20):
        sysm, psin = _system(I=1, N=5, outer_bc=synth.BC_ZERO_FLUX, terms=terms)
        ka = 10.0 ** rng.uniform(-8, -3, (1, 5))
        j = 10.0 ** rng.uniform(-8, -3, (1, 5))
        psin = rng.uniform(0, 1, (1, 5))
        sysm = dataclasses.replace(sysm, kappa_a=ka, eta=j, kappa_s=3 * ka)
        res = oracle.newton(sysm, psin, max_iter=1, rtol=0.0)
        c = sysm.c_dt
        expect = (psin + c * j) / (1.0 + c * (j + ka))
        np.testing.assert_allclose(res.psi, expect, rtol=1e-14, atol=0)
        assert res.res <= 1e-15 * max(1.0, float(np.max(c * (j + ka))))


def test_many_zones_no_transport_closed_form():
    """With diffusion and NES off every cell is the same closed form, for any zone count."""
    sysm, psin = _system(I=30, N=7, terms=EA)
    res = oracle.newton(sysm, psin, max_iter=1)
    c = sysm.c_dt
    expect = (psin + c * sysm.eta) / (1.0 + c * (sysm.eta + sysm.kappa_a))
    np.testing.assert_allclose(res.psi, expect, rtol=1e-14)


# ------------------------------------------------------------------ P2: Fermi-Dirac fixed point

@pytest.mark.parametrize("T,mu", [(10.0, 20.0), (4.0, -8.0), (0.7, 1.4), (25.0, 50.0)])
def test_fermi_dirac_is_fixed_point(T, mu):
    """Uniform medium, zero-flux boundaries, psi^n = f_FD: G(f_FD) = 0 (eq. d4 detailed balance
    for NES; j(1 - f) = kappa_a f for emission/absorption; zero gradient for diffusion), and a
    Newton step leaves f_FD unchanged."""
    sysm, f = _uniform_system(I=6, N=10, T=T, mu=mu)
    G = oracle.residual(sysm, f, f)
    assert np.max(np.abs(G)) < 1e-15
    res = oracle.newton(sysm, f, max_iter=2)
    np.testing.assert_allclose(res.psi, f, rtol=1e-13, atol=1e-300)


def test_fermi_dirac_relaxation():
    """Starting from 0.9 f_FD in a uniform medium the step moves psi toward f_FD."""
    sysm, f = _uniform_system(I=4, N=8, T=8.0, mu=16.0)
    res = oracle.newton(sysm, 0.9 * f, max_iter=10, rtol=1e-13)
    assert np.all(res.psi > 0.9 * f) and np.all(res.psi <= f * (1 + 1e-12))


# ------------------------------------------------------------------ P3/P4: conservation

def test_pure_diffusion_conserves_number_every_iterate():
    """eqs. a60-a62: with zero flux at both ends, sum_i V_i psi_{i,k} is unchanged per group,
    at every Newton iterate (the Jacobian's V-weighted column sums telescope)."""
    sysm, psin = _system(I=40, N=6, terms=D1, outer_bc=synth.BC_ZERO_FLUX)
    rng = np.random.default_rng(3)
    psin = rng.uniform(0.0, 1.0, psin.shape) * np.exp(-np.arange(40) / 6.0)[:, None]
    _, V, _, _ = oracle.geometry(sysm.r_edge)
    n0 = (V[:, None] * psin).sum(axis=0)
    psi = psin.copy()
    for _ in range(6):
        G = oracle.residual(sysm, psin, psi)
        A, bm, bp = oracle.jacobian_blocks(sysm, psi)
        psi = psi + oracle.block_thomas_solve(A, bm, bp, -G)
        np.testing.assert_allclose((V[:, None] * psi).sum(axis=0), n0, rtol=1e-12)
    # and the number actually moved: diffusion spread the profile
    assert np.max(np.abs(psi - psin)) > 1e-3


def test_nes_conserves_number():
    """eq. d3: sum_k W_k S_k = 0 for any psi, and with zero-flux diffusion the total
    sum V W psi is invariant at every iterate while energy is exchanged."""
    sysm, psin = _system(I=10, N=12, terms=D1 | NES, outer_bc=synth.BC_ZERO_FLUX)
    sysm = dataclasses.replace(sysm, nes_amp=sysm.nes_amp * 1e3)
    rng = np.random.default_rng(4)
    psi = rng.uniform(0, 1, psin.shape)
    _, W = oracle.group_energies(sysm.e_edge)
    S = ot.nes_source(sysm, psi)
    assert abs(np.sum(W * S)) < 1e-13 * np.sum(np.abs(W * S))
    _, V, _, _ = oracle.geometry(sysm.r_edge)
    VW = V[:, None] * W[None, :]
    n0 = np.sum(VW * psin)
    res = oracle.newton(sysm, psin, max_iter=4)
    np.testing.assert_allclose(np.sum(VW * res.psi), n0, rtol=1e-12)
    eps, _ = oracle.group_energies(sysm.e_edge)
    assert abs(np.sum(VW * eps * res.psi) / np.sum(VW * eps * psin) - 1) > 1e-8


def test_isoenergetic_scattering_has_no_moment0_source():
    """eq. d8b: isoenergetic scattering contributes nothing to the zeroth moment, so with
    zero gradient the residual does not depend on kappa_s."""
    sysm, f = _uniform_system(I=5, N=6, T=5.0, mu=3.0)
    psi = 0.7 * f
    G1 = oracle.residual(sysm, f, psi)
    G2 = oracle.residual(dataclasses.replace(sysm, kappa_s=sysm.kappa_s * 1e4), f, psi)
    np.testing.assert_array_equal(G1, G2)


def test_budget_identity():
    """sum_i V_i sum_k W_k G_{i,k} = N^{n+1} - N^n + B_N - Q_N - NES_N (eq. a62 summed)."""
    sysm, psin = _system(I=20, N=8)
    psi = psin * np.random.default_rng(5).uniform(0.5, 1.5, psin.shape)
    _, V, _, _ = oracle.geometry(sysm.r_edge)
    _, W = oracle.group_energies(sysm.e_edge)
    G = oracle.residual(sysm, psin, psi)
    st = oracle.step_stats(sysm, psin, psi)
    lhs = np.sum(V[:, None] * W[None, :] * G)
    np.testing.assert_allclose(lhs, st["budget"], rtol=1e-10)


# ------------------------------------------------------------------ P5: limiter and flux

def test_limiter_limits_eq_a21_a22():
    """eq. a21: lambda -> 0 gives the diffusion flux -(lambda/3) dpsi/dR; eq. a22: lambda -> inf
    gives |psi^(1)| -> psi (the edge mean), the free-streaming limit."""
    u, v, D = np.array([0.8, 0.2, 0.5]), np.array([0.3, 0.6, 0.5]), 1e5
    for lam in [1e-3, 1e-1]:
        H = oracle.edge_flux(u, v, lam, D, 1e-300)[0]
        np.testing.assert_allclose(H[:2], -(lam / 3) * (v - u)[:2] / D, rtol=1e-6)
    H = oracle.edge_flux(u, v, 1e20, D, 1e-300)[0]
    np.testing.assert_allclose(np.abs(H[:2]), 0.5 * (u + v)[:2], rtol=1e-12)
    assert H[2] == 0.0
    # flux points down the gradient (outward when psi falls outward)
    assert H[0] > 0 and H[1] < 0


def test_diffusion_operator_on_quadratic_profile():
    """Uniform radial grid, F = 1, constant lambda, psi = alpha + beta r^2: the conservative
    divergence (A H)_{i+1/2} - (A H)_{i-1/2} over V_i equals the continuum value
    div(-(lambda/3) grad psi) = -2 lambda beta exactly in interior zones."""
    I, N = 24, 3
    r = np.linspace(1e6, 5e6, I + 1)
    chi = 1e-4
    sysm, _ = _system(I=I, N=N, terms=D1, limiter=0, outer_bc=synth.BC_ZERO_FLUX)
    sysm = dataclasses.replace(sysm, r_edge=r, kappa_a=np.full((I, N), chi / 4),
                               eta=np.full((I, N), chi / 4), kappa_s=np.full((I, N), chi / 2))
    Rc = 0.5 * (r[1:] + r[:-1])
    beta = 1e-14
    psi = (0.2 + beta * Rc ** 2)[:, None] * np.ones((1, N))
    G = oracle.residual(sysm, psi, psi)
    lam = 1.0 / chi
    np.testing.assert_allclose(G[1:-1], sysm.c_dt * (-2.0 * lam * beta), rtol=1e-9)


def test_zero_state_is_finite():
    """psi = 0 everywhere (the floor path of the limiter) keeps G and J finite."""
    sysm, psin = _system(I=8, N=5)
    z = np.zeros_like(psin)
    G = oracle.residual(sysm, z, z)
    A, bm, bp = oracle.jacobian_blocks(sysm, z)
    assert np.all(np.isfinite(G)) and np.all(np.isfinite(A)) and np.all(np.isfinite(bm)) and np.all(np.isfinite(bp))


# ------------------------------------------------------------------ NES kernel symmetries

def test_nes_kernel_symmetries_d3_d4():
    """eq. d3 (weighted discrete form) W_k K^in_{kk'} = W_k' K^out_{k'k} and eq. d4
    K^in_{kk'} = exp((eps_k' - eps_k)/T) K^out_{kk'}."""
    e = 2.0 * 150.0 ** (np.arange(13) / 12.0)
    eps, W = oracle.group_energies(e)
    le = np.log(eps)
    G = np.exp(-(le[:, None] - le[None, :]) ** 2 / (2 * 0.3 ** 2))
    for T in [0.5, 3.0, 30.0]:
        k_out, k_in = oracle.nes_kernels(2e-7, T, eps, W, G)
        np.testing.assert_allclose(W[:, None] * k_in, (W[:, None] * k_out).T, rtol=1e-14, atol=1e-300)
        ratio_exp = (eps[None, :] - eps[:, None]) / T
        mask = np.abs(ratio_exp) < 600
        np.testing.assert_allclose(k_in[mask], (np.exp(ratio_exp) * k_out)[mask], rtol=1e-12, atol=1e-300)
        assert np.all(k_out >= 0) and np.all(k_in >= 0)
        # kernel diagonal equals amp * (eps/eps0)^2 * W/Wbar (G_kk = 1)
        np.testing.assert_allclose(np.diag(k_out), 2e-7 * (eps / 10) ** 2 * W / W.mean(), rtol=1e-14)


# ------------------------------------------------------------------ P6/P7: solver and Jacobian

@pytest.mark.parametrize("transpose", [False, True])
def test_block_thomas_matches_dense_lapack(transpose):
    """The block-Thomas solve equals numpy.linalg.solve of the assembled (I*N)^2 matrix."""
    for cfg_shape in [(40, 12), (7, 20), (1, 9), (25, 1)]:
        I, N = cfg_shape
        sysm, psin = _system(I=I, N=N)
        psi = psin * 1.1
        rhs = np.random.default_rng(6).standard_normal((I, N))
        A, bm, bp = oracle.jacobian_blocks(sysm, psi)
        x = oracle.block_thomas_solve(A, bm, bp, rhs, transpose=transpose)
        xd = oracle.dense_solve(sysm, psi, rhs, transpose=transpose)
        np.testing.assert_allclose(x, xd, rtol=1e-11, atol=1e-13 * np.max(np.abs(xd)))


@pytest.mark.parametrize("limiter", [0, 1])
def test_jacobian_matches_central_differences(limiter):
    """Every column of the analytic Jacobian equals a central difference of G (about 1e-7)."""
    sysm, psin = _system(I=6, N=5, limiter=limiter)
    sysm = dataclasses.replace(sysm, nes_amp=sysm.nes_amp * 1e3)
    rng = np.random.default_rng(7)
    psi = np.clip(psin * rng.uniform(0.5, 1.5, psin.shape), 0.0, 0.99)
    # no exact ties between neighbours: |psi_{i+1} - psi_i| has a kink at zero
    psi = np.where(psi < 1e-3, rng.uniform(1e-3, 5e-3, psi.shape), psi)
    J = oracle.dense_jacobian(sysm, psi)
    n = psi.size
    for col in range(n):
        h = 1e-6 * max(abs(psi.flat[col]), 1e-3)
        pp, pm = psi.copy(), psi.copy()
        pp.flat[col] += h
        pm.flat[col] -= h
        fd = (oracle.residual(sysm, psin, pp) - oracle.residual(sysm, psin, pm)).reshape(-1) / (2 * h)
        np.testing.assert_allclose(J[:, col], fd, rtol=2e-6, atol=1e-8 * np.max(np.abs(J[:, col])))


def test_newton_converges_quadratically():
    """An exact Jacobian gives quadratic convergence: e_{m+1} <= C e_m^2 with modest C."""
    w = synth.make(0).numpy()
    sysm = oracle.systems_from_workload(w)[0][3]
    psin = w["psi_n"][0, 3]
    ref = oracle.newton(sysm, psin, max_iter=12, rtol=1e-15).psi
    psi = psin.copy()
    errs = []
    for _ in range(4):
        errs.append(np.max(np.abs(psi - ref)))
        G = oracle.residual(sysm, psin, psi)
        A, bm, bp = oracle.jacobian_blocks(sysm, psi)
        psi = psi + oracle.block_thomas_solve(A, bm, bp, -G)
    assert errs[1] < 1e-3 * errs[0]
    assert errs[2] <= 50.0 * errs[1] ** 2
    assert errs[3] < 1e-12


# ------------------------------------------------------------------ P8: adjoint

def test_adjoint_dot_product():
    """<v, J^{-1} w> = <J^{-T} v, w> with the block-Thomas forward solve and the dense transpose."""
    sysm, psin = _system(I=15, N=7)
    rng = np.random.default_rng(8)
    v, wv = rng.standard_normal((2,) + psin.shape)
    A, bm, bp = oracle.jacobian_blocks(sysm, psin)
    x = oracle.block_thomas_solve(A, bm, bp, wv)
    mu = oracle.adjoint(sysm, psin, v)
    np.testing.assert_allclose(np.sum(v * x), np.sum(mu * wv), rtol=1e-11)


def test_luminosity_gradient_matches_central_differences():
    """dL/dtheta from the adjoint (J^T mu = dL/dpsi, g = -mu^T dG/dtheta) equals central finite
    differences of L(psi^{n+1}(theta)) along random relative directions (h = 1e-6)."""
    sysm, psin = _system(I=10, N=6)
    # make the medium optically thick enough that all terms matter
    sysm = dataclasses.replace(sysm, kappa_a=sysm.kappa_a * 30, eta=sysm.eta * 30,
                               kappa_s=sysm.kappa_s * 30, nes_amp=sysm.nes_amp * 300)

    def solve(sy, pn):
        return oracle.newton(sy, pn, max_iter=40, rtol=1e-15).psi

    psi = solve(sysm, psin)
    seed = oracle.luminosity_seed(sysm, psi.shape)
    mu = oracle.adjoint(sysm, psi, seed)
    g = oracle.param_vjp(sysm, psi, mu)
    rng = np.random.default_rng(9)
    h = 1e-6
    for name in ["kappa_a", "eta", "kappa_s", "nes_amp", "psi_n"]:
        for _ in range(3):
            base = psin if name == "psi_n" else getattr(sysm, name)
            d = rng.standard_normal(base.shape) * base

            def L(sign):
                if name == "psi_n":
                    return oracle.luminosity(sysm, solve(sysm, psin + sign * h * d))
                sy = dataclasses.replace(sysm, **{name: base + sign * h * d})
                return oracle.luminosity(sy, solve(sy, psin))

            fd = (L(+1) - L(-1)) / (2 * h)
            an = np.sum(g[name] * d)
            assert abs(fd - an) <= 1e-5 * abs(an) + 1e-9 * abs(oracle.luminosity(sysm, psi)), (name, fd, an)


# ------------------------------------------------------------------ planted mistakes (CPU only)

def test_pins_catch_swapped_nes_kernels(monkeypatch):
    """Plant the opposite detailed-balance sign (in and out kernels swapped): the
    Fermi-Dirac fixed point pin must fail."""
    orig = ot.nes_kernels
    monkeypatch.setattr(ot, "nes_kernels", lambda *a: orig(*a)[::-1])
    sysm, f = _uniform_system(I=3, N=8, T=4.0, mu=8.0)
    assert np.max(np.abs(oracle.residual(sysm, f, f))) > 1e-8


def test_pins_catch_missing_third_in_flux(monkeypatch):
    """Plant a flux without the 1/3 of eq. a59: the quadratic-profile pin must fail."""
    orig = ot.edge_flux
    monkeypatch.setattr(ot, "edge_flux",
                        lambda u, v, lam, D, fl, lim=1, limb=None: tuple(3 * x for x in orig(u, v, lam, D, fl, lim, limb)))
    with pytest.raises(AssertionError):
        test_diffusion_operator_on_quadratic_profile()


def test_pins_catch_transposed_nes_jacobian(monkeypatch):
    """Plant a transposed dense block in the Jacobian: the finite-difference pin must fail."""
    orig = ot.jacobian_blocks

    def bad(sysm, psi):
        A, bm, bp = orig(sysm, psi)
        return np.transpose(A, (0, 2, 1)).copy(), bm, bp
    monkeypatch.setattr(ot, "jacobian_blocks", bad)
    with pytest.raises(AssertionError):
        test_jacobian_matches_central_differences(1)


def test_block_route_of_the_multistep_adjoint_equals_the_dense_route():
    """The transposed block-Thomas route of the reverse recursion (used on full-size rays) gives the dense
    route's dJ/dpsi^0 and per-step opacity gradients."""
    ws = [synth.make(4, rays=[3], zones=20, groups=8, species=2, step=s).numpy() for s in range(3)]
    for sp in range(2):
        syss = [oracle.systems_from_workload(w)[sp][0] for w in ws]
        psis = oracle.multistep_forward(syss, ws[0]["psi_n"][sp, 0], max_iter=10, rtol=0.0)
        g_d, gr_d = oracle.multistep_adjoint(syss, psis)
        g_b, gr_b = oracle.multistep_adjoint(syss, psis, solver="block")
        np.testing.assert_allclose(g_b, g_d, rtol=1e-10, atol=1e-13 * np.max(np.abs(g_d)))
        for a, b in zip(gr_b, gr_d):
            for n in ("kappa_a", "eta", "kappa_s"):
                np.testing.assert_allclose(a[n], b[n], rtol=1e-9, atol=1e-12 * np.max(np.abs(b[n])))


def test_multistep_adjoint_matches_central_differences():
    """Three drifting steps, J = sum_s L(psi^s): the reverse recursion equals central differences of J
    with respect to psi^0 and to the absorption opacity of the first and last step."""
    ws = [synth.make(4, rays=[7], zones=8, groups=5, species=1, step=s).numpy() for s in range(3)]
    syss = [oracle.systems_from_workload(w)[0][0] for w in ws]
    syss = [dataclasses.replace(sy, kappa_a=sy.kappa_a * 1e3, eta=sy.eta * 1e3, kappa_s=sy.kappa_s * 1e3,
                                nes_amp=sy.nes_amp * 1e4) for sy in syss]
    psi0 = ws[0]["psi_n"][0, 0]

    def fwd(sy_list, p0):
        return oracle.multistep_forward(sy_list, p0, max_iter=10, rtol=0.0)

    psis = fwd(syss, psi0)
    g0, grads = oracle.multistep_adjoint(syss, psis)
    rng = np.random.default_rng(21)
    # J carries ~1e-11 relative rounding noise on this optically thick test system, so the
    # step is 1e-4 relative (truncation O(h^2) ~ 1e-8) rather than a noise-dominated 1e-6
    h = 1e-4

    def J(sy_list, p0):
        return oracle.multistep_objective(sy_list, fwd(sy_list, p0))

    d = rng.standard_normal(psi0.shape) * psi0
    fd = (J(syss, psi0 + h * d) - J(syss, psi0 - h * d)) / (2 * h)
    assert abs(fd - np.sum(g0 * d)) <= 1e-5 * abs(fd)
    for s in (0, 2):
        d = rng.standard_normal(psi0.shape) * syss[s].kappa_a
        plus = [dataclasses.replace(sy, kappa_a=sy.kappa_a + h * d) if j == s else sy for j, sy in enumerate(syss)]
        minus = [dataclasses.replace(sy, kappa_a=sy.kappa_a - h * d) if j == s else sy for j, sy in enumerate(syss)]
        fd = (J(plus, psi0) - J(minus, psi0)) / (2 * h)
        an = np.sum(grads[s]["kappa_a"] * d)
        assert abs(fd - an) <= 1e-5 * abs(an), (s, fd, an)


# ------------------------------------------------------------------ Newton globalisation

def _plain_newton(sys, psi_n, n):
    """Undamped Newton (the paper's outer iteration without the line search), n updates."""
    psi = psi_n.copy()
    hist = []
    for _ in range(n):
        G = oracle.residual(sys, psi_n, psi)
        hist.append(float(np.max(np.abs(G))))
        A, bm, bp = oracle.jacobian_blocks(sys, psi)
        psi = psi + oracle.block_thomas_solve(A, bm, bp, -G)
    hist.append(float(np.max(np.abs(oracle.residual(sys, psi_n, psi)))))
    return psi, hist


def test_line_search_takes_full_steps_where_plain_newton_converges():
    """On a system where undamped Newton converges, every full step passes the sufficient-decrease
    test, so the globalised iteration is plain Newton: identical iterates after the same updates."""
    w = synth.make(2, rays=[820]).numpy()
    sys = oracle.systems_from_workload(w)[0][0]
    psi_p, hist = _plain_newton(sys, w["psi_n"][0, 0], 3)
    assert hist[-1] < 1e-9 * hist[0]
    res = oracle.newton(sys, w["psi_n"][0, 0], max_iter=3, rtol=0.0)
    assert res.iters == 3
    np.testing.assert_array_equal(res.psi, psi_p)


def test_line_search_rescues_a_diverging_spike_system():
    """A spiked antineutrino system on which undamped Newton diverges (max|G| grows): the backtracking
    iteration decreases max|G| at every accepted step away from the target and converges (here to the
    rounding level of G, about 1e-11 of the initial residual)."""
    w = synth.make(2, rays=[592]).numpy()
    sys = oracle.systems_from_workload(w)[1][0]
    _, hist = _plain_newton(sys, w["psi_n"][1, 0], 6)
    assert hist[-1] > hist[0]                              # the paper's plain iteration fails here
    res = oracle.newton(sys, w["psi_n"][1, 0], max_iter=30, rtol=1e-12)
    assert res.converged and res.res <= 1e-10 * res.res0
    h = res.history
    for a, b in zip(h[:-1], h[1:]):
        assert b <= (1.0 - 1e-4 / 256) * a or b <= 1e3 * 1e-12 * res.res0
