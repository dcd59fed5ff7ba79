"""Pins of the energy-advection oracle (CPU): closed forms, exact integrals and conservation laws.

Each test checks the oracle against something the paper or the mathematics fixes, not against a
retyped copy of its own formulas: exact polynomial reproduction of the PPM interpolation (eqs. h9,
h12), quadrature of the parabola of eq. h22 (eqs. h60, h61), exact integrals of the swept regions
(eq. p5), number and energy conservation (eqs. p2, p3, p6-p8, a81a, a81b), the 2x2 solve behind
eqs. a81c and a81d, and the rho^(1/3) energy scaling of eq. a77.
"""
import numpy as np
import pytest

from oracle import energy_advection as ea

RNG = np.random.default_rng(1809056)


def nonuniform_grid(n, lo=1.0, hi=3.0, seed=0):
    r = np.random.default_rng(seed).uniform(0.5, 1.5, n)
    return np.concatenate([[lo], lo + np.cumsum(r) / r.sum() * (hi - lo)])


def cubic(x):
    return 1.0 + x + 0.1 * x ** 2 + 0.01 * x ** 3


def cubic_int(x):
    return x + x ** 2 / 2 + 0.1 * x ** 3 / 3 + 0.01 * x ** 4 / 4


def quad(x):
    return 2.0 + 0.3 * x - 0.2 * x ** 2


def quad_int(x):
    return 2.0 * x + 0.15 * x ** 2 - 0.2 * x ** 3 / 3


def averages(F, e):
    return (F(e[1:]) - F(e[:-1])) / np.diff(e)


def test_weights_are_eps_squared_times_width():
    """Eq. a01b: W_k = eps_k^2 (e_{k+1/2} - e_{k-1/2}) with the centres of eq. a01."""
    e = nonuniform_grid(20, 2.0, 300.0)
    assert np.allclose(ea.weights(e), ea.centers(e) ** 2 * np.diff(e), rtol=1e-14, atol=0)


def test_ppm_interface_values_reproduce_a_cubic():
    """Eq. h12 interpolates the integral of the zone averages by a quartic, so interior edge values
    of a cubic density are exact on any grid (edges whose stencil stays off the ghost groups)."""
    n = 24
    e = nonuniform_grid(n)
    aL, aR = ea.ppm_interfaces(averages(cubic_int, e), np.diff(e))
    edges = e[3:n - 1]                       # edge m = 3..n-2, right edge of groups 2..n-3
    assert np.allclose(aR[2:n - 2], cubic(edges), rtol=1e-13, atol=0)
    assert np.allclose(aL[3:n - 1], cubic(edges), rtol=1e-13, atol=0)


def test_ppm_interface_pin_catches_the_printed_h12(monkeypatch):
    """The printed eq. h12 (product d_i d_{i+1} in a denominator, 2d_i + d_{i+1} in the last term)
    fails the cubic pin: the pin decides the garble."""
    def printed(aj, aj1, dm, d0, d1, d2, sj, sj1):
        diff = aj1 - aj
        return (aj + d0 / (d0 + d1) * diff + 1.0 / (dm + d0 + d1 + d2) * (
            2.0 * d1 * d0 / (d0 * d1) * ((dm + d0) / (2.0 * d0 + d1) - (d1 + d2) / (2.0 * d0 + d1)) * diff
            - d0 * (dm + d0) / (2.0 * d0 + d1) * sj1 + d1 * (d1 + d2) / (d0 + 2.0 * d1) * sj))
    monkeypatch.setattr(ea, "interface_value", printed)
    n = 24
    e = nonuniform_grid(n)
    _, aR = ea.ppm_interfaces(averages(cubic_int, e), np.diff(e))
    assert not np.allclose(aR[2:n - 2], cubic(e[3:n - 1]), rtol=1e-6, atol=0)


def test_ppm_slopes_of_a_quadratic_are_exact():
    """Eq. h9 (with the width garble read as Delta xi_i): the mean slope times the width of a zone is
    the difference of the quadratic's edge values."""
    n = 16
    e = nonuniform_grid(n, seed=3)
    a = averages(quad_int, e)
    s = ea.ppm_slopes(ea._pad2(a), ea._pad2(np.diff(e)))
    exact = quad(e[1:]) - quad(e[:-1])
    # padded slopes 2..n-1 belong to groups 1..n-2 (groups with real neighbours on both sides)
    assert np.allclose(s[2:n], exact[1:n - 1], rtol=1e-13, atol=1e-15)


def test_monotonicity_limits():
    """Eq. h11 zeroes the slope at an extremum; eqs. h15-h16 keep edge values between the averages."""
    a = np.array([1.0, 2.0, 5.0, 3.0, 3.5, 0.2, 0.1, 4.0])
    d = np.linspace(1.0, 2.0, a.size)
    s = ea.ppm_slopes(ea._pad2(a), ea._pad2(d))
    assert s[1 + 2] == 0.0 and s[1 + 3] == 0.0        # groups 2 (maximum) and 3 (minimum)
    aL, aR = ea.ppm_interfaces(a, d)
    lo = np.minimum(a[:-1], a[1:])
    hi = np.maximum(a[:-1], a[1:])
    assert np.all(aR[:-1] >= lo) and np.all(aR[:-1] <= hi)
    assert np.array_equal(aL[1:], aR[:-1])


def test_zone_constraint_keeps_parabolas_free_of_interior_extrema():
    """After the zone constraint no group parabola has an extremum strictly inside its group, so every
    swept-region mean lies between the group's edge values, and the parabolas of a positive, steeply
    falling spectrum stay non-negative."""
    e = np.geomspace(2.0, 300.0, 21)
    eps = ea.centers(e)
    psi = 1.0 / (np.exp((eps - 6.0) / 3.0) + 1.0)
    a = psi * ea.weights(e) / np.diff(e)
    aL, aR = ea.monotone_edges(a, *ea.ppm_interfaces(a, np.diff(e)))
    Da, a6 = ea.parabola(a, aL, aR)
    x = np.linspace(0.0, 1.0, 201)[:, None]
    prof = aL + x * (Da + a6 * (1.0 - x))
    assert np.all(prof >= np.minimum(aL, aR) - 1e-15 * np.abs(a)) and np.all(prof >= 0.0)
    assert np.all(prof <= np.maximum(aL, aR) + 1e-15 * np.abs(a))
    # without the constraint the same spectrum has parabolas dipping below zero
    aL0, aR0 = ea.ppm_interfaces(a, np.diff(e))
    Da0, a60 = ea.parabola(a, aL0, aR0)
    assert np.any(aL0 + x * (Da0 + a60 * (1.0 - x)) < 0.0)


def test_remap_of_a_steep_spectrum_stays_non_negative():
    e = np.geomspace(2.0, 300.0, 21)
    eps = ea.centers(e)
    T = np.linspace(3.0, 12.0, 32)[:, None]
    psi = 0.9 / (np.exp((eps - 2.0 * T) / T) + 1.0)
    for s in (0.99, 1.01):
        out, xi, flags = ea.lapse_remap(psi, e, np.full(32, 0.9), np.full(32, 0.9 * s))
        assert np.all(flags == 0) and np.all(out >= 0.0)


def gauss_mean(f, lo, hi):
    x, w = np.polynomial.legendre.leggauss(4)
    t = 0.5 * (hi - lo) * x[:, None] + 0.5 * (hi + lo)
    return np.sum(w[:, None] * f(t), axis=0) / 2.0


def test_parabola_averages_by_quadrature():
    """Eq. h24 makes the parabola of eq. h22 average to the zone value; eqs. h60 and h61 (as read)
    are its means over the top and bottom fractions y of the zone."""
    m = 50
    a, aL, aR = RNG.uniform(0.0, 2.0, (3, m))
    y = RNG.uniform(0.0, 1.0, m)
    Da, a6 = ea.parabola(a, aL, aR)

    def prof(x):
        return aL + x * (Da + a6 * (1.0 - x))
    assert np.allclose(gauss_mean(prof, np.zeros(m), np.ones(m)), a, rtol=1e-14, atol=1e-15)
    assert np.allclose(ea.average_top(aR, Da, a6, y), gauss_mean(prof, 1.0 - y, np.ones(m)), rtol=1e-13, atol=1e-14)
    assert np.allclose(ea.average_bottom(aL, Da, a6, y), gauss_mean(prof, np.zeros(m), y), rtol=1e-13, atol=1e-14)


def test_bottom_mean_pin_catches_the_printed_h61_sign():
    """The printed eq. h61 factor (1 + 2y/3) disagrees with the integral of the parabola."""
    aL, aR, a, y = 1.0, 2.0, 1.2, 0.4
    Da, a6 = ea.parabola(a, aL, aR)
    printed = aL + 0.5 * y * (Da + (1.0 + 2.0 * y / 3.0) * a6)

    def prof(x):
        return aL + x * (Da + a6 * (1.0 - x))
    exact = gauss_mean(prof, np.zeros(1), np.full(1, y))[0]
    assert abs(printed - exact) > 1e-3
    assert abs(ea.average_bottom(aL, Da, a6, y) - exact) < 1e-14


def test_remap_fluxes_are_exact_integrals_of_a_quadratic_density():
    """Eq. p5: the flux through an edge is the number between the displaced and the fixed edge; with a
    quadratic density the PPM profile is exact in groups away from the ends, so the flux is the exact
    integral over the swept region (signed)."""
    n = 20
    tgt = nonuniform_grid(n, 2.0, 4.0, seed=5)
    shift = 0.3 * np.sin(np.arange(n + 1)) * np.minimum(np.diff(tgt, prepend=tgt[0] - 1)[:], 1.0)
    shift *= 0.3 * np.diff(tgt).min()
    src = tgt + shift
    src[0], src[-1] = tgt[0], tgt[-1]

    def dens(x):
        return 5.0 - 0.5 * x + 0.05 * x ** 2

    def dens_int(x):
        return 5.0 * x - 0.25 * x ** 2 + 0.05 * x ** 3 / 3
    N = dens_int(src[1:]) - dens_int(src[:-1])
    F, ok = ea.remap_fluxes(N, src, tgt)
    assert ok
    exact = dens_int(src) - dens_int(tgt)
    # the exact values are differences of antiderivatives near 20: rounding of about 1e-15 absolute
    assert np.allclose(F[3:n - 2], exact[3:n - 2], rtol=0, atol=1e-14)
    assert not np.allclose(F[3:n - 2], 0.0, rtol=0, atol=1e-4)
    assert F[0] == 0.0 and F[-1] == 0.0


def random_state(shape, n, seed):
    r = np.random.default_rng(seed)
    psi = r.uniform(0.0, 0.9, shape + (n,)) * np.exp(-np.linspace(0, 4, n))
    return psi


def test_remap_conserves_number_and_energy():
    """Eqs. p6-p8: any xi conserves the number; the one of eq. p8 also conserves the energy."""
    n = 20
    tgt = np.geomspace(2.0, 300.0, n + 1)
    r = np.random.default_rng(7)
    s = 1.0 + 0.02 * r.standard_normal((64, n + 1))
    src = tgt * s
    N = random_state((64,), n, 8) * ea.weights(src)
    N_new, xi, ok = ea.remap(N, src, np.broadcast_to(tgt, src.shape))
    assert ok.all()
    assert np.allclose(N_new.sum(-1), N.sum(-1), rtol=1e-14, atol=0)
    e_src, e_tgt = ea.centers(src), ea.centers(tgt)
    assert np.allclose((N_new * e_tgt).sum(-1), (N * e_src).sum(-1), rtol=1e-13, atol=0)


def test_no_displacement_leaves_psi_unchanged():
    n = 20
    e = np.geomspace(2.0, 300.0, n + 1)
    psi = random_state((10,), n, 9)
    out, xi, flags = ea.energy_advect(psi, e)
    assert np.allclose(out, psi, rtol=4e-16, atol=0) and np.all(xi == 1.0) and np.all(flags == 0)
    out, xi, flags = ea.lapse_remap(psi, e, np.full(10, 0.8), np.full(10, 0.8))
    assert np.allclose(out, psi, rtol=4e-16, atol=0) and np.all(flags == 0)


@pytest.mark.parametrize("x", [1e-3, 1e-2])
def test_homologous_compression_scales_energy_by_rho_cube_root(x):
    """Eq. a77: in the diffusion limit a homologous compression (dR/R = db/b = -x) shifts every energy
    by s = 1 + x, which is (rho^{n+1}/rho^n)^{1/3} to first order; the number per unit mass is kept
    (eq. a78) and the remap keeps the energy (eq. p8), so the mean energy grows by exactly s."""
    n = 20
    e = np.geomspace(2.0, 300.0, n + 1)
    psi = random_state((16,), n, 11)
    rho_ratio = 1.0 / (1.0 - x) ** 3
    out, xi, flags = ea.energy_advect(psi, e, rho_old=1.0, rho_new=rho_ratio, dlnR=-x, dlnb=-x)
    assert np.all(flags == 0)
    n0, e0 = ea.number_and_energy(psi, e)
    n1, e1 = ea.number_and_energy(out, e)
    assert np.allclose(n1, rho_ratio * n0, rtol=1e-14, atol=0)
    assert np.allclose((e1 / n1) / (e0 / n0), 1.0 + x, rtol=1e-13, atol=0)
    assert abs((1.0 + x) - rho_ratio ** (1.0 / 3.0)) < 2.0 * x * x


def test_smooth_spectrum_needs_a_small_energy_correction():
    """For a Fermi-Dirac spectrum that is negligible at the grid ends, the PPM fluxes of a homologous
    compression carry nearly the right energy by themselves: xi of eq. p8 is close to 1."""
    n = 20
    e = np.geomspace(2.0, 300.0, n + 1)
    eps = ea.centers(e)
    T = np.linspace(4.0, 8.0, 8)[:, None]
    psi = 1.0 / (np.exp((eps - 2.0 * T) / T) + 1.0)
    out, xi, flags = ea.energy_advect(psi, e, rho_new=1.0 / 0.99 ** 3, dlnR=-0.01, dlnb=-0.01)
    assert np.all(flags == 0)
    assert np.all(np.abs(xi - 1.0) < 0.05), xi


def test_lapse_remap_conserves_number_and_energy():
    """Eqs. p2 and p3: after a lapse change the number and the energy in each zone are unchanged,
    each measured on its own local grid E/a."""
    n = 20
    E = np.geomspace(2.0, 300.0, n + 1)
    r = np.random.default_rng(12)
    a0 = r.uniform(0.7, 0.95, 32)
    a1 = a0 * (1.0 + 0.01 * r.standard_normal(32))
    psi = random_state((32,), n, 13)
    out, xi, flags = ea.lapse_remap(psi, E, a0, a1)
    assert np.all(flags == 0)
    n0, e0 = ea.number_and_energy(psi, E / a0[:, None])
    n1, e1 = ea.number_and_energy(out, E / a1[:, None])
    assert np.allclose(n1, n0, rtol=1e-14, atol=0) and np.allclose(e1, e0, rtol=1e-13, atol=0)


def test_overfill_limiter_solves_number_and_energy_balance():
    """Eqs. a81c, a81d are the solution of eqs. a81a, a81b for a given removal from group k: compare
    with a direct 2x2 solve, and check that number and energy are kept and psi <= 1 afterwards."""
    n = 12
    e = np.geomspace(2.0, 300.0, n + 1)
    psi = np.full(n, 0.5)
    psi[3] = 1.3
    out, flags = ea.overfill_limit(psi[None], e)
    out = out[0]
    eps, W = ea.centers(e), ea.weights(e)
    rm0 = 0.3
    A = np.array([[W[4], -W[5]], [W[4] * eps[4], -W[5] * eps[5]]])
    b = np.array([W[3] * rm0, W[3] * eps[3] * rm0])
    add1, rm2 = np.linalg.solve(A, b)
    assert np.isclose(out[3], 1.0, rtol=1e-15)
    assert np.isclose(out[4] - 0.5, add1, rtol=1e-12) and np.isclose(0.5 - out[5], rm2, rtol=1e-12)
    assert flags[0] == ea.FLAG_OVERFILL
    n0, e0 = ea.number_and_energy(psi, e)
    n1, e1 = ea.number_and_energy(out, e)
    assert np.isclose(n1, n0, rtol=1e-14) and np.isclose(e1, e0, rtol=1e-14)


def test_overfill_limiter_cascades_and_clamps():
    """A chain of over-filled groups is worked upward; a removal that would empty group k+2 below zero
    is scaled down (the approximate case), and number and energy are still kept."""
    n = 10
    e = np.geomspace(2.0, 300.0, n + 1)
    psi = np.array([1.5, 1.2, 0.9, 0.8, 1e-6, 0.3, 0.2, 0.1, 0.05, 0.01])
    out, flags = ea.overfill_limit(psi[None], e)
    out, flags = out[0], flags[0]
    assert flags & ea.FLAG_OVERFILL and flags & ea.FLAG_OVERFILL_CLAMP
    assert np.all(out >= 0.0)
    n0, e0 = ea.number_and_energy(psi, e)
    n1, e1 = ea.number_and_energy(out, e)
    assert np.isclose(n1, n0, rtol=1e-14) and np.isclose(e1, e0, rtol=1e-14)


def test_displacement_beyond_a_group_is_flagged_and_left_unchanged():
    n = 8
    e = np.geomspace(2.0, 300.0, n + 1)
    psi = random_state((2,), n, 14)
    out, xi, flags = ea.energy_advect(psi, e, dlnR=np.array([0.0, -0.9]), dlnb=np.array([0.0, 0.9]),
                                      eddington=np.stack([np.full(n, 0.4), np.linspace(0.34, 1.0, n)]))
    assert flags[1] == ea.FLAG_DISPLACEMENT and np.array_equal(out[1], psi[1])
    assert flags[0] == 0


# ---------------------------------------------------------------- eq. a79 against the angular physics

def beam_average(beta, x_R, x_b):
    """Eddington factor <mu^2> of an intensity I(mu) ~ exp(beta mu), and the intensity-weighted mean of
    the first-order energy change of a beam at direction cosine mu in a fluid element stretched radially by
    db/b = x_b and transversely by dR/R = x_R: the momentum component along each axis scales inversely
    with the element's length along it, so d ln eps = -mu^2 x_b - (1 - mu^2) x_R.  Gauss-Legendre
    quadrature over mu in [-1, 1]."""
    mu, wq = np.polynomial.legendre.leggauss(64)
    I = wq * np.exp(beta * mu)
    eta2 = float(np.sum(I * mu * mu) / np.sum(I))
    s = 1.0 + float(np.sum(I * (-mu * mu * x_b - (1.0 - mu * mu) * x_R)) / np.sum(I))
    return eta2, s


@pytest.mark.parametrize("beta", [0.0, 2.0, 8.0, 40.0])
def test_eq_a79_energy_shift_is_the_beam_average(beta):
    """Eq. a79 with dR/R != db/b and a constant Eddington factor: every group edge moves by the beam
    average s above, so the mean energy of each zone changes by exactly s (the remap keeps number and
    energy) and its number by the density ratio of eq. a78 (the element's volume changes by
    (1 + dR/R)^2 (1 + db/b))."""
    n = 20
    e = np.geomspace(2.0, 300.0, n + 1)
    x_R, x_b = -3e-3, 5e-3
    eta2, s = beam_average(beta, x_R, x_b)
    psi = random_state((16,), n, 21)
    rho_ratio = 1.0 / ((1.0 + x_R) ** 2 * (1.0 + x_b))
    out, xi, flags = ea.energy_advect(psi, e, rho_old=1.0, rho_new=rho_ratio, dlnR=x_R, dlnb=x_b,
                                      eddington=np.full((16, n), eta2))
    assert np.all(flags == 0)
    n0, e0 = ea.number_and_energy(psi, e)
    n1, e1 = ea.number_and_energy(out, e)
    assert np.allclose(n1, rho_ratio * n0, rtol=1e-14, atol=0)
    assert np.allclose((e1 / n1) / (e0 / n0), s, rtol=1e-13, atol=0)


def test_eq_a79_pin_catches_a_sign_flip_of_the_eddington_term(monkeypatch):
    """A planted sign error in the (db/b - dR/R) eta2 term of eq. a79 fails the beam-average pin."""
    def flipped(e_edge, dlna, dlnR, dlnb, eddington, shape):
        h = ea.edge_eddington(eddington, shape)
        dlna, dlnR, dlnb = (np.asarray(x, dtype=np.float64)[..., None] for x in (dlna, dlnR, dlnb))
        return (1.0 + (dlna - dlnR) + (dlnb - dlnR) * h) * e_edge
    monkeypatch.setattr(ea, "lagrangian_displacement", flipped)
    with pytest.raises(AssertionError):
        test_eq_a79_energy_shift_is_the_beam_average(2.0)


def test_eq_a79_per_group_eddington_factors():
    """Groups 0-9 with one angular distribution and 10-19 with another: the edges inside each set move by
    that set's beam average, the edge between them by the mean of the two (its Eddington factor is the
    mean of its groups' and eq. a79 is linear in it), and the end edges by their group's.  The energy
    after the step is the number of each displaced group (eq. a78) at its displaced centre (eq. a01),
    which the remap keeps."""
    n = 20
    e = np.geomspace(2.0, 300.0, n + 1)
    x_R, x_b = 4e-3, -6e-3
    (h_lo, s_lo), (h_hi, s_hi) = beam_average(0.5, x_R, x_b), beam_average(12.0, x_R, x_b)
    edd = np.where(np.arange(n) < 10, h_lo, h_hi)[None, :].repeat(8, 0)
    psi = random_state((8,), n, 22)
    rho_ratio = 1.0 / ((1.0 + x_R) ** 2 * (1.0 + x_b))
    out, xi, flags = ea.energy_advect(psi, e, rho_new=rho_ratio, dlnR=x_R, dlnb=x_b, eddington=edd)
    assert np.all(flags == 0)
    s_edge = np.where(np.arange(n + 1) < 10, s_lo, s_hi)
    s_edge[10] = 0.5 * (s_lo + s_hi)
    moved = e * s_edge
    N_moved = rho_ratio * ea.weights(e) * psi
    e_expected = np.sum(N_moved * ea.centers(moved), axis=-1)
    n1, e1 = ea.number_and_energy(out, e)
    assert np.allclose(n1, N_moved.sum(-1), rtol=1e-14, atol=0)
    assert np.allclose(e1, e_expected, rtol=1e-13, atol=0)


def test_lagrangian_lapse_change_equals_homologous_compression():
    """In eq. a79 the lapse enters as da/a - dR/R and in eq. a78 through rho a^3: a lapse change
    a^{n+1}/a^n = 1 + x at fixed rho, R and b is the same update as a homologous compression
    dR/R = db/b = -x with rho^{n+1}/rho^n = (1 + x)^3 at a fixed lapse, whatever the Eddington factors
    (the eta2 term vanishes for both), and shifts the mean energy by exactly 1 + x."""
    n = 20
    e = np.geomspace(2.0, 300.0, n + 1)
    psi = random_state((12,), n, 23)
    edd = np.clip(np.random.default_rng(24).uniform(1 / 3, 1.0, (12, n)), 1 / 3, 1.0)
    x = 7e-3
    a0 = np.random.default_rng(25).uniform(0.7, 0.95, 12)
    lap, _, fl_a = ea.energy_advect(psi, e, a_old=a0, a_new=a0 * (1.0 + x), eddington=edd)
    hom, _, fl_h = ea.energy_advect(psi, e, rho_new=(1.0 + x) ** 3, dlnR=-x, dlnb=-x, eddington=edd)
    assert np.all(fl_a == 0) and np.all(fl_h == 0)
    assert np.allclose(lap, hom, rtol=1e-13, atol=1e-15)
    n0, e0 = ea.number_and_energy(psi, e)
    n1, e1 = ea.number_and_energy(lap, e)
    assert np.allclose(n1, (1.0 + x) ** 3 * n0, rtol=1e-14, atol=0)
    assert np.allclose((e1 / n1) / (e0 / n0), 1.0 + x, rtol=1e-13, atol=0)


# ---------------------------------------------------------------- float64 rounding of the update

def gpu_test_inputs(S, R, I, N, seed, scale=1.0, psi_hi=0.9):
    """The recipe of the device parity test: Fermi-Dirac spectra, percent-level rho/lapse/radius changes,
    group- and zone-dependent Eddington factors."""
    r = np.random.default_rng(seed)
    e_edge = 2.0 * 150.0 ** (np.arange(N + 1) / N)
    eps = ea.centers(e_edge)
    T = r.uniform(3.0, 12.0, (S, R, I, 1))
    psi = psi_hi / (np.exp((eps - 2.0 * T) / T) + 1.0)
    rho_old = r.uniform(1e8, 1e12, (R, I))
    rho_new = rho_old * (1.0 + 0.01 * scale * r.standard_normal((R, I)))
    a_old = r.uniform(0.8, 0.99, (R, I))
    a_new = a_old * (1.0 + 0.005 * scale * r.standard_normal((R, I)))
    dlnR = 0.01 * scale * r.standard_normal((R, I))
    dlnb = 0.01 * scale * r.standard_normal((R, I))
    edd = np.clip(1.0 / 3.0 + 0.3 * r.uniform(0, 1, (S, R, I, 1)) * np.linspace(0, 1, N), 1 / 3, 1)
    return dict(e_edge=e_edge, psi=psi, rho_old=rho_old, rho_new=rho_new, a_old=a_old, a_new=a_new,
                dlnR=dlnR, dlnb=dlnb, edd=edd)


@pytest.mark.parametrize("shape", [(2, 3, 40, 20), (1, 4, 30, 13), (1, 2, 50, 8)])
def test_float64_rounding_of_the_update_is_zone_relative(shape):
    """The update of the oracle in float64 against the same steps in long double (np.longdouble, 64-bit
    mantissa): the difference of each group is a few ulp of its zone's largest occupation (below 1e-13 of
    it), while relative to the group itself it reaches far more in tail groups whose inflow and outflow
    nearly cancel.  This is why the device parity bar for psi is zone-relative (1e-12), and xi's relative
    rounding of about 2^-53 / |s - 1| is why its bar is 1e-8."""
    d = gpu_test_inputs(*shape, seed=sum(shape))
    ld = {k: np.asarray(v, dtype=np.longdouble) for k, v in d.items()}
    kw = lambda z: dict(rho_old=z["rho_old"], rho_new=z["rho_new"], a_old=z["a_old"], a_new=z["a_new"],  # noqa: E731
                        dlnR=z["dlnR"], dlnb=z["dlnb"], eddington=z["edd"])
    p64, xi64, f64 = ea.energy_advect(d["psi"], d["e_edge"], **kw(d))
    pld, xild, fld = ea.energy_advect(ld["psi"], ld["e_edge"], **kw(ld))
    assert pld.dtype == np.longdouble
    assert np.array_equal(f64, fld)
    pld = pld.astype(np.float64)
    scale = np.maximum(np.abs(pld).max(-1, keepdims=True), 1e-30)
    zone = float(np.max(np.abs(p64 - pld) / scale))
    own = float(np.max(np.abs(p64 - pld) / np.maximum(np.abs(pld), 1e-30)))
    xrel = float(np.max(np.abs(xi64 - xild.astype(np.float64)) / np.abs(xild.astype(np.float64))))
    assert zone < 1e-13
    assert own > 10.0 * zone          # relative to the group itself the rounding is far larger
    assert xrel < 1e-9
