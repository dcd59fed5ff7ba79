"""FP64 CPU oracle of the implicit MGFLD transport step (test infrastructure only).

Notation follows the paper (CHIMERA, arXiv 1809.05608):
  psi      zeroth angular moment psi^(0) of the occupation (dimensionless)
  H        first moment psi^(1) at a zone edge (the flux, eq. a59)
  lambda   transport mean free path (eq. a17), 1/lambda = kappa_a + eta + kappa_s
           (absorption plus emission inverse mean free paths, eq. d10, plus the
           isoenergetic scattering opacity, eq. d8c)
  F        flux limiter: F_intrp (eq. a20), or min(F_intrp, F_geom) (eqs. a23-a26a)
  R_nu     neutrinosphere radius of a group (eqs. a23, a25, a62af)
  V_i, A   zone volume and edge area with the common 4*pi dropped and Gamma = 1
  eps_k    group-centre energies (eq. a01), W_k = eps_k^2 d eps_k (eq. a01b)
The lapse a is 1 (no lapse input), so E = eps (eq. a8a).

One "system" is one (species, ray): I radial zones x N energy groups.  The
unknowns are psi^{n+1}_{i,k}; the residual is c*dt times eq. a58 with the
source of eq. a54 (emission/absorption with Pauli blocking) and the zeroth
moment of eq. d8 / eq. d40 (inelastic NES-like scattering, Phi_0 terms).

Readings where the paper is silent or garbled:
  * eq. a01 prints eps_k instead of eps_k^2 on the left; the square is restored
    so that eq. a01b holds.
  * the limiter's psi in eq. a20 is the edge mean (psi_i + psi_{i+1})/2, floored
    at psi_floor; |d psi/dR| uses the same one-sided difference as eq. a59.
  * limiter 1 is F_intrp alone; limiter 2 is F = min(F_intrp, F_geom) (eq. a26a) with R_nu(eps_k)
    an input.  In F_geom (eq. a23) the comoving limb cosine is the fixed-frame one (beta = 0 in eq.
    a24: the transport step takes no matter velocity) without ray bending (G = 1 in eq. a26: no
    gravitational mass is an input), psi^(0) at the edge is the same floored edge mean as in F_intrp,
    and R is the edge radius; inside the neutrinosphere (R <= R_nu) F_geom = 1.
  * outer boundary 1 is free streaming, psi^(1) = psi^(0) of the last zone (the limit of eq. a22);
    outer boundary 2 is the paper's constant-luminosity condition (eq. a62af) with the neutrinosphere
    radius squared (the printed 1/4 R_nu is read as 1/4 R_nu^2, the first-order form of
    (1 + mu_nu) R^2 / 2): a ghost zone I+1 centred at the mirror of the last zone's centre across the
    outer edge, holding psi_{I+1} = psi_I (R_I^2 - R_nu^2/4) / (R_{I+1}^2 - R_nu^2/4) (the ratio
    clipped to [0, 1]), with the last zone's mean free path; the outer flux is then the ordinary
    limited edge flux of eq. a59 between zone I and the ghost.  Boundary 0 is zero flux; the inner
    boundary has zero flux.
  * NES enters moment 0 through the Phi_0 terms only and is excluded from the
    transport opacity, so the off-diagonal radial blocks stay diagonal (eq. a62ae).
  * the NES kernel obeys the in/out symmetry (eq. d3) in the weighted discrete
    form W_k K^in_{kk'} = W_k' K^out_{k'k} and detailed balance (eq. d4), with the
    directly computed part carrying a min(1, e^{-x}) factor.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.linalg

EPS0_MEV = 10.0          # NES reference energy (kernel scale eps_k eps_k' / eps0^2)
C_LIGHT = 2.99792458e10  # cm/s, used only for the luminosity (number per unit time)

TERM_DIFFUSION = 1
TERM_EMABS = 2
TERM_NES = 4

LIMITER_NONE, LIMITER_INTRP, LIMITER_GEOM = 0, 1, 2
BC_ZERO_FLUX, BC_FREE_STREAM, BC_GEOMETRIC = 0, 1, 2


@dataclasses.dataclass
class System:
    """Inputs of one (species, ray) system, all float64 numpy arrays."""
    r_edge: np.ndarray      # [I+1] cm
    e_edge: np.ndarray      # [N+1] MeV
    temp: np.ndarray        # [I] MeV
    kappa_a: np.ndarray     # [I][N] cm^-1
    eta: np.ndarray         # [I][N] cm^-1 (emissivity j)
    kappa_s: np.ndarray     # [I][N] cm^-1
    nes_amp: np.ndarray     # [I] cm^-1
    nes_g: np.ndarray       # [N][N]
    c_dt: float             # cm
    inner_bc: int = 0
    outer_bc: int = 1
    terms: int = 7
    limiter: int = 1
    psi_floor: float = 1e-300
    lapse: Optional[np.ndarray] = None        # [I] lapse a_i at zone centres (None: a = 1)
    lapse_edge: Optional[np.ndarray] = None   # [I+1] lapse at zone edges
    r_nu: Optional[np.ndarray] = None         # [N] neutrinosphere radius R_nu(eps_k), cm (limiter 2, outer_bc 2)

    @property
    def I(self) -> int:
        return self.kappa_a.shape[0]

    @property
    def N(self) -> int:
        return self.kappa_a.shape[1]


def systems_from_workload(w: dict) -> List[List[System]]:
    """Split workload arrays (layouts [S][R][I][N], [R][I], [S][R][I]) into systems[s][r]."""
    out = []
    for s in range(w["S"]):
        row = []
        for r in range(w["R"]):
            row.append(System(
                r_edge=w["r_edge"][r], e_edge=w["e_edge"], temp=w["temp"][r],
                kappa_a=w["kappa_a"][s, r], eta=w["eta"][s, r], kappa_s=w["kappa_s"][s, r],
                nes_amp=w["nes_amp"][s, r], nes_g=w["nes_g"], c_dt=w["c_dt"],
                inner_bc=w["inner_bc"], outer_bc=w["outer_bc"], terms=w["terms"],
                limiter=w["limiter"], psi_floor=w["psi_floor"],
                lapse=w["lapse"][r] if w.get("lapse") is not None else None,
                lapse_edge=w["lapse_edge"][r] if w.get("lapse_edge") is not None else None,
                r_nu=w["r_nu"][s] if w.get("r_nu") is not None else None))
        out.append(row)
    return out


# ---------------------------------------------------------------- grids

def group_energies(e_edge: np.ndarray):
    """Group centres eps_k (eq. a01 with eps_k^2 on the left) and weights W_k (eq. a01b)."""
    lo, hi = e_edge[:-1], e_edge[1:]
    eps = np.sqrt((hi ** 2 + hi * lo + lo ** 2) / 3.0)
    W = (hi ** 3 - lo ** 3) / 3.0
    return eps, W


def geometry(r_edge: np.ndarray):
    """Zone centres R_i, volumes V_i, edge areas A_{i+1/2}, centre distances D_{i+1/2}.

    Definitions stated after eq. a59: R_i is the mean of its edges, V_i the shell
    volume and A the edge area, the common 4*pi dropped and Gamma = 1.
    Returns R [I], V [I], A [I+1] (edge 0 is the inner edge), D [I-1] (interior edges).
    """
    Rc = 0.5 * (r_edge[:-1] + r_edge[1:])
    V = (r_edge[1:] ** 3 - r_edge[:-1] ** 3) / 3.0
    A = r_edge ** 2
    D = Rc[1:] - Rc[:-1]
    return Rc, V, A, D


# ---------------------------------------------------------------- physics pieces

def nes_kernels(amp: float, T: float, eps: np.ndarray, W: np.ndarray, G: np.ndarray):
    """Out/in NES kernels K^out_{kk'}, K^in_{kk'} of one zone (Phi_0 terms of eq. d8).

    K^out_{kk'} = amp (eps_k eps_k'/eps0^2) G_{kk'} (W_k'/Wbar) min(1, exp(-(eps_k' - eps_k)/T))
    K^in_{kk'}  = amp (eps_k eps_k'/eps0^2) G_{kk'} (W_k'/Wbar) min(1, exp(+(eps_k' - eps_k)/T))
    so that K^in/K^out = exp((eps_k' - eps_k)/T) (detailed balance, eq. d4) and
    W_k K^in_{kk'} = W_k' K^out_{k'k} (in/out symmetry, eq. d3, with the phase-space
    weight of the discrete sum of eq. d40).
    """
    Wbar = W.mean()
    base = amp * np.outer(eps, eps) / EPS0_MEV ** 2 * G * (W / Wbar)[None, :]
    x = (eps[None, :] - eps[:, None]) / T          # (eps_k' - eps_k)/T, row k, column k'
    k_out = base * np.exp(np.minimum(-x, 0.0))     # min(1, e^{-x})
    k_in = base * np.exp(np.minimum(x, 0.0))       # min(1, e^{+x})
    return k_out, k_in


def limb_factor(R, r_nu):
    """(1 + mu_nu)/2 at radius R for neutrinosphere radii r_nu [N] (eqs. a24-a26 with beta = 0 and
    G = 1): mu_nu = sqrt(1 - (R_nu/R)^2).  NaN where R <= R_nu (no geometric limit inside the
    neutrinosphere, F_geom = 1)."""
    r_nu = np.asarray(r_nu, dtype=np.float64)
    out = np.full(r_nu.shape, np.nan)
    outside = R > r_nu
    out[outside] = 0.5 * (1.0 + np.sqrt(1.0 - (r_nu[outside] / R) ** 2))
    return out


def edge_flux(u, v, lam, D, floor, limiter=1, limb=None):
    """Flux H = psi^(1) at an edge and its partial derivatives.

    eq. a59 with the limiter of eq. a20 (Gamma = 1):
        H = -(lam/3) F (v - u)/D,   F = [1 + lam |v - u| / (3 D m)]^{-1},
        m = max((u + v)/2, floor)
    i.e. H = -lam m (v - u) / (3 D m + lam |v - u|).  With limiter=0, F = 1.  With limiter=2,
    F = min(F_intrp, F_geom) (eq. a26a), F_geom = limb m / ((1/3) lam |v - u| / D) (eq. a23) where
    limb = (1 + mu_nu)/2 is finite (outside the neutrinosphere) and F_geom = 1 elsewhere; where
    F_geom is the smaller, H = -limb m sign(v - u) (eq. a26b), independent of lam.
    Returns H, dH/du, dH/dv, dH/dlam (arrays over groups).
    """
    delta = v - u
    if limiter == 0:
        H = -lam * delta / (3.0 * D)
        dH_dd = -lam / (3.0 * D)
        return H, -dH_dd, dH_dd, -delta / (3.0 * D)
    mean = 0.5 * (u + v)
    m = np.maximum(mean, floor)
    above = (mean > floor).astype(np.float64)
    den = 3.0 * D * m + lam * np.abs(delta)
    r = m / den
    q = delta / den
    H = -lam * delta * r
    dH_ddelta = -3.0 * D * lam * r * r            # d/d(delta) at fixed m
    dH_dm = -lam * lam * q * np.abs(q) * above     # d/dm at fixed delta
    dH_du = -dH_ddelta + 0.5 * dH_dm
    dH_dv = dH_ddelta + 0.5 * dH_dm
    dH_dlam = -3.0 * D * delta * r * r
    if limiter == 2:
        if limb is None:
            raise ValueError("limiter 2 needs the neutrinosphere radii")
        limb = np.broadcast_to(np.asarray(limb, dtype=np.float64), np.shape(H))
        ad = np.abs(delta)
        F_intrp = 3.0 * D * m / den
        with np.errstate(divide="ignore", invalid="ignore"):
            F_geom = np.where(np.isfinite(limb) & (ad > 0), limb * m / (lam * ad / (3.0 * D)), 1.0)
        F = np.minimum(F_intrp, F_geom)
        geom = F_geom < F_intrp
        sgn = np.sign(delta)
        H = np.where(geom, -lam / 3.0 * F * delta / D, H)
        g = np.where(geom, limb, 0.0)
        dH_du = np.where(geom, -0.5 * g * sgn * above, dH_du)
        dH_dv = np.where(geom, -0.5 * g * sgn * above, dH_dv)
        dH_dlam = np.where(geom, 0.0, dH_dlam)
    return H, dH_du, dH_dv, dH_dlam


def outer_ghost(sys: System):
    """Ghost zone of the geometric outer boundary (eq. a62af with R_nu^2): its centre R_{I+1}, the ratio
    psi_{I+1}/psi_I = (R_I^2 - R_nu^2/4) / (R_{I+1}^2 - R_nu^2/4) per group (clipped to [0, 1]), and the
    distance D = R_{I+1} - R_I of the outer edge."""
    if sys.r_nu is None:
        raise ValueError("the geometric outer boundary needs the neutrinosphere radii")
    Rc = geometry(sys.r_edge)[0]
    R_I = Rc[-1]
    R_g = 2.0 * sys.r_edge[-1] - R_I
    q = 0.25 * np.asarray(sys.r_nu, dtype=np.float64) ** 2
    den = R_g ** 2 - q
    ratio = np.where(den > 0, np.clip((R_I ** 2 - q) / np.where(den > 0, den, 1.0), 0.0, 1.0), 0.0)
    return R_g, ratio, R_g - R_I


def lapse_factors(sys: System):
    """Lapse at zone centres a_i [I] and edges a_{i+1/2} [I+1] (ones without a lapse).

    With a lapse, eq. a58 times a_i c dt puts a_i^3 / V_i in front of the flux difference, the edge
    areas become A_{i+1/2} / a_{i+1/2}^2, and the emission/absorption and NES sources carry a_i.  The
    energy grid e_edge then holds energies at infinity E (eq. a8a): a zone's groups sit at the local
    energies E / a_i, at which the opacities are given and the NES kernels evaluated."""
    I = sys.kappa_a.shape[0]
    a = np.ones(I) if sys.lapse is None else np.asarray(sys.lapse, dtype=np.float64)
    ae = np.ones(I + 1) if sys.lapse_edge is None else np.asarray(sys.lapse_edge, dtype=np.float64)
    if (sys.lapse is None) != (sys.lapse_edge is None):
        raise ValueError("lapse and lapse_edge go together")
    return a, ae


def _weights(sys: System):
    """Per-zone factor a_i^3 / V_i of the flux difference and per-edge areas A / a^2 (eq. a58)."""
    _, V, A, _ = geometry(sys.r_edge)
    a, ae = lapse_factors(sys)
    return a ** 3 / V, A / ae ** 2, a


def _lambda(sys: System):
    return 1.0 / (sys.kappa_a + sys.eta + sys.kappa_s)


def _edge_fluxes(sys: System, psi: np.ndarray):
    """H at all I+1 edges [I+1][N] plus derivatives at interior edges."""
    I, N = psi.shape
    _, _, _, D = geometry(sys.r_edge)
    lam = _lambda(sys)
    H = np.zeros((I + 1, N))
    dHu = np.zeros((I + 1, N))
    dHv = np.zeros((I + 1, N))
    dHl = np.zeros((I + 1, N))
    lam_e = np.zeros((I + 1, N))
    def limb(e):
        return limb_factor(sys.r_edge[e], sys.r_nu) if sys.limiter == LIMITER_GEOM else None

    for e in range(1, I):                            # edge e = i + 1/2 between zones e-1 and e
        lam_e[e] = np.sqrt(lam[e - 1] * lam[e])     # geometric mean, stated after eq. a59
        H[e], dHu[e], dHv[e], dHl[e] = edge_flux(psi[e - 1], psi[e], lam_e[e], D[e - 1],
                                                 sys.psi_floor, sys.limiter, limb(e))
    # inner boundary: zero flux (H[0] = 0).  Outer boundary:
    if sys.outer_bc == BC_FREE_STREAM:
        H[I] = psi[I - 1]                            # free streaming, psi^(1) = psi^(0)
        dHu[I] = 1.0
    elif sys.outer_bc == BC_GEOMETRIC:               # ghost zone of eq. a62af
        _, ratio, D_out = outer_ghost(sys)
        lam_e[I] = lam[I - 1]
        H[I], du, dv, dHl[I] = edge_flux(psi[I - 1], ratio * psi[I - 1], lam_e[I], D_out,
                                         sys.psi_floor, sys.limiter, limb(I))
        dHu[I] = du + ratio * dv                     # the ghost value moves with psi_I
    return H, dHu, dHv, dHl, lam_e


def nes_source(sys: System, psi: np.ndarray, unit_amplitude: bool = False):
    """S_{i,k}: zeroth moment of the NES collision term (eq. d8, Phi_0 terms; eq. d40), with the kernels
    at the zone's local energies (E / a_i with a lapse)."""
    I, N = psi.shape
    eps, W = group_energies(sys.e_edge)
    a, _ = lapse_factors(sys)
    S = np.zeros((I, N))
    for i in range(I):
        amp = 1.0 if unit_amplitude else sys.nes_amp[i]
        k_out, k_in = _off_diagonal(*nes_kernels(amp, sys.temp[i], eps / a[i], W, sys.nes_g))
        p = psi[i]
        S[i] = (1.0 - p) * (k_in @ p) - p * (k_out @ (1.0 - p))
    return S


def _off_diagonal(*kernels):
    """Kernels without the k' = k terms.  Scattering that keeps the energy group has no
    zeroth-moment source (eq. d8b): its in and out terms cancel identically, so they are
    left out rather than summed and cancelled in floating point."""
    out = []
    for K in kernels:
        K = K.copy()
        np.fill_diagonal(K, 0.0)
        out.append(K)
    return out


# ---------------------------------------------------------------- residual and Jacobian

def residual(sys: System, psi_n: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """G(psi) = a_i c dt times eq. a58, per cell [I][N] (a = 1 without a lapse).

    G_{i,k} = psi - psi^n + c dt { a_i^3 (A_{i+1/2} H_{i+1/2} / a_{i+1/2}^2 - A_{i-1/2} H_{i-1/2} / a_{i-1/2}^2) / V_i
                                   + a_i [ - eta (1 - psi) + kappa_a psi - S_{i,k} ] }
    """
    vf, Aw, a = _weights(sys)
    G = psi - psi_n
    if sys.terms & TERM_DIFFUSION:
        H = _edge_fluxes(sys, psi)[0]
        G = G + sys.c_dt * (Aw[1:, None] * H[1:] - Aw[:-1, None] * H[:-1]) * vf[:, None]
    if sys.terms & TERM_EMABS:
        G = G + sys.c_dt * a[:, None] * (-sys.eta * (1.0 - psi) + sys.kappa_a * psi)
    if sys.terms & TERM_NES:
        G = G - sys.c_dt * a[:, None] * nes_source(sys, psi)
    return G


def jacobian_blocks(sys: System, psi: np.ndarray):
    """Exact Jacobian of G in block-tridiagonal form (eq. a62ae).

    Returns A [I][N][N] (dense diagonal blocks), bm [I][N], bp [I][N] (the diagonal
    off-diagonal blocks coupling zone i to zones i-1 and i+1).
    """
    I, N = psi.shape
    vf, Aed, a = _weights(sys)
    eps, W = group_energies(sys.e_edge)
    c = sys.c_dt
    blocks = np.zeros((I, N, N))
    bm = np.zeros((I, N))
    bp = np.zeros((I, N))
    diag = np.ones((I, N))
    if sys.terms & TERM_DIFFUSION:
        _, dHu, dHv, _, _ = _edge_fluxes(sys, psi)
        for i in range(I):
            # G_i contains +A_{i+1/2} H_{i+1/2}(psi_i, psi_{i+1}) - A_{i-1/2} H_{i-1/2}(psi_{i-1}, psi_i)
            diag[i] += c * (Aed[i + 1] * dHu[i + 1] - Aed[i] * dHv[i]) * vf[i]
            if i + 1 < I:
                bp[i] = c * Aed[i + 1] * dHv[i + 1] * vf[i]
            if i > 0:
                bm[i] = -c * Aed[i] * dHu[i] * vf[i]
    if sys.terms & TERM_EMABS:
        diag += c * a[:, None] * (sys.eta + sys.kappa_a)
    for i in range(I):
        blocks[i][np.diag_indices(N)] = diag[i]
        if sys.terms & TERM_NES:
            k_out, k_in = _off_diagonal(*nes_kernels(sys.nes_amp[i], sys.temp[i], eps / a[i], W, sys.nes_g))
            p = psi[i]
            ca = c * a[i]
            # -c a dS_k/dpsi_m : dense part for every m (the m = k term included) ...
            blocks[i] -= ca * ((1.0 - p)[:, None] * k_in + p[:, None] * k_out)
            # ... plus the diagonal derivative through the explicit (1 - psi_k), psi_k factors
            blocks[i][np.diag_indices(N)] += ca * (k_in @ p + k_out @ (1.0 - p))
    return blocks, bm, bp


def dense_jacobian(sys: System, psi: np.ndarray) -> np.ndarray:
    """The full (I*N) x (I*N) Jacobian, row/column index i*N + k."""
    blocks, bm, bp = jacobian_blocks(sys, psi)
    I, N = psi.shape
    J = np.zeros((I * N, I * N))
    for i in range(I):
        J[i * N:(i + 1) * N, i * N:(i + 1) * N] = blocks[i]
        if i > 0:
            J[i * N:(i + 1) * N, (i - 1) * N:i * N] = np.diag(bm[i])
        if i + 1 < I:
            J[i * N:(i + 1) * N, (i + 1) * N:(i + 2) * N] = np.diag(bp[i])
    return J


# ---------------------------------------------------------------- linear solves

def block_thomas_solve(blocks, bm, bp, rhs, transpose: bool = False):
    """Solve J x = rhs (or J^T x = rhs) by block-Thomas elimination.

    Forward sweep: Ahat_i = A_i - diag(bm_i) C_{i-1}, y_i = Ahat_i^{-1}(rhs_i - bm_i * y_{i-1}),
    C_i = Ahat_i^{-1} diag(bp_i), each Ahat_i factored by LU with partial pivoting.
    Back substitution: x_{I-1} = y_{I-1}, x_i = y_i - C_i x_{i+1}.
    J^T has blocks A_i^T and off-diagonals bp_{i-1} (below) and bm_{i+1} (above).
    """
    I, N = rhs.shape
    if transpose:
        blocks = np.transpose(blocks, (0, 2, 1))
        lower = np.zeros_like(bm)
        upper = np.zeros_like(bp)
        lower[1:] = bp[:-1]
        upper[:-1] = bm[1:]
        bm, bp = lower, upper
    C = np.zeros((I, N, N))
    y = np.zeros((I, N))
    for i in range(I):
        Ahat = blocks[i].copy()
        g = rhs[i].copy()
        if i > 0:
            Ahat -= bm[i][:, None] * C[i - 1]
            g -= bm[i] * y[i - 1]
        lu = scipy.linalg.lu_factor(Ahat)
        y[i] = scipy.linalg.lu_solve(lu, g)
        C[i] = scipy.linalg.lu_solve(lu, np.diag(bp[i]))
    x = np.zeros((I, N))
    x[I - 1] = y[I - 1]
    for i in range(I - 2, -1, -1):
        x[i] = y[i] - C[i] @ x[i + 1]
    return x


def dense_solve(sys: System, psi: np.ndarray, rhs: np.ndarray, transpose: bool = False):
    """Second, independent route: assemble the dense J and call LAPACK (numpy.linalg.solve)."""
    J = dense_jacobian(sys, psi)
    if transpose:
        J = J.T
    return np.linalg.solve(J, rhs.reshape(-1)).reshape(rhs.shape)


# ---------------------------------------------------------------- Newton iteration

@dataclasses.dataclass
class NewtonResult:
    psi: np.ndarray
    iters: int
    res0: float
    res: float
    converged: bool
    history: list


ARMIJO_C = 1e-4          # sufficient-decrease constant of the backtracking line search
ALPHA_MIN = 2.0 ** -8    # shortest step tried before a step is taken regardless


def newton(sys: System, psi_n: np.ndarray, psi0: Optional[np.ndarray] = None,
           max_iter: int = 30, rtol: float = 0.0) -> NewtonResult:
    """Backward-Euler Newton iteration (eq. a62aa) for psi^{n+1} of one system.

    Starts from psi0 (default psi^n).  Each update solves J delta = -G (eq. a62ae) and is
    globalised by backtracking on r = max|G|: the trial psi + delta is accepted when
    r_trial <= (1 - 1e-4 alpha) r, else alpha is halved (the trial becomes psi + alpha delta)
    down to alpha = 2^-8, which is taken regardless.  Within 1000x
    of the target (the rounding level of G when rtol = 0) a full step is taken without the test.  The paper's scheme is plain
    Newton; without the line search the strongly spiked stress rays diverge (psi overshoots
    the Pauli limit 1 and the residual grows), with it they converge quadratically.
    Stopping (rtol > 0): r <= target = max(rtol r_0, rounding level of G), or no halving of r
    within 1000x of the target; rtol = 0 runs exactly max_iter updates.
    """
    psi = (psi_n if psi0 is None else psi0).copy()
    G = residual(sys, psi_n, psi)
    r = float(np.max(np.abs(G)))
    res0 = r
    hist = [r]
    iters = 0
    prev = np.inf
    target = 0.0
    for _ in range(max_iter):
        if r == 0.0 or not np.isfinite(r):
            break
        target = max(rtol * res0, residual_rounding_level(sys, psi_n, psi))
        if rtol > 0.0 and (r <= target or (r <= 1e3 * target and r > 0.5 * prev)):
            break              # reached, or stalled: the update is below the resolution of psi
        blocks, bm, bp = jacobian_blocks(sys, psi)
        delta = block_thomas_solve(blocks, bm, bp, -G)
        iters += 1
        trial = psi + delta
        alpha = 1.0
        Gt = residual(sys, psi_n, trial)
        rt = float(np.max(np.abs(Gt)))
        near = r <= 1e3 * target
        while not near and not rt <= (1.0 - ARMIJO_C * alpha) * r and alpha > ALPHA_MIN:
            alpha = 0.5 * alpha
            trial = psi + alpha * delta
            Gt = residual(sys, psi_n, trial)
            rt = float(np.max(np.abs(Gt)))
        prev = r
        psi, G, r = trial, Gt, rt
        hist.append(r)
    if rtol > 0.0:
        target = max(rtol * res0, residual_rounding_level(sys, psi_n, psi))
    conv = (r <= target) if rtol > 0.0 else True
    return NewtonResult(psi=psi, iters=iters, res0=res0, res=r, converged=bool(conv), history=hist)


def residual_rounding_level(sys: System, psi_n: np.ndarray, psi: np.ndarray) -> float:
    """32 ulp of the largest per-cell sum of the magnitudes of G's terms plus |psi| |dG/dpsi|.

    G is a sum of terms that nearly cancel near the solution, and a change of psi by one
    ulp moves G by about |dG/dpsi| ulp(psi); below this level the computed residual is
    rounding, so the stopping rule asks for no progress beyond it.
    """
    vf, A, a = _weights(sys)
    c = sys.c_dt
    mag = np.abs(psi) + np.abs(psi_n)
    jd = np.ones_like(psi)              # bound of |dG_ik/dpsi_ik|
    if sys.terms & TERM_DIFFUSION:
        H, dHu, dHv, _, _ = _edge_fluxes(sys, psi)
        mag = mag + c * (np.abs(A[1:, None] * H[1:]) + np.abs(A[:-1, None] * H[:-1])) * vf[:, None]
        jd = jd + c * (A[1:, None] * np.abs(dHu[1:]) + A[:-1, None] * np.abs(dHv[:-1])) * vf[:, None]
    if sys.terms & TERM_EMABS:
        mag = mag + c * a[:, None] * (np.abs(sys.kappa_a * psi) + np.abs(sys.eta * (1.0 - psi)))
        jd = jd + c * a[:, None] * (sys.kappa_a + sys.eta)
    if sys.terms & TERM_NES:
        eps, W = group_energies(sys.e_edge)
        for i in range(psi.shape[0]):
            k_out, k_in = _off_diagonal(*nes_kernels(sys.nes_amp[i], sys.temp[i], eps / a[i], W, sys.nes_g))
            p = psi[i]
            si, so = k_in @ p, k_out @ (1.0 - p)
            mag[i] += c * a[i] * (np.abs(1.0 - p) * np.abs(si) + np.abs(p) * np.abs(so))
            jd[i] += c * a[i] * (np.abs(si) + np.abs(so))
    mag = mag + np.abs(psi) * jd
    return 32.0 * np.finfo(np.float64).eps * float(np.max(mag))


# ---------------------------------------------------------------- conservation sums and luminosity

def step_stats(sys: System, psi_n: np.ndarray, psi: np.ndarray) -> dict:
    """FP64 sums of one system (number conservation, eqs. a60-a62).

    n_tot   = sum_i V_i sum_k W_k psi_{i,k}         (neutrino number, constants dropped)
    e_tot   = sum_i V_i sum_k W_k eps_k psi_{i,k}   (energy)
    q_n     = c dt sum V W [eta (1 - psi) - kappa_a psi]   (emission minus absorption)
    nes_n   = c dt sum V W S                          (NES number source, zero by eq. d3)
    b_n     = c dt A_{I+1/2} sum_k W_k H_{I+1/2,k}     (number through the outer surface)
    budget  = n_tot - n_tot^n + b_n - q_n - nes_n    (equals sum V W G)
    lum_n   = c A_{I+1/2} sum_k W_k H_{I+1/2,k}        (number luminosity, 4pi and (hc)^-3 dropped)
    With a lapse, V_i becomes V_i / a_i^3 (the local phase-space weight is W / a^3), A_{I+1/2} becomes
    A_{I+1/2} / a_{I+1/2}^2, the sources carry a_i, and e_tot is the energy at infinity (E = a eps).
    """
    vf, A, a = _weights(sys)
    eps, W = group_energies(sys.e_edge)
    I, N = psi.shape
    VW = (1.0 / vf)[:, None] * W[None, :]
    n_tot = float(np.sum(VW * psi))
    n_old = float(np.sum(VW * psi_n))
    e_tot = float(np.sum(VW * eps[None, :] * psi))
    q_n = float(sys.c_dt * np.sum(VW * a[:, None] * (sys.eta * (1.0 - psi) - sys.kappa_a * psi))) \
        if sys.terms & TERM_EMABS else 0.0
    nes_n = float(sys.c_dt * np.sum(VW * a[:, None] * nes_source(sys, psi))) if sys.terms & TERM_NES else 0.0
    if sys.terms & TERM_DIFFUSION and sys.outer_bc != BC_ZERO_FLUX:
        h_out = _edge_fluxes(sys, psi)[0][I]
    else:
        h_out = np.zeros(N)
    b_n = float(sys.c_dt * A[I] * np.sum(W * h_out))
    return dict(n_tot=n_tot, e_tot=e_tot, q_n=q_n, nes_n=nes_n, b_n=b_n,
                budget=n_tot - n_old + b_n - q_n - nes_n,
                lum_n=float(C_LIGHT * A[I] * np.sum(W * h_out)))


def luminosity(sys: System, psi: np.ndarray) -> float:
    """L_N = c A_{I+1/2} sum_k W_k H_{I+1/2,k}: number leaving the outer surface per unit time (eq. a62;
    with a lapse A_{I+1/2} / a_{I+1/2}^2)."""
    _, A, _ = _weights(sys)
    _, W = group_energies(sys.e_edge)
    I = psi.shape[0]
    if not (sys.terms & TERM_DIFFUSION) or sys.outer_bc == BC_ZERO_FLUX:
        return 0.0
    return float(C_LIGHT * A[I] * np.sum(W * _edge_fluxes(sys, psi)[0][I]))


def luminosity_seed(sys: System, shape, psi: Optional[np.ndarray] = None) -> np.ndarray:
    """dL_N/dpsi as a cell array: nonzero only in the outermost zone.  The outer flux of the free-streaming
    boundary is psi_I itself; that of the geometric boundary depends on psi_I through the limited flux
    to the ghost zone, so its derivative needs the state psi."""
    _, A, _ = _weights(sys)
    _, W = group_energies(sys.e_edge)
    I, N = shape
    seed = np.zeros((I, N))
    if (sys.terms & TERM_DIFFUSION) and sys.outer_bc == BC_FREE_STREAM:
        seed[I - 1] = C_LIGHT * A[I] * W
    elif (sys.terms & TERM_DIFFUSION) and sys.outer_bc == BC_GEOMETRIC:
        if psi is None:
            raise ValueError("the geometric outer boundary's seed depends on psi")
        seed[I - 1] = C_LIGHT * A[I] * W * _edge_fluxes(sys, psi)[1][I]
    return seed


# ---------------------------------------------------------------- adjoint

def adjoint(sys: System, psi: np.ndarray, seed: np.ndarray, solver: str = "dense") -> np.ndarray:
    """mu solving J(psi)^T mu = seed: through the dense transpose (numpy.linalg.solve), or with
    solver="block" by the transposed block-Thomas elimination (the same system; the block route is
    pinned to the dense one, and serves full-size rays where a dense 10^4-square solve is slow)."""
    if solver == "block":
        blocks, bm, bp = jacobian_blocks(sys, psi)
        return block_thomas_solve(blocks, bm, bp, seed, transpose=True)
    return dense_solve(sys, psi, seed, transpose=True)


def param_vjp(sys: System, psi: np.ndarray, mu: np.ndarray) -> dict:
    """-mu^T dG/dtheta for theta in (kappa_a, eta, kappa_s, nes_amp, psi_n).

    dG/dkappa_a = c dt a_i psi and dG/deta = -c dt a_i (1 - psi) on the own cell (eq. a54 form
    times the lapse a_i of eq. a58, a = 1 without one); all three opacities also reach G_{i-1},
    G_i, G_{i+1} through lambda_i, the edge means lambda_{i+-1/2} = sqrt(lambda_i lambda_{i+-1})
    and the edge fluxes (eq. a59), with d lambda_e / d chi_i = -lambda_e lambda_i / 2 for
    chi = 1/lambda, each edge weighted by a^3/V of the zone and A/a^2 of the edge;
    dG/d amp_i = -c dt a_i S_{i,k}/amp_i; dG/dpsi^n = -1.
    """
    I, N = psi.shape
    vf, Aw, a = _weights(sys)         # a^3 / V per zone, A / a^2 per edge, a per zone
    c = sys.c_dt
    lam = _lambda(sys)
    g_chi = np.zeros((I, N))      # mu-weighted dG/dchi_i through the edge fluxes
    if sys.terms & TERM_DIFFUSION:
        _, _, _, dHl, lam_e = _edge_fluxes(sys, psi)
        for e in range(1, I):          # interior edge between zones e-1 and e
            # G_{e-1} += c (A/a^2)_e H_e (a^3/V)_{e-1};  G_e -= c (A/a^2)_e H_e (a^3/V)_e
            w = c * Aw[e] * (mu[e - 1] * vf[e - 1] - mu[e] * vf[e])     # mu-weighted dG/dH_e
            for zone in (e - 1, e):
                dlam_dchi = -0.5 * lam_e[e] * lam[zone]
                g_chi[zone] += w * dHl[e] * dlam_dchi
        # the geometric outer boundary's flux carries the last zone's mean free path (lam_e = lam_I)
        w_out = c * Aw[I] * mu[I - 1] * vf[I - 1]
        g_chi[I - 1] += w_out * dHl[I] * (-lam[I - 1] * lam[I - 1])
    g_ka = g_chi.copy()
    g_eta = g_chi.copy()
    g_ks = g_chi.copy()
    if sys.terms & TERM_EMABS:
        g_ka += mu * c * a[:, None] * psi
        g_eta += mu * (-c * a[:, None] * (1.0 - psi))
    g_amp = np.zeros(I)
    if sys.terms & TERM_NES:
        S1 = nes_source(sys, psi, unit_amplitude=True)
        g_amp = np.sum(mu * (-c * a[:, None] * S1), axis=1)
    return dict(kappa_a=-g_ka, eta=-g_eta, kappa_s=-g_ks, nes_amp=-g_amp, psi_n=mu.copy())


# ---------------------------------------------------------------- batch helpers

def newton_batch(w: dict, max_iter: int, rtol: float, systems=None):
    """Run `newton` on (s, r) systems of a workload dict; returns psi [S][R][I][N] and per-system info."""
    syss = systems_from_workload(w)
    psi = np.array(w["psi_n"], copy=True)
    info = {}
    pairs = systems if systems is not None else [(s, r) for s in range(w["S"]) for r in range(w["R"])]
    for s, r in pairs:
        res = newton(syss[s][r], w["psi_n"][s, r], max_iter=max_iter, rtol=rtol)
        psi[s, r] = res.psi
        info[(s, r)] = res
    return psi, info


def residual_batch(w: dict, psi: np.ndarray) -> np.ndarray:
    syss = systems_from_workload(w)
    G = np.zeros_like(psi)
    for s in range(w["S"]):
        for r in range(w["R"]):
            G[s, r] = residual(syss[s][r], w["psi_n"][s, r], psi[s, r])
    return G


# ---------------------------------------------------------------- multi-step objective and adjoint

def multistep_forward(systems: list, psi0: np.ndarray, max_iter: int = 40, rtol: float = 1e-14) -> list:
    """psi^1..psi^S of S consecutive implicit steps; step s uses systems[s] and psi^n = psi^{s-1}."""
    out = []
    psi = psi0
    for sysm in systems:
        psi = newton(sysm, psi, max_iter=max_iter, rtol=rtol).psi
        out.append(psi)
    return out


def multistep_objective(systems: list, psis: list) -> float:
    """J = sum_s L_N(psi^s): the number leaving the outer surface over the steps (dt dropped)."""
    return float(sum(luminosity(sy, p) for sy, p in zip(systems, psis)))


def multistep_adjoint(systems: list, psis: list, solver: str = "dense"):
    """Reverse recursion for J = sum_s L_N(psi^s).

    With lambda_s the total derivative of J with respect to psi^s,
      lambda_S = dL/dpsi^S,  J_s^T mu_s = lambda_s,  lambda_{s-1} = dL/dpsi^{s-1} + mu_s
    (psi^{s-1} enters step s only as psi^n, and dG_s/dpsi^n = -1), so dJ/dpsi^0 = mu_1 and
    dJ/dtheta_s = -mu_s^T dG_s/dtheta_s.  Returns (dJ/dpsi^0, [param_vjp of each step]).
    """
    S = len(systems)
    grads = [None] * S
    mu_next = np.zeros_like(psis[0])
    for s in range(S - 1, -1, -1):
        seed = luminosity_seed(systems[s], psis[s].shape) + mu_next
        mu = adjoint(systems[s], psis[s], seed, solver=solver)
        grads[s] = param_vjp(systems[s], psis[s], mu)
        mu_next = mu
    return mu_next, grads
