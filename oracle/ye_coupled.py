"""FP64 CPU oracle of the Y_e-coupled transport step (TEST INFRASTRUCTURE).

Extends the single-species oracle (`oracle.transport`) with the electron-fraction equation of
the paper's Lagrangian transport step (CHIMERA, arXiv 1809.05608, "Lagrangian Transport Step"
and "Solution of the Transport Equations"):

* eq. a62a: the differenced Y_e equation, coupling the electron neutrinos and antineutrinos of a
  ray through their emission/absorption sources;
* eqs. a62ac, a62ad: the linearised transport equations with the Y_e correction on their source
  side, and the linearised Y_e equation with the psi corrections of both species;
* eq. a62ae: the combined block-tridiagonal system of N_nu x N_k + 1 unknowns per zone, here
  the two coupled species, so 2N + 1 (psi of nu_e, psi of anti-nu_e, Y_e);
* eqs. a62b, a62d: the internal-energy change of the matter and the temperature update computed
  after the implicit solve;
* eqs. d11-d22 (optional): neutrino-antineutrino pair creation and annihilation coupling the two
  species of the block, with the angular cutoff factor chi = min(chi_1, chi_2) on the annihilation
  kernel.

Only `tests/` may import this module.  It shares no code with the HIP path.

Readings (the paper is silent or garbled here):
  * the transport mean free path is frozen at Y_e^n during the step: eq. a62ae couples zone i
    to its neighbours only through the same unknown (diagonal Bm, Bp), and eq. a62ac puts the
    Y_e correction on the source side, so Y_e enters only the emission/absorption source;
  * the absorption and emission opacities of the two coupled species are linear in Y_e over the
    step, kappa_a(Y_e) = kappa_a + (Y_e - Y_e^n) dkappa_a/dY_e and likewise for eta, with the
    derivatives supplied as inputs (they come from the EoS/opacity tables in a full code);
  * the NES kernels and the isoenergetic scattering do not depend on Y_e;
  * m_B, the baryon mass of eq. a62a, is the atomic mass unit;
  * eq. a62d is used in its thermodynamically consistent form
        T^{n+1} = T^n + (e^{n+1} - e^n - (Y_e^{n+1} - Y_e^n) (de/dY_e)_{rho,T}) / (de/dT)_{rho,Y_e}
    (the printed "+" and the subscript "rho, Y_e" on de/dY_e are read as a garble of a first-order
    expansion of e(T, Y_e) at fixed rho);
  * energies of eq. a62b are in MeV per baryon; e and its derivatives are inputs in those units;
  * pair processes enter moment 0 through the Phi_0 terms of eq. d14 (the Phi_1 terms, products of the
    two species' first moments, are dropped as for the NES kernel); in the discrete form the sums over
    eps' carry the weights W_k' (eq. a01b), the annihilation kernel is Q^a_{kk'} = a_i g_{kk'} W_k'/Wbar
    with a symmetric shape g (so that W_k Q^a_{kk'} is symmetric and pairs conserve nu - anti-nu
    number), and the creation kernel is Q^p = exp(-(eps_k + eps_k')/T) Q^a (eq. d12: the electron and
    positron carry the pair's energy);
  * chi_1 (eq. d16) takes the zone-centred flux factors psi1/psi0 of both species as inputs, so it does
    not depend on the unknowns; its printed closed form, 1 - (1/6) eta eta', does not follow from the
    ratio of angular integrals that eq. d16 states as its definition, which evaluates to
    1 - (3/2) eta eta' for f = psi0 + 3 mu psi1; the definition is taken; chi_2 (eq. d19) uses R = the zone centre and the cosines of eq. d22,
    whose "sign" is Fortran's SIGN(a, b) (|a| with the sign of b): mu = sqrt(1 - x^2) for x = R_nu/R <= 1
    and -sqrt(x^2 - 1) clipped at -1 inside the neutrinosphere;
  * the pair sources join the collision energy of the temperature update (the pair's energy comes from
    the matter's electrons and positrons);
  * with a lapse a_i (eq. a58 with a != 1) the species rows are a_i c dt times eq. a58 as in the
    single-species oracle, so their Y_e-dependent source terms carry a_i too, and the neutrinos of zone i
    number (V_i / a_i^3) sum_k W_k psi (the local phase space W / a^3 at the local energies E / a_i);
    eq. a62a then exchanges electrons with that number at the rate of the species rows: its source is
    c dt zeta a_i^-2 sum_k W_k (S_nue - S_nuebar) with the caller's local-energy opacities (a_i from the
    source and a_i^-3 from the phase space), which keeps the lepton number
    sum_i V_i [rho Y_e / m_B + (4 pi/(hc)^3) a_i^-3 sum_k W_k (psi_nue - psi_nuebar)] (pinned); the pair
    processes and the temperature update are written for a = 1 and refuse a lapse.

Parity status: pinned by `tests/test_oracle_ye.py` (total lepton-number conservation, total
energy conservation through the temperature update, the decoupled limit against the
single-species oracle, central differences of the Jacobian, block-Thomas against a dense solve);
none of its functions is "parity unpinned".
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import transport as tr
from .transport import (System, TERM_EMABS, TERM_NES, geometry, group_energies, residual_rounding_level,
                        nes_source, block_thomas_solve, NewtonResult, ARMIJO_C, ALPHA_MIN)

M_B_G = 1.66053906660e-24        # g, baryon mass of eq. a62a (atomic mass unit)
HC_MEV_CM = 1.23984198e-10       # MeV cm
FOUR_PI_HC3 = 4.0 * np.pi / HC_MEV_CM ** 3     # MeV^-3 cm^-3: number density per unit W psi


@dataclasses.dataclass
class CoupledSystem:
    """One ray's nu_e and anti-nu_e systems plus the zone data of the Y_e equation."""
    nue: System                 # species q = 1 of eq. a62ad (electron neutrinos)
    nuebar: System              # species q = 2 (electron antineutrinos)
    rho: np.ndarray             # [I] g cm^-3
    ye_n: np.ndarray            # [I] Y_e at step n
    dka_dye: np.ndarray         # [2][I][N] dkappa_a/dY_e of nu_e, anti-nu_e (cm^-1)
    deta_dye: np.ndarray        # [2][I][N] deta/dY_e (cm^-1)
    pair_amp: Optional[np.ndarray] = None    # [I] cm^-1, pair-kernel amplitude (None: no pair processes)
    pair_g: Optional[np.ndarray] = None      # [N][N] symmetric shape of the pair kernels
    pair_eta1: Optional[np.ndarray] = None   # [2][I][N] flux factors psi1/psi0 of nu_e and anti-nu_e

    @property
    def I(self) -> int:
        return self.nue.I

    @property
    def N(self) -> int:
        return self.nue.N

    @property
    def M(self) -> int:
        return 2 * self.N + 1


def coupled_systems(w: dict, ye: dict) -> list:
    """CoupledSystem of every ray from workload arrays (`Workload.numpy()`) and `YeInputs.numpy()`."""
    sy = tr.systems_from_workload(w)
    pairs = ye.get("pair_amp") is not None
    return [CoupledSystem(nue=sy[0][r], nuebar=sy[1][r], rho=ye["rho"][r], ye_n=ye["ye_n"][r],
                          dka_dye=ye["dka_dye"][:, r], deta_dye=ye["deta_dye"][:, r],
                          pair_amp=ye["pair_amp"][r] if pairs else None, pair_g=ye["pair_g"] if pairs else None,
                          pair_eta1=ye["pair_eta1"][:, r] if pairs else None)
            for r in range(w["R"])]


# ---------------------------------------------------------------- pair processes (eqs. d11-d22)

def limb_cosine(x):
    """Cosine of eq. d22 for x = R_nu/R: sqrt(1 - x^2) outside the neutrinosphere (eq. d17), and
    -sqrt(x^2 - 1) clipped at -1 inside it."""
    x = np.asarray(x, dtype=np.float64)
    v = 1.0 - x * x
    return np.maximum(np.copysign(np.sqrt(np.abs(v)), v), -1.0)


def chi1(eta1_nu, eta1_nubar):
    """Angular factor of the annihilation rate for nearly isotropic distributions: the ratio that defines
    eq. d16, evaluated for f = psi0 + 3 mu psi1 (eq. d15), is 1 - (3/2)(psi1/psi0)(psi1bar/psi0bar)
    (the averages of (1 - n.n')^2 are 4/3 isotropic and -2 psi1 psi1bar from the dipoles)."""
    return 1.0 - 1.5 * np.asarray(eta1_nu) * np.asarray(eta1_nubar)


def chi2(mu, mubar):
    """Angular factor for radiation beamed from the neutrinospheres (eq. d19)."""
    mu, mubar = np.asarray(mu), np.asarray(mubar)
    return (8.0 + (mu * mubar - 3.0) * (1.0 + mu) * (1.0 + mubar)) / 8.0


def pair_chi(cs: CoupledSystem) -> np.ndarray:
    """chi_{i,k,k'} = min(chi_1, chi_2) (eq. d21) for a nu_e of group k and an anti-nu_e of group k' in
    zone i: [I][N][N]."""
    Rc = geometry(cs.nue.r_edge)[0]
    mu = limb_cosine(cs.nue.r_nu[None, :] / Rc[:, None])            # [I][N]
    mub = limb_cosine(cs.nuebar.r_nu[None, :] / Rc[:, None])
    c1 = chi1(cs.pair_eta1[0][:, :, None], cs.pair_eta1[1][:, None, :])
    c2 = chi2(mu[:, :, None], mub[:, None, :])
    return np.minimum(c1, c2)


def pair_kernels(cs: CoupledSystem):
    """Annihilation and creation kernels [I][N][N] seen from the nu_e (row k, anti-nu_e group k') and from
    the anti-nu_e (row k', nu_e group k): Q^a_{kk'} = a g_{kk'} W_k'/Wbar, Qbar^a_{k'k} = a g_{kk'} W_k/Wbar,
    and the creation kernels times exp(-(eps_k + eps_k')/T) (eq. d12)."""
    eps, W = group_energies(cs.nue.e_edge)
    Wbar = W.mean()
    base = cs.pair_amp[:, None, None] * cs.pair_g[None, :, :]
    qa = base * (W / Wbar)[None, None, :]
    qba = np.transpose(base, (0, 2, 1)) * (W / Wbar)[None, None, :]
    boltz = np.exp(-(eps[:, None] + eps[None, :])[None] / cs.nue.temp[:, None, None])
    return qa, boltz * qa, qba, np.transpose(boltz, (0, 2, 1)) * qba


def pair_sources(cs: CoupledSystem, pe: np.ndarray, pa: np.ndarray):
    """Zeroth-moment pair sources of both species (eq. d14, Phi_0 terms), [I][N] each:
        S_nu,k = (1 - psi_k) sum_k' Q^p_{kk'} (1 - psibar_k') - psi_k sum_k' Q^a_{kk'} chi_{kk'} psibar_k'
    and the same with the roles of the species exchanged."""
    qa, qp, qba, qbp = pair_kernels(cs)
    chi = pair_chi(cs)
    chib = np.transpose(chi, (0, 2, 1))
    s_e = (1.0 - pe) * np.einsum("ikl,il->ik", qp, 1.0 - pa) - pe * np.einsum("ikl,il->ik", qa * chi, pa)
    s_a = (1.0 - pa) * np.einsum("ikl,il->ik", qbp, 1.0 - pe) - pa * np.einsum("ikl,il->ik", qba * chib, pe)
    return s_e, s_a


def zeta(cs: CoupledSystem) -> np.ndarray:
    """4 pi m_B / ((hc)^3 rho) per zone: converts sum_k W_k (source) to a Y_e rate (eq. a62a)."""
    return FOUR_PI_HC3 * M_B_G / cs.rho


def lapse(cs: CoupledSystem) -> np.ndarray:
    """Lapse a_i at the zone centres (ones without a lapse); the pair processes take none."""
    if cs.nue.lapse is None:
        return np.ones(cs.I)
    if cs.pair_amp is not None:
        raise NotImplementedError("the pair processes are written for a = 1")
    return np.asarray(cs.nue.lapse, dtype=np.float64)


def pack(psi_e: np.ndarray, psi_a: np.ndarray, ye: np.ndarray) -> np.ndarray:
    """Per-zone unknowns u_i = (psi_nue[0..N), psi_nuebar[0..N), Y_e) -> [I][2N+1]."""
    return np.concatenate([psi_e, psi_a, ye[:, None]], axis=1)


def unpack(u: np.ndarray, N: int):
    return u[:, :N], u[:, N:2 * N], u[:, 2 * N]


def _ea_source(sys: System, dka: np.ndarray, deta: np.ndarray, dy: np.ndarray, psi: np.ndarray):
    """Emission minus absorption, eta(Y_e) (1 - psi) - kappa_a(Y_e) psi, with linear Y_e dependence."""
    ka = sys.kappa_a + dy[:, None] * dka
    et = sys.eta + dy[:, None] * deta
    return et * (1.0 - psi) - ka * psi


def residual(cs: CoupledSystem, u_n: np.ndarray, u: np.ndarray) -> np.ndarray:
    """G(u) [I][2N+1]: the two species residuals (c dt times eq. a58) with Y_e-dependent
    emission/absorption, and c dt times eq. a62a for Y_e:
        G_Y = Y_e - Y_e^n + c dt zeta sum_k W_k (S^ea_nue - S^ea_nuebar)
    """
    N = cs.N
    pe_n, pa_n, _ = unpack(u_n, N)
    pe, pa, ye = unpack(u, N)
    dy = ye - cs.ye_n
    c = cs.nue.c_dt
    a = lapse(cs)
    out = np.empty_like(u)
    for q, (sys, p_n, p) in enumerate(((cs.nue, pe_n, pe), (cs.nuebar, pa_n, pa))):
        G = tr.residual(sys, p_n, p)            # opacities at Y_e^n
        if sys.terms & TERM_EMABS:
            # the Y_e-dependent part of a (-eta (1 - psi) + kappa_a psi)
            G = G + c * (a * dy)[:, None] * (cs.dka_dye[q] * p - cs.deta_dye[q] * (1.0 - p))
        out[:, q * N:(q + 1) * N] = G
    if cs.pair_amp is not None:
        s_e, s_a = pair_sources(cs, pe, pa)
        out[:, :N] -= c * s_e
        out[:, N:2 * N] -= c * s_a
    out[:, 2 * N] = dy
    if cs.nue.terms & TERM_EMABS:
        _, W = group_energies(cs.nue.e_edge)
        s_e = _ea_source(cs.nue, cs.dka_dye[0], cs.deta_dye[0], dy, pe)
        s_a = _ea_source(cs.nuebar, cs.dka_dye[1], cs.deta_dye[1], dy, pa)
        out[:, 2 * N] += c * zeta(cs) / a ** 2 * ((s_e - s_a) @ W)
    return out


def jacobian_blocks(cs: CoupledSystem, u: np.ndarray):
    """Exact Jacobian of G in the block-tridiagonal form of eq. a62ae: A [I][M][M] (M = 2N+1),
    bm [I][M], bp [I][M].  Y_e has no radial coupling (its bm, bp entries are zero)."""
    N, I, M = cs.N, cs.I, cs.M
    pe, pa, ye = unpack(u, N)
    dy = ye - cs.ye_n
    c = cs.nue.c_dt
    _, W = group_energies(cs.nue.e_edge)
    a = lapse(cs)
    z = zeta(cs) / a ** 2                      # the Y_e row's rate per unit sum_k W_k S
    A = np.zeros((I, M, M))
    bm = np.zeros((I, M))
    bp = np.zeros((I, M))
    for q, (sys, p) in enumerate(((cs.nue, pe), (cs.nuebar, pa))):
        Aq, bmq, bpq = tr.jacobian_blocks(sys, p)
        sl = slice(q * N, (q + 1) * N)
        A[:, sl, sl] = Aq
        bm[:, sl] = bmq
        bp[:, sl] = bpq
        dka, deta = cs.dka_dye[q], cs.deta_dye[q]
        if sys.terms & TERM_EMABS:
            # d/dpsi of c dY (dka psi - deta (1 - psi)), and the Y_e column d G_q / dY_e
            idx = np.arange(q * N, (q + 1) * N)
            A[:, idx, idx] += c * (a * dy)[:, None] * (dka + deta)
            A[:, sl, 2 * N] = c * a[:, None] * (dka * p - deta * (1.0 - p))
            # Y_e row: dG_Y/dpsi_q,k = +-c zeta W_k dS^ea_q/dpsi = -+c zeta W_k (eta(Y) + kappa_a(Y))
            ka = sys.kappa_a + dy[:, None] * dka
            et = sys.eta + dy[:, None] * deta
            sign = 1.0 if q == 0 else -1.0
            A[:, 2 * N, sl] = -sign * c * z[:, None] * W[None, :] * (et + ka)
    if cs.pair_amp is not None:
        # -c dS_pair/dpsi: own diagonal c [sum Q^p (1 - psibar) + sum Q^a chi psibar], and the cross-species
        # block c [(1 - psi_k) Q^p_{kk'} + psi_k Q^a_{kk'} chi_{kk'}]
        qa, qp, qba, qbp = pair_kernels(cs)
        chi = pair_chi(cs)
        chib = np.transpose(chi, (0, 2, 1))
        for (r0, c0, p, pb, qpp, qaa, ch) in ((0, N, pe, pa, qp, qa, chi), (N, 0, pa, pe, qbp, qba, chib)):
            idx = np.arange(r0, r0 + N)
            A[:, idx, idx] += c * (np.einsum("ikl,il->ik", qpp, 1.0 - pb) + np.einsum("ikl,il->ik", qaa * ch, pb))
            A[:, r0:r0 + N, c0:c0 + N] += c * ((1.0 - p)[:, :, None] * qpp + p[:, :, None] * qaa * ch)
    A[:, 2 * N, 2 * N] = 1.0
    if cs.nue.terms & TERM_EMABS:
        dS = lambda q, p: cs.deta_dye[q] * (1.0 - p) - cs.dka_dye[q] * p      # noqa: E731  dS^ea/dY_e
        A[:, 2 * N, 2 * N] += c * z * ((dS(0, pe) - dS(1, pa)) @ W)
    return A, bm, bp


def dense_jacobian(cs: CoupledSystem, u: np.ndarray) -> np.ndarray:
    """The full (I*M) x (I*M) Jacobian, row/column index i*M + alpha."""
    A, bm, bp = jacobian_blocks(cs, u)
    I, M = cs.I, cs.M
    J = np.zeros((I * M, I * M))
    for i in range(I):
        J[i * M:(i + 1) * M, i * M:(i + 1) * M] = A[i]
        if i > 0:
            J[i * M:(i + 1) * M, (i - 1) * M:i * M] = np.diag(bm[i])
        if i + 1 < I:
            J[i * M:(i + 1) * M, (i + 1) * M:(i + 2) * M] = np.diag(bp[i])
    return J


def rounding_level(cs: CoupledSystem, u_n: np.ndarray, u: np.ndarray) -> float:
    """Rounding level of G: the larger of the two species' levels (transport oracle definition)
    and 32 ulp of the largest per-zone sum of |terms of G_Y| + |Y_e| |dG_Y/dY_e|, where the terms of
    the emission/absorption source count separately, |eta (1 - psi)| + |kappa_a psi|, as they do in
    the species rows."""
    N = cs.N
    pe_n, pa_n, _ = unpack(u_n, N)
    pe, pa, ye = unpack(u, N)
    dy = ye - cs.ye_n
    c = cs.nue.c_dt
    _, W = group_energies(cs.nue.e_edge)
    z = zeta(cs) / lapse(cs) ** 2
    lev = max(residual_rounding_level(cs.nue, pe_n, pe), residual_rounding_level(cs.nuebar, pa_n, pa))
    mag = np.abs(ye) + np.abs(cs.ye_n)
    if cs.nue.terms & TERM_EMABS:
        for q, (sys, p) in enumerate(((cs.nue, pe), (cs.nuebar, pa))):
            ka = sys.kappa_a + dy[:, None] * cs.dka_dye[q]
            et = sys.eta + dy[:, None] * cs.deta_dye[q]
            mag = mag + c * z * ((np.abs(et * (1.0 - p)) + np.abs(ka * p)) @ W)
    A, _, _ = jacobian_blocks(cs, u)
    mag = mag + np.abs(ye) * np.abs(A[:, 2 * N, 2 * N])
    lev = max(lev, 32.0 * np.finfo(np.float64).eps * float(np.max(mag)))
    if cs.pair_amp is not None:
        # the pair terms of the species rows, counted as the other source terms are: |psi|, their
        # magnitudes, and |psi| times their derivative with respect to the row's own psi (|psi^n| is in the
        # species rows' own level)
        qa, qp, qba, qbp = pair_kernels(cs)
        chi = pair_chi(cs)
        chib = np.transpose(chi, (0, 2, 1))
        for p, pb, qpp, qaa, ch in ((pe, pa, qp, qa, chi), (pa, pe, qbp, qba, chib)):
            cre = np.einsum("ikl,il->ik", qpp, 1.0 - pb)
            ann = np.einsum("ikl,il->ik", qaa * ch, pb)
            m = np.abs(p) + c * (np.abs((1.0 - p) * cre) + np.abs(p * ann)) + np.abs(p) * c * (cre + ann)
            lev = max(lev, 32.0 * np.finfo(np.float64).eps * float(np.max(m)))
    return lev


def newton(cs: CoupledSystem, u_n: np.ndarray, u0: Optional[np.ndarray] = None,
           max_iter: int = 30, rtol: float = 0.0) -> NewtonResult:
    """Backward-Euler Newton iteration (eq. a62aa) for psi of both species and Y_e of one ray:
    each update solves the (2N+1)-block system of eq. a62ae by block-Thomas, with the same
    backtracking line search and stopping rule as the single-species oracle."""
    u = (u_n if u0 is None else u0).copy()
    G = residual(cs, u_n, u)
    r = float(np.max(np.abs(G)))
    res0 = r
    hist = [r]
    iters = 0
    prev = np.inf
    target = 0.0
    for _ in range(max_iter):
        if r == 0.0 or not np.isfinite(r):
            break
        target = max(rtol * res0, rounding_level(cs, u_n, u))
        if rtol > 0.0 and (r <= target or (r <= 1e3 * target and r > 0.5 * prev)):
            break
        A, bm, bp = jacobian_blocks(cs, u)
        delta = block_thomas_solve(A, bm, bp, -G)
        iters += 1
        trial = u + delta
        alpha = 1.0
        Gt = residual(cs, u_n, trial)
        rt = float(np.max(np.abs(Gt)))
        near = r <= 1e3 * target
        while not near and not rt <= (1.0 - ARMIJO_C * alpha) * r and alpha > ALPHA_MIN:
            alpha = 0.5 * alpha
            trial = u + alpha * delta
            Gt = residual(cs, u_n, trial)
            rt = float(np.max(np.abs(Gt)))
        prev = r
        u, G, r = trial, Gt, rt
        hist.append(r)
    if rtol > 0.0:
        target = max(rtol * res0, rounding_level(cs, u_n, u))
    conv = (r <= target) if rtol > 0.0 else True
    return NewtonResult(psi=u, iters=iters, res0=res0, res=r, converged=bool(conv), history=hist)


# ---------------------------------------------------------------- conservation and the T update

def lepton_number(cs: CoupledSystem, u: np.ndarray) -> float:
    """Total lepton number of the ray divided by 4 pi (volumes without 4 pi, eqs. a51-a55):
        sum_i V_i [rho_i Y_e,i / m_B + (4 pi/(hc)^3) a_i^-3 sum_k W_k (psi_nue - psi_nuebar)]
    (a = 1 without a lapse)."""
    _, V, _, _ = geometry(cs.nue.r_edge)
    _, W = group_energies(cs.nue.e_edge)
    pe, pa, ye = unpack(u, cs.N)
    a = lapse(cs)
    return float(np.sum(V * (cs.rho * ye / M_B_G + FOUR_PI_HC3 / a ** 3 * ((pe - pa) @ W))))


def collision_energy_source(sys: System, psi: np.ndarray, dka=None, deta=None, dy=None) -> np.ndarray:
    """c dt times the energy-weighted collision source per zone, sum_k eps_k W_k (S^ea + S^NES)
    (MeV^4; isoenergetic scattering exchanges no energy)."""
    eps, W = group_energies(sys.e_edge)
    src = np.zeros_like(psi)
    if sys.terms & TERM_EMABS:
        if dka is None:
            src = src + sys.eta * (1.0 - psi) - sys.kappa_a * psi
        else:
            src = src + _ea_source(sys, dka, deta, dy, psi)
    if sys.terms & TERM_NES:
        src = src + nes_source(sys, psi)
    return sys.c_dt * (src @ (eps * W))


def temperature_update(cs: CoupledSystem, others: list, u: np.ndarray, psi_others: list,
                       stat_weights, temp_n: np.ndarray, de_dT: np.ndarray, de_dye: np.ndarray):
    """Internal-energy change of the matter (eq. a62b) and the temperature after the step (eq. a62d).

    others / psi_others: the remaining species' systems of the ray and their new psi; stat_weights:
    the statistical weight of every species, the coupled pair first (typically 1, 1, 2, 2).
    de = -(4 pi/(hc)^3) (m_B/rho) sum_q w_q sum_k eps_k W_k c dt S_q (MeV per baryon);
    T^{n+1} = T^n + (de - (Y_e^{n+1} - Y_e^n) de/dY_e) / (de/dT).
    Returns (de [I], T^{n+1} [I]).
    """
    if cs.nue.lapse is not None:
        raise NotImplementedError("the temperature update is written for a = 1")
    pe, pa, ye = unpack(u, cs.N)
    dy = ye - cs.ye_n
    src = stat_weights[0] * collision_energy_source(cs.nue, pe, cs.dka_dye[0], cs.deta_dye[0], dy)
    src = src + stat_weights[1] * collision_energy_source(cs.nuebar, pa, cs.dka_dye[1], cs.deta_dye[1], dy)
    if cs.pair_amp is not None:
        eps, W = group_energies(cs.nue.e_edge)
        s_e, s_a = pair_sources(cs, pe, pa)
        src = src + cs.nue.c_dt * (stat_weights[0] * (s_e @ (eps * W)) + stat_weights[1] * (s_a @ (eps * W)))
    for w, sys, p in zip(stat_weights[2:], others, psi_others):
        src = src + w * collision_energy_source(sys, p)
    de = -FOUR_PI_HC3 * M_B_G / cs.rho * src
    return de, temp_n + (de - dy * de_dye) / de_dT


def neutrino_energy(sys: System, psi: np.ndarray) -> float:
    """sum_i V_i (4 pi/(hc)^3) sum_k eps_k W_k psi (MeV, volumes without 4 pi)."""
    _, V, _, _ = geometry(sys.r_edge)
    eps, W = group_energies(sys.e_edge)
    return float(FOUR_PI_HC3 * np.sum(V * (psi @ (eps * W))))
