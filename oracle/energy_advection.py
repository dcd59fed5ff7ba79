"""FP64 CPU oracle of the neutrino energy-advection step (TEST INFRASTRUCTURE).

Follows the paper (CHIMERA, arXiv 1809.05608), "Neutrino Energy Advection" and "Neutrino Energy
Advection due to Changes in the Lapse" in the transport appendix, with the PPM machinery of the
"PPM Interpolation Scheme" section of the hydrodynamics appendix:

* eqs. a78-a80: the Lagrangian energy step.  The group edges are displaced by the factor of
  eq. a79 and psi is rescaled so that the number of neutrinos per unit mass is unchanged;
* eq. a81 with eqs. p5-p8: the remap of the displaced grid back onto the fixed grid.  The number
  density per unit energy, eps^2 psi, gets a piecewise parabolic profile in energy (eqs. h9-h24); the number in
  the region swept by each edge moves across it, and the fluxes are scaled by one factor xi per
  zone so that the energy is conserved as well as the number;
* eqs. a81a-a81d: the Pauli over-fill limiter, which moves the excess of an over-filled group to
  the next two groups conserving number and energy;
* eqs. p1-p8: the same remap applied to a change of the lapse, where the local energy grid
  E/a moves from E/a^n to E/a^{n+1}.

Arrays are [..., N] with the energy group last; every leading index is an independent
(species, ray, zone).  Energies in MeV; N_k = W_k psi_k is the number in group k without the
common factor 4 pi (eq. p4).

Only `tests/` may import this module.  It shares no code with the HIP path.

Readings (the paper is silent, garbled or inconsistent here):
  * PPM variable and geometry: the zone average is a_k = N_k / dE_k (proportional to
    eps_k^2 psi_k by eq. a01b) on the energy coordinate, with the planar (phi-direction) forms of
    eqs. h6-h14 and h24 (dV/dxi = 1, a* = a);
  * eq. h9 prints "Delta_i" for the width Delta xi_i; eq. h12 prints (Delta xi_i Delta xi_{i+1}) for
    the sum (Delta xi_i + Delta xi_{i+1}) in the first denominator, and (2 Delta xi_i + Delta xi_{i+1})
    for (Delta xi_i + 2 Delta xi_{i+1}) in the second: the corrected forms reproduce a cubic exactly,
    which the printed ones do not (the pins check this);
  * eq. h61 prints (1 + 4/3 ...) where the integral of the parabola of eq. h22 over the first
    fraction y of a zone gives (1 - 2y/3), the same factor as eq. h60 (the pins integrate the
    parabola numerically);
  * eq. h11 with Delta a_{i+1/2} Delta a_{i-1/2} = 0 gives a zero slope (a flat side);
  * the paper states that its monotonicity constraints keep new maxima and minima from appearing, but
    prints only the limits on the slopes and edge values (eqs. h11, h15, h16), which do not keep the
    parabola of a zone from overshooting inside it; on a steeply falling spectrum the overshoot goes
    below zero and the remap then produces negative occupations.  The zone constraint of the PPM
    paper it cites (Colella and Woodward 1984) is applied to each group's edge values before the
    parabola is formed: flat at a local extremum of the averages, otherwise the far edge moved until
    the parabola's extremum sits on the zone edge;
  * two ghost groups at each end of the energy grid repeat the end group's average and width, and
    the fluxes through the two outer grid edges are zero (the paper's condition for eq. p5 to
    conserve number);
  * edge displacement: a swept region wider than the group it comes from, or a displaced grid that
    is no longer increasing, is outside the method; such a zone is left unchanged and flagged;
  * the Eddington factor of eq. a79 at a group edge is the mean of the two adjacent groups' values
    (the end edges take the adjacent group's value); without one, 1/3 (the diffusion limit);
  * eq. p8 prints the denominator without its sum over k; it is sum_k (F_{k-1/2} - F_{k+1/2}) eps_k
    on the new grid; when that sum is zero, xi = 1;
  * eq. a81 runs the limiter from k = 0 while groups k+1 and k+2 exist (0-based k <= N-3); when the
    removal from k+2 would exceed psi_{k+2}, the removal from k is scaled down so that psi_{k+2}
    becomes zero (the "approximate" case of the paper).
"""
from __future__ import annotations

from typing import Optional

import numpy as np

MODE_LAGRANGIAN = 0      # eqs. a78-a81d
MODE_LAPSE = 1           # eqs. p1-p8, then the limiter of eqs. a81a-a81d

FLAG_DISPLACEMENT = 1    # a swept region exceeds its group: zone unchanged
FLAG_OVERFILL = 2        # the limiter moved neutrinos
FLAG_OVERFILL_CLAMP = 4  # the limiter hit the psi_{k+2} >= 0 bound (approximate case)


def _work_dtype(x) -> type:
    """float64, or the wider floating type of x (np.longdouble), so that the same steps can be
    repeated in extended precision to measure their own rounding."""
    return np.result_type(np.asarray(x).dtype, np.float64)


# ---------------------------------------------------------------- grid quantities (eqs. a01, a01b, p4)

def centers(edges: np.ndarray) -> np.ndarray:
    """Group-centre energies of eq. a01 (with the square restored): eps_k^2 = (e+^2 + e+ e- + e-^2)/3."""
    lo, hi = edges[..., :-1], edges[..., 1:]
    return np.sqrt((hi * hi + hi * lo + lo * lo) / 3.0)


def weights(edges: np.ndarray) -> np.ndarray:
    """W_k = (e+^3 - e-^3)/3 = eps_k^2 d eps_k (eq. a01b; eq. p4 without 4 pi)."""
    lo, hi = edges[..., :-1], edges[..., 1:]
    return (hi ** 3 - lo ** 3) / 3.0


# ---------------------------------------------------------------- PPM in energy (eqs. h9-h17, h22-h24)

def _pad2(x: np.ndarray) -> np.ndarray:
    """Two ghost entries at each end of the last axis, repeating the end values."""
    return np.concatenate([x[..., :1], x[..., :1], x, x[..., -1:], x[..., -1:]], axis=-1)


def ppm_slopes(a: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Limited mean slopes delta_m a_j of the zones of padded arrays (eqs. h9-h11, planar).

    a, d: zone averages and widths with ghosts; returns slopes for zones 1..len-2 of the padded
    arrays (the first and last padded zones have no slope)."""
    am, a0, ap = a[..., :-2], a[..., 1:-1], a[..., 2:]
    dm, d0, dp = d[..., :-2], d[..., 1:-1], d[..., 2:]
    dplus = ap - a0                # Delta a_{j+1/2}
    dminus = a0 - am               # Delta a_{j-1/2}
    da = d0 / (dm + d0 + dp) * ((2.0 * dm + d0) / (dp + d0) * dplus + (d0 + 2.0 * dp) / (dm + d0) * dminus)
    lim = np.minimum(np.abs(da), np.minimum(2.0 * np.abs(dplus), 2.0 * np.abs(dminus))) * np.sign(da)
    return np.where(dplus * dminus > 0.0, lim, 0.0)


def interface_value(aj, aj1, dm, d0, d1, d2, sj, sj1):
    """Value at the edge between zones j and j+1 of the cubic through the neighbouring averages (eq. h12,
    planar, garbles corrected): zone averages aj, aj1, widths dm, d0, d1, d2 of zones j-1..j+2, and the
    limited slopes sj, sj1 of zones j and j+1."""
    diff = aj1 - aj
    return (aj + d0 / (d0 + d1) * diff
            + 1.0 / (dm + d0 + d1 + d2) * (
                2.0 * d1 * d0 / (d0 + d1) * ((dm + d0) / (2.0 * d0 + d1) - (d2 + d1) / (2.0 * d1 + d0)) * diff
                - d0 * (dm + d0) / (2.0 * d0 + d1) * sj1
                + d1 * (d1 + d2) / (d0 + 2.0 * d1) * sj))


def ppm_interfaces(a: np.ndarray, d: np.ndarray):
    """Left and right edge values a_L, a_R of every group (eqs. h12, h15-h17, planar, with ghosts).

    a, d: [..., N] averages and widths.  Returns (aL, aR), each [..., N]."""
    ap, dp = _pad2(a), _pad2(d)
    s = ppm_slopes(ap, dp)                       # slopes of padded zones 1..N+2
    # interfaces j+1/2 between padded zones j and j+1 for j = 1..N+1 (N+1 interfaces: the grid edges)
    j = np.arange(1, a.shape[-1] + 2)
    aj, aj1 = ap[..., j], ap[..., j + 1]
    dm, d0, d1, d2 = dp[..., j - 1], dp[..., j], dp[..., j + 1], dp[..., j + 2]
    sj, sj1 = s[..., j - 1], s[..., j]           # s index = padded zone - 1
    val = interface_value(aj, aj1, dm, d0, d1, d2, sj, sj1)
    val = np.maximum(val, np.minimum(aj, aj1))   # eq. h15
    val = np.minimum(val, np.maximum(aj, aj1))   # eq. h16
    # val[..., m] is the edge below group m (m = 0..N); eq. h17: a_L of group m = a_R of group m-1
    return val[..., :-1], val[..., 1:]


def parabola(a: np.ndarray, aL: np.ndarray, aR: np.ndarray):
    """Delta a and a_6 of eqs. h23, h24 (planar): the parabola of eq. h22 averages to a over the zone."""
    return aR - aL, 6.0 * (a - 0.5 * (aL + aR))


def monotone_edges(a: np.ndarray, aL: np.ndarray, aR: np.ndarray):
    """Edge values of each zone adjusted so that its parabola has no extremum inside the zone: flat at a
    local extremum of the averages, else the edge on the far side of an interior extremum is moved
    until the extremum sits on the zone edge (the zone constraint of Colella and Woodward's PPM)."""
    Da, a6 = parabola(a, aL, aR)
    flat = (aR - a) * (a - aL) <= 0.0
    lo_fix = ~flat & (Da * a6 > Da * Da)
    hi_fix = ~flat & (-Da * Da > Da * a6)
    aL2 = np.where(flat, a, np.where(lo_fix, 3.0 * a - 2.0 * aR, aL))
    aR2 = np.where(flat, a, np.where(hi_fix, 3.0 * a - 2.0 * aL, aR))
    return aL2, aR2


def average_top(aR, Da, a6, y):
    """Mean of the parabola of eq. h22 over the top fraction y of its zone (eq. h60, the swept width in
    place of c_s dt)."""
    return aR - 0.5 * y * (Da - (1.0 - 2.0 * y / 3.0) * a6)


def average_bottom(aL, Da, a6, y):
    """Mean of the parabola of eq. h22 over the bottom fraction y of its zone (eq. h61, read with the
    factor (1 - 2y/3) that integrating eq. h22 gives)."""
    return aL + 0.5 * y * (Da + (1.0 - 2.0 * y / 3.0) * a6)


# ---------------------------------------------------------------- remap (eqs. p5-p8, a81)

def remap_fluxes(N: np.ndarray, src_edges: np.ndarray, tgt_edges: np.ndarray):
    """Number moved through each grid edge when the groups of the displaced grid `src_edges` holding
    numbers N are mapped onto `tgt_edges` (eq. p5).  F[..., m] is the flux through edge m (m = 0..N),
    positive upward; the two outer edges carry none.  Returns (F, ok) where ok is False for zones whose
    swept region at some edge is wider than the group it is taken from."""
    dS = src_edges[..., 1:] - src_edges[..., :-1]
    a = N / dS
    aL, aR = monotone_edges(a, *ppm_interfaces(a, dS))
    Da, a6 = parabola(a, aL, aR)
    delta = src_edges[..., 1:-1] - tgt_edges[..., 1:-1]          # eq. h101 at interior edges
    up = delta > 0.0
    y_up = np.where(up, delta / dS[..., :-1], 0.0)               # top part of group k moves up
    y_dn = np.where(up, 0.0, -delta / dS[..., 1:])               # bottom part of group k+1 moves down
    f_up = average_top(aR[..., :-1], Da[..., :-1], a6[..., :-1], y_up) * delta
    f_dn = average_bottom(aL[..., 1:], Da[..., 1:], a6[..., 1:], y_dn) * delta
    inner = np.where(delta == 0.0, 0.0, np.where(up, f_up, f_dn))
    ok = np.all((y_up <= 1.0) & (y_dn <= 1.0), axis=-1) & np.all(dS > 0.0, axis=-1)
    zero = np.zeros(N.shape[:-1] + (1,))
    return np.concatenate([zero, inner, zero], axis=-1), ok


def remap(N: np.ndarray, src_edges: np.ndarray, tgt_edges: np.ndarray):
    """Numbers on the target grid conserving number (eq. p5) and energy (eqs. p6-p8).

    Returns (N_new, xi, ok)."""
    F, ok = remap_fluxes(N, src_edges, tgt_edges)
    D = F[..., :-1] - F[..., 1:]                                  # -F_{k+1/2} + F_{k-1/2}
    e_src, e_tgt = centers(src_edges), centers(tgt_edges)
    energy = np.sum(N * e_src, axis=-1)                           # eq. p3, before
    num = energy - np.sum(N * e_tgt, axis=-1)
    den = np.sum(D * e_tgt, axis=-1)
    xi = np.where(den != 0.0, num / np.where(den != 0.0, den, 1.0), 1.0)   # eq. p8
    return N + xi[..., None] * D, xi, ok                          # eq. p6


# ---------------------------------------------------------------- over-fill limiter (eqs. a81a-a81d)

def overfill_limit(psi: np.ndarray, edges: np.ndarray):
    """Limit psi <= 1 group by group from the lowest, moving the excess of group k into k+1 and out of
    k+2 so that number (eq. a81a) and energy (eq. a81b) are unchanged (eqs. a81c, a81d).

    Returns (psi_new, flags)."""
    psi = np.array(psi, dtype=_work_dtype(psi), copy=True)
    eps = centers(edges)
    de = edges[..., 1:] - edges[..., :-1]
    flags = np.zeros(psi.shape[:-1], dtype=np.int32)
    n = psi.shape[-1]
    for k in range(n - 2):
        over = psi[..., k] > 1.0
        if not np.any(over):
            continue
        e0, e1, e2 = eps[..., k], eps[..., k + 1], eps[..., k + 2]
        w0, w1, w2 = e0 * e0 * de[..., k], e1 * e1 * de[..., k + 1], e2 * e2 * de[..., k + 2]
        rm0 = np.where(over, psi[..., k] - 1.0, 0.0)
        add1 = (e2 - e0) * w0 / ((e2 - e1) * w1) * rm0                 # eq. a81c
        rm2 = (e1 - e0) * w0 / ((e2 - e1) * w2) * rm0                   # eq. a81d
        clamp = over & (rm2 > psi[..., k + 2])
        scale = np.where(clamp, psi[..., k + 2] / np.where(clamp, rm2, 1.0), 1.0)
        rm0, add1, rm2 = rm0 * scale, add1 * scale, np.where(clamp, psi[..., k + 2], rm2)
        psi[..., k] -= rm0
        psi[..., k + 1] += add1
        psi[..., k + 2] -= rm2
        flags |= np.where(over, FLAG_OVERFILL, 0) | np.where(clamp, FLAG_OVERFILL_CLAMP, 0)
    return psi, flags


# ---------------------------------------------------------------- the steps

def edge_eddington(eddington: Optional[np.ndarray], shape) -> np.ndarray:
    """Eddington factor at the N+1 group edges: mean of the neighbours, end edges from the end groups."""
    if eddington is None:
        return np.full(shape[:-1] + (shape[-1] + 1,), 1.0 / 3.0)
    h = eddington
    mid = 0.5 * (h[..., :-1] + h[..., 1:])
    return np.concatenate([h[..., :1], mid, h[..., -1:]], axis=-1)


def lagrangian_displacement(e_edge, dlna, dlnR, dlnb, eddington, shape):
    """Displaced edges of eq. a79: E' = [1 + (da/a - dR/R) - (db/b - dR/R) eta2] E at every edge.

    dlna, dlnR, dlnb: arrays broadcasting to the leading shape (one value per zone)."""
    h = edge_eddington(eddington, shape)
    dt = _work_dtype(e_edge)
    dlna, dlnR, dlnb = (np.asarray(x, dtype=dt)[..., None] for x in (dlna, dlnR, dlnb))
    s = 1.0 + (dlna - dlnR) - (dlnb - dlnR) * h
    return s * e_edge


def energy_advect(psi, e_edge, rho_old=1.0, rho_new=1.0, a_old=1.0, a_new=1.0, dlnR=0.0, dlnb=0.0,
                  eddington=None):
    """The three-part energy update of eqs. a78-a81d for psi [..., N] on the fixed grid e_edge [N+1].

    Zone quantities (rho, lapse a, dR/R, db/b) broadcast to the leading shape.  Returns
    (psi_new, xi, flags)."""
    dt = _work_dtype(psi)
    psi = np.asarray(psi, dtype=dt)
    shape = psi.shape
    tgt = np.broadcast_to(e_edge, shape[:-1] + (shape[-1] + 1,))
    a_old, a_new = np.asarray(a_old, dtype=dt), np.asarray(a_new, dtype=dt)
    dlna = a_new / a_old - 1.0
    src = lagrangian_displacement(e_edge, dlna, dlnR, dlnb, eddington, shape)
    # eq. a78: psi' (E^2 dE)' = (rho a^3)^{n+1} / (rho a^3)^n psi (E^2 dE), i.e. N' = r W psi
    r = (np.asarray(rho_new) * a_new ** 3) / (np.asarray(rho_old) * a_old ** 3)
    N = np.asarray(r, dtype=dt)[..., None] * weights(tgt) * psi
    return _remap_and_limit(psi, N, src, tgt)


def lapse_remap(psi, e_edge, a_old, a_new):
    """Remap of psi after a change of the lapse (eqs. p1-p8), then the over-fill limiter.

    The local grid edges move from E/a^n to E/a^{n+1} (eq. p1); psi on the old grid holds
    N_k = psi_k W_k(E/a^n) neutrinos (eq. p2).  Returns (psi_new, xi, flags)."""
    dt = _work_dtype(psi)
    psi = np.asarray(psi, dtype=dt)
    shape = psi.shape
    a_old = np.asarray(a_old, dtype=dt)[..., None]
    a_new = np.asarray(a_new, dtype=dt)[..., None]
    src = np.broadcast_to(e_edge / a_old, shape[:-1] + (shape[-1] + 1,))
    tgt = np.broadcast_to(e_edge / a_new, shape[:-1] + (shape[-1] + 1,))
    N = weights(src) * psi
    return _remap_and_limit(psi, N, src, tgt)


def _remap_and_limit(psi, N, src, tgt):
    N_new, xi, ok = remap(N, src, tgt)
    psi_new = N_new / weights(tgt)
    psi_new, flags = overfill_limit(psi_new, tgt)
    psi_new = np.where(ok[..., None], psi_new, psi)
    xi = np.where(ok, xi, 1.0)
    flags = np.where(ok, flags, FLAG_DISPLACEMENT).astype(np.int32)
    return psi_new, xi, flags


def number_and_energy(psi: np.ndarray, edges: np.ndarray):
    """Sum_k W_k psi_k and sum_k W_k eps_k psi_k on the grid `edges` (eqs. p2, p3 without 4 pi)."""
    W, e = weights(edges), centers(edges)
    return np.sum(W * psi, axis=-1), np.sum(W * e * psi, axis=-1)
