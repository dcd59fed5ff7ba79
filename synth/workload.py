"""Synthetic stellar-profile workloads for the implicit MGFLD transport step.

The paper's production runs use progenitor models and tabulated opacities that
are not available here, so every input is a seeded analytic stand-in with the
paper's production shapes: 20 energy groups, 4 species, about 540 radial zones
(Transport Sources section; Code Comparison section; the 540x180x180 3-D grid of
the hydrodynamics tests).

Recipe (one workload = S species x R rays x I zones x N groups):

* radial zone edges log-spaced from 1e6 cm to 1e9 cm; zone centres are edge means;
* energy-group edges log-spaced from 2 MeV to 300 MeV; opacities are evaluated at
  the group centre energy whose square is the mean of e_lo^2, e_lo*e_hi, e_hi^2
  (the zone-centre definition of the paper's energy grid, eq. a01 with the
  square restored, which keeps eq. a01b exact);
* rho(r) = max(1e14 (r/1e6)^-3 * exp(0.1 z_rho), 1e6) g/cm^3 and
  T(r) = 30 (r/1e6)^-0.7 * exp(0.1 z_T) MeV, with one standard-normal draw per ray
  and per quantity (a lognormal ray-to-ray perturbation with sigma 0.1);
* chemical potential mu = +2T for nu_e and nu_x, -2T for the antineutrinos;
* absorption opacity kappa_a = 1e-6 (rho/1e14) (eps/10 MeV)^2 cm^-1;
  emissivity from detailed balance with Fermi-Dirac, eta = f_s kappa_a exp(-(eps-mu)/T)
  with f_s = 0.5 for the heavy-lepton species; isoenergetic scattering kappa_s = 2 kappa_a;
* NES-like kernel: amplitude a = 1e-7 (rho/1e14) cm^-1 per zone and a symmetric
  Gaussian G[k][k'] = exp(-(ln eps_k - ln eps_k')^2 / (2 * 0.3^2));
* initial state psi^n = 0.9 f_FD(eps; mu, T);
* c*dt with dt = 1e-6 s;
* neutrinosphere radius R_nu(eps) = 3e6 cm (eps / 10 MeV)^0.5 for every species (the radius at which the
  Eddington-factor stand-in of the energy-advection inputs turns over); used only by the geometric
  flux limiter and the geometric outer boundary (off by default).

Extras per configuration: opacity spikes on 5% of the rays (stress case) and a
smooth 1% per-step drift of rho and T (multi-step case).

No array here is computed by the transport method: the oracle and the device
path both take these arrays as given inputs.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np
import torch

C_LIGHT = 2.99792458e10          # cm/s
SEED = 180905608
DT = 1.0e-6                      # s

TERM_DIFFUSION = 1
TERM_EMABS = 2
TERM_NES = 4
TERMS_ALL = TERM_DIFFUSION | TERM_EMABS | TERM_NES

BC_ZERO_FLUX = 0
BC_FREE_STREAM = 1
BC_GEOMETRIC = 2                 # constant luminosity through a geometric ghost zone (eq. a62af)

LIMITER_NONE = 0
LIMITER_INTRP = 1
LIMITER_GEOM = 2                 # min(F_intrp, F_geom), eqs. a20, a23-a26a

R_NU_CM = 3.0e6                  # neutrinosphere radius of a 10 MeV neutrino

# name, rays, zones, groups, species
CONFIGS = {
    0: dict(name="fp64-16r-64z-12g-1s", R=16, I=64, N=12, S=1),
    1: dict(name="fp64-180r-540z-20g-4s", R=180, I=540, N=20, S=4),
    2: dict(name="mixed-4096r-540z-20g-4s-spikes", R=4096, I=540, N=20, S=4),
    3: dict(name="adjoint-1024r-540z-20g-1s", R=1024, I=540, N=20, S=1),
    4: dict(name="multistep-16384r-540z-20g-4s", R=16384, I=540, N=20, S=4),
}

N_SPIKE_FRACTION = 0.05
SPIKE_HALF_WIDTH = 8             # 17 zones
DRIFT_AMPLITUDE = 0.01


@dataclasses.dataclass
class Workload:
    """One batch of independent (species, ray) systems, all arrays float64.

    Layouts: cell arrays [S][R][I][N] (group fastest), zone arrays [R][I],
    per-system-zone arrays [S][R][I], radial edges [R][I+1], energy edges [N+1],
    NES shape matrix [N][N].
    """
    name: str
    S: int
    R: int
    I: int
    N: int
    c_dt: float
    r_edge: torch.Tensor
    e_edge: torch.Tensor
    temp: torch.Tensor
    kappa_a: torch.Tensor
    eta: torch.Tensor
    kappa_s: torch.Tensor
    psi_n: torch.Tensor
    nes_amp: torch.Tensor
    nes_g: torch.Tensor
    inner_bc: int = BC_ZERO_FLUX
    outer_bc: int = BC_FREE_STREAM
    terms: int = TERMS_ALL
    limiter: int = 1
    psi_floor: float = 1e-300
    r_nu: Optional[torch.Tensor] = None      # [S][N] neutrinosphere radius R_nu(eps_k) per species, cm

    @property
    def n_systems(self) -> int:
        return self.S * self.R

    @property
    def n_cells(self) -> int:
        return self.S * self.R * self.I * self.N

    def tensors(self):
        t = dict(r_edge=self.r_edge, e_edge=self.e_edge, temp=self.temp,
                 kappa_a=self.kappa_a, eta=self.eta, kappa_s=self.kappa_s,
                 psi_n=self.psi_n, nes_amp=self.nes_amp, nes_g=self.nes_g)
        if self.r_nu is not None:
            t["r_nu"] = self.r_nu
        return t

    def to(self, device) -> "Workload":
        kw = {k: v.to(device).contiguous() for k, v in self.tensors().items()}
        return dataclasses.replace(self, **kw)

    def numpy(self) -> dict:
        """All arrays as contiguous float64 numpy arrays plus the scalars."""
        out = {k: np.ascontiguousarray(v.detach().cpu().numpy()) for k, v in self.tensors().items()}
        out.update(S=self.S, R=self.R, I=self.I, N=self.N, c_dt=self.c_dt,
                   inner_bc=self.inner_bc, outer_bc=self.outer_bc, terms=self.terms,
                   limiter=self.limiter, psi_floor=self.psi_floor)
        return out

    def select_rays(self, rays: Sequence[int]) -> "Workload":
        idx = torch.as_tensor(list(rays), dtype=torch.long, device=self.r_edge.device)
        return dataclasses.replace(
            self, R=len(rays),
            r_edge=self.r_edge.index_select(0, idx).contiguous(),
            temp=self.temp.index_select(0, idx).contiguous(),
            kappa_a=self.kappa_a.index_select(1, idx).contiguous(),
            eta=self.eta.index_select(1, idx).contiguous(),
            kappa_s=self.kappa_s.index_select(1, idx).contiguous(),
            psi_n=self.psi_n.index_select(1, idx).contiguous(),
            nes_amp=self.nes_amp.index_select(1, idx).contiguous())


def _rng(cfg: int, *extra: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(SEED, spawn_key=(cfg,) + extra)))


def _group_energies(e_edge: torch.Tensor) -> torch.Tensor:
    lo, hi = e_edge[:-1], e_edge[1:]
    return torch.sqrt((hi * hi + hi * lo + lo * lo) / 3.0)


def _fermi_dirac(x: torch.Tensor) -> torch.Tensor:
    """1/(1+e^x) evaluated without overflow (e^-x/(1+e^-x) for x > 0)."""
    e = torch.exp(-x.abs())
    return torch.where(x > 0, e / (1.0 + e), 1.0 / (1.0 + e))


def _species_sign_weight(S: int):
    sign = [1.0, -1.0, 1.0, -1.0][:S]
    weight = [1.0, 1.0, 0.5, 0.5][:S]
    return sign, weight


def _profiles(cfg: int, R_full: int, I: int, rays: np.ndarray, step: int):
    """rho [R][I], T [R][I], r_edge [I+1] for the selected rays (numpy, float64)."""
    rng = _rng(cfg)
    z_rho = rng.standard_normal(R_full)
    z_T = rng.standard_normal(R_full)
    r_edge = 1e6 * 1000.0 ** (np.arange(I + 1, dtype=np.float64) / I)
    r_c = 0.5 * (r_edge[1:] + r_edge[:-1])
    x = r_c / 1e6
    rho = 1e14 * x[None, :] ** -3.0 * np.exp(0.1 * z_rho[rays])[:, None]
    T = 30.0 * x[None, :] ** -0.7 * np.exp(0.1 * z_T[rays])[:, None]
    rho = np.maximum(rho, 1e6)
    if step > 0:
        # smooth 1% drift per step, an independent phase per (ray, step) and quantity
        phase_arg = 2.0 * math.pi * np.log(x) / math.log(1000.0)
        for s in range(1, step + 1):
            drng = _rng(cfg, 2, s)
            ph_rho = drng.uniform(0.0, 2.0 * math.pi, R_full)[rays]
            ph_T = drng.uniform(0.0, 2.0 * math.pi, R_full)[rays]
            rho = rho * (1.0 + DRIFT_AMPLITUDE * np.sin(phase_arg[None, :] + ph_rho[:, None]))
            T = T * (1.0 + DRIFT_AMPLITUDE * np.sin(phase_arg[None, :] + ph_T[:, None]))
            rho = np.maximum(rho, 1e6)
    return rho, T, r_edge


def _spikes(cfg: int, R_full: int, I: int):
    """(ray ids, centre zones, multiplicative factors) of the opacity spikes."""
    rng = _rng(cfg)
    rng.standard_normal(R_full)
    rng.standard_normal(R_full)
    n = int(round(N_SPIKE_FRACTION * R_full))
    ids = rng.choice(R_full, size=n, replace=False)
    centres = rng.integers(0, I, size=n)
    factors = 10.0 * np.exp(rng.standard_normal(n))
    return ids, centres, factors


def _build(name, cfg, S, R_full, I, N, rays, step, spikes, device, c_dt=C_LIGHT * DT) -> Workload:
    rays = np.asarray(rays, dtype=np.int64)
    R = len(rays)
    rho_np, T_np, r_edge_np = _profiles(cfg, R_full, I, rays, step)
    dev = torch.device(device)
    f64 = torch.float64
    rho = torch.as_tensor(rho_np, dtype=f64, device=dev)
    T = torch.as_tensor(T_np, dtype=f64, device=dev)
    r_edge = torch.as_tensor(r_edge_np, dtype=f64, device=dev).expand(R, I + 1).contiguous()
    e_edge = 2.0 * 150.0 ** (torch.arange(N + 1, dtype=f64, device=dev) / N)
    eps = _group_energies(e_edge)                                     # [N]

    kappa_a = 1e-6 * (rho / 1e14)[:, :, None] * (eps / 10.0)[None, None, :] ** 2   # [R][I][N]
    sign, weight = _species_sign_weight(S)
    ka, et, ks, pn = [], [], [], []
    for q in range(S):
        mu = sign[q] * 2.0 * T
        x = (eps[None, None, :] - mu[:, :, None]) / T[:, :, None]
        f = _fermi_dirac(x)
        eta_q = weight[q] * kappa_a * torch.exp(-x)
        ka.append(kappa_a)
        et.append(eta_q)
        ks.append(2.0 * kappa_a)
        pn.append(0.9 * f)
    kappa_a = torch.stack(ka).contiguous()
    eta = torch.stack(et).contiguous()
    kappa_s = torch.stack(ks).contiguous()
    psi_n = torch.stack(pn).contiguous()

    if spikes:
        ids, centres, factors = _spikes(cfg, R_full, I)
        pos = {int(r): j for j, r in enumerate(rays)}
        for rid, c, fac in zip(ids, centres, factors):
            if int(rid) not in pos:
                continue
            j = pos[int(rid)]
            lo, hi = max(0, int(c) - SPIKE_HALF_WIDTH), min(I, int(c) + SPIKE_HALF_WIDTH + 1)
            kappa_a[:, j, lo:hi, :] *= fac
            eta[:, j, lo:hi, :] *= fac
            kappa_s[:, j, lo:hi, :] *= fac

    nes_amp = (1e-7 * rho / 1e14)[None].expand(S, R, I).contiguous()
    le = torch.log(eps)
    nes_g = torch.exp(-((le[:, None] - le[None, :]) ** 2) / (2.0 * 0.3 ** 2)).contiguous()
    r_nu = (R_NU_CM * torch.sqrt(eps / 10.0))[None].expand(S, N).contiguous()
    return Workload(name=name, S=S, R=R, I=I, N=N, c_dt=float(c_dt), r_edge=r_edge,
                    e_edge=e_edge.contiguous(), temp=T.contiguous(), kappa_a=kappa_a, eta=eta,
                    kappa_s=kappa_s, psi_n=psi_n, nes_amp=nes_amp, nes_g=nes_g, r_nu=r_nu)


@dataclasses.dataclass
class YeInputs:
    """Extra inputs of the Y_e-coupled step for species 0 (nu_e) and 1 (anti-nu_e) of a workload.

    rho [R][I] g/cm^3 and ye_n [R][I]; dka_dye, deta_dye [2][R][I][N] cm^-1 (derivatives of the
    absorption and emission opacities of the two species with respect to Y_e); de_dT [R][I]
    (MeV per baryon per MeV) and de_dye [R][I] (MeV per baryon), the matter's internal-energy
    derivatives used by the post-solve temperature update.
    """
    rho: torch.Tensor
    ye_n: torch.Tensor
    dka_dye: torch.Tensor
    deta_dye: torch.Tensor
    de_dT: torch.Tensor
    de_dye: torch.Tensor
    pair_amp: Optional[torch.Tensor] = None    # [R][I] cm^-1, amplitude of the nu_e / anti-nu_e pair kernels
    pair_g: Optional[torch.Tensor] = None      # [N][N] symmetric pair-kernel shape
    pair_eta1: Optional[torch.Tensor] = None   # [2][R][I][N] flux factors psi1/psi0 of nu_e, anti-nu_e

    def to(self, device):
        return YeInputs(**{f.name: (None if getattr(self, f.name) is None else getattr(self, f.name).to(device))
                           for f in dataclasses.fields(self)})

    def numpy(self) -> dict:
        return {f.name: getattr(self, f.name).detach().cpu().numpy() for f in dataclasses.fields(self)
                if getattr(self, f.name) is not None}


def ye_inputs(w: Workload, cfg: int, rays: Optional[Sequence[int]] = None, step: int = 0,
              R_full: Optional[int] = None, pairs: bool = False) -> YeInputs:
    """Synthetic Y_e-coupling data for workload `w` (made by `make(cfg, rays=rays, step=step, ...)`,
    or by `make_custom(seed_cfg=cfg, R=R_full, ...)` with `R_full` given).

    * rho: the workload's own density profile (same seeds);
    * Y_e^n(r) = 0.5 - 0.22 exp(-((log10 r - 6)/0.8)^2): 0.28 at the inner edge, 0.5 outside;
    * absorption on free nucleons: kappa_a of nu_e scales with the neutron fraction 1 - Y_e and that
      of anti-nu_e with the proton fraction Y_e, so dkappa_a/dY_e = -kappa_a/(1 - Y_e) and
      +kappa_a/Y_e; the emissivities follow at fixed chemical potentials, deta/dY_e = eta (dkappa_a/dY_e)/kappa_a;
    * de/dT = 1.5 + 0.5 T/MeV and de/dY_e = -10 T (MeV per baryon): smooth stand-ins for the EoS;
    * with `pairs`: nu_e / anti-nu_e pair kernels of amplitude 1e-7 (T/10 MeV)^3 cm^-1 and symmetric shape
      (eps_k eps_k'/(10 MeV)^2) exp(-(ln eps_k - ln eps_k')^2 / (2 0.5^2)), and flux factors
      psi1/psi0 = x^2/(1 + x^2), x = r / R_nu(eps) (0 deep inside the neutrinosphere, towards 1 outside).
    """
    if w.S < 2:
        raise ValueError("the Y_e coupling needs species 0 (nu_e) and 1 (anti-nu_e)")
    if R_full is None:
        R_full = CONFIGS[cfg]["R"]
    if rays is None:
        rays = range(R_full)
    rays = np.asarray(rays, dtype=np.int64)
    rho_np, _, _ = _profiles(cfg, R_full, w.I, rays, step)
    dev = w.kappa_a.device
    f64 = torch.float64
    rho = torch.as_tensor(rho_np, dtype=f64, device=dev).contiguous()
    rc = 0.5 * (w.r_edge[:, :-1] + w.r_edge[:, 1:])
    ye_n = (0.5 - 0.22 * torch.exp(-((torch.log10(rc) - 6.0) / 0.8) ** 2)).contiguous()
    frac = torch.stack([-1.0 / (1.0 - ye_n), 1.0 / ye_n])[:, :, :, None]        # [2][R][I][1]
    dka = (frac * w.kappa_a[:2]).contiguous()
    deta = (frac * w.eta[:2]).contiguous()
    de_dT = (1.5 + 0.5 * w.temp).contiguous()
    de_dye = (-10.0 * w.temp).contiguous()
    y = YeInputs(rho=rho, ye_n=ye_n, dka_dye=dka, deta_dye=deta, de_dT=de_dT, de_dye=de_dye)
    if pairs:
        eps = _group_energies(w.e_edge.to(dev))
        le = torch.log(eps)
        g = (eps[:, None] * eps[None, :] / 100.0) * torch.exp(-((le[:, None] - le[None, :]) ** 2) / (2.0 * 0.5 ** 2))
        x = rc[None, :, :, None] / w.r_nu[:2].to(dev)[:, None, None, :]                # [2][R][I][N]
        y = dataclasses.replace(y, pair_amp=(1e-7 * (w.temp / 10.0) ** 3).contiguous(), pair_g=g.contiguous(),
                                pair_eta1=(x * x / (1.0 + x * x)).contiguous())
    return y


@dataclasses.dataclass
class EadvInputs:
    """Inputs of the energy-advection step of a workload between its drift steps `step` and `step + 1`.

    rho_old, rho_new [R][I] g/cm^3; lapse_old, lapse_new [R][I]; dlnR, dlnb [R][I] (fractional changes
    of the areal radius and of the radial stretch over the hydro step); eddington [S][R][I][N].
    """
    rho_old: torch.Tensor
    rho_new: torch.Tensor
    lapse_old: torch.Tensor
    lapse_new: torch.Tensor
    dlnR: torch.Tensor
    dlnb: torch.Tensor
    eddington: torch.Tensor

    def numpy(self) -> dict:
        return {f.name: getattr(self, f.name).cpu().numpy() for f in dataclasses.fields(self)}


LAPSE_R0_CM = 2.04e5        # the paper's redshift test: a(R) = sqrt(1 - R0/R), R0 = 2.04 km


def eadv_inputs(w: Workload, cfg: int, rays: Optional[Sequence[int]] = None, step: int = 0,
                R_full: Optional[int] = None) -> EadvInputs:
    """Synthetic energy-advection inputs for workload `w` (made by `make(cfg, rays=rays, step=step)`).

    * rho before and after: the workload's density at drift steps `step` and `step + 1`;
    * a homologous stand-in for the hydro step, dR/R = db/b = -(1/3) ln(rho_new/rho_old);
    * lapse a = sqrt(1 - R0/r) at the zone centre, with R0 growing by 1% per step;
    * Eddington factor 1/3 + (2/3) x^2/(1 + x^2), x = r / (R_nu (eps/10 MeV)^0.5): 1/3 (diffusion) deep
      inside, rising towards 1 (free streaming) outside a group-dependent neutrinosphere.
    """
    if R_full is None:
        R_full = CONFIGS[cfg]["R"]
    if rays is None:
        rays = range(R_full)
    rays = np.asarray(rays, dtype=np.int64)
    rho0, _, r_edge = _profiles(cfg, R_full, w.I, rays, step)
    rho1, _, _ = _profiles(cfg, R_full, w.I, rays, step + 1)
    dev = w.kappa_a.device
    f64 = torch.float64
    rc = 0.5 * (r_edge[1:] + r_edge[:-1])
    a0 = np.sqrt(1.0 - LAPSE_R0_CM * 1.01 ** step / rc)
    a1 = np.sqrt(1.0 - LAPSE_R0_CM * 1.01 ** (step + 1) / rc)
    dln = -np.log(rho1 / rho0) / 3.0
    eps = _group_energies(w.e_edge.to(dev)).cpu().numpy()
    x = rc[:, None] / (R_NU_CM * np.sqrt(eps / 10.0))[None, :]                 # [I][N]
    edd = 1.0 / 3.0 + (2.0 / 3.0) * x * x / (1.0 + x * x)
    t = lambda v: torch.as_tensor(np.ascontiguousarray(v), dtype=f64, device=dev)
    R = len(rays)
    zone = lambda v: t(np.broadcast_to(v, (R, w.I)))
    return EadvInputs(rho_old=t(rho0), rho_new=t(rho1), lapse_old=zone(a0), lapse_new=zone(a1), dlnR=t(dln),
                      dlnb=t(dln), eddington=t(edd).expand(w.S, R, w.I, w.N).contiguous())


def make(cfg: int, *, rays: Optional[Sequence[int]] = None, zones: Optional[int] = None,
         groups: Optional[int] = None, species: Optional[int] = None, step: int = 0,
         device="cpu") -> Workload:
    """Inputs of workload `cfg` (0..4).

    `rays` selects a subset of the configuration's rays (per-ray random draws are
    made for the full ray count, so a subset equals the same rays of the full
    workload).  `zones`, `groups`, `species` shrink the shape for quick tests
    while keeping the recipe.  `step` applies that many drift steps (multi-step case).
    """
    c = CONFIGS[cfg]
    R_full = c["R"]
    I = zones or c["I"]
    N = groups or c["N"]
    S = species or c["S"]
    if rays is None:
        rays = range(R_full)
    spikes = cfg == 2
    name = c["name"]
    return _build(name, cfg, S, R_full, I, N, rays, step, spikes, device)


def make_custom(*, S=1, R=2, I=16, N=8, seed_cfg=0, device="cpu", **kw) -> Workload:
    """A small workload with the standard recipe at an arbitrary shape."""
    w = _build(f"custom-{R}r-{I}z-{N}g-{S}s", seed_cfg, S, R, I, N, range(R), 0, False, device)
    return dataclasses.replace(w, **kw)
