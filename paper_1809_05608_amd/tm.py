"""Python binding of libtm (include/tm.h): argument marshalling only.

Every step of the transport path runs in the HIP kernels of libtm.so; this module
checks tensor shapes/dtypes/devices, passes raw device pointers and the current
HIP stream through ctypes, and turns status codes into exceptions.  PyTorch is
used for device memory and streams only.  There is no CPU fallback: importing
works without a GPU, but every call raises if the library or a device is missing.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtm.so")

TM_OK = 0
STATUS_NAMES = {0: "TM_OK", 1: "TM_ERR_INVALID_ARG", 2: "TM_ERR_HIP", 3: "TM_ERR_SINGULAR",
                4: "TM_ERR_NOT_CONVERGED", 5: "TM_ERR_NONFINITE", 6: "TM_ERR_WORKSPACE"}
TERM_DIFFUSION, TERM_EMABS, TERM_NES = 1, 2, 4
PREC_FP64, PREC_MIXED = 0, 1
FLAG_NOT_CONVERGED, FLAG_NONFINITE, FLAG_ZERO_PIVOT, FLAG_PIVOT_FALLBACK = 1, 2, 4, 8
EADV_LAGRANGIAN, EADV_LAPSE = 0, 1
EADV_FLAG_DISPLACEMENT, EADV_FLAG_OVERFILL, EADV_FLAG_OVERFILL_CLAMP = 1, 2, 4

EXPORTED = ["tm_create", "tm_destroy", "tm_workspace_bytes", "tm_set_workspace", "tm_assemble",
            "tm_factor_solve", "tm_factor_solve_noalloc", "tm_newton_step", "tm_adjoint_step", "tm_luminosity_seed", "tm_ye_workspace_bytes",
            "tm_ye_newton_step", "tm_temperature_update", "tm_energy_advect", "tm_set_kernel_timing",
            "tm_kernel_time_ms", "tm_status_string", "tm_last_error"]


class TMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_rays", ctypes.c_int32), ("n_zones", ctypes.c_int32),
                ("n_groups", ctypes.c_int32), ("c_dt", ctypes.c_double), ("inner_bc", ctypes.c_int32),
                ("outer_bc", ctypes.c_int32), ("terms", ctypes.c_uint32), ("limiter", ctypes.c_int32),
                ("psi_floor", ctypes.c_double), ("precision", ctypes.c_int32)]


class Inputs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("r_edge", "e_edge", "kappa_a", "eta", "kappa_s", "temp", "nes_amp", "nes_g", "lapse", "lapse_edge",
                 "r_nu")]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("res_inf", "res0_inf", "n_tot", "e_tot", "budget_n", "lum_n", "iters", "flags")]


class YeInputs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("rho", "ye_n", "dka_dye", "deta_dye", "pair_amp", "pair_g",
                                               "pair_eta1")]


class EadvInputs(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32)] + [(n, ctypes.c_void_p) for n in
                                             ("rho_old", "rho_new", "lapse_old", "lapse_new", "dlnR", "dlnb",
                                              "eddington")]


class YeStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("res_inf", "res0_inf", "lepton", "iters", "flags")]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libtm.so and declare its C signatures (no device is touched)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libtm.so not built at {path}; run `python -m paper_1809_05608_amd.build`")
    lib = ctypes.CDLL(path)
    P, V, D, I32 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_double, ctypes.c_int32
    lib.tm_create.argtypes = [P(Problem), V, P(V)]
    lib.tm_destroy.argtypes = [V]
    lib.tm_workspace_bytes.argtypes = [P(Problem), ctypes.c_int64]
    lib.tm_workspace_bytes.restype = ctypes.c_size_t
    lib.tm_set_workspace.argtypes = [V, V, ctypes.c_size_t]
    lib.tm_assemble.argtypes = [V, P(Inputs), V, V, V, V]
    lib.tm_factor_solve.argtypes = [V, P(Inputs), V, V, V, I32]
    lib.tm_factor_solve_noalloc.argtypes = [V, P(Inputs), V, V, V, I32, V]
    lib.tm_newton_step.argtypes = [V, P(Inputs), V, V, I32, D, P(Stats)]
    lib.tm_adjoint_step.argtypes = [V, P(Inputs), V, V, V, V, V, V, V, V]
    lib.tm_luminosity_seed.argtypes = [V, P(Inputs), V, V]
    lib.tm_ye_workspace_bytes.argtypes = [P(Problem), ctypes.c_int64]
    lib.tm_ye_workspace_bytes.restype = ctypes.c_size_t
    lib.tm_ye_newton_step.argtypes = [V, P(Inputs), P(YeInputs), V, V, V, I32, D, P(YeStats)]
    lib.tm_temperature_update.argtypes = [V, P(Inputs), P(YeInputs), V, V, P(D), V, V, V, V]
    lib.tm_energy_advect.argtypes = [V, P(Inputs), P(EadvInputs), V, V, V]
    lib.tm_set_kernel_timing.argtypes = [V, I32]
    lib.tm_kernel_time_ms.argtypes = [V, P(D)]
    lib.tm_status_string.argtypes = [ctypes.c_int]
    lib.tm_status_string.restype = ctypes.c_char_p
    lib.tm_last_error.argtypes = [V]
    lib.tm_last_error.restype = ctypes.c_char_p
    for name in ("tm_create", "tm_destroy", "tm_set_workspace", "tm_assemble", "tm_factor_solve",
                 "tm_factor_solve_noalloc",
                 "tm_newton_step", "tm_adjoint_step", "tm_luminosity_seed", "tm_ye_newton_step",
                 "tm_temperature_update", "tm_energy_advect", "tm_set_kernel_timing", "tm_kernel_time_ms"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def make_problem(S, R, I, N, c_dt, *, outer_bc=1, terms=7, limiter=1, psi_floor=1e-300,
                 precision=PREC_FP64) -> Problem:
    return Problem(S, R, I, N, float(c_dt), 0, outer_bc, terms, limiter, float(psi_floor), precision)


def problem_of(w, precision=PREC_FP64) -> Problem:
    """tm_problem of a synth.Workload."""
    return make_problem(w.S, w.R, w.I, w.N, w.c_dt, outer_bc=w.outer_bc, terms=w.terms,
                        limiter=w.limiter, psi_floor=w.psi_floor, precision=precision)


@dataclasses.dataclass
class DeviceFields:
    """The tm_inputs arrays as device float64 tensors."""
    r_edge: torch.Tensor
    e_edge: torch.Tensor
    kappa_a: torch.Tensor
    eta: torch.Tensor
    kappa_s: torch.Tensor
    temp: torch.Tensor
    nes_amp: torch.Tensor
    nes_g: torch.Tensor
    lapse: Optional[torch.Tensor] = None        # [R][I] lapse at zone centres (None: a = 1)
    lapse_edge: Optional[torch.Tensor] = None   # [R][I+1] lapse at zone edges
    r_nu: Optional[torch.Tensor] = None         # [S][N] neutrinosphere radii (geometric limiter / boundary)

    @classmethod
    def of(cls, w, **override):
        d = {k: getattr(w, k) for k in ("r_edge", "e_edge", "kappa_a", "eta", "kappa_s", "temp",
                                         "nes_amp", "nes_g")}
        d["r_nu"] = getattr(w, "r_nu", None)
        d.update(override)
        return cls(**d)


class Context:
    """One tm_ctx: a problem shape bound to the current HIP stream of the current device."""

    def __init__(self, problem: Problem, stream: Optional[torch.cuda.Stream] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("libtm needs a ROCm GPU; none is visible")
        self.lib = load_library()
        self.problem = problem
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream or torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = self.lib.tm_create(ctypes.byref(problem), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != TM_OK:
            raise TMError(st, "tm_create failed")
        self._h = h
        self._ws = None

    def close(self):
        if getattr(self, "_h", None):
            self.lib.tm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ helpers
    @property
    def shape_cell(self):
        p = self.problem
        return (p.n_species, p.n_rays, p.n_zones, p.n_groups)

    def _check(self, st: int):
        if st != TM_OK:
            msg = self.lib.tm_last_error(self._h)
            raise TMError(st, msg.decode() if msg else "")

    def _cell(self, t: torch.Tensor, name: str):
        if t is None:
            raise ValueError(f"{name} is required")
        if t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor on {self.device}")
        if tuple(t.shape) != self.shape_cell:
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {self.shape_cell}")
        return t

    def _inputs(self, f: DeviceFields) -> Inputs:
        p = self.problem
        exp = {"r_edge": (p.n_rays, p.n_zones + 1), "e_edge": (p.n_groups + 1,), "kappa_a": self.shape_cell,
               "eta": self.shape_cell, "kappa_s": self.shape_cell, "temp": (p.n_rays, p.n_zones),
               "nes_amp": (p.n_species, p.n_rays, p.n_zones), "nes_g": (p.n_groups, p.n_groups)}
        if (f.lapse is None) != (f.lapse_edge is None):
            raise ValueError("lapse and lapse_edge go together")
        if f.lapse is not None:
            exp.update(lapse=(p.n_rays, p.n_zones), lapse_edge=(p.n_rays, p.n_zones + 1))
        if f.r_nu is not None:
            exp.update(r_nu=(p.n_species, p.n_groups))
        for name, shape in exp.items():
            t = getattr(f, name)
            if t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float64 tensor on {self.device}")
            if tuple(t.shape) != shape:
                raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")
        self._keep = f
        return Inputs(*[_ptr(getattr(f, n)) for n in ("r_edge", "e_edge", "kappa_a", "eta", "kappa_s", "temp",
                                                       "nes_amp", "nes_g", "lapse", "lapse_edge", "r_nu")])

    def set_workspace(self, nbytes: int):
        """Give the context a caller-owned workspace of `nbytes` (a torch uint8 tensor)."""
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._check(self.lib.tm_set_workspace(self._h, _ptr(self._ws), ctypes.c_size_t(nbytes)))

    def workspace_bytes(self, batch_systems: int = 0) -> int:
        return int(self.lib.tm_workspace_bytes(ctypes.byref(self.problem), batch_systems))

    # ------------------------------------------------------------------ entry points
    def assemble(self, f: DeviceFields, psi_n, psi, residual, blocks=None):
        self._cell(psi_n, "psi_n"), self._cell(psi, "psi"), self._cell(residual, "residual")
        if blocks is not None:
            p = self.problem
            want = self.shape_cell + (p.n_groups + 2,)
            if tuple(blocks.shape) != want or blocks.dtype != torch.float64 or not blocks.is_contiguous():
                raise ValueError(f"blocks must be contiguous float64 of shape {want}")
        inp = self._inputs(f)
        self._check(self.lib.tm_assemble(self._h, ctypes.byref(inp), _ptr(psi_n), _ptr(psi), _ptr(residual),
                                         _ptr(blocks)))

    def factor_solve(self, f: DeviceFields, psi, rhs, x, transpose=False):
        self._cell(psi, "psi"), self._cell(rhs, "rhs"), self._cell(x, "x")
        inp = self._inputs(f)
        self._check(self.lib.tm_factor_solve(self._h, ctypes.byref(inp), _ptr(psi), _ptr(rhs), _ptr(x),
                                             int(bool(transpose))))

    def set_kernel_timing(self, enable: bool):
        """Bracket the diagonal-pivot factor launches of later solves with HIP events (measurement aid)."""
        self._check(self.lib.tm_set_kernel_timing(self._h, 1 if enable else 0))

    def kernel_time_ms(self) -> float:
        """Milliseconds between the events of the last bracketed factor launch (waits for it)."""
        ms = ctypes.c_double(0.0)
        self._check(self.lib.tm_kernel_time_ms(self._h, ctypes.byref(ms)))
        return ms.value

    def factor_solve_noalloc(self, f: DeviceFields, psi, rhs, x, transpose=False, flags=None):
        """tm_factor_solve_noalloc: the solve with the library's static scratch (no allocation, no
        synchronisation); `flags` (int32 [S][R] on the device) receives the per-system flag bits."""
        self._cell(psi, "psi"), self._cell(rhs, "rhs"), self._cell(x, "x")
        if flags is not None:
            p = self.problem
            if (flags.dtype != torch.int32 or flags.device != self.device or not flags.is_contiguous()
                    or tuple(flags.shape) != (p.n_species, p.n_rays)):
                raise ValueError(f"flags must be a contiguous int32 tensor of shape {(p.n_species, p.n_rays)}")
        inp = self._inputs(f)
        self._check(self.lib.tm_factor_solve_noalloc(self._h, ctypes.byref(inp), _ptr(psi), _ptr(rhs), _ptr(x),
                                                     int(bool(transpose)), _ptr(flags)))

    def newton_step(self, f: DeviceFields, psi_n, psi, max_iter: int, rtol: float, with_stats=True,
                    raise_on_status=True):
        """Run the Newton iteration in place on psi; returns (status, stats dict of device tensors)."""
        self._cell(psi_n, "psi_n"), self._cell(psi, "psi")
        inp = self._inputs(f)
        ns = self.problem.n_species * self.problem.n_rays
        stats = None
        st_struct = None
        if with_stats:
            d = dict(device=self.device)
            stats = {n: torch.empty(ns, dtype=torch.float64, **d) for n in
                     ("res_inf", "res0_inf", "n_tot", "e_tot", "budget_n", "lum_n")}
            stats.update({n: torch.empty(ns, dtype=torch.int32, **d) for n in ("iters", "flags")})
            st_struct = Stats(*[_ptr(stats[n]) for n in ("res_inf", "res0_inf", "n_tot", "e_tot", "budget_n",
                                                          "lum_n", "iters", "flags")])
        st = self.lib.tm_newton_step(self._h, ctypes.byref(inp), _ptr(psi_n), _ptr(psi), int(max_iter),
                                     float(rtol), ctypes.byref(st_struct) if st_struct is not None else None)
        if raise_on_status and st not in (TM_OK,):
            self._check(st)
        return st, stats

    def adjoint_step(self, f: DeviceFields, psi_n, psi_np1, seed, mu, g_kappa_a=None, g_eta=None,
                     g_kappa_s=None, g_nes_amp=None):
        self._cell(psi_np1, "psi_np1"), self._cell(seed, "seed"), self._cell(mu, "mu")
        for name, t in (("g_kappa_a", g_kappa_a), ("g_eta", g_eta), ("g_kappa_s", g_kappa_s)):
            if t is not None:
                self._cell(t, name)
        inp = self._inputs(f)
        self._check(self.lib.tm_adjoint_step(self._h, ctypes.byref(inp), _ptr(psi_n), _ptr(psi_np1), _ptr(seed),
                                             _ptr(mu), _ptr(g_kappa_a), _ptr(g_eta), _ptr(g_kappa_s),
                                             _ptr(g_nes_amp)))

    # ------------------------------------------------------------------ Y_e-coupled step
    def _zone(self, t: torch.Tensor, name: str):
        p = self.problem
        if t is None:
            raise ValueError(f"{name} is required")
        if t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor on {self.device}")
        if tuple(t.shape) != (p.n_rays, p.n_zones):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {(p.n_rays, p.n_zones)}")
        return t

    def _ye_inputs(self, y) -> YeInputs:
        """y: an object with rho, ye_n [R][I] and dka_dye, deta_dye [2][R][I][N] device tensors."""
        p = self.problem
        self._zone(y.rho, "rho"), self._zone(y.ye_n, "ye_n")
        pair = (2, p.n_rays, p.n_zones, p.n_groups)
        for name in ("dka_dye", "deta_dye"):
            t = getattr(y, name)
            if t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous() or tuple(t.shape) != pair:
                raise ValueError(f"{name} must be a contiguous float64 tensor of shape {pair} on {self.device}")
        extra = {}
        if getattr(y, "pair_amp", None) is not None:
            self._zone(y.pair_amp, "pair_amp")
            for name, shape in (("pair_g", (p.n_groups, p.n_groups)), ("pair_eta1", pair)):
                t = getattr(y, name)
                if t is None or t.dtype != torch.float64 or t.device != self.device or not t.is_contiguous() \
                        or tuple(t.shape) != shape:
                    raise ValueError(f"{name} must be a contiguous float64 tensor of shape {shape} on {self.device}")
            extra = {n: getattr(y, n) for n in ("pair_amp", "pair_g", "pair_eta1")}
        self._keep_ye = y
        return YeInputs(*[_ptr(getattr(y, n)) for n in ("rho", "ye_n", "dka_dye", "deta_dye")],
                        *[_ptr(extra.get(n)) for n in ("pair_amp", "pair_g", "pair_eta1")])

    def ye_workspace_bytes(self, batch_rays: int = 0) -> int:
        return int(self.lib.tm_ye_workspace_bytes(ctypes.byref(self.problem), batch_rays))

    def ye_newton_step(self, f: DeviceFields, y, psi_n, psi, ye, max_iter: int, rtol: float, with_stats=True,
                       raise_on_status=True):
        """Coupled Newton iteration for species 0, 1 and Y_e, in place on psi and ye; returns (status, stats)."""
        self._cell(psi_n, "psi_n"), self._cell(psi, "psi"), self._zone(ye, "ye")
        inp, yin = self._inputs(f), self._ye_inputs(y)
        R = self.problem.n_rays
        stats = None
        st_struct = None
        if with_stats:
            d = dict(device=self.device)
            stats = {n: torch.empty(R, dtype=torch.float64, **d) for n in ("res_inf", "res0_inf", "lepton")}
            stats.update({n: torch.empty(R, dtype=torch.int32, **d) for n in ("iters", "flags")})
            st_struct = YeStats(*[_ptr(stats[n]) for n in ("res_inf", "res0_inf", "lepton", "iters", "flags")])
        st = self.lib.tm_ye_newton_step(self._h, ctypes.byref(inp), ctypes.byref(yin), _ptr(psi_n), _ptr(psi),
                                        _ptr(ye), int(max_iter), float(rtol),
                                        ctypes.byref(st_struct) if st_struct is not None else None)
        if raise_on_status and st != TM_OK:
            self._check(st)
        return st, stats

    def temperature_update(self, f: DeviceFields, y, psi, ye, stat_weights, de_dT, de_dye, temp_out, de_out=None):
        """Matter energy change and temperature after the step (zone arrays temp_out, de_out)."""
        self._cell(psi, "psi"), self._zone(ye, "ye"), self._zone(de_dT, "de_dT"), self._zone(de_dye, "de_dye")
        self._zone(temp_out, "temp_out")
        if de_out is not None:
            self._zone(de_out, "de_out")
        S = self.problem.n_species
        if len(stat_weights) != S:
            raise ValueError(f"stat_weights needs {S} values")
        w = (ctypes.c_double * S)(*[float(v) for v in stat_weights])
        inp, yin = self._inputs(f), self._ye_inputs(y)
        self._check(self.lib.tm_temperature_update(self._h, ctypes.byref(inp), ctypes.byref(yin), _ptr(psi), _ptr(ye),
                                                   w, _ptr(de_dT), _ptr(de_dye), _ptr(de_out), _ptr(temp_out)))

    def energy_advect(self, e_edge, psi, *, mode=EADV_LAGRANGIAN, rho_old=None, rho_new=None, lapse_old=None,
                      lapse_new=None, dlnR=None, dlnb=None, eddington=None, xi=None, flags=None):
        """Energy-advection update of psi in place (eqs. a78-a81d, or the lapse remap of eqs. p1-p8).

        e_edge [N+1]; zone arrays [R][I]; eddington a cell array; xi (float64) and flags (int32) [S][R][I]."""
        p = self.problem
        self._cell(psi, "psi")
        if e_edge.dtype != torch.float64 or e_edge.device != self.device or tuple(e_edge.shape) != (p.n_groups + 1,):
            raise ValueError(f"e_edge must be a float64 tensor of shape {(p.n_groups + 1,)} on {self.device}")
        zones = {"rho_old": rho_old, "rho_new": rho_new, "lapse_old": lapse_old, "lapse_new": lapse_new,
                 "dlnR": dlnR, "dlnb": dlnb}
        for name, t in zones.items():
            if t is not None:
                self._zone(t, name)
        if eddington is not None:
            self._cell(eddington, "eddington")
        sysz = (p.n_species, p.n_rays, p.n_zones)
        for name, t, dt in (("xi", xi, torch.float64), ("flags", flags, torch.int32)):
            if t is not None and (t.dtype != dt or t.device != self.device or not t.is_contiguous()
                                  or tuple(t.shape) != sysz):
                raise ValueError(f"{name} must be a contiguous {dt} tensor of shape {sysz} on {self.device}")
        inp = Inputs(None, _ptr(e_edge), None, None, None, None, None, None)
        ea = EadvInputs(int(mode), *[_ptr(zones[n]) for n in ("rho_old", "rho_new", "lapse_old", "lapse_new",
                                                              "dlnR", "dlnb")], _ptr(eddington))
        self._check(self.lib.tm_energy_advect(self._h, ctypes.byref(inp), ctypes.byref(ea), _ptr(psi), _ptr(xi),
                                              _ptr(flags)))

    def luminosity_seed(self, f: DeviceFields, seed, add=None):
        """seed = dL_N/dpsi (outer-boundary number luminosity) + add (cell arrays)."""
        self._cell(seed, "seed")
        if add is not None:
            self._cell(add, "add")
        inp = self._inputs(f)
        self._check(self.lib.tm_luminosity_seed(self._h, ctypes.byref(inp), _ptr(add), _ptr(seed)))


# ---------------------------------------------------------------------- autograd

class TransportStep(torch.autograd.Function):
    """psi^{n+1} = step(kappa_a, eta, kappa_s, psi^n) with a hand-written adjoint.

    forward: tm_newton_step (converged to `rtol`); backward: tm_adjoint_step, which
    solves J(psi^{n+1})^T mu = grad and returns -mu^T dG/dtheta for the opacities and
    mu for psi^n.  The fixed inputs (grids, temperature, NES kernel) carry no gradient.
    """

    @staticmethod
    def forward(ctx, kappa_a, eta, kappa_s, psi_n, tmctx: Context, fixed: DeviceFields, max_iter: int, rtol: float):
        f = dataclasses.replace(fixed, kappa_a=kappa_a.contiguous(), eta=eta.contiguous(), kappa_s=kappa_s.contiguous())
        psi = psi_n.detach().clone()
        tmctx.newton_step(f, psi_n.detach().contiguous(), psi, max_iter, rtol, with_stats=False)
        ctx.tmctx = tmctx
        ctx.fixed = fixed
        ctx.save_for_backward(kappa_a, eta, kappa_s, psi_n, psi)
        return psi

    @staticmethod
    def backward(ctx, grad):
        kappa_a, eta, kappa_s, psi_n, psi = ctx.saved_tensors
        f = dataclasses.replace(ctx.fixed, kappa_a=kappa_a.contiguous(), eta=eta.contiguous(),
                                kappa_s=kappa_s.contiguous())
        mu = torch.empty_like(psi)
        need = ctx.needs_input_grad
        gka = torch.empty_like(psi) if need[0] else None
        get = torch.empty_like(psi) if need[1] else None
        gks = torch.empty_like(psi) if need[2] else None
        ctx.tmctx.adjoint_step(f, psi_n, psi, grad.contiguous(), mu, gka, get, gks, None)
        return gka, get, gks, (mu if need[3] else None), None, None, None, None
