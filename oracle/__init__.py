"""CPU oracle for the implicit ray-by-ray MGFLD transport step (TEST INFRASTRUCTURE).

A plain, slow, FP64 NumPy implementation of what the device path computes,
written from the paper (Bruenn et al., CHIMERA, arXiv 1809.05608): Neutrino
Transport section, "Lagrangian Transport Step" (eqs. a57-a62) and "Solution of
the Transport Equations" (eqs. a62aa-a62af); Transport Sources section
(eqs. d1-d8c, d10, d40).

Only `tests/`, `__graft_entry__.smoke()` and the `cpu_baseline` leg of
`bench.py` may import this package.  It shares no code with the HIP path and
must never be used as a fallback for it.

The Y_e-coupled step (electron-fraction equation, eq. a62a, and the temperature update, eqs.
a62b and a62d) is in `oracle.ye_coupled`; the energy-advection step (Lagrangian energy shift,
PPM remap, Pauli over-fill limiter, lapse remap; eqs. a78-a81d, p1-p8) in
`oracle.energy_advection`, pinned by `tests/test_oracle_energy.py`.

Parity status: every function below is pinned by `tests/test_oracle_pins.py`
(closed forms, invariants, brute-force dense solves, finite differences);
none is "parity unpinned".  The synthetic-workload recipe itself (module
`synth`) is a generator choice and is not pinned by the paper.
"""
from .transport import (  # noqa: F401
    System, systems_from_workload, group_energies, geometry, nes_kernels, edge_flux,
    residual, jacobian_blocks, dense_jacobian, block_thomas_solve, dense_solve,
    newton, step_stats, luminosity, luminosity_seed, adjoint, param_vjp,
    newton_batch, residual_batch, multistep_forward, multistep_objective, multistep_adjoint,
)
from . import ye_coupled  # noqa: F401
from . import energy_advection  # noqa: F401
