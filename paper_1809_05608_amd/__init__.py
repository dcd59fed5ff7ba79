"""MI355X-native implicit ray-by-ray MGFLD neutrino-transport step (CHIMERA, arXiv 1809.05608).

The compute path is libtm.so (HIP kernels for gfx950 behind the C ABI of
include/tm.h); `paper_1809_05608_amd.tm` is its ctypes binding.
"""
from .tm import (  # noqa: F401
    Context, DeviceFields, Problem, TMError, TransportStep, load_library,
    make_problem, problem_of, PREC_FP64, PREC_MIXED,
)
