"""MI355X-native BDDC-preconditioned CG for unfitted (cut-cell) Q1 meshes.

The product is libcutbddc.so (HIP kernels for gfx950 behind the C ABI of
include/cutbddc.h); `cutbddc` is its ctypes binding and `autograd` wraps the
solve in a torch.autograd.Function.
"""
from .cutbddc import BatchSolver, Solver, CBError, load_library, LIB_PATH  # noqa: F401
