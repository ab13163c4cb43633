"""MI355X-native Trotter-step engine for the graph tensor-network quantum
annealer of arXiv:2409.12240.

The compute path is libgtqa.so (HIP kernels for gfx950 behind the C ABI of
include/gtqa.h); `gtqa` is its ctypes binding and `serve` the
continuous-batching request loop built on the pool API.
"""

__all__ = ["gtqa"]
