"""GPU fill of seeded payloads (same bytes as synth.gen.payload), for inputs too
large to generate on the host.  Loads synth/libsynth.so (built by the package
build); raises ImportError if it is missing."""

import ctypes
import os

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsynth.so")
if not os.path.exists(LIB):
    raise ImportError("synth/libsynth.so is not built")
try:   # torch's HIP runtime first (the library links the system one)
    import torch as _torch
    if _torch.cuda.is_available():
        _torch.cuda.init()
except ImportError:
    pass
_lib = ctypes.CDLL(LIB)
_lib.synth_fill.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                            ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]
_lib.synth_fill.restype = ctypes.c_int

DATA, UPDATE_DATA = 2, 6


def fill(tensor, seed, stripe, t, first_block=0, purpose=DATA, stream=None):
    """Fill a contiguous uint8 CUDA tensor holding nblocks x t bytes."""
    import torch
    assert tensor.is_cuda and tensor.is_contiguous() and tensor.numel() % t == 0
    s = torch.cuda.current_stream().cuda_stream if stream is None else getattr(stream, "cuda_stream", stream)
    rc = _lib.synth_fill(tensor.data_ptr(), tensor.numel() // t, t, first_block, seed, purpose, stripe, s)
    if rc != 0:
        raise RuntimeError("synth_fill failed (%d)" % rc)
