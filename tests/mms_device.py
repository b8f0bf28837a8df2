"""ctypes access to the test-only input kernel (tests/mms_input_kernel.hip):
phi(t) and the scaled manufactured force of the travelling examples written
into caller-provided CUDA tensors, one launch per call."""
import ctypes
import os

import torch

import mms_inputs as MI

_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmmsinput.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise ImportError("libmmsinput.so not built: run tests/build_mms_input.py")
        _lib = ctypes.CDLL(_LIB)
        d, i, P = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        _lib.mms_travel_fields.restype = i
        _lib.mms_travel_fields.argtypes = [i, i, i, i, d, d, d, d, P, P, P]
    return _lib


def travel_fields(ex, N, t, fscale, phi, force):
    """phi(t) into `phi` [n] and fscale * F_MMS(t) into `force` [d, n]."""
    dims = MI.setup(ex, N, 0.6)[1]
    rc = _load().mms_travel_fields(ex, dims[0], dims[1], dims[2], MI.L / N, float(t), MI.NU,
                                   float(fscale), ctypes.c_void_p(phi.data_ptr()),
                                   ctypes.c_void_p(force.data_ptr()),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc:
        raise RuntimeError("mms_travel_fields failed (%d)" % rc)
