"""Thin ctypes binding of libswstencil.so (include/swstencil.h): one
diffusion step of a float32 grid, on a zero-padded grid or with bounds
checks.  Argument marshalling only; there is no CPU fallback."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswstencil.so")
EXPORTED = ("sw_diffuse_padded", "sw_diffuse_checked", "sw_pad_grid")

_lib = None


def load_library(path: str = LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libswstencil.so is not built (run __graft_entry__.build())")
    from paper_2208_12350_amd.binding import _init_torch_runtime
    _init_torch_runtime()   # PyTorch's HIP runtime first, as for libswalign
    lib = ctypes.CDLL(path)
    lib.sw_diffuse_padded.restype = ctypes.c_int
    lib.sw_diffuse_padded.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_float, ctypes.c_void_p]
    lib.sw_diffuse_checked.restype = ctypes.c_int
    lib.sw_diffuse_checked.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_float, ctypes.c_void_p]
    lib.sw_pad_grid.restype = ctypes.c_int
    lib.sw_pad_grid.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_void_p]
    _lib = lib
    return lib


def _stream(t, stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream(t.device)
    return ctypes.c_void_p(s.cuda_stream)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("%s failed with status %d" % (what, rc))


def padded_pitch(nx: int) -> int:
    """Row pitch of the padded layout: nx + 2 rounded up to 64 floats."""
    return (nx + 2 + 63) // 64 * 64


def pad(grid, pitch=None, stream=None):
    """Padded copy (torch float32 [ny+2, pitch]) of a torch float32 [ny, nx] grid."""
    import torch
    ny, nx = grid.shape
    pitch = padded_pitch(nx) if pitch is None else pitch
    out = torch.empty((ny + 2, pitch), dtype=torch.float32, device=grid.device)
    _check(load_library().sw_pad_grid(grid.data_ptr(), out.data_ptr(), nx, ny, pitch, _stream(grid, stream)),
           "sw_pad_grid")
    return out


def diffuse_padded(src, dst, nx: int, ny: int, D: float, stream=None):
    """One step from padded `src` into padded `dst` (same shape)."""
    assert src.shape == dst.shape and src.shape[0] == ny + 2 and src.is_contiguous() and dst.is_contiguous()
    _check(load_library().sw_diffuse_padded(src.data_ptr(), dst.data_ptr(), nx, ny, src.shape[1], D,
                                            _stream(src, stream)), "sw_diffuse_padded")


def diffuse_checked(src, dst, D: float, stream=None):
    """One step from unpadded `src` [ny, nx] into `dst`."""
    assert src.shape == dst.shape and src.is_contiguous() and dst.is_contiguous()
    ny, nx = src.shape
    _check(load_library().sw_diffuse_checked(src.data_ptr(), dst.data_ptr(), nx, ny, D, _stream(src, stream)),
           "sw_diffuse_checked")
