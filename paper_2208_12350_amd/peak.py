"""Measure the VALU issue rates the sweep roofline assumes (libswprobe.so).

    python -m paper_2208_12350_amd.peak

Prints one JSON line: lane-instructions per second for each probed
instruction, and the published-figure peak they are compared with
(256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane-instructions/s).
"""
import ctypes
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KINDS = {"v_pk_add_u16": 0, "v_pk_maximum3_f16": 1, "v_max3_u32": 2, "v_add_u32": 3}
PUBLISHED = 256 * 4 * 16 * 2.4e9


def measure(device=0, iters=4096, blocks=256 * 16):
    from paper_2208_12350_amd.binding import _init_torch_runtime
    _init_torch_runtime()   # PyTorch's HIP runtime first, as for libswalign
    lib = ctypes.CDLL(os.path.join(HERE, "libswprobe.so"))
    lib.sw_probe_valu.restype = ctypes.c_int
    lib.sw_probe_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_double)]
    out = {}
    for name, kind in KINDS.items():
        v = ctypes.c_double(0)
        rc = lib.sw_probe_valu(device, kind, iters, blocks, ctypes.byref(v))
        if rc != 0:
            raise RuntimeError("sw_probe_valu(%s) returned %d" % (name, rc))
        out[name] = v.value
    return out


def main():
    rates = measure()
    print(json.dumps({"published_lane_instr_per_s": PUBLISHED,
                      "measured": {k: round(v / 1e12, 3) for k, v in rates.items()},
                      "unit": "T lane-instructions/s",
                      "fraction_of_published": {k: round(v / PUBLISHED, 4) for k, v in rates.items()}}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
