"""Measured MI355X ceilings used as roofline references (binding of libdrceil.so)."""

from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdrceil.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the package first")
        _lib = C.CDLL(LIB_PATH)
        _lib.drceil_run.argtypes = [C.c_int, C.c_size_t, C.c_int, C.POINTER(C.c_double)]
        _lib.drceil_run.restype = C.c_int
        _lib.drceil_xcc_hist.argtypes = [C.c_int, C.POINTER(C.c_int)]
        _lib.drceil_xcc_hist.restype = C.c_int
    return _lib


def run(which: int, footprint: int = 0, iters: int = 64) -> float:
    v = C.c_double()
    rc = _load().drceil_run(which, footprint, iters, C.byref(v))
    if rc != 0:
        raise RuntimeError(f"ceiling benchmark {which} failed ({rc})")
    return v.value


def copy_bandwidth(nbytes=2 << 30):
    return run(0, nbytes)


def atomics_device(footprint):
    return run(1, footprint)


def atomics_per_xcd(footprint):
    return run(2, footprint)


def atomics_grouped(footprint, group):
    return run(5 if group == 64 else 6, footprint)


def atomic_rows_f64(footprint):
    """FP64 atomic adds on random 64-byte rows of 8 doubles: rows per second."""
    return run(7, footprint)


def atomic_rows_f32(footprint):
    """FP32 atomic adds on random 64-byte rows of 16 floats: rows per second."""
    return run(8, footprint)


def lds_atomics():
    return run(3, 0, 256)


def exp_rate():
    return run(4, 0, 1024)


def xcc_hist(blocks=4096):
    h = (C.c_int * 8)()
    rc = _load().drceil_xcc_hist(blocks, h)
    if rc != 0:
        raise RuntimeError("xcc histogram failed")
    return list(h)


if __name__ == "__main__":
    import sys
    if len(sys.argv) > 2 and sys.argv[1] == "copy":
        # one copy of the given number of bytes (read + write), warm-up plus timed launch
        print(f"copy {copy_bandwidth(int(sys.argv[2])) / 1e9:.0f} GB/s", flush=True)
        sys.exit(0)
    print("xcc histogram", xcc_hist(), flush=True)
    print(f"copy {copy_bandwidth() / 1e9:.0f} GB/s (read + write)", flush=True)
    for fp in (1 << 20, 8 << 20, 128 << 20, 1 << 30, 8 << 30):
        print(f"atomics {fp >> 20} MiB: device scope {atomics_device(fp) / 1e9:.2f} G/s, "
              f"per-XCD workgroup scope {atomics_per_xcd(fp) / 1e9:.2f} G/s", flush=True)
    for fp in (8 << 20, 1 << 30):
        print(f"atomics {fp >> 20} MiB in 64-float groups {atomics_grouped(fp, 64) / 1e9:.1f} G lane-ops/s, "
              f"8-float groups {atomics_grouped(fp, 8) / 1e9:.1f} G lane-ops/s", flush=True)
    for fp in (8 << 20, 16 << 20, 128 << 20, 1 << 30):
        print(f"FP64 atomic rows (8 doubles), {fp >> 20} MiB: {atomic_rows_f64(fp) / 1e9:.2f} G rows/s; "
              f"FP32 atomic rows (16 floats): {atomic_rows_f32(fp) / 1e9:.2f} G rows/s", flush=True)
    print(f"FP32 atomic rows (16 floats), 8192 MiB: {atomic_rows_f32(8 << 30) / 1e9:.2f} G rows/s", flush=True)
    print(f"LDS atomics {lds_atomics() / 1e12:.2f} T/s", flush=True)
    print(f"exp {exp_rate() / 1e12:.2f} T/s", flush=True)
