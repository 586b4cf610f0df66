"""Sustained int16x2 VALU rate of the GPU (libswprobe.so): long streams of
independent packed saturating adds and subtracts on every lane, timed with
HIP events.  bench.py reports it beside the rate derived from unit counts and
clock, so that the kernel's roofline fraction can be read against both."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def measure(grid: int = 2048, trips: int = 20000) -> float:
    """Packed int16 operations per second (two per instruction per lane)."""
    lib = ctypes.CDLL(os.path.join(HERE, "libswprobe.so"))
    lib.swprobe_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    out = ctypes.c_double(0.0)
    rc = lib.swprobe_valu(grid, trips, ctypes.byref(out))
    if rc != 0:
        raise RuntimeError("VALU probe failed with HIP error %d" % rc)
    return out.value


def measure_i32(grid: int = 2048, trips: int = 20000) -> float:
    """32-bit integer operations per second (v_add_u32 and v_max_i32 streams,
    written as the instructions themselves so that their count is exact)."""
    lib = ctypes.CDLL(os.path.join(HERE, "libswprobe.so"))
    lib.swprobe_valu_i32.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    out = ctypes.c_double(0.0)
    rc = lib.swprobe_valu_i32(grid, trips, ctypes.byref(out))
    if rc != 0:
        raise RuntimeError("VALU probe failed with HIP error %d" % rc)
    return out.value


if __name__ == "__main__":
    print("int16x2: %.2f Tops/s" % (measure() / 1e12))
    print("int32:   %.2f Tops/s" % (measure_i32() / 1e12))
