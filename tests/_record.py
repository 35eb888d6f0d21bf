"""Stated errors of the GPU tests: each test prints its measured errors and,
when SKELFMM_RECORD names a file, appends them there as one JSON line, so a
run's figures can be collected without parsing captured output."""
import json
import os


def record(case: str, **values):
    line = {"case": case, **{k: (float(v) if isinstance(v, (int, float)) or hasattr(v, "__float__") else v)
                             for k, v in values.items()}}
    print("[record]", json.dumps(line), flush=True)
    path = os.environ.get("SKELFMM_RECORD")
    if path:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "a") as f:
            f.write(json.dumps(line) + "\n")


# Float32 / complex64 applies against O2 on the same (float32-rounded) charges:
# what is left is the float32 arithmetic of the path -- T and every stored
# vector rounded to float32 once per level, the kernel value from a rounded
# |d|^2 and the hardware reciprocal square root (about one unit in the last
# place), float32 partial sums of at most a few terms before float64
# accumulation.  Each output is a sum whose terms carry independent roundings
# of a few units u = 2^-24, so its relative error is a small multiple of u;
# the bar allows 16 u.
F32_VS_O2 = 16 * 2.0 ** -24


def maxrel(a, b):
    """max |a - b| / max |b| (the paper's error measure, beside the relative l2)."""
    import numpy as np
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
