"""Shared helpers for the GPU parity tests (HIP path through the C ABI vs the
CPU oracle on identical seeded inputs)."""
import sys

import numpy as np


def banner(msg):
    """Name the case before the GPU work starts, so a failing run says which."""
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


# Tolerances on fields (relative L2 against the FP64 oracle).
TOL = {"fp64": 1e-12, "fp32": 2e-5}
