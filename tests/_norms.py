"""Error norms of the GPU tests.

Parity with the oracle (same tree, lists and order, so the same linear map up
to rounding) is asserted element-wise: both the relative L2 norm and the
relative max norm max|a - b| / max|b| (over every element of an output,
all field components included) must meet the bound.  Accuracy against the
direct sum is the method's truncation error, stated by the workloads as a
relative L2 bound over the targets; the relative max norm (the paper's
relative L-infinity error of Sec. III.A) is reported beside it.
"""
import numpy as np


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_max(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


def parity(a, b) -> float:
    """The larger of the relative L2 and relative max errors."""
    return max(rel_l2(a, b), rel_max(a, b))
