"""Regular segmented reduction and complete reduction, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 6.1.3 names three reduction patterns by how the accumulator is indexed:
never (a complete reduction, `for i. acc += values.i`), by a subset of the loop
indices (a regular segmented reduction, `for i j. acc!i += values.i.j`), or by
an arbitrary expression (the irregular scatter and the histogram, in
`oracle.scatter`). Each value is added one at a time, in index order, with
math.fsum's exact summation (correctly rounded to FP64).
"""
from __future__ import annotations

import math

import numpy as np


def reduce_rows(values) -> np.ndarray:
    """out[i] = sum_j values[i, j] (the accumulator indexed by the outer index)."""
    v = np.asarray(values, dtype=np.float64)
    return np.array([math.fsum(v[i]) for i in range(v.shape[0])], dtype=np.float64)


def reduce_all(values) -> float:
    """sum_i values[i] over every element (the accumulator never indexed)."""
    return math.fsum(np.asarray(values, dtype=np.float64).ravel())
