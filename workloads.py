"""Seeded synthetic inputs for the five workloads of the scatter-accumulate AD path.

This module only draws random numbers and lays them out; it contains none of the
method's arithmetic. Both the HIP path (through its Python binding) and the FP64
oracle are fed from here, so that they see bit-identical inputs.

Conventions (the paper fixes none of these; they are this project's readings):
  * generator: numpy ``Generator(PCG64(seed))``;
  * "N(m, s)" means mean m and standard deviation s;
  * draw order for a GMM instance: x, alphas, means, qd, l;
  * the strictly-lower-triangular parameters ``l[k]`` of component k hold
    Q_k[a, b] (a > b) at position a*(a-1)/2 + b (row-major over the strict
    lower triangle);
  * Zipf(s) draws k >= 1 from numpy's unbounded Zipf sampler; a table index is
    (k - 1) mod rows, a histogram key is k mod bins.
"""
from __future__ import annotations

import dataclasses

import numpy as np

# Workload sizes (one place, so tests and the benchmark agree).
GMM_SMALL = dict(N=1000, D=2, K=5, seed=0)            # FP64 end to end
GMM_LARGE = dict(N=100_000, D=64, K=200, seed=1)      # BF16 MFMA products
SCATTER = dict(rows=1_000_000, row_len=128, n=4_194_304, s=1.1, seed=2)
HISTOGRAM = dict(bins=65_536, n=1 << 26, s=1.1, seed=2)
BATCHED = dict(B=512, N=(1000, 50_000), D=(8, 16, 32), K=(10, 100), seed=3)
STENCIL = dict(H=4096, W=4096, steps=1000, every=32, seed=4)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def n_lower(D: int) -> int:
    """Number of strictly-lower-triangular entries of a D x D matrix."""
    return D * (D - 1) // 2


@dataclasses.dataclass
class GMMInputs:
    alphas: np.ndarray  # [K]
    means: np.ndarray   # [K, D]
    qd: np.ndarray      # [K, D]   log of the diagonal of Q_k
    l: np.ndarray       # [K, D(D-1)/2]  strictly lower part of Q_k
    x: np.ndarray       # [N, D]

    @property
    def N(self) -> int:
        return self.x.shape[0]

    @property
    def D(self) -> int:
        return self.x.shape[1]

    @property
    def K(self) -> int:
        return self.alphas.shape[0]

    def astype(self, dtype) -> "GMMInputs":
        return GMMInputs(*(np.ascontiguousarray(a, dtype=dtype) for a in
                           (self.alphas, self.means, self.qd, self.l, self.x)))

    def params(self):
        return self.alphas, self.means, self.qd, self.l


def gmm_inputs(N: int, D: int, K: int, seed: int, dtype=np.float64) -> GMMInputs:
    """x ~ N(0,1), alphas ~ N(0,1), means ~ N(0,1), qd ~ N(0,0.1), l ~ N(0,0.1).

    Values are drawn in FP64 and cast once to ``dtype``; the oracle then runs in
    FP64 on exactly the cast values.
    """
    r = _rng(seed)
    x = r.normal(0.0, 1.0, (N, D))
    alphas = r.normal(0.0, 1.0, K)
    means = r.normal(0.0, 1.0, (K, D))
    qd = r.normal(0.0, 0.1, (K, D))
    l = r.normal(0.0, 0.1, (K, n_lower(D)))
    return GMMInputs(alphas, means, qd, l, x).astype(dtype)


def gmm_small(dtype=np.float64) -> GMMInputs:
    c = GMM_SMALL
    return gmm_inputs(c["N"], c["D"], c["K"], c["seed"], dtype)


def gmm_large(dtype=np.float32) -> GMMInputs:
    c = GMM_LARGE
    return gmm_inputs(c["N"], c["D"], c["K"], c["seed"], dtype)


def batched_shapes(B: int | None = None, seed: int | None = None):
    """Per-instance (N, D, K): N ~ U[1000, 50000], D uniform over {8,16,32},
    K ~ U[10, 100] (integer bounds inclusive). Returns an int64 array [B, 3]."""
    c = BATCHED
    B = c["B"] if B is None else B
    seed = c["seed"] if seed is None else seed
    r = _rng(seed)
    N = r.integers(c["N"][0], c["N"][1], size=B, endpoint=True)
    D = r.choice(np.array(c["D"]), size=B)
    K = r.integers(c["K"][0], c["K"][1], size=B, endpoint=True)
    return np.stack([N, D, K], axis=1).astype(np.int64)


def batched_inputs(shapes: np.ndarray, seed: int | None = None, dtype=np.float32):
    """One GMMInputs per instance; instance b uses seed (base + 1 + b)."""
    base = BATCHED["seed"] if seed is None else seed
    return [gmm_inputs(int(N), int(D), int(K), base + 1 + b, dtype)
            for b, (N, D, K) in enumerate(shapes)]


def pack_batched(insts):
    """Concatenate per-instance arrays in instance order (the packed layout the
    batched entry points take): alphas, means, qd, l, x as flat FP arrays."""
    cat = lambda name: np.ascontiguousarray(
        np.concatenate([getattr(g, name).reshape(-1) for g in insts]))
    return tuple(cat(n) for n in ("alphas", "means", "qd", "l", "x"))


def zipf_table_indices(n: int, rows: int, s: float, seed: int) -> np.ndarray:
    """int32 indices (k - 1) mod rows, k ~ Zipf(s)."""
    k = _rng(seed).zipf(s, n)
    return ((k - 1) % rows).astype(np.int32)


@dataclasses.dataclass
class ScatterInputs:
    table: np.ndarray  # [rows, row_len] f32
    idx: np.ndarray    # [n] int32
    w: np.ndarray      # [n] f32
    g: np.ndarray      # [n, row_len] f32 (upstream cotangent of the gather)


def scatter_inputs(rows: int, row_len: int, n: int, s: float = 1.1, seed: int = 2,
                   with_table: bool = True) -> ScatterInputs:
    """Draw order: idx, w, g, then the table. FP32 drawn directly (no FP64 copy
    of the 2 GiB arrays)."""
    r = _rng(seed)
    idx = ((r.zipf(s, n) - 1) % rows).astype(np.int32)
    w = r.uniform(-1.0, 1.0, n).astype(np.float32)
    g = r.standard_normal((n, row_len), dtype=np.float32)
    table = (r.standard_normal((rows, row_len), dtype=np.float32)
             if with_table else None)
    return ScatterInputs(table, idx, w, g)


def histogram_keys(n: int, bins: int, s: float = 1.1, seed: int = 2) -> np.ndarray:
    """uint32 keys k mod bins, k ~ Zipf(s), drawn in blocks to bound memory."""
    r = _rng(seed)
    out = np.empty(n, dtype=np.uint32)
    step = 1 << 22
    for i in range(0, n, step):
        m = min(step, n - i)
        out[i:i + m] = (r.zipf(s, m) % bins).astype(np.uint32)
    return out


def stencil_inputs(H: int, W: int, seed: int = 4):
    """u0 ~ N(0,1), target ~ N(0,1), both [H, W] f32, drawn in that order."""
    r = _rng(seed)
    u0 = r.standard_normal((H, W), dtype=np.float32)
    target = r.standard_normal((H, W), dtype=np.float32)
    return u0, target
