"""Indexed read (gather), its transpose (scatter-accumulate) and the histogram, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

  gather     out[j, :] = w[j] * T[idx[j], :]          -- `for j. w.j * T.(idx.j)`,
             array indexing (Sec. 2.1) inside a `for`.
  scatter    the transpose of `gather` with respect to T: rule
             LetIndexingTranspose (Fig. "transposition rules") turns the read
             `T.(idx.j)` into the accumulation `dT!(idx.j) += w.j * g.j` into a
             sliced cotangent reference (Sec. 2.3.3, Sec. 5.3.3), run under
             `runAccum` starting from zero (Sec. 2.3.2). Its transpose with
             respect to w is dw[j] = <T[idx[j]], g[j]> (MulLeftTranspose).
  histogram  `for i. hist!(keys.i) += 1` (Sec. 2.3.3, Sec. 6.1.2): an integer
             accumulation, exact under any order.
  gather_jvp the forward mode of `gather` (the linear map that `linearize`
             returns, Sec. 5.1): the tangent of a product is the product rule,
             the tangent of an indexed read reads the tangent array at the same
             index, and the integer idx carries no tangent.
"""
from __future__ import annotations

import numpy as np


def gather(T, idx, w, rows_out=None):
    """out[j] = w[j] * T[idx[j]] for every j, or only for j in rows_out."""
    T = np.asarray(T, dtype=np.float64)
    idx = np.asarray(idx, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    js = np.arange(idx.shape[0]) if rows_out is None else np.asarray(rows_out)
    out = np.empty((js.shape[0], T.shape[1]))
    for n, j in enumerate(js):
        out[n] = w[j] * T[idx[j]]
    return out


def scatter(n_rows, idx, w, g, check_bounds=False):
    """dT = runAccum (for j. dT!(idx.j) += w.j * g.j), starting from zero.

    Indices outside [0, n_rows) are skipped and counted when check_bounds is set
    (an index built from an ordinal needs a run-time check, Sec. 6.3).
    Returns dT, or (dT, n_out_of_range) when check_bounds is set.
    Each update is accumulated one at a time, in index order j = 0, 1, ...
    """
    idx = np.asarray(idx, dtype=np.int64)
    g = np.asarray(g, dtype=np.float64)
    w = np.ones(idx.shape[0]) if w is None else np.asarray(w, dtype=np.float64)
    dT = np.zeros((n_rows, g.shape[1]))
    bad = 0
    for j in range(idx.shape[0]):
        v = idx[j]
        if v < 0 or v >= n_rows:
            bad += 1
            continue
        dT[v] += w[j] * g[j]
    return (dT, bad) if check_bounds else dT


def scatter_rows(rows, idx, w, g):
    """Selected rows of `scatter`: dT[v] = sum over {j : idx[j] = v} of w[j] g[j],
    accumulated in index order. For sampled checks at sizes where the full
    table is too large to build on the host."""
    idx = np.asarray(idx)
    out = np.zeros((len(rows), g.shape[1]))
    for n, v in enumerate(rows):
        js = np.nonzero(idx == v)[0]
        acc = np.zeros(g.shape[1])
        for j in js:
            acc += float(w[j]) * np.asarray(g[j], dtype=np.float64)
        out[n] = acc
    return out


def scatter_dw(T, idx, g, rows_out=None):
    """dw[j] = sum_c T[idx[j], c] * g[j, c]: transpose of the gather w.r.t. w."""
    idx = np.asarray(idx, dtype=np.int64)
    js = np.arange(idx.shape[0]) if rows_out is None else np.asarray(rows_out)
    out = np.empty(js.shape[0])
    for n, j in enumerate(js):
        out[n] = float(np.dot(np.asarray(T[idx[j]], np.float64),
                              np.asarray(g[j], np.float64)))
    return out


def histogram(keys, n_bins, check_bounds=False):
    """hist = runAccum (for i. hist!(keys.i) += 1), in int64, one key at a time.

    Returns hist, or (hist, n_out_of_range) when check_bounds is set.
    """
    keys = np.asarray(keys).astype(np.int64)
    h = np.zeros(n_bins, dtype=np.int64)
    inside = (keys >= 0) & (keys < n_bins)
    # one increment per key; np.add.at applies repeated indices one at a time
    np.add.at(h, keys[inside], 1)
    bad = int(keys.shape[0] - np.count_nonzero(inside))
    return (h, bad) if check_bounds else h


def gather_jvp(T, idx, w, tT, tw, rows_out=None):
    """Tangent of out[j] = w[j] * T[idx[j]] along (tT, tw):
    tout[j] = tw[j] * T[idx[j]] + w[j] * tT[idx[j]], for every j or only for j in
    rows_out. Rows whose index lies outside [0, len(T)) are zero (the library's
    out-of-range convention)."""
    T = np.asarray(T, dtype=np.float64)
    tT = np.asarray(tT, dtype=np.float64)
    idx = np.asarray(idx, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    tw = np.asarray(tw, dtype=np.float64)
    js = np.arange(idx.shape[0]) if rows_out is None else np.asarray(rows_out)
    out = np.zeros((js.shape[0], T.shape[1]))
    for n, j in enumerate(js):
        v = idx[j]
        if 0 <= v < T.shape[0]:
            out[n] = tw[j] * T[v] + w[j] * tT[v]
    return out
