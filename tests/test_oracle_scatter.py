"""Pins for the gather / scatter-accumulate / histogram oracle: the dense one-hot
product (the work-inefficient form the paper's Accum avoids, Sec. 5.3.3 and
Sec. 6.1.2), the adjoint identity, np.bincount, closed forms, and planted
mistakes."""
import numpy as np
import pytest

import workloads
from oracle import scatter


def one_hot(idx, rows):
    S = np.zeros((idx.shape[0], rows))
    S[np.arange(idx.shape[0]), idx] = 1.0
    return S


@pytest.mark.parametrize("rows,n,R,seed", [(50, 1000, 8, 0), (7, 300, 3, 1), (1000, 64, 5, 2)])
def test_scatter_equals_dense_transposed_product(rows, n, R, seed):
    si = workloads.scatter_inputs(rows, R, n, 1.1, seed)
    S = one_hot(si.idx, rows)
    dense = S.T @ (si.w.astype(np.float64)[:, None] * si.g.astype(np.float64))
    assert np.allclose(scatter.scatter(rows, si.idx, si.w, si.g), dense, rtol=1e-12, atol=1e-12)
    dense_fwd = np.diag(si.w.astype(np.float64)) @ S @ si.table.astype(np.float64)
    assert np.allclose(scatter.gather(si.table, si.idx, si.w), dense_fwd, rtol=1e-13, atol=1e-13)


def test_adjoint_identity():
    si = workloads.scatter_inputs(40, 6, 500, 1.1, 3)
    lhs = np.sum(scatter.gather(si.table, si.idx, si.w) * si.g)
    rhs = np.sum(si.table * scatter.scatter(40, si.idx, si.w, si.g))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_dw_by_central_differences():
    si = workloads.scatter_inputs(30, 4, 50, 1.1, 4)
    dw = scatter.scatter_dw(si.table, si.idx, si.g)
    w = si.w.astype(np.float64)
    for j in (0, 7, 49):
        e = np.zeros_like(w)
        e[j] = 1e-6
        up = np.sum(scatter.gather(si.table, si.idx, w + e) * si.g)
        dn = np.sum(scatter.gather(si.table, si.idx, w - e) * si.g)
        assert np.isclose((up - dn) / 2e-6, dw[j], rtol=1e-7, atol=1e-9)


def test_all_indices_equal():
    rng = np.random.default_rng(0)
    g = rng.standard_normal((200, 5))
    w = rng.uniform(-1, 1, 200)
    idx = np.full(200, 3)
    dT = scatter.scatter(10, idx, w, g)
    assert np.allclose(dT[3], (w[:, None] * g).sum(0), rtol=1e-12)
    assert np.count_nonzero(np.delete(dT, 3, axis=0)) == 0


def test_scatter_rows_matches_full():
    si = workloads.scatter_inputs(100, 4, 2000, 1.1, 5)
    full = scatter.scatter(100, si.idx, si.w, si.g)
    rows = [0, 1, 5, 99]
    assert np.allclose(scatter.scatter_rows(rows, si.idx, si.w, si.g), full[rows],
                       rtol=1e-13, atol=1e-13)


def test_out_of_range_indices_counted_and_skipped():
    idx = np.array([0, 5, -1, 9, 10, 3])
    g = np.ones((6, 2))
    dT, bad = scatter.scatter(10, idx, None, g, check_bounds=True)
    assert bad == 2 and dT.sum() == 8
    h, bad = scatter.histogram(np.array([1, 1, 70000, 2]), 4, check_bounds=True)
    assert bad == 1 and list(h) == [0, 2, 1, 0]


@pytest.mark.parametrize("n,bins,seed", [(100_000, 65536, 0), (5000, 17, 1)])
def test_histogram_equals_bincount(n, bins, seed):
    keys = workloads.histogram_keys(n, bins, 1.1, seed)
    h = scatter.histogram(keys, bins)
    assert np.array_equal(h, np.bincount(keys.astype(np.int64), minlength=bins))
    assert h.sum() == n


def test_planted_histogram_mistake_is_caught(monkeypatch):
    """Plant a classic mistake in the oracle: fancy-index `+=` instead of an
    unbuffered accumulation (repeated keys then count once). The bincount pin
    must catch it."""
    import types
    keys = workloads.histogram_keys(10_000, 64, 1.1, 0)

    def bad_add_at(a, i, v):
        a[i] += v

    fake = types.SimpleNamespace(**{n: getattr(np, n) for n in dir(np) if not n.startswith("__")})
    fake.add = types.SimpleNamespace(at=bad_add_at)
    monkeypatch.setattr(scatter, "np", fake)
    h = scatter.histogram(keys, 64)
    monkeypatch.undo()
    assert not np.array_equal(h, np.bincount(keys.astype(np.int64), minlength=64))


def test_zipf_statistics_of_the_table_indices():
    """The hottest row of the Zipf(1.1) table indices takes ~9.5% of all
    updates (1/zeta(1.1)); this is what makes the scatter contended."""
    idx = workloads.zipf_table_indices(1 << 20, 1_000_000, 1.1, 2)
    share = np.mean(idx == 0)
    assert 0.085 < share < 0.105


def test_gather_jvp_by_central_differences():
    """The gather is bilinear in (T, w), so the central difference of the
    primal along (tT, tw) equals the tangent up to rounding, for any step."""
    si = workloads.scatter_inputs(40, 6, 300, 1.1, 5)
    rng = np.random.default_rng(5)
    tT = rng.standard_normal(si.table.shape)
    tw = rng.standard_normal(si.w.shape)
    T, w = si.table.astype(np.float64), si.w.astype(np.float64)
    h = 0.5
    up = scatter.gather(T + h * tT, si.idx, w + h * tw)
    dn = scatter.gather(T - h * tT, si.idx, w - h * tw)
    got = scatter.gather_jvp(T, si.idx, w, tT, tw)
    assert np.allclose((up - dn) / (2 * h), got, rtol=1e-12, atol=1e-12)


def test_gather_jvp_vjp_dot_product_identity():
    """<J t, g> = <t, J^T g>: the forward mode against the transposed gather
    (scatter) and the weight cotangent (scatter_dw), both pinned above."""
    si = workloads.scatter_inputs(60, 5, 700, 1.1, 6)
    rng = np.random.default_rng(6)
    tT = rng.standard_normal(si.table.shape)
    tw = rng.standard_normal(si.w.shape)
    lhs = np.sum(scatter.gather_jvp(si.table, si.idx, si.w, tT, tw) * si.g)
    rhs = (np.sum(tT * scatter.scatter(60, si.idx, si.w, si.g))
           + np.dot(tw, scatter.scatter_dw(si.table, si.idx, si.g)))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_gather_jvp_special_cases():
    """Zero tangents give zero; a tangent along T alone is the gather of tT;
    along w alone it is tw times the gathered rows; out-of-range rows are zero."""
    si = workloads.scatter_inputs(20, 4, 100, 1.1, 7)
    T, w, idx = si.table.astype(np.float64), si.w.astype(np.float64), si.idx
    z = scatter.gather_jvp(T, idx, w, np.zeros_like(T), np.zeros_like(w))
    assert np.all(z == 0)
    tT = np.arange(T.size, dtype=np.float64).reshape(T.shape)
    assert np.array_equal(scatter.gather_jvp(T, idx, w, tT, np.zeros_like(w)),
                          scatter.gather(tT, idx, w))
    tw = np.linspace(-1, 1, w.size)
    assert np.array_equal(scatter.gather_jvp(T, idx, w, np.zeros_like(T), tw),
                          scatter.gather(T, idx, tw))
    bad = np.array([-1, 20, 3], dtype=np.int64)
    got = scatter.gather_jvp(T, bad, w[:3], tT, tw[:3])
    assert np.all(got[:2] == 0) and np.allclose(got[2], tw[2] * T[3] + w[2] * tT[3])
