"""Pins for the reduction oracle: closed forms on integer data, the relation of
the two patterns, and the one-hot form of a segmented reduction."""
import numpy as np

from oracle import reduce


def test_closed_forms_on_integers():
    n = 10_000
    v = np.arange(1, n + 1, dtype=np.float64)
    assert reduce.reduce_all(v) == n * (n + 1) // 2
    m = np.arange(12, dtype=np.float64).reshape(3, 4)        # rows 0..3, 4..7, 8..11
    assert np.array_equal(reduce.reduce_rows(m), [6.0, 22.0, 38.0])


def test_complete_is_the_sum_of_the_segments():
    rng = np.random.default_rng(1)
    v = rng.standard_normal((37, 53))
    assert np.isclose(reduce.reduce_all(v), reduce.reduce_all(reduce.reduce_rows(v)), rtol=1e-14)


def test_segmented_equals_a_one_hot_scatter():
    """acc!i += values.i.j is the scatter of every element to its row index."""
    from oracle import scatter
    rng = np.random.default_rng(2)
    v = rng.standard_normal((9, 7))
    idx = np.repeat(np.arange(9), 7)
    dense = scatter.scatter(9, idx, None, v.reshape(-1, 1))[:, 0]
    assert np.allclose(reduce.reduce_rows(v), dense, rtol=1e-13, atol=1e-13)


def test_exact_summation_beats_cancellation():
    v = np.array([1e16, 1.0, -1e16, 1.0])
    assert reduce.reduce_all(v) == 2.0
    assert np.array_equal(reduce.reduce_rows(np.zeros((4, 0))), np.zeros(4))
