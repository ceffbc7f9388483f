"""The oracle against the stored fixtures under tests/golden/ (a hand-worked
example of the paper's histogram, and regression values written by
tests/golden/make_golden.py from the oracle)."""
import json
import os

import numpy as np

import workloads
from oracle import gmm, scatter, stencil

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def test_paper_histogram_example():
    ex = load("histogram_paper_example.json")
    assert scatter.histogram(np.array(ex["keys"]), ex["bins"]).tolist() == ex["hist"]


def test_gmm_small_regression():
    ex = load("gmm_small_f64.json")
    g = workloads.gmm_small()
    F, f = gmm.objective(*g.params(), g.x)
    assert np.isclose(F, ex["F"], rtol=1e-13)
    for got, key in zip(gmm.vjp(*g.params(), g.x, f), ("d_alphas", "d_means", "d_qd", "d_l")):
        assert np.allclose(got, np.array(ex[key]), rtol=1e-12, atol=1e-12)


def test_stencil_regression():
    ex = load("stencil_8x8_5steps.json")
    u0, target = workloads.stencil_inputs(8, 8, 4)
    L, uT, grad = stencil.loss_and_grad(u0, target, 5)
    assert np.isclose(L, ex["L"], rtol=1e-13)
    assert np.allclose(grad[0], ex["grad_row0"], rtol=1e-12, atol=1e-13)


def test_histogram_regression():
    ex = load("histogram_4096_37.json")
    keys = workloads.histogram_keys(4096, 37, 1.1, 7)
    assert scatter.histogram(keys, 37).tolist() == ex["hist"]
