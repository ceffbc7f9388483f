"""Writes the stored expected values under tests/golden/ by calling only the
oracle package (and the seeded input generators). Re-run after an intentional
change to the oracle's arithmetic:  python tests/golden/make_golden.py"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import gmm, scatter, stencil  # noqa: E402


def dump(name, obj):
    with open(os.path.join(HERE, name), "w") as fh:
        json.dump(obj, fh, indent=1)
        fh.write("\n")


def main():
    g = workloads.gmm_small()
    F, f = gmm.objective(*g.params(), g.x)
    da, dm, dq, dl = gmm.vjp(*g.params(), g.x, f)
    dump("gmm_small_f64.json", {
        "source": "oracle.gmm on workloads.gmm_small() (N=1000, D=2, K=5, seed 0)",
        "F": F, "f_first8": f[:8].tolist(),
        "d_alphas": da.tolist(), "d_means": dm.tolist(), "d_qd": dq.tolist(), "d_l": dl.tolist()})

    u0, target = workloads.stencil_inputs(8, 8, 4)
    L, uT, grad = stencil.loss_and_grad(u0, target, 5)
    dump("stencil_8x8_5steps.json", {
        "source": "oracle.stencil on workloads.stencil_inputs(8, 8, seed 4), 5 steps",
        "L": L, "uT_row0": uT[0].tolist(), "grad_row0": grad[0].tolist()})

    keys = workloads.histogram_keys(4096, 37, 1.1, 7)
    dump("histogram_4096_37.json", {
        "source": "oracle.scatter.histogram on workloads.histogram_keys(4096, 37, 1.1, seed 7)",
        "hist": scatter.histogram(keys, 37).tolist()})


if __name__ == "__main__":
    main()
