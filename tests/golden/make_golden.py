"""Writes the stored expected values of the GPU parity tests.

Calls only the CPU oracle and the seeded input generator.  Run from the
repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2605_30128_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def tiny_rchfsi():
    """R-ChFSI on the tiny periodic cube (4^3 cells, p=4, 4 wells, 4 atoms x 4
    projectors): 32 wanted of a 40-column subspace, Chebyshev degree 20,
    run to a residual of 1e-10 from the seeded start block."""
    cfg = synth.CONFIGS["tiny"]
    p = synth.make_config("tiny")
    o = oracle.Oracle(p)
    lmax = o.lanczos(20, synth.random_block(p.ndof, 1, 2000)[:, 0])
    X0 = synth.random_block(p.ndof, cfg["nsub"], 2001)
    t = time.time()
    out = o.chfsi(X0, cfg["n_wanted"], cfg["cheb_degree"], lmax, tol=1e-10, max_iter=300)
    rec = dict(config="tiny", n_wanted=cfg["n_wanted"], nsub=cfg["nsub"], degree=cfg["cheb_degree"],
               lanczos_seed=2000, x0_seed=2001, lmax=lmax, tol=1e-10, iters=out["iters"],
               eigenvalues=out["ritz"].tolist(), hist_res=out["hist_res"].tolist(),
               seconds=time.time() - t)
    with open(os.path.join(HERE, "tiny_rchfsi.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print("tiny:", out["iters"], "iterations", out["hist_res"][-1], rec["seconds"], "s")


if __name__ == "__main__":
    oracle.build(force=False)
    tiny_rchfsi()
