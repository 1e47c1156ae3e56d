"""Writes c3_crop_10000.npz: the FP64 oracle's fields after 10^4 steps of the 2048 x 2048 ventilated
workload (inlet u = 0.01, seed R = 8 at (300, 1024)), on the crop rows [768, 1280) x columns [44, 556)
around the crystal, rounded to float32.  It calls only the oracle (about 12 minutes on 8 cores).

    python tests/golden/make_c3_crop.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2101_07163_amd import workloads as W  # noqa: E402  (the workload's parameters)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_crop_10000.npz")


def main(steps: int = 10000) -> None:
    cfg = W.C3
    (r0, r1), (c0, c1) = cfg["crop"]
    o = oracle.Oracle(oracle.Params.from_dict(cfg)).init_seed(*cfg["seed"], cfg["w_init"], cfg["U0"])
    t0 = time.time()
    done = 0
    while done < steps:
        n = min(500, steps - done)
        o.step(n)
        done += n
        print("step %d  %.0f s" % (done, time.time() - t0), flush=True)
    F = o.fields()
    crop = {k: F[k][r0:r1, c0:c1].astype(np.float32) for k in ("phi", "U", "rho", "ux", "uy")}
    np.savez_compressed(OUT, steps=np.int64(steps), rows=np.array([r0, r1]), cols=np.array([c0, c1]), **crop)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
