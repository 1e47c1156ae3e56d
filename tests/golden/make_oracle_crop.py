"""Writes the FP64 oracle's fields after a full-length run of a ventilated workload, on a 512 x 512 crop
around the crystal, rounded to float32 (the GPU tests compare the same crop of their own run):

    python tests/golden/make_oracle_crop.py c3   # 2048^2, inlet u = 0.01, 10^4 steps -> c3_crop_10000.npz
    python tests/golden/make_oracle_crop.py c2   # 1024^2, inlet u = 0.02, 2*10^4 steps -> c2_crop_20000.npz

It calls only the oracle (about 26 and 8 minutes on 8 cores).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2101_07163_amd import workloads as W  # noqa: E402  (the workloads' parameters)

HERE = os.path.dirname(os.path.abspath(__file__))
# workload, crop (rows, columns) around the seed, output file
CASES = {
    "c3": (W.C3, W.C3["crop"], "c3_crop_10000.npz"),
    "c2": (W.C2, ((256, 768), (44, 556)), "c2_crop_20000.npz"),
}


def main(name: str) -> None:
    cfg, ((r0, r1), (c0, c1)), fname = CASES[name]
    steps = cfg["steps"]
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
    out = os.path.join(HERE, fname)
    np.savez_compressed(out, steps=np.int64(steps), rows=np.array([r0, r1]), cols=np.array([c0, c1]), **crop)
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c3")
