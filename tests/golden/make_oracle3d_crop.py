"""Writes the 3D FP64 oracle's fields after the full run of the 3D ventilated workload (256 x 128 x 128,
inlet u = 0.01, seed R = 8, 2000 steps), on the box around the crystal (phi > -0.9, widened by 8 cells),
rounded to float32; the GPU test compares the same box of its own run:

    python tests/golden/make_oracle3d_crop.py [out.npz]   # default: tests/golden/f4_crop_2000.npz

It calls only the oracle (about 20 minutes on 8 cores).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2101_07163_amd import workloads as W  # noqa: E402  (the workload's parameters)

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "f4_crop_2000.npz")
PAD = 8


def main(out: str = OUT) -> None:
    cfg = W.F4_3D
    steps = cfg["steps"]
    o = oracle.Oracle3D(oracle.Params3D.from_dict(cfg)).init_seed(*cfg["seed"], cfg["w_init"], cfg["U0"])
    t0 = time.time()
    done = 0
    while done < steps:
        n = min(100, steps - done)
        o.step(n)
        done += n
        print("step %d  %.0f s" % (done, time.time() - t0), flush=True)
    F = o.fields()
    zs, ys, xs = np.nonzero(F["phi"] > -0.9)
    nz, ny, nx = F["phi"].shape
    box = [(max(0, int(a.min()) - PAD), min(n, int(a.max()) + 1 + PAD)) for a, n in ((zs, nz), (ys, ny), (xs, nx))]
    (z0, z1), (y0, y1), (x0, x1) = box
    arrays = {k: F[k][z0:z1, y0:y1, x0:x1].astype(np.float32) for k in ("phi", "U", "ux")}
    np.savez_compressed(out, steps=np.int64(steps), box=np.array(box, dtype=np.int64), **arrays)
    print("wrote", out, "box", box, flush=True)


if __name__ == "__main__":
    main(*sys.argv[1:2])
