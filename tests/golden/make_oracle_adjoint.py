"""Writes the FP64 oracle's discrete adjoint of the 512^2 adjoint workload (no flow, periodic, seed
R = 6 at the centre, 5000 steps, checkpoints every ceil(sqrt(5000)) steps): the loss
L = sum (phi_T - phi*)^2 against the shape phi* grown with eps = 0.06, U0 = 0.55, and its gradients at
eps = 0.04, U_init = 0.5 + 0.02 xi (xi ~ N(0, 1), default_rng(2101)), with U_init rounded to float32
(the GPU reads it in FP32):

    python tests/golden/make_oracle_adjoint.py   # -> c5_adjoint_5000.npz (about 3 minutes on 8 cores)

Stored: phi* (float64), dL/dU_init (float32: the GPU test compares cell by cell at 1e-3 of its largest
magnitude), dL/deps and L (float64).  It calls only the oracle.
"""
import dataclasses
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2101_07163_amd import workloads as W  # noqa: E402  (the workload's parameters and draw)

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "c5_adjoint_5000.npz")


def main() -> None:
    cfg = dict(W.C5)
    steps = cfg["steps"]
    p = oracle.Params.from_dict(cfg)
    U = W.c5_U_init(cfg).astype(np.float32).astype(np.float64)
    t0 = time.time()
    target = oracle.final_phi(dataclasses.replace(p, eps=cfg["eps_target"]), cfg["seed"], cfg["w_init"],
                              np.full_like(U, cfg["U0_target"]), steps)
    print("target  %.0f s" % (time.time() - t0), flush=True)
    L, dU, de, phiT = oracle.adjoint(p, cfg["seed"], cfg["w_init"], U, target, steps)
    print("adjoint %.0f s: L %.9e  dL/deps %.9e  sum dL/dU %.9e" % (time.time() - t0, L, de, dU.sum()), flush=True)
    np.savez_compressed(OUT, steps=np.int64(steps), target=target, dU=dU.astype(np.float32),
                        deps=np.float64(de), L=np.float64(L), dU0=np.float64(dU.sum()))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
