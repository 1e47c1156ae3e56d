"""Writes how far the FP64 oracle's own phase field moves under noise of FP32 size, for the long
ventilated runs, and the oracle's fields of every member of the 64-crystal sweep:

    python tests/golden/make_oracle_spread.py v512 c2 c4 c3

For each case the oracle runs twice from the same initial state: as is, and with every population and
phi_prev multiplied by (1 + sigma sqrt(k) xi) every k = 10 steps, xi ~ N(0, 1) (a seeded draw), sigma =
2^-23 per step: one FP32 unit in the last place per value and step, about what the few roundings a
step applies to each stored value add up to.  The spread is the largest |phi_noisy - phi| over the
compared region at each checkpoint.  A FP32 run of the same case cannot be expected closer to the
oracle than this spread where it exceeds the 1e-4 target; the GPU tests bound their error by
max(1e-4, 2 x spread).

Cases (regions are the cells the GPU tests compare):
  v512  the 2048^2 workload's physics on 512^2 (seed (150, 256)), 10^4 steps, whole lattice
  c2    the 1024^2 workload over 2*10^4 steps, the stored crop rows [256, 768) x columns [44, 556)
  c3    the 2048^2 workload over 10^4 steps, the stored crop (reference: c3_crop_10000.npz)
  c4    each of the 64 crystals over 5000 steps, the box around its crystal (phi > -0.9, widened by
        16 cells); also stores each crystal's phi and U on that box (float32) in c4_members_5000.npz

Results go to oracle_spread.json (merged with what is there).  The sweep's members can also be split
between machines: "c4part FIRST LAST DIR" computes members FIRST..LAST-1 into DIR, and "c4merge DIR" adds
them to the stored files (each member depends only on its own parameters and seed); "c4areas DIR"
records, for the members whose spread exceeds 1e-2, the crystal areas of the reference and perturbed
runs, which c4merge adds as well.  It calls only the oracle; c3 takes
about an hour and c4 about four on 8 cores (c4 resumes after the last member stored).
"""
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2101_07163_amd import workloads as W  # noqa: E402  (the workloads' parameters)

HERE = os.path.dirname(os.path.abspath(__file__))
JSON = os.path.join(HERE, "oracle_spread.json")
C4_NPZ = os.path.join(HERE, "c4_members_5000.npz")
SIGMA = 2.0 ** -23  # relative noise per value and step
EVERY = 10


def v512_cfg():
    cfg = dict(W.C3)
    cfg.update(nx=512, ny=512, seed=(150.0, 256.0, 8.0))
    return cfg


def new(cfg):
    return oracle.Oracle(oracle.Params.from_dict(cfg)).init_seed(*cfg["seed"], cfg["w_init"], cfg["U0"])


class Draws:
    """The standard normal arrays of successive perturbations (f, g, h, phi_prev in that order, f only
    with flow), drawn from one seeded generator in a worker thread while the oracle steps; the sequence
    is the one a plain loop over the same generator gives."""

    def __init__(self, o, rng):
        names = ("f", "g", "h", "phip") if o.p.flow else ("g", "h", "phip")
        ny, nx = o.shape
        q = {"f": 9, "g": 5, "h": 9, "phip": 0}
        self.shapes = [(n, (q[n], ny, nx) if q[n] else (ny, nx)) for n in names]
        self.rng = rng
        self.pool = ThreadPoolExecutor(max_workers=1)
        self.next = self.pool.submit(self._draw)

    def _draw(self):
        return {n: self.rng.standard_normal(shape) for n, shape in self.shapes}

    def take(self):
        z = self.next.result()
        self.next = self.pool.submit(self._draw)
        return z

    def close(self):
        self.next.result()
        self.pool.shutdown()


def perturb(o, draws, k):
    s = o.get_state()
    a = SIGMA * np.sqrt(k)
    z = draws.take()
    if not o.p.flow:
        s["f"] = None
    for name, zn in z.items():
        zn *= a
        zn += 1.0
        s[name] *= zn
    o.set_state(**s)


def spread_run(cfg, steps, checkpoints, region, seed, ref_at_end=None, log="", keep=None):
    """phi spread at each checkpoint over region ((r0, r1), (c0, c1)); the reference runs alongside
    unless its phi on the region at the last checkpoint is given (ref_at_end).  keep (a dict), if
    given, receives the perturbed run's phi on the region at the last checkpoint."""
    (r0, r1), (c0, c1) = region
    noisy = new(cfg)
    draws = Draws(noisy, np.random.default_rng(seed))
    ref = None if ref_at_end is not None else new(cfg)
    out = {}
    done, t0 = 0, time.time()
    while done < steps:
        k = min(EVERY, steps - done)
        noisy.step(k)
        if ref is not None:
            ref.step(k)
        done += k
        perturb(noisy, draws, k)
        if done % 1000 == 0:
            print("%s perturbed run step %d" % (log, done), flush=True)
        if done in checkpoints:
            a = noisy.fields()["phi"][r0:r1, c0:c1]
            b = ref.fields()["phi"][r0:r1, c0:c1] if ref is not None else ref_at_end
            out[str(done)] = float(np.abs(a - b).max())
            if keep is not None:
                keep["phi"] = a.copy()
            print("%s step %d spread %.3e (%.0f s)" % (log, done, out[str(done)], time.time() - t0), flush=True)
    draws.close()
    return out


def load():
    return json.load(open(JSON)) if os.path.exists(JSON) else {}


def save(d):
    with open(JSON + ".tmp", "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(JSON + ".tmp", JSON)


def header():
    return {"sigma_per_step": SIGMA, "every": EVERY, "noise": "relative, N(0, 1), seeded"}


def case_v512():
    cfg = v512_cfg()
    d = dict(header(), region=[[0, 512], [0, 512]],
             spread_phi=spread_run(cfg, 10000, {2500, 5000, 10000}, ((0, 512), (0, 512)), 512, log="v512"))
    return d


def case_c2():
    region = ((256, 768), (44, 556))
    return dict(header(), region=[list(region[0]), list(region[1])],
                spread_phi=spread_run(W.C2, 20000, {5000, 10000, 15000, 20000}, region, 1024, log="c2"))


def case_c3():
    data = np.load(os.path.join(HERE, "c3_crop_10000.npz"))
    (r0, r1), (c0, c1) = W.C3["crop"]
    ref = data["phi"].astype(np.float64)
    return dict(header(), region=[[r0, r1], [c0, c1]], reference="c3_crop_10000.npz (float32)",
                spread_phi=spread_run(W.C3, 10000, {10000}, ((r0, r1), (c0, c1)), 2048, ref_at_end=ref, log="c3"))


def crystal_box(phi, pad=16):
    ys, xs = np.nonzero(phi > -0.9)
    ny, nx = phi.shape
    return ((max(0, int(ys.min()) - pad), min(ny, int(ys.max()) + 1 + pad)),
            (max(0, int(xs.min()) - pad), min(nx, int(xs.max()) + 1 + pad)))


def c4_member(i, cfg, steps):
    """Arrays and record of sweep member i: its phi and U on the box around its crystal after the full
    run, and the oracle's spread there."""
    ref = new(cfg)
    for done in range(0, steps, 1000):
        ref.step(min(1000, steps - done))
        print("c4[%d] reference run step %d" % (i, min(done + 1000, steps)), flush=True)
    F = ref.fields()
    (r0, r1), (c0, c1) = crystal_box(F["phi"])
    arrays = {"phi_%d" % i: F["phi"][r0:r1, c0:c1].astype(np.float32),
              "U_%d" % i: F["U"][r0:r1, c0:c1].astype(np.float32),
              "box_%d" % i: np.array([r0, r1, c0, c1], dtype=np.int64)}
    sp = spread_run(cfg, steps, {steps}, ((r0, r1), (c0, c1)), 7163 + i,
                    ref_at_end=F["phi"][r0:r1, c0:c1], log="c4[%d] %dx%d" % (i, cfg["nx"], cfg["ny"]))
    member = {"i": i, "nx": cfg["nx"], "eps": cfg["eps"], "U0": cfg["U0"], "u_in": cfg["u_in"],
              "box": [[r0, r1], [c0, c1]], "spread_phi": sp[str(steps)]}
    return arrays, member


def store_c4(arrays, members, steps):
    np.savez_compressed(C4_NPZ + ".tmp.npz", steps=np.int64(steps), **{k: v for k, v in arrays.items() if k != "steps"})
    os.replace(C4_NPZ + ".tmp.npz", C4_NPZ)
    d = load()
    d["c4"] = dict(header(), steps=steps, members=sorted(members, key=lambda m: m["i"]))
    save(d)


def case_c4():
    cfgs = W.c4_domains()
    steps = cfgs[0]["steps"]
    arrays, members = {}, []
    if os.path.exists(C4_NPZ):  # resume
        old = np.load(C4_NPZ)
        arrays = {k: old[k] for k in old.files}
        members = load().get("c4", {}).get("members", [])
    t0 = time.time()
    have = {m["i"] for m in members}
    for i in range(len(cfgs)):
        if i in have:
            continue
        a, m = c4_member(i, cfgs[i], steps)
        arrays.update(a)
        members.append(m)
        store_c4(arrays, members, steps)
        print("c4 member %d done (%.0f s)" % (i, time.time() - t0), flush=True)
    return load()["c4"]


def c4_areas(outdir, *only, threshold=1e-2):
    """For the sweep members whose stored spread exceeds threshold (their phase field after 5000 steps
    is not reproducible pointwise under one-ulp noise): the crystal area (cells with phi > 0 on the
    stored box) of the reference run and of the same perturbed run as the spread's, into
    outdir/c4_areas.json; c4_merge adds them to the stored records."""
    cfgs = W.c4_domains()
    steps = cfgs[0]["steps"]
    os.makedirs(outdir, exist_ok=True)
    out = {}
    for m in load()["c4"]["members"]:
        if m["spread_phi"] <= threshold or (only and str(m["i"]) not in only):
            continue
        i = m["i"]
        (r0, r1), (c0, c1) = m["box"]
        ref = new(cfgs[i])
        for done in range(0, steps, 1000):
            ref.step(min(1000, steps - done))
            print("c4[%d] reference run step %d" % (i, min(done + 1000, steps)), flush=True)
        phi = ref.fields()["phi"][r0:r1, c0:c1]
        keep = {}
        spread_run(cfgs[i], steps, {steps}, ((r0, r1), (c0, c1)), 7163 + i, ref_at_end=phi,
                   log="c4[%d] area" % i, keep=keep)
        out[str(i)] = [int((phi > 0).sum()), int((keep["phi"] > 0).sum())]
        json.dump(out, open(os.path.join(outdir, "c4_areas%s.json" % ("_" + "_".join(only) if only else "")), "w"),
                  indent=1, sort_keys=True)
        print("c4 member %d areas %s" % (i, out[str(i)]), flush=True)


def c4_part(first, last, outdir):
    """Members first..last-1 into outdir/c4_part.npz and outdir/c4_part.json (for a second machine);
    c4_merge adds such a part to the stored files."""
    cfgs = W.c4_domains()
    steps = cfgs[0]["steps"]
    arrays, members = {}, []
    os.makedirs(outdir, exist_ok=True)
    for i in range(int(first), int(last)):
        a, m = c4_member(i, cfgs[i], steps)
        arrays.update(a)
        members.append(m)
        np.savez_compressed(os.path.join(outdir, "c4_part.npz"), **arrays)
        json.dump(members, open(os.path.join(outdir, "c4_part.json"), "w"), indent=1, sort_keys=True)
        print("c4 member %d done" % i, flush=True)


def c4_merge(outdir):
    steps = W.c4_domains()[0]["steps"]
    old = np.load(C4_NPZ)
    arrays = {k: old[k] for k in old.files}
    members = load()["c4"]["members"]
    have = {m["i"] for m in members}
    areas = {}
    for f in sorted(os.listdir(outdir)):
        if f.startswith("c4_areas") and f.endswith(".json"):
            areas.update(json.load(open(os.path.join(outdir, f))))
    if areas:
        for m in members:
            if str(m["i"]) in areas:
                m["area_ref"], m["area_perturbed"] = areas[str(m["i"])]
    part_file = os.path.join(outdir, "c4_part.json")
    part = np.load(os.path.join(outdir, "c4_part.npz")) if os.path.exists(part_file) else None
    for m in (json.load(open(part_file)) if part is not None else []):
        if m["i"] in have:
            continue
        for k in ("phi", "U", "box"):
            arrays["%s_%d" % (k, m["i"])] = part["%s_%d" % (k, m["i"])]
        members.append(m)
    store_c4(arrays, members, steps)
    print("merged; %d members stored" % len(members), flush=True)


CASES = {"v512": case_v512, "c2": case_c2, "c3": case_c3, "c4": case_c4}


def main(names):
    for n in names:
        r = CASES[n]()
        d = load()
        d[n] = r
        save(d)
        print("wrote", JSON, n, flush=True)


if __name__ == "__main__":
    if sys.argv[1:2] == ["c4part"]:
        c4_part(*sys.argv[2:5])
    elif sys.argv[1:2] == ["c4areas"]:
        c4_areas(*sys.argv[2:])
    elif sys.argv[1:2] == ["c4merge"]:
        c4_merge(sys.argv[2])
    else:
        main(sys.argv[1:] or ["v512"])
