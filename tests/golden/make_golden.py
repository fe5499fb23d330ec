"""Write the stored end-to-end results of the FP64 oracle that the GPU parity
tests compare with.  Calls only the oracle (oracle/) and the seeded input
generator; nothing here comes from the HIP path.

The oracle runs the plain iteration of the paper: Sinkhorn on every cell
(Remark "Sinkhorn algorithm"; stop on the L1 X-marginal error after a
Y-iteration, Sec. 6.2), no acceleration and no Newton steps, over the whole
multi-scale eps schedule (Algorithm 2 with the refinement of Sec. 6.4).

Stored per workload: W2^2 = <c, pi> of the last half-iteration's cell plans,
the objective, the L1 marginal errors, nnz, and per basic cell (all of them,
or a seeded sample) the mass |nu_i| and the barycentre of nu_i in pixel
units of the finest grid (row, col): the basic-cell transport targets.

Usage: python tests/golden/make_golden.py {config2,config3,power3} [n_threads]
(config 3 takes about an hour and a half on 8 cores).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import ddo  # noqa: E402
from paper_2001_10986_amd import datagen  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def basic_summary(o, W, sample=None):
    e = o.export()
    rp, col, val = e["row_ptr"], e["col"], e["val"]
    nb = len(rp) - 1
    ids = np.arange(nb) if sample is None else np.sort(
        np.random.default_rng(0).choice(nb, size=sample, replace=False))
    mass, br, bc = [], [], []
    for b in ids:
        v = val[rp[b]:rp[b + 1]]
        c = col[rp[b]:rp[b + 1]]
        m = float(v.sum())
        mass.append(m)
        br.append(float(np.dot(v, c // W) / m))
        bc.append(float(np.dot(v, c % W) / m))
    return {"ids": [int(i) for i in ids], "mass": mass, "mean_row": br, "mean_col": bc}


def run(name, mu, nu, cfg, n_threads, sample=None):
    t = time.time()
    o = ddo.Oracle(mu, nu, s=cfg["s"], n_levels=cfg["n_levels"], eps=cfg["stages"][0][1],
                   accel=0, newton_after=0, n_threads=n_threads, cost_p=cfg.get("cost_p", 2.0))
    st = o.run_schedule(cfg["stages"])
    c = o.cost()
    out = {
        "workload": name,
        "oracle": "FP64, plain Sinkhorn per cell (accel 0, newton_after 0), Err 1e-5, "
                  "trunc 1e-15, loop cap 50000 with the eps safeguard",
        "stages": [list(s) for s in cfg["stages"]],
        "cost_p": cfg.get("cost_p", 2.0),
        "w2_sq": c["cost"], "obj": c["obj"], "err_x": c["err_x"], "err_y": c["err_y"],
        "mass_drift": c["mass_drift"], "nnz": int(c["nnz"]),
        "loops_total": int(st["loops_total"]), "loops_max": int(st["loops_max"]),
        "n_failed": int(st["n_failed"]), "n_safeguard": int(st["n_safeguard"]),
        "basic": basic_summary(o, mu.shape[1], sample),
        "seconds": time.time() - t,
    }
    return out


def main():
    which = sys.argv[1]
    n_threads = int(sys.argv[2]) if len(sys.argv) > 2 else 0
    if which == "config2":
        mu, nu, cfg = datagen.config2_pair()
        out = run("config 2: 256x256 pair (images 0, 1; 8 blobs), levels 64->256, "
                  "eps 1 -> (1/256)^2", mu, nu, cfg, n_threads)
    elif which == "power3":
        mu, nu = datagen.small_pair(64, 4, seed=17)
        cfg = dict(s=4, n_levels=2, cost_p=3.0,
                   stages=datagen.eps_schedule(64, 2, p=3.0, level_factor=16.0,
                                               final_eps=16.0 / 64 ** 3))
        out = run("64x64 pair (4 blobs, seed 17), cost |x-y|^3, levels 32->64, eps 1 -> "
                  "16 (1/64)^3", mu, nu, cfg, n_threads)
    elif which == "config3":
        mu, nu, cfg = datagen.config3_pair()
        out = run("config 3: 1024x1024 pair (16 blobs + U[0,0.1]*max noise), levels "
                  "64->1024, eps 1 -> (1/1024)^2", mu, nu, cfg, n_threads, sample=4096)
    else:
        raise SystemExit(f"unknown workload {which}")
    path = os.path.join(HERE, f"oracle_plain_{which}.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")
    print(f"{path}: W2^2 {out['w2_sq']:.15g}, {out['seconds']:.0f} s")


if __name__ == "__main__":
    main()
