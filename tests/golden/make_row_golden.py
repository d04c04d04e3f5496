"""Write the oracle's results for one full-size row absorption to JSON.

Calls only the FP64 oracle (oracle/) and the seeded input generators
(workloads/). The GPU parity tests compare the device library against the
file this writes; nothing in it comes from the device path.

    python tests/golden/make_row_golden.py --config 2 [--max-cols 8] [--workers 6]
    python tests/golden/make_row_golden.py --config 4 --sites 2 --workers 6

Stored: per site the kept count and the sketch width of every sector, the
singular values of every sector, the log-norm, and the gauge-invariant
network value s_row = <new environment | bottom> for a seeded random bottom
environment (bond = the environment catalogue of the configuration, seed 5).

Committed rows: config 2 (about 30 min on 8 host cores). A whole config-4
row is out of reach of the oracle on such a host (about 1.5 h per site at
sketch widths near 570). ``--sites 2`` stores its first two sites instead
(kept counts, widths and singular values; the sites' results do not depend
on the later sites), on a host with more cores: on 8 cores the oracle's
site 1 ran for more than 3.8 hours. The parity tests check sampled
columns of a full-size site and the chi = 500 lattice whose boundary MPS is
exact.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as wl  # noqa: E402
from oracle.zipup import absorb_row  # noqa: E402
from oracle.expect import overlap  # noqa: E402
from oracle.flops import row_flops  # noqa: E402


def problem(cfg):
    if cfg == 2:
        return wl.config2_row(), wl.legs_dense(4, 6, 6, 128)["env"]
    if cfg == 3:
        return wl.config3_row(), wl.legs_u1u1(256)["env"]
    if cfg == 4:
        return wl.config4_row(), wl.legs_su2(500)["env"]
    raise ValueError(cfg)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--max-cols", type=int, default=8)
    ap.add_argument("--workers", type=int, default=1,
                    help="sectors evaluated in this many processes (same results)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--sites", type=int, default=0,
                    help="stop after this many sites (their kept counts and singular values "
                         "are those of the whole row); 0: the whole row")
    a = ap.parse_args()
    t0 = time.time()
    row, bond = problem(a.config)
    log = lambda s: print(f"[{time.time() - t0:8.1f}s] {s}", flush=True)
    log(f"config {a.config}: chi {row.chi} p {row.oversample} q {row.power_iters}")
    record = []
    env, lg, info = absorb_row(row.sym, row.T, row.A, row.W, row.chi, row.oversample,
                               row.power_iters, a.seed, row=row.row, record=record,
                               max_cols=a.max_cols, progress=log, workers=a.workers,
                               stop_after=a.sites or None)
    if a.sites:
        out = dict(config=a.config, seed=a.seed, chi=row.chi, oversample=row.oversample,
                   power_iters=row.power_iters, row=row.row, sites=a.sites,
                   cpu_seconds=time.time() - t0,
                   kept=[[int(k) for k in ks] for ks in info["kept"]],
                   k=[[int(k) for k in ks] for ks in info["k"]],
                   m=[[int(k) for k in ks] for ks in info["m"]],
                   n=[[int(k) for k in ks] for ks in info["n"]],
                   gap=[float(g) for g in info["gap"]],
                   sigma=[[list(map(float, s)) for s in ss] for ss in info["sigma"]])
        path = a.out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                     f"config{a.config}_row_sites{a.sites}.json")
        with open(path, "w") as f:
            json.dump(out, f)
        log(f"wrote {path}: first {a.sites} sites")
        return
    log("absorbed; flops and network value")
    flops = row_flops(record, info, row.power_iters)
    bot = wl.random_bottom_env(row.sym, env, bond, np.random.default_rng(5))
    v = overlap(env, bot)
    out = dict(config=a.config, seed=a.seed, chi=row.chi, oversample=row.oversample,
               power_iters=row.power_iters, row=row.row, log_norm=lg,
               s_row_sign=int(np.sign(v)), s_row_log=math.log(abs(v)) + lg,
               overlap=v, alg_flops=flops, cpu_seconds=time.time() - t0,
               kept=[[int(k) for k in ks] for ks in info["kept"]],
               k=[[int(k) for k in ks] for ks in info["k"]],
               m=[[int(k) for k in ks] for ks in info["m"]],
               n=[[int(k) for k in ks] for ks in info["n"]],
               gap=[float(g) for g in info["gap"]],
               discarded=[float(d) for d in info["discarded"]],
               sigma=[[list(map(float, s)) for s in ss] for ss in info["sigma"]])
    path = a.out or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                 f"config{a.config}_row.json")
    with open(path, "w") as f:
        json.dump(out, f)
    log(f"wrote {path}: log_norm {lg:.12f} s_row {out['s_row_sign']} exp({out['s_row_log']:.12f})"
        f" flops {flops:.4e}")


if __name__ == "__main__":
    main()
