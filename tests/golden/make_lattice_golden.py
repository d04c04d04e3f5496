"""Write the oracle's <W> of the 8x8 lattice whose boundary MPS is exact at
chi = 500 (``workloads.lowrank_su2_lattice``) to JSON.

Calls only the FP64 oracle (oracle/) and the seeded input generators
(workloads/); nothing in it comes from the device path. The GPU test
``test_gpu_headline.py`` compares the library's <W> = Z_W / Z_1 (FP64 and
mixed precision) with the values stored here.

    python tests/golden/make_lattice_golden.py

Stored: sign and log |Z| of Z_W and Z_1, <W>, and per row and site the kept
counts and the number of factorisation passes.
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

import workloads as wl  # noqa: E402
from oracle.zipup import absorb_row  # noqa: E402
from oracle.expect import overlap  # noqa: E402


def value(lat, W, prm, log, max_cols):
    env = wl.trivial_env(lat.sym, lat.Lx)
    lg = 0.0
    rows = []
    for y in range(lat.Ly):
        t0 = time.time()
        env, lg, info = absorb_row(lat.sym, env, lat.A[y], W[y], prm["chi"], prm["oversample"],
                                   prm["power_iters"], prm["seed"], row=y, log_norm=lg,
                                   max_cols=max_cols)
        rows.append(dict(kept=[[int(v) for v in k] for k in info["kept"]],
                         passes=[len(p) for p in info["passes"]], log_norm=lg))
        log(f"row {y}: kept {[sum(k) for k in info['kept']]} in {time.time() - t0:.1f}s")
    v = overlap(env, wl.bottom_closing(env))
    return (1 if v > 0 else -1), lg + math.log(abs(v)), rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-cols", type=int, default=16)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    t0 = time.time()
    log = lambda s: print(f"[{time.time() - t0:8.1f}s] {s}", flush=True)
    prm = wl.LOWRANK_PARAMS
    lat, ident = wl.lowrank_su2_lattice(seed=prm["seed"])
    sw, lw, rows_w = value(lat, lat.W, prm, log, a.max_cols)
    s1, l1, rows_1 = value(lat, ident, prm, log, a.max_cols)
    ratio = sw * s1 * math.exp(lw - l1)
    out = dict(lattice="lowrank_su2_lattice 8x8", params=prm, Z_W=dict(sign=sw, log=lw),
               Z_1=dict(sign=s1, log=l1), W=ratio, rows_W=rows_w, rows_1=rows_1,
               cpu_seconds=time.time() - t0)
    path = a.out or os.path.join(os.path.dirname(os.path.abspath(__file__)), "lowrank_lattice.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    log(f"wrote {path}: <W> = {ratio:.15e}")


if __name__ == "__main__":
    main()
