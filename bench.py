#!/usr/bin/env python3
"""Benchmark of the gfx950 row absorption: one interior row of the 8x8
SU(2)-reduced synthetic workload (reduced D = 6, w = 4, d = 3, chi = 500,
oversampling 20, two power iterations) absorbed into its boundary MPS with
randomized-SVD truncation at every bond.

A step is one full row absorption (8 sites: sketch, chain applications,
orthonormalisation, projection, core factorisation, cut, new environment and
remainder) on inputs resident in HBM. The timed steps run the library as a
caller would (slices of a site spread over four streams); the per-kernel
figures of the roofline come from one more step on one stream with every
launch timed by HIP events. Prints one JSON line.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--config 4]
                    [--precision mixed-vs-fp64|fp64|fp32] [--one-stream]
                    [--lattice] [--config 5] [--calibrate-copy]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "row-absorb+rSVD TFLOP/s, 8x8 D=6 χ=500; mixed vs FP64 speedup @ ≤1e-6 rel err"
PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16": 2516.6}   # dense MFMA TFLOP/s, MI355X
HBM_PEAK = 8000.0                                       # GB/s, MI355X HBM3E


def workload(cfg):
    import workloads as wl
    if cfg == 4:
        row = wl.config4_row()
        desc = ("SU(2)-reduced synthetic 8x8 interior row: D=6 (2j 0,1,2 x 3,2,1), w=4, d=3, "
                "chi=500 (env 2j<=6), p=20, q=2, fermionic signs, random blocks N(0,1)/sqrt(numel)")
        bond = wl.legs_su2(500)["env"]
    elif cfg == 2:
        row = wl.config2_row()
        desc = "dense 8x8 interior row, Hubbard comb PEPO w=6, d=4, D=6, chi=128, p=8, q=1"
        bond = wl.legs_dense(4, 6, 6, 128)["env"]
    elif cfg == 3:
        row = wl.config3_row()
        desc = "U(1)xU(1) 8x8 interior row, D=6 (5 sectors), w=6, d=4, chi=256 (15 sectors), p=8, q=1"
        bond = wl.legs_u1u1(256)["env"]
    else:
        raise SystemExit(f"unknown config {cfg}")
    return row, desc, bond


def bench_config5_row(a):
    """Config 5 on the row's own residuals: the U(1)xU(1) chi = 256 row of
    config 3 absorbed by fpeps_env_absorb with rSVD truncation (p = 8, q = 1)
    and, at every site, controlled bond expansion by ceil(0.1 chi) = 26
    directions taken from the range of (1 - U U^T) M_x (1 - V^T V) on the
    implicit site operator (projector splitting, q = 0). A step is one row;
    the same row without expansion is timed beside it."""
    import torch
    import workloads as wl
    from paper_2511_01039_amd import Context, DeviceTensor, opts_for
    cfg = wl.CONFIG5
    row = wl.config3_row()
    ctx = Context(0)
    dev = lambda ts: [DeviceTensor.from_host(t) for t in ts]
    T, A, W = dev(row.T), dev(row.A), dev(row.W)
    res = {}
    for extra in (cfg["cbe_extra"], 0):
        o = opts_for(row.sym, chi=cfg["chi"], oversample=cfg["oversample"],
                     power_iters=cfg["power_iters"], cbe_extra=extra, seed=0, row=row.row)
        caps = None
        for _ in range(a.warmup):
            out, lg, rep = ctx.env_absorb(T, A, W, o, caps=caps)
            caps = [(max(256, max(l.nsect for l in t.legs)), max(t.blocks.shape[0], 1),
                     max(t.nelem, 1)) for t in out]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        flops = 0.0
        for i in range(a.steps):
            out, lg, rep = ctx.env_absorb(T, A, W, o, caps=caps)
            flops += rep["alg_flops"]
            print(f"config 5 row, cbe_extra {extra}, step {i}: {rep['seconds']:.3f} s device",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / a.steps
        kept = [int(t.legs[4].dims.sum()) for t in out[:-1]]   # new bond dimensions
        res[extra] = dict(sec=sec, flops=flops / a.steps, kept=kept)
    e = res[cfg["cbe_extra"]]
    line = {"metric": "row absorption with controlled bond expansion, per-row latency",
            "value": 1e3 * e["sec"], "unit": "ms", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": 1e3 * e["sec"], "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "config 5: the 8x8 U(1)xU(1) chi=256 row of config 3, rSVD "
                                   "truncation p=8 q=1 and CBE by 26 directions (p=8, q=0) at every "
                                   "site on the implicit site operator",
                       "alg_flops_per_step": e["flops"], "tflops": e["flops"] / e["sec"] / 1e12,
                       "bond_dims_after_expansion": e["kept"],
                       "without_cbe_ms_per_step": 1e3 * res[0]["sec"],
                       "without_cbe_bond_dims": res[0]["kept"]}}
    print(json.dumps(line), flush=True)


def bench_config5(a):
    """Batched bond expansion over one row of config 3: for each interior site
    of the U(1)xU(1) chi = 256 row, the per-sector shapes of its site operator
    (from the library) are filled with seeded explicit matrices of decaying
    spectrum; a step is, for every site, one rSVD truncation of all its
    sectors (chi = 256, p = 8, q = 1, one cut over the sectors) and one
    controlled bond expansion by ceil(0.1 chi) = 26 directions orthogonal to
    the kept left and right spaces (q = 0). All sites go in one grouped
    truncation call and one grouped expansion call (each site its own
    problem); ``--per-site`` makes one call of each per site instead."""
    import torch
    import numpy as np
    import workloads as wl
    from workloads.tensor import Leg
    from paper_2511_01039_amd import Context, DeviceTensor, opts_for, make_opts
    cfg = wl.CONFIG5
    row = wl.config3_row()
    env = wl.legs_u1u1(256)["env"]
    ctx = Context(0)
    rng = np.random.default_rng(0)
    dev = DeviceTensor.from_host
    sites = []
    for x in range(1, len(row.T) - 1):
        T, A, W = row.T[x], row.A[x], row.W[x]
        legs = [env, T.legs[0].flipped(), A.legs[1].flipped(), W.legs[2].flipped(), A.legs[1]]
        legs = [Leg(l.labels, l.dims, d) for l, d in zip(legs, (1, -1, -1, -1, 1))]
        Rt = wl.random_tensor(row.sym, legs, rng)
        _, m, n = ctx.site_shape(dev(Rt), dev(T), dev(A), dev(W), opts_for(row.sym))
        g = torch.Generator(device="cuda").manual_seed(1000 + x)
        mats = []
        for mi, ni in zip(m, n):
            r = int(min(mi, ni))
            s = torch.exp(-torch.arange(r, device="cuda", dtype=torch.float64) / cfg["decay"])
            Am = torch.randn(int(mi), r, generator=g, device="cuda", dtype=torch.float64) / math.sqrt(mi)
            Bm = torch.randn(r, int(ni), generator=g, device="cuda", dtype=torch.float64) / math.sqrt(ni)
            mats.append(((Am * s) @ Bm).contiguous())
        sites.append(mats)
    ropts = make_opts(chi=cfg["chi"], oversample=cfg["oversample"], power_iters=cfg["power_iters"],
                      seed=0, tag=0)
    copts = make_opts(cbe_extra=cfg["cbe_extra"], oversample=cfg["cbe_oversample"], seed=0, tag=1)

    def truncate_expand(mats, group):
        U, R, sig, kept, rep = ctx.rsvd_truncate(mats, ropts, group=group)
        # kept right space V (rows orthonormal): R = S V^T
        Us, Vs = [], []
        for u, rr, sg, k in zip(U, R, sig, kept):
            sg_t = torch.as_tensor(np.asarray(sg[:k]), device="cuda", dtype=torch.float64)
            Us.append(u)
            Vs.append((rr / sg_t[:, None]).contiguous() if k > 0 else rr)
        Q, csig, ckept, crep = ctx.cbe_expand(mats, Us, Vs, copts, group=group)
        return rep["alg_flops"] + crep["alg_flops"]

    all_mats = [a for mats in sites for a in mats]
    all_group = [g for g, mats in enumerate(sites) for _ in mats]

    def step():
        if a.per_site:
            return sum(truncate_expand(mats, None) for mats in sites)
        return truncate_expand(all_mats, all_group)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flops = 0.0
    for _ in range(a.steps):
        flops += step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / a.steps
    nmat = sum(len(s) for s in sites)
    sides = [int(min(t.shape)) for s in sites for t in s]
    line = {"metric": "batched rSVD truncation + bond expansion of one row, per-row latency",
            "value": 1e3 * sec, "unit": "ms", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": 1e3 * sec, "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "config 5: bond expansion over the interior sites of the 8x8 "
                                   "U(1)xU(1) chi=256 row; per site all sector matrices "
                                   f"({nmat} matrices, sides {min(sides)}-{max(sides)}), "
                                   "rSVD chi=256 p=8 q=1 then CBE 26 directions p=8 q=0",
                       "calls": "one per site" if a.per_site else "one grouped call per kind",
                       "alg_flops_per_step": flops / a.steps,
                       "tflops": flops / a.steps / sec / 1e12}}
    print(json.dumps(line), flush=True)


def bench_lattice(a):
    """<W> = Z_W / Z_1 of the full 8x8 SU(2)-synthetic lattice at the shapes of
    the headline row (reduced D = 6, w = 4, d = 3; chi = 500, p = 20, q = 2):
    every row absorbed top to bottom, then closed. W is a near-identity PEPO
    (1 + 0.5 R per site), so that <W> is of order one; with a purely random W
    the value is exponentially small and dominated by cancellation. Runs in
    FP64 and in mixed precision with sketch seed 0, and in FP64 with seed 1
    (the spread of the randomized method itself); prints the values, their
    relative differences, the log-norms and the times."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2511_01039_amd import Context, DeviceTensor, opts_for
    lat = wl.config4_lattice()
    W = wl.near_identity_pepo(lat.sym, wl.legs_su2(500), lat.Lx, lat.Ly, np.random.default_rng(1))
    ident = wl.identity_pepo(lat.sym, lat.Lx, lat.Ly, lat.A[0][0].legs[0])
    ctx = Context(0)
    dev = lambda ts: [DeviceTensor.from_host(t) for t in ts]
    A = [dev(r) for r in lat.A]

    def value(W, precision, seed=0):
        Wd = [dev(r) for r in W]
        env = dev(wl.trivial_env(lat.sym, lat.Lx))
        lg, flops = 0.0, 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for y in range(lat.Ly):
            env, lg, rep = ctx.env_absorb(env, A[y], Wd[y],
                                          opts_for(lat.sym, chi=500, oversample=20, power_iters=2,
                                                   seed=seed, row=y, precision=precision),
                                          log_norm=lg)
            flops += rep["alg_flops"]
            print(f"{precision} seed {seed} row {y}: {rep['seconds']:.3f} s", file=sys.stderr,
                  flush=True)
        v = ctx.expect(env, dev(wl.bottom_closing(env)))
        torch.cuda.synchronize()
        return (1 if v > 0 else -1), lg + math.log(abs(v)), time.perf_counter() - t0, flops

    res = {}
    for key, prec, seed in (("fp64", "fp64", 0), ("fp32", "fp32", 0), ("seed1", "fp64", 1)):
        zw, z1 = value(W, prec, seed), value(ident, prec, seed)
        res[key] = dict(W=zw[0] * z1[0] * math.exp(zw[1] - z1[1]), seconds=zw[2] + z1[2],
                        flops=zw[3] + z1[3], log_zw=zw[1], log_z1=z1[1])
    rel = abs(res["fp32"]["W"] - res["fp64"]["W"]) / abs(res["fp64"]["W"])
    # the method's own spread: FP64 with another sketch seed
    seed_rel = abs(res["seed1"]["W"] - res["fp64"]["W"]) / abs(res["fp64"]["W"])
    line = {"metric": "<W> of the 8x8 SU(2)-synthetic lattice, chi=500: mixed vs FP64",
            "value": res["fp64"]["seconds"] / res["fp32"]["seconds"], "unit": "speedup",
            "n_gpus": 1, "steps": 1, "warmup": 0, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "full 8x8 SU(2)-synthetic lattice (reduced D=6, w=4, d=3, "
                                   "fermionic signs), near-identity W, Z_W and Z_1 top to "
                                   "bottom, chi=500 p=20 q=2"},
            "W_fp64": res["fp64"]["W"], "W_mixed": res["fp32"]["W"], "rel_err": rel,
            "log_zw_diff": abs(res["fp32"]["log_zw"] - res["fp64"]["log_zw"]),
            "log_z1_diff": abs(res["fp32"]["log_z1"] - res["fp64"]["log_z1"]),
            "log_z1_fp64": res["fp64"]["log_z1"],
            "W_fp64_seed1": res["seed1"]["W"], "seed_rel": seed_rel,
            "log_z1_seed_diff": abs(res["seed1"]["log_z1"] - res["fp64"]["log_z1"]),
            "seconds_fp64": res["fp64"]["seconds"], "seconds_mixed": res["fp32"]["seconds"],
            "tflops_fp64": res["fp64"]["flops"] / res["fp64"]["seconds"] / 1e12,
            "tflops_mixed": res["fp32"]["flops"] / res["fp32"]["seconds"] / 1e12}
    print(json.dumps(line), flush=True)


def profiled_traffic(kernel, precision="fp64"):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE runs, calibrated against a plain
    copy), or None when there is none or the kernel source has changed since
    the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_config4_{precision}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    src = fields.get("kernel_source")
    if not src or "traffic_bytes_per_launch" not in fields:
        return None
    src_path = os.path.join(ROOT, src)
    if not os.path.exists(src_path):
        return None
    if hashlib.sha256(open(src_path, "rb").read()).hexdigest() != fields.get("kernel_source_sha256"):
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(row, row_flops, budget_s=20.0, one_thread_s=8.0):
    """The FP64 oracle as it stands, on a bounded sample of the same unit.
    The unit's dominant work (over 95% of its flops) is the chain: here the
    oracle applies M_x at the first interior site (x = 1; a random remainder
    of the structure the truncation of site 0 gives) to the site's full
    first-pass sketch (k_J = min(m_J, n_J, ceil(chi m_J / sum m) + p)
    columns), 4 columns of one sector at a time, until ``budget_s`` of work
    on every host thread; then one piece on one thread. The rate times the
    row's algorithmic flops gives the oracle's estimated time for the row."""
    import numpy as np
    import workloads as wl
    from threadpoolctl import threadpool_limits, threadpool_info
    from workloads.tensor import Leg
    from oracle.blocks import BT
    from oracle.chain import SiteOperator
    from oracle.zipup import SiteProblem
    from oracle.flops import chain_flops
    from oracle.rsvd import sketch_widths
    x = 1
    rng = np.random.default_rng(0)
    T, A, W = row.T[x], row.A[x], row.W[x]
    env = T.legs[0]
    legs = [Leg(env.labels, env.dims, 1), T.legs[0].flipped(), A.legs[1].flipped(),
            W.legs[2].flipped(), A.legs[1]]
    legs = [Leg(l.labels, l.dims, d) for l, d in zip(legs, (1, -1, -1, -1, 1))]
    Rt = wl.random_tensor(row.sym, legs, rng)
    names = ["c", "a", "lk", "lw", "lb"]
    R = BT(names, dict(zip(names, Rt.legs)), Rt.to_dict())
    sp = SiteProblem(SiteOperator(row.sym, R, T, A, W))
    k = sketch_widths(sp.m, sp.n, row.chi, row.oversample)
    ncol = 4
    # tasks: 4 columns of one sector each (sector by sector, largest first)
    order = sorted(range(len(k)), key=lambda J: -sp.n[J])
    tasks = [(J, c0) for J in order for c0 in range(0, k[J], ncol)]

    def run_tasks(limit_s, max_tasks):
        done_flops, secs, count = 0.0, 0.0, 0
        for J, c0 in tasks:
            kc = [min(ncol, k[J] - c0) if i == J else 0 for i in range(len(k))]
            X = [rng.standard_normal((n, w)) for n, w in zip(sp.n, kc)]
            t0 = time.perf_counter()
            sp.apply_m(X)
            secs += time.perf_counter() - t0
            done_flops += float(chain_flops(sp, kc))
            count += 1
            if secs >= limit_s or count >= max_tasks:
                break
        return done_flops, secs, count

    threads = max((p.get("num_threads", 1) for p in threadpool_info()), default=1)
    f_all, s_all, c_all = run_tasks(budget_s, 10 ** 6)
    with threadpool_limits(limits=1):
        f_one, s_one, c_one = run_tasks(one_thread_s, 1)
    rate = f_all / s_all
    return {"value": rate / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"oracle M_x X at site 1 of the same row with the site's first-pass sketch "
                      f"widths ({sum(k)} columns over {len(sp.sect)} sectors), {ncol} columns "
                      f"of one sector at a time, largest sectors first: {c_all} of "
                      f"{len(tasks)} pieces, {f_all:.3e} flops in {s_all:.1f} s on "
                      f"{threads} threads",
            "one_thread": {"value": f_one / s_one / 1e12, "unit": "TFLOP/s",
                           "sample": f"{c_one} piece, {f_one:.3e} flops in {s_one:.1f} s"},
            "row_seconds_estimate": row_flops / rate}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--precision", default="mixed-vs-fp64", choices=["mixed-vs-fp64", "fp64", "fp32"],
                    help="mixed-vs-fp64 (default): time both paths on the same row and report the "
                         "mixed one if its network value is within 1e-6 of FP64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", type=int, default=2,
                    help="tile candidates of the autotuner, run on the headline row in its first "
                         "warmup step (slice budget and GEMM tiles measured on the row); 0: the "
                         "planner's model")
    ap.add_argument("--tune-file", default="",
                    help="load this tuned table (written by --save-tune) instead of tuning")
    ap.add_argument("--save-tune", default="", help="write the tuned table to this file")
    ap.add_argument("--per-site", action="store_true",
                    help="config 5 --explicit: one truncation and one expansion call per site")
    ap.add_argument("--explicit", action="store_true",
                    help="config 5 on seeded explicit matrices of the sites' sector shapes "
                         "(grouped truncation and expansion calls) instead of the row's own "
                         "residuals")
    ap.add_argument("--slice-budget-gib", type=float, default=0.0,
                    help="workspace per slice set in GiB (0: the library's default)")
    ap.add_argument("--one-stream", action="store_true",
                    help="run every slice on one stream (no overlap of slices)")
    ap.add_argument("--lattice", action="store_true",
                    help="<W> of the full 8x8 lattice at the headline shapes, FP64 and mixed")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 4 times (the known-size "
                         "reference for HBM byte counters) and exit")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the row absorption runs on a single MI355X; "
              "--gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if a.calibrate_copy:
        n = 1 << 27                      # 2^27 doubles = 1 GiB
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy": {"bytes_read_per_copy": 8 * n,
                                             "bytes_written_per_copy": 8 * n, "copies": 4}}))
        return
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.config == 5:
        if a.explicit:
            bench_config5(a)
        else:
            bench_config5_row(a)
        return
    if a.lattice:
        bench_lattice(a)
        return
    from paper_2511_01039_amd import Context, DeviceTensor, opts_for
    from paper_2511_01039_amd.binding import FLAG_TIME_KERNELS, FLAG_ONE_STREAM
    import numpy as np
    import workloads as wl
    row, desc, bond = workload(a.config)
    dev = lambda ts: [DeviceTensor.from_host(t) for t in ts]
    T, A, W = dev(row.T), dev(row.A), dev(row.W)
    ctx = Context(0)

    def run(precision, steps, warmup, tune_here):
        """``warmup`` untimed + ``steps`` timed absorptions of the row;
        device-resident inputs. The last warmup step (or one more step when
        there is none) is the kernel-timing step."""
        kw = dict(chi=row.chi, oversample=row.oversample, power_iters=row.power_iters, seed=0,
                  row=row.row, precision=precision, slice_budget=int(a.slice_budget_gib * 2**30))
        # timed steps: the library's default four streams (slices overlap);
        # kernel figures: one more step on one stream with every launch timed
        # by HIP events (overlapping launches would stretch each other's
        # durations)
        base = FLAG_ONE_STREAM if a.one_stream else 0
        opts = opts_for(row.sym, flags=base, **kw)
        kopts = opts_for(row.sym, flags=FLAG_ONE_STREAM | FLAG_TIME_KERNELS, **kw)
        caps = None
        krep = None
        tune = None
        for i in range(warmup):
            last = i == warmup - 1
            if i == 0 and tune_here:
                # slice budget and GEMM tiles measured on this row (untimed);
                # the context keeps them for every later absorption
                t0 = time.perf_counter()
                out, lg, rep = ctx.env_absorb(T, A, W, opts, caps=caps, autotune=a.autotune)
                n, b = ctx.tune_info()
                tune = {"tile_candidates": a.autotune, "tuned_signatures": n,
                        "slice_budget_gib": b / 2**30,
                        "tuning_seconds": time.perf_counter() - t0}
                print(f"{precision} autotune: {n} step signatures, slice budget "
                      f"{b / 2**30:.0f} GiB, {tune['tuning_seconds']:.1f} s", file=sys.stderr,
                      flush=True)
                caps = [(max(256, max(l.nsect for l in t.legs)), max(t.blocks.shape[0], 1),
                         max(t.nelem, 1)) for t in out]
                if not last:
                    continue
            out, lg, rep = ctx.env_absorb(T, A, W, kopts if last else opts, caps=caps)
            print(f"{precision} warmup {i}{' (kernel-timing, one stream)' if last else ''}: "
                  f"{rep['seconds']:.3f} s device", file=sys.stderr, flush=True)
            caps = [(max(256, max(l.nsect for l in t.legs)), max(t.blocks.shape[0], 1),
                     max(t.nelem, 1)) for t in out]
            if last:
                krep = rep
        r = dict(flops=0.0, dev_s=0.0, alg_bytes=0.0)
        cls = {k: 0.0 for k in ("layer_launches", "layer_seconds", "layer_flops", "layer_bytes",
                                "gemm_launches", "gemm_seconds", "gemm_flops", "gemm_bytes")}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            out, lg, rep = ctx.env_absorb(T, A, W, opts, caps=caps)
            r["flops"] += rep["alg_flops"]
            r["alg_bytes"] += rep["alg_bytes"]
            r["dev_s"] += rep["seconds"]
            print(f"{precision} step {i}: {rep['seconds']:.3f} s device", file=sys.stderr,
                  flush=True)
        torch.cuda.synchronize()
        r["sec"] = (time.perf_counter() - t0) / steps
        r["value"] = r["flops"] / steps / r["sec"] / 1e12
        r["steps"] = steps
        if krep is None:
            _, _, krep = ctx.env_absorb(T, A, W, kopts, caps=caps)
            print(f"{precision} kernel-timing step (one stream): {krep['seconds']:.3f} s device",
                  file=sys.stderr, flush=True)
        for k in cls:
            cls[k] = krep[k]
        r["kernel_step_s"] = krep["seconds"]
        r["cls"], r["out"], r["lg"] = cls, out, lg
        r["tune"] = tune
        # singular values of every truncated site (the kernel-timing step's,
        # same arithmetic as the timed steps)
        r["sig"] = [ctx.absorb_diag(x)[0] for x in range(len(out) - 1)]
        return r

    precs = ["fp64", "fp32"] if a.precision == "mixed-vs-fp64" else [a.precision]
    # the headline path times exactly --steps steps; the mixed path beside it
    # (a comparison) at most 3 after at most 1 warmup step
    res = {}
    # the autotuner runs once, on the headline path's row, in its first
    # warmup step; a saved table (--tune-file) replaces it
    if a.tune_file:
        ctx.tune_load(a.tune_file)
    for i, p in enumerate(precs):
        res[p] = run(p, a.steps if i == 0 else min(a.steps, 3),
                     a.warmup if i == 0 else min(a.warmup, 1),
                     i == 0 and a.autotune > 0 and not a.tune_file)
    if a.save_tune and ctx.tune_info()[0] >= 0:
        ctx.tune_save(a.save_tune)
    # mixed vs FP64: the gauge-invariant network value of the new environment
    # against one fixed random bottom environment, both on the device
    cmp = None
    if len(precs) == 2:
        bot = dev(wl.random_bottom_env(row.sym, res["fp64"]["out"], bond,
                                       np.random.default_rng(5)))
        v64, v32 = ctx.expect(res["fp64"]["out"], bot), ctx.expect(res["fp32"]["out"], bot)
        rel = abs(v32 / v64 * math.exp(res["fp32"]["lg"] - res["fp64"]["lg"]) - 1.0)
        # context for that difference: the same FP64 absorption with another
        # sketch seed (untimed)
        caps = [(max(256, max(l.nsect for l in t.legs)), max(t.blocks.shape[0], 1),
                 max(t.nelem, 1)) for t in res["fp64"]["out"]]
        o1 = opts_for(row.sym, chi=row.chi, oversample=row.oversample,
                      power_iters=row.power_iters, seed=1, row=row.row, precision="fp64",
                      slice_budget=int(a.slice_budget_gib * 2**30))
        out1, lg1, _ = ctx.env_absorb(T, A, W, o1, caps=caps)
        v1 = ctx.expect(out1, bot)
        seed_rel = abs(v1 / v64 * math.exp(lg1 - res["fp64"]["lg"]) - 1.0)
        cmp = {"speedup": res["fp64"]["sec"] / res["fp32"]["sec"], "s_row_rel_err": rel,
               "tolerance": 1e-6, "fp64_value": res["fp64"]["value"],
               "fp64_ms_per_step": 1e3 * res["fp64"]["sec"],
               "mixed_value": res["fp32"]["value"], "mixed_ms_per_step": 1e3 * res["fp32"]["sec"],
               "mixed_steps": res["fp32"]["steps"],
               "fp64_other_seed_s_row_rel": seed_rel,
               # largest norm-wise relative difference of a site's singular
               # values (all computed ones, kept and cut) between the two paths
               "sigma_rel_max": max(
                   (float(np.linalg.norm(a32 - a64) / max(np.linalg.norm(a64), 1e-300))
                    for a32, a64 in zip(res["fp32"]["sig"], res["fp64"]["sig"])
                    if a32.shape == a64.shape and a64.size), default=float("nan"))}
    # the reported figure: the first path (FP64 by default), timed over
    # exactly --steps steps; the mixed path's speedup and error sit beside it
    rep_prec = precs[0]
    R = res[rep_prec]
    cls = R["cls"]
    # Dominant kernel by measured time, with its ALGORITHMIC work per launch
    # (the oracle's count: 2 m n k over the block pairs the launch
    # contracts) over its average launch duration. The layer-step kernel
    # (ket, PEPO and bra contractions) runs on the FP64 vector ALU (peak
    # 256 CU x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz = 78.6 TFLOP/s); the
    # environment/remainder kernel on MFMA (FP64 78.6, FP32 157.3 TFLOP/s).
    # Counter traffic (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated on a
    # plain copy) is reported beside it and against the path's algorithmic
    # bytes (T, R, ket and PEPO read once and the output written once per
    # chain application; the chain intermediates are not algorithmic).
    lay_s, gem_s = cls["layer_seconds"], cls["gemm_seconds"]
    nl, ng = max(cls["layer_launches"], 1), max(cls["gemm_launches"], 1)
    layer_tfs = cls["layer_flops"] / lay_s / 1e12 if lay_s > 0 else 0.0
    gemm_tfs = cls["gemm_flops"] / gem_s / 1e12 if gem_s > 0 else 0.0
    layer_traffic = profiled_traffic("k_rt_f64", rep_prec)
    gemm_traffic = profiled_traffic("k_gemm_f64", rep_prec)
    gemm_peak = PEAK["fp64"]
    if lay_s >= gem_s:
        roof = {"bound": "alu", "achieved": layer_tfs, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                "frac": layer_tfs / PEAK["fp64"], "traffic": layer_traffic,
                "kernel": "k_rt_f64 (ket/PEPO/bra layer steps and transposes; FP64 vector FMA)",
                "launches_per_step": cls["layer_launches"], "avg_launch_ms": 1e3 * lay_s / nl,
                "flops_per_launch": cls["layer_flops"] / nl,
                "counter_vs_intermediate_bytes": (layer_traffic / (cls["layer_bytes"] / nl))
                if layer_traffic else None}
    else:
        roof = {"bound": "mfma", "achieved": gemm_tfs, "peak": gemm_peak, "unit": "TFLOP/s",
                "frac": gemm_tfs / gemm_peak, "traffic": gemm_traffic,
                "kernel": "k_gemm (environment/remainder contractions, FP64 MFMA)",
                "launches_per_step": cls["gemm_launches"], "avg_launch_ms": 1e3 * gem_s / ng,
                "flops_per_launch": cls["gemm_flops"] / ng}
    roof["kernels"] = {
        "k_rt_f64": {"seconds_per_step": lay_s, "TFLOP/s": layer_tfs,
                     "frac_fp64_alu": layer_tfs / PEAK["fp64"],
                     "intermediate_GB/s": cls["layer_bytes"] / lay_s / 1e9 if lay_s > 0 else 0.0,
                     "counter_bytes_per_launch": layer_traffic},
        "k_gemm": {"seconds_per_step": gem_s, "TFLOP/s": gemm_tfs,
                   "frac_fp64_mfma": gemm_tfs / PEAK["fp64"],
                   "counter_bytes_per_launch": gemm_traffic}}
    alg_b = R["alg_bytes"] / R["steps"]
    counter_step = None
    if layer_traffic and gemm_traffic:
        counter_step = layer_traffic * cls["layer_launches"] + gemm_traffic * cls["gemm_launches"]
    roof["path"] = {"alg_flops_per_step": R["flops"] / R["steps"], "alg_bytes_per_step": alg_b,
                    "row_frac_fp64_peak": R["value"] / PEAK["fp64"],
                    "counter_bytes_per_step": counter_step,
                    "counter_over_algorithmic_bytes": (counter_step / alg_b)
                    if counter_step and alg_b > 0 else None}
    roof["timing"] = ("HIP events around every launch in an untimed step of the same row on "
                      "one stream (the last warmup step; launches do not overlap); the timed "
                      "steps spread slices over four streams")
    line = {"metric": METRIC, "value": R["value"], "unit": "TFLOP/s", "n_gpus": 1,
            "steps": a.steps, "warmup": a.warmup, "ms_per_step": R["sec"] * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            # FP64: every product and sum in FP64. Mixed: the two outer chain
            # products of the range finder on FP32 MFMA (FP32 sums per 16-deep
            # K tile, tiles added in FP64), the rest FP64
            "dtype": "f32+f64" if rep_prec == "fp32" else "f64", "data": "synthetic",
            "config": {"workload": desc, "lattice": "8x8", "chi": row.chi,
                       "precision": "mixed (FP32 MFMA outer chain products of the range finder)"
                       if rep_prec == "fp32" else "fp64",
                       "alg_flops_per_step": R["flops"] / R["steps"],
                       "device_seconds_per_step": R["dev_s"] / R["steps"]},
            "roofline": roof,
            # how the slice budget and GEMM tiles of the timed steps were chosen
            "autotune": R.get("tune") or ({"loaded": a.tune_file} if a.tune_file else None)}
    if cmp is not None:
        line["mixed_vs_fp64"] = cmp
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(row, R["flops"] / R["steps"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
