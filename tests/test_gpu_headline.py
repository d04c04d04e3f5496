"""Headline parity at the target shapes (needs a GPU): the 8x8 lattice at
reduced D = 6, w = 4, d = 3 with chi = 500, p = 20, q = 2 whose boundary MPS
is exact at chi (``workloads.lowrank_su2_lattice``), <W> = Z_W / Z_1
absorbed row by row on the device, against the FP64 oracle's value stored
in tests/golden/lowrank_lattice.json (written by make_lattice_golden.py from
the oracle only). FP64 within 1e-11 relative, mixed precision within 1e-6;
kept counts of every row and site exact. Full config-4 / 2 / 3 rows against
their stored oracle rows (kept counts, singular values, log-norm, s_row)
where the golden files exist."""
import json
import math
import os

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01039_amd import Context
    c = Context(0)
    yield c
    c.close()


def dev(ts):
    from paper_2511_01039_amd import DeviceTensor
    return [DeviceTensor.from_host(t) for t in ts]


def lattice_Z(ctx, lat, W, prm, precision):
    from paper_2511_01039_amd import opts_for
    env = dev(wl.trivial_env(lat.sym, lat.Lx))
    lg = 0.0
    kept, secs = [], 0.0
    for y in range(lat.Ly):
        env, lg, rep = ctx.env_absorb(env, dev(lat.A[y]), dev(W[y]),
                                      opts_for(lat.sym, chi=prm["chi"], oversample=prm["oversample"],
                                               power_iters=prm["power_iters"], seed=prm["seed"],
                                               row=y, precision=precision), log_norm=lg)
        kept.append([int(sum(ctx.absorb_diag(x)[2])) for x in range(lat.Lx - 1)])
        secs += rep["seconds"]
    closing = dev(wl.bottom_closing([t.to_host() for t in env]))
    sg, la = ctx.expect_log(env, closing, lg, 0.0)
    return sg, la, kept, secs


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-6)])
def test_lowrank_lattice_W(ctx, precision, tol):
    g = json.load(open(os.path.join(GOLDEN, "lowrank_lattice.json")))
    prm = g["params"]
    lat, ident = wl.lowrank_su2_lattice(seed=prm["seed"])
    sw, lw, kw, tw = lattice_Z(ctx, lat, lat.W, prm, precision)
    s1, l1, k1, t1 = lattice_Z(ctx, lat, ident, prm, precision)
    got = sw * s1 * math.exp(lw - l1)
    want = g["W"]
    rel = abs(got - want) / abs(want)
    print(f"8x8 <W> {precision}: oracle {want:.15e} gpu {got:.15e} rel {rel:.2e} "
          f"(log Z_W {lw:.12f} / {g['Z_W']['log']:.12f}; device {tw + t1:.2f} s)")
    assert [[sum(x) for x in r["kept"]] for r in g["rows_W"]] == kw
    assert [[sum(x) for x in r["kept"]] for r in g["rows_1"]] == k1
    assert sw == g["Z_W"]["sign"] and s1 == g["Z_1"]["sign"]
    assert rel < tol
    assert abs(lw - g["Z_W"]["log"]) < tol * max(1.0, abs(lw))
