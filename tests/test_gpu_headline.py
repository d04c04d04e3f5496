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
from oracle.expect import overlap

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


ROWS = {2: ("config2_row", lambda: wl.legs_dense(4, 6, 6, 128)["env"]),
        3: ("config3_row", lambda: wl.legs_u1u1(256)["env"]),
        4: ("config4_row", lambda: wl.legs_su2(500)["env"])}
ROW_GOLDENS = [c for c in sorted(ROWS) if os.path.exists(os.path.join(GOLDEN, f"config{c}_row.json"))]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("cfg", ROW_GOLDENS)
def test_full_row_matches_golden(ctx, cfg, precision):
    """A full-size row of the configuration absorbed on the device against
    the oracle's stored row: kept counts of every site and sector exact,
    singular values of every site, the log-norm and the network value
    s_row = <new environment | seeded random bottom> within 1e-11 relative
    in FP64, and in mixed precision within max(1e-6, 2^-24 / g) (g the
    smallest relative gap at a cut of the oracle's row: a cut subspace
    moves by the rounding over the gap, Davis-Kahan); s_row, which cancels,
    within that bound times its condition number where that is larger."""
    from paper_2511_01039_amd import opts_for
    g = json.load(open(os.path.join(GOLDEN, f"config{cfg}_row.json")))
    name, bond = ROWS[cfg]
    row = getattr(wl, name)()
    out, lg, rep = ctx.env_absorb(dev(row.T), dev(row.A), dev(row.W),
                                  opts_for(row.sym, chi=g["chi"], oversample=g["oversample"],
                                           power_iters=g["power_iters"], seed=g["seed"],
                                           row=g["row"], precision=precision))
    fp64 = precision == "fp64"
    gaps = [x for x in g["gap"] if np.isfinite(x)]
    tol = 1e-11 if fp64 else max(1e-6, 2.0 ** -24 / max(min(gaps) if gaps else 1.0, 1e-300))
    worst = 0.0
    for x in range(len(out) - 1):
        sig, sec, kept = ctx.absorb_diag(x)
        assert [int(v) for v in kept] == g["kept"][x]
        want = np.concatenate([np.asarray(s) for s in g["sigma"][x]])
        assert sig.shape == want.shape
        worst = max(worst, float(np.abs(sig - want).max() / want.max()))
    env_h = [t.to_host() for t in out]
    bot_h = wl.random_bottom_env(row.sym, env_h, bond(), np.random.default_rng(5))
    sg, la = ctx.expect_log(out, dev(bot_h), lg, 0.0)
    dlog = abs(la - g["s_row_log"])
    # s_row is an overlap with a random environment, which cancels: a
    # relative change d of the environment (as a vector) moves it by up to
    # kappa d, kappa = |env| |bot| / |<env|bot>| (norms by the oracle's
    # contraction). d is bounded by the cut subspaces' rounding over their
    # gap at each of the L - 1 truncated sites.
    kappa = math.sqrt(overlap(env_h, mirror(env_h)) * overlap(mirror(bot_h), bot_h)) / \
        abs(overlap(env_h, bot_h))
    u = 2.0 ** -53 if fp64 else 2.0 ** -24
    d = (len(out) - 1) * u / max(min(gaps) if gaps else 1.0, 1e-300)
    tol_s = max(tol, kappa * d)
    print(f"config {cfg} {precision}: s_row log {la:.12f} oracle {g['s_row_log']:.12f} "
          f"(rel {dlog:.2e}, kappa {kappa:.3e}, bound {tol_s:.2e}), log-norm diff "
          f"{abs(lg - g['log_norm']):.2e}, sigma max diff {worst:.2e} of the largest, bound "
          f"{tol:.2e}, device {rep['seconds']:.3f} s")
    assert sg == g["s_row_sign"]
    assert dlog < tol_s
    assert abs(lg - g["log_norm"]) < tol * max(1.0, abs(g["log_norm"]))
    assert worst < (1e-10 if fp64 else tol)


def mirror(env):
    """The environment with its bundle legs reversed (same blocks and data):
    the plain overlap of an environment with its mirror is its squared norm."""
    from workloads.tensor import Leg, Tensor
    out = []
    for t in env:
        legs = [Leg(t.legs[0].labels, t.legs[0].dims, -t.legs[0].dir)] + \
            [t.legs[i].flipped() for i in (1, 2, 3)] + \
            [Leg(t.legs[4].labels, t.legs[4].dims, -t.legs[4].dir)]
        out.append(Tensor(legs, t.blocks, t.offsets, t.data))
    return out


SITE_GOLDENS = [c for c in sorted(ROWS)
                if os.path.exists(os.path.join(GOLDEN, f"config{c}_row_sites2.json"))]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("cfg", SITE_GOLDENS)
def test_row_first_sites_match_golden(ctx, cfg, precision):
    """The headline row at full size (config 4: 8x8 SU(2)-synthetic, D = 6,
    chi = 500, p = 20, q = 2) absorbed on the device, against the oracle's
    first two sites of the same row (the whole row is out of the oracle's
    reach on the host): the kept count of every sector exact (in mixed
    precision when the cut's smallest relative gap g exceeds 1e-5, so that
    rounding cannot move it), and the singular values of every sector within
    1e-10 of the largest in FP64 (max(1e-6, 2^-24 / g) in mixed precision)."""
    from paper_2511_01039_amd import opts_for
    g = json.load(open(os.path.join(GOLDEN, f"config{cfg}_row_sites2.json")))
    name, _ = ROWS[cfg]
    row = getattr(wl, name)()
    out, lg, rep = ctx.env_absorb(dev(row.T), dev(row.A), dev(row.W),
                                  opts_for(row.sym, chi=g["chi"], oversample=g["oversample"],
                                           power_iters=g["power_iters"], seed=g["seed"],
                                           row=g["row"], precision=precision))
    fp64 = precision == "fp64"
    gaps = [x for x in g["gap"] if np.isfinite(x)]
    tol = 1e-10 if fp64 else max(1e-6, 2.0 ** -24 / max(min(gaps) if gaps else 1.0, 1e-300))
    for x in range(g["sites"]):
        sig, sec, kept = ctx.absorb_diag(x)
        if fp64 or (gaps and min(gaps) > 1e-5):
            assert [int(v) for v in kept] == g["kept"][x], x
        want = np.concatenate([np.asarray(s) for s in g["sigma"][x]])
        assert sig.shape == want.shape, x
        err = float(np.abs(sig - want).max() / want.max())
        print(f"config {cfg} {precision} site {x}: kept {sum(g['kept'][x])}, sigma max diff "
              f"{err:.2e} of the largest (bound {tol:.1e}), row {rep['seconds']:.2f} s")
        assert err < tol
