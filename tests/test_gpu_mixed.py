"""Mixed precision (FPEPS_FP32) against the FP64 oracle (needs a GPU).

In this mode the environment and remainder products of the earlier
range-finder applications run on FP32 MFMA from FP32 copies of T and R, the
chain intermediates are stored in FP32, and the last range-finder product,
the projection and the factorisations stay FP64. The chain itself is checked
norm-wise per sector (elements near zero carry the FP32 rounding of their
larger neighbours); each case also checks that the error is above the FP64
level, i.e. that the FP32 path is really in use.

Bound for truncated results. The FP32 rounding perturbs M by about
u = 2^-24 relative; the kept subspace of a cut whose relative gap is g then
moves by about u / g (Davis & Kahan, SIAM J. Numer. Anal. 7 (1970) 1), and
every gauge-invariant value built on it with it. The bound is
max(1e-6, u / g) with g the smallest relative gap at a cut of the run (the
oracle's own): 1e-6 where the cuts are well separated (the target bound of
the headline <W>, test_gpu_headline.py, whose cut keeps the exact rank),
larger where a cut splits a near-degenerate pair.
"""
import math

import numpy as np
import pytest

import workloads as wl
from workloads.tensor import Leg

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-6
U32 = 2.0 ** -24


def gap_tol(*infos):
    """max(1e-6, u / g), g the smallest relative gap at a cut in the
    oracle's runs (lists of per-row info dicts or single info dicts)."""
    gaps = []
    for inf in infos:
        for i in (inf if isinstance(inf, list) else [inf]):
            gaps += [g for g in i["gap"] if np.isfinite(g)]
    g = min(gaps) if gaps else 1.0
    return max(MIXED_TOL, U32 / max(g, 1e-300))


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01039_amd import Context
    c = Context(0)
    yield c
    c.close()


def dev(t):
    from paper_2511_01039_amd import DeviceTensor
    return DeviceTensor.from_host(t)


def devs(ts):
    return [dev(t) for t in ts]


def normwise(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = [
    ("none", dict(kind="none", L=3, d=2, D=3, w=2, chi=9)),
    ("u1u1", dict(kind="u1u1", L=3, env_scale=3, virt_scale=2)),
    ("su2", dict(kind="su2", L=3, env_scale=4, virt_scale=2)),
]


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_site_chain_mixed_matches_oracle(ctx, name, kw):
    """a3 in mixed precision: M_x X and M_x^T Y per sector within 1e-6
    (norm-wise) of the FP64 oracle."""
    import torch
    from oracle.blocks import BT
    from oracle.chain import SiteOperator
    from oracle.zipup import SiteProblem
    from paper_2511_01039_amd import opts_for
    row = wl.small_row(seed=5, **kw)
    rng = np.random.default_rng(11)
    x = 1
    T, A, W = row.T[x], row.A[x], row.W[x]
    cat = row.meta["cat"]["env"]
    legs = [cat, T.legs[0].flipped(), A.legs[1].flipped(), W.legs[2].flipped(), A.legs[1]]
    legs = [Leg(l.labels, l.dims, d) for l, d in zip(legs, (1, -1, -1, -1, 1))]
    Rt = wl.random_tensor(row.sym, legs, rng)
    names = ["c", "a", "lk", "lw", "lb"]
    sp = SiteProblem(SiteOperator(row.sym, BT(names, dict(zip(names, Rt.legs)), Rt.to_dict()),
                                  T, A, W))
    opts = opts_for(row.sym, precision="fp32")
    widths = [1, 5, 37]
    k = [widths[i % 3] for i in range(len(sp.sect))]
    errs = []
    for transpose in (False, True):
        rows_in = sp.m if transpose else sp.n
        rows_out = sp.n if transpose else sp.m
        Xs = [rng.standard_normal((r, kk)) for r, kk in zip(rows_in, k)]
        want = sp.apply_mt(Xs) if transpose else sp.apply_m(Xs)
        xin = torch.from_numpy(np.concatenate([a.ravel() for a in Xs])).cuda()
        tot = sum(r * kk for r, kk in zip(rows_out, k))
        y, _ = ctx.site_apply(dev(Rt), dev(T), dev(A), dev(W), opts, k, xin,
                              transpose=transpose, out_elems=tot)
        y = y[:tot].cpu().numpy()
        p = 0
        for r, kk, w in zip(rows_out, k, want):
            g = y[p:p + r * kk].reshape(r, kk)
            p += r * kk
            if w.size:
                errs.append(normwise(g, w))
    err = max(errs)
    print(f"{name}: mixed chain norm-wise rel err {err:.2e}")
    assert err < MIXED_TOL
    assert err > 1e-13   # FP32 storage in use


ROWS = [
    ("none", dict(kind="none", L=4, d=2, D=3, w=2, chi=9), 12),
    ("u1u1", dict(kind="u1u1", L=4, env_scale=2, virt_scale=2), 14),
    ("su2", dict(kind="su2", L=4, env_scale=3, virt_scale=2), 10),
]


@pytest.mark.parametrize("name,kw,chi", ROWS, ids=[r[0] for r in ROWS])
def test_absorb_row_mixed_matches_oracle(ctx, name, kw, chi):
    """a1-a8 in mixed precision: one row absorbed with rSVD truncation. The
    network value against a fixed random bottom environment and the
    log-norm within max(1e-6, u / g) of the FP64 oracle; singular values
    norm-wise within 1e-6 per site."""
    from oracle.zipup import absorb_row
    from oracle.expect import overlap
    from paper_2511_01039_amd import opts_for
    row = wl.small_row(seed=3, oversample=4, power_iters=1, **kw)
    env, lg, info = absorb_row(row.sym, row.T, row.A, row.W, chi, 4, 1, 17, row=row.row)
    out, glg, rep = ctx.env_absorb(devs(row.T), devs(row.A), devs(row.W),
                                   opts_for(row.sym, chi=chi, oversample=4, power_iters=1, seed=17,
                                            row=row.row, precision="fp32"))
    for x in range(len(env) - 1):
        sig, sec, kept = ctx.absorb_diag(x)
        want = np.concatenate([np.asarray(s) for s in info["sigma"][x]])
        assert normwise(sig, want) < MIXED_TOL
    bot = wl.random_bottom_env(row.sym, env, row.meta["cat"]["env"], np.random.default_rng(5))
    v_or = overlap(env, bot) * math.exp(lg)
    v_gpu = ctx.expect(out, devs(bot)) * math.exp(glg)
    rel = abs(v_gpu - v_or) / abs(v_or)
    tol = gap_tol(info)
    print(f"{name}: mixed s_row oracle {v_or:.15e} gpu {v_gpu:.15e} rel {rel:.2e} "
          f"log_norm diff {abs(glg - lg):.2e} gap {rep['min_rel_gap']:.2e} bound {tol:.2e}")
    assert abs(glg - lg) < tol * max(1.0, abs(lg))
    assert rel < tol
    assert rel > 1e-15   # FP32 storage in use


def test_config1_network_value_mixed(ctx):
    """Config 1 (4x4, chi = 32, p = 8, q = 1): <W> = Z_W / Z_1 in mixed
    precision within 1e-6 of the FP64 oracle."""
    from oracle.expect import network_value, ratio, closing_env
    from paper_2511_01039_amd import opts_for
    lat = wl.config1_lattice()
    prm = wl.config1_params()
    ident = wl.identity_pepo(lat.sym, 4, 4, lat.A[0][0].legs[0])

    def gpu_value(W):
        env = devs(wl.trivial_env(lat.sym, 4))
        lg = 0.0
        for y in range(4):
            env, lg, _ = ctx.env_absorb(env, devs(lat.A[y]), devs(W[y]),
                                        opts_for(lat.sym, chi=prm["chi"], oversample=prm["oversample"],
                                                 power_iters=prm["power_iters"], seed=prm["seed"],
                                                 row=y, precision="fp32"),
                                        log_norm=lg)
        v = ctx.expect(env, devs(closing_env([t.to_host() for t in env])))
        return (1 if v > 0 else -1), lg + math.log(abs(v))

    got = ratio(gpu_value(lat.W), gpu_value(ident))
    ow = network_value(lat.sym, lat.A, lat.W, prm["chi"], prm["oversample"], prm["power_iters"],
                       prm["seed"])
    o1 = network_value(lat.sym, lat.A, ident, prm["chi"], prm["oversample"], prm["power_iters"],
                       prm["seed"])
    want = ratio(ow[:2], o1[:2])
    tol = gap_tol(ow[2], o1[2])
    rel = abs(got - want) / abs(want)
    print(f"config1 mixed <W>: oracle {want:.15e} gpu {got:.15e} rel {rel:.2e} bound {tol:.2e}")
    assert rel < tol


def test_su2_lattice_network_value_mixed(ctx):
    """The 3x3 SU(2)-synthetic lattice of the FP64 test in mixed precision:
    <W> within 1e-6 of the FP64 oracle."""
    from oracle.expect import network_value, ratio
    from test_gpu_parity import lattice_value
    lat = wl.su2_lattice(3, 3, wl.legs_su2_mini(env_scale=2, virt_scale=1), seed=4)
    ident = wl.identity_pepo(lat.sym, 3, 3, lat.A[0][0].legs[0])
    got = ratio(lattice_value(ctx, lat, lat.W, 12, 4, 1, 7, "fp32"),
                lattice_value(ctx, lat, ident, 12, 4, 1, 7, "fp32"))
    ow = network_value(lat.sym, lat.A, lat.W, 12, 4, 1, 7)
    o1 = network_value(lat.sym, lat.A, ident, 12, 4, 1, 7)
    want = ratio(ow[:2], o1[:2])
    tol = gap_tol(ow[2], o1[2])
    rel = abs(got - want) / abs(want)
    print(f"su2 3x3 mixed <W>: oracle {want:.15e} gpu {got:.15e} rel {rel:.2e} bound {tol:.2e}")
    assert rel < tol
