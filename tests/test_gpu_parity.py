"""Parity of the gfx950 library with the FP64 oracle (needs a GPU).

Every case runs the device path through the C ABI and the oracle on the same
seeded inputs; comparisons are element by element where the output is unique
(chain products, singular values, network values) and through gauge-
invariant quantities where it is not (isometries: projectors and overlaps).
"""
import math

import numpy as np
import pytest

import workloads as wl
from workloads.tensor import Leg, Tensor

pytestmark = pytest.mark.gpu


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


def remainder_tensor(sym, row, x, cat_c, rng):
    T, A, W = row.T[x], row.A[x], row.W[x]
    legs = [cat_c, T.legs[0].flipped(), A.legs[1].flipped(), W.legs[2].flipped(), A.legs[1]]
    legs = [Leg(l.labels, l.dims, d) for l, d in zip(legs, (1, -1, -1, -1, 1))]
    return wl.random_tensor(sym, legs, rng)


def rel_err(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


CASES = [
    ("none", dict(kind="none", L=3, d=2, D=3, w=2, chi=9)),
    ("u1u1", dict(kind="u1u1", L=3, env_scale=3, virt_scale=2)),
    ("su2", dict(kind="su2", L=3, env_scale=4, virt_scale=2)),
]


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_site_chain_matches_oracle(ctx, name, kw):
    """a3: Y = M_x X and Z = M_x^T Y' element by element, several tiles and
    ragged tails per block (widths 1, 5, 37)."""
    import torch
    from oracle.blocks import BT
    from oracle.chain import SiteOperator
    from oracle.zipup import SiteProblem
    from paper_2511_01039_amd import opts_for
    row = wl.small_row(seed=5, **kw)
    rng = np.random.default_rng(11)
    x = 1
    Rt = remainder_tensor(row.sym, row, x, row.meta["cat"]["env"], rng)
    names = ["c", "a", "lk", "lw", "lb"]
    R = BT(names, dict(zip(names, Rt.legs)), Rt.to_dict())
    sp = SiteProblem(SiteOperator(row.sym, R, row.T[x], row.A[x], row.W[x]))
    opts = opts_for(row.sym)
    lab, m, n = ctx.site_shape(dev(Rt), dev(row.T[x]), dev(row.A[x]), dev(row.W[x]), opts)
    assert [tuple(l) for l in lab] == [tuple(np.atleast_1d(J)) for J, _ in sp.sect]
    assert list(m) == sp.m and list(n) == sp.n
    widths = [1, 5, 37]
    k = [widths[i % 3] for i in range(len(sp.sect))]
    X = [rng.standard_normal((nn, kk)) for nn, kk in zip(sp.n, k)]
    want = sp.apply_m(X)
    xin = torch.from_numpy(np.concatenate([a.ravel() for a in X])).cuda()
    tot = sum(mm * kk for mm, kk in zip(sp.m, k))
    y, rep = ctx.site_apply(dev(Rt), dev(row.T[x]), dev(row.A[x]), dev(row.W[x]), opts, k, xin,
                            transpose=False, out_elems=tot)
    y = y[:tot].cpu().numpy()
    got, p = [], 0
    for mm, kk in zip(sp.m, k):
        got.append(y[p:p + mm * kk].reshape(mm, kk))
        p += mm * kk
    err = max(rel_err(g, w) for g, w in zip(got, want) if w.size)
    print(f"{name}: sectors {len(sp.sect)} m {sum(sp.m)} n {sum(sp.n)} fwd rel err {err:.2e} "
          f"flops {rep['alg_flops']:.3e}")
    assert err < 1e-12
    # transpose
    Z = [rng.standard_normal((mm, kk)) for mm, kk in zip(sp.m, k)]
    want_t = sp.apply_mt(Z)
    zin = torch.from_numpy(np.concatenate([a.ravel() for a in Z])).cuda()
    tot_t = sum(nn * kk for nn, kk in zip(sp.n, k))
    yt, _ = ctx.site_apply(dev(Rt), dev(row.T[x]), dev(row.A[x]), dev(row.W[x]), opts, k, zin,
                           transpose=True, out_elems=tot_t)
    yt = yt[:tot_t].cpu().numpy()
    got_t, p = [], 0
    for nn, kk in zip(sp.n, k):
        got_t.append(yt[p:p + nn * kk].reshape(nn, kk))
        p += nn * kk
    err_t = max(rel_err(g, w) for g, w in zip(got_t, want_t) if w.size)
    print(f"{name}: bwd rel err {err_t:.2e}")
    assert err_t < 1e-12


def test_site_chain_slicing_is_invariant(ctx):
    """Peak-memory slicing (budget forcing one slice per sector and column
    splits) gives the same products bit for bit."""
    import torch
    from paper_2511_01039_amd import opts_for
    row = wl.small_row("u1u1", L=3, seed=2, env_scale=3, virt_scale=2)
    rng = np.random.default_rng(1)
    Rt = remainder_tensor(row.sym, row, 1, row.meta["cat"]["env"], rng)
    o = opts_for(row.sym)
    lab, m, n = ctx.site_shape(dev(Rt), dev(row.T[1]), dev(row.A[1]), dev(row.W[1]), o)
    k = [7] * len(m)
    X = torch.from_numpy(rng.standard_normal(int(sum(n)) * 7)).cuda()
    tot = int(sum(m)) * 7
    y0, r0 = ctx.site_apply(dev(Rt), dev(row.T[1]), dev(row.A[1]), dev(row.W[1]), o, k, X,
                            out_elems=tot)
    o2 = opts_for(row.sym, slice_budget=20000)
    y1, r1 = ctx.site_apply(dev(Rt), dev(row.T[1]), dev(row.A[1]), dev(row.W[1]), o2, k, X,
                            out_elems=tot)
    print("slices", r0["nslices"], r1["nslices"], "peak", r0["peak_workspace"], r1["peak_workspace"])
    assert r1["nslices"] > r0["nslices"]
    assert r1["peak_workspace"] < r0["peak_workspace"]
    assert torch.equal(y0[:tot], y1[:tot])


def test_streams_match_one_stream(ctx):
    """Slices are spread round-robin over four streams by default; with at
    least five slices (so that one stream takes two), the products are the
    same bit for bit as with every slice on one stream, forward and
    transposed."""
    import torch
    from paper_2511_01039_amd import opts_for
    from paper_2511_01039_amd.binding import FLAG_ONE_STREAM
    row = wl.small_row("u1u1", L=3, seed=2, env_scale=3, virt_scale=2)
    rng = np.random.default_rng(3)
    Rt = remainder_tensor(row.sym, row, 1, row.meta["cat"]["env"], rng)
    o = opts_for(row.sym)
    lab, m, n = ctx.site_shape(dev(Rt), dev(row.T[1]), dev(row.A[1]), dev(row.W[1]), o)
    k = [5] * len(m)
    X0 = torch.from_numpy(rng.standard_normal(int(sum(n)) * 5)).cuda()
    tot0 = int(sum(m)) * 5
    # the largest of these budgets that gives at least five slices
    for budget in (20000, 8000, 3000, 1200):
        _, r = ctx.site_apply(dev(Rt), dev(row.T[1]), dev(row.A[1]), dev(row.W[1]),
                              opts_for(row.sym, slice_budget=budget), k, X0, out_elems=tot0)
        if r["nslices"] >= 5:
            break
    print("budget", budget, "slices", r["nslices"])
    assert r["nslices"] >= 5
    for transpose in (False, True):
        rows_in, rows_out = (m, n) if transpose else (n, m)
        X = torch.from_numpy(rng.standard_normal(int(sum(rows_in)) * 5)).cuda()
        tot = int(sum(rows_out)) * 5
        ys = []
        for flags in (0, FLAG_ONE_STREAM):
            o2 = opts_for(row.sym, slice_budget=budget, flags=flags)
            y, r = ctx.site_apply(dev(Rt), dev(row.T[1]), dev(row.A[1]), dev(row.W[1]), o2, k, X,
                                  transpose=transpose, out_elems=tot)
            assert r["nslices"] >= 5
            ys.append(y[:tot].clone())
        assert torch.equal(ys[0], ys[1])


def prescribed(m, n, sig, seed):
    rng = np.random.default_rng(seed)
    r = len(sig)
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return U @ np.diag(sig) @ V.T


def test_rsvd_truncate_matches_oracle(ctx):
    """a4-a6 on explicit matrices: same sketch, same kept counts, singular
    values and projectors as the oracle; truncation across the batch."""
    import torch
    from oracle.rsvd import rsvd_explicit
    from paper_2511_01039_amd import make_opts
    rng = np.random.default_rng(0)
    mats = [prescribed(300, 250, 1.0 / (1 + np.arange(120)) ** 0.7, 1),
            rng.standard_normal((70, 190)), rng.standard_normal((33, 33)),
            prescribed(129, 65, np.linspace(2, 1, 40), 4)]
    for q in (0, 2):
        want = rsvd_explicit(mats, chi=60, p=7, q=q, seed=42, tag=3)
        U, R, sig, kept, rep = ctx.rsvd_truncate([torch.from_numpy(a).cuda() for a in mats],
                                                 make_opts(chi=60, oversample=7, power_iters=q,
                                                           seed=42, tag=3))
        assert list(kept) == list(want["kept"])
        for i in range(len(mats)):
            if kept[i] == 0:
                continue
            e = rel_err(sig[i], want["sigma"][i])
            u = U[i].cpu().numpy()
            pe = np.abs(u @ u.T - want["U"][i] @ want["U"][i].T).max()
            ur = u @ R[i].cpu().numpy()
            re = rel_err(ur, want["U"][i] @ want["R"][i])
            ue = rel_err(u, want["U"][i])
            print(f"q={q} mat {i}: kept {kept[i]} sigma err {e:.2e} proj err {pe:.2e} UR err {re:.2e} U err {ue:.2e}")
            assert e < 1e-11 and pe < 1e-10 and re < 1e-10
            assert ue < 1e-9   # same canonical column signs


def test_cbe_expand_matches_oracle(ctx):
    """a7 on explicit matrices: the truncated complement equals the oracle's
    (split projectors) and is orthogonal to the kept space."""
    import torch
    from oracle.cbe import cbe_explicit
    from paper_2511_01039_amd import make_opts
    rng = np.random.default_rng(7)
    mats, U, V = [], [], []
    for (m, n, r) in [(140, 120, 12), (66, 200, 8), (30, 29, 5)]:
        mats.append(rng.standard_normal((m, n)))
        U.append(np.linalg.qr(rng.standard_normal((m, r)))[0])
        V.append(np.linalg.qr(rng.standard_normal((n, r)))[0].T)
    want = cbe_explicit(mats, U, V, chi_extra=20, p=6, seed=9, tag=2)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    Q, sig, kept, rep = ctx.cbe_expand([t(a) for a in mats], [t(u) for u in U], [t(v) for v in V],
                                       make_opts(cbe_extra=20, oversample=6, seed=9, tag=2))
    assert list(kept) == list(want["kept"])
    for i in range(3):
        if kept[i] == 0:
            continue
        q = Q[i].cpu().numpy()
        assert np.abs(q.T @ U[i]).max() < 1e-12
        assert np.abs(q.T @ q - np.eye(q.shape[1])).max() < 1e-12
        pe = np.abs(q @ q.T - want["Q"][i] @ want["Q"][i].T).max()
        print(f"cbe mat {i}: kept {kept[i]} proj err {pe:.2e} sigma err {rel_err(sig[i], want['sigma'][i]):.2e}"
              f" Q err {rel_err(q, want['Q'][i]):.2e}")
        assert pe < 1e-10
        assert rel_err(q, want["Q"][i]) < 1e-9
        assert rel_err(sig[i], want["sigma"][i]) < 1e-11


ROWS = [
    ("none", dict(kind="none", L=4, d=2, D=3, w=2, chi=9), 12),
    ("u1u1", dict(kind="u1u1", L=4, env_scale=2, virt_scale=2), 14),
    ("su2", dict(kind="su2", L=4, env_scale=3, virt_scale=2), 10),
]


@pytest.mark.parametrize("name,kw,chi", ROWS, ids=[r[0] for r in ROWS])
def test_absorb_row_matches_oracle(ctx, name, kw, chi):
    """a1-a6 + a8: one row absorbed with rSVD truncation. Kept counts and
    singular values per site, the log-norm, and the network value against a
    fixed random bottom environment (gauge invariant) agree with the oracle."""
    from oracle.zipup import absorb_row
    from oracle.expect import overlap
    from paper_2511_01039_amd import opts_for
    row = wl.small_row(seed=3, oversample=4, power_iters=1, **kw)
    env, lg, info = absorb_row(row.sym, row.T, row.A, row.W, chi, 4, 1, 17, row=row.row)
    out, glg, rep = ctx.env_absorb(devs(row.T), devs(row.A), devs(row.W),
                                   opts_for(row.sym, chi=chi, oversample=4, power_iters=1, seed=17,
                                            row=row.row))
    for x in range(len(env) - 1):
        sig, sec, kept = ctx.absorb_diag(x)
        assert list(kept) == list(info["kept"][x]), (x, kept, info["kept"][x])
        want = np.concatenate([np.asarray(s) for s in info["sigma"][x]])
        assert rel_err(sig, want) < 1e-11
    bot = wl.random_bottom_env(row.sym, env, row.meta["cat"]["env"], np.random.default_rng(5))
    v_or = overlap(env, bot) * math.exp(lg)
    gpu_host = [t.to_host() for t in out]
    v_mix = overlap(gpu_host, bot) * math.exp(glg)
    v_gpu = ctx.expect(out, devs(bot)) * math.exp(glg)
    print(f"{name}: log_norm {lg:.12f} / {glg:.12f}  s_row oracle {v_or:.15e} gpu {v_gpu:.15e} "
          f"rel {abs(v_gpu - v_or) / abs(v_or):.2e}  flops {rep['alg_flops']:.3e} gap {rep['min_rel_gap']:.2e}")
    assert abs(glg - lg) < 1e-11 * max(1.0, abs(lg))
    assert abs(v_mix - v_or) < 1e-11 * abs(v_or)
    assert abs(v_gpu - v_or) < 1e-11 * abs(v_or)


def test_absorb_row_reuses_plans(ctx):
    """A dense 6-site row whose interior sites share their block structure
    (12 kept at every site): sites after the first interior one reuse the
    previous site's analysis and plans with their own layer data. Kept
    counts, singular values, log-norm and s_row still agree with the oracle."""
    from oracle.zipup import absorb_row
    from oracle.expect import overlap
    from paper_2511_01039_amd import opts_for
    row = wl.small_row(seed=3, oversample=4, power_iters=1, kind="none", L=6, d=2, D=3, w=2,
                       chi=9)
    env, lg, info = absorb_row(row.sym, row.T, row.A, row.W, 12, 4, 1, 17, row=row.row)
    out, glg, rep = ctx.env_absorb(devs(row.T), devs(row.A), devs(row.W),
                                   opts_for(row.sym, chi=12, oversample=4, power_iters=1, seed=17,
                                            row=row.row))
    print(f"plan reuses {rep['plan_reuses']}")
    assert rep["plan_reuses"] >= 2
    for x in range(len(env) - 1):
        sig, sec, kept = ctx.absorb_diag(x)
        assert list(kept) == list(info["kept"][x]), (x, kept, info["kept"][x])
        want = np.concatenate([np.asarray(s) for s in info["sigma"][x]])
        assert rel_err(sig, want) < 1e-11
    bot = wl.random_bottom_env(row.sym, env, row.meta["cat"]["env"], np.random.default_rng(5))
    v_or = overlap(env, bot) * math.exp(lg)
    v_gpu = ctx.expect(out, devs(bot)) * math.exp(glg)
    assert abs(glg - lg) < 1e-11 * max(1.0, abs(lg))
    assert abs(v_gpu - v_or) < 1e-11 * abs(v_or)


def test_config1_network_value(ctx):
    """Config 1: 4x4 dense lattice, <W> = Z_W / Z_1 top to bottom with chi = 32,
    rSVD (p = 8, q = 1): FP64 device path vs the oracle within 1e-11."""
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
                                                 power_iters=prm["power_iters"], seed=prm["seed"], row=y),
                                        log_norm=lg)
        v = ctx.expect(env, devs(closing_env([t.to_host() for t in env])))
        return (1 if v > 0 else -1), lg + math.log(abs(v))

    gw, g1 = gpu_value(lat.W), gpu_value(ident)
    ow = network_value(lat.sym, lat.A, lat.W, prm["chi"], prm["oversample"], prm["power_iters"], prm["seed"])
    o1 = network_value(lat.sym, lat.A, ident, prm["chi"], prm["oversample"], prm["power_iters"], prm["seed"])
    got, want = ratio(gw, g1), ratio(ow, o1)
    print(f"config1 <W>: oracle {want:.15e} gpu {got:.15e} rel {abs(got - want) / abs(want):.2e}")
    assert abs(got - want) < 1e-11 * abs(want)


FULL = [
    # (config, precision, tolerance): FP64 element by element, mixed norm-wise
    (4, "fp64", 1e-12), (4, "fp32", 1e-6),
    (2, "fp64", 1e-12), (2, "fp32", 1e-6),
]


@pytest.mark.parametrize("cfg,precision,tol", FULL,
                         ids=[f"config{c}-{p}" for c, p, _ in FULL])
def test_site_chain_full_size(ctx, cfg, precision, tol):
    """a3 at the full size of the benchmark workloads: the interior site x = 1
    of the 8x8 SU(2)-synthetic chi = 500 row (config 4: 12 sectors,
    432000 x 155348) and of the dense Hubbard-comb chi = 128 row (config 2),
    with a random remainder of the row's structure and one or two sketch
    columns per sector (so that the oracle finishes in seconds). M_x X and
    M_x^T Y against the oracle, element by element in FP64 and norm-wise per
    sector in mixed precision."""
    import torch
    from oracle.blocks import BT
    from oracle.chain import SiteOperator
    from oracle.zipup import SiteProblem
    from paper_2511_01039_amd import opts_for
    if cfg == 4:
        row, env = wl.config4_row(), wl.legs_su2(500)["env"]
    else:
        row, env = wl.config2_row(), wl.legs_dense(4, 6, 6, 128)["env"]
    rng = np.random.default_rng(21)
    x = 1
    T, A, W = row.T[x], row.A[x], row.W[x]
    Rt = remainder_tensor(row.sym, row, x, env, rng)
    names = ["c", "a", "lk", "lw", "lb"]
    sp = SiteProblem(SiteOperator(row.sym, BT(names, dict(zip(names, Rt.legs)), Rt.to_dict()),
                                  T, A, W))
    if cfg == 4:
        assert len(sp.sect) == 12 and sum(sp.m) == 432000 and sum(sp.n) == 155348
    opts = opts_for(row.sym, precision=precision)
    k = [1 + (i % 2) for i in range(len(sp.sect))]
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
        p, errs = 0, []
        for r, kk, w in zip(rows_out, k, want):
            g = y[p:p + r * kk].reshape(r, kk)
            p += r * kk
            if w.size:
                errs.append(rel_err(g, w) if precision == "fp64" else
                            float(np.linalg.norm(g - w) / np.linalg.norm(w)))
        print(f"config{cfg} site chain {precision} {'bwd' if transpose else 'fwd'}: "
              f"sectors {len(sp.sect)} m {sum(sp.m)} n {sum(sp.n)} max rel err {max(errs):.2e}")
        assert max(errs) < tol


def test_config5_bond_expansion_site_matches_oracle(ctx):
    """a7 at the sizes of the bond-expansion workload (config 5): the largest
    sector matrices of interior site 1 of the U(1)xU(1) chi = 256 row (shapes
    from the site operator), seeded explicit matrices of decaying spectrum;
    one rSVD truncation over the sectors (chi = 256, p = 8, q = 1) and one
    bond expansion by 26 directions (p = 8, q = 0) against the oracle: kept
    counts, singular values, projectors; Q orthogonal to U and orthonormal."""
    import torch
    from oracle.blocks import BT
    from oracle.chain import SiteOperator
    from oracle.zipup import SiteProblem
    from oracle.rsvd import rsvd_explicit
    from oracle.cbe import cbe_explicit
    from paper_2511_01039_amd import make_opts
    cfg = wl.CONFIG5
    row = wl.config3_row()
    rng = np.random.default_rng(3)
    x = 1
    Rt = remainder_tensor(row.sym, row, x, wl.legs_u1u1(256)["env"], rng)
    names = ["c", "a", "lk", "lw", "lb"]
    sp = SiteOperator(row.sym, BT(names, dict(zip(names, Rt.legs)), Rt.to_dict()),
                      row.T[x], row.A[x], row.W[x])
    prob = SiteProblem(sp)
    shapes = sorted(zip(prob.m, prob.n), key=lambda t: -min(t))[:6]
    assert min(shapes[0]) >= 500
    mats = [wl.decaying_matrix(m, n, rng, cfg["decay"]) for m, n in shapes]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    want = rsvd_explicit(mats, chi=cfg["chi"], p=cfg["oversample"], q=cfg["power_iters"],
                         seed=0, tag=0)
    U, R, sig, kept, _ = ctx.rsvd_truncate([t(a) for a in mats],
                                           make_opts(chi=cfg["chi"], oversample=cfg["oversample"],
                                                     power_iters=cfg["power_iters"], seed=0, tag=0))
    assert list(kept) == list(want["kept"])
    Uh, Vh = [], []
    for i in range(len(mats)):
        u = U[i].cpu().numpy()
        assert rel_err(sig[i], want["sigma"][i]) < 1e-11
        assert np.abs(u @ u.T - want["U"][i] @ want["U"][i].T).max() < 1e-10
        Uh.append(want["U"][i])
        Vh.append(want["R"][i] / np.asarray(want["sigma"][i])[:, None])
    cw = cbe_explicit(mats, Uh, Vh, chi_extra=cfg["cbe_extra"], p=cfg["cbe_oversample"], seed=0,
                      tag=1)
    Q, csig, ckept, _ = ctx.cbe_expand([t(a) for a in mats], [t(u) for u in Uh],
                                       [t(v) for v in Vh],
                                       make_opts(cbe_extra=cfg["cbe_extra"],
                                                 oversample=cfg["cbe_oversample"], seed=0, tag=1))
    assert list(ckept) == list(cw["kept"])
    for i in range(len(mats)):
        if ckept[i] == 0:
            continue
        q = Q[i].cpu().numpy()
        assert np.abs(q.T @ Uh[i]).max() < 1e-12
        assert np.abs(q.T @ q - np.eye(q.shape[1])).max() < 1e-12
        assert np.abs(q @ q.T - cw["Q"][i] @ cw["Q"][i].T).max() < 1e-10
        assert rel_err(csig[i], cw["sigma"][i]) < 1e-11
    print(f"config5 site: shapes {shapes} kept {list(kept)} cbe kept {list(ckept)}")


def test_grouped_truncations_match_oracle_per_group(ctx):
    """a9: several independent truncation problems (the per-site truncations
    of a row) in one grouped call. Each group has its own widths and cut and
    the sketch counters of its own call (tag + group), so every group agrees
    with the oracle run on that group alone: kept counts, singular values and
    projectors; then the grouped bond expansion likewise."""
    import torch
    from oracle.rsvd import rsvd_explicit
    from oracle.cbe import cbe_explicit
    from paper_2511_01039_amd import make_opts
    rng = np.random.default_rng(11)
    shapes = [[(300, 250), (120, 200), (80, 80)], [(400, 150), (60, 90)], [(200, 220)]]
    mats, group = [], []
    for g, sh in enumerate(shapes):
        for m, n in sh:
            mats.append(wl.decaying_matrix(m, n, rng, 20.0))
            group.append(g)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    chi, p, q = 40, 8, 1
    U, R, sig, kept, rep = ctx.rsvd_truncate([t(a) for a in mats],
                                             make_opts(chi=chi, oversample=p, power_iters=q,
                                                       seed=0, tag=5), group=group)
    Uh, Vh = [None] * len(mats), [None] * len(mats)
    for g in range(len(shapes)):
        idx = [i for i in range(len(mats)) if group[i] == g]
        want = rsvd_explicit([mats[i] for i in idx], chi=chi, p=p, q=q, seed=0, tag=5 + g)
        assert [int(kept[i]) for i in idx] == list(want["kept"]), g
        assert sum(int(kept[i]) for i in idx) <= chi
        for j, i in enumerate(idx):
            u = U[i].cpu().numpy()
            assert rel_err(sig[i], want["sigma"][j]) < 1e-11
            assert np.abs(u @ u.T - want["U"][j] @ want["U"][j].T).max() < 1e-10
            Uh[i] = want["U"][j]
            Vh[i] = want["R"][j] / np.asarray(want["sigma"][j])[:, None]
    Q, csig, ckept, _ = ctx.cbe_expand([t(a) for a in mats], [t(u) for u in Uh],
                                       [t(v) for v in Vh],
                                       make_opts(cbe_extra=6, oversample=4, seed=0, tag=7),
                                       group=group)
    for g in range(len(shapes)):
        idx = [i for i in range(len(mats)) if group[i] == g]
        cw = cbe_explicit([mats[i] for i in idx], [Uh[i] for i in idx], [Vh[i] for i in idx],
                          chi_extra=6, p=4, seed=0, tag=7 + g)
        assert [int(ckept[i]) for i in idx] == list(cw["kept"]), g
        for j, i in enumerate(idx):
            if ckept[i] == 0:
                continue
            qq = Q[i].cpu().numpy()
            assert np.abs(qq.T @ Uh[i]).max() < 1e-12
            assert np.abs(qq @ qq.T - cw["Q"][j] @ cw["Q"][j].T).max() < 1e-10
            assert rel_err(csig[i], cw["sigma"][j]) < 1e-11
    print(f"grouped: kept {list(kept)} cbe kept {list(ckept)}")
    # one group holding every matrix is the ungrouped call, bit for bit; an
    # empty group id in between changes nothing for the others
    sub = [t(a) for a in mats[:3]]
    o = make_opts(chi=chi, oversample=p, power_iters=q, seed=0, tag=5)
    U0, _, _, k0, _ = ctx.rsvd_truncate(sub, o)
    U1, _, _, k1, _ = ctx.rsvd_truncate(sub, o, group=[0, 0, 0])
    assert list(k0) == list(k1)
    for a, b in zip(U0, U1):
        assert torch.equal(a, b)
    U2, _, _, k2, _ = ctx.rsvd_truncate(sub, o, group=[0, 2, 2])
    want0 = rsvd_explicit(mats[:1], chi=chi, p=p, q=q, seed=0, tag=5)
    want2 = rsvd_explicit(mats[1:3], chi=chi, p=p, q=q, seed=0, tag=7)
    assert [int(v) for v in k2] == list(want0["kept"]) + list(want2["kept"])


def lattice_value(ctx, lat, W, chi, p, q, seed, precision="fp64"):
    """<top|closing> after absorbing every row top to bottom on the device:
    (sign, log |Z|)."""
    from oracle.expect import closing_env
    from paper_2511_01039_amd import opts_for
    Ly, Lx = len(lat.A), len(lat.A[0])
    env = devs(wl.trivial_env(lat.sym, Lx))
    lg = 0.0
    for y in range(Ly):
        env, lg, _ = ctx.env_absorb(env, devs(lat.A[y]), devs(W[y]),
                                    opts_for(lat.sym, chi=chi, oversample=p, power_iters=q,
                                             seed=seed, row=y, precision=precision),
                                    log_norm=lg)
    v = ctx.expect(env, devs(closing_env([t.to_host() for t in env])))
    return (1 if v > 0 else -1), lg + math.log(abs(v))


def test_su2_lattice_network_value(ctx):
    """a1-a8 on a whole SU(2)-synthetic lattice (3x3, fermionic signs, random
    PEPO): <W> = Z_W / Z_1 top to bottom with chi = 12, rSVD p = 4, q = 1,
    FP64 device path vs the oracle within 1e-11."""
    from oracle.expect import network_value, ratio
    lat = wl.su2_lattice(3, 3, wl.legs_su2_mini(env_scale=2, virt_scale=1), seed=4)
    ident = wl.identity_pepo(lat.sym, 3, 3, lat.A[0][0].legs[0])
    got = ratio(lattice_value(ctx, lat, lat.W, 12, 4, 1, 7), lattice_value(ctx, lat, ident, 12, 4, 1, 7))
    want = ratio(network_value(lat.sym, lat.A, lat.W, 12, 4, 1, 7)[:2],
                 network_value(lat.sym, lat.A, ident, 12, 4, 1, 7)[:2])
    print(f"su2 3x3 <W>: oracle {want:.15e} gpu {got:.15e} rel {abs(got - want) / abs(want):.2e}")
    assert abs(got - want) < 1e-11 * abs(want)
