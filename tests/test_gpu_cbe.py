"""Bond expansion inside the row absorption against the oracle (needs a
GPU): every truncated site of the row is expanded by the most weighty
directions of (1 - U U^T) M_x (1 - V^T V) on the implicit operator (Sec. 4,
Figs. 3-5); the new environment is [U | Q] and the remainder [U | Q]^T M_x.
Compared: the bond of every site (truncation plus expansion per sector),
the log-norm, the network value against a fixed random bottom environment
(gauge invariant), the flop count, and the isometry of every site."""
import math

import numpy as np
import pytest

import workloads as wl

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


def dev(ts):
    from paper_2511_01039_amd import DeviceTensor
    return [DeviceTensor.from_host(t) for t in ts]


ROWS = [
    ("none", dict(kind="none", L=4, d=2, D=3, w=2, chi=9), 8, 3),
    ("u1u1", dict(kind="u1u1", L=4, env_scale=2, virt_scale=2), 10, 4),
    ("su2", dict(kind="su2", L=4, env_scale=3, virt_scale=2), 6, 3),
]


@pytest.mark.parametrize("name,kw,chi,extra", ROWS, ids=[r[0] for r in ROWS])
def test_absorb_row_with_expansion_matches_oracle(ctx, name, kw, chi, extra):
    from oracle.zipup import absorb_row
    from oracle.expect import overlap
    from oracle.flops import row_flops
    from paper_2511_01039_amd import opts_for
    row = wl.small_row(seed=3, oversample=4, power_iters=1, **kw)
    record = []
    env, lg, info = absorb_row(row.sym, row.T, row.A, row.W, chi, 4, 1, 17, row=row.row,
                               record=record, cbe_extra=extra)
    out, glg, rep = ctx.env_absorb(dev(row.T), dev(row.A), dev(row.W),
                                   opts_for(row.sym, chi=chi, oversample=4, power_iters=1,
                                            seed=17, row=row.row, cbe_extra=extra))
    gh = [t.to_host() for t in out]
    for x in range(len(env) - 1):
        assert list(gh[x].legs[4].dims) == list(env[x].legs[4].dims), x
        # isometry of the expanded site over its rows, per sector
        cols = {}
        for key, b in gh[x].to_dict().items():
            cols.setdefault(key[-1], []).append(b.reshape(-1, b.shape[-1]))
        for mats in cols.values():
            U = np.vstack(mats)
            assert np.abs(U.T @ U - np.eye(U.shape[1])).max() < 1e-12
    bot = wl.random_bottom_env(row.sym, env, row.meta["cat"]["env"], np.random.default_rng(5))
    v_or = overlap(env, bot) * math.exp(lg)
    sg, la = ctx.expect_log(out, dev(bot), glg, 0.0)
    v_gpu = sg * math.exp(la)
    want_f = row_flops(record, info, 1)
    print(f"{name}: bonds {[int(t.legs[4].total) for t in gh[:-1]]} log_norm {lg:.12f}/{glg:.12f} "
          f"s_row {v_or:.15e}/{v_gpu:.15e} rel {abs(v_gpu - v_or) / abs(v_or):.2e} "
          f"flops {want_f:.6e}/{rep['alg_flops']:.6e}")
    assert abs(glg - lg) < 1e-11 * max(1.0, abs(lg))
    assert abs(v_gpu - v_or) < 1e-11 * abs(v_or)
    assert rep["alg_flops"] == pytest.approx(want_f, rel=1e-12)
