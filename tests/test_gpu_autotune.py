"""Autotuner of the row absorption (fpeps_autotune_absorb): slice budget and
GEMM tiles chosen by measurement, kept in the context and in a text file.

The tuned row must still agree with the FP64 oracle; later absorptions use
the table (bit-identical to the tuned run); a saved table loaded into a
cleared context reproduces them; a table that forces other tiles on every
step still gives oracle parity; a malformed file is refused."""
import math

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

GIB = 1 << 30


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01039_amd import Context
    c = Context(0)
    yield c
    c.close()


def devs(ts):
    from paper_2511_01039_amd import DeviceTensor
    return [DeviceTensor.from_host(t) for t in ts]


def rel_err(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def check_against_oracle(ctx, row, out, glg, env, lg, info):
    from oracle.expect import overlap
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
    return v_gpu


def same(a, b):
    import torch
    return all(x.nelem == y.nelem and torch.equal(x.data[:x.nelem], y.data[:y.nelem])
               for x, y in zip(a, b))


def test_autotuned_row(ctx, tmp_path):
    from oracle.zipup import absorb_row
    from paper_2511_01039_amd import opts_for
    from paper_2511_01039_amd.binding import FpepsError
    row = wl.small_row(seed=3, oversample=4, power_iters=1, kind="su2", L=4, env_scale=3,
                       virt_scale=2)
    chi = 10
    env, lg, info = absorb_row(row.sym, row.T, row.A, row.W, chi, 4, 1, 17, row=row.row)
    opts = opts_for(row.sym, chi=chi, oversample=4, power_iters=1, seed=17, row=row.row)
    T, A, W = devs(row.T), devs(row.A), devs(row.W)
    ctx.tune_clear()
    assert ctx.tune_info() == (-1, 0)
    out, glg, rep = ctx.env_absorb(T, A, W, opts, autotune=3)
    n, budget = ctx.tune_info()
    print(f"tuned signatures {n}, slice budget {budget / GIB:.0f} GiB, "
          f"final run {rep['seconds'] * 1e3:.2f} ms")
    # one of the candidates: 32 GiB, 64 GiB or the default (<= 128 GiB)
    assert n > 0 and (budget in (32 * GIB, 64 * GIB) or 0 < budget <= 128 * GIB)
    check_against_oracle(ctx, row, out, glg, env, lg, info)
    # later absorptions use the table: the same result as the tuned run
    out2, glg2, _ = ctx.env_absorb(T, A, W, opts)
    assert glg2 == glg and same(out, out2)
    # on-disk cache: save, clear, load
    path = str(tmp_path / "tune.txt")
    ctx.tune_save(path)
    ctx.tune_clear()
    with pytest.raises(FpepsError):
        ctx.tune_save(path)          # nothing to save
    commented = tmp_path / "commented.txt"
    commented.write_text("# a tuned table\n" + open(path).read() + "# end\n")
    ctx.tune_load(str(commented))
    assert ctx.tune_info() == (n, budget)
    out3, glg3, _ = ctx.env_absorb(T, A, W, opts)
    assert glg3 == glg and same(out, out3)
    # a malformed file is refused and the table kept
    bad = tmp_path / "bad.txt"
    bad.write_text("fpeps-tune 1\nslice_budget 0\n0123 100 100\n")
    with pytest.raises(FpepsError):
        ctx.tune_load(str(bad))
    assert ctx.tune_info() == (n, budget)
    # every step forced onto another tile shape: still oracle parity
    lines = open(path).read().splitlines()
    forced = [lines[0], lines[1]]
    alt = {(128, 128): (16, 256), (16, 256): (256, 16)}
    for ln in lines[2:]:
        sig, mt, nt = ln.split()
        mt, nt = alt.get((int(mt), int(nt)), (128, 128))
        forced.append(f"{sig} {mt} {nt}")
    fpath = tmp_path / "forced.txt"
    fpath.write_text("\n".join(forced) + "\n")
    ctx.tune_load(str(fpath))
    out4, glg4, _ = ctx.env_absorb(T, A, W, opts)
    check_against_oracle(ctx, row, out4, glg4, env, lg, info)
    ctx.tune_clear()
