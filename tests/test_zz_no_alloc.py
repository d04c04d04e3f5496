"""fpeps_expect_noalloc (needs a GPU): the network value computed with every
workspace buffer in the library's static device array equals
fpeps_expect's, bit for bit, on two calls in a row, the second on a smaller
problem (the array keeps the first call's contents); a problem too large for
the array is refused with FPEPS_ERR_CAPACITY."""
import math

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def dev(ts):
    from paper_2511_01039_amd import DeviceTensor
    return [DeviceTensor.from_host(t) for t in ts]


def envs(kind, L, seed, **kw):
    from oracle.zipup import absorb_row
    row = wl.small_row(kind, L=L, seed=seed, oversample=4, power_iters=1, **kw)
    env, lg, _ = absorb_row(row.sym, row.T, row.A, row.W, 10, 4, 1, 17, row=row.row)
    bot = wl.random_bottom_env(row.sym, env, row.meta["cat"]["env"], np.random.default_rng(5))
    return env, bot, lg


def test_noalloc_expect_equals_expect():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01039_amd import Context
    from paper_2511_01039_amd.binding import FpepsError
    import ctypes as C
    from paper_2511_01039_amd.binding import ALLOC_FN, FREE_FN
    ctx = Context(0)
    # every device allocation of the library goes through this hook: count
    # them (the blocks come from torch's caching allocator)
    calls = {"alloc": 0}
    stream = torch.cuda.ExternalStream(ctx.stream, device=0)

    def _alloc(nbytes, user):
        calls["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes), 0, stream)

    def _free(ptr, user):
        torch.cuda.caching_allocator_delete(ptr)

    cbs = (ALLOC_FN(_alloc), FREE_FN(_free))
    ctx.check(ctx.lib.fpeps_set_allocator(ctx.h, cbs[0], cbs[1], None))
    big = envs("su2", 5, 3, env_scale=3, virt_scale=2)
    small = envs("u1u1", 3, 4, env_scale=1, virt_scale=1)
    for env, bot, lg in (big, small):
        top_d, bot_d = dev(env), dev(bot)
        torch.cuda.synchronize()
        before, n0 = torch.cuda.memory_allocated(), calls["alloc"]
        got = ctx.expect_log_noalloc(top_d, bot_d, lg, 0.5)
        torch.cuda.synchronize()
        assert calls["alloc"] == n0 and torch.cuda.memory_allocated() == before
        want = ctx.expect_log(top_d, bot_d, lg, 0.5)
        print(f"noalloc {got} expect {want}; library allocations by fpeps_expect "
              f"{calls['alloc'] - n0}")
        assert got[0] == want[0] and got[1] == want[1]
    # a problem beyond the 64 MiB array: refused with a capacity error
    cat = wl.legs_dense(2, 2, 1, 3000)
    L = 3
    legs = [[wl.configs.with_dirs([cat["bnd"] if x == 0 else cat["env"], cat["virt"], cat["pepo"],
                                   cat["virt"], cat["bnd"] if x == L - 1 else cat["env"]],
                                  wl.ENV_DIRS) for x in range(L)]]
    rng = np.random.default_rng(0)
    top = [wl.random_tensor(wl.Sym(), lg_, rng) for lg_ in legs[0]]
    bot = wl.random_bottom_env(wl.Sym(), top, cat["env"], rng)
    with pytest.raises(FpepsError) as e:
        ctx.expect_log_noalloc(dev(top), dev(bot))
    assert "ERR_CAPACITY" in str(e.value) and "scratch" in str(e.value)
    ctx.close()
    del cbs
