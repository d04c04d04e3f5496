"""The boundary's context services on the device (needs a GPU): the
workspace allocator hook and the network value as (sign, log |Z|)."""
import math

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def dev(ts):
    from paper_2511_01039_amd import DeviceTensor
    return [DeviceTensor.from_host(t) for t in ts]


def test_torch_allocator_gives_the_same_row_bit_for_bit():
    """A context whose workspace comes from PyTorch's caching allocator
    absorbs a row to the same bits as one using hipMalloc, and its workspace
    is memory PyTorch accounts for; a new allocator first returns the old
    workspace."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01039_amd import Context, opts_for
    row = wl.small_row("su2", L=4, seed=3, oversample=4, power_iters=1, env_scale=3, virt_scale=2)
    o = opts_for(row.sym, chi=10, oversample=4, power_iters=1, seed=17, row=row.row)
    outs = []
    for use_torch in (False, True):
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        ctx = Context(0, torch_allocator=use_torch)
        out, lg, rep = ctx.env_absorb(dev(row.T), dev(row.A), dev(row.W), o)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated() - before
        print(f"torch allocator {use_torch}: workspace {rep['workspace_bytes']:.0f} B, "
              f"torch-accounted growth {held} B")
        if use_torch:
            assert held >= rep["workspace_bytes"] > 0
            ctx.use_hip_allocator()          # gives the workspace back to torch
            torch.cuda.synchronize()
            assert torch.cuda.memory_allocated() - before < held
        outs.append(([t.data[:t.nelem].clone() for t in out], lg))
        ctx.close()
    for a, b in zip(outs[0][0], outs[1][0]):
        assert torch.equal(a, b)
    assert outs[0][1] == outs[1][1]


def test_expect_returns_sign_and_log_of_large_values():
    """fpeps_expect adds the two log-norms and returns (sign, log |Z|); a
    value whose magnitude is outside the range of a double (log-norms of
    +-800) still comes back exactly, and its scaled value equals the plain
    overlap."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01039_amd import Context, opts_for
    from oracle.zipup import absorb_row
    from oracle.expect import overlap
    row = wl.small_row("u1u1", L=4, seed=3, oversample=4, power_iters=1, env_scale=2, virt_scale=2)
    env, lg, _ = absorb_row(row.sym, row.T, row.A, row.W, 14, 4, 1, 17, row=row.row)
    bot = wl.random_bottom_env(row.sym, env, row.meta["cat"]["env"], np.random.default_rng(5))
    v = overlap(env, bot)
    ctx = Context(0)
    for ln_t, ln_b in ((0.0, 0.0), (800.0, 700.0), (-900.0, 20.0)):
        sg, la = ctx.expect_log(dev(env), dev(bot), ln_t, ln_b)
        assert sg == (1 if v > 0 else -1)
        assert abs(la - (math.log(abs(v)) + ln_t + ln_b)) < 1e-12 * max(1.0, abs(la))
    ctx.close()
