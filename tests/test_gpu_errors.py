"""Error paths of the C ABI forced from the host (needs a GPU for the
context): every case is refused by a host-side check, so no kernel meets a
bad buffer. An output too small for the cut returns FPEPS_ERR_CAPACITY with
the required sizes in the report, and a retry with those sizes succeeds; null
arguments return FPEPS_ERR_ARG; a ket whose legs do not match the
environment returns FPEPS_ERR_SHAPE; a prepared effective operator refuses a
vector of the wrong size. The context stays usable after every error."""
import ctypes as C

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

ERR_ARG, ERR_SHAPE, ERR_CAPACITY = -1, -2, -7


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


def test_capacity_error_reports_required_sizes(ctx):
    from paper_2511_01039_amd import opts_for
    from paper_2511_01039_amd.binding import CTensor, COpts, CReport, OutTensor
    row = wl.small_row("u1u1", L=3, seed=2, oversample=4, power_iters=1, env_scale=1,
                       virt_scale=1)
    T, A, W = devs(row.T), devs(row.A), devs(row.W)
    opts = opts_for(row.sym, chi=8, oversample=4, power_iters=1, seed=1, row=row.row)
    L = len(T)
    keep = []
    ein = (CTensor * L)(*[t.ctensor(keep) for t in T])
    kin = (CTensor * L)(*[t.ctensor(keep) for t in A])
    pin = (CTensor * L)(*[t.ctensor(keep) for t in W])
    outs = [OutTensor(5, ein[0].nlab, 256, 2, 4) for _ in range(L)]
    oarr = (CTensor * L)(*[o.ct for o in outs])
    ln = C.c_double(0.0)
    rep = CReport()
    rc = ctx.lib.fpeps_env_absorb(ctx.h, L, ein, kin, pin, C.byref(opts), oarr, C.byref(ln),
                                  C.byref(rep))
    assert rc == ERR_CAPACITY
    assert rep.required_elem > 4 and rep.required_blocks >= 1
    assert b"capacity" in ctx.lib.fpeps_last_error(ctx.h).lower()
    # the same call with the reported sizes goes through
    out, lg, r = ctx.env_absorb(T, A, W, opts,
                                caps=[(256, max(rep.required_blocks, 1) * 4,
                                       max(rep.required_elem, 1) * 4)] * L)
    assert np.isfinite(lg) and len(out) == L


def test_null_arguments_and_shape_mismatch(ctx):
    from paper_2511_01039_amd import opts_for
    from paper_2511_01039_amd.binding import CTensor, CReport
    rep = CReport()
    rc = ctx.lib.fpeps_env_absorb(ctx.h, 3, None, None, None, None, None, None, C.byref(rep))
    assert rc == ERR_ARG
    # a ket whose virtual legs do not match the environment's bundle legs
    row = wl.small_row("u1u1", L=3, seed=2, oversample=4, power_iters=1, env_scale=1,
                       virt_scale=1)
    other = wl.small_row("u1u1", L=3, seed=2, oversample=4, power_iters=1, env_scale=1,
                         virt_scale=2)
    from paper_2511_01039_amd.binding import FpepsError
    with pytest.raises(FpepsError) as e:
        ctx.env_absorb(devs(row.T), devs(other.A), devs(other.W),
                       opts_for(row.sym, chi=8, oversample=4, power_iters=1, seed=1,
                                row=row.row))
    assert e.value.code in (ERR_SHAPE, ERR_ARG)
    # the context still works
    out, lg, _ = ctx.env_absorb(devs(row.T), devs(row.A), devs(row.W),
                                opts_for(row.sym, chi=8, oversample=4, power_iters=1, seed=1,
                                         row=row.row))
    assert np.isfinite(lg)


def test_prepared_operator_refuses_wrong_vector_size(ctx):
    import torch
    from paper_2511_01039_amd import DeviceTensor, opts_for
    from paper_2511_01039_amd.binding import FpepsError
    h = wl.heff_inputs("u1u1", seed=3, env_scale=2, virt_scale=1)
    dv = {n: DeviceTensor.from_host(h[n]) for n in ("T", "L", "B", "R", "W", "A")}
    op, y, _ = ctx.heff_prepare(dv["T"], dv["L"], dv["B"], dv["R"], dv["W"], dv["A"],
                                opts_for(h["sym"]))
    a = torch.zeros(dv["A"].nelem + 1, dtype=torch.float64, device="cuda")
    op.a_elems = dv["A"].nelem + 1
    with pytest.raises(FpepsError):
        op.apply(a)
    op.a_elems = dv["A"].nelem
    yy, _ = op.apply(a[:-1].contiguous())
    assert float(yy[:y.nelem].abs().max()) == 0.0
    op.close()
