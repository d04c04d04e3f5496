"""The effective single-site operator (Fig. 2(b)) on the device against the
oracle (needs a GPU): y = H_eff A element by element for dense,
U(1)xU(1) and SU(2)-synthetic inputs, several tiles and ragged block sizes,
and the algorithmic flop count."""
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


CASES = [
    ("none", dict(d=2, D=3, w=2, chi=20)),
    ("u1u1", dict(env_scale=4, virt_scale=2)),
    ("su2", dict(env_scale=5, virt_scale=2)),
]


@pytest.mark.parametrize("kind,kw", CASES, ids=[c[0] for c in CASES])
def test_heff_matches_oracle(ctx, kind, kw):
    from oracle.heff import heff_apply, heff_flops
    from oracle.blocks import to_tensor
    from paper_2511_01039_amd import DeviceTensor, opts_for
    h = wl.heff_inputs(kind, seed=7, **kw)
    want = to_tensor(heff_apply(h["sym"], h["T"], h["L"], h["B"], h["R"], h["W"], h["A"]))
    dv = {n: DeviceTensor.from_host(h[n]) for n in ("T", "L", "B", "R", "W", "A")}
    y, rep = ctx.heff_apply(dv["T"], dv["L"], dv["B"], dv["R"], dv["W"], dv["A"],
                            opts_for(h["sym"]))
    got = y.to_host()
    for lg, lw in zip(got.legs, want.legs):
        assert lg.same_sectors(lw) and lg.dir == lw.dir
    gd, wd = got.to_dict(), want.to_dict()
    assert set(gd) >= {k for k, v in wd.items() if np.abs(v).max() > 0}
    scale = max(float(np.abs(want.data).max()), 1e-300)
    err = 0.0
    for k in set(gd) | set(wd):
        a = gd.get(k)
        b = wd.get(k)
        if a is None:
            a = np.zeros_like(b)
        if b is None:
            b = np.zeros_like(a)
        err = max(err, float(np.abs(a - b).max()))
    print(f"{kind}: blocks {len(gd)} elements {got.data.shape[0]} max rel err {err / scale:.2e} "
          f"flops {rep['alg_flops']:.4e}")
    assert err < 1e-12 * scale
    assert rep["alg_flops"] == pytest.approx(heff_flops(h["T"], h["L"], h["B"], h["R"], h["W"],
                                                        h["A"]), rel=1e-12)


@pytest.mark.parametrize("kind,kw", CASES, ids=[c[0] for c in CASES])
def test_prepared_operator_replays_equal_eager(ctx, kind, kw):
    """The prepared operator (T L and B R once, the three vector-dependent
    products replayed as a HIP graph): every replay, with other device work
    and synchronisations between them, equals the eager fpeps_heff_apply of
    the same vector bit for bit; one replay matches the oracle; the flops of
    preparation and replay add up to the oracle's count; after the context's
    workspace is released the handle refuses to replay."""
    import torch
    from oracle.heff import heff_apply, heff_flops
    from oracle.blocks import to_tensor
    from paper_2511_01039_amd import DeviceTensor, opts_for
    from paper_2511_01039_amd.binding import FpepsError
    h = wl.heff_inputs(kind, seed=11, **kw)
    dv = {n: DeviceTensor.from_host(h[n]) for n in ("T", "L", "B", "R", "W", "A")}
    opts = opts_for(h["sym"])
    op, y0, prep = ctx.heff_prepare(dv["T"], dv["L"], dv["B"], dv["R"], dv["W"], dv["A"], opts)
    ye, erep = ctx.heff_apply(dv["T"], dv["L"], dv["B"], dv["R"], dv["W"], dv["A"], opts)
    n = ye.nelem
    assert y0.nelem == n and torch.equal(y0.data[:n], ye.data[:n])
    A = dv["A"]
    g = torch.Generator(device="cuda").manual_seed(3)
    for i in range(4):
        a = torch.randn(A.nelem, generator=g, device="cuda", dtype=torch.float64)
        yr, rrep = op.apply(a)
        # other device work and a host synchronisation between replays
        junk = torch.randn(256, 256, device="cuda", dtype=torch.float64)
        (junk @ junk).sum().item()
        Ai = DeviceTensor(A.legs, A.blocks, A.offsets, a, A.nelem)
        yi, _ = ctx.heff_apply(dv["T"], dv["L"], dv["B"], dv["R"], dv["W"], Ai, opts)
        assert torch.equal(yr[:n], yi.data[:n]), f"replay {i} differs from the eager product"
        if i == 0:
            host = h["A"]
            Ah = type(host)(list(host.legs), host.blocks, host.offsets, a.cpu().numpy())
            want = to_tensor(heff_apply(h["sym"], h["T"], h["L"], h["B"], h["R"], h["W"], Ah))
            got = yi.to_host()
            gd, wd = got.to_dict(), want.to_dict()
            scale = max(float(np.abs(want.data).max()), 1e-300)
            err = max(float(np.abs(gd[k] - wd[k]).max()) for k in wd if k in gd)
            assert all(k in gd or np.abs(v).max() == 0 for k, v in wd.items())
            assert err < 1e-12 * scale
    assert prep["alg_flops"] + rrep["alg_flops"] == pytest.approx(
        heff_flops(h["T"], h["L"], h["B"], h["R"], h["W"], h["A"]), rel=1e-12)
    print(f"{kind}: prepare {prep['alg_flops']:.3e} flops, replay {rrep['alg_flops']:.3e} flops "
          f"in {rrep['seconds'] * 1e3:.3f} ms")
    # a released workspace invalidates the handle
    ctx.use_hip_allocator()
    with pytest.raises(FpepsError):
        op.apply(a)
    op.close()


def test_prepared_operator_without_graph(ctx):
    """FPEPS_FLAG_NO_GRAPH: the prepared operator launches its three products
    directly instead of replaying a graph; products equal the graph replays
    bit for bit."""
    import torch
    from paper_2511_01039_amd import DeviceTensor, opts_for
    from paper_2511_01039_amd.binding import FLAG_NO_GRAPH
    kind, kw = CASES[-1]
    h = wl.heff_inputs(kind, seed=12, **kw)
    dv = {n: DeviceTensor.from_host(h[n]) for n in ("T", "L", "B", "R", "W", "A")}
    ops = [ctx.heff_prepare(dv["T"], dv["L"], dv["B"], dv["R"], dv["W"], dv["A"],
                            opts_for(h["sym"], flags=f))[0] for f in (0, FLAG_NO_GRAPH)]
    g = torch.Generator(device="cuda").manual_seed(4)
    n = ops[0].y_like.nelem
    for _ in range(3):
        a = torch.randn(dv["A"].nelem, generator=g, device="cuda", dtype=torch.float64)
        yg, _ = ops[0].apply(a)
        ye, rep = ops[1].apply(a)
        assert rep["alg_flops"] > 0
        assert torch.equal(yg[:n], ye[:n])
    for op in ops:
        op.close()
