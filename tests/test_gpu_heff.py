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
