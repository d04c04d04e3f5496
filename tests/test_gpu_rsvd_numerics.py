"""The truncation floor, sketch widening and flop count of the device
library against the oracle (needs a GPU).

* a spectrum from 1 down to 1e-12 is resolved (every value kept, each within
  a few eps of the largest), which needs the core factorisation of B itself
  rather than of its Gram matrix alone;
* a sector holding all of the spectrum is widened until it is no longer
  saturated, in the same passes as the oracle;
* the library's algorithmic flop count equals the oracle's (forward and
  mirrored chains over their own block pairs, every factorisation pass).
"""
import math

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_01039_amd import Context
    c = Context(0)
    yield c
    c.close()


def prescribed(m, n, sigma, seed):
    rng = np.random.default_rng(seed)
    r = len(sigma)
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return U @ np.diag(sigma) @ V.T, U, V


def t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_spectrum_down_to_1e12_resolved(ctx):
    from oracle.rsvd import rsvd_explicit
    from oracle.flops import explicit_flops
    from paper_2511_01039_amd import make_opts
    s = np.logspace(0, -12, 40)
    a, u, _ = prescribed(300, 200, s, 11)
    want = rsvd_explicit([a], chi=60, p=10, q=1, seed=5)
    U, R, sig, kept, rep = ctx.rsvd_truncate([t(a)], make_opts(chi=60, oversample=10,
                                                               power_iters=1, seed=5))
    print(f"kept {list(kept)} (oracle {want['kept']}), fallbacks {rep['fallbacks']}")
    assert list(kept) == want["kept"] == [40]
    print(f"max |dsigma| {np.abs(sig[0] - s).max():.2e} "
          f"(oracle {np.abs(want['sigma'][0] - s).max():.2e})")
    assert np.abs(sig[0] - s).max() < 50 * EPS * s[0]
    assert np.abs(sig[0] - want["sigma"][0]).max() < 50 * EPS * s[0]
    Uh = U[0].cpu().numpy()
    assert np.abs(Uh[:, :20] @ Uh[:, :20].T - u[:, :20] @ u[:, :20].T).max() < 1e-9
    assert np.abs(Uh.T @ Uh - np.eye(40)).max() < 1e-12
    assert rep["alg_flops"] == pytest.approx(explicit_flops([300], [200], want["passes"], 1),
                                             rel=1e-12)


def test_saturated_sector_is_widened(ctx):
    from oracle.rsvd import rsvd_explicit
    from oracle.flops import explicit_flops
    from paper_2511_01039_amd import make_opts
    sig = [np.geomspace(5.0, 0.5, 32), np.array([1e-3, 5e-4]), np.array([2e-3])]
    mats = [prescribed(200, 150, x, 20 + i)[0] for i, x in enumerate(sig)]
    want = rsvd_explicit(mats, chi=30, p=6, q=1, seed=2)
    U, R, sg, kept, rep = ctx.rsvd_truncate([t(a) for a in mats],
                                            make_opts(chi=30, oversample=6, power_iters=1, seed=2))
    print(f"passes oracle {len(want['passes'])} device {rep['rsvd_passes']} kept {list(kept)}")
    assert list(kept) == want["kept"] == [30, 0, 0]
    assert rep["rsvd_passes"] == len(want["passes"]) >= 2
    assert np.abs(sg[0] - want["sigma"][0]).max() < 1e-12 * sig[0][0]
    Uh = U[0].cpu().numpy()
    assert np.abs(Uh @ Uh.T - want["U"][0] @ want["U"][0].T).max() < 1e-10
    assert rep["alg_flops"] == pytest.approx(
        explicit_flops([200] * 3, [150] * 3, want["passes"], 1), rel=1e-12)


ROWS = [
    ("none", dict(kind="none", L=4, d=2, D=3, w=2, chi=9), 12),
    ("u1u1", dict(kind="u1u1", L=4, env_scale=2, virt_scale=2), 14),
    ("su2", dict(kind="su2", L=4, env_scale=3, virt_scale=2), 10),
]


@pytest.mark.parametrize("name,kw,chi", ROWS, ids=[r[0] for r in ROWS])
def test_row_flop_count_and_passes_match_oracle(ctx, name, kw, chi):
    """O-6: the library's alg_flops of a row absorption equals the oracle's
    count over the same passes (forward and mirrored chains counted over
    their own block pairs)."""
    from oracle.zipup import absorb_row
    from oracle.flops import row_flops
    from paper_2511_01039_amd import DeviceTensor, opts_for
    row = wl.small_row(seed=3, oversample=4, power_iters=1, **kw)
    record = []
    env, lg, info = absorb_row(row.sym, row.T, row.A, row.W, chi, 4, 1, 17, row=row.row,
                               record=record)
    dev = lambda ts: [DeviceTensor.from_host(x) for x in ts]
    out, glg, rep = ctx.env_absorb(dev(row.T), dev(row.A), dev(row.W),
                                   opts_for(row.sym, chi=chi, oversample=4, power_iters=1,
                                            seed=17, row=row.row))
    want = row_flops(record, info, 1)
    npass = sum(len(p) for p in info["passes"])
    print(f"{name}: flops oracle {want:.6e} device {rep['alg_flops']:.6e} passes {npass}/"
          f"{rep['rsvd_passes']}")
    assert rep["rsvd_passes"] == npass
    assert rep["alg_flops"] == pytest.approx(want, rel=1e-12)


def test_exactly_rank_deficient_sketch(ctx):
    """A matrix with only five nonzero rows (its sketch is rank-deficient by
    structure, so no shifted CholeskyQR pass can complete it): the
    orthonormalisation finishes by SVQB, and kept count, singular values and
    projector equal the oracle's (Householder QR)."""
    from oracle.rsvd import rsvd_explicit
    from paper_2511_01039_amd import make_opts
    a = np.zeros((300, 200))
    a[[3, 50, 77, 150, 299]] = np.random.default_rng(1).standard_normal((5, 200))
    want = rsvd_explicit([a], chi=40, p=10, q=1, seed=5)
    U, R, sig, kept, rep = ctx.rsvd_truncate([t(a)], make_opts(chi=40, oversample=10,
                                                               power_iters=1, seed=5))
    print(f"kept {list(kept)} oracle {want['kept']} fallbacks {rep['fallbacks']}")
    assert list(kept) == want["kept"] == [5]
    assert rep["fallbacks"] & 4
    assert np.abs(sig[0] - want["sigma"][0]).max() < 1e-13 * want["sigma"][0][0]
    Uh = U[0].cpu().numpy()
    assert np.abs(Uh @ Uh.T - want["U"][0] @ want["U"][0].T).max() < 1e-12
