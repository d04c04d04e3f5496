"""Pins of the oracle's effective single-site operator (Fig. 2(b)), no GPU:
a single dense einsum, the dense embedding of U(1)xU(1) blocks, a brute-force
sum with the per-pair scalars restated, and the symmetry of the operator for
exchange-symmetric environments."""
import itertools

import numpy as np
import pytest

import workloads as wl
from workloads.tensor import Leg, Tensor
from oracle.heff import heff_apply, HORDERS
from oracle.blocks import to_tensor

EIN = "atuvb,aklmc,cdefg,brshg,qplsue,pkrtd->qmhvf"


def dense_of(bt):
    return to_tensor(bt).to_dense()


def test_dense_equals_one_einsum():
    h = wl.heff_inputs("none", seed=2, d=2, D=3, w=2, chi=4)
    y = heff_apply(h["sym"], h["T"], h["L"], h["B"], h["R"], h["W"], h["A"])
    want = np.einsum(EIN, *[h[n].to_dense() for n in ("T", "L", "B", "R", "W", "A")], optimize=("greedy", 1e8))
    assert y.names == HORDERS[4]
    assert np.allclose(dense_of(y), want, rtol=1e-13, atol=1e-15)


def test_u1_blocks_equal_dense_embedding():
    h = wl.heff_inputs("u1u1", seed=3, env_scale=2, virt_scale=1)
    sym = wl.Sym("u1u1", coef_seed=3, fermionic=False)
    y = heff_apply(sym, h["T"], h["L"], h["B"], h["R"], h["W"], h["A"])
    want = np.einsum(EIN, *[h[n].to_dense() for n in ("T", "L", "B", "R", "W", "A")], optimize=("greedy", 1e8))
    got = dense_of(y)
    assert np.abs(want).max() > 0
    assert np.allclose(got, want, rtol=1e-13, atol=1e-15)


def test_symmetric_environments_give_a_symmetric_operator():
    """<A', H A> = <A, H A'> when every environment is symmetric under the
    exchange of its ket and bra legs and W is symmetric in (q, p)."""
    h = wl.heff_inputs("none", seed=4, d=2, D=2, w=2, chi=3, symmetric=True)
    rng = np.random.default_rng(0)
    A2 = Tensor.from_blocks(h["A"].legs, [(0,) * 5], [rng.standard_normal(h["A"].block(0).shape)])
    H = lambda a: dense_of(heff_apply(h["sym"], h["T"], h["L"], h["B"], h["R"], h["W"], a))
    lhs = float(np.sum(A2.to_dense() * H(h["A"])))
    rhs = float(np.sum(h["A"].to_dense() * H(A2)))
    assert abs(lhs) > 0
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_su2_scalars_brute_force():
    """Every leg two 1-dim sectors (2j = 0, 1): y equals the element-wise
    sum over all index assignments of the product of the six tensors times
    the five per-step scalars, restated here from their definition."""
    from test_oracle_blocksparse import _alpha_ref
    sym = wl.Sym("su2", coef_seed=5, fermionic=True)
    two = Leg.make([((0,), 1), ((1,), 1)])
    rng = np.random.default_rng(2)
    mk = lambda dirs: wl.random_tensor(sym, wl.configs.with_dirs([two] * len(dirs), dirs), rng)
    T, L, B, R = mk(wl.ENV_DIRS), mk((-1, -1, -1, 1, 1)), mk((-1, 1, 1, -1, 1)), mk((1, 1, 1, -1, -1))
    W, A = mk(wl.PEPO_DIRS), mk(wl.KET_DIRS)
    y = heff_apply(sym, T, L, B, R, W, A)
    names = ["a", "tk", "tw", "tb", "b", "lk", "lw", "lb", "c", "dk", "dw", "db", "d", "rk", "rw",
             "rb", "p", "q"]
    tens = [(T.to_dense(), ["a", "tk", "tw", "tb", "b"]), (L.to_dense(), ["a", "lk", "lw", "lb", "c"]),
            (A.to_dense(), ["p", "lk", "rk", "tk", "dk"]),
            (W.to_dense(), ["q", "p", "lw", "rw", "tw", "dw"]),
            (B.to_dense(), ["c", "dk", "dw", "db", "d"]), (R.to_dense(), ["b", "rk", "rw", "rb", "d"])]
    want = np.zeros((2,) * 5)
    lab = lambda v: (int(v),)
    # steps: (X names, S names, S index) in the order of the definition
    steps = [(["a", "tk", "tw", "tb", "b"], ["a", "lk", "lw", "lb", "c"]),
             (HORDERS[0], ["p", "lk", "rk", "tk", "dk"]),
             (HORDERS[1], ["q", "p", "lw", "rw", "tw", "dw"]),
             (["c", "dk", "dw", "db", "d"], ["b", "rk", "rw", "rb", "d"]),
             (HORDERS[2], HORDERS[3])]
    for idx in itertools.product(range(2), repeat=len(names)):
        ix = dict(zip(names, idx))
        v = 1.0
        for dt, nm in tens:
            v *= dt[tuple(ix[n] for n in nm)]
        if v == 0.0:
            continue
        for s, (xn, sn) in enumerate(steps):
            shared = set(xn) & set(sn)
            v *= _alpha_ref(sym, 11 + s, [lab(ix[n]) for n in xn], [lab(ix[n]) for n in sn],
                            [n in shared for n in xn], [n in shared for n in sn])
        want[tuple(ix[n] for n in HORDERS[4])] += v
    got = dense_of(y)
    assert np.abs(want).max() > 0
    assert np.allclose(got, want, rtol=1e-12, atol=1e-15)
