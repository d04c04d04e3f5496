"""The effective single-site operator applied to a PEPS tensor (oracle): the
contraction pattern of Fig. 2(b), Sec. 3.

Environment tensors around site (x, y): T (top boundary site), L (left
environment), B (bottom boundary site) and R (right environment), and the
PEPS-PEPO sandwich of the site (PEPO W and ket A, the vector of the
Davidson step):

    y[q, lb, rb, tb, db] = sum T[a, tk, tw, tb, b] L[a, lk, lw, lb, c]
                               B[c, dk, dw, db, d] R[b, rk, rw, rb, d]
                               W[q, p, lw, rw, tw, dw] A[p, lk, rk, tk, dk]

evaluated, as in Sec. 3, as ((T L) C) (B R) with the sandwich C applied
layer by layer: X1 = T L, X2 = X1 A, X3 = X2 W, X4 = B R, y = X3 X4. Each
step is a sum over block pairs with the scalar alpha of ``chain.pair_alpha``
keyed by the step (11 .. 15) and the blocks' sector labels in the leg orders
below, so the association is part of the definition for the synthetic SU(2)
scalars.
"""
from __future__ import annotations

from .blocks import BT, contract, from_tensor, pair_flops
from .chain import pair_alpha

T_NAMES = ["a", "tk", "tw", "tb", "b"]
L_NAMES = ["a", "lk", "lw", "lb", "c"]
B_NAMES = ["c", "dk", "dw", "db", "d"]
R_NAMES = ["b", "rk", "rw", "rb", "d"]
KET_NAMES = ["p", "lk", "rk", "tk", "dk"]
PEPO_NAMES = ["q", "p", "lw", "rw", "tw", "dw"]
HORDERS = [
    ["tk", "tw", "tb", "b", "lk", "lw", "lb", "c"],        # X1 = T L
    ["tw", "tb", "b", "lw", "lb", "c", "p", "rk", "dk"],   # X2 = X1 A
    ["tb", "b", "lb", "c", "rk", "dk", "q", "rw", "dw"],   # X3 = X2 W
    ["c", "dk", "dw", "db", "b", "rk", "rw", "rb"],        # X4 = B R
    ["q", "lb", "rb", "tb", "db"],                         # y = X3 X4
]


def _step(sym, step, X, S, out, symbolic=False):
    return contract(X, S, out, symbolic=symbolic,
                    alpha=lambda xk, tk, ok: pair_alpha(sym, step, X, xk, S, tk))


def heff_apply(sym, T, L, B, R, W, A, symbolic=False):
    """y = H_eff A as a block tensor (BT) with legs HORDERS[4]."""
    t, l = from_tensor(T, T_NAMES), from_tensor(L, L_NAMES)
    b, r = from_tensor(B, B_NAMES), from_tensor(R, R_NAMES)
    w, a = from_tensor(W, PEPO_NAMES), from_tensor(A, KET_NAMES)
    X1 = _step(sym, 11, t, l, HORDERS[0], symbolic)
    X2 = _step(sym, 12, X1, a, HORDERS[1], symbolic)
    X3 = _step(sym, 13, X2, w, HORDERS[2], symbolic)
    X4 = _step(sym, 14, b, r, HORDERS[3], symbolic)
    return _step(sym, 15, X3, X4, HORDERS[4], symbolic)


def heff_flops(T, L, B, R, W, A):
    """2 m n k over the block pairs of the five steps."""
    t, l = from_tensor(T, T_NAMES), from_tensor(L, L_NAMES)
    b, r = from_tensor(B, B_NAMES), from_tensor(R, R_NAMES)
    w, a = from_tensor(W, PEPO_NAMES), from_tensor(A, KET_NAMES)
    f = pair_flops(t, l)
    X1 = contract(t, l, HORDERS[0], symbolic=True)
    f += pair_flops(X1, a)
    X2 = contract(X1, a, HORDERS[1], symbolic=True)
    f += pair_flops(X2, w)
    X3 = contract(X2, w, HORDERS[2], symbolic=True)
    f += pair_flops(b, r)
    X4 = contract(b, r, HORDERS[3], symbolic=True)
    f += pair_flops(X3, X4)
    return f
