"""Dict-of-blocks tensors with named legs, and their pairwise contraction.

A ``BT`` holds, for every leg name, the leg's sector catalogue (labels, dims,
direction) and a dict ``sector tuple -> ndarray``. Contraction of two BTs
sums, over every pair of blocks that agree on the shared (contracted) legs,
``alpha(pair) * tensordot(block_x, block_t)`` into the output block keyed by
the free sectors. This is the block-by-block form of the contractions of
Sec. 3: each output block is the sum over the quantum numbers of the
contracted legs, and different output blocks never overlap.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

from workloads.tensor import Leg, Tensor


@dataclass
class BT:
    names: list          # leg names, in storage order
    legs: dict           # name -> Leg
    blocks: dict         # sector-index tuple (in ``names`` order) -> ndarray or None

    def leg_list(self):
        return [self.legs[n] for n in self.names]

    def copy(self):
        return BT(list(self.names), dict(self.legs),
                  {k: (None if v is None else v.copy()) for k, v in self.blocks.items()})

    def norm2(self):
        return float(sum(np.sum(v * v) for v in self.blocks.values()))

    def scale(self, s):
        for k in self.blocks:
            self.blocks[k] = self.blocks[k] * s


def from_tensor(t: Tensor, names) -> BT:
    assert len(names) == t.nlegs
    return BT(list(names), dict(zip(names, t.legs)),
              {tuple(int(v) for v in b): t.block(i).copy() for i, b in enumerate(t.blocks)})


def to_tensor(bt: BT) -> Tensor:
    keys = sorted(bt.blocks)
    return Tensor.from_blocks(bt.leg_list(), keys, [bt.blocks[k] for k in keys])


def block_shape(bt: BT, key):
    return tuple(int(bt.legs[n].dims[s]) for n, s in zip(bt.names, key))


def contract(X: BT, T: BT, out_names, alpha=None, symbolic=False):
    """Contract over every leg name present in both X and T.

    ``alpha(xkey, tkey, okey)`` returns the scalar of one block pair
    (default 1); keys are sector tuples in X, T and output name order.
    With ``symbolic`` only the set of output blocks is produced (values None).
    Shared legs must carry identical sector catalogues.
    """
    shared = [n for n in X.names if n in T.legs]
    for n in shared:
        assert X.legs[n].same_sectors(T.legs[n]), f"leg {n}: sector mismatch"
    xs = [X.names.index(n) for n in shared]
    ts = [T.names.index(n) for n in shared]
    xfree = [i for i, n in enumerate(X.names) if n not in shared]
    tfree = [i for i, n in enumerate(T.names) if n not in shared]
    raw_names = [X.names[i] for i in xfree] + [T.names[i] for i in tfree]
    assert sorted(raw_names) == sorted(out_names), (raw_names, out_names)
    perm = [raw_names.index(n) for n in out_names]

    groups = {}
    for tk in T.blocks:
        groups.setdefault(tuple(tk[i] for i in ts), []).append(tk)

    out = {}
    for xk, xa in X.blocks.items():
        for tk in groups.get(tuple(xk[i] for i in xs), ()):
            raw_key = tuple(xk[i] for i in xfree) + tuple(tk[i] for i in tfree)
            okey = tuple(raw_key[p] for p in perm)
            if symbolic:
                out[okey] = None
                continue
            a = 1.0 if alpha is None else alpha(xk, tk, okey)
            r = np.tensordot(xa, T.blocks[tk], axes=(xs, ts)).transpose(perm)
            if okey in out:
                out[okey] = out[okey] + a * r
            else:
                out[okey] = a * r
    legs = {n: (X.legs[n] if n in X.legs else T.legs[n]) for n in out_names}
    return BT(list(out_names), legs, out)


def pair_flops(X: BT, T: BT, symbolic_out=None):
    """2 * m * n * k summed over every contributing block pair."""
    shared = [n for n in X.names if n in T.legs]
    xs = [X.names.index(n) for n in shared]
    ts = [T.names.index(n) for n in shared]
    groups = {}
    for tk in T.blocks:
        groups.setdefault(tuple(tk[i] for i in ts), []).append(tk)
    total = 0
    for xk in X.blocks:
        xsz = int(np.prod(block_shape(X, xk)))
        for tk in groups.get(tuple(xk[i] for i in xs), ()):
            tsz = int(np.prod(block_shape(T, tk)))
            ksz = int(np.prod([X.legs[shared[j]].dims[xk[xs[j]]] for j in range(len(shared))]))
            total += 2 * xsz * tsz // max(ksz, 1)
    return total


def pair_flops_to(X: BT, T: BT, out_names, keep=None):
    """2 * m * n * k summed over the block pairs whose output block (sector
    tuple in ``out_names`` order) is in ``keep`` (every pair when None)."""
    shared = [n for n in X.names if n in T.legs]
    xs = [X.names.index(n) for n in shared]
    ts = [T.names.index(n) for n in shared]
    xfree = [i for i, n in enumerate(X.names) if n not in shared]
    tfree = [i for i, n in enumerate(T.names) if n not in shared]
    raw_names = [X.names[i] for i in xfree] + [T.names[i] for i in tfree]
    perm = [raw_names.index(n) for n in out_names]
    groups = {}
    for tk in T.blocks:
        groups.setdefault(tuple(tk[i] for i in ts), []).append(tk)
    total = 0
    for xk in X.blocks:
        xsz = int(np.prod(block_shape(X, xk)))
        for tk in groups.get(tuple(xk[i] for i in xs), ()):
            if keep is not None:
                raw = tuple(xk[i] for i in xfree) + tuple(tk[i] for i in tfree)
                if tuple(raw[q] for q in perm) not in keep:
                    continue
            tsz = int(np.prod(block_shape(T, tk)))
            ksz = int(np.prod([X.legs[shared[j]].dims[xk[xs[j]]] for j in range(len(shared))]))
            total += 2 * xsz * tsz // max(ksz, 1)
    return total
