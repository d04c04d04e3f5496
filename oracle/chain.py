"""The implicit site operator M_x of one zip-up step, applied to a block of
vectors in the fixed association "sketch first" (oracle).

Sec. 4 factorises a (chi D w D) x (chi D w D) matrix A that is never formed;
the rows of M_x here are (c, dk, dw, db) and the columns (b, rk, rw, rb):

    M_x = sum  R[c,a,lk,lw,lb] T[a,tk,tw,tb,b] A[p,lk,rk,tk,dk]
               W[q,p,lw,rw,tw,dw] A[q,lb,rb,tb,db]

The product M_x Omega is evaluated as  R (bra (W (ket (T Omega)))), one
layer at a time (Sec. 3 contracts the environment T, L, B with the
PEPS-PEPO-PEPS sandwich; the three layers are applied separately here), and
M_x^T Z is the mirrored chain. Each step is a sum over block pairs; a pair
carries alpha = (synthetic recoupling coefficient) x (parity sign), both
keyed by the step, the sectors of the intermediate on the sketch side and
the sectors of the step's tensor, so that the mirrored chain applies the
exact transpose.
"""
from __future__ import annotations

import itertools
import math
import numpy as np

from workloads.tensor import Leg
from .blocks import BT, contract, from_tensor, pair_flops, pair_flops_to
from .rng import hash_words, unit_from_hash, gaussian_block

# canonical leg orders of the intermediates of the chain
ORDERS = [
    ["b", "rk", "rw", "rb", "j"],                       # X0 = Omega
    ["a", "tk", "tw", "tb", "rk", "rw", "rb", "j"],     # X1 = T Omega
    ["a", "tw", "tb", "rw", "rb", "j", "p", "lk", "dk"],  # X2 (ket absorbed)
    ["a", "tb", "rb", "j", "lk", "dk", "q", "lw", "dw"],  # X3 (PEPO absorbed)
    ["a", "j", "lk", "dk", "lw", "dw", "lb", "db"],     # X4 (bra absorbed)
    ["c", "dk", "dw", "db", "j"],                       # Y
]
T_NAMES = ["a", "tk", "tw", "tb", "b"]
KET_NAMES = ["p", "lk", "rk", "tk", "dk"]
PEPO_NAMES = ["q", "p", "lw", "rw", "tw", "dw"]
BRA_NAMES = ["q", "lb", "rb", "tb", "db"]
R_NAMES = ["c", "a", "lk", "lw", "lb"]


def label_parity(sym, lab):
    if sym.kind == "u1u1":
        return int(lab[1]) & 1
    if sym.kind == "su2":
        return int(lab[0]) & 1
    return 0


def pair_alpha(sym, step, xbt: BT, xkey, tbt: BT, tkey):
    """alpha for one block pair of chain step ``step`` (1..5). ``xkey`` is the
    sketch-side intermediate X_{step-1} block in ORDERS[step-1] order."""
    a = 1.0
    xlabs = [xbt.legs[n].labels[s] for n, s in zip(xbt.names, xkey)]
    tlabs = [tbt.legs[n].labels[s] for n, s in zip(tbt.names, tkey)]
    if sym.kind == "su2":
        words = [step] + [int(v) for lab in xlabs for v in lab] + [int(v) for lab in tlabs for v in lab]
        a = 2.0 * unit_from_hash(hash_words(sym.coef_seed, words)) - 1.0
    if sym.fermionic:
        shared = set(xbt.names) & set(tbt.names)
        px = sum(label_parity(sym, lab) for n, lab in zip(xbt.names, xlabs) if n not in shared)
        pt = sum(label_parity(sym, lab) for n, lab in zip(tbt.names, tlabs) if n in shared)
        if (px * pt) & 1:
            a = -a
    return a


def flip(leg: Leg):
    return Leg(leg.labels, leg.dims, -leg.dir)


class SiteOperator:
    """M_x for one site: R (remainder of the previous zip-up step), T (top
    environment site), ket A and PEPO W. The bra is A with reversed legs
    unless another (real) tensor is given."""

    def __init__(self, sym, R: BT, T, A, W, bra=None):
        self.sym = sym
        self.R = R
        self.T = from_tensor(T, T_NAMES)
        self.ket = from_tensor(A, KET_NAMES)
        self.W = from_tensor(W, PEPO_NAMES)
        bra = from_tensor(A if bra is None else bra, BRA_NAMES)
        bra.legs = {n: flip(l) for n, l in bra.legs.items()}
        self.bra = bra
        self.tensors = [self.T, self.ket, self.W, self.bra, self.R]
        self._alpha_memo = {}

    # --- structure of the column space ---------------------------------
    def col_legs(self):
        return [self.T.legs["b"], self.ket.legs["rk"], self.W.legs["rw"], self.bra.legs["rb"]]

    def row_legs(self):
        return [self.R.legs["c"], self.ket.legs["dk"], self.W.legs["dw"], self.bra.legs["db"]]

    def sectors(self):
        """Sketch sectors J: list of (label, [column tuples]) in label order."""
        legs = self.col_legs()
        out = {}
        for tup in itertools.product(*[range(l.nsect) for l in legs]):
            labs = [legs[i].labels[s] for i, s in enumerate(tup)]
            for J in self._col_labels(labs, legs):
                out.setdefault(J, []).append(tup)
        return [(J, out[J]) for J in sorted(out)]

    def _col_labels(self, labs, legs):
        k = self.sym.kind
        if k == "none":
            return [(0,)]
        if k == "u1u1":
            tot = np.zeros(2, dtype=np.int64)
            for lab, leg in zip(labs, legs):
                tot -= leg.dir * np.asarray(lab, dtype=np.int64)
            return [tuple(int(v) for v in tot)]
        tj = [int(l[0]) for l in labs]
        s, mx = sum(tj), max(tj)
        res = []
        for J in range(0, s + 1):
            allj = tj + [J]
            tot = s + J
            if tot % 2 == 0 and 2 * max(mx, J) <= tot:
                res.append((J,))
        return res

    def col_dim(self, tup):
        return int(np.prod([l.dims[s] for l, s in zip(self.col_legs(), tup)]))

    def j_leg(self, labels, dims):
        lab = np.array(labels, dtype=np.int32).reshape(len(labels), -1)
        return Leg(lab, np.array(dims, dtype=np.int32), -1)

    def omega_bt(self, sect, kdims, arrays=None):
        """Omega with the given sectors (list of (J, tuples)) and widths."""
        legs = self.col_legs()
        jl = self.j_leg([J for J, _ in sect], kdims)
        names = ORDERS[0]
        bt = BT(list(names), {"b": flip(legs[0]), "rk": flip(legs[1]), "rw": flip(legs[2]),
                              "rb": flip(legs[3]), "j": jl}, {})
        for ji, (J, tuples) in enumerate(sect):
            for ti, tup in enumerate(tuples):
                shp = tuple(int(l.dims[s]) for l, s in zip(legs, tup)) + (int(kdims[ji]),)
                bt.blocks[tup + (ji,)] = None if arrays is None else arrays[ji][ti].reshape(shp)
        return bt

    # --- the chain -------------------------------------------------------
    def _alpha(self, step, xbt, xkey, tbt, tkey):
        """pair_alpha, remembered per (step, sketch-side block, step-tensor
        block): it depends only on their sector labels. The sketch-side leg
        catalogues of a step are the same in every application, except the
        sketch leg j, whose sector labels are part of the key."""
        jl = xbt.legs.get("j")
        jlab = tuple(int(v) for v in jl.labels[xkey[xbt.names.index("j")]]) if jl is not None else ()
        key = (step, xkey, tkey, jlab)
        a = self._alpha_memo.get(key)
        if a is None:
            a = pair_alpha(self.sym, step, xbt, xkey, tbt, tkey)
            self._alpha_memo[key] = a
        return a

    def apply(self, Om: BT, symbolic=False):
        X = Om
        for s in range(5):
            S = self.tensors[s]
            X = contract(X, S, ORDERS[s + 1], symbolic=symbolic,
                         alpha=(lambda xk, tk, ok, s=s, X=X, S=S:
                                self._alpha(s + 1, X, xk, S, tk)))
        return X

    def apply_t(self, Z: BT, symbolic=False):
        for s in reversed(range(5)):
            S = self.tensors[s]
            tmpl = BT(list(ORDERS[s]), {n: self._leg_of(n, Z, S) for n in ORDERS[s]}, {})
            Z = contract(Z, S, ORDERS[s], symbolic=symbolic,
                         alpha=(lambda zk, tk, ok, s=s, S=S, tmpl=tmpl:
                                self._alpha(s + 1, tmpl, ok, S, tk)))
        return Z

    @staticmethod
    def _leg_of(n, Z, S):
        return Z.legs[n] if n in Z.legs else S.legs[n]

    def chain_flops(self, Om_struct: BT):
        """Flops 2 m n k over all block pairs of one application."""
        X, total = Om_struct, 0
        for s in range(5):
            S = self.tensors[s]
            total += pair_flops(X, S)
            X = contract(X, S, ORDERS[s + 1], symbolic=True)
        return total

    def chain_flops_t(self, Y_struct: BT, col_blocks):
        """Flops 2 m n k over the block pairs of one application of the
        mirrored chain to ``Y_struct``; the last step counts only pairs whose
        output block is in ``col_blocks`` (M's domain)."""
        Z, total = Y_struct, 0
        for s in reversed(range(5)):
            S = self.tensors[s]
            total += pair_flops_to(Z, S, ORDERS[s], col_blocks if s == 0 else None)
            Z = contract(Z, S, ORDERS[s], symbolic=True)
        return total


def trivial_remainder(sym, T, A, W):
    """R_0 at the left edge: every leg of dim 1, value 1."""
    zero = Leg(np.zeros((1, sym.nlab), dtype=np.int32), np.ones(1, dtype=np.int32), 1)
    legs = {"c": zero, "a": T.legs[0], "lk": A.legs[1], "lw": W.legs[2], "lb": flip(A.legs[1])}
    for n in ("a", "lk", "lw", "lb"):
        assert legs[n].total == 1, "left boundary legs must have dim 1"
    return BT(list(R_NAMES), legs, {(0, 0, 0, 0, 0): np.ones((1, 1, 1, 1, 1))})


def sketch_arrays(sect, kdims, col_dims, seed, c1_base, site, row, stream):
    """Gaussian Omega_J for every sector: rows are the column tuples in
    order, row-major inside each tuple; element (r, c) of Omega_J uses index
    r * k_J + c of the stream (seed; c1 = sector ordinal, c2 = site,
    c3 = row | stream << 16)."""
    out = []
    for ji, (J, tuples) in enumerate(sect):
        k = int(kdims[ji])
        n = int(sum(col_dims[ji]))
        g = gaussian_block(seed, c1_base + ji, site, (row & 0xFFFF) | (stream << 16), n * k)
        g = g.reshape(n, k)
        arrs, r0 = [], 0
        for nd in col_dims[ji]:
            arrs.append(g[r0:r0 + nd])
            r0 += nd
        out.append(arrs)
    return out
