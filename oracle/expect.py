"""Network value from boundary MPSs (oracle).

The expectation value of the PEPS-PEPO-PEPS sandwich (Sec. 2, Fig. 1) is
read off once the environments are built: a top environment and a bottom
environment whose bundle legs (ket, PEPO, bra) face each other are contracted
site by site, E_x[c_t, c_b] = sum E_{x-1}[a_t, a_b] T_x[a_t, k, w, b', c_t]
Bot_x[a_b, k, w, b', c_b], left to right. The network value is
E_L * exp(log_norm_top + log_norm_bottom).
"""
from __future__ import annotations

import math
import numpy as np

from workloads.tensor import Leg, Tensor
from .blocks import BT, from_tensor, contract


def overlap(top, bottom):
    """Plain contraction of two environments (lists of [a, k, w, b', b]
    tensors). Returns the scalar value (without log-norms)."""
    zero = lambda leg: Leg(leg.labels, leg.dims, leg.dir)
    E = None
    for x, (Tt, Tb) in enumerate(zip(top, bottom)):
        tb = from_tensor(Tt, ["at", "k", "w", "bb", "ct"])
        bb = from_tensor(Tb, ["ab", "k", "w", "bb", "cb"])
        if E is None:
            assert tb.legs["at"].total == 1 and bb.legs["ab"].total == 1
            E = BT(["at", "ab"], {"at": tb.legs["at"], "ab": bb.legs["ab"]},
                   {(0, 0): np.ones((1, 1))})
        X = contract(E, tb, ["ab", "k", "w", "bb", "ct"])
        E = contract(X, bb, ["ct", "cb"])
        E = BT(["at", "ab"], {"at": E.legs["ct"], "ab": E.legs["cb"]},
               {k: v for k, v in E.blocks.items()})
    tot = 0.0
    for k, v in E.blocks.items():
        tot += float(np.sum(v))
    return tot


def closing_env(env):
    """An environment of dim-1 legs matching the open (dim-1) bundle legs of
    ``env``: used below the last row (built by the shared input module)."""
    from workloads.configs import bottom_closing
    return bottom_closing(env)


def network_value(sym, lattice_A, lattice_W, chi, p, q, seed, exact_svd=False, bra=None,
                  sv_cut=None):
    """Top-to-bottom contraction of the whole lattice. Returns (sign, log|Z|,
    info per row)."""
    from .zipup import absorb_row
    from workloads.configs import trivial_env
    Ly, Lx = len(lattice_A), len(lattice_A[0])
    env = trivial_env(sym, Lx)
    lg = 0.0
    infos = []
    for y in range(Ly):
        kw = {} if sv_cut is None else dict(sv_cut=sv_cut)
        env, lg, info = absorb_row(sym, env, lattice_A[y], lattice_W[y], chi, p, q, seed, row=y,
                                   exact_svd=exact_svd, log_norm=lg,
                                   bra=None if bra is None else bra[y], **kw)
        infos.append(info)
    v = overlap(env, closing_env(env))
    if v == 0.0:
        return 0, -math.inf, infos
    return (1 if v > 0 else -1), lg + math.log(abs(v)), infos


def ratio(a, b):
    """(sign, log) pairs -> a / b as float."""
    return a[0] * b[0] * math.exp(a[1] - b[1])
