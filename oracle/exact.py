"""Exact contraction of small dense networks into state vectors (oracle pin).

For lattices of a few sites the PEPS can be contracted to the full vector
psi[p_1 ... p_N] (row-major site order) and the PEPO applied exactly; the
network value of Fig. 1 is then psi . (W psi) without any environment
approximation.
"""
from __future__ import annotations

import numpy as np


def peps_vector(T):
    """T[y][x]: dense arrays [p, l, r, u, d] -> vector over all physical legs."""
    Ly, Lx = len(T), len(T[0])
    # S[P, c_0..c_{Lx-1}]: physical legs so far, open down legs of last row
    S = np.ones((1,) + (1,) * Lx)
    for y in range(Ly):
        S = S[:, None]                      # add the horizontal leg h (dim 1)
        for x in range(Lx):
            a = T[y][x]                     # [p, l, r, u, d]
            # S[P, h, c_0..c_x..]: h meets the left leg l, c_x the up leg u
            S = np.moveaxis(S, 2 + x, 2)    # S[P, h, u, others...]
            P, h, u = S.shape[0], S.shape[1], S.shape[2]
            rest = S.shape[3:]
            S2 = S.reshape(P, h, u, -1)
            out = np.einsum("Pluo,plrud->Pprdo", S2, a)
            p_, r_, d_ = a.shape[0], a.shape[2], a.shape[4]
            S = out.reshape((P * p_, r_, d_) + rest)
            S = np.moveaxis(S, 2, 2 + x)     # put d back in column x
        assert S.shape[1] == 1
        S = S[:, 0]
    return S.reshape(S.shape[0], -1)[:, 0] if S.ndim > 1 else S


def pepo_times_peps(A, W):
    """The PEPS W|psi> with bond D*w: site [q, (l l'), (r r'), (u u'), (d d')]."""
    out = []
    for ya, yw in zip(A, W):
        row = []
        for a, w in zip(ya, yw):
            t = np.einsum("qplrud,pLRUD->qlLrRuUdD", w, a)
            s = t.shape
            row.append(t.reshape(s[0], s[1] * s[2], s[3] * s[4], s[5] * s[6], s[7] * s[8]))
        out.append(row)
    return out


def exact_value(A, W, bra=None):
    """<bra|W|psi> for dense lattices (bra defaults to psi)."""
    psi = peps_vector(A)
    wpsi = peps_vector(pepo_times_peps(A, W))
    phi = psi if bra is None else peps_vector(bra)
    return float(phi @ wpsi), float(phi @ psi)


def pepo_matrix(W):
    """Dense operator of a PEPO on a small lattice: matrix [q..., p...]."""
    Ly, Lx = len(W), len(W[0])
    d = W[0][0].shape[0]
    N = Lx * Ly
    # treat W as a PEPS with physical leg (q, p) of dim d*d
    T = [[w.reshape((w.shape[0] * w.shape[1],) + w.shape[2:]) for w in row] for row in W]
    v = peps_vector(T).reshape((d, d) * N)
    perm = list(range(0, 2 * N, 2)) + list(range(1, 2 * N, 2))
    return v.transpose(perm).reshape(d ** N, d ** N)
