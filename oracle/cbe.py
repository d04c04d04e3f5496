"""Controlled bond expansion with the randomized SVD (oracle; Sec. 4).

CBE adds to a kept space the most weighty directions of the discarded space
(the "truncated complement"). With kept left space U (orthonormal columns)
and kept right space V (orthonormal rows) of an operator M, the discarded
part is P_U' M P_V' with the orthogonal projectors P_U' = 1 - U U^T and
P_V' = 1 - V^T V (the completeness relation of Fig. 4). Following Fig. 5 the
projectors are never formed: each is split into identity minus the
tangential projector, and one application of the operator to the Gaussian
sketch suffices (q = 0).

Split form:   Z = M Om - M (V^T (V Om)),   Y = Z - U (U^T Z).
(Fig. 5 evaluates the two bracketed clusters and subtracts; by linearity
the sketch is folded first, which halves the number of heavy products.)
Stage B of the randomized SVD then ranks the directions of Q = orth(Y) and
one global cut over all matrices keeps ``chi_extra`` of them.
"""
from __future__ import annotations

import numpy as np

from .rng import gaussian_matrix
from .rsvd import sketch_widths, global_cut, orth, SV_CUT


def residual_widths(mats, U, V, chi_extra, p):
    m = [a.shape[0] - u.shape[1] for a, u in zip(mats, U)]
    n = [a.shape[1] - v.shape[0] for a, v in zip(mats, V)]
    return sketch_widths([max(x, 0) for x in m], [max(x, 0) for x in n], chi_extra, p)


def cbe_explicit(mats, U, V, chi_extra, p, seed, tag=0, stream=1, split=True, q=0,
                 sv_cut=SV_CUT):
    """Truncated complement of every matrix; one global cut of size
    ``chi_extra``. Returns dict with Q (m_i x e_i, orthogonal to U_i),
    sigma of the kept complement directions, and counts."""
    k = residual_widths(mats, U, V, chi_extra, p)
    out_Q, S_, Ut_, Q_ = [], [], [], []
    if split:
        ap = lambda i, X: (lambda Z: Z - U[i] @ (U[i].T @ Z))(mats[i] @ (X - V[i].T @ (V[i] @ X)))
        at = lambda i, Y: (lambda Z: Z - V[i].T @ (V[i] @ Z))(mats[i].T @ (Y - U[i] @ (U[i].T @ Y)))
    else:
        PU = [np.eye(a.shape[0]) - u @ u.T for a, u in zip(mats, U)]
        PV = [np.eye(a.shape[1]) - v.T @ v for a, v in zip(mats, V)]
        ap = lambda i, X: PU[i] @ (mats[i] @ (PV[i] @ X))
        at = lambda i, Y: PV[i] @ (mats[i].T @ (PU[i] @ Y))
    for i, a in enumerate(mats):
        om = gaussian_matrix(seed, i, tag, (stream << 16), a.shape[1], k[i])
        Y = ap(i, om)
        Q = orth(Y)
        for _ in range(q):
            Q = orth(ap(i, orth(at(i, Q))))
        B = at(i, Q).T
        if B.shape[0]:
            Ut, s, _ = np.linalg.svd(B, full_matrices=False)
        else:
            Ut, s = np.zeros((0, 0)), np.zeros(0)
        Q_.append(Q); Ut_.append(Ut); S_.append(s)
    kept, disc, gap = global_cut(S_, chi_extra, sv_cut=sv_cut)
    from .zipup import fix_signs
    for i in range(len(mats)):
        q = Q_[i] @ Ut_[i][:, :kept[i]]
        out_Q.append(fix_signs(q, np.zeros((q.shape[1], 0)))[0])
    return dict(Q=out_Q, sigma=[S_[i][:kept[i]] for i in range(len(mats))], kept=kept, k=k,
                gap=gap)
