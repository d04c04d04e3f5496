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
from .rsvd import rsvd_adaptive


def residual_dims(mats, U, V):
    m = [max(a.shape[0] - u.shape[1], 0) for a, u in zip(mats, U)]
    n = [max(a.shape[1] - v.shape[0], 0) for a, v in zip(mats, V)]
    return m, n


def cbe_explicit(mats, U, V, chi_extra, p, seed, tag=0, stream=1, split=True, q=0,
                 sv_cut=None):
    """Truncated complement of every matrix; one global cut of size
    ``chi_extra``. The sketch widths follow the rule of ``rsvd`` on the
    residual's dimensions (m_i - r_i) x (n_i - r_i). Returns dict with Q
    (m_i x e_i, orthogonal to U_i), sigma of the kept complement directions,
    and counts."""
    if split:
        ap = lambda i, X: (lambda Z: Z - U[i] @ (U[i].T @ Z))(mats[i] @ (X - V[i].T @ (V[i] @ X)))
        at = lambda i, Y: (lambda Z: Z - V[i].T @ (V[i] @ Z))(mats[i].T @ (Y - U[i] @ (U[i].T @ Y)))
    else:
        PU = [np.eye(a.shape[0]) - u @ u.T for a, u in zip(mats, U)]
        PV = [np.eye(a.shape[1]) - v.T @ v for a, v in zip(mats, V)]
        ap = lambda i, X: PU[i] @ (mats[i] @ (PV[i] @ X))
        at = lambda i, Y: PV[i] @ (mats[i].T @ (PU[i] @ Y))
    mr, nr = residual_dims(mats, U, V)
    r = rsvd_adaptive(lambda X: [ap(i, x) for i, x in enumerate(X)],
                      lambda Y: [at(i, y) for i, y in enumerate(Y)], mr, nr, chi_extra, p, q,
                      lambda k: [gaussian_matrix(seed, i, tag, (stream << 16), a.shape[1], k[i])
                                 for i, a in enumerate(mats)], sv_cut=sv_cut)
    from .zipup import fix_signs
    kept, out_Q = r["kept"], []
    for i in range(len(mats)):
        qi = r["Q"][i] @ r["Ut"][i][:, :kept[i]]
        out_Q.append(fix_signs(qi, np.zeros((qi.shape[1], 0)))[0])
    return dict(Q=out_Q, sigma=[r["S"][i][:kept[i]] for i in range(len(mats))], kept=kept,
                k=r["k"], gap=r["gap"], passes=r["passes"])
