"""Randomized SVD of the oracle (Sec. 4; Halko, Martinsson & Tropp, SIAM
Rev. 53 (2011) 217, Example 1.6 with the subspace iteration of their
Algorithm 4.4 and the direct SVD of their Sec. 5.1).

Stage A: Y = M Omega; q times Y <- M qr(M^T qr(Y)); Q = qr(Y).
Stage B: B = Q^T M; B = U~ S V^T (LAPACK); U = Q U~.

Matrices come in independent sectors J (the block-diagonal structure of a
symmetric operator); the number of kept singular values is decided once over
all sectors together.
"""
from __future__ import annotations

import math
import numpy as np


def sketch_widths(m, n, chi, p):
    """k_J = min(m_J, n_J, ceil(chi m_J / sum m) + p); 0 for empty sectors."""
    tot = int(sum(m))
    out = []
    for mj, nj in zip(m, n):
        if mj <= 0 or nj <= 0 or tot <= 0:
            out.append(0)
        else:
            out.append(int(min(mj, nj, -(-chi * mj // tot) + p)))
    return out


SV_CUT = 1e-7


def global_cut(sigmas, chi, sector_keys=None, sv_cut=SV_CUT):
    """Keep the min(chi, total) largest values over all sectors, never one
    below sv_cut times the largest (numerically zero singular values have no
    defined vectors). Ties are broken by sector key (lexicographic), then by
    in-sector position. Returns kept counts per sector, the discarded weight
    sum(s^2 cut) / sum(s^2) and the relative gap
    (s_last_kept - s_first_cut)/s_last_kept."""
    keys = sector_keys if sector_keys is not None else list(range(len(sigmas)))
    allv = []
    for si, s in enumerate(sigmas):
        for i, v in enumerate(s):
            allv.append((-float(v), keys[si], i, si))
    allv.sort()
    smax = -allv[0][0] if allv else 0.0
    above = sum(1 for v in allv if -v[0] > sv_cut * smax)
    nkeep = min(chi, above)
    kept = [0] * len(sigmas)
    for e in allv[:nkeep]:
        kept[e[3]] += 1
    tot2 = sum(v * v for v, *_ in allv)
    disc2 = sum(v * v for v, *_ in allv[nkeep:])
    gap = float("inf")
    if 0 < nkeep < len(allv):
        a, b = -allv[nkeep - 1][0], -allv[nkeep][0]
        gap = (a - b) / a if a > 0 else 0.0
    return kept, (disc2 / tot2 if tot2 > 0 else 0.0), gap


def orth(Y):
    """Orthonormal basis of range(Y) (Householder QR, LAPACK geqrf/orgqr)."""
    if Y.shape[1] == 0:
        return Y.copy()
    Q, _ = np.linalg.qr(Y)
    return Q


def rsvd_sectors(apply_m, apply_mt, omegas, q):
    """Stage A + B for independent sectors. ``apply_m`` maps a list of
    per-sector n_J x k_J matrices to the list of m_J x k_J products (and
    ``apply_mt`` the reverse). Returns per-sector Q, U~, sigma, B."""
    Y = apply_m(omegas)
    Q = [orth(y) for y in Y]
    for _ in range(q):
        Z = apply_mt(Q)
        Qz = [orth(z) for z in Z]
        Y = apply_m(Qz)
        Q = [orth(y) for y in Y]
    Bt = apply_mt(Q)
    Us, Ss, Bs = [], [], []
    for bt in Bt:
        B = bt.T
        if B.shape[0] == 0:
            Us.append(np.zeros((0, 0))); Ss.append(np.zeros(0)); Bs.append(B)
            continue
        Ut, s, _ = np.linalg.svd(B, full_matrices=False)
        Us.append(Ut); Ss.append(s); Bs.append(B)
    return Q, Us, Ss, Bs


def rsvd_explicit(mats, chi, p, q, seed, tag=0, stream=0, sv_cut=SV_CUT):
    """Batched rSVD of explicit matrices with one global cut (the
    ``fpeps_rsvd_truncate`` contract). Omega_i uses the counter stream
    (seed; c1 = i, c2 = tag, c3 = stream << 16)."""
    from .rng import gaussian_matrix
    m = [a.shape[0] for a in mats]
    n = [a.shape[1] for a in mats]
    k = sketch_widths(m, n, chi, p)
    oms = [gaussian_matrix(seed, i, tag, (stream << 16), n[i], k[i]) for i in range(len(mats))]
    Q, Ut, S, B = rsvd_sectors(lambda X: [a @ x for a, x in zip(mats, X)],
                               lambda X: [a.T @ x for a, x in zip(mats, X)], oms, q)
    kept, disc, gap = global_cut(S, chi, sv_cut=sv_cut)
    from .zipup import fix_signs
    UR = [fix_signs(Q[i] @ Ut[i][:, :kept[i]], Ut[i][:, :kept[i]].T @ B[i]) for i in range(len(mats))]
    U = [u for u, _ in UR]
    R = [r for _, r in UR]
    sig = [S[i][:kept[i]] for i in range(len(mats))]
    return dict(U=U, R=R, sigma=sig, sigma_all=S, kept=kept, k=k, discarded=disc, gap=gap)
