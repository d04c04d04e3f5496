"""Randomized SVD of the oracle (Sec. 4; Halko, Martinsson & Tropp, SIAM
Rev. 53 (2011) 217, Example 1.6 with the subspace iteration of their
Algorithm 4.4 and the direct SVD of their Sec. 5.1).

Stage A: Y = M Omega; q times Y <- M qr(M^T qr(Y)); Q = qr(Y).
Stage B: B = Q^T M; B = U~ S V^T (LAPACK); U = Q U~.

Matrices come in independent sectors J (the block-diagonal structure of a
symmetric operator); the number of kept singular values is decided once over
all sectors together.

Sketch widths per sector (the paper gives none; Halko et al. Sec. 4.2 ask for
k = (target rank) + p columns): a sector starts with
k_J = min(m_J, n_J, h_J + p), h_J a guess of its kept count (the previous
site's kept count for the same sector label, else its share
ceil(chi m_J / sum m) of chi). After the global cut a sector is saturated
when its sketch does not cover it (k_J < min(m_J, n_J)) and the cut kept
more than k_J - p/2 of its values, i.e. fewer than p/2 oversampling columns
remain. Saturated sectors are widened to min(m_J, n_J, 2 k_J + p) and the
whole factorisation is repeated, until no sector is saturated.

Truncation floor: a value sigma <= eps * max_J max(m_J, n_J) * sigma_max is
never kept (eps = 2^-52): the rank tolerance of Press et al., Numerical
Recipes (3rd ed., Sec. 2.6) and of numpy.linalg.matrix_rank. Below it a
singular value is not resolved by any backward-stable factorisation of the
matrix, and its vectors are not defined.
"""
from __future__ import annotations

import numpy as np

EPS = 2.0 ** -52


def rank_floor(m, n):
    """Relative truncation floor eps * max_J max(m_J, n_J)."""
    dims = [max(int(a), int(b)) for a, b in zip(m, n)]
    return EPS * float(max(dims + [0]))


def sketch_widths(m, n, chi, p, hint=None):
    """k_J = min(m_J, n_J, h_J + p); h_J = hint[J] when given (not None),
    else ceil(chi m_J / sum m). 0 for empty sectors."""
    tot = int(sum(m))
    out = []
    for J, (mj, nj) in enumerate(zip(m, n)):
        if mj <= 0 or nj <= 0 or tot <= 0:
            out.append(0)
            continue
        h = hint[J] if hint is not None and hint[J] is not None else -(-chi * mj // tot)
        out.append(int(min(mj, nj, int(h) + p)))
    return out


def saturated(k, kept, m, n, p):
    """Sectors whose sketch does not cover them and whose cut kept more than
    k_J - p/2 values (2 kept + p > 2 k)."""
    return [kj > 0 and kj < min(mj, nj) and 2 * c + p > 2 * kj
            for kj, c, mj, nj in zip(k, kept, m, n)]


def grown_widths(k, sat, m, n, p):
    return [int(min(mj, nj, 2 * kj + p)) if s else int(kj)
            for kj, s, mj, nj in zip(k, sat, m, n)]


def global_cut(sigmas, chi, sector_keys=None, floor=0.0):
    """Keep the min(chi, total) largest values over all sectors, never one
    at or below floor times the largest. Ties are broken by sector key
    (lexicographic), then by in-sector position. Returns kept counts per
    sector, the discarded weight sum(s^2 cut) / sum(s^2) and the relative
    gap (s_last_kept - s_first_cut)/s_last_kept."""
    keys = sector_keys if sector_keys is not None else list(range(len(sigmas)))
    allv = []
    for si, s in enumerate(sigmas):
        for i, v in enumerate(s):
            allv.append((-float(v), keys[si], i, si))
    allv.sort()
    smax = -allv[0][0] if allv else 0.0
    above = sum(1 for v in allv if -v[0] > floor * smax)
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


def rsvd_adaptive(apply_m, apply_mt, m, n, chi, p, q, omega_fn, keys=None, hint=None,
                  sv_cut=None):
    """The randomized SVD of a sector-diagonal operator with the width rule
    of this module: start from sketch_widths(m, n, chi, p, hint), widen the
    saturated sectors and repeat until none is. ``omega_fn(k)`` returns the
    per-sector Gaussian sketches (n_J x k_J) for widths k (a sector's sketch
    depends on its own width only). A sector that is not widened would give
    its previous factorisation again, so a repeat pass factorises the
    widened sectors only and the others keep theirs; every pass ends with
    the global cut over all sectors. ``sv_cut`` (a relative floor) replaces
    the rank floor when given. Returns a dict with Q, Ut, sigma (all
    computed values), B, kept, k (final widths), the discarded weight, gap,
    and passes = [(k, kept)] of every factorisation pass, k listing the
    widths factorised in that pass (0 for a sector it left as it was)."""
    floor = sv_cut if sv_cut is not None and sv_cut > 0 else rank_floor(m, n)
    k = sketch_widths(m, n, chi, p, hint)
    Q, Ut, S, B = rsvd_sectors(apply_m, apply_mt, omega_fn(k), q)
    kept, disc, gap = global_cut(S, chi, keys, floor)
    passes = [(list(k), list(kept))]
    while True:
        sat = saturated(k, kept, m, n, p)
        if not any(sat):
            break
        grow = [g if s else 0 for g, s in zip(grown_widths(k, sat, m, n, p), sat)]
        Q2, Ut2, S2, B2 = rsvd_sectors(apply_m, apply_mt, omega_fn(grow), q)
        for J, g in enumerate(grow):
            if g > 0:
                Q[J], Ut[J], S[J], B[J] = Q2[J], Ut2[J], S2[J], B2[J]
                k[J] = g
        kept, disc, gap = global_cut(S, chi, keys, floor)
        passes.append((list(grow), list(kept)))
    return dict(Q=Q, Ut=Ut, S=S, B=B, kept=kept, k=list(k), discarded=disc, gap=gap,
                passes=passes, floor=floor)


def final_widths(passes):
    """Widths each sector ends with: its last factorised width over
    ``passes`` (rsvd_adaptive's pass list)."""
    k = list(passes[0][0])
    for kv, _ in passes[1:]:
        k = [b if b > 0 else a for a, b in zip(k, kv)]
    return k


def rsvd_explicit(mats, chi, p, q, seed, tag=0, stream=0, sv_cut=None):
    """Batched rSVD of explicit matrices with one global cut (the
    ``fpeps_rsvd_truncate`` contract). Omega_i uses the counter stream
    (seed; c1 = i, c2 = tag, c3 = stream << 16)."""
    from .rng import gaussian_matrix
    from .zipup import fix_signs
    m = [a.shape[0] for a in mats]
    n = [a.shape[1] for a in mats]
    r = rsvd_adaptive(lambda X: [a @ x for a, x in zip(mats, X)],
                      lambda X: [a.T @ x for a, x in zip(mats, X)], m, n, chi, p, q,
                      lambda k: [gaussian_matrix(seed, i, tag, (stream << 16), n[i], k[i])
                                 for i in range(len(mats))], sv_cut=sv_cut)
    kept, Q, Ut, B = r["kept"], r["Q"], r["Ut"], r["B"]
    UR = [fix_signs(Q[i] @ Ut[i][:, :kept[i]], Ut[i][:, :kept[i]].T @ B[i]) for i in range(len(mats))]
    return dict(U=[u for u, _ in UR], R=[x for _, x in UR],
                sigma=[r["S"][i][:kept[i]] for i in range(len(mats))], sigma_all=r["S"],
                kept=kept, k=r["k"], discarded=r["discarded"], gap=r["gap"], passes=r["passes"])
