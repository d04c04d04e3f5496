"""Algorithmic flop count of a row absorption (oracle).

Definition used for every throughput figure:
* chain: 2 m n k over every block pair of every chain step. The rSVD of a
  truncated site applies M (the forward chain) 1 + q times and M^T (the
  mirrored chain, counted over its own block pairs) 1 + q times; the final
  site applies M once. The mirrored chain counts, at its last step, only
  the pairs whose output lands on a column tuple of M (M^T acts on M's
  domain);
* orthonormalisation of an m x k block: 2 m k^2 - 2 k^3 / 3 (Householder QR,
  Golub & Van Loan, Matrix Computations, 4th ed., Alg. 5.2.1);
* core SVD of the k x n block B: 2 n k^2 + 11 k^3 (R-SVD of the n x k
  transpose, singular values and right vectors; Golub & Van Loan,
  Fig. 8.6.1);
* U = Q U~: 2 m k c and R = U~^T B: 2 k c n with c kept columns, once per
  truncated site.
Every factorisation pass of a site counts (a site whose saturated sectors
were widened is factorised again with the wider sketch). Anything an
implementation adds (padding, masked tiles, extra passes of a
split-precision product) is not counted.
"""
from __future__ import annotations

from .rsvd import final_widths


def chain_flops(sp, kvec):
    """Forward chain M X with per-sector widths ``kvec``."""
    op = sp.op
    om = op.omega_bt(sp.sect, kvec)
    om.blocks = {k: v for k, v in om.blocks.items() if kvec[k[-1]] > 0}
    return op.chain_flops(om)


def chain_flops_t(sp, kvec):
    """Mirrored chain M^T Y with per-sector widths ``kvec``."""
    return sp.op.chain_flops_t(sp.y_struct(kvec), sp.col_blocks(kvec))


def pass_flops(sp, kvec, q):
    f = (1 + q) * (chain_flops(sp, kvec) + chain_flops_t(sp, kvec))
    for m, n, k in zip(sp.m, sp.n, kvec):
        if k == 0:
            continue
        f += (q + 1) * (2 * m * k * k - 2 * k ** 3 / 3.0) + q * (2 * n * k * k - 2 * k ** 3 / 3.0)
        f += 2 * n * k * k + 11 * k ** 3
    return f


def site_flops(sp, passes, q, cbe_passes=(), cbe_kept=None):
    """``passes``: [(k, kept)] of every factorisation of the site;
    ``cbe_passes`` those of its bond expansion (``cbe_kept`` directions
    added). An expansion pass applies M and M^T once each with the projector
    splits around them (4 c k (m + n) per application, c the truncation's
    kept count), orthonormalises once and factorises; then Q = Q_s U~
    (2 m k e) and the expansion's remainder rows M^T Q (mirrored chain at
    widths e)."""
    f = 0.0
    for kvec, _ in passes:
        f += pass_flops(sp, kvec, q)
    kvec, kept = final_widths(passes), passes[-1][1]
    for m, n, k, c in zip(sp.m, sp.n, kvec, kept):
        if k > 0:
            f += 2 * m * k * c + 2 * k * c * n
    for kc, _ in cbe_passes:
        f += chain_flops(sp, kc) + chain_flops_t(sp, kc)
        for m, n, k, c in zip(sp.m, sp.n, kc, kept):
            if k > 0:
                f += 8.0 * c * k * (m + n)
                f += 2 * m * k * k - 2 * k ** 3 / 3.0
                f += 2 * n * k * k + 11 * k ** 3
    if cbe_passes:
        kc = final_widths(cbe_passes)
        f += chain_flops_t(sp, cbe_kept)
        for m, k, e in zip(sp.m, kc, cbe_kept):
            if k > 0:
                f += 2.0 * m * k * e
    return f


def row_flops(record, info, q):
    """``record``/``info`` as filled by zipup.absorb_row(record=[...])."""
    total = 0.0
    for r in record:
        total += site_flops(r["sp"], r["passes"], q, r.get("cbe_passes") or (),
                            r.get("cbe_kept"))
    return total


def explicit_flops(m, n, passes, q, r=None):
    """Explicit matrices (``rsvd_explicit``, ``cbe_explicit`` with kept ranks
    ``r``): per pass 1 + q products with A and with A^T (2 m n k each), for
    an expansion the projector splits (4 r k (m + n) per product pair),
    orthonormalisation and core SVD as for a site; the factors U = Q U~
    (2 m k c) and, for a truncation, R = U~^T B (2 k c n) once."""
    f = 0.0
    for kvec, _ in passes:
        for i, k in enumerate(kvec):
            if k <= 0:
                continue
            mi, ni = m[i], n[i]
            f += (2 + 2 * q) * 2.0 * mi * ni * k
            if r is not None:
                f += (2 + 2 * q) * 4.0 * r[i] * k * (mi + ni)
            f += (q + 1) * (2 * mi * k * k - 2 * k ** 3 / 3.0) + q * (2 * ni * k * k - 2 * k ** 3 / 3.0)
            f += 2 * ni * k * k + 11 * k ** 3
    kvec, kept = final_widths(passes), passes[-1][1]
    for i, (k, c) in enumerate(zip(kvec, kept)):
        if k > 0:
            f += 2.0 * m[i] * k * c + (0.0 if r is not None else 2.0 * k * c * n[i])
    return f
