"""Algorithmic flop count of a row absorption (oracle).

Definition used for every throughput figure:
* chain: 2 m n k over every contributing block pair of every chain step,
  for each of the 2 + 2q applications of M or M^T per truncated site
  (one for the final site);
* orthonormalisation of an m x k block: 2 m k^2 - 2 k^3 / 3 (Householder QR);
* core SVD of the k x n block B: 2 n k^2 + 12 k^3;
* U = Q U~: 2 m k c and R = U~^T B: 2 k c n with c kept columns.
Anything an implementation adds (padding, masked tiles, extra passes of a
split-precision product) is not counted.
"""
from __future__ import annotations


def chain_flops(sp, kvec):
    op = sp.op
    om = op.omega_bt(sp.sect, kvec)
    om.blocks = {k: v for k, v in om.blocks.items() if kvec[k[-1]] > 0}
    return op.chain_flops(om)


def site_flops(sp, kvec, kept, q):
    f = chain_flops(sp, kvec) * (2 + 2 * q)
    for m, n, k, c in zip(sp.m, sp.n, kvec, kept):
        if k == 0:
            continue
        f += (q + 1) * (2 * m * k * k - 2 * k ** 3 / 3.0) + q * (2 * n * k * k - 2 * k ** 3 / 3.0)
        f += 2 * n * k * k + 12 * k ** 3
        f += 2 * m * k * c + 2 * k * c * n
    return f


def row_flops(record, info, q):
    """``record``/``info`` as filled by zipup.absorb_row(record=[...])."""
    total = 0.0
    for r, kept in zip(record, info["kept"]):
        total += site_flops(r["sp"], r["kvec"], kept, q)
    return total
