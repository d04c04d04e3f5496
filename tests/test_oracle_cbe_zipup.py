"""Pins of the oracle's bond expansion inside the zip-up (no GPU): on a small
row the expansion of each site is checked against the explicitly formed
operator M_x and its residual (1 - U U^T) M_x (1 - V^T V)."""
import numpy as np
import pytest

import workloads as wl
from oracle.zipup import SiteProblem, absorb_row, cbe_site, fix_signs
from oracle.chain import SiteOperator, trivial_remainder
from oracle.rsvd import rsvd_adaptive
from oracle.zipup import sketch_arrays


def explicit(sp):
    mats = []
    for ji in range(len(sp.sect)):
        cols = [np.eye(sp.n[i]) if i == ji else np.zeros((sp.n[i], 0)) for i in range(len(sp.sect))]
        mats.append(sp.apply_m(cols)[ji])
    return mats


@pytest.mark.parametrize("kind", ["u1u1", "su2"])
def test_site_expansion_is_top_subspace_of_the_residual(kind):
    """Site 0 of a small row: the expansion Q is orthogonal to U, orthonormal,
    and (the sketch covers the residual) spans the top left singular
    subspace of the explicit residual (LAPACK) chosen by one cut over the
    sectors; the remainder rows are Q^T M."""
    row = wl.small_row(kind, L=3, seed=5, oversample=4, power_iters=1, env_scale=2, virt_scale=1)
    R = trivial_remainder(row.sym, row.T[0], row.A[0], row.W[0])
    sp = SiteProblem(SiteOperator(row.sym, R, row.T[0], row.A[0], row.W[0]))
    labels = [J for J, _ in sp.sect]
    chi, p, e_want = 3, 40, 4
    r = rsvd_adaptive(sp.apply_m, sp.apply_mt, sp.m, sp.n, chi, p, 1,
                      lambda kv: [np.vstack(o) if len(o) else np.zeros((0, kv[i]))
                                  for i, o in enumerate(sketch_arrays(sp.sect, kv, sp.col_dims,
                                                                      7, 0, 0, 0, 0))], labels)
    kept = r["kept"]
    UR = [fix_signs(r["Q"][J] @ r["Ut"][J][:, :kept[J]], r["Ut"][J][:, :kept[J]].T @ r["B"][J])
          for J in range(len(kept))]
    U = [u for u, _ in UR]
    Rm = [x for _, x in UR]
    Qc, Rc, e, passes, k = cbe_site(sp, U, Rm, r["S"], kept, e_want, p, 7, 0, 0, labels)
    assert sum(e) == e_want
    M = explicit(sp)
    res_sig, res_vec = [], []
    for J in range(len(kept)):
        u = U[J]
        v = Rm[J] / r["S"][J][:kept[J]][:, None] if kept[J] else Rm[J]
        Pu = np.eye(sp.m[J]) - u @ u.T
        Pv = np.eye(sp.n[J]) - v.T @ v
        res = Pu @ M[J] @ Pv
        ur, s, _ = np.linalg.svd(res)
        res_sig.append(s)
        res_vec.append(ur)
        q = Qc[J]
        if q.shape[1]:
            if u.shape[1]:
                assert np.abs(q.T @ u).max() < 1e-12
            assert np.abs(q.T @ q - np.eye(q.shape[1])).max() < 1e-12
            assert np.abs(Rc[J] - q.T @ M[J]).max() < 1e-12 * np.abs(M[J]).max()
        # the sketch covers the residual of this sector: exact top subspace
        assert k[J] >= min(sp.m[J] - kept[J], sp.n[J] - kept[J])
    # one cut over the sectors: the e largest residual values overall
    allv = sorted(((v, J) for J, s in enumerate(res_sig) for v in s), reverse=True)[:e_want]
    for J in range(len(kept)):
        assert e[J] == sum(1 for _, j in allv if j == J)
        if e[J]:
            top = res_vec[J][:, :e[J]]
            assert np.abs(Qc[J] @ Qc[J].T - top @ top.T).max() < 1e-9


def test_expanded_row_isometries():
    """A whole row with expansion: every bond grows by the expansion's
    directions and every new environment site is an isometry over its rows."""
    row = wl.small_row("su2", L=4, seed=3, oversample=4, power_iters=1, env_scale=3, virt_scale=2)
    rec0, rec1 = [], []
    e0, l0, i0 = absorb_row(row.sym, row.T, row.A, row.W, 6, 4, 1, 17, row=row.row, record=rec0)
    e1, l1, i1 = absorb_row(row.sym, row.T, row.A, row.W, 6, 4, 1, 17, row=row.row, record=rec1,
                            cbe_extra=3)
    assert [sum(c["kept"]) for c in i1["cbe"]] == [3] * (len(row.T) - 1)
    for site in e1[:-1]:
        blocks = site.to_dict()
        # columns of each sector (last leg) orthonormal over the rows
        cols = {}
        for key, b in blocks.items():
            cols.setdefault(key[-1], []).append(b.reshape(-1, b.shape[-1]))
        for mats in cols.values():
            U = np.vstack(mats)
            assert np.abs(U.T @ U - np.eye(U.shape[1])).max() < 1e-12
    # every bond of the expanded row is its truncation plus the expansion
    for k1, c in zip(i1["kept"], i1["cbe"]):
        assert sum(k1) == sum(c["kept"]) + min(6, sum(k1) - sum(c["kept"]))


def test_sign_gauge_rule():
    """The canonical gauge of a truncated factorisation U R: each column of U
    (with the matching row of R) is flipped so that its leading entry is
    positive, the leading entry being the first in row order whose magnitude
    lies within a relative 1e-5 of the column's largest. Entries 2e-5 below
    the largest do not count as ties; entries 5e-6 below do."""
    U = np.array([[0.3, -0.5, 0.5],
                  [-0.6, 0.5 * (1 - 5e-6), -0.5 * (1 + 1e-6)],
                  [0.6 * (1 - 2e-5), 0.1, 0.2]])
    R = np.arange(9.0).reshape(3, 3)
    U2, R2 = fix_signs(U, R)
    # column 0: the largest is row 1 (negative), row 2 is outside the window
    # column 1: rows 0 and 1 tie; row 0 leads and is negative
    # column 2: rows 0 and 1 tie; row 0 leads and is positive (no flip)
    assert U2[1, 0] > 0 and U2[0, 1] > 0 and U2[0, 2] > 0
    assert np.array_equal(U2[:, 2], U[:, 2]) and np.array_equal(R2[2], R[2])
    assert np.array_equal(U2[:, :2], -U[:, :2]) and np.array_equal(R2[:2], -R[:2])
    assert np.allclose(U2 @ R2, U @ R, rtol=0, atol=0)


def test_partial_row_equals_the_whole_row_prefix():
    """Stopping the absorption after s sites (used for the first sites of a
    row too large for the oracle) gives those sites' kept counts, widths and
    singular values exactly as the whole row does: a site depends only on the
    sites to its left."""
    from oracle.zipup import absorb_row
    row = wl.small_row("su2", L=4, seed=3, oversample=4, power_iters=1, env_scale=3, virt_scale=2)
    _, _, full = absorb_row(row.sym, row.T, row.A, row.W, 10, 4, 1, 17, row=row.row)
    env, _, part = absorb_row(row.sym, row.T, row.A, row.W, 10, 4, 1, 17, row=row.row,
                              stop_after=2)
    assert len(env) == 2 and len(part["kept"]) == 2
    for x in range(2):
        assert list(part["kept"][x]) == list(full["kept"][x])
        assert list(part["k"][x]) == list(full["k"][x])
        for a, b in zip(part["sigma"][x], full["sigma"][x]):
            assert np.array_equal(np.asarray(a), np.asarray(b))
