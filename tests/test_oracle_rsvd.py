"""Pins of the oracle's randomized SVD and CBE against LAPACK and the
published error bounds (no GPU)."""
import math

import numpy as np
import pytest

from oracle.rsvd import (rsvd_explicit, sketch_widths, global_cut, saturated, grown_widths,
                         rank_floor, EPS)
from oracle.cbe import cbe_explicit


def prescribed(m, n, sigma, seed):
    rng = np.random.default_rng(seed)
    r = len(sigma)
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return U @ np.diag(sigma) @ V.T, U, V


def test_exact_recovery_when_sketch_covers_rank():
    """rank <= k: sigma and the projector U U^T equal LAPACK's."""
    mats, want = [], []
    for i, (m, n, r) in enumerate([(60, 45, 7), (30, 80, 5), (20, 20, 3)]):
        s = np.sort(np.random.default_rng(i).uniform(0.5, 3.0, r))[::-1]
        a, u, _ = prescribed(m, n, s, 10 + i)
        mats.append(a)
        want.append((s, u))
    out = rsvd_explicit(mats, chi=15, p=8, q=0, seed=4)
    allsig = np.sort(np.concatenate([w[0] for w in want]))[::-1]
    got = np.sort(np.concatenate(out["sigma"]))[::-1]
    assert np.allclose(got, allsig, rtol=1e-12, atol=0)
    for (s, u), U, R, a in zip(want, out["U"], out["R"], mats):
        assert U.shape[1] == len(s)
        assert np.abs(U @ U.T - u @ u.T).max() < 1e-12
        assert np.abs(U.T @ U - np.eye(U.shape[1])).max() < 1e-13
        assert np.abs(U @ R - a).max() < 1e-12 * np.abs(a).max()


def test_global_cut_across_sectors_matches_lapack():
    """Truncated to chi over several sectors = the chi largest singular
    values of the block-diagonal matrix (LAPACK on the assembled matrix)."""
    rng = np.random.default_rng(0)
    mats = [rng.standard_normal((12, 9)), rng.standard_normal((7, 15)), rng.standard_normal((5, 5))]
    out = rsvd_explicit(mats, chi=10, p=20, q=0, seed=1)
    big = np.zeros((24, 29))
    big[:12, :9] = mats[0]; big[12:19, 9:24] = mats[1]; big[19:, 24:] = mats[2]
    s = np.linalg.svd(big, compute_uv=False)
    assert np.allclose(np.sort(np.concatenate(out["sigma"]))[::-1], s[:10], rtol=1e-12)
    assert sum(out["kept"]) == 10


def halko_expected_bound(sig, k, p):
    """Halko, Martinsson, Tropp (2011) Thm. 10.6: expected spectral error of
    the Gaussian range finder with k + p samples."""
    tail = np.sqrt(np.sum(sig[k:] ** 2))
    return (1 + math.sqrt(k / (p - 1))) * sig[k] + math.e * math.sqrt(k + p) / p * tail


def test_range_finder_error_within_halko_bound_and_power_iterations_help():
    m, n, k, p = 300, 250, 20, 10
    sig = 1.0 / (1.0 + np.arange(150)) ** 1.2
    a, _, _ = prescribed(m, n, sig, 3)
    bound = halko_expected_bound(sig, k, p)
    errs = {0: [], 1: [], 2: []}
    for seed in range(8):
        for q in (0, 1, 2):
            out = rsvd_explicit([a], chi=k + p, p=0, q=q, seed=seed)
            U = out["U"][0]
            errs[q].append(np.linalg.norm(a - U @ (U.T @ a), 2))
    mean0 = np.mean(errs[0])
    assert mean0 <= bound
    assert min(errs[0]) >= sig[k + p] * (1 - 1e-12)           # Eckart-Young
    assert np.mean(errs[2]) < np.mean(errs[1]) < mean0


def test_truncated_error_not_below_optimal():
    """Eckart-Young: the truncated rSVD can never beat the truncated SVD."""
    rng = np.random.default_rng(5)
    a = rng.standard_normal((80, 70)) @ np.diag(0.9 ** np.arange(70)) @ rng.standard_normal((70, 70))
    s = np.linalg.svd(a, compute_uv=False)
    for q in (0, 1, 2):
        out = rsvd_explicit([a], chi=10, p=5, q=q, seed=2)
        err = np.linalg.norm(a - out["U"][0] @ out["R"][0])
        assert err >= np.sqrt(np.sum(s[10:] ** 2)) * (1 - 1e-12)


def test_sketch_widths_rule():
    assert sketch_widths([100, 50, 0], [80, 200, 10], chi=30, p=4) == [24, 14, 0]
    assert sketch_widths([3], [1000], chi=500, p=20) == [3]
    # a hint (the previous site's kept count) replaces the proportional share
    assert sketch_widths([100, 50, 40], [80, 200, 90], chi=30, p=4, hint=[2, None, 50]) == [6, 12, 40]


def test_saturation_rule_and_growth():
    k, m, n = [10, 10, 10, 7], [50, 50, 50, 7], [60, 60, 60, 9]
    # 10 - 4/2 = 8: kept 9 or 10 saturates, 8 does not; a covered sector never
    assert saturated(k, [9, 8, 10, 7], m, n, p=4) == [True, False, True, False]
    assert grown_widths(k, [True, False, True, False], m, n, p=4) == [24, 10, 24, 7]
    assert grown_widths([30], [True], [50], [40], p=4) == [40]


def test_weight_in_one_sector_is_found_by_widening():
    """All of the spectrum in one of three equal sectors: the proportional
    widths (chi/3 + p) saturate that sector; widening it recovers LAPACK's
    chi largest values of the block-diagonal matrix exactly (its rank is
    covered by the widened sketch) and the kept count is chi there."""
    sig = [np.geomspace(5.0, 0.5, 32), np.array([1e-3, 5e-4]), np.array([2e-3])]
    mats = [prescribed(200, 150, s, 20 + i)[0] for i, s in enumerate(sig)]
    out = rsvd_explicit(mats, chi=30, p=6, q=1, seed=2)
    assert len(out["passes"]) >= 2
    assert out["passes"][0][0] == [16, 16, 16]
    assert out["passes"][0][1][0] == 16          # saturated at the proportional width
    assert out["kept"] == [30, 0, 0]
    big = np.zeros((600, 450))
    for i, a in enumerate(mats):
        big[200 * i:200 * (i + 1), 150 * i:150 * (i + 1)] = a
    s = np.linalg.svd(big, compute_uv=False)
    assert np.allclose(out["sigma"][0], s[:30], rtol=1e-12)
    u = np.linalg.svd(mats[0])[0][:, :30]
    assert np.abs(out["U"][0] @ out["U"][0].T - u @ u.T).max() < 1e-10


def test_repeat_pass_factorises_widened_sectors_only():
    """A repeat pass lists width 0 for the sectors it leaves, and leaving
    them changes nothing: the result equals factorising every sector again
    at the final widths (the same sketch columns, so the same values) and
    cutting over all of them."""
    from oracle.rng import gaussian_matrix
    from oracle.rsvd import rsvd_sectors, final_widths
    sig = [np.geomspace(5.0, 0.5, 32), np.geomspace(1.0, 0.2, 12), np.array([2e-3])]
    mats = [prescribed(200, 150, s, 20 + i)[0] for i, s in enumerate(sig)]
    out = rsvd_explicit(mats, chi=30, p=6, q=1, seed=2)
    assert len(out["passes"]) >= 2
    for (k0, _), (k1, _) in zip(out["passes"], out["passes"][1:]):
        assert any(v > 0 for v in k1) and any(v == 0 for v in k1)
    assert final_widths(out["passes"]) == out["k"]
    omegas = [gaussian_matrix(2, i, 0, 0, 150, out["k"][i]) for i in range(3)]
    Q, Ut, S, B = rsvd_sectors(lambda X: [a @ x for a, x in zip(mats, X)],
                               lambda X: [a.T @ x for a, x in zip(mats, X)], omegas, 1)
    kept, _, _ = global_cut(S, 30, None, rank_floor([200] * 3, [150] * 3))
    assert kept == out["kept"]
    for i in range(3):
        assert np.array_equal(S[i][:kept[i]], out["sigma"][i])


def test_spectrum_down_to_1e12_is_resolved_and_kept():
    """Prescribed singular values from 1 to 1e-12 (above the rank floor
    eps max(m, n) = 6.7e-14): all are kept, and each agrees with the
    prescribed value to a few eps times the largest (backward stability)."""
    s = np.logspace(0, -12, 40)
    a, u, _ = prescribed(300, 200, s, 11)
    out = rsvd_explicit([a], chi=60, p=10, q=1, seed=5)
    assert rank_floor([300], [200]) == pytest.approx(300 * EPS)
    assert out["kept"] == [40]
    assert np.abs(out["sigma"][0] - s).max() < 50 * EPS * s[0]
    # vectors to eps sigma_max / gap (Davis-Kahan): the top 20 (gap ~ 1e-6)
    assert np.abs(out["U"][0][:, :20] @ out["U"][0][:, :20].T - u[:, :20] @ u[:, :20].T).max() < 1e-9


def test_global_cut_ties_and_counts():
    kept, disc, gap = global_cut([np.array([3.0, 1.0]), np.array([3.0, 2.0])], 3, ["b", "a"])
    assert kept == [1, 2]
    assert disc == pytest.approx(1.0 / 23.0)
    assert gap == pytest.approx(0.5)


def test_cbe_invariants_and_split_equals_explicit_projectors():
    rng = np.random.default_rng(7)
    mats, U, V = [], [], []
    for (m, n, r) in [(40, 35, 5), (25, 50, 4), (12, 9, 2)]:
        mats.append(rng.standard_normal((m, n)))
        U.append(np.linalg.qr(rng.standard_normal((m, r)))[0])
        V.append(np.linalg.qr(rng.standard_normal((n, r)))[0].T)
    a = cbe_explicit(mats, U, V, chi_extra=8, p=4, seed=3)
    b = cbe_explicit(mats, U, V, chi_extra=8, p=4, seed=3, split=False)
    assert sum(a["kept"]) == 8 and a["kept"] == b["kept"]
    for qa, qb, u in zip(a["Q"], b["Q"], U):
        if qa.shape[1] == 0:
            continue
        assert np.abs(qa.T @ u).max() < 1e-13
        assert np.abs(qa.T @ qa - np.eye(qa.shape[1])).max() < 1e-13
        assert np.abs(qa @ qa.T - qb @ qb.T).max() < 1e-12


def test_cbe_spans_top_subspace_of_residual():
    """With the sketch covering the residual's rank, the expansion is the top
    left singular subspace of (1 - U U^T) M (1 - V^T V) (LAPACK)."""
    rng = np.random.default_rng(9)
    m, n, r = 30, 26, 3
    M = rng.standard_normal((m, 8)) @ rng.standard_normal((8, n))
    u = np.linalg.qr(rng.standard_normal((m, r)))[0]
    v = np.linalg.qr(rng.standard_normal((n, r)))[0].T
    res = (np.eye(m) - u @ u.T) @ M @ (np.eye(n) - v.T @ v)
    out = cbe_explicit([M], [u], [v], chi_extra=4, p=10, seed=0)
    Ur, s, _ = np.linalg.svd(res)
    Q = out["Q"][0]
    assert np.abs(Q @ Q.T - Ur[:, :4] @ Ur[:, :4].T).max() < 1e-10
    assert np.allclose(out["sigma"][0], s[:4], rtol=1e-10)


def test_numerically_zero_singular_values_are_never_kept():
    """Rank-deficient sectors: with chi above the total rank the cut keeps
    exactly the rank (values below sv_cut * max carry no defined vectors)."""
    mats = [prescribed(40, 30, np.linspace(3, 1, 6), 1)[0], prescribed(20, 50, np.linspace(2, 1, 3), 2)[0]]
    out = rsvd_explicit(mats, chi=25, p=10, q=1, seed=3)
    assert out["kept"] == [6, 3]
    for U in out["U"]:
        assert np.abs(U.T @ U - np.eye(U.shape[1])).max() < 1e-13
