"""Pins of the oracle's boundary-MPS contraction against exact results,
invariants and special cases (no GPU)."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle.exact import exact_value, peps_vector, pepo_matrix
from oracle.expect import network_value, ratio, overlap, closing_env
from oracle.zipup import absorb_row



def dense(lat):
    return [[t.block(0) for t in row] for row in lat]


def test_peps_vector_two_sites_by_hand():
    lat = wl.config1_lattice(Lx=2, Ly=1)
    a0, a1 = lat.A[0][0].block(0), lat.A[0][1].block(0)
    want = np.einsum("ar,br->ab", a0[:, 0, :, 0, 0], a1[:, :, 0, 0, 0]).ravel()
    assert np.allclose(peps_vector([[a0, a1]]), want, rtol=1e-14, atol=0)
    lat = wl.config1_lattice(Lx=1, Ly=2)
    a0, a1 = lat.A[0][0].block(0), lat.A[1][0].block(0)
    want = np.einsum("ad,bd->ab", a0[:, 0, 0, 0, :], a1[:, 0, 0, :, 0]).ravel()
    assert np.allclose(peps_vector([[a0], [a1]]), want, rtol=1e-14, atol=0)


CHI_INF = 10 ** 9   # keeps every direction: k = min(m, n) at every site


@pytest.mark.parametrize("shape,D,exact_svd", [((3, 3), 3, False), ((4, 4), 2, False),
                                               ((2, 3), 3, False), ((3, 2), 3, False),
                                               ((3, 3), 3, True), ((2, 3), 3, True)])
def test_untruncated_zipup_equals_state_vector(shape, D, exact_svd):
    """Without truncation the boundary-MPS value equals psi.(W psi) of the
    contracted state vector (3x3 and 4x4 networks)."""
    Lx, Ly = shape
    lat = wl.config1_lattice(Lx=Lx, Ly=Ly, D=D)
    chi = CHI_INF
    zw, z1 = exact_value(dense(lat.A), dense(lat.W))
    vw = network_value(lat.sym, lat.A, lat.W, chi, 8, 1, 0, exact_svd=exact_svd)
    ident = wl.identity_pepo(lat.sym, Lx, Ly, lat.A[0][0].legs[0])
    v1 = network_value(lat.sym, lat.A, ident, chi, 8, 1, 0, exact_svd=exact_svd)
    assert vw[0] * math.exp(vw[1]) == pytest.approx(zw, rel=1e-12)
    assert v1[0] * math.exp(v1[1]) == pytest.approx(z1, rel=1e-12)
    assert ratio(vw, v1) == pytest.approx(zw / z1, rel=1e-12)


def test_identity_pepo_is_norm():
    lat = wl.config1_lattice(Lx=3, Ly=3)
    psi = peps_vector(dense(lat.A))
    ident = wl.identity_pepo(lat.sym, 3, 3, lat.A[0][0].legs[0])
    v = network_value(lat.sym, lat.A, ident, CHI_INF, 8, 1, 0)
    assert v[0] == 1
    assert math.exp(v[1]) == pytest.approx(float(psi @ psi), rel=1e-12)


@pytest.mark.parametrize("chi", [2, 4, 7])
def test_scaled_identity_gives_exact_scale_at_any_chi(chi):
    """W = c * 1 (the scale on one site): every truncation of Z_W and Z_1 is
    the same, so <W> = c exactly even when chi truncates heavily. (A bra
    different from the ket avoids the exact degeneracies that the swap
    symmetry of <psi|psi> produces in the singular values.) The cut gaps are
    as small as 5e-3 here, which amplifies rounding: 1e-10 relative."""
    lat = wl.config1_lattice(Lx=4, Ly=4)
    other = wl.config1_lattice(Lx=4, Ly=4, seed=3)
    c = -2.75
    leg = lat.A[0][0].legs[0]
    wc = wl.identity_pepo(lat.sym, 4, 4, leg, scale=c)
    w1 = wl.identity_pepo(lat.sym, 4, 4, leg)
    vc = network_value(lat.sym, lat.A, wc, chi, 3, 1, 5, bra=other.A)
    v1 = network_value(lat.sym, lat.A, w1, chi, 3, 1, 5, bra=other.A)
    assert ratio(vc, v1) == pytest.approx(c, rel=1e-10)


def test_random_pepo_is_symmetric_operator():
    lat = wl.config1_lattice(Lx=2, Ly=2)
    H = pepo_matrix(dense(lat.W))
    assert np.abs(H - H.T).max() <= 1e-13 * np.abs(H).max()


def test_hermiticity_two_different_states():
    """<phi|W|psi> = <psi|W|phi> at chi = infinity for a symmetric W."""
    lat = wl.config1_lattice(Lx=3, Ly=3)
    other = wl.config1_lattice(Lx=3, Ly=3, seed=11)
    a = network_value(lat.sym, lat.A, lat.W, CHI_INF, 8, 1, 0, bra=other.A)
    b = network_value(lat.sym, other.A, lat.W, CHI_INF, 8, 1, 0, bra=lat.A)
    ex, _ = exact_value(dense(lat.A), dense(lat.W), bra=dense(other.A))
    assert a[0] * math.exp(a[1]) == pytest.approx(ex, rel=1e-12)
    assert a[0] * math.exp(a[1]) == pytest.approx(b[0] * math.exp(b[1]), rel=1e-12)


def test_overlap_of_top_and_bottom_halves():
    """Absorbing the top half downwards and the bottom half upwards (rows
    flipped) gives the same network value as the full top-down sweep."""
    lat = wl.config1_lattice(Lx=3, Ly=4, D=2)
    sym = lat.sym
    zw, _ = exact_value(dense(lat.A), dense(lat.W))
    env = wl.trivial_env(sym, 3)
    lg = 0.0
    for y in range(2):
        env, lg, _ = absorb_row(sym, env, lat.A[y], lat.W[y], CHI_INF, 8, 1, 0, row=y,
                                log_norm=lg)

    def flip_ud(t, is_pepo):
        from workloads.tensor import Tensor, Leg
        perm = [0, 1, 2, 3, 5, 4] if is_pepo else [0, 1, 2, 4, 3]
        legs = [t.legs[i] for i in perm]
        legs = [Leg(l.labels, l.dims, l.dir) for l in legs]
        return Tensor.from_blocks(legs, [tuple(int(b[i]) for i in perm) for b in t.blocks],
                                  [t.block(j).transpose(perm) for j in range(t.nblocks)])

    bot = wl.trivial_env(sym, 3)
    lb = 0.0
    for y in (3, 2):
        bot, lb, _ = absorb_row(sym, bot, [flip_ud(a, False) for a in lat.A[y]],
                                [flip_ud(w, True) for w in lat.W[y]], CHI_INF, 8, 1, 0, row=y,
                                log_norm=lb)
    v = overlap(env, bot) * math.exp(lg + lb)
    assert v == pytest.approx(zw, rel=1e-12)
