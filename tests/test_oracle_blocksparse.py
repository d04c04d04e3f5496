"""Pins of the oracle's block-sparse chain: dense embedding, a brute-force
sum with per-pair scalars, the exact transpose, the block-diagonal sector
structure, the comb PEPO and the flop count (no GPU)."""
import itertools
import math

import numpy as np
import pytest

import workloads as wl
from workloads.tensor import Leg, Tensor
from oracle.blocks import BT, from_tensor
from oracle.chain import SiteOperator, trivial_remainder, ORDERS, flip
from oracle.exact import pepo_matrix
from oracle.zipup import SiteProblem
from oracle.flops import chain_flops, chain_flops_t
from oracle.rng import splitmix64_mix


def random_remainder(sym, row, x, cat_c, rng):
    """A random R[c, a, lk, lw, lb] obeying the flux rule of ``sym``."""
    T, A, W = row.T[x], row.A[x], row.W[x]
    legs = [cat_c, flip(T.legs[0]), flip(A.legs[1]), flip(W.legs[2]), A.legs[1]]
    legs = [Leg(l.labels, l.dims, d) for l, d in zip(legs, (1, -1, -1, -1, 1))]
    t = wl.random_tensor(sym, legs, rng)
    return BT(["c", "a", "lk", "lw", "lb"], dict(zip(["c", "a", "lk", "lw", "lb"], legs)),
              t.to_dict())


def sector_offsets(leg):
    return np.concatenate([[0], np.cumsum(leg.dims)[:-1]]).astype(int)


def dense_index_rows(legs, keys):
    """Flat dense indices (row-major over ``legs``) of the rows of the
    stacked blocks ``keys`` (each block row-major)."""
    tot = [l.total for l in legs]
    out = []
    for key in keys:
        ranges = [range(sector_offsets(l)[s], sector_offsets(l)[s] + l.dims[s])
                  for l, s in zip(legs, key)]
        for idx in itertools.product(*ranges):
            out.append(int(np.ravel_multi_index(idx, tot)))
    return np.array(out, dtype=np.int64)


def explicit_sector_matrices(sp):
    mats = []
    for ji in range(len(sp.sect)):
        cols = [np.eye(sp.n[i]) if i == ji else np.zeros((sp.n[i], 0)) for i in range(len(sp.sect))]
        mats.append(sp.apply_m(cols)[ji])
    return mats


def u1_problem(fermionic):
    row = wl.small_row("u1u1", L=3, chi=15, seed=2)
    sym = wl.Sym("u1u1", coef_seed=2, fermionic=fermionic)
    rng = np.random.default_rng(5)
    R = random_remainder(sym, row, 1, row.meta["cat"]["env"], rng)
    return sym, row, R


def test_u1_blocks_equal_dense_embedding_and_are_block_diagonal():
    """U(1)xU(1) without signs: the block engine's M_J equals the densely
    embedded operator restricted to sector J, and the dense operator has no
    entries between different sectors."""
    sym, row, R = u1_problem(False)
    x = 1
    op = SiteOperator(sym, R, row.T[x], row.A[x], row.W[x])
    sp = SiteProblem(op)
    mats = explicit_sector_matrices(sp)
    # dense operator from the embedded tensors
    Td, Ad, Wd = row.T[x].to_dense(), row.A[x].to_dense(), row.W[x].to_dense()
    Rd = Tensor.from_blocks([R.legs[n] for n in R.names], sorted(R.blocks),
                            [R.blocks[k] for k in sorted(R.blocks)]).to_dense()
    Md = np.einsum("calmn,atwsb,plrtd,qpmuwe,qnvsf->cdefbruv", Rd, Td, Ad, Wd, Ad, optimize=True)
    Md = Md.reshape(np.prod(Md.shape[:4]), -1)
    row_legs = op.row_legs()
    col_legs = op.col_legs()
    used_r, used_c = np.zeros(Md.shape[0], bool), np.zeros(Md.shape[1], bool)
    for ji, (J, tuples) in enumerate(sp.sect):
        ri = dense_index_rows(row_legs, [k[:4] for k in sp.row_keys[ji]])
        ci = dense_index_rows(col_legs, tuples)
        assert np.allclose(mats[ji], Md[np.ix_(ri, ci)], rtol=1e-13, atol=1e-15)
        assert not used_r[ri].any(), "a row appears in two sectors"
        used_r[ri] = True
        used_c[ci] = True
    mask = np.zeros_like(Md, dtype=bool)
    for ji, (J, tuples) in enumerate(sp.sect):
        ri = dense_index_rows(row_legs, [k[:4] for k in sp.row_keys[ji]])
        ci = dense_index_rows(col_legs, tuples)
        mask[np.ix_(ri, ci)] = True
    assert np.abs(Md[~mask]).max() == 0.0


def _alpha_ref(sym, step, xlabs, tlabs, x_shared_mask, t_shared_mask):
    """The per-pair scalar, restated: synthetic coefficient from a fold of
    SplitMix64 over (step, labels) and the parity sign."""
    a = 1.0
    if sym.kind == "su2":
        h = sym.coef_seed
        for w in [step] + [v for l in xlabs for v in l] + [v for l in tlabs for v in l]:
            h = splitmix64_mix((h + 0x9E3779B97F4A7C15 + (w % 2 ** 64)) % 2 ** 64)
        a = 2.0 * ((h >> 11) * 2.0 ** -53) - 1.0
    if sym.fermionic:
        par = (lambda l: l[0] & 1) if sym.kind == "su2" else (lambda l: l[1] & 1)
        px = sum(par(l) for l, s in zip(xlabs, x_shared_mask) if not s)
        pt = sum(par(l) for l, s in zip(tlabs, t_shared_mask) if s)
        if (px * pt) % 2:
            a = -a
    return a


def test_su2_chain_equals_brute_force_sum():
    """Every leg two 1-dim sectors (2j = 0, 1): the chain equals the direct
    sum over all index assignments of the product of the six tensors times
    the product of the five per-step scalars."""
    sym = wl.Sym("su2", coef_seed=9, fermionic=True)
    two = Leg.make([((0,), 1), ((1,), 1)])
    rng = np.random.default_rng(1)
    A = wl.random_tensor(sym, wl.configs.with_dirs([two] * 5, wl.KET_DIRS), rng)
    W = wl.random_tensor(sym, wl.configs.with_dirs([two] * 6, wl.PEPO_DIRS), rng)
    T = wl.random_tensor(sym, wl.configs.with_dirs([two] * 5, wl.ENV_DIRS), rng)
    Rt = wl.random_tensor(sym, [two] * 5, rng)
    R = BT(["c", "a", "lk", "lw", "lb"], dict(zip(["c", "a", "lk", "lw", "lb"], Rt.legs)), Rt.to_dict())
    op = SiteOperator(sym, R, T, A, W)
    sect = op.sectors()
    nJ = len(sect)
    om = op.omega_bt(sect, [1] * nJ, [[rng.standard_normal((1, 1)) for _ in tup] for _, tup in sect])
    Y = op.apply(om)
    # dense arrays: every sector has dim 1, so index = sector index
    Rd = np.zeros((2,) * 5); Td = T.to_dense(); Ad = A.to_dense(); Wd = W.to_dense()
    for k, v in R.blocks.items():
        Rd[k] = v.ravel()[0]
    Od = np.zeros((2, 2, 2, 2, nJ))
    for k, v in om.blocks.items():
        Od[k] = v.ravel()[0]
    Jlab = [J for J, _ in sect]
    names = ["c", "a", "lk", "lw", "lb", "tk", "tw", "tb", "b", "p", "q", "rk", "rw", "rb",
             "dk", "dw", "db", "j"]
    dims = [2] * 17 + [nJ]
    grids = np.indices(dims).reshape(len(dims), -1)
    ix = dict(zip(names, grids))
    lab = lambda n, v: (int(v),) if n != "j" else tuple(Jlab[int(v)])
    tens = [(Td, ["a", "tk", "tw", "tb", "b"]), (Ad, ["p", "lk", "rk", "tk", "dk"]),
            (Wd, ["q", "p", "lw", "rw", "tw", "dw"]), (Ad, ["q", "lb", "rb", "tb", "db"]),
            (Rd, ["c", "a", "lk", "lw", "lb"])]
    prod = Od[tuple(ix[n] for n in ORDERS[0])]
    for d, nm in tens:
        prod = prod * d[tuple(ix[n] for n in nm)]
    nz = np.nonzero(prod)[0]
    alpha = np.ones(nz.size)
    for s, (d, nm) in enumerate(tens):
        xn = ORDERS[s]
        shared = set(xn) & set(nm)
        cache = {}
        for t, e in enumerate(nz):
            key = tuple(int(ix[n][e]) for n in xn + nm)
            if key not in cache:
                xl = [lab(n, ix[n][e]) for n in xn]
                tl = [lab(n, ix[n][e]) for n in nm]
                cache[key] = _alpha_ref(sym, s + 1, xl, tl, [n in shared for n in xn],
                                        [n in shared for n in nm])
            alpha[t] *= cache[key]
    want = np.zeros((2, 2, 2, 2, nJ))
    np.add.at(want, tuple(ix[n][nz] for n in ORDERS[5]), prod[nz] * alpha)
    got = np.zeros_like(want)
    for k, v in Y.blocks.items():
        got[k] = v.ravel()[0]
    assert np.abs(want).max() > 0
    assert np.allclose(got, want, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("kind", ["u1u1", "su2", "none"])
def test_transpose_chain_is_exact_transpose(kind):
    """<Z, M Om> = <M^T Z, Om> for random Om, Z, including the synthetic
    coefficients and parity signs."""
    row = wl.small_row(kind, L=3, chi=15, seed=4)
    rng = np.random.default_rng(0)
    R = random_remainder(row.sym, row, 1, row.meta["cat"]["env"], rng)
    op = SiteOperator(row.sym, R, row.T[1], row.A[1], row.W[1])
    sp = SiteProblem(op)
    k = [3] * len(sp.sect)
    Om = [rng.standard_normal((n, kk)) for n, kk in zip(sp.n, k)]
    Z = [rng.standard_normal((m, kk)) for m, kk in zip(sp.m, k)]
    MO = sp.apply_m(Om)
    MZ = sp.apply_mt(Z)
    lhs = sum(float(np.sum(z * y)) for z, y in zip(Z, MO))
    rhs = sum(float(np.sum(w * o)) for w, o in zip(MZ, Om))
    assert lhs == pytest.approx(rhs, rel=1e-12)
    assert abs(lhs) > 0


def test_dense_flop_count_closed_form():
    """Dense legs: one application costs
    2 [2 chi^2 k (DwD)^2 + 2 chi k d w^2 D^6 + chi k D^4 d^2 w^4]."""
    d, D, w, chi, k = 2, 3, 2, 5, 4
    cat = wl.legs_dense(d, D, w, chi)
    rng = np.random.default_rng(0)
    legsA = wl.configs.with_dirs([cat["phys"], cat["virt"], cat["virt"], cat["virt"], cat["virt"]],
                                 wl.KET_DIRS)
    legsW = wl.configs.with_dirs([cat["phys"], cat["phys"]] + [cat["pepo"]] * 4, wl.PEPO_DIRS)
    A = wl.random_tensor(wl.Sym(), legsA, rng)
    W = wl.random_tensor(wl.Sym(), legsW, rng)
    T = wl.random_tensor(wl.Sym(), wl.configs.env_site_legs(cat, A.legs[3], W.legs[4], False, False), rng)
    Rt = wl.random_tensor(wl.Sym(), [cat["env"], T.legs[0], A.legs[1], W.legs[2], A.legs[1]], rng)
    R = BT(["c", "a", "lk", "lw", "lb"], dict(zip(["c", "a", "lk", "lw", "lb"], Rt.legs)), Rt.to_dict())
    sp = SiteProblem(SiteOperator(wl.Sym(), R, T, A, W))
    S = D * w * D
    want = 2 * (2 * chi ** 2 * k * S ** 2 + 2 * chi * k * d * w ** 2 * D ** 6
                + chi * k * D ** 4 * d ** 2 * w ** 4)
    assert chain_flops(sp, [k]) == want
    # the mirrored chain has the transposed products of the same shapes
    assert chain_flops_t(sp, [k]) == want


def spin_ops(tj):
    """S_z and S_+ of spin j = tj / 2 in the basis m = j, j-1, ..., -j."""
    j = tj / 2.0
    ms = j - np.arange(tj + 1)
    sz = np.diag(ms)
    sp = np.zeros((tj + 1, tj + 1))
    for i in range(1, tj + 1):          # S_+ |m> = sqrt(j(j+1) - m(m+1)) |m+1>
        m = ms[i]
        sp[i - 1, i] = math.sqrt(j * (j + 1) - m * (m + 1))
    return sz, sp


def total_spins(tjs):
    """The set of 2J whose multiplets occur in the product of spins tjs/2:
    eigenvalues J(J+1) of the total S^2 = S_z^2 + (S_+ S_- + S_- S_+)/2 built
    from the spin matrices of every factor."""
    dims = [tj + 1 for tj in tjs]
    N = int(np.prod(dims))
    Sz, Sp = np.zeros((N, N)), np.zeros((N, N))
    for i, tj in enumerate(tjs):
        sz, sp = spin_ops(tj)
        left, right = np.eye(int(np.prod(dims[:i]))), np.eye(int(np.prod(dims[i + 1:])))
        Sz += np.kron(np.kron(left, sz), right)
        Sp += np.kron(np.kron(left, sp), right)
    S2 = Sz @ Sz + 0.5 * (Sp @ Sp.T + Sp.T @ Sp)
    lam = np.linalg.eigvalsh(S2)
    twoJ = np.rint(np.sqrt(1.0 + 4.0 * np.maximum(lam, 0)) - 1.0).astype(int)
    assert np.allclose(twoJ / 2.0 * (twoJ / 2.0 + 1.0), lam, atol=1e-8)
    return set(int(v) for v in twoJ)


def test_su2_column_sectors_are_the_spins_of_the_coupled_legs():
    """Config-4 catalogue (environment 2j = 0..6, virtual 2j <= 2, PEPO
    2j <= 1): the sketch sectors J of every column tuple (b, rk, rw, rb) are
    exactly the total spins of the product of its four spins, found by
    diagonalising the total S^2 of the spin matrices (not by the triangle
    rule the operator uses)."""
    sym = wl.Sym("su2", coef_seed=1, fermionic=True)
    cat = wl.legs_su2(14)
    rng = np.random.default_rng(0)
    A = wl.random_tensor(sym, wl.configs.peps_site_legs(cat, 1, 1, 3, 3), rng)
    W = wl.random_tensor(sym, wl.configs.pepo_site_legs(cat, 1, 1, 3, 3), rng)
    T = wl.random_tensor(sym, wl.configs.env_site_legs(cat, A.legs[3], W.legs[4], False, False), rng)
    row = wl.RowProblem(sym, [T] * 3, [A] * 3, [W] * 3, 14, 2, 1)
    R = random_remainder(sym, row, 1, cat["env"], rng)
    op = SiteOperator(sym, R, T, A, W)
    legs = op.col_legs()
    assert [int(l[0]) for l in legs[0].labels] == list(range(7))
    got = {}
    for J, tuples in op.sectors():
        for t in tuples:
            got.setdefault(tuple(t), set()).add(int(J[0]))
    checked = 0
    for t in itertools.product(*[range(l.nsect) for l in legs]):
        tjs = [int(legs[i].labels[s][0]) for i, s in enumerate(t)]
        assert got.get(tuple(t), set()) == total_spins(tjs), (t, tjs)
        checked += 1
    assert checked == 7 * 3 * 2 * 3


# ---------------------------------------------------------------------------
# the Hubbard-shaped comb PEPO
# ---------------------------------------------------------------------------
def kron_all(ops):
    out = np.ones((1, 1))
    for o in ops:
        out = np.kron(out, o)
    return out


def jw_hubbard_chain(L, t, U, mu):
    """1D Hubbard chain with exact Jordan-Wigner strings (site-major order,
    up before down inside a site)."""
    o = wl.hubbard_local_ops()
    I, F = o["I"], o["F"]

    def c(i, which):
        return kron_all([F] * i + [o[which]] + [I] * (L - i - 1))

    H = np.zeros((4 ** L, 4 ** L))
    for i in range(L):
        nu, nd = c(i, "cdu") @ c(i, "cu"), c(i, "cdd") @ c(i, "cd")
        H += U * nu @ nd - mu * (nu + nd)
    for i in range(L - 1):
        for s in ("u", "d"):
            hop = c(i, "cd" + s) @ c(i + 1, "c" + s)
            H += -t * (hop + hop.T)
    return H


def local_hop_hubbard(Lx, Ly, t, U, mu):
    """Nearest-neighbour Hubbard with the local form of every bond, i before
    j in row-major order: -t sum_s [(c+_s F)_i (c_s)_j - (c_s F)_i (c+_s)_j]
    (exact Jordan-Wigner for in-row neighbours, intervening strings dropped
    for vertical ones)."""
    o = wl.hubbard_local_ops()
    N = Lx * Ly
    I = o["I"]

    def at(ops):
        return kron_all([ops.get(i, I) for i in range(N)])

    H = np.zeros((4 ** N, 4 ** N))
    onsite = U * o["nu"] @ o["nd"] - mu * (o["nu"] + o["nd"])
    for i in range(N):
        H += at({i: onsite})
    bonds = []
    for y in range(Ly):
        for x in range(Lx):
            i = y * Lx + x
            if x + 1 < Lx:
                bonds.append((i, i + 1))
            if y + 1 < Ly:
                bonds.append((i, i + Lx))
    for i, j in bonds:
        for s in ("u", "d"):
            H += -t * at({i: o["cd" + s] @ o["F"], j: o["c" + s]})
            H += t * at({i: o["c" + s] @ o["F"], j: o["cd" + s]})
    return H


def comb_matrix(Lx, Ly, t=1.0, U=8.0, mu=0.3):
    Ws = wl.hubbard_pepo(Lx, Ly, t, U, mu)
    return pepo_matrix([[w.to_dense() for w in row] for row in Ws])


@pytest.mark.parametrize("L", [2, 3, 4])
def test_comb_pepo_chain_is_jordan_wigner_hubbard(L):
    H = comb_matrix(L, 1)
    ref = jw_hubbard_chain(L, 1.0, 8.0, 0.3)
    assert np.abs(H - ref).max() < 1e-12
    assert np.abs(H - H.T).max() < 1e-12


@pytest.mark.parametrize("shape", [(2, 2), (3, 2), (2, 3), (1, 3)])
def test_comb_pepo_lattice_equals_local_bond_form(shape):
    Lx, Ly = shape
    H = comb_matrix(Lx, Ly)
    ref = local_hop_hubbard(Lx, Ly, 1.0, 8.0, 0.3)
    assert np.abs(H - ref).max() < 1e-12
    assert np.abs(H - H.T).max() < 1e-12


def test_comb_pepo_interior_site_has_19_transitions():
    W = wl.hubbard_pepo_site(2, 2, 5, 5)
    assert W.nblocks == 19


def test_sector_parallel_and_chunked_evaluation_is_bitwise_equal():
    """The oracle's memory and time bounding (column chunks, sectors in
    worker processes) changes no bit of a row absorption: each sector's
    blocks are summed in the same order either way."""
    from oracle.zipup import absorb_row
    row = wl.small_row("su2", L=4, seed=3, oversample=4, power_iters=1, env_scale=3, virt_scale=2)
    e1, l1, i1 = absorb_row(row.sym, row.T, row.A, row.W, 10, 4, 1, 17, row=row.row)
    e2, l2, i2 = absorb_row(row.sym, row.T, row.A, row.W, 10, 4, 1, 17, row=row.row, workers=3,
                            max_cols=2)
    assert l1 == l2
    assert i1["kept"] == i2["kept"]
    for s1, s2 in zip(i1["sigma"], i2["sigma"]):
        assert all(np.array_equal(a, b) for a, b in zip(s1, s2))
    for a, b in zip(e1, e2):
        assert np.array_equal(a.data, b.data)
