"""Seeded synthetic inputs for the boundary-MPS row absorption.

The workloads stand in for the Hubbard benchmarks of the paper (Sec. 5:
U = 8, nearest-neighbour hopping, open boundaries, lattices up to 8x8,
environment bond chi = 500, U(1) and SU(2) symmetric PEPS with D <= 8 / 6).
No trained state exists, so every tensor is random with the stated shapes.

Leg conventions (one fixed reading; the tensor diagrams of Figs. 2-7 are
not available):

* ket site ``A[p, l, r, u, d]``           dirs (+1, +1, -1, +1, -1)
* PEPO site ``W[q, p, l, r, u, d]``       dirs (+1, -1, +1, -1, +1, -1);
  ``q`` is the bra-side physical leg, ``p`` the ket-side one. The bra is the
  ket tensor itself (real data) with every direction reversed.
* environment site ``T[a, k, w, b', b]``  dirs (+1, -1, -1, +1, -1):
  left bond, the three downward legs (ket, PEPO, bra) and the right bond.

Only data generation lives here; nothing in this module contracts or
factorises tensors.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import itertools
import math
import numpy as np

from .tensor import Leg, Tensor

KET_DIRS = (1, 1, -1, 1, -1)
PEPO_DIRS = (1, -1, 1, -1, 1, -1)
ENV_DIRS = (1, -1, -1, 1, -1)


# --------------------------------------------------------------------------
# symmetry descriptors
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Sym:
    """kind: 'none' (no rule), 'u1u1' (labels (dn, 2Sz), abelian flux rule)
    or 'su2' (labels (2j,), multiplet triangle rule, synthetic recoupling
    coefficients). ``coef_seed`` keys the synthetic coefficients;
    ``fermionic`` switches on parity signs per contracted block pair."""
    kind: str = "none"
    coef_seed: int = 0
    fermionic: bool = False

    @property
    def nlab(self):
        return {"none": 1, "u1u1": 2, "su2": 1}[self.kind]

    def zero_label(self):
        return (0,) * self.nlab


def block_allowed(sym: Sym, labels, dirs) -> bool:
    """Which sector tuples the generated inputs populate."""
    if sym.kind == "none":
        return True
    if sym.kind == "u1u1":
        tot = np.zeros(2, dtype=np.int64)
        for lab, d in zip(labels, dirs):
            tot += d * np.asarray(lab, dtype=np.int64)
        return bool(np.all(tot == 0))
    if sym.kind == "su2":
        tj = [int(l[0]) for l in labels]
        s = sum(tj)
        return s % 2 == 0 and 2 * max(tj) <= s
    raise ValueError(sym.kind)


def largest_remainder(weights, total, minimum=1):
    """Integer dims proportional to ``weights`` summing to ``total``; each at
    least ``minimum`` (Hamilton's largest-remainder apportionment)."""
    w = np.asarray(weights, dtype=np.float64)
    n = len(w)
    dims = np.full(n, minimum, dtype=np.int64)
    rest = total - minimum * n
    quota = w / w.sum() * rest
    base = np.floor(quota).astype(np.int64)
    dims += base
    left = rest - int(base.sum())
    order = sorted(range(n), key=lambda i: (-(quota[i] - base[i]), i))
    for i in order[:left]:
        dims[i] += 1
    return [int(v) for v in dims]


# --------------------------------------------------------------------------
# random block-sparse tensors
# --------------------------------------------------------------------------
def random_tensor(sym, legs, rng, scale="numel", allowed=None):
    """All allowed sector tuples, lexicographic, entries N(0,1) scaled by
    1/sqrt(numel) of the whole tensor."""
    tuples = []
    for tup in itertools.product(*[range(l.nsect) for l in legs]):
        labs = [tuple(legs[i].labels[s]) for i, s in enumerate(tup)]
        ok = block_allowed(sym, labs, [l.dir for l in legs]) if allowed is None else allowed(tup)
        if ok:
            tuples.append(tup)
    t = Tensor.from_blocks(legs, tuples)
    t.data[:] = rng.standard_normal(t.data.shape[0])
    if scale == "numel" and t.data.shape[0] > 0:
        t.data /= math.sqrt(t.data.shape[0])
    return t


def with_dirs(legs, dirs):
    return [Leg(l.labels.copy(), l.dims.copy(), int(d)) for l, d in zip(legs, dirs)]


# --------------------------------------------------------------------------
# leg catalogues
# --------------------------------------------------------------------------
def legs_dense(d, D, w, chi):
    return dict(phys=Leg.dense(d), virt=Leg.dense(D), pepo=Leg.dense(w), env=Leg.dense(chi),
                bnd=Leg.dense(1))


def legs_u1u1(chi=256):
    """(dn, 2Sz) sectors, shifted relative to half filling."""
    phys = Leg.make([((-1, 0), 1), ((0, 1), 1), ((0, -1), 1), ((1, 0), 1)])
    virt = Leg.make([((-1, 0), 1), ((0, -1), 1), ((0, 0), 2), ((0, 1), 1), ((1, 0), 1)])
    pepo = Leg.make([((-1, -1), 1), ((-1, 1), 1), ((0, 0), 2), ((1, -1), 1), ((1, 1), 1)])
    labs = [(dn, s) for s in (-1, 0, 1) for dn in (-2, -1, 0, 1, 2)]
    dims = largest_remainder([math.exp(-(dn * dn + s * s) / 8.0) for dn, s in labs], chi)
    order = sorted(range(len(labs)), key=lambda i: labs[i])
    env = Leg.make([(labs[i], dims[i]) for i in order])
    return dict(phys=phys, virt=virt, pepo=pepo, env=env, bnd=Leg.make([((0, 0), 1)]))


def legs_su2(chi=500, virt_mult=(3, 2, 1)):
    """Reduced multiplet legs, labels 2j."""
    phys = Leg.make([((0,), 2), ((1,), 1)])
    virt = Leg.make([((tj,), m) for tj, m in enumerate(virt_mult) if m > 0])
    pepo = Leg.make([((0,), 2), ((1,), 2)])
    tjs = list(range(0, 7))
    dims = largest_remainder([math.exp(-((tj / 2.0) ** 2) / 2.0) for tj in tjs], chi)
    env = Leg.make([((tj,), m) for tj, m in zip(tjs, dims)])
    return dict(phys=phys, virt=virt, pepo=pepo, env=env, bnd=Leg.make([((0,), 1)]))


def legs_u1u1_mini(env_scale=1, virt_scale=1):
    """A small (dn, 2Sz) catalogue for quick tests; ``*_scale`` multiplies the
    sector dimensions without changing the sector structure."""
    phys = Leg.make([((-1, 0), 1), ((0, 1), 1), ((0, -1), 1), ((1, 0), 1)])
    virt = Leg.make([((0, -1), virt_scale), ((0, 0), virt_scale), ((0, 1), virt_scale)])
    pepo = Leg.make([((-1, -1), 1), ((0, 0), 1), ((1, 1), 1)])
    env = Leg.make([((-1, 0), env_scale), ((0, -1), 2 * env_scale), ((0, 0), 2 * env_scale),
                    ((0, 1), 2 * env_scale), ((1, 0), env_scale)])
    return dict(phys=phys, virt=virt, pepo=pepo, env=env, bnd=Leg.make([((0, 0), 1)]))


def legs_su2_mini(env_scale=1, virt_scale=1):
    """A small multiplet catalogue (2j labels) for quick tests."""
    phys = Leg.make([((0,), 2), ((1,), 1)])
    virt = Leg.make([((0,), virt_scale), ((1,), virt_scale)])
    pepo = Leg.make([((0,), 1), ((1,), 1)])
    env = Leg.make([((0,), 2 * env_scale), ((1,), 2 * env_scale), ((2,), env_scale)])
    return dict(phys=phys, virt=virt, pepo=pepo, env=env, bnd=Leg.make([((0,), 1)]))


# --------------------------------------------------------------------------
# Hubbard-shaped comb PEPO (finite state machine)
# --------------------------------------------------------------------------
# bond states: 0 nothing placed yet, 1 term completed, 2..5 pending operator
NONE, DONE = 0, 1
N_STATES = 6


def hubbard_local_ops():
    """Site basis (0, up, dn, updn) with updn = c_up^dag c_dn^dag |0>."""
    cdu = np.zeros((4, 4)); cdu[1, 0] = 1.0; cdu[3, 2] = 1.0
    cdd = np.zeros((4, 4)); cdd[2, 0] = 1.0; cdd[3, 1] = -1.0
    F = np.diag([1.0, -1.0, -1.0, 1.0])
    nu = np.diag([0.0, 1.0, 0.0, 1.0])
    nd = np.diag([0.0, 0.0, 1.0, 1.0])
    return dict(cdu=cdu, cdd=cdd, cu=cdu.T.copy(), cd=cdd.T.copy(), F=F, nu=nu, nd=nd,
                I=np.eye(4))


def hubbard_site_terms(t, U, mu):
    """Emitted operator (times the string F) and the absorbing partner with its
    coefficient, for the hopping -t sum_s [c^dag_s,i c_s,j + h.c.] with i before j."""
    o = hubbard_local_ops()
    emit = [o["cdu"] @ o["F"], o["cdd"] @ o["F"], o["cu"] @ o["F"], o["cd"] @ o["F"]]
    absorb = [-t * o["cu"], -t * o["cd"], t * o["cdu"], t * o["cdd"]]
    onsite = U * (o["nu"] @ o["nd"]) - mu * (o["nu"] + o["nd"])
    return emit, absorb, onsite


def hubbard_transitions(spine):
    """Nonzero (l, r, u, d) -> operator tags for one site type."""
    tr = []
    if not spine:
        tr.append(((NONE, NONE, NONE, NONE), ("I",)))
        tr.append(((NONE, DONE, NONE, NONE), ("onsite",)))
        for k in range(4):
            tr.append(((NONE, 2 + k, NONE, NONE), ("emit", k)))
            tr.append(((NONE, NONE, NONE, 2 + k), ("emit", k)))
            tr.append(((2 + k, DONE, NONE, NONE), ("absorb", k)))
            tr.append(((NONE, DONE, 2 + k, NONE), ("absorb", k)))
        tr.append(((DONE, DONE, NONE, NONE), ("I",)))
    else:
        # spine column: the row state arriving from the left merges with the
        # spine state arriving from above; the right leg is a dummy boundary.
        tr.append(((NONE, 0, NONE, NONE), ("I",)))
        tr.append(((NONE, 0, NONE, DONE), ("onsite",)))
        for k in range(4):
            tr.append(((NONE, 0, NONE, 2 + k), ("emit", k)))
            tr.append(((2 + k, 0, NONE, DONE), ("absorb", k)))
            tr.append(((NONE, 0, 2 + k, DONE), ("absorb", k)))
        tr.append(((DONE, 0, NONE, DONE), ("I",)))
        tr.append(((NONE, 0, DONE, DONE), ("I",)))
    return tr


def hubbard_pepo_site(x, y, Lx, Ly, t=1.0, U=8.0, mu=0.0):
    """Block-sparse PEPO tensor W[q, p, l, r, u, d]; virtual legs carry one
    1-dim sector per FSM state (label = state), boundary legs one fixed state."""
    emit, absorb, onsite = hubbard_site_terms(t, U, mu)
    spine = (x == Lx - 1)
    all_states = [((s,), 1) for s in range(N_STATES)]
    leg_l = Leg.make([((NONE,), 1)]) if x == 0 else Leg.make(all_states)
    leg_r = Leg.make([((0,), 1)]) if spine else Leg.make(all_states)
    leg_u = Leg.make([((NONE,), 1)]) if y == 0 else Leg.make(all_states)
    if y == Ly - 1:
        leg_d = Leg.make([((DONE if spine else NONE,), 1)])
    else:
        leg_d = Leg.make(all_states)
    phys = Leg.dense(4)
    legs = with_dirs([phys, phys, leg_l, leg_r, leg_u, leg_d], PEPO_DIRS)

    def sidx(leg, state):
        hits = np.nonzero(leg.labels[:, 0] == state)[0]
        return int(hits[0]) if hits.size else None

    tuples, arrays = [], []
    for (l, r, u, d), tag in hubbard_transitions(spine):
        s = (0, 0, sidx(leg_l, l), sidx(leg_r, r), sidx(leg_u, u), sidx(leg_d, d))
        if any(v is None for v in s):
            continue
        if tag[0] == "I":
            op = np.eye(4)
        elif tag[0] == "onsite":
            op = onsite
        elif tag[0] == "emit":
            op = emit[tag[1]]
        else:
            op = absorb[tag[1]]
        tuples.append(s)
        arrays.append(op.reshape(4, 4, 1, 1, 1, 1))   # op[q, p]
    order = sorted(range(len(tuples)), key=lambda i: tuples[i])
    return Tensor.from_blocks(legs, [tuples[i] for i in order], [arrays[i] for i in order])


def hubbard_pepo(Lx, Ly, t=1.0, U=8.0, mu=0.0):
    return [[hubbard_pepo_site(x, y, Lx, Ly, t, U, mu) for x in range(Lx)] for y in range(Ly)]


# --------------------------------------------------------------------------
# lattices and single rows
# --------------------------------------------------------------------------
@dataclass
class Lattice:
    sym: Sym
    A: list                       # A[y][x] ket tensors
    W: list                       # W[y][x] PEPO tensors
    Lx: int = 0
    Ly: int = 0


@dataclass
class RowProblem:
    """One row absorption: top environment T[x], ket A[x], PEPO W[x]."""
    sym: Sym
    T: list
    A: list
    W: list
    chi: int
    oversample: int
    power_iters: int
    seed: int = 0
    row: int = 0
    log_norm: float = 0.0
    meta: dict = field(default_factory=dict)


def _virt_leg(cat, on_boundary):
    return cat["bnd"] if on_boundary else cat["virt"]


def peps_site_legs(cat, x, y, Lx, Ly):
    return with_dirs([cat["phys"], _virt_leg(cat, x == 0), _virt_leg(cat, x == Lx - 1),
                      _virt_leg(cat, y == 0), _virt_leg(cat, y == Ly - 1)], KET_DIRS)


def pepo_site_legs(cat, x, y, Lx, Ly):
    pb = lambda b: cat["bnd"] if b else cat["pepo"]
    return with_dirs([cat["phys"], cat["phys"], pb(x == 0), pb(x == Lx - 1), pb(y == 0),
                      pb(y == Ly - 1)], PEPO_DIRS)


def random_peps(sym, cat, Lx, Ly, rng):
    return [[random_tensor(sym, peps_site_legs(cat, x, y, Lx, Ly), rng) for x in range(Lx)]
            for y in range(Ly)]


def random_symmetric_pepo(cat, Lx, Ly, rng):
    """Dense W ~ N(0,1), then symmetrised in (q, p) per site so that the
    network operator is symmetric."""
    out = []
    for y in range(Ly):
        row = []
        for x in range(Lx):
            legs = pepo_site_legs(cat, x, y, Lx, Ly)
            shp = tuple(l.total for l in legs)
            w = rng.standard_normal(shp)
            w = 0.5 * (w + w.transpose(1, 0, 2, 3, 4, 5))
            row.append(Tensor.from_blocks(legs, [(0,) * 6], [w]))
        out.append(row)
    return out


def near_identity_pepo(sym, cat, Lx, Ly, rng, eps=0.5):
    """W = 1 + eps * R per site: R a random tensor on the PEPO legs of the
    catalogue, 1 = delta_{qp} on the first index of the trivial sector of
    every virtual leg. Such an operator (the shape of a short imaginary-time
    step) gives <W> of order one, so its relative error measures the
    contraction rather than a cancellation in a vanishing value."""
    out = []
    for y in range(Ly):
        row = []
        for x in range(Lx):
            legs = pepo_site_legs(cat, x, y, Lx, Ly)
            t = random_tensor(sym, legs, rng)
            t.data *= eps
            z = [int(np.flatnonzero((l.labels == np.asarray(sym.zero_label())).all(axis=1))[0])
                 for l in legs[2:]]
            for s in range(legs[0].nsect):
                i = t.find((s, s) + tuple(z))
                assert i is not None, "identity block must be allowed"
                b = t.block(i)
                b[:, :, 0, 0, 0, 0] += np.eye(int(legs[0].dims[s]))
            row.append(t)
        out.append(row)
    return out


def identity_pepo(sym, Lx, Ly, d_leg, scale=1.0):
    """W = delta_{qp} with trivial (dim-1) virtual legs; ``scale`` multiplies
    the (0, 0) site only."""
    out = []
    bnd = Leg.make([(sym.zero_label(), 1)])
    for y in range(Ly):
        row = []
        for x in range(Lx):
            legs = with_dirs([d_leg, d_leg, bnd, bnd, bnd, bnd], PEPO_DIRS)
            tuples = [(s, s, 0, 0, 0, 0) for s in range(d_leg.nsect)]
            arrs = []
            for s in range(d_leg.nsect):
                m = int(d_leg.dims[s])
                e = np.eye(m).reshape(m, m, 1, 1, 1, 1)
                arrs.append(e * (scale if (x == 0 and y == 0) else 1.0))
            row.append(Tensor.from_blocks(legs, tuples, arrs))
        out.append(row)
    return out


def env_site_legs(cat, ket_up, pepo_up, left_bnd, right_bnd):
    """Legs of a top-environment site whose downward legs meet the given ket
    and PEPO up legs."""
    a = cat["bnd"] if left_bnd else cat["env"]
    b = cat["bnd"] if right_bnd else cat["env"]
    return with_dirs([a, ket_up, pepo_up, ket_up, b], ENV_DIRS)


def random_top_env(sym, cat, A_row, W_row, rng):
    L = len(A_row)
    return [random_tensor(sym, env_site_legs(cat, A_row[x].legs[3], W_row[x].legs[4], x == 0,
                                             x == L - 1), rng) for x in range(L)]


def bottom_closing(env):
    """The environment below the last row: ones on dim-1 legs facing the
    open (dim-1) bundle legs of ``env`` (anything with ``.legs``)."""
    out = []
    for t in env:
        legs = []
        for i, l in enumerate(t.legs):
            if i in (0, 4):
                legs.append(Leg(np.zeros((1, l.labels.shape[1]), dtype=np.int32),
                                np.ones(1, dtype=np.int32), -l.dir))
            else:
                assert l.total == 1, "bundle legs must be closed (dim 1)"
                legs.append(Leg(l.labels.copy(), l.dims.copy(), -l.dir))
        out.append(Tensor.from_blocks(legs, [(0,) * 5], [np.ones((1,) * 5)]))
    return out


def trivial_env(sym, L):
    """The environment above the top row: every leg one dim-1 sector."""
    bnd = Leg.make([(sym.zero_label(), 1)])
    out = []
    for _ in range(L):
        legs = with_dirs([bnd] * 5, ENV_DIRS)
        out.append(Tensor.from_blocks(legs, [(0,) * 5], [np.ones((1, 1, 1, 1, 1))]))
    return out


# --------------------------------------------------------------------------
# the five benchmark configurations
# --------------------------------------------------------------------------
def config1_lattice(Lx=4, Ly=4, d=2, D=3, w=2, seed=0):
    """Plain dense network: A ~ N(0,1)/sqrt(numel), symmetric random W."""
    sym = Sym("none")
    cat = legs_dense(d, D, w, 1)
    rng = np.random.default_rng(seed)
    A = random_peps(sym, cat, Lx, Ly, rng)
    W = random_symmetric_pepo(cat, Lx, Ly, rng)
    return Lattice(sym, A, W, Lx, Ly)


def su2_lattice(Lx, Ly, cat, seed=0, fermionic=True):
    """SU(2)-synthetic lattice: random PEPS and random PEPO blocks on the
    multiplet catalogue ``cat`` (N(0,1)/sqrt(numel) per block)."""
    sym = Sym("su2", coef_seed=seed, fermionic=fermionic)
    rng = np.random.default_rng(seed)
    A = random_peps(sym, cat, Lx, Ly, rng)
    W = [[random_tensor(sym, pepo_site_legs(cat, x, y, Lx, Ly), rng) for x in range(Lx)]
         for y in range(Ly)]
    return Lattice(sym, A, W, Lx, Ly)


def config4_lattice(Lx=8, Ly=8, seed=0):
    """The full 8x8 lattice at the shapes of the headline row: reduced
    D = 6 (multiplicities 3, 2, 1), w = 4, d = 3; absorbed with chi = 500,
    p = 20, q = 2."""
    return su2_lattice(Lx, Ly, legs_su2(500), seed=seed)


def lowrank_su2_lattice(Lx=8, Ly=8, chi=500, seed=0, eps=0.5):
    """An 8x8 SU(2)-synthetic lattice at the leg shapes of the headline row
    (reduced D = 6, w = 4, d = 3, environment catalogue for chi = 500) whose
    boundary MPS is exact at chi: every ket carries its horizontal bonds on
    one state (the first state of the trivial sector; the blocks of the other
    states are zero) and every PEPO its horizontal bonds on the two states of
    the trivial sector, so after y rows the boundary bond is at most 2^y
    <= 256 < chi (vertical legs carry all six states). No truncation is
    needed, and <W> = Z_W / Z_1 depends on the arithmetic only, not on which
    values a cut keeps. The PEPO is 1 + eps R per site as in
    ``near_identity_pepo``; returns (Lattice with W, identity PEPO)."""
    sym = Sym("su2", coef_seed=seed, fermionic=True)
    cat = legs_su2(chi)
    rng = np.random.default_rng(seed)
    zero = lambda leg: int(np.flatnonzero((leg.labels == 0).all(axis=1))[0])

    A = []
    for y in range(Ly):
        row = []
        for x in range(Lx):
            legs = peps_site_legs(cat, x, y, Lx, Ly)
            zl, zr = zero(legs[1]), zero(legs[2])
            allowed = lambda tup, legs=legs, zl=zl, zr=zr: (
                tup[1] == zl and tup[2] == zr and
                block_allowed(sym, [tuple(l.labels[s]) for l, s in zip(legs, tup)],
                              [l.dir for l in legs]))
            t = random_tensor(sym, legs, rng, allowed=allowed)
            for i in range(t.nblocks):
                b = t.block(i)
                b[:, 1:, :, :, :] = 0.0
                b[:, :, 1:, :, :] = 0.0
            row.append(t)
        A.append(row)
    W = []
    for y in range(Ly):
        row = []
        for x in range(Lx):
            legs = pepo_site_legs(cat, x, y, Lx, Ly)
            zl, zr = zero(legs[2]), zero(legs[3])
            allowed = lambda tup, legs=legs, zl=zl, zr=zr: (
                tup[2] == zl and tup[3] == zr and
                block_allowed(sym, [tuple(l.labels[s]) for l, s in zip(legs, tup)],
                              [l.dir for l in legs]))
            t = random_tensor(sym, legs, rng, allowed=allowed)
            t.data *= eps
            z = [zero(l) for l in legs[2:]]
            for s in range(legs[0].nsect):
                i = t.find((s, s) + tuple(z))
                assert i is not None, "identity block must be present"
                t.block(i)[:, :, 0, 0, 0, 0] += np.eye(int(legs[0].dims[s]))
            row.append(t)
        W.append(row)
    lat = Lattice(sym, A, W, Lx, Ly)
    return lat, identity_pepo(sym, Lx, Ly, cat["phys"])


LOWRANK_PARAMS = dict(chi=500, oversample=20, power_iters=2, seed=0)


def config1_params():
    return dict(chi=32, oversample=8, power_iters=1, seed=0)


def config2_row(Lx=8, Ly=8, y=3, d=4, D=6, chi=128, seed=0, t=1.0, U=8.0, mu=0.0,
                oversample=8, power_iters=1):
    """Dense PEPS, Hubbard comb PEPO (w = 6), random dense environment."""
    sym = Sym("none")
    cat = legs_dense(d, D, 6, chi)
    rng = np.random.default_rng(seed)
    A = [random_tensor(sym, peps_site_legs(cat, x, y, Lx, Ly), rng) for x in range(Lx)]
    W = [hubbard_pepo_site(x, y, Lx, Ly, t, U, mu) for x in range(Lx)]
    T = random_top_env(sym, cat, A, W, rng)
    return RowProblem(sym, T, A, W, chi, oversample, power_iters, seed, y,
                      meta=dict(config=2, Lx=Lx, Ly=Ly, d=d, D=D, w=6))


def config3_row(Lx=8, Ly=8, y=3, chi=256, seed=0, oversample=8, power_iters=1):
    """U(1)xU(1) block-sparse row, random blocks, fermionic signs."""
    sym = Sym("u1u1", coef_seed=seed, fermionic=True)
    cat = legs_u1u1(chi)
    rng = np.random.default_rng(seed)
    A = [random_tensor(sym, peps_site_legs(cat, x, y, Lx, Ly), rng) for x in range(Lx)]
    W = [random_tensor(sym, pepo_site_legs(cat, x, y, Lx, Ly), rng) for x in range(Lx)]
    T = random_top_env(sym, cat, A, W, rng)
    return RowProblem(sym, T, A, W, chi, oversample, power_iters, seed, y,
                      meta=dict(config=3, Lx=Lx, Ly=Ly))


def config4_row(Lx=8, Ly=8, y=3, chi=500, seed=0, oversample=20, power_iters=2,
                virt_mult=(3, 2, 1)):
    """SU(2)-reduced synthetic row: multiplet legs, synthetic recoupling
    coefficients and parity signs per contracted block pair."""
    sym = Sym("su2", coef_seed=seed, fermionic=True)
    cat = legs_su2(chi, virt_mult)
    rng = np.random.default_rng(seed)
    A = [random_tensor(sym, peps_site_legs(cat, x, y, Lx, Ly), rng) for x in range(Lx)]
    W = [random_tensor(sym, pepo_site_legs(cat, x, y, Lx, Ly), rng) for x in range(Lx)]
    T = random_top_env(sym, cat, A, W, rng)
    return RowProblem(sym, T, A, W, chi, oversample, power_iters, seed, y,
                      meta=dict(config=4, Lx=Lx, Ly=Ly))


def small_row(kind="none", L=3, d=2, D=2, w=2, chi=4, seed=0, oversample=2, power_iters=1,
              interior=True, env_scale=1, virt_scale=1):
    """A small row of the requested symmetry for quick tests. For the dense
    kind ``chi`` is the environment bond; for the symmetric kinds the
    environment legs come from the mini catalogues (scaled by
    ``env_scale``) and ``chi`` is only the truncation target."""
    if kind == "none":
        sym, cat = Sym("none"), legs_dense(d, D, w, chi)
    elif kind == "u1u1":
        sym = Sym("u1u1", coef_seed=seed, fermionic=True)
        cat = legs_u1u1_mini(env_scale, virt_scale)
    elif kind == "su2":
        sym = Sym("su2", coef_seed=seed, fermionic=True)
        cat = legs_su2_mini(env_scale, virt_scale)
    else:
        raise ValueError(kind)
    Ly = 3 if interior else 1
    y = 1 if interior else 0
    rng = np.random.default_rng(seed)
    A = [random_tensor(sym, peps_site_legs(cat, x, y, L, Ly), rng) for x in range(L)]
    W = [random_tensor(sym, pepo_site_legs(cat, x, y, L, Ly), rng) for x in range(L)]
    T = random_top_env(sym, cat, A, W, rng) if interior else trivial_env(sym, L)
    return RowProblem(sym, T, A, W, chi, oversample, power_iters, seed, y,
                      meta=dict(config="small", kind=kind, cat=cat))


def heff_inputs(kind="none", seed=0, d=2, D=2, w=2, chi=3, env_scale=1, virt_scale=1,
                symmetric=False):
    """Random inputs of the effective single-site operator of Fig. 2(b) at an
    interior site: ket A[p, l, r, u, d], PEPO W[q, p, l, r, u, d], top
    boundary site T[a, k, w, b', b], left environment L[a, k, w, b', c],
    bottom boundary site B[c, k, w, b', d] and right environment
    R[b, k, w, b', d] (k, w, b' the ket, PEPO and bra legs they face).
    Directions follow the row conventions (each shared leg opposite on its
    two tensors). ``symmetric`` (dense kind only) makes every environment
    symmetric under the exchange of its ket and bra legs and W symmetric in
    (q, p), so that the operator is symmetric."""
    if kind == "none":
        sym, cat = Sym("none"), legs_dense(d, D, w, chi)
    elif kind == "u1u1":
        sym, cat = Sym("u1u1", coef_seed=seed, fermionic=True), legs_u1u1_mini(env_scale, virt_scale)
    elif kind == "su2":
        sym, cat = Sym("su2", coef_seed=seed, fermionic=True), legs_su2_mini(env_scale, virt_scale)
    else:
        raise ValueError(kind)
    rng = np.random.default_rng(seed)
    A = random_tensor(sym, peps_site_legs(cat, 1, 1, 3, 3), rng)
    W = random_tensor(sym, pepo_site_legs(cat, 1, 1, 3, 3), rng)
    env = cat["env"]
    d_ = lambda leg, dr: Leg(leg.labels.copy(), leg.dims.copy(), int(dr))
    T = random_tensor(sym, env_site_legs(cat, A.legs[3], W.legs[4], False, False), rng)
    L = random_tensor(sym, [d_(env, -1), d_(A.legs[1], -1), d_(W.legs[2], -1), d_(A.legs[1], 1),
                            d_(env, 1)], rng)
    B = random_tensor(sym, [d_(env, -1), d_(A.legs[4], 1), d_(W.legs[5], 1), d_(A.legs[4], -1),
                            d_(env, 1)], rng)
    R = random_tensor(sym, [d_(env, 1), d_(A.legs[2], 1), d_(W.legs[3], 1), d_(A.legs[2], -1),
                            d_(env, -1)], rng)
    if symmetric:
        assert kind == "none", "symmetric inputs are dense"
        for t in (T, L, B, R):
            x = t.block(0)
            x[...] = 0.5 * (x + x.transpose(0, 3, 2, 1, 4))
        w_ = W.block(0)
        w_[...] = 0.5 * (w_ + w_.transpose(1, 0, 2, 3, 4, 5))
    return dict(sym=sym, cat=cat, A=A, W=W, T=T, L=L, B=B, R=R)


def random_bottom_env(sym, top_env, bond_leg, rng):
    """A random environment whose bundle legs face those of ``top_env``
    (same sectors, reversed directions) with bonds ``bond_leg`` (dim 1 at the
    two ends). Used to read a gauge-invariant number off a new environment."""
    L = len(top_env)
    bnd = Leg.make([(sym.zero_label(), 1)])
    out = []
    for x, t in enumerate(top_env):
        a = bnd if x == 0 else bond_leg
        b = bnd if x == L - 1 else bond_leg
        legs = [Leg(a.labels, a.dims, -1)] + [t.legs[i].flipped() for i in (1, 2, 3)] + \
               [Leg(b.labels, b.dims, 1)]
        out.append(random_tensor(sym, legs, rng))
    return out


def decaying_matrix(m, n, rng, decay=32.0):
    """An m x n matrix A diag(s) B with Gaussian A (m x r), B (r x n),
    r = min(m, n) and s_i = exp(-i / decay): a decaying spectrum of the kind
    a truncation acts on (stand-in for the explicit per-sector matrices of a
    bond-expansion step)."""
    r = min(m, n)
    s = np.exp(-np.arange(r) / decay)
    A = rng.standard_normal((m, r)) / math.sqrt(m)
    B = rng.standard_normal((r, n)) / math.sqrt(n)
    return (A * s) @ B


CONFIG5 = dict(chi=256, oversample=8, power_iters=1, cbe_extra=26, cbe_oversample=8, decay=32.0)
