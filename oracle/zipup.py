"""Row absorption into a boundary MPS by a left-to-right zip-up (oracle).

The environment approximation compresses the bundle of ket, PEPO and bra
legs (dim D w D) of each new row into a bond of dimension chi (Sec. 2); the
bond is truncated with the randomized SVD of Sec. 4. Reading (the paper's
own scheme is a variational fit, Fig. 3): sweep the row from left to right;
at site x the implicit operator M_x (rows (c, dk, dw, db), columns
(b, rk, rw, rb)) is factorised as M_x ~ U R with U an isometry, which becomes
the new environment site, and R is carried to site x+1. R is divided by its
Frobenius norm after every step and the last site is normalised; the
logarithms of those norms are accumulated.
"""
from __future__ import annotations

import math
import numpy as np

from workloads.tensor import Leg, Tensor
from .blocks import BT, to_tensor
from .chain import (SiteOperator, ORDERS, R_NAMES, trivial_remainder, sketch_arrays, flip)
from .rsvd import global_cut, rank_floor, rsvd_adaptive


SIGN_TIE = 1e-5


def fix_signs(U, R):
    """Canonical gauge of a truncated factorisation U R: every column of U is
    flipped (with the matching row of R) so that its leading entry is
    positive, the leading entry being the first (in row order) whose
    magnitude is within a relative 1e-5 of the column's largest. The
    singular vectors of an SVD are unique only up to these signs; fixing them
    makes the environment, and with it the sketch of the next row,
    independent of the SVD routine. The tolerance matters when a symmetry
    (the ket-bra exchange of <psi|W|psi> with a symmetric W) makes entries
    of equal magnitude: it must exceed the rounding of the computation that
    produced U (FP32 storage of the chain intermediates perturbs such ties at
    the 1e-7 level), so that every path picks the same entry of a tied
    pair."""
    U, R = U.copy(), R.copy()
    for c in range(U.shape[1]):
        a = np.abs(U[:, c])
        if a.size == 0:
            continue
        i = int(np.nonzero(a >= a.max() * (1.0 - SIGN_TIE))[0][0])
        if U[i, c] < 0:
            U[:, c] *= -1.0
            R[c, :] *= -1.0
    return U, R


def _row_keys(bt, ji, jpos):
    return sorted(k for k in bt.blocks if k[jpos] == ji)


def _assemble(bt, keys, width):
    if not keys:
        return np.zeros((0, width))
    return np.vstack([bt.blocks[k].reshape(-1, width) for k in keys])


_WORKER_SP = None


def _sector_task(args):
    """Worker side of SiteProblem.workers: one sector, one direction."""
    transpose, J, mat = args
    sp = _WORKER_SP
    widths = [0] * len(sp.sect)
    widths[J] = mat.shape[1]
    rows = sp.n if not transpose else sp.m
    mats = [mat if i == J else np.zeros((rows[i], 0)) for i in range(len(sp.sect))]
    fn = sp._apply_mt if transpose else sp._apply_m
    out_rows = sp.m if not transpose else sp.n
    return J, sp._chunked(fn, mats, out_rows)[J]


class SiteProblem:
    """Glue between SiteOperator (block tensors) and per-sector matrices.

    ``max_cols`` (optional) applies the operator to at most that many columns
    of every sector at a time: the operator acts on each column on its own,
    so this only bounds the memory of the intermediates. ``workers`` > 1
    evaluates the sectors in that many forked processes: M is block
    diagonal over the sectors (sector J's columns reach only sector J's
    rows), and a sector's blocks are summed in the same order whether or not
    the other sectors are present, so the result is the same to the bit.
    Call close() to end the workers."""

    def __init__(self, op: SiteOperator, max_cols=None, workers=1):
        self.op = op
        self.max_cols = max_cols
        self.workers = workers
        self._pool = None
        self.sect = op.sectors()
        legs = op.col_legs()
        self.col_dims = [[op.col_dim(t) for t in tup] for _, tup in self.sect]
        self.n = [int(sum(c)) for c in self.col_dims]
        ys = op.apply(op.omega_bt(self.sect, [1] * len(self.sect)), symbolic=True)
        self.row_keys = [_row_keys(ys, ji, 4) for ji in range(len(self.sect))]
        self.row_dims = [[int(np.prod([ys.legs[n].dims[s] for n, s in zip(ys.names[:4], k[:4])]))
                          for k in keys] for keys in self.row_keys]
        self.m = [int(sum(r)) for r in self.row_dims]
        self.y_legs = ys.legs

    def omega_from_mats(self, mats):
        kd = [m.shape[1] for m in mats]
        arrs = []
        for ji, M in enumerate(mats):
            rows, r0 = [], 0
            for nd in self.col_dims[ji]:
                rows.append(M[r0:r0 + nd]); r0 += nd
            arrs.append(rows)
        bt = self.op.omega_bt(self.sect, kd, arrs)
        return bt

    def y_from_mats(self, mats):
        kd = [m.shape[1] for m in mats]
        jl = self.op.j_leg([J for J, _ in self.sect], kd)
        legs = dict(self.y_legs); legs["j"] = jl
        bt = BT(list(ORDERS[5]), legs, {})
        for ji, M in enumerate(mats):
            r0 = 0
            for key, rd in zip(self.row_keys[ji], self.row_dims[ji]):
                shp = tuple(int(legs[n].dims[s]) for n, s in zip(ORDERS[5][:4], key[:4])) + (kd[ji],)
                bt.blocks[key[:4] + (ji,)] = M[r0:r0 + rd].reshape(shp)
                r0 += rd
        return bt

    def _chunked(self, fn, mats, rows_out):
        kmax = max([m.shape[1] for m in mats] + [0])
        if not self.max_cols or kmax <= self.max_cols:
            return fn(mats)
        parts = []
        for c0 in range(0, kmax, self.max_cols):
            parts.append(fn([m[:, c0:c0 + self.max_cols] for m in mats]))
        return [np.hstack([p[i] for p in parts]) if parts else np.zeros((rows_out[i], 0))
                for i in range(len(mats))]

    def y_struct(self, kvec):
        """Structure (values None) of a row-layout block of vectors with
        per-sector widths ``kvec``; sectors of width 0 have no blocks."""
        jl = self.op.j_leg([J for J, _ in self.sect], kvec)
        legs = dict(self.y_legs); legs["j"] = jl
        bt = BT(list(ORDERS[5]), legs, {})
        for ji in range(len(self.sect)):
            if kvec[ji] > 0:
                for key in self.row_keys[ji]:
                    bt.blocks[key[:4] + (ji,)] = None
        return bt

    def col_blocks(self, kvec):
        """Column-layout block keys (b, rk, rw, rb, j) of M's domain."""
        return {tuple(t) + (ji,) for ji, (_, tuples) in enumerate(self.sect) if kvec[ji] > 0
                for t in tuples}

    def apply_m(self, mats):
        if self.workers > 1:
            return self._parallel(False, mats)
        return self._chunked(self._apply_m, mats, self.m)

    def apply_mt(self, mats):
        if self.workers > 1:
            return self._parallel(True, mats)
        return self._chunked(self._apply_mt, mats, self.n)

    def _parallel(self, transpose, mats):
        global _WORKER_SP
        if self._pool is None:
            import multiprocessing as mp
            _WORKER_SP = self
            self._pool = mp.get_context("fork").Pool(self.workers)
        rows_out = self.n if transpose else self.m
        out = [np.zeros((rows_out[i], m.shape[1])) for i, m in enumerate(mats)]
        # largest sectors first (their chains take longest)
        todo = sorted((J for J, m in enumerate(mats) if m.shape[1] > 0 and rows_out[J] > 0),
                      key=lambda J: -(self.n[J] + self.m[J]) * mats[J].shape[1])
        for J, y in self._pool.imap_unordered(_sector_task, [(transpose, J, mats[J]) for J in todo]):
            out[J] = y
        return out

    def close(self):
        if self._pool is not None:
            self._pool.close()
            self._pool.join()
            self._pool = None

    def _apply_m(self, mats):
        Y = self.op.apply(self.omega_from_mats(mats))
        out = []
        for ji in range(len(self.sect)):
            k = mats[ji].shape[1]
            blocks = []
            for key, rd in zip(self.row_keys[ji], self.row_dims[ji]):
                b = Y.blocks.get(key[:4] + (ji,))
                blocks.append(np.zeros((rd, k)) if b is None else b.reshape(rd, k))
            out.append(np.vstack(blocks) if blocks else np.zeros((0, k)))
        return out

    def _apply_mt(self, mats):
        Z = self.op.apply_t(self.y_from_mats(mats))
        out = []
        for ji, (J, tuples) in enumerate(self.sect):
            k = mats[ji].shape[1]
            blocks = []
            for tup, nd in zip(tuples, self.col_dims[ji]):
                b = Z.blocks.get(tuple(tup) + (ji,))
                blocks.append(np.zeros((nd, k)) if b is None else b.reshape(nd, k))
            out.append(np.vstack(blocks) if blocks else np.zeros((0, k)))
        return out


def _env_site(sp: SiteProblem, U_mats, kept, labels):
    """New environment site [a, k, w, b', b] from the kept U of every sector."""
    op = sp.op
    sel = [ji for ji in range(len(kept)) if kept[ji] > 0]
    jl = Leg(np.array([labels[ji] for ji in sel], dtype=np.int32).reshape(len(sel), -1),
             np.array([kept[ji] for ji in sel], dtype=np.int32), -1)
    legs = [op.R.legs["c"], op.ket.legs["dk"], op.W.legs["dw"], op.bra.legs["db"], jl]
    keys, arrs = [], []
    for newj, ji in enumerate(sel):
        r0 = 0
        for key, rd in zip(sp.row_keys[ji], sp.row_dims[ji]):
            shp = tuple(int(legs[i].dims[s]) for i, s in enumerate(key[:4])) + (kept[ji],)
            keys.append(tuple(key[:4]) + (newj,))
            arrs.append(U_mats[ji][r0:r0 + rd].reshape(shp))
            r0 += rd
    legs = [Leg(l.labels, l.dims, d) for l, d in zip(legs, (1, -1, -1, 1, -1))]
    order = sorted(range(len(keys)), key=lambda i: keys[i])
    return Tensor.from_blocks(legs, [keys[i] for i in order], [arrs[i] for i in order]), sel


def _remainder(sp: SiteProblem, R_mats, kept, labels, sel):
    """R for the next site, names [c, a, lk, lw, lb]."""
    op = sp.op
    cl = Leg(np.array([labels[ji] for ji in sel], dtype=np.int32).reshape(len(sel), -1),
             np.array([kept[ji] for ji in sel], dtype=np.int32), 1)
    legs = {"c": cl, "a": op.T.legs["b"], "lk": op.ket.legs["rk"], "lw": op.W.legs["rw"],
            "lb": op.bra.legs["rb"]}
    bt = BT(list(R_NAMES), legs, {})
    for newj, ji in enumerate(sel):
        c0 = 0
        for tup, nd in zip(sp.sect[ji][1], sp.col_dims[ji]):
            shp = (kept[ji],) + tuple(int(l.dims[s]) for l, s in zip(op.col_legs(), tup))
            bt.blocks[(newj,) + tuple(tup)] = R_mats[ji][:, c0:c0 + nd].reshape(shp)
            c0 += nd
    return bt


def cbe_site(sp, Umats, Rmats, sig, kept, cbe_extra, p, seed, x, row, labels, sv_cut=None):
    """Controlled bond expansion of one truncated site (Sec. 4, Figs. 3-5):
    with kept left space U (the new environment site) and kept right space
    V (the rows of R = U^T M divided by their singular values), the
    ``cbe_extra`` most weighty directions of the discarded part
    (1 - U U^T) M (1 - V^T V), one cut over all sectors. The projectors are
    split as in Fig. 5 and applied to the sketch first (fold):
    Z = M (Om - V^T (V Om)), Y = Z - U (U^T Z); one application (q = 0);
    sketch widths by the rule of ``rsvd`` on the residual's dimensions
    (m_J - kept_J) x (n_J - kept_J); sketch stream 1. Returns the expansion
    Q_J (sign-fixed) with its remainder rows Q_J^T M_J, the counts and the
    passes."""
    V = [r / s[:c][:, None] if c > 0 else r for r, s, c in zip(Rmats, sig, kept)]

    def am(X):
        Z = sp.apply_m([x_ - v.T @ (v @ x_) for x_, v in zip(X, V)])
        return [z - u @ (u.T @ z) for z, u in zip(Z, Umats)]

    def amt(Y):
        Z = sp.apply_mt([y - u @ (u.T @ y) for y, u in zip(Y, Umats)])
        return [z - v.T @ (v @ z) for z, v in zip(Z, V)]

    def omegas(kv):
        oms = sketch_arrays(sp.sect, kv, sp.col_dims, seed, 0, x, row, 1)
        return [np.vstack(o) if len(o) else np.zeros((0, kv[i])) for i, o in enumerate(oms)]

    mr = [mj - c for mj, c in zip(sp.m, kept)]
    nr = [nj - c for nj, c in zip(sp.n, kept)]
    r = rsvd_adaptive(am, amt, mr, nr, cbe_extra, p, 0, omegas, labels, None, sv_cut)
    e = r["kept"]
    Qc = [r["Q"][J] @ r["Ut"][J][:, :e[J]] for J in range(len(e))]
    Qc = [fix_signs(qc, np.zeros((qc.shape[1], 0)))[0] for qc in Qc]
    # the remainder rows of the expansion: Q^T M (not projected)
    Rc = [z.T for z in sp.apply_mt(Qc)]
    return Qc, Rc, e, r["passes"], r["k"]


def absorb_row(sym, T, A, W, chi, p, q, seed, row=0, exact_svd=False, log_norm=0.0,
               bra=None, record=None, max_cols=None, progress=None, sv_cut=None, workers=1,
               cbe_extra=0, stop_after=None):
    """Absorb one row (ket A[x], PEPO W[x]) into the top environment T[x].

    Returns (new environment sites, log_norm, info). With ``exact_svd`` the
    operator of every sector is formed explicitly and factorised by LAPACK
    (truncated SVD), which bounds the error of the randomized version.
    The sketch width of a sector starts from the previous site's kept count
    for the same sector label (the proportional share at the first site and
    for new labels); see ``rsvd``. ``sv_cut`` replaces the rank floor.
    ``stop_after`` = s ends the absorption after the truncation of site s - 1
    (interior sites only; the results of sites 0 .. s-1 are those of the
    whole row, and the returned environment is partial)."""
    L = len(T)
    R = trivial_remainder(sym, T[0], A[0], W[0])
    env = []
    info = dict(sigma=[], kept=[], k=[], m=[], n=[], discarded=[], gap=[], nu=[], passes=[])
    prev_kept = None
    for x in range(L):
        op = SiteOperator(sym, R, T[x], A[x], W[x], bra=None if bra is None else bra[x])
        sp = SiteProblem(op, max_cols, workers)
        if progress:
            progress(f"site {x}: sectors {len(sp.sect)} m {sum(sp.m)} n {sum(sp.n)}")
        labels = [J for J, _ in sp.sect]
        if x == L - 1:
            assert sum(sp.n) == 1, "right boundary legs must have dim 1"
            ji = next(i for i, nn in enumerate(sp.n) if nn == 1)
            mats = [np.zeros((nn, 0)) for nn in sp.n]
            mats[ji] = np.ones((1, 1))
            Y = sp.apply_m(mats)
            sp.close()
            nu = math.sqrt(sum(float(np.sum(y * y)) for y in Y))
            kept = [m.shape[1] for m in Y]
            site, _ = _env_site(sp, [y / nu for y in Y], kept, labels)
            env.append(site)
            log_norm += math.log(nu)
            info["nu"].append(nu)
            break
        if exact_svd:
            S_, U_, B_ = [], [], []
            for ji in range(len(sp.sect)):
                Mf = sp.apply_m([np.eye(sp.n[i]) if i == ji else np.zeros((sp.n[i], 0))
                                 for i in range(len(sp.sect))])[ji]
                if Mf.size == 0:
                    U_.append(np.zeros((Mf.shape[0], 0))); S_.append(np.zeros(0)); B_.append(Mf)
                    continue
                u, s, vt = np.linalg.svd(Mf, full_matrices=False)
                U_.append(u); S_.append(s); B_.append(Mf)
            fl = sv_cut if sv_cut else rank_floor(sp.m, sp.n)
            kept, disc, gap = global_cut(S_, chi, labels, fl)
            Umats = [U_[i][:, :kept[i]] for i in range(len(kept))]
            Rmats = [Umats[i].T @ B_[i] for i in range(len(kept))]
            kvec = [len(s) for s in S_]
        else:
            hint = None if prev_kept is None else [prev_kept.get(tuple(J)) for J in labels]

            def omegas(kv):
                oms = sketch_arrays(sp.sect, kv, sp.col_dims, seed, 0, x, row, 0)
                return [np.vstack(o) if len(o) else np.zeros((0, kv[i])) for i, o in enumerate(oms)]

            r = rsvd_adaptive(sp.apply_m, sp.apply_mt, sp.m, sp.n, chi, p, q, omegas, labels,
                              hint, sv_cut)
            Q, Ut, S_, Bm, kept, kvec = r["Q"], r["Ut"], r["S"], r["B"], r["kept"], r["k"]
            disc, gap = r["discarded"], r["gap"]
            info["passes"].append(r["passes"])
            prev_kept = {tuple(J): c for J, c in zip(labels, kept)}
            Umats = [Q[i] @ Ut[i][:, :kept[i]] for i in range(len(kept))]
            Rmats = [Ut[i][:, :kept[i]].T @ Bm[i] for i in range(len(kept))]
        fixed = [fix_signs(u, r) for u, r in zip(Umats, Rmats)]
        Umats = [f[0] for f in fixed]
        Rmats = [f[1] for f in fixed]
        cbe_passes, cbe_k, cbe_e = [], None, [0] * len(kept)
        if cbe_extra > 0 and not exact_svd:
            Qc, Rc, cbe_e, cbe_passes, cbe_k = cbe_site(sp, Umats, Rmats, S_, kept, cbe_extra, p,
                                                        seed, x, row, labels, sv_cut)
            Umats = [np.hstack([u, qc]) for u, qc in zip(Umats, Qc)]
            Rmats = [np.vstack([r_, rc]) for r_, rc in zip(Rmats, Rc)]
            kept = [c + e for c, e in zip(kept, cbe_e)]
            prev_kept = {tuple(J): c for J, c in zip(labels, kept)}
        info.setdefault("cbe", []).append(dict(kept=list(cbe_e), passes=cbe_passes))
        sp.close()
        site, sel = _env_site(sp, Umats, kept, labels)
        env.append(site)
        R = _remainder(sp, Rmats, kept, labels, sel)
        nu = math.sqrt(R.norm2())
        R.scale(1.0 / nu)
        log_norm += math.log(nu)
        for key, val in (("sigma", S_), ("kept", kept), ("k", kvec), ("m", sp.m), ("n", sp.n),
                         ("discarded", disc), ("gap", gap), ("nu", nu)):
            info[key].append(val)
        if record is not None:
            record.append(dict(x=x, sp=sp, kvec=kvec,
                               passes=info["passes"][-1] if not exact_svd else [(kvec, kept)],
                               cbe_passes=cbe_passes, cbe_kept=list(cbe_e)))
        if stop_after is not None and x + 1 >= stop_after:
            break
    return env, log_norm, info
