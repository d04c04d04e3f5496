"""ctypes binding of the C ABI in include/fpeps.h (argument marshalling only).

Tensor structure (legs, blocks) lives in numpy arrays on the host; tensor
data lives in torch float64 tensors on the GPU. Every computation happens in
the gfx950 library ``libfpeps.so``; when it cannot be loaded the binding
raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import numpy as np

# workspace allocator callbacks of fpeps_set_allocator
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfpeps.so")

FPEPS_OK = 0
STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_SHAPE", -3: "ERR_SYMMETRY", -4: "ERR_NOMEM",
          -5: "ERR_HIP", -6: "ERR_NUMERIC", -7: "ERR_CAPACITY", -8: "ERR_UNSUPPORTED",
          -9: "ERR_NODEVICE"}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
SYM = {"none": 0, "u1u1": 1, "su2": 2}
FLAG_NO_GRAPH, FLAG_CHECK_FINITE, FLAG_TIME_KERNELS, FLAG_ONE_STREAM = 1, 2, 4, 8


class FpepsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class CTensor(C.Structure):
    _fields_ = [("nlegs", C.c_int32), ("nlab", C.c_int32), ("max_sect", C.c_int32),
                ("nsect", C.POINTER(C.c_int32)), ("dirs", C.POINTER(C.c_int32)),
                ("labels", C.POINTER(C.c_int32)), ("dims", C.POINTER(C.c_int32)),
                ("nblocks", C.c_int32), ("max_blocks", C.c_int32),
                ("block_sect", C.POINTER(C.c_int32)), ("block_off", C.POINTER(C.c_int64)),
                ("data", C.c_void_p), ("nelem", C.c_int64), ("max_elem", C.c_int64)]


class COpts(C.Structure):
    _fields_ = [("chi", C.c_int32), ("oversample", C.c_int32), ("power_iters", C.c_int32),
                ("cbe_extra", C.c_int32), ("seed", C.c_uint64), ("row", C.c_int32),
                ("precision", C.c_int32), ("symmetry", C.c_int32), ("fermionic", C.c_int32),
                ("coef_seed", C.c_uint64), ("slice_budget", C.c_int64), ("flags", C.c_uint32),
                ("tag", C.c_int32), ("sv_cut", C.c_double)]


class CReport(C.Structure):
    _fields_ = [("alg_flops", C.c_double), ("seconds", C.c_double),
                ("discarded_weight", C.c_double), ("min_rel_gap", C.c_double),
                ("log_norm", C.c_double), ("peak_workspace", C.c_double),
                ("kept_total", C.c_int32), ("nslices", C.c_int32), ("fallbacks", C.c_uint32),
                ("required_blocks", C.c_int32), ("required_elem", C.c_int64),
                ("required_sect", C.c_int32), ("kernel_launches", C.c_int32),
                ("kernel_seconds", C.c_double), ("kernel_flops", C.c_double),
                ("layer_launches", C.c_int32), ("layer_seconds", C.c_double),
                ("layer_flops", C.c_double), ("layer_bytes", C.c_double),
                ("gemm_launches", C.c_int32), ("gemm_seconds", C.c_double),
                ("gemm_flops", C.c_double), ("gemm_bytes", C.c_double),
                ("plan_reuses", C.c_int32), ("rsvd_passes", C.c_int32),
                ("workspace_bytes", C.c_double), ("alg_bytes", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def _check_dense(ts):
    """The library reads matrices as contiguous row-major float64 on the GPU."""
    import torch
    for t in ts:
        if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
            raise FpepsError(-1, "expected contiguous float64 CUDA tensors")


def load():
    """Load libfpeps.so (raises if it is missing: there is no other path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FpepsError(-9, f"{LIB_PATH} is not built; run paper_2511_01039_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    T = P(CTensor)
    sig = {
        "fpeps_version": ([], C.c_char_p),
        "fpeps_create": ([P(C.c_void_p), C.c_int32, C.c_void_p], C.c_int),
        "fpeps_destroy": ([C.c_void_p], C.c_int),
        "fpeps_set_stream": ([C.c_void_p, C.c_void_p], C.c_int),
        "fpeps_last_error": ([C.c_void_p], C.c_char_p),
        "fpeps_env_absorb": ([C.c_void_p, C.c_int32, T, T, T, P(COpts), T, P(C.c_double),
                              P(CReport)], C.c_int),
        "fpeps_absorb_diag": ([C.c_void_p, C.c_int32, C.c_int32, P(C.c_double), P(C.c_int32),
                               P(C.c_int32), P(C.c_int32), P(C.c_int32)], C.c_int),
        "fpeps_site_shape": ([C.c_void_p, T, T, T, T, P(COpts), C.c_int32, P(C.c_int32),
                              P(C.c_int32), P(C.c_int64), P(C.c_int64)], C.c_int),
        "fpeps_site_apply": ([C.c_void_p, T, T, T, T, P(COpts), C.c_int32, P(C.c_int32),
                              C.c_void_p, C.c_void_p, P(CReport)], C.c_int),
        "fpeps_rsvd_truncate": ([C.c_void_p, C.c_int32, P(C.c_int64), P(C.c_int64),
                                 P(C.c_void_p), P(COpts), P(C.c_void_p), P(C.c_void_p),
                                 P(C.c_int32), P(C.c_double), P(CReport)], C.c_int),
        "fpeps_cbe_expand": ([C.c_void_p, C.c_int32, P(C.c_int64), P(C.c_int64),
                              P(C.c_void_p), P(C.c_int32), P(C.c_void_p), P(C.c_void_p),
                              P(COpts), P(C.c_void_p), P(C.c_int32), P(C.c_double),
                              P(CReport)], C.c_int),
        "fpeps_rsvd_truncate_grouped": ([C.c_void_p, C.c_int32, P(C.c_int64), P(C.c_int64),
                                         P(C.c_void_p), P(C.c_int32), P(COpts), P(C.c_void_p),
                                         P(C.c_void_p), P(C.c_int32), P(C.c_double), P(CReport)],
                                        C.c_int),
        "fpeps_cbe_expand_grouped": ([C.c_void_p, C.c_int32, P(C.c_int64), P(C.c_int64),
                                      P(C.c_void_p), P(C.c_int32), P(C.c_int32), P(C.c_void_p),
                                      P(C.c_void_p), P(COpts), P(C.c_void_p), P(C.c_int32),
                                      P(C.c_double), P(CReport)], C.c_int),
        "fpeps_expect": ([C.c_void_p, C.c_int32, T, T, C.c_double, C.c_double, P(C.c_int32),
                          P(C.c_double)], C.c_int),
        "fpeps_set_allocator": ([C.c_void_p, ALLOC_FN, FREE_FN, C.c_void_p], C.c_int),
        "fpeps_expect_noalloc": ([C.c_void_p, C.c_int32, T, T, C.c_double, C.c_double,
                                  P(C.c_int32), P(C.c_double)], C.c_int),
        "fpeps_heff_apply": ([C.c_void_p, T, T, T, T, T, T, P(COpts), T, P(CReport)], C.c_int),
        "fpeps_heff_prepare": ([C.c_void_p, T, T, T, T, T, T, P(COpts), T, P(C.c_void_p),
                                P(CReport)], C.c_int),
        "fpeps_heff_apply_prepared": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                       P(CReport)], C.c_int),
        "fpeps_heff_release": ([C.c_void_p], C.c_int),
        "fpeps_autotune_absorb": ([C.c_void_p, C.c_int32, T, T, T, P(COpts), C.c_int32, T,
                                   P(C.c_double), P(CReport)], C.c_int),
        "fpeps_tune_save": ([C.c_void_p, C.c_char_p], C.c_int),
        "fpeps_tune_load": ([C.c_void_p, C.c_char_p], C.c_int),
        "fpeps_tune_clear": ([C.c_void_p], C.c_int),
        "fpeps_tune_info": ([C.c_void_p, P(C.c_int32), P(C.c_int64)], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def exported_symbols():
    return ["fpeps_version", "fpeps_create", "fpeps_destroy", "fpeps_set_stream",
            "fpeps_last_error", "fpeps_set_allocator", "fpeps_env_absorb", "fpeps_absorb_diag", "fpeps_site_shape",
            "fpeps_site_apply", "fpeps_rsvd_truncate", "fpeps_rsvd_truncate_grouped",
            "fpeps_cbe_expand", "fpeps_cbe_expand_grouped", "fpeps_expect",
            "fpeps_heff_apply", "fpeps_heff_prepare", "fpeps_heff_apply_prepared",
            "fpeps_heff_release", "fpeps_expect_noalloc", "fpeps_autotune_absorb",
            "fpeps_tune_save", "fpeps_tune_load", "fpeps_tune_clear", "fpeps_tune_info"]


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


@dataclass
class DeviceTensor:
    """Block-sparse tensor: host structure + torch float64 data on the GPU."""
    legs: list               # workloads.tensor.Leg
    blocks: np.ndarray       # int32 [nblocks, nlegs]
    offsets: np.ndarray      # int64 [nblocks]
    data: object             # torch.Tensor float64 (cuda)
    nelem: int

    @staticmethod
    def from_host(t, device="cuda"):
        import torch
        d = torch.from_numpy(np.ascontiguousarray(t.data)).to(device=device, dtype=torch.float64)
        return DeviceTensor(list(t.legs), np.ascontiguousarray(t.blocks, dtype=np.int32),
                            np.ascontiguousarray(t.offsets, dtype=np.int64), d, int(t.data.size))

    def to_host(self):
        from workloads.tensor import Tensor
        data = self.data[:self.nelem].detach().to("cpu").numpy().astype(np.float64)
        return Tensor(list(self.legs), self.blocks.copy(), self.offsets.copy(), data)

    def ctensor(self, keep):
        """ctypes view; ``keep`` collects arrays that must outlive the call."""
        nl = len(self.legs)
        nlab = int(self.legs[0].labels.shape[1]) if nl else 1
        ms = max(int(l.nsect) for l in self.legs) if nl else 1
        nsect = _i32([l.nsect for l in self.legs])
        dirs = _i32([l.dir for l in self.legs])
        labels = np.zeros((nl, ms, nlab), dtype=np.int32)
        dims = np.zeros((nl, ms), dtype=np.int32)
        for i, l in enumerate(self.legs):
            labels[i, :l.nsect] = l.labels
            dims[i, :l.nsect] = l.dims
        bs = np.ascontiguousarray(self.blocks, dtype=np.int32).reshape(-1)
        bo = np.ascontiguousarray(self.offsets, dtype=np.int64)
        keep += [nsect, dirs, labels, dims, bs, bo]
        ct = CTensor(nl, nlab, ms, _ptr(nsect, C.c_int32), _ptr(dirs, C.c_int32),
                     _ptr(labels, C.c_int32), _ptr(dims, C.c_int32), len(bo), len(bo),
                     _ptr(bs, C.c_int32), _ptr(bo, C.c_int64),
                     C.c_void_p(self.data.data_ptr()), self.nelem, self.nelem)
        return ct


class OutTensor:
    """Capacity-bounded output tensor filled by the library."""

    def __init__(self, nlegs, nlab, max_sect, max_blocks, max_elem, device="cuda"):
        import torch
        self.nsect = np.zeros(nlegs, np.int32)
        self.dirs = np.zeros(nlegs, np.int32)
        self.labels = np.zeros((nlegs, max_sect, nlab), np.int32)
        self.dims = np.zeros((nlegs, max_sect), np.int32)
        self.block_sect = np.zeros((max_blocks, nlegs), np.int32)
        self.block_off = np.zeros(max_blocks, np.int64)
        self.data = torch.empty(max(int(max_elem), 1), dtype=torch.float64, device=device)
        self.ct = CTensor(nlegs, nlab, max_sect, _ptr(self.nsect, C.c_int32),
                          _ptr(self.dirs, C.c_int32), _ptr(self.labels, C.c_int32),
                          _ptr(self.dims, C.c_int32), 0, max_blocks,
                          _ptr(self.block_sect, C.c_int32), _ptr(self.block_off, C.c_int64),
                          C.c_void_p(self.data.data_ptr()), 0, int(max_elem))

    def result(self):
        from workloads.tensor import Leg
        ct = self.ct
        legs = []
        for l in range(ct.nlegs):
            ns = int(self.nsect[l])
            legs.append(Leg(self.labels[l, :ns].copy(), self.dims[l, :ns].copy(), int(self.dirs[l])))
        nb = ct.nblocks
        return DeviceTensor(legs, self.block_sect[:nb].copy(), self.block_off[:nb].copy(), self.data,
                            int(ct.nelem))


def make_opts(chi=1, oversample=0, power_iters=0, cbe_extra=0, seed=0, row=0, precision="fp64",
              symmetry="none", fermionic=False, coef_seed=0, slice_budget=0, flags=0, tag=0,
              sv_cut=0.0):
    return COpts(int(chi), int(oversample), int(power_iters), int(cbe_extra), int(seed) & (2**64 - 1),
                 int(row), PREC[precision], SYM[symmetry], int(bool(fermionic)),
                 int(coef_seed) & (2**64 - 1), int(slice_budget), int(flags), int(tag), float(sv_cut))


def opts_for(sym, **kw):
    """Options from a workloads.Sym plus keyword overrides."""
    return make_opts(symmetry=sym.kind, fermionic=sym.fermionic, coef_seed=sym.coef_seed, **kw)


class Context:
    """One library context on one GPU, bound to torch's current stream."""

    def __init__(self, device=0, stream=None, torch_allocator=False):
        import torch
        self.lib = load()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self.stream = stream
        h = C.c_void_p()
        rc = self.lib.fpeps_create(C.byref(h), int(device), C.c_void_p(stream))
        if rc != FPEPS_OK:
            raise FpepsError(rc, "fpeps_create failed (no gfx950 device?)")
        self.h = h
        self._alloc_cbs = None
        if torch_allocator:
            self.use_torch_allocator()

    def use_torch_allocator(self):
        """Take the library's workspace from PyTorch's caching allocator
        (blocks on the context's stream) instead of hipMalloc."""
        import torch
        dev, stream = self.device, torch.cuda.ExternalStream(self.stream, device=self.device)

        def _alloc(nbytes, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
            except Exception:       # out of memory: the library reports FPEPS_ERR_NOMEM
                return None

        def _free(ptr, user):
            torch.cuda.caching_allocator_delete(ptr)

        cbs = (ALLOC_FN(_alloc), FREE_FN(_free))
        self.check(self.lib.fpeps_set_allocator(self.h, cbs[0], cbs[1], None))
        self._alloc_cbs = cbs        # the library calls them until the context is closed

    def use_hip_allocator(self):
        self.check(self.lib.fpeps_set_allocator(self.h, ALLOC_FN(), FREE_FN(), None))
        self._alloc_cbs = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.fpeps_destroy(self.h)
            self.h = None
        self._alloc_cbs = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc):
        if rc != FPEPS_OK:
            raise FpepsError(rc, self.lib.fpeps_last_error(self.h).decode())

    # ---------------------------------------------------------------------
    def env_absorb(self, env_in, ket, pepo, opts, log_norm=0.0, caps=None, autotune=0):
        """Absorb one row. Returns (list of DeviceTensor, log_norm, report).
        ``autotune`` > 0: fpeps_autotune_absorb with that many tile
        candidates (the context keeps the tuned table)."""
        L = len(env_in)
        keep = []
        ein = (CTensor * L)(*[t.ctensor(keep) for t in env_in])
        kin = (CTensor * L)(*[t.ctensor(keep) for t in ket])
        pin = (CTensor * L)(*[t.ctensor(keep) for t in pepo])
        caps = caps or [output_caps(env_in, ket, pepo, x, opts.chi) for x in range(L)]
        for attempt in range(2):
            outs = [OutTensor(5, ein[0].nlab, *caps[x]) for x in range(L)]
            oarr = (CTensor * L)(*[o.ct for o in outs])
            ln = C.c_double(log_norm)
            rep = CReport()
            if autotune:
                rc = self.lib.fpeps_autotune_absorb(self.h, L, ein, kin, pin, C.byref(opts),
                                                    int(autotune), oarr, C.byref(ln),
                                                    C.byref(rep))
            else:
                rc = self.lib.fpeps_env_absorb(self.h, L, ein, kin, pin, C.byref(opts), oarr,
                                               C.byref(ln), C.byref(rep))
            if rc == -7 and attempt == 0:
                caps = [(max(c[0], rep.required_sect), max(c[1], rep.required_blocks),
                         max(c[2], rep.required_elem)) for c in caps]
                continue
            self.check(rc)
            for o, oc in zip(outs, oarr):
                o.ct = oc
            return [o.result() for o in outs], ln.value, rep.as_dict()
        raise FpepsError(-7, "capacity")

    def tune_save(self, path):
        self.check(self.lib.fpeps_tune_save(self.h, os.fsencode(path)))

    def tune_load(self, path):
        self.check(self.lib.fpeps_tune_load(self.h, os.fsencode(path)))

    def tune_clear(self):
        self.check(self.lib.fpeps_tune_clear(self.h))

    def tune_info(self):
        """(tuned step signatures or -1 without a table, tuned slice budget in bytes)."""
        n, b = C.c_int32(), C.c_int64()
        self.check(self.lib.fpeps_tune_info(self.h, C.byref(n), C.byref(b)))
        return n.value, b.value

    def absorb_diag(self, site, capacity=1 << 16):
        sig = np.zeros(capacity)
        sec = np.zeros(capacity, np.int32)
        kept = np.zeros(capacity, np.int32)
        cnt, ns = C.c_int32(), C.c_int32()
        self.check(self.lib.fpeps_absorb_diag(self.h, int(site), capacity, _ptr(sig, C.c_double),
                                              _ptr(sec, C.c_int32), C.byref(cnt), C.byref(ns),
                                              _ptr(kept, C.c_int32)))
        return sig[:cnt.value].copy(), sec[:cnt.value].copy(), kept[:ns.value].copy()

    def site_shape(self, R, T, A, W, opts, capacity=4096):
        keep = []
        ns = C.c_int32()
        nlab = int(T.legs[0].labels.shape[1])
        lab = np.zeros((capacity, nlab), np.int32)
        m = np.zeros(capacity, np.int64)
        n = np.zeros(capacity, np.int64)
        cts = [x.ctensor(keep) for x in (R, T, A, W)]
        self.check(self.lib.fpeps_site_shape(self.h, *[C.byref(c) for c in cts], C.byref(opts),
                                             capacity, C.byref(ns), _ptr(lab, C.c_int32),
                                             _ptr(m, C.c_int64), _ptr(n, C.c_int64)))
        k = ns.value
        return lab[:k].copy(), m[:k].copy(), n[:k].copy()

    def site_apply(self, R, T, A, W, opts, k, x, transpose=False, out_elems=None):
        """x: torch float64 device tensor (per-sector matrices); returns y."""
        import torch
        _check_dense([x])
        keep = []
        kk = _i32(k)
        cts = [t.ctensor(keep) for t in (R, T, A, W)]
        y = torch.empty(max(int(out_elems), 1), dtype=torch.float64, device=x.device)
        rep = CReport()
        self.check(self.lib.fpeps_site_apply(self.h, *[C.byref(c) for c in cts], C.byref(opts),
                                             int(bool(transpose)), _ptr(kk, C.c_int32),
                                             C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                             C.byref(rep)))
        return y, rep.as_dict()

    def rsvd_truncate(self, mats, opts, group=None):
        """mats: list of 2-D torch float64 device tensors; group (optional): the
        truncation problem of every matrix (fpeps_rsvd_truncate_grouped).
        Returns U, R, sigma, kept, report."""
        import torch
        _check_dense(mats)
        nm = len(mats)
        m = np.array([a.shape[0] for a in mats], np.int64)
        n = np.array([a.shape[1] for a in mats], np.int64)
        A = (C.c_void_p * nm)(*[a.data_ptr() for a in mats])
        U = [torch.empty(max(int(mi * min(mi, ni)), 1), dtype=torch.float64, device=mats[0].device)
             for mi, ni in zip(m, n)]
        R = [torch.empty(max(int(min(mi, ni) * ni), 1), dtype=torch.float64, device=mats[0].device)
             for mi, ni in zip(m, n)]
        Up = (C.c_void_p * nm)(*[u.data_ptr() for u in U])
        Rp = (C.c_void_p * nm)(*[r.data_ptr() for r in R])
        kept = np.zeros(nm, np.int32)
        sig = np.zeros(int(sum(min(a, b) for a, b in zip(m, n))) + 1)
        rep = CReport()
        if group is None:
            self.check(self.lib.fpeps_rsvd_truncate(self.h, nm, _ptr(m, C.c_int64),
                                                    _ptr(n, C.c_int64), A, C.byref(opts), Up, Rp,
                                                    _ptr(kept, C.c_int32), _ptr(sig, C.c_double),
                                                    C.byref(rep)))
        else:
            g = _i32(group)
            if g.shape != (nm,):
                raise FpepsError(-1, "group must list one problem id per matrix")
            self.check(self.lib.fpeps_rsvd_truncate_grouped(self.h, nm, _ptr(m, C.c_int64),
                                                            _ptr(n, C.c_int64), A,
                                                            _ptr(g, C.c_int32), C.byref(opts), Up,
                                                            Rp, _ptr(kept, C.c_int32),
                                                            _ptr(sig, C.c_double), C.byref(rep)))
        Us = [U[i][:int(m[i] * kept[i])].reshape(int(m[i]), int(kept[i])) for i in range(nm)]
        Rs = [R[i][:int(n[i] * kept[i])].reshape(int(kept[i]), int(n[i])) for i in range(nm)]
        sigs, p = [], 0
        for i in range(nm):
            sigs.append(sig[p:p + kept[i]].copy())
            p += kept[i]
        return Us, Rs, sigs, kept, rep.as_dict()

    def cbe_expand(self, mats, U, V, opts, group=None):
        """Bond expansion directions orthogonal to U and V (group as in
        rsvd_truncate). Returns Q, sigma, kept, report."""
        import torch
        _check_dense(mats)
        nm = len(mats)
        m = np.array([a.shape[0] for a in mats], np.int64)
        n = np.array([a.shape[1] for a in mats], np.int64)
        r = np.array([u.shape[1] for u in U], np.int32)
        A = (C.c_void_p * nm)(*[a.data_ptr() for a in mats])
        # contiguous copies held until the call returns (a temporary's
        # data_ptr would dangle)
        Uc = [u.contiguous() for u in U]
        Vc = [v.contiguous() for v in V]
        Up = (C.c_void_p * nm)(*[u.data_ptr() for u in Uc])
        Vp = (C.c_void_p * nm)(*[v.data_ptr() for v in Vc])
        Q = [torch.empty(max(int(mi * min(mi, ni)), 1), dtype=torch.float64, device=mats[0].device)
             for mi, ni in zip(m, n)]
        Qp = (C.c_void_p * nm)(*[q.data_ptr() for q in Q])
        kept = np.zeros(nm, np.int32)
        sig = np.zeros(int(sum(min(a, b) for a, b in zip(m, n))) + 1)
        rep = CReport()
        if group is None:
            self.check(self.lib.fpeps_cbe_expand(self.h, nm, _ptr(m, C.c_int64),
                                                 _ptr(n, C.c_int64), A, _ptr(r, C.c_int32), Up, Vp,
                                                 C.byref(opts), Qp, _ptr(kept, C.c_int32),
                                                 _ptr(sig, C.c_double), C.byref(rep)))
        else:
            g = _i32(group)
            if g.shape != (nm,):
                raise FpepsError(-1, "group must list one problem id per matrix")
            self.check(self.lib.fpeps_cbe_expand_grouped(self.h, nm, _ptr(m, C.c_int64),
                                                         _ptr(n, C.c_int64), A, _ptr(g, C.c_int32),
                                                         _ptr(r, C.c_int32), Up, Vp, C.byref(opts),
                                                         Qp, _ptr(kept, C.c_int32),
                                                         _ptr(sig, C.c_double), C.byref(rep)))
        Qs = [Q[i][:int(m[i] * kept[i])].reshape(int(m[i]), int(kept[i])) for i in range(nm)]
        sigs, p = [], 0
        for i in range(nm):
            sigs.append(sig[p:p + kept[i]].copy())
            p += kept[i]
        return Qs, sigs, kept, rep.as_dict()

    def expect_log(self, top, bottom, log_norm_top=0.0, log_norm_bottom=0.0):
        """Network value of two environments as (sign, log |Z|)."""
        keep = []
        L = len(top)
        ta = (CTensor * L)(*[t.ctensor(keep) for t in top])
        ba = (CTensor * L)(*[t.ctensor(keep) for t in bottom])
        sg = C.c_int32()
        la = C.c_double()
        self.check(self.lib.fpeps_expect(self.h, L, ta, ba, C.c_double(log_norm_top),
                                         C.c_double(log_norm_bottom), C.byref(sg), C.byref(la)))
        return int(sg.value), float(la.value)

    def heff_apply(self, T, L, B, R, W, A, opts, caps=None):
        """y = H_eff A (Fig. 2(b)); returns (DeviceTensor y, report)."""
        keep = []
        cts = [t.ctensor(keep) for t in (T, L, B, R, W, A)]
        nlab = cts[0].nlab
        caps = caps or (256, 1 << 16, max(1, int(A.nelem) * 64))
        for attempt in range(2):
            out = OutTensor(5, nlab, *caps)
            rep = CReport()
            rc = self.lib.fpeps_heff_apply(self.h, *[C.byref(c) for c in cts], C.byref(opts),
                                           C.byref(out.ct), C.byref(rep))
            if rc == -7 and attempt == 0:
                caps = (max(caps[0], rep.required_sect), max(caps[1], rep.required_blocks),
                        max(caps[2], rep.required_elem))
                continue
            self.check(rc)
            return out.result(), rep.as_dict()
        raise FpepsError(-7, "capacity")

    def heff_prepare(self, T, L, B, R, W, A, opts, caps=None):
        """The prepared effective operator for vectors shaped like A:
        returns (HeffOperator, DeviceTensor y = H_eff A, report)."""
        keep = []
        cts = [t.ctensor(keep) for t in (T, L, B, R, W, A)]
        nlab = cts[0].nlab
        caps = caps or (256, 1 << 16, max(1, int(A.nelem) * 64))
        for attempt in range(2):
            out = OutTensor(5, nlab, *caps)
            rep = CReport()
            h = C.c_void_p()
            rc = self.lib.fpeps_heff_prepare(self.h, *[C.byref(c) for c in cts], C.byref(opts),
                                             C.byref(out.ct), C.byref(h), C.byref(rep))
            if rc == -7 and attempt == 0:
                caps = (max(caps[0], rep.required_sect), max(caps[1], rep.required_blocks),
                        max(caps[2], rep.required_elem))
                continue
            self.check(rc)
            y = out.result()
            return HeffOperator(self, h, int(A.nelem), y), y, rep.as_dict()
        raise FpepsError(-7, "capacity")

    def expect_log_noalloc(self, top, bottom, log_norm_top=0.0, log_norm_bottom=0.0):
        """expect_log with no device allocation (fpeps_expect_noalloc)."""
        keep = []
        L = len(top)
        ta = (CTensor * L)(*[t.ctensor(keep) for t in top])
        ba = (CTensor * L)(*[t.ctensor(keep) for t in bottom])
        sg = C.c_int32()
        la = C.c_double()
        self.check(self.lib.fpeps_expect_noalloc(self.h, L, ta, ba, C.c_double(log_norm_top),
                                                 C.c_double(log_norm_bottom), C.byref(sg),
                                                 C.byref(la)))
        return int(sg.value), float(la.value)

    def expect(self, top, bottom):
        """The same as a plain float (no log-norms applied)."""
        sg, la = self.expect_log(top, bottom)
        return sg * math.exp(la) if sg else 0.0


class HeffOperator:
    """A prepared effective operator (fpeps_heff_prepare): apply() replays
    the captured products for a new vector of the prepared structure."""

    def __init__(self, ctx, handle, a_elems, y_like):
        self.ctx, self.h, self.a_elems, self.y_like = ctx, handle, a_elems, y_like

    def apply(self, a_data, y_data=None):
        """a_data: torch float64 device tensor with the vector's elements;
        returns (y_data, report)."""
        import torch
        if y_data is None:
            y_data = torch.empty(max(self.y_like.nelem, 1), dtype=torch.float64,
                                 device=a_data.device)
        rep = CReport()
        self.ctx.check(self.ctx.lib.fpeps_heff_apply_prepared(
            self.h, C.c_void_p(a_data.data_ptr()), int(self.a_elems),
            C.c_void_p(y_data.data_ptr()), int(y_data.numel()), C.byref(rep)))
        return y_data, rep.as_dict()

    def close(self):
        if self.h:
            self.ctx.check(self.ctx.lib.fpeps_heff_release(self.h))
            self.h = None


def output_caps(env_in, ket, pepo, x, chi):
    """First-guess capacities (sectors per leg, blocks, elements) of the new
    environment site x. Elements: at most chi kept columns over rows of
    (chi, D, w, D) dims. If a guess is short the library reports the sizes it
    needs and the call is repeated once with them."""
    dk, dw = ket[x].legs[4], pepo[x].legs[5]
    rows = max(chi, 1) * int(dk.total) * int(dw.total) * int(dk.total)
    max_sect = max(256, int(env_in[x].legs[0].nsect), int(env_in[x].legs[4].nsect))
    max_blocks = 1 << 16
    max_elem = int(rows * max(chi, 1))
    return (int(max_sect), int(max_blocks), max(int(max_elem), 1))
