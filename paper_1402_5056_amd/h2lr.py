"""Thin ctypes binding of the h2lr C ABI (include/h2lr.h).

Argument marshalling only: every computation runs in the HIP library.  The
functions keep the C names; handles are opaque integers wrapped in small
classes that free them.  Device buffers are torch tensors on a ROCm device
(passed by ``data_ptr()``); host arrays are numpy arrays.  A non-zero status
raises :class:`H2Error`.  Importing this module fails loudly if the library
has not been built; there is no fallback implementation.
"""

from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# H2LR_LIBRARY selects another build of the same library (side-by-side
# comparisons of builds); by default the in-tree one.
LIB_PATH = os.environ.get("H2LR_LIBRARY") or os.path.join(_HERE, "libh2lr.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"h2lr library not built: {LIB_PATH} missing (run paper_1402_5056_amd/build.py)")
try:
    # torch ships its own HIP runtime (same soname as the system one); loading
    # it first makes this library bind to that runtime instead of loading a
    # second HIP/HSA runtime into the process.
    import torch  # noqa: F401
except ImportError:  # host-only use (trees) without torch
    pass
_lib = C.CDLL(LIB_PATH)

H2_OK = 0
STATUS = {0: "H2_OK", -1: "H2_ERR_ARG", -2: "H2_ERR_NOMEM", -3: "H2_ERR_HIP", -4: "H2_ERR_NOT_SPD",
          -5: "H2_ERR_RANK_CAP", -6: "H2_ERR_NONZERO_FARFIELD", -7: "H2_ERR_NOT_CONVERGED",
          -8: "H2_ERR_STATE", -9: "H2_ERR_ZERO_PIVOT"}
MAX_RANK = 32
MAX_LEAF = 32
MAX_COLS = 64
MAX_UPDATE_RANK = 32
NOALLOC_MAX_N = 262144
PROF_LEN = 204
UPDATE_STEPS = ("a4 R-factors", "a5 weights", "a6 recompression", "a7 couplings",
                "a8 R-factor refresh", "a9 nearfield")
MODES = {"block_rel": 0, "const_rel": 1, "none": 2}


class H2Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class h2_trunc(C.Structure):
    _fields_ = [("eps", C.c_double), ("mode", C.c_int32), ("rank_cap", C.c_int32), ("precision", C.c_int32),
                ("accumulate", C.c_int32), ("level_factor", C.c_double)]


_vp = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_d = C.c_double
_P = C.POINTER

_SIG = {
    "h2_ctx_create": [C.c_int, _vp, _P(_vp)],
    "h2_ctx_destroy": [_vp],
    "h2_ctx_synchronize": [_vp],
    "h2_ctree_build": [_vp, _i32, _i64, _vp, _i32, _P(_vp)],
    "h2_ctree_build_dd": [_vp, _i32, _i64, _vp, _i32, _P(_vp)],
    "h2_ctree_info": [_vp, _P(_i64), _P(_i64), _P(_i32)],
    "h2_ctree_export": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "h2_ctree_destroy": [_vp],
    "h2_btree_build": [_vp, _vp, _d, _P(_vp)],
    "h2_btree_info": [_vp, _P(_i64), _P(_i64), _P(_i64), _P(_i32)],
    "h2_btree_export": [_vp, _vp, _vp, _vp, _vp],
    "h2_btree_find": [_vp, _i64, _i64, _P(_i64)],
    "h2_btree_destroy": [_vp],
    "h2_mat_from_csr": [_vp, _vp, _i64, _vp, _vp, _vp, _i32, _P(_vp)],
    "h2_mat_copy": [_vp, _P(_vp)],
    "h2_mat_assign": [_vp, _vp],
    "h2_mat_destroy": [_vp],
    "h2_mat_stats": [_vp, _P(_i64), _P(_i32), _P(_i32)],
    "h2_mat_ranks": [_vp, _vp, _vp],
    "h2_estimate_bytes": [_vp, _i32, _P(_i64)],
    "h2_mat_bytes": [_vp, _P(_i64)],
    "h2_profile": [_vp, _i32, _vp, _i32],
    "h2_mat_flops": [_vp, _P(_d), _i32],
    "h2_lowrank_update": [_vp, _i64, _i32, _vp, _i64, _vp, _i64, _P(h2_trunc)],
    "h2_matvec": [_vp, _i32, _d, _vp, _d, _vp, _i32],
    "h2_cholesky": [_vp, _P(h2_trunc)],
    "h2_lr": [_vp, _P(h2_trunc)],
    "h2_lr_solve": [_vp, _vp, _vp, _i32],
    "h2_product": [_vp, _d, _vp, _vp, _P(h2_trunc)],
    "h2_cholesky_batched": [_P(_vp), _i32, _P(h2_trunc), _P(C.c_int)],
    "h2_lowrank_update_batched": [_P(_vp), _i32, _P(_i32), _P(_i64), _P(_i32), _P(_vp), _P(_i64), _P(_vp),
                                  _P(_i64), _P(h2_trunc), _P(C.c_int)],
    "h2_cholesky_launch": [_P(_vp), _i32, _P(h2_trunc), _P(_vp)],
    "h2_lowrank_update_accumulated": [_vp, _i32, _P(_i64), _P(_i32), _P(_vp), _P(_i64), _P(_vp), _P(_i64),
                                      _P(h2_trunc), _P(_i64)],
    "h2_precond_config": [_vp, _i32, _i32],
    "h2_autotune_precond": [_vp, _i32, _i32, C.c_char_p, _P(_i32), _P(_d), _P(_i32), _P(_d)],
    "h2_update_cholesky_launch": [_P(_vp), _i32, _P(_i32), _P(_i64), _P(_i32), _P(_vp), _P(_i64), _P(_vp),
                                  _P(_i64), _P(_vp), _i32, _P(h2_trunc), _P(_vp)],
    "h2_job_query": [_vp, _P(_i32)],
    "h2_job_finish": [_vp, _P(C.c_int)],
    "h2_pcg_batched": [_P(_vp), _P(_vp), _P(_vp), _P(_vp), _P(_i32), _i32, _d, _i32, _P(_i32), _P(_d),
                       _P(C.c_int)],
    "h2_pcg_batched_graph": [_P(_vp), _P(_vp), _P(_vp), _P(_vp), _P(_i32), _i32, _d, _i32, _P(_i32), _P(_d),
                             _P(C.c_int)],
    "h2_precond": [_vp, _vp, _vp, _i32],
    "h2_trsv": [_vp, _i32, _vp, _vp, _i32],
    "h2_tri_invert": [_vp, _vp],
    "h2_mat_is_inverse": [_vp, _P(_i32)],
    "h2_csr_create": [_vp, _i64, _vp, _vp, _vp, _P(_vp)],
    "h2_csr_destroy": [_vp],
    "h2_spmv": [_vp, _vp, _vp],
    "h2_pcg": [_vp, _vp, _vp, _vp, _d, _i32, _P(_i32), _P(_d)],
    "h2_pcg_noalloc": [_vp, _vp, _vp, _vp, _d, _i32, _P(_i32), _P(_d)],
}
for _name, _args in _SIG.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.h2_last_error.argtypes = []
_lib.h2_last_error.restype = C.c_char_p

EXPORTED = tuple(_SIG) + ("h2_last_error",)


def _check(status: int):
    if status != H2_OK:
        raise H2Error(status, (_lib.h2_last_error() or b"").decode())


def _ptr(t) -> int:
    """Device pointer of a torch tensor (must be contiguous float64/int)."""
    return t.data_ptr()


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


PRECISIONS = {"fp64": 0, "mixed": 1, "mixed_bf16": 2}


def trunc(eps: float = 1e-4, mode: str = "block_rel", rank_cap: int = MAX_RANK,
          precision: str = "fp64", accumulate: bool = False, level_factor: float = 1.0) -> h2_trunc:
    return h2_trunc(float(eps), MODES[mode] if isinstance(mode, str) else int(mode), int(rank_cap),
                    PRECISIONS[precision] if isinstance(precision, str) else int(precision), int(bool(accumulate)),
                    float(level_factor))


_LIVE = weakref.WeakSet()


class _Handle:
    _destroy = None
    _order = 0          # destruction order at exit: matrices first, context last

    def __init__(self, h, keep=()):
        self.h = h
        self._keep = keep   # keep referenced objects alive
        _LIVE.add(self)

    def close(self):
        if self.h is not None and self._destroy is not None:
            getattr(_lib, self._destroy)(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # Never call into the HIP runtime while the interpreter shuts down.
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


@atexit.register
def _forget_all():
    """At interpreter exit, drop every live handle without calling into the
    HIP runtime (the operating system reclaims device memory)."""
    for h in list(_LIVE):
        h.h = None


class Ctx(_Handle):
    _destroy = "h2_ctx_destroy"
    _order = 4


class CTree(_Handle):
    _destroy = "h2_ctree_destroy"
    _order = 3


class BTree(_Handle):
    _destroy = "h2_btree_destroy"
    _order = 2


class Mat(_Handle):
    _destroy = "h2_mat_destroy"
    _order = 0


class Csr(_Handle):
    _destroy = "h2_csr_destroy"
    _order = 1


def h2_ctx_create(device: int = 0, stream: int | None = None) -> Ctx:
    h = _vp()
    _check(_lib.h2_ctx_create(int(device), _vp(stream or 0), C.byref(h)))
    return Ctx(h.value)


def h2_ctx_synchronize(ctx: Ctx):
    _check(_lib.h2_ctx_synchronize(ctx.h))


def h2_ctree_build(ctx: Ctx, coords: np.ndarray, leaf_size: int = 32) -> CTree:
    c = _np(coords, np.int32)
    h = _vp()
    _check(_lib.h2_ctree_build(ctx.h, c.shape[1], c.shape[0], c.ctypes.data, int(leaf_size), C.byref(h)))
    return CTree(h.value, keep=(ctx,))


def h2_ctree_build_dd(ctx: Ctx, coords: np.ndarray, leaf_size: int = 32) -> CTree:
    c = _np(coords, np.int32)
    h = _vp()
    _check(_lib.h2_ctree_build_dd(ctx.h, c.shape[1], c.shape[0], c.ctypes.data, int(leaf_size),
                                  C.byref(h)))
    return CTree(h.value, keep=(ctx,))


def h2_ctree_info(ct: CTree):
    n, nc, depth = _i64(), _i64(), _i32()
    _check(_lib.h2_ctree_info(ct.h, C.byref(n), C.byref(nc), C.byref(depth)))
    return n.value, nc.value, depth.value


def h2_ctree_export(ct: CTree) -> dict:
    n, nc, _ = h2_ctree_info(ct)
    out = {"perm": np.zeros(n, np.int64)}
    for k in ("offset", "size", "level", "son0", "son1", "parent"):
        out[k] = np.zeros(nc, np.int32)
    _check(_lib.h2_ctree_export(ct.h, out["perm"].ctypes.data, out["offset"].ctypes.data,
                                out["size"].ctypes.data, out["level"].ctypes.data,
                                out["son0"].ctypes.data, out["son1"].ctypes.data,
                                out["parent"].ctypes.data))
    return out


def h2_btree_build(ctx: Ctx, ct: CTree, eta: float = 2.0) -> BTree:
    h = _vp()
    _check(_lib.h2_btree_build(ctx.h, ct.h, float(eta), C.byref(h)))
    return BTree(h.value, keep=(ctx, ct))


def h2_btree_info(bt: BTree):
    nb, na, nn, csp = _i64(), _i64(), _i64(), _i32()
    _check(_lib.h2_btree_info(bt.h, C.byref(nb), C.byref(na), C.byref(nn), C.byref(csp)))
    return nb.value, na.value, nn.value, csp.value


def h2_btree_export(bt: BTree) -> dict:
    nb = h2_btree_info(bt)[0]
    out = {k: np.zeros(nb, np.int32) for k in ("row", "col", "kind", "parent")}
    _check(_lib.h2_btree_export(bt.h, out["row"].ctypes.data, out["col"].ctypes.data,
                                out["kind"].ctypes.data, out["parent"].ctypes.data))
    return out


def h2_btree_find(bt: BTree, t: int, s: int) -> int:
    b = _i64()
    _check(_lib.h2_btree_find(bt.h, int(t), int(s), C.byref(b)))
    return b.value


def _csr_arrays(A):
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    return A.shape[0], _np(A.indptr, np.int64), _np(A.indices, np.int32), _np(A.data, np.float64)


def h2_mat_from_csr(ctx: Ctx, bt: BTree, A, lower: bool = False) -> Mat:
    n, rp, ci, v = _csr_arrays(A)
    h = _vp()
    _check(_lib.h2_mat_from_csr(ctx.h, bt.h, n, rp.ctypes.data, ci.ctypes.data, v.ctypes.data,
                                1 if lower else 0, C.byref(h)))
    return Mat(h.value, keep=(ctx, bt))


def h2_mat_copy(m: Mat) -> Mat:
    h = _vp()
    _check(_lib.h2_mat_copy(m.h, C.byref(h)))
    return Mat(h.value, keep=m._keep)


def h2_mat_assign(dst: Mat, src: Mat):
    _check(_lib.h2_mat_assign(dst.h, src.h))


def h2_mat_stats(m: Mat):
    v, kr, kc = _i64(), _i32(), _i32()
    _check(_lib.h2_mat_stats(m.h, C.byref(v), C.byref(kr), C.byref(kc)))
    return v.value, kr.value, kc.value


def h2_mat_ranks(m: Mat, nclusters: int):
    """(row ranks, column ranks) as int32 arrays of nclusters entries."""
    kr = np.zeros(nclusters, dtype=np.int32)
    kc = np.zeros(nclusters, dtype=np.int32)
    _check(_lib.h2_mat_ranks(m.h, kr.ctypes.data, kc.ctypes.data))
    return kr, kc


def h2_mat_flops(m: Mat, reset: bool = False) -> float:
    f = _d()
    _check(_lib.h2_mat_flops(m.h, C.byref(f), 1 if reset else 0))
    return f.value


OPS = ["", "addlr", "expand", "bapply", "rmul_s", "copy_near", "ident", "near_add", "temp_init",
       "temp_add", "potrf", "trsm", "trsv", "sub", "copy", "sv_zero", "sv_push", "sv_leaf", "sv_cross",
       "sv_up", "trtri", "trmv", "neg", "near_trmul", "getrf", "addlr_temps"]
STAGES = ["zero-check", "rfactors", "path-weights", "subtree-weights", "recompress", "couplings",
          "nearfield", "commit"]


# per-wave sub-steps of the low-rank update (seconds summed over waves) and counts
WAVE_TICKS = ["rfactor build", "rfactor qr", "weight omega", "weight stack", "weight qr",
              "recompress build", "recompress M", "recompress svd", "recompress out", "coupling",
              "rho refresh"]
WAVE_COUNTS = ["weight calls", "weight blocks", "weight nonempty", "qr calls", "qr cols", "qr rows",
               "rho refresh"]


def h2_profile(m: Mat, enable: bool = True):
    """Return the previous counters as a dict and (re)enable collection."""
    buf = np.zeros(PROF_LEN, np.int64)
    _check(_lib.h2_profile(m.h, 1 if enable else 0, buf.ctypes.data, PROF_LEN))
    out = {}
    for i, name in enumerate(OPS):
        if name and buf[i]:
            out[name] = (int(buf[i]), buf[32 + i] * 1e-8)
    out["stages"] = {name: buf[64 + i] * 1e-8 for i, name in enumerate(STAGES)}
    out["stages"]["  of which svd"] = buf[64 + 11] * 1e-8
    out["jacobi"] = {"calls": int(buf[64 + 13]), "sweeps": int(buf[64 + 12]), "cols": int(buf[64 + 14])}
    out["bapply_classes"] = {c: (int(buf[88 + i]), buf[80 + i] * 1e-8) for i, c in
                             enumerate(["1", "2-3", "4-15", "16-63", "64-255", "256+"])}
    out["wave_ticks"] = {name: buf[96 + i] * 1e-8 for i, name in enumerate(WAVE_TICKS)}
    out["wave_counts"] = {name: int(buf[112 + i]) for i, name in enumerate(WAVE_COUNTS)}
    out["update_levels"] = {lv: (int(buf[144 + lv]), buf[128 + lv] * 1e-8) for lv in range(16) if buf[144 + lv]}
    out["leaf_stages"] = {name: buf[160 + i] * 1e-8 for i, name in enumerate(STAGES)}
    out["svd_classes"] = {c: (int(buf[172 + i]), buf[168 + i] * 1e-8) for i, c in
                          enumerate(["<=8", "<=16", "<=32", ">32"])}
    out["temp_classes"] = {c: (int(buf[184 + i]), buf[176 + i] * 1e-8) for i, c in
                           enumerate(["<=32", "<=128", "<=512", "<=2048", ">2048"])}
    out["step_flops"] = {name: float(buf[192 + i]) for i, name in enumerate(UPDATE_STEPS)}
    out["step_bytes"] = {name: float(buf[198 + i]) for i, name in enumerate(UPDATE_STEPS)}
    return out


def h2_lowrank_update(m: Mat, block: int, X, Y, tr: h2_trunc):
    """X (#t0 x k), Y (#s0 x k): float64 torch tensors on the device,
    column-major (pass ``x.t().contiguous().t()`` or Fortran-ordered data)."""
    k = X.shape[1]
    assert Y.shape[1] == k
    _check(_lib.h2_lowrank_update(m.h, int(block), int(k), _ptr(X), X.stride(1) if k > 1 else X.shape[0],
                                  _ptr(Y), Y.stride(1) if k > 1 else Y.shape[0], C.byref(tr)))


def h2_matvec(m: Mat, x, y, trans: bool = False, alpha: float = 1.0, beta: float = 0.0):
    """x, y: (n,) or (nrhs, n) contiguous float64 device tensors (each row one
    vector, i.e. column-major n x nrhs)."""
    nrhs = 1 if x.dim() == 1 else x.shape[0]
    _check(_lib.h2_matvec(m.h, 1 if trans else 0, float(alpha), _ptr(x), float(beta), _ptr(y), nrhs))


def h2_cholesky(m: Mat, tr: h2_trunc):
    _check(_lib.h2_cholesky(m.h, C.byref(tr)))


def h2_lr(m: Mat, tr: h2_trunc):
    _check(_lib.h2_lr(m.h, C.byref(tr)))


def h2_lr_solve(m: Mat, r, z):
    """z = R^{-1} L^{-1} r with the factors of h2_lr; r, z as for h2_precond."""
    nrhs = 1 if r.dim() == 1 else r.shape[0]
    _check(_lib.h2_lr_solve(m.h, _ptr(r), _ptr(z), nrhs))


def h2_product(z: Mat, alpha: float, x: Mat, y: Mat, tr: h2_trunc):
    _check(_lib.h2_product(z.h, float(alpha), x.h, y.h, C.byref(tr)))


def h2_estimate_bytes(bt: BTree, lower: bool = True) -> int:
    v = _i64()
    _check(_lib.h2_estimate_bytes(bt.h, 1 if lower else 0, C.byref(v)))
    return v.value


def h2_mat_bytes(m: Mat) -> int:
    v = _i64()
    _check(_lib.h2_mat_bytes(m.h, C.byref(v)))
    return v.value


def _update_arrays(mats, updates):
    """Flat host arrays of a batch of local updates (h2_lowrank_update_batched)."""
    k = len(mats)
    flat = [u for ups in updates for u in ups]
    nu = max(len(flat), 1)

    def ld(T):
        return T.stride(1) if T.shape[1] > 1 else T.shape[0]
    return ((_vp * max(k, 1))(*[m.h for m in mats]), (_i32 * max(k, 1))(*[len(u) for u in updates]),
            (_i64 * nu)(*[int(b) for b, _, _ in flat]), (_i32 * nu)(*[int(X.shape[1]) for _, X, _ in flat]),
            (_vp * nu)(*[_ptr(X) for _, X, _ in flat]), (_i64 * nu)(*[ld(X) for _, X, _ in flat]),
            (_vp * nu)(*[_ptr(Y) for _, _, Y in flat]), (_i64 * nu)(*[ld(Y) for _, _, Y in flat]))


def h2_lowrank_update_accumulated(m: Mat, updates, tr: h2_trunc) -> int:
    """updates: list of (block, X, Y) as for h2_lowrank_update, merged into
    one local update; returns the merged block."""
    _, _, blocks, ks, Xs, ldx, Ys, ldy = _update_arrays([m], [updates])
    mb = _i64()
    _check(_lib.h2_lowrank_update_accumulated(m.h, len(updates), blocks, ks, Xs, ldx, Ys, ldy, C.byref(tr),
                                              C.byref(mb)))
    return mb.value


def h2_lowrank_update_batched(mats, updates, tr: h2_trunc, check: bool = True):
    """updates[i]: list of (block, X, Y) for mats[i] (at most 4), X, Y
    column-major device tensors as for h2_lowrank_update.  Returns the
    per-matrix status list."""
    k = len(mats)
    arr, nupd, blocks, ks, Xs, ldx, Ys, ldy = _update_arrays(mats, updates)
    st = (C.c_int * k)()
    status = _lib.h2_lowrank_update_batched(arr, k, nupd, blocks, ks, Xs, ldx, Ys, ldy, C.byref(tr), st)
    codes = list(st)
    if check:
        _check(status)
    return codes


def h2_cholesky_batched(mats, tr: h2_trunc):
    """Factorise the matrices in one launch; returns the per-matrix status
    list.  Raises H2Error for the first failure (the others are factorised)."""
    arr = (_vp * len(mats))(*[m.h for m in mats])
    st = (C.c_int * len(mats))()
    status = _lib.h2_cholesky_batched(arr, len(mats), C.byref(tr), st)
    codes = list(st)
    _check(status)
    return codes


class Job:
    """A launched batch (h2_cholesky_launch, h2_update_cholesky_launch);
    holds its matrices (and the update factors it reads) until finish()."""

    def __init__(self, h, mats, keep=()):
        self.h = h
        self.mats = list(mats)
        self.keep = list(keep)

    def done(self) -> bool:
        v = _i32()
        _check(_lib.h2_job_query(self.h, C.byref(v)))
        return bool(v.value)

    def __del__(self):
        # an unfinished job still holds its matrices: wait and release them
        if getattr(self, "h", None) is not None and _lib is not None:
            h, self.h = self.h, None
            _lib.h2_job_finish(h, None)

    def finish(self, check: bool = True):
        """Per-matrix status list; raises H2Error for the first failure when
        check is true."""
        if self.h is None:
            raise H2Error(-1, "job already finished")
        st = (C.c_int * len(self.mats))()
        h, self.h = self.h, None
        status = _lib.h2_job_finish(h, st)
        codes = list(st)
        self.mats = []
        self.keep = []
        if check:
            _check(status)
        return codes


def h2_cholesky_launch(mats, tr: h2_trunc) -> Job:
    arr = (_vp * len(mats))(*[m.h for m in mats])
    h = _vp()
    _check(_lib.h2_cholesky_launch(arr, len(mats), C.byref(tr), C.byref(h)))
    return Job(h.value, mats)


def h2_update_cholesky_launch(umats, updates, cmats, tr: h2_trunc) -> Job:
    """Local updates of umats (updates as for h2_lowrank_update_batched) and
    Cholesky factorisations of cmats in one launch; the job's status list
    has the updated matrices first."""
    arr, nupd, blocks, ks, Xs, ldx, Ys, ldy = _update_arrays(umats, updates)
    carr = (_vp * max(len(cmats), 1))(*[m.h for m in cmats])
    h = _vp()
    _check(_lib.h2_update_cholesky_launch(arr, len(umats), nupd, blocks, ks, Xs, ldx, Ys, ldy, carr, len(cmats),
                                          C.byref(tr), C.byref(h)))
    keep = [T for ups in updates for _, X, Y in ups for T in (X, Y)]
    return Job(h.value, list(umats) + list(cmats), keep)


def h2_pcg_batched(csrs, mats, bs, xs, rtol: float = 1e-8, maxit: int = 500, check: bool = True,
                   graph: bool = False):
    """bs[i], xs[i]: device float64 tensors of shape (n_i,) or (k_i, n_i)
    (k_i right-hand sides, contiguous).  Returns (iters, relres, status),
    flat lists with one entry per right-hand side; raises H2Error for the
    first failure when check is true.  graph: replay the iterations from a
    captured HIP graph (h2_pcg_batched_graph)."""
    k = len(mats)
    A = (_vp * k)(*[a.h for a in csrs])
    Ls = (_vp * k)(*[m.h for m in mats])
    B = (_vp * k)(*[_ptr(b) for b in bs])
    X = (_vp * k)(*[_ptr(x) for x in xs])
    cols = [1 if b.dim() == 1 else b.shape[0] for b in bs]
    for b, x, c in zip(bs, xs, cols):
        if not (b.is_contiguous() and x.is_contiguous() and b.shape == x.shape):
            raise H2Error(-1, "right-hand sides and solutions must be contiguous and of equal shape")
    nr = (_i32 * k)(*cols)
    tot = sum(cols)
    it = (_i32 * tot)()
    rel = (_d * tot)()
    st = (C.c_int * tot)()
    fn = _lib.h2_pcg_batched_graph if graph else _lib.h2_pcg_batched
    status = fn(A, Ls, B, X, nr, k, float(rtol), int(maxit), it, rel, st)
    if check:
        _check(status)
    return list(it), list(rel), list(st)


def h2_tri_invert(m: Mat, tr: h2_trunc):
    _check(_lib.h2_tri_invert(m.h, C.byref(tr)))


def h2_mat_is_inverse(m: Mat) -> bool:
    v = _i32()
    _check(_lib.h2_mat_is_inverse(m.h, C.byref(v)))
    return bool(v.value)


def h2_trsv(m: Mat, r, z, trans: bool = False):
    """z = L^{-1} r (or L^{-*} r); r, z as for h2_precond."""
    nrhs = 1 if r.dim() == 1 else r.shape[0]
    _check(_lib.h2_trsv(m.h, 1 if trans else 0, _ptr(r), _ptr(z), nrhs))


def h2_precond(m: Mat, r, z):
    nrhs = 1 if r.dim() == 1 else r.shape[0]
    _check(_lib.h2_precond(m.h, _ptr(r), _ptr(z), nrhs))


def h2_precond_config(m: Mat, nrhs: int, threads: int):
    _check(_lib.h2_precond_config(m.h, int(nrhs), int(threads)))


def h2_autotune_precond(m: Mat, nrhs: int = 1, reps: int = 5, cache_path: str | None = None):
    """Returns (threads, ms per application, from_cache, {threads: ms} of
    every shape timed)."""
    t, ms, fc, by = _i32(), _d(), _i32(), (_d * 3)()
    path = cache_path.encode() if cache_path else None
    _check(_lib.h2_autotune_precond(m.h, int(nrhs), int(reps), path, C.byref(t), C.byref(ms), C.byref(fc), by))
    return t.value, ms.value, bool(fc.value), ({} if fc.value else dict(zip((128, 256, 512), list(by))))


def h2_csr_create(ctx: Ctx, A) -> Csr:
    n, rp, ci, v = _csr_arrays(A)
    h = _vp()
    _check(_lib.h2_csr_create(ctx.h, n, rp.ctypes.data, ci.ctypes.data, v.ctypes.data, C.byref(h)))
    return Csr(h.value, keep=(ctx,))


def h2_spmv(a: Csr, x, y):
    _check(_lib.h2_spmv(a.h, _ptr(x), _ptr(y)))


def h2_pcg(a: Csr, m: Mat, b, x, rtol: float = 1e-8, maxit: int = 1000):
    it, rel = _i32(), _d()
    st = _lib.h2_pcg(a.h, m.h, _ptr(b), _ptr(x), float(rtol), int(maxit), C.byref(it), C.byref(rel))
    if st != H2_OK and st != -7:
        _check(st)
    return it.value, rel.value, st == H2_OK


def h2_pcg_noalloc(a: Csr, m: Mat, b, x, rtol: float = 1e-8, maxit: int = 1000):
    it, rel = _i32(), _d()
    st = _lib.h2_pcg_noalloc(a.h, m.h, _ptr(b), _ptr(x), float(rtol), int(maxit), C.byref(it), C.byref(rel))
    if st != H2_OK and st != -7:
        _check(st)
    return it.value, rel.value, st == H2_OK
