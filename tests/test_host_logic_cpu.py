"""Host logic of the C ABI on the CPU: the library is loaded in a child
process against a host-only stand-in for the HIP runtime (memory is host
memory, kernels do nothing), so argument checks, job and busy bookkeeping
and the byte accounting run without a GPU.  No numerical result is checked
here; the GPU tests do that."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1402_5056_amd", "libh2lr.so")

CHILD = textwrap.dedent(r'''
    import ctypes as C, sys
    import numpy as np
    sys.path.insert(0, ROOT)
    import workloads as w
    lib = C.CDLL(LIB)
    vp = C.c_void_p
    lib.h2_last_error.restype = C.c_char_p

    class trunc(C.Structure):
        _fields_ = [("eps", C.c_double), ("mode", C.c_int32), ("rank_cap", C.c_int32), ("precision", C.c_int32),
                    ("accumulate", C.c_int32), ("level_factor", C.c_double)]

    def ok(st):
        assert st == 0, lib.h2_last_error()

    ctx = vp(); ok(lib.h2_ctx_create(0, None, C.byref(ctx)))
    keep = []

    def matrix(side, leaf, lower):
        p = w.problem(side, sigma_seed=3, rhs_seed=1); A = p["A"].tocsr()
        xy = np.ascontiguousarray(p["coords"], dtype=np.int32)
        ct = vp(); ok(lib.h2_ctree_build(ctx, C.c_int32(2), C.c_int64(len(xy)), xy.ctypes.data_as(vp), C.c_int32(leaf), C.byref(ct)))
        bt = vp(); ok(lib.h2_btree_build(ctx, ct, C.c_double(2.0), C.byref(bt)))
        rp = np.ascontiguousarray(A.indptr, np.int64); ci = np.ascontiguousarray(A.indices, np.int32); v = np.ascontiguousarray(A.data)
        keep.extend([xy, rp, ci, v])
        est = C.c_int64(); ok(lib.h2_estimate_bytes(bt, C.c_int32(lower), C.byref(est)))
        m = vp(); ok(lib.h2_mat_from_csr(ctx, bt, C.c_int64(A.shape[0]), rp.ctypes.data_as(vp), ci.ctypes.data_as(vp), v.ctypes.data_as(vp), C.c_int32(lower), C.byref(m)))
        now = C.c_int64(); ok(lib.h2_mat_bytes(m, C.byref(now)))
        assert now.value == est.value, (now.value, est.value)
        return m, A.shape[0]

    tr = trunc(1e-6, 0, 32, 0)
    (L1, n1), (L2, n2), (F, nf) = matrix(16, 8, 1), matrix(24, 16, 1), matrix(16, 8, 0)
    arr = (vp * 2)(L1.value, L2.value)
    st = (C.c_int * 2)()
    # launch: the matrices are busy until the job is finished
    job = vp(); ok(lib.h2_cholesky_launch(arr, 2, C.byref(tr), C.byref(job)))
    assert lib.h2_cholesky(L1, C.byref(tr)) == -1
    assert lib.h2_mat_assign(L1, L2) == -1
    assert lib.h2_mat_destroy(L2) == -8
    d = C.c_int32(); ok(lib.h2_job_query(job, C.byref(d)))
    ok(lib.h2_job_finish(job, st)); assert list(st) == [0, 0]
    ok(lib.h2_cholesky(L1, C.byref(tr)))
    # truncation parameters are checked before any device work: mode, rank
    # cap, eps, precision, the accumulation flag and the level factor
    nan, inf = float("nan"), float("inf")
    for bad in (trunc(1e-6, 3, 32, 0), trunc(1e-6, -1, 32, 0), trunc(1e-6, 0, 0, 0), trunc(1e-6, 0, 33, 0),
                trunc(-1e-6, 0, 32, 0), trunc(nan, 0, 32, 0), trunc(inf, 0, 32, 0), trunc(1e-6, 0, 32, 3),
                trunc(1e-6, 0, 32, 0, 2), trunc(1e-6, 0, 32, 0, -1), trunc(1e-6, 0, 32, 0, 0, 1.5),
                trunc(1e-6, 0, 32, 0, 0, -0.5), trunc(1e-6, 0, 32, 0, 0, nan)):
        assert lib.h2_cholesky(L1, C.byref(bad)) == -1, (bad.mode, bad.rank_cap, bad.eps, bad.level_factor)
        assert b"must" in lib.h2_last_error(), lib.h2_last_error()
        assert lib.h2_cholesky_batched(arr, 2, C.byref(bad), st) == -1
    for good in (trunc(1e-6, 1, 32, 1, 1, 0.5), trunc(0.0, 2, 1, 2, 0, 1.0), trunc(1e-6, 0, 32, 0, 0, 0.0)):
        ok(lib.h2_cholesky(L1, C.byref(good)))
    ok(lib.h2_cholesky(L1, None))                     # no parameters: exact arithmetic
    # batch argument checks
    dup = (vp * 2)(L1.value, L1.value)
    assert lib.h2_cholesky_batched(dup, 2, C.byref(tr), st) == -1
    assert lib.h2_cholesky_batched(arr, 0, C.byref(tr), st) == -1
    full = (vp * 1)(F.value)
    assert lib.h2_cholesky_batched(full, 1, C.byref(tr), st) == -1   # not a lower factor
    # batched updates: counts and block range checked before any device work
    X = np.zeros((nf, 2))
    one = (vp * 1)(F.value)
    nup = (C.c_int32 * 1)(1); blk = (C.c_int64 * 1)(0); ks = (C.c_int32 * 1)(2)
    xs = (vp * 1)(X.ctypes.data); ld = (C.c_int64 * 1)(nf); s1 = (C.c_int * 1)()
    ok(lib.h2_lowrank_update_batched(one, 1, nup, blk, ks, xs, ld, xs, ld, C.byref(tr), s1))
    nup5 = (C.c_int32 * 1)(5)
    assert lib.h2_lowrank_update_batched(one, 1, nup5, blk, ks, xs, ld, xs, ld, C.byref(tr), s1) == -1
    bad = (C.c_int64 * 1)(10 ** 7)
    assert lib.h2_lowrank_update_batched(one, 1, nup, bad, ks, xs, ld, xs, ld, C.byref(tr), s1) == -1
    # single triangular solves need a lower factor and trans in {0, 1}
    r = np.zeros(nf)
    assert lib.h2_trsv(F, C.c_int32(0), r.ctypes.data_as(vp), r.ctypes.data_as(vp), C.c_int32(1)) == -1
    r1 = np.zeros(n1)
    assert lib.h2_trsv(L1, C.c_int32(2), r1.ctypes.data_as(vp), r1.ctypes.data_as(vp), C.c_int32(1)) == -1
    ok(lib.h2_trsv(L1, C.c_int32(1), r1.ctypes.data_as(vp), r1.ctypes.data_as(vp), C.c_int32(1)))
    # batched PCG: per-system column counts within [1, H2_MAX_COLS]
    A1 = w.problem(16, sigma_seed=3, rhs_seed=1)["A"].tocsr()
    rp = np.ascontiguousarray(A1.indptr, np.int64); ci = np.ascontiguousarray(A1.indices, np.int32)
    vv = np.ascontiguousarray(A1.data); keep.extend([rp, ci, vv])
    csr = vp(); ok(lib.h2_csr_create(ctx, C.c_int64(n1), rp.ctypes.data_as(vp), ci.ctypes.data_as(vp), vv.ctypes.data_as(vp), C.byref(csr)))
    b = np.zeros(n1 * 65); x = np.zeros(n1 * 65)
    As = (vp * 1)(csr.value); Ls = (vp * 1)(L1.value); bs = (vp * 1)(b.ctypes.data); xs1 = (vp * 1)(x.ctypes.data)
    for k, want in ((65, -1), (0, -1), (3, 0)):
        nr = (C.c_int32 * 1)(k)
        got = lib.h2_pcg_batched(As, Ls, bs, xs1, nr, 1, C.c_double(1e-8), C.c_int32(10), None, None, None)
        assert got == want, (k, got, lib.h2_last_error())
    # updates on trees with block rows of more than 64 admissible blocks are
    # refused (the domain-decomposition 256 x 256 tree at eta 4 has 89)
    pd = w.problem(256, rhs_seed=1); Ad = pd["A"].tocsr()
    xyd = np.ascontiguousarray(pd["coords"], dtype=np.int32)
    ctd = vp(); ok(lib.h2_ctree_build_dd(ctx, C.c_int32(2), C.c_int64(len(xyd)), xyd.ctypes.data_as(vp), C.c_int32(32), C.byref(ctd)))
    btd = vp(); ok(lib.h2_btree_build(ctx, ctd, C.c_double(4.0), C.byref(btd)))
    csp = C.c_int32(); ok(lib.h2_btree_info(btd, None, None, None, C.byref(csp))); assert csp.value == 89
    rpd = np.ascontiguousarray(Ad.indptr, np.int64); cid = np.ascontiguousarray(Ad.indices, np.int32); vd = np.ascontiguousarray(Ad.data)
    keep.extend([xyd, rpd, cid, vd])
    Ld = vp(); ok(lib.h2_mat_from_csr(ctx, btd, C.c_int64(Ad.shape[0]), rpd.ctypes.data_as(vp), cid.ctypes.data_as(vp), vd.ctypes.data_as(vp), C.c_int32(1), C.byref(Ld)))
    assert lib.h2_cholesky(Ld, C.byref(tr)) == -1 and b"not validated" in lib.h2_last_error()
    assert lib.h2_tri_invert(Ld, C.byref(tr)) == -1
    ok(lib.h2_mat_destroy(Ld))
    print("host logic ok")
''')


@pytest.fixture(scope="module")
def stub_dir(tmp_path_factory):
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    d = tmp_path_factory.mktemp("hipstub")
    ver = d / "ver.map"
    # symbol versions of the runtime: graphs hip_4.3, the stream-ordered
    # allocator hip_5.1, the device properties hip_6.0
    ver.write_text("hip_4.2 { global: *; };\n"
                   "hip_4.3 { global: hipStreamBeginCapture; hipStreamEndCapture; hipGraphInstantiate; "
                   "hipGraphLaunch; hipGraphExecDestroy; hipGraphDestroy; } hip_4.2;\n"
                   "hip_5.1 { global: hipMallocAsync; hipFreeAsync; hipDeviceGetDefaultMemPool; "
                   "hipMemPoolSetAttribute; } hip_4.3;\n"
                   "hip_6.0 { global: hipGetDevicePropertiesR0600; } hip_5.1;\n")
    src = os.path.join(ROOT, "tests", "host_stub", "hip_host_stub.c")
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", "-o", str(d / "libamdhip64.so.7"), src,
                    f"-Wl,--version-script={ver}", "-Wl,-soname,libamdhip64.so.7"], check=True)
    return str(d)


def test_host_logic_under_stub_runtime(stub_dir):
    env = dict(os.environ, LD_LIBRARY_PATH=stub_dir)
    code = f"ROOT = {ROOT!r}\nLIB = {LIB!r}\n" + CHILD
    res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "host logic ok" in res.stdout
