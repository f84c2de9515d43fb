"""Host logic of the serving loop on the CPU: admission by the HBM budget,
first-come-first-served order, rejection of oversized requests, release of
memory, per-request results.  The library and torch are replaced by small
stand-ins (the factorisation "finishes" after a fixed number of polls, the
solve is a sparse direct solve); no method arithmetic is under test here."""
import types

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as w


class _Arr:
    def __init__(self, a):
        self.a = np.array(a, dtype=np.float64)

    def cpu(self):
        return self

    def numpy(self):
        return self.a


def _fake_torch():
    class Stream:
        def __init__(self, device=0):
            self.cuda_stream = 0

        def synchronize(self):
            pass

    class _Ctx:
        def __init__(self, s):
            pass

        def __enter__(self):
            return self

        def __exit__(self, *a):
            return False

    cuda = types.SimpleNamespace(Stream=Stream, stream=_Ctx)
    return types.SimpleNamespace(cuda=cuda, tensor=lambda a, device=None: _Arr(a),
                                 zeros_like=lambda t: _Arr(np.zeros_like(t.a)))


class _FakeLib:
    """Stand-in for the binding: records the device bytes in use."""
    STATUS = {0: "H2_OK", -4: "H2_ERR_NOT_SPD", -7: "H2_ERR_NOT_CONVERGED"}

    def __init__(self, polls=3):
        self.polls = polls
        self.launched = []

    class _H:
        def __init__(self, **kw):
            self.__dict__.update(kw)

        def close(self):
            pass

    def trunc(self, *a):
        return a

    def h2_ctx_create(self, device, stream=None):
        return self._H(device=device)

    def h2_ctree_build(self, ctx, coords, leaf):
        return self._H(n=len(coords))

    def h2_btree_build(self, ctx, ct, eta):
        return self._H(n=ct.n)

    def h2_estimate_bytes(self, bt, lower):
        return 1000 * bt.n

    def h2_mat_from_csr(self, ctx, bt, A, lower=False):
        return self._H(A=A)

    def h2_csr_create(self, ctx, A):
        return self._H(A=A)

    def h2_cholesky_launch(self, mats, tr):
        lib = self
        self.launched.append(len(mats))

        class Job:
            left = lib.polls

            def done(self):
                self.left -= 1
                return self.left <= 0

            def finish(self, check=True):
                return [0] * len(mats)
        return Job()

    def h2_pcg_batched(self, csrs, mats, bs, xs, rtol, maxit, check=True, graph=False):
        its = []
        for c, b, x in zip(csrs, bs, xs):
            B = b.a.reshape(-1, c.A.shape[0])
            x.a[...] = np.stack([spla.spsolve(c.A.tocsc(), B[j]) for j in range(B.shape[0])]).reshape(x.a.shape)
            its += [1] * B.shape[0]
        return its, [0.0] * len(its), [0] * len(its)


@pytest.fixture()
def serve(monkeypatch):
    from paper_1402_5056_amd import serve as s
    monkeypatch.setattr(s, "torch", _fake_torch())
    lib = _FakeLib()
    monkeypatch.setattr(s, "h2lr", lib)
    monkeypatch.setattr(s, "TASK_BYTES_PER_DOF", 0)
    return s, lib


def _reqs(s, specs):
    out = []
    for i, (arrival, side, nrhs) in enumerate(specs):
        p = w.problem(side, sigma_seed=i, rhs_seed=i)
        out.append(s.Request(i, arrival, p["A"], p["coords"], w.gaussian(p["A"].shape[0], nrhs, 50 + i)))
    return out


def test_budget_fifo_and_rejection(serve):
    s, lib = serve
    # estimates: 1000 bytes per unknown; sides 16 -> 225, 24 -> 529, 40 -> 1521 unknowns
    specs = [(0.0, 16, 1), (0.0, 24, 2), (0.0, 16, 3), (0.0, 40, 1), (0.0, 24, 1)]
    srv = s.Server(600_000, slots=2, max_batch=8)
    reqs = srv.run(_reqs(s, specs), poll=0.0)
    assert [r.status for r in reqs] == ["done", "done", "done", "rejected", "done"]
    assert srv.peak <= 600_000
    assert srv.used == 0
    # first come first served: each side-24 request (529,000 B) fits only
    # alone and blocks the queue behind it, so every launch holds one problem
    assert all(k == 1 for k in lib.launched)
    for r in reqs:
        if r.status == "done":
            X = r.result
            res = np.linalg.norm(r.B - r.A @ X) / np.linalg.norm(r.B)
            assert res < 1e-10
            assert r.latency >= 0.0 and len(r.iters) == r.B.shape[1]


def test_batching_when_budget_allows(serve):
    s, lib = serve
    specs = [(0.0, 16, 1)] * 6
    srv = s.Server(10**9, slots=2, max_batch=2)
    reqs = srv.run(_reqs(s, specs), poll=0.0)
    assert all(r.status == "done" for r in reqs)
    assert sum(lib.launched) == 6 and max(lib.launched) == 2
    assert srv.max_inflight == 2


def test_release_policy_argument(serve):
    s, _ = serve
    with pytest.raises(ValueError):
        s.Server(1, release="sometimes")
