"""The allocation-free entry point rsvd_solve_noalloc (the library's fixed
device scratch in place of a caller workspace) gives the same results as
rsvd_solve on the same inputs: bit for bit, since both run the same
deterministic kernels.  Two calls in a row, the second on a smaller
problem, then the first again, so a stale scratch state would show; a
problem larger than the scratch is refused before anything is enqueued."""

import ctypes

import numpy as np
import pytest
import torch

from paper_2402_17794_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2402_17794_amd import rsvd
    rsvd.load_library()
    return rsvd


def _input(m, n, dtype, seed):
    sig = W.spectrum_geometric(min(m, n), 0.97)
    A = W.known_spectrum(m, n, sig, seed, seed + 1)
    return torch.from_numpy(A).to("cuda:0", dtype)


def _pair(R, A, k, p, q, seed, residual=0):
    kw = dict(k=k, p=p, q=q, seed=seed, residual=residual)
    ref = R.Solver(A, **kw)()
    na = R.Solver(A, noalloc=True, **kw)
    assert na.ws is None
    na()
    torch.cuda.synchronize()
    return ref, na


def _assert_same(ref, na):
    for name in ("U", "S", "Vt", "info"):
        a, b = getattr(ref, name).cpu(), getattr(na, name).cpu()
        assert torch.equal(a, b), name
    if ref.res is not None:
        assert torch.equal(ref.res.cpu(), na.res.cpu())
    assert int(ref.info.item()) == 0


def test_noalloc_equals_workspace_solve_then_smaller(R):
    print("noalloc: call 1, 4096 x 2048 f32, k=100 p=10 q=2, residual both", flush=True)
    A1 = _input(4096, 2048, torch.float32, 11)
    ref1, na1 = _pair(R, A1, 100, 10, 2, 3, residual=3)
    _assert_same(ref1, na1)
    S = na1.S.cpu().numpy()
    assert np.all(np.diff(S) <= 0) and S[0] > 0
    print("noalloc: call 2 (smaller), 1000 x 700 f64, k=20 p=10 q=1", flush=True)
    A2 = _input(1000, 700, torch.float64, 21)
    ref2, na2 = _pair(R, A2, 20, 10, 1, 5)
    _assert_same(ref2, na2)
    print("noalloc: call 3, the first problem again", flush=True)
    na1b = R.Solver(A1, k=100, p=10, q=2, seed=3, residual=3, noalloc=True)()
    torch.cuda.synchronize()
    _assert_same(ref1, na1b)


def test_noalloc_refuses_a_problem_beyond_the_scratch(R):
    lib = R.load_library()
    h = R._handle("cuda:0")
    M = R.rsvd_matrix(0x100000, R.RSVD_F32, 0, 32768, 16384, 16384)
    prm = R.make_params(256, 16, 2)
    nb = ctypes.c_size_t()
    assert lib.rsvd_workspace_size(h, ctypes.byref(M), ctypes.byref(prm), ctypes.byref(nb)) == 0
    assert nb.value > R.NOALLOC_SCRATCH_BYTES
    res = R.rsvd_result(0x1000, 256, 0x1000, 0x1000, 16384, None, 0x1000, None, 0)
    st = lib.rsvd_solve_noalloc(h, ctypes.byref(M), ctypes.byref(prm), ctypes.byref(res), None)
    assert st == R.RSVD_ERR_TOO_LARGE
    assert b"scratch" in lib.rsvd_status_string(st)
