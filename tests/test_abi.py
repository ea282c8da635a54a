"""The C-ABI library loads on the CPU and exports every function that
include/rsvd.h declares; host-only entry points (sizes, validation, status
strings) answer without a GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsvd.h")
LIB = os.path.join(ROOT, "paper_2402_17794_amd", "librsvd.so")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsvd_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("librsvd.so not built: run `python -m paper_2402_17794_amd.build`")
    from paper_2402_17794_amd import rsvd
    return rsvd.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert "rsvd_solve" in names and "rsvd_create" in names
    for name in names:
        assert hasattr(lib, name), name
    from paper_2402_17794_amd import rsvd
    assert set(rsvd.EXPORTS) == set(names)


def test_host_only_entry_points(lib):
    from paper_2402_17794_amd import rsvd
    assert lib.rsvd_l_used(512, 256, 20, 10) == 30
    assert lib.rsvd_l_used(804, 1092, 800, 10) == 804
    assert lib.rsvd_status_string(0) == b"ok"
    assert lib.rsvd_status_string(4) == b"workspace too small"
    A = rsvd.rsvd_matrix(0x1000, rsvd.RSVD_F32, 0, 8192, 8192, 8192)
    nb = ctypes.c_size_t()
    good = rsvd.make_params(100, 10, 2)
    assert lib.rsvd_workspace_size(None, ctypes.byref(A), ctypes.byref(good), ctypes.byref(nb)) == 0
    assert nb.value > 8192 * 112 * 4 * 3
    for k, p, q in [(0, 10, 0), (8193, 0, 0), (10, -1, 0), (10, 5, -2)]:
        bad = rsvd.make_params(k, p, q)
        assert lib.rsvd_workspace_size(None, ctypes.byref(A), ctypes.byref(bad), ctypes.byref(nb)) == 1
    wide = rsvd.make_params(400, 10, 0)          # l = 410 > 288
    assert lib.rsvd_workspace_size(None, ctypes.byref(A), ctypes.byref(wide), ctypes.byref(nb)) == 2
    badld = rsvd.rsvd_matrix(0x1000, rsvd.RSVD_F32, 0, 10, 20, 19)
    assert lib.rsvd_workspace_size(None, ctypes.byref(badld), ctypes.byref(good), ctypes.byref(nb)) == 1
    # solve with a NULL handle is rejected before any device work
    assert lib.rsvd_solve(None, ctypes.byref(A), ctypes.byref(good), None, None, 0, None) == 1
    assert lib.rsvd_solve_noalloc(None, ctypes.byref(A), ctypes.byref(good), None, None) == 1
    assert b"scratch" in lib.rsvd_status_string(rsvd.RSVD_ERR_TOO_LARGE)


def test_single_pass_argument_checks(lib):
    """Algorithms 5 and 6: the host checks of their limits (no GPU needed)."""
    from paper_2402_17794_amd import rsvd
    nb = ctypes.c_size_t()
    sq = rsvd.rsvd_matrix(0x1000, rsvd.RSVD_F32, 0, 4096, 4096, 4096)
    rect = rsvd.rsvd_matrix(0x1000, rsvd.RSVD_F64, 0, 3000, 2000, 2000)

    def ws(A, **kw):
        args = dict(k=100, p=10, q=0)
        args.update(kw)
        p = rsvd.make_params(args.pop("k"), args.pop("p"), args.pop("q"), **args)
        return lib.rsvd_workspace_size(None, ctypes.byref(A), ctypes.byref(p), ctypes.byref(nb))

    for alg in (5, 6):
        assert ws(sq, algorithm=alg) == 0 and nb.value > 4096 * 224 * 4
        assert ws(sq, algorithm=alg, q=1) == 2                   # single pass: no power iterations
        assert ws(sq, algorithm=alg, k=120) == 2                 # l = 130 > 128
        assert ws(sq, algorithm=alg, residual=1) == 2
        assert ws(sq, algorithm=alg, return_full_l=1) == 2
        assert ws(sq, algorithm=alg, test_matrix=rsvd.TEST_SRFT) == 2
    assert ws(rect, algorithm=6) == 0
    assert ws(rect, algorithm=5) == 1                            # Algorithm 5 needs a square A
    assert ws(sq, algorithm=7) == 1
    bf = rsvd.rsvd_matrix(0x1000, rsvd.RSVD_BF16, 0, 4096, 4096, 4096)
    assert ws(bf, algorithm=6) == 2
    # Algorithm 6 holds the row-tile partials of A^T Omega_r: 32 tiles of 128 rows.
    assert ws(sq, algorithm=6) == 0 and nb.value >= 32 * 4096 * 112 * 4
    assert lib.rsvd_dual_sketch_workspace_size(ctypes.byref(sq), 110, ctypes.byref(nb)) == 0
    assert nb.value >= 32 * 4096 * 112 * 4
    assert lib.rsvd_dual_sketch_workspace_size(ctypes.byref(sq), 129, ctypes.byref(nb)) == 2


def test_workspace_grows_with_the_block_jacobi_scratch(lib):
    """The workspace holds the block Jacobi's X (kMaxL^2 doubles) and its
    per-sweep words for any l, so an l > 128 solve needs nothing else."""
    from paper_2402_17794_amd import rsvd
    A = rsvd.rsvd_matrix(0x1000, rsvd.RSVD_F32, 0, 4096, 2048, 2048)
    nb = ctypes.c_size_t()
    p = rsvd.make_params(256, 16, 1)            # l = 272
    assert lib.rsvd_workspace_size(None, ctypes.byref(A), ctypes.byref(p), ctypes.byref(nb)) == 0
    assert nb.value >= 288 * 288 * 8 + 4096 * 272 * 4


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus 2 exits with status 2 and says why,
    before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
