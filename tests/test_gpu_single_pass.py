"""The single-pass Algorithms 5 and 6 (Section 3.4) on the GPU, against the
FP64 oracle (oracle/single_pass.py), through the C ABI.

Tolerances:
* Two-sided sketch: any summation order satisfies |Y - Y*| <= K u |A||Omega|
  (K the reduction length) plus the test matrix's own rounding (FP32:
  2^-20 (|z| + 1) per entry, FP64: 1e-14 (|z| + 1)).  On a matrix with at
  most two nonzeros per row and per column (entries +-1, +-2, +-1/2) every
  output element is one product or the correctly rounded sum of two, so the
  kernel's Y_c and Y_r equal A times the test matrices it wrote, bit for bit;
  that pins its indexing for both tilings (FP32 and FP64 differ).
* FP64 solves: singular values within 1e-10 sigma_1 (normwise); the joint
  least-squares system of Algorithm 6 and the square system of Algorithm 5
  amplify rounding by their conditioning (kappa(Q^T Omega) of a square
  Gaussian, up to ~1e3 on these sizes), still far below this.  Vectors of
  separated singular values within 1e-7.  Exact-rank inputs are recovered
  to 1e-11.
* FP32 solves: Algorithm 6 meets the 1e-5 sigma_1 normwise bar of the
  two-pass method (its joint system is overdetermined and well conditioned).
  Algorithm 5 solves the square system C (Q^T Omega) = Q^T Y, which
  amplifies the FP32 rounding of the sketch (u = 2^-24 of ||A||) by
  kappa(Q^T Omega): the bound is 8 kappa u |lambda_1| with kappa taken from
  the oracle's Q and Omega (about 2.4e-4 on the test matrix, where 6.4e-5 is
  measured).
"""

import numpy as np
import pytest
import torch

from oracle import philox as OP
from oracle.single_pass import rsvd_alg5, rsvd_alg6
from paper_2402_17794_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2402_17794_amd import rsvd
    rsvd.load_library()
    return rsvd


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _cuda(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def _u(dtype):
    return 2.0 ** -24 if dtype == torch.float32 else 2.0 ** -53


def _omega_tol(dtype):
    return (2.0 ** -20) if dtype == torch.float32 else 1e-14


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("m,n,l,seed", [(1000, 700, 40, 3), (257, 1111, 17, 5), (130, 129, 128, 1),
                                        (2048, 2048, 110, 0)])
def test_dual_sketch_matches_oracle(R, dtype, m, n, l, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    Ad = _cuda(A, dtype)
    Yc, Yr, Oc, Or = (_np(t) for t in R.dual_sketch(Ad, l, seed))
    torch.cuda.synchronize()
    A = _np(Ad)                                      # the values the kernel read
    oc, orr = OP.omega(seed, n, l, stream=0), OP.omega(seed, m, l, stream=1)
    tol = _omega_tol(dtype)
    assert np.all(np.abs(Oc - oc) <= tol * (np.abs(oc) + 1.0))
    assert np.all(np.abs(Or - orr) <= tol * (np.abs(orr) + 1.0))
    u = _u(dtype)
    bc = (n * u + tol) * (np.abs(A) @ (np.abs(oc) + 1.0)) + 1e-300
    br = (m * u + tol) * (np.abs(A.T) @ (np.abs(orr) + 1.0)) + 1e-300
    assert np.all(np.abs(Yc - A @ oc) <= bc)
    assert np.all(np.abs(Yr - A.T @ orr) <= br)


def _two_permutation_matrix(m, n, seed):
    """At most two nonzeros per row and per column, values +-1, +-2, +-1/2."""
    rng = np.random.default_rng(seed)
    A = np.zeros((m, n))
    vals = np.array([1.0, -1.0, 2.0, -2.0, 0.5, -0.5])
    for _ in range(2):
        if m <= n:
            cols = rng.permutation(n)[:m]
            rows = np.arange(m)
        else:
            rows = rng.permutation(m)[:n]
            cols = np.arange(n)
        free = A[rows, cols] == 0
        A[rows[free], cols[free]] = rng.choice(vals, size=int(free.sum()))
    return A


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("m,n,l", [(1500, 1100, 48), (1100, 1500, 110), (333, 4100, 7)])
def test_dual_sketch_indexing_exact(R, dtype, m, n, l):
    A = _two_permutation_matrix(m, n, m + n)
    Ad = _cuda(A, dtype)
    Yc, Yr, Oc, Or = R.dual_sketch(Ad, l, 11)
    torch.cuda.synchronize()
    np_t = np.float32 if dtype == torch.float32 else np.float64
    An, Ocn, Orn = A.astype(np_t), Oc.cpu().numpy(), Or.cpu().numpy()

    def exact(A_, X):
        """Each output is one product or the rounded sum of two: form it in
        the storage type from the (at most two) nonzeros of each row."""
        out = np.zeros((A_.shape[0], X.shape[1]), dtype=np_t)
        for i in range(A_.shape[0]):
            nz = np.nonzero(A_[i])[0]
            acc = np.zeros(X.shape[1], dtype=np_t)
            for j in nz:
                acc = (acc + np_t(A_[i, j]) * X[j]).astype(np_t)
            out[i] = acc
        return out

    assert np.array_equal(Yc.cpu().numpy(), exact(An, Ocn))
    assert np.array_equal(Yr.cpu().numpy(), exact(An.T, Orn))


def _vec_err(Ug, Ur, idx):
    """Largest entry difference of the columns idx (signs already fixed)."""
    return max(float(np.max(np.abs(Ug[:, i] - Ur[:, i]))) for i in idx)


@pytest.mark.parametrize("m,n,k,p", [(600, 400, 20, 10), (513, 777, 30, 6), (1200, 1200, 100, 10)])
def test_alg6_matches_oracle_fp64(R, m, n, k, p):
    sig = W.spectrum_geometric(min(m, n), 0.9)
    A = W.known_spectrum(m, n, sig, 7, 8)
    out = R.solve(_cuda(A, torch.float64), k=k, p=p, seed=4, algorithm=6)
    torch.cuda.synchronize()
    ref = rsvd_alg6(A, k, p, seed=4)
    assert out["info_tensor"].item() == 0
    S = _np(out["S"])
    assert np.max(np.abs(S - ref["S"])) <= 1e-10 * ref["S"][0]
    sep = [i for i in range(min(k, 10)) if abs(ref["S"][i] - ref["S"][i + 1]) > 1e-3 * ref["S"][0]]
    assert _vec_err(_np(out["U"]), ref["U"], sep) <= 1e-7
    assert _vec_err(_np(out["Vt"]).T, ref["Vt"].T, sep) <= 1e-7


def test_alg6_exact_rank_fp64(R):
    A, sig = W.exact_rank(900, 700, 12, 3, 4, top=2.0, ratio=0.75)
    out = R.solve(_cuda(A, torch.float64), k=12, p=8, seed=1, algorithm=6)
    torch.cuda.synchronize()
    S, U, Vt = _np(out["S"]), _np(out["U"]), _np(out["Vt"])
    assert np.max(np.abs(S - sig[:12])) <= 1e-11 * sig[0]
    assert np.max(np.abs((U * S) @ Vt - A)) <= 1e-11 * sig[0]


def test_alg6_matches_oracle_fp32(R):
    sig = W.spectrum_geometric(1500, 0.95, 1e-6)
    A = W.known_spectrum(2000, 1500, sig, 1, 2).astype(np.float32)
    out = R.solve(_cuda(A, torch.float32), k=50, p=10, seed=0, algorithm=6)
    torch.cuda.synchronize()
    ref = rsvd_alg6(A.astype(np.float64), 50, 10, seed=0)
    err = np.max(np.abs(_np(out["S"]) - ref["S"])) / ref["S"][0]
    print(f"alg6 fp32 2000x1500 k=50: normwise sigma error {err:.3e}")
    assert err <= 1e-5


def _sym(n, seed, indefinite=True, ratio=0.9):
    lam = W.spectrum_geometric(n, ratio)
    if indefinite:
        lam = W.alternating_signs(lam)
    return W.symmetric_spectrum(n, lam, seed), lam


@pytest.mark.parametrize("n,k,p,indef", [(500, 20, 10, True), (701, 40, 8, False), (1024, 100, 12, True)])
def test_alg5_matches_oracle_fp64(R, n, k, p, indef):
    A, lam = _sym(n, 9, indef)
    out = R.solve(_cuda(A, torch.float64), k=k, p=p, seed=2, algorithm=5)
    torch.cuda.synchronize()
    ref = rsvd_alg5(A, k, p, seed=2)
    assert out["info_tensor"].item() == 0
    D = _np(out["S"])
    assert np.max(np.abs(D - ref["D"])) <= 1e-10 * abs(ref["D"][0])
    U = _np(out["U"])
    assert np.max(np.abs(_np(out["Vt"]) - U.T)) <= 1e-14
    sep = [i for i in range(min(k, 10))
           if min(abs(abs(ref["D"][i]) - abs(ref["D"][j])) for j in range(k) if j != i) > 1e-3 * abs(ref["D"][0])]
    assert _vec_err(U, ref["U"], sep) <= 1e-7


def test_alg5_exact_rank_fp64(R):
    n, r = 800, 12
    lam = np.zeros(n)
    lam[:r] = W.alternating_signs(0.8 ** np.arange(r))
    A = W.symmetric_spectrum(n, lam, 31)
    out = R.solve(_cuda(A, torch.float64), k=r, p=8, seed=3, algorithm=5)
    torch.cuda.synchronize()
    order = np.argsort(-np.abs(lam[:r]), kind="stable")
    D, U = _np(out["S"]), _np(out["U"])
    assert np.max(np.abs(D - lam[:r][order])) <= 1e-11
    assert np.max(np.abs((U * D) @ U.T - A)) <= 1e-11


def test_alg5_matches_oracle_fp32(R):
    A, lam = _sym(1500, 5, True, 0.95)
    A32 = A.astype(np.float32)
    out = R.solve(_cuda(A32, torch.float32), k=50, p=10, seed=0, algorithm=5)
    torch.cuda.synchronize()
    ref = rsvd_alg5(A32.astype(np.float64), 50, 10, seed=0)
    err = np.max(np.abs(_np(out["S"]) - ref["D"])) / abs(ref["D"][0])
    kappa = np.linalg.cond(ref["Q"].T @ ref["omega"])
    print(f"alg5 fp32 1500 k=50: normwise eigenvalue error {err:.3e}, kappa(Q^T Omega) {kappa:.3e}")
    assert err <= 8 * kappa * 2.0 ** -24


def test_single_pass_full_size_fp32(R):
    """The 8192 x 8192 FP32 workload of the benchmark (sigma_i = max(0.95^i,
    1e-6), Haar factors), k = 100, p = 10, Algorithm 6 against the oracle."""
    sig = W.spectrum_geometric(8192, 0.95, 1e-6)
    Ad = W.known_spectrum(8192, 8192, sig, 1, 2, device="cuda").to(torch.float32)
    out = R.solve(Ad, k=100, p=10, seed=0, algorithm=6)
    torch.cuda.synchronize()
    A = _np(Ad)
    ref = rsvd_alg6(A, 100, 10, seed=0)
    err = np.max(np.abs(_np(out["S"]) - ref["S"])) / ref["S"][0]
    print(f"alg6 fp32 8192^2 k=100: normwise sigma error {err:.3e}")
    assert out["info_tensor"].item() == 0
    assert err <= 1e-5


@pytest.mark.parametrize("alg", [5, 6])
def test_single_pass_nan_reports_nonfinite(R, alg):
    A, _ = _sym(300, 4)
    A[17, 5] = np.nan
    out = R.solve(_cuda(A, torch.float64), k=10, p=5, seed=0, algorithm=alg)
    torch.cuda.synchronize()
    info = out["info_tensor"].item()
    assert info & (R.INFO_NONFINITE | R.INFO_SINGULAR_SYSTEM)


@pytest.mark.parametrize("alg", [5, 6])
def test_single_pass_noalloc_matches(R, alg):
    A, _ = _sym(640, 6)
    Ad = _cuda(A, torch.float64)
    a = R.solve(Ad, k=16, p=8, seed=9, algorithm=alg)
    b = R.solve(Ad, k=16, p=8, seed=9, algorithm=alg, noalloc=True)
    torch.cuda.synchronize()
    assert torch.equal(a["S"], b["S"]) and torch.equal(a["U"], b["U"]) and torch.equal(a["Vt"], b["Vt"])
