"""End-to-end parity of the GPU solve (Algorithm 4) with the FP64 oracle,
through the C ABI, on the same seeded inputs and the same seeded test matrix.

Tolerances:
* FP64 solve: singular values within 1e-12 sigma_1 (normwise), vectors of
  well-separated singular values within 1e-9, residual within 1e-9 relative.
* FP32 solve: top-k singular values within 1e-5 sigma_1 (normwise; FP32
  rounding perturbs every singular value by about u ||A||) and within 1e-5
  relative where sigma_i >= 1e-2 sigma_1 (below it the rounding floor u ||A||
  approaches 1e-5 sigma_i), the Frobenius residual
  within 1% of the oracle's (plus the FP32 floor 16 u ||A||_F, which matters
  only when the exact residual vanishes), and every singular vector whose
  gap to its neighbours exceeds 1e-4 sigma_1 within 8 u sigma_1 / gap_i
  (u = 2^-24) of the oracle's.
* Vectors are compared up to the sign of each column; the GPU's own output
  is separately checked to satisfy the sign convention.
"""

import numpy as np
import pytest
import torch

from oracle.rsvd import residual_norms, rsvd_alg4
from paper_2402_17794_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2402_17794_amd import rsvd
    rsvd.load_library()
    return rsvd


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _align(X, Xref):
    """Flip columns of X to the sign of Xref's."""
    s = np.sign(np.sum(X * Xref, axis=0))
    s[s == 0] = 1.0
    return X * s[None, :]


def _check_sign_convention(Vt):
    for i in range(Vt.shape[0]):
        idx = int(np.argmax(np.abs(Vt[i])))
        assert Vt[i, idx] >= 0.0


def _gaps(S):
    """gap_i = distance from sigma_i to its nearest neighbour among the returned values."""
    gaps = np.full(S.size, np.inf)
    gaps[:-1] = np.minimum(gaps[:-1], S[:-1] - S[1:])
    gaps[1:] = np.minimum(gaps[1:], S[:-1] - S[1:])
    return gaps


def _separated(S, rel=1e-3):
    """Indices i whose sigma_i is separated from its neighbours by rel * sigma_1."""
    gaps = np.full(S.size, np.inf)
    gaps[:-1] = np.minimum(gaps[:-1], S[:-1] - S[1:])
    gaps[1:] = np.minimum(gaps[1:], S[:-1] - S[1:])
    return np.nonzero(gaps > rel * S[0])[0]


def test_c1_fp64_512x256(R):
    """The FP64 configuration: 512 x 256, sigma_i = 0.8^i, k=20, p=10, q=0, seed 0."""
    sig = W.spectrum_geometric(256, 0.8)
    A = W.known_spectrum(512, 256, sig, 1, 2)
    out = R.solve(torch.from_numpy(A).cuda(), k=20, p=10, q=0, seed=0, residual=True, return_q=True)
    torch.cuda.synchronize()
    ref = rsvd_alg4(A, 20, 10, 0, seed=0)
    S = _np(out["S"])
    assert out["l"] == 30
    assert out["info_tensor"].item() == 0
    assert np.max(np.abs(S - ref["S"])) <= 1e-12 * ref["S"][0]
    U, Vt = _np(out["U"]), _np(out["Vt"])
    assert np.max(np.abs(U - ref["U"])) <= 1e-9
    assert np.max(np.abs(Vt - ref["Vt"])) <= 1e-9
    _check_sign_convention(Vt)
    spec, fro = residual_norms(A, ref["Q"])
    assert abs(_np(out["residual_t"])[1] - fro) <= 1e-9 * fro
    Qg = _np(out["Q"])
    assert np.max(np.abs(Qg - ref["Q"])) <= 1e-9


@pytest.mark.parametrize("m,n,k,p,q,seed", [(1000, 600, 20, 10, 0, 0), (600, 1000, 25, 5, 1, 3),
                                            (777, 333, 50, 10, 2, 9), (2048, 2048, 50, 10, 1, 0),
                                            (300, 3000, 100, 10, 2, 1), (129, 65, 60, 10, 1, 2),
                                            (1200, 400, 150, 10, 1, 5)])
def test_fp32_solve_matches_oracle(R, m, n, k, p, q, seed):
    d = min(m, n)
    sig = W.spectrum_geometric(d, 0.95, 1e-6)
    A = W.known_spectrum(m, n, sig, 1, 2)
    A32 = A.astype(np.float32)
    Ad = A32.astype(np.float64)                      # the oracle sees the same (rounded) matrix
    out = R.solve(torch.from_numpy(A32).cuda(), k=k, p=p, q=q, seed=seed, residual=True)
    torch.cuda.synchronize()
    ref = rsvd_alg4(Ad, k, p, q, seed=seed)
    S = _np(out["S"])
    assert np.max(np.abs(S - ref["S"])) <= 1e-5 * ref["S"][0]
    # top-k relative error too, where sigma_i >= 1e-2 sigma_1: below that the
    # FP32 rounding of the products (about u ||A||, u = 2^-24) is itself near
    # 1e-5 sigma_i and only the normwise bound above holds
    big = ref["S"] >= 1e-2 * ref["S"][0]
    assert np.max(np.abs(S - ref["S"])[big] / ref["S"][big]) <= 1e-5
    _, fro = residual_norms(Ad, ref["Q"])
    # 1% of the oracle's residual, above the FP32 rounding floor u ||A||_F
    # (when l = min(m, n) the exact residual is zero).
    floor = 16 * 2.0 ** -24 * np.linalg.norm(Ad)
    assert abs(_np(out["residual_t"])[1] - fro) <= 1e-2 * fro + floor
    U, Vt = _np(out["U"]), _np(out["Vt"])
    assert np.max(np.abs(U.T @ U - np.eye(k))) <= 1e-5
    assert np.max(np.abs(Vt @ Vt.T - np.eye(k))) <= 1e-5
    _check_sign_convention(Vt)
    # Singular vectors, gap-scaled: the FP32 run differs from the FP64 one by a
    # perturbation of about u ||A|| (u = 2^-24), which turns singular vector i
    # by at most about u sigma_1 / gap_i (Wedin); allowed: 8 u sigma_1 / gap_i,
    # on every index whose gap exceeds 1e-4 sigma_1 (measured: at most 0.62).
    gap = _gaps(ref["S"])
    idx = np.nonzero(gap > 1e-4 * ref["S"][0])[0]
    tol = 8 * 2.0 ** -24 * ref["S"][0] / gap[idx]
    Ua = _align(U[:, idx], ref["U"][:, idx])
    errU = np.linalg.norm(Ua - ref["U"][:, idx], axis=0)
    Va = _align(Vt[idx].T, ref["Vt"][idx].T)
    errV = np.linalg.norm(Va - ref["Vt"][idx].T, axis=0)
    print(f"vector error / (u sigma_1 / gap): U {np.max(errU / tol * 8):.2f}, V {np.max(errV / tol * 8):.2f}")
    assert np.all(errU <= tol) and np.all(errV <= tol)


def test_fp64_wide_l(R):
    """l = 200 > 128: the Cholesky and Jacobi kernels run on their device-memory path."""
    sig = W.spectrum_geometric(500, 0.97)
    A = W.known_spectrum(900, 500, sig, 7, 8)
    out = R.solve(torch.from_numpy(A).cuda(), k=190, p=10, q=0, seed=3)
    torch.cuda.synchronize()
    ref = rsvd_alg4(A, 190, 10, 0, seed=3)
    assert np.max(np.abs(_np(out["S"]) - ref["S"])) <= 1e-12 * ref["S"][0]
    U, Vt = _np(out["U"]), _np(out["Vt"])
    idx = _separated(ref["S"], 1e-3)[:20]
    assert np.max(np.abs(_align(U[:, idx], ref["U"][:, idx]) - ref["U"][:, idx])) <= 1e-8
    assert np.max(np.abs(U.T @ U - np.eye(190))) <= 1e-12


@pytest.mark.parametrize("m,n,k,p,ratio", [(500, 260, 120, 9, 0.97), (600, 320, 280, 8, 0.98)])
def test_fp64_block_jacobi_edges(R, m, n, k, p, ratio):
    """l = 129 (9 blocks of 16, one zero block added) and l = 288 (the largest l,
    18 blocks): the block-pair Jacobi and the blocked Cholesky against the oracle."""
    sig = W.spectrum_geometric(n, ratio)
    A = W.known_spectrum(m, n, sig, 11, 12)
    out = R.solve(torch.from_numpy(A).cuda(), k=k, p=p, q=0, seed=9)
    torch.cuda.synchronize()
    ref = rsvd_alg4(A, k, p, 0, seed=9)
    assert out["l"] == k + p
    assert out["info_tensor"].item() & R.INFO_JACOBI_NOT_CONVERGED == 0
    assert np.max(np.abs(_np(out["S"]) - ref["S"])) <= 1e-12 * ref["S"][0]
    U, Vt = _np(out["U"]), _np(out["Vt"])
    assert np.max(np.abs(U.T @ U - np.eye(k))) <= 1e-12
    assert np.max(np.abs(Vt @ Vt.T - np.eye(k))) <= 1e-12
    _check_sign_convention(Vt)
    idx = _separated(ref["S"], 1e-3)[:20]
    assert np.max(np.abs(_align(U[:, idx], ref["U"][:, idx]) - ref["U"][:, idx])) <= 1e-8


def test_rank_deficient_block_jacobi(R):
    """Rank 100 with l = 140: the Gram of B is singular, so the small SVD's
    Cholesky takes its shifted retry and the block Jacobi meets zero columns."""
    A, sig = W.exact_rank(600, 300, 100, 5, 6)
    out = R.solve(torch.from_numpy(A).cuda(), k=140, p=0, q=0, seed=2, return_full_l=True)
    torch.cuda.synchronize()
    S = _np(out["S"])
    assert out["l"] == 140
    assert np.max(np.abs(S[:100] - sig[:100])) <= 1e-12 * sig[0]
    assert np.max(S[100:]) <= 1e-6 * sig[0]
    assert np.all(np.diff(S) <= 0.0)


def test_exact_rank_full_size_takes_the_fallback(R):
    """8192 x 8192 FP32 of exact rank 50 with k = 100, p = 10, q = 2: every
    Y of the power scheme has rank 50 < l = 110, so every orthonormalisation
    takes the Householder fallback at full size; the 50 singular values are
    recovered to FP32 accuracy, the other 50 returned ones are at the
    rounding level, and U, V are orthonormal."""
    m = n = 8192
    r = 50
    sig = 0.8 ** np.arange(r)
    U = W.haar(m, r, 31)
    V = W.haar(n, r, 32)
    A = ((U * sig[None, :]) @ V.T).astype(np.float32)
    out = R.solve(torch.from_numpy(A).cuda(), k=100, p=10, q=2, seed=0)
    torch.cuda.synchronize()
    info = out["info_tensor"].item()
    assert info & R.INFO_QR_FALLBACK and not info & R.INFO_FALLBACK_TIMEOUT
    S = _np(out["S"])
    assert np.max(np.abs(S[:r] - sig)) <= 1e-5 * sig[0]
    assert np.max(S[r:]) <= 1e-5 * sig[0]
    Ug, Vt = _np(out["U"]), _np(out["Vt"])
    assert np.max(np.abs(Ug.T @ Ug - np.eye(100))) <= 1e-5
    assert np.max(np.abs(Vt[:r] @ Vt[:r].T - np.eye(r))) <= 1e-5
    # the leading singular subspace is recovered
    assert np.linalg.norm(U[:, :10] - Ug[:, :10] @ (Ug[:, :10].T @ U[:, :10]), 2) <= 1e-4


def test_exact_rank_fp64(R):
    A, sig = W.exact_rank(700, 300, 12, 5, 6)
    out = R.solve(torch.from_numpy(A).cuda(), k=12, p=8, q=1, seed=4, residual=True)
    torch.cuda.synchronize()
    S = _np(out["S"])
    assert np.max(np.abs(S - sig[:12])) <= 1e-12 * sig[0]
    assert _np(out["residual_t"])[1] <= 1e-12 * sig[0]


def test_zero_matrix_and_full_width(R):
    out = R.solve(torch.zeros((200, 50), dtype=torch.float64, device="cuda"), k=5, p=5, q=1)
    torch.cuda.synchronize()
    assert np.all(_np(out["S"]) == 0.0)
    assert out["info_tensor"].item() & R.INFO_QR_FALLBACK
    # l = min(m, n): an exact SVD
    sig = W.spectrum_geometric(40, 0.7)
    A = W.known_spectrum(90, 40, sig, 3, 4)
    out = R.solve(torch.from_numpy(A).cuda(), k=40, p=10, q=0)
    torch.cuda.synchronize()
    assert out["l"] == 40
    assert np.max(np.abs(_np(out["S"]) - sig)) <= 1e-12 * sig[0]


def test_return_full_l_and_determinism(R):
    A = W.eq41_matrix(2.0, 5, 6).astype(np.float32)
    Ad = torch.from_numpy(A).cuda()
    a = R.solve(Ad, k=25, p=5, q=1, seed=1, return_full_l=True)
    b = R.solve(Ad, k=25, p=5, q=1, seed=1, return_full_l=True)
    torch.cuda.synchronize()
    assert a["U"].shape == (3000, 30) and a["Vt"].shape == (30, 300)
    for key in ("U", "S", "Vt"):
        assert torch.equal(a[key], b[key])
    ref = rsvd_alg4(A.astype(np.float64), 25, 5, 1, seed=1, return_full_l=True)
    assert np.max(np.abs(_np(a["S"]) - ref["S"])) <= 1e-5 * ref["S"][0]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_nonfinite_input_is_reported(R, dtype):
    """A NaN in A reaches the Gram matrices: the solve completes (every loop
    is bounded) and reports RSVD_INFO_NONFINITE."""
    sig = W.spectrum_geometric(300, 0.9)
    A = W.known_spectrum(500, 300, sig, 3, 4)
    A[123, 45] = np.nan
    out = R.solve(torch.from_numpy(A).to(dtype).cuda(), k=20, p=10, q=1, seed=0)
    torch.cuda.synchronize()
    assert out["info_tensor"].item() & R.INFO_NONFINITE


@pytest.mark.parametrize("m,n,k", [(500, 300, 40), (700, 400, 190)])
def test_jacobi_sweep_cap_is_reported(R, m, n, k):
    """A sweep cap of 1 stops the small SVD's Jacobi iteration before it
    converges (both forms: l <= 128 in registers, l > 128 block pairs) and
    sets RSVD_INFO_JACOBI_NOT_CONVERGED; the default cap does not."""
    sig = W.spectrum_geometric(n, 0.97)
    Ad = torch.from_numpy(W.known_spectrum(m, n, sig, 5, 6)).cuda()
    capped = R.solve(Ad, k=k, p=10, q=0, seed=1, jacobi_max_sweeps=1)
    full = R.solve(Ad, k=k, p=10, q=0, seed=1)
    torch.cuda.synchronize()
    assert capped["info_tensor"].item() & R.INFO_JACOBI_NOT_CONVERGED
    assert full["info_tensor"].item() == 0


def test_invalid_arguments_raise(R):
    A = torch.zeros((10, 8), dtype=torch.float32, device="cuda")
    for k, p, q in [(0, 1, 0), (9, 0, 0), (2, -1, 0)]:
        with pytest.raises(R.RsvdError):
            R.solve(A, k=k, p=p, q=q)
