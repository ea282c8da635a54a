"""Canonical angles (Section 4.3, Theorem 5) and the adaptive range finder
(Appendix A) on the GPU, against the oracle (oracle/angles.py,
oracle/bounds.py, oracle/adaptive.py).

Tolerances: the GPU sines come from the FP64 Gram of the projection
residual E = (I - U2 U2^T) U1, so their error is about u ||E||^2 / s + u
(u = 2^-53) in FP64 (bound used: 64 u (1 + ||E||^2 / max(s, 1e-6))); FP32
inputs carry their own rounding of about 2^-24, so sines are compared to
2e-6 there.  The adaptive range finder draws the same test vectors as the
oracle, so in FP64, on spectra without singular values near the tolerance,
both take the same decisions: the same number of columns and the same
estimate (to 1e-9 relative); in FP32 the rounding can move a block's
singular value across the keep threshold, so the basis size is compared to
within one block.  Every result meets the tolerance.
"""

import numpy as np
import pytest
import torch

from oracle import adaptive as OA
from oracle import angles as OG
from oracle import bounds
from oracle.philox import omega
from paper_2402_17794_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2402_17794_amd import rsvd
    rsvd.load_library()
    return rsvd


def _bases(rows, k, l, seed, scale):
    rng = np.random.default_rng(seed)
    U1 = np.linalg.qr(rng.standard_normal((rows, k)))[0]
    U2 = np.linalg.qr(np.concatenate([U1 + scale * rng.standard_normal((rows, k)),
                                      rng.standard_normal((rows, l - k))], axis=1))[0]
    return U1, U2


@pytest.mark.parametrize("rows,k,l,scale", [(3000, 25, 30, 1e-3), (500, 7, 12, 0.3), (8192, 100, 110, 1e-2),
                                            (1000, 16, 16, 1e-5)])
def test_canonical_sines_match_oracle(R, rows, k, l, scale):
    U1, U2 = _bases(rows, k, l, rows + k, scale)
    ref = OG.canonical_sines(U1, U2)
    g = R.canonical_sines(torch.from_numpy(U1).cuda(), torch.from_numpy(U2).cuda()).cpu().numpy()
    u = 2.0 ** -53
    e2 = np.linalg.norm(U1 - U2 @ (U2.T @ U1), 2) ** 2
    assert np.all(np.abs(g - ref) <= 64 * u * (1 + e2 / np.maximum(ref, 1e-6)))
    g32 = R.canonical_sines(torch.from_numpy(U1).float().cuda(), torch.from_numpy(U2).float().cuda()).cpu().numpy()
    assert np.all(np.abs(g32 - ref) <= 2e-6)


def test_canonical_sines_edge_cases(R):
    """A subspace against itself (all sines 0) and against an orthogonal one
    (all sines 1)."""
    U = np.linalg.qr(np.random.default_rng(1).standard_normal((400, 20)))[0]
    Ud = torch.from_numpy(U).cuda()
    assert np.max(R.canonical_sines(Ud[:, :8].contiguous(), Ud).cpu().numpy()) <= 1e-7
    s = R.canonical_sines(Ud[:, :8].contiguous(), Ud[:, 8:].contiguous()).cpu().numpy()
    assert np.all(np.abs(s - 1.0) <= 1e-12)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_theorem5_on_the_gpu_sketch(R, q):
    """Section 4.3 setting: eq. (4.1) stand-in with gap 2 after sigma_15,
    k = 25, p = 5.  The canonical sines between U_k and the GPU's full
    l-column U (range(Q) of Algorithm 4) meet Theorem 5's bound and equal the
    oracle's for the same test matrix."""
    from oracle.rsvd import rsvd_alg4
    m, n, k, p = 3000, 300, 25, 5
    sig = W.eq41_spectrum(n, 2.0)
    U = W.haar(m, n, 1)
    V = W.haar(n, n, 2)
    A = (U * sig[None, :]) @ V.T
    out = R.solve(torch.from_numpy(A).cuda(), k=k, p=p, q=q, seed=3, return_full_l=True)
    torch.cuda.synchronize()
    Uk = torch.from_numpy(np.ascontiguousarray(U[:, :k])).cuda()
    st = R.canonical_sines(Uk, out["U"]).cpu().numpy()
    bt, _ = bounds.thm5(sig, k, q, omega(3, n, k + p), V)
    assert np.all(st <= bt * (1 + 1e-9) + 1e-12)
    ref = OG.canonical_sines(U[:, :k], rsvd_alg4(A, k, p, q, seed=3, return_full_l=True)["U"])
    assert np.all(np.abs(st - ref) <= 1e-9 + 1e-6 * ref)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("tol,block", [(1e-2, 16), (1e-4, 8), (3e-4, 32)])
def test_adaptive_range_matches_oracle(R, dtype, tol, block):
    sig = W.spectrum_geometric(600, 0.93)
    A = W.known_spectrum(1200, 600, sig, 5, 6)
    if dtype == torch.float32:
        A = A.astype(np.float32).astype(np.float64)
    Q, est, conv = R.adaptive_range(torch.from_numpy(A).to(dtype).cuda(), tol, block=block, seed=4)
    ref = OA.adaptive_range_finder(A, tol, block=block, seed=4)
    assert conv and ref["converged"]
    Qg = Q.cpu().numpy().astype(np.float64)
    eps = 1e-12 if dtype == torch.float64 else 1e-5
    assert np.max(np.abs(Qg.T @ Qg - np.eye(Qg.shape[1]))) <= eps
    assert np.linalg.svd(A - Qg @ (Qg.T @ A), compute_uv=False)[0] <= tol
    if dtype == torch.float64:
        assert Q.shape[1] == ref["l"]
        assert abs(est - ref["est"]) <= 1e-9 * ref["est"]
    else:
        # FP32 rounding can move a singular value of a block across the keep
        # threshold tol / (10 sqrt(2/pi)): several bases are then correct; the
        # size stays within a block of the oracle's
        assert abs(Q.shape[1] - ref["l"]) <= block


def test_adaptive_range_exact_rank_and_cap(R):
    A, _ = W.exact_rank(2000, 900, 37, 7, 8)
    Q, est, conv = R.adaptive_range(torch.from_numpy(A).cuda(), 1e-9, block=16, seed=1)
    assert conv and Q.shape[1] == 37 and est <= 1e-9
    Qg = Q.cpu().numpy()
    assert np.linalg.norm(A - Qg @ (Qg.T @ A)) <= 1e-12 * np.linalg.norm(A)
    sig = W.spectrum_geometric(400, 0.97)
    B = W.known_spectrum(800, 400, sig, 9, 10)
    Q, est, conv = R.adaptive_range(torch.from_numpy(B).cuda(), 1e-12, block=16, max_l=64, seed=2)
    ref = OA.adaptive_range_finder(B, 1e-12, block=16, max_l=64, seed=2)
    assert not conv and not ref["converged"] and Q.shape[1] == ref["l"]
