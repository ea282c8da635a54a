"""The SRFT test matrix (FastRandRF, Appendix A) on the GPU against the
oracle (oracle/srft.py):

* sampled columns: bit-exact (integer work: Philox words, Floyd's algorithm);
* the materialised matrix: FP64 within 1e-13 (|z| + 1), FP32 within
  2^-20 (|z| + 1) (hardware cosine of an exactly reduced argument);
* a whole solve with the SRFT sketch (q = 0: FastRandRF followed by Stage 2;
  q = 1, 2: the same power scheme) against the oracle run with the same
  materialised test matrix: FP64 sigma within 1e-12 sigma_1, FP32 within
  1e-5 sigma_1 (normwise), and exact recovery of an exact-rank matrix.
"""

import numpy as np
import pytest
import torch

from oracle import srft as OS
from oracle.rsvd import residual_norms, rsvd_alg4
from paper_2402_17794_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_2402_17794_amd import rsvd
    rsvd.load_library()
    return rsvd


@pytest.mark.parametrize("n,l,seed", [(64, 10, 0), (1000, 110, 3), (257, 257, 1), (8192, 110, 0), (70000, 288, 7)])
def test_srft_matrix_matches_oracle(R, n, l, seed):
    ref = OS.srft_omega(seed, n, l)
    g64, c64 = R.srft_omega(n, l, seed, torch.float64)
    assert np.array_equal(c64.cpu().numpy(), OS.srft_columns(seed, n, l))
    assert np.all(np.abs(g64.cpu().numpy() - ref) <= 1e-13 * (np.abs(ref) + 1.0))
    g32, c32 = R.srft_omega(n, l, seed, torch.float32)
    assert np.array_equal(c32.cpu().numpy(), OS.srft_columns(seed, n, l))
    assert np.all(np.abs(g32.cpu().numpy().astype(np.float64) - ref) <= 2.0 ** -20 * (np.abs(ref) + 1.0))


@pytest.mark.parametrize("dtype,q", [(torch.float64, 0), (torch.float64, 1), (torch.float32, 0), (torch.float32, 2)])
def test_srft_solve_matches_oracle(R, dtype, q):
    m, n, k, p = 1500, 900, 40, 10
    sig = W.spectrum_geometric(n, 0.95)
    A = W.known_spectrum(m, n, sig, 41, 42)
    if dtype == torch.float32:
        A = A.astype(np.float32).astype(np.float64)
    out = R.solve(torch.from_numpy(A).to(dtype).cuda(), k=k, p=p, q=q, seed=6, test_matrix=R.TEST_SRFT)
    torch.cuda.synchronize()
    ref = rsvd_alg4(A, k, p, q, omega=OS.srft_omega(6, n, k + p))
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert out["info_tensor"].item() == 0
    assert np.max(np.abs(out["S"].cpu().numpy() - ref["S"])) <= tol * ref["S"][0]


def test_srft_solve_exact_rank(R):
    A, sig = W.exact_rank(2000, 700, 20, 8, 9)
    out = R.solve(torch.from_numpy(A).cuda(), k=20, p=20, q=0, seed=1, test_matrix=R.TEST_SRFT, residual=True,
                  return_q=True)
    torch.cuda.synchronize()
    assert np.max(np.abs(out["S"].cpu().numpy() - sig[:20])) <= 1e-12 * sig[0]
    assert out["residual_t"].cpu().numpy()[1] <= 1e-12 * np.linalg.norm(sig)
