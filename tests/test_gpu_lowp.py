"""The precision layer on the GPU, through the C ABI: BF16 and column-scaled
FP8 E4M3 storage of A.

* Quantizers: bit-exact against the oracle's definition (oracle/quant.py).
* Products: the GPU rounds the skinny operand to A's format exactly as the
  oracle's `operand_fp8` / `bf16_bits` do, so the product of the decoded
  operands is known exactly in FP64; the GPU result differs from it only by
  the accumulation: |Y - Y*| <= K u32 |A^| |X^| (u32 = 2^-24) plus the
  rounding of the final scale products for BF16.  The FP8 instruction does
  not round its sum of 32 products as a correctly rounded FP32 sum would:
  measured on gfx950 its error reaches about 2^-16 of the sum of the
  magnitudes of the 32 products, so FP8 adds 2^-14 |A^| |X^| (one such term
  per instruction, bounded by the total).  For the sketch the test matrix is
  generated in FP32 on the GPU, so the bound is against the exact product
  A^ Omega with the operand's rounding added: 2^-8 (BF16) or 2^-4 (FP8)
  relative per element, plus the FP8 subnormal quantum.
* Solves: the singular values come from the Rayleigh-Ritz projection on the
  FP32 copy of A, so sigma_i <= sigma_i(A) exactly (interlacing) up to FP32
  rounding; their distance to the FP64 oracle run with the same number of
  passes (q + 1) on the FP32 copy is the error the precision costs, bounded
  here (normwise, / sigma_1) by 2e-4 for BF16 and 5e-3 for FP8 at these
  sizes (the measured errors are reported by bench.py).
"""

import numpy as np
import pytest
import torch

from oracle import quant as Qz
from oracle.philox import omega as oracle_omega
from oracle.rsvd import rsvd_alg4
from paper_2402_17794_amd import workloads as W

pytestmark = pytest.mark.gpu

FP8_MFMA = 2.0 ** -14       # per-instruction accumulation error of the FP8 product (see above)


@pytest.fixture(scope="module")
def R():
    from paper_2402_17794_amd import rsvd
    rsvd.load_library()
    return rsvd


def _matrix(m, n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) * np.logspace(-2, 1, n)[None, :]
    A[:, 3] = 0.0
    A[5, :] = np.float32(1.5) * (2.0 ** -7)          # exact ties after scaling in some columns
    return A.astype(np.float32)


@pytest.mark.parametrize("m,n", [(257, 130), (64, 48), (1000, 777)])
def test_quantizers_bit_exact(R, m, n):
    A = _matrix(m, n, m + n)
    Ad = torch.from_numpy(A).cuda()
    qb = R.quantize(Ad, R.RSVD_BF16)
    qf = R.quantize(Ad, R.RSVD_FP8_E4M3)
    torch.cuda.synchronize()
    bits = qb.data.cpu().numpy().view(np.uint16)
    assert np.array_equal(bits, Qz.bf16_bits(A))
    Aq, s = Qz.quantize_fp8(A)
    assert np.array_equal(qf.data.cpu().numpy(), Aq)
    assert np.array_equal(qf.col_scale.cpu().numpy(), s)


def test_fp8_rounding_at_every_code_boundary(R):
    """Columns whose largest entry is 448 are quantized with the scale 448 /
    448 = 1, so their entries meet the E4M3 rounding unscaled: every midpoint
    between neighbouring codes (ties to even), one FP32 step either side of
    it, every code itself, the normal/subnormal boundary and values past 448,
    with both signs; bit for bit against the oracle's quantizer."""
    codes = np.arange(0x7f, dtype=np.uint8)                       # 0 .. 0x7e, then 448
    vals = Qz.dequantize_fp8(codes[:, None], np.ones(1, dtype=np.float32))[:, 0].astype(np.float64)
    vals = vals[np.isfinite(vals)]
    mids = (vals[:-1] + vals[1:]) / 2
    pts = np.concatenate([vals, mids, 2.0 ** -6 * np.array([1.0, 0.999, 1.001]), [448.0, 449.0, 464.0, 470.0, 1e6]])
    x = pts.astype(np.float32)
    x = np.concatenate([x, np.nextafter(x, np.float32(0)), np.nextafter(x, np.float32(np.inf))])
    x = np.concatenate([x, -x])
    x = np.minimum(np.abs(x), np.float32(448.0)) * np.sign(x)   # the column maximum stays 448
    x[0] = np.float32(448.0)
    A = np.zeros((x.size, 3), dtype=np.float32)
    A[:, 0] = x
    A[:, 1] = -x
    A[:, 2] = x[::-1]
    qf = R.quantize(torch.from_numpy(A).cuda(), R.RSVD_FP8_E4M3)
    torch.cuda.synchronize()
    Aq, s = Qz.quantize_fp8(A)
    assert np.all(s == 1.0)
    assert np.array_equal(qf.data.cpu().numpy(), Aq)


def _decoded(fmt, q):
    if fmt == 2:
        return Qz.dequantize_bf16(q.data.cpu().numpy().view(np.uint16))
    return Qz.dequantize_fp8(q.data.cpu().numpy(), q.col_scale.cpu().numpy())


@pytest.mark.parametrize("fmt", [2, 3])
@pytest.mark.parametrize("m,n,nc", [(1000, 777, 30), (333, 4099, 110), (2048, 512, 272), (130, 129, 1)])
def test_lowp_products(R, fmt, m, n, nc):
    A = _matrix(m, n, 7 * m + n)
    q = R.quantize(torch.from_numpy(A).cuda(), fmt)
    Ah = _decoded(fmt, q)
    s = q.col_scale.cpu().numpy() if fmt == 3 else None
    u = 2.0 ** -24
    rng = np.random.default_rng(nc)
    # Y = A X
    X = rng.standard_normal((n, nc)).astype(np.float32)
    Y = R.gemm(q, torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    if fmt == 2:
        Xh = Qz.dequantize_bf16(Qz.bf16_bits(X))
        ref, bound = Ah @ Xh, n * u * (np.abs(Ah) @ np.abs(Xh))
    else:
        Xq, t = Qz.operand_fp8(X, row_scale=s)
        Xd = Qz.e4m3_value(Xq).astype(np.float64)
        Aqd = Qz.e4m3_value(q.data.cpu().numpy()).astype(np.float64)
        ref = (Aqd @ Xd) * t[None, :]
        bound = ((n + 4) * u + FP8_MFMA) * (np.abs(Aqd) @ np.abs(Xd)) * t[None, :]
    assert np.all(np.abs(Y - ref) <= bound + 1e-30)
    # Z = A^T Y
    Yin = rng.standard_normal((m, nc)).astype(np.float32)
    Z = R.gemm(q, torch.from_numpy(Yin).cuda(), trans=True).cpu().numpy().astype(np.float64)
    if fmt == 2:
        Yh = Qz.dequantize_bf16(Qz.bf16_bits(Yin))
        ref, bound = Ah.T @ Yh, m * u * (np.abs(Ah.T) @ np.abs(Yh))
    else:
        Yq, t = Qz.operand_fp8(Yin)
        Yd = Qz.e4m3_value(Yq).astype(np.float64)
        Aqd = Qz.e4m3_value(q.data.cpu().numpy()).astype(np.float64)
        ref = s[:, None] * (Aqd.T @ Yd) * t[None, :]
        bound = ((m + 4) * u + FP8_MFMA) * s[:, None] * (np.abs(Aqd.T) @ np.abs(Yd)) * t[None, :]
    assert np.all(np.abs(Z - ref) <= bound + 1e-30)
    # sketch with the generated test matrix
    S = R.gemm(q, None, seed=5, ncols=nc).cpu().numpy().astype(np.float64)
    Om = oracle_omega(5, n, nc)
    rel = 2.0 ** -8 if fmt == 2 else 2.0 ** -4
    sub = 0.0
    if fmt == 3:
        # half the FP8 subnormal quantum of the scaled test matrix, 2^-10 t with
        # t = 5.77 max(s) / 448, times the unscaled codes of A it multiplies
        Aqd = Qz.e4m3_value(q.data.cpu().numpy()).astype(np.float64)
        sub = 2.0 ** -10 * 5.77 * np.max(s) / 448.0 * np.sum(np.abs(Aqd), axis=1)[:, None]
    acc = n * u + (FP8_MFMA if fmt == 3 else 0.0)
    bound = (rel + 2.0 ** -19 + acc) * (np.abs(Ah) @ (np.abs(Om) + 1.0)) + sub
    assert np.all(np.abs(S - Ah @ Om) <= bound)


@pytest.mark.parametrize("fmt,tol", [(2, 2e-4), (3, 5e-3)])
def test_lowp_solve(R, fmt, tol):
    m, n, k, p, q = 2048, 1024, 64, 16, 2
    sig = W.spectrum_power(n, 1.5)
    A32 = W.known_spectrum(m, n, sig, 1, 2).astype(np.float32)
    Ad = A32.astype(np.float64)
    qa = R.quantize(torch.from_numpy(A32).cuda(), fmt)
    out = R.solve(qa, k=k, p=p, q=q, seed=0, residual=2, return_q=True)
    torch.cuda.synchronize()
    S = out["S"].cpu().numpy()
    exact = np.linalg.svd(Ad, compute_uv=False)[:k]
    assert np.all(S <= exact * (1 + 1e-6) + 1e-6 * exact[0])                 # interlacing on the FP32 A
    ref = rsvd_alg4(Ad, k, p, q + 1, seed=0)                                # same number of passes
    assert np.max(np.abs(S - ref["S"])) <= tol * ref["S"][0]
    Qg = out["Q"].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(Qg.T @ Qg - np.eye(Qg.shape[1]))) <= 2e-6
    U, Vt = out["U"].cpu().numpy().astype(np.float64), out["Vt"].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(U.T @ U - np.eye(k))) <= 2e-5 and np.max(np.abs(Vt @ Vt.T - np.eye(k))) <= 2e-5
    E = Ad - Qg @ (Qg.T @ Ad)
    assert abs(out["residual_t"].cpu().numpy()[1] - np.linalg.norm(E)) <= 1e-3 * np.linalg.norm(E)
    assert out["info_tensor"].item() == 0


def test_lowp_argument_checks(R):
    A = torch.zeros((64, 40), dtype=torch.float32, device="cuda")
    q = R.quantize(A, R.RSVD_FP8_E4M3, keep_master=False)
    with pytest.raises(R.RsvdError):
        R.solve(q, k=4, p=2, residual=2)                     # residual needs the FP32 copy
    q.col_scale = None
    with pytest.raises(R.RsvdError):
        R.solve(q, k=4, p=2)                                 # FP8 without scales
