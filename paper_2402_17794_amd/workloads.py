"""Seeded synthetic input matrices shaped like the paper's test problems.

This module only draws inputs; it holds none of the randomized-SVD
arithmetic.  Both the GPU path and the FP64 CPU oracle are fed the matrices
produced here.  Random draws use numpy's PCG64 generator (`default_rng`), not
the Philox generator of the test matrix, so that the inputs are independent
of the method's own random numbers.

Families
  known_spectrum  A = U diag(sigma) V^T with Haar-distributed U, V (thin QR of
                  a Gaussian matrix with the signs of diag(R) folded in, the
                  standard recipe for the Haar measure).
  spectra         the singular-value profiles of the benchmark configurations:
                  geometric 0.8^i (512 x 256), max(0.95^i, 1e-6) (8192^2),
                  1/i (2048^2 slow decay), i^-1.5 (mixed precision,
                  32768 x 16384).
  eq41_spectrum   the test family of eq. (4.1) (Section 4.2): singular values
                  gap/j for j <= r and 1/j after, m x n = 3000 x 300, r = 15.
                  The paper builds it from sparse nonnegative vectors of
                  unspecified density; this stand-in uses Haar factors so the
                  spectrum is exactly the stated one.
  image           the image-restoration stand-in (Section 4.1 uses a
                  photograph that is not available): a 2048 x 2048 sum of 60
                  separable Gaussian bumps, min-max normalised to [0, 1], plus
                  i.i.d. N(0, 0.05^2) noise.
  exact_rank      A = U diag(sigma_1..r) V^T of exact rank r.
  symmetric_spectrum  symmetric A = U diag(lambda) U^T with Haar U (the
                  Hermitian inputs of the single-pass Algorithm 5), with
                  alternating_signs for indefinite spectra.
"""

import numpy as np


def _rng(seed):
    return np.random.default_rng(int(seed))


def haar(rows, cols, seed, device=None):
    """rows x cols matrix with orthonormal columns, Haar-distributed.

    With `device` set to a torch CUDA device the QR runs there in float64
    (the Gaussian draw stays on the host, so the matrix depends only on the
    seed up to the rounding of the QR); the result is returned as a float64
    torch tensor on that device."""
    if cols > rows:
        raise ValueError("haar needs rows >= cols")
    G = _rng(seed).standard_normal((rows, cols))
    if device is None:
        Q, R = np.linalg.qr(G)
        d = np.where(np.diag(R) < 0, -1.0, 1.0)
        return Q * d[None, :]
    import torch
    Gt = torch.from_numpy(G).to(device)
    Q, R = torch.linalg.qr(Gt)
    d = torch.where(torch.diagonal(R) < 0, -1.0, 1.0).to(Q.dtype)
    return Q * d[None, :]


def known_spectrum(m, n, sigma, seed_u=1, seed_v=2, device=None):
    """A = U diag(sigma) V^T (float64).  len(sigma) must be min(m, n).
    On a torch device, returns a float64 tensor there."""
    d = min(m, n)
    sigma = np.asarray(sigma, dtype=np.float64)
    if sigma.shape != (d,):
        raise ValueError("sigma must have min(m, n) entries")
    U = haar(m, d, seed_u, device)
    V = haar(n, d, seed_v, device)
    if device is None:
        return (U * sigma[None, :]) @ V.T
    import torch
    s = torch.from_numpy(sigma).to(U.device)
    return (U * s[None, :]) @ V.T


def symmetric_spectrum(n, lam, seed=1, device=None):
    """Symmetric A = U diag(lam) U^T (float64) with Haar U (n x n); lam has n
    entries (signed: A may be indefinite).  On a torch device, returns a
    float64 tensor there, symmetrised exactly."""
    lam = np.asarray(lam, dtype=np.float64)
    if lam.shape != (n,):
        raise ValueError("lam must have n entries")
    U = haar(n, n, seed, device)
    if device is None:
        A = (U * lam[None, :]) @ U.T
        return 0.5 * (A + A.T)
    import torch
    s = torch.from_numpy(lam).to(U.device)
    A = (U * s[None, :]) @ U.T
    return 0.5 * (A + A.T)


def alternating_signs(values):
    """values with signs + - + - ... (an indefinite spectrum of the same
    magnitudes)."""
    v = np.asarray(values, dtype=np.float64)
    return v * np.where(np.arange(v.size) % 2 == 0, 1.0, -1.0)


def spectrum_geometric(d, ratio, floor=0.0):
    """sigma_i = max(ratio^i, floor), i = 1..d."""
    i = np.arange(1, d + 1, dtype=np.float64)
    return np.maximum(ratio ** i, floor)


def spectrum_power(d, alpha):
    """sigma_i = i^-alpha, i = 1..d."""
    i = np.arange(1, d + 1, dtype=np.float64)
    return i ** (-float(alpha))


def eq41_spectrum(d, gap, r=15):
    """Eq. (4.1): sigma_j = gap / j for j <= r, 1 / j for j > r."""
    j = np.arange(1, d + 1, dtype=np.float64)
    return np.where(j <= r, gap / j, 1.0 / j)


def eq41_matrix(gap, seed_u=1, seed_v=2, m=3000, n=300, r=15):
    return known_spectrum(m, n, eq41_spectrum(min(m, n), gap, r), seed_u, seed_v)


def exact_rank(m, n, r, seed_u=1, seed_v=2, top=1.0, ratio=0.7):
    """Exact rank-r matrix with sigma_i = top * ratio^(i-1), i <= r, 0 after."""
    d = min(m, n)
    sigma = np.zeros(d)
    sigma[:r] = top * ratio ** np.arange(r)
    return known_spectrum(m, n, sigma, seed_u, seed_v), sigma


def image(size=2048, bumps=60, noise=0.05, seed_bumps=3, seed_noise=4):
    """Image-shaped test matrix: sum of `bumps` separable Gaussian bumps with
    centres uniform in [0, size)^2, standard deviations uniform in [20, 200]
    pixels and amplitudes uniform in [0, 1]; min-max normalised to [0, 1];
    then i.i.d. N(0, noise^2) added (no clipping).  Row index = y, column
    index = x.  The noiseless part has rank <= bumps."""
    rb = _rng(seed_bumps)
    cx = rb.uniform(0.0, size, bumps)
    cy = rb.uniform(0.0, size, bumps)
    w = rb.uniform(20.0, 200.0, bumps)
    a = rb.uniform(0.0, 1.0, bumps)
    x = np.arange(size, dtype=np.float64)
    gy = np.exp(-((x[:, None] - cy[None, :]) ** 2) / (2.0 * w[None, :] ** 2))   # size x bumps
    gx = np.exp(-((x[:, None] - cx[None, :]) ** 2) / (2.0 * w[None, :] ** 2))
    img = (gy * a[None, :]) @ gx.T
    img = (img - img.min()) / (img.max() - img.min())
    return img + noise * _rng(seed_noise).standard_normal((size, size))


# Benchmark configurations: (m, n, k, p, q, dtype, spectrum description).
CONFIGS = {
    "c1_fp64_512x256": dict(m=512, n=256, k=20, p=10, q=0, dtype="f64",
                            spectrum=("geometric", 0.8, 0.0)),
    "c2_fp32_8192": dict(m=8192, n=8192, k=100, p=10, q=2, dtype="f32",
                         spectrum=("geometric", 0.95, 1e-6)),
    "c3a_fp32_image_2048": dict(m=2048, n=2048, k=50, p=10, q=1, dtype="f32",
                                spectrum=("image",)),
    "c3b_fp32_slow_2048": dict(m=2048, n=2048, k=50, p=10, q=1, dtype="f32",
                               spectrum=("power", 1.0)),
    # Serving: 2000 FP32 requests, Poisson arrivals at 200 req/s (serving_trace below).
    "c5_serving": dict(serving=True, count=2000, rate=200.0, dtype="f32", budget_gb=16, streams=16),
    # Mixed precision: FP32 master, solved as FP32, BF16 and column-scaled FP8.
    "c4_mixed_32768x16384": dict(m=32768, n=16384, k=256, p=16, q=2, dtype="f32",
                                 spectrum=("power", 1.5), lowp=True),
}


def config_sigma(name):
    c = CONFIGS[name]
    d = min(c["m"], c["n"])
    kind = c["spectrum"][0]
    if kind == "geometric":
        return spectrum_geometric(d, c["spectrum"][1], c["spectrum"][2])
    if kind == "power":
        return spectrum_power(d, c["spectrum"][1])
    return None


def config_matrix(name, device=None):
    """The float64 input matrix of a named configuration (numpy array, or a
    torch float64 tensor on `device` for the known-spectrum families)."""
    c = CONFIGS[name]
    if c["spectrum"][0] == "image":
        A = image(c["m"])
        if device is None:
            return A
        import torch
        return torch.from_numpy(A).to(device)
    return known_spectrum(c["m"], c["n"], config_sigma(name), 1, 2, device)


# ---------------------------------------------------------------- serving --
# The request stream of the serving workload: Poisson arrivals, m and n
# log-uniform in [256, 8192] (rounded to the half-octave grid below), k
# uniform in {10..128} (at most min(m, n)), p = 10, q uniform in {0, 1, 2};
# spectra alternate geometric (ratio U[0.9, 0.99]) and polynomial (i^-alpha,
# alpha U[1, 2]), sigma_1 = 1.  Matrices are A = U_m[:, :d] diag(sigma) V_n[:, :d]^T
# with one pair of Haar factors per grid size (a pool shared by the requests
# of that size; each request has its own spectrum), formed on the device.
SERVING_GRID = [int(round(256 * 2.0 ** (h / 2))) for h in range(11)]        # 256 ... 8192


def serving_trace(count=2000, rate=200.0, seed=5):
    rng = _rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, count))
    lg = np.log(np.array(SERVING_GRID, dtype=np.float64))
    snap = lambda x: SERVING_GRID[int(np.argmin(np.abs(lg - x)))]
    out = []
    for r in range(count):
        m = snap(rng.uniform(lg[0], lg[-1]))
        n = snap(rng.uniform(lg[0], lg[-1]))
        k = min(int(rng.integers(10, 129)), min(m, n))
        q = int(rng.integers(0, 3))
        spec = ("geometric", float(rng.uniform(0.9, 0.99))) if r % 2 == 0 else ("power", float(rng.uniform(1.0, 2.0)))
        out.append(dict(arrival=float(arrivals[r]), m=m, n=n, k=k, p=10, q=q, spectrum=spec, seed=r))
    return out


def request_sigma(req):
    d = min(req["m"], req["n"])
    kind, x = req["spectrum"]
    return spectrum_geometric(d, x) / x if kind == "geometric" else spectrum_power(d, x)


class HaarPool:
    """One pair of Haar factors per grid size on a torch device (FP64 QR,
    stored in FP32), for the serving workload's matrices."""

    def __init__(self, device, sizes):
        self.U, self.V = {}, {}
        for s in sizes:
            self.U[s] = haar(s, s, 16000 + s, device).float()
            self.V[s] = haar(s, s, 17000 + s, device).float()

    def matrix(self, req):
        import torch
        m, n = req["m"], req["n"]
        d = min(m, n)
        sig = torch.from_numpy(request_sigma(req)).float().to(self.U[m].device)
        return ((self.U[m][:, :d] * sig[None, :]) @ self.V[n][:, :d].T).contiguous()
