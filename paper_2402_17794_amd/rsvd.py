"""Thin Python binding of librsvd.so (ctypes).

Argument marshalling only: torch tensors provide device memory and the
stream; every step of the computation runs in the library's HIP kernels.
The names follow the C ABI in include/rsvd.h.  There is no fallback: if the
library is missing or a call fails, an exception is raised.
"""

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librsvd.so")

RSVD_F64, RSVD_F32, RSVD_BF16, RSVD_FP8_E4M3 = 0, 1, 2, 3
INFO_QR_FALLBACK = 1
INFO_SHIFTED_CHOLESKY = 2
INFO_JACOBI_NOT_CONVERGED = 4
INFO_NONFINITE = 8

_DTYPES = {torch.float64: RSVD_F64, torch.float32: RSVD_F32}


class rsvd_matrix(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("col_scale", ctypes.c_void_p), ("master", ctypes.c_void_p), ("ld_master", ctypes.c_int64)]


class LowPrecisionMatrix:
    """A stored as BF16 (uint16 patterns in an int16 tensor) or column-scaled
    FP8 E4M3 (uint8 tensor + float32 col_scale), optionally with the FP32
    master copy used for the Rayleigh-Ritz projection and the residual."""

    def __init__(self, data, fmt, col_scale=None, master=None):
        self.data, self.fmt, self.col_scale, self.master = data, fmt, col_scale, master
        self.shape = tuple(data.shape)
        self.device = data.device
        self.dtype = torch.float32            # dtype of the outputs

    def matrix(self):
        m = rsvd_matrix(self.data.data_ptr(), self.fmt, 0, self.shape[0], self.shape[1], self.data.stride(0))
        if self.col_scale is not None:
            m.col_scale = self.col_scale.data_ptr()
        if self.master is not None:
            m.master = self.master.data_ptr()
            m.ld_master = self.master.stride(0)
        return m


ORTH_AUTO, ORTH_CHOLQR2, ORTH_HOUSEHOLDER = 0, 1, 2
INFO_ORTH_BREAKDOWN = 16
INFO_FALLBACK_TIMEOUT = 32
INFO_SINGULAR_SYSTEM = 64


class rsvd_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("p", ctypes.c_int64), ("q", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("residual", ctypes.c_int32), ("return_full_l", ctypes.c_int32),
                ("orth", ctypes.c_int32), ("residual_iters", ctypes.c_int32),
                ("extra_power_pass", ctypes.c_int32), ("algorithm", ctypes.c_int32),
                ("jacobi_max_sweeps", ctypes.c_int32), ("test_matrix", ctypes.c_int32), ("reserved1", ctypes.c_int32)]


TEST_GAUSSIAN, TEST_SRFT = 0, 1


def make_params(k, p=10, q=0, seed=0, residual=0, return_full_l=False, orth=ORTH_AUTO, residual_iters=0,
                extra_power_pass=-1, algorithm=4, jacobi_max_sweeps=0, test_matrix=TEST_GAUSSIAN):
    return rsvd_params(k, p, q, seed, residual, int(return_full_l), int(orth), int(residual_iters),
                       int(extra_power_pass), int(algorithm), int(jacobi_max_sweeps), int(test_matrix), 0)


class rsvd_result(ctypes.Structure):
    _fields_ = [("U", ctypes.c_void_p), ("ldu", ctypes.c_int64), ("S", ctypes.c_void_p),
                ("Vt", ctypes.c_void_p), ("ldvt", ctypes.c_int64), ("residual", ctypes.c_void_p),
                ("info", ctypes.c_void_p), ("Q", ctypes.c_void_p), ("ldq", ctypes.c_int64),
                ("jacobi_sweeps", ctypes.c_void_p)]


EXPORTS = ["rsvd_create", "rsvd_destroy", "rsvd_l_used", "rsvd_workspace_size", "rsvd_solve", "rsvd_solve_noalloc",
           "rsvd_srft_omega", "rsvd_canonical_sines_workspace_size", "rsvd_canonical_sines",
           "rsvd_adaptive_range_workspace_size", "rsvd_adaptive_range",
           "rsvd_dual_sketch_workspace_size", "rsvd_dual_sketch",
           "rsvd_status_string", "rsvd_profile_enable", "rsvd_profile_read", "rsvd_quantize", "rsvd_omega",
           "rsvd_philox_words", "rsvd_gemm_workspace_size", "rsvd_gemm", "rsvd_orth_workspace_size", "rsvd_orth",
           "rsvd_server_create", "rsvd_server_submit", "rsvd_server_poll", "rsvd_server_wait", "rsvd_server_drain",
           "rsvd_server_stats", "rsvd_server_destroy", "rsvd_server_use_graphs", "rsvd_server_graph_stats",
           "rsvd_server_release", "rsvd_server_pause"]

_lib = None


def load_library(path=LIB_PATH):
    """Load librsvd.so and declare the C signatures (no GPU needed)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2402_17794_amd.build`")
    lib = ctypes.CDLL(path)
    P, I64, I32, U64, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_size_t
    sig = {
        "rsvd_create": ([ctypes.POINTER(P), ctypes.c_int], I32),
        "rsvd_destroy": ([P], I32),
        "rsvd_l_used": ([I64, I64, I64, I64], I64),
        "rsvd_workspace_size": ([P, ctypes.POINTER(rsvd_matrix), ctypes.POINTER(rsvd_params), ctypes.POINTER(SZ)],
                                I32),
        "rsvd_solve": ([P, ctypes.POINTER(rsvd_matrix), ctypes.POINTER(rsvd_params), ctypes.POINTER(rsvd_result),
                        P, SZ, P], I32),
        "rsvd_solve_noalloc": ([P, ctypes.POINTER(rsvd_matrix), ctypes.POINTER(rsvd_params),
                                ctypes.POINTER(rsvd_result), P], I32),
        "rsvd_status_string": ([I32], ctypes.c_char_p),
        "rsvd_profile_enable": ([P, I32], I32),
        "rsvd_profile_read": ([P, I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)], I32),
        "rsvd_quantize": ([I32, P, I64, I64, I64, P, I64, P, P], I32),
        "rsvd_server_create": ([ctypes.POINTER(P), ctypes.c_int, SZ, ctypes.c_int, I32], I32),
        "rsvd_server_submit": ([P, ctypes.POINTER(rsvd_matrix), ctypes.POINTER(rsvd_params),
                                ctypes.POINTER(rsvd_result), P, ctypes.POINTER(U64)], I32),
        "rsvd_server_release": ([P, U64], I32),
        "rsvd_server_pause": ([P, I32], I32),
        "rsvd_server_poll": ([P, U64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(I32)], I32),
        "rsvd_server_wait": ([P, U64, ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_double)], I32),
        "rsvd_server_drain": ([P], I32),
        "rsvd_server_stats": ([P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)], I32),
        "rsvd_server_destroy": ([P], I32),
        "rsvd_server_use_graphs": ([P, I32], I32),
        "rsvd_server_graph_stats": ([P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64)], I32),
        "rsvd_omega": ([I32, U64, ctypes.c_uint32, I64, I64, P, I64, P], I32),
        "rsvd_philox_words": ([U64, ctypes.c_uint32, P, I64, P, P], I32),
        "rsvd_srft_omega": ([I32, U64, I64, I64, P, I64, P, P], I32),
        "rsvd_canonical_sines_workspace_size": ([I32, I64, I64, I64, ctypes.POINTER(SZ)], I32),
        "rsvd_canonical_sines": ([P, I32, I64, I64, P, I64, I64, P, I64, P, P, SZ, P], I32),
        "rsvd_adaptive_range_workspace_size": ([ctypes.POINTER(rsvd_matrix), I32, I64, ctypes.POINTER(SZ)], I32),
        "rsvd_adaptive_range": ([P, ctypes.POINTER(rsvd_matrix), ctypes.c_double, I32, I64, U64, P, I64,
                                 ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I32), P, SZ, P],
                                I32),
        "rsvd_dual_sketch_workspace_size": ([ctypes.POINTER(rsvd_matrix), I64, ctypes.POINTER(SZ)], I32),
        "rsvd_dual_sketch": ([P, ctypes.POINTER(rsvd_matrix), U64, I64, P, I64, P, I64, P, I64, P, I64, P, SZ, P],
                             I32),
        "rsvd_gemm_workspace_size": ([ctypes.POINTER(rsvd_matrix), I32, I64, ctypes.POINTER(SZ)], I32),
        "rsvd_gemm": ([P, ctypes.POINTER(rsvd_matrix), I32, P, I64, U64, I64, P, I64, P, SZ, P], I32),
        "rsvd_orth_workspace_size": ([I32, I64, I64, ctypes.POINTER(SZ)], I32),
        "rsvd_orth": ([P, I32, I64, I64, P, I64, P, I64, I32, P, P, SZ, P], I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    if path == LIB_PATH:
        _lib = lib
    return lib


class RsvdError(RuntimeError):
    """A non-zero rsvd_status; `status` holds the code."""

    def __init__(self, msg, status=0):
        super().__init__(msg)
        self.status = status


def _check(status):
    if status != 0:
        msg = load_library().rsvd_status_string(status).decode()
        raise RsvdError(f"librsvd: {msg} (status {status})", status)


_handles = {}


def _handle(device):
    idx = torch.device(device).index
    idx = torch.cuda.current_device() if idx is None else idx
    if idx not in _handles:
        h = ctypes.c_void_p()
        _check(load_library().rsvd_create(ctypes.byref(h), idx))
        _handles[idx] = h
    return _handles[idx]


def _stream_ptr(stream, device):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _as_matrix(A):
    if isinstance(A, LowPrecisionMatrix):
        return A.matrix()
    if A.dim() != 2 or not A.is_cuda or A.dtype not in _DTYPES:
        raise ValueError("A must be a 2-D float32/float64 CUDA tensor")
    if A.stride(1) != 1:
        raise ValueError("A must be row-major (stride(1) == 1)")
    return rsvd_matrix(A.data_ptr(), _DTYPES[A.dtype], 0, A.shape[0], A.shape[1], max(A.stride(0), A.shape[1]),
                       None, None, 0)


def quantize(A, fmt, keep_master=True, stream=None):
    """BF16 (fmt = RSVD_BF16) or column-scaled FP8 (RSVD_FP8_E4M3) copy of a
    row-major float32 CUDA tensor, made by the library's kernels; the rows
    are padded to a 16-byte multiple.  keep_master: A itself becomes the
    FP32 copy for the Rayleigh-Ritz projection."""
    if A.dtype != torch.float32 or A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a row-major float32 CUDA tensor")
    m, n = A.shape
    if fmt == RSVD_BF16:
        data = torch.empty((m, (n + 7) // 8 * 8), dtype=torch.int16, device=A.device)[:, :n]
        scale = None
    elif fmt == RSVD_FP8_E4M3:
        data = torch.empty((m, (n + 15) // 16 * 16), dtype=torch.uint8, device=A.device)[:, :n]
        scale = torch.empty((n,), dtype=torch.float32, device=A.device)
    else:
        raise ValueError("fmt must be RSVD_BF16 or RSVD_FP8_E4M3")
    _check(load_library().rsvd_quantize(fmt, ctypes.c_void_p(A.data_ptr()), m, n, A.stride(0),
                                        ctypes.c_void_p(data.data_ptr()), data.stride(0),
                                        ctypes.c_void_p(scale.data_ptr()) if scale is not None else None,
                                        _stream_ptr(stream, A.device)))
    return LowPrecisionMatrix(data, fmt, scale, A if keep_master else None)


def _workspace(nbytes, device):
    # 256-byte alignment: torch's caching allocator returns 512-byte aligned blocks.
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def l_used(m, n, k, p):
    return int(load_library().rsvd_l_used(m, n, k, p))


def workspace_size(A, k, p=10, q=0, return_full_l=False):
    lib = load_library()
    M = _as_matrix(A)
    prm = make_params(k, p, q, return_full_l=return_full_l)
    nb = ctypes.c_size_t()
    _check(lib.rsvd_workspace_size(_handle(A.device), ctypes.byref(M), ctypes.byref(prm), ctypes.byref(nb)))
    return nb.value


RESIDUAL_SPECTRAL, RESIDUAL_FROBENIUS = 1, 2


def _residual_mode(residual):
    """True keeps the Frobenius norm alone; an int selects the header's bits."""
    if residual is True:
        return RESIDUAL_FROBENIUS
    if not residual:
        return 0
    return int(residual)


RSVD_ERR_TOO_LARGE = 6
RSVD_ERR_QUEUE_FULL = 7
NOALLOC_SCRATCH_BYTES = 64 << 20


class Solver:
    """Reusable solve for one (shape, dtype, k, p, q): owns the output tensors
    and the workspace, so repeated calls allocate nothing.  residual: False,
    True (Frobenius), or the header's bit mask (1 spectral estimate, 2
    Frobenius, 3 both); residual_iters: power iterations of the spectral
    estimate (0 = library default).  noalloc: call rsvd_solve_noalloc, which
    uses the library's fixed device scratch instead of a workspace (no
    workspace tensor is made).  orth: ORTH_AUTO, ORTH_CHOLQR2 or
    ORTH_HOUSEHOLDER (force_householder=True is ORTH_HOUSEHOLDER);
    algorithm: 4 (default), 3 (no orth between the power products), or the
    single-pass 5 (symmetric A: S holds signed eigenvalues, Vt = U^T) and 6
    (general A, two sketches from one read);
    jacobi_max_sweeps: sweep cap of the small SVD (0 = default)."""

    def __init__(self, A, k, p=10, q=0, seed=0, residual=False, return_full_l=False, force_householder=False,
                 return_q=False, stream=None, residual_iters=0, extra_power_pass=-1, noalloc=False, orth=ORTH_AUTO,
                 algorithm=4, jacobi_max_sweeps=0, test_matrix=TEST_GAUSSIAN):
        self.lib = load_library()
        self.A = A
        self.M = _as_matrix(A)
        m, n = A.shape
        self.l = l_used(m, n, k, p)
        r = self.l if return_full_l else k
        dev = A.device
        residual = _residual_mode(residual)
        self.params = make_params(k, p, q, seed, residual, return_full_l,
                                  ORTH_HOUSEHOLDER if force_householder else orth, residual_iters, extra_power_pass,
                                  algorithm, jacobi_max_sweeps, test_matrix)
        self.U = torch.empty((m, r), dtype=A.dtype, device=dev)
        self.S = torch.empty((r,), dtype=torch.float64, device=dev)
        self.Vt = torch.empty((r, n), dtype=A.dtype, device=dev)
        self._words = torch.empty((2,), dtype=torch.int32, device=dev)
        self.info, self.sweeps = self._words[:1], self._words[1:]        # RSVD_INFO_* bits, Jacobi sweeps
        self.res = torch.zeros((2,), dtype=torch.float64, device=dev) if residual else None
        self.Q = torch.empty((m, self.l), dtype=A.dtype, device=dev) if return_q else None
        nb = ctypes.c_size_t()
        self.h = _handle(dev)
        self.noalloc = bool(noalloc)
        _check(self.lib.rsvd_workspace_size(self.h, ctypes.byref(self.M), ctypes.byref(self.params),
                                            ctypes.byref(nb)))
        self.ws = None if self.noalloc else _workspace(nb.value, dev)
        self.result = rsvd_result(self.U.data_ptr(), r, self.S.data_ptr(), self.Vt.data_ptr(), n,
                                  self.res.data_ptr() if residual else None, self.info.data_ptr(),
                                  self.Q.data_ptr() if return_q else None, self.l, self.sweeps.data_ptr())
        self.stream = stream

    def set_seed(self, seed):
        self.params.seed = seed

    def __call__(self):
        if self.noalloc:
            _check(self.lib.rsvd_solve_noalloc(self.h, ctypes.byref(self.M), ctypes.byref(self.params),
                                               ctypes.byref(self.result), _stream_ptr(self.stream, self.A.device)))
            return self
        _check(self.lib.rsvd_solve(self.h, ctypes.byref(self.M), ctypes.byref(self.params), ctypes.byref(self.result),
                                   ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                   _stream_ptr(self.stream, self.A.device)))
        return self


def solve(A, k, p=10, q=0, seed=0, residual=False, return_full_l=False, force_householder=False, return_q=False,
          stream=None, residual_iters=0, extra_power_pass=-1, noalloc=False, orth=ORTH_AUTO, algorithm=4,
          jacobi_max_sweeps=0, test_matrix=TEST_GAUSSIAN):
    """Randomized SVD (Algorithm 4; Algorithm 3, 5 or 6 with algorithm=3, 5, 6) of a
    CUDA tensor A.  Returns a dict with U (m x r), S (r, float64), Vt
    (r x n), info (int), l, and optionally residual_t ([spectral estimate,
    Frobenius norm] of A - QQ^T A, float64 tensor) and Q (m x l).
    noalloc: use rsvd_solve_noalloc."""
    s = Solver(A, k, p, q, seed, residual, return_full_l, force_householder, return_q, stream, residual_iters,
               extra_power_pass, noalloc, orth, algorithm, jacobi_max_sweeps, test_matrix)()
    out = dict(U=s.U, S=s.S, Vt=s.Vt, l=s.l, info_tensor=s.info, jacobi_sweeps_tensor=s.sweeps)
    if residual:
        out["residual_t"] = s.res
    if return_q:
        out["Q"] = s.Q
    return out


class Request:
    """A submitted server request: owns its output tensors (and keeps A
    alive) until it is done."""

    def __init__(self, server, A, k, p, q, seed, return_full_l, extra_power_pass, algorithm=4):
        m, n = A.shape
        self.A, self.l = A, l_used(m, n, k, p)
        r = self.l if return_full_l else k
        dev = A.device
        self.U = torch.empty((m, r), dtype=A.dtype, device=dev)
        self.S = torch.empty((r,), dtype=torch.float64, device=dev)
        self.Vt = torch.empty((r, n), dtype=A.dtype, device=dev)
        self.info = torch.empty((1,), dtype=torch.int32, device=dev)    # assigned by the solve
        self._M = _as_matrix(A)
        self._params = make_params(k, p, q, seed, 0, return_full_l, extra_power_pass=extra_power_pass,
                                   algorithm=algorithm)
        self._result = rsvd_result(self.U.data_ptr(), r, self.S.data_ptr(), self.Vt.data_ptr(), n, None,
                                   self.info.data_ptr(), None, self.l)
        # The server's streams do not wait for torch's: the request waits for
        # this event, recorded after whatever made A and the outputs.
        self._ready = torch.cuda.Event()
        self._ready.record(torch.cuda.current_stream(dev))
        t = ctypes.c_uint64()
        _check(server.lib.rsvd_server_submit(server.ptr, ctypes.byref(self._M), ctypes.byref(self._params),
                                             ctypes.byref(self._result), ctypes.c_void_p(self._ready.cuda_event),
                                             ctypes.byref(t)))
        self.ticket = t.value
        self.server = server
        self._latency = None

    def done(self):
        if self._latency is not None:
            return True
        d, st = ctypes.c_int(), ctypes.c_int32()
        _check(self.server.lib.rsvd_server_poll(self.server.ptr, self.ticket, ctypes.byref(d), ctypes.byref(st)))
        return bool(d.value)

    def wait(self):
        """Block until done and release the server's record of the request;
        returns the latency in ms (submit to completion)."""
        if self._latency is not None:
            return self._latency
        st, lat = ctypes.c_int32(), ctypes.c_double()
        _check(self.server.lib.rsvd_server_wait(self.server.ptr, self.ticket, ctypes.byref(st), ctypes.byref(lat)))
        _check(self.server.lib.rsvd_server_release(self.server.ptr, self.ticket))
        self._latency = lat.value
        _check(st.value)
        return lat.value


class Server:
    """Continuous-batching request server (rsvd_server_*): requests are
    admitted by HBM footprint into `n_streams` concurrent slots."""

    def __init__(self, device="cuda:0", hbm_budget_bytes=16 << 30, n_streams=4, max_pending=0):
        self.lib = load_library()
        dev = torch.device(device)
        idx = dev.index if dev.index is not None else torch.cuda.current_device()
        self.ptr = ctypes.c_void_p()
        _check(self.lib.rsvd_server_create(ctypes.byref(self.ptr), idx, int(hbm_budget_bytes), int(n_streams),
                                           int(max_pending)))

    def submit(self, A, k, p=10, q=0, seed=0, return_full_l=False, extra_power_pass=-1, algorithm=4):
        """Queue a solve (RsvdError with status RSVD_ERR_QUEUE_FULL when
        max_pending requests already wait)."""
        return Request(self, A, k, p, q, seed, return_full_l, extra_power_pass, algorithm)

    def pause(self, paused=True):
        """Hold (or resume) admissions; queued requests wait."""
        _check(self.lib.rsvd_server_pause(self.ptr, int(paused)))

    def drain(self):
        _check(self.lib.rsvd_server_drain(self.ptr))

    def use_graphs(self, enable=True):
        """Launch later admissions as captured per-bucket graphs, or directly
        (the default).  While graphs are on, other code must not synchronise
        the whole device (HIP refuses it during a capture): wait on streams,
        events or the server's tickets instead."""
        _check(self.lib.rsvd_server_use_graphs(self.ptr, int(enable)))

    def graph_stats(self):
        """(requests launched as graphs, executable graphs instantiated,
        requests launched directly after a failed capture)."""
        n, inst, fb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(self.lib.rsvd_server_graph_stats(self.ptr, ctypes.byref(n), ctypes.byref(inst), ctypes.byref(fb)))
        return n.value, inst.value, fb.value

    def stats(self):
        p50, p99, sps, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(self.lib.rsvd_server_stats(self.ptr, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(sps),
                                          ctypes.byref(n)))
        return {"p50_ms": p50.value, "p99_ms": p99.value, "solves_per_s": sps.value, "completed": n.value}

    def close(self):
        if self.ptr:
            _check(self.lib.rsvd_server_destroy(self.ptr))
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PROFILE_SKETCH, PROFILE_NN, PROFILE_TN, PROFILE_ALL, PROFILE_PROJ32, PROFILE_STAGE1, PROFILE_JACOBI = 0, 1, 2, 3, 4, 5, 6
PROFILE_DUAL = 7


def profile_enable(device, enable=True):
    """Time every product with A of later solves on `device` with HIP events."""
    _check(load_library().rsvd_profile_enable(_handle(device), int(enable)))


def profile_read(device, kind=PROFILE_ALL):
    """(total milliseconds, records) of the recorded products of `kind`, or of
    the range finders (Stage 1) of the profiled solves for PROFILE_STAGE1."""
    tot = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(load_library().rsvd_profile_read(_handle(device), kind, ctypes.byref(tot), ctypes.byref(cnt)))
    return tot.value, cnt.value


def omega(n, l, seed, dtype=torch.float32, stream_id=0, device="cuda"):
    """The test matrix of Algorithm 4 step 1, materialised on the device."""
    out = torch.empty((n, l), dtype=dtype, device=device)
    _check(load_library().rsvd_omega(_DTYPES[dtype], seed, stream_id, n, l, ctypes.c_void_p(out.data_ptr()), l,
                                     _stream_ptr(None, out.device)))
    return out


def srft_omega(n, l, seed, dtype=torch.float32, device="cuda"):
    """The SRFT test matrix (FastRandRF), materialised: (Omega n x l, the l
    sampled DCT columns as an int32 tensor)."""
    out = torch.empty((n, l), dtype=dtype, device=device)
    cols = torch.empty((l,), dtype=torch.int32, device=device)
    _check(load_library().rsvd_srft_omega(_DTYPES[dtype], seed, n, l, ctypes.c_void_p(out.data_ptr()), l,
                                          ctypes.c_void_p(cols.data_ptr()), _stream_ptr(None, out.device)))
    return out, cols


def canonical_sines(U1, U2):
    """Sines of the canonical angles between range(U1) and range(U2) (both
    with orthonormal columns, U1 no wider than U2), ascending, float64."""
    lib = load_library()
    if U1.dtype != U2.dtype or U1.dtype not in _DTYPES or U1.stride(1) != 1 or U2.stride(1) != 1:
        raise ValueError("U1, U2: row-major CUDA tensors of one float dtype")
    rows, k = U1.shape
    l = U2.shape[1]
    nb = ctypes.c_size_t()
    _check(lib.rsvd_canonical_sines_workspace_size(_DTYPES[U1.dtype], rows, k, l, ctypes.byref(nb)))
    ws = _workspace(nb.value, U1.device)
    out = torch.empty((k,), dtype=torch.float64, device=U1.device)
    _check(lib.rsvd_canonical_sines(_handle(U1.device), _DTYPES[U1.dtype], rows, k, ctypes.c_void_p(U1.data_ptr()),
                                    U1.stride(0), l, ctypes.c_void_p(U2.data_ptr()), U2.stride(0),
                                    ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    _stream_ptr(None, U1.device)))
    return out


def adaptive_range(A, tol, block=16, max_l=None, seed=0):
    """Adaptive randomized range finder: (Q m x l, estimate, converged).
    max_l defaults to the largest basis the library handles for this block
    (288 - round16(block)), or min(m, n) if smaller."""
    lib = load_library()
    M = _as_matrix(A)
    m, n = A.shape
    if max_l is None:
        max_l = min(m, n, 288 - (int(block) + 15) // 16 * 16)
    max_l = int(max_l)
    nb = ctypes.c_size_t()
    _check(lib.rsvd_adaptive_range_workspace_size(ctypes.byref(M), int(block), max_l, ctypes.byref(nb)))
    ws = _workspace(nb.value, A.device)
    cap = min(max_l, m, n)
    Q = torch.empty((m, cap), dtype=A.dtype, device=A.device)
    l, est, conv = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int32()
    _check(lib.rsvd_adaptive_range(_handle(A.device), ctypes.byref(M), float(tol), int(block), max_l, seed,
                                   ctypes.c_void_p(Q.data_ptr()), cap, ctypes.byref(l), ctypes.byref(est),
                                   ctypes.byref(conv), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream_ptr(None, A.device)))
    return Q[:, :l.value], est.value, bool(conv.value)


def philox_words(seed, ctr, stream_id=0):
    """Raw Philox4x32-10 words for an (N, 2) int32 tensor of (g, j) counters."""
    ctr = ctr.contiguous()
    out = torch.empty((ctr.shape[0], 4), dtype=torch.int32, device=ctr.device)
    _check(load_library().rsvd_philox_words(seed, stream_id, ctypes.c_void_p(ctr.data_ptr()), ctr.shape[0],
                                            ctypes.c_void_p(out.data_ptr()), _stream_ptr(None, ctr.device)))
    return out


def gemm(A, X=None, trans=False, seed=0, ncols=None):
    """Y = A X (trans False) or A^T X (trans True) with the solve's MFMA
    kernels; X None (trans False) means the generated test matrix."""
    lib = load_library()
    M = _as_matrix(A)
    if X is not None:
        if X.dtype != A.dtype or X.stride(1) != 1:
            raise ValueError("X must match A's dtype (float32 for a low-precision A) and be row-major")
        ncols = X.shape[1]
    rows = A.shape[1] if trans else A.shape[0]
    nb = ctypes.c_size_t()
    _check(lib.rsvd_gemm_workspace_size(ctypes.byref(M), int(trans), ncols, ctypes.byref(nb)))
    ws = _workspace(nb.value, A.device)
    Y = torch.empty((rows, ncols), dtype=A.dtype, device=A.device)
    _check(lib.rsvd_gemm(_handle(A.device), ctypes.byref(M), int(trans),
                         ctypes.c_void_p(X.data_ptr()) if X is not None else None,
                         X.stride(0) if X is not None else 0, seed, ncols, ctypes.c_void_p(Y.data_ptr()), ncols,
                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(None, A.device)))
    return Y


def dual_sketch(A, l, seed=0):
    """Two-sided sketch of Algorithm 6 from one read of A: returns
    (Y_c = A Omega_c, Y_r = A^T Omega_r, Omega_c, Omega_r) with the test
    matrices of streams 0 (n x l) and 1 (m x l) as the kernel generated them."""
    lib = load_library()
    M = _as_matrix(A)
    m, n = A.shape
    nb = ctypes.c_size_t()
    _check(lib.rsvd_dual_sketch_workspace_size(ctypes.byref(M), l, ctypes.byref(nb)))
    ws = _workspace(nb.value, A.device)
    kw = dict(dtype=A.dtype, device=A.device)
    Yc, Yr, Oc, Or = torch.empty((m, l), **kw), torch.empty((n, l), **kw), torch.empty((n, l), **kw), \
        torch.empty((m, l), **kw)
    _check(lib.rsvd_dual_sketch(_handle(A.device), ctypes.byref(M), seed, l, ctypes.c_void_p(Yc.data_ptr()), l,
                                ctypes.c_void_p(Yr.data_ptr()), l, ctypes.c_void_p(Oc.data_ptr()), l,
                                ctypes.c_void_p(Or.data_ptr()), l, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                _stream_ptr(None, A.device)))
    return Yc, Yr, Oc, Or


def orth(Y, force_householder=False, mode=None):
    """Orthonormal basis of range(Y) (CholeskyQR2 with Householder fallback;
    mode: ORTH_AUTO, ORTH_CHOLQR2 or ORTH_HOUSEHOLDER, force_householder=True
    is ORTH_HOUSEHOLDER).  Returns (Q, info)."""
    if mode is None:
        mode = ORTH_HOUSEHOLDER if force_householder else ORTH_AUTO
    lib = load_library()
    if Y.dtype not in _DTYPES or Y.stride(1) != 1:
        raise ValueError("Y must be a row-major float32/float64 CUDA tensor")
    rows, l = Y.shape
    nb = ctypes.c_size_t()
    _check(lib.rsvd_orth_workspace_size(_DTYPES[Y.dtype], rows, l, ctypes.byref(nb)))
    ws = _workspace(nb.value, Y.device)
    Q = torch.empty_like(Y)
    info = torch.zeros((1,), dtype=torch.int32, device=Y.device)
    _check(lib.rsvd_orth(_handle(Y.device), _DTYPES[Y.dtype], rows, l, ctypes.c_void_p(Y.data_ptr()), Y.stride(0),
                         ctypes.c_void_p(Q.data_ptr()), l, int(mode), ctypes.c_void_p(info.data_ptr()),
                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(None, Y.device)))
    return Q, info
