"""MI355X (gfx950) randomized SVD: the Gaussian range finder with
re-orthonormalised power iterations, projection, small SVD and lift
(Algorithm 4 of the thesis), as HIP kernels behind a C-ABI library.

`rsvd` is the thin ctypes binding over librsvd.so; `workloads` draws the
seeded synthetic inputs.
"""

__all__ = ["rsvd", "workloads"]
