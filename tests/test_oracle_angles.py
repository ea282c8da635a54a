"""Pins of the canonical-angle oracle and of the Theorem 5 bound:
closed-form angles in a plane, the identity sin^2 + cos^2 = 1 between two
different computations (a projection residual and a product), invariance
under rotations of either basis, and Theorem 5's bounds holding for the
oracle's Algorithm 3 and Algorithm 4 sketches on the Section 4.3 test
matrix (eq. (4.1) stand-in, gap 2, k = 25, p = 5, q = 0, 1, 2) for every seed."""

import numpy as np
import pytest

from oracle import angles, bounds
from oracle.philox import omega
from oracle.rsvd import rsvd_alg3, rsvd_alg4
from paper_2402_17794_amd import workloads as W


@pytest.mark.parametrize("theta", [0.0, 1e-6, 0.3, np.pi / 2])
def test_plane_angle_closed_form(theta):
    U1 = np.array([[1.0], [0.0], [0.0]])
    U2 = np.array([[np.cos(theta)], [np.sin(theta)], [0.0]])
    s = angles.canonical_sines(U1, U2)
    assert abs(s[0] - np.sin(theta)) <= 1e-15 + 1e-12 * np.sin(theta)


def test_two_angles_and_a_common_direction():
    """range(U1) = span(e1, e2), range(U2) = span(e1, cos t e2 + sin t e3,
    e4): canonical sines 0 and sin t."""
    t = 0.7
    U1 = np.eye(5)[:, :2]
    U2 = np.stack([np.eye(5)[0], np.cos(t) * np.eye(5)[1] + np.sin(t) * np.eye(5)[2], np.eye(5)[3]], axis=1)
    assert np.allclose(angles.canonical_sines(U1, U2), [0.0, np.sin(t)], atol=1e-15)


def test_sines_and_cosines_are_consistent_and_invariant():
    rng = np.random.default_rng(3)
    U1 = np.linalg.qr(rng.standard_normal((200, 7)))[0]
    U2 = np.linalg.qr(U1 @ rng.standard_normal((7, 7)) + 0.3 * rng.standard_normal((200, 7)))[0]
    U2 = np.concatenate([U2, np.linalg.qr(rng.standard_normal((200, 5)))[0]], axis=1)
    U2 = np.linalg.qr(U2)[0]
    s = angles.canonical_sines(U1, U2)
    c = angles.canonical_cosines(U1, U2)
    assert np.max(np.abs(s ** 2 + c ** 2 - 1.0)) <= 1e-13
    R1 = np.linalg.qr(rng.standard_normal((7, 7)))[0]
    R2 = np.linalg.qr(rng.standard_normal((12, 12)))[0]
    assert np.max(np.abs(angles.canonical_sines(U1 @ R1, U2 @ R2) - s)) <= 1e-13


@pytest.mark.parametrize("alg", [rsvd_alg3, rsvd_alg4])
@pytest.mark.parametrize("q", [0, 1, 2])
def test_theorem5_bounds_hold(alg, q):
    m, n, k, p = 3000, 300, 25, 5
    sig = W.eq41_spectrum(n, 2.0)
    U = W.haar(m, n, 1)
    V = W.haar(n, n, 2)
    A = (U * sig[None, :]) @ V.T
    for seed in range(4):
        out = alg(A, k, p, q, seed=seed, return_full_l=True)
        Om = omega(seed, n, k + p)
        bt, bv = bounds.thm5(sig, k, q, Om, V)
        st = angles.canonical_sines(U[:, :k], out["U"])
        sv = angles.canonical_sines(V[:, :k], out["Vt"].T)
        assert np.all(st <= bt * (1 + 1e-9) + 1e-13), (seed, np.max(st - bt))
        assert np.all(sv <= bv * (1 + 1e-9) + 1e-13), (seed, np.max(sv - bv))
        if q == 0:
            assert np.max(st) > 1e-6          # the q = 0 angles are not trivially zero
