"""Pins for the oracle's hydrodynamic interaction (Eqs. 1-3): the RPY tensor
blocks, the Cholesky factor of the 3N x 3N diffusion tensor, the drift
D F / kT and the correlated random displacement sqrt(2 dt) L xi."""
import math

import numpy as np
import pytest

from oracle import ora
from paper_2206_05851_amd import workloads as wl


def _full_tensor(r, a, kT=1.0, zeta=1.0):
    N = r.shape[0]
    D = np.zeros((3 * N, 3 * N))
    for i in range(N):
        for j in range(N):
            D[3 * i:3 * i + 3, 3 * j:3 * j + 3] = (kT / zeta) * np.eye(3) if i == j else \
                ora.rpy_block(kT, zeta, a, r[j] - r[i])
    return D


def test_rpy_block_symmetry_continuity_and_oseen_limit():
    a, kT, zeta = 1.0, 1.3, 0.7
    D0 = kT / zeta
    rng = np.random.default_rng(0)
    for _ in range(10):
        r = rng.normal(size=3) * 2
        B = ora.rpy_block(kT, zeta, a, r)
        assert np.allclose(B, B.T, rtol=0, atol=1e-15)
        assert np.allclose(B, ora.rpy_block(kT, zeta, a, -r), rtol=0, atol=1e-15)
    e = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    lo = ora.rpy_block(kT, zeta, a, e * 2 * a * (1 - 1e-12))
    hi = ora.rpy_block(kT, zeta, a, e * 2 * a * (1 + 1e-12))
    assert np.allclose(lo, hi, rtol=0, atol=1e-10)          # continuous at r = 2a
    far = 1e4
    B = ora.rpy_block(kT, zeta, a, e * far)
    oseen = D0 * 0.75 * a / far * (np.eye(3) + np.outer(e, e))
    assert np.allclose(B, oseen, rtol=1e-7, atol=0)          # Oseen tensor far away
    assert np.allclose(ora.rpy_block(kT, zeta, a, e * 1e-12), D0 * np.eye(3), atol=1e-10)   # coincident


def test_rpy_block_is_divergence_free():
    # sum_y d D_xy / d r_y = 0 in both branches (no Ito drift term in Eq. 1)
    a = 1.0
    rng = np.random.default_rng(1)
    h = 1e-5
    for q in (0.7, 1.5, 2.5, 4.0, 9.0):
        r = rng.normal(size=3)
        r *= q / np.linalg.norm(r)
        div = np.zeros(3)
        for y in range(3):
            e = np.zeros(3)
            e[y] = h
            div += (ora.rpy_block(1.0, 1.0, a, r + e)[:, y] - ora.rpy_block(1.0, 1.0, a, r - e)[:, y]) / (2 * h)
        assert np.allclose(div, 0.0, atol=1e-8), (q, div)


def test_full_tensor_is_positive_definite_including_overlaps():
    rng = np.random.default_rng(2)
    for _ in range(20):
        N = int(rng.integers(2, 12))
        r = rng.normal(size=(N, 3)) * rng.uniform(0.3, 3.0)     # many pairs overlap (r < 2a)
        ev = np.linalg.eigvalsh(_full_tensor(r, 1.0))
        assert ev.min() > 0


def test_cholesky_matches_library_and_rejects_indefinite():
    rng = np.random.default_rng(3)
    for n in (1, 3, 12, 45):
        X = rng.normal(size=(n, n))
        A = X @ X.T + n * np.eye(n)
        assert np.allclose(ora.cholesky(A), np.linalg.cholesky(A), rtol=1e-12, atol=1e-12)
    assert ora.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]])) is None


@pytest.mark.parametrize("axis", [0, 2])
def test_noise_free_dumbbell_relaxes_with_rpy_mobility(axis):
    # Dumbbell, bond Q along one axis, |Q| = q >= 2a: each bead moves by
    # dt D F / kT with F = +-H Q, so Q' = Q - dt (2H/kT) (D0 - D_par) Q with the
    # RPY component along the bond D_par = D0 (3a/4q)(2 - 4a^2/(3q^2)) (Eq. 3).
    H, kT, zeta, a, q, dt = 2.0, 1.0, 1.5, 0.8, 2.3, 1e-3
    D0 = kT / zeta
    r = np.zeros((2, 3))
    r[1, axis] = q
    desc = wl.group(2, 1, dt, wl.HOOKEAN, H, kT=kT, zeta=zeta, noise_scale=0.0, hi_radius=a)
    o = ora.Oracle([desc], 0, 1, 1)
    o.init_chains([r])
    o.step(1)
    Q = np.diff(o.positions()[0][0], axis=0)[0]
    Dpar = D0 * 0.75 * a / q * (2.0 - 4.0 * a * a / (3.0 * q * q))
    assert np.isclose(Q[axis], q * (1 - dt * 2 * H / kT * (D0 - Dpar)), rtol=1e-13)
    assert np.allclose(np.delete(Q, axis), 0.0, atol=1e-15)


def test_vanishing_radius_recovers_free_draining_step():
    # a -> 0: D -> (kT/zeta) I, L -> sqrt(kT/zeta) I, so the HI step (drift and
    # correlated noise through the Cholesky factor) equals the free-draining one.
    N = 6
    g = wl.group(N, 3, 1e-3, wl.FENE, 1.5, 30.0, wl.SHEAR, 2.0, kT=1.2, zeta=0.8)
    p = wl.equilibrium_parent(N, wl.FENE, 1.5, 30.0, 1.2, seed=4)
    fd = ora.Oracle([g], 5, 10, 1)
    fd.init_chains([p])
    fd.step(10)
    hi = ora.Oracle([dict(g, hi_radius=1e-9)], 5, 10, 1)
    hi.init_chains([p])
    hi.step(10)
    assert np.allclose(hi.positions()[0], fd.positions()[0], rtol=0, atol=1e-8)


def test_equilibrium_statics_do_not_depend_on_hi():
    # Free-draining or with RPY HI, Brownian dynamics samples exp(-U/kT):
    # for a Hookean chain every bond has <Q Q^T> = (kT/H) I and distinct
    # bonds are uncorrelated. A wrong noise factor (not L with L L^T = D)
    # would change these moments; the EM bias is O(dt).
    N, H, R, dt = 4, 1.0, 2000, 2e-3
    g = wl.group(N, R, dt, wl.HOOKEAN, H, hi_radius=0.35)
    o = ora.Oracle([g], 17, 2000, 2)
    o.init_chains([wl.equilibrium_parent(N, seed=9)])
    o.step(4000)                                           # 8 time units
    Q = np.diff(o.positions()[0], axis=1)                  # [R][N-1][3]
    for j in range(N - 1):
        C = np.einsum("ka,kb->ab", Q[:, j], Q[:, j]) / R
        se = math.sqrt(2.0 / R) / H
        assert np.allclose(np.diag(C), 1.0 / H, atol=5 * se + 0.02), (j, C)
        assert np.allclose(C - np.diag(np.diag(C)), 0.0, atol=5 * se)
    c01 = np.mean(np.sum(Q[:, 0] * Q[:, 1], axis=1))
    assert abs(c01) < 5 * math.sqrt(3.0 / R) / H


def test_hi_rejects_gradients_and_negative_radius():
    g = wl.group(4, 2, 1e-3, hi_radius=0.5)
    with pytest.raises(ora.OracleError):
        ora.Oracle([g], 0, 1, 1, tangents=True)
    with pytest.raises(ora.OracleError):
        ora.Oracle([dict(g, hi_radius=-1.0)], 0, 1, 1)
