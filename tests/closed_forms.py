"""Closed forms for the free-draining chain, written in bond space.

These are independent of the oracle, which works in bead positions: for a
Hookean chain the Euler-Maruyama map is linear in the bond vectors
Q_j = r_{j+1} - r_j, so the mean and covariance of every bond at every step
are known exactly, as are steady states and their continuous-time limits.
"""
import numpy as np

HOOKEAN, FENE = 0, 1
QUIESCENT, UNIAXIAL, PLANAR, SHEAR = 0, 1, 2, 3


def rouse_B(n_bonds):
    """Bond-space Rouse matrix tridiag(-1, 2, -1) of size N-1."""
    B = 2.0 * np.eye(n_bonds)
    if n_bonds > 1:
        i = np.arange(n_bonds - 1)
        B[i, i + 1] = -1.0
        B[i + 1, i] = -1.0
    return B


def flow_matrix(flow, rate):
    """kappa such that v = kappa . r (shear: v_x = rate * z)."""
    K = np.zeros((3, 3))
    if flow == UNIAXIAL:
        K[0, 0], K[1, 1], K[2, 2] = rate, -0.5 * rate, -0.5 * rate
    elif flow == PLANAR:
        K[0, 0], K[1, 1] = rate, -rate
    elif flow == SHEAR:
        K[0, 2] = rate
    return K


def em_matrices(n_beads, H, zeta, kT, dt, flow, rate, noise_scale=1.0):
    """Hookean EM map on the stacked bond vector [Qx; Qy; Qz] (3(N-1)):
    Q' = M Q + eta, Cov(eta) = sigma^2 kron(I3, B), sigma^2 = 2 kT dt / zeta."""
    nb = n_beads - 1
    B = rouse_B(nb)
    K = flow_matrix(flow, rate)
    M = np.kron(np.eye(3), np.eye(nb) - (H * dt / zeta) * B) + dt * np.kron(K, np.eye(nb))
    sig2 = noise_scale ** 2 * 2.0 * kT * dt / zeta
    Qn = sig2 * np.kron(np.eye(3), B)
    return M, Qn


def bonds_of(xyz):
    """[.., N, 3] positions -> stacked bond vectors [.., 3(N-1)] ordered [x..., y..., z...]."""
    Q = np.diff(xyz, axis=-2)                  # [.., N-1, 3]
    return np.swapaxes(Q, -1, -2).reshape(Q.shape[:-2] + (-1,))


def moments_after(n_steps, Q0, M, Qn):
    """Exact mean and covariance of the bond vector after n EM steps from Q0."""
    m = Q0.copy()
    S = np.zeros((len(Q0), len(Q0)))
    for _ in range(n_steps):
        m = M @ m
        S = M @ S @ M.T + Qn
    return m, S


def stationary_cov(M, Qn, iters=200000, tol=1e-15):
    """Fixed point of S = M S M^T + Qn (discrete Lyapunov) by doubling."""
    S = Qn.copy()
    A = M.copy()
    for _ in range(64):
        S_new = S + A @ S @ A.T
        A = A @ A
        if np.max(np.abs(S_new - S)) < tol * max(1.0, np.max(np.abs(S_new))):
            return S_new
        S = S_new
    return S


def shear_xz_profile(n_beads, H, zeta, kT, rate):
    """Continuous-time steady <Q_x Q_z>_j for a Hookean chain in simple shear:
    rate * zeta * kT * j (N - j) / (2 H^2 N), j = 1..N-1."""
    j = np.arange(1, n_beads)
    return rate * zeta * kT * j * (n_beads - j) / (2.0 * H * H * n_beads)


def fene_dumbbell_q2(H, b, kT):
    """Equilibrium <Q^2> of a FENE dumbbell: 3 (kT/H) b / (b + 5)."""
    return 3.0 * kT / H * b / (b + 5.0)


def maxwell_tension(H, kT):
    """Mean and variance of f = H |Q| for Q ~ Normal(0, kT/H I3)."""
    return np.sqrt(8.0 * H * kT / np.pi), H * kT * (3.0 - 8.0 / np.pi)
