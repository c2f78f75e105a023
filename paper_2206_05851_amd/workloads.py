"""Seeded synthetic inputs shared by the GPU library's tests/bench and the oracle.

This module holds no part of the method's arithmetic: it only draws parent
conformations and workload parameters, and converts a Weissenberg number into
a strain rate. Both the HIP path and the oracle receive the same FP64 arrays.

Units are the paper's reduced units (Sec. II): lengths in bead radius, energy
in kT, time in the single-bead diffusion time, so kT = zeta = 1 by default.
"""
import math

import numpy as np

HOOKEAN, FENE, HARMONIC = 0, 1, 2
QUIESCENT, UNIAXIAL, PLANAR, SHEAR = 0, 1, 2, 3


def rouse_lambda1(n_beads, H=1.0, zeta=1.0):
    """Longest relaxation time of a free-draining Rouse chain of N beads:
    lambda_1 = zeta / (8 H sin^2(pi / 2N))."""
    return zeta / (8.0 * H * math.sin(math.pi / (2.0 * n_beads)) ** 2)


def wi_to_rate(wi, n_beads, H=1.0, zeta=1.0):
    """Strain (or shear) rate for Weissenberg number Wi = rate * lambda_1."""
    return wi / rouse_lambda1(n_beads, H, zeta)


def equilibrium_bonds(n_bonds, spring, H, b, kT, rng):
    """Independent equilibrium bond vectors of a free-draining chain.

    Hookean: each component ~ Normal(0, kT/H).
    FENE: density proportional to (1 - Q^2/Q0^2)^(b/2), Q0^2 = b kT / H, drawn
    by rejection from the Hookean Gaussian with acceptance
    (1 - t)^(b/2) exp(b t / 2), t = Q^2/Q0^2 (zero for t >= 1).
    """
    sd = math.sqrt(kT / H)
    if spring == HOOKEAN:
        return rng.normal(0.0, sd, size=(n_bonds, 3))
    q0sq = b * kT / H
    out = np.empty((n_bonds, 3))
    filled = 0
    while filled < n_bonds:
        cand = rng.normal(0.0, sd, size=(max(16, 2 * (n_bonds - filled)), 3))
        t = (cand * cand).sum(axis=1) / q0sq
        with np.errstate(invalid="ignore", divide="ignore"):
            acc = np.where(t < 1.0, np.exp(0.5 * b * (np.log1p(-np.minimum(t, 1.0 - 1e-300)) + t)),
                           0.0)
        keep = cand[rng.random(len(cand)) < acc]
        take = min(len(keep), n_bonds - filled)
        out[filled:filled + take] = keep[:take]
        filled += take
    return out


def equilibrium_parent(n_beads, spring=HOOKEAN, H=1.0, b=0.0, kT=1.0, seed=0):
    """Parent conformation [N][3] (FP64): cumulative sum of equilibrium bonds,
    shifted so that its centre of mass is at the origin."""
    rng = np.random.default_rng(seed)
    bonds = equilibrium_bonds(n_beads - 1, spring, H, b, kT, rng)
    r = np.zeros((n_beads, 3))
    r[1:] = np.cumsum(bonds, axis=0)
    r -= r.mean(axis=0)
    return r


def group(n_beads, n_replicas, dt, spring=HOOKEAN, H=1.0, b=0.0, flow=QUIESCENT, rate=0.0,
          kT=1.0, zeta=1.0, noise_scale=1.0, stream_id=0, rest_length=0.0, lj_eps=0.0, lj_rmin=0.0,
          hi_radius=0.0):
    return dict(n_beads=int(n_beads), n_replicas=int(n_replicas), spring=int(spring),
                H=float(H), b=float(b), flow=int(flow), rate=float(rate), kT=float(kT),
                zeta=float(zeta), dt=float(dt), noise_scale=float(noise_scale),
                stream_id=int(stream_id), rest_length=float(rest_length), lj_eps=float(lj_eps),
                lj_rmin=float(lj_rmin), hi_radius=float(hi_radius))


# ---------------------------------------------------------------------------
# The five workload shapes. Each returns (groups, parents, run) where run holds
# seed, steps, sample_every and the Bell constants.
# ---------------------------------------------------------------------------
def rouse_fp64_small(n_replicas=64):
    """Hookean Rouse chain N=10, H=kT=zeta=1, uniaxial Wi=0.3, dt=1e-3,
    replicas cloned from one equilibrium conformation, 50 windows of 100
    steps, FP64, Philox seed 0."""
    N = 10
    g = group(N, n_replicas, 1e-3, HOOKEAN, 1.0, 0.0, UNIAXIAL, wi_to_rate(0.3, N))
    parent = equilibrium_parent(N, HOOKEAN, seed=100)
    return [g], [parent], dict(seed=0, steps=5000, sample_every=100, precision=64,
                               k0=1e-6, x_dagger=0.1)


def fene50(n_replicas=1024, steps=10000):
    """FENE chain N=50, b=100, uniaxial Wi=2, dt=1e-4, 1024 replicas,
    10^4 steps, per-spring mean/std every 100 steps, Bell k0=1e-6, x=0.1."""
    N = 50
    g = group(N, n_replicas, 1e-4, FENE, 1.0, 100.0, UNIAXIAL, wi_to_rate(2.0, N))
    parent = equilibrium_parent(N, FENE, 1.0, 100.0, seed=101)
    return [g], [parent], dict(seed=1, steps=steps, sample_every=100, precision=32,
                               k0=1e-6, x_dagger=0.1)


def batched512(n_groups=512, steps=5000, seed=3):
    """512 FENE chains: N ~ U{20..200}, b ~ U[50,200]; first half planar
    elongation Wi ~ U[0.5,5], second half simple shear Wi ~ U[1,50];
    R ~ U{16,32,64,128,256}; dt=1e-4, 5000 steps, sample every 100."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(20, 201, size=n_groups)
    bs = rng.uniform(50.0, 200.0, size=n_groups)
    Rs = rng.choice(np.array([16, 32, 64, 128, 256]), size=n_groups)
    half = n_groups // 2
    wis = np.concatenate([rng.uniform(0.5, 5.0, size=half),
                          rng.uniform(1.0, 50.0, size=n_groups - half)])
    groups, parents = [], []
    for i in range(n_groups):
        N = int(Ns[i])
        flow = PLANAR if i < half else SHEAR
        groups.append(group(N, int(Rs[i]), 1e-4, FENE, 1.0, float(bs[i]), flow,
                            wi_to_rate(float(wis[i]), N), stream_id=i))
        parents.append(equilibrium_parent(N, FENE, 1.0, float(bs[i]), seed=10000 + i))
    return groups, parents, dict(seed=seed, steps=steps, sample_every=100, precision=32,
                                 k0=1e-6, x_dagger=0.1)


def adjoint100(n_replicas=4096, steps=2000):
    """FENE chain N=100, b=100, uniaxial Wi=4, 4096 replicas, dt=1e-4, 2000
    steps, checkpoints every 100 steps, gradient w.r.t. (rate, H, b)."""
    N = 100
    g = group(N, n_replicas, 1e-4, FENE, 1.0, 100.0, UNIAXIAL, wi_to_rate(4.0, N))
    parent = equilibrium_parent(N, FENE, 1.0, 100.0, seed=102)
    return [g], [parent], dict(seed=2, steps=steps, sample_every=100, precision=32,
                               k0=1e-6, x_dagger=0.1, checkpoint_every=100)


def large1000(n_replicas=8192, steps=20000):
    """FENE chain N=1000, b=400, start-up uniaxial Wi=10, 8192 replicas,
    dt=5e-5, 2e4 steps, RSF and TSF windows of 500 steps, Bell events."""
    N = 1000
    g = group(N, n_replicas, 5e-5, FENE, 1.0, 400.0, UNIAXIAL, wi_to_rate(10.0, N))
    parent = equilibrium_parent(N, FENE, 1.0, 400.0, seed=103)
    return [g], [parent], dict(seed=4, steps=steps, sample_every=500, precision=32,
                               k0=1e-6, x_dagger=0.1, tsf=True)


def rsf50(n_replicas=1000, n_windows=20):
    """RSF sampling cycle (Sec. II) on a FENE chain N=50, b=100, in simple
    shear at Wi=50: one parent trajectory (parent noise tag) halted every 750
    steps, 1000 replicas re-cloned from it and evolved for S=750 steps
    (dt=1e-4), 20 windows; ISF and TSF from the parent, RSF from the
    replicas, sigma(N_R) over blocks of 10, 20, 40 and 50 replicas, Bell rates
    and MFTU with k0=1e-6, x=0.1."""
    N = 50
    g = group(N, n_replicas, 1e-4, FENE, 1.0, 100.0, SHEAR, wi_to_rate(50.0, N))
    parent = equilibrium_parent(N, FENE, 1.0, 100.0, seed=104)
    return [g], [parent], dict(seed=5, sample_every=750, parent_steps=750, n_windows=n_windows,
                               precision=32, k0=1e-6, x_dagger=0.1, blocks=(10, 20, 40, 50))


def collapsed_parent(n_beads, seed=0, spacing=2.0, jitter=0.05):
    """Compact self-avoiding conformation [N][3] for the collapsed-polymer
    model: a serpentine path through a cubic lattice of the given spacing (the
    bond rest length and the LJ minimum, 2a), so bonded and nearest
    non-bonded beads sit at 2a; plus seeded Gaussian jitter; centre of mass
    at the origin."""
    side = 1
    while side ** 3 < n_beads:
        side += 1
    sites = []
    for z in range(side):
        ys = range(side) if z % 2 == 0 else range(side - 1, -1, -1)
        for yi, y in enumerate(ys):
            xs = range(side) if (z * side + yi) % 2 == 0 else range(side - 1, -1, -1)
            for x in xs:
                sites.append((x, y, z))
    r = spacing * np.array(sites[:n_beads], dtype=np.float64)
    r += np.random.default_rng(seed).normal(0.0, jitter, size=r.shape)
    return r - r.mean(axis=0)


def collapsed50(n_replicas=1000, n_windows=20):
    """The paper's collapsed polymer (Sec. II) without hydrodynamic
    interaction: N=50 beads, harmonic backbone springs kappa=400 kT/a^2 with
    rest length 2a, LJ self-association u=1 kT between non-adjacent beads,
    zeta=1 (time in units of the single-bead diffusion time), dt=1e-5, simple
    shear at gamma-dot=30; RSF cycle with a parent re-cloned into 1000
    replicas every 750 steps (S = 0.0075), 20 windows."""
    N = 50
    g = group(N, n_replicas, 1e-5, HARMONIC, 400.0, 0.0, SHEAR, 30.0, rest_length=2.0, lj_eps=1.0,
              lj_rmin=2.0)
    parent = collapsed_parent(N, seed=105)
    return [g], [parent], dict(seed=6, sample_every=750, parent_steps=750, n_windows=n_windows,
                               precision=32, k0=1e-6, x_dagger=0.1, blocks=(10, 20, 40, 50))


def hi50(n_replicas=50, n_windows=4):
    """The paper's full model (Sec. II): N=50 beads, harmonic backbone
    kappa=400 kT/a^2 with rest length 2a, LJ u=1 kT between non-adjacent
    beads, hydrodynamic interaction through the RPY tensor (Eqs. 2-3, a=1),
    simple shear gamma-dot=30, dt=1e-5; RSF cycle with N_R=50 replicas
    re-cloned from the parent every 750 steps (S = 0.0075), 4 windows."""
    N = 50
    g = group(N, n_replicas, 1e-5, HARMONIC, 400.0, 0.0, SHEAR, 30.0, rest_length=2.0, lj_eps=1.0,
              lj_rmin=2.0, hi_radius=1.0)
    parent = collapsed_parent(N, seed=106)
    return [g], [parent], dict(seed=7, sample_every=750, parent_steps=750, n_windows=n_windows,
                               precision=32, k0=1e-6, x_dagger=0.1, blocks=(10, 25, 50))
