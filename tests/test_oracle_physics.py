"""Pins for the oracle's dynamics: spring laws, flows, the Euler-Maruyama
update of Eq. (1) with the free-draining tensor Eq. (2), and the sampled
tension of Eq. (4) (zero rest length), each checked against something other
than the oracle: bond-space closed forms, potentials, Newton solutions and
textbook equilibrium results."""
import numpy as np
import pytest
from scipy import optimize

import closed_forms as cf
from oracle import ora
from paper_2206_05851_amd import workloads as wl


def g(N, R, dt, **kw):
    return wl.group(N, R, dt, **kw)


# ---- spring law ---------------------------------------------------------------
@pytest.mark.parametrize("kind,H,b", [(ora.HOOKEAN, 1.0, 0.0), (ora.HOOKEAN, 2.5, 0.0),
                                      (ora.FENE, 1.0, 100.0), (ora.FENE, 3.0, 20.0)])
def test_spring_force_is_potential_gradient(kind, H, b):
    kT = 1.3
    rng = np.random.default_rng(1)

    def U(Q):
        if kind == ora.HOOKEAN:
            return 0.5 * H * Q @ Q
        q0sq = b * kT / H
        return -0.5 * H * q0sq * np.log(1.0 - Q @ Q / q0sq)

    for _ in range(50):
        Q = rng.normal(0, 1.0, 3)
        if kind == ora.FENE:
            Q *= rng.uniform(0.05, 0.95) * np.sqrt(b * kT / H) / np.linalg.norm(Q)
        F, gf, f, clamped = ora.spring(kind, H, b, kT, Q)
        num = np.array([(U(Q + e) - U(Q - e)) / 2e-6 for e in 1e-6 * np.eye(3)])
        assert np.allclose(F, num, rtol=1e-6, atol=1e-8)
        assert np.isclose(f, np.linalg.norm(F), rtol=1e-14)       # tension = |force|
        assert not clamped


def test_fene_guard_clamps_at_one_minus_delta():
    H, b, kT = 1.0, 100.0, 1.0
    Q0 = 10.0
    for s, expect in [(0.998, False), (0.9995, True), (1.2, True)]:
        Q = np.array([np.sqrt(s) * Q0, 0.0, 0.0])
        F, gf, f, clamped = ora.spring(ora.FENE, H, b, kT, Q)
        assert clamped == expect
        if expect:
            assert np.isclose(gf, 1.0 / 1e-3, rtol=1e-12)
        else:
            assert np.isclose(gf, 1.0 / (1.0 - s), rtol=1e-9)


def test_flow_fields():
    r = np.array([1.5, -2.0, 0.7])
    assert np.allclose(ora.flow_velocity(ora.SHEAR, 3.0, r), [3.0 * 0.7, 0, 0])
    assert np.allclose(ora.flow_velocity(ora.UNIAXIAL, 2.0, r), [3.0, 2.0, -0.7])
    assert np.allclose(ora.flow_velocity(ora.PLANAR, 2.0, r), [3.0, 4.0, 0.0])
    assert np.allclose(ora.flow_velocity(ora.QUIESCENT, 2.0, r), 0)
    for fl in (ora.UNIAXIAL, ora.PLANAR, ora.SHEAR):   # incompressible: trace(kappa) = 0
        K = np.array([ora.flow_velocity(fl, 1.7, e) for e in np.eye(3)]).T
        assert abs(np.trace(K)) < 1e-15
        assert np.allclose(K, cf.flow_matrix(fl, 1.7))


# ---- deterministic Hookean dynamics = bond-space matrix power ---------------------
@pytest.mark.parametrize("flow,rate", [(ora.QUIESCENT, 0.0), (ora.UNIAXIAL, 0.7),
                                       (ora.PLANAR, -0.4), (ora.SHEAR, 3.0)])
def test_hookean_noise_off_matches_bond_space_matrix_power(flow, rate):
    N, dt, H, zeta, kT, n = 7, 2e-3, 1.7, 1.3, 0.9, 400
    parent = wl.equilibrium_parent(N, seed=5)
    o = ora.Oracle([g(N, 2, dt, H=H, zeta=zeta, kT=kT, flow=flow, rate=rate, noise_scale=0.0)],
                   seed=0, sample_every=100, max_windows=10)
    o.init_chains([parent])
    o.step(n)
    M, _ = cf.em_matrices(N, H, zeta, kT, dt, flow, rate)
    Qn = np.linalg.matrix_power(M, n) @ cf.bonds_of(parent)
    for rep in o.positions()[0]:
        assert np.allclose(cf.bonds_of(rep), Qn, rtol=1e-11, atol=1e-12)
    # tension samples are |F| = H |Q| of the same bonds at each window end
    smp = o.samples()[0]
    Q4 = (np.linalg.matrix_power(M, 400) @ cf.bonds_of(parent)).reshape(3, N - 1)
    assert np.allclose(smp[3, 0], H * np.linalg.norm(Q4, axis=0), rtol=1e-11)


def test_centre_of_mass_moves_with_flow_only():
    # noise off: springs exert no net force, so r_cm' = (I + dt kappa) r_cm
    N, dt, rate, n = 6, 1e-3, 0.8, 300
    parent = wl.equilibrium_parent(N, seed=2) + np.array([1.0, -2.0, 0.5])
    o = ora.Oracle([g(N, 1, dt, flow=ora.UNIAXIAL, rate=rate, noise_scale=0.0)], 0, 50, 10)
    o.init_chains([parent])
    o.step(n)
    A = np.eye(3) + dt * cf.flow_matrix(ora.UNIAXIAL, rate)
    expect = np.linalg.matrix_power(A, n) @ parent.mean(axis=0)
    assert np.allclose(o.positions()[0][0].mean(axis=0), expect, rtol=1e-12)


# ---- stochastic Hookean dynamics: exact EM moments -------------------------------
@pytest.mark.parametrize("flow,rate,noise_map", [(ora.UNIAXIAL, 0.5, 0), (ora.SHEAR, 4.0, 0),
                                                (ora.UNIAXIAL, 0.5, 1), (ora.SHEAR, 4.0, 1),
                                                (ora.UNIAXIAL, 0.5, 2), (ora.SHEAR, 4.0, 2)])
def test_hookean_moments_match_exact_em_recursion(flow, rate, noise_map):
    # the exact recursion holds only for independent standard normals at
    # every (step, bead, component): both noise maps must give them
    N, R, dt, H, kT, zeta, n = 6, 4000, 1e-2, 1.0, 1.0, 1.0, 150
    parent = wl.equilibrium_parent(N, seed=3)
    o = ora.Oracle([g(N, R, dt, H=H, kT=kT, zeta=zeta, flow=flow, rate=rate)], seed=42,
                   sample_every=50, max_windows=10, noise_map=noise_map)
    o.init_chains([parent])
    o.step(n)
    Q = cf.bonds_of(o.positions()[0])                  # [R, 3(N-1)]
    M, Qn = cf.em_matrices(N, H, zeta, kT, dt, flow, rate)
    m, S = cf.moments_after(n, cf.bonds_of(parent), M, Qn)
    z_mean = (Q.mean(axis=0) - m) / np.sqrt(np.diag(S) / R)
    assert np.max(np.abs(z_mean)) < 4.5, z_mean
    C = np.cov(Q.T)
    sd = np.sqrt((S ** 2 + np.outer(np.diag(S), np.diag(S))) / (R - 1))   # Gaussian SE of cov
    z_cov = (C - S) / sd
    assert np.max(np.abs(z_cov)) < 5.0
    assert np.mean(z_cov ** 2) < 1.5
    if flow == ora.SHEAR:   # the x-z cross covariance is the flow signature
        nb = N - 1
        xz = np.diag(S[:nb, 2 * nb:])
        assert np.all(xz > 0) and np.all(np.diag(C[:nb, 2 * nb:]) > 0)


def test_hookean_dumbbell_variance():
    # EM-exact stationary <Q^2> = 3 (kT/H) / (1 - H dt / zeta)
    R, dt, H = 8000, 2e-2, 1.0
    parent = np.array([[0.0, 0.0, 0.0], [0.3, 0.0, 0.0]])
    o = ora.Oracle([g(2, R, dt, H=H)], seed=8, sample_every=100, max_windows=10)
    o.init_chains([parent])
    o.step(600)             # 6 time units = 24 relaxation times zeta/4H
    Q = np.diff(o.positions()[0], axis=1)[:, 0, :]
    q2 = (Q ** 2).sum(axis=1)
    expect = 3.0 / (1.0 - H * dt)
    assert abs(q2.mean() - expect) < 4.5 * q2.std() / np.sqrt(R)


def test_em_weak_order_one_hookean_dumbbell():
    # Euler-Maruyama is weakly first order: the stationary bias of <Q^2> about
    # the continuous 3 kT/H halves when dt halves. The EM-exact biases give the
    # ratio [1/(1 - 0.08) - 1] / [1/(1 - 0.04) - 1] = 2.087 (1 would mean no
    # convergence, 4 second order). Estimated from the oracle's tension
    # samples f = H |Q| over 10 decorrelated windows of 8000 replicas each.
    H, R = 1.0, 8000
    parent = np.array([[0.0, 0.0, 0.0], [0.3, 0.0, 0.0]])
    bias, se = [], []
    for dt, S in ((0.08, 25), (0.04, 50)):
        o = ora.Oracle([g(2, R, dt, H=H)], seed=31, sample_every=S, max_windows=12)
        o.init_chains([parent])
        o.step(12 * S)        # windows 2 time units = 8 relaxation times zeta/4H apart
        q2 = (o.samples()[0][2:, :, 0] / H) ** 2
        bias.append(q2.mean() - 3.0 / H)
        se.append(q2.std() / np.sqrt(q2.size))
    ratio = bias[0] / bias[1]
    ratio_se = ratio * np.hypot(se[0] / bias[0], se[1] / bias[1])
    expect = (1.0 / (1.0 - 0.08) - 1.0) / (1.0 / (1.0 - 0.04) - 1.0)
    assert abs(ratio - expect) < 4.0 * ratio_se, (ratio, ratio_se)
    assert abs(ratio - 1.0) > 4.0 * ratio_se and abs(ratio - 4.0) > 4.0 * ratio_se


def test_fene_dumbbell_equilibrium_q2():
    # <Q^2> = 3 (kT/H) b/(b+5) for the FENE dumbbell; EM bias O(dt) << SE here
    R, dt, H, b = 8000, 1e-3, 1.0, 10.0
    parent = np.array([[0.0, 0.0, 0.0], [0.5, 0.2, 0.0]])
    o = ora.Oracle([g(2, R, dt, spring=ora.FENE, H=H, b=b)], seed=9, sample_every=100,
                   max_windows=40)
    o.init_chains([parent])
    o.step(3000)
    Q = np.diff(o.positions()[0], axis=1)[:, 0, :]
    q2 = (Q ** 2).sum(axis=1)
    expect = cf.fene_dumbbell_q2(H, b, 1.0)
    assert abs(q2.mean() - expect) < 4.5 * q2.std() / np.sqrt(R)
    assert abs(q2.mean() - 3.0) > 10 * q2.std() / np.sqrt(R)   # distinguishes FENE from Hookean


def test_rouse_equilibrium_tension_is_maxwell():
    # independent equilibrium parents; tension f = H|Q| with Q ~ N(0, kT/H I)
    N, G, R, dt = 8, 48, 16, 1e-3
    groups = [g(N, R, dt, stream_id=i) for i in range(G)]
    parents = [wl.equilibrium_parent(N, seed=500 + i) for i in range(G)]
    o = ora.Oracle(groups, seed=3, sample_every=200, max_windows=10)
    o.init_chains(parents)
    o.step(1000)
    mean, std = o.average_forces()
    per_group = mean.reshape(5, G, N - 1).mean(axis=(0, 2))
    mu, var = cf.maxwell_tension(1.0, 1.0)
    assert abs(per_group.mean() - mu) < 4.5 * per_group.std() / np.sqrt(G)
    # replicas of one parent stay correlated over these times, so the marginal
    # variance is taken over all groups' samples of the last window
    last = np.stack([s[-1] for s in o.samples()])          # [G, R, N-1]
    pooled_var = last.var()
    assert abs(pooled_var - var) < 0.1 * var
    assert np.all(std > 0)


def test_replica_std_is_unbiased_maxwell_spread():
    # Pins the replica standard deviation (denominator R - 1) of the RSF and TSF
    # estimates. Hookean dumbbells (one spring) with H = kT = zeta = 1: the bond
    # relaxes at rate 2H/zeta and its EM-stationary variance per component is
    # v = (kT/H) / (1 - H dt/zeta). Windows of S dt = 5 time units leave every
    # replica of a window independent of its clone source and of the previous
    # window (correlation e^-10), so each window's replica variance over R = 3
    # replicas is an unbiased estimate of the Maxwell variance v H^2 (3 - 8/pi).
    # A denominator R would give 2/3 of it; the band below is 4.5 standard errors.
    R, G, dt, S, W = 3, 400, 0.01, 500, 10
    groups = [g(2, R, dt, stream_id=i) for i in range(G)]
    parents = [wl.equilibrium_parent(2, seed=900 + i) for i in range(G)]
    o = ora.Oracle(groups, seed=11, sample_every=S, max_windows=W, tsf=True)
    o.init_chains(parents)
    o.step(S * W)
    mean, std, tmean, tstd = o.average_forces(tsf=True)
    v = 1.0 / (1.0 - dt)
    mu_exact, var_exact = np.sqrt(8.0 * v / np.pi), v * (3.0 - 8.0 / np.pi)
    s2 = std[1:] ** 2                                   # first window still remembers the parent
    se = s2.std() / np.sqrt(s2.size)
    assert abs(s2.mean() - var_exact) < 4.5 * se, (s2.mean(), var_exact, se)
    assert abs(s2.mean() - (R - 1) / R * var_exact) > 10 * se
    assert abs(mean[1:].mean() - mu_exact) < 4.5 * mean[1:].std() / np.sqrt(mean[1:].size)
    # the same outputs against numpy's ddof=1 statistics of the oracle's samples
    smp, tsmp = o.samples(tsf=True)
    per = np.stack([x[:, :, 0] for x in smp], axis=1)   # [W][G][R]
    tper = np.stack([x[:, :, 0] for x in tsmp], axis=1)
    assert np.allclose(std, per.std(axis=2, ddof=1), rtol=1e-12, atol=0)
    assert np.allclose(mean, per.mean(axis=2), rtol=1e-13, atol=0)
    assert np.allclose(tstd, tper.std(axis=2, ddof=1), rtol=1e-12, atol=0)
    assert np.allclose(tmean, tper.mean(axis=2), rtol=1e-13, atol=0)
    # R = 1: the spread is defined as 0
    one = ora.Oracle([g(2, 1, dt)], seed=11, sample_every=S, max_windows=1)
    one.init_chains([parents[0]])
    one.step(S)
    assert one.average_forces()[1][0, 0] == 0.0


def _mean_tension_gaussian(m, cov3, H, n=400000, seed=0):
    """E[H |Q|] for Q ~ Normal(m, cov3), by numpy Monte Carlo (independent RNG)."""
    rng = np.random.default_rng(seed)
    L = np.linalg.cholesky(cov3 + 1e-300 * np.eye(3))
    Q = m + rng.standard_normal((n, 3)) @ L.T
    f = H * np.linalg.norm(Q, axis=1)
    return f.mean()


def test_transient_rsf_profile_matches_exact_gaussian():
    # Small version of the N=10 uniaxial Hookean case: each window's replica
    # mean tension has an exact expectation (Gaussian bonds with the EM mean
    # and covariance), evaluated here by independent Monte Carlo.
    N, R, dt, S, W = 10, 1024, 1e-3, 100, 4
    rate = wl.wi_to_rate(0.3, N)
    parent = wl.equilibrium_parent(N, seed=100)
    o = ora.Oracle([g(N, R, dt, flow=ora.UNIAXIAL, rate=rate)], seed=0, sample_every=S,
                   max_windows=W)
    o.init_chains([parent])
    o.step(S * W)
    mean, std = o.average_forces()
    M, Qn = cf.em_matrices(N, 1.0, 1.0, 1.0, dt, ora.UNIAXIAL, rate)
    Q0 = cf.bonds_of(parent)
    nb = N - 1
    for w in range(W):
        m, Sig = cf.moments_after(S * (w + 1), Q0, M, Qn)
        for j in range(nb):
            idx = [j, nb + j, 2 * nb + j]
            e = _mean_tension_gaussian(m[idx], Sig[np.ix_(idx, idx)], 1.0, seed=w * 100 + j)
            z = (mean[w, j] - e) / (std[w, j] / np.sqrt(R))
            assert abs(z) < 4.5, (w, j, z)


def test_shear_steady_profile_closed_form_vs_recursion():
    # the continuous parabolic <Qx Qz>_j is the dt -> 0 limit of the EM fixed point
    N, rate = 9, 2.0
    for dt in (1e-3, 5e-4):
        M, Qn = cf.em_matrices(N, 1.0, 1.0, 1.0, dt, ora.SHEAR, rate)
        S = cf.stationary_cov(M, Qn)
        nb = N - 1
        xz = np.diag(S[:nb, 2 * nb:])
        exact = cf.shear_xz_profile(N, 1.0, 1.0, 1.0, rate)
        assert np.allclose(xz, exact, rtol=5 * dt)


def test_stretched_fene_steady_state_matches_newton():
    # Noise off, strong uniaxial flow: the EM fixed point satisfies the force
    # balance kappa.r_i + Fnet_i/zeta = 0 exactly; solve it by Newton in 1-D
    # and compare, and check the parabolic tension T_j = zeta*rate*sum_{i>j} x_i.
    N, H, b, rate, dt = 10, 1.0, 50.0, 0.2, 2e-3
    q0sq = b / H
    x0 = 0.5 * (np.arange(N) - (N - 1) / 2)
    parent = np.stack([x0, 1e-3 * np.sin(np.arange(N)), 1e-3 * np.cos(np.arange(N))], axis=1)
    parent -= parent.mean(axis=0)
    o = ora.Oracle([g(N, 1, dt, spring=ora.FENE, H=H, b=b, flow=ora.UNIAXIAL, rate=rate,
                      noise_scale=0.0)], seed=0, sample_every=1000, max_windows=100)
    o.init_chains([parent])
    o.step(100000)
    r = o.positions()[0][0]
    x = r[:, 0] - r[:, 0].mean()

    def resid(xs):
        q = np.diff(xs)
        F = H * q / (1.0 - q * q / q0sq)
        Fnet = np.concatenate([F, [0.0]]) - np.concatenate([[0.0], F])
        return rate * xs + Fnet

    xs = optimize.fsolve(resid, x, xtol=1e-14)
    assert np.max(np.abs(resid(xs))) < 1e-10
    assert np.allclose(x, xs, atol=1e-9)
    assert np.max(np.abs(r[:, 1:])) < 1e-8
    mean, _ = o.average_forces()
    T = np.array([rate * xs[j + 1:].sum() for j in range(N - 1)])
    assert np.allclose(mean[-1], T, rtol=1e-8)
    # parabolic: nearly j(N-j) shaped, maximal in the middle, symmetric
    assert np.argmax(T) in (N // 2 - 1, N // 2)
    assert np.allclose(T, T[::-1], rtol=1e-8)


def test_rsf_standard_error_scales_as_inverse_sqrt_replicas():
    # Spread of the RSF estimate over independent replica sets: sigma ~ N_R^-1/2
    N, G, dt, S = 6, 200, 1e-3, 100
    parent = wl.equilibrium_parent(N, seed=21)
    sig = {}
    for R in (10, 40):
        groups = [g(N, R, dt, stream_id=i) for i in range(G)]
        o = ora.Oracle(groups, seed=R, sample_every=S, max_windows=1)
        o.init_chains([parent] * G)
        o.step(S)
        mean, _ = o.average_forces()
        sig[R] = mean[0].reshape(G, N - 1)[:, 2].std(ddof=1)
    ratio = sig[40] / sig[10]
    assert abs(ratio - 0.5) < 0.5 * 4 * np.sqrt(2.0 / G), ratio


def test_batch_and_replica_subset_invariance():
    N1, N2, dt = 7, 12, 1e-3
    d1 = g(N1, 8, dt, spring=ora.FENE, b=30.0, flow=ora.SHEAR, rate=2.0, stream_id=3)
    d2 = g(N2, 5, dt, flow=ora.PLANAR, rate=0.3, stream_id=9)
    p1 = wl.equilibrium_parent(N1, ora.FENE, 1.0, 30.0, seed=1)
    p2 = wl.equilibrium_parent(N2, seed=2)
    both = ora.Oracle([d1, d2], seed=77, sample_every=20, max_windows=5)
    both.init_chains([p1, p2])
    both.step(100)
    alone = ora.Oracle([d2], seed=77, sample_every=20, max_windows=5)
    alone.init_chains([p2])
    alone.step(100)
    assert np.array_equal(both.samples()[1], alone.samples()[0])
    sub = ora.Oracle([d1], seed=77, sample_every=20, max_windows=5)
    sub.set_replicas(0, 3, 6)
    sub.init_chains([p1])
    sub.step(100)
    assert np.array_equal(both.samples()[0][:, 3:6], sub.samples()[0])


def test_tsf_is_time_average_of_per_step_tension():
    N, R, dt, S = 5, 3, 1e-3, 10
    d = g(N, R, dt, spring=ora.FENE, b=20.0, flow=ora.UNIAXIAL, rate=0.5)
    p = wl.equilibrium_parent(N, ora.FENE, 1.0, 20.0, seed=4)
    o = ora.Oracle([d], seed=5, sample_every=S, max_windows=3, tsf=True)
    o.init_chains([p])
    step1 = ora.Oracle([d], seed=5, sample_every=1, max_windows=30)
    step1.init_chains([p])
    o.step(3 * S)
    step1.step(3 * S)
    every = step1.samples()[0]                        # [30][R][N-1], per step
    smp, tsf = o.samples(tsf=True)
    assert np.allclose(tsf[0], every.reshape(3, S, R, N - 1).mean(axis=1), rtol=1e-13)
    assert np.array_equal(smp[0], every[S - 1::S])


def test_invalid_inputs_rejected():
    with pytest.raises(ora.OracleError):
        ora.Oracle([g(1, 4, 1e-3)], 0, 10, 1)
    with pytest.raises(ora.OracleError):
        ora.Oracle([g(4, 0, 1e-3)], 0, 10, 1)
    with pytest.raises(ora.OracleError):
        ora.Oracle([g(4, 2, 0.0)], 0, 10, 1)
    with pytest.raises(ora.OracleError):
        ora.Oracle([g(4, 2, 1e-3, spring=ora.FENE, b=0.0)], 0, 10, 1)
    o = ora.Oracle([g(3, 2, 1e-3, spring=ora.FENE, b=4.0)], 0, 10, 1)
    with pytest.raises(ora.OracleError):
        o.step(5)                                     # before init
    with pytest.raises(ora.OracleError):               # |Q| = 2.5 >= Q0 = 2
        o.init_chains([np.array([[0, 0, 0], [2.5, 0, 0], [3.0, 0, 0.0]])])
    o.init_chains([np.array([[0, 0, 0], [1.0, 0, 0], [2.0, 0, 0.0]])])
    with pytest.raises(ora.OracleError):
        o.step(20)                                    # 2 windows > capacity 1
