"""Pins for the oracle's RSF sampling cycle (Sec. II: the parent is halted,
re-cloned into N_R replicas that evolve for S, sampled once; the parent then
continues), its ISF/TSF companions, the block spread sigma(N_R) (Figs. 2, 5),
the MFTU estimator (Sec. III) and the replica-fidelity diagnostics of Eq. 5
and R_Gz (Sec. IV)."""
import math

import numpy as np
import pytest

import closed_forms as cf
from oracle import ora
from paper_2206_05851_amd import workloads as wl
from test_oracle_rng import philox_py


def _tensions(Qs, nb, H):
    """Stacked bond vector(s) [..., 3 nb] -> spring tensions H |Q_j| [..., nb]."""
    Q = np.asarray(Qs).reshape(Qs.shape[:-1] + (3, nb))
    return H * np.sqrt((Q ** 2).sum(axis=-2))


def _pair(desc, parent, seed, S, P, W, R, tsf=True):
    par = ora.Oracle([dict(desc, n_replicas=1)], seed, P, W, tsf=tsf)
    par.set_tag(ora.TAG_PARENT)
    par.init_chains([parent])
    rep = ora.Oracle([dict(desc, n_replicas=R)], seed, S, W)
    return par, rep


@pytest.mark.parametrize("flow,rate", [(wl.UNIAXIAL, 0.4), (wl.SHEAR, 3.0), (wl.PLANAR, 0.7)])
def test_rsf_cycle_noise_off_matches_matrix_powers(flow, rate):
    # Hookean, noise off: the bond map is Q -> M Q, so the parent after
    # (w+1)P steps, its per-step tensions over the window and the replicas
    # after S more steps are matrix powers of M applied to Q0.
    N, H, dt, S, P, W = 6, 1.3, 2e-3, 7, 5, 4
    desc = wl.group(N, 3, dt, H=H, flow=flow, rate=rate, noise_scale=0.0)
    parent = wl.equilibrium_parent(N, H=H, seed=11)
    par, rep = _pair(desc, parent, 5, S, P, W, 3)
    rep.rsf_cycle(par, W, P)
    isf, isf_std, tsf, _ = par.average_forces(tsf=True)
    rsf, rsf_std = rep.average_forces()
    M, _ = cf.em_matrices(N, H, 1.0, 1.0, dt, flow, rate, noise_scale=0.0)
    Q = cf.bonds_of(parent)
    nb = N - 1
    for w in range(W):
        steps = [np.linalg.matrix_power(M, n) @ Q for n in range(w * P + 1, (w + 1) * P + 1)]
        Qp = steps[-1]
        assert np.allclose(isf[w], _tensions(Qp, nb, H), rtol=1e-12, atol=0)
        assert np.allclose(tsf[w], np.mean([_tensions(q, nb, H) for q in steps], axis=0), rtol=1e-12, atol=0)
        Qr = np.linalg.matrix_power(M, S) @ Qp
        assert np.allclose(rsf[w], _tensions(Qr, nb, H), rtol=1e-12, atol=0)
    # identical replicas: std is zero up to the rounding of the mean
    assert np.max(rsf_std) < 1e-14 * np.max(rsf) and np.all(isf_std == 0.0)


def test_rsf_replicas_match_exact_gaussian_given_parent():
    # Hookean, replicas with noise: given the parent bonds Qp at the re-clone,
    # the replica bonds after S steps are Normal(M^S Qp, Sigma_S) exactly.
    N, H, dt, S, P, R = 4, 1.0, 1e-2, 30, 20, 4000
    desc = wl.group(N, R, dt, H=H, flow=wl.UNIAXIAL, rate=0.3)
    parent = wl.equilibrium_parent(N, H=H, seed=3)
    par, rep = _pair(desc, parent, 8, S, P, 2, R)
    rep.rsf_cycle(par, 2, P)
    Qp = cf.bonds_of(par.positions()[0][0])
    M, Qn = cf.em_matrices(N, H, 1.0, 1.0, dt, wl.UNIAXIAL, 0.3)
    m, C = cf.moments_after(S, Qp, M, Qn)
    Qr = cf.bonds_of(rep.positions()[0])
    se = np.sqrt(np.diag(C) / R)
    assert np.all(np.abs(Qr.mean(axis=0) - m) < 4.5 * se)
    emp = np.cov(Qr.T)
    sd = np.sqrt(np.outer(np.diag(C), np.diag(C)) + C ** 2) / np.sqrt(R)
    assert np.all(np.abs(emp - C) < 5.0 * sd)


def test_rsf_windows_draw_independent_noise():
    # With a linear (Hookean) map the replica displacement from M^S Qp is a
    # linear function of that window's noise alone: if two windows reused the
    # same counters, replica k's displacements would be identical.
    N, H, dt, S, P, R = 3, 1.0, 1e-2, 10, 10, 2000
    desc = wl.group(N, R, dt, H=H)
    parent = wl.equilibrium_parent(N, H=H, seed=4)
    par, rep = _pair(desc, parent, 2, S, P, 2, R)
    M, _ = cf.em_matrices(N, H, 1.0, 1.0, dt, wl.QUIESCENT, 0.0)
    MS = np.linalg.matrix_power(M, S)
    d = []
    for _ in range(2):
        rep.rsf_cycle(par, 1, P)
        Qp = cf.bonds_of(par.positions()[0][0])
        d.append(cf.bonds_of(rep.positions()[0]) - MS @ Qp)
    for c in range(d[0].shape[1]):
        corr = np.corrcoef(d[0][:, c], d[1][:, c])[0, 1]
        assert abs(corr) < 4.0 / math.sqrt(R)
    assert rep.n_windows == 2


def _normals_py(words):
    u = [((x >> 9) + 0.5) * 2.0 ** -23 for x in words]
    r0, r1 = math.sqrt(-2 * math.log(u[0])), math.sqrt(-2 * math.log(u[2]))
    return [r0 * math.cos(2 * math.pi * u[1]), r0 * math.sin(2 * math.pi * u[1]),
            r1 * math.cos(2 * math.pi * u[3])]


def test_parent_step_uses_parent_tag():
    # One step of a 2-bead Hookean parent: r_i += dt (kappa r_i + F_i/zeta) + sigma xi_i
    # with xi_i from counter (0, i, 0, 1<<24 | group) (pure-Python Philox).
    H, dt, rate, seed, gid = 1.7, 1e-3, 0.9, 0x1234_5678_9ABC, 5
    desc = wl.group(2, 1, dt, H=H, flow=wl.PLANAR, rate=rate, stream_id=gid)
    r = np.array([[0.1, -0.4, 0.3], [0.9, 0.2, -0.5]])
    par = ora.Oracle([desc], seed, 1, 1)
    par.set_tag(ora.TAG_PARENT)
    par.init_chains([r])
    par.step(1)
    got = par.positions()[0][0]
    Q = r[1] - r[0]
    F = [H * Q, -H * Q]
    kap = np.diag([rate, -rate, 0.0])
    sigma = math.sqrt(2 * dt)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    for i in range(2):
        xi = np.array(_normals_py(philox_py((0, i, 0, (1 << 24) | gid), key)))
        exp = r[i] + dt * (kap @ r[i] + F[i]) + sigma * xi
        assert np.allclose(got[i], exp, rtol=0, atol=1e-14)
    # the replica tag draws a different displacement
    rep = ora.Oracle([desc], seed, 1, 1)
    rep.init_chains([r])
    rep.step(1)
    assert np.max(np.abs(rep.positions()[0][0] - got)) > 1e-3


def test_reclone_only_at_window_boundaries():
    desc = wl.group(3, 2, 1e-3)
    o = ora.Oracle([desc], 0, 10, 5)
    p = wl.equilibrium_parent(3, seed=0)
    o.init_chains([p])
    o.step(15)
    with pytest.raises(ora.OracleError):
        o.reclone([p])
    o.step(5)
    o.reclone([p])
    o.step(10)
    assert o.n_windows == 3


def test_block_sigma_definition_and_inverse_sqrt_scaling():
    # sigma(N_R): std over consecutive blocks of N_R replicas of the block-mean
    # tension; independent replicas give sigma = std / sqrt(N_R) (the paper's
    # N_R^-1/2 law, Figs. 2 and 5).
    N, R, S = 8, 1600, 40
    desc = wl.group(N, R, 1e-2)
    o = ora.Oracle([desc], 9, S, 2)
    o.init_chains([wl.equilibrium_parent(N, seed=2)])
    o.step(2 * S)
    smp = o.samples()[0]                   # [W][R][N-1]
    for nr in (10, 40):
        B = R // nr
        bm = smp[:, :B * nr].reshape(2, B, nr, N - 1).mean(axis=2)
        ref = bm.std(axis=1, ddof=1)
        assert np.allclose(o.block_sigma(nr), ref, rtol=1e-12, atol=0)
    s10, s40 = o.block_sigma(10), o.block_sigma(40)
    ratio = np.mean(s10) / np.mean(s40)
    assert abs(ratio - 2.0) < 0.2
    full = smp.std(axis=1, ddof=1)
    assert abs(np.mean(s10) / np.mean(full / math.sqrt(10)) - 1.0) < 0.1
    # ragged tail: the last R mod N_R replicas are not used
    assert np.allclose(o.block_sigma(R), 0.0)


def test_mftu_is_inverse_mean_total_rate():
    # Worked example (Sec. III / supplementary vWF section): constant mean
    # force 0.28 pN on 25 domains, k0 = 7e-4, f_u = 1.1 -> 44.30 s.
    o = ora.Oracle([wl.group(26, 1, 1e-3)], 0, 1, 4)
    mean = np.full((4, 25), 0.28)
    _, rsum = o.bell_rates(mean, k0=7e-4, x_dagger=1.0 / 1.1)
    m = o.mftu(rsum)
    assert abs(m[0] - 44.30) < 0.01
    # fluctuating profiles: 1/<K> over windows, never more than <1/K> (Jensen)
    rng = np.random.default_rng(0)
    mean = rng.normal(0.28, 0.5, size=(4, 25))
    _, rsum = o.bell_rates(mean, k0=7e-4, x_dagger=1.0 / 1.1)
    m = o.mftu(rsum)
    assert np.isclose(m[0], 4.0 / rsum[:, 0].sum(), rtol=1e-14)
    assert m[0] <= np.mean(1.0 / rsum[:, 0])


def test_mftu_events_trial_zero_uses_the_bell_event_draws():
    # trial 0 over the sampled windows draws exactly the uniforms of
    # bell_rates' events, so its first window is the first row with an event
    N, W, S, dt = 12, 30, 10, 1e-2
    o = ora.Oracle([wl.group(N, 1, dt, stream_id=5)], 3, S, W)
    rng = np.random.default_rng(1)
    mean = rng.uniform(5.0, 25.0, size=(W, N - 1))
    rates, rsum, ev = o.bell_rates(mean, k0=0.02, x_dagger=0.1, events=True)
    rows = np.nonzero(ev.any(axis=1))[0]
    assert rows.size > 0
    _, first = o.mftu_events(rates, 1, W)
    assert first[0, 0] == rows[0]
    # no event at all within the cap: censored
    _, first = o.mftu_events(np.zeros_like(rates), 3, 50)
    assert np.all(first == -1)
    m, _ = o.mftu_events(np.zeros_like(rates), 3, 50)
    assert np.isinf(m[0])


def test_mftu_events_geometric_first_passage():
    # Piecewise-constant rates held per window: window v of a trial unfolds
    # some spring with probability p_v = 1 - exp(-K_v S dt) (K_v the summed
    # rate, springs independent), so the first window is distributed as
    # P(v) = prod_{i<v} (1 - p_i) p_v over the repeated rate profile. Its mean
    # and the censored fraction are checked against that law by brute force.
    N, S, dt = 6, 10, 1e-2
    o = ora.Oracle([wl.group(N, 1, dt, stream_id=2)], 7, S, 3)
    dtw = S * dt
    rates = np.array([[0.5, 0.2, 0.1, 0.05, 0.15], [2.0, 0.0, 0.0, 0.0, 0.0], [0.1, 0.1, 0.1, 0.1, 0.1]])
    K = rates.sum(axis=1)
    p = -np.expm1(-K * dtw)
    T, cap = 20000, 400
    m, first = o.mftu_events(rates, T, cap)
    v = first[:, 0]
    surv, pmf = 1.0, np.zeros(cap)
    for i in range(cap):
        pmf[i] = surv * p[i % 3]
        surv *= 1.0 - p[i % 3]
    assert surv < 1e-12 and np.all(v >= 0)
    ev = np.sum((np.arange(cap) + 1) * pmf)
    got = (v + 1).astype(float)
    assert abs(got.mean() - ev) < 4.5 * got.std() / np.sqrt(T)
    assert abs(m[0] - ev * dtw) < 4.5 * dtw * got.std() / np.sqrt(T)
    for i in range(3):                              # the first windows' frequencies
        assert abs(np.mean(v == i) - pmf[i]) < 4.5 * np.sqrt(pmf[i] * (1 - pmf[i]) / T)
    # constant rate: the estimator tends to S dt / p, i.e. 1/K + S dt / 2 for K S dt << 1
    one = rates[2:3]
    m1, f1 = o.mftu_events(one, T, 5000)
    p1 = p[2]
    assert abs(m1[0] - dtw / p1) < 4.5 * dtw * np.sqrt(1 - p1) / p1 / np.sqrt(T)
    # censoring at 5 windows: the survivors are (1 - p)^5 of the trials and the
    # censored mean (total time / events) is still an estimate of S dt / p
    m5, f5 = o.mftu_events(one, T, 5)
    cens = np.mean(f5[:, 0] < 0)
    assert abs(cens - (1 - p1) ** 5) < 4.5 * np.sqrt(cens * (1 - cens) / T)
    assert abs(m5[0] / (dtw / p1) - 1.0) < 0.1


def test_conformation_hand_values():
    # Eq. 5 on a 3-bead example: source on the x axis, replica displaced.
    src = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [2.0, 0.0, 0.0]])
    desc = wl.group(3, 1, 1e-3, noise_scale=0.0)
    o = ora.Oracle([desc], 0, 1, 1)
    o.init_chains([src])
    dbar, rg2, srg2, db = o.conformation(per_bead=True)
    assert np.all(dbar == 0.0) and np.all(db == 0.0)
    # rod of 3 beads, spacing 1: Rg^2 = l^2 (N^2 - 1) / 12 = 2/3, all in x
    assert np.allclose(srg2[0], [2.0 / 3.0, 0.0, 0.0], rtol=1e-15, atol=0)
    assert np.allclose(rg2[0], srg2[0], rtol=1e-15, atol=0)
    # one noise-free step: springs contract toward the middle bead
    o.step(1)
    r = o.positions()[0][0]
    hr, hs = r - r.mean(axis=0), src - src.mean(axis=0)
    dbar, rg2, _, db = o.conformation(per_bead=True)
    assert np.allclose(db.reshape(3, 3), np.abs(hr - hs), rtol=0, atol=1e-15)
    assert np.allclose(dbar[0], np.abs(hr - hs).mean(axis=0), rtol=0, atol=1e-15)
    # x: ends move in by dt * H = 1e-3 each; dbar_x = 2e-3 / 3
    assert np.isclose(dbar[0, 0], 2e-3 / 3.0, rtol=1e-9)


def test_rg2_of_rod_and_translation_invariance():
    N, l = 7, 0.8
    rod = np.zeros((N, 3))
    rod[:, 2] = l * np.arange(N) + 5.0      # along z, off the origin
    o = ora.Oracle([wl.group(N, 2, 1e-3, noise_scale=0.0)], 0, 1, 1)
    o.init_chains([rod])
    _, rg2, srg2 = o.conformation()
    assert np.allclose(srg2[0], [0.0, 0.0, l * l * (N * N - 1) / 12.0], rtol=1e-14, atol=0)
    assert np.allclose(rg2, srg2[0], rtol=1e-14, atol=0)


def test_equilibrium_radius_of_gyration_components():
    # Hookean chain at the EM stationary state: with r = L Q (L: cumulative sum
    # of bonds), the centre-of-mass frame is A = (I - 11^T/N) L and each
    # component of Rg^2 averages tr(A C A^T)/N, C the stationary bond
    # covariance of the discrete map (continuous limit (kT/H)(N^2-1)/(6N)).
    N, H, dt, R = 5, 1.0, 1e-2, 4000
    desc = wl.group(N, R, dt, H=H)
    o = ora.Oracle([desc], 21, 1000, 2)
    o.init_chains([wl.equilibrium_parent(N, H=H, seed=7)])
    o.step(2000)                           # 20 time units, > 10 Rouse times
    _, rg2, _ = o.conformation()
    M, Qn = cf.em_matrices(N, H, 1.0, 1.0, dt, wl.QUIESCENT, 0.0)
    nb = N - 1
    C = cf.stationary_cov(M, Qn)[:nb, :nb]
    L = np.tril(np.ones((N, nb)), -1)
    A = (np.eye(N) - np.ones((N, N)) / N) @ L
    exp = np.trace(A @ C @ A.T) / N
    assert abs(exp / ((N * N - 1) / (6.0 * N) / H) - 1.0) < 0.02
    se = rg2.std(axis=0, ddof=1) / math.sqrt(R)
    assert np.all(np.abs(rg2.mean(axis=0) - exp) < 4.5 * se)
