"""GPU parity of noise map 2 against the oracle's map 2. Under map 2 the beads
of a step form groups of four, and bead 4q + r takes normal r of the Philox
blocks with bead word 3q + c as its component c: three blocks serve four
bead-steps with no carry between steps. The fused path runs it on lanes of 8,
12 or 16 beads. Covered here: every such tile, partial groups and lanes, split
calls, TSF, batches, graph replay, the RSF cycle's dual launch and the plain
path. Tolerances are those of test_gpu_parity: FP32 relative 1e-4 on
per-replica samples over windows of at most 200 steps, FP64 1e-10."""
import numpy as np
import pytest

from gpu_util import announce, rel_err, require_gpu, run_gpu, run_oracle
from paper_2206_05851_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL32 = 1e-4
TOL64 = 1e-10


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def test_map2_tiles_bitwise_equal_and_match_oracle():
    # N = 301: the chain's last group of four holds one bead, and every tile's
    # last lane is partial; M = 8 runs one replica per wavefront, M = 12 and 16
    # pack two and three. Calls of 37, 13 and 150 steps split the windows.
    from paper_2206_05851_amd import ra
    N, R, seed = 301, 12, 23
    g = wl.group(N, R, 5e-5, wl.FENE, 1.0, 200.0, wl.UNIAXIAL, wl.wi_to_rate(5.0, N), stream_id=5)
    parent = wl.equilibrium_parent(N, wl.FENE, 1.0, 200.0, seed=91)
    o = run_oracle([g], [parent], seed, 200, 25, noise_map=2)
    ref = None
    for M in (8, 12, 16):
        announce("noise map 2 N=%d M=%d" % (N, M))
        rep = ra.Replicas([g], seed, sample_every=25, max_windows=8, noise_map=2, tile_policy=1000 + M)
        rep.init_chains([parent])
        for c in (37, 13, 150):
            rep.step(c)
        smp = rep.samples()[0].cpu().numpy()
        bonds = rep.bonds()[0].cpu().numpy()
        rep.sync_status()
        assert rep.tile_info()[0] == [M]
        if ref is None:
            ref = (smp, bonds)
            e = rel_err(smp, o.samples()[0])
            announce("noise map 2 rel err samples %.2e" % e)
            assert e < TOL32
            assert np.max(np.abs(bonds - np.diff(o.positions()[0], axis=1))) < 1e-4
        else:
            assert np.array_equal(smp, ref[0]) and np.array_equal(bonds, ref[1]), M
    announce("noise map 0 differs")
    rep0 = run_gpu([g], [parent], seed, 200, 25)
    assert not np.array_equal(rep0.samples()[0].cpu().numpy(), ref[0])
    rep0.sync_status()


@pytest.mark.parametrize("N,M,R", [(1000, 16, 6), (1024, 16, 6), (512, 8, 6), (257, 12, 1), (257, 8, 3)])
def test_map2_long_chains_match_oracle(N, M, R):
    # the headline's chain length, the longest chain of the family (all 64
    # lanes full), the longest at 8 beads per lane, and the shortest chain
    # the wide-lane family takes (one bead in its last group of four), with a
    # single replica and with three packed into one wavefront
    g = wl.group(N, R, 5e-5, wl.FENE, 1.0, 400.0, wl.UNIAXIAL, wl.wi_to_rate(10.0, N), stream_id=2)
    parent = wl.equilibrium_parent(N, wl.FENE, 1.0, 400.0, seed=N + 1)
    announce("noise map 2 N=%d M=%d R=%d 200 steps" % (N, M, R))
    rep = run_gpu([g], [parent], 4, 200, 100, noise_map=2, tile_policy=1000 + M)
    assert rep.tile_info()[0] == [M]
    mean, std = rep.average_forces()
    smp = rep.samples()[0].cpu().numpy()
    rep.sync_status()
    o = run_oracle([g], [parent], 4, 200, 100, noise_map=2)
    rm, rs = o.average_forces()
    if R == 1:   # one replica: no spread on either side
        assert np.all(std.cpu().numpy() == 0) and np.all(rs == 0)
        rs_err = 0.0
    else:
        rs_err = rel_err(std.cpu().numpy(), rs)
    e = (rel_err(smp, o.samples()[0]), rel_err(mean.cpu().numpy(), rm), rs_err)
    announce("N=%d rel err samples %.2e mean %.2e std %.2e" % ((N,) + e))
    assert max(e) < TOL32


def test_map2_tsf_graph_and_batch():
    # a batch with a short chain (8 beads per lane, packed replicas) beside two
    # long ones, TSF on, two calls; graph replay gives the same bits, and each
    # long group gives the same bits alone
    gs = [wl.group(300, 10, 5e-5, wl.FENE, 1.0, 150.0, wl.SHEAR, 20.0, stream_id=1),
          wl.group(520, 4, 5e-5, wl.HOOKEAN, 1.0, 0.0, wl.PLANAR, 0.02, stream_id=2),
          wl.group(40, 30, 1e-4, wl.FENE, 1.0, 80.0, wl.UNIAXIAL, 0.5, stream_id=3)]
    ps = [wl.equilibrium_parent(g["n_beads"], g["spring"], g["H"], g["b"], seed=40 + i) for i, g in enumerate(gs)]
    o = run_oracle(gs, ps, 31, 150, 30, tsf=True, noise_map=2)
    announce("noise map 2 batch, TSF, eager")
    rep = run_gpu(gs, ps, 31, 0, 30, max_windows=5, tsf=True, noise_map=2)
    for c in (61, 89):
        rep.step(c)
    smp, tsf = rep.samples(tsf=True)
    rep.sync_status()
    assert all(m % 4 == 0 for m in rep.tile_info()[0])
    osmp = o.samples()
    otsf = o.samples(tsf=True)[1]
    for k in range(3):
        assert rel_err(smp[k].cpu().numpy(), osmp[k]) < TOL32, k
        assert rel_err(tsf[k].cpu().numpy(), otsf[k]) < TOL32, k
    announce("noise map 2 batch, graph replay")
    repg = run_gpu(gs, ps, 31, 0, 30, max_windows=5, tsf=True, noise_map=2, use_graph=True)
    for c in (61, 89):
        repg.step(c)
    smpg, tsfg = repg.samples(tsf=True)
    repg.sync_status()
    for k in range(3):
        assert np.array_equal(smpg[k].cpu().numpy(), smp[k].cpu().numpy())
        assert np.array_equal(tsfg[k].cpu().numpy(), tsf[k].cpu().numpy())
    for k in (0, 1):
        announce("noise map 2 group %d alone" % k)
        alone = run_gpu([gs[k]], [ps[k]], 31, 0, 30, max_windows=5, tsf=True, noise_map=2)
        for c in (61, 89):   # the same calls: TSF register sums are folded at call ends
            alone.step(c)
        a, at = alone.samples(tsf=True)
        alone.sync_status()
        assert np.array_equal(a[0].cpu().numpy(), smp[k].cpu().numpy())
        assert np.array_equal(at[0].cpu().numpy(), tsf[k].cpu().numpy())


def test_map2_rsf_cycle_matches_oracle():
    # the RSF cycle's dual launch (replicas of window w beside the parent's
    # next segment) on the wide-lane kernels under map 2
    import torch
    from oracle import ora
    from paper_2206_05851_amd import ra
    g = wl.group(300, 16, 5e-5, wl.FENE, 1.0, 150.0, wl.SHEAR, wl.wi_to_rate(20.0, 300), stream_id=4)
    parent = wl.equilibrium_parent(300, wl.FENE, 1.0, 150.0, seed=12)
    S, P, W, seed = 40, 30, 4, 19
    announce("noise map 2 rsf cycle N=300")
    gp = ra.Replicas([dict(g, n_replicas=1)], seed, sample_every=P, max_windows=W, tsf=True, noise_tag=1,
                     noise_map=2)
    gp.init_chains([parent])
    gr = ra.Replicas([g], seed, sample_every=S, max_windows=W, noise_map=2)
    gr.rsf_cycle(gp, W, P)
    isf, _, tsf, _ = gp.average_forces(tsf=True)
    rsf, rstd = gr.average_forces()
    torch.cuda.synchronize()
    gp.sync_status()
    gr.sync_status()
    op = ora.Oracle([dict(g, n_replicas=1)], seed, P, W, tsf=True, noise_map=2)
    op.set_tag(ora.TAG_PARENT)
    op.init_chains([parent])
    orr = ora.Oracle([g], seed, S, W, noise_map=2)
    orr.rsf_cycle(op, W, P)
    oisf, _, otsf, _ = op.average_forces(tsf=True)
    orsf, orstd = orr.average_forces()
    e = [rel_err(isf.cpu().numpy(), oisf, 1e-3), rel_err(tsf.cpu().numpy(), otsf, 1e-3),
         rel_err(rsf.cpu().numpy(), orsf, 1e-3), rel_err(rstd.cpu().numpy(), orstd, 1e-3)]
    announce("isf %.2e tsf %.2e rsf %.2e std %.2e" % tuple(e))
    assert max(e) < TOL32


@pytest.mark.parametrize("precision,tol", [(32, TOL32), (64, TOL64)])
def test_map2_plain_path_matches_oracle(precision, tol):
    # the plain path draws a bead's three blocks in its own thread; any chain
    # length (the 4-bead groups do not depend on a tile)
    for N in (37, 300):
        g = wl.group(N, 6, 5e-5, wl.FENE, 1.0, 150.0, wl.UNIAXIAL, wl.wi_to_rate(5.0, N), stream_id=7)
        parent = wl.equilibrium_parent(N, wl.FENE, 1.0, 150.0, seed=N)
        announce("noise map 2 plain path N=%d precision=%d" % (N, precision))
        rep = run_gpu([g], [parent], 5, 100, 50, precision=precision, plain=True, noise_map=2)
        smp = rep.samples()[0].cpu().numpy()
        rep.sync_status()
        o = run_oracle([g], [parent], 5, 100, 50, noise_map=2)
        assert rel_err(smp, o.samples()[0]) < tol


def test_map2_autotuner_picks_whole_groups(tmp_path, monkeypatch):
    # tile_policy 1 under map 2 times only 8, 12 and 16 beads per lane (whole
    # groups of four), the short chain too, on the batch's wide-lane kernels;
    # whatever it picks, the results are the cost model's bits
    import torch
    monkeypatch.setenv("RA_AUTOTUNE_CACHE", str(tmp_path / "t.jsonl"))
    gs = [wl.group(300, 8, 5e-5, wl.FENE, 1.0, 150.0, wl.SHEAR, 20.0, stream_id=1),
          wl.group(700, 3, 5e-5, wl.FENE, 1.0, 300.0, wl.UNIAXIAL, wl.wi_to_rate(5.0, 700), stream_id=2),
          wl.group(40, 20, 1e-4, wl.HOOKEAN, 1.0, 0.0, wl.PLANAR, 0.3, stream_id=3)]
    ps = [wl.equilibrium_parent(g["n_beads"], g["spring"], g["H"], g["b"], seed=60 + i) for i, g in enumerate(gs)]
    announce("noise map 2 autotuner")
    tuned = run_gpu(gs, ps, 8, 100, 50, tile_policy=1, noise_map=2)
    cost = run_gpu(gs, ps, 8, 100, 50, noise_map=2)
    assert all(m in (8, 12, 16) for m in tuned.tile_info()[0])
    for x, y in zip(tuned.samples(), cost.samples()):
        assert bool(torch.equal(x, y))
    tuned.sync_status()
    cost.sync_status()
    lines = (tmp_path / "t.jsonl").read_text().splitlines()
    assert len(lines) == 9                        # 3 lengths x 3 workgroup sizes
    assert all('"noise_map": 2' in ln and '"family": 16' in ln for ln in lines)


@pytest.mark.parametrize("M,K", [(16, 50), (12, 7), (8, -1)])
def test_map2_adjoint_matches_oracle_tangents(M, K):
    # the adjoint's segment recompute under map 2 on every wide tile; K = 7
    # starts segments mid-window, K = -1 keeps every state (no recompute)
    import torch
    N, R, steps, S = 300, 24, 200, 50
    g = wl.group(N, R, 5e-5, wl.FENE, 1.3, 120.0, wl.UNIAXIAL, wl.wi_to_rate(3.0, N), stream_id=3)
    parent = wl.equilibrium_parent(N, wl.FENE, 1.3, 120.0, seed=33)
    rng = np.random.default_rng(M)
    W = steps // S
    gm = rng.normal(size=(W, N - 1))
    gr = rng.normal(size=(W, N - 1)) * 1e5
    announce("noise map 2 adjoint N=%d M=%d K=%d" % (N, M, K))
    rep = run_gpu([g], [parent], 11, steps, S, checkpoint_every=K, max_steps=steps, noise_map=2,
                  tile_policy=1000 + M)
    assert rep.tile_info()[0] == [M]
    mean, _ = rep.average_forces()
    g_gpu = rep.backward(mean, torch.from_numpy(gm).cuda(), torch.from_numpy(gr).cuda(), 1e-6, 0.1).cpu().numpy()
    rep.sync_status()
    o = run_oracle([g], [parent], 11, steps, S, tangents=True, noise_map=2)
    g_ref = o.backward(gm, gr, 1e-6, 0.1)
    scale = np.maximum(np.abs(g_ref), 1e-3 * np.max(np.abs(g_ref)))
    err = np.max(np.abs(g_gpu - g_ref) / scale)
    announce("noise map 2 adjoint max rel err %.2e" % err)
    assert err < 1e-4, (g_gpu, g_ref)
