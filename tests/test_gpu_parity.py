"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs. Tolerance for FP32 state: relative 1e-4 on per-replica
samples and on the replica-averaged profile over windows of at most 200 steps;
FP64 state: relative 1e-10. Integer work (Philox words, events) is bit-exact."""
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


def test_noise_words_bit_exact_and_normals():
    import torch
    from oracle import ora
    from paper_2206_05851_amd import ra
    rng = np.random.default_rng(0)
    n = 20000
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:8] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 2, 3, 4], [99, 7, 1023, 1], [0, 1, 0, 0],
               [5, 0, 0, 2 << 24], [12345, 49, 1023, 0], [0, 0, 0xFFFFFFFF, 0]]
    seed = 0x0123456789ABCDEF
    announce("debug_noise n=%d" % n)
    words, n32, n64 = ra.debug_noise(torch.from_numpy(ctr.view(np.int32)).cuda(), seed)
    torch.cuda.synchronize()
    words = words.cpu().numpy().view(np.uint32)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    ref_w = np.array([ora.philox(c, key) for c in ctr], dtype=np.uint32)
    assert np.array_equal(words, ref_w)
    ref_n = np.array([ora.normals(w) for w in ref_w])
    e32 = np.max(np.abs(n32.cpu().numpy() - ref_n))
    e64 = np.max(np.abs(n64.cpu().numpy() - ref_n))
    announce("normals max abs err fp32 %.3e fp64 %.3e" % (e32, e64))
    assert e32 < 5e-6
    assert e64 < 1e-13


def test_fp64_rouse_n10_full_parity():
    groups, parents, run = wl.rouse_fp64_small(n_replicas=64)
    announce("C1 shape FP64: N=10 R=64 5000 steps")
    rep = run_gpu(groups, parents, run["seed"], run["steps"], run["sample_every"], precision=64)
    mean, std = rep.average_forces()
    smp = rep.samples()[0].cpu().numpy()
    rep.sync_status()
    o = run_oracle(groups, parents, run["seed"], run["steps"], run["sample_every"])
    rm, rs = o.average_forces()
    e = (rel_err(smp, o.samples()[0]), rel_err(mean.cpu().numpy(), rm), rel_err(std.cpu().numpy(), rs))
    announce("fp64 rel err samples %.2e mean %.2e std %.2e" % e)
    assert max(e) < TOL64
    assert mean.shape == (50, 9)


def test_fp32_fene50_parity_200_steps():
    groups, parents, run = wl.fene50(n_replicas=1024, steps=200)
    announce("C2 shape: FENE N=50 R=1024 200 steps")
    rep = run_gpu(groups, parents, run["seed"], 200, 100)
    mean, std = rep.average_forces()
    smp = rep.samples()[0].cpu().numpy()
    rep.sync_status()
    o = run_oracle(groups, parents, run["seed"], 200, 100)
    rm, rs = o.average_forces()
    e = (rel_err(smp, o.samples()[0]), rel_err(mean.cpu().numpy(), rm), rel_err(std.cpu().numpy(), rs))
    announce("fp32 rel err samples %.2e mean %.2e std %.2e" % e)
    assert max(e) < TOL32
    assert rep.tile_info() == ([1], [1])


@pytest.mark.parametrize("precision,tol", [(32, TOL32), (64, TOL64)])
def test_degenerate_sizes_match_oracle(precision, tol):
    # one replica (std defined as 0), the two-bead dumbbell (a single spring),
    # a one-replica chain filling a whole wavefront, zero-step calls, and calls
    # that end inside a window; on the fused path and on the plain path
    from paper_2206_05851_amd import ra
    cases = [wl.group(2, 1, 1e-3, wl.FENE, 1.0, 10.0, wl.UNIAXIAL, 0.5, stream_id=2),
             wl.group(2, 7, 1e-3, wl.HOOKEAN, 1.0, 0.0, wl.SHEAR, 2.0, stream_id=3),
             wl.group(64, 1, 1e-4, wl.FENE, 1.0, 60.0, wl.PLANAR, 0.3, stream_id=4)]
    for i, g in enumerate(cases):
        parent = wl.equilibrium_parent(g["n_beads"], g["spring"], g["H"], g["b"], seed=20 + i)
        o = run_oracle([g], [parent], 13, 100, 20)
        om, osd = o.average_forces()
        for plain in (False, True):
            announce("degenerate case %d N=%d R=%d precision=%d plain=%d"
                     % (i, g["n_beads"], g["n_replicas"], precision, plain))
            rep = ra.Replicas([g], 13, sample_every=20, max_windows=5, precision=precision, plain=plain)
            rep.init_chains([parent])
            b0 = rep.bonds()[0].cpu().numpy()
            rep.step(0)
            assert np.array_equal(rep.bonds()[0].cpu().numpy(), b0)
            for n in (0, 55, 0, 45):
                rep.step(n)
            mean, std = rep.average_forces()
            smp = rep.samples()[0].cpu().numpy()
            rep.sync_status()
            assert smp.shape == (5, g["n_replicas"], g["n_beads"] - 1)
            assert rel_err(smp, o.samples()[0]) < tol
            assert rel_err(mean.cpu().numpy(), om) < tol
            if g["n_replicas"] == 1:
                assert np.all(std.cpu().numpy() == 0.0) and np.all(osd == 0.0)
            else:
                assert rel_err(std.cpu().numpy(), osd) < tol


@pytest.mark.parametrize("precision,tol", [(32, TOL32), (64, TOL64)])
def test_plain_path_parity(precision, tol):
    N = 30
    g = wl.group(N, 96, 1e-4, wl.FENE, 1.0, 60.0, wl.SHEAR, 40.0)
    parent = wl.equilibrium_parent(N, wl.FENE, 1.0, 60.0, seed=7)
    announce("plain path precision %d" % precision)
    rep = run_gpu([g], [parent], 11, 200, 50, plain=True, precision=precision)
    mean, std = rep.average_forces()
    smp = rep.samples()[0].cpu().numpy()
    bonds = rep.bonds()[0].cpu().numpy()
    rep.sync_status()
    o = run_oracle([g], [parent], 11, 200, 50)
    rm, rs = o.average_forces()
    ob = np.diff(o.positions()[0], axis=1)
    e = (rel_err(smp, o.samples()[0]), rel_err(mean.cpu().numpy(), rm), rel_err(std.cpu().numpy(), rs),
         rel_err(bonds, ob, floor=1.0))
    announce("plain rel err samples %.2e mean %.2e std %.2e bonds %.2e" % e)
    assert max(e) < tol


def test_tile_choice_is_bitwise_invariant():
    N, R = 37, 50
    g = wl.group(N, R, 1e-4, wl.FENE, 1.0, 80.0, wl.SHEAR, 20.0)
    parent = wl.equilibrium_parent(N, wl.FENE, 1.0, 80.0, seed=9)
    ref = None
    for M in (1, 2, 3, 4):
        announce("tile M=%s" % M)
        rep = run_gpu([g], [parent], 5, 150, 50, tile_policy=1000 + M)
        assert rep.kernel_family() == 4
        assert rep.tile_info()[0] == [M]
        smp = rep.samples()[0].cpu().numpy()
        rep.sync_status()
        if ref is None:
            ref = smp
            o = run_oracle([g], [parent], 5, 150, 50)
            assert rel_err(smp, o.samples()[0]) < TOL32
        else:
            assert np.array_equal(smp, ref), M


@pytest.mark.parametrize("precision,tol", [(32, TOL32), (64, TOL64)])
def test_noise_map_one_parity_tiles_and_plain(precision, tol):
    # noise map 1 against the oracle's map 1. S = 25 puts window ends off the
    # 4-step grid and the step calls (37, 13, 150) start off it, so the fused
    # loop's unaligned heads, carry rebuilds and tails all run; every tile M =
    # 1..4 must give the same bits, and the plain path the oracle's values
    from paper_2206_05851_amd import ra
    N, R, seed = 50, 40, 17
    g = wl.group(N, R, 1e-4, wl.FENE, 1.0, 60.0, wl.UNIAXIAL, 0.5, stream_id=6)
    parent = wl.equilibrium_parent(N, wl.FENE, 1.0, 60.0, seed=61)
    o = run_oracle([g], [parent], seed, 200, 25, noise_map=1)
    ref = None
    for M in (1, 2, 3, 4):
        announce("noise map 1 precision=%d M=%d" % (precision, M))
        rep = ra.Replicas([g], seed, precision=precision, sample_every=25, max_windows=8, noise_map=1,
                          tile_policy=1000 + M)
        rep.init_chains([parent])
        for c in (37, 13, 150):
            rep.step(c)
        smp = rep.samples()[0].cpu().numpy()
        rep.sync_status()
        assert rep.tile_info()[0] == [M]
        if ref is None:
            ref = smp
            assert rel_err(smp, o.samples()[0]) < tol
        else:
            assert np.array_equal(smp, ref), M
    announce("noise map 0 differs; plain path under map 1")
    rep0 = run_gpu([g], [parent], seed, 200, 25, precision=precision)
    assert not np.array_equal(rep0.samples()[0].cpu().numpy(), ref)
    rep0.sync_status()
    repp = run_gpu([g], [parent], seed, 200, 25, precision=precision, plain=True, noise_map=1)
    assert rel_err(repp.samples()[0].cpu().numpy(), o.samples()[0]) < tol
    repp.sync_status()


@pytest.mark.parametrize("M", [1, 3])
def test_noise_map_one_tiny_calls_equal_one_call(M):
    # calls of 1-3 steps start every launch inside a group of four, so each
    # builds its carry from the blocks of the group's earlier steps; windows of
    # 5 steps end off the grid too. Bit-equal to one call, and to the oracle.
    from paper_2206_05851_amd import ra
    N = 40
    g = wl.group(N, 24, 1e-4, wl.FENE, 1.0, 60.0, wl.PLANAR, 0.7, stream_id=8)
    parent = wl.equilibrium_parent(N, wl.FENE, 1.0, 60.0, seed=81)
    chunks = [1, 2, 3, 1, 1, 3, 2, 2, 1, 3, 1, 2, 3, 3, 2, 1, 1, 2, 3, 3]   # 40 steps
    out = []
    for calls in (chunks, [sum(chunks)]):
        announce("noise map 1 M=%d, %d calls" % (M, len(calls)))
        rep = ra.Replicas([g], 37, sample_every=5, max_windows=8, noise_map=1, tile_policy=1000 + M)
        rep.init_chains([parent])
        for c in calls:
            rep.step(c)
        out.append((rep.samples()[0].cpu().numpy(), rep.bonds()[0].cpu().numpy()))
        rep.sync_status()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    o = run_oracle([g], [parent], 37, 40, 5, noise_map=1)
    assert rel_err(out[0][0], o.samples()[0]) < TOL32


def test_noise_map_one_tsf_graph_and_batch():
    # TSF (per-step tensions) and graph replay under map 1, in a batch of
    # uneven chains (M = 1 and packed replicas), each group against the oracle
    gs = [wl.group(50, 30, 1e-4, wl.FENE, 1.0, 80.0, wl.SHEAR, 20.0, stream_id=1),
          wl.group(20, 45, 1e-4, wl.HOOKEAN, 1.0, 0.0, wl.PLANAR, 0.4, stream_id=2),
          wl.group(200, 6, 1e-4, wl.FENE, 1.0, 120.0, wl.UNIAXIAL, 0.02, stream_id=3)]
    ps = [wl.equilibrium_parent(g["n_beads"], g["spring"], g["H"], g["b"], seed=70 + i) for i, g in enumerate(gs)]
    o = run_oracle(gs, ps, 29, 150, 30, tsf=True, noise_map=1)
    announce("noise map 1 batch, TSF, eager")
    rep = run_gpu(gs, ps, 29, 0, 30, max_windows=5, tsf=True, noise_map=1)
    for c in (61, 89):
        rep.step(c)
    smp, tsf = rep.samples(tsf=True)
    rep.sync_status()
    osmp = o.samples()
    otsf = o.samples(tsf=True)[1]
    for k in range(3):
        assert rel_err(smp[k].cpu().numpy(), osmp[k]) < TOL32
        assert rel_err(tsf[k].cpu().numpy(), otsf[k]) < TOL32
    announce("noise map 1 batch, graph replay")
    repg = run_gpu(gs, ps, 29, 0, 30, max_windows=5, tsf=True, noise_map=1, use_graph=True)
    for c in (61, 89):
        repg.step(c)
    smpg, tsfg = repg.samples(tsf=True)
    repg.sync_status()
    for k in range(3):
        assert np.array_equal(smpg[k].cpu().numpy(), smp[k].cpu().numpy())
        assert np.array_equal(tsfg[k].cpu().numpy(), tsf[k].cpu().numpy())


def test_batch_is_bitwise_invariant():
    gs = [wl.group(20, 40, 1e-4, wl.FENE, 1.0, 50.0, wl.PLANAR, 0.5, stream_id=4),
          wl.group(63, 17, 2e-4, wl.HOOKEAN, 2.0, 0.0, wl.UNIAXIAL, 0.01, stream_id=9),
          wl.group(150, 9, 1e-4, wl.FENE, 1.0, 150.0, wl.SHEAR, 5.0, stream_id=1)]
    ps = [wl.equilibrium_parent(g["n_beads"], g["spring"], g["H"], g["b"], seed=i) for i, g in enumerate(gs)]
    announce("batch of 3 vs alone")
    rep = run_gpu(gs, ps, 21, 100, 25)
    both = [s.cpu().numpy() for s in rep.samples()]
    rep.sync_status()
    for i in range(3):
        alone = run_gpu([gs[i]], [ps[i]], 21, 100, 25)
        a = alone.samples()[0].cpu().numpy()
        alone.sync_status()
        assert np.array_equal(both[i], a), i
    o = run_oracle(gs, ps, 21, 100, 25)
    for i, s in enumerate(o.samples()):
        assert rel_err(both[i], s) < TOL32, i


def test_graph_replay_matches_eager_bitwise():
    N = 50
    g = wl.group(N, 128, 1e-4, wl.FENE, 1.0, 100.0, wl.UNIAXIAL, 0.05)
    parent = wl.equilibrium_parent(N, wl.FENE, 1.0, 100.0, seed=3)
    announce("graph replay")
    eager = run_gpu([g], [parent], 8, 0, 50, max_windows=8)
    graph = run_gpu([g], [parent], 8, 0, 50, max_windows=8, use_graph=True)
    for _ in range(4):
        eager.step(100)
        graph.step(100)
    a = eager.samples()[0].cpu().numpy()
    b = graph.samples()[0].cpu().numpy()
    eager.sync_status()
    graph.sync_status()
    assert np.array_equal(a, b)
    assert a.shape[0] == 8


def test_long_chain_parity():
    N = 1000
    g = wl.group(N, 12, 5e-5, wl.FENE, 1.0, 400.0, wl.UNIAXIAL, wl.wi_to_rate(10.0, N))
    parent = wl.equilibrium_parent(N, wl.FENE, 1.0, 400.0, seed=103)
    announce("N=1000 R=12 200 steps")
    rep = run_gpu([g], [parent], 4, 200, 100)
    assert rep.tile_info()[0] == [16]
    mean, std = rep.average_forces()
    smp = rep.samples()[0].cpu().numpy()
    rep.sync_status()
    o = run_oracle([g], [parent], 4, 200, 100)
    rm, rs = o.average_forces()
    e = (rel_err(smp, o.samples()[0]), rel_err(mean.cpu().numpy(), rm), rel_err(std.cpu().numpy(), rs))
    announce("N=1000 rel err samples %.2e mean %.2e std %.2e" % e)
    assert max(e) < TOL32


@pytest.mark.parametrize("N,M", [(256, 4), (1024, 16)])
def test_largest_chain_of_each_family(N, M):
    # the longest chain each one-wave family holds: every one of the 64 lanes
    # carries M beads, the last lane's last bead included
    g = wl.group(N, 5, 5e-5, wl.FENE, 1.0, 400.0, wl.PLANAR, wl.wi_to_rate(5.0, N))
    parent = wl.equilibrium_parent(N, wl.FENE, 1.0, 400.0, seed=N)
    announce("largest chain N=%d" % N)
    rep = run_gpu([g], [parent], 8, 200, 100, tile_policy=1000 + M)
    assert rep.tile_info() == ([M], [1])
    smp = rep.samples()[0].cpu().numpy()
    bonds = rep.bonds()[0].cpu().numpy()
    rep.sync_status()
    o = run_oracle([g], [parent], 8, 200, 100)
    e = (rel_err(smp, o.samples()[0]), np.max(np.abs(bonds - np.diff(o.positions()[0], axis=1))))
    announce("N=%d rel err samples %.2e bonds abs %.2e" % ((N,) + e))
    assert e[0] < TOL32 and e[1] < 1e-4


def test_mixed_batch_parity():
    groups, parents, run = wl.batched512(n_groups=512, steps=200)
    pick = [0, 1, 17, 255, 256, 300, 511]
    gs = [groups[i] for i in pick]
    for g in gs:
        g["n_replicas"] = min(g["n_replicas"], 32)
    ps = [parents[i] for i in pick]
    announce("mixed batch of %d groups, 200 steps" % len(gs))
    rep = run_gpu(gs, ps, run["seed"], 200, 100)
    mean, std = rep.average_forces()
    smp = [s.cpu().numpy() for s in rep.samples()]
    rep.sync_status()
    o = run_oracle(gs, ps, run["seed"], 200, 100)
    rm, rs = o.average_forces()
    for i, s in enumerate(o.samples()):
        assert rel_err(smp[i], s) < TOL32, i
    assert rel_err(mean.cpu().numpy(), rm) < TOL32
    assert rel_err(std.cpu().numpy(), rs) < TOL32


def test_tsf_parity():
    N = 40
    g = wl.group(N, 32, 1e-4, wl.FENE, 1.0, 100.0, wl.UNIAXIAL, 0.5)
    parent = wl.equilibrium_parent(N, wl.FENE, 1.0, 100.0, seed=5)
    announce("TSF")
    for plain in (False, True):
        rep = run_gpu([g], [parent], 6, 200, 50, tsf=True, plain=plain)
        m, s, tm, ts = rep.average_forces(tsf=True)
        smp, tsmp = rep.samples(tsf=True)
        rep.sync_status()
        o = run_oracle([g], [parent], 6, 200, 50, tsf=True)
        rm, rs, rtm, rts = o.average_forces(tsf=True)
        osm, otsm = o.samples(tsf=True)
        assert rel_err(tsmp[0].cpu().numpy(), otsm[0]) < TOL32
        assert rel_err(tm.cpu().numpy(), rtm) < TOL32
        assert rel_err(ts.cpu().numpy(), rts) < TOL32
        assert rel_err(m.cpu().numpy(), rm) < TOL32


def test_tsf_window_straddles_calls():
    N = 25
    g = wl.group(N, 16, 1e-4, wl.FENE, 1.0, 100.0, wl.SHEAR, 3.0)
    parent = wl.equilibrium_parent(N, wl.FENE, 1.0, 100.0, seed=2)
    rep = run_gpu([g], [parent], 3, 0, 40, max_windows=5, tsf=True)
    for n in (13, 27, 60, 100):
        rep.step(n)
    smp, tsmp = rep.samples(tsf=True)
    rep.sync_status()
    o = run_oracle([g], [parent], 3, 200, 40, tsf=True)
    osm, otsm = o.samples(tsf=True)
    assert rel_err(tsmp[0].cpu().numpy(), otsm[0]) < TOL32
    assert rel_err(smp[0].cpu().numpy(), osm[0]) < TOL32


def test_bell_rates_and_events_parity():
    import torch
    groups, parents, run = wl.fene50(n_replicas=64, steps=300)
    groups = groups + [wl.group(12, 8, 1e-4, wl.HOOKEAN, 1.0, 0.0, wl.PLANAR, 0.2, kT=1.5, stream_id=5)]
    parents = parents + [wl.equilibrium_parent(12, seed=1)]
    o = run_oracle(groups, parents, run["seed"], 300, 100)
    rm, _ = o.average_forces()
    rep = run_gpu(groups, parents, run["seed"], 300, 100)
    announce("Bell rates on the oracle's profile")
    for k0, xd in ((1e-6, 0.1), (0.3, 2.0)):
        mean = torch.from_numpy(rm).cuda()
        rates, rsum, ev = rep.bell_rates(mean, k0, xd, events=True)
        r_rates, r_rsum, r_ev = o.bell_rates(rm, k0, xd, events=True)
        assert rel_err(rates.cpu().numpy(), r_rates) < 1e-13
        assert rel_err(rsum.cpu().numpy(), r_rsum) < 1e-13
        assert np.array_equal(ev.cpu().numpy(), r_ev)
    rep.sync_status()


def test_fene_guard_counts_and_fp64_band():
    N = 6
    Q0 = 10.0
    parent = np.zeros((N, 3))
    steps = [0.5, np.sqrt(0.9995) * Q0, 1.0, np.sqrt(0.95) * Q0, 0.7]
    parent[1:, 0] = np.cumsum(steps)
    g = wl.group(N, 64, 1e-4, wl.FENE, 1.0, 100.0, wl.UNIAXIAL, 0.1)
    announce("FENE guard")
    rep = run_gpu([g], [parent], 13, 100, 50)
    smp = rep.samples()[0].cpu().numpy()
    counts = rep.guard_counts()
    rep.sync_status()
    o = run_oracle([g], [parent], 13, 100, 50)
    assert counts[0] == o.clamps(0) and counts[0] >= 64
    assert rel_err(smp, o.samples()[0]) < TOL32


def test_invalid_parent_detected_on_device():
    from paper_2206_05851_amd import ra
    N = 4
    parent = np.zeros((N, 3))
    parent[1:, 0] = [1.0, 12.0, 13.0]            # bond of 11 > Q0 = 10
    g = wl.group(N, 8, 1e-4, wl.FENE, 1.0, 100.0)
    rep = run_gpu([g], [parent], 1, 50, 50)
    with pytest.raises(ra.RAError) as ei:
        rep.sync_status()
    assert ei.value.code == ra.RA_EINVAL
    # a valid parent on the same context clears the flag
    parent[1:, 0] = [1.0, 2.0, 3.0]
    rep.init_chains([parent])
    rep.step(50)
    rep.sync_status()


def test_errors_on_capacity_and_order():
    from paper_2206_05851_amd import ra
    g = wl.group(5, 4, 1e-3)
    rep = ra.Replicas([g], 0, sample_every=10, max_windows=2)
    with pytest.raises(ra.RAError) as ei:
        rep.step(5)
    assert ei.value.code == ra.RA_ESTATE
    rep.init_chains([wl.equilibrium_parent(5)])
    rep.step(20)
    with pytest.raises(ra.RAError) as ei:
        rep.step(10)
    assert ei.value.code == ra.RA_EINVAL
    with pytest.raises(ra.RAError):
        rep.backward(None, None)
    # the binding checks shapes and dtypes before a pointer reaches the C ABI
    import torch
    mean, _ = rep.average_forces()
    for bad in (mean[:, :-1].contiguous(), mean.float(), mean[:1].reshape(-1)):
        with pytest.raises(ValueError):
            rep.bell_rates(bad, 1e-6, 0.1)
    with pytest.raises(ValueError):
        rep.average_forces(out=(mean[:1].clone(), mean.clone()))
    with pytest.raises(ValueError):
        rep.init_chains(torch.zeros(3 * 5 - 1, dtype=torch.float64, device=mean.device))
    with pytest.raises(ValueError):
        rep.mftu(torch.zeros(2, 3, dtype=torch.float64, device=mean.device))
    rep.sync_status()


def test_autotuner_tiles_bit_equal_and_cache_round_trip(tmp_path, monkeypatch):
    # tile_policy 1 times the legal tiles (and workgroup sizes) per chain
    # length; whatever it picks, the results are the cost model's bits. Its
    # results persist in the RA_AUTOTUNE_CACHE file: a copy of that file gives
    # the same tiles without timing (nothing is appended), and an entry written
    # by hand is obeyed.
    import shutil
    from paper_2206_05851_amd import ra
    gs = [wl.group(20, 40, 1e-4, wl.FENE, 1.0, 60.0, wl.SHEAR, 20.0, stream_id=1),
          wl.group(50, 30, 1e-4, wl.FENE, 1.0, 100.0, wl.UNIAXIAL, 0.3, stream_id=2),
          wl.group(130, 20, 1e-4, wl.HOOKEAN, 1.0, 0.0, wl.PLANAR, 0.2, stream_id=3)]
    ps = [wl.equilibrium_parent(20, wl.FENE, 1.0, 60.0, seed=1), wl.equilibrium_parent(50, wl.FENE, 1.0, 100.0, seed=2),
          wl.equilibrium_parent(130, seed=3)]
    a = tmp_path / "a.jsonl"
    monkeypatch.setenv("RA_AUTOTUNE_CACHE", str(a))
    announce("autotuner: tuning 3 chain lengths")
    tuned = run_gpu(gs, ps, 5, 150, 50, tile_policy=1)
    cost = run_gpu(gs, ps, 5, 150, 50, tile_policy=0)
    for x, y in zip(tuned.samples(), cost.samples()):
        assert torch_equal(x, y)
    tiles = tuned.tile_info()
    tuned.sync_status()
    lines = a.read_text().splitlines()
    assert len(lines) == 9                        # 3 lengths x 3 workgroup sizes
    b = tmp_path / "b.jsonl"
    shutil.copy(a, b)
    monkeypatch.setenv("RA_AUTOTUNE_CACHE", str(b))
    again = ra.Replicas(gs, 5, sample_every=50, max_windows=3, tile_policy=1)
    assert again.tile_info() == tiles
    assert b.read_text() == a.read_text()
    again.close()
    c = tmp_path / "c.jsonl"
    c.write_text("".join('{"N": 50, "spring": 1, "precision": 32, "family": 4, "wpb": %d, "noise_map": 0, '
                         '"M": 4, "ms_per_replica": 1e-9}\n' % w for w in (1, 2, 4)))
    monkeypatch.setenv("RA_AUTOTUNE_CACHE", str(c))
    forced = ra.Replicas(gs, 5, sample_every=50, max_windows=3, tile_policy=1)
    assert forced.tile_info()[0][1] == 4
    forced.close()


def torch_equal(x, y):
    import torch
    return bool(torch.equal(x, y))
