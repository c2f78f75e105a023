"""GPU hydrodynamic-interaction kernel (Eqs. 1-3: RPY tensor, Cholesky-factor
correlated noise, D F / kT drift) against the oracle on the same seeds and
counters."""
import numpy as np
import pytest

from gpu_util import announce, rel_err, require_gpu, run_gpu, run_oracle
from paper_2206_05851_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _lds_limit():
    import torch
    return torch.cuda.get_device_properties(0).shared_memory_per_block


def _fits(N, precision):
    # packed tensor (at least the drift partials 4 x 16 NB), positions, forces,
    # normals, drift, displacement, and the double-buffered elimination panel
    n = 3 * N
    nb = next(b for b in (2, 4, 6, 8, 10, 12) if 16 * b >= n)
    width = 2 if (precision == 64 and nb >= 10) else 4
    elems = max(n * (n + 1) // 2, 64 * nb) + 16 * 64 + 2 * 16 * nb * width
    return elems * (8 if precision == 64 else 4) <= _lds_limit()


CASES = [
    ("Hookean N=8 quiescent", lambda: wl.group(8, 5, 1e-3, wl.HOOKEAN, 1.0, hi_radius=0.35), 1e-3),
    ("paper model N=20 shear", lambda: wl.group(20, 4, 1e-5, wl.HARMONIC, 400.0, 0.0, wl.SHEAR, 30.0,
                                                rest_length=2.0, lj_eps=1.0, lj_rmin=2.0, hi_radius=1.0), 1e-5),
    ("FENE N=50 uniaxial", lambda: wl.group(50, 3, 1e-4, wl.FENE, 1.0, 100.0, wl.UNIAXIAL, 0.05, hi_radius=0.4),
     1e-4),
    ("Hookean N=64 planar, largest tile", lambda: wl.group(64, 2, 1e-3, wl.HOOKEAN, 1.0, 0.0, wl.PLANAR, 0.2,
                                                           hi_radius=0.3), 1e-3),
]


def _parent(g, seed):
    if g["spring"] == wl.HARMONIC:
        return wl.collapsed_parent(g["n_beads"], seed=seed)
    return wl.equilibrium_parent(g["n_beads"], g["spring"], g["H"], g["b"], seed=seed)


@pytest.mark.parametrize("name,mk,dt", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", [32, 64])
def test_hi_kernel_matches_oracle(name, mk, dt, precision):
    g = mk()
    if not _fits(g["n_beads"], precision):
        pytest.skip("N=%d at precision %d needs more LDS per workgroup than the device's %d B"
                    % (g["n_beads"], precision, _lds_limit()))
    p = _parent(g, 4)
    steps, S = 200, 50
    announce("hi %s precision %d (LDS limit %d B)" % (name, precision, _lds_limit()))
    rep = run_gpu([g], [p], 11, steps, S, precision=precision, tsf=True)
    assert rep.kernel_family() == 3
    smp, tsf = rep.samples(tsf=True)
    bonds = rep.bonds()[0].cpu().numpy()
    rep.sync_status()
    o = run_oracle([g], [p], 11, steps, S, tsf=True)
    osmp, otsf = o.samples(tsf=True)
    obonds = np.diff(o.positions()[0], axis=1)
    fl = float(np.sqrt(g["H"] * g["kT"]))
    tol = 1e-4 if precision == 32 else 1e-9
    e = [rel_err(smp[0].cpu().numpy(), osmp[0], fl), rel_err(tsf[0].cpu().numpy(), otsf[0], fl),
         np.max(np.abs(bonds - obonds))]
    announce("samples %.2e tsf %.2e bonds abs %.2e" % tuple(e))
    assert e[0] < tol and e[1] < tol and e[2] < tol


def test_hi_differs_from_free_draining_and_batches_bitwise():
    g = wl.group(12, 6, 1e-3, wl.HOOKEAN, 1.0, hi_radius=0.45, stream_id=2)
    g2 = wl.group(7, 3, 1e-3, wl.HOOKEAN, 1.0, hi_radius=0.3, stream_id=5)
    p, p2 = _parent(g, 1), _parent(g2, 2)
    both = run_gpu([g, g2], [p, p2], 3, 100, 50, use_graph=True)
    a = both.samples()
    alone = run_gpu([g], [p], 3, 100, 50).samples()[0]
    assert np.array_equal(a[0].cpu().numpy(), alone.cpu().numpy())
    fd = run_gpu([dict(g, hi_radius=0.0)], [p], 3, 100, 50).samples()[0]
    assert np.max(np.abs(fd.cpu().numpy() - alone.cpu().numpy())) > 1e-3


def test_hi_rsf_cycle_matches_oracle():
    from oracle import ora
    from paper_2206_05851_amd import ra
    g = wl.group(16, 6, 1e-3, wl.FENE, 1.0, 50.0, wl.SHEAR, 0.5, hi_radius=0.4)
    p = _parent(g, 6)
    S, P, W = 40, 30, 3
    par = ra.Replicas([dict(g, n_replicas=1)], 9, sample_every=P, max_windows=W, tsf=True, noise_tag=1)
    par.init_chains([p])
    rep = ra.Replicas([g], 9, sample_every=S, max_windows=W)
    rep.rsf_cycle(par, W, P)
    isf, _, tsf, _ = [t.cpu().numpy() for t in par.average_forces(tsf=True)]
    rsf, _ = [t.cpu().numpy() for t in rep.average_forces()]
    op = ora.Oracle([dict(g, n_replicas=1)], 9, P, W, tsf=True)
    op.set_tag(ora.TAG_PARENT)
    op.init_chains([p])
    orr = ora.Oracle([g], 9, S, W)
    orr.rsf_cycle(op, W, P)
    oisf, _, otsf, _ = op.average_forces(tsf=True)
    orsf, _ = orr.average_forces()
    e = [rel_err(isf, oisf, 1.0), rel_err(tsf, otsf, 1.0), rel_err(rsf, orsf, 1.0)]
    announce("hi rsf: " + " ".join("%.1e" % x for x in e))
    assert max(e) < 1e-4


def test_hi_full_size_hi50_first_window_per_replica():
    # The hi50 workload in full (the paper's model with HI: 50 replicas and the
    # parent, 4 windows of 750 steps), launched as bench.py runs it (parent on
    # its own stream, graphs on); the oracle replays the parent and replicas
    # 0..1 of the first window with the same counters.
    import torch
    from oracle import ora
    from paper_2206_05851_amd import ra
    groups, parents, run = wl.hi50()
    g = groups[0]
    S, P, W = run["sample_every"], run["parent_steps"], run["n_windows"]
    announce("hi50 full size")
    pstream = torch.cuda.Stream()
    par = ra.Replicas([dict(g, n_replicas=1)], run["seed"], sample_every=P, max_windows=W, tsf=True, noise_tag=1,
                      stream=pstream, use_graph=True)
    par.init_chains(parents)
    rep = ra.Replicas(groups, run["seed"], sample_every=S, max_windows=W, use_graph=True)
    rep.rsf_cycle(par, W, P)
    smp = rep.samples()[0].cpu().numpy()
    psmp = par.samples()[0].cpu().numpy()
    par.sync_status()
    rep.sync_status()
    assert rep.kernel_family() == 3
    assert np.all(np.isfinite(smp)) and smp.shape == (W, 50, 49)
    op = ora.Oracle([dict(g, n_replicas=1)], run["seed"], P, 1, tsf=True)
    op.set_tag(ora.TAG_PARENT)
    op.init_chains(parents)
    orr = ora.Oracle(groups, run["seed"], S, 1)
    orr.set_replicas(0, 0, 2)
    orr.rsf_cycle(op, 1, P)
    fl = float(np.sqrt(g["H"] * g["kT"]))
    e = [rel_err(psmp[0], op.samples()[0][0], fl), rel_err(smp[0, :2], orr.samples()[0][0], fl)]
    announce("hi50 window 0: parent rel err %.2e, replicas 0-1 rel err %.2e" % tuple(e))
    assert max(e) < 1e-4
