"""Shared helpers for the GPU tests (no method arithmetic here)."""
import os

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_05851_amd import ra
    if not os.path.exists(ra.LIB_PATH):
        pytest.fail("libra.so is not built (run __graft_entry__.build())")
    torch.cuda.set_device(0)


def announce(msg):
    print("[gpu-test] " + msg, flush=True)


def rel_err(a, b, floor=0.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), floor)) if a.size else 0.0


def run_gpu(groups, parents, seed, steps, S, max_windows=None, **kw):
    from paper_2206_05851_amd import ra
    rep = ra.Replicas(groups, seed, sample_every=S,
                      max_windows=max_windows if max_windows is not None else steps // S, **kw)
    rep.init_chains(parents)
    if steps:
        rep.step(steps)
    return rep


def run_oracle(groups, parents, seed, steps, S, max_windows=None, **kw):
    from oracle import ora
    o = ora.Oracle(groups, seed, S, max_windows if max_windows is not None else steps // S, **kw)
    o.init_chains(parents)
    if steps:
        o.step(steps)
    return o


def cpu_threads():
    """Host threads for oracle runs: the cores this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_mean_parallel(groups, parents, seed, steps, S, noise_map=0, threads=None):
    """Replica-mean profile [W][N-1] of a one-group oracle run, its replicas
    split into contiguous ranges run on host threads (the counters carry the
    global replica index, so every range draws the noise of the full run);
    the ranges' means are combined weighted by their sizes."""
    import concurrent.futures
    from oracle import ora
    assert len(groups) == 1
    R = groups[0]["n_replicas"]
    nt = min(threads or cpu_threads(), R)
    edges = [R * i // nt for i in range(nt + 1)]

    def part(i):
        o = ora.Oracle(groups, seed, S, steps // S, noise_map=noise_map)
        o.set_replicas(0, edges[i], edges[i + 1])
        o.init_chains(parents)
        o.step(steps)
        m, _ = o.average_forces()
        o.close()
        return (edges[i + 1] - edges[i]) * m

    with concurrent.futures.ThreadPoolExecutor(max_workers=nt) as ex:
        parts = list(ex.map(part, range(nt)))
    return sum(parts) / R
