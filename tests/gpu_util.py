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
