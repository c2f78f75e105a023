"""CPU checks of the C ABI: the library loads, exports every symbol that
include/ra.h declares, and rejects invalid descriptors on the host before any
device work (no GPU needed for these paths)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2206_05851_amd import ra
    if not os.path.exists(ra.LIB_PATH):
        from paper_2206_05851_amd import build
        build.build()
    return ra.library()


def header_symbols():
    text = open(os.path.join(ROOT, "include", "ra.h")).read()
    return sorted(set(re.findall(r"RA_API\s+[\w\s\*]+?\b(ra_\w+)\s*\(", text)))


def test_header_declares_the_five_calls():
    syms = header_symbols()
    for name in ("ra_init_chains", "ra_step", "ra_average_forces", "ra_bell_rates", "ra_backward"):
        assert name in syms


def test_every_declared_symbol_is_exported(lib):
    from paper_2206_05851_amd import ra
    syms = header_symbols()
    assert sorted(ra.EXPORTS) == syms
    for name in syms:
        assert hasattr(lib, name), name
    # and nothing from the oracle leaks into the product library
    with pytest.raises(AttributeError):
        getattr(lib, "rao_philox4x32_10")


def test_struct_sizes_match_header():
    from paper_2206_05851_amd import ra
    text = open(os.path.join(ROOT, "include", "ra.h")).read()
    assert "112 bytes" in text and "56 bytes" in text
    assert ctypes.sizeof(ra.ChainDesc) == 112
    assert ctypes.sizeof(ra.RunDesc) == 56


def _create(lib, desc_kw, run_kw):
    from paper_2206_05851_amd import ra
    d = ra.make_desc(dict(dict(n_beads=10, n_replicas=4, dt=1e-3), **desc_kw), 0)
    arr = (ra.ChainDesc * 1)(d)
    run = ra.RunDesc(**dict(dict(seed=0, precision=32, sample_every=10, max_windows=4), **run_kw))
    p = ctypes.c_void_p()
    rc = lib.ra_create(ctypes.byref(p), arr, 1, ctypes.byref(run), None)
    return rc, lib.ra_last_error(None).decode()


@pytest.mark.parametrize("desc_kw,run_kw,frag", [
    (dict(n_beads=1), {}, "n_beads"),
    (dict(n_beads=2000), {}, "n_beads"),
    (dict(n_beads=300), dict(precision=64), "n_beads"),
    (dict(n_replicas=0), {}, "n_replicas"),
    (dict(dt=0.0), {}, "dt"),
    (dict(dt=float("nan")), {}, "dt"),
    (dict(spring=1, b=0.0), {}, "FENE"),
    (dict(spring=7), {}, "spring"),
    (dict(flow=9), {}, "flow"),
    (dict(stream_id=1 << 24), {}, "stream_id"),
    (dict(noise_scale=-1.0), {}, "noise_scale"),
    ({}, dict(precision=16), "precision"),
    ({}, dict(sample_every=0), "sample_every"),
    ({}, dict(max_windows=65536), "max_windows"),
    ({}, dict(checkpoint_every=10, precision=64), "adjoint"),
    ({}, dict(checkpoint_every=10, plain=1), "adjoint"),
    ({}, dict(checkpoint_every=-1, precision=64), "adjoint"),
    ({}, dict(checkpoint_every=-2), "negative"),
    ({}, dict(waves_per_block=3), "waves_per_block"),
    ({}, dict(noise_tag=2), "noise_tag"),
    (dict(spring=2, rest_length=-1.0), {}, "rest_length"),
    (dict(lj_eps=1.0, lj_rmin=0.0), {}, "lj_rmin"),
    (dict(lj_eps=-1.0), {}, "lj_eps"),
    (dict(spring=2, rest_length=2.0, n_beads=65), {}, "n_beads"),
    (dict(spring=2, rest_length=2.0), dict(checkpoint_every=10), "adjoint"),
    (dict(spring=2, rest_length=2.0), dict(plain=1), "plain"),
    (dict(hi_radius=-0.5), {}, "hi_radius"),
    (dict(hi_radius=0.5, n_beads=65), {}, "n_beads"),
    (dict(hi_radius=0.5), dict(checkpoint_every=10), "adjoint"),
    (dict(hi_radius=0.5), dict(plain=1), "plain"),
    ({}, dict(noise_map=3), "noise_map"),
    ({}, dict(noise_map=-1), "noise_map"),
    ({}, dict(noise_map=2), "noise_map"),
    (dict(n_beads=300), dict(noise_map=2, checkpoint_every=10, precision=64), "adjoint"),
    (dict(spring=2, rest_length=2.0), dict(noise_map=2), "noise_map"),
    (dict(n_beads=300), dict(noise_map=1), "noise_map"),
    (dict(spring=2, rest_length=2.0), dict(noise_map=1), "noise_map"),
    (dict(hi_radius=0.5), dict(noise_map=1), "noise_map"),
])
def test_invalid_descriptors_rejected_on_host(lib, desc_kw, run_kw, frag):
    rc, msg = _create(lib, desc_kw, run_kw)
    assert rc == -1
    assert frag in msg


def test_null_context_calls_fail_cleanly(lib):
    assert lib.ra_step(None, 10) == -1
    assert lib.ra_init_chains(None, None) == -1
    assert lib.ra_backward(None, None, None, None, 0.0, 0.0, None) == -1
    assert lib.ra_reclone(None, None) == -1
    assert lib.ra_rsf_cycle(None, None, 1, 1) == -1
    assert lib.ra_block_sigma(None, 1, None) == -1
    assert lib.ra_mftu(None, None, 1, None) == -1
    assert lib.ra_conformation(None, None, None, None, None) == -1
    assert lib.ra_checkpoint_interval(None, None) == -1
    lib.ra_destroy(None)


def test_mixed_model_classes_rejected_on_host(lib):
    from paper_2206_05851_amd import ra
    run = ra.RunDesc(seed=0, precision=32, sample_every=10, max_windows=4)
    for extra in (dict(hi_radius=0.5), dict(spring=2, rest_length=2.0), dict(lj_eps=1.0, lj_rmin=1.0)):
        d0 = ra.make_desc(dict(n_beads=10, n_replicas=4, dt=1e-3), 0)
        d1 = ra.make_desc(dict(dict(n_beads=10, n_replicas=4, dt=1e-3), **extra), 1)
        arr = (ra.ChainDesc * 2)(d0, d1)
        p = ctypes.c_void_p()
        assert lib.ra_create(ctypes.byref(p), arr, 2, ctypes.byref(run), None) == -1
        assert "only" in lib.ra_last_error(None).decode()


def test_tile_policy_values_checked(lib):
    for bad in (2, 3, 1000, 1017, -1):
        rc, msg = _create(lib, {}, dict(tile_policy=bad))
        assert rc == -1 and "tile_policy" in msg, bad


def test_static_run_rejections_on_host(lib):
    # every case fails in host validation, before the device is touched; the
    # dummy parent pointer is never dereferenced (skipped where a GPU exists,
    # so no case can reach a kernel)
    import torch
    from paper_2206_05851_amd import ra
    if torch.cuda.is_available():
        pytest.skip("host-only check")

    def call(desc_kw, run_kw, n_steps, parent=ctypes.c_void_p(0x1000), outs=True):
        d = ra.make_desc(dict(dict(n_beads=50, n_replicas=64, dt=1e-4, spring=1, b=100.0), **desc_kw), 0)
        run = ra.RunDesc(**dict(dict(seed=0, precision=32, sample_every=10, max_windows=4), **run_kw))
        out = ctypes.c_void_p(0x2000) if outs else None
        rc = lib.ra_run_static(ctypes.byref(d), ctypes.byref(run), parent, n_steps, out, out, None)
        return rc, lib.ra_last_error(None).decode()

    cases = [
        (dict(n_replicas=8192, n_beads=1000), {}, 1000, "scratch"),
        ({}, {}, 15, "multiple"),
        ({}, {}, 0, "multiple"),
        ({}, dict(tsf=1), 10, "TSF"),
        ({}, dict(checkpoint_every=10, max_steps=10), 10, "checkpoints"),
        ({}, dict(plain=1), 10, "fused"),
        ({}, dict(tile_policy=1), 10, "autotuning"),
        (dict(spring=2, rest_length=2.0), {}, 10, "chain model"),
        (dict(hi_radius=0.5), {}, 10, "chain model"),
        (dict(n_beads=300), dict(noise_map=1), 10, "noise_map"),
        ({}, dict(noise_map=2), 10, "noise_map"),
        (dict(n_beads=1), {}, 10, "n_beads"),
    ]
    for desc_kw, run_kw, n, frag in cases:
        rc, msg = call(desc_kw, run_kw, n)
        assert rc == -1 and frag in msg, (desc_kw, run_kw, n, msg)
    rc, msg = call({}, {}, 10, parent=None)
    assert rc == -1 and "null" in msg
    rc, msg = call({}, {}, 10, outs=False)
    assert rc == -1 and "output" in msg


def test_plain_fp64_long_chain_tile_on_host(lib):
    # an FP64 plain-path context of 1000 beads is valid; its work list is laid
    # out with a tile that holds the chain in one wavefront (on a host without
    # a GPU the call then fails at allocation, with a code, not a crash)
    import torch
    if torch.cuda.is_available():
        pytest.skip("host-only check")
    rc, msg = _create(lib, dict(n_beads=1000, n_replicas=8), dict(precision=64, plain=1))
    assert rc in (-2, -3), (rc, msg)
    rc, msg = _create(lib, dict(n_beads=300), dict(precision=64))
    assert rc == -1 and "n_beads" in msg
