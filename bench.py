"""Benchmark: replica-averaged Brownian dynamics on one MI355X.

Headline workload (one "step" = the whole hot path once), the largest
single-GPU configuration:
  large1000: FENE chain, N = 1000 beads, b = 400, start-up uniaxial elongation
  at Wi = 10, dt = 5e-5, 8192 replicas cloned from one equilibrium parent,
  2 x 10^4 Euler-Maruyama steps, replica-averaged (RSF) and time-averaged
  (TSF) tension profiles over windows of 500 steps (40 windows), FP32 state,
  FP64 averages, Bell rates k0 = 1e-6, x = 0.1 with one event draw per spring
  and window
  = ra_init_chains + ra_step(2 x 10^4) + ra_average_forces (RSF and TSF)
    + ra_bell_rates (rates, rate sums, events),
  inputs (parent conformation) resident in HBM before the timed region.

value = replica*bead*steps per second (8192 * 1000 * 2 x 10^4 per step / time).

The roofline object is for the fused forward kernel of the headline: its
duration is taken with HIP events on the stream it is launched on, and its
algorithmic work is the VALU lane-slots per replica*bead*step (below) times
the replica*bead*steps of one launch. cpu_baseline is the FP64 oracle on a
bounded sample of the same workload (replica ranges, all steps) on the host's
cores, one thread and all threads, and the GPU's samples are compared with it.

Also reported, each measured after warm-up: the plain unbatched GPU path on
the headline (one launch per EM step, state in HBM; a 2000-step prefix,
extrapolated) and on fene50; fene50 itself (N = 50, 1024 replicas, 10^4 steps);
the adjoint (N = 100, 4096 replicas, 2000 steps, checkpoints every 100); the
batched run (512 uneven FENE chains, one graph-captured persistent launch,
cost-model and autotuned tiles); the RSF sampling cycle (a parent trajectory
re-cloned into 1000 replicas every 750 steps, 20 windows, with ISF/TSF/RSF,
sigma(N_R) and MFTU) on the FENE chain, on the paper's collapsed polymer
(rest-length springs + LJ) and on the full model with hydrodynamic interaction.
The roofline fraction of each chain workload under the same slot count is
listed in roofline_fractions.
"""
import argparse
import concurrent.futures
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "replica·bead·steps/s and adjoint steps/s vs plain GPU path at 1e-4 rel err"

# Peak VALU issue rate of one MI355X in lane-slots: 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz = 39.3 T lane-slots/s. One lane-slot is one lane of one VALU
# instruction issue (a wave64 instruction occupies its SIMD's VALU for 4
# cycles); it is the published 157.3 TFLOP/s FP32 vector peak divided by 2
# flops per FMA and by 2 for the packed FP32 forms, which integer work cannot use.
VALU_PEAK_LANE_SLOTS = 256 * 4 * 16 * 2.4e9
# Algorithmic lane-slots per replica*bead*step of the FENE forward step: the
# gfx950 VALU instructions the step needs, one slot each, the same count for
# every tile layout. Transcendentals (v_log, v_sqrt, v_sin, v_cos, v_rcp) are
# not counted: they execute on the transcendental unit beside the VALU (on
# large1000 the kernel issues 1.05x more VALU instructions than 4-cycle slots
# exist in its active cycles; without the transcendentals, 0.95x).
#   Philox4x32-10: 10 rounds x (2 v_mad_u64_u32 + 2 v_bitop3_b32)           = 40
#   uniform maps: 4 words x (v_alignbit_b32 + subtract)                        =  8
#   Box-Muller, 3 normals: 2 log scalings + 3 radius products                  =  5
#     (beside them on the transcendental unit: 2 log, 2 sqrt, 3 sin/cos)
#   FENE bond update: |Q|^2 (3), s, 1 - s, guard compare, g Q (3), neighbour
#     Laplacian by DPP (9), noise difference by DPP (3), flow + EM increment
#     (8), add (3)                                                            = 31
#     (beside them: the reciprocal 1/(1 - s))
# With noise map 1 a Philox block gives four normals and serves 4/3 bead-steps:
#   Philox 40 x 3/4 = 30; uniform maps 8 x 3/4 = 6; Box-Muller with both outputs
#   of the second pair (2 log scalings + 4 radius products) x 3/4 = 4.5;
#   FENE bond update 31.
# Noise map 2 (beads in groups of four, three blocks per group and step) draws
# and transforms the same 3/4 block per bead-step as map 1.
SLOTS_PER_BEAD_STEP = {0: 40 + 8 + 5 + 31, 1: 30 + 6 + 4.5 + 31, 2: 30 + 6 + 4.5 + 31}
# HBM bytes per launch of the headline's forward kernel, read with rocprofv3
# counters (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 KiB, both factors from a 1 GiB
# device copy in the same runs). Valid only for the kernel they were taken on:
# the digest of the kernel's sources (device code and its argument block), the
# launch tile (beads per lane, replicas per wavefront, kernel family) and the
# noise map are recorded with the figure, and traffic is reported as null when
# any of them differs.
FWD_TRAFFIC = {"sha256": "4db2b2d7ac6e4b9e7fead47e53ba5fac9fdcdb728271da68bd6cfff70a7bbcf5", "noise_map": 2,
               "tile": (16, 1, 16), "bytes": (48764.958 * 2.0 + 2655974.031) * 1024}
FWD_SOURCES = ("ra_kernels.hip", "ra_chain.hpp", "ra_device.hpp", "ra_types.hpp", "ra_launch.hpp")


def fwd_sources_digest(files=FWD_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2206_05851_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


# The pair kernel's lane-slots per replica*bead*step on collapsed50 (N = 50):
# non-transcendental VALU instructions per wavefront-step (one bead per lane)
# of fwd_pair_dual_kernel<float>, from rocprofv3 --pmc SQ_INSTS_VALU
# SQ_INSTS_VALU_TRANS_F32 SQ_WAVES: (636,828,191 - 43,547,252) / 1001 wavefronts
# / 750 steps. It holds for the pair kernel sources with this digest only.
PAIR_SOURCES = ("ra_pair.hip", "ra_chain.hpp", "ra_device.hpp", "ra_dpp.hpp")
PAIR_SLOTS = {"sha256": "ad605e15eed9f61ce0d2c49a4d6ed60cbfd68a769bb007705ed98ffad3646d11",
              "slots": (636828191.0 - 43547252.0) / 1001 / 750}
FP32_VECTOR_PEAK = 157.3e12   # FLOP/s, packed FP32 included


def hi_flops_per_replica_step(n_beads):
    """Dense linear algebra of one HI step on the 3N x 3N tensor: Cholesky
    n^3/3, the drift D F 2 n^2 and the displacement L xi n^2 flops."""
    n = 3 * n_beads
    return n ** 3 / 3.0 + 3.0 * n * n


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def time_once(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


class EventTimer:
    """HIP events around one call on a given stream; mean duration in ms."""

    def __init__(self, stream):
        self.stream = stream
        self.pairs = []

    def run(self, fn):
        import torch
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        r = fn()
        e1.record(self.stream)
        self.pairs.append((e0, e1))
        return r

    def mean_ms(self):
        import numpy as np
        return float(np.mean([a.elapsed_time(b) for a, b in self.pairs]))


def roofline_frac(slots, work, seconds):
    return slots * work / seconds / VALU_PEAK_LANE_SLOTS


# ---------------------------------------------------------------------------
# FP64 oracle baseline (host cores) on replica ranges of a one-group workload
# ---------------------------------------------------------------------------
def oracle_range(groups, parents, run, k_begin, k_end, noise_map=0):
    """The whole pass (clone, all steps, RSF/TSF averages, Bell rates and
    events) of the oracle on replicas [k_begin, k_end); returns seconds and the
    per-replica samples (and TSF samples)."""
    from oracle import ora
    tsf = bool(run.get("tsf", False))
    t0 = time.perf_counter()
    o = ora.Oracle(groups, run["seed"], run["sample_every"], run["steps"] // run["sample_every"], tsf=tsf,
                   noise_map=noise_map)
    o.set_replicas(0, k_begin, k_end)
    o.init_chains(parents)
    o.step(run["steps"])
    mean = o.average_forces(tsf=tsf)[0]
    o.bell_rates(mean, run["k0"], run["x_dagger"], events=tsf)
    secs = time.perf_counter() - t0
    smp = o.samples(tsf=tsf)
    o.close()
    if tsf:
        return secs, smp[0][0], smp[1][0]
    return secs, smp[0], None


def cpu_baseline(groups, parents, run, single_replicas, per_thread, threads, noise_map=0):
    import numpy as np
    N, T = groups[0]["n_beads"], run["steps"]
    log("cpu baseline: oracle, 1 thread, replicas 0..%d x %d steps" % (single_replicas - 1, T))
    t1, _, _ = oracle_range(groups, parents, run, 0, single_replicas, noise_map)
    log("cpu baseline: oracle, %d threads x %d replicas x %d steps" % (threads, per_thread, T))
    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda i: oracle_range(groups, parents, run, i * per_thread, (i + 1) * per_thread,
                                                   noise_map), range(threads)))
    tall = time.perf_counter() - t0
    n_all = threads * per_thread
    smp = np.concatenate([p[1] for p in parts], axis=1)
    tsmp = np.concatenate([p[2] for p in parts], axis=1) if parts[0][2] is not None else None
    return {"single": (single_replicas * N * T / t1, t1), "all": (n_all * N * T / tall, tall, n_all),
            "samples": smp, "tsf_samples": tsmp}


def oracle_samples(groups, parents, run, n_replicas, threads, noise_map):
    """Per-replica samples of replicas [0, n_replicas) of a one-group workload
    (the oracle's whole pass, replicas split over host threads)."""
    import numpy as np
    per = -(-n_replicas // threads)
    edges = [(k, min(k + per, n_replicas)) for k in range(0, n_replicas, per)]
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda e: oracle_range(groups, parents, run, e[0], e[1], noise_map), edges))
    smp = np.concatenate([p[1] for p in parts], axis=1)
    tsmp = np.concatenate([p[2] for p in parts], axis=1) if parts[0][2] is not None else None
    return smp, tsmp


def oracle_all_cores(jobs, threads):
    """Run oracle jobs (callables returning the replica*bead*steps they did)
    on a pool of host threads; returns (work, seconds)."""
    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        work = sum(ex.map(lambda f: f(), jobs))
    return work, time.perf_counter() - t0


def oracle_job(group, parent, run, k_begin, k_end, noise_map, tangents=False):
    """One oracle run of replicas [k_begin, k_end) of one chain: clone, all
    steps, replica averages (and the gradient by forward-mode tangents)."""
    def job():
        import numpy as np
        from oracle import ora
        S = run["sample_every"]
        o = ora.Oracle([group], run["seed"], S, run["steps"] // S, tangents=tangents, noise_map=noise_map)
        o.set_replicas(0, k_begin, k_end)
        o.init_chains([parent])
        o.step(run["steps"])
        m, _ = o.average_forces()
        if tangents:
            o.backward(np.ones_like(m), None, run["k0"], run["x_dagger"])
        o.close()
        return (k_end - k_begin) * group["n_beads"] * run["steps"]
    return job


def oracle_rates(threads, noise_map, gpu):
    """The FP64 oracle on all host threads (replicas or whole chains split
    over the threads) for the correctness and measurement workloads besides
    the headline: rouse_fp64_small, fene50 and adjoint100 (gradient) in
    full, batched512 on its first 16 chains (extrapolated by work). gpu maps
    a workload to the GPU's rate for the same quantity, when bench.py
    measured it."""
    from paper_2206_05851_amd import workloads as wl

    def split(groups, parents, run, nm, tangents=False):
        jobs = []
        for g, p in zip(groups, parents):
            R = g["n_replicas"]
            parts = min(R, 4 * threads)
            for i in range(parts):
                kb, ke = R * i // parts, R * (i + 1) // parts
                if ke > kb:
                    jobs.append(oracle_job(g, p, run, kb, ke, nm, tangents))
        return jobs

    res = {"cores": threads, "unit": "replica·bead·steps/s", "kind": "oracle (FP64, threads over replicas)"}
    cases = [("rouse_fp64_small", wl.rouse_fp64_small(), 0, False, "all 64 replicas x 5000 steps"),
             ("fene50", wl.fene50(), noise_map, False, "all 1024 replicas x 10^4 steps"),
             ("adjoint100_gradient", wl.adjoint100(), noise_map, True,
              "all 4096 replicas x 2000 steps, forward with tangents + gradient"),
             ("batched512_first16", None, noise_map, False,
              "chains 0..15 of 512 in full, their replicas split over the threads; a rate per "
              "replica*bead*step, which extrapolates by work to all 512 chains")]
    for name, wload, nm, tangents, sample in cases:
        if wload is None:
            groups, parents, run = wl.batched512()
            groups, parents = groups[:16], parents[:16]
        else:
            groups, parents, run = wload
        log("oracle on %d threads: %s" % (threads, name))
        work, secs = oracle_all_cores(split(groups, parents, run, nm, tangents), threads)
        res[name] = {"value": work / secs, "seconds": secs, "sample": sample}
        if name in gpu:
            res[name]["gpu_value"] = gpu[name]
            res[name]["gpu_over_oracle"] = gpu[name] / (work / secs)
    return res


def accuracy(got, ref, first_windows):
    """Max relative errors: every sample, and the replica-mean profile of the
    compared replicas, over all windows and over the first windows."""
    import numpy as np
    rel = np.abs(got - ref) / np.abs(ref)
    prof = np.abs(got.mean(axis=1) - ref.mean(axis=1)) / np.abs(ref.mean(axis=1))
    return {"samples": float(rel.max()), "samples_first": float(rel[:first_windows].max()),
            "profile": float(prof.max()), "profile_first": float(prof[:first_windows].max())}


# ---------------------------------------------------------------------------
# Extras
# ---------------------------------------------------------------------------
def rsf_cycle_bench(workload, desc, dev, name, noise_map=0):
    """One RSF cycle (parent context on its own stream, re-clone per window)
    with the estimators built on it, timed after a warm-up cycle."""
    import numpy as np
    import torch
    from paper_2206_05851_amd import ra
    rg, rp, rrun = workload
    rS, rP, rW = rrun["sample_every"], rrun["parent_steps"], rrun["n_windows"]
    pstream = torch.cuda.Stream()
    rpar = ra.Replicas([dict(x, n_replicas=1) for x in rg], rrun["seed"], sample_every=rP, max_windows=rW,
                       tsf=True, noise_tag=1, stream=pstream, use_graph=True, device=dev, noise_map=noise_map)
    rrep = ra.Replicas(rg, rrun["seed"], sample_every=rS, max_windows=rW, use_graph=True, device=dev,
                       noise_map=noise_map)
    mftu = {}
    rpd = torch.from_numpy(np.concatenate([np.ravel(x) for x in rp])).to(dev)

    def cycle():
        rpar.init_chains(rpd)
        rrep.init_chains(rpd)
        rrep.rsf_cycle(rpar, rW, rP)
        isf, _, tsf, _ = rpar.average_forces(tsf=True)
        rsf, _ = rrep.average_forces()
        for b in rrun["blocks"]:
            rrep.block_sigma(b)
        rrep.conformation()
        for key, prof in (("isf", isf), ("tsf", tsf), ("rsf", rsf)):
            _, rs = rpar.bell_rates(prof, rrun["k0"], rrun["x_dagger"])
            mftu[key] = rpar.mftu(rs)

    cycle()
    t = min(time_once(cycle) for _ in range(2))
    rpar.sync_status()
    rrep.sync_status()
    work = rg[0]["n_replicas"] * rg[0]["n_beads"] * rS * rW
    res = {"workload": name + ": " + desc, "value": work / t,
           "unit": "replica·bead·steps/s (whole cycle incl. parent)", "ms_per_cycle": 1e3 * t,
           "us_per_window": 1e6 * t / rW, "mftu": {k: float(v[0]) for k, v in mftu.items()},
           "noise_map": noise_map}
    # MFTU by sampling unfolding events over the cycle's rate profiles (1024
    # trials, up to 2^20 windows each), beside 1/<sum k> above
    isf, _, tsf, _ = rpar.average_forces(tsf=True)
    rsf, _ = rrep.average_forces()
    ev = {}
    t_ev = 0.0
    for key, prof in (("isf", isf), ("tsf", tsf), ("rsf", rsf)):
        rates, _ = rpar.bell_rates(prof, rrun["k0"], rrun["x_dagger"])
        t0 = time.perf_counter()
        m, f = rpar.mftu_events(rates, 1024, 1 << 20)
        torch.cuda.synchronize()
        t_ev += time.perf_counter() - t0
        ev[key] = {"mftu": float(m[0]), "censored": float((f[:, 0] < 0).float().mean().item())}
    res["mftu_events"] = dict(ev, trials=1024, max_windows=1 << 20, ms=1e3 * t_ev)
    rpar.close()
    rrep.close()
    # roofline over the whole cycle's wall time (forward launches, re-clones,
    # the parent, the estimators): a lower bound on the kernels' own fraction
    g0 = rg[0]
    if g0.get("hi_radius", 0.0) > 0.0:
        reps = (g0["n_replicas"] + 1) * rS * rW / t   # replica-steps/s, the parent included
        flops = hi_flops_per_replica_step(g0["n_beads"])
        res["roofline"] = {"bound": "fp32_vector", "unit": "TFLOP/s", "peak": FP32_VECTOR_PEAK / 1e12,
                           "achieved": flops * reps / 1e12, "frac": flops * reps / FP32_VECTOR_PEAK,
                           "flops_per_replica_step": flops,
                           "note": "dense linear algebra of the step (Cholesky n^3/3, D F 2n^2, L xi n^2, "
                                   "n = 3N) over the cycle's wall time; 51 chains occupy 51 of 256 CUs"}
    else:
        pair = g0.get("lj_eps", 0.0) > 0.0 or g0["spring"] == 2
        if pair:
            slots = PAIR_SLOTS["slots"] if fwd_sources_digest(PAIR_SOURCES) == PAIR_SLOTS["sha256"] else None
        else:
            slots = SLOTS_PER_BEAD_STEP[noise_map]
        rate = (g0["n_replicas"] + 1) * g0["n_beads"] * rS * rW / t
        res["roofline"] = {"bound": "alu", "unit": "T VALU lane-slots/s", "peak": VALU_PEAK_LANE_SLOTS / 1e12,
                           "lane_slots_per_replica_bead_step": slots,
                           "achieved": None if slots is None else slots * rate / 1e12,
                           "frac": None if slots is None else slots * rate / VALU_PEAK_LANE_SLOTS,
                           "note": "over the cycle's wall time, the parent included; "
                                   + ("pair kernel slots measured by counters at N = 50" if pair
                                      else "the chain kernels' slot count")}
    log("%s: %.2f ms per cycle (%.1f us per window)" % (name, 1e3 * t, 1e6 * t / rW))
    return res


def oracle_cycle_rates(workload, threads, reps_per_thread, windows):
    """The oracle's RSF cycle (parent with noise tag 1, replicas re-cloned
    every window) on a bounded sample: replicas [0, reps_per_thread) on one
    thread, and reps_per_thread per thread on all threads (each thread runs
    its own copy of the parent). Rates count replica*bead*steps only."""
    from oracle import ora
    groups, parents, run = workload
    g = groups[0]
    S, P = run["sample_every"], run["parent_steps"]

    def job(k0):
        op = ora.Oracle([dict(g, n_replicas=1)], run["seed"], P, windows, tsf=True)
        op.set_tag(ora.TAG_PARENT)
        op.init_chains(parents)
        orr = ora.Oracle(groups, run["seed"], S, windows)
        orr.set_replicas(0, k0, k0 + reps_per_thread)
        orr.rsf_cycle(op, windows, P)
        orr.average_forces()
        op.close()
        orr.close()
        return reps_per_thread * g["n_beads"] * S * windows

    t0 = time.perf_counter()
    w1 = job(0)
    t1 = time.perf_counter() - t0
    work, ta = oracle_all_cores([lambda i=i: job(i * reps_per_thread) for i in range(threads)], threads)
    return {"kind": "oracle", "unit": "replica·bead·steps/s", "cores": threads,
            "value": work / ta, "seconds": ta, "single_thread": {"value": w1 / t1, "seconds": t1},
            "sample": "RSF cycle of %d windows: the parent and %d replicas per thread (%d on %d threads; "
                      "one thread for the single-thread rate), replica work only" % (
                          windows, reps_per_thread, reps_per_thread * threads, threads)}


def sigma_sweep_bench(dev, noise_map):
    """sigma(N_R) of the RSF estimate against the evolution time S (the
    analogue of Figs. 2 and 5): the rsf50 chain's RSF cycle at several S
    (parent steps P = S), 20 windows each, sigma over blocks of N_R replicas
    for the middle spring (window mean) and over all springs; beside them the
    spread over windows of the parent's ISF and TSF of the middle spring."""
    import numpy as np
    import torch
    from paper_2206_05851_amd import ra
    from paper_2206_05851_amd import workloads as wl
    rg, rp, rrun = wl.rsf50()
    rpd = torch.from_numpy(np.concatenate([np.ravel(x) for x in rp])).to(dev)
    W, mid = rrun["n_windows"], rg[0]["n_beads"] // 2 - 1
    rows = []
    t0 = time.perf_counter()
    for S in (75, 250, 750, 2500):
        par = ra.Replicas([dict(x, n_replicas=1) for x in rg], rrun["seed"], sample_every=S, max_windows=W,
                          tsf=True, noise_tag=1, device=dev, noise_map=noise_map)
        rep = ra.Replicas(rg, rrun["seed"], sample_every=S, max_windows=W, device=dev, noise_map=noise_map)
        par.init_chains(rpd)
        rep.init_chains(rpd)
        rep.rsf_cycle(par, W, S)
        isf, _, tsf, _ = [x.cpu().numpy() for x in par.average_forces(tsf=True)]
        row = {"S_steps": S, "S_time": S * rg[0]["dt"],
               "isf_spread_mid": float(isf[:, mid].std(ddof=1)), "tsf_spread_mid": float(tsf[:, mid].std(ddof=1))}
        for b in (10, 20, 40):
            sig = rep.block_sigma(b).cpu().numpy()
            row["sigma_NR%d_mid" % b] = float(sig[:, mid].mean())
            row["sigma_NR%d_all" % b] = float(sig.mean())
        par.sync_status()
        rep.sync_status()
        par.close()
        rep.close()
        rows.append(row)
    log("sigma sweep: %d evolution times in %.2f s" % (len(rows), time.perf_counter() - t0))
    return {"workload": "rsf50 chain (FENE N=50 b=100, shear Wi=50), RSF cycles at S = 75, 250, 750, 2500 steps "
                        "(dt = 1e-4), parent steps P = S, 1000 replicas, 20 windows; sigma over blocks of N_R = "
                        "10, 20, 40", "noise_map": noise_map, "rows": rows}


def fene50_bench(dev, noise_map, passes=10):
    """fene50 (N = 50, 1024 replicas, 10^4 steps) fused, and its plain path."""
    import numpy as np
    import torch
    from paper_2206_05851_amd import ra
    from paper_2206_05851_amd import workloads as wl
    groups, parents, run = wl.fene50()
    g = groups[0]
    R, N, T, S = g["n_replicas"], g["n_beads"], run["steps"], run["sample_every"]
    W = T // S
    parent = torch.from_numpy(np.ascontiguousarray(parents[0]).reshape(-1)).to(dev)
    rep = ra.Replicas(groups, run["seed"], sample_every=S, max_windows=W, device=dev, noise_map=noise_map)
    timer = EventTimer(torch.cuda.current_stream())
    mean = torch.empty((W, N - 1), dtype=torch.float64, device=dev)
    std = torch.empty_like(mean)

    def one(record):
        rep.init_chains(parent)
        if record:
            timer.run(lambda: rep.step(T))
        else:
            rep.step(T)
        rep.average_forces(out=(mean, std))
        rep.bell_rates(mean, run["k0"], run["x_dagger"])

    for _ in range(2):
        one(False)
    # the pass and the kernel both as means over the same timed passes
    t = float(np.mean([time_once(lambda: one(True)) for _ in range(passes)]))
    rep.sync_status()
    work = R * N * T
    kms = timer.mean_ms()
    out = {"workload": "fene50: FENE N=50 b=100, uniaxial Wi=2, dt=1e-4, R=1024, 10^4 steps, sample every 100, "
                       "Bell rates", "value": work / t, "ms_per_step": 1e3 * t, "kernel_ms": kms,
           "noise_map": noise_map,
           "roofline_frac": roofline_frac(SLOTS_PER_BEAD_STEP[noise_map], work, kms * 1e-3)}
    # plain unbatched path, same workload and counters
    plain = ra.Replicas(groups, run["seed"], sample_every=S, max_windows=W, plain=True, device=dev,
                        noise_map=noise_map)
    pm = torch.empty_like(mean)
    ps = torch.empty_like(mean)

    def plain_pass():
        plain.init_chains(parent)
        plain.step(T)
        plain.average_forces(out=(pm, ps))
        plain.bell_rates(pm, run["k0"], run["x_dagger"])

    plain_pass()
    tp = min(time_once(plain_pass) for _ in range(2))
    plain.sync_status()
    out["plain_path"] = {"value": work / tp, "ms_per_step": 1e3 * tp, "speedup_fused_over_plain": tp / t,
                         "max_rel_diff_profile_vs_fused": torch.max(torch.abs(pm - mean) / mean).item()}
    plain.close()
    rep.close()
    log("fene50: %.3f ms per pass (kernel %.3f ms), plain %.2f ms" % (1e3 * t, kms, 1e3 * tp))
    return out


def adjoint_bench(dev, noise_map):
    import numpy as np
    import torch
    from paper_2206_05851_amd import ra
    from paper_2206_05851_amd import workloads as wl
    ag, ap_, arun = wl.adjoint100()
    ga = ag[0]
    apar = torch.from_numpy(np.ascontiguousarray(ap_[0]).reshape(-1)).to(dev)
    W = arun["steps"] // arun["sample_every"]
    gm = torch.ones((W, ga["n_beads"] - 1), dtype=torch.float64, device=dev)
    awork = ga["n_replicas"] * ga["n_beads"] * arun["steps"]
    res = {}
    for label, K in (("every_100", arun["checkpoint_every"]), ("auto_interval", ra.CKPT_AUTO)):
        adj = ra.Replicas(ag, arun["seed"], sample_every=arun["sample_every"], max_windows=W,
                          checkpoint_every=K, max_steps=arun["steps"], device=dev, noise_map=noise_map)

        def fwd():
            adj.init_chains(apar)
            adj.step(arun["steps"])

        def bwd():
            m, _ = adj.average_forces()
            return adj.backward(m, gm, None)

        fwd()
        bwd()
        tf = min(time_once(fwd) for _ in range(2))
        tb = min(time_once(bwd) for _ in range(2))
        adj.sync_status()
        res[label] = {"checkpoint_every": adj.checkpoint_interval(), "value": awork / tb,
                      "forward_value": awork / tf, "backward_ms": 1e3 * tb, "forward_ms": 1e3 * tf,
                      "backward_over_forward": tb / tf}
        adj.close()
        log("adjoint %s: fwd %.2f ms bwd %.2f ms" % (label, 1e3 * tf, 1e3 * tb))
    out = {"workload": "adjoint100: FENE N=100 b=100, uniaxial Wi=4, R=4096, dt=1e-4, 2000 steps, "
                       "gradient of the profile w.r.t. (rate, H, b)",
           "value": res["every_100"]["value"], "unit": "replica·bead·steps/s (backward incl. recompute)",
           "noise_map": noise_map,
           "forward_roofline_frac": roofline_frac(SLOTS_PER_BEAD_STEP[noise_map], awork,
                                                  res["every_100"]["forward_ms"] * 1e-3)}
    out.update(res)
    return out


def batched_bench(dev, noise_map):
    import numpy as np
    import torch
    from paper_2206_05851_amd import ra
    from paper_2206_05851_amd import workloads as wl
    bg, bp, brun = wl.batched512()
    bpar = torch.from_numpy(np.concatenate([np.ascontiguousarray(p).reshape(-1) for p in bp])).to(dev)
    bwork = sum(x["n_replicas"] * x["n_beads"] for x in bg) * brun["steps"]
    res = {}
    for label, policy in (("cost_model", 0), ("autotuned", 1)):
        t_tune = time.perf_counter()
        bat = ra.Replicas(bg, brun["seed"], sample_every=brun["sample_every"],
                          max_windows=brun["steps"] // brun["sample_every"], use_graph=True, device=dev,
                          tile_policy=policy, noise_map=noise_map)
        t_tune = time.perf_counter() - t_tune
        timer = EventTimer(torch.cuda.current_stream())

        def one():
            bat.init_chains(bpar)
            timer.run(lambda: bat.step(brun["steps"]))
            m, s = bat.average_forces()
            bat.bell_rates(m, brun["k0"], brun["x_dagger"])

        one()
        timer.pairs.clear()
        t = min(time_once(one) for _ in range(3))
        bat.sync_status()
        kms = timer.mean_ms()
        res[label] = {"ms_per_step": 1e3 * t, "kernel_ms": kms, "create_s": t_tune,
                      "roofline_frac": roofline_frac(SLOTS_PER_BEAD_STEP[noise_map], bwork, kms * 1e-3)}
        bat.close()
        log("batched (%s): %.2f ms per pass, kernel %.2f ms" % (label, 1e3 * t, kms))
    best = min(res.values(), key=lambda r: r["ms_per_step"])
    out = {"workload": "batched512: 512 FENE chains N~U{20..200}, b~U[50,200], planar Wi~U[0.5,5] / shear "
                       "Wi~U[1,50], R~U{16..256}, 5000 steps, one graph-captured persistent launch",
           "value": bwork / (best["ms_per_step"] * 1e-3), "noise_map": noise_map}
    out.update(res)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="other_map,plain,fene50,adjoint,batched,rsf50,sigma_sweep,collapsed50,"
                                      "hi50,oracle_rates",
                    help="comma-separated extra workloads to measure")
    ap.add_argument("--cpu-single-replicas", type=int, default=2,
                    help="oracle replicas on one thread (all 2 x 10^4 steps)")
    ap.add_argument("--cpu-replicas-per-thread", type=int, default=2,
                    help="oracle replicas per thread on all threads")
    ap.add_argument("--noise-map", type=int, default=1, choices=(0, 1),
                    help="ra_run_desc.noise_map of fene50, its plain path, the adjoint, batched and rsf50 "
                         "(1: four normals per Philox block, three blocks per four bead-steps; the headline's "
                         "16 beads per lane take --head-map)")
    ap.add_argument("--head-map", type=int, default=2, choices=(0, 2),
                    help="ra_run_desc.noise_map of the headline (16 beads per lane: map 0, one Philox block per "
                         "bead-step, or map 2, three blocks per four beads)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2206_05851_amd import ra
    from paper_2206_05851_amd import workloads as wl

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    groups, parents, run = wl.large1000()
    g = groups[0]
    R, N, T, S = g["n_replicas"], g["n_beads"], run["steps"], run["sample_every"]
    W = T // S
    parent = torch.from_numpy(np.ascontiguousarray(parents[0]).reshape(-1)).to(dev)
    head_map = args.head_map   # noise map 1 is compiled for at most 4 beads per lane
    rep = ra.Replicas(groups, run["seed"], precision=32, sample_every=S, max_windows=W, tsf=True, device=dev,
                      noise_map=head_map)
    outs = [torch.empty((W, N - 1), dtype=torch.float64, device=dev) for _ in range(4)]
    timer = EventTimer(torch.cuda.current_stream())

    def one_step(record):
        rep.init_chains(parent)
        if record:
            timer.run(lambda: rep.step(T))
        else:
            rep.step(T)
        m, s, tm, ts = rep.average_forces(tsf=True)
        return rep.bell_rates(m, run["k0"], run["x_dagger"], events=True)

    log("headline large1000: warmup %d" % args.warmup)
    for _ in range(args.warmup):
        one_step(False)
    rep.sync_status()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    rep.sync_status()
    del outs
    work_per_step = R * N * T
    value = work_per_step * args.steps / elapsed
    kernel_ms = timer.mean_ms()
    slots = SLOTS_PER_BEAD_STEP[head_map]
    achieved = slots * work_per_step / (kernel_ms * 1e-3)
    log("large1000: %.1f ms/step, kernel %.1f ms, %.3e replica-bead-steps/s, frac %.3f" %
        (1e3 * elapsed / args.steps, kernel_ms, value, achieved / VALU_PEAK_LANE_SLOTS))
    tiles = rep.tile_info()
    family = rep.kernel_family()
    traffic = (FWD_TRAFFIC["bytes"] if FWD_TRAFFIC["sha256"] and fwd_sources_digest() == FWD_TRAFFIC["sha256"]
               and FWD_TRAFFIC.get("noise_map") == head_map
               and FWD_TRAFFIC.get("tile") == (tiles[0][0], tiles[1][0], family) else None)
    out = {
        "metric": METRIC, "value": value, "unit": "replica·bead·steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded FENE equilibrium parent; Philox noise, noise map %d)" % head_map,
        "config": {"workload": "large1000: FENE N=1000 b=400, start-up uniaxial Wi=10 (rate=%.6g), dt=5e-5, "
                               "R=8192, 2x10^4 steps, RSF+TSF windows of 500, FP64 averages, Bell rates + events"
                               % g["rate"],
                   "global_batch": R, "seq_len": N, "parallelism": "none (1 GPU)",
                   "beads_per_lane": tiles[0][0], "replicas_per_wave": tiles[1][0],
                   "kernel_family": family, "noise_map": head_map},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_LANE_SLOTS / 1e12,
                     "unit": "T VALU lane-slots/s", "frac": achieved / VALU_PEAK_LANE_SLOTS,
                     "traffic": traffic, "kernel": "fwd_kernel<float,16,2,%d,1>" % head_map, "kernel_ms": kernel_ms,
                     "lane_slots_per_replica_bead_step": slots,
                     "replica_bead_steps_per_launch": work_per_step},
    }
    fracs = {"large1000": out["roofline"]["frac"]}

    n_cmp = 0
    cpu = None
    if not args.no_cpu_baseline:
        threads = max(1, min(16, cpu_cores()))
        cpu = cpu_baseline(groups, parents, run, args.cpu_single_replicas, args.cpu_replicas_per_thread, threads,
                           head_map)
        r1, t1 = cpu["single"]
        ra_, ta, n_cmp = cpu["all"]
        out["cpu_baseline"] = {
            "value": ra_, "unit": "replica·bead·steps/s", "cores": threads, "kind": "oracle",
            "sample": "FP64 oracle, replicas 0..%d of 8192 (%d per thread on %d threads), all 2x10^4 steps, "
                      "RSF+TSF averages, Bell rates and events (%.1f s); rate per replica*bead*step, which "
                      "extrapolates linearly to the full workload (replicas are independent)"
                      % (n_cmp - 1, args.cpu_replicas_per_thread, threads, ta),
            "single_thread": {"value": r1, "replicas": args.cpu_single_replicas, "seconds": t1},
            "host_cores": cpu_cores()}
        log("cpu: %.3e (1 thread), %.3e (%d threads) replica-bead-steps/s" % (r1, ra_, threads))
        smp, tsmp = rep.samples(tsf=True)
        got = smp[0][:, :n_cmp].cpu().numpy()
        tgot = tsmp[0][:, :n_cmp].cpu().numpy()
        del smp, tsmp
        acc = accuracy(got, cpu["samples"], 1)
        tacc = accuracy(tgot, cpu["tsf_samples"], 1)
        out["accuracy_vs_oracle"] = {"replicas": n_cmp, "rsf": acc, "tsf": tacc,
                                     "note": "max relative error over all 40 windows; *_first: first window "
                                             "(500 steps); profile = replica mean of the compared replicas"}
        log("GPU vs oracle: samples %.2e (first window %.2e), profile %.2e; TSF samples %.2e"
            % (acc["samples"], acc["samples_first"], acc["profile"], tacc["samples"]))

    extras = set() if args.no_extras else set(x for x in args.extras.split(",") if x)
    if "other_map" in extras:
        # the same headline pass under the other noise map the wide lanes take
        # (three timed passes after one warm-up), for comparison
        om = 0 if head_map == 2 else 2
        rep_o = ra.Replicas(groups, run["seed"], precision=32, sample_every=S, max_windows=W, tsf=True,
                            device=dev, noise_map=om)
        timer_o = EventTimer(torch.cuda.current_stream())

        def pass_o(record):
            rep_o.init_chains(parent)
            if record:
                timer_o.run(lambda: rep_o.step(T))
            else:
                rep_o.step(T)
            m, s, tm, ts = rep_o.average_forces(tsf=True)
            return rep_o.bell_rates(m, run["k0"], run["x_dagger"], events=True)

        pass_o(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            pass_o(True)
        torch.cuda.synchronize()
        to = (time.perf_counter() - t0) / 3
        rep_o.sync_status()
        kms_o = timer_o.mean_ms()
        out["headline_other_noise_map"] = {
            "noise_map": om, "ms_per_step": 1e3 * to, "kernel_ms": kms_o, "value": work_per_step / to,
            "lane_slots_per_replica_bead_step": SLOTS_PER_BEAD_STEP[om],
            "roofline_frac": roofline_frac(SLOTS_PER_BEAD_STEP[om], work_per_step, kms_o * 1e-3),
            "note": "the headline pass under the other noise map of the 16-beads-per-lane kernels, 3 timed passes"}
        rep_o.close()
        log("large1000 under noise map %d: %.1f ms per pass, kernel %.1f ms" % (om, 1e3 * to, kms_o))
    if "plain" in extras:
        # plain unbatched path on the headline: a 2000-step prefix (4 windows),
        # timed after a warm-up, extrapolated to the 2x10^4 steps
        # The plain kernel (one thread per bead) runs noise map 0, its cheapest:
        # under map 2 each bead's thread would draw its group's three blocks.
        Tp = 2000
        plain_map = 0
        out["plain_path"] = {"workload": "large1000, plain path (one launch per EM step and group, bead "
                                         "positions in HBM), first 2000 steps (4 windows), extrapolated to "
                                         "2x10^4; FP32 (positions lose digits at N = 1000) and FP64; noise "
                                         "map 0 (one Philox block per bead-step, the plain kernel's cheapest)",
                             "noise_map": plain_map}
        plain_ref = None
        if cpu is not None:
            plain_ref = oracle_samples(groups, parents, dict(run, steps=Tp), n_cmp, max(1, min(16, cpu_cores())),
                                       plain_map)
        for prec in (32, 64):
            plain = ra.Replicas(groups, run["seed"], precision=prec, sample_every=S, max_windows=Tp // S,
                                tsf=True, plain=True, device=dev, noise_map=plain_map)

            def plain_pass():
                plain.init_chains(parent)
                plain.step(Tp)
                m, s, tm, ts = plain.average_forces(tsf=True)
                plain.bell_rates(m, run["k0"], run["x_dagger"], events=True)

            plain_pass()
            tp = time_once(plain_pass)
            plain.sync_status()
            pv = R * N * Tp / tp
            res = {"value": pv, "ms_per_step_extrapolated": 1e3 * tp * T / Tp, "speedup_fused_over_plain": value / pv}
            if plain_ref is not None:
                psmp, ptsmp = plain.samples(tsf=True)
                res["accuracy_vs_oracle"] = {
                    "rsf": accuracy(psmp[0][:, :n_cmp].cpu().numpy(), plain_ref[0], 1),
                    "tsf": accuracy(ptsmp[0][:, :n_cmp].cpu().numpy(), plain_ref[1], 1)}
                del psmp, ptsmp
            out["plain_path"]["fp%d" % prec] = res
            plain.close()
            log("plain large1000 FP%d: %.1f ms for %d steps (x%.0f extrapolated)" % (prec, 1e3 * tp, Tp, T / Tp))
        if cpu is not None:
            out["plain_path"]["fused_accuracy_same_windows"] = accuracy(got[:Tp // S], cpu["samples"][:Tp // S], 1)
    rep.close()

    if "fene50" in extras:
        out["fene50"] = fene50_bench(dev, args.noise_map)
        fracs["fene50"] = out["fene50"]["roofline_frac"]
    if "adjoint" in extras:
        out["adjoint"] = adjoint_bench(dev, args.noise_map)
        fracs["adjoint100_forward"] = out["adjoint"]["forward_roofline_frac"]
    if "batched" in extras:
        out["batched"] = batched_bench(dev, args.noise_map)
        fracs["batched512"] = out["batched"]["cost_model"]["roofline_frac"]
    for rname, rdesc in (("rsf50", "RSF cycle, FENE N=50 b=100, shear Wi=50, parent + 1000 replicas "
                                   "re-cloned every 750 steps, S=750, 20 windows, ISF/TSF/RSF, "
                                   "sigma(N_R=10,20,40,50), Bell rates and MFTU"),
                         ("collapsed50", "RSF cycle on the collapsed polymer without HI: N=50, harmonic "
                                         "backbone kappa=400 rest length 2, LJ u=1 between non-adjacent "
                                         "beads, shear 30, dt=1e-5, parent + 1000 replicas re-cloned every "
                                         "750 steps (S=0.0075), 20 windows, ISF/TSF/RSF, sigma(N_R), MFTU"),
                         ("hi50", "RSF cycle on the paper's full model: N=50, harmonic backbone kappa=400 "
                                  "rest length 2, LJ u=1, RPY hydrodynamic interaction a=1 (Cholesky noise "
                                  "every step), shear 30, dt=1e-5, parent + N_R=50 replicas re-cloned every "
                                  "750 steps, 4 windows, ISF/TSF/RSF, sigma(N_R), MFTU")):
        if rname in extras:
            # noise map 1 covers the chain model only (not the pair and HI models)
            out[rname] = rsf_cycle_bench(getattr(wl, rname)(), rdesc, dev, rname,
                                         args.noise_map if rname == "rsf50" else 0)
            fracs[rname + "_cycle"] = out[rname]["roofline"]["frac"]
            if not args.no_cpu_baseline:
                reps, wins = {"rsf50": (4, 20), "collapsed50": (2, 20), "hi50": (1, 4)}[rname]
                log("oracle %s cycle: %d replicas per thread, %d windows" % (rname, reps, wins))
                out[rname]["oracle"] = oracle_cycle_rates(getattr(wl, rname)(), max(1, min(16, cpu_cores())),
                                                          reps, wins)
                out[rname]["oracle"]["gpu_over_oracle"] = out[rname]["value"] / out[rname]["oracle"]["value"]
    if "sigma_sweep" in extras:
        out["sigma_sweep"] = sigma_sweep_bench(dev, args.noise_map)
    if "oracle_rates" in extras and not args.no_cpu_baseline:
        gpu = {}
        if "fene50" in out:
            gpu["fene50"] = out["fene50"]["value"]
        if "adjoint" in out:
            a100 = out["adjoint"]["every_100"]
            gpu["adjoint100_gradient"] = (out["adjoint"]["value"] * a100["backward_ms"]
                                          / (a100["backward_ms"] + a100["forward_ms"]))
        if "batched" in out:
            gpu["batched512_first16"] = out["batched"]["value"]
        out["oracle_rates"] = oracle_rates(max(1, min(16, cpu_cores())), args.noise_map, gpu)
        out["oracle_rates"]["note"] = ("gpu_value: fene50 whole pass; adjoint100 forward + backward (checkpoints "
                                       "every 100 steps); batched512: all 512 chains on the GPU against the "
                                       "oracle's per-bead-step rate on the first 16")
    out["roofline_fractions"] = {"slots_per_replica_bead_step": SLOTS_PER_BEAD_STEP, "frac": fracs}

    if args.copy_calibration:
        x = torch.empty(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        y = torch.empty_like(x)
        x.fill_(1.0)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
