"""Benchmark: replica-averaged Brownian dynamics on one MI355X.

Headline workload (one "step" = the whole hot path once):
  FENE chain, N = 50 beads, b = 100, uniaxial elongation at Wi = 2,
  dt = 1e-4, 1024 replicas cloned from one equilibrium parent,
  10^4 Euler-Maruyama steps, tension sampled every 100 steps (100 windows),
  FP32 state, FP64 replica mean/std, Bell rates k0 = 1e-6, x = 0.1.
  = ra_init_chains + ra_step(10^4) + ra_average_forces + ra_bell_rates,
  inputs (parent conformation) resident in HBM before the timed region.
  Noise map 1 (--noise-map, default 1): each Philox block gives four normals,
  three blocks serve four bead-steps; the oracle baseline draws the same.

value = replica*bead*steps per second (1024 * 50 * 10^4 per step / time).

Also reported, each measured once after warm-up: the plain unbatched GPU path
on the same workload (one launch per EM step, state in HBM; speedup), the
adjoint (N = 100, 4096 replicas, 2000 steps, checkpoints every 100), the
batched run (512 uneven FENE chains, one graph-captured persistent launch),
the 1000-bead transient (8192 replicas, 2e4 steps, RSF + TSF) and the RSF
sampling cycle (a parent trajectory re-cloned into 1000 replicas every 750
steps, 20 windows, with ISF/TSF/RSF, sigma(N_R) and MFTU) on the FENE chain,
on the paper's collapsed polymer (rest-length springs + LJ) and on the full
model with hydrodynamic interaction (parent + 50 replicas, 4 windows).
The roofline object is for the fused forward kernel; its time is taken with
HIP events on the stream the kernel runs on. cpu_baseline is the FP64 oracle
on a bounded sample of the same workload, on the host's cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "replica·bead·steps/s and adjoint steps/s vs plain GPU path at 1e-4 rel err"

# Peak VALU issue rate of one MI355X in lane-slots: 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz = 39.3 T lane-slots/s. One lane-slot is one lane of one full-rate
# VALU instruction (a wave64 instruction occupies a SIMD for 4 cycles); it is
# the published 157.3 TFLOP/s FP32 vector peak divided by 2 flops per FMA and
# by 2 for the packed FP32 forms, which integer work cannot use.
VALU_PEAK_LANE_SLOTS = 256 * 4 * 16 * 2.4e9
# Algorithmic lane-slots per replica*bead*step of the FENE forward step, at the
# issue cost of the gfx950 instruction that each operation needs (a
# transcendental occupies 2 slots, everything else 1):
#   Philox4x32-10: 10 rounds x (2 products 32x32->64 + 2 three-input XORs) = 40
#   uniform maps: 4 words x (exponent splice + subtract)                      =  8
#   Box-Muller: 2 log + 2 sqrt + 3 sin/cos (2 slots each) + 5 scalings        = 19
#   FENE bond update (spring law, flow, neighbour exchange, EM combine)      = 32
VALU_SLOTS_PER_BEAD_STEP_FENE = 40 + 8 + 19 + 32
# With noise map 1 a Philox block gives four normals and serves 4/3 bead-steps:
#   Philox 40 x 3/4 = 30; uniform maps 8 x 3/4 = 6; Box-Muller with both outputs
#   of the second pair, 2 log + 2 sqrt + 4 sin/cos (2 slots each) + 6 scalings
#   = 22 per block, x 3/4 = 16.5; FENE bond update 32
VALU_SLOTS_PER_BEAD_STEP_FENE_MAP1 = 30 + 6 + 16.5 + 32
# HBM bytes per launch of the forward kernel on the headline workload, read with
# rocprofv3 counters (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 KiB, both factors from
# a 1 GiB device copy). Valid only for the kernel sources they were taken on:
# the digest of those sources is recorded with the figure, and bench.py reports
# null when the sources have changed since.
FWD_TRAFFIC = {"sha256": "59e3a42a4fdb70ba6f5abdc9b5a3c9c26073053b867d8cb3bc54d0182f0d7ae7", "noise_map": 1,
               "bytes": (429.625 * 2.0 + 20592.0) * 1024}
FWD_SOURCES = ("ra_kernels.hip", "ra_chain.hpp", "ra_device.hpp", "ra_types.hpp", "ra_launch.hpp",
               "ra_host.cpp", "ra_tune.cpp", "ra_tune.hpp")


def fwd_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in FWD_SOURCES:
        with open(os.path.join(ROOT, "paper_2206_05851_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def cpu_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def cpu_baseline(groups, parents, run, n_replicas, noise_map=0):
    """FP64 oracle on replicas [0, n_replicas) of the headline workload, all
    steps, plus the replica averages and Bell rates (single thread)."""
    from oracle import ora
    g = dict(groups[0])
    t0 = time.perf_counter()
    o = ora.Oracle([g], run["seed"], run["sample_every"], run["steps"] // run["sample_every"],
                   noise_map=noise_map)
    o.set_replicas(0, 0, n_replicas)
    o.init_chains(parents)
    o.step(run["steps"])
    mean, std = o.average_forces()
    o.bell_rates(mean, run["k0"], run["x_dagger"])
    dt = time.perf_counter() - t0
    work = n_replicas * g["n_beads"] * run["steps"]
    return work / dt, dt, o.samples()[0]


def time_once(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


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
    rpar.close()
    rrep.close()
    log("%s: %.2f ms per cycle (%.1f us per window)" % (name, 1e3 * t, 1e6 * t / rW))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default="plain,adjoint,batched,large1000,rsf50,collapsed50,hi50",
                    help="comma-separated extra workloads to measure once")
    ap.add_argument("--cpu-replicas", type=int, default=384)
    ap.add_argument("--tile-policy", type=int, default=0,
                    help="ra_run_desc.tile_policy for the headline workload (0 = cost model)")
    ap.add_argument("--noise-map", type=int, default=1, choices=(0, 1),
                    help="ra_run_desc.noise_map of the headline, plain, adjoint, batched and rsf50 workloads "
                         "(1: four normals per Philox block)")
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
    groups, parents, run = wl.fene50()
    g = groups[0]
    R, N, T, S = g["n_replicas"], g["n_beads"], run["steps"], run["sample_every"]
    W = T // S
    parent = torch.from_numpy(np.ascontiguousarray(parents[0]).reshape(-1)).to(dev)
    rep = ra.Replicas(groups, run["seed"], precision=32, sample_every=S, max_windows=W, device=dev,
                      tile_policy=args.tile_policy, noise_map=args.noise_map)
    slots = VALU_SLOTS_PER_BEAD_STEP_FENE_MAP1 if args.noise_map else VALU_SLOTS_PER_BEAD_STEP_FENE
    mean = torch.empty((W, N - 1), dtype=torch.float64, device=dev)
    std = torch.empty_like(mean)
    stream = torch.cuda.current_stream()
    ev = []

    def one_step(record):
        rep.init_chains(parent)
        if record:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        rep.step(T)
        if record:
            e1.record(stream)
            ev.append((e0, e1))
        rep.average_forces(out=(mean, std))
        return rep.bell_rates(mean, run["k0"], run["x_dagger"])

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        one_step(False)
    rep.sync_status()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rates, rsum = one_step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    rep.sync_status()
    work_per_step = R * N * T
    value = work_per_step * args.steps / elapsed
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    achieved = slots * work_per_step / (kernel_ms * 1e-3)
    log("fused: %.3f ms/step, kernel %.3f ms, %.3e replica-bead-steps/s" %
        (1e3 * elapsed / args.steps, kernel_ms, value))
    gpu_samples = rep.samples()[0]
    tiles = rep.tile_info()
    family = rep.kernel_family()
    traffic = (FWD_TRAFFIC["bytes"] if family == 4 and args.tile_policy == 0
               and args.noise_map == FWD_TRAFFIC.get("noise_map", 0)
               and fwd_sources_digest() == FWD_TRAFFIC["sha256"] else None)
    kernel_name = {4: "fwd_kernel<float,4,1,%d>" % args.noise_map,
                   16: "fwd_kernel<float,16,2,0>"}[family]

    out = {
        "metric": METRIC, "value": value, "unit": "replica·bead·steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded FENE equilibrium parent; Philox noise, noise map %d)" % args.noise_map,
        "config": {"workload": "fene50: FENE N=50 b=100, uniaxial Wi=2 (rate=%.6g), dt=1e-4, "
                               "R=1024, 10^4 steps, sample every 100, FP64 averages, Bell rates"
                               % g["rate"],
                   "global_batch": R, "seq_len": N, "parallelism": "none (1 GPU)",
                   "beads_per_lane": tiles[0][0], "replicas_per_wave": tiles[1][0],
                   "kernel_family": family, "noise_map": args.noise_map},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_LANE_SLOTS / 1e12,
                     "unit": "T VALU lane-slots/s", "frac": achieved / VALU_PEAK_LANE_SLOTS,
                     "traffic": traffic, "kernel": kernel_name, "kernel_ms": kernel_ms,
                     "lane_slots_per_replica_bead_step": slots},
    }

    extras = set() if args.no_extras else set(x for x in args.extras.split(",") if x)
    if "plain" in extras:
        # plain unbatched path, same workload and counters
        plain = ra.Replicas(groups, run["seed"], precision=32, sample_every=S, max_windows=W,
                            plain=True, device=dev, noise_map=args.noise_map)
        pm = torch.empty_like(mean)
        ps = torch.empty_like(mean)

        def plain_step():
            plain.init_chains(parent)
            plain.step(T)
            plain.average_forces(out=(pm, ps))
            plain.bell_rates(pm, run["k0"], run["x_dagger"])

        plain_step()
        tp = min(time_once(plain_step) for _ in range(2))
        plain.sync_status()
        diff = torch.max(torch.abs(pm - mean) / mean).item()
        out["plain_path"] = {"value": work_per_step / tp, "ms_per_step": 1e3 * tp,
                             "speedup_fused_over_plain": (work_per_step / (elapsed / args.steps)) /
                             (work_per_step / tp),
                             "max_rel_diff_profile_vs_fused": diff}
        plain.close()
        log("plain: %.3f ms/step" % (1e3 * tp))

    if "adjoint" in extras:
        ag, ap_, arun = wl.adjoint100()
        ga = ag[0]
        apar = torch.from_numpy(np.ascontiguousarray(ap_[0]).reshape(-1)).to(dev)
        adj = ra.Replicas(ag, arun["seed"], precision=32, sample_every=arun["sample_every"],
                          max_windows=arun["steps"] // arun["sample_every"],
                          checkpoint_every=arun["checkpoint_every"], max_steps=arun["steps"], device=dev,
                          noise_map=args.noise_map)
        gm = torch.ones((arun["steps"] // arun["sample_every"], ga["n_beads"] - 1),
                        dtype=torch.float64, device=dev)

        def adj_fwd():
            adj.init_chains(apar)
            adj.step(arun["steps"])

        def adj_bwd():
            m, _ = adj.average_forces()
            return adj.backward(m, gm, None)

        adj_fwd()
        adj_bwd()
        tf = time_once(adj_fwd)
        tb = time_once(adj_bwd)
        adj.sync_status()
        adj.close()
        # the same gradient with the library's automatic checkpoint interval:
        # the 2001 states (9.8 GB) fit in HBM, so every state is kept and the
        # backward recomputes nothing
        adj = ra.Replicas(ag, arun["seed"], precision=32, sample_every=arun["sample_every"],
                          max_windows=arun["steps"] // arun["sample_every"],
                          checkpoint_every=ra.CKPT_AUTO, max_steps=arun["steps"], device=dev,
                          noise_map=args.noise_map)
        adj_fwd()
        adj_bwd()
        tf1 = time_once(adj_fwd)
        tb1 = time_once(adj_bwd)
        k_auto = adj.checkpoint_interval()
        adj.sync_status()
        adj.close()
        awork = ga["n_replicas"] * ga["n_beads"] * arun["steps"]
        out["adjoint"] = {"workload": "adjoint100: FENE N=100 b=100, uniaxial Wi=4, R=4096, dt=1e-4, "
                                      "2000 steps, checkpoints every 100",
                          "value": awork / tb, "unit": "replica·bead·steps/s (backward incl. recompute)",
                          "forward_value": awork / tf, "backward_ms": 1e3 * tb, "forward_ms": 1e3 * tf,
                          "auto_interval": {"checkpoint_every": k_auto, "value": awork / tb1,
                                            "forward_value": awork / tf1, "backward_ms": 1e3 * tb1,
                                            "forward_ms": 1e3 * tf1}}
        log("adjoint: fwd %.2f ms bwd %.2f ms; automatic interval %d: fwd %.2f ms bwd %.2f ms"
            % (1e3 * tf, 1e3 * tb, k_auto, 1e3 * tf1, 1e3 * tb1))

    if "batched" in extras:
        # batched uneven chains, one graph-captured persistent launch per call
        bg, bp, brun = wl.batched512()
        bpar = torch.from_numpy(np.concatenate([np.ascontiguousarray(p).reshape(-1) for p in bp])).to(dev)
        bat = ra.Replicas(bg, brun["seed"], precision=32, sample_every=brun["sample_every"],
                          max_windows=brun["steps"] // brun["sample_every"], use_graph=True, device=dev,
                          noise_map=args.noise_map)

        def bat_step():
            bat.init_chains(bpar)
            bat.step(brun["steps"])
            m, s = bat.average_forces()
            bat.bell_rates(m, brun["k0"], brun["x_dagger"])

        bat_step()
        tbat = min(time_once(bat_step) for _ in range(2))
        bat.sync_status()
        bat.close()
        # the same batch with tiles chosen by the timing autotuner (each chain
        # length timed alone on 256 replicas) instead of the cost model
        bat = ra.Replicas(bg, brun["seed"], precision=32, sample_every=brun["sample_every"],
                          max_windows=brun["steps"] // brun["sample_every"], use_graph=True, device=dev,
                          tile_policy=1, noise_map=args.noise_map)
        bat_step()
        ttun = min(time_once(bat_step) for _ in range(2))
        bat.sync_status()
        bat.close()
        bwork = sum(x["n_replicas"] * x["n_beads"] for x in bg) * brun["steps"]
        out["batched"] = {"workload": "batched512: 512 FENE chains N~U{20..200}, b~U[50,200], planar "
                                      "Wi~U[0.5,5] / shear Wi~U[1,50], R~U{16..256}, 5000 steps",
                          "value": bwork / tbat, "ms_per_step": 1e3 * tbat, "graph": True,
                          "tiles": "cost model", "autotuned_tiles_ms_per_step": 1e3 * ttun}
        log("batched: %.2f ms (cost-model tiles), %.2f ms (autotuned tiles)" % (1e3 * tbat, 1e3 * ttun))

    if "large1000" in extras:
        # 1000-bead transient with TSF
        lg, lp, lrun = wl.large1000()
        lpar = torch.from_numpy(np.ascontiguousarray(lp[0]).reshape(-1)).to(dev)
        big = ra.Replicas(lg, lrun["seed"], precision=32, sample_every=lrun["sample_every"],
                          max_windows=lrun["steps"] // lrun["sample_every"], tsf=True, device=dev)

        def big_step():
            big.init_chains(lpar)
            big.step(lrun["steps"])
            m, s, tm, ts = big.average_forces(tsf=True)
            big.bell_rates(m, lrun["k0"], lrun["x_dagger"], events=True)

        big_step()
        tbig = time_once(big_step)
        big.sync_status()
        lwork = lg[0]["n_replicas"] * lg[0]["n_beads"] * lrun["steps"]
        out["large1000"] = {"workload": "large1000: FENE N=1000 b=400, start-up uniaxial Wi=10, R=8192, "
                                        "dt=5e-5, 2e4 steps, RSF+TSF windows of 500, Bell events",
                            "value": lwork / tbig, "ms_per_step": 1e3 * tbig}
        big.close()
        log("large1000: %.1f ms" % (1e3 * tbig))

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

    if args.copy_calibration:
        x = torch.empty(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        y = torch.empty_like(x)
        x.fill_(1.0)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    if not args.no_cpu_baseline:
        nr = args.cpu_replicas
        log("cpu baseline: oracle on %d replicas x %d steps" % (nr, T))
        rate, secs, ref = cpu_baseline(groups, parents, run, nr, args.noise_map)
        got = gpu_samples[:, :nr].cpu().numpy()
        rel = np.abs(got - ref) / np.abs(ref)
        err = float(np.max(rel))
        # the accuracy gate: replica-averaged forces over windows of at most
        # 200 steps (and the profile of the same replicas over the whole run)
        prof = np.abs(got.mean(axis=1) - ref.mean(axis=1)) / np.abs(ref.mean(axis=1))
        out["max_rel_err_vs_oracle_profile_first_200_steps"] = float(np.max(prof[:200 // S]))
        out["max_rel_err_vs_oracle_profile"] = float(np.max(prof))
        out["max_rel_err_vs_oracle_samples_first_200_steps"] = float(np.max(rel[:200 // S]))
        out["cpu_baseline"] = {"value": rate, "unit": "replica·bead·steps/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "FP64 oracle, replicas 0..%d of 1024, all 10^4 steps, averages and "
                                         "Bell rates, single thread (%.1f s; host has %d cores)"
                                         % (nr - 1, secs, cpu_cores())}
        out["max_rel_err_vs_oracle"] = err   # every sample of every window of the 10^4 steps
        log("cpu: %.3e replica-bead-steps/s, GPU vs oracle max rel err %.2e (samples), %.2e (profile)"
            % (rate, err, out["max_rel_err_vs_oracle_profile"]))

    rep.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
