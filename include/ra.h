/*
 * ra.h — C ABI of the MI355X (gfx950) replica-averaged Brownian-dynamics library.
 *
 * Method (Kania, Nguyen, Oztekin, Webb, "Replica-Averaging: An algorithm to
 * study mechano-reactive processes for polymers under flow conditions"):
 *   - a parent bead-spring chain is halted and cloned into N_R replicas,
 *     each driven by its own random stream (RSF description, Sec. II);
 *   - every replica is advanced by the Brownian-dynamics update of Eq. (1),
 *     here with only the self term of the diffusion tensor, Eq. (2)
 *     (free-draining), under a homogeneous flow v = kappa . r;
 *   - after an evolution time S the tension of each spring (Eq. (4): signed
 *     for the rest-length spring, the magnitude for zero-rest-length Hookean
 *     and FENE springs) is sampled once per replica
 *     and averaged over replicas (RSF); optionally it is also averaged over
 *     the steps of the window (TSF, Sec. II);
 *   - the averaged tension feeds a Bell-type rate k = k0 exp(x_dagger f/kT)
 *     (Sec. III, the A2-domain unfolding rate law).
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers (hipMalloc'd or torch CUDA tensors)
 *     unless marked "host". The caller owns every argument buffer; the
 *     library owns the context, chain state, samples and checkpoints.
 *   - Work is enqueued on the stream given to ra_create and is asynchronous:
 *     outputs are valid after that stream is synchronised. Calls on one
 *     context must not overlap from several host threads.
 *   - Errors are returned as ra_status codes, never by exit or exception;
 *     ra_last_error returns a text for the last failure on a context.
 *     Errors found on the device (an invalid parent chain, a non-finite
 *     tension) are latched in the context and reported by ra_sync_status.
 *   - Layout of a profile: [window][spring], springs of all groups
 *     concatenated in group order, sum_g (N_g - 1) per window, FP64.
 *   - Spring j of a chain joins beads j and j+1 (0-based), N-1 springs.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key =
 *     (seed low, seed high) and counter = (step, bead, replica,
 *     tag<<24 | stream_id); tag 0 drives replica noise, tag 1 a parent
 *     trajectory (noise_tag = 1), tag 2 Bell events.
 *     A group's results depend only on its descriptor, its parent, the seed
 *     and the step count: never on which other groups share the context.
 */
#ifndef RA_H
#define RA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RA_API __attribute__((visibility("default")))

typedef struct ra_ctx ra_ctx;

#define RA_CKPT_AUTO (-1)   /* ra_run_desc.checkpoint_every: choose the interval (see there) */

typedef enum {
    RA_OK = 0,
    RA_EINVAL = -1,     /* invalid argument or descriptor; nothing changed */
    RA_ENOMEM = -2,     /* device or host allocation failed */
    RA_EDEVICE = -3,    /* a HIP call failed (text in ra_last_error) */
    RA_EUNSTABLE = -4,  /* a sampled tension was NaN/Inf */
    RA_ESTATE = -5      /* call out of order (e.g. ra_step before ra_init_chains) */
} ra_status;

typedef enum { RA_HOOKEAN = 0, RA_FENE = 1, RA_HARMONIC = 2 } ra_spring;
typedef enum { RA_QUIESCENT = 0, RA_UNIAXIAL = 1, RA_PLANAR = 2, RA_SHEAR = 3 } ra_flow;

/* One group = one parent chain and its replicas (host struct, 112 bytes).
 * Spring force on bead j from spring j: F = H g Q, Q = r_{j+1} - r_j, with
 *   Hookean  g = 1, tension f = H |Q|;
 *   FENE     g = 1/(1 - min(|Q|^2/Q0^2, 1 - 1e-3)), Q0^2 = b kT/H, f = H g |Q|;
 *   HARMONIC g = 1 - r0/|Q| (rest length r0, the Sec. II backbone spring
 *            kappa/2 (r - 2a)^2 with kappa = H), signed tension f = H (|Q| - r0)
 *            (Eq. 4).
 * Optional Lennard-Jones self-association between non-adjacent beads
 * (|i - j| >= 2, Sec. II): U = lj_eps [(lj_rmin/r)^12 - 2 (lj_rmin/r)^6].
 * Groups with a HARMONIC spring or lj_eps > 0 run the pair-interaction kernel
 * (N <= 64, no adjoint); a context holds either only such groups or none.
 * Hydrodynamic interaction (hi_radius = a > 0): D_ii = kT/zeta I (Eq. 2, zeta
 * = 6 pi eta a), D_ij the RPY tensor of Eq. 3, drift dt D F / kT and random
 * displacement sqrt(2 dt) L xi with D = L L^T (Cholesky) every step; any spring
 * law and LJ; one workgroup per replica (N <= 64 within the device's LDS per
 * workgroup: 3N(3N+1)/2 + 1024 elements); a context holds only HI groups or
 * none; no adjoint, no plain path.
 * Flow: uniaxial kappa = rate*diag(1,-1/2,-1/2); planar rate*diag(1,-1,0);
 * shear v_x = rate * z (the paper's convention, Sec. II). */
typedef struct {
    int32_t  n_beads;      /* N, 2 <= N <= 1024 (FP64 fused: N <= 256; pair and HI kernels: N <= 64) */
    int32_t  n_replicas;   /* R >= 1 */
    int32_t  spring;       /* ra_spring */
    int32_t  flow;         /* ra_flow */
    double   H;            /* spring constant > 0 */
    double   b;            /* FENE extensibility > 0 (FENE only) */
    double   rate;         /* strain rate or shear rate (not a Weissenberg number) */
    double   kT;           /* thermal energy > 0 */
    double   zeta;         /* bead friction > 0 */
    double   dt;           /* time step > 0 */
    double   noise_scale;  /* 1 = physical noise; 0 = deterministic */
    double   rest_length;  /* HARMONIC rest length r0 >= 0 (ignored otherwise) */
    double   lj_eps;       /* LJ well depth >= 0 (0 = no LJ) */
    double   lj_rmin;      /* LJ minimum position > 0 when lj_eps > 0 */
    double   hi_radius;    /* bead radius a of the RPY tensor (Eqs. 2-3); 0 = free draining */
    uint32_t stream_id;    /* group id in the random counter, < 2^24 */
    uint32_t pad_;
} ra_chain_desc;

/* Run options (host struct, 56 bytes). */
typedef struct {
    uint64_t seed;              /* Philox key */
    int32_t  precision;         /* 32: FP32 state, FP64 averages; 64: all FP64 */
    int32_t  sample_every;      /* S >= 1: sample after every S-th step */
    int32_t  max_windows;       /* capacity of the per-replica sample store, 0..65535 */
    int32_t  tsf;               /* 1: also keep per-replica window time averages */
    int32_t  checkpoint_every;  /* K > 0 enables ra_backward (precision 32 only), keeping the
                                   state every K steps; RA_CKPT_AUTO: every step when the
                                   trajectory, (max_steps + 1) states, fits in a quarter of
                                   the free device memory, else every ceil(sqrt(max_steps)) */
    int32_t  max_steps;         /* steps since ra_init_chains the checkpoints must hold */
    int32_t  plain;             /* 1: plain path, one launch per step, state in HBM */
    int32_t  use_graph;         /* 1: capture ra_step's launch sequence in a hipGraph */
    int32_t  tile_policy;       /* 0 cost model; 1 autotune by timing; 1000 + m: force
                                   m beads per lane where legal (m <= 16) */
    int32_t  waves_per_block;   /* 0 = default (4) */
    int32_t  noise_tag;         /* 0: replica noise; 1: parent trajectory (RSF cycle, Sec. II) */
    int32_t  noise_map;         /* 0: one Philox block per (step, bead), three normals;
                                   1: each block gives four normals (both of Box-Muller's
                                   second pair): steps 4m..4m+2 use the first three of
                                   their own block, step 4m+3 the fourth normals of those
                                   three blocks (three blocks per four steps). Chain
                                   model only, at most 4 beads per lane (FP32 N <= 256);
                                   2: the beads of a step in groups of four, bead 4q + r
                                   takes normal r of the blocks with bead word 3q + c as
                                   its component c (three blocks per four beads). Chain
                                   model only, fused path with 8-16 beads per lane (FP32,
                                   a group with N > 256) or the plain path */
} ra_run_desc;

/* Create a context: validates every descriptor (RA_EINVAL with nothing
 * allocated on any violation), chooses a tile per group, allocates all device
 * memory it will use, and records the HIP stream (NULL = null stream). */
RA_API ra_status ra_create(ra_ctx** out, const ra_chain_desc* groups, int32_t n_groups,
                           const ra_run_desc* run, void* hip_stream);

/* RSF clone (Sec. II): every replica of group g starts from its parent.
 * parent_xyz: device FP64, N_g*3 values per group (x,y,z per bead), groups
 * concatenated. Resets the step counter, windows, TSF sums and guard counts.
 * A FENE bond with |Q| >= Q0 or a non-finite coordinate is detected on the
 * device; ra_sync_status then returns RA_EINVAL and ra_step does no work. */
RA_API ra_status ra_init_chains(ra_ctx* ctx, const double* parent_xyz);

/* Advance every replica of every group by n_steps Euler-Maruyama steps of
 * Eq. (1) (free-draining, Eq. (2)), sampling spring tensions after each
 * step whose 1-based index since init is a multiple of S. Fails with
 * RA_EINVAL if the window capacity, the checkpoint capacity or 2^32 total
 * steps would be exceeded. */
RA_API ra_status ra_step(ra_ctx* ctx, int64_t n_steps);

/* RSF estimate (Sec. II): replica mean of the sampled tensions and their
 * replica standard deviation (denominator R-1; 0 when R = 1), FP64, for all
 * windows sampled since init. mean/std: device [W][sum_g(N_g-1)]; tsf_mean,
 * tsf_std the same for the window time averages (need tsf=1). Any output may
 * be NULL. n_windows (host, may be NULL) receives W. */
RA_API ra_status ra_average_forces(ra_ctx* ctx, double* mean, double* std,
                                   double* tsf_mean, double* tsf_std, int64_t* n_windows);

/* Bell-type rates (Sec. III): rates[w][s] = k0 exp(x_dagger mean[w][s] / kT_g),
 * rate_sum[w][g] = sum over the springs of group g (its inverse is the mean
 * first-passage time to any event). events[w][s] (uint8, may be NULL) = 1
 * with probability 1 - exp(-rates * S * dt_g), from one tag-2 Philox block per
 * (window, spring, group): counter (w, j, 0, 2<<24 | stream_id), uniform
 * u = (2m + 1) 2^-53 from the top 52 bits m of its first two words (hi:lo). mean: device [n_windows][sum_g(N_g-1)]. */
RA_API ra_status ra_bell_rates(ra_ctx* ctx, const double* mean, int64_t n_windows,
                               double k0, double x_dagger, double* rates,
                               double* rate_sum, uint8_t* events);

/* Pathwise adjoint with the noise held fixed: gradient of
 *   J = sum_{w,s} grad_mean[w][s] * mean[w][s] + sum_{w,s} grad_rates[w][s] * rates[w][s]
 * with respect to (rate, H, b) of every group, through all steps since init.
 * mean: the profile from ra_average_forces (device, used for the rates term);
 * grad_rates may be NULL; grad_params: device FP64 [n_groups][3]. Needs
 * checkpoint_every != 0; replays each K-step segment from its checkpoint
 * (with K = 1 it reads every state and recomputes only the last step).
 * FENE springs on the guard are treated as having ds = 0. */
RA_API ra_status ra_backward(ra_ctx* ctx, const double* mean, const double* grad_mean,
                             const double* grad_rates, double k0, double x_dagger,
                             double* grad_params);

/* RSF re-clone (Sec. II): at a force-sampling time the parent chain is halted
 * and every replica of group g restarts from the current state of group g's
 * first chain in `parent` (a context with the same groups and chain lengths,
 * normally one chain per group and noise_tag = 1, same precision, fused path).
 * The context's step count must be a multiple of S and is kept: the replicas
 * of window w continue with counters (w*S + s, bead, replica, group),
 * distinct from every other window's, and earlier windows stay available to
 * ra_average_forces. The context must have been created but need not have
 * been initialised. Stream-ordered after the parent's queued work when both
 * contexts use the same stream; otherwise the caller orders the two streams
 * (ra_rsf_cycle does). The re-cloned conformation becomes the reference of
 * ra_conformation. After a re-clone ra_backward returns RA_ESTATE until the
 * next ra_init_chains. */
RA_API ra_status ra_reclone(ra_ctx* ctx, const ra_ctx* parent);

/* The RSF sampling cycle (Sec. II) for n_windows windows, continuing from the
 * windows already sampled: per window the parent context advances
 * parent_steps steps (its sample_every must equal parent_steps, so each
 * window also records the parent's instantaneous tensions (ISF) and, with
 * tsf = 1, their time average over the window (TSF)); the replicas are
 * re-cloned from it and evolve S steps; their tensions are sampled once at the
 * end (RSF). When the two contexts have different streams, the parent's next
 * window overlaps the replicas' current one (ordered by HIP events). Capacity
 * of both contexts is checked before anything is enqueued. */
RA_API ra_status ra_rsf_cycle(ra_ctx* ctx, ra_ctx* parent, int64_t n_windows, int64_t parent_steps);

/* Spread of the RSF estimate for N_R = block replicas (Figs. 2 and 5): per
 * window and spring, the R replicas of a group are split into
 * B = floor(R/block) consecutive blocks, each block mean is one RSF estimate,
 * and sigma = their standard deviation (denominator B-1; 0 when B < 2).
 * sigma: device FP64 [W][sum_g(N_g-1)]; block >= 1. */
RA_API ra_status ra_block_sigma(ra_ctx* ctx, int32_t block, double* sigma);

/* Mean first-passage time to any event on a chain (MFTU, Sec. III, Table 1):
 * mftu[g] = 1 / (mean over the n_windows windows of rate_sum[w][g]), the mean
 * of an exponential first-event time with the run-averaged total rate.
 * rate_sum: device FP64 [n_windows][n_groups] from ra_bell_rates; mftu: device
 * FP64 [n_groups]; n_windows >= 1. */
RA_API ra_status ra_mftu(ra_ctx* ctx, const double* rate_sum, int64_t n_windows, double* mftu);

/* MFTU by sampling unfolding events (Sec. III, Table 1), for n_trials
 * independent trials per group: window v = 0, 1, ... of a trial carries the
 * rates of sampled window v mod n_windows (the rate profile repeats), and
 * spring j of group g unfolds in window v when the tag-2 53-bit uniform of counter
 * (v, j, trial, 2<<24 | stream_id) is below 1 - exp(-rates[v mod W][j] S dt_g)
 * (trial 0 over the sampled windows draws exactly ra_bell_rates's events). A
 * trial's first-passage time is the end of its first window with any
 * unfolding, (v + 1) S dt_g; a trial with none in max_windows windows is
 * censored at max_windows S dt_g. mftu[g] = (sum of all trials' times) /
 * (number of trials with an event), the censored maximum-likelihood mean of an
 * exponential waiting time (+Inf when no trial has an event); for a constant
 * total rate K it estimates S dt / (1 - exp(-K S dt)) = 1/K + S dt/2 + ...
 * rates: device FP64 [n_windows][sum_g(N_g-1)] from ra_bell_rates;
 * first_window: device int64 [n_trials][n_groups] (first window or -1);
 * mftu: device FP64 [n_groups]. 1 <= n_trials <= 65535, 1 <= max_windows < 2^32. */
RA_API ra_status ra_mftu_events(ra_ctx* ctx, const double* rates, int64_t n_windows, int32_t n_trials,
                                int64_t max_windows, int64_t* first_window, double* mftu);

/* Replica fidelity (Sec. IV, Eq. 5) and radius of gyration, from the current
 * state of every replica, in the centre-of-mass frame:
 *   dbar[q][a]   = (1/N) sum_i |rhat_a^i(q) - rhat_a^i(source)|,
 *   d_bead[b][a] = the same term for one bead, b = (replica, bead) flattened,
 *   rg2[q][a]    = (1/N) sum_i rhat_a^i(q)^2 (a = z gives R_Gz^2),
 *   src_rg2[g][a] likewise for group g's source conformation,
 * where source is the conformation of the last ra_init_chains or ra_reclone
 * and q runs over all replicas, groups concatenated. Device FP64 outputs
 * [sum_g R_g][3], [sum_g R_g N_g][3], [sum_g R_g][3], [n_groups][3]; any may
 * be NULL. Fused path only. */
RA_API ra_status ra_conformation(ra_ctx* ctx, double* dbar, double* d_bead, double* rg2, double* src_rg2);

/* Synchronise the context's stream and report device-side errors:
 * RA_EINVAL (invalid parent), RA_EUNSTABLE (non-finite tension, or a
 * non-positive pivot in the Cholesky factorization of the RPY tensor of a
 * hydrodynamic-interaction group) or RA_OK. */
RA_API ra_status ra_sync_status(ra_ctx* ctx);

/* Host copy of the per-group FENE guard counts (synchronises). out: host int64[n_groups]. */
RA_API ra_status ra_guard_counts(ra_ctx* ctx, int64_t* out);

/* Per-replica tension samples since init, device FP64
 * [W][sum_g R_g (N_g-1)] ([replica][spring] per group); tsf_out likewise. */
RA_API ra_status ra_get_samples(ra_ctx* ctx, double* out, double* tsf_out);

/* Current bond vectors Q_j = r_{j+1} - r_j of every replica, device FP64
 * [sum_g R_g (N_g-1) 3]. */
RA_API ra_status ra_get_bonds(ra_ctx* ctx, double* out);

/* The checkpoint interval in use (RA_CKPT_AUTO resolved at ra_create; 0 when
 * the context keeps no checkpoints). With an interval of 1 ra_backward reads
 * every step's state instead of recomputing it. */
RA_API ra_status ra_checkpoint_interval(ra_ctx* ctx, int32_t* steps);

/* Tile chosen per group (host int32[n_groups] each): beads per lane and
 * replicas per wavefront; kernel_family (host int32[1], may be NULL): 2 = the
 * pair-interaction kernel (one bead per lane; LJ and rest-length springs),
 * 3 = hydrodynamic-interaction kernel (one workgroup per replica), 4 = 1-4
 * beads per lane, 16 = 6-16 beads per lane, 0 = plain path. */
RA_API ra_status ra_tile_info(ra_ctx* ctx, int32_t* beads_per_lane, int32_t* replicas_per_wave,
                              int32_t* kernel_family);

/* Noise stream check: for n counters (device uint32 [n][4]) and key = seed,
 * writes the Philox words (device uint32 [n][4]) and the three normals in
 * FP32 and FP64 (device [n][3]); NULL outputs are skipped. Uses the same
 * device functions as the simulation kernels. */
RA_API ra_status ra_debug_noise(const uint32_t* counters, int64_t n, uint64_t seed,
                                uint32_t* words, float* normals32, double* normals64,
                                void* hip_stream);

/* Allocation-free run, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): for one chain group (Hookean or FENE, no LJ, no HI) it does what
 * ra_create + ra_init_chains + ra_step(n_steps) + ra_average_forces do, with
 * the same kernels and bit-identical mean and std, but keeps its descriptors,
 * counters, bond state and per-replica samples in a static device array of
 * RA_STATIC_SCRATCH_MAX bytes instead of allocating. It calls no allocating
 * routine (the array's device address is looked up once per device, on the
 * first call there, with hipGetSymbolAddress).
 *   group, run: host structs as for ra_create; run must select the fused path
 *     without TSF, checkpoints, graph capture, autotuning (tile_policy 0 or
 *     1000 + m) or the parent noise tag; run->max_windows is ignored.
 *   parent_xyz: device FP64 [N][3]; n_steps: a positive multiple of
 *     sample_every (W = n_steps / sample_every windows, W <= 65535).
 *   mean, std: device FP64 [W][N-1] (either may be NULL, not both).
 *   Scratch needed: R (N-1) (3 + W) values of the state precision plus ~2 KB;
 *     RA_EINVAL (text in ra_last_error(NULL)) if it exceeds the limit.
 *   Errors found on the device (an invalid parent, a non-finite tension)
 *     set every element of mean and std to NaN.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (each call rewrites what it reads): calls that overlap on
 * one device, from several streams or host threads, race. */
#define RA_STATIC_SCRATCH_MAX (64ll << 20)
RA_API ra_status ra_run_static(const ra_chain_desc* group, const ra_run_desc* run, const double* parent_xyz,
                               int64_t n_steps, double* mean, double* std, void* hip_stream);

RA_API const char* ra_last_error(const ra_ctx* ctx);
RA_API void ra_destroy(ra_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
