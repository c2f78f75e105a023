// ra_kernels.hip — gfx950 kernels of the replica-averaged BD library.
//
// Fused forward path (one launch per ra_step):
//   one wavefront per work item = P replicas of one group; a replica occupies
//   L = ceil(N/M) consecutive lanes, lane t holding beads/springs
//   [t*M, t*M + M). The chain lives in VGPRs as bond vectors Q_j = r_{j+1} - r_j
//   for the whole time loop; neighbour springs and neighbour-bead noise come
//   from the adjacent lane by DPP wave shifts. Every slot past the last spring
//   of a replica holds Q = 0 (so its force is 0), which makes the chain ends
//   and the seams between packed replicas need no extra masking.
// The step itself (bond form of Eq. (1) with Eq. (2)) is in ra_chain.hpp.
#include "ra_chain.hpp"
#include "ra_launch.hpp"

namespace ra {

// ---------------------------------------------------------------------------
// Fused persistent forward: all n_steps of one work item in registers.
// ---------------------------------------------------------------------------
// Noise run-ahead per beads-per-lane: with one bead per lane the wave has
// little independent work per step, so U steps of noise (U independent Philox
// chains per lane) are generated before the U physics steps consume them.
template <int M> struct RunAhead { static constexpr int U = M == 1 ? 4 : (M == 2 ? 2 : 1); };

// Fused persistent forward over all n_steps of one work item. The step loop is
// cut into segments between events (window end, checkpoint), so the inner
// loop holds nothing but noise generation and the bond update (plus the
// per-step tension sum when TSF is on).
template <typename T, int M, bool FENE, bool UNIFORM_K, bool TSF, int NMAP>
__device__ __forceinline__ void run_forward_impl(const FwdArgs& a, const GroupDev& G, int gidx, int k_first,
                                                 int64_t n0_64) {
    constexpr int U = RunAhead<M>::U;
    // Kernel arguments are read once into locals: the step lambdas below must
    // not take the address of the by-value argument block (that would copy it
    // to scratch memory).
    const int S = a.S, K = a.K;
    const int64_t smp_total = a.smp_total, state_total = a.state_total;
    T* const state = (T*)a.state;
    int32_t* const status = a.status;
    unsigned long long* const clamp_ctr = a.clamps + gidx;
    const int n_steps = (int)a.n_steps;
    const TileGeom tg = tile_geom<UNIFORM_K>(G, k_first, M);
    const RoundKeys keys = round_keys(a.key0, a.key1);
    Lane<T, M> s;
    bool valid[M];
    load_lane<T, M>(s, valid, state, G, tg);
    const SlotCoef<T, M> kc = slot_coef<T, M>(G, valid);
    const int nm1 = G.N - 1;
    const uint32_t n0 = (uint32_t)n0_64;       // total steps stay below 2^32
    const uint32_t bead0 = (uint32_t)tg.j0, rep = (uint32_t)tg.k;
    // per-lane output cursors, bumped once per window / checkpoint
    const int64_t lane_off = G.smp_off + (int64_t)tg.k * nm1 + tg.j0;
    T* smp_w = (T*)a.samples + (int64_t)(n0 / (uint32_t)S) * smp_total + lane_off;
    T* tsf_w = TSF ? (T*)a.tsf + (int64_t)(n0 / (uint32_t)S) * smp_total + lane_off : nullptr;
    const int64_t ckpt_total = a.ckpt_total;
    T* ck_w = K > 0 ? ckpt_item<T, M>((T*)a.ckpt, G, k_first) + (int64_t)((n0 + (uint32_t)K - 1) / (uint32_t)K) * ckpt_total
                    : nullptr;
    double* const tacc_g = TSF ? a.tsf_acc + lane_off : nullptr;
    int to_smp = S - (int)(n0 % (uint32_t)S);                              // steps to the next window end
    int to_ck = K > 0 ? (int)((K - (int)(n0 % (uint32_t)K)) % K) : INT32_MAX;  // steps to the next checkpoint
    // TSF: each step's force evaluation adds the tension of the state it
    // starts from (slot_force), so a window's states n+1 .. n+S are the
    // evaluations of steps n+1 .. n+S-1 plus the window-end state, which the
    // sample computes anyway; the evaluation of step n (the previous window's
    // last state) is cancelled by starting the sum at minus that tension.
    // The sums stay in registers over at most TSF_FLUSH steps and are folded
    // into the FP64 window sum in global memory only when a window is longer
    // or continues in a later launch. Tensions are nonnegative, so a register
    // sum of at most 512 terms (and the one cancelled term) carries a relative
    // error of a few hundred ulp at most (below 3.1e-5).
    constexpr int TSF_FLUSH = 512;
    // 6-16 beads per lane under noise map 0 keep the separate tension pass after
    // each step: their register budget (two wavefronts per SIMD) has no room for
    // the fused sums beside sixteen Philox chains. Under map 2 (twelve chains)
    // the fused sums fit; the spills they cause sit outside the step loop, and
    // the 16-bead kernel is 4% faster than with the separate pass.
    constexpr bool FUSED = TSF && (M <= 4 || NMAP == 2);
    T tpart[M];
    T* const tsum = FUSED ? tpart : nullptr;
#pragma unroll
    for (int m = 0; m < M; ++m) tpart[m] = (T)0;
    if constexpr (FUSED) {
        if (n0_64 % S == 0) {                // the launch starts a window
            T f[M];
            tensions<T, M, FENE>(s, G, f);
#pragma unroll
            for (int m = 0; m < M; ++m) tpart[m] = -f[m];
        }
    }
    // the window sum in global memory holds part of the current window: true
    // when the launch starts inside a window, and after every mid-window fold
    bool acc_live = (n0_64 % S) != 0;
    // fend: the window-end tensions (window_end), which also start the next window's sum
    auto flush_tsf = [&](bool window_end, const T (&fend)[M]) {
        if constexpr (TSF) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (valid[m]) {
                    const double acc = (acc_live ? tacc_g[m] : 0.0) + (double)tpart[m];
                    if (window_end) tsf_w[m] = (T)((acc + (FUSED ? (double)fend[m] : 0.0)) / (double)S);
                    else tacc_g[m] = acc;
                }
                tpart[m] = (FUSED && window_end) ? -fend[m] : (T)0;
            }
            acc_live = !window_end;
        }
    };
    int clamps = 0;
    // the separate pass: the tensions of the state after each step
    auto accumulate_tsf = [&]() {
        if constexpr (TSF && !FUSED) {
            T f[M];
            tensions<T, M, FENE>(s, G, f);
#pragma unroll
            for (int m = 0; m < M; ++m) tpart[m] += f[m];
        }
    };
    // noise map 1: with one or two beads per lane the steps run in aligned
    // groups of four. The next group's three Philox blocks per slot are drawn
    // at the top of each group (integer work independent of the steps), and
    // each step transforms the blocks it uses just before it, which spreads
    // the transcendentals over the group (against transforming the next
    // group's blocks along with their draw, 3.5% faster on fene50; against
    // the carry, 5% faster on two beads per lane). A run's unaligned head and
    // its tail, and wider lanes, take the carry step by step. The carry lives
    // for the whole launch (built once for its first step): segments follow
    // each other in step order, an aligned group neither needs nor changes
    // it, and a partial group is always stepped through the carry, so it
    // holds the current group's fourth normals.
    [[maybe_unused]] Carry<T, M> cy;
    if constexpr (NMAP == 1) init_carry<T, M>(cy, G, n0, bead0, rep, keys);
    auto run_steps_map1 = [&](uint32_t n, int len) {
        int i = 0;
        if constexpr (M <= 2) {
            for (; i < len && ((n + (uint32_t)i) & 3u) != 0u; ++i) {
                em_step_map1<T, M, FENE, FUSED>(s, cy, G, valid, kc, n + (uint32_t)i, bead0, rep, keys, clamps, tsum);
                accumulate_tsf();
            }
            if (i + 4 <= len) {
                Words w[3][M];
#pragma unroll
                for (int q = 0; q < 3; ++q)
#pragma unroll
                    for (int m = 0; m < M; ++m)
                        w[q][m] = philox10(n + (uint32_t)(i + q), bead0 + (uint32_t)m, rep, G.stream, keys);
                for (; i + 4 <= len; i += 4) {
                    asm volatile(".p2align 6");
                    Words nw[3][M];
#pragma unroll
                    for (int q = 0; q < 3; ++q)
#pragma unroll
                        for (int m = 0; m < M; ++m)
                            nw[q][m] = philox10(n + (uint32_t)(i + 4 + q), bead0 + (uint32_t)m, rep, G.stream, keys);
                    Noise<T, M> e3;
#pragma unroll
                    for (int u = 0; u < 3; ++u) {
                        Noise<T, M> e;
#pragma unroll
                        for (int m = 0; m < M; ++m) {
                            T d;
                            normals4(w[u][m], e.x[m], e.y[m], e.z[m], d);
                            if (u == 0) e3.x[m] = d;
                            if (u == 1) e3.y[m] = d;
                            if (u == 2) e3.z[m] = d;
                        }
                        physics_step<T, M, FENE, FUSED>(s, e, G, valid, kc, clamps, tsum);
                        accumulate_tsf();
                    }
                    physics_step<T, M, FENE, FUSED>(s, e3, G, valid, kc, clamps, tsum);
                    accumulate_tsf();
#pragma unroll
                    for (int q = 0; q < 3; ++q)
#pragma unroll
                        for (int m = 0; m < M; ++m) w[q][m] = nw[q][m];
                }
            }
        }
        // the rest: with one or two beads per lane a tail of at most three
        // steps that starts aligned (the carry is refilled before it is read);
        // wider lanes step through the carry from the start
        for (; i < len; ++i) {
            em_step_map1<T, M, FENE, FUSED>(s, cy, G, valid, kc, n + (uint32_t)i, bead0, rep, keys, clamps, tsum);
            accumulate_tsf();
        }
    };
    auto run_steps = [&](uint32_t n, int len) {   // len steps starting at global step n
        if constexpr (NMAP == 1) {
            run_steps_map1(n, len);
            return;
        }
        if constexpr (NMAP == 2) {
            for (int i = 0; i < len; ++i) {
                em_step_map2<T, M, FENE, FUSED>(s, G, valid, kc, n + (uint32_t)i, bead0, rep, keys, clamps, tsum);
                accumulate_tsf();
            }
            return;
        }
        int i = 0;
        if constexpr (U > 1) {
            // software pipeline: the noise of block b+1 is generated in the same
            // basic block as the updates of block b, so the scheduler can fill the
            // update chain's latencies with independent Philox work (one spare
            // block of noise is generated past the end and discarded)
            if constexpr (M == 1) {
                // one bead per lane: the next U steps' blocks are drawn ahead and
                // each step transforms its own block just before it (6% faster
                // on fene50 than transforming along with the draw; with two beads
                // per lane the draw-and-transform pipeline below is 2% faster)
                if (U <= len) {
                    Words w[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) w[u] = philox10(n + (uint32_t)u, bead0, rep, G.stream, keys);
                    for (; i + U <= len; i += U) {
                        asm volatile(".p2align 6");
                        Words nw[U];
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            nw[u] = philox10(n + (uint32_t)(i + U + u), bead0, rep, G.stream, keys);
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            Noise<T, M> e;
                            normals3(w[u], e.x[0], e.y[0], e.z[0]);
                            physics_step<T, M, FENE, FUSED>(s, e, G, valid, kc, clamps, tsum);
                            accumulate_tsf();
                        }
#pragma unroll
                        for (int u = 0; u < U; ++u) w[u] = nw[u];
                    }
                }
            } else if (U <= len) {
                Noise<T, M> e[U];
#pragma unroll
                for (int u = 0; u < U; ++u) gen_noise<T, M>(e[u], G, n + (uint32_t)u, bead0, rep, keys);
                for (; i + U <= len; i += U) {
                    // start the loop body on a 64-byte boundary: its speed depends on
                    // where its 4- and 8-byte instructions fall in the fetch lines
                    // (measured: unaligned placements cost up to 10%)
                    asm volatile(".p2align 6");
                    Noise<T, M> f[U];
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        gen_noise<T, M>(f[u], G, n + (uint32_t)(i + U + u), bead0, rep, keys);
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        physics_step<T, M, FENE, FUSED>(s, e[u], G, valid, kc, clamps, tsum);
                        accumulate_tsf();
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) e[u] = f[u];
                }
            }
        }
        for (; i < len; ++i) {
            em_step<T, M, FENE, FUSED>(s, G, valid, kc, n + (uint32_t)i, bead0, rep, keys, clamps, tsum);
            accumulate_tsf();
        }
    };

    int left = n_steps;
    int to_flush = TSF_FLUSH;
    uint32_t n = n0;
    while (left > 0) {
        if (to_ck == 0) {                      // checkpoint before step n
            store_ckpt<T, M>(s, ck_w, G);
            ck_w += ckpt_total;
            to_ck = K;
        }
        int len = min(left, min(to_smp, to_ck));
        if constexpr (TSF) len = min(len, to_flush);
        run_steps(n, len);
        n += (uint32_t)len;
        left -= len;
        to_ck -= len;
        to_smp -= len;
        to_flush -= len;
        if (to_smp == 0) {                     // window end after step n - 1
            T f[M];
            tensions<T, M, FENE>(s, G, f);
            bool bad = false;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (valid[m]) {
                    smp_w[m] = f[m];
                    bad |= !__builtin_isfinite(f[m]);
                }
            }
            flush_tsf(true, f);
            to_flush = TSF_FLUSH;
            smp_w += smp_total;
            if constexpr (TSF) tsf_w += smp_total;
            if (bad) atomicOr(status, 2);
            to_smp = S;
        } else if (TSF && (to_flush == 0 || left == 0)) {
            const T none[M] = {};
            flush_tsf(false, none);
            to_flush = TSF_FLUSH;
        }
    }
    store_lane<T, M>(s, valid, state, G, tg);
    flush_clamps(clamps, clamp_ctr);
}

// With 1-4 beads per lane the group's constants are copied into a local value
// once: read through the reference, the step loop re-loads them from memory
// every iteration (measured: one extra vector load per step). Wider lanes keep
// the reference, as the copy would not fit their register budget.
// Noise map 1 is compiled for 1-4 beads per lane only (the host rejects it
// for wider lanes, whose register budget has no room for the carry), noise
// map 2 for 8, 12 and 16 beads per lane only, each in kernels of its own, so
// each map gets its own register allocation.
template <typename T, int M, bool FENE, bool UNIFORM_K, bool TSF, int NMAP>
__device__ __forceinline__ void run_forward(const FwdArgs& a, const GroupDev& Gm, int k_first, int64_t n0_64) {
    const int gidx = (int)(&Gm - a.groups);
    if constexpr (M <= 4) {
        const GroupDev G = Gm;
        run_forward_impl<T, M, FENE, UNIFORM_K, TSF, NMAP>(a, G, gidx, k_first, n0_64);
    } else {
        static_assert(NMAP != 1, "noise map 1 is compiled for 1-4 beads per lane");
        run_forward_impl<T, M, FENE, UNIFORM_K, TSF, NMAP>(a, Gm, gidx, k_first, n0_64);
    }
}

// TSFK: 0 compiles the variants without TSF, 1 those with TSF (kernels of
// their own, so the time-average sums do not raise the register budget of
// runs without them), 2 both, chosen per context at run time (the RSF
// cycle's dual launch: the parent keeps TSF, the replicas do not).
template <typename T, int M, int NMAP, int TSFK>
__device__ __forceinline__ void dispatch_spring(const FwdArgs& a, const GroupDev& G, int k_first, int64_t n0) {
    const bool tsf = a.tsf != nullptr;
#define RA_FWD(FENE_, UK_, TSF_) run_forward<T, M, FENE_, UK_, TSF_, NMAP>(a, G, k_first, n0)
#define RA_TSF(FENE_, UK_)                                        \
    do {                                                          \
        if constexpr (TSFK == 0) RA_FWD(FENE_, UK_, false);       \
        else if constexpr (TSFK == 1) RA_FWD(FENE_, UK_, true);   \
        else if (tsf) RA_FWD(FENE_, UK_, true);                   \
        else RA_FWD(FENE_, UK_, false);                           \
    } while (0)
    if constexpr (sizeof(T) == 8) {           // FP64 correctness path: fewer variants
        if (G.spring == 1) RA_TSF(true, false);
        else RA_TSF(false, false);
    } else {
        const bool uk = G.P == 1;
        if (G.spring == 1) {
            if (uk) RA_TSF(true, true);
            else RA_TSF(true, false);
        } else {
            if (uk) RA_TSF(false, true);
            else RA_TSF(false, false);
        }
    }
#undef RA_TSF
#undef RA_FWD
    (void)tsf;
}

// WAVES_PER_EU is a register budget hint: family 4 needs none (about 100
// VGPRs); family 16 is held to 2 resident waves per SIMD (256 registers), which
// it fits without spilling — left alone the scheduler hoists all 16 Philox
// chains and falls to 1 wave, and asking for 3-4 waves makes it spill.
template <typename T, int FAMILY, int NMAP, int TSFK>
__device__ __forceinline__ void fwd_item(const FwdArgs& a, int item) {
    if (item >= a.n_items) return;
    if (*(const volatile int*)a.status & 1) return;   // invalid parent: no work
    const Item it = a.items[item];
    const GroupDev& G = a.groups[it.g];
    const int64_t n0 = *a.step0;
    if constexpr (FAMILY == 4) {
        switch (G.M) {
        case 1: dispatch_spring<T, 1, NMAP, TSFK>(a, G, it.k0, n0); break;
        case 2: dispatch_spring<T, 2, NMAP, TSFK>(a, G, it.k0, n0); break;
        case 3: dispatch_spring<T, 3, NMAP, TSFK>(a, G, it.k0, n0); break;
        case 4: dispatch_spring<T, 4, NMAP, TSFK>(a, G, it.k0, n0); break;
        default: break;
        }
    } else if constexpr (NMAP == 2) {   // the host picks 8, 12 or 16 beads per lane under map 2
        switch (G.M) {
        case 8: dispatch_spring<T, 8, 2, TSFK>(a, G, it.k0, n0); break;
        case 12: dispatch_spring<T, 12, 2, TSFK>(a, G, it.k0, n0); break;
        case 16: dispatch_spring<T, 16, 2, TSFK>(a, G, it.k0, n0); break;
        default: break;
        }
    } else {
        switch (G.M) {
        case 6: dispatch_spring<T, 6, 0, TSFK>(a, G, it.k0, n0); break;
        case 8: dispatch_spring<T, 8, 0, TSFK>(a, G, it.k0, n0); break;
        case 12: dispatch_spring<T, 12, 0, TSFK>(a, G, it.k0, n0); break;
        case 16: dispatch_spring<T, 16, 0, TSFK>(a, G, it.k0, n0); break;
        default: break;
        }
    }
}

template <typename T, int FAMILY, int WAVES_PER_EU, int NMAP, int TSFK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES_PER_EU)))
void fwd_kernel(FwdArgs a) {
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    fwd_item<T, FAMILY, NMAP, TSFK>(a, (int)blockIdx.x * (int)(blockDim.x >> 6) + wave);
}

// Two contexts in one launch (the RSF cycle's replicas of window w and the
// parent's next segment): blocks [0, blocks_a) run a's work list, the rest b's.
// One launch keeps the two concurrent whatever hardware queues the streams
// map to, and the parent's few waves get SIMDs of their own.
template <typename T, int FAMILY, int WAVES_PER_EU, int NMAP = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WAVES_PER_EU)))
void fwd_dual_kernel(FwdArgs a, FwdArgs b, int blocks_a) {
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wpb = (int)(blockDim.x >> 6);
    if ((int)blockIdx.x < blocks_a) fwd_item<T, FAMILY, NMAP, 2>(a, (int)blockIdx.x * wpb + wave);
    else fwd_item<T, FAMILY, NMAP, 2>(b, ((int)blockIdx.x - blocks_a) * wpb + wave);
}

__global__ void advance_kernel(int64_t* step, int64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *step += n;
}

// Clears the status word, the per-group guard counters and the device step
// counter: a kernel rather than memset nodes, so a caller may capture the
// clone sequence in a graph.
__global__ void reset_kernel(int32_t* status, unsigned long long* clamps, int n_groups, int64_t* step) {
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t == 0) {
        *status = 0;
        *step = 0;
    }
    for (int g = t; g < n_groups; g += (int)(gridDim.x * blockDim.x)) clamps[g] = 0ull;
}

// ---------------------------------------------------------------------------
// Clone (RSF, Sec. II): Q_j = parent_{j+1} - parent_j in FP64, then rounded to
// the state precision, for every replica; the parent is validated here.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void clone_kernel(const GroupDev* __restrict__ groups, const double* __restrict__ parent,
                             const int64_t* __restrict__ par_off, T* __restrict__ state,
                             double* __restrict__ tsf_acc, int32_t* status) {
    const GroupDev& G = groups[blockIdx.y];
    const int nm1 = G.N - 1;
    const int64_t total = (int64_t)G.R * nm1;
    const double* p = parent + par_off[blockIdx.y];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / nm1;
        const int j = (int)(e - k * nm1);
        const double qx = p[3 * (j + 1)] - p[3 * j];
        const double qy = p[3 * (j + 1) + 1] - p[3 * j + 1];
        const double qz = p[3 * (j + 1) + 2] - p[3 * j + 2];
        bool bad = !(__builtin_isfinite(qx) && __builtin_isfinite(qy) && __builtin_isfinite(qz));
        if (G.spring == 1 && !((qx * qx + qy * qy + qz * qz) * G.inv_q0sq_d < 1.0)) bad = true;
        if (bad && k == 0) atomicOr(status, 1);
        const int64_t o = G.state_off + e * 3;
        state[o] = (T)qx;
        state[o + 1] = (T)qy;
        state[o + 2] = (T)qz;
        if (tsf_acc) tsf_acc[G.smp_off + e] = 0.0;
    }
}

// Plain path clone: bead positions of every replica = parent.
template <typename T>
__global__ void clone_pos_kernel(const GroupDev* __restrict__ groups, const double* __restrict__ parent,
                                 const int64_t* __restrict__ par_off, T* __restrict__ pos,
                                 double* __restrict__ tsf_acc, int32_t* status) {
    const GroupDev& G = groups[blockIdx.y];
    const int64_t per = (int64_t)G.N * 3;
    const int64_t total = (int64_t)G.R * per;
    const double* p = parent + par_off[blockIdx.y];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e % per;
        pos[G.pos_off + e] = (T)p[c];
        if (e < per) {
            bool bad = !__builtin_isfinite(p[c]);
            if (G.spring == 1 && c % 3 == 0 && c + 3 < per) {
                const double qx = p[c + 3] - p[c], qy = p[c + 4] - p[c + 1], qz = p[c + 5] - p[c + 2];
                if (!((qx * qx + qy * qy + qz * qz) * G.inv_q0sq_d < 1.0)) bad = true;
            }
            if (bad) atomicOr(status, 1);
        }
    }
    if (tsf_acc) {
        const int64_t ns = (int64_t)G.R * (G.N - 1);
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ns;
             e += (int64_t)gridDim.x * blockDim.x)
            tsf_acc[G.smp_off + e] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Plain path: one launch per step per group, bead positions in HBM, one
// thread per (replica, bead), bead form of Eq. (1) with the same counters.
// ---------------------------------------------------------------------------
template <typename T, bool FENE>
__device__ __forceinline__ void bond_force(const T* r0, const T* r1, const GroupDev& G, T& fx, T& fy,
                                           T& fz, int& clamps) {
    const T qx = r1[0] - r0[0], qy = r1[1] - r0[1], qz = r1[2] - r0[2];
    T g = (T)1;
    if constexpr (FENE) {
        const T q2 = fmadd(qx, qx, fmadd(qy, qy, qz * qz));
        g = fene_g(qx, qy, qz, q2, (T)G.inv_q0sq, G.inv_q0sq_d, clamps);
    }
    fx = g * qx;
    fy = g * qy;
    fz = g * qz;
}

template <typename T, bool FENE>
__global__ __launch_bounds__(256) void plain_step_kernel(const GroupDev* __restrict__ groups, int g,
                                                         const T* __restrict__ rin, T* __restrict__ rout,
                                                         const int32_t* status, uint32_t n, uint32_t key0,
                                                         uint32_t key1, unsigned long long* clamp_ctr) {
    const GroupDev& G = groups[g];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)G.R * G.N) return;
    if (*status & 1) return;
    const int64_t k = e / G.N;
    const int i = (int)(e - k * G.N);
    const T* r = rin + G.pos_off + k * G.N * 3;
    const Co<T> c{G};
    int clamps = 0;
    T fx = 0, fy = 0, fz = 0;
    if (i <= G.N - 2) {
        T ax, ay, az;
        bond_force<T, FENE>(r + 3 * i, r + 3 * (i + 1), G, ax, ay, az, clamps);
        fx += ax; fy += ay; fz += az;
    }
    if (i >= 1) {
        T bx, by, bz;
        int dummy = 0;
        bond_force<T, FENE>(r + 3 * (i - 1), r + 3 * i, G, bx, by, bz, dummy);
        fx -= bx; fy -= by; fz -= bz;
    }
    T ex, ey, ez;
    if (G.nmap == 1 && (n & 3u) == 3u) {   // map 1: fourth normals of steps n-3 .. n-1
        T a_, b_, c_;
        normals4(philox10(n - 3u, (uint32_t)i, (uint32_t)k, G.stream, key0, key1), a_, b_, c_, ex);
        normals4(philox10(n - 2u, (uint32_t)i, (uint32_t)k, G.stream, key0, key1), a_, b_, c_, ey);
        normals4(philox10(n - 1u, (uint32_t)i, (uint32_t)k, G.stream, key0, key1), a_, b_, c_, ez);
    } else if (G.nmap == 2) {              // map 2: normal i mod 4 of the blocks 3 (i / 4) + c
        const uint32_t b = 3u * ((uint32_t)i >> 2);
        const int r = i & 3;
        T v[4];
        normals4(philox10(n, b, (uint32_t)k, G.stream, key0, key1), v[0], v[1], v[2], v[3]);
        ex = r == 0 ? v[0] : r == 1 ? v[1] : r == 2 ? v[2] : v[3];
        normals4(philox10(n, b + 1u, (uint32_t)k, G.stream, key0, key1), v[0], v[1], v[2], v[3]);
        ey = r == 0 ? v[0] : r == 1 ? v[1] : r == 2 ? v[2] : v[3];
        normals4(philox10(n, b + 2u, (uint32_t)k, G.stream, key0, key1), v[0], v[1], v[2], v[3]);
        ez = r == 0 ? v[0] : r == 1 ? v[1] : r == 2 ? v[2] : v[3];
    } else {
        normals3(philox10(n, (uint32_t)i, (uint32_t)k, G.stream, key0, key1), ex, ey, ez);
    }
    const T x = r[3 * i], y = r[3 * i + 1], z = r[3 * i + 2];
    const T ix = fmadd(c.kx(), x, fmadd(c.kxz(), z, fmadd(c.cF(), fx, c.sigma() * ex)));
    const T iy = fmadd(c.ky(), y, fmadd(c.cF(), fy, c.sigma() * ey));
    const T iz = fmadd(c.kz(), z, fmadd(c.cF(), fz, c.sigma() * ez));
    T* o = rout + G.pos_off + k * G.N * 3 + 3 * i;
    o[0] = x + ix;
    o[1] = y + iy;
    o[2] = z + iz;
    if (clamps) atomicAdd(clamp_ctr + g, (unsigned long long)clamps);
}

template <typename T, bool FENE>
__global__ __launch_bounds__(256) void plain_sample_kernel(const GroupDev* __restrict__ groups, int g,
                                                           const T* __restrict__ pos, T* __restrict__ samples,
                                                           T* __restrict__ tsfo, double* __restrict__ tsf_acc,
                                                           int window_end, int S, int32_t* status) {
    const GroupDev& G = groups[g];
    const int nm1 = G.N - 1;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)G.R * nm1) return;
    const int64_t k = e / nm1;
    const int j = (int)(e - k * nm1);
    const T* r = pos + G.pos_off + k * G.N * 3 + 3 * j;
    int dummy = 0;
    T fx, fy, fz;
    bond_force<T, FENE>(r, r + 3, G, fx, fy, fz, dummy);
    const T f = Co<T>{G}.H() * fast_sqrt(fmadd(fx, fx, fmadd(fy, fy, fz * fz)));
    const int64_t o = G.smp_off + e;
    if (tsf_acc) {
        const double acc = tsf_acc[o] + (double)f;
        if (window_end) {
            tsfo[o] = (T)(acc / (double)S);
            tsf_acc[o] = 0.0;
        } else {
            tsf_acc[o] = acc;
        }
    }
    if (window_end) {
        samples[o] = f;
        if (!__builtin_isfinite(f)) atomicOr(status, 2);
    }
}

// ---------------------------------------------------------------------------
// Replica reduction (RSF estimate, Sec. II): per (window, spring) the replica
// mean and the R-1 standard deviation, FP64, two passes, fixed order:
// wave v of RED_WAVES sums replicas [v*c, (v+1)*c) (c = ceil(R/RED_WAVES)) in
// order, the waves' sums combine in wave order. Loads are unrolled so each
// lane keeps several rows in flight; the second pass re-reads the block's
// rows, which are still in L2.
// ---------------------------------------------------------------------------
constexpr int RED_WAVES = 16;

template <typename T>
__global__ __launch_bounds__(WAVE * RED_WAVES) void reduce_kernel(const GroupDev* __restrict__ groups,
                                                               const ColTile* __restrict__ tiles,
                                                               const T* __restrict__ smp, int64_t smp_total,
                                                               int64_t spr_total, double* __restrict__ mean,
                                                               double* __restrict__ stdv) {
    __shared__ double part[RED_WAVES][WAVE];
    const ColTile tile = tiles[blockIdx.x];
    const int64_t w = blockIdx.y;
    const GroupDev& G = groups[tile.g];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x >> 6;
    const int nm1 = G.N - 1;
    const int j = tile.j0 + lane;
    const bool ok = j < nm1;
    const int chunk = (G.R + RED_WAVES - 1) / RED_WAVES;
    const int kb = min(G.R, wv * chunk);
    const int ke = min(G.R, kb + chunk);
    const T* base = smp + w * smp_total + G.smp_off + (ok ? j : 0);
    double acc = 0.0;
    if (ok) {
#pragma unroll 8
        for (int k = kb; k < ke; ++k) acc += (double)base[(int64_t)k * nm1];
    }
    part[wv][lane] = acc;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int v = 0; v < RED_WAVES; ++v) tot += part[v][lane];
    const double mu = tot / (double)G.R;
    __syncthreads();
    double ss = 0.0;
    if (ok) {
#pragma unroll 8
        for (int k = kb; k < ke; ++k) {
            const double d = (double)base[(int64_t)k * nm1] - mu;
            ss = fmadd(d, d, ss);
        }
    }
    part[wv][lane] = ss;
    __syncthreads();
    if (wv == 0 && ok) {
        double sst = 0.0;
#pragma unroll
        for (int v = 0; v < RED_WAVES; ++v) sst += part[v][lane];
        const int64_t o = w * spr_total + G.spr_off + j;
        if (mean) mean[o] = mu;
        if (stdv) stdv[o] = G.R > 1 ? sqrt(sst / (double)(G.R - 1)) : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Bell-type rates (Sec. III) and event draws, one wavefront per (group, window).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void bell_kernel(const GroupDev* __restrict__ groups, int n_groups,
                                                  const double* __restrict__ mean, int64_t spr_total,
                                                  double k0, double xd, double* __restrict__ rates,
                                                  double* __restrict__ rate_sum, uint8_t* __restrict__ events,
                                                  int S, uint32_t key0, uint32_t key1) {
    const int g = blockIdx.x;
    const int64_t w = blockIdx.y;
    const GroupDev& G = groups[g];
    const int lane = threadIdx.x;
    double acc = 0.0;
    for (int j = lane; j < G.N - 1; j += WAVE) {
        const int64_t o = w * spr_total + G.spr_off + j;
        const double k = k0 * exp(xd * mean[o] / G.kT);
        if (rates) rates[o] = k;
        acc += k;
        if (events) {
            const Words u = philox10((uint32_t)w, (uint32_t)j, 0u, (2u << 24) | (G.stream & 0xFFFFFFu), key0, key1);
            const double p = -expm1(-k * (double)S * G.dt);
            events[o] = u01_f64_53(u.x, u.y) < p ? 1 : 0;
        }
    }
    // fixed-order butterfly over the 64 lanes
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, WAVE);
    if (lane == 0 && rate_sum) rate_sum[w * n_groups + g] = acc;
}

// ---------------------------------------------------------------------------
// Inspection helpers.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void to_f64_kernel(const T* __restrict__ src, double* __restrict__ dst, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = (double)src[e];
}

template <typename T>
__global__ void pos_to_bonds_kernel(const GroupDev* __restrict__ groups, const T* __restrict__ pos,
                                    double* __restrict__ out) {
    const GroupDev& G = groups[blockIdx.y];
    const int nm1 = G.N - 1;
    const int64_t total = (int64_t)G.R * nm1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / nm1;
        const int j = (int)(e - k * nm1);
        const T* r = pos + G.pos_off + k * G.N * 3 + 3 * j;
        for (int a = 0; a < 3; ++a) out[G.state_off + e * 3 + a] = (double)r[3 + a] - (double)r[a];
    }
}

__global__ void debug_noise_kernel(const uint32_t* __restrict__ ctr, int64_t n, uint32_t key0, uint32_t key1,
                                   uint32_t* __restrict__ words, float* __restrict__ n32,
                                   double* __restrict__ n64) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const Words w = philox10(ctr[4 * e], ctr[4 * e + 1], ctr[4 * e + 2], ctr[4 * e + 3], key0, key1);
    if (words) {
        words[4 * e] = w.x;
        words[4 * e + 1] = w.y;
        words[4 * e + 2] = w.z;
        words[4 * e + 3] = w.w;
    }
    if (n32) {
        float a, b, c;
        normals3(w, a, b, c);
        n32[3 * e] = a;
        n32[3 * e + 1] = b;
        n32[3 * e + 2] = c;
    }
    if (n64) {
        double a, b, c;
        normals3(w, a, b, c);
        n64[3 * e] = a;
        n64[3 * e + 1] = b;
        n64[3 * e + 2] = c;
    }
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
static dim3 grid1d(int64_t n, int block) {
    int64_t b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > 65535) b = 65535;
    return dim3((unsigned)b);
}

#ifndef FAMILY16_WAVES
#define FAMILY16_WAVES 2
#endif

template <typename T, int FAMILY, int WPE, int NMAP>
static void launch_fwd_tsf(const FwdArgs& a, dim3 grid, dim3 block, hipStream_t st) {
    if (a.tsf) hipLaunchKernelGGL((fwd_kernel<T, FAMILY, WPE, NMAP, 1>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((fwd_kernel<T, FAMILY, WPE, NMAP, 0>), grid, block, 0, st, a);
}

hipError_t launch_forward(const FwdArgs& a, int precision, int family, int waves_per_block, int nmap,
                          hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    const int wpb = waves_per_block;
    dim3 grid((a.n_items + wpb - 1) / wpb), block(WAVE * wpb);
    if (precision == 64) {
        if (nmap == 1) launch_fwd_tsf<double, 4, 1, 1>(a, grid, block, st);
        else launch_fwd_tsf<double, 4, 1, 0>(a, grid, block, st);
    } else if (family == 4) {
        if (nmap == 1) launch_fwd_tsf<float, 4, 1, 1>(a, grid, block, st);
        else launch_fwd_tsf<float, 4, 1, 0>(a, grid, block, st);
    } else {
        if (nmap == 2) launch_fwd_tsf<float, 16, FAMILY16_WAVES, 2>(a, grid, block, st);
        else launch_fwd_tsf<float, 16, FAMILY16_WAVES, 0>(a, grid, block, st);
    }
    return hipGetLastError();
}

hipError_t launch_forward_dual(const FwdArgs& a, const FwdArgs& b, int precision, int family, int waves_per_block,
                               int nmap, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    const int wpb = waves_per_block;
    const int ba = (a.n_items + wpb - 1) / wpb, bb = (b.n_items + wpb - 1) / wpb;
    if (ba + bb == 0) return hipSuccess;
    dim3 grid((unsigned)(ba + bb)), block(WAVE * wpb);
    if (precision == 64) {
        if (nmap == 1) hipLaunchKernelGGL((fwd_dual_kernel<double, 4, 1, 1>), grid, block, 0, st, a, b, ba);
        else hipLaunchKernelGGL((fwd_dual_kernel<double, 4, 1>), grid, block, 0, st, a, b, ba);
    } else if (family == 4) {
        if (nmap == 1) hipLaunchKernelGGL((fwd_dual_kernel<float, 4, 1, 1>), grid, block, 0, st, a, b, ba);
        else hipLaunchKernelGGL((fwd_dual_kernel<float, 4, 1>), grid, block, 0, st, a, b, ba);
    } else {
        if (nmap == 2) hipLaunchKernelGGL((fwd_dual_kernel<float, 16, FAMILY16_WAVES, 2>), grid, block, 0, st, a, b, ba);
        else hipLaunchKernelGGL((fwd_dual_kernel<float, 16, FAMILY16_WAVES>), grid, block, 0, st, a, b, ba);
    }
    return hipGetLastError();
}

hipError_t launch_advance(int64_t* step, int64_t n, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, st, step, n);
    return hipGetLastError();
}

hipError_t launch_reset(int32_t* status, unsigned long long* clamps, int n_groups, int64_t* step, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(256), 0, st, status, clamps, n_groups, step);
    return hipGetLastError();
}

hipError_t launch_clone(const GroupDev* groups, int n_groups, int64_t max_elems, const double* parent,
                        const int64_t* par_off, void* state, double* tsf_acc, int32_t* status, int precision,
                        bool plain, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    dim3 grid((unsigned)std::min<int64_t>((max_elems + 255) / 256, 4096), (unsigned)n_groups), block(256);
    if (plain) {
        if (precision == 64)
            hipLaunchKernelGGL(clone_pos_kernel<double>, grid, block, 0, st, groups, parent, par_off,
                               (double*)state, tsf_acc, status);
        else
            hipLaunchKernelGGL(clone_pos_kernel<float>, grid, block, 0, st, groups, parent, par_off,
                               (float*)state, tsf_acc, status);
    } else {
        if (precision == 64)
            hipLaunchKernelGGL(clone_kernel<double>, grid, block, 0, st, groups, parent, par_off,
                               (double*)state, tsf_acc, status);
        else
            hipLaunchKernelGGL(clone_kernel<float>, grid, block, 0, st, groups, parent, par_off,
                               (float*)state, tsf_acc, status);
    }
    return hipGetLastError();
}

hipError_t launch_plain_step(const GroupDev* groups, int g, int64_t n_threads, bool fene, const void* rin,
                             void* rout, const int32_t* status, uint32_t n, uint32_t key0, uint32_t key1,
                             unsigned long long* clamps, int precision, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    dim3 grid((unsigned)((n_threads + 255) / 256)), block(256);
    if (precision == 64) {
        if (fene) hipLaunchKernelGGL((plain_step_kernel<double, true>), grid, block, 0, st, groups, g,
                                     (const double*)rin, (double*)rout, status, n, key0, key1, clamps);
        else hipLaunchKernelGGL((plain_step_kernel<double, false>), grid, block, 0, st, groups, g,
                                (const double*)rin, (double*)rout, status, n, key0, key1, clamps);
    } else {
        if (fene) hipLaunchKernelGGL((plain_step_kernel<float, true>), grid, block, 0, st, groups, g,
                                     (const float*)rin, (float*)rout, status, n, key0, key1, clamps);
        else hipLaunchKernelGGL((plain_step_kernel<float, false>), grid, block, 0, st, groups, g,
                                (const float*)rin, (float*)rout, status, n, key0, key1, clamps);
    }
    return hipGetLastError();
}

hipError_t launch_plain_sample(const GroupDev* groups, int g, int64_t n_threads, bool fene, const void* pos,
                               void* samples_w, void* tsf_w, double* tsf_acc, int window_end, int S,
                               int32_t* status, int precision, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    dim3 grid((unsigned)((n_threads + 255) / 256)), block(256);
    if (precision == 64) {
        if (fene) hipLaunchKernelGGL((plain_sample_kernel<double, true>), grid, block, 0, st, groups, g,
                                     (const double*)pos, (double*)samples_w, (double*)tsf_w, tsf_acc,
                                     window_end, S, status);
        else hipLaunchKernelGGL((plain_sample_kernel<double, false>), grid, block, 0, st, groups, g,
                                (const double*)pos, (double*)samples_w, (double*)tsf_w, tsf_acc,
                                window_end, S, status);
    } else {
        if (fene) hipLaunchKernelGGL((plain_sample_kernel<float, true>), grid, block, 0, st, groups, g,
                                     (const float*)pos, (float*)samples_w, (float*)tsf_w, tsf_acc,
                                     window_end, S, status);
        else hipLaunchKernelGGL((plain_sample_kernel<float, false>), grid, block, 0, st, groups, g,
                                (const float*)pos, (float*)samples_w, (float*)tsf_w, tsf_acc,
                                window_end, S, status);
    }
    return hipGetLastError();
}

hipError_t launch_reduce(const GroupDev* groups, const ColTile* tiles, int n_tiles, int64_t n_windows,
                         const void* smp, int64_t smp_total, int64_t spr_total, double* mean, double* stdv,
                         int precision, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    if (n_tiles == 0 || n_windows == 0) return hipSuccess;
    dim3 grid((unsigned)n_tiles, (unsigned)n_windows), block(WAVE * RED_WAVES);
    if (precision == 64)
        hipLaunchKernelGGL(reduce_kernel<double>, grid, block, 0, st, groups, tiles, (const double*)smp,
                           smp_total, spr_total, mean, stdv);
    else
        hipLaunchKernelGGL(reduce_kernel<float>, grid, block, 0, st, groups, tiles, (const float*)smp,
                           smp_total, spr_total, mean, stdv);
    return hipGetLastError();
}

hipError_t launch_bell(const GroupDev* groups, int n_groups, int64_t n_windows, const double* mean,
                       int64_t spr_total, double k0, double xd, double* rates, double* rate_sum,
                       uint8_t* events, int S, uint32_t key0, uint32_t key1, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    if (n_windows == 0) return hipSuccess;
    dim3 grid((unsigned)n_groups, (unsigned)n_windows), block(64);
    hipLaunchKernelGGL(bell_kernel, grid, block, 0, st, groups, n_groups, mean, spr_total, k0, xd, rates,
                       rate_sum, events, S, key0, key1);
    return hipGetLastError();
}

hipError_t launch_to_f64(const void* src, double* dst, int64_t n, int precision, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    if (n == 0) return hipSuccess;
    if (precision == 64)
        hipLaunchKernelGGL(to_f64_kernel<double>, grid1d(n, 256), dim3(256), 0, st, (const double*)src, dst, n);
    else
        hipLaunchKernelGGL(to_f64_kernel<float>, grid1d(n, 256), dim3(256), 0, st, (const float*)src, dst, n);
    return hipGetLastError();
}

hipError_t launch_pos_to_bonds(const GroupDev* groups, int n_groups, int64_t max_elems, const void* pos,
                               double* out, int precision, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    dim3 grid((unsigned)std::min<int64_t>((max_elems + 255) / 256, 4096), (unsigned)n_groups), block(256);
    if (precision == 64)
        hipLaunchKernelGGL(pos_to_bonds_kernel<double>, grid, block, 0, st, groups, (const double*)pos, out);
    else
        hipLaunchKernelGGL(pos_to_bonds_kernel<float>, grid, block, 0, st, groups, (const float*)pos, out);
    return hipGetLastError();
}

hipError_t launch_debug_noise(const uint32_t* ctr, int64_t n, uint32_t key0, uint32_t key1, uint32_t* words,
                              float* n32, double* n64, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(debug_noise_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ctr, n, key0,
                       key1, words, n32, n64);
    return hipGetLastError();
}

}  // namespace ra
