// ra_rsf.hip — device work of the RSF sampling cycle and of the estimators
// built on it:
//   - re-clone (Sec. II): every replica restarts from the current state of a
//     parent chain that runs its own trajectory in another context;
//   - the centre-of-mass-frame conformation each replica set was cloned from;
//   - the spread sigma(N_R) of the RSF estimate over blocks of N_R replicas
//     (Figs. 2 and 5);
//   - the mean first-passage time to any event of a chain (MFTU, Sec. III),
//     from the mean total rate and by sampling unfolding events;
//   - replica fidelity D-bar (Eq. 5) and radius-of-gyration components
//     (R_Gz, Sec. IV).
// None of these is on the per-step path; they run once per window or per
// analysis call, with fixed summation orders so results are reproducible.
#include "ra_device.hpp"
#include "ra_launch.hpp"

namespace ra {

// ---------------------------------------------------------------------------
// Wave helpers (FP64): fixed-shape butterfly sum and an inclusive Hillis-Steele
// scan over the 64 lanes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

__device__ __forceinline__ double wave_incl_scan_d(double v, int lane) {
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        const double u = __shfl_up(v, off, WAVE);
        if (lane >= off) v += u;
    }
    return v;
}

// Lane l of a wave owns beads [l*c, min(N, (l+1)*c)), c = ceil(N/64), and the
// bonds with the same indices (bond m joins beads m and m+1). base = position
// of the lane's first bead relative to bead 0: the exclusive scan of the
// lanes' bond sums.
template <typename T>
struct ChainScan {
    const T* q;          // bonds [N-1][3]
    int N, c, i0, i1;
    double bx, by, bz;   // position of bead i0

    __device__ ChainScan(const T* bonds, int n, int lane) : q(bonds), N(n) {
        c = (N + WAVE - 1) / WAVE;
        i0 = min(N, lane * c);
        i1 = min(N, i0 + c);
        double tx = 0.0, ty = 0.0, tz = 0.0;
        for (int m = i0; m < min(i1, N - 1); ++m) {
            tx += (double)q[3 * m];
            ty += (double)q[3 * m + 1];
            tz += (double)q[3 * m + 2];
        }
        bx = wave_incl_scan_d(tx, lane) - tx;
        by = wave_incl_scan_d(ty, lane) - ty;
        bz = wave_incl_scan_d(tz, lane) - tz;
    }
};

// Centre-of-mass-frame positions of a chain given by its bonds, written to
// out[N][3] (FP64). One wave.
template <typename T>
__device__ void com_frame_from_bonds(const T* bonds, int N, double* out, int lane) {
    ChainScan<T> cs(bonds, N, lane);
    double x = cs.bx, y = cs.by, z = cs.bz, sx = 0.0, sy = 0.0, sz = 0.0;
    for (int i = cs.i0; i < cs.i1; ++i) {
        sx += x; sy += y; sz += z;
        if (i < N - 1) { x += (double)bonds[3 * i]; y += (double)bonds[3 * i + 1]; z += (double)bonds[3 * i + 2]; }
    }
    const double cx = wave_sum_d(sx) / N, cy = wave_sum_d(sy) / N, cz = wave_sum_d(sz) / N;
    x = cs.bx; y = cs.by; z = cs.bz;
    for (int i = cs.i0; i < cs.i1; ++i) {
        out[3 * i] = x - cx;
        out[3 * i + 1] = y - cy;
        out[3 * i + 2] = z - cz;
        if (i < N - 1) { x += (double)bonds[3 * i]; y += (double)bonds[3 * i + 1]; z += (double)bonds[3 * i + 2]; }
    }
}

// Clone source from FP64 bead positions: src = parent - centre of mass.
__global__ __launch_bounds__(64) void src_from_xyz_kernel(const GroupDev* __restrict__ groups,
                                                          const double* __restrict__ parent,
                                                          const int64_t* __restrict__ par_off,
                                                          double* __restrict__ src) {
    const GroupDev& G = groups[blockIdx.x];
    const int lane = threadIdx.x;
    const double* p = parent + par_off[blockIdx.x];
    double* o = src + par_off[blockIdx.x];
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int i = lane; i < G.N; i += WAVE) { sx += p[3 * i]; sy += p[3 * i + 1]; sz += p[3 * i + 2]; }
    const double cx = wave_sum_d(sx) / G.N, cy = wave_sum_d(sy) / G.N, cz = wave_sum_d(sz) / G.N;
    for (int i = lane; i < G.N; i += WAVE) {
        o[3 * i] = p[3 * i] - cx;
        o[3 * i + 1] = p[3 * i + 1] - cy;
        o[3 * i + 2] = p[3 * i + 2] - cz;
    }
}

// ---------------------------------------------------------------------------
// Re-clone: state of every replica of group g := replica 0 of the parent
// context's group g. A FENE bond at or past full extension (or non-finite)
// marks the parent invalid (status bit 1), as at the first clone. In the same
// launch: the first wave of block (0, g) writes group g's clone source (the
// parent's beads in its centre-of-mass frame, for Eq. 5), and one thread sets
// the replicas' device step counter to the window start.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void reclone_kernel(const GroupDev* __restrict__ groups, const GroupDev* __restrict__ pgroups,
                               const T* __restrict__ pstate, T* __restrict__ state,
                               double* __restrict__ tsf_acc, int32_t* status, const int64_t* __restrict__ par_off,
                               double* __restrict__ src, int64_t* step, int64_t step_value) {
    const GroupDev& G = groups[blockIdx.y];
    const GroupDev& PG = pgroups[blockIdx.y];
    const int nm1 = G.N - 1;
    const int64_t total = (int64_t)G.R * nm1;
    const T* p = pstate + PG.state_off;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = e / nm1;
        const int j = (int)(e - k * nm1);
        const T qx = p[3 * j], qy = p[3 * j + 1], qz = p[3 * j + 2];
        if (k == 0) {
            const double x = qx, y = qy, z = qz;
            bool bad = !(__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z));
            if (G.spring == 1 && !((x * x + y * y + z * z) * G.inv_q0sq_d < 1.0)) bad = true;
            if (bad) atomicOr(status, 1);
        }
        const int64_t o = G.state_off + e * 3;
        state[o] = qx;
        state[o + 1] = qy;
        state[o + 2] = qz;
        if (tsf_acc) tsf_acc[G.smp_off + e] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x < WAVE)
        com_frame_from_bonds<T>(p, G.N, src + par_off[blockIdx.y], (int)threadIdx.x);
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) step[0] = step_value;
}

// Both step counters of a dual launch advance in one kernel.
__global__ void advance2_kernel(int64_t* a, int64_t na, int64_t* b, int64_t nb) {
    if (threadIdx.x == 0) {
        a[0] += na;
        b[0] += nb;
    }
}

// ---------------------------------------------------------------------------
// Replica fidelity (Eq. 5) and radius of gyration, one wave per replica.
// rep_off[g] = first replica of group g in the outputs (n_groups + 1 entries).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void conformation_kernel(const GroupDev* __restrict__ groups, int n_groups,
                                                           const int64_t* __restrict__ rep_off,
                                                           const T* __restrict__ state,
                                                           const int64_t* __restrict__ par_off,
                                                           const double* __restrict__ src,
                                                           double* __restrict__ dbar, double* __restrict__ d_bead,
                                                           double* __restrict__ rg2) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t q = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (q >= rep_off[n_groups]) return;
    int lo = 0, hi = n_groups - 1;   // group with rep_off[g] <= q < rep_off[g + 1]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rep_off[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    const int g = lo;
    const GroupDev& G = groups[g];
    const int64_t k = q - rep_off[g];
    const int N = G.N;
    const T* bonds = state + G.state_off + k * (int64_t)(N - 1) * 3;
    const double* s = src + par_off[g];
    ChainScan<T> cs(bonds, N, lane);
    double x = cs.bx, y = cs.by, z = cs.bz, sx = 0.0, sy = 0.0, sz = 0.0;
    for (int i = cs.i0; i < cs.i1; ++i) {
        sx += x; sy += y; sz += z;
        if (i < N - 1) { x += (double)bonds[3 * i]; y += (double)bonds[3 * i + 1]; z += (double)bonds[3 * i + 2]; }
    }
    const double cx = wave_sum_d(sx) / N, cy = wave_sum_d(sy) / N, cz = wave_sum_d(sz) / N;
    double dx = 0.0, dy = 0.0, dz = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    double* db = d_bead ? d_bead + (G.pos_off / 3 + k * N) * 3 : nullptr;
    x = cs.bx; y = cs.by; z = cs.bz;
    for (int i = cs.i0; i < cs.i1; ++i) {
        const double hx = x - cx, hy = y - cy, hz = z - cz;
        const double ex = fabs(hx - s[3 * i]), ey = fabs(hy - s[3 * i + 1]), ez = fabs(hz - s[3 * i + 2]);
        dx += ex; dy += ey; dz += ez;
        gx += hx * hx; gy += hy * hy; gz += hz * hz;
        if (db) { db[3 * i] = ex; db[3 * i + 1] = ey; db[3 * i + 2] = ez; }
        if (i < N - 1) { x += (double)bonds[3 * i]; y += (double)bonds[3 * i + 1]; z += (double)bonds[3 * i + 2]; }
    }
    dx = wave_sum_d(dx); dy = wave_sum_d(dy); dz = wave_sum_d(dz);
    gx = wave_sum_d(gx); gy = wave_sum_d(gy); gz = wave_sum_d(gz);
    const int64_t o = (rep_off[g] + k) * 3;
    if (lane == 0) {
        if (dbar) { dbar[o] = dx / N; dbar[o + 1] = dy / N; dbar[o + 2] = dz / N; }
        if (rg2) { rg2[o] = gx / N; rg2[o + 1] = gy / N; rg2[o + 2] = gz / N; }
    }
}

// Radius-of-gyration components of each group's clone source.
__global__ __launch_bounds__(64) void src_rg2_kernel(const GroupDev* __restrict__ groups,
                                                     const int64_t* __restrict__ par_off,
                                                     const double* __restrict__ src, double* __restrict__ out) {
    const GroupDev& G = groups[blockIdx.x];
    const double* s = src + par_off[blockIdx.x];
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int i = threadIdx.x; i < G.N; i += WAVE) {
        gx += s[3 * i] * s[3 * i];
        gy += s[3 * i + 1] * s[3 * i + 1];
        gz += s[3 * i + 2] * s[3 * i + 2];
    }
    gx = wave_sum_d(gx); gy = wave_sum_d(gy); gz = wave_sum_d(gz);
    if (threadIdx.x == 0) {
        out[3 * blockIdx.x] = gx / G.N;
        out[3 * blockIdx.x + 1] = gy / G.N;
        out[3 * blockIdx.x + 2] = gz / G.N;
    }
}

// ---------------------------------------------------------------------------
// sigma(N_R): per (window, spring), B = floor(R/block) consecutive blocks;
// each block's mean tension is one RSF estimate; sigma = their standard
// deviation (B - 1). Wave v of 16 takes a contiguous sixteenth of the blocks
// in order; the sixteenths combine in order; two passes (mean, then deviations).
// ---------------------------------------------------------------------------
constexpr int BSIG_WAVES = 16;

template <typename T>
__global__ __launch_bounds__(1024) void block_sigma_kernel(const GroupDev* __restrict__ groups,
                                                           const ColTile* __restrict__ tiles,
                                                           const T* __restrict__ smp, int64_t smp_total,
                                                           int64_t spr_total, int block,
                                                           double* __restrict__ sigma) {
    constexpr int NW = BSIG_WAVES;
    __shared__ double part[NW][WAVE];
    const ColTile tile = tiles[blockIdx.x];
    const int64_t w = blockIdx.y;
    const GroupDev& G = groups[tile.g];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x >> 6;
    const int nm1 = G.N - 1;
    const int j = tile.j0 + lane;
    const bool ok = j < nm1;
    const int B = G.R / block;
    const int cb = (B + NW - 1) / NW;
    const int b0 = min(B, wv * cb), b1 = min(B, b0 + cb);
    const T* base = smp + w * smp_total + G.smp_off + (ok ? j : 0);
    auto block_mean = [&](int b) {
        double m = 0.0;
        for (int q = 0; q < block; ++q) m += (double)base[(int64_t)(b * block + q) * nm1];
        return m / block;
    };
    auto combine = [&]() {   // the wavefronts' partials in wavefront order
        double t = 0.0;
#pragma unroll
        for (int v = 0; v < NW; ++v) t += part[v][lane];
        return t;
    };
    double acc = 0.0;
    if (ok)
        for (int b = b0; b < b1; ++b) acc += block_mean(b);
    part[wv][lane] = acc;
    __syncthreads();
    const double mu = B > 0 ? combine() / B : 0.0;
    __syncthreads();
    double ss = 0.0;
    if (ok)
        for (int b = b0; b < b1; ++b) {
            const double e = block_mean(b) - mu;
            ss = fma(e, e, ss);
        }
    part[wv][lane] = ss;
    __syncthreads();
    if (wv == 0 && ok) {
        const double tot = combine();
        sigma[w * spr_total + G.spr_off + j] = B > 1 ? sqrt(tot / (double)(B - 1)) : 0.0;
    }
}

// mftu[g] = 1 / (mean over windows of rate_sum[w][g]); one wave per group.
__global__ __launch_bounds__(64) void mftu_kernel(const double* __restrict__ rate_sum, int64_t n_windows,
                                                  int n_groups, double* __restrict__ mftu) {
    const int g = blockIdx.x;
    double acc = 0.0;
    for (int64_t w = threadIdx.x; w < n_windows; w += WAVE) acc += rate_sum[w * n_groups + g];
    acc = wave_sum_d(acc);
    if (threadIdx.x == 0) mftu[g] = 1.0 / (acc / (double)n_windows);
}

// MFTU by sampling unfolding events. Window v carries the rates of sampled
// window v mod n_windows, and spring j unfolds there when the tag-2 53-bit
// uniform of counter (v, j, trial, 2<<24 | stream) is below 1 - exp(-k S dt)
// (trial 0 over the sampled windows draws exactly ra_bell_rates's events).
// The first window with any unfolding, or -1 after max_windows, is the trial's
// first passage.
//
// The uniform is u = (2m + 1) 2^-53 with m the top 52 bits of its two words,
// so u < p holds exactly when m is below the count of such m, ceil((p 2^53 - 1) / 2)
// (0 when p 2^53 <= 1, 2^52 when p >= 1): p 2^53 is exact, and for
// 1 < p 2^53 < 2^53 so are the subtraction and the halving. The per-draw test is
// one 64-bit integer compare against a threshold computed once per (window,
// spring) from the same FP64 expression.
__device__ __forceinline__ uint64_t event_threshold(double p) {
    const double x = p * 0x1p53;
    if (!(x > 1.0)) return 0;   // no m, also for NaN
    if (x >= 0x1p53) return (uint64_t)1 << 52;
    return (uint64_t)ceil((x - 1.0) * 0.5);
}

// Thresholds in LDS, one workgroup of four wavefronts per (trial, group):
// thread t takes window base + t, so lane order within a wavefront and the
// wavefront index are window order; every thread draws all springs of its
// window. The earliest window with a vote in any wavefront ends the trial for
// the whole workgroup.
constexpr int EVENT_THREADS = 256;
constexpr size_t EVENT_LDS_MAX = 32 << 10;   // thresholds in LDS up to this size, else the kernel below

__global__ __launch_bounds__(EVENT_THREADS) void first_event_lds_kernel(
    const GroupDev* __restrict__ groups, const double* __restrict__ rates, int64_t n_windows, int64_t spr_total,
    int64_t max_windows, int S, uint32_t key0, uint32_t key1, int64_t* __restrict__ first_window, int n_groups) {
    extern __shared__ uint64_t thr[];   // [n_windows][N - 1]
    __shared__ int64_t found[EVENT_THREADS / WAVE];
    const int trial = blockIdx.x;
    const int g = blockIdx.y;
    const GroupDev& G = groups[g];
    const int tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & (WAVE - 1);
    const int nm1 = G.N - 1;
    const double window_time = (double)S * G.dt;
    const uint32_t ctr3 = (2u << 24) | (G.stream & 0xFFFFFFu);
    const RoundKeys keys = round_keys<false>(key0, key1);
    const int64_t n_thr = n_windows * nm1;
    for (int64_t i = tid; i < n_thr; i += EVENT_THREADS) {
        const int64_t w = i / nm1, j = i - w * nm1;
        const double k = rates[w * spr_total + G.spr_off + j];
        thr[i] = event_threshold(-expm1(-k * window_time));
    }
    __syncthreads();
    const uint32_t nw = (uint32_t)n_windows;
    for (int64_t base = 0; base < max_windows; base += EVENT_THREADS) {
        const int64_t v = base + tid;
        bool hit = false;
        if (v < max_windows) {
            const uint64_t* tw = thr + (int64_t)((uint32_t)v % nw) * nm1;
            for (int j = 0; j < nm1; ++j) {
                const Words u = philox10((uint32_t)v, (uint32_t)j, (uint32_t)trial, ctr3, keys);
                const uint64_t m = ((uint64_t)u.x << 20) | (uint64_t)(u.y >> 12);
                hit |= m < tw[j];
            }
        }
        const uint64_t b = __builtin_amdgcn_ballot_w64(hit);
        if (lane == 0) found[wv] = b ? base + WAVE * wv + __builtin_ctzll(b) : -1;
        __syncthreads();
        int64_t f = -1;
#pragma unroll
        for (int q = 0; q < EVENT_THREADS / WAVE; ++q) {
            const int64_t x = found[q];
            if (f < 0 && x >= 0) f = x;
        }
        __syncthreads();   // found[] is rewritten by the next round
        if (f >= 0) {
            if (tid == 0) first_window[(int64_t)trial * n_groups + g] = f;
            return;
        }
    }
    if (tid == 0) first_window[(int64_t)trial * n_groups + g] = -1;
}

// The same without the LDS table (chains whose thresholds do not fit): one
// wavefront per (trial, group), the lanes cover the springs and the wave walks
// the windows in order, the rate read and the FP64 test per draw.
__global__ __launch_bounds__(64) void first_event_kernel(const GroupDev* __restrict__ groups,
                                                         const double* __restrict__ rates, int64_t n_windows,
                                                         int64_t spr_total, int64_t max_windows, int S,
                                                         uint32_t key0, uint32_t key1,
                                                         int64_t* __restrict__ first_window, int n_groups) {
    const int trial = blockIdx.x;
    const int g = blockIdx.y;
    const GroupDev& G = groups[g];
    const int lane = threadIdx.x;
    const int nm1 = G.N - 1;
    const double window_time = (double)S * G.dt;
    const uint32_t ctr3 = (2u << 24) | (G.stream & 0xFFFFFFu);
    const RoundKeys keys = round_keys<false>(key0, key1);
    int64_t first = -1;
    int64_t w = 0;
    for (int64_t v = 0; v < max_windows; ++v) {
        bool hit = false;
        for (int j = lane; j < nm1; j += WAVE) {
            const double k = rates[w * spr_total + G.spr_off + j];
            const Words u = philox10((uint32_t)v, (uint32_t)j, (uint32_t)trial, ctr3, keys);
            hit |= u01_f64_53(u.x, u.y) < -expm1(-k * window_time);
        }
        if (__builtin_amdgcn_ballot_w64(hit) != 0) {
            first = v;
            break;
        }
        if (++w == n_windows) w = 0;
    }
    if (lane == 0) first_window[(int64_t)trial * n_groups + g] = first;
}

// The censored maximum-likelihood mean of the first-passage times: all
// trials' times (first-passage or censoring) over the number of events; one
// wavefront per group, trials summed in fixed order.
__global__ __launch_bounds__(64) void mftu_events_kernel(const GroupDev* __restrict__ groups,
                                                         const int64_t* __restrict__ first_window, int n_trials,
                                                         int64_t max_windows, int S, int n_groups,
                                                         double* __restrict__ mftu) {
    const int g = blockIdx.x;
    const double window_time = (double)S * groups[g].dt;
    double total = 0.0, events = 0.0;
    for (int t = threadIdx.x; t < n_trials; t += WAVE) {
        const int64_t f = first_window[(int64_t)t * n_groups + g];
        total += (double)(f >= 0 ? f + 1 : max_windows) * window_time;
        events += f >= 0 ? 1.0 : 0.0;
    }
    total = wave_sum_d(total);
    events = wave_sum_d(events);
    if (threadIdx.x == 0) mftu[g] = events > 0.0 ? total / events : __builtin_inf();
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t launch_reclone(const GroupDev* groups, const GroupDev* pgroups, int n_groups, int64_t max_elems,
                          const void* pstate, void* state, double* tsf_acc, int32_t* status, const int64_t* par_off,
                          double* src, int64_t* step, int64_t step_value, int precision, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    const int64_t blocks = std::min<int64_t>(1024, (max_elems + 255) / 256);
    dim3 grid((unsigned)std::max<int64_t>(1, blocks), (unsigned)n_groups), block(256);
    if (precision == 64)
        hipLaunchKernelGGL(reclone_kernel<double>, grid, block, 0, st, groups, pgroups, (const double*)pstate,
                           (double*)state, tsf_acc, status, par_off, src, step, step_value);
    else
        hipLaunchKernelGGL(reclone_kernel<float>, grid, block, 0, st, groups, pgroups, (const float*)pstate,
                           (float*)state, tsf_acc, status, par_off, src, step, step_value);
    return hipGetLastError();
}

hipError_t launch_advance2(int64_t* a, int64_t na, int64_t* b, int64_t nb, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    hipLaunchKernelGGL(advance2_kernel, dim3(1), dim3(64), 0, st, a, na, b, nb);
    return hipGetLastError();
}

hipError_t launch_src_from_xyz(const GroupDev* groups, int n_groups, const double* parent, const int64_t* par_off,
                               double* src, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    hipLaunchKernelGGL(src_from_xyz_kernel, dim3((unsigned)n_groups), dim3(64), 0, st, groups, parent, par_off, src);
    return hipGetLastError();
}

hipError_t launch_conformation(const GroupDev* groups, int n_groups, const int64_t* rep_off, int64_t n_reps,
                               const void* state, const int64_t* par_off, const double* src, double* dbar,
                               double* d_bead, double* rg2, double* src_rg2, int precision, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    if (n_reps > 0 && (dbar || d_bead || rg2)) {
        dim3 grid((unsigned)((n_reps + 3) / 4)), block(256);
        if (precision == 64)
            hipLaunchKernelGGL(conformation_kernel<double>, grid, block, 0, st, groups, n_groups, rep_off,
                               (const double*)state, par_off, src, dbar, d_bead, rg2);
        else
            hipLaunchKernelGGL(conformation_kernel<float>, grid, block, 0, st, groups, n_groups, rep_off,
                               (const float*)state, par_off, src, dbar, d_bead, rg2);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (src_rg2) hipLaunchKernelGGL(src_rg2_kernel, dim3((unsigned)n_groups), dim3(64), 0, st, groups, par_off, src,
                                    src_rg2);
    return hipGetLastError();
}

hipError_t launch_block_sigma(const GroupDev* groups, const ColTile* tiles, int n_tiles, int64_t n_windows,
                              const void* smp, int64_t smp_total, int64_t spr_total, int block, double* sigma,
                              int precision, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    if (n_tiles == 0 || n_windows == 0) return hipSuccess;
    dim3 grid((unsigned)n_tiles, (unsigned)n_windows), blk(WAVE * BSIG_WAVES);
    if (precision == 64)
        hipLaunchKernelGGL(block_sigma_kernel<double>, grid, blk, 0, st, groups, tiles, (const double*)smp, smp_total,
                           spr_total, block, sigma);
    else
        hipLaunchKernelGGL(block_sigma_kernel<float>, grid, blk, 0, st, groups, tiles, (const float*)smp, smp_total,
                           spr_total, block, sigma);
    return hipGetLastError();
}

hipError_t launch_mftu_events(const GroupDev* groups, int n_groups, const double* rates, int64_t n_windows,
                              int64_t spr_total, int n_trials, int64_t max_windows, int S, uint32_t key0,
                              uint32_t key1, int max_springs, int64_t* first_window, double* mftu, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    const size_t lds = (size_t)n_windows * (size_t)std::max(max_springs, 1) * sizeof(uint64_t);
    if (n_windows <= 0xFFFFFFFFll && lds <= EVENT_LDS_MAX)
        hipLaunchKernelGGL(first_event_lds_kernel, dim3((unsigned)n_trials, (unsigned)n_groups), dim3(EVENT_THREADS),
                           lds, st, groups, rates, n_windows, spr_total, max_windows, S, key0, key1, first_window,
                           n_groups);
    else
        hipLaunchKernelGGL(first_event_kernel, dim3((unsigned)n_trials, (unsigned)n_groups), dim3(64), 0, st, groups,
                           rates, n_windows, spr_total, max_windows, S, key0, key1, first_window, n_groups);
    hipLaunchKernelGGL(mftu_events_kernel, dim3((unsigned)n_groups), dim3(64), 0, st, groups, first_window, n_trials,
                       max_windows, S, n_groups, mftu);
    return hipGetLastError();
}

hipError_t launch_mftu(const double* rate_sum, int64_t n_windows, int n_groups, double* mftu, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    hipLaunchKernelGGL(mftu_kernel, dim3((unsigned)n_groups), dim3(64), 0, st, rate_sum, n_windows, n_groups, mftu);
    return hipGetLastError();
}

}  // namespace ra
