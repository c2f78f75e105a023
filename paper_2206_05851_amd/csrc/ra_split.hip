// ra_split.hip — forward kernel for one bead per lane with noise produced by
// a second wavefront.
//
// When a batch has about one wavefront per SIMD (e.g. 1024 replicas of a
// 50-bead chain), a single instruction stream per SIMD cannot hide its own
// latencies, and the scalar unit and the VALU never work for different waves
// at once. Here each work item gets two wavefronts in the same block: the
// physics wave keeps the chain in VGPRs exactly as the one-wave kernel does,
// and a noise wave fills an LDS double buffer with the Philox/Box-Muller
// normals of the next SPLIT_CHUNK steps. The noise wave walks the flattened
// (step, bead) space so all 64 of its lanes do useful work whatever N is.
// Both waves pass the same number of block barriers, one per chunk.
//
// The normals and the bond update are the same device functions as in the
// one-wave kernel, so trajectories are bit-identical to it.
#include "ra_chain.hpp"
#include "ra_launch.hpp"

namespace ra {

constexpr int SPLIT_PAIRS = 4;          // (physics, noise) wavefront pairs per block
constexpr int SPLIT_CHUNK = 16;         // steps per LDS buffer
constexpr int SPLIT_ROW = WAVE + 1;     // one slot per lane + a zero slot for lane 63's neighbour

struct SplitBuf {
    float v[2][SPLIT_CHUNK][3][SPLIT_ROW];
};

// Normals of steps [base, base + cnt) of one work item into B[step][xyz][lane].
template <bool UNIFORM_K>
__device__ __forceinline__ void split_fill(float (&B)[SPLIT_CHUNK][3][SPLIT_ROW], const GroupDev& G,
                                           int k_first, uint32_t base, int cnt, const RoundKeys& keys,
                                           int lane) {
    const int N = G.N;
    const int PN = UNIFORM_K ? N : G.P * N;   // bead lanes in use (lane = replica slot * N + bead)
    const int total = cnt * PN;
    int step = 0, lc = lane;
    while (lc >= PN) { lc -= PN; ++step; }
    for (int v0 = 0; v0 < total; v0 += WAVE) {
        if (v0 + lane < total) {
            int bead = lc, seg = 0;
            if constexpr (!UNIFORM_K) {
                while (bead >= N) { bead -= N; ++seg; }
            }
            const Words w = philox10(base + (uint32_t)step, (uint32_t)bead, (uint32_t)(k_first + seg),
                                     G.stream, keys);
            float x, y, z;
            normals3(w, x, y, z);
            B[step][0][lc] = x;
            B[step][1][lc] = y;
            B[step][2][lc] = z;
        }
        lc += WAVE;
        while (lc >= PN) { lc -= PN; ++step; }
    }
}

template <bool UNIFORM_K>
__device__ void split_produce(const FwdArgs& a, const GroupDev& G, int k_first, uint32_t n0, int n_steps,
                              int nc, SplitBuf& buf) {
    const RoundKeys keys = round_keys(a.key0, a.key1);
    const int lane = threadIdx.x & (WAVE - 1);
    split_fill<UNIFORM_K>(buf.v[0], G, k_first, n0, min(SPLIT_CHUNK, n_steps), keys, lane);
    for (int c = 0; c < nc; ++c) {
        __syncthreads();
        if (c + 1 < nc) {
            const int start = (c + 1) * SPLIT_CHUNK;
            split_fill<UNIFORM_K>(buf.v[(c + 1) & 1], G, k_first, n0 + (uint32_t)start,
                                  min(SPLIT_CHUNK, n_steps - start), keys, lane);
        }
    }
}

// The physics wave: run_forward for M = 1 without TSF, noise read from LDS.
template <bool FENE, bool UNIFORM_K>
__device__ void split_consume(const FwdArgs& a, const GroupDev& G, int k_first, uint32_t n0, int n_steps,
                              int nc, SplitBuf& buf) {
    using T = float;
    constexpr int M = 1;
    const int S = a.S, K = a.K;
    const int64_t smp_total = a.smp_total, state_total = a.state_total;
    T* const state = (T*)a.state;
    int32_t* const status = a.status;
    unsigned long long* const clamp_ctr = a.clamps + (&G - a.groups);
    const TileGeom tg = tile_geom<UNIFORM_K>(G, k_first, M);
    const int lane = threadIdx.x & (WAVE - 1);
    Lane<T, M> s;
    bool valid[M];
    load_lane<T, M>(s, valid, state, G, tg);
    const SlotCoef<T, M> kc = slot_coef<T, M>(G, valid);
    const int nm1 = G.N - 1;
    const int64_t lane_off = G.smp_off + (int64_t)tg.k * nm1 + tg.j0;
    T* smp_w = (T*)a.samples + (int64_t)(n0 / (uint32_t)S) * smp_total + lane_off;
    T* ck_w = K > 0 ? (T*)a.ckpt + (int64_t)((n0 + (uint32_t)K - 1) / (uint32_t)K) * state_total : nullptr;
    int to_smp = S - (int)(n0 % (uint32_t)S);
    int to_ck = K > 0 ? (int)((K - (int)(n0 % (uint32_t)K)) % K) : INT32_MAX;
    int clamps = 0;
    // the physics wave is the critical path: issue it first, the noise wave fills the gaps
    __builtin_amdgcn_s_setprio(2);
    for (int c = 0; c < nc; ++c) {
        __syncthreads();
        const float (&B)[SPLIT_CHUNK][3][SPLIT_ROW] = buf.v[c & 1];
        const int cnt = min(SPLIT_CHUNK, n_steps - c * SPLIT_CHUNK);
        // own and next-lane normals of step i, read one step ahead
        T ex = B[0][0][lane], ey = B[0][1][lane], ez = B[0][2][lane];
        T nx = B[0][0][lane + 1], ny = B[0][1][lane + 1], nz = B[0][2][lane + 1];
        for (int i = 0; i < cnt; ++i) {
            const int ip = i + 1 < cnt ? i + 1 : i;
            const T ex1 = B[ip][0][lane], ey1 = B[ip][1][lane], ez1 = B[ip][2][lane];
            const T nx1 = B[ip][0][lane + 1], ny1 = B[ip][1][lane + 1], nz1 = B[ip][2][lane + 1];
            if (to_ck == 0) {
                store_lane<T, M>(s, valid, ck_w, G, tg);
                ck_w += state_total;
                to_ck = K;
            }
            physics_step_core<T, M, FENE>(
                s, [&](int, T& x, T& y, T& z) { x = ex; y = ey; z = ez; },
                [&](T, T, T, T& x, T& y, T& z) { x = nx; y = ny; z = nz; }, G, valid, kc, clamps);
            ex = ex1; ey = ey1; ez = ez1;
            nx = nx1; ny = ny1; nz = nz1;
            --to_ck;
            if (--to_smp == 0) {
                T f[M];
                tensions<T, M, FENE>(s, G, f);
                bool bad = false;
                if (valid[0]) {
                    smp_w[0] = f[0];
                    bad = !__builtin_isfinite(f[0]);
                }
                smp_w += smp_total;
                if (bad) atomicOr(status, 2);
                to_smp = S;
            }
        }
    }
    __builtin_amdgcn_s_setprio(0);
    store_lane<T, M>(s, valid, state, G, tg);
    flush_clamps(clamps, clamp_ctr);
}

__global__ __launch_bounds__(WAVE * 2 * SPLIT_PAIRS) void fwd_split_kernel(FwdArgs a) {
    __shared__ SplitBuf bufs[SPLIT_PAIRS];
    // zero the buffers: lanes past the last bead (and the pad slot) read 0.0
    float* flat = &bufs[0].v[0][0][0][0];
    constexpr int n_floats = (int)(SPLIT_PAIRS * sizeof(SplitBuf) / sizeof(float));
    for (int i = threadIdx.x; i < n_floats; i += blockDim.x) flat[i] = 0.0f;
    __syncthreads();
    if (*(const volatile int*)a.status & 1) return;   // invalid parent: the whole block leaves together
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const bool producer = wave >= SPLIT_PAIRS;
    const int pair = producer ? wave - SPLIT_PAIRS : wave;
    const int item = (int)blockIdx.x * SPLIT_PAIRS + pair;
    const int n_steps = (int)a.n_steps;
    const int nc = (n_steps + SPLIT_CHUNK - 1) / SPLIT_CHUNK;
    const uint32_t n0 = (uint32_t)*a.step0;
    SplitBuf& buf = bufs[pair];
    if (item >= a.n_items) {   // no work, but every wave passes every barrier
        for (int c = 0; c < nc; ++c) __syncthreads();
        return;
    }
    const Item it = a.items[item];
    const GroupDev& G = a.groups[it.g];
    const bool uk = G.P == 1;
    if (producer) {
        if (uk) split_produce<true>(a, G, it.k0, n0, n_steps, nc, buf);
        else split_produce<false>(a, G, it.k0, n0, n_steps, nc, buf);
    } else if (G.spring == 1) {
        if (uk) split_consume<true, true>(a, G, it.k0, n0, n_steps, nc, buf);
        else split_consume<true, false>(a, G, it.k0, n0, n_steps, nc, buf);
    } else {
        if (uk) split_consume<false, true>(a, G, it.k0, n0, n_steps, nc, buf);
        else split_consume<false, false>(a, G, it.k0, n0, n_steps, nc, buf);
    }
}

hipError_t launch_forward_split(const FwdArgs& a, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    dim3 grid((a.n_items + SPLIT_PAIRS - 1) / SPLIT_PAIRS), block(WAVE * 2 * SPLIT_PAIRS);
    hipLaunchKernelGGL(fwd_split_kernel, grid, block, 0, st, a);
    return hipGetLastError();
}

}  // namespace ra
