// ra_adjoint.hip — pathwise adjoint of the fused forward path (FP32 state).
//
// Objective J = sum_{w,j} lam_mu[w][j] * mean_k f_j^{w,k}, where lam_mu is
// dJ/d(replica-mean tension) (Bell-rate cotangents are folded into it first).
// With the noise held fixed, every EM step Q^{n+1} = Phi(Q^n; rate, H, b) is
// a smooth map, and reverse mode runs
//   lambda^n = (dPhi/dQ)^T lambda^{n+1} + dJ/dQ^n (sample injections),
//   dJ/dtheta += lambda^{n+1} . dPhi/dtheta + direct dJ/dtheta at samples.
// The forward stored Q every K steps; each K-step segment is recomputed
// from its checkpoint with the same step function (bitwise-identical
// trajectory) into a per-wavefront HBM buffer, then swept backwards.
//
// Bond form: Phi_j = Q_j + dt kappa Q_j + cF [G_{j+1} - 2 G_j + G_{j-1}] + noise,
// G_j = g_j Q_j. The Laplacian is symmetric, so
//   (dPhi/dQ)^T lambda at j = lambda_j + (dt kappa)^T lambda_j + cF J_j mu_j,
//   mu_j = lambda_{j+1} - 2 lambda_j + lambda_{j-1},
//   J_j = dG_j/dQ_j = g I + 2 g^2 / Q0^2 Q Q^T (FENE off the guard), g I on it.
#include "ra_chain.hpp"
#include "ra_launch.hpp"

namespace ra {

// g, s and the guard flag, computed exactly as the forward computes g.
template <bool FENE>
__device__ __forceinline__ void factor_gs(float qx, float qy, float qz, const GroupDev& G, float& g, float& s,
                                          bool& smooth) {
    if constexpr (!FENE) {
        g = 1.0f; s = 0.0f; smooth = false;
        return;
    } else {
        const float q2 = fmadd(qx, qx, fmadd(qy, qy, qz * qz));
        const float sf = q2 * G.inv_q0sq;
        g = fast_rcp(1.0f - sf);
        s = sf;
        smooth = true;
        // wave vote, as in the forward step: the FP64 recomputation runs only
        // in wavefronts where some lane is near full extension
        if (__builtin_expect(__builtin_amdgcn_ballot_w64(sf > FENE_FP64_BAND) != 0, 0)) {
            if (sf > FENE_FP64_BAND) {
                const double dx = qx, dy = qy, dz = qz;
                double sd = (dx * dx + dy * dy + dz * dz) * G.inv_q0sq_d;
                smooth = !(sd > 1.0 - FENE_DELTA);
                if (!smooth) sd = 1.0 - FENE_DELTA;
                g = (float)(1.0 / (1.0 - sd));
                s = (float)sd;
            }
        }
    }
}

template <int M>
__device__ __forceinline__ void seg_store(float* seg, int step, const Lane<float, M>& s, int lane) {
#pragma unroll
    for (int m = 0; m < M; ++m) {
        float* p = seg + ((int64_t)(step * M + m) * 3) * WAVE + lane;
        p[0] = s.qx[m];
        p[WAVE] = s.qy[m];
        p[2 * WAVE] = s.qz[m];
    }
}
template <int M>
__device__ __forceinline__ void seg_load(const float* seg, int step, Lane<float, M>& s, int lane) {
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const float* p = seg + ((int64_t)(step * M + m) * 3) * WAVE + lane;
        s.qx[m] = p[0];
        s.qy[m] = p[WAVE];
        s.qz[m] = p[2 * WAVE];
    }
}

// dJ/dQ and direct dJ/dtheta of the sampled tension f = H g |Q| at window w.
template <int M, bool FENE>
__device__ __forceinline__ void inject(const Lane<float, M>& q, const bool (&valid)[M], const GroupDev& G,
                                       const AdjArgs& a, const TileGeom& tg, int64_t w, float (&lx)[M],
                                       float (&ly)[M], float (&lz)[M], double& gH, double& gb) {
    const float H = G.H;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const float c = valid[m] ? (float)(a.lam_mu[w * a.spr_total + G.spr_off + tg.j0 + m] / (double)G.R)
                                 : 0.0f;
        float g, s;
        bool smooth;
        factor_gs<FENE>(q.qx[m], q.qy[m], q.qz[m], G, g, s, smooth);
        const float q2 = fmadd(q.qx[m], q.qx[m], fmadd(q.qy[m], q.qy[m], q.qz[m] * q.qz[m]));
        const float len = fast_sqrt(q2);
        // df/dQ = H (g + 2 g^2 s) Q/|Q| off the guard, H g Q/|Q| on it (Hookean: s = 0)
        const float coef = len > 0.0f ? H * (smooth ? fmadd(2.0f * g * g, s, g) : g) / len : 0.0f;
        lx[m] = fmadd(c * coef, q.qx[m], lx[m]);
        ly[m] = fmadd(c * coef, q.qy[m], ly[m]);
        lz[m] = fmadd(c * coef, q.qz[m], lz[m]);
        // df/dH = g |Q| (1 + g s), df/db = -H g^2 (s/b) |Q| off the guard
        const float dH = smooth ? g * len * fmadd(g, s, 1.0f) : g * len;
        const float db = (FENE && smooth) ? -H * g * g * (s / (float)G.b) * len : 0.0f;
        gH += (double)(c * dH);
        gb += (double)(c * db);
    }
}

// FP32 partial sums of one reverse sweep (a segment, or one step when every
// state is kept), turned into the (rate, H, b) gradient terms by rev_flush:
//   rate: lambda . d(dt kappa Q)/d rate = dt (fx Sxx + fy Syy + fz Szz + fxz Sxz)
//         with (fx, fy, fz, fxz) the flow pattern and S_ab = sum lambda_a Q_b;
//   H:    dtz (S1 + S2), b: -cF S2 / b, with S1 = sum g mu.Q and
//         S2 = sum g^2 s mu.Q (s and the 2/Q0^2 term are 0 on the guard and
//         for Hookean springs).
struct RevSums {
    float sxx, syy, szz, sxz, s1, s2;
};

__device__ __forceinline__ void rev_flush(const RevSums& r, const GroupDev& G, double& gr, double& gH, double& gb) {
    const double dt = G.dt;
    double pr = 0.0;
    if (G.flow == 1) pr = dt * ((double)r.sxx - 0.5 * ((double)r.syy + (double)r.szz));
    else if (G.flow == 2) pr = dt * ((double)r.sxx - (double)r.syy);
    else if (G.flow == 3) pr = dt * (double)r.sxz;
    gr += pr;
    gH += (G.dt / G.zeta) * ((double)r.s1 + (double)r.s2);
    if (G.spring == 1) gb += -(double)G.cF * (double)r.s2 / G.b;
}

// Reverse step through Phi at the state q = Q^n; lambda holds lambda^{n+1}.
// kc.cF is 0 on slots that are not a spring of an active replica: their
// lambda starts at 0, gets no injection, and with a zero coefficient on the
// neighbour term stays 0 without a per-step select (their Q is 0, so they add
// nothing to the theta sums either).
template <int M, bool FENE>
__device__ __forceinline__ void reverse_step(const Lane<float, M>& q, const SlotCoef<float, M>& kc, const GroupDev& G,
                                             float (&lx)[M], float (&ly)[M], float (&lz)[M], RevSums& r) {
    const float kx = G.kx, ky = G.ky, kz = G.kz, kxz = G.kxz;
    const float plx = from_prev_lane(lx[M - 1]), ply = from_prev_lane(ly[M - 1]), plz = from_prev_lane(lz[M - 1]);
    const float nlx = from_next_lane(lx[0]), nly = from_next_lane(ly[0]), nlz = from_next_lane(lz[0]);
    float ux[M], uy[M], uz[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const float nx = (m + 1 < M) ? lx[m + 1 < M ? m + 1 : m] : nlx;
        const float ny = (m + 1 < M) ? ly[m + 1 < M ? m + 1 : m] : nly;
        const float nz = (m + 1 < M) ? lz[m + 1 < M ? m + 1 : m] : nlz;
        const float qx = (m > 0) ? lx[m > 0 ? m - 1 : 0] : plx;
        const float qy = (m > 0) ? ly[m > 0 ? m - 1 : 0] : ply;
        const float qz = (m > 0) ? lz[m > 0 ? m - 1 : 0] : plz;
        ux[m] = fmadd(-2.0f, lx[m], nx + qx);
        uy[m] = fmadd(-2.0f, ly[m], ny + qy);
        uz[m] = fmadd(-2.0f, lz[m], nz + qz);
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        float g, s;
        bool smooth;
        factor_gs<FENE>(q.qx[m], q.qy[m], q.qz[m], G, g, s, smooth);
        const float Qx = q.qx[m], Qy = q.qy[m], Qz = q.qz[m];
        // rate terms with lambda^{n+1}
        r.sxx = fmadd(lx[m], Qx, r.sxx);
        r.syy = fmadd(ly[m], Qy, r.syy);
        r.szz = fmadd(lz[m], Qz, r.szz);
        r.sxz = fmadd(lx[m], Qz, r.sxz);
        const float muQ = fmadd(ux[m], Qx, fmadd(uy[m], Qy, uz[m] * Qz));
        // lambda^n = lambda + (dt kappa)^T lambda + cF J mu with
        // J mu = g mu + (2 g^2 / Q0^2) (Q.mu) Q off the guard, g mu on it
        const float cg = kc.cF[m] * g;
        const float t = g * muQ;
        r.s1 += t;
        float ce = 0.0f;
        if constexpr (FENE) {
            const float ge = g * t;
            r.s2 = fmadd(ge, smooth ? s : 0.0f, r.s2);
            ce = kc.cF[m] * (smooth ? ge * (2.0f * G.inv_q0sq) : 0.0f);
        }
        const float nx = lx[m] + fmadd(kx, lx[m], fmadd(cg, ux[m], ce * Qx));
        const float ny = ly[m] + fmadd(ky, ly[m], fmadd(cg, uy[m], ce * Qy));
        const float nz = lz[m] + fmadd(kz, lz[m], fmadd(kxz, lx[m], fmadd(cg, uz[m], ce * Qz)));
        lx[m] = nx;
        ly[m] = ny;
        lz[m] = nz;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

template <int M, bool FENE, int NMAP>
__device__ __forceinline__ void run_adjoint(const AdjArgs& a, const GroupDev& G, int item, int k_first) {
    // kernel arguments into locals (the loops must not address the argument block)
    const int S = a.S, K = a.K;
    const int64_t n_end = a.n_end, ckpt_total = a.ckpt_total, spr_total = a.spr_total;
    const float* const ckpt = ckpt_item<const float, M>((const float*)a.ckpt, G, k_first);
    const double* const lam_mu = a.lam_mu;
    float* const seg = a.segbuf + a.seg_off[item];
    double* const partial = a.partial + 3 * item;
    const TileGeom tg = tile_geom(G, k_first, M);
    const int lane = threadIdx.x & (WAVE - 1);
    Lane<float, M> s, q, qn;
    bool valid[M];
    float lx[M], ly[M], lz[M];
#pragma unroll
    for (int m = 0; m < M; ++m) lx[m] = ly[m] = lz[m] = 0.0f;
    double gr = 0.0, gH = 0.0, gb = 0.0;      // FP64 totals
    int dummy = 0;
    const RoundKeys keys = round_keys<false>(a.key0, a.key1);
    SlotCoef<float, M> kc;
    constexpr int STRIDE = M * 3 * WAVE;      // floats per stored state
    const AdjArgs* ap = &a;                   // for inject(); not touched in the step loops
    const int n_seg = (int)((n_end + K - 1) / K);
    if (K == 1 && n_end > 0) {
        // Every state is a checkpoint: no recompute. The state after the last
        // step is rebuilt by one step from the last checkpoint; the sweep then
        // reads Q^n from checkpoint n (one step ahead), in the same order and
        // expressions as the segment loop below with segments of one step.
        const float* cp = ckpt + (int64_t)(n_end - 1) * ckpt_total;
        load_ckpt<float, M>(qn, valid, cp, G, tg);
        kc = slot_coef<float, M>(G, valid);
        s = qn;
        if constexpr (NMAP == 1) {
            Carry<float, M> cy;
            init_carry<float, M>(cy, G, (uint32_t)(n_end - 1), (uint32_t)tg.j0, (uint32_t)tg.k, keys);
            em_step_map1<float, M, FENE>(s, cy, G, valid, kc, (uint32_t)(n_end - 1), (uint32_t)tg.j0, (uint32_t)tg.k,
                                         keys, dummy);
        } else if constexpr (NMAP == 2) {
            em_step_map2<float, M, FENE>(s, G, valid, kc, (uint32_t)(n_end - 1), (uint32_t)tg.j0, (uint32_t)tg.k, keys,
                                         dummy);
        } else {
            em_step<float, M, FENE>(s, G, valid, kc, (uint32_t)(n_end - 1), (uint32_t)tg.j0, (uint32_t)tg.k, keys,
                                    dummy);
        }
        int rr = (int)(n_end % S);
        int w = (int)(n_end / S) - 1;
        RevSums rs{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        for (int n = (int)n_end - 1; n >= 0; --n) {
            q = qn;
            cp -= ckpt_total;
            if (n > 0) load_ckpt<float, M>(qn, valid, cp, G, tg);
            if (rr == 0) {
                double dH = 0.0, db = 0.0;
                inject<M, FENE>(s, valid, G, *ap, tg, w, lx, ly, lz, dH, db);
                gH += dH;
                gb += db;
                --w;
            }
            reverse_step<M, FENE>(q, kc, G, lx, ly, lz, rs);
            // FP32 partials over at most 128 steps, as the segments below hold
            // theirs over one checkpoint interval
            if ((n & 127) == 0) {
                rev_flush(rs, G, gr, gH, gb);
                rs = RevSums{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            }
            s = q;
            rr = rr == 0 ? S - 1 : rr - 1;
        }
    }
    for (int sgi = (K == 1 && n_end > 0) ? -1 : n_seg - 1; sgi >= 0; --sgi) {
        const int s0 = sgi * K;
        const int s1 = (int)min(n_end, (int64_t)s0 + K);
        load_ckpt<float, M>(s, valid, ckpt + (int64_t)sgi * ckpt_total, G, tg);
        kc = slot_coef<float, M>(G, valid);
        float* wp = seg;
        if constexpr (NMAP == 1) {
            Carry<float, M> cy;
            init_carry<float, M>(cy, G, (uint32_t)s0, (uint32_t)tg.j0, (uint32_t)tg.k, keys);
            int n = s0;
            if constexpr (M <= 2) {
                // aligned groups of four steps as in the forward: the group's
                // three blocks per slot drawn first, each step's transform just
                // before the step (the same normals as the carry gives)
                for (; n < s1 && (n & 3) != 0; ++n) {
                    seg_store<M>(wp, 0, s, lane);
                    wp += STRIDE;
                    em_step_map1<float, M, FENE>(s, cy, G, valid, kc, (uint32_t)n, (uint32_t)tg.j0, (uint32_t)tg.k,
                                                 keys, dummy);
                }
                for (; n + 4 <= s1; n += 4) {
                    Words w[3][M];
#pragma unroll
                    for (int q = 0; q < 3; ++q)
#pragma unroll
                        for (int m = 0; m < M; ++m)
                            w[q][m] = philox10((uint32_t)(n + q), (uint32_t)tg.j0 + (uint32_t)m, (uint32_t)tg.k, G.stream,
                                               keys);
                    Noise<float, M> e3;
#pragma unroll
                    for (int u = 0; u < 3; ++u) {
                        Noise<float, M> e;
#pragma unroll
                        for (int m = 0; m < M; ++m) {
                            float d;
                            normals4(w[u][m], e.x[m], e.y[m], e.z[m], d);
                            if (u == 0) e3.x[m] = d;
                            if (u == 1) e3.y[m] = d;
                            if (u == 2) e3.z[m] = d;
                        }
                        seg_store<M>(wp, 0, s, lane);
                        wp += STRIDE;
                        physics_step<float, M, FENE>(s, e, G, valid, kc, dummy);
                    }
                    seg_store<M>(wp, 0, s, lane);
                    wp += STRIDE;
                    physics_step<float, M, FENE>(s, e3, G, valid, kc, dummy);
                }
            }
            for (; n < s1; ++n) {
                seg_store<M>(wp, 0, s, lane);
                wp += STRIDE;
                em_step_map1<float, M, FENE>(s, cy, G, valid, kc, (uint32_t)n, (uint32_t)tg.j0, (uint32_t)tg.k, keys,
                                             dummy);
            }
        } else if constexpr (NMAP == 2) {
            for (int n = s0; n < s1; ++n) {
                seg_store<M>(wp, 0, s, lane);
                wp += STRIDE;
                em_step_map2<float, M, FENE>(s, G, valid, kc, (uint32_t)n, (uint32_t)tg.j0, (uint32_t)tg.k, keys,
                                             dummy);
            }
        } else {
            for (int n = s0; n < s1; ++n) {
                seg_store<M>(wp, 0, s, lane);
                wp += STRIDE;
                em_step<float, M, FENE>(s, G, valid, kc, (uint32_t)n, (uint32_t)tg.j0, (uint32_t)tg.k, keys, dummy);
            }
        }
        // s = Q^{s1}; sweep n = s1-1 .. s0, injecting at states n+1 that were sampled.
        // rr = (n + 1) mod S, w = window of state n + 1 when rr == 0
        int rr = s1 % S;
        int w = s1 / S - 1;
        RevSums rs{0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};   // FP32 partials of this segment
        const float* rp = seg + (int64_t)(s1 - 1 - s0) * STRIDE;
        seg_load<M>(rp, 0, qn, lane);           // Q^{s1-1}, loaded one step ahead
        for (int n = s1 - 1; n >= s0; --n) {
            q = qn;
            if (n > s0) seg_load<M>(rp - STRIDE, 0, qn, lane);
            rp -= STRIDE;
            if (rr == 0) {
                double dH = 0.0, db = 0.0;
                inject<M, FENE>(s, valid, G, *ap, tg, w, lx, ly, lz, dH, db);
                gH += dH;
                gb += db;
                --w;
            }
            reverse_step<M, FENE>(q, kc, G, lx, ly, lz, rs);
            s = q;
            rr = rr == 0 ? S - 1 : rr - 1;
        }
        rev_flush(rs, G, gr, gH, gb);
    }
    (void)spr_total;
    (void)lam_mu;
    gr = wave_sum(gr);
    gH = wave_sum(gH);
    gb = wave_sum(gb);
    if (lane == 0) {
        partial[0] = gr;
        partial[1] = gH;
        partial[2] = gb;
    }
}

// One kernel per beads-per-lane M, launched over the contiguous range of the
// (M-sorted) work list that uses it, so each M gets its own register budget.
template <int M, int NMAP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(M <= 2 ? 4 : 1)))
void adjoint_kernel(AdjArgs a, int item_begin, int item_end) {
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int item = item_begin + (int)blockIdx.x * (int)(blockDim.x >> 6) + wave;
    if (item >= item_end) return;
    const Item it = a.items[item];
    const GroupDev& G = a.groups[it.g];
    if constexpr (M <= 4) {
        // the group's constants as a local value: read through the reference,
        // the recompute loop re-loads them from memory every step
        const GroupDev Gl = G;
        if (Gl.spring == 1) run_adjoint<M, true, NMAP>(a, Gl, item, it.k0);
        else run_adjoint<M, false, NMAP>(a, Gl, item, it.k0);
    } else {   // noise map 1 is not compiled for wider lanes (rejected on the host)
        static_assert(NMAP != 1, "noise map 1 is compiled for 1-4 beads per lane");
        if (G.spring == 1) run_adjoint<M, true, NMAP>(a, G, item, it.k0);
        else run_adjoint<M, false, NMAP>(a, G, item, it.k0);
    }
}

// lam_mu[w][s] = grad_mean + grad_rates * dk/dmean, dk/dmean = k * x_dagger / kT.
__global__ __launch_bounds__(64) void lam_mu_kernel(const GroupDev* __restrict__ groups, const double* __restrict__ mean,
                                                    const double* __restrict__ gm, const double* __restrict__ grt,
                                                    double k0, double xd, int64_t spr_total, double* __restrict__ out) {
    const GroupDev& G = groups[blockIdx.x];
    const int64_t w = blockIdx.y;
    for (int j = threadIdx.x; j < G.N - 1; j += WAVE) {
        const int64_t o = w * spr_total + G.spr_off + j;
        double v = gm ? gm[o] : 0.0;
        if (grt) v += grt[o] * k0 * exp(xd * mean[o] / G.kT) * xd / G.kT;
        out[o] = v;
    }
}

// grad[g][p] = sum over the group's work items, one block per group in a
// fixed order: thread t sums items t, t + GR_THREADS, ... in order, then the
// threads' sums combine by a fixed-shape tree.
constexpr int GR_THREADS = 256;

__global__ __launch_bounds__(GR_THREADS) void grad_reduce_kernel(const int32_t* __restrict__ begin_count,
                                                                const double* __restrict__ partial,
                                                                double* __restrict__ grad) {
    __shared__ double sh[3][GR_THREADS];
    const int g = blockIdx.x;
    const int t = threadIdx.x;
    const int b = begin_count[2 * g], n = begin_count[2 * g + 1];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int i = t; i < n; i += GR_THREADS) {
        const double* q = partial + 3 * (int64_t)(b + i);
        a0 += q[0];
        a1 += q[1];
        a2 += q[2];
    }
    sh[0][t] = a0;
    sh[1][t] = a1;
    sh[2][t] = a2;
    __syncthreads();
    for (int h = GR_THREADS / 2; h >= 1; h >>= 1) {
        if (t < h) {
            sh[0][t] += sh[0][t + h];
            sh[1][t] += sh[1][t + h];
            sh[2][t] += sh[2][t + h];
        }
        __syncthreads();
    }
    if (t < 3) grad[3 * g + t] = sh[t][0];
}

hipError_t launch_adjoint(const AdjArgs& a, int M, int item_begin, int item_end, int waves_per_block, int nmap,
                          hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    const int n = item_end - item_begin;
    if (n <= 0) return hipSuccess;
    const int wpb = waves_per_block;
    dim3 grid((n + wpb - 1) / wpb), block(WAVE * wpb);
    if (nmap == 1) {
        switch (M) {
        case 1: hipLaunchKernelGGL((adjoint_kernel<1, 1>), grid, block, 0, st, a, item_begin, item_end); break;
        case 2: hipLaunchKernelGGL((adjoint_kernel<2, 1>), grid, block, 0, st, a, item_begin, item_end); break;
        case 3: hipLaunchKernelGGL((adjoint_kernel<3, 1>), grid, block, 0, st, a, item_begin, item_end); break;
        case 4: hipLaunchKernelGGL((adjoint_kernel<4, 1>), grid, block, 0, st, a, item_begin, item_end); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (nmap == 2) {   // whole groups of four beads per lane: 8, 12 or 16
        switch (M) {
        case 8: hipLaunchKernelGGL((adjoint_kernel<8, 2>), grid, block, 0, st, a, item_begin, item_end); break;
        case 12: hipLaunchKernelGGL((adjoint_kernel<12, 2>), grid, block, 0, st, a, item_begin, item_end); break;
        case 16: hipLaunchKernelGGL((adjoint_kernel<16, 2>), grid, block, 0, st, a, item_begin, item_end); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (M) {
    case 1: hipLaunchKernelGGL((adjoint_kernel<1, 0>), grid, block, 0, st, a, item_begin, item_end); break;
    case 2: hipLaunchKernelGGL((adjoint_kernel<2, 0>), grid, block, 0, st, a, item_begin, item_end); break;
    case 3: hipLaunchKernelGGL((adjoint_kernel<3, 0>), grid, block, 0, st, a, item_begin, item_end); break;
    case 4: hipLaunchKernelGGL((adjoint_kernel<4, 0>), grid, block, 0, st, a, item_begin, item_end); break;
    case 6: hipLaunchKernelGGL((adjoint_kernel<6, 0>), grid, block, 0, st, a, item_begin, item_end); break;
    case 8: hipLaunchKernelGGL((adjoint_kernel<8, 0>), grid, block, 0, st, a, item_begin, item_end); break;
    case 12: hipLaunchKernelGGL((adjoint_kernel<12, 0>), grid, block, 0, st, a, item_begin, item_end); break;
    case 16: hipLaunchKernelGGL((adjoint_kernel<16, 0>), grid, block, 0, st, a, item_begin, item_end); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lam_mu(const GroupDev* groups, int n_groups, int64_t n_windows, const double* mean,
                         const double* grad_mean, const double* grad_rates, double k0, double xd,
                         int64_t spr_total, double* lam_mu, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    if (n_windows == 0) return hipSuccess;
    hipLaunchKernelGGL(lam_mu_kernel, dim3((unsigned)n_groups, (unsigned)n_windows), dim3(64), 0, st, groups,
                       mean, grad_mean, grad_rates, k0, xd, spr_total, lam_mu);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const int32_t* item_begin, int n_groups, const double* partial,
                              double* grad_params, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    if (n_groups == 0) return hipSuccess;
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((unsigned)n_groups), dim3(GR_THREADS), 0, st, item_begin,
                       partial, grad_params);
    return hipGetLastError();
}

}  // namespace ra
