// ra_pair.hip — forward kernel of the collapsed-polymer force field (Sec. II):
// backbone springs (rest-length harmonic kappa/2 (r - r0)^2, or the Hookean
// and FENE laws) plus Lennard-Jones self-association between non-adjacent
// beads, free-draining (Eq. 1 with the self term Eq. 2 only).
//
// One bead per lane, P = floor(64/N) replicas per wavefront (N <= 64). The
// state stays the bond vectors Q_j (as in the chain kernels, so FP32 keeps
// bond-scale precision however far the chain drifts in the flow); the bead
// positions relative to bead 0 are rebuilt every step by a wave scan of the
// bonds (DPP with one replica per wavefront, lane shuffles per segment with
// several) and shared through LDS for the O(N^2) pair forces. The
// bond update is the difference of the bead updates of beads j+1 and j:
//   Q_j' = Q_j + dt kappa Q_j + (dt/zeta) (F_{j+1} - F_j) + sigma (xi_{j+1} - xi_j)
// with F_i the total force on bead i (springs + LJ).
#include "ra_chain.hpp"
#include "ra_dpp.hpp"
#include "ra_launch.hpp"

namespace ra {

template <typename T> struct PairCo;
template <> struct PairCo<float> {
    const GroupDev& G;
    __device__ float dtz() const { return G.dtz; }
    __device__ float r0() const { return G.r0; }
};
template <> struct PairCo<double> {
    const GroupDev& G;
    __device__ double dtz() const { return G.dtz_d; }
    __device__ double r0() const { return G.r0_d; }
};

// Force of the spring on bond Q acting on its first bead (toward the second).
template <typename T, int SPRING>
__device__ __forceinline__ void pair_spring_force(T qx, T qy, T qz, const GroupDev& G, T& fx, T& fy, T& fz,
                                                  int& clamps) {
    const T H = Co<T>{G}.H();
    const T q2 = fmadd(qx, qx, fmadd(qy, qy, qz * qz));
    T g;
    if constexpr (SPRING == 0) {
        g = (T)1;
    } else if constexpr (SPRING == 1) {
        g = fene_g(qx, qy, qz, q2, (T)G.inv_q0sq, G.inv_q0sq_d, clamps);
    } else {
        const T q = fast_sqrt(q2);
        g = q > (T)0 ? (T)1 - PairCo<T>{G}.r0() * fast_rcp(q) : (T)0;
    }
    const T Hg = H * g;
    fx = Hg * qx;
    fy = Hg * qy;
    fz = Hg * qz;
}

// Spring tension of Eq. 4: signed H (|Q| - r0) for the rest-length spring,
// H g |Q| for the zero-rest-length laws.
template <typename T, int SPRING>
__device__ __forceinline__ T pair_tension(T qx, T qy, T qz, const GroupDev& G) {
    const T H = Co<T>{G}.H();
    const T q2 = fmadd(qx, qx, fmadd(qy, qy, qz * qz));
    const T q = fast_sqrt(q2);
    if constexpr (SPRING == 2) {
        return H * (q - PairCo<T>{G}.r0());
    } else if constexpr (SPRING == 1) {
        int dummy = 0;
        return H * fene_g(qx, qy, qz, q2, (T)G.inv_q0sq, G.inv_q0sq_d, dummy) * q;
    } else {
        return H * q;
    }
}

// Inclusive scan of v over the lanes of each replica segment (bead index i
// within the segment): after it, lane i holds the sum over beads 0..i.
template <typename T>
__device__ __forceinline__ T segment_scan(T v, int i) {
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        const T u = __shfl_up(v, (unsigned)off, WAVE);
        if (i >= off) v += u;
    }
    return v;
}

template <typename T, int SPRING, bool LJ>
__device__ __forceinline__ void run_pair(const FwdArgs& a, const GroupDev& Gm, int k_first, T (*xs)[4]) {
    // the group's constants as a local value: read through the reference,
    // the step loop re-loads them from memory every iteration
    const GroupDev G = Gm;
    const int gidx = (int)(&Gm - a.groups);
    const int lane = threadIdx.x & (WAVE - 1);
    const int N = G.N, nm1 = N - 1;
    const int seg = lane / N;
    const int i = lane - seg * N;
    const int k = k_first + seg;
    const bool rep_ok = seg < G.P && k < G.R;
    const bool bond_ok = rep_ok && i < nm1;
    T* const state = (T*)a.state;
    const int64_t sidx = ((int64_t)k * nm1 + i);
    T qx = (T)0, qy = (T)0, qz = (T)0;
    if (bond_ok) {
        const int64_t o = G.state_off + sidx * 3;
        qx = state[o];
        qy = state[o + 1];
        qz = state[o + 2];
    }
    const Co<T> c{G};
    const PairCo<T> pc{G};
    // coefficients are zero on lanes without a bond
    const T kx = bond_ok ? c.kx() : (T)0, ky = bond_ok ? c.ky() : (T)0, kz = bond_ok ? c.kz() : (T)0;
    const T kxz = bond_ok ? c.kxz() : (T)0;
    const T dtz = bond_ok ? pc.dtz() : (T)0, sg = bond_ok ? c.sigma() : (T)0;
    // LJ in units of rmin: positions scaled by 1/rmin, the pair sum scaled
    // back by 12 u / rmin at the end
    const T irm = (T)(1.0 / sqrt(G.ljr2_d)), ljf = (T)(G.lj12u_d / sqrt(G.ljr2_d));
    // LDS rows of this lane's replica: its positions twice over (rows
    // tb .. tb + 2N - 1), so that partner i + t is row tb + i + t for every
    // t < N; lanes past the last segment read segment 0 and write nothing
    const bool seg_ok = seg < G.P;
    const bool one_seg = G.P == 1;
    const int tb = seg_ok ? 2 * N * seg : 0;
    const RoundKeys keys = round_keys(a.key0, a.key1);
    const uint32_t n0 = (uint32_t)*a.step0;
    const int S = a.S;
    const int64_t smp_total = a.smp_total;
    const bool tsf = a.tsf != nullptr;
    double acc = 0.0;
    if (tsf && bond_ok) acc = a.tsf_acc[G.smp_off + sidx];
    int to_smp = S - (int)(n0 % (uint32_t)S);
    int64_t w = (int64_t)(n0 / (uint32_t)S);
    int clamps = 0;
    const int n_steps = (int)a.n_steps;
    for (int st = 0; st < n_steps; ++st) {
        const uint32_t n = n0 + (uint32_t)st;
        T gx, gy, gz;
        pair_spring_force<T, SPRING>(qx, qy, qz, G, gx, gy, gz, clamps);
        // net force on bead i: spring i pulls toward i+1, spring i-1 pulls back
        // (the previous lane of bead 0 is the bondless last bead of the
        // previous replica, or lane -1, and contributes 0)
        T Fx = gx - from_prev_lane(gx), Fy = gy - from_prev_lane(gy), Fz = gz - from_prev_lane(gz);
        if constexpr (LJ) {
            // one replica per wavefront (N > 32): the whole-wave DPP scan;
            // else the segmented scan by lane shuffles
            T sx, sy, sz;
            if (one_seg) {
                sx = wave_scan_incl(qx);
                sy = wave_scan_incl(qy);
                sz = wave_scan_incl(qz);
            } else {
                sx = segment_scan(qx, i);
                sy = segment_scan(qy, i);
                sz = segment_scan(qz, i);
            }
            const T px = (sx - qx) * irm, py = (sy - qy) * irm, pz = (sz - qz) * irm;
            if (seg_ok) {
                xs[tb + i][0] = px;
                xs[tb + i][1] = py;
                xs[tb + i][2] = pz;
                xs[tb + i + N][0] = px;
                xs[tb + i + N][1] = py;
                xs[tb + i + N][2] = pz;
            }
            // this wave alone uses its LDS rows: make the writes visible to
            // its own reads (and keep the next step's writes after them)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // Partners i + t (mod N) of the replica, read from the doubled
            // table at rows i + t (no wrap test). t = 2 .. N - 2 are never
            // bonded neighbours nor the bead itself, so that loop carries no
            // mask; t = 1 and t = N - 1 meet the bonded neighbours except across
            // the wrap-around (bead N-1 with bead 0), where the pair counts
            // for N >= 3. In units of rmin: s = rmin^2 / r^2 is the reciprocal
            // of the scaled r^2, and the pair term is s (s^6 - s^3) dx'.
            const T* row = xs[tb + i];
            T lx = (T)0, ly = (T)0, lz = (T)0;
            const bool wrap_first = N >= 3 && i == nm1, wrap_last = N >= 3 && i == 0;
            {
                const T dx = px - row[4 * 1], dy = py - row[4 * 1 + 1], dz = pz - row[4 * 1 + 2];
                const T s = fast_rcp(fmadd(dx, dx, fmadd(dy, dy, dz * dz)));
                const T s3 = s * s * s;
                // a select, not a product: drops the Inf/NaN of a coincident
                // bonded neighbour
                const T h = wrap_first ? s * fmadd(s3, s3, -s3) : (T)0;
                lx = h * dx;
                ly = h * dy;
                lz = h * dz;
            }
            // t = 2 .. N - 1 in blocks of 8 (independent reciprocal chains for
            // the single wavefront per SIMD, all eight LDS reads in flight):
            // whole blocks of t < N - 1 unmasked, then one block that holds
            // t = N - 1 (the wrap-around pair of bead 0) and reads row N - 1
            // with weight 0 past it
            int t0 = 2;
            auto load8 = [&](T (&bx)[8], T (&by)[8], T (&bz)[8], int tb0) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const T* r = row + 4 * (tb0 + u);
                    bx[u] = r[0];
                    by[u] = r[1];
                    bz[u] = r[2];
                }
            };
            auto pairs8 = [&](const T (&bx)[8], const T (&by)[8], const T (&bz)[8]) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const T dx = px - bx[u], dy = py - by[u], dz = pz - bz[u];
                    const T s = fast_rcp(fmadd(dx, dx, fmadd(dy, dy, dz * dz)));
                    const T s3 = s * s * s;
                    const T h = s * fmadd(s3, s3, -s3);
                    lx = fmadd(h, dx, lx);
                    ly = fmadd(h, dy, ly);
                    lz = fmadd(h, dz, lz);
                }
            };
            if constexpr (sizeof(T) == 4) {
                // FP32: whole blocks with their reads at the top. The pipelined
                // form below was slower here (37.9 against 33.6 ms for
                // collapsed50's 15,000 steps) and faster in FP64 (14.5 against
                // 17.3 ms for 3,000 steps), where the reciprocal is a division.
                for (; t0 + 8 <= nm1; t0 += 8) {
                    T ax[8], ay[8], az[8];
                    load8(ax, ay, az, t0);
                    pairs8(ax, ay, az);
                }
            } else if (t0 + 8 <= nm1) {
                // FP64: software pipeline over whole blocks, two register
                // buffers in turn, so that the next block's eight reads are
                // issued before this block's arithmetic
                T ax[8], ay[8], az[8], bx[8], by[8], bz[8];
                load8(ax, ay, az, t0);
                for (;;) {
                    const bool more_b = t0 + 16 <= nm1;
                    if (more_b) load8(bx, by, bz, t0 + 8);
                    pairs8(ax, ay, az);
                    t0 += 8;
                    if (!more_b) break;
                    const bool more_a = t0 + 16 <= nm1;
                    if (more_a) load8(ax, ay, az, t0 + 8);
                    pairs8(bx, by, bz);
                    t0 += 8;
                    if (!more_a) break;
                }
            }
            if (t0 <= nm1) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int t = t0 + u;
                    const T* r = row + 4 * (t < nm1 ? t : nm1);
                    const bool use = t < nm1 || (t == nm1 && wrap_last);
                    const T dx = px - r[0], dy = py - r[1], dz = pz - r[2];
                    const T s = fast_rcp(fmadd(dx, dx, fmadd(dy, dy, dz * dz)));
                    const T s3 = s * s * s;
                    // a select: drops the Inf/NaN of a coincident bonded neighbour
                    const T h = use ? s * fmadd(s3, s3, -s3) : (T)0;
                    lx = fmadd(h, dx, lx);
                    ly = fmadd(h, dy, ly);
                    lz = fmadd(h, dz, lz);
                }
            }
            lx *= ljf;
            ly *= ljf;
            lz *= ljf;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            Fx += lx;
            Fy += ly;
            Fz += lz;
        }
        T ex, ey, ez;
        normals3(philox10(n, (uint32_t)i, (uint32_t)k, G.stream, keys), ex, ey, ez);
        const T Fnx = from_next_lane(Fx), Fny = from_next_lane(Fy), Fnz = from_next_lane(Fz);
        const T enx = from_next_lane(ex), eny = from_next_lane(ey), enz = from_next_lane(ez);
        const T ix = fmadd(kx, qx, fmadd(kxz, qz, fmadd(dtz, Fnx - Fx, sg * (enx - ex))));
        const T iy = fmadd(ky, qy, fmadd(dtz, Fny - Fy, sg * (eny - ey)));
        const T iz = fmadd(kz, qz, fmadd(dtz, Fnz - Fz, sg * (enz - ez)));
        // lanes without a bond keep Q = 0 whatever their neighbours hold
        qx = bond_ok ? qx + ix : (T)0;
        qy = bond_ok ? qy + iy : (T)0;
        qz = bond_ok ? qz + iz : (T)0;
        const bool window_end = --to_smp == 0;
        if (tsf || window_end) {
            const T f = pair_tension<T, SPRING>(qx, qy, qz, G);
            if (tsf) acc += (double)f;
            if (window_end) {
                bool bad = false;
                if (bond_ok) {
                    const int64_t o = w * smp_total + G.smp_off + sidx;
                    ((T*)a.samples)[o] = f;
                    bad = !__builtin_isfinite((double)f);
                    if (tsf) {
                        ((T*)a.tsf)[o] = (T)(acc / (double)S);
                        acc = 0.0;
                    }
                }
                if (bad) atomicOr(a.status, 2);
                to_smp = S;
                ++w;
            }
        }
    }
    if (bond_ok) {
        const int64_t o = G.state_off + sidx * 3;
        state[o] = qx;
        state[o + 1] = qy;
        state[o + 2] = qz;
        if (tsf) a.tsf_acc[G.smp_off + sidx] = acc;
    }
    flush_clamps(clamps, a.clamps + gidx);
}

template <typename T>
__device__ __forceinline__ void pair_item(const FwdArgs& a, int item, T (*xs)[4]) {
    if (item >= a.n_items) return;
    if (*(const volatile int*)a.status & 1) return;   // invalid parent: no work
    const Item it = a.items[item];
    const GroupDev& G = a.groups[it.g];
    const bool lj = G.lj12u_d > 0.0;
    switch (G.spring * 2 + (lj ? 1 : 0)) {
    case 0: run_pair<T, 0, false>(a, G, it.k0, xs); break;
    case 1: run_pair<T, 0, true>(a, G, it.k0, xs); break;
    case 2: run_pair<T, 1, false>(a, G, it.k0, xs); break;
    case 3: run_pair<T, 1, true>(a, G, it.k0, xs); break;
    case 4: run_pair<T, 2, false>(a, G, it.k0, xs); break;
    default: run_pair<T, 2, true>(a, G, it.k0, xs); break;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void fwd_pair_kernel(FwdArgs a) {
    __shared__ T xs[4][2 * WAVE][4];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    pair_item<T>(a, (int)blockIdx.x * (int)(blockDim.x >> 6) + wave, xs[wave]);
}

// Two contexts in one launch (see fwd_dual_kernel): blocks [0, blocks_a) run a.
template <typename T>
__global__ __launch_bounds__(256) void fwd_pair_dual_kernel(FwdArgs a, FwdArgs b, int blocks_a) {
    __shared__ T xs[4][2 * WAVE][4];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wpb = (int)(blockDim.x >> 6);
    if ((int)blockIdx.x < blocks_a) pair_item<T>(a, (int)blockIdx.x * wpb + wave, xs[wave]);
    else pair_item<T>(b, ((int)blockIdx.x - blocks_a) * wpb + wave, xs[wave]);
}

hipError_t launch_forward_pair(const FwdArgs& a, int precision, int waves_per_block, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    if (a.n_items <= 0 || a.n_steps <= 0) return hipSuccess;
    const int wpb = waves_per_block;
    dim3 grid((a.n_items + wpb - 1) / wpb), block(WAVE * wpb);
    if (precision == 64) hipLaunchKernelGGL(fwd_pair_kernel<double>, grid, block, 0, st, a);
    else hipLaunchKernelGGL(fwd_pair_kernel<float>, grid, block, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_forward_pair_dual(const FwdArgs& a, const FwdArgs& b, int precision, int waves_per_block,
                                    hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    const int wpb = waves_per_block;
    const int ba = (a.n_items + wpb - 1) / wpb, bb = (b.n_items + wpb - 1) / wpb;
    if (ba + bb == 0) return hipSuccess;
    dim3 grid((unsigned)(ba + bb)), block(WAVE * wpb);
    if (precision == 64) hipLaunchKernelGGL(fwd_pair_dual_kernel<double>, grid, block, 0, st, a, b, ba);
    else hipLaunchKernelGGL(fwd_pair_dual_kernel<float>, grid, block, 0, st, a, b, ba);
    return hipGetLastError();
}

}  // namespace ra
