// ra_chain.hpp — per-lane chain state and the bond-form Euler-Maruyama step,
// shared by the forward kernels and the adjoint's segment recompute (which
// must reproduce the forward trajectory bit for bit).
//
// Bond form of Eq. (1) with the free-draining tensor Eq. (2):
//   Q_j' = Q_j + dt kappa Q_j + (H dt/zeta) [G_{j+1} - 2 G_j + G_{j-1}]
//          + sigma (xi_{j+1} - xi_j),   G_j = g_j Q_j,  sigma = sqrt(2 kT dt/zeta)
// which is the difference of the bead update r_i' = r_i + dt (kappa r_i +
// Fnet_i/zeta) + sigma xi_i for beads j+1 and j. The increment is formed
// first and added once, so FP32 keeps the small flow term dt*rate*Q exactly
// as accurate as the other terms.
#pragma once
#include "ra_device.hpp"
#include "ra_types.hpp"

namespace ra {

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T> struct Co;
template <> struct Co<float> {
    const GroupDev& G;
    __device__ float kx() const { return G.kx; }
    __device__ float ky() const { return G.ky; }
    __device__ float kz() const { return G.kz; }
    __device__ float kxz() const { return G.kxz; }
    __device__ float cF() const { return G.cF; }
    __device__ float sigma() const { return G.sigma; }
    __device__ float H() const { return G.H; }
    __device__ float iq() const { return G.inv_q0sq; }
};
template <> struct Co<double> {
    const GroupDev& G;
    __device__ double kx() const { return G.kx_d; }
    __device__ double ky() const { return G.ky_d; }
    __device__ double kz() const { return G.kz_d; }
    __device__ double kxz() const { return G.kxz_d; }
    __device__ double cF() const { return G.cF_d; }
    __device__ double sigma() const { return G.sigma_d; }
    __device__ double H() const { return G.H_d; }
    __device__ double iq() const { return G.inv_q0sq_d; }
};

// State of one lane: M bond slots.
template <typename T, int M> struct Lane {
    T qx[M], qy[M], qz[M];
};

// g_j for every slot (1 for Hookean), clamp count accumulated.
template <typename T, int M, bool FENE>
__device__ __forceinline__ void spring_factors(const Lane<T, M>& s, const GroupDev& G, T (&g)[M],
                                               int& clamps) {
#pragma unroll
    for (int m = 0; m < M; ++m) {
        if constexpr (FENE) {
            const T q2 = fmadd(s.qx[m], s.qx[m], fmadd(s.qy[m], s.qy[m], s.qz[m] * s.qz[m]));
            g[m] = fene_g(s.qx[m], s.qy[m], s.qz[m], q2, (T)G.inv_q0sq, G.inv_q0sq_d, clamps);
        } else {
            g[m] = (T)1;
        }
    }
}

// Normals of the M beads of the lane at one step (bead j uses the counter
// (step, bead j, replica, tag|group)); independent of the chain state, so the
// forward kernel generates several steps ahead for instruction-level parallelism.
template <typename T, int M> struct Noise {
    T x[M], y[M], z[M];
};

template <typename T, int M>
__device__ __forceinline__ void gen_noise(Noise<T, M>& e, const GroupDev& G, uint32_t n, uint32_t bead0,
                                          uint32_t replica, const RoundKeys& keys) {
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const Words w = philox10(n, bead0 + (uint32_t)m, replica, G.stream, keys);
        normals3(w, e.x[m], e.y[m], e.z[m]);
    }
}

// Noise map 1: the block of step n gives four normals; steps 4m..4m+2 use the
// first three of their own block, step 4m+3 the fourth normals of the blocks
// of steps 4m, 4m+1, 4m+2 (as x, y, z). Three blocks serve four steps, and
// every step still gets three independent standard normals. The fourth
// normals wait in a per-slot carry until step 4m+3.
template <typename T, int M> struct Carry {
    T c0[M], c1[M], c2[M];
};

// Normals of step n under map 1, updating the carry (r = n mod 4 is
// wave-uniform, so the branch is uniform and the carry slot a select).
template <typename T, int M>
__device__ __forceinline__ void gen_noise_map1(Noise<T, M>& e, Carry<T, M>& cy, const GroupDev& G, uint32_t n,
                                               uint32_t bead0, uint32_t replica, const RoundKeys& keys) {
    const uint32_t r = n & 3u;
    if (r == 3u) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            e.x[m] = cy.c0[m];
            e.y[m] = cy.c1[m];
            e.z[m] = cy.c2[m];
        }
        return;
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        T d;
        normals4(philox10(n, bead0 + (uint32_t)m, replica, G.stream, keys), e.x[m], e.y[m], e.z[m], d);
        cy.c0[m] = r == 0u ? d : cy.c0[m];
        cy.c1[m] = r == 1u ? d : cy.c1[m];
        cy.c2[m] = r == 2u ? d : cy.c2[m];
    }
}

// Carry for a run that starts at step n: the fourth normals of the blocks of
// steps 4m .. n-1 of n's group of four (none when n is a multiple of 4).
template <typename T, int M>
__device__ __forceinline__ void init_carry(Carry<T, M>& cy, const GroupDev& G, uint32_t n, uint32_t bead0,
                                           uint32_t replica, const RoundKeys& keys) {
    const uint32_t r = n & 3u;
#pragma unroll
    for (int m = 0; m < M; ++m) cy.c0[m] = cy.c1[m] = cy.c2[m] = (T)0;
    for (uint32_t q = 0; q < r; ++q) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            T a, b, c, d;
            normals4(philox10(n - r + q, bead0 + (uint32_t)m, replica, G.stream, keys), a, b, c, d);
            cy.c0[m] = q == 0u ? d : cy.c0[m];
            cy.c1[m] = q == 1u ? d : cy.c1[m];
            cy.c2[m] = q == 2u ? d : cy.c2[m];
        }
    }
}

// G_j = g_j Q_j of slot m (spring factor evaluated once per slot and step).
// With TSF the slot's tension f = H g |Q| of the same state is added to
// tsum[m] (Eq. 4, zero rest length): the step's force evaluation is the TSF
// sample of the state it starts from, so no second spring-law evaluation is
// needed for the time average.
template <typename T, int M, bool FENE, bool TSF = false>
__device__ __forceinline__ void slot_force(const Lane<T, M>& s, const GroupDev& G, int m, T& fx, T& fy, T& fz,
                                           int& clamps, T* tsum = nullptr) {
    T g = (T)1;
    T q2 = (T)0;
    if constexpr (FENE || TSF) q2 = fmadd(s.qx[m], s.qx[m], fmadd(s.qy[m], s.qy[m], s.qz[m] * s.qz[m]));
    if constexpr (FENE) g = fene_g(s.qx[m], s.qy[m], s.qz[m], q2, (T)G.inv_q0sq, G.inv_q0sq_d, clamps);
    if constexpr (TSF) tsum[m] = fmadd(Co<T>{G}.H() * g, fast_sqrt(q2), tsum[m]);
    fx = g * s.qx[m];
    fy = g * s.qy[m];
    fz = g * s.qz[m];
}

// Per-slot force and noise coefficients (H dt/zeta and sigma), zero on slots
// that are not a spring of an active replica. Such slots hold Q = 0, so with
// zero coefficients their increment is exactly 0 and they stay 0 without a
// per-step select. Used for up to 4 slots per lane; wider lanes keep the
// coefficients in scalar registers and select instead.
template <typename T, int M> struct SlotCoef {
    T cF[M], sg[M];
};

template <typename T, int M>
__device__ __forceinline__ SlotCoef<T, M> slot_coef(const GroupDev& G, const bool (&valid)[M]) {
    const Co<T> c{G};
    SlotCoef<T, M> k;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        k.cF[m] = valid[m] ? c.cF() : (T)0;
        k.sg[m] = valid[m] ? c.sigma() : (T)0;
    }
    return k;
}

template <int M> struct MaskedSlots { static constexpr bool value = M <= 4; };

// One Euler-Maruyama step of every slot of the lane. xi(m, x, y, z) yields
// the normals of bead j0 + m (precomputed or generated on demand — the value
// is the same). The update of slot m needs G and xi of slots m-1..m+1 only,
// so both roll through three-slot windows; the lane's first/last slots meet
// the neighbour lanes' through DPP. valid[m] masks slots that are not a
// spring of an active replica.
// xnext(e0, en) gives the next lane's bead-0 normals (by DPP from e0 unless the
// caller has them at hand, e.g. in LDS).
template <typename T, int M, bool FENE, bool TSF = false, typename NoiseFn, typename NextFn>
__device__ __forceinline__ void physics_step_core(Lane<T, M>& s, NoiseFn&& xi, NextFn&& xnext,
                                                  const GroupDev& G, const bool (&valid)[M],
                                                  const SlotCoef<T, M>& kc, int& clamps, T* tsum = nullptr) {
    const Co<T> c{G};
    T f0x, f0y, f0z, flx, fly, flz;
    slot_force<T, M, FENE, TSF>(s, G, 0, f0x, f0y, f0z, clamps, tsum);
    if constexpr (M > 1) {
        slot_force<T, M, FENE, TSF>(s, G, M - 1, flx, fly, flz, clamps, tsum);
    } else {
        flx = f0x; fly = f0y; flz = f0z;
    }
    const T fpx = from_prev_lane(flx), fpy = from_prev_lane(fly), fpz = from_prev_lane(flz);
    const T fnx = from_next_lane(f0x), fny = from_next_lane(f0y), fnz = from_next_lane(f0z);
    T e0x, e0y, e0z, enx, eny, enz;
    xi(0, e0x, e0y, e0z);
    xnext(e0x, e0y, e0z, enx, eny, enz);
    const T kx = c.kx(), ky = c.ky(), kz = c.kz(), kxz = c.kxz();
    T Px = fpx, Py = fpy, Pz = fpz;   // G of slot m-1
    T Cx = f0x, Cy = f0y, Cz = f0z;   // G of slot m
    T Ex = e0x, Ey = e0y, Ez = e0z;   // xi of bead m
#pragma unroll
    for (int m = 0; m < M; ++m) {
        T Nx, Ny, Nz, Xx, Xy, Xz;     // G of slot m+1, xi of bead m+1
        if (m + 1 < M) {
            if (m + 1 == M - 1) { Nx = flx; Ny = fly; Nz = flz; }
            else slot_force<T, M, FENE, TSF>(s, G, m + 1 < M ? m + 1 : m, Nx, Ny, Nz, clamps, tsum);
            xi(m + 1, Xx, Xy, Xz);
        } else {
            Nx = fnx; Ny = fny; Nz = fnz;
            Xx = enx; Xy = eny; Xz = enz;
        }
        const T lx = fmadd((T)-2, Cx, Nx + Px);
        const T ly = fmadd((T)-2, Cy, Ny + Py);
        const T lz = fmadd((T)-2, Cz, Nz + Pz);
        constexpr bool masked = MaskedSlots<M>::value;
        const T cF = masked ? kc.cF[m] : c.cF();
        const T sg = masked ? kc.sg[m] : c.sigma();
        const T ix = fmadd(kx, s.qx[m], fmadd(kxz, s.qz[m], fmadd(cF, lx, sg * (Xx - Ex))));
        const T iy = fmadd(ky, s.qy[m], fmadd(cF, ly, sg * (Xy - Ey)));
        const T iz = fmadd(kz, s.qz[m], fmadd(cF, lz, sg * (Xz - Ez)));
        if constexpr (masked) {
            s.qx[m] += ix;
            s.qy[m] += iy;
            s.qz[m] += iz;
        } else {
            s.qx[m] = valid[m] ? s.qx[m] + ix : (T)0;
            s.qy[m] = valid[m] ? s.qy[m] + iy : (T)0;
            s.qz[m] = valid[m] ? s.qz[m] + iz : (T)0;
        }
        Px = Cx; Py = Cy; Pz = Cz;
        Cx = Nx; Cy = Ny; Cz = Nz;
        Ex = Xx; Ey = Xy; Ez = Xz;
    }
}

template <typename T, int M, bool FENE, bool TSF = false, typename NoiseFn>
__device__ __forceinline__ void physics_step_fn(Lane<T, M>& s, NoiseFn&& xi, const GroupDev& G,
                                                const bool (&valid)[M], const SlotCoef<T, M>& kc,
                                                int& clamps, T* tsum = nullptr) {
    physics_step_core<T, M, FENE, TSF>(
        s, xi,
        [](T ex, T ey, T ez, T& nx, T& ny, T& nz) {
            nx = from_next_lane(ex);
            ny = from_next_lane(ey);
            nz = from_next_lane(ez);
        },
        G, valid, kc, clamps, tsum);
}

template <typename T, int M, bool FENE, bool TSF = false>
__device__ __forceinline__ void physics_step(Lane<T, M>& s, const Noise<T, M>& e, const GroupDev& G,
                                             const bool (&valid)[M], const SlotCoef<T, M>& kc, int& clamps,
                                             T* tsum = nullptr) {
    physics_step_fn<T, M, FENE, TSF>(
        s, [&](int m, T& x, T& y, T& z) { x = e.x[m]; y = e.y[m]; z = e.z[m]; }, G, valid, kc, clamps, tsum);
}

// One full Euler-Maruyama step at global step n (noise + update).
template <typename T, int M, bool FENE, bool TSF = false>
__device__ __forceinline__ void em_step(Lane<T, M>& s, const GroupDev& G, const bool (&valid)[M],
                                        const SlotCoef<T, M>& kc, uint32_t n, uint32_t bead0,
                                        uint32_t replica, const RoundKeys& keys, int& clamps, T* tsum = nullptr) {
    physics_step_fn<T, M, FENE, TSF>(
        s,
        [&](int m, T& x, T& y, T& z) {
            normals3(philox10(n, bead0 + (uint32_t)m, replica, G.stream, keys), x, y, z);
        },
        G, valid, kc, clamps, tsum);
}

// One step at global step n under map 1 (noise from and into the carry).
template <typename T, int M, bool FENE, bool TSF = false>
__device__ __forceinline__ void em_step_map1(Lane<T, M>& s, Carry<T, M>& cy, const GroupDev& G,
                                             const bool (&valid)[M], const SlotCoef<T, M>& kc, uint32_t n,
                                             uint32_t bead0, uint32_t replica, const RoundKeys& keys, int& clamps,
                                             T* tsum = nullptr) {
    Noise<T, M> e;
    gen_noise_map1<T, M>(e, cy, G, n, bead0, replica, keys);
    physics_step<T, M, FENE, TSF>(s, e, G, valid, kc, clamps, tsum);
}

// Noise map 2, for lanes of a multiple of four beads (the lane's first bead
// is then a multiple of four too): the beads are taken in groups of four,
// j = 4q + r, and the three blocks of counters (step, 3q + c, replica,
// tag|group), c = 0, 1, 2, give four normals each; bead 4q + r takes normal r
// of block c as its component c. Three blocks serve four bead-steps, as under
// map 1, but with no carry from step to step. The step's Philox blocks are
// drawn first (integer work with twelve independent chains at 16 beads per
// lane) and each group's Box-Muller transform runs when the update reaches
// the group's first bead, which spreads the transcendentals over the step
// (measured on 16 beads per lane: 2% faster than transforming all twelve
// blocks up front, 4% faster than drawing and transforming each group at its
// first bead).
template <typename T, int M, bool FENE, bool TSF = false>
__device__ __forceinline__ void em_step_map2(Lane<T, M>& s, const GroupDev& G, const bool (&valid)[M],
                                             const SlotCoef<T, M>& kc, uint32_t n, uint32_t bead0,
                                             uint32_t replica, const RoundKeys& keys, int& clamps,
                                             T* tsum = nullptr) {
    static_assert(M % 4 == 0, "noise map 2 takes the beads of a lane in groups of four");
    Words w[M / 4][3];
#pragma unroll
    for (int g = 0; g < M / 4; ++g) {
        const uint32_t b = 3u * ((bead0 >> 2) + (uint32_t)g);
#pragma unroll
        for (int c = 0; c < 3; ++c) w[g][c] = philox10(n, b + (uint32_t)c, replica, G.stream, keys);
    }
    T gx[4], gy[4], gz[4];
    physics_step_fn<T, M, FENE, TSF>(
        s,
        [&](int m, T& x, T& y, T& z) {
            if ((m & 3) == 0) {
                normals4(w[m >> 2][0], gx[0], gx[1], gx[2], gx[3]);
                normals4(w[m >> 2][1], gy[0], gy[1], gy[2], gy[3]);
                normals4(w[m >> 2][2], gz[0], gz[1], gz[2], gz[3]);
            }
            x = gx[m & 3];
            y = gy[m & 3];
            z = gz[m & 3];
        },
        G, valid, kc, clamps, tsum);
}

// Tension f_j = H g_j |Q_j| (Eq. 4, zero rest length) of every slot.
template <typename T, int M, bool FENE>
__device__ __forceinline__ void tensions(const Lane<T, M>& s, const GroupDev& G, T (&f)[M]) {
    int dummy = 0;
    T g[M];
    spring_factors<T, M, FENE>(s, G, g, dummy);
    const T H = Co<T>{G}.H();
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const T q2 = fmadd(s.qx[m], s.qx[m], fmadd(s.qy[m], s.qy[m], s.qz[m] * s.qz[m]));
        f[m] = H * g[m] * fast_sqrt(q2);
    }
}

struct TileGeom {
    int t, k;          // lane position in its replica, replica index
    bool rep_ok;       // lane belongs to an existing replica
    int j0;            // first bead/spring of the lane
};

// With UNIFORM_K (one replica per wavefront, P = 1) every lane carries the
// wave-uniform replica index, so the replica word of the Philox counter stays
// in a scalar register and part of the first rounds runs on the scalar unit.
template <bool UNIFORM_K = false>
__device__ __forceinline__ TileGeom tile_geom(const GroupDev& G, int k_first, int M) {
    const int lane = threadIdx.x & (WAVE - 1);
    TileGeom tg;
    if constexpr (UNIFORM_K) {
        tg.t = lane;
        tg.k = k_first;
        tg.rep_ok = (lane < G.L) && (k_first < G.R);
    } else {
        const int seg = lane / G.L;
        tg.t = lane - seg * G.L;
        tg.k = k_first + seg;
        tg.rep_ok = (seg < G.P) && (tg.k < G.R);
    }
    tg.j0 = tg.t * M;
    return tg;
}

template <typename T, int M>
__device__ __forceinline__ void load_lane(Lane<T, M>& s, bool (&valid)[M], const T* __restrict__ src,
                                          const GroupDev& G, const TileGeom& tg) {
    const int nm1 = G.N - 1;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int j = tg.j0 + m;
        valid[m] = tg.rep_ok && j < nm1;
        T x = (T)0, y = (T)0, z = (T)0;
        if (valid[m]) {
            const int64_t o = G.state_off + ((int64_t)tg.k * nm1 + j) * 3;
            x = src[o];
            y = src[o + 1];
            z = src[o + 2];
        }
        s.qx[m] = x;
        s.qy[m] = y;
        s.qz[m] = z;
    }
}

template <typename T, int M>
__device__ __forceinline__ void store_lane(const Lane<T, M>& s, const bool (&valid)[M], T* __restrict__ dst,
                                           const GroupDev& G, const TileGeom& tg) {
    const int nm1 = G.N - 1;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        if (valid[m]) {
            const int64_t o = G.state_off + ((int64_t)tg.k * nm1 + tg.j0 + m) * 3;
            dst[o] = s.qx[m];
            dst[o + 1] = s.qy[m];
            dst[o + 2] = s.qz[m];
        }
    }
}

// Checkpoint rows of one work item: [slot m][xyz][lane], U = P L lanes per
// row, so each store or load instruction covers U consecutive values. Slots
// that are not a spring of a replica hold 0.
template <typename T, int M>
__device__ __forceinline__ T* ckpt_item(T* base, const GroupDev& G, int k_first) {
    return base + G.ck_off + (int64_t)(k_first / G.P) * (M * 3 * G.P * G.L);
}

template <typename T, int M>
__device__ __forceinline__ void store_ckpt(const Lane<T, M>& s, T* __restrict__ dst, const GroupDev& G) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int U = G.P * G.L;
    if (lane < U) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            dst[(3 * m) * U + lane] = s.qx[m];
            dst[(3 * m + 1) * U + lane] = s.qy[m];
            dst[(3 * m + 2) * U + lane] = s.qz[m];
        }
    }
}

template <typename T, int M>
__device__ __forceinline__ void load_ckpt(Lane<T, M>& s, bool (&valid)[M], const T* __restrict__ src,
                                          const GroupDev& G, const TileGeom& tg) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int U = G.P * G.L;
    const int nm1 = G.N - 1;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        valid[m] = tg.rep_ok && tg.j0 + m < nm1;
        T x = (T)0, y = (T)0, z = (T)0;
        if (valid[m] && lane < U) {
            x = src[(3 * m) * U + lane];
            y = src[(3 * m + 1) * U + lane];
            z = src[(3 * m + 2) * U + lane];
        }
        s.qx[m] = x;
        s.qy[m] = y;
        s.qz[m] = z;
    }
}

__device__ __forceinline__ void flush_clamps(int clamps, unsigned long long* counter) {
    if (clamps) atomicAdd(counter, (unsigned long long)clamps);
}

}  // namespace ra
