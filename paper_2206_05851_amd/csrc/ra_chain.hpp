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

// One Euler-Maruyama step of every slot of the lane, at global step n.
// valid[m] masks slots that are not a spring of an active replica.
template <typename T, int M, bool FENE>
__device__ __forceinline__ void em_step(Lane<T, M>& s, const GroupDev& G, const bool (&valid)[M],
                                        uint32_t n, uint32_t bead0, uint32_t replica,
                                        uint32_t key0, uint32_t key1, int& clamps) {
    const Co<T> c{G};
    T g[M];
    spring_factors<T, M, FENE>(s, G, g, clamps);
    T fx[M], fy[M], fz[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        fx[m] = g[m] * s.qx[m];
        fy[m] = g[m] * s.qy[m];
        fz[m] = g[m] * s.qz[m];
    }
    const T fpx = from_prev_lane(fx[M - 1]), fpy = from_prev_lane(fy[M - 1]), fpz = from_prev_lane(fz[M - 1]);
    const T fnx = from_next_lane(fx[0]), fny = from_next_lane(fy[0]), fnz = from_next_lane(fz[0]);
    T ex[M], ey[M], ez[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const Words w = philox10(n, bead0 + (uint32_t)m, replica, G.stream, key0, key1);
        normals3(w, ex[m], ey[m], ez[m]);
    }
    const T enx = from_next_lane(ex[0]), eny = from_next_lane(ey[0]), enz = from_next_lane(ez[0]);
    const T kx = c.kx(), ky = c.ky(), kz = c.kz(), kxz = c.kxz(), cF = c.cF(), sg = c.sigma();
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const T nx = (m + 1 < M) ? fx[m + 1 < M ? m + 1 : m] : fnx;
        const T ny = (m + 1 < M) ? fy[m + 1 < M ? m + 1 : m] : fny;
        const T nz = (m + 1 < M) ? fz[m + 1 < M ? m + 1 : m] : fnz;
        const T px = (m > 0) ? fx[m > 0 ? m - 1 : 0] : fpx;
        const T py = (m > 0) ? fy[m > 0 ? m - 1 : 0] : fpy;
        const T pz = (m > 0) ? fz[m > 0 ? m - 1 : 0] : fpz;
        const T lx = fmadd((T)-2, fx[m], nx + px);
        const T ly = fmadd((T)-2, fy[m], ny + py);
        const T lz = fmadd((T)-2, fz[m], nz + pz);
        const T xnx = (m + 1 < M) ? ex[m + 1 < M ? m + 1 : m] : enx;
        const T xny = (m + 1 < M) ? ey[m + 1 < M ? m + 1 : m] : eny;
        const T xnz = (m + 1 < M) ? ez[m + 1 < M ? m + 1 : m] : enz;
        const T ix = fmadd(kx, s.qx[m], fmadd(kxz, s.qz[m], fmadd(cF, lx, sg * (xnx - ex[m]))));
        const T iy = fmadd(ky, s.qy[m], fmadd(cF, ly, sg * (xny - ey[m])));
        const T iz = fmadd(kz, s.qz[m], fmadd(cF, lz, sg * (xnz - ez[m])));
        s.qx[m] = valid[m] ? s.qx[m] + ix : (T)0;
        s.qy[m] = valid[m] ? s.qy[m] + iy : (T)0;
        s.qz[m] = valid[m] ? s.qz[m] + iz : (T)0;
    }
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

__device__ __forceinline__ TileGeom tile_geom(const GroupDev& G, int k_first, int M) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int seg = lane / G.L;
    TileGeom tg;
    tg.t = lane - seg * G.L;
    tg.k = k_first + seg;
    tg.rep_ok = (seg < G.P) && (tg.k < G.R);
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

__device__ __forceinline__ void flush_clamps(int clamps, unsigned long long* counter) {
    if (clamps) atomicAdd(counter, (unsigned long long)clamps);
}

}  // namespace ra
