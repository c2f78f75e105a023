// ra_hi.hip — forward kernel with hydrodynamic interaction (Eqs. 1-3).
//
// Per step and replica: the 3N x 3N Rotne-Prager-Yamakawa diffusion tensor D
// (Eq. 2 on the diagonal, Eq. 3 off it) from the current positions, the drift
// dt D F / kT, and the random displacement sqrt(2 dt) L xi with D = L L^T
// (Cholesky), xi the per-bead normals of the replica counter. Forces F are the
// springs (Hookean, FENE or rest-length harmonic) plus optional LJ between
// non-adjacent beads, as in the pair kernel.
//
// One workgroup (256 threads) per replica. D is assembled in LDS as a packed
// lower triangle (n = 3N <= 192: at most 18528 elements), from which the drift
// D F is taken; the factorization then runs on a copy of the lower triangle
// held in registers (see factor_apply), exchanging one column per step of the
// elimination through LDS. Wave 0 keeps the bond state in registers (lane i = bond i),
// rebuilds positions by a wave scan, forms spring/LJ forces and the noise,
// and applies the bond-form update Q_j += dt kappa Q_j + (Y_{j+1} - Y_j), Y the
// bead displacements without the flow term.
#include "ra_chain.hpp"
#include "ra_dpp.hpp"
#include "ra_launch.hpp"

namespace ra {

constexpr int HI_THREADS = 256;

template <typename T> struct HiCo;
template <> struct HiCo<float> {
    const GroupDev& G;
    __device__ float r0() const { return G.r0; }
    __device__ float lj12u() const { return G.lj12u; }
    __device__ float ljr2() const { return G.ljr2; }
};
template <> struct HiCo<double> {
    const GroupDev& G;
    __device__ double r0() const { return G.r0_d; }
    __device__ double lj12u() const { return G.lj12u_d; }
    __device__ double ljr2() const { return G.ljr2_d; }
};

__device__ __forceinline__ int tri(int i) { return (i * (i + 1)) >> 1; }

// Lane force of the spring on bond Q (on its first bead, toward the second).
template <typename T>
__device__ __forceinline__ void hi_spring(T qx, T qy, T qz, const GroupDev& G, T& fx, T& fy, T& fz, int& clamps) {
    const T H = Co<T>{G}.H();
    const T q2 = fmadd(qx, qx, fmadd(qy, qy, qz * qz));
    T g = (T)1;
    if (G.spring == 1) {
        g = fene_g(qx, qy, qz, q2, (T)G.inv_q0sq, G.inv_q0sq_d, clamps);
    } else if (G.spring == 2) {
        const T q = fast_sqrt(q2);
        g = q > (T)0 ? (T)1 - HiCo<T>{G}.r0() * fast_rcp(q) : (T)0;
    }
    fx = H * g * qx;
    fy = H * g * qy;
    fz = H * g * qz;
}

template <typename T>
__device__ __forceinline__ T hi_tension(T qx, T qy, T qz, const GroupDev& G) {
    const T H = Co<T>{G}.H();
    const T q2 = fmadd(qx, qx, fmadd(qy, qy, qz * qz));
    const T q = fast_sqrt(q2);
    if (G.spring == 2) return H * (q - HiCo<T>{G}.r0());
    if (G.spring == 1) {
        int dummy = 0;
        return H * fene_g(qx, qy, qz, q2, (T)G.inv_q0sq, G.inv_q0sq_d, dummy) * q;
    }
    return H * q;
}

// RPY block of Eq. 3 over D0 = kT/zeta for the pair separation (dx, dy, dz):
// D_ab = D0 (ci delta_ab + cr rhat_a rhat_b).
template <typename T>
__device__ __forceinline__ void rpy_coeffs(T dx, T dy, T dz, T a, T& ci, T& cr, T& ux, T& uy, T& uz) {
    const T r2 = fmadd(dx, dx, fmadd(dy, dy, dz * dz));
    const T q = fast_sqrt(r2);
    const T iq = q > (T)0 ? fast_rcp(q) : (T)0;
    ux = dx * iq;
    uy = dy * iq;
    uz = dz * iq;
    if (q >= (T)2 * a) {
        const T s = (T)0.75 * a * iq;
        const T a2r2 = a * a * iq * iq;
        ci = s * fmadd((T)2 / (T)3, a2r2, (T)1);
        cr = s * fmadd((T)-2, a2r2, (T)1);
    } else {
        const T t = q / a;
        ci = fmadd((T)(-9.0 / 32.0), t, (T)1);
        cr = (T)(3.0 / 32.0) * t;
    }
}

// Columns per exchange in the elimination (a panel): 4, or 2 for the FP64
// instances with the largest register tiles (register and LDS budget).
__host__ __device__ constexpr int hi_panel(bool fp64, int nb) { return (fp64 && nb >= 10) ? 2 : 4; }

// Drift, Cholesky factor and displacement for the packed tensor A (n = 3N rows).
//
// The lower triangle is loaded into registers: thread (tx, ty) of the 16 x 16
// grid owns rows i = ty + 16a and columns j = tx + 16b (b <= a); every loop
// over a and b is unrolled so the register indices are compile-time constants.
//
// Drift D F: from the registers, as row sums (reduced over tx) plus the
// transposed contributions of the strictly lower part (reduced over ty, per
// wavefront in registers and over the four wavefronts through LDS, in the
// space of A, which is free once it has been loaded). Fixed order throughout.
//
// Factorization: square-root-free right-looking elimination R_ij -= R_ik R_jk / R_kk,
// W columns (a panel) per exchange: the owners of the panel's columns publish
// their raw values (all earlier panels applied) through a double-buffered LDS
// panel, one barrier per panel; every thread then eliminates within the panel
// the values it needs (its rows, its columns and the W x W diagonal block) in
// the same expressions and order as the register update, so all copies of a
// panel value are bit-identical, and applies the rank-W update to its
// registers. A non-positive pivot sets status bit 4 after the loop.
//
// Then L = R diag(1/sqrt(R_jj)), y = L xi by 16-lane butterflies (fixed order)
// and Y_i = dt/kT (D F)_i + nsc y_i.
template <typename T, int NB>
__device__ __forceinline__ void factor_apply(T* A, int n, int tx, int ty, T* cbuf, const T* X, const T* F, T* DF,
                                             T* Y, T drift, T nsc, int32_t* status) {
    constexpr int NP = 16 * NB;
    constexpr int W = hi_panel(sizeof(T) == 8, NB);
    T R[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        const int i = ty + 16 * a;
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int j = tx + 16 * b;
            const bool ok = i < n && j <= i;
            const T v = A[ok ? tri(i) + j : 0];
            R[a][b] = ok ? v : (T)0;
        }
    }
    // drift: row part pr (all j <= i) and column part qc (j < i, transposed)
    T fr[NB], fc[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        const T u = F[ty + 16 * a], v = F[tx + 16 * a];
        fr[a] = ty + 16 * a < n ? u : (T)0;
        fc[a] = tx + 16 * a < n ? v : (T)0;
    }
    T pr[NB], qc[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        pr[a] = (T)0;
        qc[a] = (T)0;
    }
#pragma unroll
    for (int a = 0; a < NB; ++a) {
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            pr[a] = fmadd(R[a][b], fc[b], pr[a]);
            const T r = (b == a && tx == ty) ? (T)0 : R[a][b];
            qc[b] = fmadd(r, fr[a], qc[b]);
        }
    }
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        pr[a] = row16_sum(pr[a]);
        qc[a] += __shfl_xor(qc[a], 16, WAVE);
        qc[a] += __shfl_xor(qc[a], 32, WAVE);
    }
    __syncthreads();   // every thread has read A: its space takes the per-wavefront column parts
    {
        T* colp = A + (ty >> 2) * NP;
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            if (tx == 0) DF[ty + 16 * a] = pr[a];
            if ((ty & 3) == 0) colp[tx + 16 * a] = qc[a];
        }
    }
    bool bad = false;
#pragma unroll
    for (int bk = 0; bk < NB; ++bk) {
        for (int kp = 0; kp < 16 / W; ++kp) {
            const int k0 = 16 * bk + W * kp;   // panel: columns k0 .. k0 + W - 1
            if (k0 >= n) break;
            // 16 / W is even, so the buffers alternate across block columns too
            T* cb = (T*)__builtin_assume_aligned(cbuf + (kp & 1) * (NP * W), 16);
            const int own = tx - W * kp;
            if (own >= 0 && own < W) {
#pragma unroll
                for (int a = bk; a < NB; ++a) cb[(ty + 16 * a) * W + own] = R[a][bk];
            }
            __syncthreads();
            // raw panel values (all updates of earlier panels applied) at this
            // thread's rows (ri) and columns (rj), and the W x W diagonal block
            T ri[NB][W], rj[NB][W], D[W][W];
#pragma unroll
            for (int a = bk; a < NB; ++a)
#pragma unroll
                for (int m = 0; m < W; ++m) {
                    ri[a][m] = cb[(ty + 16 * a) * W + m];
                    rj[a][m] = cb[(tx + 16 * a) * W + m];
                }
#pragma unroll
            for (int l = 0; l < W; ++l)
#pragma unroll
                for (int m = 0; m < W; ++m) D[l][m] = cb[(k0 + l) * W + m];
            // Eliminate within the panel, column by column, with the same
            // expressions as the register update below (scaled row value times
            // raw column value, accumulated in column order), so every copy of
            // a panel value is bit-identical to its owner's register.
            T inv[W];
#pragma unroll
            for (int m = 0; m < W; ++m) {
                const bool live = k0 + m < n;
                bad |= live && !(D[m][m] > (T)0);
                inv[m] = live ? fast_rcp(D[m][m]) : (T)0;
#pragma unroll
                for (int r = m + 1; r < W; ++r) {
                    const T c = D[r][m] * inv[m];
#pragma unroll
                    for (int l = m + 1; l <= r; ++l) D[r][l] = fmadd(-c, D[l][m], D[r][l]);
                }
#pragma unroll
                for (int a = bk; a < NB; ++a) {
                    ri[a][m] *= inv[m];   // from here on the scaled row value R_im / d_m
                    const T cjm = rj[a][m] * inv[m];
#pragma unroll
                    for (int l = m + 1; l < W; ++l) {
                        ri[a][l] = fmadd(-ri[a][m], D[l][m], ri[a][l]);
                        rj[a][l] = fmadd(-cjm, D[l][m], rj[a][l]);
                    }
                }
            }
            // rows and columns at or above each panel column take no update
#pragma unroll
            for (int m = 0; m < W; ++m) {
                if (ty <= W * kp + m) ri[bk][m] = (T)0;
                if (tx <= W * kp + m) rj[bk][m] = (T)0;
            }
#pragma unroll
            for (int a = bk; a < NB; ++a)
#pragma unroll
                for (int b = bk; b <= a; ++b)
#pragma unroll
                    for (int m = 0; m < W; ++m) R[a][b] = fmadd(-ri[a][m], rj[b][m], R[a][b]);
        }
    }
    if (tx == 0 && ty == 0 && bad) atomicOr(status, 4);
    __syncthreads();
    T* dg = cbuf;   // pivots d_j
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        const int i = ty + 16 * a;
        if (tx == ty && i < n) dg[i] = R[a][a];
    }
    __syncthreads();
    T sx[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = tx + 16 * b;
        const T dj = dg[j < n ? j : 0], x = X[j];
        sx[b] = j < n ? x / fast_sqrt(dj) : (T)0;
    }
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        const int i = ty + 16 * a;
        T part = (T)0;
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const T r = (b == a && tx > ty) ? (T)0 : R[a][b];
            part = fmadd(r, sx[b], part);
        }
        part = row16_sum(part);
        if (tx == 0 && i < n) {
            const T df = DF[i] + A[i] + A[NP + i] + A[2 * NP + i] + A[3 * NP + i];
            Y[i] = fmadd(drift, df, nsc * part);
        }
    }
}

template <typename T, int NB>
__device__ __forceinline__ void run_hi(const FwdArgs& a, const GroupDev& G, int k, T* lds) {
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const bool w0 = tid < WAVE;
    const int N = G.N, nm1 = N - 1, n = 3 * N;
    T* A = lds;                       // packed lower triangle, tri(n) elements (at least 4 x 16 NB)
    // region offsets are multiples of 4 elements (16-byte aligned panel rows)
    T* P = A + (((tri(n) > 64 * NB ? tri(n) : 64 * NB) + 3) & ~3);   // positions [N][4]
    T* F = P + 4 * WAVE;              // forces [n]
    T* X = F + 3 * WAVE;              // normals [n]
    T* DF = X + 3 * WAVE;             // D F [n]
    T* Y = DF + 3 * WAVE;             // bead displacement without flow [n]
    T* C = Y + 3 * WAVE;              // Cholesky panel exchange, 2 x 16 NB x panel width
    const bool bond_ok = w0 && lane < nm1;
    const bool bead_ok = w0 && lane < N;
    T* const state = (T*)a.state;
    const int64_t sidx = (int64_t)k * nm1 + lane;
    T qx = (T)0, qy = (T)0, qz = (T)0;
    if (bond_ok) {
        const int64_t o = G.state_off + sidx * 3;
        qx = state[o];
        qy = state[o + 1];
        qz = state[o + 2];
    }
    const Co<T> c{G};
    const HiCo<T> hc{G};
    const T kx = c.kx(), ky = c.ky(), kz = c.kz(), kxz = c.kxz();
    const T D0 = (T)(G.kT / G.zeta);
    const T drift = (T)(G.dt / G.kT);                                 // dt / kT
    const T nsc = (T)(G.sigma_d * sqrt(G.zeta / G.kT));               // noise_scale sqrt(2 dt)
    const T ahi = (T)G.hi_a_d;
    const bool lj = G.lj12u_d > 0.0;
    const T lj12u = hc.lj12u(), ljr2 = hc.ljr2();
    const RoundKeys keys = round_keys(a.key0, a.key1);
    const uint32_t n0 = (uint32_t)*a.step0;
    const int S = a.S;
    const bool tsf = a.tsf != nullptr;
    double acc = 0.0;
    if (tsf && bond_ok) acc = a.tsf_acc[G.smp_off + sidx];
    int to_smp = S - (int)(n0 % (uint32_t)S);
    int64_t w = (int64_t)(n0 / (uint32_t)S);
    int clamps = 0;
    const int tx = tid & 15, ty = tid >> 4;
    const int n_steps = (int)a.n_steps;
    for (int st = 0; st < n_steps; ++st) {
        const uint32_t nstep = n0 + (uint32_t)st;
        // 1. positions, spring forces, noise (wave 0)
        if (w0) {
            const T px = wave_scan_incl(qx) - qx;
            const T py = wave_scan_incl(qy) - qy;
            const T pz = wave_scan_incl(qz) - qz;
            P[4 * lane] = px;
            P[4 * lane + 1] = py;
            P[4 * lane + 2] = pz;
            T gx, gy, gz;
            hi_spring(qx, qy, qz, G, gx, gy, gz, clamps);
            if (bead_ok) {
                F[3 * lane] = gx - from_prev_lane(gx);
                F[3 * lane + 1] = gy - from_prev_lane(gy);
                F[3 * lane + 2] = gz - from_prev_lane(gz);
                T ex, ey, ez;
                normals3(philox10(nstep, (uint32_t)lane, (uint32_t)k, G.stream, keys), ex, ey, ez);
                X[3 * lane] = ex;
                X[3 * lane + 1] = ey;
                X[3 * lane + 2] = ez;
            }
        }
        __syncthreads();
        // LJ between non-adjacent beads: wavefront v sums over the beads j of
        // its quarter of the chain for every bead i (lane), into its own rows
        // of the (not yet used) panel buffer
        if (lj) {
            const int wv = tid >> 6;
            const int q = (N + 3) >> 2;
            const int j0 = wv * q, j1 = j0 + q < N ? j0 + q : N;
            const bool mine = lane < N;
            const T px = P[4 * lane], py = P[4 * lane + 1], pz = P[4 * lane + 2];
            T fx = (T)0, fy = (T)0, fz = (T)0;
            for (int j = j0; j < j1; ++j) {
                const T dx = px - P[4 * j], dy = py - P[4 * j + 1], dz = pz - P[4 * j + 2];
                const int dj = j - lane;
                const bool use = mine && (dj >= 2 || dj <= -2);
                // excluded pairs get a zero coefficient below (the select also
                // drops the self pair's Inf/NaN from 1/r^2 at r = 0)
                const T r2 = fmadd(dx, dx, fmadd(dy, dy, dz * dz));
                const T inv = fast_rcp(r2);
                const T s1 = ljr2 * inv;
                const T s3 = s1 * s1 * s1;
                const T cc = use ? lj12u * inv * fmadd(s3, s3, -s3) : (T)0;
                fx = fmadd(cc, dx, fx);
                fy = fmadd(cc, dy, fy);
                fz = fmadd(cc, dz, fz);
            }
            if (mine) {
                T* fl = C + wv * n + 3 * lane;
                fl[0] = fx;
                fl[1] = fy;
                fl[2] = fz;
            }
        }
        // 2. D: one pair (i >= j) at a time, its 3x3 block (lower part on the diagonal)
        const int n_pairs = tri(N);
        for (int p = tid; p < n_pairs; p += HI_THREADS) {
            int i = (int)((fast_sqrt(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
            while (tri(i) > p) --i;
            while (tri(i + 1) <= p) ++i;
            const int j = p - tri(i);
            if (i == j) {
                const int r0 = 3 * i;
                A[tri(r0) + r0] = D0;
                A[tri(r0 + 1) + r0] = (T)0;
                A[tri(r0 + 1) + r0 + 1] = D0;
                A[tri(r0 + 2) + r0] = (T)0;
                A[tri(r0 + 2) + r0 + 1] = (T)0;
                A[tri(r0 + 2) + r0 + 2] = D0;
            } else {
                T ci, cr, ux, uy, uz;
                rpy_coeffs(P[4 * j] - P[4 * i], P[4 * j + 1] - P[4 * i + 1], P[4 * j + 2] - P[4 * i + 2], ahi, ci,
                           cr, ux, uy, uz);
                const T u[3] = {ux, uy, uz};
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    T* row = A + tri(3 * i + x) + 3 * j;
#pragma unroll
                    for (int y = 0; y < 3; ++y) row[y] = D0 * fmadd(cr, u[x] * u[y], x == y ? ci : (T)0);
                }
            }
        }
        __syncthreads();
        if (lj) {
            // total force: springs + the four LJ partial sums in fixed order
            if (bead_ok) {
#pragma unroll
                for (int c3 = 0; c3 < 3; ++c3) {
                    const int r = 3 * lane + c3;
                    F[r] += ((C[r] + C[n + r]) + C[2 * n + r]) + C[3 * n + r];
                }
            }
            __syncthreads();
        }
        // 3-5. drift, Cholesky in registers and the displacement Y = dt D F / kT + sqrt(2 dt) L xi
        factor_apply<T, NB>(A, n, tx, ty, C, X, F, DF, Y, drift, nsc, a.status);
        __syncthreads();
        // 6. bond update and sampling (wave 0)
        if (w0) {
            if (bond_ok) {
                const T ix = fmadd(kx, qx, fmadd(kxz, qz, Y[3 * lane + 3] - Y[3 * lane]));
                const T iy = fmadd(ky, qy, Y[3 * lane + 4] - Y[3 * lane + 1]);
                const T iz = fmadd(kz, qz, Y[3 * lane + 5] - Y[3 * lane + 2]);
                qx += ix;
                qy += iy;
                qz += iz;
            }
            const bool window_end = --to_smp == 0;
            if (tsf || window_end) {
                const T f = hi_tension(qx, qy, qz, G);
                if (tsf) acc += (double)f;
                if (window_end) {
                    bool bad = false;
                    if (bond_ok) {
                        const int64_t o = w * a.smp_total + G.smp_off + sidx;
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
    }
    if (bond_ok) {
        const int64_t o = G.state_off + sidx * 3;
        state[o] = qx;
        state[o + 1] = qy;
        state[o + 2] = qz;
        if (tsf) a.tsf_acc[G.smp_off + sidx] = acc;
    }
    if (w0) flush_clamps(clamps, a.clamps + (&G - a.groups));
}

// One kernel per register tile NB (16-row blocks of the tensor): the host
// picks the smallest NB with 16 NB >= 3 N_max, so each instance gets its own
// register allocation.
template <typename T, int NB>
__device__ __forceinline__ void hi_item(const FwdArgs& a, int item, T* lds) {
    if (item >= a.n_items) return;
    if (*(const volatile int*)a.status & 1) return;   // invalid parent: no work (whole block)
    const Item it = a.items[item];
    const GroupDev& G = a.groups[it.g];
    if (it.k0 >= G.R) return;
    run_hi<T, NB>(a, G, it.k0, lds);
}

template <typename T, int NB>
__global__ __launch_bounds__(HI_THREADS) void fwd_hi_kernel(FwdArgs a) {
    extern __shared__ __align__(16) unsigned char hi_lds[];
    hi_item<T, NB>(a, (int)blockIdx.x, (T*)hi_lds);
}

// Two contexts in one launch (see fwd_dual_kernel): blocks [0, n_items of a) run a.
template <typename T, int NB>
__global__ __launch_bounds__(HI_THREADS) void fwd_hi_dual_kernel(FwdArgs a, FwdArgs b) {
    extern __shared__ __align__(16) unsigned char hi_lds[];
    if ((int)blockIdx.x < a.n_items) hi_item<T, NB>(a, (int)blockIdx.x, (T*)hi_lds);
    else hi_item<T, NB>(b, (int)blockIdx.x - a.n_items, (T*)hi_lds);
}

// Register tile of the kernel instance launched for nb = ceil(3 N_max / 16).
static int hi_nb_instance(int nb) { return nb <= 2 ? 2 : nb <= 4 ? 4 : nb <= 6 ? 6 : nb <= 8 ? 8 : nb <= 10 ? 10 : 12; }

size_t hi_lds_bytes(int max_beads, int precision) {
    const int n = 3 * max_beads;
    const size_t a_elems = (std::max((size_t)n * (n + 1) / 2, (size_t)64 * hi_nb_instance((n + 15) / 16)) + 3) & ~(size_t)3;
    const int nbi = hi_nb_instance((n + 15) / 16);
    const size_t elems = a_elems + 4 * WAVE + 12 * WAVE + (size_t)2 * 16 * nbi * hi_panel(precision == 64, nbi);
    return elems * (precision == 64 ? 8 : 4);
}

template <typename T>
static void launch_hi_nb(const FwdArgs& a, int nb, dim3 grid, dim3 block, size_t lds, hipStream_t st) {
    if (nb <= 2) hipLaunchKernelGGL((fwd_hi_kernel<T, 2>), grid, block, lds, st, a);
    else if (nb <= 4) hipLaunchKernelGGL((fwd_hi_kernel<T, 4>), grid, block, lds, st, a);
    else if (nb <= 6) hipLaunchKernelGGL((fwd_hi_kernel<T, 6>), grid, block, lds, st, a);
    else if (nb <= 8) hipLaunchKernelGGL((fwd_hi_kernel<T, 8>), grid, block, lds, st, a);
    else if (nb <= 10) hipLaunchKernelGGL((fwd_hi_kernel<T, 10>), grid, block, lds, st, a);
    else hipLaunchKernelGGL((fwd_hi_kernel<T, 12>), grid, block, lds, st, a);
}

hipError_t launch_forward_hi(const FwdArgs& a, int precision, int max_beads, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    if (a.n_items <= 0 || a.n_steps <= 0) return hipSuccess;
    if (max_beads < 2 || max_beads > WAVE) return hipErrorInvalidValue;
    const size_t lds = hi_lds_bytes(max_beads, precision);   // checked against the device limit by the host
    const int nb = (3 * max_beads + 15) / 16;
    dim3 grid((unsigned)a.n_items), block(HI_THREADS);
    if (precision == 64) launch_hi_nb<double>(a, nb, grid, block, lds, st);
    else launch_hi_nb<float>(a, nb, grid, block, lds, st);
    return hipGetLastError();
}

template <typename T>
static void launch_hi_dual_nb(const FwdArgs& a, const FwdArgs& b, int nb, dim3 grid, dim3 block, size_t lds,
                              hipStream_t st) {
    if (nb <= 2) hipLaunchKernelGGL((fwd_hi_dual_kernel<T, 2>), grid, block, lds, st, a, b);
    else if (nb <= 4) hipLaunchKernelGGL((fwd_hi_dual_kernel<T, 4>), grid, block, lds, st, a, b);
    else if (nb <= 6) hipLaunchKernelGGL((fwd_hi_dual_kernel<T, 6>), grid, block, lds, st, a, b);
    else if (nb <= 8) hipLaunchKernelGGL((fwd_hi_dual_kernel<T, 8>), grid, block, lds, st, a, b);
    else if (nb <= 10) hipLaunchKernelGGL((fwd_hi_dual_kernel<T, 10>), grid, block, lds, st, a, b);
    else hipLaunchKernelGGL((fwd_hi_dual_kernel<T, 12>), grid, block, lds, st, a, b);
}

hipError_t launch_forward_hi_dual(const FwdArgs& a, const FwdArgs& b, int precision, int max_beads, hipStream_t st) {
    (void)hipGetLastError();   // report only this launch's own error
    if (a.n_items + b.n_items <= 0) return hipSuccess;
    if (max_beads < 2 || max_beads > WAVE) return hipErrorInvalidValue;
    const size_t lds = hi_lds_bytes(max_beads, precision);
    const int nb = (3 * max_beads + 15) / 16;
    dim3 grid((unsigned)(a.n_items + b.n_items)), block(HI_THREADS);
    if (precision == 64) launch_hi_dual_nb<double>(a, b, nb, grid, block, lds, st);
    else launch_hi_dual_nb<float>(a, b, nb, grid, block, lds, st);
    return hipGetLastError();
}

}  // namespace ra
