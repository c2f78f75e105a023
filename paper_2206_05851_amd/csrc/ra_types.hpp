// ra_types.hpp — host/device shared descriptors of the library's kernels.
#pragma once
#include <stdint.h>

namespace ra {

constexpr int WAVE = 64;

// Per-group constants, precomputed on the host in FP64 (both precisions kept
// so that the FP32 kernels never round a sum like 1 + dt*rate).
struct GroupDev {
    int32_t N, R;            // beads, replicas
    int32_t M, L, P;         // beads per lane, lanes per replica, replicas per wave
    int32_t spring;          // 0 Hookean, 1 FENE, 2 rest-length harmonic
    uint32_t stream;         // counter word: tag<<24 | stream_id (tag 0)
    int32_t flow;            // 0..3 (shear adds the x <- z coupling)
    int32_t nmap;            // noise map: 0 one Philox block per bead-step, 1 four normals per block
    // bond-form EM increment: dQ = kdiag.*Q + kxz*Qz e_x + cF*lap(gQ) + sigma*(xi_{j+1}-xi_j)
    float kx, ky, kz, kxz;   // dt * kappa entries
    float cF;                // H * dt / zeta
    float sigma;             // noise_scale * sqrt(2 kT dt / zeta)
    float H, inv_q0sq;       // tension f = H g |Q|; s = |Q|^2 * inv_q0sq
    double kx_d, ky_d, kz_d, kxz_d, cF_d, sigma_d, H_d, inv_q0sq_d;
    double kT, zeta, dt, b;  // for Bell rates, events and gradients
    double rate;
    int64_t state_off;       // first element of this group's [R][N-1][3] bond state
    int64_t smp_off;         // first element of this group's [R][N-1] block in a window
    int64_t spr_off;         // first spring of this group in a profile row
    int64_t pos_off;         // first element of this group's [R][N][3] positions (plain path)
    int64_t ck_off;          // first element of this group's work items in a checkpoint, whose
                             // layout per item is [slot M][xyz][lane < P L] (lane-contiguous rows)
    // pair-interaction model (Sec. II collapsed polymer): spring 2 = rest-length
    // harmonic, F = H (|Q| - r0) Q/|Q|; LJ u [(rmin/r)^12 - 2 (rmin/r)^6] between
    // beads |i - j| >= 2, force (12u/r^2) [(rmin/r)^12 - (rmin/r)^6] (r_i - r_j)
    float dtz, r0, lj12u, ljr2;          // dt/zeta, rest length, 12 u, rmin^2
    double dtz_d, r0_d, lj12u_d, ljr2_d;
    double hi_a_d;                       // RPY bead radius (Eqs. 2-3), 0 = free draining
};

// One wavefront of work: replicas [k0, k0 + P) of group g.
struct Item {
    int32_t g;
    int32_t k0;
};

// Column tile of the replica reduction: springs [j0, j0 + 64) of group g.
struct ColTile {
    int32_t g;
    int32_t j0;
};

}  // namespace ra
