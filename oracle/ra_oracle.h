/*
 * ra_oracle.h — FP64 CPU oracle for replica-averaged Brownian dynamics.
 *
 * TEST INFRASTRUCTURE ONLY. This header and ra_oracle.c form a plain, slow,
 * obviously-correct reference of what the GPU library computes. Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it. The product path never links, calls or falls back to it, and it shares
 * no code, header, constant table or helper with the HIP library.
 *
 * Model (Kania, Nguyen, Oztekin, Webb, "Replica-Averaging", Sec. II):
 *   - bead-spring chain of N beads, spring j joins beads j and j+1;
 *   - Brownian-dynamics update Eq. (1), free-draining (D_ii = kT/zeta * I,
 *     D_ij = 0) or with hydrodynamic interaction through the RPY tensor of
 *     Eqs. (2)-(3) when hi_radius > 0;
 *   - random displacement with zero mean and covariance 2*D*dt (Eq. 1 text),
 *     Gaussian: sqrt(2 dt) L xi with L the Cholesky factor of D and xi from a
 *     counter-based Philox4x32-10 stream (L = sqrt(kT/zeta) I free-draining);
 *   - homogeneous flow v = kappa . r (Sec. II; shear v = gdot * z * x-hat);
 *   - spring tension sampled per spring (Eq. 4: signed kappa (r - r0) for
 *     rest-length harmonic springs, H g |Q| for zero-rest-length Hookean and
 *     FENE springs), averaged over replicas (RSF, Sec. II) and over time
 *     within a window (TSF, Sec. II);
 *   - optional Lennard-Jones self-association between non-adjacent beads
 *     (Sec. II, collapsed-polymer model);
 *   - Bell-type rate k = k0 * exp(x_dagger * f / kT) (Sec. III, vWF rate law).
 *
 * All arithmetic is IEEE double; the only library calls are libm's
 * log/sqrt/cos/sin/exp/expm1.
 */
#ifndef RA_ORACLE_H
#define RA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { RAO_HOOKEAN = 0, RAO_FENE = 1, RAO_HARMONIC = 2 };
enum { RAO_QUIESCENT = 0, RAO_UNIAXIAL = 1, RAO_PLANAR = 2, RAO_SHEAR = 3 };
enum { RAO_OK = 0, RAO_EINVAL = -1, RAO_ENOMEM = -2, RAO_ESTATE = -5 };

/* Philox counter tag (top 8 bits of the fourth counter word). */
enum { RAO_TAG_REPLICA = 0, RAO_TAG_PARENT = 1, RAO_TAG_EVENT = 2 };

typedef struct {
    int32_t  n_beads;      /* N >= 2 */
    int32_t  n_replicas;   /* R >= 1 */
    int32_t  spring;       /* RAO_HOOKEAN | RAO_FENE */
    int32_t  flow;         /* RAO_QUIESCENT | RAO_UNIAXIAL | RAO_PLANAR | RAO_SHEAR */
    double   H;            /* spring constant */
    double   b;            /* FENE extensibility; Q0^2 = b*kT/H */
    double   rate;         /* strain rate (elongation) or shear rate */
    double   kT, zeta, dt;
    double   noise_scale;  /* 1 = physical noise, 0 = deterministic */
    double   rest_length;  /* RAO_HARMONIC: zero-force bond length (2a in Sec. II) */
    double   lj_eps;       /* Lennard-Jones well depth u between non-adjacent beads (0 = off) */
    double   lj_rmin;      /* position of the LJ minimum (2a in Sec. II) */
    double   hi_radius;    /* bead radius a of the RPY tensor, Eqs. 2-3 (0 = free draining) */
    uint32_t stream_id;    /* group id in the Philox counter, < 2^24 */
    uint32_t pad_;
} rao_group;

/* FENE guard: s = |Q|^2/Q0^2 is clamped at 1 - RAO_FENE_DELTA. */
#define RAO_FENE_DELTA 1.0e-3

/* ---- primitives ------------------------------------------------------- */
void   rao_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double rao_uniform(uint32_t x);
double rao_uniform53(uint32_t hi, uint32_t lo);
void   rao_normals(const uint32_t x[4], double xi[3]);
void   rao_noise(uint64_t seed, uint32_t step, uint32_t bead, uint32_t replica,
                 uint32_t tag, uint32_t group, double xi[3]);
/* xi[0..2] as rao_normals, xi[3] = r1 sin(2 pi u3) */
void   rao_normals4(const uint32_t x[4], double xi[4]);
/* per-bead normals of one step under noise map 0 (rao_noise), 1 (four
 * normals per block; step 4m+3 takes the fourth normals of steps 4m..4m+2)
 * or 2 (bead 4q + r takes normal r of the blocks with bead word 3q + c) */
void   rao_noise_mapped(uint64_t seed, uint32_t step, uint32_t bead, uint32_t replica,
                        uint32_t tag, uint32_t group, int32_t map, double xi[3]);
/* spring force F (on bead j, toward bead j+1), factor g (F = H g Q), tension f;
 * p2 is b for FENE and the rest length for RAO_HARMONIC; returns 1 if clamped */
int    rao_spring(int spring, double H, double p2, double kT, const double Q[3],
                  double F[3], double* g, double* f);
/* RPY diffusion tensor block D_ij (i != j) of Eq. 3 for r = r_j - r_i, with
 * D_ii = kT/zeta I (Eq. 2, zeta = 6 pi eta a): row-major 3x3 into D */
void   rao_rpy_block(double kT, double zeta, double a, const double r[3], double D[9]);
/* in-place lower Cholesky of the row-major n x n matrix A (A = L L^T, upper
 * part zeroed); returns 0, or -1 if a pivot is not positive */
int    rao_cholesky(int n, double* A);
/* Lennard-Jones force on bead i from bead j (Sec. II): U = u [(rmin/r)^12 - 2 (rmin/r)^6],
 * d = r_i - r_j; F = (12 u / r^2) [(rmin/r)^12 - (rmin/r)^6] d; returns U */
double rao_lj(double u, double rmin, const double d[3], double F[3]);
void   rao_flow_velocity(int flow, double rate, const double r[3], double v[3]);

/* ---- context API mirroring the library's calls ------------------------ */
typedef struct rao_ctx rao_ctx;

int  ra_oracle_create(rao_ctx** out, const rao_group* groups, int32_t n_groups,
                      uint64_t seed, int32_t sample_every, int32_t max_windows,
                      int32_t tsf, int32_t tangents);
/* simulate only replicas [k_begin, k_end) of group g (counters keep global k) */
int  ra_oracle_set_replicas(rao_ctx* c, int32_t g, int32_t k_begin, int32_t k_end);
/* clone: parent_xyz holds N_g*3 doubles per group, concatenated in group order */
int  ra_oracle_init_chains(rao_ctx* c, const double* parent_xyz);
int  ra_oracle_step(rao_ctx* c, int64_t n_steps);
int64_t ra_oracle_n_windows(const rao_ctx* c);
int64_t ra_oracle_total_springs(const rao_ctx* c);
/* [W][sum_g (N_g-1)] FP64; std with R-1 (0 if R == 1); any pointer may be NULL */
int  ra_oracle_average_forces(rao_ctx* c, double* mean, double* std,
                              double* tsf_mean, double* tsf_std);
/* rates[W][S], rate_sum[W][G]; events[W][S] (may be NULL) */
int  ra_oracle_bell_rates(rao_ctx* c, const double* mean, int64_t n_windows,
                          double k0, double x_dagger, double* rates,
                          double* rate_sum, uint8_t* events);
/* forward-mode pathwise gradient of J = sum gm*mean + sum gr*rates w.r.t.
 * (rate, H, b) per group; needs tangents=1 at create; grad_rates may be NULL */
int  ra_oracle_backward(rao_ctx* c, const double* grad_mean, const double* grad_rates,
                        double k0, double x_dagger, double* grad_params);
/* noise tag of the context's trajectories: RAO_TAG_REPLICA (default) or RAO_TAG_PARENT */
int  ra_oracle_set_tag(rao_ctx* c, uint32_t tag);
/* noise map of the context's trajectories: 0 (default), 1 or 2, see rao_noise_mapped */
int  ra_oracle_set_noise_map(rao_ctx* c, int32_t map);
/* RSF re-clone (Sec. II): every replica restarts from parent_xyz; the step
 * count (a multiple of S) is kept, and so are earlier windows */
int  ra_oracle_reclone(rao_ctx* c, const double* parent_xyz);
/* RSF cycle (Sec. II): per window the parent context (one chain per group,
 * sample_every = parent_steps) advances parent_steps steps, the replicas are
 * re-cloned from it and advance S steps */
int  ra_oracle_rsf_cycle(rao_ctx* rep, rao_ctx* par, int64_t n_windows, int64_t parent_steps);
/* sigma[W][sum_g (N_g-1)]: std over floor(R/block) consecutive replica blocks of the block mean */
int  ra_oracle_block_sigma(const rao_ctx* c, int32_t block, double* sigma);
/* mftu[g] = 1 / (mean over windows of rate_sum[w][g]) */
int  ra_oracle_mftu(const rao_ctx* c, const double* rate_sum, int64_t n_windows, double* mftu);
int  ra_oracle_mftu_events(const rao_ctx* c, const double* rates, int64_t n_windows, int32_t n_trials,
                           int64_t max_windows, int64_t* first_window, double* mftu);
/* Eq. 5 fidelity dbar[k][3], per-bead d_bead[k][i][3], squared radius of
 * gyration components rg2[k][3] and src_rg2[g][3] of the clone source */
int  ra_oracle_conformation(const rao_ctx* c, double* dbar, double* d_bead, double* rg2,
                            double* src_rg2);
/* per-replica tension samples [W][sum_g Rsub_g*(N_g-1)] and TSF values */
int  ra_oracle_get_samples(const rao_ctx* c, double* out, double* tsf_out);
/* bead positions [sum_g Rsub_g*N_g*3] */
int  ra_oracle_get_positions(const rao_ctx* c, double* out);
int64_t ra_oracle_clamps(const rao_ctx* c, int32_t g);
const char* ra_oracle_last_error(const rao_ctx* c);
void ra_oracle_destroy(rao_ctx* c);

#ifdef __cplusplus
}
#endif
#endif
