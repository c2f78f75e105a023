/*
 * ra_oracle.c — FP64 CPU oracle for replica-averaged Brownian dynamics.
 *
 * TEST INFRASTRUCTURE ONLY (see ra_oracle.h). Plain loops over replicas,
 * beads and components in bead-position form, written for a reader to check
 * against the paper by eye; no blocking, fusion or reordering.
 *
 * Paper: Kania, Nguyen, Oztekin, Webb, "Replica-Averaging: An algorithm to
 * study mechano-reactive processes for polymers under flow conditions".
 */
#include "ra_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies, with a  */
/* Weyl-sequence key schedule. The paper under study fixes only the moments  */
/* of the random displacement (Eq. 1 text); the generator is our choice.     */
/* ------------------------------------------------------------------------ */
void rao_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;   /* round multipliers */
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;   /* key increments    */
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 32-bit word -> uniform in (0,1): the top 23 bits j give u = (j + 1/2) 2^-23,
 * an odd multiple of 2^-24 that is exact in binary32 and binary64. */
double rao_uniform(uint32_t x)
{
    return ((double)(x >> 9) + 0.5) * 0x1p-23;
}

/* Two 32-bit words -> uniform in (0,1) for unfolding-event draws: the top 52
 * bits m of the 64-bit word hi:lo give u = (2m + 1) 2^-53, an odd multiple of
 * 2^-53 (exact in binary64). Event probabilities per window reach 1e-7 and
 * below, under the 2^-24 grid of the one-word map. */
double rao_uniform53(uint32_t hi, uint32_t lo)
{
    uint64_t m = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return (double)(2 * m + 1) * 0x1p-53;
}

/* Box-Muller: three standard normals from four uniforms (the second radius
 * uses only its cosine branch). */
void rao_normals(const uint32_t x[4], double xi[3])
{
    const double two_pi = 6.283185307179586476925286766559;
    double u0 = rao_uniform(x[0]), u1 = rao_uniform(x[1]);
    double u2 = rao_uniform(x[2]), u3 = rao_uniform(x[3]);
    double r0 = sqrt(-2.0 * log(u0));
    double r1 = sqrt(-2.0 * log(u2));
    xi[0] = r0 * cos(two_pi * u1);
    xi[1] = r0 * sin(two_pi * u1);
    xi[2] = r1 * cos(two_pi * u3);
}

/* Box-Muller with both outputs of the second pair: xi[3] = r1 sin(2 pi u3),
 * the normal rao_normals leaves out (independent of the other three). */
void rao_normals4(const uint32_t x[4], double xi[4])
{
    const double two_pi = 6.283185307179586476925286766559;
    rao_normals(x, xi);
    double r1 = sqrt(-2.0 * log(rao_uniform(x[2])));
    xi[3] = r1 * sin(two_pi * rao_uniform(x[3]));
}

/* Counter layout: (step, bead-or-spring, replica, tag<<24 | group);
 * key = (seed low 32 bits, seed high 32 bits). Each replica gets its own
 * stream through the replica word, which plays the role of the paper's
 * per-replica unique seed (RSF description, Sec. II). */
void rao_noise(uint64_t seed, uint32_t step, uint32_t bead, uint32_t replica,
               uint32_t tag, uint32_t group, double xi[3])
{
    uint32_t ctr[4] = { step, bead, replica, (tag << 24) | (group & 0xFFFFFFu) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t x[4];
    rao_philox4x32_10(ctr, key, x);
    rao_normals(x, xi);
}

/* The per-bead normals of one step under a noise map. Map 0: one Philox
 * block per (step, bead), rao_noise. Map 1: the block of step n gives four
 * normals; steps n = 4m, 4m+1, 4m+2 take the first three of their own block,
 * and step 4m+3 takes the fourth normals of the blocks of steps 4m, 4m+1 and
 * 4m+2 (x, y, z in that order). Map 2: the beads of a step form groups of
 * four, bead = 4q + r; the blocks with the bead word 3q, 3q+1 and 3q+2 give
 * four normals each, and bead 4q + r takes normal r of block 3q + c as its
 * component c (x, y, z for c = 0, 1, 2). Under every map each (step, bead)
 * gets three independent standard normals; maps 1 and 2 use three blocks per
 * four bead-steps. */
void rao_noise_mapped(uint64_t seed, uint32_t step, uint32_t bead, uint32_t replica,
                      uint32_t tag, uint32_t group, int32_t map, double xi[3])
{
    if (map == 2) {
        uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
        uint32_t q = bead / 4u, r = bead % 4u;
        for (uint32_t c = 0; c < 3; ++c) {
            uint32_t ctr[4] = { step, 3u * q + c, replica, (tag << 24) | (group & 0xFFFFFFu) };
            uint32_t x[4];
            double four[4];
            rao_philox4x32_10(ctr, key, x);
            rao_normals4(x, four);
            xi[c] = four[r];
        }
        return;
    }
    if (map == 0 || step % 4u != 3u) {
        rao_noise(seed, step, bead, replica, tag, group, xi);
        return;
    }
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    for (uint32_t q = 0; q < 3; ++q) {
        uint32_t ctr[4] = { step - 3u + q, bead, replica, (tag << 24) | (group & 0xFFFFFFu) };
        uint32_t x[4];
        double four[4];
        rao_philox4x32_10(ctr, key, x);
        rao_normals4(x, four);
        xi[q] = four[3];
    }
}

/* ------------------------------------------------------------------------ */
/* Spring law. Hookean: F = H Q. FENE: F = H Q / (1 - |Q|^2/Q0^2), with      */
/* Q0^2 = b kT / H; s = |Q|^2/Q0^2 is clamped at 1 - delta (guard). The       */
/* tension is the magnitude f = H g |Q| — Eq. (4) with zero rest length.     */
/* Returns 1 when the guard clamped s.                                        */
/* ------------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static int spring_factor(int spring, double H, double p2, double kT, const double Q[3],
                         double* g, double* s_out)
{
    if (spring == RAO_HOOKEAN) { *g = 1.0; *s_out = 0.0; return 0; }
    if (spring == RAO_HARMONIC) {
        /* rest length r0 = p2: F = H (|Q| - r0) Q/|Q| = H g Q, g = 1 - r0/|Q| */
        double q = sqrt(dot3(Q, Q));
        *g = q > 0.0 ? 1.0 - p2 / q : 0.0;
        *s_out = 0.0;
        return 0;
    }
    double q0sq = p2 * kT / H;
    double s = dot3(Q, Q) / q0sq;
    int clamped = 0;
    if (s > 1.0 - RAO_FENE_DELTA) { s = 1.0 - RAO_FENE_DELTA; clamped = 1; }
    *g = 1.0 / (1.0 - s);
    *s_out = s;
    return clamped;
}

int rao_spring(int spring, double H, double p2, double kT, const double Q[3],
               double F[3], double* g, double* f)
{
    double s;
    int clamped = spring_factor(spring, H, p2, kT, Q, g, &s);
    for (int a = 0; a < 3; ++a) F[a] = H * (*g) * Q[a];
    if (spring == RAO_HARMONIC) *f = H * (sqrt(dot3(Q, Q)) - p2);   /* signed, Eq. 4 */
    else *f = H * (*g) * sqrt(dot3(Q, Q));
    return clamped;
}

/* Lennard-Jones pair (Sec. II collapsed-polymer model). */
double rao_lj(double u, double rmin, const double d[3], double F[3])
{
    double r2 = dot3(d, d);
    double x6 = pow(rmin * rmin / r2, 3.0);          /* (rmin/r)^6 */
    double c = 12.0 * u / r2 * (x6 * x6 - x6);
    for (int a = 0; a < 3; ++a) F[a] = c * d[a];
    return u * (x6 * x6 - 2.0 * x6);
}

/* Rotne-Prager-Yamakawa block (Eq. 3) for two beads of radius a at
 * separation r, in units of D0 = kT/zeta (zeta = 6 pi eta a, Eq. 2):
 *   r >= 2a: (3a/4r) [(1 + 2a^2/(3r^2)) I + (1 - 2a^2/r^2) rhat rhat]
 *   r <  2a: (1 - 9r/(32a)) I + (3r/(32a)) rhat rhat
 * (the second line is the paper's overlap form with kT/(8 pi eta r) (r/2a)
 * rewritten over D0). */
void rao_rpy_block(double kT, double zeta, double a, const double r[3], double D[9])
{
    const double D0 = kT / zeta;
    const double q = sqrt(dot3(r, r));
    double ci, cr;
    if (q >= 2.0 * a) {
        ci = 0.75 * a / q * (1.0 + 2.0 * a * a / (3.0 * q * q));
        cr = 0.75 * a / q * (1.0 - 2.0 * a * a / (q * q));
    } else {
        ci = 1.0 - 9.0 * q / (32.0 * a);
        cr = 3.0 * q / (32.0 * a);
    }
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) {
            double rr = q > 0.0 ? r[x] * r[y] / (q * q) : 0.0;
            D[3 * x + y] = D0 * ((x == y ? ci : 0.0) + cr * rr);
        }
}

/* Cholesky-Banachiewicz: row by row, L_ij = (A_ij - sum_{m<j} L_im L_jm) / L_jj,
 * L_ii = sqrt(A_ii - sum_{m<i} L_im^2). */
int rao_cholesky(int n, double* A)
{
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double sum = A[i * n + j];
            for (int m = 0; m < j; ++m) sum -= A[i * n + m] * A[j * n + m];
            if (i == j) {
                if (!(sum > 0.0)) return -1;
                A[i * n + i] = sqrt(sum);
            } else {
                A[i * n + j] = sum / A[j * n + j];
            }
        }
        for (int j = i + 1; j < n; ++j) A[i * n + j] = 0.0;
    }
    return 0;
}

/* Second spring parameter: b (FENE) or the rest length (harmonic). */
static double spring_p2(const rao_group* d)
{
    return d->spring == RAO_HARMONIC ? d->rest_length : d->b;
}

/* Homogeneous flow v = kappa . r. Shear follows the paper's convention
 * v = gdot * z * x-hat (Sec. II); elongations are the standard forms. */
void rao_flow_velocity(int flow, double rate, const double r[3], double v[3])
{
    v[0] = v[1] = v[2] = 0.0;
    switch (flow) {
    case RAO_UNIAXIAL: v[0] = rate * r[0]; v[1] = -0.5 * rate * r[1]; v[2] = -0.5 * rate * r[2]; break;
    case RAO_PLANAR:   v[0] = rate * r[0]; v[1] = -rate * r[1]; v[2] = 0.0; break;
    case RAO_SHEAR:    v[0] = rate * r[2]; break;
    default: break;
    }
}

/* ------------------------------------------------------------------------ */
/* Context                                                                    */
/* ------------------------------------------------------------------------ */
struct rao_ctx {
    int32_t  n_groups;
    rao_group* groups;
    uint64_t seed;
    int32_t  sample_every, max_windows, tsf, tangents;
    int32_t* k_begin;      /* simulated replica range per group */
    int32_t* k_end;
    int64_t* pos_off;      /* offset (in doubles) of group g in pos[] */
    int64_t* smp_off;      /* offset of group g in one window of samples */
    int64_t* spr_off;      /* offset of group g in one window of the profile */
    int64_t  n_pos, n_smp, n_spr;
    double*  pos;          /* [g][k][i][3] */
    double*  tan;          /* [p][g][k][i][3], p = rate, H, b */
    double*  samples;      /* [w][smp] */
    double*  tsf_samples;  /* [w][smp] */
    double*  tsf_acc;      /* [smp] running window sums */
    double*  dmu;          /* [w][spr][3] sum over replicas of df/dtheta */
    int64_t* clamps;       /* per group */
    double*  src;          /* [g][i][3] conformation the replicas were last cloned from */
    uint32_t tag;          /* noise tag of this context's trajectories */
    int32_t  noise_map;    /* 0, 1 or 2, see rao_noise_mapped */
    int64_t  step;         /* steps taken since init */
    int64_t  n_windows;
    int      initialised;
    char     err[256];
};

static int fail(rao_ctx* c, int code, const char* msg)
{
    if (c) snprintf(c->err, sizeof c->err, "%s", msg);
    return code;
}

const char* ra_oracle_last_error(const rao_ctx* c) { return c ? c->err : "null context"; }

void ra_oracle_destroy(rao_ctx* c)
{
    if (!c) return;
    free(c->groups); free(c->k_begin); free(c->k_end);
    free(c->pos_off); free(c->smp_off); free(c->spr_off);
    free(c->pos); free(c->tan); free(c->samples); free(c->tsf_samples);
    free(c->tsf_acc); free(c->dmu); free(c->clamps); free(c->src);
    free(c);
}

static int layout(rao_ctx* c)
{
    int64_t p = 0, s = 0, q = 0;
    for (int g = 0; g < c->n_groups; ++g) {
        int64_t rs = c->k_end[g] - c->k_begin[g];
        int64_t n = c->groups[g].n_beads;
        c->pos_off[g] = p; p += rs * n * 3;
        c->smp_off[g] = s; s += rs * (n - 1);
        c->spr_off[g] = q; q += n - 1;
    }
    c->n_pos = p; c->n_smp = s; c->n_spr = q;
    free(c->pos); free(c->tan); free(c->samples); free(c->tsf_samples);
    free(c->tsf_acc); free(c->dmu);
    c->pos = calloc((size_t)(p ? p : 1), sizeof(double));
    c->tan = c->tangents ? calloc((size_t)(3 * p + 1), sizeof(double)) : NULL;
    c->samples = calloc((size_t)(c->max_windows * s + 1), sizeof(double));
    c->tsf_samples = c->tsf ? calloc((size_t)(c->max_windows * s + 1), sizeof(double)) : NULL;
    c->tsf_acc = c->tsf ? calloc((size_t)(s + 1), sizeof(double)) : NULL;
    c->dmu = c->tangents ? calloc((size_t)(c->max_windows * q * 3 + 1), sizeof(double)) : NULL;
    if (!c->pos || !c->samples || (c->tangents && (!c->tan || !c->dmu)) ||
        (c->tsf && (!c->tsf_samples || !c->tsf_acc)))
        return fail(c, RAO_ENOMEM, "out of host memory");
    c->initialised = 0;
    return RAO_OK;
}

int ra_oracle_create(rao_ctx** out, const rao_group* groups, int32_t n_groups,
                     uint64_t seed, int32_t sample_every, int32_t max_windows,
                     int32_t tsf, int32_t tangents)
{
    if (!out) return RAO_EINVAL;
    *out = NULL;
    if (!groups || n_groups < 1 || sample_every < 1 || max_windows < 0) return RAO_EINVAL;
    for (int g = 0; g < n_groups; ++g) {
        const rao_group* d = &groups[g];
        if (d->n_beads < 2 || d->n_replicas < 1 || !(d->dt > 0) || !(d->kT > 0) ||
            !(d->zeta > 0) || !(d->H > 0) || d->spring < 0 || d->spring > 2 ||
            d->flow < 0 || d->flow > 3 || d->stream_id > 0xFFFFFFu ||
            (d->spring == RAO_FENE && !(d->b > 0)) ||
            (d->spring == RAO_HARMONIC && !(d->rest_length >= 0)) ||
            !(d->lj_eps >= 0) || (d->lj_eps > 0 && !(d->lj_rmin > 0)) ||
            !(d->hi_radius >= 0) || !isfinite(d->hi_radius))
            return RAO_EINVAL;
        if (tangents && (d->spring == RAO_HARMONIC || d->lj_eps > 0 || d->hi_radius > 0))
            return RAO_EINVAL;   /* gradients cover the free-draining Hookean and FENE chain only */
    }
    rao_ctx* c = calloc(1, sizeof *c);
    if (!c) return RAO_ENOMEM;
    c->n_groups = n_groups;
    c->groups = malloc(sizeof(rao_group) * (size_t)n_groups);
    c->k_begin = malloc(sizeof(int32_t) * (size_t)n_groups);
    c->k_end = malloc(sizeof(int32_t) * (size_t)n_groups);
    c->pos_off = malloc(sizeof(int64_t) * (size_t)n_groups);
    c->smp_off = malloc(sizeof(int64_t) * (size_t)n_groups);
    c->spr_off = malloc(sizeof(int64_t) * (size_t)n_groups);
    c->clamps = calloc((size_t)n_groups, sizeof(int64_t));
    int64_t n_src = 0;
    for (int g = 0; g < n_groups; ++g) n_src += 3 * (int64_t)groups[g].n_beads;
    c->src = calloc((size_t)n_src, sizeof(double));
    if (!c->groups || !c->k_begin || !c->k_end || !c->pos_off || !c->smp_off ||
        !c->spr_off || !c->clamps || !c->src) { ra_oracle_destroy(c); return RAO_ENOMEM; }
    memcpy(c->groups, groups, sizeof(rao_group) * (size_t)n_groups);
    for (int g = 0; g < n_groups; ++g) { c->k_begin[g] = 0; c->k_end[g] = groups[g].n_replicas; }
    c->seed = seed; c->sample_every = sample_every; c->max_windows = max_windows;
    c->tsf = tsf ? 1 : 0; c->tangents = tangents ? 1 : 0;
    c->tag = RAO_TAG_REPLICA;
    int rc = layout(c);
    if (rc != RAO_OK) { ra_oracle_destroy(c); return rc; }
    *out = c;
    return RAO_OK;
}

int ra_oracle_set_replicas(rao_ctx* c, int32_t g, int32_t k_begin, int32_t k_end)
{
    if (!c || g < 0 || g >= c->n_groups || k_begin < 0 || k_end <= k_begin ||
        k_end > c->groups[g].n_replicas)
        return fail(c, RAO_EINVAL, "bad replica range");
    c->k_begin[g] = k_begin; c->k_end[g] = k_end;
    return layout(c);
}

int64_t ra_oracle_n_windows(const rao_ctx* c) { return c ? c->n_windows : 0; }
int64_t ra_oracle_total_springs(const rao_ctx* c) { return c ? c->n_spr : 0; }
int64_t ra_oracle_clamps(const rao_ctx* c, int32_t g)
{
    return (c && g >= 0 && g < c->n_groups) ? c->clamps[g] : -1;
}

/* Copy the parent conformation into every simulated replica and remember it
 * as the clone source; rejects a FENE bond at or past full extension and
 * non-finite coordinates. */
static int clone_from(rao_ctx* c, const double* parent_xyz)
{
    int64_t par = 0;
    for (int g = 0; g < c->n_groups; ++g) {
        const rao_group* d = &c->groups[g];
        int n = d->n_beads;
        const double* p = parent_xyz + par;
        if (d->spring == RAO_FENE) {
            double q0sq = d->b * d->kT / d->H;
            for (int j = 0; j + 1 < n; ++j) {
                double Q[3] = { p[3 * (j + 1)] - p[3 * j], p[3 * (j + 1) + 1] - p[3 * j + 1],
                                p[3 * (j + 1) + 2] - p[3 * j + 2] };
                if (!(dot3(Q, Q) < q0sq))
                    return fail(c, RAO_EINVAL, "parent FENE bond at or beyond full extension");
            }
        }
        for (int i = 0; i < 3 * n; ++i)
            if (!isfinite(p[i])) return fail(c, RAO_EINVAL, "non-finite parent coordinate");
        par += 3 * n;
    }
    par = 0;
    for (int g = 0; g < c->n_groups; ++g) {
        int n = c->groups[g].n_beads;
        const double* p = parent_xyz + par;
        int rs = c->k_end[g] - c->k_begin[g];
        for (int k = 0; k < rs; ++k)
            memcpy(c->pos + c->pos_off[g] + (int64_t)k * n * 3, p, sizeof(double) * 3 * (size_t)n);
        memcpy(c->src + par, p, sizeof(double) * 3 * (size_t)n);
        par += 3 * n;
    }
    if (c->tan) memset(c->tan, 0, sizeof(double) * (size_t)(3 * c->n_pos));
    if (c->tsf_acc) memset(c->tsf_acc, 0, sizeof(double) * (size_t)c->n_smp);
    return RAO_OK;
}

/* RSF clone (Sec. II): every replica starts from the parent conformation. */
int ra_oracle_init_chains(rao_ctx* c, const double* parent_xyz)
{
    if (!c || !parent_xyz) return fail(c, RAO_EINVAL, "null argument");
    int rc = clone_from(c, parent_xyz);
    if (rc != RAO_OK) return rc;
    for (int g = 0; g < c->n_groups; ++g) c->clamps[g] = 0;
    c->step = 0; c->n_windows = 0; c->initialised = 1;
    return RAO_OK;
}

int ra_oracle_set_tag(rao_ctx* c, uint32_t tag)
{
    if (!c || (tag != RAO_TAG_REPLICA && tag != RAO_TAG_PARENT))
        return fail(c, RAO_EINVAL, "tag must be REPLICA or PARENT");
    c->tag = tag;
    return RAO_OK;
}

int ra_oracle_set_noise_map(rao_ctx* c, int32_t map)
{
    if (!c || map < 0 || map > 2) return fail(c, RAO_EINVAL, "noise map must be 0, 1 or 2");
    c->noise_map = map;
    return RAO_OK;
}

/* RSF re-clone (Sec. II): at a force-sampling time the parent is halted and
 * every replica restarts from its current conformation. The replicas keep
 * their step count, a multiple of S, so the replicas of each window draw their
 * own counters (w*S + s); samples of earlier windows are kept. */
int ra_oracle_reclone(rao_ctx* c, const double* parent_xyz)
{
    if (!c || !parent_xyz) return fail(c, RAO_EINVAL, "null argument");
    if (c->step % c->sample_every != 0)
        return fail(c, RAO_EINVAL, "re-clone only at a window boundary (step count a multiple of S)");
    if (c->tangents) return fail(c, RAO_ESTATE, "re-clone is not differentiated");
    int rc = clone_from(c, parent_xyz);
    if (rc != RAO_OK) return rc;
    c->initialised = 1;
    return RAO_OK;
}

/* The RSF sampling cycle (Sec. II). Window w: the parent chain (context par,
 * one replica per group, parent noise tag) continues its own trajectory for
 * parent_steps steps, which par samples as one window (ISF at the end, TSF
 * over the steps when par keeps TSF); the parent is halted, the replicas are
 * re-cloned from its conformation and evolve for S steps, and each replica's
 * spring tensions are sampled once at the end (RSF window w). The replicas'
 * windows continue from those already sampled. */
int ra_oracle_rsf_cycle(rao_ctx* rep, rao_ctx* par, int64_t n_windows, int64_t parent_steps)
{
    if (!rep || !par || n_windows < 0 || parent_steps < 1) return fail(rep, RAO_EINVAL, "bad argument");
    if (par->n_groups != rep->n_groups || par->sample_every != parent_steps || !par->initialised)
        return fail(rep, RAO_EINVAL, "parent context must match groups, sample every parent_steps, be initialised");
    for (int g = 0; g < rep->n_groups; ++g)
        if (par->groups[g].n_beads != rep->groups[g].n_beads || par->k_end[g] - par->k_begin[g] != 1)
            return fail(rep, RAO_EINVAL, "parent context needs one chain of the same length per group");
    double* xyz = malloc(sizeof(double) * (size_t)(par->n_pos + 1));
    if (!xyz) return fail(rep, RAO_ENOMEM, "out of host memory");
    int rc = RAO_OK;
    for (int64_t w = 0; w < n_windows && rc == RAO_OK; ++w) {
        rc = ra_oracle_step(par, parent_steps);
        if (rc != RAO_OK) { fail(rep, rc, ra_oracle_last_error(par)); break; }
        memcpy(xyz, par->pos, sizeof(double) * (size_t)par->n_pos);
        rc = ra_oracle_reclone(rep, xyz);
        if (rc == RAO_OK) rc = ra_oracle_step(rep, rep->sample_every);
    }
    free(xyz);
    return rc;
}

/* Pathwise derivatives of the spring force for the forward-mode tangents.
 * dF = (dF/dQ) dQ + dF/dtheta_p, p in {rate, H, b}. */
static void spring_tangent(int spring, double H, double b, double kT, const double Q[3],
                           double g, double s, int clamped, int p, const double dQ[3],
                           double dF[3])
{
    int smooth = (spring == RAO_FENE) && !clamped;   /* dg/ds = g^2 only if unclamped */
    double q0sq = (spring == RAO_FENE) ? b * kT / H : 1.0;
    double qdq = dot3(Q, dQ);
    for (int a = 0; a < 3; ++a) {
        double v = H * g * dQ[a];
        if (smooth) v += H * 2.0 * g * g * qdq / q0sq * Q[a];
        if (p == 1) v += smooth ? g * Q[a] * (1.0 + g * s) : g * Q[a];
        if (p == 2 && smooth) v += -H * g * g * (s / b) * Q[a];
        dF[a] = v;
    }
}

static double tension_tangent(int spring, double H, double b, double g, double s,
                              int clamped, int p, const double Q[3], const double dQ[3])
{
    int smooth = (spring == RAO_FENE) && !clamped;
    double q = sqrt(dot3(Q, Q));
    double df = 0.0;
    if (q > 0.0) df = H * (g + (smooth ? 2.0 * g * g * s : 0.0)) * dot3(Q, dQ) / q;
    if (p == 1) df += smooth ? g * q * (1.0 + g * s) : g * q;
    if (p == 2 && smooth) df += -H * g * g * (s / b) * q;
    return df;
}

/* Eq. (1) with hydrodynamic interaction: the 3N x 3N tensor D of Eqs. (2)-(3)
 * from the step-n positions, drift dt (v + D F / kT), random displacement
 * sqrt(2 dt) L xi with D = L L^T (Cholesky) and xi the per-bead normals of the
 * replica counter. hi holds (3N)^2 + 3N doubles. */
static int hi_update(rao_ctx* c, const rao_group* d, int k, uint32_t n, double* r, const double* F,
                     double* hi)
{
    const int N = d->n_beads, n3 = 3 * N;
    double* D = hi;
    double* xi = hi + (size_t)n3 * n3;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            double B[9];
            if (i == j) {
                for (int e = 0; e < 9; ++e) B[e] = (e % 4 == 0) ? d->kT / d->zeta : 0.0;
            } else {
                double rij[3] = { r[3 * j] - r[3 * i], r[3 * j + 1] - r[3 * i + 1], r[3 * j + 2] - r[3 * i + 2] };
                rao_rpy_block(d->kT, d->zeta, d->hi_radius, rij, B);
            }
            for (int x = 0; x < 3; ++x)
                for (int y = 0; y < 3; ++y) D[(3 * i + x) * n3 + 3 * j + y] = B[3 * x + y];
        }
    double* step = malloc(sizeof(double) * (size_t)n3);
    if (!step) return fail(c, RAO_ENOMEM, "out of host memory");
    for (int a = 0; a < n3; ++a) {          /* drift: dt (v + D F / kT) */
        double df = 0.0;
        for (int b = 0; b < n3; ++b) df += D[a * n3 + b] * F[b];
        step[a] = d->dt * df / d->kT;
    }
    for (int i = 0; i < N; ++i) {
        double v[3];
        rao_flow_velocity(d->flow, d->rate, r + 3 * i, v);
        for (int x = 0; x < 3; ++x) step[3 * i + x] += d->dt * v[x];
        rao_noise_mapped(c->seed, n, (uint32_t)i, (uint32_t)k, c->tag, d->stream_id, c->noise_map, xi + 3 * i);
    }
    if (rao_cholesky(n3, D) != 0) {
        free(step);
        return fail(c, RAO_EINVAL, "diffusion tensor is not positive definite");
    }
    const double sc = d->noise_scale * sqrt(2.0 * d->dt);
    for (int a = 0; a < n3; ++a) {          /* random displacement sqrt(2 dt) L xi */
        double y = 0.0;
        for (int b = 0; b <= a; ++b) y += D[a * n3 + b] * xi[b];
        step[a] += sc * y;
    }
    for (int a = 0; a < n3; ++a) r[a] += step[a];
    free(step);
    return RAO_OK;
}

/* One Euler-Maruyama step of Eq. (1) with the free-draining tensor Eq. (2)
 * for replica k of group g: all beads advance together from the step-n
 * state; the random displacement has covariance 2 (kT/zeta) dt I. */
static int em_step_replica(rao_ctx* c, int g, int kk, uint32_t n,
                           double* Fbuf, double* Fnet, double* dF, double* dFnet, double* hi)
{
    const rao_group* d = &c->groups[g];
    const int N = d->n_beads;
    const int k = c->k_begin[g] + kk;
    const int rs = c->k_end[g] - c->k_begin[g];
    double* r = c->pos + c->pos_off[g] + (int64_t)kk * N * 3;
    const double sigma = d->noise_scale * sqrt(2.0 * d->kT * d->dt / d->zeta);

    /* spring forces from the step-n positions */
    for (int j = 0; j + 1 < N; ++j) {
        double Q[3], F[3], gj, f, s;
        for (int a = 0; a < 3; ++a) Q[a] = r[3 * (j + 1) + a] - r[3 * j + a];
        int clamped = rao_spring(d->spring, d->H, spring_p2(d), d->kT, Q, F, &gj, &f);
        spring_factor(d->spring, d->H, spring_p2(d), d->kT, Q, &gj, &s);
        c->clamps[g] += clamped;
        for (int a = 0; a < 3; ++a) Fbuf[3 * j + a] = F[a];
        if (c->tangents) {
            for (int p = 0; p < 3; ++p) {
                const double* t = c->tan + (int64_t)p * c->n_pos + c->pos_off[g] + (int64_t)kk * N * 3;
                double dQ[3];
                for (int a = 0; a < 3; ++a) dQ[a] = t[3 * (j + 1) + a] - t[3 * j + a];
                spring_tangent(d->spring, d->H, d->b, d->kT, Q, gj, s, clamped, p, dQ,
                               dF + (int64_t)p * 3 * N + 3 * j);
            }
        }
    }
    /* net spring force on bead i: pulled forward by spring i, back by spring i-1 */
    for (int i = 0; i < N; ++i)
        for (int a = 0; a < 3; ++a) {
            double v = 0.0;
            if (i <= N - 2) v += Fbuf[3 * i + a];
            if (i >= 1) v -= Fbuf[3 * (i - 1) + a];
            Fnet[3 * i + a] = v;
            if (c->tangents)
                for (int p = 0; p < 3; ++p) {
                    double w = 0.0;
                    if (i <= N - 2) w += dF[(int64_t)p * 3 * N + 3 * i + a];
                    if (i >= 1) w -= dF[(int64_t)p * 3 * N + 3 * (i - 1) + a];
                    dFnet[(int64_t)p * 3 * N + 3 * i + a] = w;
                }
        }
    /* Lennard-Jones self-association between non-adjacent beads (|i - j| >= 2) */
    if (d->lj_eps > 0)
        for (int i = 0; i < N; ++i)
            for (int j = i + 2; j < N; ++j) {
                double dv[3], F[3];
                for (int a = 0; a < 3; ++a) dv[a] = r[3 * i + a] - r[3 * j + a];
                rao_lj(d->lj_eps, d->lj_rmin, dv, F);
                for (int a = 0; a < 3; ++a) {
                    Fnet[3 * i + a] += F[a];
                    Fnet[3 * j + a] -= F[a];
                }
            }
    if (d->hi_radius > 0) return hi_update(c, d, k, n, r, Fnet, hi);
    /* position update */
    for (int i = 0; i < N; ++i) {
        double xi[3], v[3];
        rao_noise_mapped(c->seed, n, (uint32_t)i, (uint32_t)k, c->tag, d->stream_id, c->noise_map, xi);
        rao_flow_velocity(d->flow, d->rate, r + 3 * i, v);
        if (c->tangents) {
            for (int p = 0; p < 3; ++p) {
                double* t = c->tan + (int64_t)p * c->n_pos + c->pos_off[g] + (int64_t)kk * N * 3;
                double dv[3];
                rao_flow_velocity(d->flow, d->rate, t + 3 * i, dv);
                if (p == 0) {   /* d(kappa . r)/d rate = (kappa/rate) . r */
                    double pat[3];
                    rao_flow_velocity(d->flow, 1.0, r + 3 * i, pat);
                    for (int a = 0; a < 3; ++a) dv[a] += pat[a];
                }
                for (int a = 0; a < 3; ++a)
                    t[3 * i + a] += d->dt * (dv[a] + dFnet[(int64_t)p * 3 * N + 3 * i + a] / d->zeta);
            }
        }
        for (int a = 0; a < 3; ++a)
            Fnet[3 * i + a] = d->dt * (v[a] + Fnet[3 * i + a] / d->zeta) + sigma * xi[a];
    }
    for (int i = 0; i < 3 * N; ++i) r[i] += Fnet[i];
    (void)rs;
    return RAO_OK;
}

/* Tension of every spring of replica kk (after the step), for RSF/TSF. */
static void sample_replica(rao_ctx* c, int g, int kk, int window_end, int64_t w)
{
    const rao_group* d = &c->groups[g];
    const int N = d->n_beads;
    const int rs = c->k_end[g] - c->k_begin[g];
    const double* r = c->pos + c->pos_off[g] + (int64_t)kk * N * 3;
    for (int j = 0; j + 1 < N; ++j) {
        double Q[3], F[3], gj, f, s;
        for (int a = 0; a < 3; ++a) Q[a] = r[3 * (j + 1) + a] - r[3 * j + a];
        int clamped = rao_spring(d->spring, d->H, spring_p2(d), d->kT, Q, F, &gj, &f);
        spring_factor(d->spring, d->H, spring_p2(d), d->kT, Q, &gj, &s);
        int64_t idx = c->smp_off[g] + (int64_t)kk * (N - 1) + j;
        if (c->tsf) c->tsf_acc[idx] += f;
        if (!window_end) continue;
        c->samples[w * c->n_smp + idx] = f;
        if (c->tsf) {
            c->tsf_samples[w * c->n_smp + idx] = c->tsf_acc[idx] / (double)c->sample_every;
            c->tsf_acc[idx] = 0.0;
        }
        if (c->tangents) {
            for (int p = 0; p < 3; ++p) {
                const double* t = c->tan + (int64_t)p * c->n_pos + c->pos_off[g] + (int64_t)kk * N * 3;
                double dQ[3];
                for (int a = 0; a < 3; ++a) dQ[a] = t[3 * (j + 1) + a] - t[3 * j + a];
                c->dmu[(w * c->n_spr + c->spr_off[g] + j) * 3 + p] +=
                    tension_tangent(d->spring, d->H, d->b, gj, s, clamped, p, Q, dQ) / (double)rs;
            }
        }
    }
}

int ra_oracle_step(rao_ctx* c, int64_t n_steps)
{
    if (!c) return RAO_EINVAL;
    if (!c->initialised) return fail(c, RAO_ESTATE, "step before init_chains");
    if (n_steps < 0) return fail(c, RAO_EINVAL, "negative step count");
    int64_t end = c->step + n_steps;
    if (end > 0xFFFFFFFFll) return fail(c, RAO_EINVAL, "step counter exceeds 32 bits");
    if (end / c->sample_every > c->max_windows) return fail(c, RAO_EINVAL, "window capacity exceeded");
    int nmax = 2;
    for (int g = 0; g < c->n_groups; ++g) if (c->groups[g].n_beads > nmax) nmax = c->groups[g].n_beads;
    double* Fbuf = malloc(sizeof(double) * 3 * (size_t)nmax);
    double* Fnet = malloc(sizeof(double) * 3 * (size_t)nmax);
    double* dF = malloc(sizeof(double) * 9 * (size_t)nmax);
    double* dFnet = malloc(sizeof(double) * 9 * (size_t)nmax);
    double* hi = malloc(sizeof(double) * ((size_t)9 * nmax * nmax + 3 * (size_t)nmax));
    if (!Fbuf || !Fnet || !dF || !dFnet || !hi) {
        free(Fbuf); free(Fnet); free(dF); free(dFnet); free(hi);
        return fail(c, RAO_ENOMEM, "out of host memory");
    }
    int rc = RAO_OK;
    for (; c->step < end && rc == RAO_OK; ++c->step) {
        uint32_t n = (uint32_t)c->step;
        int window_end = ((c->step + 1) % c->sample_every) == 0;
        int64_t w = (c->step + 1) / c->sample_every - 1;
        for (int g = 0; g < c->n_groups && rc == RAO_OK; ++g) {
            int rs = c->k_end[g] - c->k_begin[g];
            for (int kk = 0; kk < rs && rc == RAO_OK; ++kk) {
                rc = em_step_replica(c, g, kk, n, Fbuf, Fnet, dF, dFnet, hi);
                if (c->tsf || window_end) sample_replica(c, g, kk, window_end, w);
            }
        }
        if (window_end) c->n_windows = w + 1;
    }
    free(Fbuf); free(Fnet); free(dF); free(dFnet); free(hi);
    return rc;
}

/* RSF estimate (Sec. II): replica mean of the sampled tension and the
 * replica standard deviation (denominator R-1), two-pass. */
static void replica_stats(const rao_ctx* c, const double* smp, double* mean, double* std)
{
    for (int64_t w = 0; w < c->n_windows; ++w)
        for (int g = 0; g < c->n_groups; ++g) {
            int N = c->groups[g].n_beads;
            int rs = c->k_end[g] - c->k_begin[g];
            for (int j = 0; j + 1 < N; ++j) {
                double sum = 0.0;
                for (int kk = 0; kk < rs; ++kk)
                    sum += smp[w * c->n_smp + c->smp_off[g] + (int64_t)kk * (N - 1) + j];
                double mu = sum / rs;
                double ss = 0.0;
                for (int kk = 0; kk < rs; ++kk) {
                    double e = smp[w * c->n_smp + c->smp_off[g] + (int64_t)kk * (N - 1) + j] - mu;
                    ss += e * e;
                }
                int64_t o = w * c->n_spr + c->spr_off[g] + j;
                if (mean) mean[o] = mu;
                if (std) std[o] = rs > 1 ? sqrt(ss / (rs - 1)) : 0.0;
            }
        }
}

int ra_oracle_average_forces(rao_ctx* c, double* mean, double* std,
                             double* tsf_mean, double* tsf_std)
{
    if (!c) return RAO_EINVAL;
    replica_stats(c, c->samples, mean, std);
    if (tsf_mean || tsf_std) {
        if (!c->tsf) return fail(c, RAO_ESTATE, "TSF not enabled");
        replica_stats(c, c->tsf_samples, tsf_mean, tsf_std);
    }
    return RAO_OK;
}

/* Bell-type rate law (Sec. III): k = k0 exp(x_dagger f / kT) per spring, the
 * summed rate per chain, and optionally one event draw per spring per window
 * with probability 1 - exp(-k * window length). */
int ra_oracle_bell_rates(rao_ctx* c, const double* mean, int64_t n_windows,
                         double k0, double x_dagger, double* rates,
                         double* rate_sum, uint8_t* events)
{
    if (!c || !mean || n_windows < 0) return RAO_EINVAL;
    uint32_t key[2] = { (uint32_t)c->seed, (uint32_t)(c->seed >> 32) };
    for (int64_t w = 0; w < n_windows; ++w)
        for (int g = 0; g < c->n_groups; ++g) {
            const rao_group* d = &c->groups[g];
            double sum = 0.0;
            for (int j = 0; j + 1 < d->n_beads; ++j) {
                int64_t o = w * c->n_spr + c->spr_off[g] + j;
                double k = k0 * exp(x_dagger * mean[o] / d->kT);
                if (rates) rates[o] = k;
                sum += k;
                if (events) {
                    uint32_t ctr[4] = { (uint32_t)w, (uint32_t)j, 0u,
                                        ((uint32_t)RAO_TAG_EVENT << 24) | d->stream_id };
                    uint32_t x[4];
                    rao_philox4x32_10(ctr, key, x);
                    double p = -expm1(-k * c->sample_every * d->dt);
                    events[o] = rao_uniform53(x[0], x[1]) < p ? 1 : 0;
                }
            }
            if (rate_sum) rate_sum[w * c->n_groups + g] = sum;
        }
    return RAO_OK;
}

int ra_oracle_backward(rao_ctx* c, const double* grad_mean, const double* grad_rates,
                       double k0, double x_dagger, double* grad_params)
{
    if (!c || !grad_params) return RAO_EINVAL;
    if (!c->tangents) return fail(c, RAO_ESTATE, "tangents not enabled");
    double* mean = malloc(sizeof(double) * (size_t)(c->n_windows * c->n_spr + 1));
    if (!mean) return fail(c, RAO_ENOMEM, "out of host memory");
    replica_stats(c, c->samples, mean, NULL);
    for (int g = 0; g < c->n_groups; ++g) {
        const rao_group* d = &c->groups[g];
        double acc[3] = { 0.0, 0.0, 0.0 };
        for (int64_t w = 0; w < c->n_windows; ++w)
            for (int j = 0; j + 1 < d->n_beads; ++j) {
                int64_t o = w * c->n_spr + c->spr_off[g] + j;
                double lam = grad_mean ? grad_mean[o] : 0.0;
                if (grad_rates) {
                    double k = k0 * exp(x_dagger * mean[o] / d->kT);
                    lam += grad_rates[o] * k * x_dagger / d->kT;
                }
                for (int p = 0; p < 3; ++p) acc[p] += lam * c->dmu[o * 3 + p];
            }
        for (int p = 0; p < 3; ++p) grad_params[3 * g + p] = acc[p];
    }
    free(mean);
    return RAO_OK;
}

/* Spread of the RSF estimator for N_R = block replicas (Figs. 2 and 5):
 * the R replicas of a group are split into B = floor(R/block) consecutive
 * blocks, each block's mean tension is one RSF estimate, and sigma is their
 * standard deviation (denominator B-1) per window and spring. */
int ra_oracle_block_sigma(const rao_ctx* c, int32_t block, double* sigma)
{
    if (!c || !sigma || block < 1) return RAO_EINVAL;
    for (int64_t w = 0; w < c->n_windows; ++w)
        for (int g = 0; g < c->n_groups; ++g) {
            int N = c->groups[g].n_beads;
            int rs = c->k_end[g] - c->k_begin[g];
            int B = rs / block;
            for (int j = 0; j + 1 < N; ++j) {
                double sum = 0.0;
                for (int b = 0; b < B; ++b) {
                    double m = 0.0;
                    for (int q = 0; q < block; ++q)
                        m += c->samples[w * c->n_smp + c->smp_off[g] + (int64_t)(b * block + q) * (N - 1) + j];
                    sum += m / block;
                }
                double mu = B > 0 ? sum / B : 0.0;
                double ss = 0.0;
                for (int b = 0; b < B; ++b) {
                    double m = 0.0;
                    for (int q = 0; q < block; ++q)
                        m += c->samples[w * c->n_smp + c->smp_off[g] + (int64_t)(b * block + q) * (N - 1) + j];
                    double e = m / block - mu;
                    ss += e * e;
                }
                sigma[w * c->n_spr + c->spr_off[g] + j] = B > 1 ? sqrt(ss / (B - 1)) : 0.0;
            }
        }
    return RAO_OK;
}

/* Mean first-passage time to any event on a chain (MFTU, Sec. III): with
 * the per-chain total rate K_w = sum_j k_j held over each window, and K
 * stationary over the run, the first event time is exponential with mean
 * 1 / <K>, <K> the average of K_w over the windows. */
/* MFTU by sampling unfolding events (Sec. III, Table 1), trial by trial:
 * window v = 0, 1, ... of a trial carries the rates of sampled window
 * v mod n_windows; each spring unfolds in window v with probability
 * 1 - exp(-k S dt), decided by the tag-2 uniform of counter (v, spring,
 * trial, group). The trial's first-passage time is the end of the first
 * window with any unfolding, (v + 1) S dt; a trial without one in max_windows
 * windows contributes max_windows S dt and no event. mftu = total time of all
 * trials / number of trials with an event (the maximum-likelihood mean of an
 * exponential waiting time under censoring), +Inf if no trial has one. */
int ra_oracle_mftu_events(const rao_ctx* c, const double* rates, int64_t n_windows, int32_t n_trials,
                          int64_t max_windows, int64_t* first_window, double* mftu)
{
    if (!c || !rates || !mftu || n_windows < 1 || n_trials < 1 || max_windows < 1 ||
        max_windows > (int64_t)0xFFFFFFFF)
        return RAO_EINVAL;
    uint32_t key[2] = { (uint32_t)c->seed, (uint32_t)(c->seed >> 32) };
    for (int g = 0; g < c->n_groups; ++g) {
        const rao_group* d = &c->groups[g];
        const double window_time = c->sample_every * d->dt;
        double total = 0.0;
        int64_t n_events = 0;
        for (int32_t t = 0; t < n_trials; ++t) {
            int64_t first = -1;
            for (int64_t v = 0; v < max_windows && first < 0; ++v) {
                int64_t w = v % n_windows;
                for (int j = 0; j + 1 < d->n_beads; ++j) {
                    double k = rates[w * c->n_spr + c->spr_off[g] + j];
                    uint32_t ctr[4] = { (uint32_t)v, (uint32_t)j, (uint32_t)t,
                                        ((uint32_t)RAO_TAG_EVENT << 24) | d->stream_id };
                    uint32_t x[4];
                    rao_philox4x32_10(ctr, key, x);
                    if (rao_uniform53(x[0], x[1]) < -expm1(-k * window_time)) first = v;
                }
            }
            if (first_window) first_window[(int64_t)t * c->n_groups + g] = first;
            if (first >= 0) {
                total += (double)(first + 1) * window_time;
                n_events += 1;
            } else {
                total += (double)max_windows * window_time;
            }
        }
        mftu[g] = n_events > 0 ? total / (double)n_events : INFINITY;
    }
    return RAO_OK;
}

int ra_oracle_mftu(const rao_ctx* c, const double* rate_sum, int64_t n_windows, double* mftu)
{
    if (!c || !rate_sum || !mftu || n_windows < 1) return RAO_EINVAL;
    for (int g = 0; g < c->n_groups; ++g) {
        double sum = 0.0;
        for (int64_t w = 0; w < n_windows; ++w) sum += rate_sum[w * c->n_groups + g];
        mftu[g] = 1.0 / (sum / (double)n_windows);
    }
    return RAO_OK;
}

/* Centre-of-mass-frame coordinates of one chain: out[i][a] = r[i][a] - r_cm[a]. */
static void com_frame(const double* r, int N, double* out)
{
    double cm[3] = { 0.0, 0.0, 0.0 };
    for (int i = 0; i < N; ++i)
        for (int a = 0; a < 3; ++a) cm[a] += r[3 * i + a];
    for (int a = 0; a < 3; ++a) cm[a] /= N;
    for (int i = 0; i < N; ++i)
        for (int a = 0; a < 3; ++a) out[3 * i + a] = r[3 * i + a] - cm[a];
}

/* Replica fidelity (Sec. IV, Eq. 5): for replica k and component a,
 * dbar[k][a] = (1/N) sum_i |rhat_a^i(k) - rhat_a^i(source)|, rhat the
 * centre-of-mass-frame coordinates and source the conformation the replicas
 * were last cloned from; d_bead[k][i][a] the same without the bead average.
 * rg2[k][a] = (1/N) sum_i (rhat_a^i)^2, the component contributions to the
 * squared radius of gyration (R_Gz^2 is a = z); src_rg2[g][a] likewise for
 * the source. Replicas are the simulated ones, groups concatenated. Any
 * output may be NULL. */
int ra_oracle_conformation(const rao_ctx* c, double* dbar, double* d_bead, double* rg2, double* src_rg2)
{
    if (!c || !c->initialised) return RAO_EINVAL;
    int nmax = 2;
    for (int g = 0; g < c->n_groups; ++g) if (c->groups[g].n_beads > nmax) nmax = c->groups[g].n_beads;
    double* hs = malloc(sizeof(double) * 3 * (size_t)nmax);
    double* hr = malloc(sizeof(double) * 3 * (size_t)nmax);
    if (!hs || !hr) { free(hs); free(hr); return RAO_ENOMEM; }
    int64_t src_off = 0, kglob = 0, bglob = 0;
    for (int g = 0; g < c->n_groups; ++g) {
        int N = c->groups[g].n_beads;
        int rs = c->k_end[g] - c->k_begin[g];
        com_frame(c->src + src_off, N, hs);
        if (src_rg2)
            for (int a = 0; a < 3; ++a) {
                double v = 0.0;
                for (int i = 0; i < N; ++i) v += hs[3 * i + a] * hs[3 * i + a];
                src_rg2[3 * g + a] = v / N;
            }
        for (int k = 0; k < rs; ++k, ++kglob) {
            com_frame(c->pos + c->pos_off[g] + (int64_t)k * N * 3, N, hr);
            for (int a = 0; a < 3; ++a) {
                double dsum = 0.0, rsum = 0.0;
                for (int i = 0; i < N; ++i) {
                    double d = fabs(hr[3 * i + a] - hs[3 * i + a]);
                    if (d_bead) d_bead[(bglob + (int64_t)k * N + i) * 3 + a] = d;
                    dsum += d;
                    rsum += hr[3 * i + a] * hr[3 * i + a];
                }
                if (dbar) dbar[kglob * 3 + a] = dsum / N;
                if (rg2) rg2[kglob * 3 + a] = rsum / N;
            }
        }
        bglob += (int64_t)rs * N;
        src_off += 3 * N;
    }
    free(hs); free(hr);
    return RAO_OK;
}

int ra_oracle_get_samples(const rao_ctx* c, double* out, double* tsf_out)
{
    if (!c) return RAO_EINVAL;
    if (out) memcpy(out, c->samples, sizeof(double) * (size_t)(c->n_windows * c->n_smp));
    if (tsf_out) {
        if (!c->tsf) return RAO_ESTATE;
        memcpy(tsf_out, c->tsf_samples, sizeof(double) * (size_t)(c->n_windows * c->n_smp));
    }
    return RAO_OK;
}

int ra_oracle_get_positions(const rao_ctx* c, double* out)
{
    if (!c || !out) return RAO_EINVAL;
    memcpy(out, c->pos, sizeof(double) * (size_t)c->n_pos);
    return RAO_OK;
}
