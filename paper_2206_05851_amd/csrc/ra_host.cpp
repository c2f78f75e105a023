// ra_host.cpp — implementation of the C ABI declared in include/ra.h.
//
// Owns the context: descriptor validation, per-group tile choice, device
// memory, the LPT-ordered work list of the persistent forward kernel, hipGraph
// capture of ra_step, and the adjoint's checkpoint and segment stores.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "ra.h"
#include "ra_launch.hpp"
#include "ra_tune.hpp"
#include "ra_types.hpp"

using namespace ra;

struct ra_ctx {
    std::vector<ra_chain_desc> descs;
    ra_run_desc run{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int family = 4;
    int wpb = 4;
    std::vector<GroupDev> hgroups;
    std::vector<Item> hitems;
    std::vector<ColTile> htiles;
    std::vector<int32_t> item_begin, item_count;   // per group, in the sorted work list
    GroupDev* dgroups = nullptr;
    Item* ditems = nullptr;
    ColTile* dtiles = nullptr;
    int64_t* dpar_off = nullptr;
    int32_t* ditem_begin = nullptr;
    int64_t state_total = 0, smp_total = 0, spr_total = 0, pos_total = 0, ckpt_total = 0;
    int64_t max_group_elems = 0;
    void* state = nullptr;          // fused path bond state
    void* pos[2] = {nullptr, nullptr};
    int cur = 0;                    // plain path: current position buffer
    void* samples = nullptr;
    void* tsf = nullptr;
    double* tsf_acc = nullptr;
    void* ckpt = nullptr;
    int64_t n_ckpt = 0;
    float* segbuf = nullptr;
    int64_t* dseg_off = nullptr;
    double* partial = nullptr;
    double* lam_mu = nullptr;
    int32_t* status = nullptr;
    unsigned long long* clamps = nullptr;
    int64_t* dstep = nullptr;
    double* src = nullptr;          // [sum_g N_g][3] centre-of-mass frame of the clone source
    int64_t* drep_off = nullptr;    // [n_groups + 1] first replica of each group
    int64_t n_reps = 0;
    hipEvent_t ev_parent = nullptr, ev_reclone = nullptr;   // RSF cycle across two streams
    int64_t step = 0;
    bool initialised = false;
    bool recloned = false;          // a re-clone since the last init (no adjoint)
    int hi_nmax = 0;                // largest N of an HI context (sizes the kernel's LDS)
    std::map<int64_t, hipGraphExec_t> graphs;
    std::string err;
};

namespace {

thread_local std::string g_err;

ra_status fail(ra_ctx* c, ra_status code, const std::string& msg) {
    if (c) c->err = msg;
    else g_err = msg;
    return code;
}

#define HIPCHK(ctx, expr)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(ctx, e_ == hipErrorOutOfMemory ? RA_ENOMEM : RA_EDEVICE,               \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                    \
    } while (0)

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Groups with hydrodynamic interaction run the HI kernel; other groups of the
// collapsed-polymer force field run the pair-interaction kernel.
bool is_hi_group(const ra_chain_desc& d) { return d.hi_radius > 0.0; }
bool is_pair_group(const ra_chain_desc& d) {
    return !is_hi_group(d) && (d.spring == RA_HARMONIC || d.lj_eps > 0.0);
}

}  // namespace

namespace ra {

void set_global_error(const std::string& msg) { g_err = msg; }

ra_status validate(const ra_chain_desc* g, int32_t n, const ra_run_desc* r, std::string& why) {
    char buf[256];
    if (!g || n < 1 || !r) { why = "null descriptor or n_groups < 1"; return RA_EINVAL; }
    if (r->precision != 32 && r->precision != 64) { why = "precision must be 32 or 64"; return RA_EINVAL; }
    if (r->sample_every < 1) { why = "sample_every must be >= 1"; return RA_EINVAL; }
    if (r->max_windows < 0 || r->checkpoint_every < RA_CKPT_AUTO || r->max_steps < 0 || r->waves_per_block < 0) {
        why = "negative capacity";
        return RA_EINVAL;
    }
    if (r->max_windows > 65535) {   // per-window kernels put the window on the grid's y dimension
        why = "max_windows must be <= 65535";
        return RA_EINVAL;
    }
    if (r->checkpoint_every != 0 && (r->precision != 32 || r->plain)) {
        why = "the adjoint (checkpoint_every != 0) needs precision 32 and the fused path";
        return RA_EINVAL;
    }
    if (r->noise_tag != 0 && r->noise_tag != 1) { why = "noise_tag must be 0 or 1"; return RA_EINVAL; }
    if (r->tile_policy != 0 && r->tile_policy != 1 && !(r->tile_policy > 1000 && r->tile_policy <= 1016)) {
        why = "tile_policy must be 0 (cost model), 1 (autotune) or 1000 + m (m beads per lane)";
        return RA_EINVAL;
    }
    if (r->noise_map < 0 || r->noise_map > 2) { why = "noise_map must be 0, 1 or 2"; return RA_EINVAL; }
    const int wpb = r->waves_per_block ? r->waves_per_block : 4;
    if (wpb != 1 && wpb != 2 && wpb != 4) { why = "waves_per_block must be 0, 1, 2 or 4"; return RA_EINVAL; }
    int n_pair = 0, n_hi = 0;
    for (int i = 0; i < n; ++i) {
        if (!(std::isfinite(g[i].hi_radius) && g[i].hi_radius >= 0)) {
            std::snprintf(buf, sizeof buf, "group %d: hi_radius must be finite and >= 0", i);
            why = buf;
            return RA_EINVAL;
        }
        n_pair += is_pair_group(g[i]) ? 1 : 0;
        n_hi += is_hi_group(g[i]) ? 1 : 0;
    }
    if ((n_pair > 0 && n_pair < n) || (n_hi > 0 && n_hi < n)) {
        why = "a context holds only pair-interaction groups (HARMONIC spring or LJ), only "
              "hydrodynamic-interaction groups (hi_radius > 0), or only chain-model groups";
        return RA_EINVAL;
    }
    if ((n_pair > 0 || n_hi > 0) && r->checkpoint_every != 0) {
        why = "the adjoint covers the free-draining Hookean and FENE chain model only";
        return RA_EINVAL;
    }
    if ((n_pair > 0 || n_hi > 0) && r->noise_map != 0) {
        why = "noise_map 1 and 2 cover the free-draining Hookean and FENE chain model only";
        return RA_EINVAL;
    }
    if ((n_pair > 0 || n_hi > 0) && r->plain) {
        why = "the pair-interaction and HI models have no plain path";
        return RA_EINVAL;
    }
    for (int i = 0; i < n; ++i) {
        const ra_chain_desc& d = g[i];
        // FP64 fused kernels hold up to 4 beads per lane; the plain path has no lane limit
        const int nmax = (n_pair || n_hi) ? WAVE : (r->precision == 64 && !r->plain) ? 256 : 1024;
        const char* bad = nullptr;
        if (d.n_beads < 2 || d.n_beads > nmax) bad = "n_beads out of range";
        else if (d.n_replicas < 1) bad = "n_replicas < 1";
        else if (d.spring != RA_HOOKEAN && d.spring != RA_FENE && d.spring != RA_HARMONIC) bad = "unknown spring";
        else if (d.spring == RA_HARMONIC && !(std::isfinite(d.rest_length) && d.rest_length >= 0))
            bad = "HARMONIC needs a finite rest_length >= 0";
        else if (!(std::isfinite(d.lj_eps) && d.lj_eps >= 0)) bad = "lj_eps must be finite and >= 0";
        else if (d.lj_eps > 0 && !finite_pos(d.lj_rmin)) bad = "LJ needs finite lj_rmin > 0";
        else if (d.flow < RA_QUIESCENT || d.flow > RA_SHEAR) bad = "unknown flow";
        else if (!finite_pos(d.H) || !finite_pos(d.kT) || !finite_pos(d.zeta) || !finite_pos(d.dt))
            bad = "H, kT, zeta and dt must be finite and > 0";
        else if (d.spring == RA_FENE && !finite_pos(d.b)) bad = "FENE needs finite b > 0";
        else if (!std::isfinite(d.rate)) bad = "rate must be finite";
        else if (!std::isfinite(d.noise_scale) || d.noise_scale < 0) bad = "noise_scale must be finite and >= 0";
        else if (d.stream_id > 0xFFFFFFu) bad = "stream_id must be < 2^24";
        if (bad) {
            std::snprintf(buf, sizeof buf, "group %d: %s", i, bad);
            why = buf;
            return RA_EINVAL;
        }
    }
    return RA_OK;
}

GroupDev make_group(const ra_chain_desc& d, int M, int tag, int nmap) {
    GroupDev G{};
    G.nmap = nmap;
    G.N = d.n_beads;
    G.R = d.n_replicas;
    G.M = M;
    G.L = (d.n_beads + M - 1) / M;
    G.P = WAVE / G.L;
    G.spring = d.spring;
    G.stream = ((uint32_t)tag << 24) | (d.stream_id & 0xFFFFFFu);   // tag 0 replicas, 1 parent
    G.flow = d.flow;
    double kx = 0, ky = 0, kz = 0, kxz = 0;
    switch (d.flow) {
    case RA_UNIAXIAL: kx = d.rate; ky = -0.5 * d.rate; kz = -0.5 * d.rate; break;
    case RA_PLANAR: kx = d.rate; ky = -d.rate; break;
    case RA_SHEAR: kxz = d.rate; break;
    default: break;
    }
    G.kx_d = d.dt * kx; G.ky_d = d.dt * ky; G.kz_d = d.dt * kz; G.kxz_d = d.dt * kxz;
    G.cF_d = d.H * d.dt / d.zeta;
    G.sigma_d = d.noise_scale * std::sqrt(2.0 * d.kT * d.dt / d.zeta);
    G.H_d = d.H;
    G.inv_q0sq_d = d.spring == RA_FENE ? d.H / (d.b * d.kT) : 0.0;
    G.kx = (float)G.kx_d; G.ky = (float)G.ky_d; G.kz = (float)G.kz_d; G.kxz = (float)G.kxz_d;
    G.cF = (float)G.cF_d; G.sigma = (float)G.sigma_d; G.H = (float)G.H_d; G.inv_q0sq = (float)G.inv_q0sq_d;
    G.kT = d.kT; G.zeta = d.zeta; G.dt = d.dt; G.b = d.b; G.rate = d.rate;
    G.dtz_d = d.dt / d.zeta;
    G.r0_d = d.spring == RA_HARMONIC ? d.rest_length : 0.0;
    G.lj12u_d = 12.0 * d.lj_eps;
    G.ljr2_d = d.lj_eps > 0.0 ? d.lj_rmin * d.lj_rmin : 0.0;
    G.dtz = (float)G.dtz_d; G.r0 = (float)G.r0_d; G.lj12u = (float)G.lj12u_d; G.ljr2 = (float)G.ljr2_d;
    G.hi_a_d = d.hi_radius;
    return G;
}

}  // namespace ra

namespace {

template <typename T>
ra_status dalloc(ra_ctx* c, T** p, size_t count) {
    *p = nullptr;
    if (count == 0) return RA_OK;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, RA_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    return RA_OK;
}

}  // namespace

extern "C" {

const char* ra_last_error(const ra_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

void ra_destroy(ra_ctx* c) {
    if (!c) return;
    // teardown: errors are not actionable here, so their codes are dropped
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    // pos[1] points into the pos[0] allocation and is not freed on its own
    void* ptrs[] = {c->dgroups, c->ditems, c->dtiles, c->dpar_off, c->ditem_begin, c->state, c->pos[0],
                    c->samples, c->tsf, c->tsf_acc, c->ckpt, c->segbuf, c->dseg_off,
                    c->partial, c->lam_mu, c->status, c->clamps, c->dstep, c->src, c->drep_off};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (c->ev_parent) (void)hipEventDestroy(c->ev_parent);
    if (c->ev_reclone) (void)hipEventDestroy(c->ev_reclone);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

ra_status ra_create(ra_ctx** out, const ra_chain_desc* groups, int32_t n_groups, const ra_run_desc* run,
                    void* hip_stream) {
    return ra::create_context(out, groups, n_groups, run, hip_stream, 0);
}

}  // extern "C"

ra_status ra::create_context(ra_ctx** out, const ra_chain_desc* groups, int32_t n_groups, const ra_run_desc* run,
                             void* hip_stream, int force_family) {
    if (!out) return fail(nullptr, RA_EINVAL, "out is null");
    *out = nullptr;
    std::string why;
    if (validate(groups, n_groups, run, why) != RA_OK) return fail(nullptr, RA_EINVAL, why);
    ra_ctx* c = new ra_ctx();
    c->descs.assign(groups, groups + n_groups);
    c->run = *run;
    c->wpb = run->waves_per_block ? run->waves_per_block : 4;
    c->stream = (hipStream_t)hip_stream;
    if (run->use_graph && !c->stream) {
        if (hipStreamCreate(&c->stream) != hipSuccess) {
            ra_destroy(c);
            return fail(nullptr, RA_EDEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }

    // tiles: beads per lane M per group, one kernel family for the whole batch
    std::vector<int> Ms(n_groups);
    int family = 4;
    for (int i = 0; i < n_groups; ++i)
        if (groups[i].n_beads > 4 * WAVE) family = 16;
    if (run->precision == 64 && !run->plain) family = 4;   // the plain path only uses the tile for its work list
    if (force_family == 16 && run->precision == 32 && !run->plain) family = 16;   // a tuner probe of a batch's group
    const bool pair = is_pair_group(groups[0]);   // validated: all groups or none
    const bool hi = is_hi_group(groups[0]);
    if (pair) family = 2;
    if (hi) {
        family = 3;
        int nmax = 2;
        for (int i = 0; i < n_groups; ++i) nmax = std::max(nmax, groups[i].n_beads);
        int dev = 0, lds_max = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
            ra_destroy(c);
            return fail(nullptr, RA_EDEVICE, "cannot query the LDS size per workgroup");
        }
        const size_t need = hi_lds_bytes(nmax, run->precision);
        if (need > (size_t)lds_max) {
            char b2[200];
            std::snprintf(b2, sizeof b2, "n_beads %d needs %zu B of LDS per workgroup for the HI kernel at "
                          "precision %d; the device has %d", nmax, need, run->precision, lds_max);
            ra_destroy(c);
            return fail(nullptr, RA_EINVAL, b2);
        }
        c->hi_nmax = nmax;
    }
    for (int i = 0; i < n_groups; ++i) {
        int forced = run->tile_policy > 1000 ? run->tile_policy - 1000 : 0;
        Ms[i] = (pair || hi) ? 1
                             : choose_beads_per_lane(groups[i].n_beads, groups[i].n_replicas, family, forced,
                                                     run->noise_map);
    }
    if (run->tile_policy == 1 && !run->plain && !pair && !hi) {
        int wpb = run->waves_per_block;   // 0: the tuner chooses the workgroup size too
        ra_status st = autotune_tiles(c->descs, *run, family, wpb, c->stream, Ms, why);
        c->wpb = wpb;
        if (st != RA_OK) {
            ra_destroy(c);
            return fail(nullptr, st, "autotune: " + why);
        }
    }
    c->family = family;
    if (run->noise_map == 1 && !run->plain && family != 4) {
        ra_destroy(c);
        return fail(nullptr, RA_EINVAL, "noise_map 1 needs at most 4 beads per lane (n_beads <= 256) on the fused path");
    }
    if (run->noise_map == 2 && !run->plain && family != 16) {
        ra_destroy(c);
        return fail(nullptr, RA_EINVAL, "noise_map 2 needs 8-16 beads per lane on the fused path: precision 32 and a "
                                        "group with n_beads > 256");
    }

    for (int i = 0; i < n_groups; ++i) {
        if ((groups[i].n_beads + Ms[i] - 1) / Ms[i] > WAVE) {   // a replica must fit in one wavefront
            ra_destroy(c);
            return fail(nullptr, RA_EINVAL, "group " + std::to_string(i) + ": no tile holds its chain in a wavefront");
        }
    }

    // layout
    std::vector<int64_t> par_off(n_groups);
    int64_t par = 0;
    for (int i = 0; i < n_groups; ++i) {
        GroupDev G = make_group(groups[i], Ms[i], run->noise_tag, run->noise_map);
        if (hi) G.P = 1;   // one replica per workgroup
        const int64_t nm1 = G.N - 1;
        G.state_off = c->state_total;
        G.smp_off = c->smp_total;
        G.spr_off = c->spr_total;
        G.pos_off = c->pos_total;
        c->state_total += (int64_t)G.R * nm1 * 3;
        G.ck_off = c->ckpt_total;   // checkpoint rows: [item][slot][xyz][P L lanes]
        c->ckpt_total += (int64_t)((G.R + G.P - 1) / G.P) * G.M * 3 * G.P * G.L;
        c->smp_total += (int64_t)G.R * nm1;
        c->spr_total += nm1;
        c->pos_total += (int64_t)G.R * G.N * 3;
        c->max_group_elems = std::max<int64_t>(c->max_group_elems, (int64_t)G.R * G.N * 3);
        par_off[i] = par;
        par += 3 * (int64_t)G.N;
        c->hgroups.push_back(G);
        for (int j0 = 0; j0 < nm1; j0 += WAVE) c->htiles.push_back(ColTile{i, j0});
    }
    // work list: one wavefront per P replicas, longest (largest M) first
    for (int i = 0; i < n_groups; ++i) {
        const GroupDev& G = c->hgroups[i];
        for (int k0 = 0; k0 < G.R; k0 += G.P) c->hitems.push_back(Item{i, k0});
    }
    std::stable_sort(c->hitems.begin(), c->hitems.end(), [&](const Item& a, const Item& b) {
        return c->hgroups[a.g].M > c->hgroups[b.g].M;
    });
    if (c->hitems.size() > (size_t)INT32_MAX / 2) {
        ra_destroy(c);
        return fail(nullptr, RA_EINVAL, "too many work items");
    }
    c->item_begin.assign(n_groups, -1);
    c->item_count.assign(n_groups, 0);
    for (size_t it = 0; it < c->hitems.size(); ++it) {
        const int g = c->hitems[it].g;
        if (c->item_begin[g] < 0) c->item_begin[g] = (int32_t)it;
        c->item_count[g]++;
    }

    const size_t esz = run->precision == 64 ? 8 : 4;
    if (c->run.checkpoint_every == RA_CKPT_AUTO) {
        // every state when the whole trajectory fits in a quarter of the free
        // device memory (the backward then recomputes nothing), else the
        // interval that minimises checkpoints + segment buffer, sqrt(max_steps)
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
        const double need = ((double)run->max_steps + 1.0) * (double)c->ckpt_total * (double)esz;
        c->run.checkpoint_every =
            need <= 0.25 * (double)free_b ? 1 : std::max(1, (int)std::ceil(std::sqrt((double)std::max(1, run->max_steps))));
    }
    ra_status st = RA_OK;
#define ALLOC(ptr, n)                                              \
    do {                                                           \
        st = dalloc(c, &(ptr), (size_t)(n));                       \
        if (st != RA_OK) { std::string m_ = c->err; ra_destroy(c); \
                           return fail(nullptr, st, m_); }         \
    } while (0)
    // host-to-device copy during set-up; on failure the context is released
#define HCOPY(dst, src, bytes)                                                              \
    do {                                                                                    \
        const hipError_t e_ = hipMemcpy((dst), (src), (bytes), hipMemcpyHostToDevice);      \
        if (e_ != hipSuccess) { ra_destroy(c);                                              \
                                return fail(nullptr, RA_EDEVICE,                            \
                                            std::string("hipMemcpy: ") + hipGetErrorString(e_)); } \
    } while (0)
    char* p8 = nullptr;
    ALLOC(c->dgroups, n_groups);
    ALLOC(c->ditems, c->hitems.size());
    ALLOC(c->dtiles, c->htiles.size());
    ALLOC(c->dpar_off, n_groups);
    ALLOC(c->status, 1);
    ALLOC(c->clamps, n_groups);
    ALLOC(c->dstep, 1);
    ALLOC(c->src, par);
    ALLOC(c->drep_off, n_groups + 1);
    if (run->plain) {
        ALLOC(p8, 2 * c->pos_total * esz);
        c->pos[0] = p8;
        c->pos[1] = p8 + c->pos_total * esz;
    } else {
        ALLOC(p8, c->state_total * esz);
        c->state = p8;
    }
    ALLOC(p8, (int64_t)run->max_windows * c->smp_total * esz);
    c->samples = p8;
    if (run->tsf) {
        ALLOC(p8, (int64_t)run->max_windows * c->smp_total * esz);
        c->tsf = p8;
        ALLOC(c->tsf_acc, c->smp_total);
    }
    if (c->run.checkpoint_every > 0) {
        const int K = c->run.checkpoint_every;
        c->n_ckpt = ((int64_t)run->max_steps + K - 1) / K + 1;
        ALLOC(p8, c->n_ckpt * c->ckpt_total * esz);
        c->ckpt = p8;
        std::vector<int64_t> seg_off(c->hitems.size());
        int64_t tot = 0;
        for (size_t it = 0; it < c->hitems.size(); ++it) {
            seg_off[it] = tot;
            tot += (int64_t)K * c->hgroups[c->hitems[it].g].M * 3 * WAVE;
        }
        ALLOC(c->segbuf, tot);
        ALLOC(c->dseg_off, c->hitems.size());
        ALLOC(c->partial, 3 * c->hitems.size());
        ALLOC(c->lam_mu, (int64_t)run->max_windows * c->spr_total);
        ALLOC(c->ditem_begin, 2 * n_groups);
        HCOPY(c->dseg_off, seg_off.data(), seg_off.size() * sizeof(int64_t));
        std::vector<int32_t> ib(2 * n_groups);
        for (int i = 0; i < n_groups; ++i) { ib[2 * i] = c->item_begin[i]; ib[2 * i + 1] = c->item_count[i]; }
        HCOPY(c->ditem_begin, ib.data(), ib.size() * sizeof(int32_t));
    }
    HCOPY(c->dgroups, c->hgroups.data(), n_groups * sizeof(GroupDev));
    HCOPY(c->ditems, c->hitems.data(), c->hitems.size() * sizeof(Item));
    HCOPY(c->dtiles, c->htiles.data(), c->htiles.size() * sizeof(ColTile));
    HCOPY(c->dpar_off, par_off.data(), n_groups * sizeof(int64_t));
    {
        std::vector<int64_t> ro(n_groups + 1, 0);
        for (int i = 0; i < n_groups; ++i) ro[i + 1] = ro[i] + groups[i].n_replicas;
        c->n_reps = ro[n_groups];
        HCOPY(c->drep_off, ro.data(), ro.size() * sizeof(int64_t));
    }
    {
        const hipError_t e = hipMemset(c->src, 0, par * sizeof(double));
        if (e != hipSuccess) {
            ra_destroy(c);
            return fail(nullptr, RA_EDEVICE, std::string("hipMemset: ") + hipGetErrorString(e));
        }
    }
    {
        const hipError_t e = launch_reset(c->status, c->clamps, n_groups, c->dstep, c->stream);
        if (e != hipSuccess) {
            ra_destroy(c);
            return fail(nullptr, RA_EDEVICE, std::string("reset kernel: ") + hipGetErrorString(e));
        }
    }
#undef ALLOC
#undef HCOPY
    *out = c;
    return RA_OK;
}

extern "C" {

ra_status ra_init_chains(ra_ctx* c, const double* parent_xyz) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    if (!parent_xyz) return fail(c, RA_EINVAL, "parent_xyz is null");
    const int ng = (int)c->descs.size();
    // device-side resets are kernels ordered on the context's stream
    HIPCHK(c, launch_reset(c->status, c->clamps, ng, c->dstep, c->stream));
    const bool plain = c->run.plain != 0;
    c->cur = 0;
    HIPCHK(c, launch_clone(c->dgroups, ng, c->max_group_elems, parent_xyz, c->dpar_off,
                           plain ? c->pos[0] : c->state, c->tsf_acc, c->status, c->run.precision, plain,
                           c->stream));
    HIPCHK(c, launch_src_from_xyz(c->dgroups, ng, parent_xyz, c->dpar_off, c->src, c->stream));
    c->step = 0;
    c->initialised = true;
    c->recloned = false;
    return RA_OK;
}

static FwdArgs fwd_args(const ra_ctx* c) {
    FwdArgs a{};
    a.groups = c->dgroups;
    a.items = c->ditems;
    a.n_items = (int32_t)c->hitems.size();
    a.S = c->run.sample_every;
    a.K = c->run.checkpoint_every;
    a.key0 = (uint32_t)c->run.seed;
    a.key1 = (uint32_t)(c->run.seed >> 32);
    a.state = c->state;
    a.samples = c->samples;
    a.tsf = c->tsf;
    a.tsf_acc = c->tsf_acc;
    a.ckpt = c->ckpt;
    a.smp_total = c->smp_total;
    a.state_total = c->state_total;
    a.ckpt_total = c->ckpt_total;
    a.step0 = c->dstep;
    a.status = c->status;
    a.clamps = c->clamps;
    return a;
}

// Forward launches of n_steps on stream st (the context's own stream unless a
// caller orders it on another one), each followed by the step-counter advance.
static ra_status enqueue_forward(ra_ctx* c, int64_t n_steps, hipStream_t st) {
    FwdArgs a = fwd_args(c);
    // the kernel counts steps in 32-bit ints: split very long calls
    const int64_t chunk = (int64_t)1 << 30;
    for (int64_t done = 0; done < n_steps; done += chunk) {
        a.n_steps = std::min(chunk, n_steps - done);
        if (c->family == 2) HIPCHK(c, launch_forward_pair(a, c->run.precision, c->wpb, st));
        else if (c->family == 3) HIPCHK(c, launch_forward_hi(a, c->run.precision, c->hi_nmax, st));
        else HIPCHK(c, launch_forward(a, c->run.precision, c->family, c->wpb, c->run.noise_map, st));
        HIPCHK(c, launch_advance(c->dstep, a.n_steps, st));
    }
    return RA_OK;
}

static ra_status enqueue_forward(ra_ctx* c, int64_t n_steps) { return enqueue_forward(c, n_steps, c->stream); }

// n_a steps of context a and n_b steps of context b in one launch on a's
// stream (same kernel family, precision and waves per block), then both
// step-counter advances.
static ra_status enqueue_forward_dual(ra_ctx* ca, int64_t n_a, ra_ctx* cb, int64_t n_b) {
    FwdArgs a = fwd_args(ca), b = fwd_args(cb);
    a.n_steps = n_a;
    b.n_steps = n_b;
    hipStream_t st = ca->stream;
    if (ca->family == 2) HIPCHK(ca, launch_forward_pair_dual(a, b, ca->run.precision, ca->wpb, st));
    else if (ca->family == 3)
        HIPCHK(ca, launch_forward_hi_dual(a, b, ca->run.precision, std::max(ca->hi_nmax, cb->hi_nmax), st));
    else HIPCHK(ca, launch_forward_dual(a, b, ca->run.precision, ca->family, ca->wpb, ca->run.noise_map, st));
    HIPCHK(ca, launch_advance2(ca->dstep, n_a, cb->dstep, n_b, st));
    return RA_OK;
}

static ra_status enqueue_plain(ra_ctx* c, int64_t n_steps) {
    const int S = c->run.sample_every;
    const size_t esz = c->run.precision == 64 ? 8 : 4;
    const uint32_t k0 = (uint32_t)c->run.seed, k1 = (uint32_t)(c->run.seed >> 32);
    for (int64_t i = 0; i < n_steps; ++i) {
        const int64_t n = c->step + i;
        const bool window_end = ((n + 1) % S) == 0;
        const int64_t w = (n + 1) / S - 1;
        for (size_t g = 0; g < c->hgroups.size(); ++g) {
            const GroupDev& G = c->hgroups[g];
            HIPCHK(c, launch_plain_step(c->dgroups, (int)g, (int64_t)G.R * G.N, G.spring == 1, c->pos[c->cur],
                                        c->pos[1 - c->cur], c->status, (uint32_t)n, k0, k1, c->clamps,
                                        c->run.precision, c->stream));
        }
        c->cur = 1 - c->cur;
        if (window_end || c->run.tsf) {
            char* smp = (char*)c->samples + (window_end ? w : 0) * c->smp_total * esz;
            char* tsf = c->tsf ? (char*)c->tsf + (window_end ? w : 0) * c->smp_total * esz : nullptr;
            for (size_t g = 0; g < c->hgroups.size(); ++g) {
                const GroupDev& G = c->hgroups[g];
                HIPCHK(c, launch_plain_sample(c->dgroups, (int)g, (int64_t)G.R * (G.N - 1), G.spring == 1,
                                              c->pos[c->cur], smp, tsf, c->tsf_acc, window_end ? 1 : 0, S,
                                              c->status, c->run.precision, c->stream));
            }
        }
    }
    HIPCHK(c, launch_advance(c->dstep, n_steps, c->stream));
    return RA_OK;
}

ra_status ra_step(ra_ctx* c, int64_t n_steps) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    if (!c->initialised) return fail(c, RA_ESTATE, "ra_step before ra_init_chains");
    if (n_steps < 0) return fail(c, RA_EINVAL, "negative step count");
    if (n_steps == 0) return RA_OK;
    const int64_t end = c->step + n_steps;
    if (end > (int64_t)0xFFFFFFFF) return fail(c, RA_EINVAL, "total steps would exceed 2^32");
    if (end / c->run.sample_every > c->run.max_windows) return fail(c, RA_EINVAL, "window capacity exceeded");
    if (c->run.checkpoint_every > 0 && end > c->run.max_steps)
        return fail(c, RA_EINVAL, "checkpoint capacity (max_steps) exceeded");
    ra_status st;
    if (c->run.plain) {
        st = enqueue_plain(c, n_steps);
    } else if (c->run.use_graph) {
        auto it = c->graphs.find(n_steps);
        if (it == c->graphs.end()) {
            hipGraph_t graph;
            HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            st = enqueue_forward(c, n_steps);
            hipError_t e = hipStreamEndCapture(c->stream, &graph);
            if (st != RA_OK) {
                if (e == hipSuccess) (void)hipGraphDestroy(graph);
                return st;
            }
            HIPCHK(c, e);
            hipGraphExec_t exec;
            hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIPCHK(c, ei);
            it = c->graphs.emplace(n_steps, exec).first;
        }
        HIPCHK(c, hipGraphLaunch(it->second, c->stream));
        st = RA_OK;
    } else {
        st = enqueue_forward(c, n_steps);
    }
    if (st == RA_OK) c->step = end;
    return st;
}

ra_status ra_average_forces(ra_ctx* c, double* mean, double* stdv, double* tsf_mean, double* tsf_std,
                            int64_t* n_windows) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    if (!c->initialised) return fail(c, RA_ESTATE, "ra_average_forces before ra_init_chains");
    if ((tsf_mean || tsf_std) && !c->tsf) return fail(c, RA_ESTATE, "TSF output requested but tsf=0");
    const int64_t W = c->step / c->run.sample_every;
    if (n_windows) *n_windows = W;
    if (mean || stdv)
        HIPCHK(c, launch_reduce(c->dgroups, c->dtiles, (int)c->htiles.size(), W, c->samples, c->smp_total,
                                c->spr_total, mean, stdv, c->run.precision, c->stream));
    if (tsf_mean || tsf_std)
        HIPCHK(c, launch_reduce(c->dgroups, c->dtiles, (int)c->htiles.size(), W, c->tsf, c->smp_total,
                                c->spr_total, tsf_mean, tsf_std, c->run.precision, c->stream));
    return RA_OK;
}

ra_status ra_bell_rates(ra_ctx* c, const double* mean, int64_t n_windows, double k0, double x_dagger,
                        double* rates, double* rate_sum, uint8_t* events) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    if (!mean || n_windows < 0 || n_windows > c->run.max_windows)
        return fail(c, RA_EINVAL, "mean is null or n_windows out of range");
    if (!std::isfinite(k0) || !std::isfinite(x_dagger)) return fail(c, RA_EINVAL, "k0 and x_dagger must be finite");
    HIPCHK(c, launch_bell(c->dgroups, (int)c->hgroups.size(), n_windows, mean, c->spr_total, k0, x_dagger, rates,
                          rate_sum, events, c->run.sample_every, (uint32_t)c->run.seed,
                          (uint32_t)(c->run.seed >> 32), c->stream));
    return RA_OK;
}

ra_status ra_backward(ra_ctx* c, const double* mean, const double* grad_mean, const double* grad_rates,
                      double k0, double x_dagger, double* grad_params) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    if (c->run.checkpoint_every <= 0) return fail(c, RA_ESTATE, "ra_backward needs checkpoint_every > 0");
    if (!c->initialised) return fail(c, RA_ESTATE, "ra_backward before ra_init_chains");
    if (c->recloned) return fail(c, RA_ESTATE, "ra_backward does not differentiate through a re-clone");
    if (!grad_params) return fail(c, RA_EINVAL, "grad_params is null");
    if (grad_rates && !mean) return fail(c, RA_EINVAL, "grad_rates needs mean");
    const int ng = (int)c->hgroups.size();
    const int64_t W = c->step / c->run.sample_every;
    HIPCHK(c, launch_lam_mu(c->dgroups, ng, W, mean, grad_mean, grad_rates, k0, x_dagger, c->spr_total,
                            c->lam_mu, c->stream));
    AdjArgs a{};
    a.groups = c->dgroups;
    a.items = c->ditems;
    a.n_items = (int32_t)c->hitems.size();
    a.S = c->run.sample_every;
    a.K = c->run.checkpoint_every;
    a.key0 = (uint32_t)c->run.seed;
    a.key1 = (uint32_t)(c->run.seed >> 32);
    a.ckpt = c->ckpt;
    a.state_total = c->state_total;
    a.ckpt_total = c->ckpt_total;
    a.n_end = c->step;
    a.lam_mu = c->lam_mu;
    a.spr_total = c->spr_total;
    a.segbuf = c->segbuf;
    a.seg_off = c->dseg_off;
    a.partial = c->partial;
    // one launch per beads-per-lane value over its contiguous range of the work list
    for (size_t b = 0; b < c->hitems.size();) {
        const int M = c->hgroups[c->hitems[b].g].M;
        size_t e = b;
        while (e < c->hitems.size() && c->hgroups[c->hitems[e].g].M == M) ++e;
        HIPCHK(c, launch_adjoint(a, M, (int)b, (int)e, c->wpb, c->run.noise_map, c->stream));
        b = e;
    }
    HIPCHK(c, launch_grad_reduce(c->ditem_begin, ng, c->partial, grad_params, c->stream));
    return RA_OK;
}

// ---------------------------------------------------------------------------
// RSF cycle (Sec. II): re-clone from a parent context, the cycle driver, and
// the estimators built on the sampled windows.
// ---------------------------------------------------------------------------
static ra_status check_parent(ra_ctx* c, const ra_ctx* p) {
    if (!p) return fail(c, RA_EINVAL, "parent is null");
    if (p == c) return fail(c, RA_EINVAL, "parent must be another context");
    if (c->run.plain || p->run.plain) return fail(c, RA_EINVAL, "re-clone needs the fused path in both contexts");
    if (p->run.precision != c->run.precision) return fail(c, RA_EINVAL, "parent precision differs");
    if (p->descs.size() != c->descs.size()) return fail(c, RA_EINVAL, "parent has a different number of groups");
    for (size_t g = 0; g < c->descs.size(); ++g)
        if (p->descs[g].n_beads != c->descs[g].n_beads)
            return fail(c, RA_EINVAL, "parent group " + std::to_string(g) + " has a different chain length");
    if (!p->initialised) return fail(c, RA_ESTATE, "parent context not initialised");
    return RA_OK;
}

// The capacity checks of ra_step for n_steps more steps, without enqueuing.
static bool step_fits(const ra_ctx* c, int64_t n_steps, std::string& why) {
    const int64_t end = c->step + n_steps;
    if (end > (int64_t)0xFFFFFFFF) { why = "total steps would exceed 2^32"; return false; }
    if (end / c->run.sample_every > c->run.max_windows) { why = "window capacity exceeded"; return false; }
    if (c->run.checkpoint_every > 0 && end > c->run.max_steps) { why = "checkpoint capacity exceeded"; return false; }
    return true;
}

ra_status ra_reclone(ra_ctx* c, const ra_ctx* parent) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    ra_status st = check_parent(c, parent);
    if (st != RA_OK) return st;
    if (c->step % c->run.sample_every != 0)
        return fail(c, RA_EINVAL, "re-clone only at a window boundary (step count a multiple of S)");
    const int ng = (int)c->hgroups.size();
    // one launch: replica states, clone source, and the device step counter
    HIPCHK(c, launch_reclone(c->dgroups, parent->dgroups, ng, c->max_group_elems, parent->state, c->state, c->tsf_acc,
                             c->status, c->dpar_off, c->src, c->dstep, c->step, c->run.precision, c->stream));
    c->initialised = true;
    c->recloned = true;
    return RA_OK;
}

ra_status ra_rsf_cycle(ra_ctx* c, ra_ctx* parent, int64_t n_windows, int64_t parent_steps) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    ra_status st = check_parent(c, parent);
    if (st != RA_OK) return st;
    if (n_windows < 0 || parent_steps < 1) return fail(c, RA_EINVAL, "n_windows < 0 or parent_steps < 1");
    if (n_windows > (int64_t)0xFFFFFFFF || parent_steps > (int64_t)0xFFFFFFFF)
        return fail(c, RA_EINVAL, "total steps would exceed 2^32");
    if (parent->run.sample_every != parent_steps)
        return fail(c, RA_EINVAL, "the parent context must sample every parent_steps steps");
    const int S = c->run.sample_every;
    if (c->step % S != 0) return fail(c, RA_EINVAL, "the replicas are not at a window boundary");
    std::string why;
    if (!step_fits(parent, n_windows * parent_steps, why)) return fail(c, RA_EINVAL, "parent: " + why);
    if (!step_fits(c, n_windows * (int64_t)S, why)) return fail(c, RA_EINVAL, why);
    const bool two = parent->stream != c->stream;
    if (two && !c->ev_parent) {
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_parent, hipEventDisableTiming));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_reclone, hipEventDisableTiming));
    }
    // One-launch schedule: the parent's segment w+1 runs in the same launch as
    // the replicas' window w (fwd_dual_kernel and its pair/HI forms), all on
    // the replicas' stream, so the two overlap on any queue mapping.
    const bool dual = n_windows > 0 && c->family == parent->family && c->wpb == parent->wpb &&
                      c->run.noise_map == parent->run.noise_map &&
                      (c->family == 2 || c->family == 3 || c->family == 4 || c->family == 16) &&
                      S <= (1 << 30) && parent_steps <= (1 << 30);
    if (dual) {
        if (two) {   // the parent's queued work comes first
            HIPCHK(c, hipEventRecord(c->ev_parent, parent->stream));
            HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_parent, 0));
        }
        st = enqueue_forward(parent, parent_steps, c->stream);
        if (st != RA_OK) return fail(c, st, "parent: " + parent->err);
        parent->step += parent_steps;
        for (int64_t w = 0; w < n_windows; ++w) {
            st = ra_reclone(c, parent);
            if (st != RA_OK) return st;
            const bool both = w + 1 < n_windows;
            st = both ? enqueue_forward_dual(c, S, parent, parent_steps) : enqueue_forward(c, S);
            if (st != RA_OK) return st;
            if (both) parent->step += parent_steps;
            c->step += S;
        }
        if (two) {   // later parent work waits for the cycle
            HIPCHK(c, hipEventRecord(c->ev_reclone, c->stream));
            HIPCHK(c, hipStreamWaitEvent(parent->stream, c->ev_reclone, 0));
        }
        return RA_OK;
    }
    for (int64_t w = 0; w < n_windows; ++w) {
        // the parent's next window may start once the last re-clone has read its state
        if (two && w > 0) HIPCHK(c, hipStreamWaitEvent(parent->stream, c->ev_reclone, 0));
        st = ra_step(parent, parent_steps);
        if (st != RA_OK) return fail(c, st, "parent: " + parent->err);
        if (two) {
            HIPCHK(c, hipEventRecord(c->ev_parent, parent->stream));
            HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_parent, 0));
        }
        st = ra_reclone(c, parent);
        if (st != RA_OK) return st;
        if (two) HIPCHK(c, hipEventRecord(c->ev_reclone, c->stream));
        st = ra_step(c, S);
        if (st != RA_OK) return st;
    }
    // later work on the parent's stream must not overwrite the state before the last re-clone read it
    if (two && n_windows > 0) HIPCHK(c, hipStreamWaitEvent(parent->stream, c->ev_reclone, 0));
    return RA_OK;
}

ra_status ra_block_sigma(ra_ctx* c, int32_t block, double* sigma) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    if (!sigma || block < 1) return fail(c, RA_EINVAL, "sigma is null or block < 1");
    if (!c->initialised) return fail(c, RA_ESTATE, "ra_block_sigma before ra_init_chains");
    const int64_t W = c->step / c->run.sample_every;
    HIPCHK(c, launch_block_sigma(c->dgroups, c->dtiles, (int)c->htiles.size(), W, c->samples, c->smp_total,
                                 c->spr_total, block, sigma, c->run.precision, c->stream));
    return RA_OK;
}

ra_status ra_mftu(ra_ctx* c, const double* rate_sum, int64_t n_windows, double* mftu) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    if (!rate_sum || !mftu || n_windows < 1) return fail(c, RA_EINVAL, "null argument or n_windows < 1");
    HIPCHK(c, launch_mftu(rate_sum, n_windows, (int)c->hgroups.size(), mftu, c->stream));
    return RA_OK;
}

ra_status ra_mftu_events(ra_ctx* c, const double* rates, int64_t n_windows, int32_t n_trials, int64_t max_windows,
                         int64_t* first_window, double* mftu) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    if (!rates || !first_window || !mftu) return fail(c, RA_EINVAL, "null argument");
    if (n_windows < 1 || n_trials < 1 || n_trials > 65535 || max_windows < 1 || max_windows > (int64_t)0xFFFFFFFF)
        return fail(c, RA_EINVAL, "need n_windows >= 1, 1 <= n_trials <= 65535, 1 <= max_windows < 2^32");
    const int ng = (int)c->hgroups.size();
    if (ng > 65535) return fail(c, RA_EINVAL, "more than 65535 groups");
    int max_springs = 1;
    for (const auto& g : c->hgroups) max_springs = std::max(max_springs, g.N - 1);
    HIPCHK(c, launch_mftu_events(c->dgroups, ng, rates, n_windows, c->spr_total, n_trials, max_windows,
                                 c->run.sample_every, (uint32_t)c->run.seed, (uint32_t)(c->run.seed >> 32),
                                 max_springs, first_window, mftu, c->stream));
    return RA_OK;
}

ra_status ra_conformation(ra_ctx* c, double* dbar, double* d_bead, double* rg2, double* src_rg2) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    if (c->run.plain) return fail(c, RA_EINVAL, "ra_conformation needs the fused path");
    if (!c->initialised) return fail(c, RA_ESTATE, "ra_conformation before ra_init_chains");
    HIPCHK(c, launch_conformation(c->dgroups, (int)c->hgroups.size(), c->drep_off, c->n_reps, c->state, c->dpar_off,
                                  c->src, dbar, d_bead, rg2, src_rg2, c->run.precision, c->stream));
    return RA_OK;
}

ra_status ra_sync_status(ra_ctx* c) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    int32_t s = 0;
    HIPCHK(c, hipMemcpy(&s, c->status, sizeof s, hipMemcpyDeviceToHost));
    if (s & 1) return fail(c, RA_EINVAL, "invalid parent chain: FENE bond at or beyond Q0, or non-finite coordinate");
    if (s & 2) return fail(c, RA_EUNSTABLE, "non-finite tension sampled");
    if (s & 4) return fail(c, RA_EUNSTABLE, "non-positive pivot in the Cholesky factorization of the RPY tensor");
    return RA_OK;
}

ra_status ra_guard_counts(ra_ctx* c, int64_t* out) {
    if (!c || !out) return fail(c, RA_EINVAL, "null argument");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<unsigned long long> v(c->hgroups.size());
    HIPCHK(c, hipMemcpy(v.data(), c->clamps, v.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < v.size(); ++i) out[i] = (int64_t)v[i];
    return RA_OK;
}

ra_status ra_get_samples(ra_ctx* c, double* out, double* tsf_out) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    if (tsf_out && !c->tsf) return fail(c, RA_ESTATE, "tsf=0");
    const int64_t W = c->step / c->run.sample_every;
    if (out) HIPCHK(c, launch_to_f64(c->samples, out, W * c->smp_total, c->run.precision, c->stream));
    if (tsf_out) HIPCHK(c, launch_to_f64(c->tsf, tsf_out, W * c->smp_total, c->run.precision, c->stream));
    return RA_OK;
}

ra_status ra_get_bonds(ra_ctx* c, double* out) {
    if (!c || !out) return fail(c, RA_EINVAL, "null argument");
    if (c->run.plain)
        HIPCHK(c, launch_pos_to_bonds(c->dgroups, (int)c->hgroups.size(), c->max_group_elems, c->pos[c->cur], out,
                                      c->run.precision, c->stream));
    else
        HIPCHK(c, launch_to_f64(c->state, out, c->state_total, c->run.precision, c->stream));
    return RA_OK;
}

ra_status ra_checkpoint_interval(ra_ctx* c, int32_t* steps) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    if (!steps) return fail(c, RA_EINVAL, "steps is null");
    *steps = c->run.checkpoint_every;
    return RA_OK;
}

ra_status ra_tile_info(ra_ctx* c, int32_t* beads_per_lane, int32_t* replicas_per_wave, int32_t* kernel_family) {
    if (!c) return fail(nullptr, RA_EINVAL, "null context");
    if (kernel_family) *kernel_family = c->run.plain ? 0 : c->family;
    for (size_t i = 0; i < c->hgroups.size(); ++i) {
        if (beads_per_lane) beads_per_lane[i] = c->hgroups[i].M;
        if (replicas_per_wave) replicas_per_wave[i] = c->hgroups[i].P;
    }
    return RA_OK;
}

ra_status ra_debug_noise(const uint32_t* counters, int64_t n, uint64_t seed, uint32_t* words, float* normals32,
                         double* normals64, void* hip_stream) {
    if (n < 0 || (n > 0 && !counters)) return fail(nullptr, RA_EINVAL, "bad counters");
    hipError_t e = launch_debug_noise(counters, n, (uint32_t)seed, (uint32_t)(seed >> 32), words, normals32,
                                      normals64, (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(nullptr, RA_EDEVICE, hipGetErrorString(e));
    return RA_OK;
}

}  // extern "C"
