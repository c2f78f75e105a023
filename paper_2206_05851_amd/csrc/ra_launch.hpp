// ra_launch.hpp — kernel argument blocks and host launchers (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>

#include <string>

#include "ra.h"
#include "ra_types.hpp"

namespace ra {

// Host-side helpers shared by the entry points (ra_host.cpp).
// Validates descriptors and run options as ra_create does (RA_EINVAL + text).
ra_status validate(const ra_chain_desc* g, int32_t n, const ra_run_desc* r, std::string& why);
// Per-group device constants for beads-per-lane M, counter tag and noise map.
GroupDev make_group(const ra_chain_desc& d, int M, int tag, int nmap);
// Text returned by ra_last_error(NULL) on this thread.
void set_global_error(const std::string& msg);
// ra_create, with force_family = 16 selecting the 6-16 beads-per-lane kernels
// (FP32 fused path) even when every chain has at most 256 beads; 0 chooses as
// ra_create does. The autotuner times one group of a wide-lane batch this way,
// so the probe runs the kernels the batch will run.
ra_status create_context(ra_ctx** out, const ra_chain_desc* groups, int32_t n_groups, const ra_run_desc* run,
                         void* hip_stream, int force_family);

struct FwdArgs {
    const GroupDev* groups;
    const Item* items;
    int32_t n_items;
    int32_t S;                 // sample every S steps
    int32_t K;                 // checkpoint every K steps (0: none)
    uint32_t key0, key1;       // Philox key = seed
    void* state;               // bond state, T[state_total]
    void* samples;             // T[max_windows][smp_total]
    void* tsf;                 // T[max_windows][smp_total] or nullptr
    double* tsf_acc;           // running window sums [smp_total] or nullptr
    void* ckpt;                // T[n_ckpt][ckpt_total] or nullptr (per item: [M][3][lanes used])
    int64_t smp_total;         // sample elements per window
    int64_t state_total;       // bond-state elements
    int64_t ckpt_total;        // elements per checkpoint
    const int64_t* step0;      // device: steps since init before this launch
    int64_t n_steps;
    int32_t* status;           // bit 0: invalid parent, bit 1: non-finite tension
    unsigned long long* clamps;
};

struct AdjArgs {
    const GroupDev* groups;
    const Item* items;
    int32_t n_items;
    int32_t S, K;
    uint32_t key0, key1;
    const void* ckpt;          // forward checkpoints T[n_ckpt][ckpt_total]
    int64_t state_total;
    int64_t ckpt_total;
    int64_t n_end;             // steps since init covered by the adjoint
    const double* lam_mu;      // dJ/d mean [W][spr_total]
    int64_t spr_total;
    float* segbuf;             // per item: K states of the wave's lanes
    const int64_t* seg_off;    // per item offset into segbuf (floats)
    double* partial;           // per item [3]: d/d(rate, H, b)
};

// nmap: noise map of the context (1 selects the kernels compiled for map 1)
hipError_t launch_forward(const FwdArgs& a, int precision, int family, int waves_per_block, int nmap,
                          hipStream_t st);
hipError_t launch_advance(int64_t* step, int64_t n, hipStream_t st);
hipError_t launch_reset(int32_t* status, unsigned long long* clamps, int n_groups, int64_t* step, hipStream_t st);
hipError_t launch_clone(const GroupDev* groups, int n_groups, int64_t max_elems, const double* parent,
                        const int64_t* par_off, void* state, double* tsf_acc, int32_t* status, int precision,
                        bool plain, hipStream_t st);
hipError_t launch_plain_step(const GroupDev* groups, int g, int64_t n_threads, bool fene, const void* rin,
                             void* rout, const int32_t* status, uint32_t n, uint32_t key0, uint32_t key1,
                             unsigned long long* clamps, int precision, hipStream_t st);
hipError_t launch_plain_sample(const GroupDev* groups, int g, int64_t n_threads, bool fene, const void* pos,
                               void* samples_w, void* tsf_w, double* tsf_acc, int window_end, int S,
                               int32_t* status, int precision, hipStream_t st);
hipError_t launch_reduce(const GroupDev* groups, const ColTile* tiles, int n_tiles, int64_t n_windows,
                         const void* smp, int64_t smp_total, int64_t spr_total, double* mean, double* stdv,
                         int precision, hipStream_t st);
hipError_t launch_bell(const GroupDev* groups, int n_groups, int64_t n_windows, const double* mean,
                       int64_t spr_total, double k0, double xd, double* rates, double* rate_sum,
                       uint8_t* events, int S, uint32_t key0, uint32_t key1, hipStream_t st);
hipError_t launch_to_f64(const void* src, double* dst, int64_t n, int precision, hipStream_t st);
hipError_t launch_pos_to_bonds(const GroupDev* groups, int n_groups, int64_t max_elems, const void* pos,
                               double* out, int precision, hipStream_t st);
hipError_t launch_debug_noise(const uint32_t* ctr, int64_t n, uint32_t key0, uint32_t key1, uint32_t* words,
                              float* n32, double* n64, hipStream_t st);
hipError_t launch_adjoint(const AdjArgs& a, int M, int item_begin, int item_end, int waves_per_block, int nmap,
                          hipStream_t st);
hipError_t launch_lam_mu(const GroupDev* groups, int n_groups, int64_t n_windows, const double* mean,
                         const double* grad_mean, const double* grad_rates, double k0, double xd,
                         int64_t spr_total, double* lam_mu, hipStream_t st);
hipError_t launch_grad_reduce(const int32_t* item_begin, int n_groups, const double* partial,
                              double* grad_params, hipStream_t st);

// pair-interaction (collapsed-polymer) forward kernel (ra_pair.hip)
hipError_t launch_forward_pair(const FwdArgs& a, int precision, int waves_per_block, hipStream_t st);
// two contexts (same kernel family) in one launch: blocks of a first, then b
hipError_t launch_forward_dual(const FwdArgs& a, const FwdArgs& b, int precision, int family, int waves_per_block,
                               int nmap, hipStream_t st);
hipError_t launch_forward_pair_dual(const FwdArgs& a, const FwdArgs& b, int precision, int waves_per_block,
                                    hipStream_t st);
hipError_t launch_forward_hi_dual(const FwdArgs& a, const FwdArgs& b, int precision, int max_beads, hipStream_t st);

// hydrodynamic-interaction forward kernel (ra_hi.hip)
size_t hi_lds_bytes(int max_beads, int precision);
hipError_t launch_forward_hi(const FwdArgs& a, int precision, int max_beads, hipStream_t st);

// RSF cycle and estimators (ra_rsf.hip)
hipError_t launch_reclone(const GroupDev* groups, const GroupDev* pgroups, int n_groups, int64_t max_elems,
                          const void* pstate, void* state, double* tsf_acc, int32_t* status, const int64_t* par_off,
                          double* src, int64_t* step, int64_t step_value, int precision, hipStream_t st);
hipError_t launch_advance2(int64_t* a, int64_t na, int64_t* b, int64_t nb, hipStream_t st);
hipError_t launch_src_from_xyz(const GroupDev* groups, int n_groups, const double* parent, const int64_t* par_off,
                               double* src, hipStream_t st);
hipError_t launch_conformation(const GroupDev* groups, int n_groups, const int64_t* rep_off, int64_t n_reps,
                               const void* state, const int64_t* par_off, const double* src, double* dbar,
                               double* d_bead, double* rg2, double* src_rg2, int precision, hipStream_t st);
hipError_t launch_block_sigma(const GroupDev* groups, const ColTile* tiles, int n_tiles, int64_t n_windows,
                              const void* smp, int64_t smp_total, int64_t spr_total, int block, double* sigma,
                              int precision, hipStream_t st);
hipError_t launch_mftu(const double* rate_sum, int64_t n_windows, int n_groups, double* mftu, hipStream_t st);
hipError_t launch_mftu_events(const GroupDev* groups, int n_groups, const double* rates, int64_t n_windows,
                              int64_t spr_total, int n_trials, int64_t max_windows, int S, uint32_t key0,
                              uint32_t key1, int max_springs, int64_t* first_window, double* mftu, hipStream_t st);

}  // namespace ra
