// ra_static.hip — the allocation-free entry point ra_run_static: one chain
// group's RSF clone, Euler-Maruyama steps and replica averages (Sec. II) with
// every scratch buffer (descriptors, counters, bond state, per-replica
// samples) in a file-scope device array instead of library allocations.
// It runs the same kernels as the context path, so its results are
// bit-identical to ra_create + ra_init_chains + ra_step + ra_average_forces.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>
#include <string>

#include "ra.h"
#include "ra_launch.hpp"
#include "ra_tune.hpp"
#include "ra_types.hpp"

namespace ra {

constexpr size_t STATIC_SCRATCH_BYTES = (size_t)64 << 20;
static_assert(STATIC_SCRATCH_BYTES == (size_t)RA_STATIC_SCRATCH_MAX, "ra.h states the scratch size");

// Each device holds its own copy of this array for the life of the process.
// Host code never uses the name as an address: the per-device address comes
// from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per device.
hipError_t scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// Clears the call's counters (status, guard count, step) and writes the
// group descriptor, the work list (wavefront i: replicas [i P, i P + P)) and
// the reduction's column tiles into the scratch array: the previous call's
// contents are never read.
__global__ void static_setup_kernel(GroupDev G, GroupDev* groups, Item* items, int n_items, ColTile* tiles,
                                    int n_tiles, int32_t* status, unsigned long long* clamps, int64_t* step,
                                    int64_t* par_off) {
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int stride = (int)(gridDim.x * blockDim.x);
    if (t == 0) {
        groups[0] = G;
        *status = 0;
        *clamps = 0ull;
        *step = 0;
        par_off[0] = 0;
    }
    for (int i = t; i < n_items; i += stride) items[i] = Item{0, i * G.P};
    for (int i = t; i < n_tiles; i += stride) tiles[i] = ColTile{0, i * WAVE};
}

// An invalid parent (no steps were run) or a non-finite tension: every output
// element becomes NaN, the in-band error of this entry point.
__global__ void static_poison_kernel(const int32_t* status, double* mean, double* stdv, int64_t n) {
    if (*(const volatile int32_t*)status == 0) return;
    const double nan = __builtin_nan("");
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        if (mean) mean[e] = nan;
        if (stdv) stdv[e] = nan;
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

ra_status fail_static(ra_status code, const std::string& msg) {
    set_global_error(msg);
    return code;
}

}  // namespace
}  // namespace ra

using namespace ra;

extern "C" ra_status ra_run_static(const ra_chain_desc* group, const ra_run_desc* run, const double* parent_xyz,
                                   int64_t n_steps, double* mean, double* stdv, void* hip_stream) {
    if (!group || !run || !parent_xyz) return fail_static(RA_EINVAL, "ra_run_static: null argument");
    if (!mean && !stdv) return fail_static(RA_EINVAL, "ra_run_static: no output");
    std::string why;
    if (validate(group, 1, run, why) != RA_OK) return fail_static(RA_EINVAL, "ra_run_static: " + why);
    const ra_chain_desc& d = *group;
    if (d.spring == RA_HARMONIC || d.lj_eps > 0.0 || d.hi_radius > 0.0)
        return fail_static(RA_EINVAL, "ra_run_static: chain model only (Hookean or FENE, no LJ, no HI)");
    if (run->plain || run->tsf || run->checkpoint_every != 0 || run->use_graph || run->tile_policy == 1 ||
        run->noise_tag != 0)
        return fail_static(RA_EINVAL, "ra_run_static: fused path without TSF, checkpoints, graph, autotuning "
                                      "or parent noise tag");
    const int S = run->sample_every;
    if (n_steps < 1 || n_steps > (int64_t)0xFFFFFFFF || n_steps % S != 0)
        return fail_static(RA_EINVAL, "ra_run_static: n_steps must be a positive multiple of sample_every below 2^32");
    const int64_t W = n_steps / S;
    if (W > 65535) return fail_static(RA_EINVAL, "ra_run_static: more than 65535 windows");

    const int family = (d.n_beads > 4 * WAVE && run->precision == 32) ? 16 : 4;
    if (run->noise_map == 1 && family != 4)
        return fail_static(RA_EINVAL, "ra_run_static: noise_map 1 needs n_beads <= 256");
    if (run->noise_map == 2 && family != 16)
        return fail_static(RA_EINVAL, "ra_run_static: noise_map 2 needs n_beads > 256 at precision 32");
    const int forced = run->tile_policy > 1000 ? run->tile_policy - 1000 : 0;
    const int M = choose_beads_per_lane(d.n_beads, d.n_replicas, family, forced, run->noise_map);
    GroupDev G = make_group(d, M, 0, run->noise_map);
    const int64_t nm1 = d.n_beads - 1;
    G.state_off = 0;
    G.smp_off = 0;
    G.spr_off = 0;
    G.pos_off = 0;
    const int n_items = (d.n_replicas + G.P - 1) / G.P;
    const int n_tiles = (int)((nm1 + WAVE - 1) / WAVE);
    const size_t esz = run->precision == 64 ? 8 : 4;
    const int64_t state_total = (int64_t)d.n_replicas * nm1 * 3;
    const int64_t smp_total = (int64_t)d.n_replicas * nm1;

    // scratch layout, every part on a 256-byte boundary
    size_t off = 0;
    const size_t o_groups = off;  off = align256(off + sizeof(GroupDev));
    const size_t o_items = off;   off = align256(off + sizeof(Item) * (size_t)n_items);
    const size_t o_tiles = off;   off = align256(off + sizeof(ColTile) * (size_t)n_tiles);
    const size_t o_status = off;  off = align256(off + sizeof(int32_t));
    const size_t o_clamps = off;  off = align256(off + sizeof(unsigned long long));
    const size_t o_step = off;    off = align256(off + sizeof(int64_t));
    const size_t o_paroff = off;  off = align256(off + sizeof(int64_t));
    const size_t o_state = off;   off = align256(off + esz * (size_t)state_total);
    const size_t o_smp = off;
    const double smp_bytes = (double)esz * (double)smp_total * (double)W;
    if ((double)off + smp_bytes > (double)STATIC_SCRATCH_BYTES) {
        char b[200];
        std::snprintf(b, sizeof b, "ra_run_static: needs %.0f bytes of scratch (state, samples, descriptors); "
                      "the limit is %zu", (double)off + smp_bytes, STATIC_SCRATCH_BYTES);
        return fail_static(RA_EINVAL, b);
    }

    void* base_v = nullptr;
    hipError_t e = scratch_address(&base_v);
    if (e != hipSuccess) return fail_static(RA_EDEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    unsigned char* base = (unsigned char*)base_v;
    GroupDev* groups = (GroupDev*)(base + o_groups);
    Item* items = (Item*)(base + o_items);
    ColTile* tiles = (ColTile*)(base + o_tiles);
    int32_t* status = (int32_t*)(base + o_status);
    unsigned long long* clamps = (unsigned long long*)(base + o_clamps);
    int64_t* step = (int64_t*)(base + o_step);
    int64_t* par_off = (int64_t*)(base + o_paroff);
    void* state = base + o_state;
    void* samples = base + o_smp;
    hipStream_t st = (hipStream_t)hip_stream;

#define SCHK(expr)                                                                                   \
    do {                                                                                             \
        const hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail_static(RA_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)
    (void)hipGetLastError();   // report only this call's own errors
    const int setup_blocks = std::min(1024, std::max(1, (n_items + 255) / 256));
    hipLaunchKernelGGL(static_setup_kernel, dim3(setup_blocks), dim3(256), 0, st, G, groups, items, n_items, tiles,
                       n_tiles, status, clamps, step, par_off);
    SCHK(hipGetLastError());
    SCHK(launch_clone(groups, 1, (int64_t)d.n_replicas * d.n_beads * 3, parent_xyz, par_off, state, nullptr, status,
                      run->precision, false, st));
    FwdArgs a{};
    a.groups = groups;
    a.items = items;
    a.n_items = n_items;
    a.S = S;
    a.K = 0;
    a.key0 = (uint32_t)run->seed;
    a.key1 = (uint32_t)(run->seed >> 32);
    a.state = state;
    a.samples = samples;
    a.smp_total = smp_total;
    a.state_total = state_total;
    a.step0 = step;
    a.status = status;
    a.clamps = clamps;
    const int wpb = run->waves_per_block ? run->waves_per_block : 4;
    const int64_t chunk = (int64_t)1 << 30;   // the kernel counts steps in 32-bit ints
    for (int64_t done = 0; done < n_steps; done += chunk) {
        a.n_steps = std::min(chunk, n_steps - done);
        SCHK(launch_forward(a, run->precision, family, wpb, run->noise_map, st));
        SCHK(launch_advance(step, a.n_steps, st));
    }
    SCHK(launch_reduce(groups, tiles, n_tiles, W, samples, smp_total, nm1, mean, stdv, run->precision, st));
    const int64_t n_out = W * nm1;
    hipLaunchKernelGGL(static_poison_kernel, dim3((unsigned)std::min<int64_t>((n_out + 255) / 256, 1024)), dim3(256),
                       0, st, status, mean, stdv, n_out);
    SCHK(hipGetLastError());
#undef SCHK
    return RA_OK;
}
