// ra_tune.cpp — cost-model and timing autotuner for the per-group tile.
#include "ra_tune.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <sstream>
#include <fstream>
#include <tuple>

namespace ra {

const std::vector<int>& family_beads_per_lane(int family) {
    static const std::vector<int> small{1, 2, 3, 4};
    static const std::vector<int> large{6, 8, 12, 16};
    return family == 4 ? small : large;
}

static bool legal(int n_beads, int M) { return (n_beads + M - 1) / M <= 64; }

int choose_beads_per_lane(int n_beads, int n_replicas, int family, int forced) {
    const auto& cand = family_beads_per_lane(family);
    if (forced > 0 && legal(n_beads, forced))
        for (int m : cand)
            if (m == forced) return m;
    int best = -1;
    long long best_cost = 0;
    for (int M : cand) {
        if (!legal(n_beads, M)) continue;
        const int L = (n_beads + M - 1) / M;
        const int P = 64 / L;
        const long long cost = (long long)M * ((n_replicas + P - 1) / P);
        if (best < 0 || cost < best_cost) { best = M; best_cost = cost; }
    }
    return best < 0 ? cand.back() : best;
}

namespace {

using Key = std::tuple<int, int, int, int, int>;   // N, spring, precision, family, wpb
constexpr int TUNE_WAVES_PER_SIMD = 4;             // timing runs fill every SIMD this many times
std::mutex g_mu;
std::map<Key, int> g_cache;
bool g_loaded = false;

void load_cache_file() {
    if (g_loaded) return;
    g_loaded = true;
    const char* path = std::getenv("RA_AUTOTUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    if (!f) return;
    // one entry per line: {"N": .., "spring": .., "precision": .., "family": .., "wpb": .., "M": ..}
    std::string line;
    while (std::getline(f, line)) {
        int v[6];
        if (std::sscanf(line.c_str(),
                        " {\"N\": %d, \"spring\": %d, \"precision\": %d, \"family\": %d, \"wpb\": %d, \"M\": %d}",
                        &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) == 6)
            g_cache[Key{v[0], v[1], v[2], v[3], v[4]}] = v[5];
    }
}

void append_cache_file(const Key& k, int M) {
    const char* path = std::getenv("RA_AUTOTUNE_CACHE");
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << "{\"N\": " << std::get<0>(k) << ", \"spring\": " << std::get<1>(k) << ", \"precision\": "
      << std::get<2>(k) << ", \"family\": " << std::get<3>(k) << ", \"wpb\": " << std::get<4>(k)
      << ", \"M\": " << M << "}\n";
}

// Time 96 fused steps of one group with a forced tile M and enough replicas
// to give every SIMD TUNE_WAVES_PER_SIMD wavefronts of that packing, so the
// candidates are ranked by throughput (as in a saturated batch), not by the
// latency of a few wavefronts. Returns ms per replica, or -1.
double time_tile(const ra_chain_desc& d, const ra_run_desc& run, int M, int wpb, hipStream_t st) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    const int lanes = (d.n_beads + M - 1) / M;
    const int per_wave = std::max(1, 64 / lanes);
    ra_chain_desc g = d;
    g.n_replicas = TUNE_WAVES_PER_SIMD * 4 * cus * per_wave;
    ra_run_desc r{};
    r.seed = run.seed;
    r.precision = run.precision;
    r.sample_every = 64;
    r.max_windows = 2;
    r.tile_policy = 1000 + M;
    r.waves_per_block = wpb;
    r.noise_map = run.noise_map;
    ra_ctx* ctx = nullptr;
    if (ra_create(&ctx, &g, 1, &r, st) != RA_OK) return -1.0;
    // straight parent along x with unit bonds (inside any FENE extension b >= 2)
    std::vector<double> parent(3 * (size_t)d.n_beads, 0.0);
    for (int i = 0; i < d.n_beads; ++i) parent[3 * i] = 0.5 * i;
    double* dp = nullptr;
    double ms = -1.0;
    hipEvent_t e0, e1;
    if (hipMalloc((void**)&dp, parent.size() * sizeof(double)) == hipSuccess &&
        hipMemcpy(dp, parent.data(), parent.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
        hipEventCreate(&e0) == hipSuccess) {
        if (hipEventCreate(&e1) == hipSuccess) {
            if (ra_init_chains(ctx, dp) == RA_OK && ra_step(ctx, 32) == RA_OK) {
                (void)hipEventRecord(e0, st);
                if (ra_step(ctx, 96) == RA_OK) {
                    (void)hipEventRecord(e1, st);
                    if (hipEventSynchronize(e1) == hipSuccess) {
                        float t = 0.f;
                        (void)hipEventElapsedTime(&t, e0, e1);
                        ms = t / g.n_replicas;
                    }
                }
            }
            (void)hipEventDestroy(e1);
        }
        (void)hipEventDestroy(e0);
    }
    // a timing probe: failures above leave ms < 0 and the candidate unused
    (void)hipStreamSynchronize(st);
    if (dp) (void)hipFree(dp);
    ra_destroy(ctx);
    return ms;
}

}  // namespace

ra_status autotune_tiles(const std::vector<ra_chain_desc>& descs, const ra_run_desc& run, int family,
                         int waves_per_block, hipStream_t stream, std::vector<int>& Ms, std::string& why) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_file();
    for (size_t i = 0; i < descs.size(); ++i) {
        const ra_chain_desc& d = descs[i];
        const Key k{d.n_beads, d.spring, run.precision, family, waves_per_block};
        auto it = g_cache.find(k);
        if (it != g_cache.end()) { Ms[i] = it->second; continue; }
        double best_ms = -1.0;
        int best = Ms[i];
        for (int M : family_beads_per_lane(family)) {
            if (!legal(d.n_beads, M)) continue;
            const double ms = time_tile(d, run, M, waves_per_block, stream);   // per replica
            if (ms < 0) { why = "timing run failed"; return RA_EDEVICE; }
            if (best_ms < 0 || ms < best_ms) { best_ms = ms; best = M; }
        }
        Ms[i] = best;
        g_cache[k] = best;
        append_cache_file(k, best);
    }
    return RA_OK;
}

}  // namespace ra
