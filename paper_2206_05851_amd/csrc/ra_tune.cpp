// ra_tune.cpp — cost-model and timing autotuner for the per-group tile and
// the launch's wavefronts per workgroup.
#include "ra_tune.hpp"

#include "ra_launch.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <tuple>

namespace ra {

const std::vector<int>& family_beads_per_lane(int family) {
    static const std::vector<int> small{1, 2, 3, 4};
    static const std::vector<int> large{6, 8, 12, 16};
    return family == 4 ? small : large;
}

static bool legal(int n_beads, int M) { return (n_beads + M - 1) / M <= 64; }

bool map_allows(int nmap, int M) { return nmap != 2 || M % 4 == 0; }

int choose_beads_per_lane(int n_beads, int n_replicas, int family, int forced, int nmap) {
    const auto& cand = family_beads_per_lane(family);
    if (forced > 0 && legal(n_beads, forced) && map_allows(nmap, forced))
        for (int m : cand)
            if (m == forced) return m;
    int best = -1;
    long long best_cost = 0;
    for (int M : cand) {
        if (!legal(n_beads, M) || !map_allows(nmap, M)) continue;
        const int L = (n_beads + M - 1) / M;
        const int P = 64 / L;
        const long long cost = (long long)M * ((n_replicas + P - 1) / P);
        if (best < 0 || cost < best_cost) { best = M; best_cost = cost; }
    }
    return best < 0 ? cand.back() : best;
}

namespace {

// One tuning result: the fastest M for a chain length and spring law under a
// precision, kernel family, wavefronts per workgroup and noise map, and its
// time per replica for 96 steps (to compare workgroup sizes across a batch).
using Key = std::tuple<int, int, int, int, int, int>;   // N, spring, precision, family, wpb, noise_map
struct Entry {
    int M;
    double ms_per_replica;
};
constexpr int TUNE_WAVES_PER_SIMD = 4;             // timing runs fill every SIMD this many times

// The process keeps one table of results per cache file (the empty path when
// RA_AUTOTUNE_CACHE is unset): the library's only process-wide state. Tuning
// results depend on the device model and the library build, not on a
// context, so contexts with the same groups share them.
std::mutex g_mu;
std::map<std::string, std::map<Key, Entry>> g_tables;

std::map<Key, Entry>& table_for(const std::string& path) {
    auto it = g_tables.find(path);
    if (it != g_tables.end()) return it->second;
    std::map<Key, Entry>& t = g_tables[path];
    if (path.empty()) return t;
    std::ifstream f(path);
    // one entry per line: {"N": .., "spring": .., "precision": .., "family": .., "wpb": ..,
    //                      "noise_map": .., "M": .., "ms_per_replica": ..}
    std::string line;
    while (f && std::getline(f, line)) {
        int v[7];
        double ms = 0.0;
        if (std::sscanf(line.c_str(),
                        " {\"N\": %d, \"spring\": %d, \"precision\": %d, \"family\": %d, \"wpb\": %d, "
                        "\"noise_map\": %d, \"M\": %d, \"ms_per_replica\": %lf}",
                        &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6], &ms) == 8)
            t[Key{v[0], v[1], v[2], v[3], v[4], v[5]}] = Entry{v[6], ms};
    }
    return t;
}

void append_cache_file(const std::string& path, const Key& k, const Entry& e) {
    if (path.empty()) return;
    std::ofstream f(path, std::ios::app);
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "{\"N\": %d, \"spring\": %d, \"precision\": %d, \"family\": %d, \"wpb\": %d, "
                  "\"noise_map\": %d, \"M\": %d, \"ms_per_replica\": %.9g}\n",
                  std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
                  std::get<5>(k), e.M, e.ms_per_replica);
    f << buf;
}

// Time 96 fused steps of one group with a forced tile M of the batch's kernel
// family (a short chain in a wide-lane batch runs the wide-lane kernels) and enough replicas
// to give every SIMD TUNE_WAVES_PER_SIMD wavefronts of that packing, so the
// candidates are ranked by throughput (as in a saturated batch), not by the
// latency of a few wavefronts. Returns ms per replica, or -1.
double time_tile(const ra_chain_desc& d, const ra_run_desc& run, int family, int M, int wpb, hipStream_t st) {
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
    if (create_context(&ctx, &g, 1, &r, st, family) != RA_OK) return -1.0;
    // straight parent along x; its bonds stay inside the FENE extension
    // (half of Q0 = sqrt(b kT/H), at most 0.5), so the timed kernel does the
    // work of a valid chain
    double bond = 0.5;
    if (d.spring == RA_FENE) bond = std::min(0.5, 0.5 * std::sqrt(d.b * d.kT / d.H));
    std::vector<double> parent(3 * (size_t)d.n_beads, 0.0);
    for (int i = 0; i < d.n_beads; ++i) parent[3 * i] = bond * i;
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
    // a timing probe: failures above leave ms < 0 and the candidate unused;
    // an invalid parent would time a kernel that skips its work
    if (ms >= 0 && ra_sync_status(ctx) != RA_OK) ms = -1.0;
    (void)hipStreamSynchronize(st);
    if (dp) (void)hipFree(dp);
    ra_destroy(ctx);
    return ms;
}

}  // namespace

ra_status autotune_tiles(const std::vector<ra_chain_desc>& descs, const ra_run_desc& run, int family,
                         int& waves_per_block, hipStream_t stream, std::vector<int>& Ms, std::string& why) {
    std::lock_guard<std::mutex> lk(g_mu);
    const char* env = std::getenv("RA_AUTOTUNE_CACHE");
    const std::string path = env ? env : "";
    std::map<Key, Entry>& table = table_for(path);
    // candidate workgroup sizes: the caller's, or all three when it left the choice open
    std::vector<int> wpbs = waves_per_block ? std::vector<int>{waves_per_block} : std::vector<int>{1, 2, 4};
    double best_total = -1.0;
    std::vector<int> best_Ms = Ms;
    int best_wpb = waves_per_block ? waves_per_block : 4;
    for (int wpb : wpbs) {
        std::vector<int> Mw(descs.size());
        double total = 0.0;   // predicted batch time: sum over groups of R x time per replica
        for (size_t i = 0; i < descs.size(); ++i) {
            const ra_chain_desc& d = descs[i];
            const Key k{d.n_beads, d.spring, run.precision, family, wpb, run.noise_map};
            auto it = table.find(k);
            if (it == table.end()) {
                Entry best{Ms[i], -1.0};
                for (int M : family_beads_per_lane(family)) {
                    if (!legal(d.n_beads, M) || !map_allows(run.noise_map, M)) continue;
                    const double ms = time_tile(d, run, family, M, wpb, stream);
                    if (ms < 0) { why = "timing run failed"; return RA_EDEVICE; }
                    if (best.ms_per_replica < 0 || ms < best.ms_per_replica) best = Entry{M, ms};
                }
                it = table.emplace(k, best).first;
                append_cache_file(path, k, best);
            }
            Mw[i] = it->second.M;
            total += it->second.ms_per_replica * d.n_replicas;
        }
        if (best_total < 0 || total < best_total) {
            best_total = total;
            best_Ms = Mw;
            best_wpb = wpb;
        }
    }
    Ms = best_Ms;
    waves_per_block = best_wpb;
    return RA_OK;
}

}  // namespace ra
