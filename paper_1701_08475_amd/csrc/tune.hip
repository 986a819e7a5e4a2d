// Autotuner of the build's result-invariant choices, and its on-disk cache.
//
// Knobs: choices that change which kernel or launch shape runs, never the
// arithmetic of a result (each has a bit-identity test, and knng_autotune
// checks every candidate against the default build on the caller's data):
//   assign_unroll   FP32 rows per lane group and step in the assignment (1, 2)
//   filter          FP32 rows: later passes filtered by the reduced copy (0, 1)
//   assign_m_u      uint8 rows per step in the matrix-core assignment (1, 2)
//   assign_m_pd     uint8 loads ahead in the matrix-core assignment (1, 2)
//   chunk_order     chunks dispatched by their first row id (0, 1)
//   leaf_wide       re-ranked leaves on the 16-lane-group kernel (0, 1)
//   leaf_buckets    reduced-precision leaves in size buckets (0, 1)
//   merge_network   bitonic merge instead of the per-row insertion (0, 1)
// A knob's value comes from its environment variable if set, else from the
// tuned set of the current call (knng_build_ex with knng_options.tune_cache),
// else from the built-in default.
//
// Cache file: text, one line per build shape, "key|name=value ...", the last
// line of a key winning; written by knng_autotune (replacing that key's line).
#include "knng_internal.hpp"
#include "knng.h"

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

namespace knng {
namespace {

struct KnobDef {
    const char* name;
    const char* env;
    int dflt;
    int cand[2];
};
constexpr KnobDef kKnobDefs[kKnobs] = {
    {"assign_unroll", "KNNG_ASSIGN_UNROLL", 2, {1, 2}},
    {"filter", "KNNG_PARTITION_FILTER", 1, {0, 1}},
    {"assign_m_u", "KNNG_ASSIGN_M_U", 1, {1, 2}},
    {"assign_m_pd", "KNNG_ASSIGN_M_PD", 1, {1, 2}},
    {"chunk_order", "KNNG_CHUNK_ORDER", 1, {0, 1}},
    {"leaf_wide", "KNNG_LEAF_WIDE", 1, {0, 1}},
    {"leaf_buckets", "KNNG_LEAF_BUCKETS", 1, {0, 1}},
    {"merge_network", "KNNG_MERGE_NETWORK", 0, {0, 1}},
};

thread_local const int* t_tuned = nullptr;  // kKnobs values (-1: default) or null

using KeyMap = std::map<std::string, std::vector<int>>;
std::mutex g_cache_mu;
std::map<std::string, KeyMap> g_cache;  // path -> key -> values

std::vector<int> parse_values(const std::string& rest) {
    std::vector<int> v(kKnobs, -1);
    std::istringstream in(rest);
    std::string tok;
    while (in >> tok) {
        const size_t eq = tok.find('=');
        if (eq == std::string::npos) continue;
        const std::string nm = tok.substr(0, eq);
        for (int i = 0; i < kKnobs; ++i)
            if (nm == kKnobDefs[i].name) v[i] = std::atoi(tok.c_str() + eq + 1);
    }
    return v;
}

// Lines of the file as (key, rest); unreadable or missing file: none.
std::vector<std::pair<std::string, std::string>> read_lines(const std::string& path) {
    std::vector<std::pair<std::string, std::string>> out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t bar = line.find('|');
        if (bar == std::string::npos || bar == 0) continue;
        out.emplace_back(line.substr(0, bar), line.substr(bar + 1));
    }
    return out;
}

const KeyMap& cache_of(const std::string& path) {
    auto it = g_cache.find(path);
    if (it != g_cache.end()) return it->second;
    KeyMap m;
    for (const auto& kv : read_lines(path)) m[kv.first] = parse_values(kv.second);
    return g_cache.emplace(path, std::move(m)).first->second;
}

__global__ void k_count_diff(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b,
                             int64_t words, unsigned long long* __restrict__ diff) {
    unsigned long long d = 0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < words;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        d += a[i] != b[i] ? 1ull : 0ull;
    if (d) atomicAdd(diff, d);
}

}  // namespace

int knob(Knob id, int fallback_default) {
    const KnobDef& kd = kKnobDefs[id];
    if (const char* e = std::getenv(kd.env)) return std::atoi(e);
    if (t_tuned != nullptr && t_tuned[id] >= 0) return t_tuned[id];
    return fallback_default;
}

int knob_default(Knob id) { return kKnobDefs[id].dflt; }

std::string tune_key(int64_t n, int D, int k, int T, int L, int precision, int rerank, int compact,
                     int plain, int min_leaf, int max_iter) {
    int n2 = 0;
    while ((int64_t{1} << (n2 + 1)) <= n) ++n2;
    char b[200];
    std::snprintf(b, sizeof b, "D=%d k=%d T=%d L=%d prec=%d rerank=%d compact=%d plain=%d "
                  "min_leaf=%d max_iter=%d log2n=%d", D, k, T, L, precision, rerank, compact,
                  plain, min_leaf, max_iter, n2);
    return b;
}

TuneScope::TuneScope(const char* path, const std::string& key) {
    if (path == nullptr || path[0] == '\0') return;
    std::lock_guard<std::mutex> g(g_cache_mu);
    const KeyMap& m = cache_of(path);
    auto it = m.find(key);
    if (it == m.end()) return;
    for (int i = 0; i < kKnobs; ++i) vals_[i] = it->second[i];
    prev_ = t_tuned;
    t_tuned = vals_;
    active_ = true;
}

TuneScope::TuneScope(const int* vals) {
    for (int i = 0; i < kKnobs; ++i) vals_[i] = vals[i];
    prev_ = t_tuned;
    t_tuned = vals_;
    active_ = true;
}

TuneScope::~TuneScope() {
    if (active_) t_tuned = prev_;
}

}  // namespace knng

extern "C" int knng_autotune(const float* data, int64_t n, int32_t D, int32_t k, int32_t n_trees,
                             int32_t leaf_max, uint64_t seed, const knng_options* opt,
                             const char* cache_path, int32_t* chosen_out, hipStream_t stream) {
    using namespace knng;
    if (cache_path == nullptr || cache_path[0] == '\0')
        return report_error(KNNG_ERR_INVALID_ARG, "knng_autotune: cache_path is empty");
    knng_options o;
    knng_default_options(&o);
    if (opt != nullptr) {
        if (opt->struct_size != static_cast<int32_t>(sizeof(knng_options)))
            return report_error(KNNG_ERR_INVALID_ARG, "knng_options.struct_size is %d, expected %d",
                                opt->struct_size, static_cast<int>(sizeof(knng_options)));
        o = *opt;
    }
    o.tune_cache = nullptr;  // the tuner sets every knob itself
    o.time_kernels = 0;
    int dev = 0;
    const hipError_t de = hipGetDevice(&dev);
    if (de != hipSuccess)
        return report_error(KNNG_ERR_HIP, "knng_autotune: no current device: %s", hipGetErrorString(de));
    const hipError_t se = hipSetDevice(dev);
    if (se != hipSuccess)
        return report_error(KNNG_ERR_HIP, "knng_autotune: device %d: %s", dev, hipGetErrorString(se));
    const size_t words = static_cast<size_t>(n) * static_cast<size_t>(k);
    int32_t *ref_ids = nullptr, *ids = nullptr;
    float *ref_d = nullptr, *d = nullptr;
    unsigned long long* diff = nullptr;
    hipError_t e = hipMalloc(&ref_ids, words * 4);
    if (e == hipSuccess) e = hipMalloc(&ref_d, words * 4);
    if (e == hipSuccess) e = hipMalloc(&ids, words * 4);
    if (e == hipSuccess) e = hipMalloc(&d, words * 4);
    if (e == hipSuccess) e = hipMalloc(&diff, sizeof(unsigned long long));
    int rc = e == hipSuccess ? KNNG_OK
                             : report_error(KNNG_ERR_OOM, "knng_autotune: output buffers: %s",
                                            hipGetErrorString(e));
    int best[kKnobs];
    for (int i = 0; i < kKnobs; ++i) best[i] = knob_default(static_cast<Knob>(i));
    // one build with the knobs `vals`, its wall time (the call returns after
    // its stream is synchronised)
    auto run = [&](const int* vals, int32_t* oi, float* od, double* ms) -> int {
        TuneScope ts(vals);
        const auto t0 = std::chrono::steady_clock::now();
        const int r = knng_build_ex(data, n, D, k, n_trees, leaf_max, seed, oi, od, &o, nullptr,
                                    stream);
        *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                  .count();
        return r;
    };
    auto timed = [&](const int* vals, double* ms) -> int {
        double a = 0, b = 0;
        int r = run(vals, ids, d, &a);
        if (r == KNNG_OK) r = run(vals, ids, d, &b);
        *ms = a < b ? a : b;
        return r;
    };
    auto same_as_ref = [&](bool* same) -> int {
        unsigned long long h = 0;
        hipError_t q = hipMemsetAsync(diff, 0, sizeof h, stream);
        if (q == hipSuccess) {
            k_count_diff<<<1024, 256, 0, stream>>>(reinterpret_cast<const uint32_t*>(ref_ids),
                                                   reinterpret_cast<const uint32_t*>(ids),
                                                   static_cast<int64_t>(words), diff);
            k_count_diff<<<1024, 256, 0, stream>>>(reinterpret_cast<const uint32_t*>(ref_d),
                                                   reinterpret_cast<const uint32_t*>(d),
                                                   static_cast<int64_t>(words), diff);
            q = hipGetLastError();
        }
        if (q == hipSuccess) q = hipMemcpyAsync(&h, diff, sizeof h, hipMemcpyDeviceToHost, stream);
        if (q == hipSuccess) q = hipStreamSynchronize(stream);
        *same = h == 0;
        return q == hipSuccess ? KNNG_OK
                               : report_error(KNNG_ERR_HIP, "knng_autotune: compare: %s",
                                              hipGetErrorString(q));
    };
    double ms_best = 0;
    if (rc == KNNG_OK) {
        double w = 0;
        rc = run(best, ref_ids, ref_d, &w);  // the reference (default knobs), also a warm-up
    }
    if (rc == KNNG_OK) rc = timed(best, &ms_best);
    for (int i = 0; i < kKnobs && rc == KNNG_OK; ++i) {
        for (int c = 0; c < 2 && rc == KNNG_OK; ++c) {
            const int v = kKnobDefs[i].cand[c];
            if (v == best[i]) continue;
            int trial[kKnobs];
            for (int j = 0; j < kKnobs; ++j) trial[j] = best[j];
            trial[i] = v;
            double ms = 0;
            rc = timed(trial, &ms);
            bool same = false;
            if (rc == KNNG_OK) rc = same_as_ref(&same);
            if (rc != KNNG_OK) break;
            if (!same) {
                rc = report_error(KNNG_ERR_HIP, "knng_autotune: %s=%d changed the graph",
                                  kKnobDefs[i].name, v);
                break;
            }
            if (ms < 0.98 * ms_best) {  // a clear gain only
                best[i] = v;
                ms_best = ms;
            }
        }
    }
    if (rc == KNNG_OK) {
        // the cache line: replace this shape's key
        const std::string key = tune_key(n, D, k, n_trees, leaf_max, o.precision, o.rerank_factor,
                                         o.compact, o.plain, o.min_leaf == 0 ? k + 1 : o.min_leaf,
                                         o.max_iter == 0 ? 10 : o.max_iter);
        std::string rest;
        for (int i = 0; i < kKnobs; ++i) {
            char b[64];
            std::snprintf(b, sizeof b, "%s%s=%d", i ? " " : "", kKnobDefs[i].name, best[i]);
            rest += b;
        }
        std::lock_guard<std::mutex> g(g_cache_mu);
        auto lines = read_lines(cache_path);
        std::string tmp = std::string(cache_path) + ".tmp";
        {
            std::ofstream f(tmp, std::ios::trunc);
            for (const auto& kv : lines)
                if (kv.first != key) f << kv.first << '|' << kv.second << '\n';
            f << key << '|' << rest << '\n';
            if (!f) rc = report_error(KNNG_ERR_INVALID_ARG, "knng_autotune: cannot write %s", tmp.c_str());
        }
        if (rc == KNNG_OK && std::rename(tmp.c_str(), cache_path) != 0)
            rc = report_error(KNNG_ERR_INVALID_ARG, "knng_autotune: cannot replace %s", cache_path);
        if (rc == KNNG_OK) g_cache[cache_path][key] = parse_values(rest);
        if (rc == KNNG_OK && chosen_out != nullptr)
            for (int i = 0; i < kKnobs; ++i) chosen_out[i] = best[i];
    }
    hipFree(ref_ids);
    hipFree(ref_d);
    hipFree(ids);
    hipFree(d);
    hipFree(diff);
    return rc;
}
