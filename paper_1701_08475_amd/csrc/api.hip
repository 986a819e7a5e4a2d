// C ABI of libknng (declared in include/knng.h): argument checks, stream-
// ordered workspace, and the order of the stages of Algorithm 1 (Sec. 3.1):
// partition every tree (two-means bisection down to leaves), compare all
// pairs inside every leaf, union the rounds' candidate lists into G.
#include "knng.h"
#include "knng_internal.hpp"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <cstdint>
#include <mutex>
#include <optional>
#include <vector>

namespace {

thread_local char g_err[512] = "";

int set_err(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

}  // namespace

namespace knng {
int report_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}
}  // namespace knng

namespace {

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

struct Resolved {
    int precision = KNNG_FP32;
    int rerank = 2;
    int min_leaf = 0;
    int max_iter = 10;
    int plain = 0;
    int check_finite = 1;
    int time_kernels = 0;
    int compact = 1;
};

int resolve(const knng_options* opt, int k, Resolved* r) {
    if (opt != nullptr) {
        if (opt->struct_size != static_cast<int32_t>(sizeof(knng_options)))
            return set_err(KNNG_ERR_INVALID_ARG, "knng_options.struct_size is %d, expected %d",
                           opt->struct_size, static_cast<int>(sizeof(knng_options)));
        r->precision = opt->precision;
        r->rerank = opt->rerank_factor;
        r->min_leaf = opt->min_leaf;
        r->max_iter = opt->max_iter;
        r->plain = opt->plain;
        r->check_finite = opt->check_finite;
        r->time_kernels = opt->time_kernels;
        r->compact = opt->compact;
    }
    if (r->min_leaf == 0) r->min_leaf = k + 1;
    if (r->max_iter == 0) r->max_iter = 10;
    if (r->precision < KNNG_FP32 || r->precision > KNNG_FP8_E4M3)
        return set_err(KNNG_ERR_INVALID_ARG, "unknown precision %d", r->precision);
    if (r->rerank < 1) return set_err(KNNG_ERR_INVALID_ARG, "rerank_factor must be >= 1");
    if (r->min_leaf < 1) return set_err(KNNG_ERR_INVALID_ARG, "min_leaf must be >= 1");
    if (r->max_iter < 1) return set_err(KNNG_ERR_INVALID_ARG, "max_iter must be >= 1");
    return KNNG_OK;
}

int check_common(const float* data, int64_t n, int32_t D, int32_t k, int32_t n_trees,
                 const int32_t* ids_out, const float* dists_out) {
    if (data == nullptr || ids_out == nullptr || dists_out == nullptr)
        return set_err(KNNG_ERR_INVALID_ARG, "null pointer argument");
    if (!aligned16(data) || !aligned16(ids_out) || !aligned16(dists_out))
        return set_err(KNNG_ERR_INVALID_ARG, "pointers must be 16-byte aligned");
    if (n < 2 || n > 2147483647LL) return set_err(KNNG_ERR_INVALID_ARG, "n=%lld out of [2, 2^31-1]",
                                                  static_cast<long long>(n));
    if (D < 1) return set_err(KNNG_ERR_INVALID_ARG, "D=%d must be >= 1", D);
    if (D > knng::kMaxDim || (D % 4 != 0 && D > 1024))
        return set_err(KNNG_ERR_UNSUPPORTED, "D=%d not supported (D <= 4096, or <= 1024 if D %% 4 != 0)", D);
    if (k < 1 || k > n - 1) return set_err(KNNG_ERR_INVALID_ARG, "k=%d out of [1, n-1]", k);
    if (k > 512) return set_err(KNNG_ERR_UNSUPPORTED, "k=%d exceeds 512", k);
    if (n_trees < 1) return set_err(KNNG_ERR_INVALID_ARG, "n_trees=%d must be >= 1", n_trees);
    return KNNG_OK;
}

// The re-ranked matrix-core leaf kernels keep c = max(rerank k, k) <= 128
// candidates and k <= 64 neighbours per row; leaves above 256 points at most
// 64 candidates.
bool reduced_leaf_fits(int k, int rerank, int leaf_max) {
    const int64_t c = std::max<int64_t>(static_cast<int64_t>(rerank) * k, k);
    return k <= 64 && c <= 128 && (leaf_max <= 256 || c <= 64);
}
// The exact BF16 leaf kernels keep the k best: k <= 128, and k <= 64 for
// leaves above 256 points.
bool exact_leaf_fits(int k, int leaf_max) { return k <= 128 && (leaf_max <= 256 || k <= 64); }

struct Events {
    hipEvent_t e[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool ok = false;
    explicit Events(bool want) {
        if (!want) return;
        ok = true;
        for (auto& x : e)
            if (hipEventCreate(&x) != hipSuccess) ok = false;
    }
    void record(int i, hipStream_t s) {
        if (ok) hipEventRecord(e[i], s);
    }
    float ms(int a, int b) {
        float t = 0.f;
        if (ok && hipEventElapsedTime(&t, e[a], e[b]) == hipSuccess) return t;
        return 0.f;
    }
    ~Events() {
        for (auto& x : e)
            if (x) hipEventDestroy(x);
    }
};

int hip_fail(hipError_t e, const char* what) {
    return set_err(e == hipErrorOutOfMemory ? KNNG_ERR_OOM : KNNG_ERR_HIP, "%s: %s", what,
                   hipGetErrorString(e));
}

// One pass over the input: *u8 (nullable) <- all values are integers in
// [0, 255].  Returns KNNG_ERR_NONFINITE for NaN/Inf input.
int scan_input(const float* data, int64_t count, bool want_finite, int* u8, hipStream_t s) {
    int32_t* flags = nullptr;
    hipError_t e = knng::ws_malloc(reinterpret_cast<void**>(&flags), 2 * sizeof(int32_t), s);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync");
    int rc = knng::prep_scan(data, count, flags, s);
    int32_t h[2] = {0, 0};
    if (rc == KNNG_OK) {
        e = hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = hip_fail(e, "input scan");
    } else {
        rc = set_err(KNNG_ERR_HIP, "input-scan launch failed");
    }
    knng::ws_free(flags, s);
    if (rc == KNNG_OK && want_finite && h[0]) rc = set_err(KNNG_ERR_NONFINITE, "input holds NaN or Inf");
    if (u8) *u8 = (h[1] == 0 && h[0] == 0) ? 1 : 0;
    return rc;
}

int check_finite(const float* data, int64_t count, hipStream_t s) {
    return scan_input(data, count, true, nullptr, s);
}


}  // namespace

extern "C" {

void knng_default_options(knng_options* o) {
    if (o == nullptr) return;
    std::memset(o, 0, sizeof(*o));
    o->struct_size = static_cast<int32_t>(sizeof(knng_options));
    o->precision = KNNG_FP32;
    o->rerank_factor = 2;
    o->min_leaf = 0;
    o->max_iter = 10;
    o->plain = 0;
    o->check_finite = 1;
    o->time_kernels = 0;
    o->compact = 1;
    o->reserved = 0;
    o->tune_cache = nullptr;
}

const char* knng_status_string(int status) {
    switch (status) {
        case KNNG_OK: return "ok";
        case KNNG_ERR_INVALID_ARG: return "invalid argument";
        case KNNG_ERR_UNSUPPORTED: return "unsupported";
        case KNNG_ERR_OOM: return "out of device memory";
        case KNNG_ERR_HIP: return "HIP error";
        case KNNG_ERR_NONFINITE: return "non-finite input";
        default: return "unknown status";
    }
}

const char* knng_last_error(void) { return g_err; }

int knng_version(void) { return 103; }

int knng_build_ex(const float* data, int64_t n, int32_t D, int32_t k, int32_t n_trees,
                  int32_t leaf_max, uint64_t seed, int32_t* ids_out, float* dists_out,
                  const knng_options* opt, knng_stats* stats_out, hipStream_t stream) {
    g_err[0] = '\0';
    int rc = check_common(data, n, D, k, n_trees, ids_out, dists_out);
    if (rc != KNNG_OK) return rc;
    Resolved o;
    rc = resolve(opt, k, &o);
    if (rc != KNNG_OK) return rc;
    if (leaf_max < 2 * o.min_leaf - 1)
        return set_err(KNNG_ERR_INVALID_ARG, "leaf_max=%d < 2*min_leaf-1=%d", leaf_max,
                       2 * o.min_leaf - 1);
    if (leaf_max > knng::kMaxLeaf)
        return set_err(KNNG_ERR_UNSUPPORTED, "leaf_max=%d exceeds %d", leaf_max, knng::kMaxLeaf);
    const int lm_eff = leaf_max < n ? leaf_max : static_cast<int>(n);
    // Which matrix-core leaf kernels can serve this request: the re-ranked
    // first pass keeps c = max(rerank_factor k, k) candidates per row, the
    // exact BF16 pass (integer data) keeps k.
    const bool reduced_fits = reduced_leaf_fits(k, o.rerank, lm_eff);
    const bool exact_fits = exact_leaf_fits(k, lm_eff);
    if (o.precision != KNNG_FP32 && !reduced_fits && !(o.precision == KNNG_BF16 && exact_fits))
        return set_err(KNNG_ERR_UNSUPPORTED,
                       "the re-ranked leaf kernel keeps k <= 64 and rerank_factor*k <= 128 "
                       "(<= 64 for leaves above 256 points); k=%d, rerank_factor=%d, leaf_max=%d",
                       k, o.rerank, lm_eff);

    hipStream_t s = stream;
    // tuned choices (knng_autotune's cache) for this shape, if any
    const knng::TuneScope tune(opt != nullptr ? opt->tune_cache : nullptr,
                               knng::tune_key(n, D, k, n_trees, leaf_max, o.precision, o.rerank,
                                              o.compact, o.plain, o.min_leaf, o.max_iter));
    knng::DeviceLock dlock;  // workspace blocks: one call per device at a time
    Events ev(stats_out != nullptr);
    knng::KernelTimer timer(o.time_kernels != 0 && stats_out != nullptr);
    ev.record(0, s);
    int all_u8 = 0;
    if (o.check_finite || (o.compact && D % 16 == 0)) {
        rc = scan_input(data, n * static_cast<int64_t>(D), o.check_finite != 0, &all_u8, s);
        if (rc != KNNG_OK) return rc;
    }
    const bool use_u8 = o.compact && D % 16 == 0 && all_u8;

    const int T = n_trees;
    const int slots = o.plain ? 1 : T;  // trees partitioned per call
    const int64_t lcap = static_cast<int64_t>(slots) * knng::max_leaves_per_tree(n, o.min_leaf);
    int32_t* perm = nullptr;
    knng::LeafRec* leaves = nullptr;
    int32_t* cand_ids = nullptr;
    float* cand_d = nullptr;
    const bool direct = (T == 1);  // one tree: its candidate lists are G
    char err[400] = "";
    int launches = 0;
    knng::PartitionResult pres;
    int64_t pairs = 0;
    int64_t n_leaves_total = 0;
    hipError_t e;
    unsigned long long* dpairs = nullptr;
    std::vector<unsigned long long> hpairs(knng::kStatWords, 0ull);
    uint8_t* x8 = nullptr;
    // BF16 holds integers 0..255 exactly, and with 2 D 255^2 < 2^24 (D <= 129)
    // every product, norm, sum of two norms and partial sum of the first pass
    // is an exact FP32 integer, so its distances equal d32 bit for bit.  Such
    // data takes that path for FP32 and BF16 requests alike (not in the plain
    // schedule, nor with compact=0) when its kernel serves (k, leaf_max);
    // otherwise FP32 requests take the FP32 direct kernel.
    const bool exact_bf16 = all_u8 != 0 && D <= 129 && o.compact && !o.plain && exact_fits &&
                            (o.precision == KNNG_FP32 || o.precision == KNNG_BF16);
    const int leaf_prec = exact_bf16 ? KNNG_BF16 : o.precision;
    if (leaf_prec != KNNG_FP32 && !exact_bf16 && !reduced_fits)
        return set_err(KNNG_ERR_UNSUPPORTED,
                       "BF16 with rerank_factor*k = %d needs the exact first pass (integer "
                       "data 0..255, D <= 129)", o.rerank * k);
    knng::ReducedRows rr{nullptr, nullptr, nullptr, knng::reduced_rows_dp(D), exact_bf16,
                         knng::reduced_rows_stride(leaf_prec, D)};

    e = knng::ws_malloc(reinterpret_cast<void**>(&perm), sizeof(int32_t) * slots * n, s);
    if (e == hipSuccess)
        e = knng::ws_malloc(reinterpret_cast<void**>(&leaves), sizeof(knng::LeafRec) * lcap, s);
    if (e == hipSuccess && !direct)
        e = knng::ws_malloc(reinterpret_cast<void**>(&cand_ids), sizeof(int32_t) * T * n * k, s);
    if (e == hipSuccess && !direct)
        e = knng::ws_malloc(reinterpret_cast<void**>(&cand_d), sizeof(float) * T * n * k, s);
    if (e == hipSuccess)
        e = knng::ws_malloc(reinterpret_cast<void**>(&dpairs),
                           sizeof(unsigned long long) * knng::kStatWords, s);
    if (e == hipSuccess)
        e = hipMemsetAsync(dpairs, 0, sizeof(unsigned long long) * knng::kStatWords, s);
    if (e == hipSuccess && use_u8)
        e = knng::ws_malloc(reinterpret_cast<void**>(&x8), static_cast<size_t>(n) * D, s);
    if (e == hipSuccess && leaf_prec != KNNG_FP32)
        e = knng::ws_malloc(reinterpret_cast<void**>(&rr.Xr),
                           knng::reduced_rows_bytes(leaf_prec, n, D), s);
    if (e == hipSuccess && leaf_prec != KNNG_FP32)
        e = knng::ws_malloc(reinterpret_cast<void**>(&rr.nrm), sizeof(float) * n, s);
    if (e == hipSuccess && leaf_prec != KNNG_FP32)
        e = knng::ws_malloc(reinterpret_cast<void**>(&rr.sinv), sizeof(float) * n, s);
    if (e != hipSuccess) {
        rc = hip_fail(e, "workspace allocation");
        goto done;
    }
    if (use_u8 && knng::prep_to_u8(data, n * static_cast<int64_t>(D), x8, s) != KNNG_OK) {
        rc = set_err(KNNG_ERR_HIP, "uint8 copy launch failed");
        goto done;
    }
    if (leaf_prec != KNNG_FP32 && knng::prep_reduced(leaf_prec, data, n, D, &rr, s) != KNNG_OK) {
        rc = set_err(KNNG_ERR_HIP, "reduced-copy launch failed");
        goto done;
    }
    ev.record(1, s);
    if (direct) {
        cand_ids = ids_out;
        cand_d = dists_out;
    }

    for (int t0 = 0; t0 < T; t0 += slots) {
        knng::PartitionArgs pa{};
        pa.X = data;
        pa.X8 = x8;
        pa.n = n;
        pa.D = D;
        pa.n_trees = slots;
        pa.tree0 = t0;
        pa.leaf_max = leaf_max;
        pa.min_leaf = o.min_leaf;
        pa.max_iter = o.max_iter;
        pa.seed = seed;
        pa.perm = perm;
        pa.leaves = leaves;
        pa.leaves_cap = lcap;
        pa.node_log = nullptr;
        pa.node_log_cap = 0;
        pa.timer = &timer;
        pa.stream = s;
        // FP32 rows with a reduced copy: the partition's later passes read
        // the copy first (same labels and centres, fewer bytes)
        pa.filter = (leaf_prec != KNNG_FP32 && !o.plain) ? &rr : nullptr;
        pa.precision = leaf_prec;
        knng::PartitionResult r;
        rc = knng::partition_run(pa, &r, err, sizeof(err));
        if (rc != KNNG_OK) {
            set_err(rc, "partition: %s", err);
            goto done;
        }
        pres.assign_rows += r.assign_rows;
        pres.subtree_rows += r.subtree_rows;
        pres.filter_rows += r.filter_rows;
        pres.filter_exact_rows += r.filter_exact_rows;
        pres.splits += r.splits;
        pres.repairs += r.repairs;
        pres.levels = r.levels > pres.levels ? r.levels : pres.levels;
        launches += r.launches;
        n_leaves_total += r.n_leaves;
        if (t0 == 0) ev.record(2, s);
        knng::LeafArgs la{};
        la.X = data;
        la.n = n;
        la.D = D;
        la.k = k;
        la.n_trees = slots;
        la.perm = perm;
        la.leaves = leaves;
        la.n_leaves = r.n_leaves;
        la.leaf_max = leaf_max < n ? leaf_max : static_cast<int>(n);
        la.precision = leaf_prec;
        la.rerank = exact_bf16 ? k : o.rerank * k;  // the exact pass keeps the k best
        la.cand_ids = cand_ids + static_cast<size_t>(t0) * n * k;
        la.cand_d = cand_d + static_cast<size_t>(t0) * n * k;
        la.pairs = dpairs;
        la.timer = &timer;
        la.stream = s;
        rc = leaf_prec == KNNG_FP32 ? knng::leaf_run(la, &launches, err, sizeof(err))
                                    : knng::leaf_run_mfma(la, rr, &launches, err, sizeof(err));
        if (rc != KNNG_OK) {
            set_err(rc, "leaf search: %s", err);
            goto done;
        }
    }
    ev.record(3, s);
    if (!direct) {
        knng::MergeArgs ma{};
        ma.n = n;
        ma.k = k;
        ma.n_trees = T;
        ma.cand_ids = cand_ids;
        ma.cand_d = cand_d;
        ma.ids_out = ids_out;
        ma.dists_out = dists_out;
        ma.timer = &timer;
        ma.stream = s;
        rc = knng::merge_run(ma, &launches, err, sizeof(err));
        if (rc != KNNG_OK) {
            set_err(rc, "merge: %s", err);
            goto done;
        }
    }
    ev.record(4, s);
    e = hipMemcpyAsync(hpairs.data(), dpairs, sizeof(unsigned long long) * hpairs.size(),
                       hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(e, "build");
    pairs = static_cast<int64_t>(knng::stat_total(hpairs.data()));

done:
    if (perm) knng::ws_free(perm, s);
    if (leaves) knng::ws_free(leaves, s);
    if (dpairs) knng::ws_free(dpairs, s);
    if (x8) knng::ws_free(x8, s);
    if (rr.Xr) knng::ws_free(rr.Xr, s);
    if (rr.nrm) knng::ws_free(rr.nrm, s);
    if (rr.sinv) knng::ws_free(rr.sinv, s);
    if (!direct) {
        if (cand_ids) knng::ws_free(cand_ids, s);
        if (cand_d) knng::ws_free(cand_d, s);
    }
    e = hipStreamSynchronize(s);
    if (rc == KNNG_OK && e != hipSuccess) rc = hip_fail(e, "build");
    if (rc == KNNG_OK && stats_out != nullptr) {
        std::memset(stats_out, 0, sizeof(*stats_out));
        stats_out->assign_rows = pres.assign_rows;
        stats_out->subtree_rows = pres.subtree_rows;
        stats_out->filter_rows = pres.filter_rows;
        stats_out->filter_exact_rows = pres.filter_exact_rows;
        stats_out->ordered_pairs = pairs;
        stats_out->leaves = n_leaves_total;
        stats_out->splits = pres.splits;
        stats_out->repairs = pres.repairs;
        stats_out->levels = pres.levels;
        stats_out->launches = launches;
        stats_out->ms_prep = ev.ms(0, 1);
        if (o.plain) {  // stages interleave per tree: report partition+leaf together
            stats_out->ms_partition = ev.ms(1, 3);
            stats_out->ms_leaf = 0.f;
        } else {
            stats_out->ms_partition = ev.ms(1, 2);
            stats_out->ms_leaf = ev.ms(2, 3);
        }
        stats_out->ms_merge = ev.ms(3, 4);
        stats_out->ms_total = ev.ms(0, 4);
        float kms[knng::kKClasses];
        int kn[knng::kKClasses];
        timer.collect(kms, kn);
        stats_out->ms_k_assign = kms[knng::kKAssign];
        stats_out->n_k_assign = kn[knng::kKAssign];
        stats_out->ms_k_leaf = kms[knng::kKLeaf];
        stats_out->n_k_leaf = kn[knng::kKLeaf];
        stats_out->ms_k_merge = kms[knng::kKMerge];
        stats_out->n_k_merge = kn[knng::kKMerge];
        stats_out->compact_used = use_u8 ? 1 : 0;
        stats_out->exact_first_pass = exact_bf16 ? 1 : 0;
    }
    return rc;
}

int knng_build(const float* data, int64_t n, int32_t D, int32_t k, int32_t n_trees,
               int32_t leaf_max, uint64_t seed, int32_t* ids_out, float* dists_out,
               hipStream_t stream) {
    return knng_build_ex(data, n, D, k, n_trees, leaf_max, seed, ids_out, dists_out, nullptr,
                         nullptr, stream);
}

int knng_partition(const float* data, int64_t n, int32_t D, int32_t leaf_max, int32_t min_leaf,
                   int32_t max_iter, uint64_t seed, int32_t tree, int32_t* perm_out,
                   int32_t* leaf_offsets_out, int32_t* n_leaves_out, int32_t* nodes_out,
                   int32_t* n_nodes_out, hipStream_t stream) {
    g_err[0] = '\0';
    if (data == nullptr || perm_out == nullptr || leaf_offsets_out == nullptr ||
        n_leaves_out == nullptr)
        return set_err(KNNG_ERR_INVALID_ARG, "null pointer argument");
    if (!aligned16(data)) return set_err(KNNG_ERR_INVALID_ARG, "data must be 16-byte aligned");
    if (n < 2 || n > 2147483647LL) return set_err(KNNG_ERR_INVALID_ARG, "n out of [2, 2^31-1]");
    if (D < 1) return set_err(KNNG_ERR_INVALID_ARG, "D must be >= 1");
    if (D > knng::kMaxDim || (D % 4 != 0 && D > 1024))
        return set_err(KNNG_ERR_UNSUPPORTED, "D=%d not supported", D);
    if (tree < 0) return set_err(KNNG_ERR_INVALID_ARG, "tree must be >= 0");
    if (min_leaf == 0) min_leaf = 1;
    if (max_iter == 0) max_iter = 10;
    if (min_leaf < 1 || max_iter < 1) return set_err(KNNG_ERR_INVALID_ARG, "min_leaf, max_iter >= 1");
    if (leaf_max < 2 * min_leaf - 1 || leaf_max < 1)
        return set_err(KNNG_ERR_INVALID_ARG, "leaf_max < 2*min_leaf-1");

    hipStream_t s = stream;
    knng::DeviceLock dlock;  // workspace blocks: one call per device at a time
    int all_u8 = 0;
    int rc = scan_input(data, n * static_cast<int64_t>(D), true, &all_u8, s);
    if (rc != KNNG_OK) return rc;
    const bool use_u8 = D % 16 == 0 && all_u8;  // same storage choice as knng_build
    const int64_t lcap = knng::max_leaves_per_tree(n, min_leaf);
    knng::LeafRec* leaves = nullptr;
    uint8_t* x8 = nullptr;
    int32_t* dcount = nullptr;
    int32_t hcount = 0;
    char err[400] = "";
    knng::PartitionResult r;
    hipError_t e = knng::ws_malloc(reinterpret_cast<void**>(&leaves), sizeof(knng::LeafRec) * lcap, s);
    if (e == hipSuccess) e = knng::ws_malloc(reinterpret_cast<void**>(&dcount), sizeof(int32_t), s);
    if (e == hipSuccess && use_u8)
        e = knng::ws_malloc(reinterpret_cast<void**>(&x8), static_cast<size_t>(n) * D, s);
    if (e != hipSuccess) {
        rc = hip_fail(e, "workspace allocation");
        goto done;
    }
    if (use_u8 && knng::prep_to_u8(data, n * static_cast<int64_t>(D), x8, s) != KNNG_OK) {
        rc = set_err(KNNG_ERR_HIP, "uint8 copy launch failed");
        goto done;
    }
    {
        knng::PartitionArgs pa{};
        pa.X = data;
        pa.X8 = x8;
        pa.n = n;
        pa.D = D;
        pa.n_trees = 1;
        pa.tree0 = tree;
        pa.leaf_max = leaf_max;
        pa.min_leaf = min_leaf;
        pa.max_iter = max_iter;
        pa.seed = seed;
        pa.perm = perm_out;
        pa.leaves = leaves;
        pa.leaves_cap = lcap;
        pa.node_log = nodes_out;
        pa.node_log_cap = nodes_out ? n : 0;
        pa.timer = nullptr;
        pa.stream = s;
        rc = knng::partition_run(pa, &r, err, sizeof(err));
        if (rc != KNNG_OK) {
            set_err(rc, "partition: %s", err);
            goto done;
        }
    }
    rc = knng::leaves_to_offsets(leaves, r.n_leaves, n, 0, leaf_offsets_out, dcount, s);
    if (rc != KNNG_OK) {
        set_err(rc, "leaf offsets");
        goto done;
    }
    e = hipMemcpyAsync(&hcount, dcount, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        rc = hip_fail(e, "partition");
        goto done;
    }
    *n_leaves_out = hcount;
    if (n_nodes_out) *n_nodes_out = static_cast<int32_t>(r.n_log);

done:
    if (leaves) knng::ws_free(leaves, s);
    if (x8) knng::ws_free(x8, s);
    if (dcount) knng::ws_free(dcount, s);
    e = hipStreamSynchronize(s);
    if (rc == KNNG_OK && e != hipSuccess) rc = hip_fail(e, "partition");
    return rc;
}

}  // extern "C"

namespace knng {
namespace {
// Turn per-tree boundary arrays into leaf records; flags malformed input.
__global__ void k_offsets_to_leaves(const int32_t* __restrict__ off, int nl, int tree,
                                    int64_t n, LeafRec* __restrict__ out, int32_t* __restrict__ maxsz,
                                    int32_t* __restrict__ bad) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nl; i += gridDim.x * blockDim.x) {
        const int32_t a = off[i], b = off[i + 1];
        if (b <= a || a < 0 || b > n || (i == 0 && a != 0) || (i == nl - 1 && b != n))
            atomicOr(bad, 1);
        out[i] = LeafRec{tree, a, b - a, 0};
        atomicMax(maxsz, b - a);
    }
}
// bad <- 1 if a perm entry lies outside [0, n).
__global__ void k_check_perm(const int32_t* __restrict__ perm, int64_t count, int64_t n,
                             int32_t* __restrict__ bad) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        if (perm[i] < 0 || perm[i] >= n) atomicOr(bad, 1);
}
__global__ void k_zero2(int32_t* p) {
    p[0] = 0;
    p[1] = 0;
}
}  // namespace
}  // namespace knng

// Scratch memory of knng_leaf_search_noalloc: every GPU the library runs on
// holds one copy of this array until the process ends.  Host code uses the
// device address that hipGetSymbolAddress returns for the current device
// (scratch_address), never the array's name.
constexpr size_t kNoAllocScratchBytes = size_t{64} << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// This device's address of `scratch`, looked up once per device (with that
// device current) and kept.
hipError_t scratch_address(void** p) {
    *p = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* q = nullptr;
        e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = q;
    }
    *p = g_scratch_ptr[dev];
    return hipSuccess;
}

// a * b, or SIZE_MAX when it overflows
size_t mul_sat(size_t a, size_t b) {
    if (a != 0 && b > SIZE_MAX / a) return SIZE_MAX;
    return a * b;
}

// Bytes the leaf search carves from an arena: every workspace block it may
// take (leaf table, flags, input scan flags, per-tree candidate lists,
// reduced copy with norms and scales, size-bucket counters and grouped leaf
// table), each rounded to the arena's alignment.  Blocks are never reused
// within a call in arena mode, so this is the exact upper bound.
size_t leaf_search_scratch_bytes(int64_t n, int D, int k, int n_trees, int64_t total_leaves,
                                 int precision, bool check_finite) {
    size_t need = 0;
    auto add = [&](size_t b) {
        const size_t r = b == SIZE_MAX ? SIZE_MAX : knng::ws_arena_block(b);
        need = (r == SIZE_MAX || need > SIZE_MAX - r) ? SIZE_MAX : need + r;
    };
    add(mul_sat(sizeof(knng::LeafRec), static_cast<size_t>(total_leaves)));
    add(2 * sizeof(int32_t));
    if (check_finite) add(2 * sizeof(int32_t));
    if (n_trees > 1) {
        const size_t lists = mul_sat(mul_sat(static_cast<size_t>(n_trees), static_cast<size_t>(n)),
                                     static_cast<size_t>(k));
        add(mul_sat(lists, sizeof(int32_t)));
        add(mul_sat(lists, sizeof(float)));
    }
    if (precision != KNNG_FP32) {
        add(knng::reduced_rows_bytes(precision, n, D));
        add(mul_sat(sizeof(float), static_cast<size_t>(n)));
        add(mul_sat(sizeof(float), static_cast<size_t>(n)));
        add(8 * sizeof(int32_t));
        add(mul_sat(sizeof(knng::LeafRec), static_cast<size_t>(total_leaves)));
    }
    return need;
}

// knng_leaf_search and knng_leaf_search_noalloc: with noalloc, every
// workspace block comes from this device's `scratch` array.
int leaf_search_impl(const float* data, int64_t n, int32_t D, int32_t k, int32_t n_trees,
                     const int32_t* perm, const int32_t* leaf_offsets, const int32_t* n_leaves,
                     const knng_options* opt, int32_t* ids_out, float* dists_out,
                     hipStream_t stream, bool noalloc) {
    g_err[0] = '\0';
    int rc = check_common(data, n, D, k, n_trees, ids_out, dists_out);
    if (rc != KNNG_OK) return rc;
    if (perm == nullptr || leaf_offsets == nullptr || n_leaves == nullptr)
        return set_err(KNNG_ERR_INVALID_ARG, "null pointer argument");
    Resolved o;
    rc = resolve(opt, k, &o);
    if (rc != KNNG_OK) return rc;
    if (o.precision != KNNG_FP32 && !reduced_leaf_fits(k, o.rerank, 256))
        return set_err(KNNG_ERR_UNSUPPORTED,
                       "the re-ranked leaf kernel keeps k <= 64 and rerank_factor*k <= 128 "
                       "(k=%d, rerank_factor=%d)", k, o.rerank);
    int64_t total = 0;
    for (int t = 0; t < n_trees; ++t) {
        if (n_leaves[t] < 1 || n_leaves[t] > n)
            return set_err(KNNG_ERR_INVALID_ARG, "n_leaves[%d]=%d out of [1, n]", t, n_leaves[t]);
        total += n_leaves[t];
    }
    void* arena_base = nullptr;
    if (noalloc) {
        const size_t need = leaf_search_scratch_bytes(n, D, k, n_trees, total, o.precision,
                                                      o.check_finite != 0);
        if (need > kNoAllocScratchBytes)
            return set_err(KNNG_ERR_UNSUPPORTED,
                           "the request needs %zu bytes of scratch memory; the no-allocation "
                           "entry point has %zu", need, kNoAllocScratchBytes);
        const hipError_t e = scratch_address(&arena_base);
        if (e != hipSuccess) return hip_fail(e, "scratch address");
    }
    hipStream_t s = stream;
    knng::DeviceLock dlock;  // workspace blocks: one call per device at a time
    std::optional<knng::ArenaScope> arena;
    if (noalloc) arena.emplace(arena_base, kNoAllocScratchBytes);
    knng::LeafRec* leaves = nullptr;
    int32_t* flags = nullptr;  // [0] max leaf size, [1] malformed
    int32_t hflags[2] = {0, 0};
    int32_t* cand_ids = nullptr;
    float* cand_d = nullptr;
    const bool direct = (n_trees == 1);
    char err[400] = "";
    int launches = 0;
    knng::ReducedRows rr{nullptr, nullptr, nullptr, knng::reduced_rows_dp(D), false,
                         knng::reduced_rows_stride(o.precision, D)};
    hipError_t e = knng::ws_malloc(reinterpret_cast<void**>(&leaves), sizeof(knng::LeafRec) * total, s);
    if (e == hipSuccess) e = knng::ws_malloc(reinterpret_cast<void**>(&flags), sizeof(int32_t) * 2, s);
    if (e != hipSuccess) {
        rc = hip_fail(e, "workspace allocation");
        goto done;
    }
    knng::k_zero2<<<1, 1, 0, s>>>(flags);
    {
        int64_t li = 0, oi = 0;
        for (int t = 0; t < n_trees; ++t) {
            knng::k_offsets_to_leaves<<<64, 256, 0, s>>>(leaf_offsets + oi, n_leaves[t], t, n,
                                                         leaves + li, flags, flags + 1);
            li += n_leaves[t];
            oi += n_leaves[t] + 1;
        }
        knng::k_check_perm<<<1024, 256, 0, s>>>(perm, static_cast<int64_t>(n_trees) * n, n,
                                                flags + 1);
    }
    e = hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        rc = hip_fail(e, "leaf table");
        goto done;
    }
    if (hflags[1]) {
        rc = set_err(KNNG_ERR_INVALID_ARG,
                     "leaf_offsets not ascending from 0 to n, or perm entry outside [0, n)");
        goto done;
    }
    if (hflags[0] > knng::kMaxLeaf) {
        rc = set_err(KNNG_ERR_UNSUPPORTED, "leaf of %d points exceeds %d", hflags[0], knng::kMaxLeaf);
        goto done;
    }
    if (o.check_finite) {
        rc = check_finite(data, n * static_cast<int64_t>(D), s);
        if (rc != KNNG_OK) goto done;
    }
    if (direct) {
        cand_ids = ids_out;
        cand_d = dists_out;
    } else {
        e = knng::ws_malloc(reinterpret_cast<void**>(&cand_ids), sizeof(int32_t) * n_trees * n * k, s);
        if (e == hipSuccess)
            e = knng::ws_malloc(reinterpret_cast<void**>(&cand_d), sizeof(float) * n_trees * n * k, s);
        if (e != hipSuccess) {
            rc = hip_fail(e, "workspace allocation");
            goto done;
        }
    }
    if (o.precision != KNNG_FP32) {
        e = knng::ws_malloc(reinterpret_cast<void**>(&rr.Xr),
                           knng::reduced_rows_bytes(o.precision, n, D), s);
        if (e == hipSuccess) e = knng::ws_malloc(reinterpret_cast<void**>(&rr.nrm), sizeof(float) * n, s);
        if (e == hipSuccess) e = knng::ws_malloc(reinterpret_cast<void**>(&rr.sinv), sizeof(float) * n, s);
        if (e != hipSuccess) {
            rc = hip_fail(e, "workspace allocation");
            goto done;
        }
        if (knng::prep_reduced(o.precision, data, n, D, &rr, s) != KNNG_OK) {
            rc = set_err(KNNG_ERR_HIP, "reduced-copy launch failed");
            goto done;
        }
    }
    {
        knng::LeafArgs la{};
        la.X = data;
        la.n = n;
        la.D = D;
        la.k = k;
        la.n_trees = n_trees;
        la.perm = perm;
        la.leaves = leaves;
        la.n_leaves = total;
        la.leaf_max = hflags[0];
        la.precision = o.precision;
        la.rerank = o.rerank * k;
        la.cand_ids = cand_ids;
        la.cand_d = cand_d;
        la.pairs = nullptr;
        la.timer = nullptr;
        la.stream = s;
        rc = o.precision == KNNG_FP32 ? knng::leaf_run(la, &launches, err, sizeof(err))
                                      : knng::leaf_run_mfma(la, rr, &launches, err, sizeof(err));
        if (rc != KNNG_OK) {
            set_err(rc, "leaf search: %s", err);
            goto done;
        }
    }
    if (!direct) {
        knng::MergeArgs ma{};
        ma.n = n;
        ma.k = k;
        ma.n_trees = n_trees;
        ma.cand_ids = cand_ids;
        ma.cand_d = cand_d;
        ma.ids_out = ids_out;
        ma.dists_out = dists_out;
        ma.timer = nullptr;
        ma.stream = s;
        rc = knng::merge_run(ma, &launches, err, sizeof(err));
        if (rc != KNNG_OK) {
            set_err(rc, "merge: %s", err);
            goto done;
        }
    }
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = hip_fail(e, "leaf search");
done:
    if (leaves) knng::ws_free(leaves, s);
    if (flags) knng::ws_free(flags, s);
    if (rr.Xr) knng::ws_free(rr.Xr, s);
    if (rr.nrm) knng::ws_free(rr.nrm, s);
    if (rr.sinv) knng::ws_free(rr.sinv, s);
    if (!direct) {
        if (cand_ids) knng::ws_free(cand_ids, s);
        if (cand_d) knng::ws_free(cand_d, s);
    }
    e = hipStreamSynchronize(s);
    if (rc == KNNG_OK && e != hipSuccess) rc = hip_fail(e, "leaf search");
    return rc;
}

}  // namespace

extern "C" int knng_leaf_search(const float* data, int64_t n, int32_t D, int32_t k,
                                int32_t n_trees, const int32_t* perm,
                                const int32_t* leaf_offsets, const int32_t* n_leaves,
                                const knng_options* opt, int32_t* ids_out, float* dists_out,
                                hipStream_t stream) {
    return leaf_search_impl(data, n, D, k, n_trees, perm, leaf_offsets, n_leaves, opt, ids_out,
                            dists_out, stream, false);
}

extern "C" int knng_leaf_search_noalloc(const float* data, int64_t n, int32_t D, int32_t k,
                                        int32_t n_trees, const int32_t* perm,
                                        const int32_t* leaf_offsets, const int32_t* n_leaves,
                                        const knng_options* opt, int32_t* ids_out,
                                        float* dists_out, hipStream_t stream) {
    return leaf_search_impl(data, n, D, k, n_trees, perm, leaf_offsets, n_leaves, opt, ids_out,
                            dists_out, stream, true);
}

namespace {
__global__ void k_zero_u64(unsigned long long* p, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        p[i] = 0ull;
}
}  // namespace

extern "C" int knng_search(const float* data, int64_t n, int32_t D, const int32_t* graph,
                           int32_t kg, const float* queries, int64_t nq, const int32_t* seeds,
                           int32_t ns, int32_t k, int32_t rounds, int32_t* ids_out,
                           float* dists_out, hipStream_t stream) {
    return knng_search_ex(data, n, D, graph, kg, queries, nq, seeds, ns, k, rounds, ids_out,
                          dists_out, nullptr, stream);
}

namespace {
// knng_search_ex (rows as FP32, data8 null) and knng_search_u8 (rows as
// uint8, data null).
int search_impl(const float* data, const uint8_t* data8, int64_t n, int32_t D,
                const int32_t* graph, int32_t kg, const float* queries, int64_t nq,
                const int32_t* seeds, int32_t ns, int32_t k, int32_t rounds, int32_t* ids_out,
                float* dists_out, uint64_t* work_out, hipStream_t stream) {
    g_err[0] = '\0';
    const void* rows = data != nullptr ? static_cast<const void*>(data) : data8;
    if (rows == nullptr || graph == nullptr || queries == nullptr || seeds == nullptr ||
        ids_out == nullptr || dists_out == nullptr)
        return set_err(KNNG_ERR_INVALID_ARG, "null pointer argument");
    if (!aligned16(rows) || !aligned16(queries))
        return set_err(KNNG_ERR_INVALID_ARG, "data and queries must be 16-byte aligned");
    if (n < 1 || n > 2147483647LL)
        return set_err(KNNG_ERR_INVALID_ARG, "n=%lld out of [1, 2^31-1]", static_cast<long long>(n));
    if (D < 1 || D > knng::kMaxDim)
        return set_err(D < 1 ? KNNG_ERR_INVALID_ARG : KNNG_ERR_UNSUPPORTED, "D=%d out of [1, %d]", D,
                       knng::kMaxDim);
    if (kg < 1) return set_err(KNNG_ERR_INVALID_ARG, "graph degree %d must be >= 1", kg);
    if (nq < 0 || nq > 2147483647LL)
        return set_err(KNNG_ERR_INVALID_ARG, "nq=%lld out of [0, 2^31-1]", static_cast<long long>(nq));
    if (ns < 1) return set_err(KNNG_ERR_INVALID_ARG, "seeds per query %d must be >= 1", ns);
    if (k < 1) return set_err(KNNG_ERR_INVALID_ARG, "k=%d must be >= 1", k);
    if (rounds < 0) return set_err(KNNG_ERR_INVALID_ARG, "rounds=%d must be >= 0", rounds);
    if (static_cast<int64_t>(k) * kg > (1 << 20) || ns > (1 << 20))
        return set_err(KNNG_ERR_UNSUPPORTED, "k x graph degree or seeds too large");
    hipStream_t s = stream;
    knng::SearchArgs sa{data, n, D, graph, kg, queries, nq, seeds, ns, k, rounds, ids_out,
                        dists_out, s};
    sa.X8 = data8;
    char err[400] = "";
    if (work_out == nullptr) {
        int rc = knng::search_run(sa, err, sizeof(err));
        if (rc != KNNG_OK) return set_err(rc, "search: %s", err);
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "search");
        return KNNG_OK;
    }
    // work report: two spread counters in scratch memory
    knng::DeviceLock dlock;
    unsigned long long* work = nullptr;
    std::vector<unsigned long long> h(2 * knng::kStatWords, 0ull);
    hipError_t e = knng::ws_malloc(reinterpret_cast<void**>(&work),
                                   sizeof(unsigned long long) * h.size(), s);
    if (e != hipSuccess) return hip_fail(e, "workspace allocation");
    k_zero_u64<<<8, 256, 0, s>>>(work, static_cast<int>(h.size()));
    sa.work = work;
    int rc = knng::search_run(sa, err, sizeof(err));
    if (rc == KNNG_OK) {
        e = hipMemcpyAsync(h.data(), work, sizeof(unsigned long long) * h.size(),
                           hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    knng::ws_free(work, s);
    if (rc != KNNG_OK) return set_err(rc, "search: %s", err);
    if (e != hipSuccess) return hip_fail(e, "search");
    work_out[0] = knng::stat_total(h.data());
    work_out[1] = knng::stat_total(h.data() + knng::kStatWords);
    return KNNG_OK;
}
}  // namespace

extern "C" int knng_search_ex(const float* data, int64_t n, int32_t D, const int32_t* graph,
                              int32_t kg, const float* queries, int64_t nq, const int32_t* seeds,
                              int32_t ns, int32_t k, int32_t rounds, int32_t* ids_out,
                              float* dists_out, uint64_t* work_out, hipStream_t stream) {
    if (data == nullptr) {
        g_err[0] = '\0';
        return set_err(KNNG_ERR_INVALID_ARG, "null pointer argument");
    }
    return search_impl(data, nullptr, n, D, graph, kg, queries, nq, seeds, ns, k, rounds, ids_out,
                       dists_out, work_out, stream);
}

extern "C" int knng_search_u8(const uint8_t* data8, int64_t n, int32_t D, const int32_t* graph,
                              int32_t kg, const float* queries, int64_t nq, const int32_t* seeds,
                              int32_t ns, int32_t k, int32_t rounds, int32_t* ids_out,
                              float* dists_out, uint64_t* work_out, hipStream_t stream) {
    if (data8 == nullptr) {
        g_err[0] = '\0';
        return set_err(KNNG_ERR_INVALID_ARG, "null pointer argument");
    }
    return search_impl(nullptr, data8, n, D, graph, kg, queries, nq, seeds, ns, k, rounds, ids_out,
                       dists_out, work_out, stream);
}

extern "C" int knng_to_u8(const float* data, int64_t count, uint8_t* out, hipStream_t stream) {
    g_err[0] = '\0';
    if (data == nullptr || out == nullptr)
        return set_err(KNNG_ERR_INVALID_ARG, "null pointer argument");
    if (count < 0) return set_err(KNNG_ERR_INVALID_ARG, "count=%lld < 0", static_cast<long long>(count));
    if (count == 0) return KNNG_OK;
    hipStream_t s = stream;
    knng::DeviceLock dlock;
    int32_t* flags = nullptr;  // [0] NaN/Inf, [1] a value not an integer in [0, 255]
    int32_t h[2] = {0, 0};
    hipError_t e = knng::ws_malloc(reinterpret_cast<void**>(&flags), 2 * sizeof(int32_t), s);
    if (e != hipSuccess) return hip_fail(e, "workspace allocation");
    int rc = knng::prep_scan(data, count, flags, s);
    if (rc == KNNG_OK) {
        e = hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    knng::ws_free(flags, s);
    if (rc != KNNG_OK) return set_err(rc, "value scan failed");
    if (e != hipSuccess) return hip_fail(e, "value scan");
    if (h[0] || h[1])
        return set_err(KNNG_ERR_INVALID_ARG, "the values are not all integers in [0, 255]");
    rc = knng::prep_to_u8(data, count, out, s);
    if (rc != KNNG_OK) return set_err(rc, "conversion launch failed");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "conversion");
    return KNNG_OK;
}

extern "C" void knng_release_workspace(void) {
    knng::DeviceLock dlock;
    knng::ws_release_device(dlock.device());
}

// ---------------------------------------------------------------- RVQ index

extern "C" int knng_rvq_train(const float* data, int64_t n, int32_t D, const int32_t* train_ids,
                              int64_t m, int32_t K1, int32_t K2, const int32_t* init1,
                              const int32_t* init2, int32_t iters, double* words1_out,
                              double* words2_out, int32_t* codes1_out, int32_t* codes2_out,
                              int32_t* rounds_out, hipStream_t stream) {
    g_err[0] = '\0';
    if (data == nullptr || train_ids == nullptr || init1 == nullptr || init2 == nullptr ||
        words1_out == nullptr || words2_out == nullptr)
        return set_err(KNNG_ERR_INVALID_ARG, "null pointer argument");
    if (n < 1 || n > 2147483647LL)
        return set_err(KNNG_ERR_INVALID_ARG, "n=%lld out of [1, 2^31-1]", static_cast<long long>(n));
    if (D < 1 || D > knng::kMaxDim)
        return set_err(D < 1 ? KNNG_ERR_INVALID_ARG : KNNG_ERR_UNSUPPORTED, "D=%d out of [1, %d]", D,
                       knng::kMaxDim);
    if (m < 1 || m > n)
        return set_err(KNNG_ERR_INVALID_ARG, "training rows m=%lld out of [1, n]",
                       static_cast<long long>(m));
    if (K1 < 1 || K2 < 1 || K1 > knng::kRvqMaxWords || K2 > knng::kRvqMaxWords)
        return set_err(K1 < 1 || K2 < 1 ? KNNG_ERR_INVALID_ARG : KNNG_ERR_UNSUPPORTED,
                       "vocabulary sizes K1=%d, K2=%d out of [1, %d]", K1, K2, knng::kRvqMaxWords);
    if (iters < 0) return set_err(KNNG_ERR_INVALID_ARG, "iters=%d must be >= 0", iters);
    knng::DeviceLock dlock;
    int rounds[2] = {0, 0};
    knng::RvqTrainArgs ra{data, n, D, train_ids, m, K1, K2, init1, init2, iters, words1_out,
                          words2_out, codes1_out, codes2_out, rounds, stream};
    char err[400] = "";
    const int rc = knng::rvq_train_run(ra, err, sizeof(err));
    if (rc != KNNG_OK) return set_err(rc, "rvq train: %s", err);
    if (rounds_out != nullptr) {
        rounds_out[0] = rounds[0];
        rounds_out[1] = rounds[1];
    }
    return KNNG_OK;
}

extern "C" int knng_ivf_build(const float* data, int64_t n, int32_t D, const double* words1,
                              int32_t K1, const double* words2, int32_t K2, int32_t* keys_out,
                              int32_t* offsets_out, int32_t* ids_out, hipStream_t stream) {
    g_err[0] = '\0';
    if (data == nullptr || words1 == nullptr || words2 == nullptr || offsets_out == nullptr ||
        (ids_out == nullptr && n > 0))
        return set_err(KNNG_ERR_INVALID_ARG, "null pointer argument");
    if (n < 0 || n > 2147483647LL)
        return set_err(KNNG_ERR_INVALID_ARG, "n=%lld out of [0, 2^31-1]", static_cast<long long>(n));
    if (D < 1 || D > knng::kMaxDim)
        return set_err(D < 1 ? KNNG_ERR_INVALID_ARG : KNNG_ERR_UNSUPPORTED, "D=%d out of [1, %d]", D,
                       knng::kMaxDim);
    if (K1 < 1 || K2 < 1 || K1 > knng::kRvqMaxWords || K2 > knng::kRvqMaxWords)
        return set_err(K1 < 1 || K2 < 1 ? KNNG_ERR_INVALID_ARG : KNNG_ERR_UNSUPPORTED,
                       "vocabulary sizes K1=%d, K2=%d out of [1, %d]", K1, K2, knng::kRvqMaxWords);
    knng::DeviceLock dlock;
    knng::IvfBuildArgs ba{data, n, D, words1, K1, words2, K2, keys_out, offsets_out, ids_out, stream};
    char err[400] = "";
    const int rc = knng::ivf_build_run(ba, err, sizeof(err));
    if (rc != KNNG_OK) return set_err(rc, "ivf build: %s", err);
    return KNNG_OK;
}

extern "C" int knng_ivf_seeds(const float* queries, int64_t nq, int32_t D, const double* words1,
                              int32_t K1, const double* words2, int32_t K2, const int32_t* offsets,
                              const int32_t* ids, int64_t n_ids, int32_t n1, int32_t ns,
                              int32_t* seeds_out, hipStream_t stream) {
    g_err[0] = '\0';
    if (words1 == nullptr || words2 == nullptr || offsets == nullptr ||
        ((queries == nullptr || seeds_out == nullptr) && nq > 0) || (ids == nullptr && n_ids > 0))
        return set_err(KNNG_ERR_INVALID_ARG, "null pointer argument");
    if (nq < 0 || nq > 2147483647LL)
        return set_err(KNNG_ERR_INVALID_ARG, "nq=%lld out of [0, 2^31-1]", static_cast<long long>(nq));
    if (n_ids < 0 || n_ids > 2147483647LL)
        return set_err(KNNG_ERR_INVALID_ARG, "n_ids=%lld out of [0, 2^31-1]",
                       static_cast<long long>(n_ids));
    if (D < 1 || D > knng::kMaxDim)
        return set_err(D < 1 ? KNNG_ERR_INVALID_ARG : KNNG_ERR_UNSUPPORTED, "D=%d out of [1, %d]", D,
                       knng::kMaxDim);
    if (K1 < 1 || K2 < 1 || K1 > knng::kRvqMaxWords || K2 > knng::kRvqMaxWords)
        return set_err(K1 < 1 || K2 < 1 ? KNNG_ERR_INVALID_ARG : KNNG_ERR_UNSUPPORTED,
                       "vocabulary sizes K1=%d, K2=%d out of [1, %d]", K1, K2, knng::kRvqMaxWords);
    if (n1 < 1 || n1 > K1) return set_err(KNNG_ERR_INVALID_ARG, "n1=%d out of [1, K1=%d]", n1, K1);
    if (n1 * K2 > knng::kSeedMaxKeys)
        return set_err(KNNG_ERR_UNSUPPORTED, "n1 x K2 = %d keys exceeds %d", n1 * K2,
                       knng::kSeedMaxKeys);
    if (ns < 1 || ns > (1 << 20))
        return set_err(KNNG_ERR_INVALID_ARG, "seeds per query %d out of [1, 2^20]", ns);
    knng::DeviceLock dlock;
    knng::IvfSeedArgs sa{queries, nq, D, words1, K1, words2, K2, offsets, ids, n_ids, n1, ns,
                         seeds_out, stream};
    char err[400] = "";
    const int rc = knng::ivf_seeds_run(sa, err, sizeof(err));
    if (rc != KNNG_OK) return set_err(rc, "ivf seeds: %s", err);
    return KNNG_OK;
}
