// Internal interfaces of libknng: records shared by the stages and the host
// launchers each stage exports to the C-ABI layer (api.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <string>

namespace knng {

// Rows of one assignment chunk; one wavefront owns one chunk.
constexpr int kChunkRows = 1024;
// Largest cluster the leaf kernels accept.
constexpr int kMaxLeaf = 512;
// Largest dimension the partition kernels accept.
constexpr int kMaxDim = 4096;

// Device workspace cache (workspace.hip): stream-ordered use like
// hipMallocAsync / hipFreeAsync, but blocks stay cached per device between
// calls.  Calls that allocate hold the device's DeviceLock until their
// stream has been synchronised.
hipError_t ws_malloc(void** p, size_t bytes, hipStream_t s);
void ws_free(void* p, hipStream_t s);
void ws_release_device(int dev);  // frees every cached (unused) block of the device
// Arena mode of the calling thread: while an ArenaScope lives, ws_malloc
// carves kArenaAlign-aligned blocks of ws_arena_block(bytes) bytes from
// [base, base + cap) in order and returns hipErrorOutOfMemory once it is
// exhausted (it never calls hipMalloc); ws_free of those blocks does nothing.
constexpr size_t kArenaAlign = 256;
size_t ws_arena_block(size_t bytes);
class ArenaScope {
  public:
    ArenaScope(void* base, size_t cap);
    ~ArenaScope();
    ArenaScope(const ArenaScope&) = delete;
    ArenaScope& operator=(const ArenaScope&) = delete;

  private:
    alignas(8) unsigned char storage_[32];
};
class DeviceLock {
  public:
    DeviceLock();
    ~DeviceLock();
    DeviceLock(const DeviceLock&) = delete;
    DeviceLock& operator=(const DeviceLock&) = delete;
    int device() const;

  private:
    int dev_;
};

// Statistics counters (rows assigned, leaf pairs, ...) are spread over
// kStatSlots 128-byte lines: atomics from thousands of wavefronts on one
// address queue behind each other in one L2 channel.  Counter c of a block
// of counters lives at words c * kStatWords + slot * kStatStride.
constexpr int kStatSlots = 64;
constexpr int kStatStride = 16;
constexpr int kStatWords = kStatSlots * kStatStride;

__device__ __forceinline__ void stat_add(unsigned long long* c, unsigned key,
                                         unsigned long long v) {
    atomicAdd(c + (key & (kStatSlots - 1)) * kStatStride, v);
}
__device__ __forceinline__ void stat_max(unsigned long long* c, unsigned key,
                                         unsigned long long v) {
    atomicMax(c + (key & (kStatSlots - 1)) * kStatStride, v);
}
// Host side: total (or maximum) of one spread counter copied back.
inline unsigned long long stat_total(const unsigned long long* c) {
    unsigned long long t = 0;
    for (int i = 0; i < kStatSlots; ++i) t += c[i * kStatStride];
    return t;
}
inline unsigned long long stat_peak(const unsigned long long* c) {
    unsigned long long t = 0;
    for (int i = 0; i < kStatSlots; ++i) t = c[i * kStatStride] > t ? c[i * kStatStride] : t;
    return t;
}

// A node of the current level: a run [start, start+size) of perm[tree].
struct NodeRec {
    int32_t tree;    // tree slot 0..T-1 within this call
    int32_t start;
    int32_t size;
    int32_t chunk0;  // first assignment chunk of this node
};

// A finished cluster (leaf) of one tree.
struct LeafRec {
    int32_t tree;
    int32_t start;
    int32_t size;
    int32_t pad;
};

// Counters the level-finishing kernel hands back to the host.
struct LevelCounters {
    int32_t n_next;     // active nodes of the next level
    int32_t nc_next;    // assignment chunks of the next level
    int32_t n_big;      // next-level nodes spanning more than one chunk
    int32_t n_leaves;   // leaves so far
    int32_t n_log;      // bisected nodes logged so far
    int32_t n_sub;      // nodes handed to the subtree kernel so far
    int32_t seq;        // host mirror only: level whose counts are in place
};

// Status codes (mirror include/knng.h).
enum Status : int {
    kOk = 0,
    kInvalid = -1,
    kUnsupported = -2,
    kOom = -3,
    kHip = -4,
    kNonFinite = -5,
};

// Optional HIP-event timing of every launch of a few kernel classes.
enum KernelClass { kKAssign = 0, kKLeaf = 1, kKMerge = 2, kKClasses = 3 };

class KernelTimer {
  public:
    explicit KernelTimer(bool on) : on_(on) {}
    ~KernelTimer();
    KernelTimer(const KernelTimer&) = delete;
    KernelTimer& operator=(const KernelTimer&) = delete;
    bool on() const { return on_; }
    void begin(KernelClass c, hipStream_t s);
    void end(KernelClass c, hipStream_t s);
    // Sum of elapsed times per class (call after the stream completed).
    void collect(float ms[kKClasses], int count[kKClasses]);

  private:
    struct Pair { hipEvent_t a, b; int cls; };
    bool on_;
    Pair* pairs_ = nullptr;
    int n_ = 0, cap_ = 0;
    int open_ = -1;
};

// ---------------------------------------------------------------- subtrees
// Nodes of at most subtree_max_rows(D) rows (uint8 rows only) are split to
// leaves by one workgroup each (subtree.hip); roots[i].chunk0 holds the
// node's depth.
struct SubtreeArgs {
    const uint8_t* X8;
    int64_t n;
    int D;
    const NodeRec* roots;
    int n_roots;
    int32_t* perm;
    int leaf_max, min_leaf, max_iter;
    uint64_t seed;
    int tree0;
    LeafRec* leaves;
    int64_t leaves_cap;
    int32_t* node_log;
    int64_t node_log_cap;
    LevelCounters* ctr;
    unsigned long long* dstats;  // spread counters (kStatWords each): level-kernel assigned
                                 // rows (unused here), repairs, splits, deepest split
                                 // depth + 1, rows assigned inside subtree kernels
    int* overflow;               // bit 0: leaf list full, bit 1: subtree stack full
    int row_budget;              // LDS bytes for rows per workgroup: 131072 or 65536;
                                 // 0: one wavefront per subtree (kernel k_subtree_wave_u8)
    hipStream_t stream;
};
int subtree_max_rows(int D, int row_budget);  // 0: the subtree kernel does not take this D
int subtree_launch(const SubtreeArgs& a);

// One assignment pass over the chunks of the active nodes (one wavefront per
// chunk of kChunkRows rows): X, n, D, perm, nodes, chunk_node, number of
// chunks, centres C, status, n0f, labels, dots, per-chunk sums P, per-chunk
// counts, pass, max_iter, assigned-row counter, repair list, min_leaf,
// dispatch order and XCD share (dispatch_chunk in partition_dev.hpp).
template <typename TX>
using AssignFn = void (*)(const TX*, int64_t, int, const int32_t*, const NodeRec*, const int32_t*,
                          int, double*, int32_t*, int32_t*, uint8_t*, double*, double*, int32_t*,
                          int, int, unsigned long long*, int32_t*, int, const int32_t*, int);
// Matrix-core assignment passes for uint8 rows (D % 16 == 0, D <= 128):
// f[0] for a level's first pass, f[1] for the later ones; rows per step u
// (1 or 2) and pipeline depth pd (1 to 3).  f: one wavefront per chunk, four
// chunks per 256-thread workgroup (grid: chunks / 4); f4: four wavefronts
// per chunk (grid: chunks).  False if D is not covered.
bool pick_assign_u8_mfma(int D, int u, int pd, AssignFn<uint8_t>* f, AssignFn<uint8_t>* f4);

// FP32-row assignment passes (assign_f32.hip, D % 4 == 0): the level's first
// pass (chunk totals and side-1 sums), the later passes (changed rows added
// to the side-1 sums), the later passes filtered by the reduced copy (rf[fmt -
// 1] for BF16, FP16, FP8; extra arguments: the copy, 1/sigma, bytes per
// row, and two spread counters: rows of filtered passes, rows whose FP32
// values they read), and the repair's margins.
using AssignRfFn = void (*)(const float*, int64_t, int, const int32_t*, const NodeRec*,
                            const int32_t*, int, double*, int32_t*, int32_t*, uint8_t*, double*,
                            int32_t*, int, int, unsigned long long*, int32_t*, int,
                            const int32_t*, int, const uint8_t*, int, int,
                            unsigned long long*);
using RedotsFn = void (*)(const NodeRec*, const int32_t*, int64_t, const float*, int,
                          const int32_t*, const double*, const int32_t*, int, double*);
struct AssignF32Fns {
    AssignFn<float> first = nullptr;
    AssignFn<float> later = nullptr;
    AssignRfFn rf[3] = {nullptr, nullptr, nullptr};
    int rf_wpc = 1;  // wavefronts per chunk of rf (1: four chunks per workgroup; 4: one)
    RedotsFn redots = nullptr;
};
bool pick_assign_f32_fns(int D, int u, AssignF32Fns* f);

// ---------------------------------------------------------------- tuning
// Result-invariant choices of the build (csrc/tune.hip).  knob(): the
// environment variable if set, else the current call's tuned value, else
// fallback_default.
enum Knob {
    kKnobAssignUnroll, kKnobFilter, kKnobAssignMU, kKnobAssignMPD, kKnobChunkOrder,
    kKnobLeafWide, kKnobLeafBuckets, kKnobMergeNetwork, kKnobs
};
int knob(Knob id, int fallback_default);
int knob_default(Knob id);
std::string tune_key(int64_t n, int D, int k, int T, int L, int precision, int rerank, int compact,
                     int plain, int min_leaf, int max_iter);
// The tuned knob values in force on this thread for the scope's life: the
// cache file's entry for `key` (no entry: none), or explicit values.
class TuneScope {
  public:
    TuneScope(const char* cache_path, const std::string& key);
    explicit TuneScope(const int* vals);
    ~TuneScope();
    TuneScope(const TuneScope&) = delete;
    TuneScope& operator=(const TuneScope&) = delete;
  private:
    int vals_[kKnobs] = {};
    const int* prev_ = nullptr;
    bool active_ = false;
};
// Sets the library's error text for the calling thread; returns code.
int report_error(int code, const char* fmt, ...);

struct ReducedRows;

// ---------------------------------------------------------------- partition
struct PartitionArgs {
    const float* X;
    const uint8_t* X8;      // nullable: the same values stored as uint8 (all integers 0..255)
    int64_t n;
    int D;
    int n_trees;      // trees tree0 .. tree0+n_trees-1 go to slots 0..n_trees-1
    int tree0;
    int leaf_max;
    int min_leaf;
    int max_iter;
    uint64_t seed;
    int32_t* perm;          // device [n_trees][n], output
    LeafRec* leaves;        // device, capacity leaves_cap
    int64_t leaves_cap;
    int32_t* node_log;      // device nullable, [node_log_cap][4]
    int64_t node_log_cap;
    KernelTimer* timer;     // nullable
    hipStream_t stream;
    const ReducedRows* filter = nullptr;  // nullable: reduced copy of X for the filtered
                                          // passes (FP32 rows; results are unchanged)
    int precision = 0;                    // format of `filter` (1 BF16, 2 FP16, 3 FP8)
};

struct PartitionResult {
    int64_t n_leaves = 0;
    int64_t n_log = 0;
    int64_t assign_rows = 0;  // rows assigned, summed over passes (subtree kernels included)
    int64_t subtree_rows = 0; // the part of assign_rows assigned inside subtree kernels (LDS)
    int64_t filter_rows = 0;  // rows of filtered passes (labelled from the reduced copy first)
    int64_t filter_exact_rows = 0;  // rows whose FP32 values the filtered passes read
    int64_t splits = 0;
    int64_t repairs = 0;
    int levels = 0;
    int launches = 0;
};

// Runs the level-synchronous bisection of all requested trees.
int partition_run(const PartitionArgs& a, PartitionResult* res, char* err, size_t errlen);

// Upper bound on the number of leaves of n points in one tree.
inline int64_t max_leaves_per_tree(int64_t n, int min_leaf) {
    return n / (min_leaf > 0 ? min_leaf : 1) + 1;
}

// ---------------------------------------------------------------- leaves
struct LeafArgs {
    const float* X;
    int64_t n;
    int D;
    int k;
    int n_trees;
    const int32_t* perm;     // device [n_trees][n]
    const LeafRec* leaves;   // device
    int64_t n_leaves;
    int leaf_max;            // largest leaf size present
    int precision;
    int rerank;              // candidates per row for reduced precision
    int32_t* cand_ids;       // device [n_trees][n][k]
    float* cand_d;           // device [n_trees][n][k]
    unsigned long long* pairs;  // device nullable, spread counter: += m*(m-1) per leaf
    KernelTimer* timer;      // nullable
    hipStream_t stream;
};
int leaf_run(const LeafArgs& a, int* launches, char* err, size_t errlen);

// Reduced-precision copy of the rows for the MFMA first pass.
struct ReducedRows {
    uint8_t* Xr;   // [n] rows of `stride` bytes: Dp elements of the format (2 bytes
                   // BF16/FP16, 1 byte FP8), zero past D and up to the stride
    float* nrm;    // [n] squared norm of the dequantised reduced row
    float* sinv;   // [n] 1/sigma (power of two)
    int Dp;        // D rounded up to 32
    bool exact;    // first pass exact (d~ == d32): skip the re-rank
    int stride;    // bytes per row: Dp elements, the FP32 words 1/sigma and e (below),
                   // rounded up to whole 128-byte lines, so a gathered row takes whole
                   // cache lines
};
// byte offset of a reduced row's 1/sigma word: just past its Dp elements (one
// byte each for FP8-e4m3, precision 3; two for BF16 and FP16)
__host__ __device__ constexpr int reduced_rows_scale_offset(int precision, int Dp) {
    return Dp * (precision == 3 ? 1 : 2);
}
// byte offset of the FP32 word e that follows 1/sigma: an upper bound of the
// row's rounding error |sigma x - x~|_2 (Euclidean norm over the row)
__host__ __device__ constexpr int reduced_rows_err_offset(int precision, int Dp) {
    return reduced_rows_scale_offset(precision, Dp) + 4;
}
int reduced_rows_dp(int D);
int reduced_rows_stride(int precision, int D);
size_t reduced_rows_bytes(int precision, int64_t n, int D);
int prep_reduced(int precision, const float* X, int64_t n, int D, ReducedRows* rr, hipStream_t s);
int leaf_run_mfma(const LeafArgs& a, const ReducedRows& rr, int* launches, char* err,
                  size_t errlen);

// ---------------------------------------------------------------- merge
struct MergeArgs {
    int64_t n;
    int k;
    int n_trees;
    const int32_t* cand_ids;  // [n_trees][n][k]
    const float* cand_d;
    int32_t* ids_out;         // [n][k]
    float* dists_out;
    KernelTimer* timer;       // nullable
    hipStream_t stream;
};
int merge_run(const MergeArgs& a, int* launches, char* err, size_t errlen);

// ---------------------------------------------------------------- search
// E-GNNS (Alg. 2) for nq queries, one workgroup each (search.hip).
constexpr size_t kSearchLdsMax = 65536;  // visited table + rank list + query, per query
struct SearchArgs {
    const float* X;       // [n][D]
    int64_t n;
    int D;
    const int32_t* G;     // [n][kg], -1 padding
    int kg;
    const float* Q;       // [nq][D]
    int64_t nq;
    const int32_t* seeds; // [nq][ns]
    int ns;
    int k;
    int rounds;
    int32_t* ids_out;     // [nq][k]
    float* d_out;
    hipStream_t stream;
    unsigned long long* work = nullptr;  // nullable: 2 spread counters (distances, expansions)
    const uint8_t* X8 = nullptr;         // nullable: the rows as uint8 (used instead of X)
};
int search_run(const SearchArgs& a, char* err, size_t errlen);

// ---------------------------------------------------------------- RVQ index
// Two-stage residue vector quantisation, inverted lists and cascaded search
// seeds (Sec. 4.1-4.2, Eqns 1-3); csrc/ivf.hip.
constexpr int kRvqMaxWords = 256;          // words per stage
constexpr int kSeedMaxKeys = 4096;         // n1 * K2 keys ranked per query
constexpr size_t kSeedLdsMax = 65536;      // per-query seed state in LDS
struct RvqTrainArgs {
    const float* X;            // [n][D]
    int64_t n;
    int D;
    const int32_t* train_ids;  // [m] rows of X
    int64_t m;
    int K1, K2;
    const int32_t* init1;      // [K1] positions in the sample
    const int32_t* init2;      // [K2]
    int iters;
    double* W1;                // [K1][D]
    double* W2;                // [K2][D]
    int32_t* codes1;           // [m], nullable
    int32_t* codes2;           // [m], nullable
    int* rounds;               // host [2]
    hipStream_t stream;
};
int rvq_train_run(const RvqTrainArgs& a, char* err, size_t errlen);
struct IvfBuildArgs {
    const float* X;            // [n][D]
    int64_t n;
    int D;
    const double* W1;          // [K1][D]
    int K1;
    const double* W2;          // [K2][D]
    int K2;
    int32_t* keys_out;         // [n], nullable
    int32_t* offsets_out;      // [K1 K2 + 1]
    int32_t* ids_out;          // [n]
    hipStream_t stream;
};
int ivf_build_run(const IvfBuildArgs& a, char* err, size_t errlen);
struct IvfSeedArgs {
    const float* Q;            // [nq][D]
    int64_t nq;
    int D;
    const double* W1;
    int K1;
    const double* W2;
    int K2;
    const int32_t* offsets;    // [K1 K2 + 1]
    const int32_t* ids;        // [n_ids]
    int64_t n_ids;
    int n1;
    int ns;
    int32_t* seeds_out;        // [nq][ns]
    hipStream_t stream;
};
int ivf_seeds_run(const IvfSeedArgs& a, char* err, size_t errlen);

// ---------------------------------------------------------------- prep
// flags[0] <- 1 if X holds a NaN or Inf; flags[1] <- 1 if some value is not
// an integer in [0, 255] (flags: device int[2]).
int prep_scan(const float* X, int64_t count, int32_t* flags, hipStream_t s);
// X8[i] = X[i] for data whose values are all integers in [0, 255].
int prep_to_u8(const float* X, int64_t count, uint8_t* X8, hipStream_t s);

// Converts per-tree leaf lists into sorted run boundaries (knng_partition).
int leaves_to_offsets(const LeafRec* leaves, int64_t n_leaves, int64_t n, int tree,
                      int32_t* offsets_out, int32_t* count_out_dev, hipStream_t s);

}  // namespace knng
