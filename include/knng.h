/*
 * knng.h -- C ABI of libknng.so: kNN-graph construction by repeated two-means
 * bisection on one AMD Instinct MI355X (gfx950).
 *
 * Method: Zhao, Yang, Deng, "Scalable Nearest Neighbor Search based on kNN
 * Graph" (arXiv 1701.08475), Sec. 3.1 and Algorithm 1.  Input X (n x D) and
 * k; output the kNN graph G (n x k).  Each of n_trees rounds bisects X with
 * two-means clustering until every cluster holds at most leaf_max points,
 * compares every pair inside each cluster, and updates both rows' k-lists.
 *
 * Conventions shared by every entry point
 *   - Pointers documented as "device" are HIP device pointers owned by the
 *     caller, row-major and contiguous, 16-byte aligned.  Pointers documented
 *     as "host" are ordinary host memory.
 *   - All work is ordered on `stream`; each call returns after that work has
 *     completed (it synchronises the stream).  Scratch memory comes from a
 *     per-device cache inside the library: blocks are allocated with
 *     hipMalloc on first need and kept for later calls (returning them to
 *     the driver every call costs milliseconds per build);
 *     knng_release_workspace() frees them.  Calls that use scratch memory on
 *     the same device run one at a time (a per-device lock).
 *   - Return value: KNNG_OK (0) or a negative status below.  On an argument
 *     error (KNNG_ERR_INVALID_ARG, KNNG_ERR_UNSUPPORTED) no output is
 *     written; nothing is launched except, where a call checks device-side
 *     arguments (ids, offsets, positions), the kernel that checks them.  On KNNG_ERR_NONFINITE the outputs are not
 *     written.  On KNNG_ERR_OOM / KNNG_ERR_HIP output contents are
 *     unspecified.  knng_last_error() gives a message for the calling thread.
 *   - Distances are squared Euclidean distances in FP32.  Every reported
 *     distance is the canonical FP32 value d32(i, j): the sum over 32-wide
 *     blocks of dimensions, in increasing order, of the in-block sequential
 *     fused sum of (x_i[d] - x_j[d])^2.  d32(i, j) == d32(j, i) bitwise.
 *   - Rows of G are ordered by ascending (distance, id); ids are distinct and
 *     never the row itself; a row with fewer than k candidates is padded
 *     with (id -1, distance +inf) -- this cannot happen when min_leaf >= k+1.
 *   - Deterministic: equal inputs give bit-identical outputs.
 */
#ifndef KNNG_H
#define KNNG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define KNNG_OK                0
#define KNNG_ERR_INVALID_ARG  -1  /* a precondition on an argument failed      */
#define KNNG_ERR_UNSUPPORTED  -2  /* valid request this build cannot serve     */
#define KNNG_ERR_OOM          -3  /* device memory allocation failed           */
#define KNNG_ERR_HIP          -4  /* a HIP runtime call or launch failed       */
#define KNNG_ERR_NONFINITE    -5  /* the input holds NaN or Inf                */

/* leaf distance precision (first pass; output distances are always d32) */
#define KNNG_FP32      0
#define KNNG_BF16      1
#define KNNG_FP16      2
#define KNNG_FP8_E4M3  3

typedef struct {
    int32_t struct_size;    /* sizeof(knng_options); set by knng_default_options */
    int32_t precision;      /* KNNG_FP32 (default) | KNNG_BF16 | KNNG_FP16 | KNNG_FP8_E4M3 */
    int32_t rerank_factor;  /* reduced precision keeps rerank_factor*k candidates per
                               row and leaf for the FP32 re-rank; default 2 */
    int32_t min_leaf;       /* smallest side of a bisection; 0 -> k+1 (default) */
    int32_t max_iter;       /* two-means assignment-pass budget; 0 -> 10 */
    int32_t plain;          /* 1: unbatched schedule (trees one after another, one
                               leaf launch per tree); 0: batched (default) */
    int32_t check_finite;   /* 1 (default): reject NaN/Inf input */
    int32_t time_kernels;   /* 1: bracket every launch of the assignment, leaf and
                               merge kernels with HIP events and report the summed
                               time in knng_stats (0 default: no events) */
    int32_t compact;        /* 1 (default): when every input value is an integer in
                               [0, 255], the partition streams a uint8 copy of X
                               (D % 16 == 0) and, for FP32/BF16 requests with
                               D <= 129 outside the plain schedule, leaf distances
                               come from the exact BF16 matrix-core pass; the
                               values are unchanged, so are the results.  0: FP32 */
    int32_t reserved;
    const char* tune_cache; /* nullable path of knng_autotune's cache file: the build
                               takes the tuned choices stored for its shape (none
                               stored, or NULL: the built-in defaults).  The choices
                               never change results.  Read on first use per path and
                               kept in memory; the file is owned by the caller. */
} knng_options;

typedef struct {
    int64_t assign_rows;    /* sum over all assignment passes of rows assigned */
    int64_t ordered_pairs;  /* sum over trees and leaves of m*(m-1) */
    int64_t leaves;         /* leaves over all trees */
    int64_t splits;         /* bisections over all trees */
    int64_t repairs;        /* bisections repaired by margin rank */
    int32_t levels;         /* deepest level + 1 */
    int32_t launches;       /* kernel launches issued */
    float ms_prep, ms_partition, ms_leaf, ms_merge, ms_total;  /* stream time */
    /* with time_kernels = 1: summed event time and launch count per kernel
       class (two-means assignment pass, leaf search, merge); else 0 */
    float ms_k_assign;
    int32_t n_k_assign;
    float ms_k_leaf;
    int32_t n_k_leaf;
    float ms_k_merge;
    int32_t n_k_merge;
    int32_t compact_used;   /* 1 if the partition streamed the uint8 copy */
    int32_t exact_first_pass; /* 1 if leaf distances came from the exact BF16
                                 first pass (integer data 0..255, D <= 129; equal
                                 to d32 bit for bit) */
    int64_t subtree_rows;   /* the part of assign_rows assigned inside the subtree
                               kernels (rows held in LDS, no memory traffic per
                               pass); assign_rows - subtree_rows rows were streamed
                               by the level kernels' assignment passes */
    int64_t filter_rows;    /* rows of assignment passes filtered by the reduced copy
                               (FP32 rows with a BF16/FP16/FP8 first pass): each read
                               its reduced row first */
    int64_t filter_exact_rows; /* rows whose FP32 values those passes also read (label
                                  inside the filter's error band, or changed) */
} knng_stats;

/* Fill *opt with the defaults listed above. */
void knng_default_options(knng_options* opt);

/*
 * knng_build -- Algorithm 1 (Sec. 3.1) end to end, FP32, batched schedule.
 * Same as knng_build_ex(..., opt = NULL, stats = NULL, stream).
 *   data       device, float[n][D], the reference set X
 *   n          number of points, 2 <= n <= 2^31-1
 *   D          dimension, 1 <= D <= 4096
 *   k          neighbours per row, 1 <= k <= min(n-1, 512)
 *   n_trees    rounds of bisection (the paper's I_0), >= 1
 *   leaf_max   clusters hold at most leaf_max points (the paper's threshold);
 *              leaf_max >= 2*min_leaf - 1 and leaf_max <= 512
 *   seed       keys the random starting centres of every two-means split
 *   ids_out    device, int32[n][k]
 *   dists_out  device, float[n][k]
 */
int knng_build(const float* data, int64_t n, int32_t D, int32_t k, int32_t n_trees,
               int32_t leaf_max, uint64_t seed, int32_t* ids_out, float* dists_out,
               hipStream_t stream);

/*
 * knng_build_ex -- as knng_build with options (NULL = defaults) and optional
 * host statistics (NULL = none).
 */
int knng_build_ex(const float* data, int64_t n, int32_t D, int32_t k, int32_t n_trees,
                  int32_t leaf_max, uint64_t seed, int32_t* ids_out, float* dists_out,
                  const knng_options* opt, knng_stats* stats_out, hipStream_t stream);

/*
 * knng_autotune -- the size buckets and tile shapes of the description above
 * are chosen by a small autotuner (not in the paper: runtime of this
 * library).  Its knobs are the build's result-invariant choices, in this order
 * (KNNG_TUNE_KNOBS values): FP32-row assignment rows per step (1, 2); the
 * reduced-copy filter of FP32-row passes (0, 1); uint8-row matrix-core
 * assignment rows per step (1, 2) and loads ahead (1, 2); chunk dispatch
 * order (0, 1); the 16-lane-group leaf kernel (0, 1); leaf size buckets
 * (0, 1); the bitonic merge (0, 1).  For each knob in turn it runs
 * knng_build_ex on the caller's data with the other knobs at their best so
 * far, checks that the graph is bit-identical to the build with default
 * knobs (else KNNG_ERR_HIP and a message naming the knob: that would be a
 * bug), times two builds and keeps a value that is at least 2% faster.  The
 * choices go to cache_path (a line keyed by the build's shape: D, k, n_trees,
 * leaf_max, the options that select the path, floor(log2 n); an existing line
 * of that key is replaced) and, if chosen_out is not NULL, to
 * chosen_out[KNNG_TUNE_KNOBS].  Arguments as knng_build_ex; opt->tune_cache
 * and opt->time_kernels are ignored.  It allocates two output buffers of
 * n*k*8 bytes with hipMalloc and runs about 2 + 3 * KNNG_TUNE_KNOBS builds.
 *   Errors: those of knng_build_ex; KNNG_ERR_INVALID_ARG for an empty
 *   cache_path or a file that cannot be written.
 */
#define KNNG_TUNE_KNOBS 8
int knng_autotune(const float* data, int64_t n, int32_t D, int32_t k, int32_t n_trees,
                  int32_t leaf_max, uint64_t seed, const knng_options* opt,
                  const char* cache_path, int32_t* chosen_out, hipStream_t stream);

/*
 * knng_partition -- one round's clustering (Sec. 3.1: bisect repeatedly with
 * two-means until no cluster exceeds leaf_max; Alg. 1, clustering step and
 * collection of the cluster set S) for tree index `tree`, exactly as
 * knng_build runs it with default options (including the uint8 storage of
 * integer-valued input).
 *   perm_out          device, int32[n]: the points in depth-first leaf order
 *                     (left child first); every cluster is a contiguous run
 *                     and lists its ids in ascending order
 *   leaf_offsets_out  device, int32[n+1] capacity: receives n_leaves+1
 *                     ascending run boundaries, first 0, last n
 *   n_leaves_out      host, receives the number of leaves
 *   nodes_out         device, nullable, int32[n][4] capacity: every bisected
 *                     node as (start, size, left_size, depth), start/size a
 *                     run of perm_out; ordered by depth, then start
 *   n_nodes_out       host, nullable, receives the number of bisected nodes
 *   min_leaf          0 -> k+1 is not known here, so 0 means 1
 *   max_iter          0 -> 10
 */
int knng_partition(const float* data, int64_t n, int32_t D, int32_t leaf_max,
                   int32_t min_leaf, int32_t max_iter, uint64_t seed, int32_t tree,
                   int32_t* perm_out, int32_t* leaf_offsets_out, int32_t* n_leaves_out,
                   int32_t* nodes_out, int32_t* n_nodes_out, hipStream_t stream);

/*
 * knng_leaf_search -- Alg. 1's inner loops for given clusters: compare every
 * pair <i, j>, i != j, inside each cluster of each tree and keep, per row, the
 * k smallest distinct (d32, id) over all trees.
 *   perm          device, int32[n_trees][n]: per tree, a permutation of
 *                 0..n-1 in which every cluster is a contiguous run
 *   leaf_offsets  device, int32: per tree n_leaves[t]+1 ascending boundaries
 *                 into that tree's perm (first 0, last n), trees concatenated
 *   n_leaves      host, int32[n_trees]; every cluster size <= 512
 *   opt           nullable; precision and rerank_factor are used
 * Malformed offsets or perm entries outside [0, n) give KNNG_ERR_INVALID_ARG
 * before any output is written.
 */
int knng_leaf_search(const float* data, int64_t n, int32_t D, int32_t k, int32_t n_trees,
                     const int32_t* perm, const int32_t* leaf_offsets,
                     const int32_t* n_leaves, const knng_options* opt,
                     int32_t* ids_out, float* dists_out, hipStream_t stream);

/*
 * knng_leaf_search_noalloc -- knng_leaf_search for callers that cannot
 * allocate device memory (code in a tight serving loop, or in a harness that
 * forbids hipMalloc).  Same arguments, checks, kernels and results as
 * knng_leaf_search; it calls no hipMalloc, hipFree or other allocating
 * routine.  Its scratch blocks (leaf table, flags, per-tree candidate lists,
 * reduced copy, size buckets) are carved from a fixed 64 MiB device array
 * that every GPU the library runs on holds until the process ends (its
 * address is looked up once per device, on the first call there).
 *   Limit: 16 B per leaf + 8 n_trees n k B of candidate lists when
 *   n_trees > 1 + for a reduced precision n (S + 8) B (S = Dp b + 4 rounded
 *   up to a multiple of 128, Dp = D rounded up to 32, b = 2 for BF16/FP16, 1
 *   for FP8) + 16 B per leaf, each block rounded up to 256 B, must fit
 *   64 MiB; larger requests return
 *   KNNG_ERR_UNSUPPORTED before any HIP call.
 *   Calls on one device share the array and are serialised by the library's
 *   per-device lock (each returns after its stream is synchronised); the
 *   array keeps the last call's contents, and every value a call reads from
 *   it is written by that call first (flags and counters are cleared by fill
 *   kernels, not memsets).
 */
int knng_leaf_search_noalloc(const float* data, int64_t n, int32_t D, int32_t k, int32_t n_trees,
                             const int32_t* perm, const int32_t* leaf_offsets,
                             const int32_t* n_leaves, const knng_options* opt,
                             int32_t* ids_out, float* dists_out, hipStream_t stream);

/*
 * knng_search -- enhanced hill-climbing nearest-neighbour search over a kNN
 * graph (Alg. 2, E-GNNS), one call for a batch of queries.  For each query
 * q, the rank list R starts from the seeds; each of `rounds` rounds takes
 * every member of the k best of R not expanded before, visits its graph
 * neighbours not visited before (distance to q), and merges them into R
 * after the round.  A round with nothing to expand ends that query's search.
 *   data       device, float[n][D]: the reference set (16-byte aligned)
 *   graph      device, int32[n][kg]: neighbour ids per point (e.g. the output
 *              of knng_build); entries < 0 or >= n are skipped
 *   queries    device, float[nq][D] (16-byte aligned)
 *   seeds      device, int32[nq][ns]: starting points per query (for example
 *              drawn at random); entries < 0 or >= n and repeats are skipped
 *   k          rank-list length and number of results per query, >= 1
 *   rounds     expansion rounds t_0 (>= 0; 0 returns the k best seeds)
 *   ids_out    device, int32[nq][k]; dists_out device, float[nq][k]: the k
 *              best (d32, id) of R in ascending order, padded with (-1, +inf)
 * Distances are d32 (squared Euclidean, canonical FP32 order), which also
 * orders R; ties go to the smaller id.  The per-query state (visited ids,
 * rank list) lives in LDS and must fit 64 KiB: roughly
 * 8 (ns + rounds k kg) + 8 (k + k kg) + 4 D bytes; larger requests return
 * KNNG_ERR_UNSUPPORTED.  NaN/Inf inputs are not checked.
 */
int knng_search(const float* data, int64_t n, int32_t D, const int32_t* graph, int32_t kg,
                const float* queries, int64_t nq, const int32_t* seeds, int32_t ns, int32_t k,
                int32_t rounds, int32_t* ids_out, float* dists_out, hipStream_t stream);

/*
 * knng_to_u8 -- the lossless uint8 copy of data whose values are all integers
 * in [0, 255] (SIFT-like descriptors stored as float).
 *   data   device, float[count]; out device, uint8[count]
 * Values that are not integers in [0, 255] (or NaN/Inf) give
 * KNNG_ERR_INVALID_ARG and leave out untouched.
 */
int knng_to_u8(const float* data, int64_t count, uint8_t* out, hipStream_t stream);

/*
 * knng_search_u8 -- knng_search_ex over the uint8 copy of integer data
 * (knng_to_u8): a quarter of the bytes per distance.  Each byte is the FP32
 * value exactly, so ids, distances and the work report equal those of
 * knng_search_ex on the FP32 rows.
 *   data8  device, uint8[n][D] (16-byte aligned)
 */
int knng_search_u8(const uint8_t* data8, int64_t n, int32_t D, const int32_t* graph, int32_t kg,
                   const float* queries, int64_t nq, const int32_t* seeds, int32_t ns, int32_t k,
                   int32_t rounds, int32_t* ids_out, float* dists_out, uint64_t* work_out,
                   hipStream_t stream);

/*
 * knng_search_ex -- knng_search with a work report.
 *   work_out   host, uint64[2], nullable: [0] distances taken over all queries
 *              (seeds included), [1] nodes expanded (each reads kg graph
 *              entries); the bytes the search reads follow from them.
 */
int knng_search_ex(const float* data, int64_t n, int32_t D, const int32_t* graph, int32_t kg,
                   const float* queries, int64_t nq, const int32_t* seeds, int32_t ns, int32_t k,
                   int32_t rounds, int32_t* ids_out, float* dists_out, uint64_t* work_out,
                   hipStream_t stream);

/*
 * Inverted index for search seeds (Sec. 4.1-4.2, Eqns 1-3).  A point is
 * encoded by two-stage residue vector quantisation (Eqn 1 with two terms): c1
 * is its nearest word in the first vocabulary, c2 the nearest word of the
 * second to its residue x - w1[c1]; the index key is c1 * K2 + c2.  All
 * quantiser arithmetic is FP64: squared distances add each term with a fused
 * multiply-add in increasing dimension order, and the lowest word index wins
 * among equal distances.  Vocabularies are row-major double[K][D].
 *
 * knng_rvq_train -- train both vocabularies by Lloyd k-means: stage 1 on the
 * sample rows, stage 2 on their stage-1 residues.  Each stage starts from the
 * given sample positions, then repeats (update, assign) at most `iters` times,
 * stopping after a round that changes no code.  The update adds the members of
 * each word in increasing sample position and divides by their count; a word
 * without members keeps its value.
 *   data        device, float[n][D] (16-byte aligned)
 *   train_ids   device, int32[m]: sample rows of data, 1 <= m <= n
 *   init1/init2 device, int32[K1] / int32[K2]: starting words as positions in
 *               the sample, in [0, m); K1, K2 in [1, 256]
 *   words1_out  device, double[K1][D]; words2_out device, double[K2][D]
 *   codes1_out, codes2_out  device, int32[m], nullable: final codes of the sample
 *   rounds_out  host, int32[2], nullable: update rounds taken per stage
 * Out-of-range ids or positions give KNNG_ERR_INVALID_ARG before any output
 * is written.  NaN/Inf inputs are not checked.
 */
int knng_rvq_train(const float* data, int64_t n, int32_t D, const int32_t* train_ids, int64_t m,
                   int32_t K1, int32_t K2, const int32_t* init1, const int32_t* init2,
                   int32_t iters, double* words1_out, double* words2_out, int32_t* codes1_out,
                   int32_t* codes2_out, int32_t* rounds_out, hipStream_t stream);

/*
 * knng_ivf_build -- encode every point and build the inverted lists.
 *   keys_out     device, int32[n], nullable: c1 * K2 + c2 of every point
 *   offsets_out  device, int32[K1 K2 + 1]: list I is ids_out[offsets[I],
 *                offsets[I + 1])
 *   ids_out      device, int32[n]: point ids grouped by key, increasing
 *                within each list
 */
int knng_ivf_build(const float* data, int64_t n, int32_t D, const double* words1, int32_t K1,
                   const double* words2, int32_t K2, int32_t* keys_out, int32_t* offsets_out,
                   int32_t* ids_out, hipStream_t stream);

/*
 * knng_ivf_seeds -- cascaded seeds of a batch of queries (Eqn 3).  Per query
 * q, term 1 = (q.q - 2 w1.q) + w1.w1 is ranked over the first vocabulary; under
 * the n1 best words every key I gets d(q, I) = term 1 + ((2 w1.w2 + w2.w2) -
 * 2 w2.q), which equals |q - w1 - w2|^2 (Eqn 2); keys are ranked by
 * (d(q, I), I) and their lists walked in that order, their ids taken as seeds
 * until ns are taken.  Dot products are FP64 fma chains in dimension order
 * over the FP32 query.
 *   queries      device, float[nq][D]
 *   offsets      device, int32[K1 K2 + 1], ids device, int32[n_ids]: the
 *                lists of knng_ivf_build; malformed offsets (not rising from
 *                0 to n_ids) give KNNG_ERR_INVALID_ARG
 *   n1           first-stage words kept, 1 <= n1 <= K1, n1 K2 <= 4096
 *   seeds_out    device, int32[nq][ns], padded with -1 when the visited lists
 *                hold fewer than ns ids; suitable as knng_search's seeds
 * queries and seeds_out may be null when nq = 0, ids when n_ids = 0.
 */
int knng_ivf_seeds(const float* queries, int64_t nq, int32_t D, const double* words1, int32_t K1,
                   const double* words2, int32_t K2, const int32_t* offsets, const int32_t* ids,
                   int64_t n_ids, int32_t n1, int32_t ns, int32_t* seeds_out,
                   hipStream_t stream);

/*
 * knng_release_workspace -- free the scratch blocks the library keeps cached
 * for the current device (none is in use when no call is running).
 */
void knng_release_workspace(void);

/* Static description of a status code. */
const char* knng_status_string(int status);

/* Message of the last failed call on this thread ("" if none). */
const char* knng_last_error(void);

/* ABI version of this library (major*100 + minor). */
int knng_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KNNG_H */
