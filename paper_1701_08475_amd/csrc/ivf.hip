// Inverted index from two-stage residue vector quantisation (Sec. 4.1-4.2,
// Eqns 1-3) and the cascaded search seeds it supplies.
//
//  - k_nearest: the nearest vocabulary word of each point in FP64, every term
//    of the squared distance added by a fused multiply-add in dimension
//    order, the lowest index among equal distances.  One thread per point;
//    the words pass through LDS in double-buffered tiles of 32 words x 16
//    dimensions, stored dimension-major so all lanes read the same two words
//    (a broadcast).  A point is a row of X (stage 1) or its stage-1 residue
//    x - w1[c1] (stage 2), formed on the fly, with vector loads when the
//    rows allow.
//  - Lloyd's update: the training positions are bucketed by code with a
//    stable counting sort, then one thread per (word, dimension) adds its
//    members in increasing position (their row ids staged in LDS 64 at a
//    time) and divides by their count.  When the training rows are integers
//    of magnitude at most 2^24 (checked on the device once per call), every
//    first-stage sum is an exact integer below 2^53 and eight wavefronts
//    split a word's members; the result is the same bits.
//  - Inverted lists: a stable radix sort of the keys, 8 bits a pass, carries
//    the point ids, so every list comes out in increasing id order.
//  - Seeds: one workgroup per query computes the query's dot products with
//    all words, term 1 of every first-stage word, the n1 best and d(q, I) of
//    the n1 x K2 keys under them; it takes the lists in (d, key) order --
//    the first ones by repeated block minimum, the rest (rarely needed) from
//    a sort with a scan of the list sizes -- until ns ids are taken.
#include "knng_internal.hpp"
#include "wave.hpp"

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>

namespace knng {
namespace {

constexpr int kNearThreads = 256;
constexpr int kTJ = 32;  // words per LDS tile
constexpr int kDC = 16;  // dimensions per LDS tile
constexpr int kSortB = 2048;  // elements per block of the stable digit sort
constexpr int kSortT = 256;
constexpr int kSeedThreads = 256;

// codes[p] <- the nearest word of W [K][D] to point p, whose value is
// X[row(p)][d] - (W1 ? W1[c1[p]][d] : 0) with row(p) = rows ? rows[p] : p.
// changed (nullable) counts the points whose code differs from codes[p] on
// entry; codes (nullable) is written; key_out (nullable) <- c1[p] * K2 + code.
// VEC: D % 16 == 0 and 16-byte aligned rows, so each slice of a point is read
// as four float4 (and its stage-1 word as eight double2) instead of 16 loads
// of single elements, each touching 64 cache lines per wave.
// Word groups (few points): block row blockIdx.y takes word tiles
// [y tpg, (y+1) tpg) and writes its best (distance, word) to pbest / pidx
// [gridDim.y][m]; k_nearest_reduce then takes the minimum over the groups in
// word order.  With pbest == nullptr the block takes every word.
template <bool VEC>
__global__ __launch_bounds__(kNearThreads) void k_nearest(
    const float* __restrict__ X, int D, const int32_t* __restrict__ rows, int64_t m,
    const double* __restrict__ W1, const int32_t* __restrict__ c1, const double* __restrict__ W,
    int K, int32_t* __restrict__ codes, int32_t* __restrict__ changed, int32_t* __restrict__ key_out,
    int K2, int tpg, double* __restrict__ pbest, int32_t* __restrict__ pidx) {
    // two LDS buffers: the slice of step s+1 is loaded while step s computes
    __shared__ __align__(16) double s_w[2][kDC][kTJ];
    constexpr int kPer = kDC * kTJ / kNearThreads;  // tile values loaded per thread
    static_assert(kDC * kTJ % kNearThreads == 0, "whole tile per pass of the block");
    const int64_t p = blockIdx.x * static_cast<int64_t>(kNearThreads) + threadIdx.x;
    const bool live = p < m;
    const int64_t row = live ? (rows != nullptr ? rows[p] : p) : 0;
    const float* x = X + row * D;
    const int32_t base = (W1 != nullptr && live) ? c1[p] : 0;
    const double* r = W1 != nullptr ? W1 + static_cast<size_t>(base) * D : nullptr;
    double best = 0.0;
    int bj = 0;
    bool have = false;  // best holds a word of this block's range
    // steps run over (word tile j0, dimension slice d0), d0 fastest
    const int nd = (D + kDC - 1) / kDC;
    const int ntiles = (K + kTJ - 1) / kTJ;
    const int t0 = pbest != nullptr ? static_cast<int>(blockIdx.y) * tpg : 0;
    const int t1 = pbest != nullptr ? min(t0 + tpg, ntiles) : ntiles;
    const int nsteps = (t1 - t0) * nd;
    auto fetch = [&](int st, double (&q)[kPer]) {
        const int j0 = (t0 + st / nd) * kTJ, d0 = (st % nd) * kDC;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + i * kNearThreads;
            const int dd = e / kTJ, j = e % kTJ;
            const int d = d0 + dd, jj = j0 + j;
            q[i] = (d < D && jj < K) ? W[static_cast<size_t>(jj) * D + d] : 0.0;
        }
    };
    auto stash = [&](int buf, const double (&q)[kPer]) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + i * kNearThreads;
            s_w[buf][e / kTJ][e % kTJ] = q[i];
        }
    };
    double q[kPer];
    fetch(0, q);
    stash(0, q);
    __syncthreads();
    double acc[kTJ];
    for (int st = 0; st < nsteps; ++st) {
        const int j0 = (t0 + st / nd) * kTJ, d0 = (st % nd) * kDC;
        if (d0 == 0) {
#pragma unroll
            for (int j = 0; j < kTJ; ++j) acc[j] = 0.0;
        }
        if (st + 1 < nsteps) fetch(st + 1, q);
        double v[kDC];
        if constexpr (VEC) {  // whole slices: d0 + kDC <= D
#pragma unroll
            for (int i = 0; i < kDC / 4; ++i) {
                const float4 f = *reinterpret_cast<const float4*>(x + d0 + 4 * i);
                v[4 * i] = static_cast<double>(f.x);
                v[4 * i + 1] = static_cast<double>(f.y);
                v[4 * i + 2] = static_cast<double>(f.z);
                v[4 * i + 3] = static_cast<double>(f.w);
            }
            if (r != nullptr) {
#pragma unroll
                for (int i = 0; i < kDC / 2; ++i) {
                    const double2 w1 = *reinterpret_cast<const double2*>(r + d0 + 2 * i);
                    v[2 * i] = __dsub_rn(v[2 * i], w1.x);
                    v[2 * i + 1] = __dsub_rn(v[2 * i + 1], w1.y);
                }
            }
        } else {
#pragma unroll
            for (int dd = 0; dd < kDC; ++dd) {
                const int d = d0 + dd;
                double xv = 0.0;
                if (live && d < D) {
                    xv = static_cast<double>(x[d]);
                    if (r != nullptr) xv = __dsub_rn(xv, r[d]);
                }
                v[dd] = xv;
            }
        }
        const int buf = st & 1;
        // padding dimensions give t = 0 and leave the sums unchanged
#pragma unroll
        for (int dd = 0; dd < kDC; ++dd) {
#pragma unroll
            for (int j = 0; j < kTJ; j += 2) {
                const double2 w = *reinterpret_cast<const double2*>(&s_w[buf][dd][j]);
                const double t0 = __dsub_rn(v[dd], w.x);
                const double t1 = __dsub_rn(v[dd], w.y);
                acc[j] = __fma_rn(t0, t0, acc[j]);
                acc[j + 1] = __fma_rn(t1, t1, acc[j + 1]);
            }
        }
        if (d0 + kDC >= D) {  // last slice of the word tile
#pragma unroll
            for (int j = 0; j < kTJ; ++j)
                if (j0 + j < K && (!have || acc[j] < best)) {
                    best = acc[j];
                    bj = j0 + j;
                    have = true;
                }
        }
        if (st + 1 < nsteps) stash(buf ^ 1, q);
        __syncthreads();
    }
    if (pbest != nullptr) {  // this group's best; k_nearest_reduce finishes
        if (live) {
            pbest[blockIdx.y * m + p] = best;
            pidx[blockIdx.y * m + p] = bj;
        }
        return;
    }
    if (changed != nullptr) {
        const bool ch = live && codes[p] != bj;
        const uint64_t mask = __ballot(ch);
        if (lane_id() == 0 && mask != 0) atomicAdd(changed, static_cast<int32_t>(__popcll(mask)));
    }
    if (!live) return;
    if (codes != nullptr) codes[p] = bj;
    if (key_out != nullptr) key_out[p] = base * K2 + bj;
}

// The nearest word over G word groups, taken in group (= word) order with a
// strict comparison, so the lowest word index wins among equal distances;
// then as the epilogue of k_nearest.
__global__ __launch_bounds__(256) void k_nearest_reduce(
    int64_t m, int G, const double* __restrict__ pbest, const int32_t* __restrict__ pidx,
    const int32_t* __restrict__ c1, int32_t* __restrict__ codes, int32_t* __restrict__ changed,
    int32_t* __restrict__ key_out, int K2) {
    const int64_t p = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const bool live = p < m;
    double best = 0.0;
    int bj = 0;
    if (live) {
        best = pbest[p];
        bj = pidx[p];
        for (int g = 1; g < G; ++g)
            if (pbest[g * m + p] < best) {
                best = pbest[g * m + p];
                bj = pidx[g * m + p];
            }
    }
    if (changed != nullptr) {
        const bool ch = live && codes[p] != bj;
        const uint64_t mask = __ballot(ch);
        if (lane_id() == 0 && mask != 0) atomicAdd(changed, static_cast<int32_t>(__popcll(mask)));
    }
    if (!live) return;
    if (codes != nullptr) codes[p] = bj;
    if (key_out != nullptr) key_out[p] = (c1 != nullptr ? c1[p] : 0) * K2 + bj;
}

// W[j] <- value of training position init[j] (as in k_nearest).
__global__ void k_init_words(const float* __restrict__ X, int D, const int32_t* __restrict__ rows,
                             const double* __restrict__ W1, const int32_t* __restrict__ c1,
                             const int32_t* __restrict__ init, double* __restrict__ W) {
    const int j = blockIdx.x;
    const int32_t p = init[j];
    const int64_t row = rows[p];
    for (int d = threadIdx.x; d < D; d += blockDim.x) {
        double v = static_cast<double>(X[row * D + d]);
        if (W1 != nullptr) v = __dsub_rn(v, W1[static_cast<size_t>(c1[p]) * D + d]);
        W[static_cast<size_t>(j) * D + d] = v;
    }
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t count, int32_t v) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        a[i] = v;
}

// bad <- 1 if some a[i] lies outside [lo, hi).
__global__ void k_check_range(const int32_t* __restrict__ a, int64_t count, int64_t lo, int64_t hi,
                              int32_t* __restrict__ bad) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        if (a[i] < lo || a[i] >= hi) atomicOr(bad, 1);
}

// flag <- 1 if a value of a training row is not an integer of magnitude at
// most 2^24 (NaN included).  Ids outside [0, n) are skipped: the range check
// reports them.  One ballot per wave and at most one atomic per wave.
__global__ void k_check_integral(const float* __restrict__ X, int64_t n, int D,
                                 const int32_t* __restrict__ rows, int64_t m,
                                 int32_t* __restrict__ flag) {
    const int64_t total = m * D;
    bool off = false;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t r = i / D;
        const int32_t id = rows[r];
        if (id < 0 || id >= n) continue;
        const float v = X[static_cast<int64_t>(id) * D + (i - r * D)];
        if (!(fabsf(v) <= 16777216.0f) || v != rintf(v)) off = true;
    }
    if (__ballot(off) != 0 && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// bad <- 1 unless off[0] = 0, off is non-decreasing and off[nk] = total.
__global__ void k_check_offsets(const int32_t* __restrict__ off, int nk, int64_t total,
                                int32_t* __restrict__ bad) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nk; i += gridDim.x * blockDim.x)
        if (off[i + 1] < off[i] || (i == 0 && off[0] != 0) || (i == nk - 1 && off[nk] != total))
            atomicOr(bad, 1);
}

// ------------------------------------------------------ stable digit sort
// hist[dig * nb + b] <- elements of block b whose digit (key >> shift) & 255 is dig.
__global__ __launch_bounds__(kSortT) void k_digit_count(const int32_t* __restrict__ key, int64_t m,
                                                        int shift, int nb, int32_t* __restrict__ hist) {
    __shared__ int32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kSortB;
    for (int i = threadIdx.x; i < kSortB; i += kSortT) {
        const int64_t e = b0 + i;
        if (e < m) atomicAdd(&cnt[(key[e] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[static_cast<int64_t>(threadIdx.x) * nb + blockIdx.x] = cnt[threadIdx.x];
}

// In-place exclusive prefix sum of a[0, T) (one workgroup).
__global__ __launch_bounds__(1024) void k_scan_excl(int32_t* __restrict__ a, int64_t T) {
    __shared__ int32_t part[1024];
    const int64_t per = (T + 1023) / 1024;
    const int64_t lo = threadIdx.x * per;
    const int64_t hi = lo + per < T ? lo + per : T;
    int32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += a[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t v = threadIdx.x >= static_cast<unsigned>(off) ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0;
    for (int64_t i = lo; i < hi; ++i) {
        const int32_t v = a[i];
        a[i] = run;
        run += v;
    }
}

// Stable scatter by digit: block b places its elements, in order, at the
// scanned bases of hist.  val (nullable) defaults to the element index.
// Within a wave, lanes of equal digit are ranked by a match mask built from
// eight ballots; the block's four waves take their turn in order.
__global__ __launch_bounds__(kSortT) void k_digit_scatter(
    const int32_t* __restrict__ key, const int32_t* __restrict__ val, int64_t m, int shift, int nb,
    const int32_t* __restrict__ hist, int32_t* __restrict__ key_out, int32_t* __restrict__ val_out) {
    __shared__ int32_t base[256];
    base[threadIdx.x] = hist[static_cast<int64_t>(threadIdx.x) * nb + blockIdx.x];
    __syncthreads();
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kSortB;
    for (int t0 = 0; t0 < kSortB; t0 += kSortT) {
        const int64_t e = b0 + t0 + threadIdx.x;
        const bool ok = e < m;
        const int32_t k = ok ? key[e] : 0;
        const int32_t v = ok ? (val != nullptr ? val[e] : static_cast<int32_t>(e)) : 0;
        const int dig = (k >> shift) & 255;
        uint64_t same = __ballot(ok);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bb = __ballot((dig >> bit) & 1);
            same &= ((dig >> bit) & 1) ? bb : ~bb;
        }
        const int rank = __popcll(same & ((1ull << lane) - 1ull));
        const int cnt = __popcll(same);
        for (int w = 0; w < kSortT / kWave; ++w) {
            if (wave == w && ok) {
                const int32_t pos = base[dig] + rank;
                key_out[pos] = k;
                val_out[pos] = v;
                if (rank == cnt - 1) base[dig] = pos + 1;
            }
            __syncthreads();
        }
    }
}

// off[kk] <- first position whose sorted key is >= kk, kk in [0, nk]
// (off[nk] = m).  Keys in [0, nk), ascending.
__global__ void k_key_offsets(const int32_t* __restrict__ skey, int64_t m, int nk,
                              int32_t* __restrict__ off) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i <= m;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int32_t lo = i == 0 ? 0 : skey[i - 1] + 1;
        const int32_t hi = i == m ? nk : skey[i];
        for (int32_t kk = lo; kk <= hi; ++kk) off[kk] = static_cast<int32_t>(i);
    }
}

// W[j][d] <- mean of the values of the members of word j, added in
// increasing position; a word without members keeps its value.
// Grid (K, ceil(D / 64)), one wave: the row ids (and stage-1 words) of 64
// members at a time go to LDS in one load, so the in-order sum issues only
// independent row loads.  RES (stage 2: residues x - w1[c1]) is a template
// parameter: a branch on it inside the unrolled loop would make the compiler
// wait for every load before the branch, one memory latency per member.
template <bool RES>
__global__ __launch_bounds__(64) void k_word_means(
    const float* __restrict__ X, int D, const int32_t* __restrict__ rows,
    const double* __restrict__ W1, const int32_t* __restrict__ c1,
    const int32_t* __restrict__ order, const int32_t* __restrict__ woff, double* __restrict__ W) {
    __shared__ int64_t s_row[64];
    __shared__ int32_t s_w1[64];
    const int j = blockIdx.x;
    const int d = blockIdx.y * 64 + threadIdx.x;
    const int32_t a = woff[j], b = woff[j + 1];
    if (b <= a) return;  // uniform: the word keeps its value
    double s = 0.0;
    for (int32_t i0 = a; i0 < b; i0 += 64) {
        const int cnt = b - i0 < 64 ? b - i0 : 64;
        if (static_cast<int>(threadIdx.x) < cnt) {
            const int32_t p = order[i0 + threadIdx.x];
            s_row[threadIdx.x] = rows[p];
            if (RES) s_w1[threadIdx.x] = c1[p];
        }
        __syncthreads();
        if (d < D) {
#pragma unroll 8
            for (int t = 0; t < cnt; ++t) {  // loads in flight, adds in order
                double v = static_cast<double>(X[s_row[t] * D + d]);
                if (RES) v = __dsub_rn(v, W1[static_cast<size_t>(s_w1[t]) * D + d]);
                s = __dadd_rn(s, v);
            }
        }
        __syncthreads();
    }
    if (d < D) W[static_cast<size_t>(j) * D + d] = s / static_cast<double>(b - a);
}

// The same means of the first stage when every partial sum is an exact
// integer: integer rows of magnitude at most 2^24 and at most 2^29 members
// keep every sum below 2^53, so the sum is the same in any order of the
// additions.  NW wavefronts take every NW-th batch of 64 members and their
// sums are added at the end, which shortens the serial chain of a large word
// NW times.
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_word_means_exact(
    const float* __restrict__ X, int D, const int32_t* __restrict__ rows,
    const int32_t* __restrict__ order, const int32_t* __restrict__ woff, double* __restrict__ W) {
    __shared__ int64_t s_row[NW][64];
    __shared__ double s_part[NW][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = blockIdx.x;
    const int d = blockIdx.y * 64 + lane;
    const int32_t a = woff[j], b = woff[j + 1];
    if (b <= a) return;  // uniform over the block: the word keeps its value
    double s = 0.0;
    for (int32_t i0 = a + 64 * w; i0 < b; i0 += 64 * NW) {
        const int cnt = b - i0 < 64 ? b - i0 : 64;
        if (lane < cnt) s_row[w][lane] = rows[order[i0 + lane]];
        wave_lds_sync();
        if (d < D) {
#pragma unroll 8
            for (int t = 0; t < cnt; ++t) s += static_cast<double>(X[s_row[w][t] * D + d]);
        }
        wave_lds_sync();
    }
    s_part[w][lane] = s;
    __syncthreads();
    if (w == 0 && d < D) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < NW; ++q) t += s_part[q][lane];
        W[static_cast<size_t>(j) * D + d] = t / static_cast<double>(b - a);
    }
}

// -------------------------------------------------------------- seeds
// x12[j][l] = w1_j . w2_l, nw1[j] = w1_j . w1_j, nw2[l] = w2_l . w2_l (fma
// chains in dimension order) and the dimension-major copies W1T [D][K1],
// W2T [D][K2].  Grid K1, 256 threads (K2 <= 256).
__global__ __launch_bounds__(256) void k_ivf_tables(const double* __restrict__ W1, int K1,
                                                    const double* __restrict__ W2, int K2, int D,
                                                    double* __restrict__ x12, double* __restrict__ nw1,
                                                    double* __restrict__ nw2, double* __restrict__ W1T,
                                                    double* __restrict__ W2T) {
    const int j = blockIdx.x;
    const int l = threadIdx.x;
    const double* w1 = W1 + static_cast<size_t>(j) * D;
    if (l < K2) {
        const double* w2 = W2 + static_cast<size_t>(l) * D;
        double s = 0.0;
        for (int d = 0; d < D; ++d) s = __fma_rn(w1[d], w2[d], s);
        x12[static_cast<size_t>(j) * K2 + l] = s;
        if (j == 0) {
            double t = 0.0;
            for (int d = 0; d < D; ++d) t = __fma_rn(w2[d], w2[d], t);
            nw2[l] = t;
        }
        for (int d = j; d < D; d += gridDim.x) W2T[static_cast<size_t>(d) * K2 + l] = w2[d];
    }
    if (l == 0) {
        double t = 0.0;
        for (int d = 0; d < D; ++d) t = __fma_rn(w1[d], w1[d], t);
        nw1[j] = t;
    }
    for (int d = l; d < D; d += blockDim.x) W1T[static_cast<size_t>(d) * K1 + j] = w1[d];
}

__device__ __forceinline__ bool dk_less(double da, int32_t ka, double db, int32_t kb) {
    return da < db || (da == db && ka < kb);
}

// Ascending bitonic sort of (d, k) pairs, N a power of two (whole block).
__device__ void bitonic_dk(double* d, int32_t* k, int N) {
    for (int size = 2; size <= N; size <<= 1)
        for (int stride = size >> 1; stride >= 1; stride >>= 1) {
            for (int i = threadIdx.x; i < (N >> 1); i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                if (dk_less(d[hi], k[hi], d[lo], k[lo]) == up) {
                    const double td = d[lo];
                    d[lo] = d[hi];
                    d[hi] = td;
                    const int32_t tk = k[lo];
                    k[lo] = k[hi];
                    k[hi] = tk;
                }
            }
            __syncthreads();
        }
}

struct SeedShape {
    int p1;  // power of two >= K1
    int p2;  // power of two >= n1 * K2
};

size_t seed_lds_bytes(const SeedShape& sh, int D) {
    return 12 * static_cast<size_t>(sh.p2) + 8 * static_cast<size_t>(D) + 2 * 8 * 256 +
           12 * static_cast<size_t>(sh.p1);
}

__global__ __launch_bounds__(kSeedThreads) void k_ivf_seeds(
    const float* __restrict__ Q, int D, const double* __restrict__ W1T, int K1,
    const double* __restrict__ W2T, int K2, const double* __restrict__ x12,
    const double* __restrict__ nw1, const double* __restrict__ nw2, const int32_t* __restrict__ off,
    const int32_t* __restrict__ ids, int n1, int ns, SeedShape sh, int32_t* __restrict__ seeds) {
    extern __shared__ __align__(16) unsigned char smem[];
    double* sd = reinterpret_cast<double*>(smem);         // [p2] key distances
    int32_t* sc = reinterpret_cast<int32_t*>(smem);        // [p2] list-size scan (after the sort)
    int32_t* sk = reinterpret_cast<int32_t*>(sd + sh.p2);  // [p2] keys
    double* q = reinterpret_cast<double*>(sk + sh.p2);     // [D]
    double* ip1 = q + D;                                   // [256] w1.q, then term 1
    double* ip2 = ip1 + 256;                               // [256] w2.q
    double* fd = ip2 + 256;                                // [p1] term 1, sorted
    int32_t* fk = reinterpret_cast<int32_t*>(fd + sh.p1);  // [p1] first-stage words, sorted
    __shared__ double s_qq;
    __shared__ int32_t s_part[kSeedThreads];

    const int tid = threadIdx.x;
    const int64_t qi = blockIdx.x;
    for (int d = tid; d < D; d += kSeedThreads) q[d] = static_cast<double>(Q[qi * D + d]);
    __syncthreads();
    if (tid < K1) {
        double s = 0.0;
        for (int d = 0; d < D; ++d) s = __fma_rn(W1T[static_cast<size_t>(d) * K1 + tid], q[d], s);
        ip1[tid] = s;
    }
    if (tid < K2) {
        double s = 0.0;
        for (int d = 0; d < D; ++d) s = __fma_rn(W2T[static_cast<size_t>(d) * K2 + tid], q[d], s);
        ip2[tid] = s;
    }
    if (tid == 0) {
        double s = 0.0;
        for (int d = 0; d < D; ++d) s = __fma_rn(q[d], q[d], s);
        s_qq = s;
    }
    __syncthreads();
    // term 1 = (q.q - 2 w1.q) + w1.w1 of every first-stage word
    if (tid < K1) ip1[tid] = __dadd_rn(__dsub_rn(s_qq, __dmul_rn(2.0, ip1[tid])), nw1[tid]);
    __syncthreads();
    for (int j = tid; j < sh.p1; j += kSeedThreads) {
        fd[j] = j < K1 ? ip1[j] : __longlong_as_double(0x7ff0000000000000ll);
        fk[j] = j < K1 ? j : INT_MAX;
    }
    __syncthreads();
    bitonic_dk(fd, fk, sh.p1);
    // d(q, I) = term 1 + ((2 w1.w2 + w2.w2) - 2 w2.q) of the keys under the n1 best
    const int M = n1 * K2;
    const int nk = K1 * K2;
    for (int e = tid; e < sh.p2; e += kSeedThreads) {
        const int a = e / K2, l = e % K2;
        const int j = e < M ? fk[a] : INT_MAX;
        if (j < K1) {  // a padding word can only rank this high if term 1 is NaN
            const double t2 = __dsub_rn(
                __dadd_rn(__dmul_rn(2.0, x12[static_cast<size_t>(j) * K2 + l]), nw2[l]),
                __dmul_rn(2.0, ip2[l]));
            sd[e] = __dadd_rn(ip1[j], t2);
            sk[e] = j * K2 + l;
        } else {
            sd[e] = __longlong_as_double(0x7ff0000000000000ll);
            sk[e] = INT_MAX;
        }
    }
    __syncthreads();
    // The first lists by repeated block minimum of (d, key): a handful of
    // lists usually holds ns ids.  A picked key becomes (+inf, INT_MAX);
    // lists are taken in the order a full sort would give, so the rest
    // (after kPicks lists) continues from a sort of what is left.
    constexpr int kPicks = 32;
    constexpr int kWaves = kSeedThreads / kWave;
    __shared__ double s_md[kWaves];
    __shared__ int32_t s_mk[kWaves], s_me[kWaves];
    __shared__ int32_t s_pick[2];
    const int lane = tid & (kWave - 1), wv = tid / kWave;
    int taken = 0;
    bool exhausted = false;
    for (int it = 0; it < kPicks && taken < ns; ++it) {
        double bd = __longlong_as_double(0x7ff0000000000000ll);
        int32_t bk = INT_MAX, be = -1;
        for (int e = tid; e < M; e += kSeedThreads)
            if (dk_less(sd[e], sk[e], bd, bk)) {
                bd = sd[e];
                bk = sk[e];
                be = e;
            }
#pragma unroll
        for (int o = kWave / 2; o >= 1; o >>= 1) {
            const double od = shfl_xor_f64(bd, o);
            const int32_t ok = __shfl_xor(bk, o, kWave), oe = __shfl_xor(be, o, kWave);
            if (dk_less(od, ok, bd, bk)) {
                bd = od;
                bk = ok;
                be = oe;
            }
        }
        if (lane == 0) {
            s_md[wv] = bd;
            s_mk[wv] = bk;
            s_me[wv] = be;
        }
        __syncthreads();
        if (tid == 0) {
            int w0 = 0;
            for (int w = 1; w < kWaves; ++w)
                if (dk_less(s_md[w], s_mk[w], s_md[w0], s_mk[w0])) w0 = w;
            s_pick[0] = s_mk[w0];
            s_pick[1] = s_me[w0];
        }
        __syncthreads();
        const int32_t pk = s_pick[0], pe = s_pick[1];
        if (pk >= nk || pe < 0) {  // only padding keys are left
            exhausted = true;
            break;
        }
        const int32_t a0 = off[pk];
        const int take = min(off[pk + 1] - a0, ns - taken);
        for (int j = tid; j < take; j += kSeedThreads) seeds[qi * ns + taken + j] = ids[a0 + j];
        taken += take;
        if (tid == 0) {
            sd[pe] = __longlong_as_double(0x7ff0000000000000ll);
            sk[pe] = INT_MAX;
        }
        __syncthreads();
    }
    if (taken >= ns) return;
    if (exhausted) {
        for (int s = taken + tid; s < ns; s += kSeedThreads) seeds[qi * ns + s] = -1;
        return;
    }
    bitonic_dk(sd, sk, sh.p2);
    // inclusive scan of the list sizes in key order (sc overwrites sd)
    const int per = (sh.p2 + kSeedThreads - 1) / kSeedThreads;
    const int lo = tid * per;
    const int hi = lo + per < M ? lo + per : M;
    int32_t run = 0;
    // keys of padding words (NaN input only) count as empty lists
    auto list_size = [&](int e) { return sk[e] < nk ? off[sk[e] + 1] - off[sk[e]] : 0; };
    for (int e = lo; e < hi; ++e) run += list_size(e);
    s_part[tid] = run;
    __syncthreads();
    for (int o = 1; o < kSeedThreads; o <<= 1) {
        const int32_t v = tid >= o ? s_part[tid - o] : 0;
        __syncthreads();
        s_part[tid] += v;
        __syncthreads();
    }
    run = tid ? s_part[tid - 1] : 0;
    for (int e = lo; e < hi; ++e) {
        run += list_size(e);
        sc[e] = run;
    }
    __syncthreads();
    const int32_t total = M > 0 ? sc[M - 1] : 0;
    for (int s0 = taken + tid; s0 < ns; s0 += kSeedThreads) {
        const int s = s0 - taken;  // position among the ids of the lists not picked
        int32_t out = -1;
        if (s < total) {
            int a = 0, b = M - 1;  // first e with sc[e] > s
            while (a < b) {
                const int mid = (a + b) >> 1;
                if (sc[mid] > s) b = mid;
                else a = mid + 1;
            }
            const int32_t before = a ? sc[a - 1] : 0;
            out = ids[off[sk[a]] + (s - before)];
        }
        seeds[qi * ns + s0] = out;
    }
}

int nblocks(int64_t count, int per) { return static_cast<int>((count + per - 1) / per); }

constexpr int kMaxWordGroups = 8;

// Word groups for m points: enough blocks to fill the GPU (about 2048), at
// most one group per word tile.
int word_groups(int64_t m, int K) {
    const int nb = nblocks(m, kNearThreads);
    const int ntiles = (K + kTJ - 1) / kTJ;
    int G = 1;
    while (G < kMaxWordGroups && G < ntiles && static_cast<int64_t>(nb) * G < 2048) G <<= 1;
    return G < ntiles ? G : ntiles;
}

// Nearest word of every point (k_nearest), with vector loads when the rows
// allow them; pbest / pidx: scratch of word_groups(m, K) x m entries (unused
// when that is 1).
void nearest(const float* X, int D, const int32_t* rows, int64_t m, const double* W1,
             const int32_t* c1, const double* W, int K, int32_t* codes, int32_t* changed,
             int32_t* key_out, int K2, double* pbest, int32_t* pidx, hipStream_t s) {
    const bool vec = D % kDC == 0 && (reinterpret_cast<uintptr_t>(X) & 15u) == 0 &&
                     (W1 == nullptr || (reinterpret_cast<uintptr_t>(W1) & 15u) == 0);
    const int nb = nblocks(m, kNearThreads);
    const int G = word_groups(m, K);
    const int ntiles = (K + kTJ - 1) / kTJ;
    const int tpg = (ntiles + G - 1) / G;
    const dim3 grid(nb, G);
    double* pb = G > 1 ? pbest : nullptr;
    int32_t* pi = G > 1 ? pidx : nullptr;
    if (vec)
        k_nearest<true><<<grid, kNearThreads, 0, s>>>(X, D, rows, m, W1, c1, W, K, codes, changed,
                                                      key_out, K2, tpg, pb, pi);
    else
        k_nearest<false><<<grid, kNearThreads, 0, s>>>(X, D, rows, m, W1, c1, W, K, codes,
                                                       changed, key_out, K2, tpg, pb, pi);
    if (G > 1)
        k_nearest_reduce<<<nblocks(m, 256), 256, 0, s>>>(m, G, pbest, pidx, W1 != nullptr ? c1 : nullptr,
                                                        codes, changed, key_out, K2);
}

// Stable sort of (key, val) by the digit at shift (val nullable: index).
void digit_pass(const int32_t* key, const int32_t* val, int64_t m, int shift, int32_t* hist,
                int32_t* key_out, int32_t* val_out, hipStream_t s) {
    const int nb = nblocks(m, kSortB);
    k_digit_count<<<nb, kSortT, 0, s>>>(key, m, shift, nb, hist);
    k_scan_excl<<<1, 1024, 0, s>>>(hist, 256 * static_cast<int64_t>(nb));
    k_digit_scatter<<<nb, kSortT, 0, s>>>(key, val, m, shift, nb, hist, key_out, val_out);
}

// Scratch blocks of one call from the workspace cache, returned on exit
// (stream-ordered); at most kMaxBlocks per call.
struct Ws {
    static constexpr int kMaxBlocks = 16;
    hipStream_t s;
    void* blk[kMaxBlocks] = {};
    int nblk = 0;
    hipError_t e = hipSuccess;
    template <class T>
    T* get(size_t count) {
        void* p = nullptr;
        if (e == hipSuccess && nblk == kMaxBlocks) e = hipErrorOutOfMemory;
        if (e == hipSuccess) e = ws_malloc(&p, count * sizeof(T) + 16, s);
        if (e == hipSuccess) blk[nblk++] = p;
        return static_cast<T*>(p);
    }
    ~Ws() {
        for (int i = 0; i < nblk; ++i) ws_free(blk[i], s);
    }
};

int finish(hipError_t e, const char* what, char* err, size_t errlen) {
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
        std::snprintf(err, errlen, "%s: %s", what, hipGetErrorString(e));
        return kHip;
    }
    return kOk;
}

// One Lloyd run (R16) over the training positions; W holds the start words.
int kmeans_run(const float* X, int D, const int32_t* rows, int64_t m, const double* W1,
               const int32_t* c1, double* W, int K, int iters, int32_t* codes, int32_t* skey,
               int32_t* order, int32_t* hist, int32_t* woff, int32_t* dchanged, double* pbest,
               int32_t* pidx, bool exact, int* rounds_out, hipStream_t s, char* err,
               size_t errlen) {
    k_fill_i32<<<nblocks(m, 256) < 1024 ? nblocks(m, 256) : 1024, 256, 0, s>>>(codes, m, -1);
    nearest(X, D, rows, m, W1, c1, W, K, codes, nullptr, nullptr, 0, pbest, pidx, s);
    int rounds = 0;
    while (rounds < iters) {
        digit_pass(codes, nullptr, m, 0, hist, skey, order, s);
        k_key_offsets<<<nblocks(m + 1, 256) < 1024 ? nblocks(m + 1, 256) : 1024, 256, 0, s>>>(
            skey, m, K, woff);
        if (exact)
            k_word_means_exact<8><<<dim3(K, (D + 63) / 64), 512, 0, s>>>(X, D, rows, order, woff, W);
        else if (W1 != nullptr)
            k_word_means<true><<<dim3(K, (D + 63) / 64), 64, 0, s>>>(X, D, rows, W1, c1, order, woff, W);
        else
            k_word_means<false><<<dim3(K, (D + 63) / 64), 64, 0, s>>>(X, D, rows, W1, c1, order, woff, W);
        k_fill_i32<<<1, 64, 0, s>>>(dchanged, 1, 0);
        nearest(X, D, rows, m, W1, c1, W, K, codes, dchanged, nullptr, 0, pbest, pidx, s);
        int32_t h = 0;
        hipError_t e = hipMemcpyAsync(&h, dchanged, sizeof(h), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return finish(e, "k-means round", err, errlen);
        ++rounds;
        if (h == 0) break;
    }
    *rounds_out = rounds;
    return finish(hipSuccess, "k-means", err, errlen);
}

int read_flag(const int32_t* dflag, int32_t* h, hipStream_t s, char* err, size_t errlen,
              int count = 1) {
    hipError_t e = hipMemcpyAsync(h, dflag, sizeof(int32_t) * count, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return finish(e, "argument check", err, errlen);
}

}  // namespace

int rvq_train_run(const RvqTrainArgs& a, char* err, size_t errlen) {
    hipStream_t s = a.stream;
    const int64_t m = a.m;
    const int K = a.K1 > a.K2 ? a.K1 : a.K2;
    Ws ws{s};
    int32_t* flag = ws.get<int32_t>(2);  // [0] argument error, [1] rows not integral
    int32_t* codes1 = ws.get<int32_t>(m);
    int32_t* codes2 = ws.get<int32_t>(m);
    int32_t* skey = ws.get<int32_t>(m);
    int32_t* order = ws.get<int32_t>(m);
    int32_t* hist = ws.get<int32_t>(256 * static_cast<size_t>(nblocks(m, kSortB)));
    int32_t* woff = ws.get<int32_t>(K + 1);
    int32_t* changed = ws.get<int32_t>(1);
    const size_t ng = static_cast<size_t>(word_groups(m, K)) * m;  // word-group partials
    double* pbest = ws.get<double>(ng);
    int32_t* pidx = ws.get<int32_t>(ng);
    if (ws.e != hipSuccess) {
        std::snprintf(err, errlen, "workspace: %s", hipGetErrorString(ws.e));
        return kOom;
    }
    k_fill_i32<<<1, 64, 0, s>>>(flag, 2, 0);
    k_check_range<<<256, 256, 0, s>>>(a.train_ids, m, 0, a.n, flag);
    k_check_range<<<1, 256, 0, s>>>(a.init1, a.K1, 0, m, flag);
    k_check_range<<<1, 256, 0, s>>>(a.init2, a.K2, 0, m, flag);
    k_check_integral<<<512, 256, 0, s>>>(a.X, a.n, a.D, a.train_ids, m, flag + 1);
    int32_t hf[2] = {0, 0};
    int rc = read_flag(flag, hf, s, err, errlen, 2);
    if (rc != kOk) return rc;
    const int32_t bad = hf[0];
    // KNNG_MEANS_EXACT=0 keeps the in-order sums for integer rows too
    const char* ev = std::getenv("KNNG_MEANS_EXACT");
    const bool exact = hf[1] == 0 && m <= (int64_t{1} << 29) && !(ev != nullptr && ev[0] == '0');
    if (bad) {
        std::snprintf(err, errlen, "a training id is outside [0, n) or a starting position outside [0, m)");
        return kInvalid;
    }
    k_init_words<<<a.K1, 64, 0, s>>>(a.X, a.D, a.train_ids, nullptr, nullptr, a.init1, a.W1);
    rc = kmeans_run(a.X, a.D, a.train_ids, m, nullptr, nullptr, a.W1, a.K1, a.iters, codes1, skey,
                    order, hist, woff, changed, pbest, pidx, exact, a.rounds, s, err, errlen);
    if (rc != kOk) return rc;
    k_init_words<<<a.K2, 64, 0, s>>>(a.X, a.D, a.train_ids, a.W1, codes1, a.init2, a.W2);
    rc = kmeans_run(a.X, a.D, a.train_ids, m, a.W1, codes1, a.W2, a.K2, a.iters, codes2, skey,
                    order, hist, woff, changed, pbest, pidx, false, a.rounds + 1, s, err, errlen);
    if (rc != kOk) return rc;
    if (a.codes1 != nullptr)
        rc = finish(hipMemcpyAsync(a.codes1, codes1, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, s),
                    "copy", err, errlen);
    if (rc == kOk && a.codes2 != nullptr)
        rc = finish(hipMemcpyAsync(a.codes2, codes2, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, s),
                    "copy", err, errlen);
    if (rc == kOk) rc = finish(hipStreamSynchronize(s), "rvq train", err, errlen);
    return rc;
}

int ivf_build_run(const IvfBuildArgs& a, char* err, size_t errlen) {
    hipStream_t s = a.stream;
    const int64_t n = a.n;
    const int nk = a.K1 * a.K2;
    Ws ws{s};
    int32_t* c1 = ws.get<int32_t>(n);
    int32_t* key = a.keys_out != nullptr ? a.keys_out : ws.get<int32_t>(n);
    int32_t* k2 = ws.get<int32_t>(n);
    int32_t* v2 = ws.get<int32_t>(n);
    int32_t* k3 = ws.get<int32_t>(n);
    int32_t* hist = ws.get<int32_t>(256 * static_cast<size_t>(nblocks(n, kSortB)));
    const int G = std::max(word_groups(n, a.K1), word_groups(n, a.K2));
    const size_t ng = G > 1 ? static_cast<size_t>(G) * n : 1;  // word-group partials
    double* pbest = ws.get<double>(ng);
    int32_t* pidx = ws.get<int32_t>(ng);
    if (ws.e != hipSuccess) {
        std::snprintf(err, errlen, "workspace: %s", hipGetErrorString(ws.e));
        return kOom;
    }
    if (n > 0) {
        nearest(a.X, a.D, nullptr, n, nullptr, nullptr, a.W1, a.K1, c1, nullptr, nullptr, 0, pbest,
                pidx, s);
        nearest(a.X, a.D, nullptr, n, a.W1, c1, a.W2, a.K2, nullptr, nullptr, key, a.K2, pbest,
                pidx, s);
        if (nk <= 256) {
            digit_pass(key, nullptr, n, 0, hist, k3, a.ids_out, s);
        } else {
            digit_pass(key, nullptr, n, 0, hist, k2, v2, s);
            digit_pass(k2, v2, n, 8, hist, k3, a.ids_out, s);
        }
    }
    const int64_t cnt = n + 1;
    const int g = nblocks(cnt, 256) < 1024 ? nblocks(cnt, 256) : 1024;
    k_key_offsets<<<g, 256, 0, s>>>(k3, n, nk, a.offsets_out);
    return finish(hipStreamSynchronize(s), "ivf build", err, errlen);
}

int ivf_seeds_run(const IvfSeedArgs& a, char* err, size_t errlen) {
    hipStream_t s = a.stream;
    const int nk = a.K1 * a.K2;
    SeedShape sh;
    sh.p1 = 1;
    while (sh.p1 < a.K1) sh.p1 <<= 1;
    sh.p2 = 2;  // keeps the LDS arrays after the keys 8-byte aligned
    while (sh.p2 < a.n1 * a.K2) sh.p2 <<= 1;
    const size_t lds = seed_lds_bytes(sh, a.D);
    if (lds > kSeedLdsMax) {
        std::snprintf(err, errlen,
                      "seed state needs %zu bytes of LDS (n1 %d x K2 %d keys, D %d); at most %zu",
                      lds, a.n1, a.K2, a.D, kSeedLdsMax);
        return kUnsupported;
    }
    Ws ws{s};
    int32_t* flag = ws.get<int32_t>(1);
    double* x12 = ws.get<double>(static_cast<size_t>(nk));
    double* nw1 = ws.get<double>(a.K1);
    double* nw2 = ws.get<double>(a.K2);
    double* W1T = ws.get<double>(static_cast<size_t>(a.D) * a.K1);
    double* W2T = ws.get<double>(static_cast<size_t>(a.D) * a.K2);
    if (ws.e != hipSuccess) {
        std::snprintf(err, errlen, "workspace: %s", hipGetErrorString(ws.e));
        return kOom;
    }
    k_fill_i32<<<1, 64, 0, s>>>(flag, 1, 0);
    k_check_offsets<<<nblocks(nk, 256) < 256 ? nblocks(nk, 256) : 256, 256, 0, s>>>(
        a.offsets, nk, a.n_ids, flag);
    int32_t bad = 0;
    int rc = read_flag(flag, &bad, s, err, errlen);
    if (rc != kOk) return rc;
    if (bad) {
        std::snprintf(err, errlen, "offsets must rise from 0 to the number of listed ids");
        return kInvalid;
    }
    if (a.nq == 0) return kOk;
    k_ivf_tables<<<a.K1, 256, 0, s>>>(a.W1, a.K1, a.W2, a.K2, a.D, x12, nw1, nw2, W1T, W2T);
    k_ivf_seeds<<<static_cast<unsigned>(a.nq), kSeedThreads, lds, s>>>(
        a.Q, a.D, W1T, a.K1, W2T, a.K2, x12, nw1, nw2, a.offsets, a.ids, a.n1, a.ns, sh, a.seeds_out);
    return finish(hipStreamSynchronize(s), "ivf seeds", err, errlen);
}

}  // namespace knng
