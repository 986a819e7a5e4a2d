// Reduced-precision leaf search on the matrix cores (Alg. 1, comparison of
// every pair inside each cluster), for leaves of up to 512 points.
//
// First pass on MFMA: per leaf, the Gram matrix g = X~ X~^T of the reduced
// rows x~_i = rnd(sigma_i x_i) (BF16, FP16 or FP8-e4m3; sigma_i a power of
// two; FP32 accumulation) gives d~(i,j) = n~_i + n~_j - 2 g_ij / (sigma_i
// sigma_j), where n~_i is the squared norm of x~_i / sigma_i.  Per row the c
// smallest (d~, id) are selected exactly (wavefront radix selection), their
// distances are recomputed with the canonical FP32 d32 of the input rows,
// and the k smallest (d32, id) are kept.
//
// One workgroup (4 wavefronts) per leaf; rows in panels of PR (64 or 32).
// The panel's d~ block lives in LDS; afterwards each wavefront takes one row
// at a time (selection, re-rank, sort) without block barriers.
// MFMA v_mfma_f32_16x16x32_{bf16,f16,fp8_fp8}: lane l supplies row l%16 and
// elements 8*(l/16)..+7 of a 32-element K step, for A (row tile) and B
// (column tile) alike; result element i of lane l is (4*(l/16)+i, l%16).
#pragma once
#include "knng_internal.hpp"
#include "wave.hpp"

#include <cstdio>
#include <type_traits>

namespace knng {
namespace leafk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// element formats of the reduced copy
constexpr int kBF16 = 1, kF16 = 2, kFP8 = 3;

template <int FMT>
struct Frag;
template <>
struct Frag<kBF16> {
    using Store = uint16_t;
    static constexpr int kBytes = 2;
    __device__ static f32x4 mma(const uint4& a, const uint4& b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
    }
};
template <>
struct Frag<kF16> {
    using Store = uint16_t;
    static constexpr int kBytes = 2;
    __device__ static f32x4 mma(const uint4& a, const uint4& b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a),
                                                      __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
    }
};
template <>
struct Frag<kFP8> {
    using Store = uint8_t;
    static constexpr int kBytes = 1;
    __device__ static f32x4 mma(const uint2& a, const uint2& b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(__builtin_bit_cast(long, a),
                                                          __builtin_bit_cast(long, b), c, 0, 0, 0);
    }
};

// 8 elements of a row (16-bit formats: 16 bytes; FP8: 8 bytes)
template <int FMT>
using FragVec = typename std::conditional<FMT == kFP8, uint2, uint4>::type;

template <int FMT>
__device__ __forceinline__ FragVec<FMT> load_frag(const uint8_t* rowp, bool ok) {
    FragVec<FMT> v{};
    if (ok) v = *reinterpret_cast<const FragVec<FMT>*>(rowp);
    return v;
}

// Unsigned 32-bit key with the order of a float.
__device__ __forceinline__ uint32_t fkey(float v) {
    v = v + 0.0f;
    const uint32_t u = __float_as_uint(v);
    return (u >> 31) ? ~u : (u | 0x80000000u);
}

// d32 of rows a and b of X: per 32-dimension block the sequential fused sum
// of squared differences, blocks added in order (the canonical FP32 distance).
template <bool VEC4>
__device__ __forceinline__ float d32_rows(const float* __restrict__ xa, const float* __restrict__ xb,
                                          int D) {
    float tot = 0.f;
    for (int d0 = 0; d0 < D; d0 += 32) {
        const int dn = D - d0 < 32 ? D - d0 : 32;
        float blk = 0.f;
        if constexpr (VEC4) {
            for (int dd = 0; dd < dn; dd += 4) {
                const float4 p = *reinterpret_cast<const float4*>(xa + d0 + dd);
                const float4 q = *reinterpret_cast<const float4*>(xb + d0 + dd);
                float df = p.x - q.x;
                blk = __fmaf_rn(df, df, blk);
                df = p.y - q.y;
                blk = __fmaf_rn(df, df, blk);
                df = p.z - q.z;
                blk = __fmaf_rn(df, df, blk);
                df = p.w - q.w;
                blk = __fmaf_rn(df, df, blk);
            }
        } else {
            for (int dd = 0; dd < dn; ++dd) {
                const float df = xa[d0 + dd] - xb[d0 + dd];
                blk = __fmaf_rn(df, df, blk);
            }
        }
        tot = tot + blk;
    }
    return tot;
}

// The leaf's ids into LDS in ascending order, with their norms and scales:
// a stable rank sort (the rank of entry j counts smaller ids, and equal ids
// before j, so it is a permutation of 0..m-1 whatever perm holds).  Position
// order is then id order, and distance ties fall to the smaller id.  raw
// holds m ints of scratch; the caller synchronises before reading ids.
template <int MP>
__device__ __forceinline__ void load_leaf_sorted(const int32_t* __restrict__ lp, int m,
                                                 int32_t* raw, int32_t* ids, float* snrm,
                                                 float* ssinv, const float* __restrict__ nrm,
                                                 const float* __restrict__ sinv) {
    const int tid = threadIdx.x;
    for (int j = tid; j < m; j += 256) raw[j] = lp[j];
    for (int j = m + tid; j < MP; j += 256) {
        ids[j] = 0;
        snrm[j] = 0.f;
        ssinv[j] = 0.f;
    }
    __syncthreads();
    for (int j = tid; j < m; j += 256) {
        const int32_t id = raw[j];
        int r = 0;
        for (int i = 0; i < m; ++i) {
            const int32_t o = raw[i];
            r += (o < id || (o == id && i < j)) ? 1 : 0;
        }
        ids[r] = id;
        snrm[r] = nrm[id];
        ssinv[r] = sinv[id];
    }
}

// EXACT: the first pass is exact (integer data that the format holds exactly,
// with every product and partial sum below 2^24), so d~ == d32 and the
// candidates are the k best directly.  VEC4: D % 4 == 0.
template <int FMT, int MP, int PR, bool EXACT, bool VEC4>
__global__ __launch_bounds__(256) void k_leaf_mfma(
    const float* __restrict__ X, const uint8_t* __restrict__ Xr, int64_t n, int D, int Dp,
    const float* __restrict__ nrm, const float* __restrict__ sinv, int k, int c,
    const int32_t* __restrict__ perm, const LeafRec* __restrict__ leaves,
    int32_t* __restrict__ cand_ids, float* __restrict__ cand_d,
    unsigned long long* __restrict__ pairs) {
    using F = Frag<FMT>;
    constexpr int NT = MP / 16;            // column tiles
    constexpr int RTP = PR / 16;           // row tiles per panel
    constexpr int WPR = 4 / RTP;           // waves per row tile
    constexpr int AT = NT / WPR;           // column tiles per wave
    constexpr int R = MP / kWave;          // keys per lane in the selection
    constexpr int CMAX = 128;              // candidates per row (upper bound)
    static_assert(R >= 1 && AT >= 1, "tile shape");

    __shared__ float dist[PR][MP + 1];     // d~ of the panel; a row's slots then hold d32
    __shared__ int16_t sel[4][CMAX];       // selected positions of the row a wave works on
    __shared__ int32_t ids[MP];
    __shared__ float snrm[MP], ssinv[MP];

    const LeafRec lf = leaves[blockIdx.x];
    const int m = lf.size;
    const size_t base = static_cast<size_t>(lf.tree) * n + lf.start;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    load_leaf_sorted<MP>(perm + base, m, reinterpret_cast<int32_t*>(&dist[0][0]), ids, snrm, ssinv,
                         nrm, sinv);
    if (tid == 0 && pairs != nullptr)
        atomicAdd(pairs, static_cast<unsigned long long>(m) * static_cast<unsigned long long>(m - 1));
    __syncthreads();
    const int cc = EXACT ? k : c;          // candidates wanted per row
    const int ce = cc < m - 1 ? cc : m - 1;
    const size_t rstride = static_cast<size_t>(Dp) * F::kBytes;
    const int rt = wv % RTP, cp = wv / RTP;
    const int kg = lane >> 4;

    for (int p0 = 0; p0 < m; p0 += PR) {
        // ---- Gram of the panel rows against every column, on MFMA; the
        // fragments of the next K step are loaded before this step's MFMAs
        const int arow = p0 + rt * 16 + (lane & 15);
        const uint8_t* ap = Xr + static_cast<size_t>(ids[arow < m ? arow : 0]) * rstride +
                            static_cast<size_t>(8 * kg) * F::kBytes;
        const uint8_t* bp[AT];
        bool bok[AT];
#pragma unroll
        for (int t = 0; t < AT; ++t) {
            const int bcol = (cp + t * WPR) * 16 + (lane & 15);
            bok[t] = bcol < m;
            bp[t] = Xr + static_cast<size_t>(ids[bcol < m ? bcol : 0]) * rstride +
                    static_cast<size_t>(8 * kg) * F::kBytes;
        }
        f32x4 acc[AT];
#pragma unroll
        for (int t = 0; t < AT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        FragVec<FMT> a = load_frag<FMT>(ap, arow < m);
        FragVec<FMT> b[AT];
#pragma unroll
        for (int t = 0; t < AT; ++t) b[t] = load_frag<FMT>(bp[t], bok[t]);
        for (int k0 = 0; k0 < Dp; k0 += 32) {
            const size_t nx = static_cast<size_t>(k0 + 32) * F::kBytes;
            const bool more = k0 + 32 < Dp;
            const FragVec<FMT> an = load_frag<FMT>(ap + nx, more && arow < m);
            FragVec<FMT> bn[AT];
#pragma unroll
            for (int t = 0; t < AT; ++t) bn[t] = load_frag<FMT>(bp[t] + nx, more && bok[t]);
#pragma unroll
            for (int t = 0; t < AT; ++t) acc[t] = F::mma(a, b[t], acc[t]);
            a = an;
#pragma unroll
            for (int t = 0; t < AT; ++t) b[t] = bn[t];
        }
        // ---- d~ into LDS
#pragma unroll
        for (int t = 0; t < AT; ++t) {
            const int col = (cp + t * WPR) * 16 + (lane & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int rl = rt * 16 + 4 * kg + i;  // panel-local row
                const int row = p0 + rl;
                float v = __int_as_float(0x7f800000);
                if (row < m && col < m)
                    v = snrm[row] + snrm[col] - 2.f * acc[t][i] * (ssinv[row] * ssinv[col]);
                dist[rl][col] = v;
            }
        }
        __syncthreads();
        // ---- per row (one wave): exact top-ce by (d~, position), re-rank, top k
        const int rows = m - p0 < PR ? m - p0 : PR;
        for (int rl = wv; rl < rows; rl += 4) {
            const int row = p0 + rl;
            uint32_t key[R];
            bool valid[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int col = r * kWave + lane;
                valid[r] = col < m && col != row;
                key[r] = valid[r] ? fkey(dist[rl][col]) : 0xffffffffu;
            }
            // radix selection of the key of rank ce-1
            uint32_t prefix = 0u;
            int rem = ce - 1;
            for (int bit = 31; bit >= 0 && ce > 0; --bit) {
                const uint32_t hi = bit == 31 ? 0u : (0xffffffffu << (bit + 1));
                int zeros = 0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const bool in = valid[r] && ((key[r] & hi) == (prefix & hi));
                    zeros += __popcll(__ballot(in && ((key[r] >> bit) & 1u) == 0u));
                }
                if (rem >= zeros) {
                    rem -= zeros;
                    prefix |= 1u << bit;
                }
            }
            // keys < prefix, and the first rem+1 keys == prefix by position
            int taken = 0, eq_seen = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const bool lt = valid[r] && key[r] < prefix;
                const bool eq = valid[r] && key[r] == prefix;
                const unsigned long long beq = __ballot(eq);
                const int eq_rank = eq_seen + __popcll(beq & ((1ull << lane) - 1ull));
                const bool take = ce > 0 && (lt || (eq && eq_rank <= rem));
                const unsigned long long bt = __ballot(take);
                if (take)
                    sel[wv][taken + __popcll(bt & ((1ull << lane) - 1ull))] =
                        static_cast<int16_t>(r * kWave + lane);
                taken += __popcll(bt);
                eq_seen += __popcll(beq);
            }
            // candidate distances: d~ itself when exact, else d32 from the rows
            float dv[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int s = lane + r * kWave;
                dv[r] = 0.f;
                if (s < ce) {
                    const int b = sel[wv][s];
                    if constexpr (EXACT) {
                        dv[r] = dist[rl][b];
                    } else {
                        dv[r] = d32_rows<VEC4>(X + static_cast<size_t>(ids[row]) * D,
                                               X + static_cast<size_t>(ids[b]) * D, D);
                    }
                }
            }
            // the wave's reads of dist[rl] are done (same wave), reuse it
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int s = lane + r * kWave;
                if (s < ce) dist[rl][s] = dv[r];
            }
            uint64_t v[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int s = lane * 2 + r;
                v[r] = s < ce ? cand_key(dist[rl][s], ids[sel[wv][s]]) : kNoKey;
            }
            wave_bitonic_sort<2>(v);
            const size_t out = (static_cast<size_t>(lf.tree) * n + ids[row]) * k;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int e = lane * 2 + r;
                if (e < k) {
                    const bool ok = v[r] != kNoKey;
                    cand_ids[out + e] = ok ? key_id(v[r]) : -1;
                    cand_d[out + e] = ok ? key_dist(v[r]) : __int_as_float(0x7f800000);
                }
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------- small leaves
// Leaves of at most MP (64, 112 or 128) points.  The Gram on MFMA fills the
// whole leaf's block of keys in LDS; then thread t owns row t and scans it
// once, keeping its CL smallest keys in a sorted register list.
//
// EXACT (first pass exact, so d~ is the integer d32 < 2^23): the 32-bit key
// (d << 7) | position orders by (distance, position) = (distance, id), and
// insertion is one min and one max per slot; the list is the answer.
// Otherwise the key is the 64-bit (order key of d~) << 32 | position, the
// list is re-ranked with d32 by streaming the leaf's FP32 rows through LDS
// in 32-dimension blocks, and the k smallest (d32, id) are kept.
template <int FMT, int MP, int CL, int KL, bool EXACT>
__global__ __launch_bounds__(256) void k_leaf_small(
    const float* __restrict__ X, const uint8_t* __restrict__ Xr, int64_t n, int D, int Dp,
    const float* __restrict__ nrm, const float* __restrict__ sinv, int k, int c,
    const int32_t* __restrict__ perm, const LeafRec* __restrict__ leaves,
    int32_t* __restrict__ cand_ids, float* __restrict__ cand_d,
    unsigned long long* __restrict__ pairs) {
    using F = Frag<FMT>;
    static_assert(MP <= 128, "positions take 7 bits of the exact key");
    constexpr int NT = MP / 16;            // row and column tiles
    constexpr int RPW = (NT + 3) / 4;      // row tiles per wave (the last may be empty)
    // LDS: the key block, later the 32-dim FP32 blocks of the re-rank
    constexpr int kKeyWords = MP * (MP + 1);
    constexpr int kRowFloats = MP * 33;
    __shared__ uint32_t lds[kKeyWords > kRowFloats ? kKeyWords : kRowFloats];
    __shared__ int32_t ids[MP];
    __shared__ float snrm[MP], ssinv[MP];

    const LeafRec lf = leaves[blockIdx.x];
    const int m = lf.size;
    const size_t base = static_cast<size_t>(lf.tree) * n + lf.start;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    load_leaf_sorted<MP>(perm + base, m, reinterpret_cast<int32_t*>(lds), ids, snrm, ssinv, nrm,
                         sinv);
    if (tid == 0 && pairs != nullptr)
        atomicAdd(pairs, static_cast<unsigned long long>(m) * static_cast<unsigned long long>(m - 1));
    __syncthreads();

    // ---- Gram: wave w has row tiles w*RPW .. w*RPW+RPW-1 and every column tile
    {
        const size_t rstride = static_cast<size_t>(Dp) * F::kBytes;
        const int kg = lane >> 4;
        const uint8_t* ap[RPW];
        bool aok[RPW];
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            const int arow = (wv * RPW + q) * 16 + (lane & 15);
            aok[q] = arow < m;
            ap[q] = Xr + static_cast<size_t>(ids[aok[q] ? arow : 0]) * rstride +
                    static_cast<size_t>(8 * kg) * F::kBytes;
        }
        const uint8_t* bp[NT];
        bool bok[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int bcol = t * 16 + (lane & 15);
            bok[t] = bcol < m;
            bp[t] = Xr + static_cast<size_t>(ids[bok[t] ? bcol : 0]) * rstride +
                    static_cast<size_t>(8 * kg) * F::kBytes;
        }
        f32x4 acc[RPW][NT];
#pragma unroll
        for (int q = 0; q < RPW; ++q)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[q][t] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < Dp; k0 += 32) {
            const size_t off = static_cast<size_t>(k0) * F::kBytes;
            FragVec<FMT> a[RPW], b[NT];
#pragma unroll
            for (int q = 0; q < RPW; ++q) a[q] = load_frag<FMT>(ap[q] + off, aok[q]);
#pragma unroll
            for (int t = 0; t < NT; ++t) b[t] = load_frag<FMT>(bp[t] + off, bok[t]);
#pragma unroll
            for (int q = 0; q < RPW; ++q)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[q][t] = F::mma(a[q], b[t], acc[q][t]);
        }
#pragma unroll
        for (int q = 0; q < RPW; ++q)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int col = t * 16 + (lane & 15);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = (wv * RPW + q) * 16 + 4 * kg + i;
                    uint32_t key = 0xffffffffu;  // diagonal, padding
                    if (row < m && col < m && row != col) {
                        const float v =
                            snrm[row] + snrm[col] - 2.f * acc[q][t][i] * (ssinv[row] * ssinv[col]);
                        if constexpr (EXACT)
                            key = (static_cast<uint32_t>(v) << 7) | static_cast<uint32_t>(col);
                        else
                            key = fkey(v);
                    }
                    if (row < MP) lds[row * (MP + 1) + col] = key;
                }
            }
    }
    __syncthreads();

    const int t = tid;
    const bool own = t < m;
    const int ce = (c < m - 1 ? c : m - 1);
    if constexpr (EXACT) {
        // ---- thread t: the CL smallest keys of row t (sorted insertion by min/max)
        uint32_t L[CL];
#pragma unroll
        for (int i = 0; i < CL; ++i) L[i] = 0xffffffffu;
        if (own) {
            const uint32_t* krow = lds + t * (MP + 1);
            for (int j = 0; j < m; ++j) {
                uint32_t x = krow[j];
#pragma unroll
                for (int i = 0; i < CL; ++i) {
                    const uint32_t hi = max(L[i], x);
                    L[i] = min(L[i], x);
                    x = hi;
                }
            }
            const size_t out = (static_cast<size_t>(lf.tree) * n + ids[t]) * k;
#pragma unroll
            for (int e = 0; e < CL; ++e)
                if (e < k) {
                    const bool ok = e < ce;
                    cand_ids[out + e] = ok ? ids[L[e] & 127u] : -1;
                    cand_d[out + e] = ok ? static_cast<float>(L[e] >> 7) : __int_as_float(0x7f800000);
                }
        }
        return;
    } else {
        // ---- thread t: the CL smallest (d~, position) of row t
        uint64_t L[CL];
#pragma unroll
        for (int i = 0; i < CL; ++i) L[i] = ~0ull;
        if (own) {
            const uint32_t* krow = lds + t * (MP + 1);
            for (int j = 0; j < m; ++j) {
                const uint32_t kj = krow[j];
                uint64_t x = kj == 0xffffffffu ? ~0ull
                                               : (static_cast<uint64_t>(kj) << 32) | static_cast<uint32_t>(j);
#pragma unroll
                for (int i = 0; i < CL; ++i) {
                    const bool lt = x < L[i];
                    const uint64_t lo = lt ? x : L[i];
                    x = lt ? L[i] : x;
                    L[i] = lo;
                }
            }
        }
        // ---- re-rank the ce candidates with d32, 32-dim blocks through LDS
        float tot[CL];
#pragma unroll
        for (int i = 0; i < CL; ++i) tot[i] = 0.f;
        float* rows = reinterpret_cast<float*>(lds);
        __syncthreads();  // every thread is done reading the key block
        for (int d0 = 0; d0 < D; d0 += 32) {
            for (int idx = tid; idx < m * 32; idx += 256) {
                const int j = idx >> 5, dd = idx & 31;
                rows[j * 33 + dd] = d0 + dd < D ? X[static_cast<size_t>(ids[j]) * D + d0 + dd] : 0.f;
            }
            __syncthreads();
            if (own) {
                const int dn = D - d0 < 32 ? D - d0 : 32;
                const float* xr = rows + t * 33;
#pragma unroll
                for (int i = 0; i < CL; ++i) {
                    if (i < ce) {
                        const float* xc = rows + static_cast<uint32_t>(L[i]) * 33;
                        float blk = 0.f;
                        for (int dd = 0; dd < dn; ++dd) {
                            const float df = xr[dd] - xc[dd];
                            blk = __fmaf_rn(df, df, blk);
                        }
                        tot[i] = tot[i] + blk;
                    }
                }
            }
            __syncthreads();
        }
        if (own) {
            // k smallest (d32, id): 64-bit keys, d32 >= 0 (KL >= k)
            uint64_t K[KL];
#pragma unroll
            for (int i = 0; i < KL; ++i) K[i] = kNoKey;
#pragma unroll
            for (int s = 0; s < CL; ++s) {
                if (s < ce) {
                    uint64_t x = cand_key(tot[s], ids[static_cast<uint32_t>(L[s])]);
#pragma unroll
                    for (int i = 0; i < KL; ++i) {
                        const bool lt = x < K[i];
                        const uint64_t lo = lt ? x : K[i];
                        x = lt ? K[i] : x;
                        K[i] = lo;
                    }
                }
            }
            const size_t out = (static_cast<size_t>(lf.tree) * n + ids[t]) * k;
#pragma unroll
            for (int e = 0; e < KL; ++e)
                if (e < k) {
                    const bool ok = e < ce;
                    cand_ids[out + e] = ok ? key_id(K[e]) : -1;
                    cand_d[out + e] = ok ? key_dist(K[e]) : __int_as_float(0x7f800000);
                }
        }
    }
}

template <int FMT, bool EXACT, bool VEC4>
int launch_fmt(const LeafArgs& a, const ReducedRows& rr, int* launches, char* err, size_t errlen) {
    const int lm = a.leaf_max;
    // candidates per row: the k best directly when the first pass is exact
    const int c = EXACT ? a.k : (a.rerank < a.k ? a.k : a.rerank);
    auto go = [&](auto kern) -> int {
        if (a.timer) a.timer->begin(kKLeaf, a.stream);
        kern<<<static_cast<unsigned>(a.n_leaves), 256, 0, a.stream>>>(
            a.X, rr.Xr, a.n, a.D, rr.Dp, rr.nrm, rr.sinv, a.k, c, a.perm, a.leaves, a.cand_ids,
            a.cand_d, a.pairs);
        if (a.timer) a.timer->end(kKLeaf, a.stream);
        ++*launches;
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            std::snprintf(err, errlen, "leaf launch failed: %s", hipGetErrorString(e));
            return kHip;
        }
        return kOk;
    };
    // small leaves: thread per row with register candidate lists
    if (lm <= 128 && c <= 32) {
        // CL >= c candidates per row; KL >= k final list (re-rank only)
        auto small = [&](auto mp_tag) -> int {
            constexpr int MP = decltype(mp_tag)::value;
            if constexpr (EXACT) {  // list of exactly k rounded up to 4
                switch ((c + 3) / 4) {
                    case 1: case 2: return go(k_leaf_small<FMT, MP, 8, 8, true>);
                    case 3: return go(k_leaf_small<FMT, MP, 12, 12, true>);
                    case 4: return go(k_leaf_small<FMT, MP, 16, 16, true>);
                    case 5: return go(k_leaf_small<FMT, MP, 20, 20, true>);
                    case 6: return go(k_leaf_small<FMT, MP, 24, 24, true>);
                    case 7: return go(k_leaf_small<FMT, MP, 28, 28, true>);
                    default: return go(k_leaf_small<FMT, MP, 32, 32, true>);
                }
            } else {
                if (c <= 16) return go(k_leaf_small<FMT, MP, 16, 16, false>);
                return a.k <= 16 ? go(k_leaf_small<FMT, MP, 32, 16, false>)
                                 : go(k_leaf_small<FMT, MP, 32, 32, false>);
            }
        };
        if (lm <= 64) return small(std::integral_constant<int, 64>{});
        if (lm <= 112) return small(std::integral_constant<int, 112>{});
        return small(std::integral_constant<int, 128>{});
    }
    if (lm <= 64) return go(k_leaf_mfma<FMT, 64, 64, EXACT, VEC4>);
    if (lm <= 128) return go(k_leaf_mfma<FMT, 128, 64, EXACT, VEC4>);
    if (lm <= 256) return go(k_leaf_mfma<FMT, 256, 64, EXACT, VEC4>);
    return go(k_leaf_mfma<FMT, 512, 32, EXACT, VEC4>);
}

// The exact first pass exists for BF16 only (integers 0..255 with D <= 129).
template <int FMT>
int launch_fmt_any(const LeafArgs& a, const ReducedRows& rr, int* launches, char* err,
                   size_t errlen) {
    const bool v4 = a.D % 4 == 0;
    if constexpr (FMT == kBF16) {
        if (rr.exact) return v4 ? launch_fmt<FMT, true, true>(a, rr, launches, err, errlen)
                                : launch_fmt<FMT, true, false>(a, rr, launches, err, errlen);
    }
    return v4 ? launch_fmt<FMT, false, true>(a, rr, launches, err, errlen)
              : launch_fmt<FMT, false, false>(a, rr, launches, err, errlen);
}

}  // namespace leafk
}  // namespace knng
