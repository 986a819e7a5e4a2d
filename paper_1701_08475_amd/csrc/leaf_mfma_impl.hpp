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
#include <cstdlib>
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

// The leaf's ids into LDS in ascending order, with their norms and scales:
// a stable rank sort (the rank of entry j counts smaller ids, and equal ids
// before j, so it is a permutation of 0..m-1 whatever perm holds).  Position
// order is then id order, and distance ties fall to the smaller id.  raw
// holds m ints of scratch; the caller synchronises before reading ids.
template <int MP, int NT = 256>
__device__ __forceinline__ void load_leaf_sorted(const int32_t* __restrict__ lp, int m,
                                                 int32_t* raw, int32_t* ids, float* snrm,
                                                 float* ssinv, const float* __restrict__ nrm,
                                                 const float* __restrict__ sinv) {
    const int tid = threadIdx.x;
    for (int j = tid; j < m; j += NT) raw[j] = lp[j];
    for (int j = m + tid; j < MP; j += NT) {
        ids[j] = 0;
        snrm[j] = 0.f;
        ssinv[j] = 0.f;
    }
    __syncthreads();
    for (int j = tid; j < m; j += NT) {
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

// Key of rank `rank` (0-based) among the valid keys of a wavefront (R per
// lane), by radix selection on 8-bit digits with a 256-bin histogram in LDS
// (hist: 256 words owned by this wavefront).  Returns the key; *below gets
// the number of valid keys smaller than it.
template <int R>
__device__ __forceinline__ uint32_t wave_select_rank(const uint32_t (&key)[R], const bool (&valid)[R],
                                                     int rank, uint32_t* hist, int* below) {
    const int lane = threadIdx.x & 63;
    uint32_t prefix = 0u;
    int rem = rank;
#pragma unroll
    for (int shift = 24; shift >= 0; shift -= 8) {
#pragma unroll
        for (int q = 0; q < 4; ++q) hist[4 * lane + q] = 0u;
        wave_lds_sync();
        const uint32_t hi = shift == 24 ? 0u : (0xffffffffu << (shift + 8));
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (valid[r] && (key[r] & hi) == (prefix & hi)) atomicAdd(&hist[(key[r] >> shift) & 255u], 1u);
        wave_lds_sync();
        uint32_t h4[4];
        int local = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            h4[q] = hist[4 * lane + q];
            local += static_cast<int>(h4[q]);
        }
        int total;
        const int excl = wave_excl_scan(local, &total);
        // the lane whose 4 bins hold cumulative rank `rem` picks the digit
        int digit = 0, nrem = 0;
        const bool mine = excl <= rem && rem < excl + local;
        if (mine) {
            int cum = excl;
            bool done = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int hq = static_cast<int>(h4[q]);
                if (!done && rem < cum + hq) {
                    digit = 4 * lane + q;
                    nrem = rem - cum;
                    done = true;
                }
                cum += hq;
            }
        }
        const unsigned long long bm = __ballot(mine);
        const int src = static_cast<int>(__builtin_ctzll(bm));
        digit = __shfl(digit, src, kWave);
        nrem = __shfl(nrem, src, kWave);
        prefix |= static_cast<uint32_t>(digit) << shift;
        rem = nrem;
        wave_lds_sync();
    }
    *below = rank - rem;
    return prefix;
}

// Leaves of up to MP points (wave per row; NW wavefronts per workgroup).  Panels of PR rows: the Gram of
// the panel against the whole leaf on MFMA gives d~ in LDS; one wave per row
// selects its ce candidates exactly by (d~, position) (radix selection).
// EXACT (the first pass is exact: integer data that the format holds, with
// every product and partial sum below 2^24, so d~ == d32): the candidates
// are the k best and are sorted and written at once.  Otherwise their
// positions go to a leaf-wide table in LDS, and after the last panel the
// re-rank streams the leaf's FP32 rows through LDS in 32-dimension chunks:
// thread t owns row t (rows in rounds of 64 NW), accumulates d32 for up to 32
// candidates at a time (in-block FMA sum, blocks added in order) and keeps
// the k smallest (d32, id).  CS bounds the candidates per row.
template <int FMT, int MP, int PR, int CS, int KL, bool EXACT, int NW>
__global__ __launch_bounds__(NW * 64) void k_leaf_mfma(
    const float* __restrict__ X, const uint8_t* __restrict__ Xr, int64_t n, int D, int Dp,
    const float* __restrict__ nrm, const float* __restrict__ sinv, int k, int c,
    const int32_t* __restrict__ perm, const LeafRec* __restrict__ leaves,
    int32_t* __restrict__ cand_ids, float* __restrict__ cand_d,
    unsigned long long* __restrict__ pairs) {
    using F = Frag<FMT>;
    using Pos = typename std::conditional<(MP <= 256), uint8_t, uint16_t>::type;
    constexpr int NTH = NW * kWave;        // threads
    constexpr int NT = MP / 16;            // column tiles
    constexpr int RTP = PR / 16;           // row tiles per panel
    constexpr int WPR = NW / RTP;          // waves per row tile
    constexpr int AT = NT / WPR;           // column tiles per wave
    constexpr int R = MP / kWave;          // keys per lane in the selection
    constexpr int kRowStride = 36;         // floats per staged 32-dim row chunk (16-byte rows)
    constexpr int kPanel = PR * (MP + 1);
    constexpr int kStage = MP * kRowStride;
    constexpr int kRegion = kPanel > kStage ? kPanel : kStage;
    constexpr int kSel = EXACT ? NW * 128 : MP * CS;
    static_assert(R >= 1 && AT >= 1 && NW % RTP == 0 && NT % WPR == 0, "tile shape");

    __shared__ __align__(16) float region[kRegion];  // d~ panel, later FP32 row chunks
    __shared__ Pos csel[kSel];  // EXACT: per wave the selection of its row;
                                // else per row its candidate positions
    __shared__ int32_t ids[MP];
    __shared__ float snrm[MP], ssinv[MP];
    __shared__ uint32_t s_hist[NW * 256];  // per-wave radix histograms
    float(*dist)[MP + 1] = reinterpret_cast<float(*)[MP + 1]>(region);

    const LeafRec lf = leaves[blockIdx.x];
    const int m = lf.size;
    const size_t base = static_cast<size_t>(lf.tree) * n + lf.start;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    load_leaf_sorted<MP, NTH>(perm + base, m, reinterpret_cast<int32_t*>(region), ids, snrm, ssinv,
                              nrm, sinv);
    if (tid == 0 && pairs != nullptr)
        stat_add(pairs, blockIdx.x, static_cast<unsigned long long>(m) * static_cast<unsigned long long>(m - 1));
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
        // ---- per row (one wave): exact top-ce by (d~, position)
        const int rows = m - p0 < PR ? m - p0 : PR;
        for (int rl = wv; rl < rows; rl += NW) {
            const int row = p0 + rl;
            Pos* sel = EXACT ? csel + wv * 128 : csel + row * CS;
            uint32_t key[R];
            bool valid[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int col = r * kWave + lane;
                valid[r] = col < m && col != row;
                key[r] = valid[r] ? fkey(dist[rl][col]) : 0xffffffffu;
            }
            // the key of rank ce-1, by 8-bit radix selection; rem = how many
            // keys equal to it are taken, minus one
            uint32_t prefix = 0u;
            int rem = 0;
            if (ce > 0) {
                int below;
                prefix = wave_select_rank<R>(key, valid, ce - 1, s_hist + wv * 256, &below);
                rem = ce - 1 - below;
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
                    sel[taken + __popcll(bt & ((1ull << lane) - 1ull))] =
                        static_cast<Pos>(r * kWave + lane);
                taken += __popcll(bt);
                eq_seen += __popcll(beq);
            }
            if constexpr (EXACT) {
                // the candidates' d~ are their d32: sort by (d, id) and write
                uint64_t v[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int s = lane * 2 + r;
                    v[r] = s < ce ? cand_key(dist[rl][sel[s]], ids[sel[s]]) : kNoKey;
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
        }
        __syncthreads();
    }
    if constexpr (!EXACT) {
        // ---- re-rank: d32 of every (row, candidate) from LDS-staged chunks
        for (int r0 = 0; r0 < m; r0 += NTH) {
            const int row = r0 + tid;
            const bool own = row < m;
            uint64_t K[KL];
#pragma unroll
            for (int i = 0; i < KL; ++i) K[i] = kNoKey;
            for (int g0 = 0; g0 < ce; g0 += 32) {
                float tot[32];
#pragma unroll
                for (int i = 0; i < 32; ++i) tot[i] = 0.f;
                for (int d0 = 0; d0 < D; d0 += 32) {
                    __syncthreads();  // the previous chunk is no longer read
                    for (int idx = tid; idx < m * 32; idx += NTH) {
                        const int j = idx >> 5, dd = idx & 31;
                        region[j * kRowStride + dd] =
                            d0 + dd < D ? X[static_cast<size_t>(ids[j]) * D + d0 + dd] : 0.f;
                    }
                    __syncthreads();
                    if (own) {
                        float xr[32];
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const float4 v4 = *reinterpret_cast<const float4*>(
                                region + row * kRowStride + 4 * q);
                            xr[4 * q] = v4.x;
                            xr[4 * q + 1] = v4.y;
                            xr[4 * q + 2] = v4.z;
                            xr[4 * q + 3] = v4.w;
                        }
                        const int gn = ce - g0 < 32 ? ce - g0 : 32;
#pragma unroll
                        for (int i = 0; i < 32; ++i) {
                            if (i < gn) {
                                const float* xc = region + csel[row * CS + g0 + i] * kRowStride;
                                float blk = 0.f;  // padding past D adds exact zeros
#pragma unroll
                                for (int q = 0; q < 8; ++q) {
                                    const float4 v4 = *reinterpret_cast<const float4*>(xc + 4 * q);
                                    float df = xr[4 * q] - v4.x;
                                    blk = __fmaf_rn(df, df, blk);
                                    df = xr[4 * q + 1] - v4.y;
                                    blk = __fmaf_rn(df, df, blk);
                                    df = xr[4 * q + 2] - v4.z;
                                    blk = __fmaf_rn(df, df, blk);
                                    df = xr[4 * q + 3] - v4.w;
                                    blk = __fmaf_rn(df, df, blk);
                                }
                                tot[i] = tot[i] + blk;
                            }
                        }
                    }
                }
                if (own) {
                    const int gn = ce - g0 < 32 ? ce - g0 : 32;
#pragma unroll
                    for (int i = 0; i < 32; ++i) {
                        if (i < gn) {
                            uint64_t x = cand_key(tot[i], ids[csel[row * CS + g0 + i]]);
#pragma unroll
                            for (int s = 0; s < KL; ++s) {
                                const bool lt = x < K[s];
                                const uint64_t lo = lt ? x : K[s];
                                x = lt ? K[s] : x;
                                K[s] = lo;
                            }
                        }
                    }
                }
            }
            if (own) {
                const size_t out = (static_cast<size_t>(lf.tree) * n + ids[row]) * k;
#pragma unroll
                for (int e = 0; e < KL; ++e)
                    if (e < k) {
                        const bool ok = e < ce && K[e] != kNoKey;
                        cand_ids[out + e] = ok ? key_id(K[e]) : -1;
                        cand_d[out + e] = ok ? key_dist(K[e]) : __int_as_float(0x7f800000);
                    }
            }
        }
    }
}

// ------------------------------------------------------------- wide leaves
// Leaves of up to MP (256 or 512) points with the re-ranked first pass, at
// most 64 candidates per row (c <= 64, k <= 64), D % 4 == 0.  One
// workgroup (4 wavefronts) per leaf, rows in batches of 64:
//   1. per 16-row panel, the Gram of the panel against every column on MFMA
//      (each wave takes MP/64 column tiles) gives d~ in LDS; then one wave
//      per row selects its ce smallest (d~, position) exactly (radix
//      selection over the row's key range, below) into the batch's
//      candidate table;
//   2. the batch's re-rank streams the leaf's FP32 rows through LDS in
//      8-dimension chunks: one wave per row, lane j owns candidate j and
//      accumulates d32 (in-block fused sum, blocks of 32 added in order);
//   3. per row, the wave sorts its (d32, id) keys and writes the k smallest.
// Same first-pass values (same MFMA steps in the same order), same
// selection, same d32 and the same order as k_leaf_mfma: the lists are
// identical bit for bit; this layout needs about a third of the LDS, so three
// workgroups share a compute unit.
//
// Selection of the key of rank rem among the valid keys of a row (R per
// lane): the keys lie in [lo, hi] (initially the row's minimum and maximum);
// each pass counts them in 256 bins of width 2^shift over [lo, hi] (LDS
// atomics), keeps the bin holding rank rem and narrows [lo, hi] to it.  It
// stops when the kept bin's keys are all needed (then every key <= hi is
// taken) or when the bin is a single value T (then the keys < T and the first
// rem + 1 keys equal to T by position are taken).
template <int R>
__device__ __forceinline__ void wave_select_candidates(const uint32_t (&key)[R], int ce,
                                                       uint32_t* hist, uint16_t* sel) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below_me = (1ull << lane) - 1ull;
    uint32_t lo = 0xffffffffu, hi = 0u;
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (key[r] != 0xffffffffu) {
            lo = min(lo, key[r]);
            hi = max(hi, key[r]);
        }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        lo = min(lo, static_cast<uint32_t>(__shfl_xor(static_cast<int>(lo), o, kWave)));
        hi = max(hi, static_cast<uint32_t>(__shfl_xor(static_cast<int>(hi), o, kWave)));
    }
    int rem = ce - 1;
    bool single = false;  // [lo, hi] is the single value of the key of rank rem
    while (true) {
        const uint32_t span = hi - lo;
        if (span == 0u) {
            single = true;
            break;
        }
        const int bits = 32 - __clz(static_cast<int>(span));
        const int shift = bits > 8 ? bits - 8 : 0;
        *reinterpret_cast<uint4*>(hist + 4 * lane) = make_uint4(0u, 0u, 0u, 0u);
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (key[r] >= lo && key[r] <= hi) atomicAdd(&hist[(key[r] - lo) >> shift], 1u);
        wave_lds_sync();
        const uint4 h4v = *reinterpret_cast<const uint4*>(hist + 4 * lane);
        const int h4[4] = {static_cast<int>(h4v.x), static_cast<int>(h4v.y),
                           static_cast<int>(h4v.z), static_cast<int>(h4v.w)};
        const int local = h4[0] + h4[1] + h4[2] + h4[3];
        int total;
        const int excl = wave_excl_scan(local, &total);
        int digit = 0, nrem = 0, cnt = 0;
        const bool mine = excl <= rem && rem < excl + local;
        if (mine) {
            int cum = excl;
            bool done = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (!done && rem < cum + h4[q]) {
                    digit = 4 * lane + q;
                    nrem = rem - cum;
                    cnt = h4[q];
                    done = true;
                }
                cum += h4[q];
            }
        }
        const int src = static_cast<int>(__builtin_ctzll(__ballot(mine)));
        digit = __shfl(digit, src, kWave);
        nrem = __shfl(nrem, src, kWave);
        cnt = __shfl(cnt, src, kWave);
        wave_lds_sync();  // the histogram is read before the next pass clears it
        const uint32_t lo2 = lo + (static_cast<uint32_t>(digit) << shift);
        const uint32_t w = (shift == 0) ? 0u : ((1u << shift) - 1u);
        const uint32_t hi2 = (hi - lo2 > w) ? lo2 + w : hi;
        lo = lo2;
        hi = hi2;
        rem = nrem;
        if (nrem == cnt - 1) break;  // every key of the bin is needed: take keys <= hi
        if (shift == 0) {
            single = true;
            break;
        }
    }
    // keys < lo (all needed), then either every key in [lo, hi] or, when the
    // bin is the single value lo, the first rem + 1 keys equal to it
    int taken = 0, eq_seen = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool lt = single ? key[r] < lo : key[r] <= hi;
        const bool eq = single && key[r] == lo;
        const unsigned long long beq = __ballot(eq);
        const int eq_rank = eq_seen + __popcll(beq & below_me);
        const bool take = lt || (eq && eq_rank <= rem);
        const unsigned long long bt = __ballot(take);
        if (take) sel[taken + __popcll(bt & below_me)] = static_cast<uint16_t>(r * kWave + lane);
        taken += __popcll(bt);
        eq_seen += __popcll(beq);
    }
}

template <int FMT, int MP>
__global__ __launch_bounds__(256) void k_leaf_wide(
    const float* __restrict__ X, const uint8_t* __restrict__ Xr, int64_t n, int D, int Dp,
    const float* __restrict__ nrm, const float* __restrict__ sinv, int k, int c,
    const int32_t* __restrict__ perm, const LeafRec* __restrict__ leaves,
    int32_t* __restrict__ cand_ids, float* __restrict__ cand_d,
    unsigned long long* __restrict__ pairs) {
    using F = Frag<FMT>;
    constexpr int NW = 4, NTH = NW * kWave;
    constexpr int R = MP / kWave;      // keys per lane in the selection
    constexpr int NT = MP / 16;        // column tiles
    constexpr int TPW = NT / NW;       // column tiles per wave
    constexpr int RB = 64;             // rows per batch
    constexpr int RPW = RB / NW;       // rows per wave in the re-rank
    constexpr int CW = 8;              // dimensions per staged chunk
    constexpr int SS = 12;             // floats per staged row (16-byte aligned)
    constexpr int kPanel = 16 * (MP + 1);
    constexpr int kStage = MP * SS;
    constexpr int kRegion = kPanel > kStage ? kPanel : kStage;
    static_assert(R >= 1 && TPW >= 1 && NT % NW == 0, "tile shape");

    __shared__ __align__(16) float region[kRegion];  // d~ panel, later FP32 row chunks
    __shared__ uint16_t csel[RB * kWave];            // per batch row its candidate positions
    __shared__ int32_t ids[MP];
    __shared__ float snrm[MP], ssinv[MP];
    __shared__ __align__(16) uint32_t s_hist[NW * 256];
    float(*dist)[MP + 1] = reinterpret_cast<float(*)[MP + 1]>(region);

    const LeafRec lf = leaves[blockIdx.x];
    const int m = lf.size;
    const size_t base = static_cast<size_t>(lf.tree) * n + lf.start;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    load_leaf_sorted<MP, NTH>(perm + base, m, reinterpret_cast<int32_t*>(region), ids, snrm, ssinv,
                              nrm, sinv);
    if (tid == 0 && pairs != nullptr)
        stat_add(pairs, blockIdx.x, static_cast<unsigned long long>(m) * static_cast<unsigned long long>(m - 1));
    __syncthreads();
    const int ce = c < m - 1 ? c : m - 1;  // candidates per row
    const size_t rstride = static_cast<size_t>(Dp) * F::kBytes;
    const int kg = lane >> 4;

    for (int p0 = 0; p0 < m; p0 += RB) {
        const int nb = m - p0 < RB ? m - p0 : RB;
        __syncthreads();  // the previous batch's last chunk is no longer read
        // ---- selection, one 16-row panel at a time
        for (int pp = 0; pp < nb; pp += 16) {
            const int prow = p0 + pp;
            const int arow = prow + (lane & 15);
            const uint8_t* ap = Xr + static_cast<size_t>(ids[arow < m ? arow : 0]) * rstride +
                                static_cast<size_t>(8 * kg) * F::kBytes;
            const uint8_t* bp[TPW];
            bool bok[TPW];
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int bcol = (wv * TPW + t) * 16 + (lane & 15);
                bok[t] = bcol < m;
                bp[t] = Xr + static_cast<size_t>(ids[bcol < m ? bcol : 0]) * rstride +
                        static_cast<size_t>(8 * kg) * F::kBytes;
            }
            f32x4 acc[TPW];
#pragma unroll
            for (int t = 0; t < TPW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
            FragVec<FMT> a = load_frag<FMT>(ap, arow < m);
            FragVec<FMT> b[TPW];
#pragma unroll
            for (int t = 0; t < TPW; ++t) b[t] = load_frag<FMT>(bp[t], bok[t]);
            for (int k0 = 0; k0 < Dp; k0 += 32) {
                const size_t nx = static_cast<size_t>(k0 + 32) * F::kBytes;
                const bool more = k0 + 32 < Dp;
                const FragVec<FMT> an = load_frag<FMT>(ap + nx, more && arow < m);
                FragVec<FMT> bn[TPW];
#pragma unroll
                for (int t = 0; t < TPW; ++t) bn[t] = load_frag<FMT>(bp[t] + nx, more && bok[t]);
#pragma unroll
                for (int t = 0; t < TPW; ++t) acc[t] = F::mma(a, b[t], acc[t]);
                a = an;
#pragma unroll
                for (int t = 0; t < TPW; ++t) b[t] = bn[t];
            }
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const int col = (wv * TPW + t) * 16 + (lane & 15);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int rl = 4 * kg + i;
                    const int row = prow + rl;
                    float v = __int_as_float(0x7f800000);
                    if (row < m && col < m)
                        v = snrm[row] + snrm[col] - 2.f * acc[t][i] * (ssinv[row] * ssinv[col]);
                    dist[rl][col] = v;
                }
            }
            __syncthreads();
            const int prows = nb - pp < 16 ? nb - pp : 16;
            for (int rl = wv; rl < prows; rl += NW) {
                const int row = prow + rl;
                uint16_t* sel = csel + (pp + rl) * kWave;
                if (ce >= m - 1) {  // every other member is a candidate
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int col = r * kWave + lane;
                        const int e = col < row ? col : col - 1;
                        if (col < m && col != row) sel[e] = static_cast<uint16_t>(col);
                    }
                } else if (ce > 0) {
                    uint32_t key[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const int col = r * kWave + lane;
                        key[r] = (col < m && col != row) ? fkey(dist[rl][col]) : 0xffffffffu;
                    }
                    wave_select_candidates<R>(key, ce, s_hist + wv * 256, sel);
                }
            }
            __syncthreads();  // the panel is no longer read
        }
        // ---- re-rank of the batch: d32 from LDS-staged 8-dimension chunks
        float tot[RPW], blk[RPW];
        int cpos[RPW];
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            tot[q] = 0.f;
            blk[q] = 0.f;
            const int bi = wv + NW * q;
            cpos[q] = (bi < nb && lane < ce) ? static_cast<int>(csel[bi * kWave + lane]) : 0;
        }
        for (int d0 = 0; d0 < D; d0 += CW) {
            __syncthreads();  // the previous chunk (or the panel) is no longer read
            for (int idx = tid; idx < 2 * m; idx += NTH) {
                const int j = idx >> 1, hf = idx & 1;
                const int d = d0 + 4 * hf;
                float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
                if (d < D) v = *reinterpret_cast<const float4*>(X + static_cast<size_t>(ids[j]) * D + d);
                *reinterpret_cast<float4*>(region + j * SS + 4 * hf) = v;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const int bi = wv + NW * q;
                if (bi < nb) {  // uniform across the wave
                    const float* xo = region + (p0 + bi) * SS;
                    const float* xc = region + cpos[q] * SS;
                    const float4 o0 = *reinterpret_cast<const float4*>(xo);
                    const float4 o1 = *reinterpret_cast<const float4*>(xo + 4);
                    const float4 c0 = *reinterpret_cast<const float4*>(xc);
                    const float4 c1 = *reinterpret_cast<const float4*>(xc + 4);
                    float bq = blk[q];  // padding past D adds exact zeros
                    float df = o0.x - c0.x;
                    bq = __fmaf_rn(df, df, bq);
                    df = o0.y - c0.y;
                    bq = __fmaf_rn(df, df, bq);
                    df = o0.z - c0.z;
                    bq = __fmaf_rn(df, df, bq);
                    df = o0.w - c0.w;
                    bq = __fmaf_rn(df, df, bq);
                    df = o1.x - c1.x;
                    bq = __fmaf_rn(df, df, bq);
                    df = o1.y - c1.y;
                    bq = __fmaf_rn(df, df, bq);
                    df = o1.z - c1.z;
                    bq = __fmaf_rn(df, df, bq);
                    df = o1.w - c1.w;
                    bq = __fmaf_rn(df, df, bq);
                    blk[q] = bq;
                }
            }
            if (((d0 + CW) & 31) == 0 || d0 + CW >= D) {  // end of a 32-dimension block
#pragma unroll
                for (int q = 0; q < RPW; ++q) {
                    tot[q] = tot[q] + blk[q];
                    blk[q] = 0.f;
                }
            }
        }
        // ---- per row: the k smallest (d32, id), in order
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            const int bi = wv + NW * q;
            if (bi < nb) {
                uint64_t v[1];
                v[0] = lane < ce ? cand_key(tot[q], ids[cpos[q]]) : kNoKey;
                wave_bitonic_sort<1>(v);
                const size_t out = (static_cast<size_t>(lf.tree) * n + ids[p0 + bi]) * k;
                if (lane < k) {
                    const bool ok = v[0] != kNoKey;
                    cand_ids[out + lane] = ok ? key_id(v[0]) : -1;
                    cand_d[out + lane] = ok ? key_dist(v[0]) : __int_as_float(0x7f800000);
                }
            }
        }
    }
}

// ------------------------------------------------------------- small leaves
// Leaves of at most MP (64, 112 or 128) points.  The Gram on MFMA fills the
// whole leaf's block of keys in LDS; then thread t owns row t and scans it
// once, keeping its CL smallest keys in a sorted register list.
//
// EXACT (first pass exact, so d~ is the integer d32 < 2^23): the 32-bit key
// (d << 7) | position orders by (distance, position) = (distance, id), and
// insertion is one min and one max per slot; two lanes share a row (half
// the candidates each, then a merge of their lists); the list is the answer.
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
        stat_add(pairs, blockIdx.x, static_cast<unsigned long long>(m) * static_cast<unsigned long long>(m - 1));
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
        // When the leaf's reduced rows fit the key block (free until the keys
        // are written), they are copied there in one coalesced pass and the
        // Gram reads its fragments from LDS: one round trip to HBM instead of
        // one per 32-dimension step.  Rows are padded by 16 bytes so the 16
        // rows of a fragment fall in different banks.  Same products, same
        // order.
        const int rs = static_cast<int>(rstride) + 16;
        const bool staged = static_cast<size_t>(MP) * rs <= sizeof(lds);
        if (staged) {
            uint8_t* L = reinterpret_cast<uint8_t*>(lds);
            const int cpr = static_cast<int>(rstride / 16);  // 16-byte chunks per row
            for (int c = tid; c < m * cpr; c += 256) {
                const int r = c / cpr, j = c % cpr;
                *reinterpret_cast<uint4*>(L + r * rs + j * 16) = *reinterpret_cast<const uint4*>(
                    Xr + static_cast<size_t>(ids[r]) * rstride + static_cast<size_t>(j) * 16);
            }
            __syncthreads();
            int ao[RPW], bo[NT];
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const int arow = (wv * RPW + q) * 16 + (lane & 15);
                ao[q] = (aok[q] ? arow : 0) * rs + 8 * kg * F::kBytes;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int bcol = t * 16 + (lane & 15);
                bo[t] = (bok[t] ? bcol : 0) * rs + 8 * kg * F::kBytes;
            }
            for (int k0 = 0; k0 < Dp; k0 += 32) {
                const int off = k0 * F::kBytes;
                FragVec<FMT> a[RPW], b[NT];
#pragma unroll
                for (int q = 0; q < RPW; ++q) a[q] = load_frag<FMT>(L + ao[q] + off, aok[q]);
#pragma unroll
                for (int t = 0; t < NT; ++t) b[t] = load_frag<FMT>(L + bo[t] + off, bok[t]);
#pragma unroll
                for (int q = 0; q < RPW; ++q)
#pragma unroll
                    for (int t = 0; t < NT; ++t) acc[q][t] = F::mma(a[q], b[t], acc[q][t]);
            }
        } else {
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
        }
        __syncthreads();  // every wave is done with the staged rows before keys overwrite them
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
        // ---- two adjacent lanes per row (2 r, 2 r + 1): each keeps the CL
        // smallest keys of every other candidate of row r (sorted insertion
        // by min/max), then the pair merges its two sorted lists: bitonic
        // half-cleaner and merge over CP = 2^ceil(log2 CL) slots.  Keys are
        // distinct (position bits), so the first CL are the row's CL smallest.
        static_assert(2 * MP <= 256, "two lanes per row");
        constexpr int CP = CL <= 8 ? 8 : CL <= 16 ? 16 : 32;
        const int r = tid >> 1, h = tid & 1;
        uint32_t L[CL];
#pragma unroll
        for (int i = 0; i < CL; ++i) L[i] = 0xffffffffu;
        if (r < m) {
            const uint32_t* krow = lds + r * (MP + 1);
            for (int j = h; j < m; j += 2) {
                uint32_t x = krow[j];
#pragma unroll
                for (int i = 0; i < CL; ++i) {
                    const uint32_t hi = max(L[i], x);
                    L[i] = min(L[i], x);
                    x = hi;
                }
            }
        }
        uint32_t C[CP];
#pragma unroll
        for (int i = 0; i < CP; ++i) {
            const int bi = CP - 1 - i;  // the partner's list, reversed
            const uint32_t b = bi < CL ? static_cast<uint32_t>(__builtin_amdgcn_update_dpp(
                                             0, static_cast<int>(L[bi < CL ? bi : 0]), 0xB1, 0xf,
                                             0xf, false))
                                       : 0xffffffffu;
            C[i] = min(i < CL ? L[i] : 0xffffffffu, b);
        }
#pragma unroll
        for (int sd = CP / 2; sd >= 1; sd >>= 1)
#pragma unroll
            for (int i = 0; i < CP; ++i)
                if ((i & sd) == 0) {
                    const uint32_t lo = min(C[i], C[i + sd]), hi = max(C[i], C[i + sd]);
                    C[i] = lo;
                    C[i + sd] = hi;
                }
        if (r < m && h == 0) {
            const size_t out = (static_cast<size_t>(lf.tree) * n + ids[r]) * k;
#pragma unroll
            for (int e = 0; e < CL; ++e)
                if (e < k) {
                    const bool ok = e < ce;
                    cand_ids[out + e] = ok ? ids[C[e] & 127u] : -1;
                    cand_d[out + e] = ok ? static_cast<float>(C[e] >> 7) : __int_as_float(0x7f800000);
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

template <int FMT, bool EXACT>
int launch_fmt(const LeafArgs& a, const ReducedRows& rr, int* launches, char* err, size_t errlen) {
    const int lm = a.leaf_max;
    // candidates per row: the k best directly when the first pass is exact
    const int c = EXACT ? a.k : (a.rerank < a.k ? a.k : a.rerank);
    if (!EXACT && a.k > 64) {
        std::snprintf(err, errlen, "the re-ranked leaf search keeps at most 64 neighbours (k=%d)", a.k);
        return kUnsupported;
    }
    auto go = [&](auto kern, unsigned threads = 256) -> int {
        if (a.timer) a.timer->begin(kKLeaf, a.stream);
        kern<<<static_cast<unsigned>(a.n_leaves), threads, 0, a.stream>>>(
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
    // wave per row; the re-rank list holds k rounded up to 16 (k <= 64 here);
    // candidates per row at most CS.  Leaves up to 256 points: 4 waves, 32-row
    // panels above 128 points (two workgroups per CU); 512: 8 waves.
    auto big = [&](auto mp_tag, auto pr_tag, auto cs_tag, auto nw_tag) -> int {
        constexpr int MP = decltype(mp_tag)::value, PR = decltype(pr_tag)::value;
        constexpr int CS = decltype(cs_tag)::value, NW = decltype(nw_tag)::value;
        constexpr unsigned TH = NW * 64;
        if constexpr (EXACT) {
            return go(k_leaf_mfma<FMT, MP, PR, CS, 16, true, NW>, TH);
        } else {
            if (a.k <= 16) return go(k_leaf_mfma<FMT, MP, PR, CS, 16, false, NW>, TH);
            if (a.k <= 32) return go(k_leaf_mfma<FMT, MP, PR, CS, 32, false, NW>, TH);
            if (a.k <= 48) return go(k_leaf_mfma<FMT, MP, PR, CS, 48, false, NW>, TH);
            return go(k_leaf_mfma<FMT, MP, PR, CS, 64, false, NW>, TH);
        }
    };
    // leaves above 128 points with at most 64 candidates per row: the wide
    // kernel (KNNG_LEAF_WIDE=0 keeps k_leaf_mfma)
    const char* wide_env = std::getenv("KNNG_LEAF_WIDE");
    const bool wide = !EXACT && lm > 128 && c <= 64 && a.D % 4 == 0 &&
                      (wide_env == nullptr || std::atoi(wide_env) != 0);
    if (wide) {
        if (lm <= 256) return go(k_leaf_wide<FMT, 256>);
        return go(k_leaf_wide<FMT, 512>);
    }
    using I4 = std::integral_constant<int, 4>;
    using I8 = std::integral_constant<int, 8>;
    using I32 = std::integral_constant<int, 32>;
    using I64 = std::integral_constant<int, 64>;
    using I128 = std::integral_constant<int, 128>;
    using I256 = std::integral_constant<int, 256>;
    if (lm <= 64) return c <= 64 ? big(I64{}, I64{}, I64{}, I4{}) : big(I64{}, I64{}, I128{}, I4{});
    if (lm <= 128)
        return c <= 64 ? big(I128{}, I64{}, I64{}, I4{}) : big(I128{}, I64{}, I128{}, I4{});
    if (lm <= 256)
        return c <= 64 ? big(I256{}, I32{}, I64{}, I4{}) : big(I256{}, I32{}, I128{}, I4{});
    if (c > 64) {
        std::snprintf(err, errlen, "leaves above 256 points take at most 64 candidates per row (asked %d)", c);
        return kUnsupported;
    }
    return big(std::integral_constant<int, 512>{}, I32{}, I64{}, I8{});
}

// The exact first pass exists for BF16 only (integers 0..255 with D <= 129).
template <int FMT>
int launch_fmt_any(const LeafArgs& a, const ReducedRows& rr, int* launches, char* err,
                   size_t errlen) {
    if constexpr (FMT == kBF16) {
        if (rr.exact) return launch_fmt<FMT, true>(a, rr, launches, err, errlen);
    }
    return launch_fmt<FMT, false>(a, rr, launches, err, errlen);
}

}  // namespace leafk
}  // namespace knng
