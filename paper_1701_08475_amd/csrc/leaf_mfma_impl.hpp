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
    // the clusters of the partition list their ids in ascending order: then
    // the rank of entry j is j
    int unsorted = 0;
    for (int j = tid + 1; j < m; j += NT) unsorted |= raw[j - 1] < raw[j] ? 0 : 1;
    if (!__syncthreads_or(unsorted)) {
        for (int j = tid; j < m; j += NT) {
            const int32_t id = raw[j];
            ids[j] = id;
            snrm[j] = nrm[id];
            ssinv[j] = sinv[id];
        }
        return;
    }
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
    const float* __restrict__ X, const uint8_t* __restrict__ Xr, int64_t n, int D, int Dp, int rsb,
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
    const size_t rstride = static_cast<size_t>(rsb);  // bytes per row
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
// Leaves of up to MP (64 to 512) points with the re-ranked first pass, at
// most 64 candidates per row (c <= 64, k <= 64), D % 4 == 0.  One workgroup
// (4 wavefronts) per leaf, rows in batches of 64.  After the MFMA Gram, every
// step works on 16-lane groups, one row per group, four rows per wavefront:
//   1. per 16-row panel, the Gram of the panel against every column on MFMA
//      (each wave takes MP/64 column tiles) gives d~ in LDS; each 16-lane
//      group then selects its row's ce smallest (d~, position) exactly
//      (group_select, keys in registers) into the batch's candidate table,
//      as a set (each lane's picks contiguous);
//   2. the batch's re-rank streams the leaf's FP32 rows through LDS in
//      8-dimension chunks (the next chunk's loads in flight during this
//      one); lane l of a row's group owns its candidates 4l .. 4l+3 and
//      accumulates their d32 (in-block fused sum, blocks of 32 added in
//      order);
//   3. each group sorts its row's 64 (d32, id) keys (group_sort64, four per
//      lane) and writes the k smallest.
// Same first-pass values (same MFMA steps in the same order), the same
// candidate set, the same d32 and the same total order as k_leaf_mfma: the
// lists are identical bit for bit.  51 KB of LDS and at most 168 registers
// per lane: three workgroups per compute unit.

// Minimum / maximum over the 16 lanes of each aligned group (quad exchanges,
// then mirrors within 8 and within 16 lanes: every lane gets the result).
__device__ __forceinline__ uint32_t group16_min(uint32_t v) {
    v = min(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0xB1, 0xf, 0xf, false)));
    v = min(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x4E, 0xf, 0xf, false)));
    v = min(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x141, 0xf, 0xf, false)));
    v = min(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x140, 0xf, 0xf, false)));
    return v;
}
__device__ __forceinline__ uint32_t group16_max(uint32_t v) {
    v = max(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0xB1, 0xf, 0xf, false)));
    v = max(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x4E, 0xf, 0xf, false)));
    v = max(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x141, 0xf, 0xf, false)));
    v = max(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x140, 0xf, 0xf, false)));
    return v;
}

// Value of lane gl - o of the lane's aligned 16-lane group (o = 1, 2, 4, 8;
// lanes gl < o get 0): a DPP row shift, no LDS instruction.
__device__ __forceinline__ int group16_up(int v, int o) {
    switch (o) {
        case 1: return __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
        case 2: return __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);
        case 4: return __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);
        default: return __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
    }
}

// Exclusive prefix sum over the 16 lanes of each aligned group (every lane
// of the wavefront active).
__device__ __forceinline__ int group16_excl_scan(int v, int gl) {
    int incl = v;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
        const int y = group16_up(incl, o);
        if (gl >= o) incl += y;
    }
    return incl - v;
}

// Selection, per 16-lane group (one row each; lane l holds the row's keys
// kv[t] = key of position t*16 + l in registers, invalid ones ~0, and every
// key of t >= tmax invalid: those columns are skipped), of the
// row's ce smallest valid keys by (key, position).  lo, hi: the minimum and
// maximum of the lane's valid keys.  The keys of rank < ce lie in [lo, hi]
// (initially the row's minimum and maximum); a pass counts them in 128 bins
// of width 2^shift over [lo, hi] and narrows [lo, hi] to the bin holding rank
// rem.  A row stops when
//   - its kept bin's keys are all needed (then every key <= hi is taken);
//   - the bin holds at most 32 keys: they are gathered as (key, position)
//     pairs into lst (the group's 32 words x 2) and ranked against each other;
//     the pair of rank rem is the threshold, and every (key, position) up to
//     it is taken;
//   - or the bin is a single value T (then the keys < T and the first rem + 1
//     keys equal to T by position are taken).
// hist: 256 words per wave; groups 0 and 1 count in the low and high 16 bits
// of words 0..127, groups 2 and 3 in words 128..255 (at most 512 keys per
// row).  act: this group's row exists (uniform within the group).  Candidate
// positions go to sel[0..ce) of the group's row.
template <int KT>
__device__ __forceinline__ void group_select(const uint32_t (&kv)[KT], int tmax, uint32_t lo, uint32_t hi,
                                             bool act, int ce, uint32_t* hist, uint64_t* lst,
                                             uint16_t* sel) {
    static_assert(KT <= 32, "one bit per key column");
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));  // lane-derived addresses stay local to the call
    const int gq = lane >> 4, gl = lane & 15;
    const uint32_t gmask_below = (1u << gl) - 1u;
    lo = group16_min(lo);
    hi = group16_max(hi);
    int rem = ce - 1;
    bool single = false, ranked = false;
    uint64_t thr = 0;  // ranked: the (key, position) of rank rem
    bool done = !act;
    uint32_t* h = hist + (gq >> 1) * 128;
    const uint32_t inc = (gq & 1) ? 65536u : 1u;
    const int hsh = (gq & 1) ? 16 : 0;
    while (__any(!done)) {
        int shift = 0;
        if (!done && hi == lo) {
            single = true;
            done = true;
        }
        if (!done) {
            const int bits = 32 - __clz(static_cast<int>(hi - lo));
            shift = bits > 7 ? bits - 7 : 0;
        }
        *reinterpret_cast<uint4*>(hist + 4 * lane) = make_uint4(0u, 0u, 0u, 0u);
        wave_lds_sync();
        if (!done) {
            // blocks of eight key columns, a block wholly past the leaf
            // skipped; inside a block every key adds inc to its bin when it
            // lies in [lo, hi] (the invalid key ~0 never does), else 0 to a
            // bin of the lane's own (no branch per key)
            const uint32_t span = hi - lo;
#pragma unroll
            for (int t0 = 0; t0 < KT; t0 += 8) {
                if (t0 >= tmax) continue;
#pragma unroll
                for (int u = 0; u < 8 && t0 + u < KT; ++u) {
                    const uint32_t off = kv[t0 + u] - lo;
                    const bool in = off <= span;
                    atomicAdd(&h[in ? (off >> shift) : static_cast<uint32_t>(8 * gl + u)], in ? inc : 0u);
                }
            }
        }
        wave_lds_sync();
        // lane l of the group reads bins 8l .. 8l+7 of its row
        const uint4 wa = *reinterpret_cast<const uint4*>(h + 8 * gl);
        const uint4 wb = *reinterpret_cast<const uint4*>(h + 8 * gl + 4);
        wave_lds_sync();  // read before the next pass clears it
        const int cb[8] = {static_cast<int>((wa.x >> hsh) & 0xffffu), static_cast<int>((wa.y >> hsh) & 0xffffu),
                           static_cast<int>((wa.z >> hsh) & 0xffffu), static_cast<int>((wa.w >> hsh) & 0xffffu),
                           static_cast<int>((wb.x >> hsh) & 0xffffu), static_cast<int>((wb.y >> hsh) & 0xffffu),
                           static_cast<int>((wb.z >> hsh) & 0xffffu), static_cast<int>((wb.w >> hsh) & 0xffffu)};
        int local = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) local += cb[q];
        // exclusive scan over the 16 lanes of the group
        int incl = local;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const int y = group16_up(incl, o);
            if (gl >= o) incl += y;
        }
        const int excl = incl - local;
        const bool mine = !done && excl <= rem && rem < incl;
        int digit = 0, nrem = 0, cnt = 0;
        if (mine) {
            int cum = excl;
            bool got = false;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (!got && rem < cum + cb[q]) {
                    digit = 8 * gl + q;
                    nrem = rem - cum;
                    cnt = cb[q];
                    got = true;
                }
                cum += cb[q];
            }
        }
        const uint32_t gb = static_cast<uint32_t>(__ballot(mine) >> (16 * gq)) & 0xffffu;
        const int src = 16 * gq + (gb ? __builtin_ctz(gb) : 0);
        digit = __shfl(digit, src, kWave);
        nrem = __shfl(nrem, src, kWave);
        cnt = __shfl(cnt, src, kWave);
        bool rank_now = false;
        if (!done) {
            const uint32_t lo2 = lo + (static_cast<uint32_t>(digit) << shift);
            const uint32_t w = shift == 0 ? 0u : ((1u << shift) - 1u);
            hi = (hi - lo2 > w) ? lo2 + w : hi;
            lo = lo2;
            rem = nrem;
            if (nrem == cnt - 1) {
                done = true;  // every key of the bin is needed: take keys <= hi
            } else if (shift == 0) {
                single = true;
                done = true;
            } else if (cnt <= 32) {
                rank_now = true;
                done = true;
            }
        }
        if (__any(rank_now)) {
            // the bin's (key, position) pairs (in any order: the pairs are
            // distinct), then each one's rank among them; the pair of rank
            // rem is the threshold
            uint32_t inb = 0u;
            int nin = 0;
#pragma unroll
            for (int t = 0; t < KT; ++t) {
                if (t >= tmax) break;
                const bool in = rank_now && kv[t] >= lo && kv[t] <= hi;
                inb |= in ? (1u << t) : 0u;
                nin += in ? 1 : 0;
            }
            int j = group16_excl_scan(nin, gl);
#pragma unroll
            for (int t = 0; t < KT; ++t) {
                if (t >= tmax) break;
                if ((inb >> t) & 1u)
                    lst[j++] = (static_cast<uint64_t>(kv[t]) << 32) | static_cast<uint32_t>(t * 16 + gl);
            }
            wave_lds_sync();
            const uint64_t e0 = (rank_now && gl < cnt) ? lst[gl] : ~0ull;
            const uint64_t e1 = (rank_now && gl + 16 < cnt) ? lst[gl + 16] : ~0ull;
            int r0 = 0, r1 = 0;
            for (int q = 0; q < 32; ++q) {
                if (__all(q >= cnt || !rank_now)) break;
                const uint64_t v = (rank_now && q < cnt) ? lst[q] : ~0ull;
                r0 += v < e0 ? 1 : 0;
                r1 += v < e1 ? 1 : 0;
            }
            const bool h0 = rank_now && gl < cnt && r0 == rem;
            const bool h1 = rank_now && gl + 16 < cnt && r1 == rem;
            const uint64_t mine_thr = h0 ? e0 : e1;
            const uint32_t hb = static_cast<uint32_t>(__ballot(h0 || h1) >> (16 * gq)) & 0xffffu;
            const int hs = 16 * gq + (hb ? __builtin_ctz(hb) : 0);
            const uint64_t t2 = shfl_u64(mine_thr, hs);
            if (rank_now) {
                thr = t2;
                ranked = true;
            }
            wave_lds_sync();  // the list is read before it is written again
        }
    }
    if (__all(!single)) {
        // every (key, position) <= thr, thr = (hi, any position) unless ranked;
        // written in any order (the re-rank sorts the candidates)
        const uint64_t th = ranked ? thr : ((static_cast<uint64_t>(hi) << 32) | 0xffffffffull);
        uint32_t tb = 0u;
        int nt = 0;
#pragma unroll
        for (int t = 0; t < KT; ++t) {
                if (t >= tmax) break;
            const uint64_t kp = (static_cast<uint64_t>(kv[t]) << 32) | static_cast<uint32_t>(t * 16 + gl);
            const bool take = act && kp <= th;
            tb |= take ? (1u << t) : 0u;
            nt += take ? 1 : 0;
        }
        int j = group16_excl_scan(nt, gl);
#pragma unroll
        for (int t = 0; t < KT; ++t) {
            if (t >= tmax) break;
            if ((tb >> t) & 1u) sel[j++] = static_cast<uint16_t>(t * 16 + gl);
        }
        return;
    }
    // some group of the wave ends on a single value: the taken keys in
    // position order (t, lane): keys < lo (all needed), then every key in
    // [lo, hi]; or, ranked, every (key, position) <= thr; or, when the bin is
    // the single value lo, the first rem + 1 keys equal to it
    int taken = 0, eq_seen = 0;
#pragma unroll
    for (int t = 0; t < KT; ++t) {
                if (t >= tmax) break;
        const uint32_t kt = kv[t];
        const uint64_t kp = (static_cast<uint64_t>(kt) << 32) | static_cast<uint32_t>(t * 16 + gl);
        const bool lt = act && (ranked ? kp <= thr : single ? kt < lo : kt <= hi);
        const bool eq = act && single && kt == lo;
        const uint32_t beq = static_cast<uint32_t>(__ballot(eq) >> (16 * gq)) & 0xffffu;
        const int eq_rank = eq_seen + __popc(beq & gmask_below);
        const bool take = lt || (eq && eq_rank <= rem);
        const uint32_t bt = static_cast<uint32_t>(__ballot(take) >> (16 * gq)) & 0xffffu;
        if (take) sel[taken + __popc(bt & gmask_below)] = static_cast<uint16_t>(t * 16 + gl);
        taken += __popc(bt);
        eq_seen += __popc(beq);
    }
}

// exchange with lane ^ lm inside a 16-lane row, by DPP: quad permutes for 1
// and 2, a rotation by 8 within the row for 8, and for 4 the rotation by 4
// (lanes with bit 2 set) or by 12 (the others)
__device__ __forceinline__ uint32_t xchg16(uint32_t v, int lm) {
    switch (lm) {
        case 1: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0xB1, 0xf, 0xf, false));
        case 2: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x4E, 0xf, 0xf, false));
        case 8: return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x128, 0xf, 0xf, false));
        default: {
            const uint32_t a = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x124, 0xf, 0xf, false));
            const uint32_t b = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x12C, 0xf, 0xf, false));
            return (threadIdx.x & 4) ? a : b;
        }
    }
}
__device__ __forceinline__ uint64_t xchg16_u64(uint64_t v, int lm) {
    const uint32_t lo = xchg16(static_cast<uint32_t>(v), lm), hi = xchg16(static_cast<uint32_t>(v >> 32), lm);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Ascending bitonic sort of NR independent rows of 64 keys per 16-lane group,
// four keys per lane: element e of a row is lane (e >> 2) of the group,
// register e & 3.  Distances 1 and 2 stay in registers; the others exchange
// with lane xor (distance / 4), inside the group.  The NR rows' stages are
// interleaved.
template <int NR>
__device__ __forceinline__ void group_sort64(uint64_t (&v)[NR][4]) {
    const int gl = threadIdx.x & 15;
#pragma unroll
    for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
        for (int j = size >> 1; j >= 1; j >>= 1) {
            if (j >= 4) {
                const int lm = j >> 2;
                uint64_t o[NR][4];
#pragma unroll
                for (int q = 0; q < NR; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r) o[q][r] = xchg16_u64(v[q][r], lm);
                const bool lower = (gl & lm) == 0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int e = gl * 4 + r;
                    const bool take_min = ((e & size) == 0) == lower;
#pragma unroll
                    for (int q = 0; q < NR; ++q) {
                        const bool lt = v[q][r] < o[q][r];
                        v[q][r] = (take_min == lt) ? v[q][r] : o[q][r];
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int p = r ^ j;
                    if (p > r) {
                        const bool up = ((gl * 4 + r) & size) == 0;
#pragma unroll
                        for (int q = 0; q < NR; ++q) {
                            const uint64_t a = v[q][r], b = v[q][p];
                            const bool sw = up ? (a > b) : (a < b);
                            v[q][r] = sw ? b : a;
                            v[q][p] = sw ? a : b;
                        }
                    }
                }
            }
        }
    }
}

// (512-point leaves: three waves per SIMD, three workgroups per compute unit in
// 3 x 51 KB of LDS; smaller leaves: four, in at most 4 x 32 KB)
template <int FMT, int MP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MP <= 256 ? 4 : 3))) void k_leaf_wide(
    const float* __restrict__ X, const uint8_t* __restrict__ Xr, int64_t n, int D, int Dp, int rsb,
    const float* __restrict__ nrm, const float* __restrict__ sinv, int k, int c,
    const int32_t* __restrict__ perm, const LeafRec* __restrict__ leaves,
    int32_t* __restrict__ cand_ids, float* __restrict__ cand_d,
    unsigned long long* __restrict__ pairs) {
    using F = Frag<FMT>;
    constexpr int NW = 4, NTH = NW * kWave;
    constexpr int KT = MP / 16;        // keys per lane in the selection (= column tiles)
    constexpr int TPW = KT / NW;       // column tiles per wave in the Gram
    constexpr int RB = 64;             // rows per batch
    constexpr int QQ = RB / (4 * NW);  // re-rank: quads of rows per wave
    constexpr int NSW = 4;             // waves that select (four rows of a 16-row panel each)
    constexpr int CW = 8;              // dimensions per staged chunk
    constexpr int SS = 12;             // floats per staged row (16-byte aligned)
    constexpr int PF = (2 * MP + NTH - 1) / NTH;  // staged float4 per thread
    constexpr int kPanel = 16 * (MP + 1);
    constexpr int kStage = MP * SS;
    constexpr int kRegion = kPanel > kStage ? kPanel : kStage;
    static_assert(TPW >= 1 && KT % NW == 0, "tile shape");
    constexpr int kShortK = 4;         // FP8 rows of Dp <= 128: one load round per Gram group

    __shared__ __align__(16) float region[kRegion];  // d~ panel, later FP32 row chunks
    __shared__ uint16_t csel[RB * kWave];            // per batch row its candidate positions
    __shared__ int32_t ids[MP];
    __shared__ float snrm[MP], ssinv[MP];
    __shared__ __align__(16) uint32_t s_hist[NSW * 256];
    float(*dist)[MP + 1] = reinterpret_cast<float(*)[MP + 1]>(region);

    const LeafRec lf = leaves[blockIdx.x];
    const int m = lf.size;
    const size_t base = static_cast<size_t>(lf.tree) * n + lf.start;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int gq = lane >> 4, gl = lane & 15;
    load_leaf_sorted<MP, NTH>(perm + base, m, reinterpret_cast<int32_t*>(region), ids, snrm, ssinv,
                              nrm, sinv);
    if (tid == 0 && pairs != nullptr)
        stat_add(pairs, blockIdx.x, static_cast<unsigned long long>(m) * static_cast<unsigned long long>(m - 1));
    __syncthreads();
    const int ce = c < m - 1 ? c : m - 1;  // candidates per row
    const size_t rstride = static_cast<size_t>(rsb);  // bytes per row
    const int kg = lane >> 4;

    // this thread's share of an 8-dimension chunk of the leaf's FP32 rows
    auto fetch = [&](int d0, float4 (&pf)[PF]) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int idx = tid + u * NTH;
            const int j = idx >> 1, d = d0 + 4 * (idx & 1);
            pf[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j < m && d < D) pf[u] = *reinterpret_cast<const float4*>(X + static_cast<size_t>(ids[j]) * D + d);
        }
    };

    for (int p0 = 0; p0 < m; p0 += RB) {
        const int nb = m - p0 < RB ? m - p0 : RB;
        __syncthreads();  // the previous batch's last chunk is no longer read
        // ---- selection, one 16-row panel at a time
        for (int pp = 0; pp < nb; pp += 16) {
            const int prow = p0 + pp;
            // the leaf size as a per-lane value taken anew each panel: the
            // compiler would otherwise keep one lane mask per column tile
            // (col < m) live across the whole kernel
            int mv = m, lnv = lane;
            asm volatile("" : "+v"(mv), "+v"(lnv));
            const int glp = lnv & 15;  // gl, likewise taken anew
            // Gram of the panel, in groups of GT column tiles per wave; wave wv
            // takes tiles wv, wv + NW, ... so that the tiles holding columns
            // (the leaf's first m) are spread over the waves, and a group
            // wholly past the leaf is skipped (its keys are never read)
            constexpr int GT = TPW < 4 ? TPW : 4;
#pragma unroll
            for (int tg = 0; tg < TPW; tg += GT) {
                if ((tg * NW + wv) * 16 >= m) continue;
                const int arow = prow + glp;
                const uint8_t* ap = Xr + static_cast<size_t>(ids[arow < mv ? arow : 0]) * rstride +
                                    static_cast<size_t>(8 * kg) * F::kBytes;
                const uint8_t* bp[GT];
                bool bok[GT];
#pragma unroll
                for (int t = 0; t < GT; ++t) {
                    const int bcol = ((tg + t) * NW + wv) * 16 + glp;
                    bok[t] = bcol < mv;
                    bp[t] = Xr + static_cast<size_t>(ids[bcol < mv ? bcol : 0]) * rstride +
                            static_cast<size_t>(8 * kg) * F::kBytes;
                }
                f32x4 acc[GT];
#pragma unroll
                for (int t = 0; t < GT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
                if (FMT == kFP8 && Dp <= 32 * kShortK) {
                    // rows of at most kShortK 32-element steps: every step's
                    // fragments are loaded at once (one memory round trip),
                    // then the same MFMA steps in the same order
                    FragVec<FMT> as[kShortK], bs[GT][kShortK];
#pragma unroll
                    for (int q = 0; q < kShortK; ++q) {
                        const size_t off = static_cast<size_t>(32 * q) * F::kBytes;
                        const bool inq = 32 * q < Dp;
                        as[q] = load_frag<FMT>(ap + off, inq && arow < mv);
#pragma unroll
                        for (int t = 0; t < GT; ++t) bs[t][q] = load_frag<FMT>(bp[t] + off, inq && bok[t]);
                    }
#pragma unroll
                    for (int q = 0; q < kShortK; ++q)
                        if (32 * q < Dp) {
#pragma unroll
                            for (int t = 0; t < GT; ++t) acc[t] = F::mma(as[q], bs[t][q], acc[t]);
                        }
                } else {
                    FragVec<FMT> a = load_frag<FMT>(ap, arow < mv);
                    FragVec<FMT> b[GT];
#pragma unroll
                    for (int t = 0; t < GT; ++t) b[t] = load_frag<FMT>(bp[t], bok[t]);
                    for (int k0 = 0; k0 < Dp; k0 += 32) {
                        const size_t nx = static_cast<size_t>(k0 + 32) * F::kBytes;
                        const bool more = k0 + 32 < Dp;
                        const FragVec<FMT> an = load_frag<FMT>(ap + nx, more && arow < mv);
                        FragVec<FMT> bn[GT];
#pragma unroll
                        for (int t = 0; t < GT; ++t) bn[t] = load_frag<FMT>(bp[t] + nx, more && bok[t]);
#pragma unroll
                        for (int t = 0; t < GT; ++t) acc[t] = F::mma(a, b[t], acc[t]);
                        a = an;
#pragma unroll
                        for (int t = 0; t < GT; ++t) b[t] = bn[t];
                    }
                }
#pragma unroll
                for (int t = 0; t < GT; ++t) {
                    const int col = ((tg + t) * NW + wv) * 16 + glp;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int rl = 4 * kg + i;
                        const int row = prow + rl;
                        float v = __int_as_float(0x7f800000);
                        if (row < mv && col < mv)
                            v = snrm[row] + snrm[col] - 2.f * acc[t][i] * (ssinv[row] * ssinv[col]);
                        dist[rl][col] = v;
                    }
                }
            }
            __syncthreads();
            if (wv < NSW) {
                // group gq of wave wv: panel row 4 wv + gq
                const int rl = 4 * wv + gq;
                const int row = prow + rl;
                const bool act = rl < nb - pp;
                uint16_t* sel = csel + (pp + (act ? rl : 0)) * kWave;
                const int tmax = (m + 15) >> 4;  // key columns holding members
                if (ce >= m - 1) {  // every other member is a candidate
                    if (act) {
#pragma unroll
                        for (int t = 0; t < KT; ++t) {
                            if ((t & ~7) >= tmax) continue;  // (~0 keys past the leaf are inert)
                            const int col = t * 16 + glp;
                            const int e = col < row ? col : col - 1;
                            if (col < mv && col != row) sel[e] = static_cast<uint16_t>(col);
                        }
                    }
                } else if (ce > 0) {
                    // the row's d~ as order keys in registers (invalid: ~0); the
                    // row's panel line then holds the selection's pair list
                    uint32_t kv[KT];
                    uint32_t lo = 0xffffffffu, hi = 0u;
#pragma unroll
                    for (int t = 0; t < KT; ++t) kv[t] = 0xffffffffu;
#pragma unroll
                    for (int t = 0; t < KT; ++t) {
                        if ((t & ~7) >= tmax) continue;  // (~0 keys past the leaf are inert)
                        const int col = t * 16 + glp;
                        const uint32_t kt = (act && col < mv && col != row) ? fkey(dist[act ? rl : 0][col])
                                                                            : 0xffffffffu;
                        kv[t] = kt;
                        if (kt != 0xffffffffu) {
                            lo = min(lo, kt);
                            hi = max(hi, kt);
                        }
                    }
                    wave_lds_sync();
                    // (the list starts at the row's first 8-byte aligned word)
                    const int lrow = ((act ? rl : 0) * (MP + 1) + 1) & ~1;
                    group_select<KT>(kv, tmax, lo, hi, act, ce, s_hist + wv * 256,
                                     reinterpret_cast<uint64_t*>(region + lrow), sel);
                }
            }
            __syncthreads();  // the panel is no longer read
        }
        // ---- re-rank of the batch: d32 from LDS-staged 8-dimension chunks;
        // the next chunk's loads are in flight while this one is computed.
        // Wave wv, quad qq, group gq: batch row 4 QQ wv + 4 qq + gq; lane gl
        // owns candidates 4 gl + u (the selection writes each lane's picks
        // contiguously, so the 16 lanes read rows of 16 different source
        // lanes: positions of distinct residues mod 16, distinct LDS banks).
        // (table entries past a row's ce, or of rows past nb, are stale: the
        // positions are masked into the leaf and the pairs marked invalid)
        float tot[QQ][4], blk[QQ][4];
        int cby[QQ][4];      // byte offset of the candidate's staged row in region
        uint32_t cval = 0u;  // bit 4 qq + u: pair (qq, u) exists
#pragma unroll
        for (int qq = 0; qq < QQ; ++qq) {
            const int bi = 4 * QQ * wv + 4 * qq + gq;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                tot[qq][u] = 0.f;
                blk[qq][u] = 0.f;
                const int e = 4 * gl + u;
                cby[qq][u] = (static_cast<int>(csel[bi * kWave + e]) & (MP - 1)) * (SS * 4);
                cval |= (bi < nb && e < ce) ? (1u << (4 * qq + u)) : 0u;
            }
        }
        float4 pf[PF];
        fetch(0, pf);
        for (int d0 = 0; d0 < D; d0 += CW) {
            __syncthreads();  // the previous chunk (or the panel) is no longer read
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                const int idx = tid + u * NTH;
                if ((idx >> 1) < m) *reinterpret_cast<float4*>(region + (idx >> 1) * SS + 4 * (idx & 1)) = pf[u];
            }
            __syncthreads();
            if (d0 + CW < D) fetch(d0 + CW, pf);
#pragma unroll
            for (int qq = 0; qq < QQ; ++qq) {
                const int bi = 4 * QQ * wv + 4 * qq + gq;
                const float* xo = region + (p0 + (bi < nb ? bi : 0)) * SS;
                const float4 o0 = *reinterpret_cast<const float4*>(xo);
                const float4 o1 = *reinterpret_cast<const float4*>(xo + 4);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float* xc = reinterpret_cast<const float*>(reinterpret_cast<const char*>(region) + cby[qq][u]);
                    const float4 c0 = *reinterpret_cast<const float4*>(xc);
                    const float4 c1 = *reinterpret_cast<const float4*>(xc + 4);
                    float bq = blk[qq][u];  // padding past D adds exact zeros
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
                    blk[qq][u] = bq;
                }
                // one quad's loads in flight at a time (register pressure)
                __builtin_amdgcn_sched_barrier(0);
            }
            if (((d0 + CW) & 31) == 0 || d0 + CW >= D) {  // end of a 32-dimension block
#pragma unroll
                for (int qq = 0; qq < QQ; ++qq)
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        tot[qq][u] = tot[qq][u] + blk[qq][u];
                        blk[qq][u] = 0.f;
                    }
            }
        }
        // ---- per row: the k smallest (d32, id), in order; two quads of rows
        // sorted together at a time
#pragma unroll
        for (int h = 0; h < QQ / 2; ++h) {
            uint64_t v[2][4];
#pragma unroll
            for (int q2 = 0; q2 < 2; ++q2) {
                const int qq = 2 * h + q2;
                const int bi = 4 * QQ * wv + 4 * qq + gq;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = 4 * gl + u;
                    v[q2][u] = ((cval >> (4 * qq + u)) & 1u) ? cand_key(tot[qq][u], ids[cby[qq][u] / (SS * 4)]) : kNoKey;
                }
            }
            group_sort64<2>(v);
#pragma unroll
            for (int q2 = 0; q2 < 2; ++q2) {
                const int qq = 2 * h + q2;
                const int bi = 4 * QQ * wv + 4 * qq + gq;
                if (bi < nb) {
                    const size_t out = (static_cast<size_t>(lf.tree) * n + ids[p0 + bi]) * k;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int e = gl * 4 + r;
                        if (e < k) {
                            const bool ok = v[q2][r] != kNoKey;
                            cand_ids[out + e] = ok ? key_id(v[q2][r]) : -1;
                            cand_d[out + e] = ok ? key_dist(v[q2][r]) : __int_as_float(0x7f800000);
                        }
                    }
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
    const float* __restrict__ X, const uint8_t* __restrict__ Xr, int64_t n, int D, int Dp, int rsb,
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
        const size_t rstride = static_cast<size_t>(rsb);  // bytes per row
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
        const int rb = Dp * F::kBytes;  // bytes of a row the Gram reads
        const int rs = rb + 16;
        const bool staged = static_cast<size_t>(MP) * rs <= sizeof(lds);
        if (staged) {
            uint8_t* L = reinterpret_cast<uint8_t*>(lds);
            const int cpr = rb / 16;  // 16-byte chunks per row
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
            a.X, rr.Xr, a.n, a.D, rr.Dp, rr.stride, rr.nrm, rr.sinv, a.k, c, a.perm, a.leaves, a.cand_ids,
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
    // at most 64 candidates per row (and more than 32 when leaves have at most
    // 128 points): the wide kernel (knob leaf_wide = 0, KNNG_LEAF_WIDE=0,
    // keeps k_leaf_mfma)
    const bool wide = !EXACT && c <= 64 && a.D % 4 == 0 && knob(kKnobLeafWide, 1) != 0;
    if (wide) {
        if (lm <= 64) return go(k_leaf_wide<FMT, 64>);
        if (lm <= 128) return go(k_leaf_wide<FMT, 128>);
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
