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
#include "knng_internal.hpp"
#include "wave.hpp"

#include <cstdio>
#include <type_traits>

namespace knng {
namespace {

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
    for (int j = tid; j < MP; j += 256) {
        const int32_t id = j < m ? perm[base + j] : 0;
        ids[j] = id;
        snrm[j] = j < m ? nrm[id] : 0.f;
        ssinv[j] = j < m ? sinv[id] : 0.f;
    }
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

// ------------------------------------------------------------- prep
// Reduced copy of every row (one wave per row): sigma = 2^(E_max - floor(log2
// max|x|) - 1) with E_max = 15 (FP16) or 8 (FP8-e4m3) so that |sigma x| <
// 2^E_max; sigma = 1 for BF16.  x~ = round-to-nearest-even(sigma x); padding
// to Dp elements is zero.  n~ = sum of (x~ / sigma)^2 (FP32, fixed order).
__device__ __forceinline__ uint16_t to_bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    return static_cast<uint16_t>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) {
    return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

template <int FMT>
__global__ __launch_bounds__(256) void k_prep_reduced(const float* __restrict__ X, int64_t n, int D,
                                                      int Dp, uint8_t* __restrict__ Xr,
                                                      float* __restrict__ nrm,
                                                      float* __restrict__ sinv) {
    const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const int lane = threadIdx.x & 63;
    const float* x = X + row * D;
    float mx = 0.f;
    for (int d = lane; d < D; d += kWave) mx = fmaxf(mx, fabsf(x[d]));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, kWave));
    float sig = 1.f;
    if (FMT != kBF16 && mx > 0.f) {
        const int emax = FMT == kF16 ? 15 : 8;
        sig = ldexpf(1.f, emax - ilogbf(mx) - 1);
    }
    const float isg = 1.f / sig;  // exact: sig is a power of two
    float s = 0.f;
    if constexpr (FMT == kFP8) {
        uint8_t* o = Xr + row * Dp;
        for (int d0 = 2 * lane; d0 < Dp; d0 += 2 * kWave) {
            const float a = d0 < D ? x[d0] * sig : 0.f;
            const float b = d0 + 1 < D ? x[d0 + 1] * sig : 0.f;
            const uint32_t pk = static_cast<uint32_t>(__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false));
            o[d0] = static_cast<uint8_t>(pk & 255u);
            o[d0 + 1] = static_cast<uint8_t>((pk >> 8) & 255u);
            // dequantised values, to the same FP32 the MFMA multiplies
            const float da = __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(pk), 0) * isg;
            const float db = __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(pk), 1) * isg;
            s = __fmaf_rn(da, da, s);
            s = __fmaf_rn(db, db, s);
        }
    } else {
        uint16_t* o = reinterpret_cast<uint16_t*>(Xr) + row * Dp;
        for (int d = lane; d < Dp; d += kWave) {
            const float v = d < D ? x[d] * sig : 0.f;
            float dq;
            if constexpr (FMT == kBF16) {
                const uint16_t h = to_bf16_rne(v);
                o[d] = h;
                dq = bf16_to_f(h) * isg;
            } else {
                const _Float16 h = static_cast<_Float16>(v);
                o[d] = __builtin_bit_cast(uint16_t, h);
                dq = static_cast<float>(h) * isg;
            }
            s = __fmaf_rn(dq, dq, s);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, kWave);
    if (lane == 0) {
        nrm[row] = s;
        sinv[row] = isg;
    }
}

template <int FMT, bool EXACT, bool VEC4>
int launch_fmt(const LeafArgs& a, const ReducedRows& rr, int* launches, char* err, size_t errlen) {
    const int lm = a.leaf_max;
    const int c = a.rerank < a.k ? a.k : a.rerank;
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
    if (lm <= 64) return go(k_leaf_mfma<FMT, 64, 64, EXACT, VEC4>);
    if (lm <= 128) return go(k_leaf_mfma<FMT, 128, 64, EXACT, VEC4>);
    if (lm <= 256) return go(k_leaf_mfma<FMT, 256, 64, EXACT, VEC4>);
    return go(k_leaf_mfma<FMT, 512, 32, EXACT, VEC4>);
}

template <int FMT>
int launch_fmt_any(const LeafArgs& a, const ReducedRows& rr, int* launches, char* err,
                   size_t errlen) {
    const bool v4 = a.D % 4 == 0;
    if (rr.exact) return v4 ? launch_fmt<FMT, true, true>(a, rr, launches, err, errlen)
                            : launch_fmt<FMT, true, false>(a, rr, launches, err, errlen);
    return v4 ? launch_fmt<FMT, false, true>(a, rr, launches, err, errlen)
              : launch_fmt<FMT, false, false>(a, rr, launches, err, errlen);
}

}  // namespace

int reduced_rows_dp(int D) { return (D + 31) / 32 * 32; }

size_t reduced_rows_bytes(int precision, int64_t n, int D) {
    const size_t eb = precision == kFP8 ? 1 : 2;
    return static_cast<size_t>(n) * reduced_rows_dp(D) * eb;
}

int prep_reduced(int precision, const float* X, int64_t n, int D, ReducedRows* rr, hipStream_t s) {
    const unsigned blocks = static_cast<unsigned>((n + 3) / 4);
    switch (precision) {
        case kBF16: k_prep_reduced<kBF16><<<blocks, 256, 0, s>>>(X, n, D, rr->Dp, rr->Xr, rr->nrm, rr->sinv); break;
        case kF16: k_prep_reduced<kF16><<<blocks, 256, 0, s>>>(X, n, D, rr->Dp, rr->Xr, rr->nrm, rr->sinv); break;
        case kFP8: k_prep_reduced<kFP8><<<blocks, 256, 0, s>>>(X, n, D, rr->Dp, rr->Xr, rr->nrm, rr->sinv); break;
        default: return kUnsupported;
    }
    return hipGetLastError() == hipSuccess ? kOk : kHip;
}

int leaf_run_mfma(const LeafArgs& a, const ReducedRows& rr, int* launches, char* err,
                  size_t errlen) {
    const int c = a.rerank < a.k ? a.k : a.rerank;
    if (c > 128 || a.k > 128) {
        std::snprintf(err, errlen, "rerank candidates %d (k=%d) exceed 128", c, a.k);
        return kUnsupported;
    }
    switch (a.precision) {
        case kBF16: return launch_fmt_any<kBF16>(a, rr, launches, err, errlen);
        case kF16: return launch_fmt_any<kF16>(a, rr, launches, err, errlen);
        case kFP8: return launch_fmt_any<kFP8>(a, rr, launches, err, errlen);
        default:
            std::snprintf(err, errlen, "precision %d has no MFMA path", a.precision);
            return kUnsupported;
    }
}

}  // namespace knng
