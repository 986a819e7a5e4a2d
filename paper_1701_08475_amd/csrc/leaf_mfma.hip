// Reduced-precision leaf search: row preparation and format dispatch (the
// kernels are in leaf_mfma_impl.hpp, one translation unit per format).
#include "leaf_mfma_impl.hpp"

namespace knng {
namespace leafk {
int run_bf16(const LeafArgs& a, const ReducedRows& rr, int* launches, char* err, size_t errlen);
int run_f16(const LeafArgs& a, const ReducedRows& rr, int* launches, char* err, size_t errlen);
int run_fp8(const LeafArgs& a, const ReducedRows& rr, int* launches, char* err, size_t errlen);
}  // namespace leafk
namespace {
using namespace leafk;
// ------------------------------------------------------------- prep
// Reduced copy of every row (one wave per row): sigma = 2^(E_max - floor(log2
// max|x|) - 1) with E_max = 15 (FP16) or 8 (FP8-e4m3) so that |sigma x| <
// 2^E_max; sigma = 1 for BF16.  x~ = round-to-nearest-even(sigma x); the row
// holds Dp elements (zero past D), then 1/sigma as an FP32 word (so that a
// gathered row brings its scale in the same cache line), then zeros to the
// stride.  n~ = sum of (x~ / sigma)^2 (FP32, fixed order).
__device__ __forceinline__ uint16_t to_bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    return static_cast<uint16_t>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) {
    return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

template <int FMT>
__global__ __launch_bounds__(256) void k_prep_reduced(const float* __restrict__ X, int64_t n, int D,
                                                      int Dp, int rsb, uint8_t* __restrict__ Xr,
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
    // e2: sum of (sigma x_i - x~_i)^2 in FP64; sigma x_i is exact in FP64 (a
    // power-of-two scaling), each difference is exact (both lie on the grid
    // of sigma x_i's last place, within two of its binades), so are the squares
    double e2 = 0.0;
    const int Ds = rsb / (FMT == kFP8 ? 1 : 2);  // elements per row in memory (zeros past Dp)
    const int Sw = Dp + (FMT == kFP8 ? 8 : 4);     // elements Dp .. Sw-1 hold 1/sigma and e
    if constexpr (FMT == kFP8) {
        uint8_t* o = Xr + row * rsb;
        for (int d0 = 2 * lane; d0 < Ds; d0 += 2 * kWave) {
            if (d0 >= Dp && d0 < Sw) continue;
            const float a = d0 < D ? x[d0] * sig : 0.f;
            const float b = d0 + 1 < D ? x[d0 + 1] * sig : 0.f;
            const uint32_t pk = static_cast<uint32_t>(__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false));
            o[d0] = static_cast<uint8_t>(pk & 255u);
            o[d0 + 1] = static_cast<uint8_t>((pk >> 8) & 255u);
            // dequantised values, to the same FP32 the MFMA multiplies
            const float qa = __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(pk), 0);
            const float qb = __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(pk), 1);
            const double ea = (d0 < D ? static_cast<double>(x[d0]) * sig : 0.0) - qa;
            const double eb = (d0 + 1 < D ? static_cast<double>(x[d0 + 1]) * sig : 0.0) - qb;
            e2 += ea * ea + eb * eb;
            const float da = qa * isg;
            const float db = qb * isg;
            s = __fmaf_rn(da, da, s);
            s = __fmaf_rn(db, db, s);
        }
    } else {
        uint16_t* o = reinterpret_cast<uint16_t*>(Xr + row * rsb);
        for (int d = lane; d < Ds; d += kWave) {
            if (d >= Dp && d < Sw) continue;
            const float v = d < D ? x[d] * sig : 0.f;
            float q;
            if constexpr (FMT == kBF16) {
                const uint16_t h = to_bf16_rne(v);
                o[d] = h;
                q = bf16_to_f(h);
            } else {
                const _Float16 h = static_cast<_Float16>(v);
                o[d] = __builtin_bit_cast(uint16_t, h);
                q = static_cast<float>(h);
            }
            const double e = (d < D ? static_cast<double>(x[d]) * sig : 0.0) - q;
            e2 += e * e;
            const float dq = q * isg;
            s = __fmaf_rn(dq, dq, s);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        s += __shfl_xor(s, o, kWave);
        e2 += shfl_xor_f64(e2, o);
    }
    if (lane == 0) {
        nrm[row] = s;
        sinv[row] = isg;
        *reinterpret_cast<float*>(Xr + row * rsb + reduced_rows_scale_offset(FMT, Dp)) = isg;
        // e: |sigma x - x~|_2 rounded up to FP32 (the FP64 sum of at most 2^11
        // exact squares is within 2^-42 of the true one)
        const double ed = sqrt(e2 * (1.0 + 0x1p-40));
        float ef = static_cast<float>(ed);
        if (static_cast<double>(ef) < ed) ef = nextafterf(ef, __int_as_float(0x7f800000));
        *reinterpret_cast<float*>(Xr + row * rsb + reduced_rows_err_offset(FMT, Dp)) = ef;
    }
}

}  // namespace

int reduced_rows_dp(int D) { return (D + 31) / 32 * 32; }

int reduced_rows_stride(int precision, int D) {
    return (reduced_rows_err_offset(precision, reduced_rows_dp(D)) + 4 + 127) / 128 * 128;
}

size_t reduced_rows_bytes(int precision, int64_t n, int D) {
    return static_cast<size_t>(n) * reduced_rows_stride(precision, D);
}

int prep_reduced(int precision, const float* X, int64_t n, int D, ReducedRows* rr, hipStream_t s) {
    const unsigned blocks = static_cast<unsigned>((n + 3) / 4);
    switch (precision) {
        case kBF16: k_prep_reduced<kBF16><<<blocks, 256, 0, s>>>(X, n, D, rr->Dp, rr->stride, rr->Xr, rr->nrm, rr->sinv); break;
        case kF16: k_prep_reduced<kF16><<<blocks, 256, 0, s>>>(X, n, D, rr->Dp, rr->stride, rr->Xr, rr->nrm, rr->sinv); break;
        case kFP8: k_prep_reduced<kFP8><<<blocks, 256, 0, s>>>(X, n, D, rr->Dp, rr->stride, rr->Xr, rr->nrm, rr->sinv); break;
        default: return kUnsupported;
    }
    return hipGetLastError() == hipSuccess ? kOk : kHip;
}

namespace {

// Size buckets of the leaf list: leaves of at most 64, 128, 256 and 512
// points; each bucket runs the kernel shaped for its bound (fewer waves and
// less LDS per workgroup for the smaller ones).
constexpr int kBuckets = 4;
constexpr int kBucketMax[kBuckets] = {64, 128, 256, 512};

__device__ __forceinline__ int bucket_of(int size) {
    return size <= 64 ? 0 : size <= 128 ? 1 : size <= 256 ? 2 : 3;
}

// cnt[0..3] <- leaves per bucket (cnt zeroed by the caller).
__global__ void k_bucket_count(const LeafRec* __restrict__ leaves, int64_t nl,
                               int32_t* __restrict__ cnt) {
    __shared__ int32_t s[kBuckets];
    if (threadIdx.x < kBuckets) s[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < nl;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        atomicAdd(&s[bucket_of(leaves[i].size)], 1);
    __syncthreads();
    if (threadIdx.x < kBuckets && s[threadIdx.x] != 0) atomicAdd(&cnt[threadIdx.x], s[threadIdx.x]);
}

// out <- the leaves grouped by bucket, bucket b from the sum of the counts
// before it (cnt[0..3]); order inside a bucket is arbitrary (every leaf
// writes only its own rows' lists).  cursor[0..3] zeroed by the caller.  The
// slots are taken per wavefront: one atomic per bucket and step, each lane's
// slot from the ballot of its bucket.
__global__ void k_bucket_fill(const LeafRec* __restrict__ leaves, int64_t nl,
                              const int32_t* __restrict__ cnt, int32_t* __restrict__ cursor,
                              LeafRec* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    int64_t first[kBuckets];
    first[0] = 0;
    for (int q = 1; q < kBuckets; ++q) first[q] = first[q - 1] + cnt[q - 1];
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i0 = blockIdx.x * static_cast<int64_t>(blockDim.x) + (threadIdx.x & ~63); i0 < nl;
         i0 += stride) {  // uniform per wavefront
        const int64_t i = i0 + lane;
        const bool live = i < nl;
        LeafRec r{};
        int b = -1;
        if (live) {
            r = leaves[i];
            b = bucket_of(r.size);
        }
#pragma unroll
        for (int q = 0; q < kBuckets; ++q) {
            const uint64_t m = __ballot(b == q);
            if (m == 0) continue;
            int slot0 = 0;
            if (lane == __builtin_ctzll(m)) slot0 = atomicAdd(&cursor[q], __popcll(m));
            slot0 = __shfl(slot0, __builtin_ctzll(m), kWave);
            if (b == q) out[first[q] + slot0 + __popcll(m & below)] = r;
        }
    }
}

__global__ void k_zero8(int32_t* p) {
    if (threadIdx.x < 8) p[threadIdx.x] = 0;
}

int run_format(const LeafArgs& a, const ReducedRows& rr, int* launches, char* err,
               size_t errlen) {
    switch (a.precision) {
        case kBF16: return leafk::run_bf16(a, rr, launches, err, errlen);
        case kF16: return leafk::run_f16(a, rr, launches, err, errlen);
        case kFP8: return leafk::run_fp8(a, rr, launches, err, errlen);
        default:
            std::snprintf(err, errlen, "precision %d has no MFMA path", a.precision);
            return kUnsupported;
    }
}

}  // namespace

int leaf_run_mfma(const LeafArgs& a, const ReducedRows& rr, int* launches, char* err,
                  size_t errlen) {
    const int c = a.rerank < a.k ? a.k : a.rerank;
    if (c > 128 || a.k > 128) {
        std::snprintf(err, errlen, "rerank candidates %d (k=%d) exceed 128", c, a.k);
        return kUnsupported;
    }
    // one launch shaped by the largest leaf when every leaf fits 128 points
    // or the knob leaf_buckets is 0 (KNNG_LEAF_BUCKETS=0); else one launch per
    // non-empty size bucket
    const bool bucketed = knob(kKnobLeafBuckets, 1) != 0 && a.leaf_max > 128 && a.n_leaves > 0;
    if (!bucketed) return run_format(a, rr, launches, err, errlen);
    hipStream_t s = a.stream;
    int32_t* ctr = nullptr;  // [0..3] counts, [4..7] fill cursors
    LeafRec* grouped = nullptr;
    hipError_t e = ws_malloc(reinterpret_cast<void**>(&ctr), 8 * sizeof(int32_t), s);
    if (e == hipSuccess)
        e = ws_malloc(reinterpret_cast<void**>(&grouped), sizeof(LeafRec) * a.n_leaves, s);
    int rc = kOk;
    int32_t h[kBuckets] = {0, 0, 0, 0};
    if (e == hipSuccess) {
        const unsigned g = static_cast<unsigned>(std::min<int64_t>((a.n_leaves + 255) / 256, 1024));
        k_zero8<<<1, 64, 0, s>>>(ctr);
        k_bucket_count<<<g, 256, 0, s>>>(a.leaves, a.n_leaves, ctr);
        k_bucket_fill<<<g, 256, 0, s>>>(a.leaves, a.n_leaves, ctr, ctr + kBuckets, grouped);
        e = hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        *launches += 3;
    }
    if (e != hipSuccess) {
        std::snprintf(err, errlen, "leaf buckets: %s", hipGetErrorString(e));
        rc = kHip;
    }
    int64_t base = 0;
    for (int b = 0; b < kBuckets && rc == kOk; ++b) {
        if (h[b] == 0) continue;
        LeafArgs ab = a;
        ab.leaves = grouped + base;
        ab.n_leaves = h[b];
        ab.leaf_max = std::min(a.leaf_max, kBucketMax[b]);
        rc = run_format(ab, rr, launches, err, errlen);
        base += h[b];
    }
    if (grouped != nullptr) ws_free(grouped, s);
    if (ctr != nullptr) ws_free(ctr, s);
    return rc;
}

}  // namespace knng
