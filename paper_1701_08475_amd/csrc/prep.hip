// Input checks and small layout conversions around the build.
#include "knng_internal.hpp"
#include "wave.hpp"

namespace knng {
namespace {

// flags[0] <- 1 if any element is NaN or +-Inf (exponent bits all ones);
// flags[1] <- 1 if any element is not an integer in [0, 255].
__global__ __launch_bounds__(256) void k_scan(const float* __restrict__ X, int64_t count,
                                              int32_t* __restrict__ flags) {
    int bad = 0, not_u8 = 0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
         i += stride) {
        const float v = X[i];
        const uint32_t u = __float_as_uint(v);
        bad |= ((u & 0x7f800000u) == 0x7f800000u) ? 1 : 0;
        not_u8 |= (v >= 0.f && v <= 255.f && v == rintf(v)) ? 0 : 1;
    }
    // wave votes in converged code, then one lane per wave publishes
    const bool any_bad = __any(bad), any_not_u8 = __any(not_u8);
    if ((threadIdx.x & 63) == 0) {
        if (any_bad) atomicOr(flags, 1);
        if (any_not_u8) atomicOr(flags + 1, 1);
    }
}

__global__ __launch_bounds__(256) void k_to_u8(const float* __restrict__ X, int64_t count,
                                               uint8_t* __restrict__ X8) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
         i += stride)
        X8[i] = static_cast<uint8_t>(X[i]);
}

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t v) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

// mark[start] = 1 for every leaf of `tree`.
__global__ void k_mark_leaves(const LeafRec* __restrict__ leaves, int64_t n_leaves, int tree,
                              int32_t* __restrict__ mark) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n_leaves;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        if (leaves[i].tree == tree) mark[leaves[i].start] = 1;
}

// Per block of 1024 positions: number of marks.
__global__ __launch_bounds__(256) void k_block_count(const int32_t* __restrict__ mark, int64_t n,
                                                     int32_t* __restrict__ bcount) {
    __shared__ int part[4];
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * 1024;
    int c = 0;
    for (int i = threadIdx.x; i < 1024; i += 256)
        if (b0 + i < n) c += mark[b0 + i];
    c = wave_sum_i32(c);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) bcount[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// Exclusive scan of the block counts (one block, sequential chunks).
__global__ __launch_bounds__(1024) void k_scan_counts(int32_t* __restrict__ bcount, int64_t nb,
                                                      int32_t* __restrict__ total) {
    __shared__ int s[1024];
    const int tid = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t i0 = tid * per, i1 = (i0 + per < nb) ? i0 + per : nb;
    int c = 0;
    for (int64_t i = i0; i < i1; ++i) c += bcount[i];
    s[tid] = c;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int y = tid >= o ? s[tid - o] : 0;
        __syncthreads();
        s[tid] += y;
        __syncthreads();
    }
    int run = s[tid] - c;
    for (int64_t i = i0; i < i1; ++i) {
        const int v = bcount[i];
        bcount[i] = run;
        run += v;
    }
    if (tid == 1023) *total = s[1023];
}

// offsets[rank of mark] = position, in ascending position order.
__global__ __launch_bounds__(256) void k_emit_offsets(const int32_t* __restrict__ mark, int64_t n,
                                                      const int32_t* __restrict__ bstart,
                                                      int32_t* __restrict__ offsets) {
    __shared__ int wtot[4];
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * 1024;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int run = bstart[blockIdx.x];
    for (int i0 = 0; i0 < 1024; i0 += 256) {
        const int64_t p = b0 + i0 + threadIdx.x;
        const bool f = p < n && mark[p] != 0;
        const unsigned long long b = __ballot(f);
        if (lane == 0) wtot[wv] = __popcll(b);
        __syncthreads();
        int off = 0, tot = 0;
        for (int w = 0; w < 4; ++w) {
            off += w < wv ? wtot[w] : 0;
            tot += wtot[w];
        }
        if (f) offsets[run + off + __popcll(b & ((1ull << lane) - 1ull))] = static_cast<int32_t>(p);
        run += tot;
        __syncthreads();
    }
}

__global__ void k_set_last(int32_t* offsets, const int32_t* total, int32_t n) {
    offsets[*total] = n;
}

}  // namespace

int prep_scan(const float* X, int64_t count, int32_t* flags, hipStream_t s) {
    k_fill_i32<<<1, 64, 0, s>>>(flags, 2, 0);
    const int64_t want = (count + 255) / 256;
    const int blocks = static_cast<int>(want < 4096 ? (want > 0 ? want : 1) : 4096);
    k_scan<<<blocks, 256, 0, s>>>(X, count, flags);
    return hipGetLastError() == hipSuccess ? kOk : kHip;
}

int prep_to_u8(const float* X, int64_t count, uint8_t* X8, hipStream_t s) {
    const int64_t want = (count + 255) / 256;
    const int blocks = static_cast<int>(want < 8192 ? (want > 0 ? want : 1) : 8192);
    k_to_u8<<<blocks, 256, 0, s>>>(X, count, X8);
    return hipGetLastError() == hipSuccess ? kOk : kHip;
}

int leaves_to_offsets(const LeafRec* leaves, int64_t n_leaves, int64_t n, int tree,
                      int32_t* offsets_out, int32_t* count_out_dev, hipStream_t s) {
    int32_t *mark = nullptr, *bcount = nullptr;
    const int64_t nb = (n + 1023) / 1024;
    if (ws_malloc(reinterpret_cast<void**>(&mark), sizeof(int32_t) * n, s) != hipSuccess)
        return kOom;
    if (ws_malloc(reinterpret_cast<void**>(&bcount), sizeof(int32_t) * nb, s) != hipSuccess) {
        ws_free(mark, s);
        return kOom;
    }
    const int fb = static_cast<int>((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    k_fill_i32<<<fb, 256, 0, s>>>(mark, n, 0);
    k_mark_leaves<<<256, 256, 0, s>>>(leaves, n_leaves, tree, mark);
    k_block_count<<<static_cast<unsigned>(nb), 256, 0, s>>>(mark, n, bcount);
    k_scan_counts<<<1, 1024, 0, s>>>(bcount, nb, count_out_dev);
    k_emit_offsets<<<static_cast<unsigned>(nb), 256, 0, s>>>(mark, n, bcount, offsets_out);
    k_set_last<<<1, 1, 0, s>>>(offsets_out, count_out_dev, static_cast<int32_t>(n));
    const hipError_t e = hipGetLastError();
    ws_free(mark, s);
    ws_free(bcount, s);
    return e == hipSuccess ? kOk : kHip;
}

}  // namespace knng

namespace knng {

KernelTimer::~KernelTimer() {
    for (int i = 0; i < n_; ++i) {
        hipEventDestroy(pairs_[i].a);
        hipEventDestroy(pairs_[i].b);
    }
    delete[] pairs_;
}

void KernelTimer::begin(KernelClass c, hipStream_t s) {
    if (!on_) return;
    if (n_ == cap_) {
        const int nc = cap_ ? 2 * cap_ : 256;
        Pair* p = new Pair[nc];
        for (int i = 0; i < n_; ++i) p[i] = pairs_[i];
        delete[] pairs_;
        pairs_ = p;
        cap_ = nc;
    }
    Pair& q = pairs_[n_];
    if (hipEventCreate(&q.a) != hipSuccess || hipEventCreate(&q.b) != hipSuccess) {
        on_ = false;  // timing is best effort; the build goes on
        return;
    }
    q.cls = c;
    hipEventRecord(q.a, s);
    open_ = n_++;
}

void KernelTimer::end(KernelClass c, hipStream_t s) {
    if (!on_ || open_ < 0) return;
    (void)c;
    hipEventRecord(pairs_[open_].b, s);
    open_ = -1;
}

void KernelTimer::collect(float ms[kKClasses], int count[kKClasses]) {
    for (int c = 0; c < kKClasses; ++c) {
        ms[c] = 0.f;
        count[c] = 0;
    }
    for (int i = 0; i < n_; ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, pairs_[i].a, pairs_[i].b) == hipSuccess) {
            ms[pairs_[i].cls] += t;
            count[pairs_[i].cls] += 1;
        }
    }
}

}  // namespace knng
