// Wavefront-level building blocks for gfx950 (64 lanes per wavefront).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace knng {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
    uint32_t lo = static_cast<uint32_t>(v), hi = static_cast<uint32_t>(v >> 32);
    lo = __shfl_xor(lo, mask, kWave);
    hi = __shfl_xor(hi, mask, kWave);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    uint32_t lo = static_cast<uint32_t>(v), hi = static_cast<uint32_t>(v >> 32);
    lo = __shfl(lo, src, kWave);
    hi = __shfl(hi, src, kWave);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ double shfl_xor_f64(double v, int mask) {
    return __longlong_as_double(static_cast<long long>(
        shfl_xor_u64(static_cast<uint64_t>(__double_as_longlong(v)), mask)));
}

// Sum over all 64 lanes of an integer (order irrelevant).
__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Key of a candidate: non-negative FP32 distance bits above the id, so that
// unsigned order is (distance, id) order.  Invalid slots use ~0.
__device__ __forceinline__ uint64_t cand_key(float d, int32_t id) {
    return (static_cast<uint64_t>(__float_as_uint(d)) << 32) | static_cast<uint32_t>(id);
}
__device__ __forceinline__ float key_dist(uint64_t k) { return __uint_as_float(static_cast<uint32_t>(k >> 32)); }
__device__ __forceinline__ int32_t key_id(uint64_t k) { return static_cast<int32_t>(static_cast<uint32_t>(k)); }
constexpr uint64_t kNoKey = ~0ull;

// Ascending bitonic sort of 64*R keys held R per lane; element e = lane*R + r.
template <int R>
__device__ __forceinline__ void wave_bitonic_sort(uint64_t (&v)[R]) {
    const int lane = lane_id();
#pragma unroll
    for (int size = 2; size <= kWave * R; size <<= 1) {
#pragma unroll
        for (int j = size >> 1; j >= 1; j >>= 1) {
            if (j >= R) {
                const int lmask = j / R;  // partner lane = lane ^ lmask, same r
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int e = lane * R + r;
                    const uint64_t o = shfl_xor_u64(v[r], lmask);
                    const bool up = (e & size) == 0;
                    const bool lower = (lane & lmask) == 0;  // e < partner
                    const bool take_min = (up == lower);
                    const uint64_t mn = v[r] < o ? v[r] : o;
                    const uint64_t mx = v[r] < o ? o : v[r];
                    v[r] = take_min ? mn : mx;
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int p = r ^ j;
                    if (p > r) {
                        const int e = lane * R + r;
                        const bool up = (e & size) == 0;
                        const uint64_t a = v[r], b = v[p];
                        const bool sw = up ? (a > b) : (a < b);
                        v[r] = sw ? b : a;
                        v[p] = sw ? a : b;
                    }
                }
            }
        }
    }
}

// Exclusive prefix sum over lanes of a per-lane count (lane order).
__device__ __forceinline__ int wave_excl_scan(int v, int* total) {
    const int lane = lane_id();
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    *total = __shfl(x, kWave - 1, kWave);
    return x - v;
}

}  // namespace knng
