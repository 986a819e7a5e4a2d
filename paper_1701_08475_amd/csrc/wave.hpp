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

// DPP exchange of a double between lanes of a 16-lane row (every lane active).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t u = static_cast<uint64_t>(__double_as_longlong(v));
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(u)), CTRL,
                                               0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(u >> 32)),
                                               CTRL, 0xf, 0xf, false);
    return __longlong_as_double(static_cast<long long>(
        (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo)));
}

// Sum of v over each aligned group of G lanes (G a power of two <= 64), the
// same value in every lane of the group.  Each stage adds the value of a
// partner lane from the complementary half of the block (partners are
// mutual and a + b == b + a, so both hold the same sum): lane xor 1, xor 2
// (quad permutes), mirror within 8 and within 16 lanes (DPP), then xor 16
// and xor 32 (permute through LDS).
template <int G>
__device__ __forceinline__ double group_sum_f64(double v) {
    if constexpr (G >= 2) v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    if constexpr (G >= 4) v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    if constexpr (G >= 8) v += dpp_f64<0x141>(v);  // row_half_mirror
    if constexpr (G >= 16) v += dpp_f64<0x140>(v); // row_mirror
    if constexpr (G >= 32) v += shfl_xor_f64(v, 16);
    if constexpr (G >= 64) v += shfl_xor_f64(v, 32);
    return v;
}

// Orders the LDS operations of one wavefront across its lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
// FROM > 2: the keys already form sorted runs of FROM/2 elements, ascending
// in even runs and descending in odd ones, and the first stages are skipped.
template <int R, int FROM = 2>
__device__ __forceinline__ void wave_bitonic_sort(uint64_t (&v)[R]) {
    const int lane = lane_id();
#pragma unroll
    for (int size = FROM; size <= kWave * R; size <<= 1) {
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
