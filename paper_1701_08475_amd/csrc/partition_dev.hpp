// Device helpers shared by the level-synchronous partition kernels and the
// subtree kernel: the keyed starting pair, the order key of a double and a
// block-wide flag scan.
#pragma once
#include "knng_internal.hpp"
#include "wave.hpp"

namespace knng {
namespace pdev {

// Chunks of kChunkRows rows (one wavefront each) of a node of `size` rows.
__device__ __forceinline__ int chunks_of(int size) { return (size + kChunkRows - 1) / kChunkRows; }

// Chunk index taken by chunk slot cs (0 .. per_block-1) of workgroup b, or -1.
// order (nullable): chunk indices sorted by the smallest row id of the
// chunk, so that chunks that gather nearby rows run together.  xcd_per > 0:
// workgroup b (placed by the hardware on XCD b mod 8) takes the positions
// from XCD (b mod 8)'s contiguous share of xcd_per workgroups, so that
// those chunks also share one L2.
__device__ __forceinline__ int dispatch_chunk(const int32_t* order, int xcd_per, int b, int cs,
                                              int per_block, int nc) {
    const int bp = xcd_per > 0 ? (b & 7) * xcd_per + (b >> 3) : b;
    const int pos = bp * per_block + cs;
    if (pos >= nc) return -1;
    return order != nullptr ? order[pos] : pos;
}

// ------------------------------------------------------------- random pair
// Keyed starting pair.  SplitMix64 output function (Steele, Lea, Flood,
// OOPSLA 2014); each key word is absorbed as one SplitMix64 step taken from
// state (h xor word).  Key: (seed, tree, smallest member id, node size, j).
constexpr uint64_t kGolden = 0x9e3779b97f4a7c15ull;

__device__ __forceinline__ uint64_t splitmix_out(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t pair_hash(uint64_t seed, uint64_t tree, uint64_t min_id,
                                              uint64_t size, uint64_t j) {
    uint64_t h = seed;
    h = splitmix_out((h ^ tree) + kGolden);
    h = splitmix_out((h ^ min_id) + kGolden);
    h = splitmix_out((h ^ size) + kGolden);
    h = splitmix_out((h ^ j) + kGolden);
    return h;
}

// Unsigned key with the order of a double (after turning -0 into +0).
__device__ __forceinline__ uint64_t ordered_key(double v) {
    v = v + 0.0;
    const uint64_t u = static_cast<uint64_t>(__double_as_longlong(v));
    return (u >> 63) ? ~u : (u | (1ull << 63));
}

// Block-wide exclusive scan of one flag per thread (NW wavefronts).
template <int NW = 4>
__device__ __forceinline__ int block_excl_scan_flag(bool f, int* warp_tot, int* total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long b = __ballot(f);
    const int below = __popcll(b & ((1ull << lane) - 1ull));
    if (lane == 0) warp_tot[wv] = __popcll(b);
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < NW; ++i) {
        if (i < wv) off += warp_tot[i];
        tot += warp_tot[i];
    }
    __syncthreads();
    *total = tot;
    return off + below;
}

// Radix-selection step over a 256-bin histogram held in LDS (one bin per
// thread for the first 256 threads of an NW-wavefront block): finds the bin
// whose cumulative count first exceeds rem and writes (bin, rem within it)
// to *out_bin, *out_rem.  Every thread calls it; it ends with a barrier.
template <int NW = 4>
__device__ __forceinline__ void block_hist_pick(const unsigned int* hist, int rem, int* wtot,
                                                int* out_bin, int* out_rem) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int c = tid < 256 ? static_cast<int>(hist[tid]) : 0;
    int x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63 && wv < 4) wtot[wv] = x;
    __syncthreads();
    int off = 0;
    for (int i = 0; i < 4; ++i)
        if (i < wv) off += wtot[i];
    const int incl = off + x, excl = incl - c;
    if (tid < 256 && excl <= rem && rem < incl) {
        *out_bin = tid;
        *out_rem = rem - excl;
    }
    __syncthreads();
}

}  // namespace pdev
}  // namespace knng
