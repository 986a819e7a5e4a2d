// Exhaustive comparison inside every cluster (Alg. 1: every pair of distinct
// members of a cluster updates both members' rows of G), FP32 direct form.
//
// One workgroup per leaf.  Rows are taken in panels of 32; for each panel the
// 32 x m distance block is accumulated from 16-dimension tiles staged in LDS,
// then every row's m-1 candidates are sorted by a wavefront bitonic network
// and its k best (d32, id) are written to the tree's candidate buffer.
//
// d32(i, j): per 32-dimension block b, blk_b = sequential fused sum of
// (x_i[d] - x_j[d])^2 over d in b; d32 = ((blk_0 + blk_1) + blk_2) + ...
// Negating a difference is exact, so d32(i, j) == d32(j, i) bitwise, and the
// same pair gets the same bits in every tree.
#include "knng_internal.hpp"
#include "wave.hpp"

#include <cstdio>

namespace knng {
namespace {

constexpr int kPanel = 32;  // rows per panel
constexpr int kDimTile = 16;

template <int MC>  // columns per thread; leaves up to 8*MC points
__global__ __launch_bounds__(256) void k_leaf_fp32(const float* __restrict__ X, int64_t n, int D,
                                                   int k, const int32_t* __restrict__ perm,
                                                   const LeafRec* __restrict__ leaves,
                                                   int32_t* __restrict__ cand_ids,
                                                   float* __restrict__ cand_d,
                                                   unsigned long long* __restrict__ pairs) {
    constexpr int MP = 8 * MC;
    constexpr int R = MP >= kWave ? MP / kWave : 1;  // sort slots per lane
    __shared__ float colT[kDimTile][MP + 1];
    __shared__ float rowT[kDimTile][kPanel];
    __shared__ float dist[kPanel][MP + 1];
    __shared__ int32_t ids[MP];

    const LeafRec lf = leaves[blockIdx.x];
    const int m = lf.size;
    const size_t base = static_cast<size_t>(lf.tree) * n + lf.start;
    const int tid = threadIdx.x;
    for (int j = tid; j < m; j += 256) ids[j] = perm[base + j];
    if (tid == 0 && pairs != nullptr)
        stat_add(pairs, blockIdx.x, static_cast<unsigned long long>(m) * static_cast<unsigned long long>(m - 1));
    __syncthreads();

    const int ri = tid & (kPanel - 1);
    const int cg = tid >> 5;  // 0..7
    const int wv = tid >> 6, lane = tid & 63;
    for (int r0 = 0; r0 < m; r0 += kPanel) {
        float blk[MC], tot[MC];
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            blk[c] = 0.f;
            tot[c] = 0.f;
        }
        for (int d0 = 0; d0 < D; d0 += kDimTile) {
            for (int idx = tid; idx < m * kDimTile; idx += 256) {
                const int j = idx / kDimTile, dd = idx % kDimTile;
                colT[dd][j] = (d0 + dd < D) ? X[static_cast<size_t>(ids[j]) * D + d0 + dd] : 0.f;
            }
            for (int idx = tid; idx < kPanel * kDimTile; idx += 256) {
                const int i = idx / kDimTile, dd = idx % kDimTile;
                rowT[dd][i] = (r0 + i < m && d0 + dd < D)
                                  ? X[static_cast<size_t>(ids[r0 + i]) * D + d0 + dd]
                                  : 0.f;
            }
            __syncthreads();
            const int dn = min(kDimTile, D - d0);
            for (int dd = 0; dd < dn; ++dd) {
                const float xi = rowT[dd][ri];
#pragma unroll
                for (int c = 0; c < MC; ++c) {
                    const float df = xi - colT[dd][cg + 8 * c];
                    blk[c] = __fmaf_rn(df, df, blk[c]);
                }
                const int d = d0 + dd;
                if ((d & 31) == 31 || d == D - 1) {
#pragma unroll
                    for (int c = 0; c < MC; ++c) {
                        tot[c] = tot[c] + blk[c];
                        blk[c] = 0.f;
                    }
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int c = 0; c < MC; ++c) dist[ri][cg + 8 * c] = tot[c];
        __syncthreads();
        const int rows = min(kPanel, m - r0);
        for (int rr = wv; rr < rows; rr += 4) {
            const int i = r0 + rr;
            uint64_t v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int j = lane * R + r;
                v[r] = (j < m && j != i) ? cand_key(dist[rr][j], ids[j]) : kNoKey;
            }
            wave_bitonic_sort<R>(v);
            const size_t out = (static_cast<size_t>(lf.tree) * n + ids[i]) * k;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int e = lane * R + r;
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

// Rows of k beyond the sort width (k > 8*MC) are padded.
__global__ void k_pad_tail(int64_t total_rows, int k, int from, int32_t* ids, float* d) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
         i < total_rows * (k - from); i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t row = i / (k - from);
        const int e = from + static_cast<int>(i % (k - from));
        ids[row * k + e] = -1;
        d[row * k + e] = __int_as_float(0x7f800000);
    }
}

}  // namespace

int leaf_run(const LeafArgs& a, int* launches, char* err, size_t errlen) {
    if (a.n_leaves == 0) return kOk;
    if (a.precision != 0) {
        std::snprintf(err, errlen, "leaf precision %d not available in this build", a.precision);
        return kUnsupported;
    }
    if (a.leaf_max > kMaxLeaf) {
        std::snprintf(err, errlen, "leaf of %d points exceeds %d", a.leaf_max, kMaxLeaf);
        return kUnsupported;
    }
    const int lm = a.leaf_max;
    // slots = sort width of the kernel: columns e >= slots are never written
    auto launch = [&](auto kern, int slots) -> int {
        if (a.timer) a.timer->begin(kKLeaf, a.stream);
        kern<<<static_cast<unsigned>(a.n_leaves), 256, 0, a.stream>>>(
            a.X, a.n, a.D, a.k, a.perm, a.leaves, a.cand_ids, a.cand_d, a.pairs);
        if (a.timer) a.timer->end(kKLeaf, a.stream);
        ++*launches;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            std::snprintf(err, errlen, "leaf launch failed: %s", hipGetErrorString(e));
            return kHip;
        }
        if (a.k > slots) {  // a leaf fills at most slots-1 candidates
            k_pad_tail<<<1024, 256, 0, a.stream>>>(static_cast<int64_t>(a.n_trees) * a.n, a.k,
                                                   slots, a.cand_ids, a.cand_d);
            ++*launches;
        }
        return kOk;
    };
    // Rows never touched by a leaf do not exist: the leaves of a tree cover
    // all n points, so every row of every tree's buffer is written.
    if (lm <= 16) return launch(k_leaf_fp32<2>, 64);
    if (lm <= 32) return launch(k_leaf_fp32<4>, 64);
    if (lm <= 64) return launch(k_leaf_fp32<8>, 64);
    if (lm <= 128) return launch(k_leaf_fp32<16>, 128);
    if (lm <= 256) return launch(k_leaf_fp32<32>, 256);
    return launch(k_leaf_fp32<64>, 512);
}

}  // namespace knng
