// Level-synchronous two-means bisection of all trees at once (Sec. 3.1:
// "bisecting the reference set repeatedly with two means clustering" until no
// cluster exceeds the threshold; Alg. 1 "apply two means clustering",
// "collect clusters set S").
//
// Every node of a level, in every tree, advances one Lloyd pass per launch.
// A node is a contiguous run of perm[tree]; members keep ascending ids because
// each split is a stable partition.  One wavefront owns one chunk of up to
// kChunkRows rows of one node and, per row, computes in FP64
//     dot = x . w,   w = c0 - c1,   h = (|c0|^2 - |c1|^2) / 2,
// labelling the row 1 (right) iff dot < h, i.e. iff |x-c1|^2 < |x-c0|^2, so a
// point equidistant from both centres stays left.  The same pass accumulates
// per-side FP64 sums for the next centres.  All reductions run in a fixed
// order (lane butterflies, then chunks in index order), so results are
// bit-reproducible.
#include "knng_internal.hpp"
#include "wave.hpp"

#include <algorithm>
#include <cstdio>
#include <cstring>

namespace knng {
namespace {

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

// ------------------------------------------------------------- kernels
// Root nodes (or root leaves when n <= leaf_max) of every tree slot.
__global__ void k_roots(int T, int64_t n, int leaf_max, NodeRec* nodes, LeafRec* leaves,
                        LevelCounters* ctr) {
    const int nch = static_cast<int>((n + kChunkRows - 1) / kChunkRows);
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        if (n > leaf_max) {
            nodes[t] = NodeRec{t, 0, static_cast<int32_t>(n), t * nch};
        } else {
            leaves[t] = LeafRec{t, 0, static_cast<int32_t>(n), 0};
        }
    }
    if (threadIdx.x == 0) {
        const bool split = n > leaf_max;
        ctr->n_next = split ? T : 0;
        ctr->nc_next = split ? T * nch : 0;
        ctr->n_leaves = split ? 0 : T;
        ctr->n_log = 0;
    }
}

__global__ void k_iota(int32_t* perm, int64_t n, int T) {
    const int64_t total = n * T;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        perm[i] = static_cast<int32_t>(i % n);
}

// chunk -> node map of a level.
__global__ void k_chunk_map(const NodeRec* nodes, int32_t* chunk_node) {
    const NodeRec r = nodes[blockIdx.x];
    const int nch = (r.size + kChunkRows - 1) / kChunkRows;
    for (int c = threadIdx.x; c < nch; c += blockDim.x) chunk_node[r.chunk0 + c] = blockIdx.x;
}

// Starting centres c0 = x[S[a]], c1 = x[S[b]] of every node; one wave each.
__global__ __launch_bounds__(64) void k_init_nodes(const NodeRec* __restrict__ nodes,
                                                   const int32_t* __restrict__ perm,
                                                   const float* __restrict__ X, int64_t n, int D,
                                                   uint64_t seed, int tree0, double* __restrict__ W,
                                                   double* __restrict__ H,
                                                   int32_t* __restrict__ status) {
    const int node = blockIdx.x;
    const int lane = threadIdx.x;
    const NodeRec r = nodes[node];
    const size_t base = static_cast<size_t>(r.tree) * n + r.start;
    const uint64_t m = static_cast<uint64_t>(r.size);
    const uint64_t min_id = static_cast<uint64_t>(static_cast<uint32_t>(perm[base]));
    const uint64_t tg = static_cast<uint64_t>(tree0 + r.tree);
    const uint64_t u0 = pair_hash(seed, tg, min_id, m, 0);
    const uint64_t u1 = pair_hash(seed, tg, min_id, m, 1);
    const uint64_t a = u0 % m;
    uint64_t b = u1 % (m - 1);
    if (b >= a) ++b;
    const float* c0 = X + static_cast<size_t>(perm[base + a]) * D;
    const float* c1 = X + static_cast<size_t>(perm[base + b]) * D;
    double q0 = 0.0, q1 = 0.0;
    double* w = W + static_cast<size_t>(node) * D;
    for (int d = lane; d < D; d += kWave) {
        const double x0 = c0[d], x1 = c1[d];
        w[d] = x0 - x1;
        q0 = fma(x0, x0, q0);
        q1 = fma(x1, x1, q1);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        q0 += shfl_xor_f64(q0, o);
        q1 += shfl_xor_f64(q1, o);
    }
    if (lane == 0) {
        H[node] = 0.5 * (q0 - q1);
        status[node] = 0;
    }
}

// One Lloyd assignment pass over every chunk of every unfinished node.
// G lanes share one row; each lane holds NF groups of VEC consecutive
// elements (element e = (lane_in_group + G*j)*VEC + v).
template <int G, int NF, int VEC>
__global__ __launch_bounds__(256) void k_assign(
    const float* __restrict__ X, int64_t n, int D, const int32_t* __restrict__ perm,
    const NodeRec* __restrict__ nodes, const int32_t* __restrict__ chunk_node, int nc,
    const double* __restrict__ W, const double* __restrict__ H,
    const int32_t* __restrict__ status, uint8_t* __restrict__ labels,
    double* __restrict__ dots, double* __restrict__ P, int32_t* __restrict__ cnt, int pass) {
    constexpr int RPW = kWave / G;  // rows per wave step
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= nc) return;
    const int node = chunk_node[wave];
    if (status[node]) return;
    const NodeRec r = nodes[node];
    const int lane = threadIdx.x & 63;
    const int g = lane / G, l = lane % G;
    const int row0 = (wave - r.chunk0) * kChunkRows;
    const int row1 = min(r.size, row0 + kChunkRows);
    const size_t base = static_cast<size_t>(r.tree) * n + r.start;

    double w[NF][VEC];
    double a0[NF][VEC], a1[NF][VEC];
    const double* wn = W + static_cast<size_t>(node) * D;
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int e = (l + G * j) * VEC + v;
            w[j][v] = e < D ? wn[e] : 0.0;
            a0[j][v] = 0.0;
            a1[j][v] = 0.0;
        }
    const double h = H[node];
    int n1 = 0, changed = 0;

    const int iters = (row1 - row0 + RPW - 1) / RPW;
    for (int it = 0; it < iters; ++it) {
        const int row = row0 + it * RPW + g;
        const bool valid = row < row1;
        float x[NF][VEC];
        if (valid) {
            const float* xr = X + static_cast<size_t>(perm[base + row]) * D;
#pragma unroll
            for (int j = 0; j < NF; ++j) {
                const int e = (l + G * j) * VEC;
                if constexpr (VEC == 4) {
                    float4 q = e < D ? *reinterpret_cast<const float4*>(xr + e)
                                     : make_float4(0.f, 0.f, 0.f, 0.f);
                    x[j][0] = q.x;
                    x[j][VEC > 1 ? 1 : 0] = q.y;
                    x[j][VEC > 2 ? 2 : 0] = q.z;
                    x[j][VEC > 3 ? 3 : 0] = q.w;
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) x[j][v] = (e + v) < D ? xr[e + v] : 0.f;
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int v = 0; v < VEC; ++v) x[j][v] = 0.f;
        }
        double dot = 0.0;
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int v = 0; v < VEC; ++v) dot = fma(static_cast<double>(x[j][v]), w[j][v], dot);
#pragma unroll
        for (int o = G / 2; o >= 1; o >>= 1) dot += shfl_xor_f64(dot, o);
        const bool lab = dot < h;
        if (valid) {
            if (l == 0) {
                const size_t p = base + row;
                const uint8_t old = labels[p];
                labels[p] = lab ? 1 : 0;
                dots[p] = dot;
                changed += (pass > 0 && old != (lab ? 1 : 0)) ? 1 : 0;
                n1 += lab ? 1 : 0;
            }
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const double xv = static_cast<double>(x[j][v]);
                    a0[j][v] += lab ? 0.0 : xv;
                    a1[j][v] += lab ? xv : 0.0;
                }
        }
    }
    // combine the RPW row groups of the wave (fixed butterfly order)
#pragma unroll
    for (int o = G; o < kWave; o <<= 1)
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                a0[j][v] += shfl_xor_f64(a0[j][v], o);
                a1[j][v] += shfl_xor_f64(a1[j][v], o);
            }
    n1 = wave_sum_i32(n1);
    changed = wave_sum_i32(changed);
    if (g == 0) {
        double* p0 = P + static_cast<size_t>(wave) * 2 * D;
        double* p1 = p0 + D;
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                const int e = (l + G * j) * VEC + v;
                if (e < D) {
                    p0[e] = a0[j][v];
                    p1[e] = a1[j][v];
                }
            }
    }
    if (lane == 0) {
        cnt[2 * wave] = n1;
        cnt[2 * wave + 1] = changed;
    }
}

// After a pass: stop the node (nothing changed, a side empty, or the pass
// budget spent) or move its centres to the means of the two sides.
__global__ __launch_bounds__(256) void k_update(const NodeRec* __restrict__ nodes, int D,
                                                const double* __restrict__ P,
                                                const int32_t* __restrict__ cnt,
                                                double* __restrict__ W, double* __restrict__ H,
                                                int32_t* __restrict__ status,
                                                int32_t* __restrict__ n0f, int pass, int max_iter,
                                                unsigned long long* __restrict__ assigned) {
    const int node = blockIdx.x;
    if (status[node]) return;
    __shared__ int s_n1, s_changed;
    __shared__ double red[2][256];
    const NodeRec r = nodes[node];
    const int nch = (r.size + kChunkRows - 1) / kChunkRows;
    const int c0 = r.chunk0;
    if (threadIdx.x == 0) {
        int a = 0, b = 0;
        for (int c = 0; c < nch; ++c) {
            a += cnt[2 * (c0 + c)];
            b += cnt[2 * (c0 + c) + 1];
        }
        s_n1 = a;
        s_changed = b;
        atomicAdd(assigned, static_cast<unsigned long long>(r.size));
    }
    __syncthreads();
    const int n1 = s_n1, n0 = r.size - n1;
    const bool stop = n1 == 0 || n0 == 0 || (pass >= 1 && s_changed == 0) || pass + 1 >= max_iter;
    if (stop) {
        if (threadIdx.x == 0) {
            status[node] = 1;
            n0f[node] = n0;
        }
        return;
    }
    double q0 = 0.0, q1 = 0.0;
    double* w = W + static_cast<size_t>(node) * D;
    const double dn0 = static_cast<double>(n0), dn1 = static_cast<double>(n1);
    for (int d = threadIdx.x; d < D; d += 256) {
        double s0 = 0.0, s1 = 0.0;
        const double* p = P + static_cast<size_t>(c0) * 2 * D + d;
        for (int c = 0; c < nch; ++c) {
            s0 += p[0];
            s1 += p[D];
            p += 2 * static_cast<size_t>(D);
        }
        const double m0 = s0 / dn0, m1 = s1 / dn1;
        w[d] = m0 - m1;
        q0 = fma(m0, m0, q0);
        q1 = fma(m1, m1, q1);
    }
    red[0][threadIdx.x] = q0;
    red[1][threadIdx.x] = q1;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (threadIdx.x < s) {
            red[0][threadIdx.x] += red[0][threadIdx.x + s];
            red[1][threadIdx.x] += red[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) H[node] = 0.5 * (red[0][0] - red[1][0]);
}

// Block-wide exclusive scan of one flag per thread (256 threads).
__device__ __forceinline__ int block_excl_scan_flag(bool f, int* warp_tot, int* total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const unsigned long long b = __ballot(f);
    const int below = __popcll(b & ((1ull << lane) - 1ull));
    if (lane == 0) warp_tot[wv] = __popcll(b);
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < 4; ++i) {
        if (i < wv) off += warp_tot[i];
        tot += warp_tot[i];
    }
    __syncthreads();
    *total = tot;
    return off + below;
}

// Margin-rank repair of nodes with a side smaller than min_leaf: order the
// members by (mu, id), mu = |x-c0|^2 - |x-c1|^2 = 2 (h - dot), and put the
// first s on the left, s = clamp(n0, min_leaf, m - min_leaf), or floor(m/2)
// when every margin is equal.  Exact rank s is found by radix selection on
// the 64-bit key of (h - dot); equal keys go by position (= id order).
__global__ __launch_bounds__(256) void k_repair(const NodeRec* __restrict__ nodes, int64_t n,
                                                const double* __restrict__ H,
                                                const double* __restrict__ dots,
                                                uint8_t* __restrict__ labels,
                                                int32_t* __restrict__ n0f, int min_leaf,
                                                unsigned long long* __restrict__ repairs) {
    const int node = blockIdx.x;
    const NodeRec r = nodes[node];
    const int m = r.size;
    const int n0 = n0f[node];
    if (n0 >= min_leaf && m - n0 >= min_leaf) return;
    const size_t base = static_cast<size_t>(r.tree) * n + r.start;
    const double h = H[node];
    __shared__ unsigned int hist[256];
    __shared__ unsigned long long s_min[256], s_max[256];
    __shared__ unsigned long long s_prefix;
    __shared__ int s_rem;
    __shared__ int warp_tot[4];
    const int tid = threadIdx.x;

    unsigned long long kmin = ~0ull, kmax = 0ull;
    for (int p = tid; p < m; p += 256) {
        const unsigned long long key = ordered_key(h - dots[base + p]);
        kmin = key < kmin ? key : kmin;
        kmax = key > kmax ? key : kmax;
    }
    s_min[tid] = kmin;
    s_max[tid] = kmax;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (tid < s) {
            s_min[tid] = s_min[tid + s] < s_min[tid] ? s_min[tid + s] : s_min[tid];
            s_max[tid] = s_max[tid + s] > s_max[tid] ? s_max[tid + s] : s_max[tid];
        }
        __syncthreads();
    }
    const bool all_equal = s_min[0] == s_max[0];
    int s;
    if (all_equal) {
        s = m / 2;
    } else {
        s = n0 < min_leaf ? min_leaf : n0;
        s = s > m - min_leaf ? m - min_leaf : s;
    }

    // radix selection of the key of rank s (0-based)
    unsigned long long prefix = 0ull;
    int rem = s;
    for (int shift = 56; shift >= 0; shift -= 8) {
        hist[tid] = 0u;
        __syncthreads();
        const unsigned long long hi = shift == 56 ? 0ull : (~0ull << (shift + 8));
        for (int p = tid; p < m; p += 256) {
            const unsigned long long key = ordered_key(h - dots[base + p]);
            if ((key & hi) == (prefix & hi)) atomicAdd(&hist[(key >> shift) & 255ull], 1u);
        }
        __syncthreads();
        if (tid == 0) {
            int cum = 0;
            for (int dg = 0; dg < 256; ++dg) {
                const int c = static_cast<int>(hist[dg]);
                if (cum + c > rem) {
                    s_prefix = prefix | (static_cast<unsigned long long>(dg) << shift);
                    s_rem = rem - cum;
                    break;
                }
                cum += c;
            }
        }
        __syncthreads();
        prefix = s_prefix;
        rem = s_rem;
        __syncthreads();
    }
    // relabel: keys below the selected key go left, above go right, equal
    // keys go left while their running count (in position order) < rem
    int run = 0;
    for (int p0 = 0; p0 < m; p0 += 256) {
        const int p = p0 + tid;
        const bool valid = p < m;
        const unsigned long long key = valid ? ordered_key(h - dots[base + p]) : 0ull;
        const bool eq = valid && key == prefix;
        int tot;
        const int rank = run + block_excl_scan_flag(eq, warp_tot, &tot);
        if (valid) {
            const bool right = key > prefix || (eq && rank >= rem);
            labels[base + p] = right ? 1 : 0;
        }
        run += tot;
    }
    if (tid == 0) {
        n0f[node] = s;
        atomicAdd(repairs, 1ull);
    }
}

// Ones per chunk after the (possibly repaired) final labels.
__global__ __launch_bounds__(256) void k_count(int64_t n, const NodeRec* __restrict__ nodes,
                                               const int32_t* __restrict__ chunk_node, int nc,
                                               const uint8_t* __restrict__ labels,
                                               int32_t* __restrict__ cnt1) {
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= nc) return;
    const int lane = threadIdx.x & 63;
    const NodeRec r = nodes[chunk_node[wave]];
    const int row0 = (wave - r.chunk0) * kChunkRows;
    const int row1 = min(r.size, row0 + kChunkRows);
    const size_t base = static_cast<size_t>(r.tree) * n + r.start;
    int c = 0;
    for (int row = row0 + lane; row < row1; row += kWave) c += labels[base + row];
    c = wave_sum_i32(c);
    if (lane == 0) cnt1[wave] = c;
}

// Stable partition of every node: label-0 members first, then label-1, each
// in their previous (ascending id) order.  Writes into perm_tmp.
__global__ __launch_bounds__(256) void k_scatter(int64_t n, const NodeRec* __restrict__ nodes,
                                                 const int32_t* __restrict__ chunk_node, int nc,
                                                 const uint8_t* __restrict__ labels,
                                                 const int32_t* __restrict__ cnt1,
                                                 const int32_t* __restrict__ n0f,
                                                 const int32_t* __restrict__ perm,
                                                 int32_t* __restrict__ perm_tmp) {
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= nc) return;
    const int lane = threadIdx.x & 63;
    const int node = chunk_node[wave];
    const NodeRec r = nodes[node];
    const int row0 = (wave - r.chunk0) * kChunkRows;
    const int row1 = min(r.size, row0 + kChunkRows);
    const size_t base = static_cast<size_t>(r.tree) * n + r.start;
    int pre = 0;
    for (int c = r.chunk0 + lane; c < wave; c += kWave) pre += cnt1[c];
    pre = wave_sum_i32(pre);
    const int n0 = n0f[node];
    int run = 0;
    for (int it = row0; it < row1; it += kWave) {
        const int row = it + lane;
        const bool valid = row < row1;
        const bool one = valid && labels[base + row] != 0;
        const unsigned long long b = __ballot(one);
        const int ones_before = pre + run + __popcll(b & ((1ull << lane) - 1ull));
        if (valid) {
            const int np = one ? n0 + ones_before : row - ones_before;
            if (np >= 0 && np < r.size) perm_tmp[base + np] = perm[base + row];
        }
        run += __popcll(b);
    }
}

__global__ __launch_bounds__(256) void k_copyback(int64_t n, const NodeRec* __restrict__ nodes,
                                                  const int32_t* __restrict__ chunk_node, int nc,
                                                  const int32_t* __restrict__ perm_tmp,
                                                  int32_t* __restrict__ perm) {
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wave >= nc) return;
    const int lane = threadIdx.x & 63;
    const NodeRec r = nodes[chunk_node[wave]];
    const int row0 = (wave - r.chunk0) * kChunkRows;
    const int row1 = min(r.size, row0 + kChunkRows);
    const size_t base = static_cast<size_t>(r.tree) * n + r.start;
    for (int row = row0 + lane; row < row1; row += kWave) perm[base + row] = perm_tmp[base + row];
}

// Children of every node of the level: runs of size > leaf_max become the
// next level's nodes (in parent order, left first), the others become
// leaves.  One block; deterministic order.
__global__ __launch_bounds__(1024) void k_next_level(
    const NodeRec* __restrict__ cur, int n_cur, const int32_t* __restrict__ n0f, int leaf_max,
    int depth, NodeRec* __restrict__ next, LeafRec* __restrict__ leaves, int64_t leaves_cap,
    int32_t* __restrict__ node_log, int64_t node_log_cap, LevelCounters* __restrict__ ctr,
    int* __restrict__ overflow) {
    __shared__ int s_int[1024], s_leaf[1024], s_ch[1024];
    __shared__ int s_base_leaf, s_base_log;
    const int tid = threadIdx.x;
    const int per = (n_cur + 1023) / 1024;
    const int i0 = min(n_cur, tid * per), i1 = min(n_cur, i0 + per);
    int ci = 0, cl = 0, cc = 0;
    for (int i = i0; i < i1; ++i) {
        const NodeRec r = cur[i];
        const int sz[2] = {n0f[i], r.size - n0f[i]};
        for (int s = 0; s < 2; ++s) {
            if (sz[s] > leaf_max) {
                ++ci;
                cc += (sz[s] + kChunkRows - 1) / kChunkRows;
            } else {
                ++cl;
            }
        }
    }
    s_int[tid] = ci;
    s_leaf[tid] = cl;
    s_ch[tid] = cc;
    if (tid == 0) {
        s_base_leaf = ctr->n_leaves;
        s_base_log = ctr->n_log;
    }
    __syncthreads();
    // inclusive Hillis-Steele scans
    for (int o = 1; o < 1024; o <<= 1) {
        int a = 0, b = 0, c = 0;
        if (tid >= o) {
            a = s_int[tid - o];
            b = s_leaf[tid - o];
            c = s_ch[tid - o];
        }
        __syncthreads();
        s_int[tid] += a;
        s_leaf[tid] += b;
        s_ch[tid] += c;
        __syncthreads();
    }
    int oi = s_int[tid] - ci, ol = s_base_leaf + s_leaf[tid] - cl, oc = s_ch[tid] - cc;
    for (int i = i0; i < i1; ++i) {
        const NodeRec r = cur[i];
        const int n0 = n0f[i];
        if (node_log != nullptr) {
            const int64_t q = static_cast<int64_t>(s_base_log) + i;
            if (q < node_log_cap) {
                node_log[4 * q + 0] = r.start;
                node_log[4 * q + 1] = r.size;
                node_log[4 * q + 2] = n0;
                node_log[4 * q + 3] = depth;
            }
        }
        const int st[2] = {r.start, r.start + n0};
        const int sz[2] = {n0, r.size - n0};
        for (int s = 0; s < 2; ++s) {
            if (sz[s] > leaf_max) {
                next[oi++] = NodeRec{r.tree, st[s], sz[s], oc};
                oc += (sz[s] + kChunkRows - 1) / kChunkRows;
            } else {
                if (ol < leaves_cap)
                    leaves[ol] = LeafRec{r.tree, st[s], sz[s], 0};
                else
                    atomicOr(overflow, 1);
                ++ol;
            }
        }
    }
    __syncthreads();
    if (tid == 1023) {
        ctr->n_next = s_int[1023];
        ctr->nc_next = s_ch[1023];
        ctr->n_leaves = s_base_leaf + s_leaf[1023];
        ctr->n_log = s_base_log + n_cur;
    }
}

// ------------------------------------------------------------- dispatch
using AssignFn = void (*)(const float*, int64_t, int, const int32_t*, const NodeRec*,
                          const int32_t*, int, const double*, const double*, const int32_t*,
                          uint8_t*, double*, double*, int32_t*, int);

template <int VEC>
AssignFn pick_assign_vec(int D) {
    const int E = D / VEC;
    int G = 1;
    while (G < 64 && G * 4 < E) G <<= 1;
    if (G < 64) {
        switch (G) {
            case 1: return k_assign<1, 4, VEC>;
            case 2: return k_assign<2, 4, VEC>;
            case 4: return k_assign<4, 4, VEC>;
            case 8: return k_assign<8, 4, VEC>;
            case 16: return k_assign<16, 4, VEC>;
            default: return k_assign<32, 4, VEC>;
        }
    }
    if (E <= 64 * 4) return k_assign<64, 4, VEC>;
    if (E <= 64 * 8) return k_assign<64, 8, VEC>;
    if (E <= 64 * 16) return k_assign<64, 16, VEC>;
    return nullptr;
}

AssignFn pick_assign(int D) {
    return (D % 4 == 0) ? pick_assign_vec<4>(D) : pick_assign_vec<1>(D);
}

struct DevBuf {
    void* p = nullptr;
};

}  // namespace

#define KNNG_HIP(call)                                                                  \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            std::snprintf(err, errlen, "%s failed: %s", #call, hipGetErrorString(e_));  \
            rc = (e_ == hipErrorOutOfMemory) ? kOom : kHip;                             \
            goto done;                                                                  \
        }                                                                               \
    } while (0)

#define KNNG_LAUNCH()                                                                   \
    do {                                                                                \
        ++launches;                                                                     \
        hipError_t e_ = hipGetLastError();                                              \
        if (e_ != hipSuccess) {                                                         \
            std::snprintf(err, errlen, "kernel launch failed: %s", hipGetErrorString(e_)); \
            rc = kHip;                                                                  \
            goto done;                                                                  \
        }                                                                               \
    } while (0)

int partition_run(const PartitionArgs& a, PartitionResult* res, char* err, size_t errlen) {
    int rc = kOk;
    int launches = 0;
    const int64_t n = a.n;
    const int D = a.D;
    const int T = a.n_trees;
    const int L = a.leaf_max;
    hipStream_t s = a.stream;
    AssignFn assign = pick_assign(D);
    if (assign == nullptr) {
        std::snprintf(err, errlen, "dimension %d not supported by the partition kernels", D);
        return kUnsupported;
    }
    // capacities: active nodes of a level are disjoint runs of > L points
    const int64_t nmax = std::max<int64_t>(1, static_cast<int64_t>(T) * (n / (L + 1) + 1));
    const int64_t cmax = static_cast<int64_t>(T) * ((n + kChunkRows - 1) / kChunkRows + n / (L + 1) + 1);
    const size_t tn = static_cast<size_t>(T) * n;

    NodeRec* nodes[2] = {nullptr, nullptr};
    int32_t *chunk_node = nullptr, *status = nullptr, *n0f = nullptr, *cnt = nullptr,
            *cnt1 = nullptr, *perm_tmp = nullptr, *overflow = nullptr;
    double *W = nullptr, *H = nullptr, *P = nullptr, *dots = nullptr;
    uint8_t* labels = nullptr;
    LevelCounters* ctr = nullptr;
    unsigned long long* dstats = nullptr;
    LevelCounters* hctr = nullptr;
    unsigned long long hstats[2] = {0, 0};
    int hoverflow = 0;
    int cur = 0;
    int depth = 0;
    int64_t splits = 0;

    KNNG_HIP(hipHostMalloc(reinterpret_cast<void**>(&hctr), sizeof(LevelCounters), hipHostMallocDefault));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&nodes[0]), sizeof(NodeRec) * nmax, s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&nodes[1]), sizeof(NodeRec) * nmax, s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&chunk_node), sizeof(int32_t) * cmax, s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&status), sizeof(int32_t) * nmax, s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&n0f), sizeof(int32_t) * nmax, s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&W), sizeof(double) * nmax * D, s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&H), sizeof(double) * nmax, s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&P), sizeof(double) * cmax * 2 * D, s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&cnt), sizeof(int32_t) * cmax * 2, s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&cnt1), sizeof(int32_t) * cmax, s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&labels), tn, s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&dots), sizeof(double) * tn, s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&perm_tmp), sizeof(int32_t) * tn, s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&ctr), sizeof(LevelCounters), s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&dstats), sizeof(unsigned long long) * 2, s));
    KNNG_HIP(hipMallocAsync(reinterpret_cast<void**>(&overflow), sizeof(int), s));
    KNNG_HIP(hipMemsetAsync(dstats, 0, sizeof(unsigned long long) * 2, s));
    KNNG_HIP(hipMemsetAsync(overflow, 0, sizeof(int), s));
    KNNG_HIP(hipMemsetAsync(labels, 0, tn, s));

    {
        const int64_t want = (static_cast<int64_t>(tn) + 255) / 256;
        const int blocks = static_cast<int>(std::min<int64_t>(want, 65536));
        k_iota<<<blocks, 256, 0, s>>>(a.perm, n, T);
        KNNG_LAUNCH();
    }
    k_roots<<<1, 64, 0, s>>>(T, n, L, nodes[0], a.leaves, ctr);
    KNNG_LAUNCH();
    KNNG_HIP(hipMemcpyAsync(hctr, ctr, sizeof(LevelCounters), hipMemcpyDeviceToHost, s));
    KNNG_HIP(hipStreamSynchronize(s));

    while (hctr->n_next > 0) {
        if (depth > n) {  // every split shrinks both sides, so depth < n
            std::snprintf(err, errlen, "bisection did not terminate");
            rc = kHip;
            goto done;
        }
        const int na = hctr->n_next;
        const int nc = hctr->nc_next;
        const int cblocks = (nc + 3) / 4;
        k_chunk_map<<<na, 64, 0, s>>>(nodes[cur], chunk_node);
        KNNG_LAUNCH();
        k_init_nodes<<<na, 64, 0, s>>>(nodes[cur], a.perm, a.X, n, D, a.seed, a.tree0, W, H, status);
        KNNG_LAUNCH();
        for (int pass = 0; pass < a.max_iter; ++pass) {
            if (a.timer) a.timer->begin(kKAssign, s);
            assign<<<cblocks, 256, 0, s>>>(a.X, n, D, a.perm, nodes[cur], chunk_node, nc, W, H,
                                           status, labels, dots, P, cnt, pass);
            if (a.timer) a.timer->end(kKAssign, s);
            KNNG_LAUNCH();
            k_update<<<na, 256, 0, s>>>(nodes[cur], D, P, cnt, W, H, status, n0f, pass,
                                        a.max_iter, dstats);
            KNNG_LAUNCH();
        }
        k_repair<<<na, 256, 0, s>>>(nodes[cur], n, H, dots, labels, n0f, a.min_leaf, dstats + 1);
        KNNG_LAUNCH();
        k_count<<<cblocks, 256, 0, s>>>(n, nodes[cur], chunk_node, nc, labels, cnt1);
        KNNG_LAUNCH();
        k_scatter<<<cblocks, 256, 0, s>>>(n, nodes[cur], chunk_node, nc, labels, cnt1, n0f,
                                          a.perm, perm_tmp);
        KNNG_LAUNCH();
        k_copyback<<<cblocks, 256, 0, s>>>(n, nodes[cur], chunk_node, nc, perm_tmp, a.perm);
        KNNG_LAUNCH();
        k_next_level<<<1, 1024, 0, s>>>(nodes[cur], na, n0f, L, depth, nodes[cur ^ 1], a.leaves,
                                        a.leaves_cap, a.node_log, a.node_log_cap, ctr, overflow);
        KNNG_LAUNCH();
        KNNG_HIP(hipMemcpyAsync(hctr, ctr, sizeof(LevelCounters), hipMemcpyDeviceToHost, s));
        KNNG_HIP(hipStreamSynchronize(s));
        splits += na;
        cur ^= 1;
        ++depth;
    }
    KNNG_HIP(hipMemcpyAsync(hstats, dstats, sizeof(hstats), hipMemcpyDeviceToHost, s));
    KNNG_HIP(hipMemcpyAsync(&hoverflow, overflow, sizeof(int), hipMemcpyDeviceToHost, s));
    KNNG_HIP(hipStreamSynchronize(s));
    if (hoverflow) {
        std::snprintf(err, errlen, "leaf list overflow (capacity %lld)",
                      static_cast<long long>(a.leaves_cap));
        rc = kHip;
        goto done;
    }
    res->n_leaves = hctr->n_leaves;
    res->n_log = hctr->n_log;
    res->assign_rows = static_cast<int64_t>(hstats[0]);
    res->repairs = static_cast<int64_t>(hstats[1]);
    res->splits = splits;
    res->levels = depth + 1;

done:
    hipFreeAsync(nodes[0], s);
    hipFreeAsync(nodes[1], s);
    hipFreeAsync(chunk_node, s);
    hipFreeAsync(status, s);
    hipFreeAsync(n0f, s);
    hipFreeAsync(W, s);
    hipFreeAsync(H, s);
    hipFreeAsync(P, s);
    hipFreeAsync(cnt, s);
    hipFreeAsync(cnt1, s);
    hipFreeAsync(labels, s);
    hipFreeAsync(dots, s);
    hipFreeAsync(perm_tmp, s);
    hipFreeAsync(ctr, s);
    hipFreeAsync(dstats, s);
    hipFreeAsync(overflow, s);
    hipStreamSynchronize(s);
    if (hctr) hipHostFree(hctr);
    res->launches += launches;
    return rc;
}

}  // namespace knng
