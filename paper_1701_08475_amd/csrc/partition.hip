// Level-synchronous two-means bisection of all trees at once (Sec. 3.1: the
// reference set is split in two by two-means clustering, again and again,
// until no cluster holds more points than the threshold; Alg. 1, clustering
// step and collection of the cluster set S).
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
#include "partition_dev.hpp"
#include "wave.hpp"

#include <type_traits>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace knng {
namespace {
using namespace pdev;

// ------------------------------------------------------------- level setup
// Root nodes (or root leaves when n <= leaf_max) of every tree slot; roots
// of at most small_max rows go straight to the subtree list (depth 0).
__global__ void k_roots(int T, int64_t n, int leaf_max, int small_max, NodeRec* nodes,
                        int32_t* big, NodeRec* sub, LeafRec* leaves, LevelCounters* ctr) {
    const int nch = static_cast<int>((n + kChunkRows - 1) / kChunkRows);
    const bool split = n > leaf_max;
    const bool small = split && n <= small_max;
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        if (small) {
            sub[t] = NodeRec{t, 0, static_cast<int32_t>(n), 0};
        } else if (split) {
            nodes[t] = NodeRec{t, 0, static_cast<int32_t>(n), t * nch};
            big[t] = t;
        } else {
            leaves[t] = LeafRec{t, 0, static_cast<int32_t>(n), 0};
        }
    }
    if (threadIdx.x == 0) {
        const bool level = split && !small;
        ctr->n_next = level ? T : 0;
        ctr->nc_next = level ? T * nch : 0;
        ctr->n_big = (level && nch > 1) ? T : 0;
        ctr->n_leaves = split ? 0 : T;
        ctr->n_log = 0;
        ctr->n_sub = small ? T : 0;
    }
}

__global__ void k_iota(int32_t* perm, int64_t n, int T) {
    const int64_t total = n * T;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < total;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        perm[i] = static_cast<int32_t>(i % n);
}

__global__ void k_fill_u8(uint8_t* p, int64_t count) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = 0;
}

__global__ void k_zero_small(unsigned long long* stats, int words, int* flag) {
    for (int i = threadIdx.x; i < words; i += blockDim.x) stats[i] = 0ull;
    if (threadIdx.x == 0) *flag = 0;
}

// Dispatch order of a level's chunks: a counting sort by first row id >> shift
// (at most 4096 bins; order within a bin arbitrary).  One block.
__global__ __launch_bounds__(1024) void k_chunk_order(const int32_t* __restrict__ key, int nc,
                                                      int shift, int32_t* __restrict__ order) {
    constexpr int kBins = 4096;
    __shared__ int s_bin[kBins];
    __shared__ int s_part[1024];
    const int tid = threadIdx.x;
    for (int i = tid; i < kBins; i += 1024) s_bin[i] = 0;
    __syncthreads();
    for (int j = tid; j < nc; j += 1024) atomicAdd(&s_bin[key[j] >> shift], 1);
    __syncthreads();
    const int a0 = s_bin[4 * tid], a1 = s_bin[4 * tid + 1], a2 = s_bin[4 * tid + 2],
              a3 = s_bin[4 * tid + 3];
    const int own = a0 + a1 + a2 + a3;
    s_part[tid] = own;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive Hillis-Steele scan
        const int v = tid >= o ? s_part[tid - o] : 0;
        __syncthreads();
        s_part[tid] += v;
        __syncthreads();
    }
    const int b = s_part[tid] - own;
    s_bin[4 * tid] = b;
    s_bin[4 * tid + 1] = b + a0;
    s_bin[4 * tid + 2] = b + a0 + a1;
    s_bin[4 * tid + 3] = b + a0 + a1 + a2;
    __syncthreads();
    for (int j = tid; j < nc; j += 1024) order[atomicAdd(&s_bin[key[j] >> shift], 1)] = j;
}

// Starting centres c0 = x[S[a]], c1 = x[S[b]] of every node; one wave each.
// C holds per node c0[D] then c1[D] (FP64).  Also empties the level's
// repair list.
__global__ __launch_bounds__(64) void k_init_nodes(const NodeRec* __restrict__ nodes,
                                                   const int32_t* __restrict__ perm,
                                                   const float* __restrict__ X, int64_t n, int D,
                                                   uint64_t seed, int tree0,
                                                   double* __restrict__ C,
                                                   int32_t* __restrict__ status,
                                                   int32_t* __restrict__ chunk_node,
                                                   int32_t* __restrict__ chunk_key,
                                                   int32_t* __restrict__ rep) {
    const int node = blockIdx.x;
    const NodeRec r = nodes[node];
    const size_t base = static_cast<size_t>(r.tree) * n + r.start;
    const uint64_t m = static_cast<uint64_t>(r.size);
    const uint64_t min_id = static_cast<uint64_t>(static_cast<uint32_t>(perm[base]));
    const uint64_t tg = static_cast<uint64_t>(tree0 + r.tree);
    const uint64_t a = pair_hash(seed, tg, min_id, m, 0) % m;
    uint64_t b = pair_hash(seed, tg, min_id, m, 1) % (m - 1);
    if (b >= a) ++b;
    const float* x0 = X + static_cast<size_t>(perm[base + a]) * D;
    const float* x1 = X + static_cast<size_t>(perm[base + b]) * D;
    double* c = C + static_cast<size_t>(node) * 2 * D;
    for (int d = threadIdx.x; d < D; d += kWave) {
        c[d] = static_cast<double>(x0[d]);
        c[D + d] = static_cast<double>(x1[d]);
    }
    if (threadIdx.x == 0) status[node] = 0;
    // the level's chunk -> node map and, when the chunks are dispatched in
    // order of their first row id, that id (chunk_key, nullable)
    if (blockIdx.x == 0 && threadIdx.x == 0) rep[0] = 0;
    const int nch = chunks_of(r.size);
    for (int ch = threadIdx.x; ch < nch; ch += blockDim.x) {
        chunk_node[r.chunk0 + ch] = node;
        if (chunk_key != nullptr)
            chunk_key[r.chunk0 + ch] = perm[base + static_cast<size_t>(ch) * kChunkRows];
    }
}

// ------------------------------------------------------------- Lloyd pass
// FP32 rows as given (the uint8 copy has its own pass, k_assign_u8).
template <typename TX, int VEC>
struct RowVec;
template <>
struct RowVec<float, 1> {  // one float per load (rows not 16-byte aligned)
    static constexpr int kVec = 1;
    using Acc = double;
    __device__ static void load(const float* row, int e, int D, bool ok, float (&x)[1]) {
        x[0] = (ok && e < D) ? row[e] : 0.f;
    }
};
template <>
struct RowVec<float, 4> {  // 4 floats per 16-byte load
    static constexpr int kVec = 4;
    using Acc = double;
    __device__ static void load(const float* row, int e, int D, bool ok, float (&x)[4]) {
        float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
        if (ok && e < D) q = *reinterpret_cast<const float4*>(row + e);
        x[0] = q.x;
        x[1] = q.y;
        x[2] = q.z;
        x[3] = q.w;
    }
};


// One assignment pass over every chunk of every unfinished node.
// G lanes share one row; each lane holds NF vectors of VEC consecutive
// elements (element e = (lane_in_group + G*j)*VEC + v).  Each lane group
// takes U rows per step (row = row0 + (step*U + u)*RPW + group).  Loads are
// software-pipelined: the rows of step s+1 are in flight while step s is
// computed, and the row ids of step s+2 are fetched meanwhile.
//
// w and h are derived by every wave from the node's centres with the same
// lane layout, so all waves of a node use bit-identical values.  A node of
// one chunk moves its centres at the end of the pass from the wave's own
// sums; larger nodes publish per-chunk sums for k_update_big.  A node stops
// when no label changed, a side is empty, or the pass budget is spent; its
// centres are then the ones that produced its final labels.
template <typename TX, int VEC, int G, int NF, int U>
__global__ __launch_bounds__(256) void k_assign(
    const TX* __restrict__ X, int64_t n, int D, const int32_t* __restrict__ perm,
    const NodeRec* __restrict__ nodes, const int32_t* __restrict__ chunk_node, int nc,
    double* __restrict__ C, int32_t* __restrict__ status, int32_t* __restrict__ n0f,
    uint8_t* __restrict__ labels, double* __restrict__ dots, double* __restrict__ P,
    int32_t* __restrict__ cnt, int pass, int max_iter, unsigned long long* __restrict__ assigned,
    int32_t* __restrict__ rep, int min_leaf, const int32_t* __restrict__ order, int xcd_per) {
    using RV = RowVec<TX, VEC>;
    using Acc = typename RV::Acc;
    constexpr int RPW = kWave / G;  // rows per wave step
    const int wave = dispatch_chunk(order, xcd_per, blockIdx.x, threadIdx.x >> 6, 4, nc);
    if (wave < 0) return;
    const int node = chunk_node[wave];
    if (status[node]) return;
    const NodeRec r = nodes[node];
    const int lane = threadIdx.x & 63;
    const int g = lane / G, l = lane % G;
    const int nch = chunks_of(r.size);
    const int row0 = (wave - r.chunk0) * kChunkRows;
    const int row1 = min(r.size, row0 + kChunkRows);
    const size_t base = static_cast<size_t>(r.tree) * n + r.start;

    double* cn = C + static_cast<size_t>(node) * 2 * D;
    double w[NF][VEC];
    Acc a0[NF][VEC], a1[NF][VEC];
    double q0 = 0.0, q1 = 0.0;
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const int e = (l + G * j) * VEC + v;
            const double c0 = e < D ? cn[e] : 0.0;
            const double c1 = e < D ? cn[D + e] : 0.0;
            w[j][v] = c0 - c1;
            q0 = fma(c0, c0, q0);
            q1 = fma(c1, c1, q1);
            a0[j][v] = Acc(0);
            a1[j][v] = Acc(0);
        }
    q0 = group_sum_f64<G>(q0);
    q1 = group_sum_f64<G>(q1);
    const double h = 0.5 * (q0 - q1);
    int n1 = 0, changed = 0;

    const int steps = (row1 - row0 + RPW * U - 1) / (RPW * U);
    auto row_id = [&](int st, int u) -> int {
        const int row = row0 + (st * U + u) * RPW + g;
        return row < row1 ? perm[base + row] : -1;
    };
    auto load_rows = [&](const int (&id)[U], float (&x)[U][NF][VEC]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const TX* xr = X + static_cast<size_t>(id[u] < 0 ? 0 : id[u]) * D;
#pragma unroll
            for (int j = 0; j < NF; ++j) RV::load(xr, (l + G * j) * VEC, D, id[u] >= 0, x[u][j]);
        }
    };
    // the previous pass's label of a row, fetched a step ahead with its row
    // (a load consumed in its own step would wait for every load before it)
    auto old_label = [&](int st, int u, int id) -> int {
        const int row = row0 + (st * U + u) * RPW + g;
        return (pass > 0 && id >= 0 && l == 0) ? static_cast<int>(labels[base + row]) : 0;
    };
    int idc[U], idn[U], oc[U];
    float xc[U][NF][VEC];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        idc[u] = row_id(0, u);
        idn[u] = row_id(1, u);
    }
    load_rows(idc, xc);
#pragma unroll
    for (int u = 0; u < U; ++u) oc[u] = old_label(0, u, idc[u]);
    for (int st = 0; st < steps; ++st) {
        float xn[U][NF][VEC];
        int on[U];
        load_rows(idn, xn);  // rows of step st+1 (ids -1 past the end)
#pragma unroll
        for (int u = 0; u < U; ++u) on[u] = old_label(st + 1, u, idn[u]);
        int idnn[U];
#pragma unroll
        for (int u = 0; u < U; ++u) idnn[u] = row_id(st + 2, u);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int row = row0 + (st * U + u) * RPW + g;
            double dot = 0.0;
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int v = 0; v < VEC; ++v)
                    dot = fma(static_cast<double>(xc[u][j][v]), w[j][v], dot);
            dot = group_sum_f64<G>(dot);  // (the FP32-row kernels' order)
            const bool lab = dot < h;
            if (idc[u] >= 0) {
                if (l == 0) {
                    const size_t p = base + row;
                    labels[p] = lab ? 1 : 0;
                    dots[p] = dot;
                    changed += (pass > 0 && oc[u] != (lab ? 1 : 0)) ? 1 : 0;
                    n1 += lab ? 1 : 0;
                }
#pragma unroll
                for (int j = 0; j < NF; ++j)
#pragma unroll
                    for (int v = 0; v < VEC; ++v) {
                        const Acc xv = static_cast<Acc>(xc[u][j][v]);
                        a0[j][v] += lab ? Acc(0) : xv;
                        a1[j][v] += lab ? xv : Acc(0);
                    }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            idc[u] = idn[u];
            idn[u] = idnn[u];
            oc[u] = on[u];
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int v = 0; v < VEC; ++v) xc[u][j][v] = xn[u][j][v];
        }
    }
    // combine the RPW row groups of the wave (fixed butterfly order)
#pragma unroll
    for (int o = G; o < kWave; o <<= 1)
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                if constexpr (sizeof(Acc) == 8) {
                    a0[j][v] += shfl_xor_f64(a0[j][v], o);
                    a1[j][v] += shfl_xor_f64(a1[j][v], o);
                } else {
                    a0[j][v] += __shfl_xor(a0[j][v], o, kWave);
                    a1[j][v] += __shfl_xor(a1[j][v], o, kWave);
                }
            }
    n1 = wave_sum_i32(n1);
    changed = wave_sum_i32(changed);
    if (lane == 0) {
        cnt[2 * wave] = n1;  // ones of this chunk (also read by the scatter)
        cnt[2 * wave + 1] = changed;
        stat_add(assigned, static_cast<unsigned>(wave), static_cast<unsigned long long>(row1 - row0));
    }

    if (nch == 1) {  // the wave holds the whole node
        const int n0 = r.size - n1;
        const bool stop =
            n1 == 0 || n0 == 0 || (pass >= 1 && changed == 0) || pass + 1 >= max_iter;
        if (stop) {
            if (lane == 0) {
                status[node] = 1;
                n0f[node] = n0;
                if (n0 < min_leaf || n1 < min_leaf) rep[1 + atomicAdd(rep, 1)] = node;
            }
            return;
        }
        if (g == 0) {
            const double dn0 = static_cast<double>(n0), dn1 = static_cast<double>(n1);
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const int e = (l + G * j) * VEC + v;
                    if (e < D) {
                        cn[e] = static_cast<double>(a0[j][v]) / dn0;
                        cn[D + e] = static_cast<double>(a1[j][v]) / dn1;
                    }
                }
        }
        return;
    }
    if (g == 0) {  // publish this chunk's sums
        double* p0 = P + static_cast<size_t>(wave) * 2 * D;
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                const int e = (l + G * j) * VEC + v;
                if (e < D) {
                    p0[e] = static_cast<double>(a0[j][v]);
                    p0[D + e] = static_cast<double>(a1[j][v]);
                }
            }
    }
}

// One assignment pass over uint8 rows (the lossless copy of integer data in
// [0, 255], D % 16 == 0), with the labels and stop rule of k_assign.  G lanes
// share a row, each holding NF vectors of EPL (8 or 16) elements; U rows per
// lane group and step.  The side sums are exact integers, so only the side-1
// sum is accumulated in every pass (a multiply-add by the 0/1 label); the
// chunk's total is taken in the level's first pass (FIRST) and kept in
// P[wave][0][.], and the side-0 sum is total - side 1, the same integer as a
// direct sum.  P[wave][1][.] holds the chunk's side-1 sum of the pass.
//
// Memory pipeline: the chunk's row ids and previous labels go to LDS first
// (all loads in flight at once); the rows of steps st+1 .. st+PD are in
// flight while step st is computed, in PD+1 register buffers rotated by
// unrolling (a register copy of a buffer still being loaded would wait for
// the load).  Row loads are unconditional (row 0 stands in past the end), so
// the loop's only global loads are rows, counted in issue order.
template <int EPL, int G, int NF, int U, int PD, bool FIRST>
__global__ __launch_bounds__(256) void k_assign_u8(
    const uint8_t* __restrict__ X, int64_t n, int D, const int32_t* __restrict__ perm,
    const NodeRec* __restrict__ nodes, const int32_t* __restrict__ chunk_node, int nc,
    double* __restrict__ C, int32_t* __restrict__ status, int32_t* __restrict__ n0f,
    uint8_t* __restrict__ labels, double* __restrict__ dots, double* __restrict__ P,
    int32_t* __restrict__ cnt, int pass, int max_iter, unsigned long long* __restrict__ assigned,
    int32_t* __restrict__ rep, int min_leaf, const int32_t* __restrict__ order, int xcd_per) {
    using V = typename std::conditional<EPL == 16, uint4, uint2>::type;
    constexpr int kWords = EPL / 4;
    constexpr int RPW = kWave / G;  // rows per wave step
    constexpr int kFill = kChunkRows / kWave;
    __shared__ int32_t s_ids[4][kChunkRows];
    __shared__ uint8_t s_old[4][kChunkRows];

    const int wave = dispatch_chunk(order, xcd_per, blockIdx.x, threadIdx.x >> 6, 4, nc);
    if (wave < 0) return;
    const int node = chunk_node[wave];
    if (status[node]) return;
    const NodeRec r = nodes[node];
    const int lane = threadIdx.x & 63, wl = threadIdx.x >> 6;
    const int g = lane / G, l = lane % G;
    const int nch = chunks_of(r.size);
    const int row0 = (wave - r.chunk0) * kChunkRows;
    const int nrows = min(r.size - row0, kChunkRows);
    const size_t base = static_cast<size_t>(r.tree) * n + r.start + row0;

    {  // row ids and previous labels of the chunk into LDS
        int32_t pid[kFill];
        uint8_t pl[kFill];
#pragma unroll
        for (int q = 0; q < kFill; ++q) {
            const int i = min(q * kWave + lane, nrows - 1);
            pid[q] = perm[base + i];
            pl[q] = FIRST ? 0 : labels[base + i];
        }
#pragma unroll
        for (int q = 0; q < kFill; ++q) {
            const int i = q * kWave + lane;
            if (i < nrows) {
                s_ids[wl][i] = pid[q];
                s_old[wl][i] = pl[q];
            }
        }
    }

    double* cn = C + static_cast<size_t>(node) * 2 * D;
    double* p0 = P + static_cast<size_t>(wave) * 2 * D;
    double w[NF][EPL];
    uint32_t a1[NF][EPL], tot[NF][EPL];
    bool ev[NF];  // vector j of this lane lies inside the row (else its
                  // loads read the row's start: finite values with w = 0,
                  // and its sums are never stored)
    double q0 = 0.0, q1 = 0.0;
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        ev[j] = (l + G * j) * EPL < D;
#pragma unroll
        for (int v = 0; v < EPL; ++v) {
            const int e = (l + G * j) * EPL + v;
            const double c0 = e < D ? cn[e] : 0.0;
            const double c1 = e < D ? cn[D + e] : 0.0;
            w[j][v] = c0 - c1;
            q0 = fma(c0, c0, q0);
            q1 = fma(c1, c1, q1);
            // later passes start from the previous pass's side-1 sum (row
            // group 0 only; the groups are added at the end)
            a1[j][v] = (!FIRST && g == 0 && e < D) ? static_cast<uint32_t>(p0[D + e]) : 0u;
            tot[j][v] = 0u;
        }
    }
    q0 = group_sum_f64<G>(q0);
    q1 = group_sum_f64<G>(q1);
    const double h = 0.5 * (q0 - q1);
    int n1 = 0, changed = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const int steps = (nrows + RPW * U - 1) / (RPW * U);
    auto load_rows = [&](int st, V (&x)[U][NF]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = (st * U + u) * RPW + g;
            const int id = i < nrows ? s_ids[wl][i] : 0;
            const uint8_t* xr = X + static_cast<size_t>(id) * D;
#pragma unroll
            for (int j = 0; j < NF; ++j)
                x[u][j] = *reinterpret_cast<const V*>(xr + (ev[j] ? (l + G * j) * EPL : 0));
        }
    };
    auto compute = [&](int st, const V (&x)[U][NF]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = (st * U + u) * RPW + g;
            const bool valid = i < nrows;
            const int old = (!FIRST && valid) ? static_cast<int>(s_old[wl][i]) : 0;
            uint32_t xv[NF][EPL];
#pragma unroll
            for (int j = 0; j < NF; ++j) {
                uint32_t wd[kWords];
                __builtin_memcpy(wd, &x[u][j], sizeof(V));
#pragma unroll
                for (int k4 = 0; k4 < kWords; ++k4)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        xv[j][4 * k4 + b] = (wd[k4] >> (8 * b)) & 255u;
            }
            double dot = 0.0;
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int v = 0; v < EPL; ++v) dot = fma(static_cast<double>(xv[j][v]), w[j][v], dot);
            dot = group_sum_f64<G>(dot);
            const bool lab = dot < h;
            if (valid && l == 0) {
                labels[base + i] = lab ? 1 : 0;
                changed += (!FIRST && old != (lab ? 1 : 0)) ? 1 : 0;
                n1 += lab ? 1 : 0;
            }
            if constexpr (FIRST) {
                const uint32_t one = (valid && lab) ? 1u : 0u;
                const uint32_t in = valid ? 1u : 0u;
#pragma unroll
                for (int j = 0; j < NF; ++j)
#pragma unroll
                    for (int v = 0; v < EPL; ++v) {
                        a1[j][v] = __umul24(xv[j][v], one) + a1[j][v];
                        tot[j][v] = __umul24(xv[j][v], in) + tot[j][v];
                    }
            } else {
                // only rows that switched sides move the side-1 sum
                const int df = valid ? (lab ? 1 : 0) - old : 0;
                if (df != 0) {
#pragma unroll
                    for (int j = 0; j < NF; ++j)
#pragma unroll
                        for (int v = 0; v < EPL; ++v)
                            a1[j][v] = static_cast<uint32_t>(
                                __mul24(df, static_cast<int>(xv[j][v])) + static_cast<int>(a1[j][v]));
                }
            }
        }
    };
    V xb[PD + 1][U][NF];
#pragma unroll
    for (int q = 0; q < PD; ++q) load_rows(q, xb[q]);
    for (int st0 = 0; st0 < steps; st0 += PD + 1) {
#pragma unroll
        for (int ph = 0; ph <= PD; ++ph) {
            const int st = st0 + ph;
            load_rows(st + PD, xb[(ph + PD) % (PD + 1)]);  // no branch: waits stay exact
            if (st < steps) compute(st, xb[ph]);
        }
    }
    // combine the RPW row groups of the wave (exact integer sums)
#pragma unroll
    for (int o = G; o < kWave; o <<= 1)
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int v = 0; v < EPL; ++v) {
                a1[j][v] += __shfl_xor(a1[j][v], o, kWave);
                if constexpr (FIRST) tot[j][v] += __shfl_xor(tot[j][v], o, kWave);
            }
    n1 = wave_sum_i32(n1);
    changed = wave_sum_i32(changed);
    if (lane == 0) {
        cnt[2 * wave] = n1;  // ones of this chunk (also read by the scatter)
        cnt[2 * wave + 1] = changed;
        stat_add(assigned, static_cast<unsigned>(wave), static_cast<unsigned long long>(nrows));
    }

    if (nch == 1) {  // the wave holds the whole node
        const int n0 = r.size - n1;
        const bool stop =
            n1 == 0 || n0 == 0 || (pass >= 1 && changed == 0) || pass + 1 >= max_iter;
        if (stop) {
            if (lane == 0) {
                status[node] = 1;
                n0f[node] = n0;
                if (n0 < min_leaf || n1 < min_leaf) rep[1 + atomicAdd(rep, 1)] = node;
            }
            return;
        }
        if (g == 0) {
            const double dn0 = static_cast<double>(n0), dn1 = static_cast<double>(n1);
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int v = 0; v < EPL; ++v) {
                    const int e = (l + G * j) * EPL + v;
                    if (e < D) {
                        double t;
                        if constexpr (FIRST) {
                            t = static_cast<double>(tot[j][v]);
                            p0[e] = t;
                        } else {
                            t = p0[e];
                        }
                        const double s1 = static_cast<double>(a1[j][v]);
                        p0[D + e] = s1;
                        cn[e] = (t - s1) / dn0;
                        cn[D + e] = s1 / dn1;
                    }
                }
        }
        return;
    }
    if (g == 0) {  // publish this chunk's sums
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int v = 0; v < EPL; ++v) {
                const int e = (l + G * j) * EPL + v;
                if (e < D) {
                    if constexpr (FIRST) p0[e] = static_cast<double>(tot[j][v]);
                    p0[D + e] = static_cast<double>(a1[j][v]);
                }
            }
    }
}

// Centre update of the nodes spanning several chunks.  One block per (node,
// slice of 8 dimensions): 16 values (8 dims x 2 sides) x 16 chunk lanes; lane
// c sums chunks c, c+16, ... in order, then the 16 lane sums are added in
// lane order.  Every block of a node derives the same stop decision.
// totals: side 0 of P holds chunk totals (uint8 rows), so the side-0 sum is
// total - side 1.
constexpr int kUpdDims = 8;
constexpr int kUpdLanes = 16;

__global__ __launch_bounds__(256) void k_update_big(const NodeRec* __restrict__ nodes,
                                                    const int32_t* __restrict__ big, int D,
                                                    const double* __restrict__ P,
                                                    const int32_t* __restrict__ cnt,
                                                    double* __restrict__ C,
                                                    int32_t* __restrict__ status,
                                                    int32_t* __restrict__ n0f, int pass,
                                                    int max_iter, int totals,
                                                    int32_t* __restrict__ rep, int min_leaf) {
    const int slices = (D + kUpdDims - 1) / kUpdDims;
    const int node = big[blockIdx.x / slices];
    const int slice = blockIdx.x % slices;
    if (status[node]) return;
    const NodeRec r = nodes[node];
    const int nch = chunks_of(r.size);
    __shared__ int s_cnt[2][256];
    __shared__ double s_sum[kUpdLanes][2 * kUpdDims];
    const int tid = threadIdx.x;
    int a = 0, b = 0;
    for (int c = tid; c < nch; c += 256) {
        a += cnt[2 * (r.chunk0 + c)];
        b += cnt[2 * (r.chunk0 + c) + 1];
    }
    s_cnt[0][tid] = a;
    s_cnt[1][tid] = b;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (tid < s) {
            s_cnt[0][tid] += s_cnt[0][tid + s];
            s_cnt[1][tid] += s_cnt[1][tid + s];
        }
        __syncthreads();
    }
    const int n1 = s_cnt[0][0], changed = s_cnt[1][0];
    const int n0 = r.size - n1;
    const bool stop = n1 == 0 || n0 == 0 || (pass >= 1 && changed == 0) || pass + 1 >= max_iter;
    if (stop) {
        if (slice == 0 && tid == 0) {
            status[node] = 1;
            n0f[node] = n0;
            if (n0 < min_leaf || n1 < min_leaf) rep[1 + atomicAdd(rep, 1)] = node;
        }
        return;
    }
    // value v: side = v / kUpdDims, dim = slice*kUpdDims + v % kUpdDims
    const int v = tid % (2 * kUpdDims), cl = tid / (2 * kUpdDims);
    const int side = v / kUpdDims, d = slice * kUpdDims + v % kUpdDims;
    double sum = 0.0;
    if (d < D) {
        const size_t sD = static_cast<size_t>(D);
        const size_t step = static_cast<size_t>(kUpdLanes) * 2 * sD;
        const double* q = P + (static_cast<size_t>(r.chunk0) + cl) * 2 * sD + side * sD + d;
        int c = cl;
        for (; c + 3 * kUpdLanes < nch; c += 4 * kUpdLanes) {  // loads in flight, adds in order
            const double x0 = q[0];
            const double x1 = q[step];
            const double x2 = q[2 * step];
            const double x3 = q[3 * step];
            sum += x0;
            sum += x1;
            sum += x2;
            sum += x3;
            q += 4 * step;
        }
        for (; c < nch; c += kUpdLanes) {
            sum += q[0];
            q += step;
        }
    }
    s_sum[cl][v] = sum;
    __syncthreads();
    if (tid < 2 * kUpdDims && d < D) {
        double t = 0.0;
        for (int k = 0; k < kUpdLanes; ++k) t += s_sum[k][tid];
        if (totals && side == 0) {  // P holds totals and side-1 sums (exact integers)
            double t1 = 0.0;
            for (int k = 0; k < kUpdLanes; ++k) t1 += s_sum[k][tid + kUpdDims];
            t -= t1;
        }
        const double cnt_side = side ? static_cast<double>(n1) : static_cast<double>(n0);
        C[static_cast<size_t>(node) * 2 * D + side * static_cast<size_t>(D) + d] = t / cnt_side;
    }
}

// Centre update of multi-chunk nodes when they span few chunks: one block per
// node for all 2D values (thread v sums the chunks in order), so a level of
// many two- or three-chunk nodes launches one block per node, not per slice.
__global__ __launch_bounds__(256) void k_update_nodes(const NodeRec* __restrict__ nodes,
                                                      const int32_t* __restrict__ big, int D,
                                                      const double* __restrict__ P,
                                                      const int32_t* __restrict__ cnt,
                                                      double* __restrict__ C,
                                                      int32_t* __restrict__ status,
                                                      int32_t* __restrict__ n0f, int pass,
                                                      int max_iter, int totals,
                                                      int32_t* __restrict__ rep, int min_leaf) {
    const int node = big[blockIdx.x];
    if (status[node]) return;
    const NodeRec r = nodes[node];
    const int nch = chunks_of(r.size);
    __shared__ int s_n[2];
    const int tid = threadIdx.x;
    if (tid == 0) {
        int a = 0, b = 0;
        for (int c = 0; c < nch; ++c) {
            a += cnt[2 * (r.chunk0 + c)];
            b += cnt[2 * (r.chunk0 + c) + 1];
        }
        s_n[0] = a;
        s_n[1] = b;
    }
    __syncthreads();
    const int n1 = s_n[0], changed = s_n[1];
    const int n0 = r.size - n1;
    const bool stop = n1 == 0 || n0 == 0 || (pass >= 1 && changed == 0) || pass + 1 >= max_iter;
    if (stop) {
        if (tid == 0) {
            status[node] = 1;
            n0f[node] = n0;
            if (n0 < min_leaf || n1 < min_leaf) rep[1 + atomicAdd(rep, 1)] = node;
        }
        return;
    }
    const size_t sD = static_cast<size_t>(D);
    const double* q = P + static_cast<size_t>(r.chunk0) * 2 * sD;
    double* cn = C + static_cast<size_t>(node) * 2 * sD;
    for (int d = tid; d < D; d += 256) {
        double t0 = 0.0, t1 = 0.0;
        for (int c = 0; c < nch; ++c) {
            t0 += q[c * 2 * sD + d];
            t1 += q[c * 2 * sD + sD + d];
        }
        if (totals) t0 -= t1;  // P holds totals and side-1 sums (exact integers)
        cn[d] = t0 / static_cast<double>(n0);
        cn[sD + d] = t1 / static_cast<double>(n1);
    }
}

// ------------------------------------------------------------- repair
// Margin-rank repair of nodes with a side smaller than min_leaf: order the
// members by (mu, id), mu = |x-c0|^2 - |x-c1|^2 = 2 (h - dot), i.e. by
// descending dot, and put the first s on the left, s = clamp(n0, min_leaf,
// m - min_leaf), or floor(m/2) when every margin is equal.  Rank s is found
// exactly by radix selection on the 64-bit key of -dot; equal keys go by
// position (= id order).  Per-chunk ones counts are rewritten.
// Nodes whose last pass left a side below min_leaf are listed in rep
// (rep[0] = count) by the pass that stopped them; blocks walk the list.
// U8G > 0: uint8 rows, whose assignment pass keeps no margins; the block
// first recomputes the final pass's FP64 margins of the node into dots, with
// the lane layout (U8G lanes per row, U8NF vectors of 16 elements per lane)
// and summation order of k_assign_u8, so they are the same numbers.
template <int U8G, int U8NF>
__global__ __launch_bounds__(256) void k_repair(const NodeRec* __restrict__ nodes,
                                                const int32_t* __restrict__ rep,
                                                int64_t n, const uint8_t* __restrict__ X8, int D,
                                                const int32_t* __restrict__ perm,
                                                const double* __restrict__ C,
                                                double* __restrict__ dots,
                                                uint8_t* __restrict__ labels,
                                                int32_t* __restrict__ n0f, int min_leaf,
                                                int32_t* __restrict__ cnt,
                                                unsigned long long* __restrict__ repairs) {
    __shared__ unsigned int hist[256];
    __shared__ unsigned long long s_min[256], s_max[256];
    __shared__ int s_bin, s_rem;
    __shared__ int warp_tot[4];
    const int tid = threadIdx.x;
    const int nrep = rep[0];
    for (int ri = blockIdx.x; ri < nrep; ri += gridDim.x) {
    const int node = rep[1 + ri];
    const NodeRec r = nodes[node];
    const int m = r.size;
    const int n0 = n0f[node];
    if (n0 >= min_leaf && m - n0 >= min_leaf) continue;
    const size_t base = static_cast<size_t>(r.tree) * n + r.start;
    if constexpr (U8G > 0) {
        constexpr int G = U8G, NF = U8NF, RPW = kWave / G;
        const int lane = tid & 63, wv = tid >> 6, g = lane / G, l = lane % G;
        const double* cn = C + static_cast<size_t>(node) * 2 * D;
        double w[NF][16];
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int e = (l + G * j) * 16 + v;
                w[j][v] = (e < D ? cn[e] : 0.0) - (e < D ? cn[D + e] : 0.0);
            }
        constexpr int U = 4;  // rows per lane group in flight
        for (int p0 = wv * RPW * U; p0 < m; p0 += 4 * RPW * U) {  // uniform per wave
            uint4 q[U][NF];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = p0 + u * RPW + g;
                const uint8_t* xr = X8 + static_cast<size_t>(p < m ? perm[base + p] : 0) * D;
#pragma unroll
                for (int j = 0; j < NF; ++j) {
                    const int e0 = (l + G * j) * 16;
                    q[u][j] = e0 < D ? *reinterpret_cast<const uint4*>(xr + e0) : make_uint4(0u, 0u, 0u, 0u);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int p = p0 + u * RPW + g;
                double dot = 0.0;
#pragma unroll
                for (int j = 0; j < NF; ++j) {
                    const uint32_t wd[4] = {q[u][j].x, q[u][j].y, q[u][j].z, q[u][j].w};
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
                        for (int b = 0; b < 4; ++b)
                            dot = fma(static_cast<double>((wd[k4] >> (8 * b)) & 255u), w[j][4 * k4 + b],
                                      dot);
                }
                dot = group_sum_f64<G>(dot);
                if (p < m && l == 0) dots[base + p] = dot;
            }
        }
        __syncthreads();
    }

    unsigned long long kmin = ~0ull, kmax = 0ull;
    for (int p = tid; p < m; p += 256) {
        const unsigned long long key = ordered_key(-dots[base + p]);
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
            const unsigned long long key = ordered_key(-dots[base + p]);
            if ((key & hi) == (prefix & hi)) atomicAdd(&hist[(key >> shift) & 255ull], 1u);
        }
        __syncthreads();
        block_hist_pick<4>(hist, rem, warp_tot, &s_bin, &s_rem);
        prefix |= static_cast<unsigned long long>(s_bin) << shift;
        rem = s_rem;
        __syncthreads();
    }
    // relabel: keys below the selected key go left, above go right, equal
    // keys go left while their running count (in position order) < rem.
    // kChunkRows is a multiple of 256, so each step lies in one chunk.
    int run = 0, ones = 0;
    for (int p0 = 0; p0 < m; p0 += 256) {
        const int p = p0 + tid;
        const bool valid = p < m;
        const unsigned long long key = valid ? ordered_key(-dots[base + p]) : 0ull;
        const bool eq = valid && key == prefix;
        int tot;
        const int rank = run + block_excl_scan_flag(eq, warp_tot, &tot);
        const bool right = valid && (key > prefix || (eq && rank >= rem));
        if (valid) labels[base + p] = right ? 1 : 0;
        run += tot;
        int tot1;
        block_excl_scan_flag(right, warp_tot, &tot1);
        ones += tot1;
        if (p0 + 256 >= m || ((p0 + 256) % kChunkRows) == 0) {
            if (tid == 0) cnt[2 * (r.chunk0 + p0 / kChunkRows)] = ones;
            ones = 0;
        }
    }
    if (tid == 0) {
        n0f[node] = s;
        stat_add(repairs, static_cast<unsigned>(blockIdx.x), 1ull);
    }
    __syncthreads();  // shared state is reused by the next node
    }
}

// ------------------------------------------------------------- split
// Stable partition of every node: label-0 members first, then label-1, each
// in their previous (ascending id) order.  Writes into perm_tmp.
__global__ __launch_bounds__(256) void k_scatter(int64_t n, const NodeRec* __restrict__ nodes,
                                                 const int32_t* __restrict__ chunk_node, int nc,
                                                 const uint8_t* __restrict__ labels,
                                                 const int32_t* __restrict__ cnt,
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
    for (int c = r.chunk0 + lane; c < wave; c += kWave) pre += cnt[2 * c];
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

// Children of every node of the level: runs of size > small_max become the
// next level's nodes (in parent order, left first), runs of leaf_max <
// size <= small_max go to the subtree list (chunk0 = their depth), the
// others are leaves; next nodes of several chunks are also listed in `big`.
// One block; the order is deterministic.
__global__ __launch_bounds__(1024) void k_next_level(
    const NodeRec* __restrict__ cur, int n_cur, const int32_t* __restrict__ n0f, int leaf_max,
    int small_max, int depth, NodeRec* __restrict__ next, int32_t* __restrict__ big,
    NodeRec* __restrict__ sub, LeafRec* __restrict__ leaves, int64_t leaves_cap,
    int32_t* __restrict__ node_log, int64_t node_log_cap, LevelCounters* __restrict__ ctr,
    int* __restrict__ overflow, LevelCounters* __restrict__ mirror, int seq) {
    // leaves and log entries are reserved with one atomic each: subtree
    // kernels on another stream append to the same lists meanwhile
    __shared__ int s_int[1024], s_leaf[1024], s_ch[1024], s_big[1024], s_sub[1024];
    __shared__ int s_base_leaf, s_base_log, s_base_sub;
    const int tid = threadIdx.x;
    const int per = (n_cur + 1023) / 1024;
    const int i0 = min(n_cur, tid * per), i1 = min(n_cur, i0 + per);
    int ci = 0, cl = 0, cc = 0, cb = 0, cs = 0;
    for (int i = i0; i < i1; ++i) {
        const NodeRec r = cur[i];
        const int sz[2] = {n0f[i], r.size - n0f[i]};
        for (int s = 0; s < 2; ++s) {
            if (sz[s] > small_max) {
                ++ci;
                const int ch = (sz[s] + kChunkRows - 1) / kChunkRows;
                cc += ch;
                cb += ch > 1 ? 1 : 0;
            } else if (sz[s] > leaf_max) {
                ++cs;
            } else {
                ++cl;
            }
        }
    }
    s_int[tid] = ci;
    s_leaf[tid] = cl;
    s_ch[tid] = cc;
    s_big[tid] = cb;
    s_sub[tid] = cs;
    if (tid == 0) s_base_sub = ctr->n_sub;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive Hillis-Steele scans
        int a = 0, b = 0, c = 0, e = 0, f = 0;
        if (tid >= o) {
            a = s_int[tid - o];
            b = s_leaf[tid - o];
            c = s_ch[tid - o];
            e = s_big[tid - o];
            f = s_sub[tid - o];
        }
        __syncthreads();
        s_int[tid] += a;
        s_leaf[tid] += b;
        s_ch[tid] += c;
        s_big[tid] += e;
        s_sub[tid] += f;
        __syncthreads();
    }
    if (tid == 1023) {
        s_base_leaf = atomicAdd(&ctr->n_leaves, s_leaf[1023]);
        s_base_log = atomicAdd(&ctr->n_log, n_cur);
    }
    __syncthreads();
    int oi = s_int[tid] - ci, ol = s_base_leaf + s_leaf[tid] - cl, oc = s_ch[tid] - cc,
        ob = s_big[tid] - cb, os = s_base_sub + s_sub[tid] - cs;
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
            if (sz[s] > small_max) {
                const int ch = (sz[s] + kChunkRows - 1) / kChunkRows;
                if (ch > 1) big[ob++] = oi;
                next[oi++] = NodeRec{r.tree, st[s], sz[s], oc};
                oc += ch;
            } else if (sz[s] > leaf_max) {
                sub[os++] = NodeRec{r.tree, st[s], sz[s], depth + 1};
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
        ctr->n_big = s_big[1023];
        ctr->n_sub = s_base_sub + s_sub[1023];
        if (mirror != nullptr) {
            // the next level's sizes into mapped host memory, then the level
            // number: the host polls it instead of copying and synchronising
            mirror->n_next = s_int[1023];
            mirror->nc_next = s_ch[1023];
            mirror->n_big = s_big[1023];
            mirror->n_sub = s_base_sub + s_sub[1023];
            __threadfence_system();
            *reinterpret_cast<volatile int32_t*>(&mirror->seq) = seq;
        }
    }
}

// ------------------------------------------------------------- dispatch

// Rows per lane group and step; more rows keep more loads in flight.
template <typename TX, int VEC, int G, int NF>
AssignFn<TX> pick_unroll(int u) {
    switch (u) {
        case 1: return k_assign<TX, VEC, G, NF, 1>;
        case 4: return k_assign<TX, VEC, G, NF, 4>;
        default: return k_assign<TX, VEC, G, NF, 2>;
    }
}

// Smallest lane group G (<= 32) with G*NF vectors covering a row of E vectors.
template <typename TX, int VEC, int NF>
AssignFn<TX> pick_groups(int E, int u) {
    int G = 1;
    while (G < 32 && G * NF < E) G <<= 1;
    switch (G) {
        case 1: return pick_unroll<TX, VEC, 1, NF>(u);
        case 2: return pick_unroll<TX, VEC, 2, NF>(u);
        case 4: return pick_unroll<TX, VEC, 4, NF>(u);
        case 8: return pick_unroll<TX, VEC, 8, NF>(u);
        case 16: return pick_unroll<TX, VEC, 16, NF>(u);
        default: return pick_unroll<TX, VEC, 32, NF>(u);
    }
}

// FP32 rows.  epl: elements per lane (4, 8 or 16) for rows that fit 32
// lanes; wider rows use all 64 lanes.
AssignFn<float> pick_assign_f32(int D, int epl, int u) {
    if (D % 4 == 0) {
        const int E = D / 4;
        if (E <= 32 * (epl / 4)) {
            if (epl == 4) return pick_groups<float, 4, 1>(E, u);
            if (epl == 8) return pick_groups<float, 4, 2>(E, u);
            return pick_groups<float, 4, 4>(E, u);
        }
        if (E <= 64 * 4) return pick_unroll<float, 4, 64, 4>(u);
        if (E <= 64 * 8) return k_assign<float, 4, 64, 8, 1>;
        if (E <= 64 * 16) return k_assign<float, 4, 64, 16, 1>;
        return nullptr;
    }
    if (D <= 32 * 4) return pick_groups<float, 1, 4>(D, 2);
    if (D <= 64 * 4) return k_assign<float, 1, 64, 4, 2>;
    if (D <= 64 * 8) return k_assign<float, 1, 64, 8, 1>;
    if (D <= 64 * 16) return k_assign<float, 1, 64, 16, 1>;
    return nullptr;
}

using RepairFn = void (*)(const NodeRec*, const int32_t*, int64_t, const uint8_t*, int, const int32_t*,
                         const double*, double*, uint8_t*, int32_t*, int, int32_t*,
                         unsigned long long*);

// uint8 rows (D % 16 == 0): 16 elements per lane; f[0] for a level's first
// pass, f[1] for the later ones; *rep recomputes their margins for repairs.
template <int G, int NF, int U>
void pick_u8_depth(int pd, AssignFn<uint8_t>* f, RepairFn* rep) {
    if (pd == 2) {
        f[0] = k_assign_u8<16, G, NF, U, 2, true>;
        f[1] = k_assign_u8<16, G, NF, U, 2, false>;
    } else {
        f[0] = k_assign_u8<16, G, NF, U, 1, true>;
        f[1] = k_assign_u8<16, G, NF, U, 1, false>;
    }
    *rep = k_repair<G, NF>;
}

template <int G, int NF>
void pick_u8_unroll(int u, int pd, AssignFn<uint8_t>* f, RepairFn* rep) {
    switch (u) {
        case 1: pick_u8_depth<G, NF, 1>(pd, f, rep); break;
        case 2: pick_u8_depth<G, NF, 2>(pd, f, rep); break;
        default: pick_u8_depth<G, NF, 4>(pd, f, rep); break;
    }
}

bool pick_assign_u8(int D, int u, int pd, AssignFn<uint8_t>* f, RepairFn* rep) {
    const int E = D / 16;
    int G = 1;
    while (G < 64 && G < E) G <<= 1;
    f[0] = f[1] = nullptr;
    switch (G) {
        case 1: pick_u8_unroll<1, 1>(u, pd, f, rep); break;
        case 2: pick_u8_unroll<2, 1>(u, pd, f, rep); break;
        case 4: pick_u8_unroll<4, 1>(u, pd, f, rep); break;
        case 8: pick_u8_unroll<8, 1>(u, pd, f, rep); break;
        case 16: pick_u8_unroll<16, 1>(u, pd, f, rep); break;
        case 32: pick_u8_unroll<32, 1>(u, pd, f, rep); break;
        default:
            if (E <= 64) pick_u8_unroll<64, 1>(u, pd, f, rep);
            else if (E <= 128) pick_u8_depth<64, 2, 1>(pd, f, rep);
            else if (E <= 256) pick_u8_depth<64, 4, 1>(pd, f, rep);
            break;
    }
    return f[0] != nullptr;
}

// Waits until the level kernel has written the counts of level `seq` into
// the mapped host mirror; fails if the stream reports an error or goes idle
// without them.
int wait_mirror(LevelCounters* m, int seq, hipStream_t s) {
    for (long spin = 1;; ++spin) {
        if (__atomic_load_n(&m->seq, __ATOMIC_ACQUIRE) == seq) return kOk;
        if ((spin & 4095) == 0) {
            const hipError_t q = hipStreamQuery(s);
            if (q == hipSuccess) {
                // the kernel has finished: its system-scope stores land shortly
                for (long t = 0; t < (1l << 22); ++t)
                    if (__atomic_load_n(&m->seq, __ATOMIC_ACQUIRE) == seq) return kOk;
                return kHip;
            }
            if (q != hipErrorNotReady) return kHip;
        }
    }
}

int env_int(const char* name, int dflt) {
    const char* e = std::getenv(name);
    return e ? std::atoi(e) : dflt;
}

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
    // Tuned on MI355X (1M x 128 rows): FP32 rows 8 elements per lane, one row
    // per lane group and step; uint8 rows 16 elements per lane, two rows per
    // step, one step of loads ahead.  The environment may override the
    // elements per lane (FP32), rows per step and load depth for tuning runs.
    const bool use_u8 = a.X8 != nullptr && D % 16 == 0;
    int epl = env_int("KNNG_ASSIGN_EPL", 8);
    // rows per lane group and step: 2 keeps more rows in flight (FP32 rows of
    // 960 dimensions: 11% faster than 1; 4 is slower, fewer waves fit)
    int unroll = knob(kKnobAssignUnroll, 2);
    if (epl != 4 && epl != 8 && epl != 16) epl = 8;
    if (unroll != 1 && unroll != 2 && unroll != 4) unroll = 2;
    // FP32 rows with D % 4 == 0: first pass with chunk totals, later passes
    // adding the changed rows (optionally filtered by the reduced copy);
    // other D: the single FP32 kernel with full side sums every pass
    AssignF32Fns f32{};
    const bool new_f32 = !use_u8 && pick_assign_f32_fns(D, unroll, &f32);
    AssignFn<float> assign = (use_u8 || new_f32) ? nullptr : pick_assign_f32(D, epl, unroll);
    // the filter: the reduced copy (KNNG_PARTITION_FILTER=0 turns it off; the
    // results are the same either way)
    AssignRfFn rf = nullptr;
    if (new_f32 && a.filter != nullptr && a.precision >= 1 && a.precision <= 3 &&
        knob(kKnobFilter, 1) != 0)
        rf = f32.rf[a.precision - 1];
    const bool totals = use_u8 || new_f32;  // P holds chunk totals and side-1 sums
    AssignFn<uint8_t> assign8[2] = {nullptr, nullptr};
    AssignFn<uint8_t> assign8w[2] = {nullptr, nullptr};  // four wavefronts per chunk
    RepairFn repair = k_repair<0, 1>;
    const int depth8 = env_int("KNNG_ASSIGN_U8_DEPTH", 1) == 2 ? 2 : 1;
    // levels with at most this many chunks take four wavefronts per chunk
    // (all levels by default: faster on MI355X whatever the chunk count)
    const int wide_max = env_int("KNNG_ASSIGN_WIDE_MAX", 1 << 30);
    if (use_u8) {
        pick_assign_u8(D, unroll, depth8, assign8, &repair);
        // margin on the matrix cores where D allows (KNNG_ASSIGN_MFMA=0: FP64 VALU kernel)
        if (env_int("KNNG_ASSIGN_MFMA", 1) != 0) {
            AssignFn<uint8_t> fm[2], fw[2];
            if (pick_assign_u8_mfma(D, knob(kKnobAssignMU, 1),
                                    knob(kKnobAssignMPD, 1), fm, fw)) {
                assign8[0] = fm[0];
                assign8[1] = fm[1];
                assign8w[0] = fw[0];
                assign8w[1] = fw[1];
            }
        }
    }
    if (assign == nullptr && assign8[0] == nullptr && !new_f32) {
        std::snprintf(err, errlen, "dimension %d not supported by the partition kernels", D);
        return kUnsupported;
    }
    // capacities: active nodes of a level are disjoint runs of > L points
    const int64_t nmax = std::max<int64_t>(1, static_cast<int64_t>(T) * (n / (L + 1) + 1));
    const int64_t cmax =
        static_cast<int64_t>(T) * ((n + kChunkRows - 1) / kChunkRows + n / (L + 1) + 1);
    const size_t tn = static_cast<size_t>(T) * n;
    const int slices = (D + kUpdDims - 1) / kUpdDims;

    // Nodes of at most small_max rows are split to leaves by a subtree kernel
    // that keeps their uint8 rows in LDS.  Default (KNNG_SUBTREE=3): one
    // wavefront per subtree of at most 144 rows.  KNNG_SUBTREE=1 or 2: one
    // eight-wave workgroup per subtree with rows in 128 or 64 KiB of LDS
    // (slower on MI355X: per-pass barriers over few rows); 0: level passes
    // down to the leaves.
    const int sub_mode = env_int("KNNG_SUBTREE", 3);
    const int row_budget = sub_mode == 2 ? 65536 : sub_mode == 3 ? 0 : 131072;
    const int small_max = (use_u8 && sub_mode != 0)
                              ? std::max(subtree_max_rows(D, row_budget), L)
                              : L;
    // KNNG_TRACE_LEVELS=1: one line per level on stderr (nodes, chunks)
    const bool trace_levels = env_int("KNNG_TRACE_LEVELS", 0) != 0;
    unsigned long long trace_f0 = 0, trace_e0 = 0;  // filter counters at the previous level's end
    NodeRec* sub = nullptr;
    NodeRec* nodes[2] = {nullptr, nullptr};
    int32_t* big[2] = {nullptr, nullptr};
    // dispatch order of the assignment chunks: bit 0 sorted by first row id
    // (default: 2-4% faster passes, chunks that gather nearby rows run
    // together), bit 1 XCD-aware workgroup placement (slower on MI355X)
    const int order_mode = knob(kKnobChunkOrder, 1);
    const int order_min = env_int("KNNG_CHUNK_ORDER_MIN", 4096);  // chunks per level
    int key_shift = 0;
    while (((n - 1) >> key_shift) >= 4096) ++key_shift;
    int32_t *chunk_key = nullptr, *corder = nullptr;
    int32_t *chunk_node = nullptr, *rep = nullptr, *status = nullptr, *n0f = nullptr, *cnt = nullptr,
            *perm_tmp = nullptr, *overflow = nullptr;
    double *C = nullptr, *P = nullptr, *dots = nullptr;
    uint8_t* labels = nullptr;
    LevelCounters* ctr = nullptr;
    unsigned long long* dstats = nullptr;
    LevelCounters* hctr = nullptr;
    LevelCounters* dmirror = nullptr;  // device address of hctr
    std::vector<unsigned long long> hstats(7 * kStatWords, 0ull);
    int hoverflow = 0;
    int cur = 0;
    int depth = 0;
    int64_t splits = 0;
    hipStream_t s2 = nullptr;      // subtree stream (overlap with the level loop)
    // levels of at most this many chunks run beside the subtree kernels
    const int overlap_nc = env_int("KNNG_SUBTREE_OVERLAP_NC", 4096);
    hipEvent_t s2_done = nullptr;
    bool s2_used = false;
    int sub_launched = 0;

    // KNNG_SUBTREE_OVERLAP=1: subtree kernels on a second stream beside the
    // smaller levels.  Off by default: on MI355X the build is no faster
    // (the level passes slow down by what the subtree kernels save).
    if (use_u8 && sub_mode != 0 && small_max > L && env_int("KNNG_SUBTREE_OVERLAP", 0) != 0) {
        // second stream (default priority) and event for the subtree
        // kernels, one per host thread and device for the life of the process
        thread_local hipStream_t t_s2[64] = {};
        thread_local hipEvent_t t_ev[64] = {};
        int dev = 0;
        KNNG_HIP(hipGetDevice(&dev));
        if (dev >= 0 && dev < 64) {
            if (t_s2[dev] == nullptr)
                KNNG_HIP(hipStreamCreateWithFlags(&t_s2[dev], hipStreamNonBlocking));
            if (t_ev[dev] == nullptr)
                KNNG_HIP(hipEventCreateWithFlags(&t_ev[dev], hipEventDisableTiming));
            s2 = t_s2[dev];
            s2_done = t_ev[dev];
        }
    }
    {
        // pinned counter mirror, one per host thread for the life of the
        // process (freeing pinned memory would synchronise the device)
        // (mapped, coherent: the level kernel writes the next level's sizes
        // into it directly)
        thread_local LevelCounters* t_hctr = nullptr;
        thread_local LevelCounters* t_dctr = nullptr;
        if (t_hctr == nullptr) {
            KNNG_HIP(hipHostMalloc(reinterpret_cast<void**>(&t_hctr), sizeof(LevelCounters),
                                   hipHostMallocMapped | hipHostMallocPortable |
                                       hipHostMallocCoherent));
            KNNG_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&t_dctr), t_hctr, 0));
        }
        hctr = t_hctr;
        dmirror = t_dctr;
    }
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&nodes[0]), sizeof(NodeRec) * nmax, s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&nodes[1]), sizeof(NodeRec) * nmax, s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&big[0]), sizeof(int32_t) * nmax, s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&big[1]), sizeof(int32_t) * nmax, s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&sub), sizeof(NodeRec) * nmax, s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&chunk_node), sizeof(int32_t) * cmax, s));
    if (order_mode & 1) {
        KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&chunk_key), sizeof(int32_t) * cmax, s));
        KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&corder), sizeof(int32_t) * cmax, s));
    }
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&rep), sizeof(int32_t) * (nmax + 1), s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&status), sizeof(int32_t) * nmax, s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&n0f), sizeof(int32_t) * nmax, s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&C), sizeof(double) * nmax * 2 * D, s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&P), sizeof(double) * cmax * 2 * D, s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&cnt), sizeof(int32_t) * cmax * 2, s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&labels), tn, s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&dots), sizeof(double) * tn, s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&perm_tmp), sizeof(int32_t) * tn, s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&ctr), sizeof(LevelCounters), s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&dstats),
                            sizeof(unsigned long long) * 7 * kStatWords, s));
    KNNG_HIP(ws_malloc(reinterpret_cast<void**>(&overflow), sizeof(int), s));
    k_zero_small<<<1, 256, 0, s>>>(dstats, 7 * kStatWords, overflow);
    KNNG_LAUNCH();
    {
        const int64_t want = (static_cast<int64_t>(tn) + 255) / 256;
        const int blocks = static_cast<int>(std::min<int64_t>(want, 65536));
        k_fill_u8<<<blocks, 256, 0, s>>>(labels, static_cast<int64_t>(tn));
        KNNG_LAUNCH();
        k_iota<<<blocks, 256, 0, s>>>(a.perm, n, T);
        KNNG_LAUNCH();
    }
    k_roots<<<1, 64, 0, s>>>(T, n, L, small_max, nodes[0], big[0], sub, a.leaves, ctr);
    KNNG_LAUNCH();
    {  // the roots' counts, as k_roots sets them
        const int nch0 = static_cast<int>((n + kChunkRows - 1) / kChunkRows);
        const bool rsplit = n > L, rsmall = rsplit && n <= small_max, rlevel = rsplit && !rsmall;
        hctr->n_next = rlevel ? T : 0;
        hctr->nc_next = rlevel ? T * nch0 : 0;
        hctr->n_big = (rlevel && nch0 > 1) ? T : 0;
        hctr->n_sub = rsmall ? T : 0;
        __atomic_store_n(&hctr->seq, -1, __ATOMIC_RELEASE);
    }

    while (hctr->n_next > 0) {
        if (depth > n) {  // every split shrinks both sides, so depth < n
            std::snprintf(err, errlen, "bisection did not terminate");
            rc = kHip;
            goto done;
        }
        const int na = hctr->n_next;
        const int nc = hctr->nc_next;
        const int nb = hctr->n_big;
        const int cblocks = (nc + 3) / 4;
        // chunks of the multi-chunk nodes: nc less one per single-chunk node
        const bool few_chunks = nb > 0 && (nc - (na - nb)) <= 8 * nb;
        // the order pays off on levels with many chunks only
        const bool sorted = (order_mode & 1) && nc >= order_min;
        // starting pairs, the chunk -> node map (and chunk keys), repair list reset
        k_init_nodes<<<na, 64, 0, s>>>(nodes[cur], a.perm, a.X, n, D, a.seed, a.tree0, C, status,
                                       chunk_node, sorted ? chunk_key : nullptr, rep);
        KNNG_LAUNCH();
        if (sorted) {
            k_chunk_order<<<1, 1024, 0, s>>>(chunk_key, nc, key_shift, corder);
            KNNG_LAUNCH();
        }
        const int32_t* ord = sorted ? corder : nullptr;
        // workgroups of the one-chunk-per-workgroup and four-chunk kernels
        const bool wide = use_u8 && assign8w[0] != nullptr && nc <= wide_max;
        const int nwg = wide ? nc : cblocks;
        const int xper = (order_mode & 2) ? (nwg + 7) / 8 : 0;
        const unsigned agrid = static_cast<unsigned>(xper > 0 ? 8 * xper : nwg);
        // the filtered pass with a workgroup per chunk (wide rows)
        const int nwg_rf = (new_f32 && f32.rf_wpc > 1) ? nc : cblocks;
        const int xper_rf = (order_mode & 2) ? (nwg_rf + 7) / 8 : 0;
        const unsigned agrid_rf = static_cast<unsigned>(xper_rf > 0 ? 8 * xper_rf : nwg_rf);
        for (int pass = 0; pass < a.max_iter; ++pass) {
            if (a.timer) a.timer->begin(kKAssign, s);
            if (wide)
                assign8w[pass == 0 ? 0 : 1]<<<agrid, 256, 0, s>>>(
                    a.X8, n, D, a.perm, nodes[cur], chunk_node, nc, C, status, n0f, labels, dots,
                    P, cnt, pass, a.max_iter, dstats, rep, a.min_leaf, ord, xper);
            else if (use_u8)
                assign8[pass == 0 ? 0 : 1]<<<agrid, 256, 0, s>>>(
                    a.X8, n, D, a.perm, nodes[cur], chunk_node, nc, C, status, n0f, labels, dots,
                    P, cnt, pass, a.max_iter, dstats, rep, a.min_leaf, ord, xper);
            else if (new_f32 && pass > 0 && rf != nullptr)
                rf<<<agrid_rf, 256, 0, s>>>(a.X, n, D, a.perm, nodes[cur], chunk_node, nc, C, status,
                                            n0f, labels, P, cnt, pass, a.max_iter, dstats, rep,
                                            a.min_leaf, ord, xper_rf, a.filter->Xr,
                                         reduced_rows_scale_offset(a.precision, a.filter->Dp),
                                         a.filter->stride, dstats + 5 * kStatWords);
            else if (new_f32)
                (pass == 0 ? f32.first : f32.later)<<<agrid, 256, 0, s>>>(
                    a.X, n, D, a.perm, nodes[cur], chunk_node, nc, C, status, n0f, labels, dots, P,
                    cnt, pass, a.max_iter, dstats, rep, a.min_leaf, ord, xper);
            else
                assign<<<agrid, 256, 0, s>>>(a.X, n, D, a.perm, nodes[cur], chunk_node, nc, C,
                                             status, n0f, labels, dots, P, cnt, pass, a.max_iter,
                                             dstats, rep, a.min_leaf, ord, xper);
            if (a.timer) a.timer->end(kKAssign, s);
            KNNG_LAUNCH();
            if (nb > 0) {
                if (few_chunks)
                    k_update_nodes<<<nb, 256, 0, s>>>(nodes[cur], big[cur], D, P, cnt, C, status,
                                                      n0f, pass, a.max_iter, totals ? 1 : 0, rep,
                                                      a.min_leaf);
                else
                    k_update_big<<<nb * slices, 256, 0, s>>>(nodes[cur], big[cur], D, P, cnt, C,
                                                             status, n0f, pass, a.max_iter,
                                                             totals ? 1 : 0, rep, a.min_leaf);
                KNNG_LAUNCH();
            }
        }
        if (new_f32) {  // the repair ranks by the final margins: recompute them
            f32.redots<<<1024, 256, 0, s>>>(nodes[cur], rep, n, a.X, D, a.perm, C, n0f,
                                            a.min_leaf, dots);
            KNNG_LAUNCH();
        }
        repair<<<std::min(na, 2048), 256, 0, s>>>(nodes[cur], rep, n, a.X8, D, a.perm, C, dots,
                                                  labels, n0f, a.min_leaf, cnt, dstats + kStatWords);
        KNNG_LAUNCH();
        k_scatter<<<cblocks, 256, 0, s>>>(n, nodes[cur], chunk_node, nc, labels, cnt, n0f, a.perm,
                                          perm_tmp);
        KNNG_LAUNCH();
        k_copyback<<<cblocks, 256, 0, s>>>(n, nodes[cur], chunk_node, nc, perm_tmp, a.perm);
        KNNG_LAUNCH();
        if (trace_levels) {
            // (the trace waits for the level: its filter counters are copied
            // back and the level's share printed)
            std::vector<unsigned long long> ts(7 * kStatWords, 0ull);
            unsigned long long f = 0, e = 0;
            if (hipMemcpyAsync(ts.data(), dstats, sizeof(unsigned long long) * ts.size(),
                               hipMemcpyDeviceToHost, s) == hipSuccess &&
                hipStreamSynchronize(s) == hipSuccess) {
                f = stat_total(ts.data() + 5 * kStatWords);
                e = stat_total(ts.data() + 6 * kStatWords);
            }
            std::fprintf(stderr,
                         "[knng] level %d: %d nodes, %d chunks, %d multi-chunk; filtered rows %llu, "
                         "in the band or changed %llu (%.2f%%)\n",
                         depth, na, nc, nb, f - trace_f0, e - trace_e0,
                         f > trace_f0 ? 100.0 * static_cast<double>(e - trace_e0) / static_cast<double>(f - trace_f0) : 0.0);
            trace_f0 = f;
            trace_e0 = e;
        }
        k_next_level<<<1, 1024, 0, s>>>(nodes[cur], na, n0f, L, small_max, depth, nodes[cur ^ 1],
                                        big[cur ^ 1], sub, a.leaves, a.leaves_cap, a.node_log,
                                        a.node_log_cap, ctr, overflow, dmirror, depth);
        KNNG_LAUNCH();
        if (wait_mirror(hctr, depth, s) != kOk) {
            std::snprintf(err, errlen, "level %d: counters not received", depth);
            rc = kHip;
            goto done;
        }
        splits += na;
        cur ^= 1;
        ++depth;
        if (s2 != nullptr && hctr->n_sub > sub_launched && hctr->nc_next <= overlap_nc) {
            // the subtree roots so far run on the second stream while the
            // level loop goes on (disjoint perm ranges; shared lists are
            // appended with atomics), once the levels are small enough that
            // their passes no longer fill the GPU
            SubtreeArgs sa{a.X8, n, D, sub + sub_launched, hctr->n_sub - sub_launched, a.perm, L,
                           a.min_leaf, a.max_iter, a.seed, a.tree0, a.leaves, a.leaves_cap,
                           a.node_log, a.node_log_cap, ctr, dstats, overflow, row_budget, s2};
            s2_used = true;
            if (subtree_launch(sa) != kOk) {
                std::snprintf(err, errlen, "subtree kernel launch failed");
                rc = kHip;
                goto done;
            }
            ++launches;
            sub_launched = hctr->n_sub;
        }
    }
    if (hctr->n_sub > sub_launched) {
        SubtreeArgs sa{a.X8, n, D, sub + sub_launched, hctr->n_sub - sub_launched, a.perm, L,
                       a.min_leaf, a.max_iter, a.seed, a.tree0, a.leaves, a.leaves_cap, a.node_log,
                       a.node_log_cap, ctr, dstats, overflow, row_budget, s};
        if (subtree_launch(sa) != kOk) {
            std::snprintf(err, errlen, "subtree kernel launch failed");
            rc = kHip;
            goto done;
        }
        ++launches;
        sub_launched = hctr->n_sub;
    }
    if (s2_used) {  // the build stream waits for the subtree stream
        KNNG_HIP(hipEventRecord(s2_done, s2));
        KNNG_HIP(hipStreamWaitEvent(s, s2_done, 0));
        s2_used = false;
    }
    KNNG_HIP(hipMemcpyAsync(hctr, ctr, sizeof(LevelCounters), hipMemcpyDeviceToHost, s));
    KNNG_HIP(hipMemcpyAsync(hstats.data(), dstats, sizeof(unsigned long long) * hstats.size(),
                            hipMemcpyDeviceToHost, s));
    KNNG_HIP(hipMemcpyAsync(&hoverflow, overflow, sizeof(int), hipMemcpyDeviceToHost, s));
    KNNG_HIP(hipStreamSynchronize(s));
    if (hoverflow) {
        if (hoverflow & 2)
            std::snprintf(err, errlen, "subtree stack overflow");
        else
            std::snprintf(err, errlen, "leaf list overflow (capacity %lld)",
                          static_cast<long long>(a.leaves_cap));
        rc = kHip;
        goto done;
    }
    res->n_leaves = hctr->n_leaves;
    res->n_log = hctr->n_log;
    res->subtree_rows = static_cast<int64_t>(stat_total(hstats.data() + 4 * kStatWords));
    res->filter_rows = static_cast<int64_t>(stat_total(hstats.data() + 5 * kStatWords));
    res->filter_exact_rows = static_cast<int64_t>(stat_total(hstats.data() + 6 * kStatWords));
    res->assign_rows = static_cast<int64_t>(stat_total(hstats.data())) + res->subtree_rows;
    res->repairs = static_cast<int64_t>(stat_total(hstats.data() + kStatWords));
    res->splits = splits + static_cast<int64_t>(stat_total(hstats.data() + 2 * kStatWords));
    res->levels =
        std::max<int64_t>(depth, static_cast<int64_t>(stat_peak(hstats.data() + 3 * kStatWords))) + 1;
    if (a.node_log != nullptr && hctr->n_sub > 0) {
        // subtree splits are logged in completion order: restore the
        // documented (depth, start) order
        const int64_t nl = std::min<int64_t>(hctr->n_log, a.node_log_cap);
        std::vector<int32_t> h(static_cast<size_t>(nl) * 4);
        KNNG_HIP(hipMemcpyAsync(h.data(), a.node_log, h.size() * sizeof(int32_t),
                                hipMemcpyDeviceToHost, s));
        KNNG_HIP(hipStreamSynchronize(s));
        std::vector<int64_t> idx(static_cast<size_t>(nl));
        for (int64_t i = 0; i < nl; ++i) idx[i] = i;
        std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
            const int32_t dx = h[4 * x + 3], dy = h[4 * y + 3];
            return dx != dy ? dx < dy : h[4 * x] < h[4 * y];
        });
        std::vector<int32_t> o(h.size());
        for (int64_t i = 0; i < nl; ++i)
            for (int f = 0; f < 4; ++f) o[4 * i + f] = h[4 * idx[i] + f];
        KNNG_HIP(hipMemcpyAsync(a.node_log, o.data(), o.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, s));
        KNNG_HIP(hipStreamSynchronize(s));
    }

done:
    if (s2_used) {  // error path: the frees below must follow the subtree kernels
        hipEventRecord(s2_done, s2);
        hipStreamWaitEvent(s, s2_done, 0);
    }
    if (nodes[0]) ws_free(nodes[0], s);
    if (nodes[1]) ws_free(nodes[1], s);
    if (big[0]) ws_free(big[0], s);
    if (big[1]) ws_free(big[1], s);
    if (sub) ws_free(sub, s);
    if (chunk_node) ws_free(chunk_node, s);
    if (chunk_key) ws_free(chunk_key, s);
    if (corder) ws_free(corder, s);
    if (rep) ws_free(rep, s);
    if (status) ws_free(status, s);
    if (n0f) ws_free(n0f, s);
    if (C) ws_free(C, s);
    if (P) ws_free(P, s);
    if (cnt) ws_free(cnt, s);
    if (labels) ws_free(labels, s);
    if (dots) ws_free(dots, s);
    if (perm_tmp) ws_free(perm_tmp, s);
    if (ctr) ws_free(ctr, s);
    if (dstats) ws_free(dstats, s);
    if (overflow) ws_free(overflow, s);
    if (rc != kOk) hipStreamSynchronize(s);  // copies into hctr may still be pending
    res->launches += launches;
    return rc;
}

}  // namespace knng
