// Recursive two-means bisection (Alg. 2) of whole subtrees inside one
// workgroup, for uint8 rows (the lossless copy of integer data).
//
// Once a node holds at most S rows (S = 1024 for D <= 128), its rows fit in
// LDS, and every Lloyd pass, the margin-rank repair and the stable partition
// of it and of all its descendants run in one workgroup reading LDS: no HBM
// traffic after the first load and no per-level launches.  Each split takes
// exactly the steps of the level-synchronous kernels in partition.hip: the
// keyed starting pair (members in id order, key (seed, tree, smallest id,
// size, j)), passes with the same lane layout and FP64 dot order, labels
// dot < h, exact integer side sums, the stop rule (no label changed, an
// empty side or the pass budget), the repair by (mu, id) rank and the stable
// partition (label-0 members first, in id order).  Results are therefore the
// same as those of the level kernels, and the node runs of perm the same.
//
// Depth-first with an explicit stack; the smaller child is split next and
// the larger pushed, so the stack never holds more than log2(S) + 1 nodes.
#include "knng_internal.hpp"
#include "partition_dev.hpp"
#include "wave.hpp"

#include <cstdio>

namespace knng {
namespace {
using namespace pdev;

// Largest subtree (rows) per row width DM when its rows take at most RB
// bytes of LDS (128 KiB: one workgroup per CU; 64 KiB: two).
template <int DM, int RB>
constexpr int sub_rows() {
    return DM * 1024 <= RB ? 1024 : RB / DM;
}
constexpr int kStack = 32;

// NW wavefronts per workgroup; U rows per lane group and step (independent
// FMA chains in flight).
constexpr int kSubWaves = 8;
constexpr int kSubThreads = kSubWaves * kWave;
constexpr int kSubRows = 4;

template <int DM, int G, int RB>
__global__ __launch_bounds__(kSubThreads) void k_subtree_u8(
    const uint8_t* __restrict__ X8, int64_t n, int D, const NodeRec* __restrict__ roots,
    int32_t* __restrict__ perm, int leaf_max, int min_leaf, int max_iter, uint64_t seed,
    int tree0, LeafRec* __restrict__ leaves, int64_t leaves_cap, int32_t* __restrict__ node_log,
    int64_t node_log_cap, LevelCounters* __restrict__ ctr,
    unsigned long long* __restrict__ dstats, int* __restrict__ overflow) {
    constexpr int S = sub_rows<DM, RB>();
    constexpr int NW = kSubWaves, NT = kSubThreads, U = kSubRows;
    constexpr int RPW = kWave / G;  // rows per lane-group slot of a wave
    __shared__ __align__(16) uint8_t s_rows[S * DM];
    __shared__ int32_t s_ids[S];
    __shared__ uint16_t s_ord[S], s_tmp[S];
    __shared__ uint8_t s_lab[S];
    __shared__ double s_dot[S];
    __shared__ double s_cen[2 * DM];
    __shared__ uint32_t s_a1[2][DM];  // side-1 sums, by pass parity
    __shared__ uint32_t s_tot[DM];
    __shared__ uint32_t s_hist[256];
    __shared__ int s_cnt[2][2];        // (ones, changed), by pass parity
    __shared__ int s_stack[kStack][3];
    __shared__ int s_sp, s_node[3], s_pair[2], s_warp[NW], s_rem;
    __shared__ unsigned long long s_kmin[NW], s_kmax[NW], s_prefix;

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int g = lane / G, l = lane % G;
    const NodeRec root = roots[blockIdx.x];
    const int M = root.size;
    const size_t pbase = static_cast<size_t>(root.tree) * n + root.start;
    const uint64_t tg = static_cast<uint64_t>(tree0 + root.tree);
    const int vpr = D / 16;  // 16-byte vectors per row

    for (int i = tid; i < M; i += NT) {
        s_ids[i] = perm[pbase + i];
        s_ord[i] = static_cast<uint16_t>(i);
    }
    __syncthreads();
    for (int q = tid; q < M * vpr; q += NT) {
        const int r = q / vpr, c = q - r * vpr;
        reinterpret_cast<uint4*>(s_rows)[q] =
            reinterpret_cast<const uint4*>(X8 + static_cast<size_t>(s_ids[r]) * D)[c];
    }
    if (tid == 0) {
        s_stack[0][0] = 0;
        s_stack[0][1] = M;
        s_stack[0][2] = root.chunk0;  // depth of the subtree's root
        s_sp = 1;
    }
    unsigned long long assigned = 0, splits = 0, repairs = 0, maxdep = 0;
    __syncthreads();

    while (true) {
        if (tid == 0) {
            const int sp = s_sp;
            if (sp == 0) {
                s_node[1] = 0;
            } else {
                s_node[0] = s_stack[sp - 1][0];
                s_node[1] = s_stack[sp - 1][1];
                s_node[2] = s_stack[sp - 1][2];
                s_sp = sp - 1;
            }
        }
        __syncthreads();
        const int s = s_node[0], m = s_node[1], dep = s_node[2];
        if (m == 0) break;

        // ---- starting pair: members in id order are positions s .. s+m-1
        if (tid == 0) {
            const uint64_t mm = static_cast<uint64_t>(m);
            const uint64_t min_id = static_cast<uint64_t>(static_cast<uint32_t>(s_ids[s_ord[s]]));
            const uint64_t a = pair_hash(seed, tg, min_id, mm, 0) % mm;
            uint64_t b = pair_hash(seed, tg, min_id, mm, 1) % (mm - 1);
            if (b >= a) ++b;
            s_pair[0] = static_cast<int>(a);
            s_pair[1] = static_cast<int>(b);
        }
        for (int e = tid; e < DM; e += NT) {
            s_tot[e] = 0u;
            s_a1[0][e] = 0u;
            s_a1[1][e] = 0u;
        }
        if (tid < 4) s_cnt[tid >> 1][tid & 1] = 0;
        __syncthreads();
        {
            const int ra = s_ord[s + s_pair[0]], rb = s_ord[s + s_pair[1]];
            for (int e = tid; e < D; e += NT) {
                s_cen[e] = static_cast<double>(s_rows[ra * D + e]);
                s_cen[DM + e] = static_cast<double>(s_rows[rb * D + e]);
            }
        }
        __syncthreads();

        // ---- Lloyd passes
        int n1 = 0;
        for (int pass = 0; pass < max_iter; ++pass) {
            const int par = pass & 1;
            double w[16];
            double q0 = 0.0, q1 = 0.0;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int e = l * 16 + v;
                const double c0 = e < D ? s_cen[e] : 0.0;
                const double c1 = e < D ? s_cen[DM + e] : 0.0;
                w[v] = c0 - c1;
                q0 = fma(c0, c0, q0);
                q1 = fma(c1, c1, q1);
            }
            q0 = group_sum_f64<G>(q0);
            q1 = group_sum_f64<G>(q1);
            const double h = 0.5 * (q0 - q1);
            uint32_t a1[16], tot[16];
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                a1[v] = 0u;
                tot[v] = 0u;
            }
            int my1 = 0, mych = 0;
            for (int p0 = wv * U * RPW; p0 < m; p0 += NW * U * RPW) {  // uniform per wave
                uint32_t xv[U][16];
                bool valid[U];
                int pp[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    pp[u] = p0 + u * RPW + g;
                    valid[u] = pp[u] < m;
                    const int lr = valid[u] ? s_ord[s + pp[u]] : 0;
                    uint4 raw = make_uint4(0u, 0u, 0u, 0u);
                    if (l * 16 < D) raw = *reinterpret_cast<const uint4*>(s_rows + lr * D + l * 16);
                    const uint32_t wd[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
                        for (int b = 0; b < 4; ++b) xv[u][4 * k4 + b] = (wd[k4] >> (8 * b)) & 255u;
                }
                double dot[U];
#pragma unroll
                for (int u = 0; u < U; ++u) dot[u] = 0.0;
#pragma unroll
                for (int v = 0; v < 16; ++v)
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        dot[u] = fma(static_cast<double>(xv[u][v]), w[v], dot[u]);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double dt = group_sum_f64<G>(dot[u]);
                    const bool lab = dt < h;
                    if (valid[u] && l == 0) {
                        const int old = s_lab[s + pp[u]];
                        mych += (pass > 0 && old != (lab ? 1 : 0)) ? 1 : 0;
                        s_lab[s + pp[u]] = lab ? 1 : 0;
                        s_dot[s + pp[u]] = dt;
                        my1 += lab ? 1 : 0;
                    }
                    const uint32_t one = (valid[u] && lab) ? 1u : 0u;
                    const uint32_t in = valid[u] ? 1u : 0u;
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        a1[v] = __umul24(xv[u][v], one) + a1[v];
                        if (pass == 0) tot[v] = __umul24(xv[u][v], in) + tot[v];
                    }
                }
            }
#pragma unroll
            for (int o = G; o < kWave; o <<= 1)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    a1[v] += __shfl_xor(a1[v], o, kWave);
                    if (pass == 0) tot[v] += __shfl_xor(tot[v], o, kWave);
                }
            my1 = wave_sum_i32(my1);
            mych = wave_sum_i32(mych);
            if (g == 0) {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int e = l * 16 + v;
                    if (e < D) {
                        atomicAdd(&s_a1[par][e], a1[v]);
                        if (pass == 0) atomicAdd(&s_tot[e], tot[v]);
                    }
                }
            }
            if (lane == 0) {
                atomicAdd(&s_cnt[par][0], my1);
                atomicAdd(&s_cnt[par][1], mych);
            }
            assigned += static_cast<unsigned long long>(m);
            __syncthreads();
            n1 = s_cnt[par][0];
            const int ch = s_cnt[par][1];
            const int n0 = m - n1;
            const bool stop =
                n1 == 0 || n0 == 0 || (pass >= 1 && ch == 0) || pass + 1 >= max_iter;
            for (int e = tid; e < DM; e += NT) s_a1[par ^ 1][e] = 0u;  // next pass's sums
            if (tid < 2) s_cnt[par ^ 1][tid] = 0;
            if (!stop) {
                const double dn0 = static_cast<double>(n0), dn1 = static_cast<double>(n1);
                for (int e = tid; e < D; e += NT) {
                    const double t = static_cast<double>(s_tot[e]);
                    const double s1 = static_cast<double>(s_a1[par][e]);
                    s_cen[e] = (t - s1) / dn0;
                    s_cen[DM + e] = s1 / dn1;
                }
            }
            __syncthreads();
            if (stop) break;
        }
        int n0 = m - n1;

        // ---- margin-rank repair: first sel members by (mu, id) go left,
        // mu ascending = dot descending = key of -dot ascending
        if (n0 < min_leaf || n1 < min_leaf) {
            unsigned long long kmin = ~0ull, kmax = 0ull;
            for (int p = tid; p < m; p += NT) {
                const unsigned long long key = ordered_key(-s_dot[s + p]);
                kmin = key < kmin ? key : kmin;
                kmax = key > kmax ? key : kmax;
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const unsigned long long a = shfl_xor_u64(kmin, o), b = shfl_xor_u64(kmax, o);
                kmin = a < kmin ? a : kmin;
                kmax = b > kmax ? b : kmax;
            }
            if (lane == 0) {
                s_kmin[wv] = kmin;
                s_kmax[wv] = kmax;
            }
            __syncthreads();
            kmin = s_kmin[0];
            kmax = s_kmax[0];
            for (int i = 1; i < NW; ++i) {
                kmin = s_kmin[i] < kmin ? s_kmin[i] : kmin;
                kmax = s_kmax[i] > kmax ? s_kmax[i] : kmax;
            }
            int sel;
            if (kmin == kmax) {
                sel = m / 2;
            } else {
                sel = n0 < min_leaf ? min_leaf : n0;
                sel = sel > m - min_leaf ? m - min_leaf : sel;
            }
            unsigned long long prefix = 0ull;
            int rem = sel;
            for (int shift = 56; shift >= 0; shift -= 8) {
                if (tid < 256) s_hist[tid] = 0u;
                __syncthreads();
                const unsigned long long hi = shift == 56 ? 0ull : (~0ull << (shift + 8));
                for (int p = tid; p < m; p += NT) {
                    const unsigned long long key = ordered_key(-s_dot[s + p]);
                    if ((key & hi) == (prefix & hi)) atomicAdd(&s_hist[(key >> shift) & 255ull], 1u);
                }
                __syncthreads();
                if (tid == 0) {
                    int cum = 0;
                    for (int dg = 0; dg < 256; ++dg) {
                        const int c = static_cast<int>(s_hist[dg]);
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
            int run = 0;
            for (int p0 = 0; p0 < m; p0 += NT) {
                const int p = p0 + tid;
                const bool valid = p < m;
                const unsigned long long key = valid ? ordered_key(-s_dot[s + p]) : 0ull;
                const bool eq = valid && key == prefix;
                int tot;
                const int rank = run + block_excl_scan_flag<NW>(eq, s_warp, &tot);
                const bool right = valid && (key > prefix || (eq && rank >= rem));
                if (valid) s_lab[s + p] = right ? 1 : 0;
                run += tot;
            }
            n0 = sel;
            ++repairs;
            __syncthreads();
        }

        // ---- stable partition of positions s .. s+m-1 by label
        {
            int run1 = 0;
            for (int p0 = 0; p0 < m; p0 += NT) {
                const int p = p0 + tid;
                const bool valid = p < m;
                const bool one = valid && s_lab[s + p] != 0;
                int tot;
                const int ob = run1 + block_excl_scan_flag<NW>(one, s_warp, &tot);
                if (valid) s_tmp[s + (one ? n0 + ob : p - ob)] = s_ord[s + p];
                run1 += tot;
            }
            __syncthreads();
            for (int p = tid; p < m; p += NT) s_ord[s + p] = s_tmp[s + p];
        }

        // ---- log the split, emit leaves, push children (larger first)
        if (tid == 0) {
            ++splits;
            maxdep = maxdep > static_cast<unsigned long long>(dep + 1)
                         ? maxdep
                         : static_cast<unsigned long long>(dep + 1);
            if (node_log != nullptr) {
                const int64_t q = atomicAdd(&ctr->n_log, 1);
                if (q < node_log_cap) {
                    node_log[4 * q + 0] = root.start + s;
                    node_log[4 * q + 1] = m;
                    node_log[4 * q + 2] = n0;
                    node_log[4 * q + 3] = dep;
                }
            }
            const int cs[2] = {s, s + n0}, cz[2] = {n0, m - n0};
            const int first = cz[0] >= cz[1] ? 0 : 1;
            for (int t = 0; t < 2; ++t) {
                const int c = t == 0 ? first : 1 - first;
                if (cz[c] > leaf_max) {
                    if (s_sp < kStack) {
                        s_stack[s_sp][0] = cs[c];
                        s_stack[s_sp][1] = cz[c];
                        s_stack[s_sp][2] = dep + 1;
                        ++s_sp;
                    } else {
                        atomicOr(overflow, 2);
                    }
                } else {
                    const int64_t q = atomicAdd(&ctr->n_leaves, 1);
                    if (q < leaves_cap)
                        leaves[q] = LeafRec{root.tree, root.start + cs[c], cz[c], 0};
                    else
                        atomicOr(overflow, 1);
                }
            }
        }
        __syncthreads();
    }

    for (int i = tid; i < M; i += NT) perm[pbase + i] = s_ids[s_ord[i]];
    if (tid == 0) {
        atomicAdd(&dstats[0], assigned);
        atomicAdd(&dstats[1], repairs);
        atomicAdd(&dstats[2], splits);
        atomicMax(&dstats[3], maxdep);
    }
}

template <int DM, int G, int RB>
int launch_sub(const SubtreeArgs& a) {
    k_subtree_u8<DM, G, RB><<<static_cast<unsigned>(a.n_roots), kSubThreads, 0, a.stream>>>(
        a.X8, a.n, a.D, a.roots, a.perm, a.leaf_max, a.min_leaf, a.max_iter, a.seed, a.tree0,
        a.leaves, a.leaves_cap, a.node_log, a.node_log_cap, a.ctr, a.dstats, a.overflow);
    return hipGetLastError() == hipSuccess ? kOk : kHip;
}

template <int RB>
int launch_rb(const SubtreeArgs& a) {
    const int E = a.D / 16;
    if (a.D <= 64) {
        if (E <= 1) return launch_sub<64, 1, RB>(a);
        if (E <= 2) return launch_sub<64, 2, RB>(a);
        return launch_sub<64, 4, RB>(a);
    }
    if (a.D <= 128) return launch_sub<128, 8, RB>(a);
    if (a.D <= 256) return launch_sub<256, 16, RB>(a);
    return kUnsupported;
}

template <int RB>
int max_rows_rb(int D) {
    if (D % 16 != 0 || D <= 0) return 0;
    if (D <= 64) return sub_rows<64, RB>();
    if (D <= 128) return sub_rows<128, RB>();
    if (D <= 256) return sub_rows<256, RB>();
    return 0;
}

}  // namespace

// budget: LDS bytes for the rows of one workgroup (131072 or 65536)
int subtree_max_rows(int D, int budget) {
    return budget == 65536 ? max_rows_rb<65536>(D) : max_rows_rb<131072>(D);
}

int subtree_launch(const SubtreeArgs& a) {
    if (a.n_roots <= 0) return kOk;
    return a.row_budget == 65536 ? launch_rb<65536>(a) : launch_rb<131072>(a);
}

}  // namespace knng
