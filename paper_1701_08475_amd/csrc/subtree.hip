// Recursive two-means bisection (Alg. 2) of whole subtrees inside one
// workgroup, for uint8 rows (the lossless copy of integer data).
//
// Once a node holds at most S rows (S = 1024 for D <= 128), its rows fit in
// LDS, and every Lloyd pass, the margin-rank repair and the stable partition
// of it and of all its descendants run in one workgroup reading LDS: no HBM
// traffic after the first load and no per-level launches.  Each split takes
// the steps of the level-synchronous kernels in partition.hip: the keyed
// starting pair (members in id order, key (seed, tree, smallest id, size,
// j)), labels dot < h with the same FP64 values, exact integer side sums,
// the stop rule (no label changed, an empty side or the pass budget), the
// repair by (mu, id) rank and the stable partition (label-0 members first,
// in id order).  The node runs of perm are therefore the same.
//
// Margin on the matrix cores.  Centres of uint8 data lie in [0, 255], so
// w = c0 - c1 has |w| <= 255 and W = rint(w 2^22) fits 31 bits: four
// balanced int8 digit planes.  With x' = x - 128 (int8), the int8 MFMA gives
// sum_e x'_e W_e exactly, and x.W = sum x'W + 128 sum W.  Against the FP64
// margin of the level kernels, |x.W - 2^22 (x.w)| <= 0.5 sum x <= 127.5 D and
// the FP64 evaluation adds less than one unit, so |x.W - 2^22 h| > 128 D + 2
// decides dot < h exactly as the FP64 code does; rows inside that band (and
// every row of a node that needs the margin-rank repair) are evaluated with
// the FP64 code itself.  Side sums: the first pass of a node adds every row,
// later passes only the rows whose label changed.
//
// Depth-first with an explicit stack; the smaller child is split next and
// the larger pushed, so the stack never holds more than log2(S) + 1 nodes.
#include "knng_internal.hpp"
#include "partition_dev.hpp"
#include "wave.hpp"

#include <cstdio>
#include <type_traits>

namespace knng {
namespace {
using namespace pdev;

typedef int i32x4 __attribute__((ext_vector_type(4)));

// Largest subtree (rows) per row width DM when its rows take at most RB
// bytes of LDS (128 KiB: one workgroup per CU; 64 KiB: two).
template <int DM, int RB>
constexpr int sub_rows() {
    return DM * 1024 <= RB ? 1024 : RB / DM;
}
constexpr int kStack = 32;

// NW wavefronts per workgroup.
constexpr int kSubWaves = 8;
constexpr int kSubThreads = kSubWaves * kWave;
constexpr double kScale = 4194304.0;  // 2^22

__device__ __forceinline__ int dpp_i32_sum16(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false);   // xor 1
    v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false);   // xor 2
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);  // mirror in 8
    v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, false);  // mirror in 16
    return v;
}

// Row r of the LDS row store keeps its 16-byte chunk j at chunk j ^ (r & swz)
// (swz + 1 divides D / 16), which spreads the chunks that lanes of one
// instruction read from different rows over the LDS banks.
__device__ __forceinline__ int chunk_at(int r, int j, int swz) { return j ^ (r & swz); }

template <int DM, int G, int RB>
__global__ __launch_bounds__(kSubThreads) void k_subtree_u8(
    const uint8_t* __restrict__ X8, int64_t n, int D, const NodeRec* __restrict__ roots,
    int32_t* __restrict__ perm, int leaf_max, int min_leaf, int max_iter, uint64_t seed,
    int tree0, LeafRec* __restrict__ leaves, int64_t leaves_cap, int32_t* __restrict__ node_log,
    int64_t node_log_cap, LevelCounters* __restrict__ ctr,
    unsigned long long* __restrict__ dstats, int* __restrict__ overflow) {
    constexpr int S = sub_rows<DM, RB>();
    constexpr int NW = kSubWaves, NT = kSubThreads;
    constexpr int RPW = kWave / G;     // rows per wave step of the FP64 code
    constexpr int KB = (DM + 63) / 64; // 64-element blocks of the matrix-core margin
    __shared__ __align__(16) uint8_t s_rows[S * DM];
    __shared__ int32_t s_ids[S];
    __shared__ uint16_t s_ord[S], s_tmp[S];  // s_tmp: partition buffer, and the list of
                                             // rows the FP64 code decides in a pass
    __shared__ uint8_t s_lab[S];
    __shared__ double s_dot[S];
    __shared__ double s_cen[2 * DM];
    __shared__ __align__(16) int8_t s_dig[4][KB * 64];  // digit planes of W, zero past D
    __shared__ int32_t s_acc[2][DM];                    // side-1 change sums, by pass parity
    __shared__ uint32_t s_a1[DM], s_tot[DM];
    __shared__ uint32_t s_hist[256];
    __shared__ int s_cnt[2][3];  // (ones, changed, FP64 rows), by pass parity
    __shared__ unsigned long long s_sw[2];
    __shared__ int8_t s_dl[NW][16];
    __shared__ int s_stack[kStack][3];
    __shared__ int s_sp, s_node[3], s_pair[2], s_warp[NW], s_rem, s_bin;
    __shared__ unsigned long long s_kmin[NW], s_kmax[NW];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int g = lane / G, l = lane % G;     // FP64 code: lane group, lane in group
    const int tc = lane & 15, tq = lane >> 4; // matrix-core tile: column / row, k-group
    const NodeRec root = roots[blockIdx.x];
    const int M = root.size;
    const size_t pbase = static_cast<size_t>(root.tree) * n + root.start;
    const uint64_t tg = static_cast<uint64_t>(tree0 + root.tree);
    const int vpr = D / 16;  // 16-byte chunks per row
    int swz = 1;
    while (swz < 8 && (vpr % (2 * swz)) == 0) swz *= 2;
    swz -= 1;
    const double bnd = 128.0 * D + 2.0;

    for (int i = tid; i < M; i += NT) {
        s_ids[i] = perm[pbase + i];
        s_ord[i] = static_cast<uint16_t>(i);
    }
    __syncthreads();
    for (int q = tid; q < M * vpr; q += NT) {
        const int r = q / vpr, c = q - r * vpr;
        reinterpret_cast<uint4*>(s_rows)[r * vpr + chunk_at(r, c, swz)] =
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

    // FP64 margin of local row lr (every lane of a group returns it), with the
    // lane layout and summation order of the level kernels
    auto fp64_dot = [&](int lr, const double (&w)[16]) -> double {
        uint4 raw = make_uint4(0u, 0u, 0u, 0u);
        if (l * 16 < D)
            raw = *reinterpret_cast<const uint4*>(s_rows + lr * D + 16 * chunk_at(lr, l, swz));
        const uint32_t wd[4] = {raw.x, raw.y, raw.z, raw.w};
        double dot = 0.0;
#pragma unroll
        for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                dot = fma(static_cast<double>((wd[k4] >> (8 * b)) & 255u), w[4 * k4 + b], dot);
        return group_sum_f64<G>(dot);
    };

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
            s_a1[e] = 0u;
            s_acc[0][e] = 0;
            s_acc[1][e] = 0;
        }
        if (tid < 6) s_cnt[tid / 3][tid % 3] = 0;
        if (tid < 2) s_sw[tid] = 0ull;
        __syncthreads();
        {
            const int ra = s_ord[s + s_pair[0]], rb = s_ord[s + s_pair[1]];
            for (int e = tid; e < D; e += NT) {
                const int b = e & 15;
                s_cen[e] = static_cast<double>(s_rows[ra * D + 16 * chunk_at(ra, e >> 4, swz) + b]);
                s_cen[DM + e] = static_cast<double>(s_rows[rb * D + 16 * chunk_at(rb, e >> 4, swz) + b]);
            }
        }
        __syncthreads();

        // ---- Lloyd passes
        int n1 = 0;
        double w[16];
        double h = 0.0;
        // one Lloyd pass; FIRST = the node's first pass (adds every row to the
        // side and total sums); returns the stop decision
        auto run_pass = [&](auto first_tag, int pass) -> bool {
            constexpr bool first = decltype(first_tag)::value;
            const int par = pass & 1;
            // FP64 weights and threshold, exactly as the level kernels form them
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
            h = 0.5 * (q0 - q1);
            // digit planes of W = rint(w 2^22) and sum W
            for (int e = tid; e < KB * 64; e += NT) {
                int d0 = 0, d1 = 0, d2 = 0, d3 = 0;
                if (e < D) {
                    int wv_ = static_cast<int>(rint((s_cen[e] - s_cen[DM + e]) * kScale));
                    atomicAdd(&s_sw[par], static_cast<unsigned long long>(static_cast<long long>(wv_)));
                    d0 = ((wv_ + 128) & 255) - 128;
                    wv_ = (wv_ - d0) / 256;
                    d1 = ((wv_ + 128) & 255) - 128;
                    wv_ = (wv_ - d1) / 256;
                    d2 = ((wv_ + 128) & 255) - 128;
                    d3 = (wv_ - d2) / 256;
                }
                s_dig[0][e] = static_cast<int8_t>(d0);
                s_dig[1][e] = static_cast<int8_t>(d1);
                s_dig[2][e] = static_cast<int8_t>(d2);
                s_dig[3][e] = static_cast<int8_t>(d3);
            }
            __syncthreads();
            i32x4 bop[KB];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                bop[kb] = i32x4{0, 0, 0, 0};
                if (tc < 4) bop[kb] = *reinterpret_cast<const i32x4*>(&s_dig[tc][kb * 64 + 16 * tq]);
            }
            const double xw0 = 128.0 * static_cast<double>(static_cast<long long>(s_sw[par]));
            const double hs = h * kScale;
            const double colscale = tc < 4 ? static_cast<double>(1ll << (8 * tc)) : 0.0;

            int32_t acc1[KB][16];
            uint32_t tot1[first ? KB : 1][16];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    acc1[kb][t] = 0;
                    if constexpr (first) tot1[kb][t] = 0u;
                }
            bool wave_delta = false;
            int my1 = 0, mych = 0;
            for (int p0 = 16 * wv; p0 < m; p0 += 16 * NW) {  // uniform per wave
                const int pr = p0 + tc;
                const bool valid = pr < m;
                const int lr = s_ord[s + (valid ? pr : m - 1)];
                uint4 raw[KB];
                i32x4 acc = i32x4{0, 0, 0, 0};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const int jj = kb * 4 + tq;
                    raw[kb] = make_uint4(0u, 0u, 0u, 0u);
                    if (jj < vpr)
                        raw[kb] = *reinterpret_cast<const uint4*>(s_rows + lr * D +
                                                                  16 * chunk_at(lr, jj, swz));
                    const i32x4 a = i32x4{static_cast<int>(raw[kb].x ^ 0x80808080u),
                                          static_cast<int>(raw[kb].y ^ 0x80808080u),
                                          static_cast<int>(raw[kb].z ^ 0x80808080u),
                                          static_cast<int>(raw[kb].w ^ 0x80808080u)};
                    acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, bop[kb], acc, 0, 0, 0);
                }
                // lane (tq, tc): rows 4 tq + i, column (digit plane) tc
                double v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    v[i] = static_cast<double>(acc[i]) * colscale;
                    v[i] += dpp_f64<0xB1>(v[i]);
                    v[i] += dpp_f64<0x4E>(v[i]);
                }
                // lane (tq, c < 4) decides row 4 tq + c
                int dl = 0;
                if (tc < 4) {
                    const double xw = (tc == 0 ? v[0] : tc == 1 ? v[1] : tc == 2 ? v[2] : v[3]) + xw0;
                    const double mg = xw - hs;
                    const int pi = p0 + 4 * tq + tc;
                    if (pi < m) {
                        if (mg < -bnd || mg > bnd) {
                            const int lab = mg < -bnd ? 1 : 0;
                            const int old = s_lab[s + pi];
                            mych += (!first && old != lab) ? 1 : 0;
                            s_lab[s + pi] = static_cast<uint8_t>(lab);
                            my1 += lab;
                            dl = first ? lab : lab - old;
                        } else {
                            s_tmp[atomicAdd(&s_cnt[par][2], 1)] = static_cast<uint16_t>(pi);
                        }
                    }
                    s_dl[wv][4 * tq + tc] = static_cast<int8_t>(dl);
                }
                const bool any = __ballot(dl != 0) != 0ull;
                if (first || any) {
                    wave_delta = wave_delta || any;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    const int d = valid ? static_cast<int>(s_dl[wv][tc]) : 0;
                    const uint32_t in = valid ? 1u : 0u;
#pragma unroll
                    for (int kb = 0; kb < KB; ++kb) {
                        const uint32_t wd[4] = {raw[kb].x, raw[kb].y, raw[kb].z, raw[kb].w};
#pragma unroll
                        for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
                            for (int b = 0; b < 4; ++b) {
                                const int x = static_cast<int>((wd[k4] >> (8 * b)) & 255u);
                                acc1[kb][4 * k4 + b] = __mul24(d, x) + acc1[kb][4 * k4 + b];
                                if constexpr (first) tot1[kb][4 * k4 + b] += in * static_cast<uint32_t>(x);
                            }
                    }
                }
            }
            // the wave's change sums: lanes of one 16-lane row hold the same elements
            if (first || wave_delta) {
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                    for (int t = 0; t < 16; ++t) {
                        const int e = kb * 64 + 16 * tq + t;
                        const int sa = dpp_i32_sum16(acc1[kb][t]);
                        int st = 0;
                        if constexpr (first) st = dpp_i32_sum16(static_cast<int>(tot1[kb][t]));
                        if (tc == 0 && e < D) {
                            if (sa != 0) atomicAdd(&s_acc[par][e], sa);
                            if constexpr (first) atomicAdd(&s_tot[e], static_cast<uint32_t>(st));
                        }
                    }
            }
            my1 = wave_sum_i32(my1);
            mych = wave_sum_i32(mych);
            if (lane == 0) {
                atomicAdd(&s_cnt[par][0], my1);
                atomicAdd(&s_cnt[par][1], mych);
            }
            __syncthreads();
            // rows inside the error band: the FP64 code decides them
            const int nfb = s_cnt[par][2];
            if (nfb > 0) {
                int f1 = 0, fch = 0;
                for (int f0 = wv * RPW; f0 < nfb; f0 += NW * RPW) {  // uniform per wave
                    const int f = f0 + g;
                    const bool valid = f < nfb;
                    const int pi = valid ? s_tmp[f] : 0;
                    const int lr = s_ord[s + pi];
                    const double dot = fp64_dot(lr, w);
                    const int lab = dot < h ? 1 : 0;
                    const int old = valid ? static_cast<int>(s_lab[s + pi]) : 0;
                    const int dl = valid ? (first ? lab : lab - old) : 0;
                    if (valid && l == 0) {
                        fch += (!first && old != lab) ? 1 : 0;
                        s_lab[s + pi] = static_cast<uint8_t>(lab);
                        f1 += lab;
                    }
                    if (dl != 0 && l * 16 < D) {
                        const uint4 raw = *reinterpret_cast<const uint4*>(
                            s_rows + lr * D + 16 * chunk_at(lr, l, swz));
                        const uint32_t wd[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
                        for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
                            for (int b = 0; b < 4; ++b)
                                atomicAdd(&s_acc[par][l * 16 + 4 * k4 + b],
                                          dl * static_cast<int>((wd[k4] >> (8 * b)) & 255u));
                    }
                }
                f1 = wave_sum_i32(f1);
                fch = wave_sum_i32(fch);
                if (lane == 0) {
                    atomicAdd(&s_cnt[par][0], f1);
                    atomicAdd(&s_cnt[par][1], fch);
                }
                __syncthreads();
            }
            assigned += static_cast<unsigned long long>(m);
            n1 = s_cnt[par][0];
            const int ch = s_cnt[par][1];
            const int n0 = m - n1;
            const bool stop =
                n1 == 0 || n0 == 0 || (pass >= 1 && ch == 0) || pass + 1 >= max_iter;
            // next pass's accumulators start at zero
            for (int e = tid; e < DM; e += NT) s_acc[par ^ 1][e] = 0;
            if (tid < 3) s_cnt[par ^ 1][tid] = 0;
            if (tid == 0) s_sw[par ^ 1] = 0ull;
            if (!stop) {
                const double dn0 = static_cast<double>(n0), dn1 = static_cast<double>(n1);
                for (int e = tid; e < D; e += NT) {
                    const uint32_t a1 = s_a1[e] + static_cast<uint32_t>(s_acc[par][e]);
                    s_a1[e] = a1;
                    const double t = static_cast<double>(s_tot[e]);
                    const double s1 = static_cast<double>(a1);
                    s_cen[e] = (t - s1) / dn0;
                    s_cen[DM + e] = s1 / dn1;
                }
            }
            __syncthreads();
            return stop;
        };
        for (int pass = 0; pass < max_iter; ++pass) {
            const bool stop = pass == 0 ? run_pass(std::true_type{}, pass)
                                        : run_pass(std::false_type{}, pass);
            if (stop) break;
        }
        int n0 = m - n1;

        // ---- margin-rank repair: first sel members by (mu, id) go left,
        // mu ascending = dot descending = key of -dot ascending
        if (n0 < min_leaf || n1 < min_leaf) {
            // FP64 margins of the final pass (its weights are still in w, h)
            for (int p0 = wv * RPW; p0 < m; p0 += NW * RPW) {  // uniform per wave
                const int p = p0 + g;
                const bool valid = p < m;
                const double dot = fp64_dot(s_ord[s + (valid ? p : 0)], w);
                if (valid && l == 0) s_dot[s + p] = dot;
            }
            __syncthreads();
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
                block_hist_pick<NW>(s_hist, rem, s_warp, &s_bin, &s_rem);
                prefix |= static_cast<unsigned long long>(s_bin) << shift;
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
        stat_add(dstats + 4 * kStatWords, blockIdx.x, assigned);
        stat_add(dstats + kStatWords, blockIdx.x, repairs);
        stat_add(dstats + 2 * kStatWords, blockIdx.x, splits);
        stat_max(dstats + 3 * kStatWords, blockIdx.x, maxdep);
    }
}

// ------------------------------------------------------------- wave subtrees
// The same splits for subtrees of at most kWaveRows rows, one wavefront each
// (workgroup of one wavefront, rows in about 25 KiB of LDS, six per CU):
// wave-level reductions and ballots only, no block barriers.  Steps and
// arithmetic as in k_subtree_u8: keyed pair, matrix-core margin decided
// outside the error band and FP64 inside it, exact side sums (changes only
// after the first pass), stop rule, margin-rank repair on FP64 margins
// recomputed with the level kernels' order, stable partition.
// 144 rows of 128 dimensions: six waves per CU hide more of the latency of
// the wave-serial steps than four waves of 240 rows, and the extra level of
// the level kernels above them costs less (C2 build 37.0 -> 35.8 ms; 112,
// 128, 160 and 176 rows all measured between the two).
constexpr int kWaveRows = 144;

template <int DM, int G>
__global__ __launch_bounds__(64) void k_subtree_wave_u8(
    const uint8_t* __restrict__ X8, int64_t n, int D, const NodeRec* __restrict__ roots,
    int32_t* __restrict__ perm, int leaf_max, int min_leaf, int max_iter, uint64_t seed,
    int tree0, LeafRec* __restrict__ leaves, int64_t leaves_cap, int32_t* __restrict__ node_log,
    int64_t node_log_cap, LevelCounters* __restrict__ ctr,
    unsigned long long* __restrict__ dstats, int* __restrict__ overflow) {
    constexpr int S = kWaveRows;
    constexpr int RPW = kWave / G;      // rows per step of the FP64 code
    constexpr int KB = (DM + 63) / 64;  // 64-element blocks of the matrix-core margin
    constexpr int KR = (S + 63) / 64;   // positions per lane in the repair
    __shared__ __align__(16) uint8_t s_rows[S * DM];
    __shared__ int32_t s_ids[S];
    __shared__ uint8_t s_ord[S], s_tmp[S], s_lab[S];
    __shared__ double s_cen[2 * DM];
    __shared__ __align__(16) int8_t s_dig[4][KB * 64];
    __shared__ uint32_t s_a1[DM], s_tot[DM];
    __shared__ uint32_t s_hist[256];
    __shared__ double s_dot[S];
    __shared__ int8_t s_dl[16];
    __shared__ int s_stack[16][3];

    const int lane = threadIdx.x;
    const int g = lane / G, l = lane % G;
    const int tc = lane & 15, tq = lane >> 4;
    const NodeRec root = roots[blockIdx.x];
    const int M = root.size;
    const size_t pbase = static_cast<size_t>(root.tree) * n + root.start;
    const uint64_t tg = static_cast<uint64_t>(tree0 + root.tree);
    const int vpr = D / 16;
    int swz = 1;
    while (swz < 8 && (vpr % (2 * swz)) == 0) swz *= 2;
    swz -= 1;
    const double bnd = 128.0 * D + 2.0;

    for (int i = lane; i < M; i += kWave) {
        s_ids[i] = perm[pbase + i];
        s_ord[i] = static_cast<uint8_t>(i);
    }
    wave_lds_sync();
    for (int q = lane; q < M * vpr; q += kWave) {
        const int r = q / vpr, c = q - r * vpr;
        reinterpret_cast<uint4*>(s_rows)[r * vpr + chunk_at(r, c, swz)] =
            reinterpret_cast<const uint4*>(X8 + static_cast<size_t>(s_ids[r]) * D)[c];
    }
    int sp = 1;  // stack depth (uniform)
    if (lane == 0) {
        s_stack[0][0] = 0;
        s_stack[0][1] = M;
        s_stack[0][2] = root.chunk0;
    }
    unsigned long long assigned = 0, splits = 0, repairs = 0, maxdep = 0;
    wave_lds_sync();

    auto fp64_dot = [&](int lr, const double (&w)[16]) -> double {
        uint4 raw = make_uint4(0u, 0u, 0u, 0u);
        if (l * 16 < D)
            raw = *reinterpret_cast<const uint4*>(s_rows + lr * D + 16 * chunk_at(lr, l, swz));
        const uint32_t wd[4] = {raw.x, raw.y, raw.z, raw.w};
        double dot = 0.0;
#pragma unroll
        for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                dot = fma(static_cast<double>((wd[k4] >> (8 * b)) & 255u), w[4 * k4 + b], dot);
        return group_sum_f64<G>(dot);
    };

    while (sp > 0) {
        --sp;
        const int s = s_stack[sp][0], m = s_stack[sp][1], dep = s_stack[sp][2];
        wave_lds_sync();
        // ---- starting pair
        int pa, pb;
        {
            const uint64_t mm = static_cast<uint64_t>(m);
            const uint64_t min_id = static_cast<uint64_t>(static_cast<uint32_t>(s_ids[s_ord[s]]));
            const uint64_t a = pair_hash(seed, tg, min_id, mm, 0) % mm;
            uint64_t b = pair_hash(seed, tg, min_id, mm, 1) % (mm - 1);
            if (b >= a) ++b;
            pa = static_cast<int>(a);
            pb = static_cast<int>(b);
        }
        {
            const int ra = s_ord[s + pa], rb = s_ord[s + pb];
            for (int e = lane; e < DM; e += kWave) {
                s_tot[e] = 0u;
                s_a1[e] = 0u;
                if (e < D) {
                    const int b = e & 15;
                    s_cen[e] = static_cast<double>(s_rows[ra * D + 16 * chunk_at(ra, e >> 4, swz) + b]);
                    s_cen[DM + e] = static_cast<double>(s_rows[rb * D + 16 * chunk_at(rb, e >> 4, swz) + b]);
                }
            }
        }
        wave_lds_sync();

        int n1 = 0;
        double w[16];
        double h = 0.0;
        auto run_pass = [&](auto first_tag, int pass) -> bool {
            constexpr bool first = decltype(first_tag)::value;
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
            h = 0.5 * (q0 - q1);
            double swp = 0.0;  // sum of W (exact integers in FP64)
            for (int e = lane; e < KB * 64; e += kWave) {
                int d0 = 0, d1 = 0, d2 = 0, d3 = 0;
                if (e < D) {
                    int wv_ = static_cast<int>(rint((s_cen[e] - s_cen[DM + e]) * kScale));
                    swp += static_cast<double>(wv_);
                    d0 = ((wv_ + 128) & 255) - 128;
                    wv_ = (wv_ - d0) / 256;
                    d1 = ((wv_ + 128) & 255) - 128;
                    wv_ = (wv_ - d1) / 256;
                    d2 = ((wv_ + 128) & 255) - 128;
                    d3 = (wv_ - d2) / 256;
                }
                s_dig[0][e] = static_cast<int8_t>(d0);
                s_dig[1][e] = static_cast<int8_t>(d1);
                s_dig[2][e] = static_cast<int8_t>(d2);
                s_dig[3][e] = static_cast<int8_t>(d3);
            }
            swp = group_sum_f64<64>(swp);
            wave_lds_sync();
            i32x4 bop[KB];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                bop[kb] = i32x4{0, 0, 0, 0};
                if (tc < 4) bop[kb] = *reinterpret_cast<const i32x4*>(&s_dig[tc][kb * 64 + 16 * tq]);
            }
            const double xw0 = 128.0 * swp;
            const double hs = h * kScale;
            const double colscale = tc < 4 ? static_cast<double>(1ll << (8 * tc)) : 0.0;

            int32_t acc1[KB][16];
            uint32_t tot1[first ? KB : 1][16];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    acc1[kb][t] = 0;
                    if constexpr (first) tot1[kb][t] = 0u;
                }
            bool wave_delta = false;
            int my1 = 0, mych = 0, nfb = 0;
            for (int p0 = 0; p0 < m; p0 += 16) {
                const int pr = p0 + tc;
                const bool valid = pr < m;
                const int lr = s_ord[s + (valid ? pr : m - 1)];
                uint4 raw[KB];
                i32x4 acc = i32x4{0, 0, 0, 0};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const int jj = kb * 4 + tq;
                    raw[kb] = make_uint4(0u, 0u, 0u, 0u);
                    if (jj < vpr)
                        raw[kb] = *reinterpret_cast<const uint4*>(s_rows + lr * D +
                                                                  16 * chunk_at(lr, jj, swz));
                    const i32x4 a = i32x4{static_cast<int>(raw[kb].x ^ 0x80808080u),
                                          static_cast<int>(raw[kb].y ^ 0x80808080u),
                                          static_cast<int>(raw[kb].z ^ 0x80808080u),
                                          static_cast<int>(raw[kb].w ^ 0x80808080u)};
                    acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, bop[kb], acc, 0, 0, 0);
                }
                double v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    v[i] = static_cast<double>(acc[i]) * colscale;
                    v[i] += dpp_f64<0xB1>(v[i]);
                    v[i] += dpp_f64<0x4E>(v[i]);
                }
                int dl = 0;
                bool fb = false;
                const int pi = p0 + 4 * tq + tc;
                if (tc < 4 && pi < m) {
                    const double xw = (tc == 0 ? v[0] : tc == 1 ? v[1] : tc == 2 ? v[2] : v[3]) + xw0;
                    const double mg = xw - hs;
                    if (mg < -bnd || mg > bnd) {
                        const int lab = mg < -bnd ? 1 : 0;
                        const int old = s_lab[s + pi];
                        mych += (!first && old != lab) ? 1 : 0;
                        s_lab[s + pi] = static_cast<uint8_t>(lab);
                        my1 += lab;
                        dl = first ? lab : lab - old;
                    } else {
                        fb = true;
                    }
                }
                // rows inside the error band, listed in position order
                const unsigned long long bf = __ballot(fb);
                if (fb) s_tmp[nfb + __popcll(bf & ((1ull << lane) - 1ull))] = static_cast<uint8_t>(pi);
                nfb += __popcll(bf);
                if (tc < 4) s_dl[4 * tq + tc] = static_cast<int8_t>(dl);
                const bool any = __ballot(dl != 0) != 0ull;
                if (first || any) {
                    wave_delta = wave_delta || any;
                    wave_lds_sync();
                    const int d = valid ? static_cast<int>(s_dl[tc]) : 0;
                    const uint32_t in = valid ? 1u : 0u;
#pragma unroll
                    for (int kb = 0; kb < KB; ++kb) {
                        const uint32_t wd[4] = {raw[kb].x, raw[kb].y, raw[kb].z, raw[kb].w};
#pragma unroll
                        for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
                            for (int b = 0; b < 4; ++b) {
                                const int x = static_cast<int>((wd[k4] >> (8 * b)) & 255u);
                                acc1[kb][4 * k4 + b] = __mul24(d, x) + acc1[kb][4 * k4 + b];
                                if constexpr (first) tot1[kb][4 * k4 + b] += in * static_cast<uint32_t>(x);
                            }
                    }
                    wave_lds_sync();
                }
            }
            if (first || wave_delta) {
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                    for (int t = 0; t < 16; ++t) {
                        const int e = kb * 64 + 16 * tq + t;
                        const int sa = dpp_i32_sum16(acc1[kb][t]);
                        int st = 0;
                        if constexpr (first) st = dpp_i32_sum16(static_cast<int>(tot1[kb][t]));
                        if (tc == 0 && e < D) {
                            s_a1[e] += static_cast<uint32_t>(sa);
                            if constexpr (first) s_tot[e] = static_cast<uint32_t>(st);
                        }
                    }
            }
            wave_lds_sync();
            // rows inside the error band: the FP64 code decides them
            for (int f0 = 0; f0 < nfb; f0 += RPW) {
                const int f = f0 + g;
                const bool valid = f < nfb;
                const int pi = valid ? s_tmp[f] : 0;
                const int lr = s_ord[s + pi];
                const double dot = fp64_dot(lr, w);
                const int lab = dot < h ? 1 : 0;
                const int old = valid ? static_cast<int>(s_lab[s + pi]) : 0;
                const int dl = valid ? (first ? lab : lab - old) : 0;
                if (valid && l == 0) {
                    mych += (!first && old != lab) ? 1 : 0;
                    s_lab[s + pi] = static_cast<uint8_t>(lab);
                    my1 += lab;
                }
                if (dl != 0 && l * 16 < D) {
                    const uint4 raw = *reinterpret_cast<const uint4*>(
                        s_rows + lr * D + 16 * chunk_at(lr, l, swz));
                    const uint32_t wd[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
                        for (int b = 0; b < 4; ++b)
                            atomicAdd(&s_a1[l * 16 + 4 * k4 + b],
                                      static_cast<uint32_t>(dl * static_cast<int>((wd[k4] >> (8 * b)) & 255u)));
                }
            }
            assigned += static_cast<unsigned long long>(m);
            n1 = wave_sum_i32(my1);
            const int ch = wave_sum_i32(mych);
            const int n0 = m - n1;
            const bool stop =
                n1 == 0 || n0 == 0 || (pass >= 1 && ch == 0) || pass + 1 >= max_iter;
            wave_lds_sync();
            if (!stop) {
                const double dn0 = static_cast<double>(n0), dn1 = static_cast<double>(n1);
                for (int e = lane; e < D; e += kWave) {
                    const double t = static_cast<double>(s_tot[e]);
                    const double s1 = static_cast<double>(s_a1[e]);
                    s_cen[e] = (t - s1) / dn0;
                    s_cen[DM + e] = s1 / dn1;
                }
            }
            wave_lds_sync();
            return stop;
        };
        for (int pass = 0; pass < max_iter; ++pass) {
            const bool stop = pass == 0 ? run_pass(std::true_type{}, pass)
                                        : run_pass(std::false_type{}, pass);
            if (stop) break;
        }
        int n0 = m - n1;

        // ---- margin-rank repair on FP64 margins of the final pass
        if (n0 < min_leaf || n1 < min_leaf) {
            for (int f0 = 0; f0 < m; f0 += RPW) {
                const int p = f0 + g;
                const bool valid = p < m;
                const double dot = fp64_dot(s_ord[s + (valid ? p : 0)], w);
                if (valid && l == 0) s_dot[p] = dot;
            }
            wave_lds_sync();
            uint64_t key[KR];
            bool kv[KR];
#pragma unroll
            for (int r = 0; r < KR; ++r) {
                const int p = r * 64 + lane;
                kv[r] = p < m;
                key[r] = kv[r] ? ordered_key(-s_dot[p]) : 0ull;
            }
            unsigned long long kmin = ~0ull, kmax = 0ull;
#pragma unroll
            for (int r = 0; r < KR; ++r)
                if (kv[r]) {
                    kmin = key[r] < kmin ? key[r] : kmin;
                    kmax = key[r] > kmax ? key[r] : kmax;
                }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                const unsigned long long a = shfl_xor_u64(kmin, o), b = shfl_xor_u64(kmax, o);
                kmin = a < kmin ? a : kmin;
                kmax = b > kmax ? b : kmax;
            }
            int sel;
            if (kmin == kmax) {
                sel = m / 2;
            } else {
                sel = n0 < min_leaf ? min_leaf : n0;
                sel = sel > m - min_leaf ? m - min_leaf : sel;
            }
            // radix selection of the key of rank sel (0-based), 8-bit digits
            uint64_t prefix = 0ull;
            int rem = sel;
            for (int shift = 56; shift >= 0; shift -= 8) {
#pragma unroll
                for (int q = 0; q < 4; ++q) s_hist[4 * lane + q] = 0u;
                wave_lds_sync();
                const uint64_t hi = shift == 56 ? 0ull : (~0ull << (shift + 8));
#pragma unroll
                for (int r = 0; r < KR; ++r)
                    if (kv[r] && (key[r] & hi) == (prefix & hi))
                        atomicAdd(&s_hist[(key[r] >> shift) & 255ull], 1u);
                wave_lds_sync();
                uint32_t h4[4];
                int loc = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    h4[q] = s_hist[4 * lane + q];
                    loc += static_cast<int>(h4[q]);
                }
                int total;
                const int excl = wave_excl_scan(loc, &total);
                int digit = 0, nrem = 0;
                const bool mine = excl <= rem && rem < excl + loc;
                if (mine) {
                    int cum = excl;
                    bool done = false;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int hq = static_cast<int>(h4[q]);
                        if (!done && rem < cum + hq) {
                            digit = 4 * lane + q;
                            nrem = rem - cum;
                            done = true;
                        }
                        cum += hq;
                    }
                }
                const unsigned long long bm = __ballot(mine);
                const int src = static_cast<int>(__builtin_ctzll(bm));
                digit = __shfl(digit, src, kWave);
                nrem = __shfl(nrem, src, kWave);
                prefix |= static_cast<uint64_t>(digit) << shift;
                rem = nrem;
                wave_lds_sync();
            }
            // relabel: below the key left, above right, equal keys left while
            // their rank in position order is below rem
            int eq_seen = 0;
#pragma unroll
            for (int r = 0; r < KR; ++r) {
                const bool eq = kv[r] && key[r] == prefix;
                const unsigned long long be = __ballot(eq);
                const int rank = eq_seen + __popcll(be & ((1ull << lane) - 1ull));
                eq_seen += __popcll(be);
                if (kv[r]) {
                    const bool right = key[r] > prefix || (eq && rank >= rem);
                    s_lab[s + r * 64 + lane] = right ? 1 : 0;
                }
            }
            n0 = sel;
            ++repairs;
            wave_lds_sync();
        }

        // ---- stable partition by label
        {
            int ones = 0;
            for (int p0 = 0; p0 < m; p0 += kWave) {
                const int p = p0 + lane;
                const bool valid = p < m;
                const bool one = valid && s_lab[s + p] != 0;
                const unsigned long long b1 = __ballot(one);
                const int ob = ones + __popcll(b1 & ((1ull << lane) - 1ull));
                if (valid) s_tmp[one ? n0 + ob : p - ob] = s_ord[s + p];
                ones += __popcll(b1);
            }
            wave_lds_sync();
            for (int p = lane; p < m; p += kWave) s_ord[s + p] = s_tmp[p];
            wave_lds_sync();
        }

        // ---- log, leaves, children (larger pushed first)
        ++splits;
        maxdep = maxdep > static_cast<unsigned long long>(dep + 1) ? maxdep
                                                                     : static_cast<unsigned long long>(dep + 1);
        const int cs[2] = {s, s + n0}, cz[2] = {n0, m - n0};
        const int first = cz[0] >= cz[1] ? 0 : 1;
        if (lane == 0 && node_log != nullptr) {
            const int64_t q = atomicAdd(&ctr->n_log, 1);
            if (q < node_log_cap) {
                node_log[4 * q + 0] = root.start + s;
                node_log[4 * q + 1] = m;
                node_log[4 * q + 2] = n0;
                node_log[4 * q + 3] = dep;
            }
        }
        for (int t = 0; t < 2; ++t) {
            const int c = t == 0 ? first : 1 - first;
            if (cz[c] > leaf_max) {
                if (sp < 16) {
                    if (lane == 0) {
                        s_stack[sp][0] = cs[c];
                        s_stack[sp][1] = cz[c];
                        s_stack[sp][2] = dep + 1;
                    }
                    ++sp;
                } else if (lane == 0) {
                    atomicOr(overflow, 2);
                }
            } else if (lane == 0) {
                const int64_t q = atomicAdd(&ctr->n_leaves, 1);
                if (q < leaves_cap)
                    leaves[q] = LeafRec{root.tree, root.start + cs[c], cz[c], 0};
                else
                    atomicOr(overflow, 1);
            }
        }
        wave_lds_sync();
    }

    for (int i = lane; i < M; i += kWave) perm[pbase + i] = s_ids[s_ord[i]];
    if (lane == 0) {
        stat_add(dstats + 4 * kStatWords, blockIdx.x, assigned);
        stat_add(dstats + kStatWords, blockIdx.x, repairs);
        stat_add(dstats + 2 * kStatWords, blockIdx.x, splits);
        stat_max(dstats + 3 * kStatWords, blockIdx.x, maxdep);
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
    return kUnsupported;
}

template <int RB>
int max_rows_rb(int D) {
    if (D % 16 != 0 || D <= 0) return 0;
    if (D <= 64) return sub_rows<64, RB>();
    if (D <= 128) return sub_rows<128, RB>();
    return 0;
}

template <int DM, int G>
int launch_wave(const SubtreeArgs& a) {
    k_subtree_wave_u8<DM, G><<<static_cast<unsigned>(a.n_roots), 64, 0, a.stream>>>(
        a.X8, a.n, a.D, a.roots, a.perm, a.leaf_max, a.min_leaf, a.max_iter, a.seed, a.tree0,
        a.leaves, a.leaves_cap, a.node_log, a.node_log_cap, a.ctr, a.dstats, a.overflow);
    return hipGetLastError() == hipSuccess ? kOk : kHip;
}

}  // namespace

// budget: LDS bytes for the rows of one workgroup (131072 or 65536), or 0 for
// the one-wavefront subtrees
int subtree_max_rows(int D, int budget) {
    if (budget == 0) return (D % 16 == 0 && D > 0 && D <= 128) ? kWaveRows : 0;
    return budget == 65536 ? max_rows_rb<65536>(D) : max_rows_rb<131072>(D);
}

int subtree_launch(const SubtreeArgs& a) {
    if (a.n_roots <= 0) return kOk;
    if (a.row_budget == 0) {
        const int E = a.D / 16;
        if (a.D <= 64) {
            if (E <= 1) return launch_wave<64, 1>(a);
            if (E <= 2) return launch_wave<64, 2>(a);
            return launch_wave<64, 4>(a);
        }
        if (a.D <= 128) return launch_wave<128, 8>(a);
        return kUnsupported;
    }
    return a.row_budget == 65536 ? launch_rb<65536>(a) : launch_rb<131072>(a);
}

}  // namespace knng
