// Assignment passes of the level-synchronous two-means bisection over FP32
// rows (Sec. 3.1: the Lloyd step of two-means that labels every member of a
// node by its nearer centre, then moves the centres to the side means).
//
// Labels.  Per row, in FP64, dot = x . w with w = c0 - c1 and h = (|c0|^2 -
// |c1|^2) / 2; the row goes right (label 1) iff dot < h, i.e. iff |x - c1|^2 <
// |x - c0|^2, so an equidistant point stays left.  G lanes share a row, lane
// l holding NF vectors of VEC consecutive elements (element (l + G j) VEC +
// v), each lane a sequential fused chain, then a butterfly over the G lanes.
//
// Side sums.  The first pass of a level takes, per chunk of kChunkRows rows,
// the total T of its rows and the side-1 sum S1 (FP64) and stores both in
// P[chunk] (side 0 is T - S1, also in the centre update kernels).  Later
// passes list the rows whose label changed, in increasing position, and add
// +x (0 -> 1) or -x (1 -> 0) to the chunk's S1 (chunk_delta).  The order of
// every addition depends only on which rows changed, so two kernels that
// label the same rows the same way produce the same bits.
//
// The filtered later pass (k_assign_rf) first takes the margin from the
// reduced copy of the rows (the leaf search's copy: x~ = rnd(sigma x) in FP8,
// FP16 or BF16, sigma a power of two, 1/sigma stored in the row) with a bound
// B on its error against the FP64 code: where |margin| > B the label is the
// FP64 code's, provably, and the row's FP32 values are not read; rows inside
// the band run the FP64 code itself.  It then lists the changed rows exactly
// as the unfiltered pass does, so labels and centres are bit-identical with
// or without the filter; only fewer bytes are read.
//
// Bound of the filter.  Rounding to the format moves sigma x_i by at most
// half the format's spacing at x~_i, which is at most 2^-p P_i + a, with P_i
// = 2^floor(log2 |x~_i|) (0 for 0), p = 4 (FP8-e4m3), 11 (FP16) or 8 (BF16),
// and a the half subnormal spacing (2^-10, 2^-25, 2^-134).  The filter takes
// dt = sum x~_i w32_i and pp = sum P_i |w32_i| in FP32 (w32 = w rounded to
// FP32; any order, gam = (D + 8) 2^-24 relative per sum), and with |x~_i| <
// 2 P_i,
//     |dt - sigma x.w| <= (2^-p + 2 gam + 2^-22)(1 + 2 gam) pp + a |w|_1,
// so B = 1/sigma times that, plus 2^-40 (2 pp / sigma + |h|) for the FP64
// code's own error (far smaller) and a tiny absolute term for FP32
// underflow.  The rounding term 2^-p pp + a |w|_1 is the worst case over the
// row; the copy also stores e >= |sigma x - x~|_2 (computed exactly and
// rounded up), and by Cauchy-Schwarz the same sum is at most e |w32|_2, so
//     |dt - sigma x.w| <= e |w32|_2 + (2 gam + 2^-22)(1 + 2 gam) pp + a |w|_1
// holds too (the terms for the FP32 sum and for w32 are those above); for an
// FP8 copy the filter takes the smaller of the two (for FP16 and BF16 the
// first is already tight and the second's arithmetic costs more than it
// saves).  A non-finite dt, pp or e never decides a row through the bound it
// enters.
#include "knng_internal.hpp"
#include "partition_dev.hpp"
#include "wave.hpp"

namespace knng {
namespace {

// DPP permute of an FP32 value within each 16-lane row (CTRL: a row mirror
// 0x140, half-row mirror 0x141 or a quad permute); every lane active.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
using namespace pdev;

// reduced-copy formats (the leaf search's: 1 BF16, 2 FP16, 3 FP8-e4m3)
constexpr int kRfBF16 = 1, kRfF16 = 2, kRfFP8 = 3;

__device__ __forceinline__ void load_vec(const float* row, int e, int D, bool ok, float (&x)[4]) {
    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ok && e < D) q = *reinterpret_cast<const float4*>(row + e);
    x[0] = q.x;
    x[1] = q.y;
    x[2] = q.z;
    x[3] = q.w;
}

// Shared prologue: w (this lane's elements), h in the lane layout and order.
template <int G, int NF>
__device__ __forceinline__ double centres_wh(const double* cn, int D, int l, double (&w)[NF][4]) {
    double q0 = 0.0, q1 = 0.0;
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int e = (l + G * j) * 4 + v;
            const double c0 = e < D ? cn[e] : 0.0;
            const double c1 = e < D ? cn[D + e] : 0.0;
            w[j][v] = c0 - c1;
            q0 = fma(c0, c0, q0);
            q1 = fma(c1, c1, q1);
        }
    q0 = group_sum_f64<G>(q0);
    q1 = group_sum_f64<G>(q1);
    return 0.5 * (q0 - q1);
}

// The FP64 margin dot of one row: the lane's fused chain, then the group's
// sum (group_sum_f64: DPP within 16-lane rows, the same bits in every lane;
// every kernel that compares margins takes them from here).
template <int G, int NF>
__device__ __forceinline__ double row_dot(const float (&x)[NF][4], const double (&w)[NF][4]) {
    double dot = 0.0;
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) dot = fma(static_cast<double>(x[j][v]), w[j][v], dot);
    return group_sum_f64<G>(dot);
}

// Per-wave LDS of the later passes: one flag byte per row of the chunk (bit 0
// label changed, bit 1 in the filter's band, bit 2 new label, bit 3 previous
// label) and a list of row positions.
struct LaterLds {
    uint8_t flag[4][kChunkRows];
    uint16_t list[4][kChunkRows];
};

// Rows of the chunk with flag bit `bit`, in increasing position, into list
// (bit 15 of an entry: the row's new label); returns their number.
__device__ __forceinline__ int list_rows(const uint8_t* flag, int nrows, int bit, uint16_t* list) {
    const int lane = threadIdx.x & 63;
    int cntl = 0;
    for (int i0 = 0; i0 < nrows; i0 += kWave) {
        const int i = i0 + lane;
        const uint8_t f = i < nrows ? flag[i] : 0;
        const bool in = (f >> bit) & 1;
        const unsigned long long b = __ballot(in);
        if (in)
            list[cntl + __popcll(b & ((1ull << lane) - 1ull))] =
                static_cast<uint16_t>(i | (((f >> 2) & 1) << 15));
        cntl += __popcll(b);
    }
    wave_lds_sync();
    return cntl;
}

// The changed rows' contribution to the side-1 sum: +x for 0 -> 1, -x for
// 1 -> 0.  Row group g adds list entries g, g + RPW, ... in order (U in
// flight), then the groups are combined by a fixed butterfly; every lane of
// group g ends with the sum of its elements.
template <int G, int NF, int U>
__device__ __forceinline__ void chunk_delta(const float* __restrict__ X, int D,
                                            const int32_t* __restrict__ ids, const uint16_t* list,
                                            int cntl, int g, int l, double (&acc)[NF][4]) {
    constexpr int RPW = kWave / G;
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[j][v] = 0.0;
    for (int k0 = 0; k0 < cntl; k0 += RPW * U) {
        float x[U][NF][4];
        double sg[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * RPW + g;
            const bool ok = k < cntl;
            const uint16_t e = ok ? list[k] : 0;
            sg[u] = ok ? ((e >> 15) ? 1.0 : -1.0) : 0.0;
            const float* xr = X + static_cast<size_t>(ids[e & 0x7fff]) * D;
#pragma unroll
            for (int j = 0; j < NF; ++j) load_vec(xr, (l + G * j) * 4, D, ok, x[u][j]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (sg[u] != 0.0)
#pragma unroll
                for (int j = 0; j < NF; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[j][v] += sg[u] * static_cast<double>(x[u][j][v]);
    }
#pragma unroll
    for (int o = G; o < kWave; o <<= 1)
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[j][v] += shfl_xor_f64(acc[j][v], o);
}

// Shared end of the later passes: side-1 sum S1 = previous S1 + delta, the
// counts, and for a node held by this one chunk the stop rule and the new
// centres c1 = S1 / n1, c0 = (T - S1) / n0.
template <int G, int NF>
__device__ __forceinline__ void later_epilogue(const NodeRec& r, int node, int wave, int D, int g,
                                               int l, int lane, int n1, int changed, int nrows,
                                               const double (&acc)[NF][4], double* __restrict__ C,
                                               int32_t* __restrict__ status,
                                               int32_t* __restrict__ n0f, double* __restrict__ P,
                                               int32_t* __restrict__ cnt, int pass, int max_iter,
                                               unsigned long long* __restrict__ assigned,
                                               int32_t* __restrict__ rep, int min_leaf) {
    double* p0 = P + static_cast<size_t>(wave) * 2 * D;
    if (lane == 0) {
        cnt[2 * wave] = n1;
        cnt[2 * wave + 1] = changed;
        stat_add(assigned, static_cast<unsigned>(wave), static_cast<unsigned long long>(nrows));
    }
    const int nch = chunks_of(r.size);
    if (nch == 1) {
        const int n0 = r.size - n1;
        const bool stop = n1 == 0 || n0 == 0 || changed == 0 || pass + 1 >= max_iter;
        if (stop) {
            if (lane == 0) {
                status[node] = 1;
                n0f[node] = n0;
                if (n0 < min_leaf || n1 < min_leaf) rep[1 + atomicAdd(rep, 1)] = node;
            }
            return;
        }
        if (g == 0) {
            double* cn = C + static_cast<size_t>(node) * 2 * D;
            const double dn0 = static_cast<double>(n0), dn1 = static_cast<double>(n1);
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int e = (l + G * j) * 4 + v;
                    if (e < D) {
                        const double s1 = p0[D + e] + acc[j][v];
                        p0[D + e] = s1;
                        cn[e] = (p0[e] - s1) / dn0;
                        cn[D + e] = s1 / dn1;
                    }
                }
        }
        return;
    }
    if (g == 0) {
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int e = (l + G * j) * 4 + v;
                if (e < D) p0[D + e] = p0[D + e] + acc[j][v];
            }
    }
}

// ---------------------------------------------------------------- first pass
// Every row is labelled by the FP64 code; the chunk's total and side-1 sums
// go to P (and, for a node of one chunk, the new centres c0 = (sum of side
// 0) / n0, c1 = S1 / n1).  Rows of step s+1 are loaded while step s is
// computed.
template <int G, int NF, int U>
__global__ __launch_bounds__(256) void k_assign_f32_first(
    const float* __restrict__ X, int64_t n, int D, const int32_t* __restrict__ perm,
    const NodeRec* __restrict__ nodes, const int32_t* __restrict__ chunk_node, int nc,
    double* __restrict__ C, int32_t* __restrict__ status, int32_t* __restrict__ n0f,
    uint8_t* __restrict__ labels, double* __restrict__ /*dots*/, double* __restrict__ P,
    int32_t* __restrict__ cnt, int pass, int max_iter, unsigned long long* __restrict__ assigned,
    int32_t* __restrict__ rep, int min_leaf, const int32_t* __restrict__ order, int xcd_per) {
    constexpr int RPW = kWave / G;
    const int wave = dispatch_chunk(order, xcd_per, blockIdx.x, threadIdx.x >> 6, 4, nc);
    if (wave < 0) return;
    const int node = chunk_node[wave];
    if (status[node]) return;
    const NodeRec r = nodes[node];
    const int lane = threadIdx.x & 63;
    const int g = lane / G, l = lane % G;
    const int row0 = (wave - r.chunk0) * kChunkRows;
    const int row1 = min(r.size, row0 + kChunkRows);
    const size_t base = static_cast<size_t>(r.tree) * n + r.start;
    double w[NF][4];
    const double h = centres_wh<G, NF>(C + static_cast<size_t>(node) * 2 * D, D, l, w);
    double a0[NF][4], a1[NF][4];
#pragma unroll
    for (int j = 0; j < NF; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            a0[j][v] = 0.0;
            a1[j][v] = 0.0;
        }
    int n1 = 0;
    const int steps = (row1 - row0 + RPW * U - 1) / (RPW * U);
    auto row_id = [&](int st, int u) -> int {
        const int row = row0 + (st * U + u) * RPW + g;
        return row < row1 ? perm[base + row] : -1;
    };
    auto load_rows = [&](const int (&id)[U], float (&x)[U][NF][4]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float* xr = X + static_cast<size_t>(id[u] < 0 ? 0 : id[u]) * D;
#pragma unroll
            for (int j = 0; j < NF; ++j) load_vec(xr, (l + G * j) * 4, D, id[u] >= 0, x[u][j]);
        }
    };
    int idc[U], idn[U];
    float xc[U][NF][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        idc[u] = row_id(0, u);
        idn[u] = row_id(1, u);
    }
    load_rows(idc, xc);
    for (int st = 0; st < steps; ++st) {
        float xn[U][NF][4];
        load_rows(idn, xn);
        int idnn[U];
#pragma unroll
        for (int u = 0; u < U; ++u) idnn[u] = row_id(st + 2, u);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int row = row0 + (st * U + u) * RPW + g;
            const double dot = row_dot<G, NF>(xc[u], w);
            const bool lab = dot < h;
            if (idc[u] >= 0) {
                if (l == 0) {
                    labels[base + row] = lab ? 1 : 0;
                    n1 += lab ? 1 : 0;
                }
#pragma unroll
                for (int j = 0; j < NF; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double xv = static_cast<double>(xc[u][j][v]);
                        a0[j][v] += lab ? 0.0 : xv;
                        a1[j][v] += lab ? xv : 0.0;
                    }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            idc[u] = idn[u];
            idn[u] = idnn[u];
#pragma unroll
            for (int j = 0; j < NF; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) xc[u][j][v] = xn[u][j][v];
        }
    }
#pragma unroll
    for (int o = G; o < kWave; o <<= 1)
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                a0[j][v] += shfl_xor_f64(a0[j][v], o);
                a1[j][v] += shfl_xor_f64(a1[j][v], o);
            }
    n1 = wave_sum_i32(n1);
    if (lane == 0) {
        cnt[2 * wave] = n1;
        cnt[2 * wave + 1] = 0;
        stat_add(assigned, static_cast<unsigned>(wave), static_cast<unsigned long long>(row1 - row0));
    }
    const int nch = chunks_of(r.size);
    double* p0 = P + static_cast<size_t>(wave) * 2 * D;
    if (nch == 1) {
        const int n0 = r.size - n1;
        if (n1 == 0 || n0 == 0 || pass + 1 >= max_iter) {
            if (lane == 0) {
                status[node] = 1;
                n0f[node] = n0;
                if (n0 < min_leaf || n1 < min_leaf) rep[1 + atomicAdd(rep, 1)] = node;
            }
            return;
        }
    }
    if (g == 0) {
        double* cn = C + static_cast<size_t>(node) * 2 * D;
        const double dn0 = static_cast<double>(r.size - n1), dn1 = static_cast<double>(n1);
#pragma unroll
        for (int j = 0; j < NF; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int e = (l + G * j) * 4 + v;
                if (e < D) {
                    p0[e] = a0[j][v] + a1[j][v];
                    p0[D + e] = a1[j][v];
                    if (nch == 1) {
                        cn[e] = a0[j][v] / dn0;
                        cn[D + e] = a1[j][v] / dn1;
                    }
                }
            }
    }
}

// ---------------------------------------------------------------- later passes
// Every row labelled by the FP64 code (the previous label is read with the
// row); changed rows are flagged and added by chunk_delta.
template <int G, int NF, int U>
__global__ __launch_bounds__(256) void k_assign_f32_later(
    const float* __restrict__ X, int64_t n, int D, const int32_t* __restrict__ perm,
    const NodeRec* __restrict__ nodes, const int32_t* __restrict__ chunk_node, int nc,
    double* __restrict__ C, int32_t* __restrict__ status, int32_t* __restrict__ n0f,
    uint8_t* __restrict__ labels, double* __restrict__ /*dots*/, double* __restrict__ P,
    int32_t* __restrict__ cnt, int pass, int max_iter, unsigned long long* __restrict__ assigned,
    int32_t* __restrict__ rep, int min_leaf, const int32_t* __restrict__ order, int xcd_per) {
    constexpr int RPW = kWave / G;
    __shared__ LaterLds lds;
    const int wl = threadIdx.x >> 6;
    const int wave = dispatch_chunk(order, xcd_per, blockIdx.x, wl, 4, nc);
    if (wave < 0) return;
    const int node = chunk_node[wave];
    if (status[node]) return;
    const NodeRec r = nodes[node];
    const int lane = threadIdx.x & 63;
    const int g = lane / G, l = lane % G;
    const int row0 = (wave - r.chunk0) * kChunkRows;
    const int nrows = min(r.size - row0, kChunkRows);
    const size_t base = static_cast<size_t>(r.tree) * n + r.start + row0;
    uint8_t* flag = lds.flag[wl];
    double w[NF][4];
    const double h = centres_wh<G, NF>(C + static_cast<size_t>(node) * 2 * D, D, l, w);
    int n1 = 0;
    const int steps = (nrows + RPW * U - 1) / (RPW * U);
    auto row_id = [&](int st, int u) -> int {
        const int i = (st * U + u) * RPW + g;
        return i < nrows ? perm[base + i] : -1;
    };
    auto old_label = [&](int st, int u) -> int {
        const int i = (st * U + u) * RPW + g;
        return (i < nrows && l == 0) ? static_cast<int>(labels[base + i]) : 0;
    };
    auto load_rows = [&](const int (&id)[U], float (&x)[U][NF][4]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float* xr = X + static_cast<size_t>(id[u] < 0 ? 0 : id[u]) * D;
#pragma unroll
            for (int j = 0; j < NF; ++j) load_vec(xr, (l + G * j) * 4, D, id[u] >= 0, x[u][j]);
        }
    };
    int idc[U], idn[U], oc[U];
    float xc[U][NF][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        idc[u] = row_id(0, u);
        idn[u] = row_id(1, u);
        oc[u] = old_label(0, u);
    }
    load_rows(idc, xc);
    for (int st = 0; st < steps; ++st) {
        float xn[U][NF][4];
        int on[U], idnn[U];
        load_rows(idn, xn);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            on[u] = old_label(st + 1, u);
            idnn[u] = row_id(st + 2, u);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = (st * U + u) * RPW + g;
            const double dot = row_dot<G, NF>(xc[u], w);
            const int lab = dot < h ? 1 : 0;
            if (idc[u] >= 0 && l == 0) {
                labels[base + i] = static_cast<uint8_t>(lab);
                n1 += lab;
                flag[i] = static_cast<uint8_t>((lab != oc[u] ? 1 : 0) | (lab << 2));
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
                for (int v = 0; v < 4; ++v) xc[u][j][v] = xn[u][j][v];
        }
    }
    wave_lds_sync();
    uint16_t* list = lds.list[wl];
    const int changed = list_rows(flag, nrows, 0, list);
    // row ids of the listed rows are read through perm
    double acc[NF][4];
    chunk_delta<G, NF, 4>(X, D, perm + base, list, changed, g, l, acc);
    n1 = wave_sum_i32(n1);
    later_epilogue<G, NF>(r, node, wave, D, g, l, lane, n1, changed, nrows, acc, C, status, n0f, P,
                          cnt, pass, max_iter, assigned, rep, min_leaf);
}

// ---------------------------------------------------------------- filtered
// Later pass with the reduced copy as a filter (see the file comment).  Phase
// A: every row's filter margin, in a lane layout of its own (GF lanes per
// row, 16 bytes of the reduced row per lane and vector); decided rows get
// their label, rows inside the band are flagged.  Phase B: the band rows by
// the FP64 code, in its lane layout.  Phase C: the changed rows' delta, as
// in k_assign_f32_later.  The chunk's row ids stay in LDS from phase A on.
template <int CPB>
struct RfLds {
    uint8_t flag[CPB][kChunkRows];
    uint16_t list[CPB][kChunkRows];
    int32_t ids[CPB][kChunkRows];
    int n1[CPB][4];
};

// The 16 bytes of one lane vector as FP32 values (exact: every FP8, FP16 and
// BF16 value is an FP32 value).
template <int FMT>
__device__ __forceinline__ void unpack16(const uint4& q, float (&v)[FMT == kRfFP8 ? 16 : 8]) {
    const uint32_t wd[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if constexpr (FMT == kRfFP8) {
            v[4 * c + 0] = __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(wd[c]), 0);
            v[4 * c + 1] = __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(wd[c]), 1);
            v[4 * c + 2] = __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(wd[c]), 2);
            v[4 * c + 3] = __builtin_amdgcn_cvt_f32_fp8(static_cast<int>(wd[c]), 3);
        } else if constexpr (FMT == kRfF16) {
            v[2 * c] = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(wd[c] & 0xffffu)));
            v[2 * c + 1] = static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(wd[c] >> 16)));
        } else {
            v[2 * c] = __uint_as_float(wd[c] << 16);
            v[2 * c + 1] = __uint_as_float(wd[c] & 0xffff0000u);
        }
    }
}

// 2^floor(log2 |v|) for a normal FP32 v (0 for 0 and for FP32 subnormals,
// infinity for infinities and NaNs).
__device__ __forceinline__ float pow2_floor(float v) {
    return __uint_as_float(__float_as_uint(v) & 0x7f800000u);
}

template <int G, int NF, int U, int FMT, int WPC>
__global__ __launch_bounds__(256) void k_assign_rf(
    const float* __restrict__ X, int64_t n, int D, const int32_t* __restrict__ perm,
    const NodeRec* __restrict__ nodes, const int32_t* __restrict__ chunk_node, int nc,
    double* __restrict__ C, int32_t* __restrict__ status, int32_t* __restrict__ n0f,
    uint8_t* __restrict__ labels, double* __restrict__ P, int32_t* __restrict__ cnt, int pass,
    int max_iter, unsigned long long* __restrict__ assigned, int32_t* __restrict__ rep,
    int min_leaf, const int32_t* __restrict__ order, int xcd_per,
    const uint8_t* __restrict__ Xr, int soff, int rsb, unsigned long long* __restrict__ filt) {
    constexpr int RPW = kWave / G;
    // WPC wavefronts per chunk (1, or 4 for wide rows: a chunk of 1024 rows
    // of a few KB each is too much work for one wavefront when the level has
    // few chunks); wavefront `part` filters rows [part RPC, (part+1) RPC)
    constexpr int CPB = 4 / WPC, RPC = kChunkRows / WPC;
    // filter layout: the widest row of this FP64 layout (4 G NF elements) in
    // 16-byte vectors over at most 64 lanes
    constexpr int EB = FMT == kRfFP8 ? 1 : 2;
    constexpr int EV = 16 / EB;
    constexpr int VRM = G * NF * EB / 4 > 0 ? G * NF * EB / 4 : 1;
    constexpr int GF = VRM < kWave ? VRM : kWave;
    constexpr int NFF = VRM / GF;
    constexpr int UF = NFF >= 2 ? 1 : 2;
    constexpr int RPWF = kWave / GF;
    // loads run PF steps ahead of the arithmetic (ring of PF + 1 buffers)
    constexpr int PF = 3, NB = PF + 1;
    constexpr int UB = 1, PB = NF >= 4 ? 1 : 3, NBB = PB + 1;
    // half-spacing of the format at x~ <= 2^-p 2^floor(log2|x~|) + a
    constexpr double kP = FMT == kRfFP8 ? 0x1p-4 : FMT == kRfF16 ? 0x1p-11 : 0x1p-8;
    constexpr double kSub = FMT == kRfFP8 ? 0x1p-10 : FMT == kRfF16 ? 0x1p-25 : 0x1p-134;
    __shared__ RfLds<CPB> lds;
    const int wl = threadIdx.x >> 6;
    const int slot = wl / WPC, part = wl % WPC;
    // (with WPC > 1 every wavefront of the workgroup takes the same chunk, so
    // the returns below are uniform over the workgroup)
    const int wave = dispatch_chunk(order, xcd_per, blockIdx.x, slot, CPB, nc);
    if (wave < 0) return;
    const int node = chunk_node[wave];
    if (status[node]) return;
    const NodeRec r = nodes[node];
    const int lane = threadIdx.x & 63;
    const int g = lane / G, l = lane % G;
    const int gf = lane / GF, lf = lane % GF;
    const int row0 = (wave - r.chunk0) * kChunkRows;
    const int nrows = min(r.size - row0, kChunkRows);
    const size_t cbase = static_cast<size_t>(r.tree) * n + r.start + row0;
    uint8_t* cflag = lds.flag[slot];
    int32_t* crid = lds.ids[slot];
    // this wavefront's part of the chunk
    const int p0 = part * RPC;
    const int np = max(0, min(nrows - p0, RPC));
    const size_t base = cbase + p0;
    uint8_t* flag = cflag + p0;
    int32_t* rid = crid + p0;

    // the part's row ids and previous labels (bit 3 of the flag), coalesced
    {
        int32_t idv[RPC / kWave];
        uint8_t lbv[RPC / kWave];
#pragma unroll
        for (int k = 0; k < RPC / kWave; ++k) {
            const int i = k * kWave + lane;
            idv[k] = i < np ? perm[base + i] : 0;
            lbv[k] = i < np ? labels[base + i] : 0;
        }
#pragma unroll
        for (int k = 0; k < RPC / kWave; ++k) {
            const int i = k * kWave + lane;
            if (i < np) {
                rid[i] = idv[k];
                flag[i] = static_cast<uint8_t>(lbv[k] << 3);
            }
        }
    }

    const double* cn = C + static_cast<size_t>(node) * 2 * D;
    // w in FP32 in the filter layout, |w|_1 in FP64, and h (in the FP64
    // code's layout and order; its w is taken again after phase A)
    float wf[NFF][EV];
    double w1 = 0.0, w2 = 0.0;  // |w|_1; then |w32|_2 (squares exact in FP64)
#pragma unroll
    for (int j = 0; j < NFF; ++j)
#pragma unroll
        for (int t = 0; t < EV; ++t) {
            const int e = (lf + GF * j) * EV + t;
            const double we = e < D ? cn[e] - cn[D + e] : 0.0;
            wf[j][t] = static_cast<float>(we);
            w1 += fabs(we);
            if constexpr (FMT == kRfFP8) w2 += static_cast<double>(wf[j][t]) * static_cast<double>(wf[j][t]);
        }
#pragma unroll
    for (int o = GF / 2; o >= 1; o >>= 1) {
        w1 += shfl_xor_f64(w1, o);
        if constexpr (FMT == kRfFP8) w2 += shfl_xor_f64(w2, o);
    }
    // |w32|_2 rounded up, with the slack for the FP64 product e |w32|_2 / sigma
    w2 = sqrt(w2 * (1.0 + 0x1p-40)) * (1.0 + 0x1p-30);
    double h;
    {
        double w[NF][4];
        h = centres_wh<G, NF>(cn, D, l, w);
    }
    const double gam = (D + 8) * 0x1p-24;
    const double relb = (kP + 2.0 * gam + 0x1p-22) * (1.0 + 2.0 * gam);
    const double rel2 = (2.0 * gam + 0x1p-22) * (1.0 + 2.0 * gam);
    const double subw = kSub * w1 * (1.0 + 0x1p-40) + 0x1p-100;
    const double hab = fabs(h);
    wave_lds_sync();

    // ---- phase A: the filter
    int nfilt = 0, nfchg = 0;
    const int steps = (np + RPWF * UF - 1) / (RPWF * UF);
    auto issue = [&](int st, uint4 (&x)[UF][NFF], float (&si)[UF], float (&ei)[UF]) {
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            const int i = (st * UF + u) * RPWF + gf;
            const bool ok = i < np;
            const uint8_t* xr = Xr + static_cast<size_t>(ok ? rid[i] : 0) * rsb;
#pragma unroll
            for (int j = 0; j < NFF; ++j) {
                const int v = lf + GF * j;
                x[u][j] = (ok && v * EV < D) ? *reinterpret_cast<const uint4*>(xr + 16 * v)
                                             : make_uint4(0u, 0u, 0u, 0u);
            }
            if constexpr (FMT == kRfFP8) {
                // 1/sigma and e in one load (soff = Dp bytes, a multiple of 32)
                const float2 se = ok ? *reinterpret_cast<const float2*>(xr + soff) : make_float2(0.f, 0.f);
                si[u] = se.x;
                ei[u] = se.y;
            } else {
                si[u] = ok ? *reinterpret_cast<const float*>(xr + soff) : 0.f;
                ei[u] = 0.f;
            }
        }
    };
    auto decide = [&](int st, const uint4 (&x)[UF][NFF], const float (&si)[UF],
                      const float (&ei)[UF]) {
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            const int i = (st * UF + u) * RPWF + gf;
            float dt = 0.f, pp = 0.f;
#pragma unroll
            for (int j = 0; j < NFF; ++j) {
                float v[EV];
                unpack16<FMT>(x[u][j], v);
#pragma unroll
                for (int t = 0; t < EV; ++t) {
                    dt = __fmaf_rn(v[t], wf[j][t], dt);
                    pp = __fmaf_rn(pow2_floor(v[t]), fabsf(wf[j][t]), pp);
                }
            }
            // sums over the GF-lane group (every lane active): quad permutes
            // and the half-row and row mirrors by DPP, then lane xor 16 and
            // xor 32 through ds_bpermute for wider groups; each lane ends
            // with the group's sum, in an order the bound's gam covers like
            // any other
            if constexpr (GF >= 2) {
                dt += dpp_f32<0xB1>(dt);
                pp += dpp_f32<0xB1>(pp);
            }
            if constexpr (GF >= 4) {
                dt += dpp_f32<0x4E>(dt);
                pp += dpp_f32<0x4E>(pp);
            }
            if constexpr (GF >= 8) {
                dt += dpp_f32<0x141>(dt);
                pp += dpp_f32<0x141>(pp);
            }
            if constexpr (GF >= 16) {
                dt += dpp_f32<0x140>(dt);
                pp += dpp_f32<0x140>(pp);
            }
            if constexpr (GF >= 32) {
                dt += __shfl_xor(dt, 16, kWave);
                pp += __shfl_xor(pp, 16, kWave);
            }
            if constexpr (GF >= 64) {
                dt += __shfl_xor(dt, 32, kWave);
                pp += __shfl_xor(pp, 32, kWave);
            }
            // sigma-scaled error bound relb pp (FP8: the smaller of that and
            // e |w32|_2 + rel2 pp) + a |w|_1, in row units (times 1/sigma),
            // and the FP64 code's own error; a non-finite dt or pp leaves the
            // row in the band, a non-finite e keeps the first bound
            const double s = static_cast<double>(si[u]);
            const double m = static_cast<double>(dt) * s - h;
            const double pb = static_cast<double>(pp) * s;
            double eb = relb * pb;
            if constexpr (FMT == kRfFP8) {
                const double b2 = static_cast<double>(ei[u]) * s * w2 + rel2 * pb;
                eb = b2 < eb ? b2 : eb;
            }
            const double bnd = eb + subw * s + 0x1p-40 * (2.0 * pb + hab);
            if (i < np && lf == 0) {
                const int old = flag[i] >> 3;
                if (m < -bnd || m > bnd) {
                    const int lab = m < -bnd ? 1 : 0;
                    ++nfilt;
                    nfchg += lab != old ? 1 : 0;
                    flag[i] = static_cast<uint8_t>((lab != old ? 1 : 0) | (lab << 2));
                } else {
                    flag[i] = static_cast<uint8_t>(2 | (old << 3));  // band
                }
            }
        }
    };
    {
        uint4 xb[NB][UF][NFF];
        float sb[NB][UF], eb[NB][UF];
#pragma unroll
        for (int b = 0; b < PF; ++b) issue(b, xb[b], sb[b], eb[b]);
        for (int st0 = 0; st0 < steps; st0 += NB) {
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                issue(st0 + k + PF, xb[(k + PF) % NB], sb[(k + PF) % NB], eb[(k + PF) % NB]);
                decide(st0 + k, xb[k], sb[k], eb[k]);
            }
        }
    }
    wave_lds_sync();

    // ---- phase B: band rows by the FP64 code (group g takes entries g,
    // g + RPW, ...), loads PB steps ahead
    double w[NF][4];
    centres_wh<G, NF>(cn, D, l, w);
    uint16_t* list = lds.list[slot] + p0;
    const int nband = list_rows(flag, np, 1, list);
    const int bsteps = (nband + RPW * UB - 1) / (RPW * UB);
    auto issue_b = [&](int st, float (&x)[UB][NF][4], int (&pos)[UB]) {
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int k = (st * UB + u) * RPW + g;
            pos[u] = k < nband ? static_cast<int>(list[k] & 0x7fff) : -1;
            const float* xr = X + static_cast<size_t>(rid[pos[u] < 0 ? 0 : pos[u]]) * D;
#pragma unroll
            for (int j = 0; j < NF; ++j) load_vec(xr, (l + G * j) * 4, D, pos[u] >= 0, x[u][j]);
        }
    };
    auto label_b = [&](const float (&x)[UB][NF][4], const int (&pos)[UB]) {
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const double dot = row_dot<G, NF>(x[u], w);
            const int lab = dot < h ? 1 : 0;
            if (pos[u] >= 0 && l == 0) {
                const int old = (flag[pos[u]] >> 3) & 1;
                flag[pos[u]] = static_cast<uint8_t>((lab != old ? 1 : 0) | (lab << 2));
            }
        }
    };
    if (bsteps > 0) {
        float xb[NBB][UB][NF][4];
        int pb[NBB][UB];
#pragma unroll
        for (int b = 0; b < PB; ++b) issue_b(b, xb[b], pb[b]);
        for (int st0 = 0; st0 < bsteps; st0 += NBB) {
#pragma unroll
            for (int k = 0; k < NBB; ++k) {
                issue_b(st0 + k + PB, xb[(k + PB) % NBB], pb[(k + PB) % NBB]);
                label_b(xb[k], pb[k]);
            }
        }
    }
    wave_lds_sync();

    // new labels (bit 2 of the flag) back to memory, coalesced
    int n1 = 0;
#pragma unroll
    for (int k = 0; k < RPC / kWave; ++k) {
        const int i = k * kWave + lane;
        if (i < np) {
            const int lab = (flag[i] >> 2) & 1;
            labels[base + i] = static_cast<uint8_t>(lab);
            n1 += lab;
        }
    }
    n1 = wave_sum_i32(n1);
    nfilt = wave_sum_i32(nfilt);
    nfchg = wave_sum_i32(nfchg);
    if (lane == 0 && filt != nullptr) {  // rows read from the copy; rows read as FP32
        stat_add(filt, static_cast<unsigned>(wave * WPC + part), static_cast<unsigned long long>(np));
        stat_add(filt + kStatWords, static_cast<unsigned>(wave * WPC + part),
                 static_cast<unsigned long long>(np - nfilt + nfchg));
    }
    if constexpr (WPC > 1) {
        // the parts' counts, then the chunk's changed rows by its first wavefront
        if (lane == 0) lds.n1[slot][part] = n1;
        __syncthreads();
        if (part != 0) return;
        n1 = 0;
#pragma unroll
        for (int q = 0; q < WPC; ++q) n1 += lds.n1[slot][q];
    }

    // ---- phase C: the changed rows of the chunk, as in the unfiltered pass
    const int changed = list_rows(cflag, nrows, 0, lds.list[slot]);
    double acc[NF][4];
    chunk_delta<G, NF, NF >= 4 ? 1 : 2>(X, D, crid, lds.list[slot], changed, g, l, acc);
    later_epilogue<G, NF>(r, node, wave, D, g, l, lane, n1, changed, nrows, acc, C, status, n0f, P,
                          cnt, pass, max_iter, assigned, rep, min_leaf);
}

// ---------------------------------------------------------------- repair margins
// FP64 margins of every member of the nodes in the repair list (rep[0]
// count), with the labelling code's lane layout and order, into dots (the
// repair ranks the members by them).  A node of up to 2^20 elements goes to
// one workgroup; every workgroup takes a share of a larger node's rows (a
// repaired node can hold most of a level's rows).
template <int G, int NF>
__global__ __launch_bounds__(256) void k_redots_f32(const NodeRec* __restrict__ nodes,
                                                     const int32_t* __restrict__ rep, int64_t n,
                                                     const float* __restrict__ X, int D,
                                                     const int32_t* __restrict__ perm,
                                                     const double* __restrict__ C,
                                                     const int32_t* __restrict__ n0f, int min_leaf,
                                                     double* __restrict__ dots) {
    constexpr int RPW = kWave / G;
    // a node of more than 2^20 elements (rows x D) is shared by every workgroup
    const int big_rows = (1 << 20) / D;
    const int nrep = rep[0];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = lane / G, l = lane % G;
    // rows p0 + g, p0 + step + g, ... of one listed node
    auto margins = [&](int node, const NodeRec& r, int p_first, int step) {
        const int m = r.size;
        const size_t base = static_cast<size_t>(r.tree) * n + r.start;
        double w[NF][4];
        centres_wh<G, NF>(C + static_cast<size_t>(node) * 2 * D, D, l, w);
        for (int p0 = p_first; p0 < m; p0 += step) {  // uniform per wave
            const int p = p0 + g;
            float x[NF][4];
            const float* xr = X + static_cast<size_t>(p < m ? perm[base + p] : 0) * D;
#pragma unroll
            for (int j = 0; j < NF; ++j) load_vec(xr, (l + G * j) * 4, D, p < m, x[j]);
            const double dot = row_dot<G, NF>(x, w);
            if (p < m && l == 0) dots[base + p] = dot;
        }
    };
    // the repair's own test: a side below min_leaf
    auto repaired = [&](int node, int m) {
        const int n0 = n0f[node];
        return !(n0 >= min_leaf && m - n0 >= min_leaf);
    };
    // smaller nodes: one workgroup each
    for (int ri = blockIdx.x; ri < nrep; ri += gridDim.x) {
        const int node = rep[1 + ri];
        const NodeRec r = nodes[node];
        if (r.size > big_rows || !repaired(node, r.size)) continue;
        margins(node, r, wv * RPW, 4 * RPW);
    }
    // larger nodes: every workgroup takes a share (the list is scanned 64
    // entries at a time, one per lane)
    for (int r0 = 0; r0 < nrep; r0 += kWave) {
        const int ri = r0 + lane;
        int node = -1;
        if (ri < nrep) {
            node = rep[1 + ri];
            const int m = nodes[node].size;
            if (m <= big_rows || !repaired(node, m)) node = -1;
        }
        uint64_t big = __ballot(node >= 0);
        while (big) {
            const int src = __builtin_ctzll(big);
            big &= big - 1;
            const int bn = __shfl(node, src, kWave);
            margins(bn, nodes[bn], (blockIdx.x * 4 + wv) * RPW, gridDim.x * 4 * RPW);
        }
    }
}

// ---------------------------------------------------------------- pickers
template <int G, int NF>
void set_f32(int u, AssignF32Fns* f) {
    f->redots = k_redots_f32<G, NF>;
    // filtered passes: a workgroup per chunk for rows of more than 256
    // elements (the filter phase does not depend on u)
    constexpr int WPC = NF >= 4 ? 4 : 1;
    f->rf_wpc = WPC;
    f->rf[0] = k_assign_rf<G, NF, 1, kRfBF16, WPC>;
    f->rf[1] = k_assign_rf<G, NF, 1, kRfF16, WPC>;
    f->rf[2] = k_assign_rf<G, NF, 1, kRfFP8, WPC>;
    switch (u) {
        case 1:
            f->first = k_assign_f32_first<G, NF, 1>;
            f->later = k_assign_f32_later<G, NF, 1>;
            break;
        default:
            f->first = k_assign_f32_first<G, NF, 2>;
            f->later = k_assign_f32_later<G, NF, 2>;
            break;
    }
}

template <int NF>
void set_groups(int E, int u, AssignF32Fns* f) {
    int G = 1;
    while (G < 32 && G * NF < E) G <<= 1;
    switch (G) {
        case 1: set_f32<1, NF>(u, f); break;
        case 2: set_f32<2, NF>(u, f); break;
        case 4: set_f32<4, NF>(u, f); break;
        case 8: set_f32<8, NF>(u, f); break;
        case 16: set_f32<16, NF>(u, f); break;
        default: set_f32<32, NF>(u, f); break;
    }
}

}  // namespace

// Rows of D % 4 == 0: 8 elements per lane for rows that fit 32 lanes (G the
// smallest power of two with 8 G >= D), else all 64 lanes; u rows per lane
// group and step (1 or 2).
bool pick_assign_f32_fns(int D, int u, AssignF32Fns* f) {
    *f = AssignF32Fns{};
    if (D % 4 != 0) return false;
    const int E = D / 4;
    if (E <= 64) set_groups<2>(E, u, f);
    else if (E <= 64 * 4) set_f32<64, 4>(u, f);
    else if (E <= 64 * 8) set_f32<64, 8>(1, f);
    else if (E <= 64 * 16) set_f32<64, 16>(1, f);
    else return false;
    return true;
}

}  // namespace knng
