// Assignment pass of the level-synchronous two-means bisection (Alg. 2: the
// Lloyd step that labels every row of a node by its nearer centre) for
// uint8 rows, with the margin taken on the matrix cores.
//
// The label of a row is dot < h, dot = x.(c0 - c1) and h = (|c0|^2 -
// |c1|^2) / 2, both in FP64 with the lane layout and summation order of the
// FP64 assignment kernel (k_assign_u8: lane l of a group of G holds elements
// 16 l .. 16 l + 15, a sequential fma chain, then the group sum), so every
// FP64 value here is that kernel's number and every label its label.
//
// Margin on the matrix cores.  Centres of uint8 data lie in [0, 255], so
// w = c0 - c1 has |w| <= 255 and W = rint(2^22 w) fits 31 bits: four balanced
// int8 digit planes.  With x' = x - 128 (int8), v_mfma_i32_16x16x64_i8 gives
// sum_e x'_e W_e exactly, and x.W = sum x'W + 128 sum W.  Since
// |x.W - 2^22 x.w| <= 0.5 sum x <= 127.5 D and the FP64 chain differs from
// the exact x.w by far less than one unit of 2^-22, |x.W - 2^22 h| > 128 D + 2
// decides dot < h as the FP64 code does.  Rows inside that band are
// evaluated by the FP64 code itself (lanes 0 .. G-1 of the wavefront).
//
// Layout.  A chunk of kChunkRows rows is split into tiles of 16 rows, dealt
// round-robin to the four wavefronts of a workgroup (or all taken by one
// wavefront, four chunks per workgroup; slower on MI355X at every level
// size: a quarter of the tiles per wave shortens each wave's serial chain
// and the id, centre and label set-up is shared).  In a tile, lane
// (q, c) = (lane / 16, lane % 16) loads bytes 64 kb + 16 q .. + 15 of row c of
// the tile (the A operand), and the B operand holds the four digit planes in
// columns 0..3.  Output element i of lane (q, c) is digit plane c of row
// 4 q + i; a quad sum weights the planes by 256^c.  Labels are gathered with
// ballots into a 16-bit mask per tile.
//
// Side sums are exact integers.  The first pass of a level adds every row
// (total and side 1) in packed 16-bit halves (two elements per register, no
// carry: at most 64 rows of 255 per lane and chunk); later passes list the
// rows whose label changed (in place, in the LDS id list) and add or remove
// them from the previous pass's side-1 sum after the tile loop.
#include "knng_internal.hpp"
#include "partition_dev.hpp"
#include "wave.hpp"

namespace knng {
namespace {
using namespace pdev;

typedef int i32x4 __attribute__((ext_vector_type(4)));
constexpr double kMarginScale = 4194304.0;  // 2^22

// Ballot bits of lanes 16 q + c (c < 4) -> bits 4 q + c.
__device__ __forceinline__ uint32_t tile_bits(uint64_t b) {
    return static_cast<uint32_t>(b & 0xFull) | static_cast<uint32_t>((b >> 12) & 0xF0ull) |
           static_cast<uint32_t>((b >> 24) & 0xF00ull) |
           static_cast<uint32_t>((b >> 36) & 0xF000ull);
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return static_cast<uint32_t>(
        __builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, 0xf, 0xf, false));
}

// KB 64-element blocks (D <= 64 KB), G lanes per row in the FP64 code, U
// tiles per step, PD steps of loads in flight, WPC wavefronts per chunk (1:
// four chunks per workgroup; 4: one chunk per workgroup).
template <int KB, int G, int U, int PD, bool FIRST, int WPC>
__global__ __launch_bounds__(256) void k_assign_u8m(
    const uint8_t* __restrict__ X, int64_t n, int D, const int32_t* __restrict__ perm,
    const NodeRec* __restrict__ nodes, const int32_t* __restrict__ chunk_node, int nc,
    double* __restrict__ C, int32_t* __restrict__ status, int32_t* __restrict__ n0f,
    uint8_t* __restrict__ labels, double* __restrict__ /*dots: not used for uint8 rows*/,
    double* __restrict__ P, int32_t* __restrict__ cnt, int pass, int max_iter,
    unsigned long long* __restrict__ assigned, int32_t* __restrict__ rep, int min_leaf,
    const int32_t* __restrict__ order, int xcd_per) {
    static_assert(WPC == 1 || WPC == 4, "one or four wavefronts per chunk");
    constexpr int DM = KB * 64;
    constexpr int CPB = 4 / WPC;                  // chunks per workgroup
    constexpr int kFill = kChunkRows / (kWave * WPC);
    constexpr int kList = WPC == 1 ? 1 : kChunkRows / WPC;  // changed-row list per wave
    static_assert(16 * G <= DM, "FP64 lane layout exceeds the row block");
    __shared__ int32_t s_ids[CPB][kChunkRows];
    __shared__ uint8_t s_old[CPB][kChunkRows];
    __shared__ __align__(16) int8_t s_dig[4][4][DM];
    __shared__ double s_w[4][DM];
    __shared__ int32_t s_lid[WPC == 1 ? 1 : 4][kList];
    __shared__ uint8_t s_lsg[WPC == 1 ? 1 : 4][kList];
    __shared__ int32_t s_red[WPC == 1 ? 1 : 4][2 * kWave + 2];

    const int lane = threadIdx.x & 63, wl = threadIdx.x >> 6;
    const int wc = wl % WPC, cs = wl / WPC;  // wave within its chunk, chunk slot
    const int wave = dispatch_chunk(order, xcd_per, blockIdx.x, cs, CPB, nc);  // chunk index
    if (wave < 0) return;
    const int node = chunk_node[wave];
    if (status[node]) return;  // the same for every wave of the chunk
    const NodeRec r = nodes[node];
    const int tc = lane & 15, tq = lane >> 4;
    const int l = lane % G;
    const int nch = chunks_of(r.size);
    const int row0 = (wave - r.chunk0) * kChunkRows;
    const int nrows = min(r.size - row0, kChunkRows);
    const size_t base = static_cast<size_t>(r.tree) * n + r.start + row0;
    int32_t* ids = s_ids[cs];
    uint8_t* olds = s_old[cs];
    double* sw = s_w[wl];
    const int ctid = wc * kWave + lane;  // thread index within the chunk's waves

    // row ids and previous labels of the chunk: loads issued now, stored to
    // LDS after the centres are done with the same LDS space
    int32_t pid[kFill];
    uint8_t pl[kFill];
#pragma unroll
    for (int q = 0; q < kFill; ++q) {
        const int i = min(q * kWave * WPC + ctid, nrows - 1);
        pid[q] = perm[base + i];
        pl[q] = FIRST ? 0 : labels[base + i];
    }

    double* cn = C + static_cast<size_t>(node) * 2 * D;
    double* p0 = P + static_cast<size_t>(wave) * 2 * D;
    // centres, [2][DM], in the id space before the ids (every wave of the
    // chunk writes the same values)
    double* scn = reinterpret_cast<double*>(ids);
#pragma unroll
    for (int e0 = 0; e0 < DM; e0 += kWave) {
        const int e = e0 + lane;
        const double c0 = e < D ? cn[e] : 0.0;
        const double c1 = e < D ? cn[D + e] : 0.0;
        scn[e] = c0;
        scn[DM + e] = c1;
        sw[e] = c0 - c1;
    }
    wave_lds_sync();
    // h in the FP64 code's layout and order
    double h;
    {
        double q0 = 0.0, q1 = 0.0;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const double c0 = scn[16 * l + v];
            const double c1 = scn[DM + 16 * l + v];
            q0 = fma(c0, c0, q0);
            q1 = fma(c1, c1, q1);
        }
        q0 = group_sum_f64<G>(q0);
        q1 = group_sum_f64<G>(q1);
        h = 0.5 * (q0 - q1);
    }
    // W = rint(2^22 w) as four balanced int8 digit planes; sum W exact in FP64
    double wsum = 0.0;
#pragma unroll
    for (int e0 = 0; e0 < DM; e0 += kWave) {
        const int e = e0 + lane;
        int d0 = 0, d1 = 0, d2 = 0, d3 = 0;
        if (e < D) {
            int W = static_cast<int>(rint(sw[e] * kMarginScale));
            wsum += static_cast<double>(W);
            d0 = ((W + 128) & 255) - 128;
            W = (W - d0) >> 8;
            d1 = ((W + 128) & 255) - 128;
            W = (W - d1) >> 8;
            d2 = ((W + 128) & 255) - 128;
            d3 = (W - d2) >> 8;
        }
        s_dig[wl][0][e] = static_cast<int8_t>(d0);
        s_dig[wl][1][e] = static_cast<int8_t>(d1);
        s_dig[wl][2][e] = static_cast<int8_t>(d2);
        s_dig[wl][3][e] = static_cast<int8_t>(d3);
    }
    wsum = group_sum_f64<64>(wsum);
    wave_lds_sync();
    i32x4 bop[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        bop[kb] = i32x4{0, 0, 0, 0};
        if (tc < 4) bop[kb] = *reinterpret_cast<const i32x4*>(&s_dig[wl][tc][kb * 64 + 16 * tq]);
    }
    if constexpr (WPC > 1) __syncthreads();  // every wave is done with the centre scratch
#pragma unroll
    for (int q = 0; q < kFill; ++q) {
        const int i = q * kWave * WPC + ctid;
        if (i < nrows) {
            ids[i] = pid[q];
            olds[i] = pl[q];
        }
    }
    if constexpr (WPC > 1) __syncthreads();
    else wave_lds_sync();
    const double xw0 = 128.0 * wsum;
    const double hs = h * kMarginScale;
    const double bnd = 128.0 * D + 2.0;
    const double colscale = tc < 4 ? static_cast<double>(1 << (8 * tc)) : 0.0;
    int off[KB];  // byte offset of this lane's slice (slices past D read the row start; zero digits)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) off[kb] = (kb * 64 + 16 * tq < D) ? kb * 64 + 16 * tq : 0;

    // first pass: packed 16-bit sums of the lane's slice (total, side 1)
    uint32_t tot[FIRST ? KB : 1][8], one[FIRST ? KB : 1][8];
#pragma unroll
    for (int kb = 0; kb < (FIRST ? KB : 1); ++kb)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            tot[kb][k] = 0u;
            one[kb][k] = 0u;
        }
    int n1 = 0, changed = 0, nchg = 0;
    // changed-row list: in place in the id list (one wave per chunk: every
    // later read of the id list is past the current tile), else per wave
    int32_t* lid = WPC == 1 ? ids : s_lid[wl % (WPC == 1 ? 1 : 4)];
    uint8_t* lsg = WPC == 1 ? olds : s_lsg[wl % (WPC == 1 ? 1 : 4)];
    const int ntiles = (nrows + 15) >> 4;
    const int mytiles = ntiles > wc ? (ntiles - wc + WPC - 1) / WPC : 0;
    const int steps = (mytiles + U - 1) / U;

    auto load_tiles = [&](int st, uint4 (&x)[U][KB]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = min(((st * U + u) * WPC + wc) * 16 + tc, nrows - 1);
            const uint8_t* xr = X + static_cast<size_t>(ids[i]) * D;
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) x[u][kb] = *reinterpret_cast<const uint4*>(xr + off[kb]);
        }
    };
    auto compute = [&](int st, const uint4 (&x)[U][KB]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t0 = ((st * U + u) * WPC + wc) * 16;
            if (t0 >= nrows) break;
            i32x4 acc = i32x4{0, 0, 0, 0};
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                const i32x4 a = i32x4{static_cast<int>(x[u][kb].x ^ 0x80808080u),
                                      static_cast<int>(x[u][kb].y ^ 0x80808080u),
                                      static_cast<int>(x[u][kb].z ^ 0x80808080u),
                                      static_cast<int>(x[u][kb].w ^ 0x80808080u)};
                acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, bop[kb], acc, 0, 0, 0);
            }
            double v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v[i] = static_cast<double>(acc[i]) * colscale;
                v[i] += dpp_f64<0xB1>(v[i]);
                v[i] += dpp_f64<0x4E>(v[i]);
            }
            // lane (q, c < 4) decides row 4 q + c of the tile
            const int rho = 4 * tq + tc;
            const bool mine = tc < 4 && t0 + rho < nrows;
            const double mg = (tc == 0 ? v[0] : tc == 1 ? v[1] : tc == 2 ? v[2] : v[3]) + xw0 - hs;
            uint32_t m1 = tile_bits(__builtin_amdgcn_ballot_w64(mine && mg < -bnd));
            uint32_t mb =
                tile_bits(__builtin_amdgcn_ballot_w64(mine && !(mg < -bnd) && !(mg > bnd)));
            while (mb != 0u) {  // band rows: the FP64 code
                const int rr = __builtin_ctz(mb);
                mb &= mb - 1u;
                const uint4 raw = *reinterpret_cast<const uint4*>(
                    X + static_cast<size_t>(ids[t0 + rr]) * D + (16 * l < D ? 16 * l : 0));
                const uint32_t wd[4] = {raw.x, raw.y, raw.z, raw.w};
                // w re-read from LDS here (not held in registers for this rare path)
                const double* swl = sw + 16 * l;
                asm volatile("" : "+v"(swl));
                double dot = 0.0;
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        dot = fma(static_cast<double>((wd[k4] >> (8 * b)) & 255u), swl[4 * k4 + b],
                                  dot);
                dot = group_sum_f64<G>(dot);
                if (__builtin_amdgcn_readfirstlane(dot < h ? 1 : 0) != 0) m1 |= 1u << rr;
            }
            const bool vrow = t0 + tc < nrows;  // row c of the tile (this lane's loads)
            const int my = static_cast<int>((m1 >> tc) & 1u);
            if (tq == 0 && vrow) labels[base + t0 + tc] = static_cast<uint8_t>(my);
            n1 += __builtin_popcount(m1);
            if constexpr (FIRST) {
                const uint32_t mt = vrow ? 0xFFFFFFFFu : 0u;
                const uint32_t m_1 = (vrow && my) ? 0xFFFFFFFFu : 0u;
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const uint32_t wd[4] = {x[u][kb].x, x[u][kb].y, x[u][kb].z, x[u][kb].w};
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4) {
                        const uint32_t lo = wd[k4] & 0x00FF00FFu;         // elements 0, 2
                        const uint32_t hi = (wd[k4] >> 8) & 0x00FF00FFu;  // elements 1, 3
                        tot[kb][2 * k4] += lo & mt;
                        tot[kb][2 * k4 + 1] += hi & mt;
                        one[kb][2 * k4] += lo & m_1;
                        one[kb][2 * k4 + 1] += hi & m_1;
                    }
                }
            } else {
                const uint32_t vm = nrows - t0 >= 16 ? 0xFFFFu : ((1u << (nrows - t0)) - 1u);
                const uint32_t old16 = static_cast<uint32_t>(
                    __builtin_amdgcn_ballot_w64(tq == 0 && vrow && olds[t0 + tc] != 0) & 0xFFFFull);
                const uint32_t ch = (m1 ^ old16) & vm;
                if (ch != 0u) {
                    // append (id, new label); with the in-place list the slot
                    // is at most the row's own slot
                    if (tq == 0 && ((ch >> tc) & 1u)) {
                        const int k = nchg + __builtin_popcount(ch & ((1u << tc) - 1u));
                        const int32_t id = ids[t0 + tc];
                        lid[k] = id;
                        lsg[k] = static_cast<uint8_t>(my);
                    }
                    const int c = __builtin_popcount(ch);
                    nchg += c;
                    changed += c;
                }
            }
        }
    };

    uint4 xb[PD + 1][U][KB];
#pragma unroll
    for (int q = 0; q < PD; ++q) load_tiles(q, xb[q]);
    for (int st0 = 0; st0 < steps; st0 += PD + 1) {
#pragma unroll
        for (int ph = 0; ph <= PD; ++ph) {
            const int st = st0 + ph;
            load_tiles(st + PD, xb[(ph + PD) % (PD + 1)]);  // no branch: waits stay exact
            if (st < steps) compute(st, xb[ph]);
        }
    }
    wave_lds_sync();

    // side sums of the wave's rows, lane l holding elements 2 l and 2 l + 1
    int32_t s1v[2] = {0, 0};
    int32_t totv[2] = {0, 0};
    if constexpr (FIRST) {
        if constexpr (WPC > 1) __syncthreads();  // the id list is spent for every wave
        // [2][DM] scratch in the id space (WPC == 4: one quarter per wave)
        uint32_t* sc = reinterpret_cast<uint32_t*>(ids) + (WPC > 1 ? wc * (kChunkRows / WPC) : 0);
        static_assert(2 * DM <= kChunkRows / WPC, "side-sum scratch exceeds the id space");
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                // lanes c and c ^ 1 first (two 16-bit halves stay below 2^16),
                // then the halves apart over the rest of the 16 lanes
                uint32_t a = tot[kb][k], b = one[kb][k];
                a += dpp_u32<0xB1>(a);
                b += dpp_u32<0xB1>(b);
                uint32_t alo = a & 0xFFFFu, ahi = a >> 16, blo = b & 0xFFFFu, bhi = b >> 16;
                alo += dpp_u32<0x4E>(alo);
                ahi += dpp_u32<0x4E>(ahi);
                blo += dpp_u32<0x4E>(blo);
                bhi += dpp_u32<0x4E>(bhi);
                alo += dpp_u32<0x141>(alo);
                ahi += dpp_u32<0x141>(ahi);
                blo += dpp_u32<0x141>(blo);
                bhi += dpp_u32<0x141>(bhi);
                alo += dpp_u32<0x140>(alo);
                ahi += dpp_u32<0x140>(ahi);
                blo += dpp_u32<0x140>(blo);
                bhi += dpp_u32<0x140>(bhi);
                if (tc == 0) {
                    // register k: elements 4 (k / 2) + (k & 1) and + 2
                    const int e = kb * 64 + 16 * tq + 4 * (k >> 1) + (k & 1);
                    sc[e] = alo;
                    sc[e + 2] = ahi;
                    sc[DM + e] = blo;
                    sc[DM + e + 2] = bhi;
                }
            }
        wave_lds_sync();
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int e = 2 * lane + c;
            if (e < DM) {
                totv[c] = static_cast<int32_t>(sc[e]);
                s1v[c] = static_cast<int32_t>(sc[DM + e]);
            }
        }
    } else {
        if (wc == 0) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int e = 2 * lane + c;
                if (e < D) s1v[c] = static_cast<int32_t>(p0[D + e]);
            }
        }
        // changed rows: +x for 0 -> 1, -x for 1 -> 0 (four rows in flight)
        const int eo = 2 * lane < D ? 2 * lane : 0;
        for (int k0 = 0; k0 < nchg; k0 += 4) {
            uint32_t two[4];
            int sg[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = min(k0 + j, nchg - 1);
                two[j] = *reinterpret_cast<const uint16_t*>(X + static_cast<size_t>(lid[k]) * D + eo);
                sg[j] = k0 + j < nchg ? (lsg[k] ? 1 : -1) : 0;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                s1v[0] += sg[j] * static_cast<int32_t>(two[j] & 255u);
                s1v[1] += sg[j] * static_cast<int32_t>(two[j] >> 8);
            }
        }
    }
    if constexpr (WPC > 1) {
        // the chunk's waves add their sums and counts; wave 0 finishes
        int32_t* red = s_red[wl % (WPC == 1 ? 1 : 4)];
        red[2 * lane] = FIRST ? totv[0] : 0;
        red[2 * lane + 1] = FIRST ? totv[1] : 0;
        if (lane == 0) {
            red[2 * kWave] = n1;
            red[2 * kWave + 1] = changed;
        }
        __syncthreads();
        int32_t* red1 = reinterpret_cast<int32_t*>(s_lid[wl % (WPC == 1 ? 1 : 4)]);
        red1[2 * lane] = s1v[0];
        red1[2 * lane + 1] = s1v[1];
        __syncthreads();
        if (wc != 0) return;
        n1 = 0;
        changed = 0;
        for (int w = 0; w < WPC; ++w) {
            const int32_t* rw = s_red[wl + w];
            const int32_t* r1 = reinterpret_cast<const int32_t*>(s_lid[wl + w]);
            if (w > 0) {
                totv[0] += rw[2 * lane];
                totv[1] += rw[2 * lane + 1];
                s1v[0] += r1[2 * lane];
                s1v[1] += r1[2 * lane + 1];
            }
            n1 += rw[2 * kWave];
            changed += rw[2 * kWave + 1];
        }
    }

    if (lane == 0) {
        cnt[2 * wave] = n1;  // ones of this chunk (also read by the scatter)
        cnt[2 * wave + 1] = changed;
        stat_add(assigned, static_cast<unsigned>(wave), static_cast<unsigned long long>(nrows));
    }
    if (nch == 1) {  // the chunk holds the whole node
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
        const double dn0 = static_cast<double>(n0), dn1 = static_cast<double>(n1);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int e = 2 * lane + c;
            if (e < D) {
                double t;
                if constexpr (FIRST) {
                    t = static_cast<double>(totv[c]);
                    p0[e] = t;
                } else {
                    t = p0[e];
                }
                const double s1 = static_cast<double>(s1v[c]);
                p0[D + e] = s1;
                cn[e] = (t - s1) / dn0;
                cn[D + e] = s1 / dn1;
            }
        }
        return;
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {  // publish this chunk's sums
        const int e = 2 * lane + c;
        if (e < D) {
            if constexpr (FIRST) p0[e] = static_cast<double>(totv[c]);
            p0[D + e] = static_cast<double>(s1v[c]);
        }
    }
}

template <int KB, int G, int U, int WPC>
void pick_pd(int pd, AssignFn<uint8_t>* f) {
    switch (pd) {
        case 1: f[0] = k_assign_u8m<KB, G, U, 1, true, WPC>; f[1] = k_assign_u8m<KB, G, U, 1, false, WPC>; break;
        case 2: f[0] = k_assign_u8m<KB, G, U, 2, true, WPC>; f[1] = k_assign_u8m<KB, G, U, 2, false, WPC>; break;
        default: f[0] = k_assign_u8m<KB, G, U, 3, true, WPC>; f[1] = k_assign_u8m<KB, G, U, 3, false, WPC>; break;
    }
}

template <int KB, int G>
void pick_u(int u, int pd, AssignFn<uint8_t>* f, AssignFn<uint8_t>* f4) {
    if (u == 2) pick_pd<KB, G, 2, 1>(pd, f);
    else pick_pd<KB, G, 1, 1>(pd, f);
    pick_pd<KB, G, 1, 4>(pd, f4);
}

}  // namespace

bool pick_assign_u8_mfma(int D, int u, int pd, AssignFn<uint8_t>* f, AssignFn<uint8_t>* f4) {
    f[0] = f[1] = f4[0] = f4[1] = nullptr;
    if (D <= 0 || D % 16 != 0 || D > 128) return false;
    const int E = D / 16;
    if (E == 1) pick_u<1, 1>(u, pd, f, f4);
    else if (E == 2) pick_u<1, 2>(u, pd, f, f4);
    else if (E <= 4) pick_u<1, 4>(u, pd, f, f4);
    else pick_u<2, 8>(u, pd, f, f4);
    return true;
}

}  // namespace knng
