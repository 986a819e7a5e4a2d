// Enhanced hill-climbing search over a kNN graph (Alg. 2, E-GNNS): every
// round expands each member of the rank list's top-k that has not been
// expanded yet, takes the distances of the neighbours not visited before,
// and merges them into the rank list after the round.
//
// One 256-thread workgroup per query, all state in LDS:
//   - the visited set: an open-addressing table of node ids (linear probing,
//     insertion by compare-and-swap, so each id is claimed by one thread);
//     bit 31 of a slot marks a node already expanded;
//   - the rank list R: the k best keys (d32 bits << 32 | id), ascending;
//   - the round's new candidates T, appended by the threads that claimed
//     them; once R holds k entries only the candidates below its k-th key
//     can enter (keys are unique), so T is cut to those first; R u T is
//     ordered with a block bitonic sort and R takes the first k (the k-th
//     distance of R never grows, so entries beyond k can never return).
// The frontier (members of R not expanded yet) is marked by one thread per
// member of R; its order does not matter (a neighbour shared by two members
// is claimed once, with the same distance).
// A thread computes the canonical d32 of one candidate: per 32-dimension
// block a sequential fused multiply-add from 0, blocks added in order -- the
// library's output distance, so the rank order is the one the oracle takes
// in its d32 mode.  A round without an unexpanded member ends the search.
// work (nullable): spread counters of the distances taken and the nodes
// expanded, for the bytes the search reads.
#include "knng_internal.hpp"
#include "wave.hpp"

#include <cstdio>

namespace knng {
namespace {

constexpr int kSearchThreads = 256;
constexpr uint32_t kExpanded = 0x80000000u;

__device__ __forceinline__ uint32_t slot_of(int32_t id, int hbits) {
    return (static_cast<uint32_t>(id) * 2654435761u) >> (32 - hbits);
}

// Claims id in the visited table: true if this call inserted it.
__device__ __forceinline__ bool visit(int32_t* tab, int hbits, int32_t id) {
    const uint32_t mask = (1u << hbits) - 1u;
    uint32_t h = slot_of(id, hbits);
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        const int32_t old = atomicCAS(&tab[h], -1, id);
        if (old == -1) return true;
        if ((static_cast<uint32_t>(old) & ~kExpanded) == static_cast<uint32_t>(id)) return false;
        h = (h + 1u) & mask;
    }
    return false;  // unreachable: the table holds at least twice the ids that can be visited
}

// Marks a visited id expanded; returns true if it was not expanded before.
__device__ __forceinline__ bool expand(int32_t* tab, int hbits, int32_t id) {
    const uint32_t mask = (1u << hbits) - 1u;
    uint32_t h = slot_of(id, hbits);
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        const int32_t v = tab[h];
        if ((static_cast<uint32_t>(v) & ~kExpanded) == static_cast<uint32_t>(id)) {
            if (static_cast<uint32_t>(v) & kExpanded) return false;
            tab[h] = static_cast<int32_t>(static_cast<uint32_t>(id) | kExpanded);
            return true;
        }
        h = (h + 1u) & mask;
    }
    return false;
}

// Canonical d32 of the query (LDS) and row x (global).
__device__ __forceinline__ float d32_row(const float* q, const float* __restrict__ x, int D,
                                         bool vec4) {
    float tot = 0.f;
    for (int d0 = 0; d0 < D; d0 += 32) {
        const int dn = D - d0 < 32 ? D - d0 : 32;
        float blk = 0.f;
        if (vec4 && dn == 32) {
            float4 v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = reinterpret_cast<const float4*>(x + d0)[i];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float e[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float df = q[d0 + 4 * i + j] - e[j];
                    blk = __fmaf_rn(df, df, blk);
                }
            }
        } else {
            for (int dd = 0; dd < dn; ++dd) {
                const float df = q[d0 + dd] - x[d0 + dd];
                blk = __fmaf_rn(df, df, blk);
            }
        }
        tot = tot + blk;
    }
    return tot;
}

// The same d32 over a uint8 row (integer data in [0, 255]: each byte is the
// FP32 value exactly, so the result equals d32 of the FP32 row); vec16: whole
// 32-byte blocks read as two 16-byte loads.
__device__ __forceinline__ float d32_row_u8(const float* q, const uint8_t* __restrict__ x, int D,
                                            bool vec16) {
    float tot = 0.f;
    for (int d0 = 0; d0 < D; d0 += 32) {
        const int dn = D - d0 < 32 ? D - d0 : 32;
        float blk = 0.f;
        if (vec16 && dn == 32) {
            const uint4 v0 = reinterpret_cast<const uint4*>(x + d0)[0];
            const uint4 v1 = reinterpret_cast<const uint4*>(x + d0)[1];
            const uint32_t w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
            for (int i = 0; i < 8; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float e = static_cast<float>((w[i] >> (8 * j)) & 255u);
                    const float df = q[d0 + 4 * i + j] - e;
                    blk = __fmaf_rn(df, df, blk);
                }
        } else {
            for (int dd = 0; dd < dn; ++dd) {
                const float df = q[d0 + dd] - static_cast<float>(x[d0 + dd]);
                blk = __fmaf_rn(df, df, blk);
            }
        }
        tot = tot + blk;
    }
    return tot;
}

// Row distance for the row type of the reference set.
template <typename TX>
__device__ __forceinline__ float d32_of(const float* q, const TX* __restrict__ X, int32_t id, int D,
                                        bool vec) {
    if constexpr (sizeof(TX) == 1)
        return d32_row_u8(q, X + static_cast<size_t>(id) * D, D, vec);
    else
        return d32_row(q, X + static_cast<size_t>(id) * D, D, vec);
}

struct SearchShape {
    int hbits;  // visited table: 2^hbits slots
    int tcap;   // new candidates per round: k * kg (at least the seeds)
    int scap;   // sort buffer: power of two >= k + tcap
};

template <typename TX>
__global__ __launch_bounds__(kSearchThreads) void k_egnns(
    const TX* __restrict__ X, int64_t n, int D, const int32_t* __restrict__ G, int kg,
    const float* __restrict__ Q, const int32_t* __restrict__ seeds, int ns, int k, int rounds,
    SearchShape sh, int32_t* __restrict__ ids_out, float* __restrict__ d_out,
    unsigned long long* __restrict__ work) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int H = 1 << sh.hbits;
    uint64_t* keys = reinterpret_cast<uint64_t*>(smem);                  // [scap]: R then T
    float* q = reinterpret_cast<float*>(keys + sh.scap);                 // [D, padded to 4]
    int32_t* tab = reinterpret_cast<int32_t*>(q + ((D + 3) & ~3));       // [H]
    int32_t* front = tab + H;                                            // [k]
    __shared__ int s_nr, s_nt, s_nf, s_ns;
    __shared__ unsigned long long s_dist, s_exp;  // distances taken, nodes expanded

    const int tid = threadIdx.x;
    const int64_t qi = blockIdx.x;
    // vector loads: 16-byte aligned rows (FP32: D % 4 == 0; uint8: D % 16 == 0)
    const bool vec4 = (D % (sizeof(TX) == 1 ? 16 : 4)) == 0;
    for (int i = tid; i < H; i += kSearchThreads) tab[i] = -1;
    for (int d = tid; d < D; d += kSearchThreads) q[d] = Q[qi * D + d];
    if (tid == 0) {
        s_nr = 0;
        s_nt = 0;
        s_nf = 0;
        s_ns = 0;
        s_dist = 0;
        s_exp = 0;
    }

    // R lives in keys[0, k) (empty slots hold the largest key), the round's
    // new candidates in keys[k, k + nt); merge = sort keys[0, m) for the
    // power of two m >= k + nt, after which keys[0, k) is the new R
    for (int i = tid; i < k; i += kSearchThreads) keys[i] = ~0ull;
    constexpr int kCut = 8;  // candidates per thread held in registers by the cut
    auto merge = [&]() {
        const int nr = s_nr, nt = s_nt;
        int nk = nt;  // candidates that can still enter R
        if (nr == k && nt > 0 && nt <= kCut * kSearchThreads) {
            const uint64_t kth = keys[k - 1];
            uint64_t v[kCut];
#pragma unroll
            for (int j = 0; j < kCut; ++j) {
                const int i = tid + j * kSearchThreads;
                v[j] = i < nt ? keys[k + i] : ~0ull;
            }
            __syncthreads();  // every candidate read before any is moved
#pragma unroll
            for (int j = 0; j < kCut; ++j)
                if (v[j] < kth) keys[k + atomicAdd(&s_ns, 1)] = v[j];
            __syncthreads();
            nk = s_ns;
        }
        int m = 1;
        while (m < k + nk) m <<= 1;
        for (int i = k + nk + tid; i < m; i += kSearchThreads) keys[i] = ~0ull;
        __syncthreads();
        for (int size = 2; size <= m; size <<= 1)
            for (int stride = size >> 1; stride >= 1; stride >>= 1) {
                for (int i = tid; i < (m >> 1); i += kSearchThreads) {
                    const int lo = 2 * i - (i & (stride - 1));
                    const int hi = lo + stride;
                    const bool up = (lo & size) == 0;
                    const uint64_t a = keys[lo], b = keys[hi];
                    if ((a > b) == up) {
                        keys[lo] = b;
                        keys[hi] = a;
                    }
                }
                __syncthreads();
            }
        if (tid == 0) {
            s_nr = nr + nk < k ? nr + nk : k;
            s_nt = 0;
            s_ns = 0;
            s_nf = 0;
            s_dist += static_cast<unsigned long long>(nt);
        }
        __syncthreads();
    };

    __syncthreads();
    // seeds
    for (int s = tid; s < ns; s += kSearchThreads) {
        const int32_t id = seeds[qi * ns + s];
        if (id >= 0 && id < n && visit(tab, sh.hbits, id)) {
            const float d = d32_of(q, X, id, D, vec4);
            keys[k + atomicAdd(&s_nt, 1)] = cand_key(d, id);
        }
    }
    __syncthreads();
    merge();

    for (int t = 0; t < rounds; ++t) {
        // frontier: the members of R not expanded yet (front[p] = its id, or
        // -1 for a member expanded before)
        const int nr = s_nr;
        for (int p = tid; p < nr; p += kSearchThreads) {
            const int32_t id = key_id(keys[p]);
            const bool fresh = expand(tab, sh.hbits, id);
            front[p] = fresh ? id : -1;
            if (fresh) atomicAdd(&s_nf, 1);
        }
        __syncthreads();
        const int nf = s_nf;
        if (tid == 0) s_exp += static_cast<unsigned long long>(nf);
        if (nf == 0) break;
        // neighbours of the frontier not visited before
        for (int c = tid; c < nr * kg; c += kSearchThreads) {
            const int32_t f = front[c / kg];
            if (f < 0) continue;
            const int32_t id = G[static_cast<size_t>(f) * kg + c % kg];
            if (id >= 0 && id < n && visit(tab, sh.hbits, id)) {
                const float d = d32_of(q, X, id, D, vec4);
                keys[k + atomicAdd(&s_nt, 1)] = cand_key(d, id);
            }
        }
        __syncthreads();
        merge();
    }

    const int nr = s_nr;
    if (work != nullptr && tid == 0) {
        stat_add(work, static_cast<unsigned>(blockIdx.x), s_dist);
        stat_add(work + kStatWords, static_cast<unsigned>(blockIdx.x), s_exp);
    }
    for (int p = tid; p < k; p += kSearchThreads) {
        const bool ok = p < nr;
        ids_out[qi * k + p] = ok ? key_id(keys[p]) : -1;
        d_out[qi * k + p] = ok ? key_dist(keys[p]) : __int_as_float(0x7f800000);
    }
}

}  // namespace

int search_run(const SearchArgs& a, char* err, size_t errlen) {
    // visited ids are at most the seeds plus kg per expanded node, and at
    // most k nodes are expanded per round
    const int64_t bound = static_cast<int64_t>(a.ns) + static_cast<int64_t>(a.rounds) * a.k * a.kg;
    int hbits = 4;
    while ((int64_t{1} << hbits) < 2 * bound) ++hbits;
    SearchShape sh;
    sh.hbits = hbits;
    sh.tcap = a.k * a.kg > a.ns ? a.k * a.kg : a.ns;
    sh.scap = 1;
    while (sh.scap < a.k + sh.tcap) sh.scap <<= 1;
    const size_t lds = sizeof(uint64_t) * sh.scap + sizeof(float) * ((a.D + 3) & ~3) +
                       sizeof(int32_t) * ((size_t{1} << hbits) + a.k);
    if (lds > kSearchLdsMax) {
        std::snprintf(err, errlen,
                      "search state needs %zu bytes of LDS (seeds %d + rounds %d x k %d x graph "
                      "degree %d); at most %zu",
                      lds, a.ns, a.rounds, a.k, a.kg, kSearchLdsMax);
        return kUnsupported;
    }
    if (a.nq == 0) return kOk;
    if (a.X8 != nullptr)
        k_egnns<uint8_t><<<static_cast<unsigned>(a.nq), kSearchThreads, lds, a.stream>>>(
            a.X8, a.n, a.D, a.G, a.kg, a.Q, a.seeds, a.ns, a.k, a.rounds, sh, a.ids_out, a.d_out,
            a.work);
    else
        k_egnns<float><<<static_cast<unsigned>(a.nq), kSearchThreads, lds, a.stream>>>(
            a.X, a.n, a.D, a.G, a.kg, a.Q, a.seeds, a.ns, a.k, a.rounds, sh, a.ids_out, a.d_out,
            a.work);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        std::snprintf(err, errlen, "search launch failed: %s", hipGetErrorString(e));
        return kHip;
    }
    return kOk;
}

}  // namespace knng
