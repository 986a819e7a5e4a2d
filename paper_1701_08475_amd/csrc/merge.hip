// Union of the rounds' candidate lists into G (Alg. 1: the rows of G are
// refined round after round; a pair already compared is not counted twice).
//
// k <= 32: one thread per row (k_merge_rows).  Otherwise (or with the knob
// merge_network = 1, KNNG_MERGE_NETWORK=1) one wavefront per row: the row's candidates from every tree are ordered by
// (d32, id) with a bitonic network (a merge of the trees' sorted lists when
// k <= 32, else a full sort), adjacent equal keys are dropped (the same id
// always carries the same d32 bits, so duplicates are adjacent), and the
// first k survivors are written.  When the candidates of all trees do not fit
// one network, trees are merged in groups into the output row.
#include "knng_internal.hpp"
#include "wave.hpp"

#include <cstdio>
#include <cstdlib>

namespace knng {
namespace {

template <int R>
__global__ __launch_bounds__(256) void k_merge(int64_t n, int k, int t0, int t1,
                                               const int32_t* __restrict__ cid,
                                               const float* __restrict__ cd,
                                               int32_t* __restrict__ oid, float* __restrict__ od,
                                               int with_prev) {
    const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const int lane = threadIdx.x & 63;
    const int np = with_prev ? k : 0;
    const int total = np + (t1 - t0) * k;
    uint64_t v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = lane * R + r;
        v[r] = kNoKey;
        if (e < total) {
            int32_t id;
            float d;
            if (e < np) {
                id = oid[row * k + e];
                d = od[row * k + e];
            } else {
                const int q = e - np;
                const size_t src = (static_cast<size_t>(t0 + q / k) * n + row) * k + q % k;
                id = cid[src];
                d = cd[src];
            }
            if (id >= 0) v[r] = cand_key(d, id);
        }
    }
    wave_bitonic_sort<R>(v);
    // previous element of each slot (lane-1's last slot for r == 0)
    const uint64_t last_of_prev_lane = shfl_u64(v[R - 1], lane > 0 ? lane - 1 : 0);
    bool keep[R];
    int cnt = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint64_t before = r > 0 ? v[r - 1] : (lane > 0 ? last_of_prev_lane : kNoKey);
        keep[r] = v[r] != kNoKey && v[r] != before;
        cnt += keep[r] ? 1 : 0;
    }
    int kept;
    int pos = wave_excl_scan(cnt, &kept);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (keep[r]) {
            if (pos < k) {
                oid[row * k + pos] = key_id(v[r]);
                od[row * k + pos] = key_dist(v[r]);
            }
            ++pos;
        }
    }
    for (int p = kept + lane; p < k; p += kWave) {
        oid[row * k + p] = -1;
        od[row * k + p] = __int_as_float(0x7f800000);
    }
}

// k <= 32: every input list (the previous output row, then one list per
// tree) is already sorted by (d32, id), so each takes a run of 32 slots,
// loaded ascending (even runs) or reversed (odd runs), and the bitonic
// network starts at runs of 64: a merge rather than a sort.
template <int R>
__global__ __launch_bounds__(256) void k_merge_runs(int64_t n, int k, int t0, int t1,
                                                    const int32_t* __restrict__ cid,
                                                    const float* __restrict__ cd,
                                                    int32_t* __restrict__ oid,
                                                    float* __restrict__ od, int with_prev) {
    const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const int lane = threadIdx.x & 63;
    const int lists = (with_prev ? 1 : 0) + (t1 - t0);
    uint64_t v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = lane * R + r;
        const int b = e >> 5, q = e & 31;
        const int idx = (b & 1) ? 31 - q : q;  // odd runs reversed
        v[r] = kNoKey;
        if (b < lists && idx < k) {
            int32_t id;
            float d;
            if (with_prev && b == 0) {
                id = oid[row * k + idx];
                d = od[row * k + idx];
            } else {
                const size_t src =
                    (static_cast<size_t>(t0 + b - (with_prev ? 1 : 0)) * n + row) * k + idx;
                id = cid[src];
                d = cd[src];
            }
            if (id >= 0) v[r] = cand_key(d, id);
        }
    }
    wave_bitonic_sort<R, 64>(v);
    const uint64_t last_of_prev_lane = shfl_u64(v[R - 1], lane > 0 ? lane - 1 : 0);
    bool keep[R];
    int cnt = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint64_t before = r > 0 ? v[r - 1] : (lane > 0 ? last_of_prev_lane : kNoKey);
        keep[r] = v[r] != kNoKey && v[r] != before;
        cnt += keep[r] ? 1 : 0;
    }
    int kept;
    int pos = wave_excl_scan(cnt, &kept);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (keep[r]) {
            if (pos < k) {
                oid[row * k + pos] = key_id(v[r]);
                od[row * k + pos] = key_dist(v[r]);
            }
            ++pos;
        }
    }
    for (int p = kept + lane; p < k; p += kWave) {
        oid[row * k + p] = -1;
        od[row * k + p] = __int_as_float(0x7f800000);
    }
}

// k <= 32, one thread per row: the row's best K (k rounded up to 4) distinct
// keys in registers, sorted.  The first tree's list is taken as it is (sorted,
// distinct ids); every later list is read in order until its key reaches the
// current K-th best (the rest of that list is larger), and each key not yet
// held is inserted with a compare-exchange network (slot i takes
// min(old[i], max(old[i-1], key))).  Same result as the bitonic merge: the
// first k of the sorted distinct union.
template <int K, bool VEC>
__global__ __launch_bounds__(256) void k_merge_rows(int64_t n, int k, int T,
                                                    const int32_t* __restrict__ cid,
                                                    const float* __restrict__ cd,
                                                    int32_t* __restrict__ oid,
                                                    float* __restrict__ od) {
    const int64_t row = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (row >= n) return;
    uint64_t top[K];
#pragma unroll
    for (int i = 0; i < K; ++i) top[i] = kNoKey;
    if (VEC) {  // k == K: the first list in K / 4 pairs of 16-byte loads
        const size_t src = static_cast<size_t>(row) * K;
#pragma unroll
        for (int i = 0; i < K; i += 4) {
            const int4 i4 = *reinterpret_cast<const int4*>(cid + src + i);
            const float4 d4 = *reinterpret_cast<const float4*>(cd + src + i);
            top[i] = i4.x >= 0 ? cand_key(d4.x, i4.x) : kNoKey;
            top[i + 1] = i4.y >= 0 ? cand_key(d4.y, i4.y) : kNoKey;
            top[i + 2] = i4.z >= 0 ? cand_key(d4.z, i4.z) : kNoKey;
            top[i + 3] = i4.w >= 0 ? cand_key(d4.w, i4.w) : kNoKey;
        }
    } else {
        const size_t src = static_cast<size_t>(row) * k;
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (i < k) {
                const int32_t id = cid[src + i];
                if (id >= 0) top[i] = cand_key(cd[src + i], id);
            }
    }
    auto insert = [&](uint64_t key) {
        bool dup = false;
#pragma unroll
        for (int i = 0; i < K; ++i) dup |= top[i] == key;
        if (dup) return;
        uint64_t prev = 0ull;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const uint64_t cur = top[i];
            const uint64_t hi = prev > key ? prev : key;
            top[i] = cur < hi ? cur : hi;
            prev = cur;
        }
    };
    // VEC: the first four entries of the next tree's list are loaded while
    // the current list is merged
    int4 ni = make_int4(-1, -1, -1, -1);
    float4 nd = make_float4(0.f, 0.f, 0.f, 0.f);
    if (VEC && T > 1) {
        const size_t s1 = (static_cast<size_t>(n) + row) * K;
        ni = *reinterpret_cast<const int4*>(cid + s1);
        nd = *reinterpret_cast<const float4*>(cd + s1);
    }
    for (int t = 1; t < T; ++t) {
        const size_t src = (static_cast<size_t>(t) * n + row) * k;
        if (VEC) {
            int4 i4 = ni;
            float4 d4 = nd;
            if (t + 1 < T) {
                const size_t s1 = (static_cast<size_t>(t + 1) * n + row) * K;
                ni = *reinterpret_cast<const int4*>(cid + s1);
                nd = *reinterpret_cast<const float4*>(cd + s1);
            }
            // four entries per 16-byte load, loaded ahead of the tests
            for (int j0 = 0; j0 < K; j0 += 4) {
                if (j0 > 0) {
                    i4 = *reinterpret_cast<const int4*>(cid + src + j0);
                    d4 = *reinterpret_cast<const float4*>(cd + src + j0);
                }
                const int32_t iv[4] = {i4.x, i4.y, i4.z, i4.w};
                const float dv[4] = {d4.x, d4.y, d4.z, d4.w};
                bool more = true;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (more && iv[q] >= 0) {
                        const uint64_t key = cand_key(dv[q], iv[q]);
                        if (key < top[K - 1]) insert(key);
                        else more = false;  // the rest of this list is larger
                    } else {
                        more = false;  // padding: the rest of the list is empty
                    }
                }
                if (!more) break;
            }
        } else {
            for (int j = 0; j < k; ++j) {
                const int32_t id = cid[src + j];
                if (id < 0) break;  // padding: the rest of the list is empty
                const uint64_t key = cand_key(cd[src + j], id);
                if (key >= top[K - 1]) break;  // the rest of this list is larger
                insert(key);
            }
        }
    }
    const size_t dst = static_cast<size_t>(row) * k;
    auto out_id = [&](int i) { return top[i] != kNoKey ? key_id(top[i]) : -1; };
    auto out_d = [&](int i) {
        return top[i] != kNoKey ? key_dist(top[i]) : __int_as_float(0x7f800000);
    };
    if (VEC) {  // the output rows are 16-byte aligned too (k % 4 == 0)
#pragma unroll
        for (int i = 0; i < K; i += 4) {
            *reinterpret_cast<int4*>(oid + dst + i) =
                make_int4(out_id(i), out_id(i + 1), out_id(i + 2), out_id(i + 3));
            *reinterpret_cast<float4*>(od + dst + i) =
                make_float4(out_d(i), out_d(i + 1), out_d(i + 2), out_d(i + 3));
        }
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (i < k) {
                oid[dst + i] = out_id(i);
                od[dst + i] = out_d(i);
            }
    }
}

using MergeFn = void (*)(int64_t, int, int, int, const int32_t*, const float*, int32_t*, float*,
                         int);
using RowMergeFn = void (*)(int64_t, int, int, const int32_t*, const float*, int32_t*, float*);

template <bool VEC>
RowMergeFn pick_rows_vec(int k) {
    switch ((k + 3) / 4) {
        case 1: return k_merge_rows<4, VEC>;
        case 2: return k_merge_rows<8, VEC>;
        case 3: return k_merge_rows<12, VEC>;
        case 4: return k_merge_rows<16, VEC>;
        case 5: return k_merge_rows<20, VEC>;
        case 6: return k_merge_rows<24, VEC>;
        case 7: return k_merge_rows<28, VEC>;
        default: return k_merge_rows<32, VEC>;
    }
}

// 16-byte loads and stores when every list and every output row starts
// 16-byte aligned (k % 4 == 0; the candidate buffers come from
// hipMallocAsync, 256-byte aligned; the outputs are the caller's)
RowMergeFn pick_rows(int k, const void* ids, const void* d, const void* oid, const void* od) {
    auto a16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    const bool vec = k % 4 == 0 && a16(ids) && a16(d) && a16(oid) && a16(od);
    return vec ? pick_rows_vec<true>(k) : pick_rows_vec<false>(k);
}

MergeFn pick_runs(int lists) {
    if (lists <= 2) return k_merge_runs<1>;
    if (lists <= 4) return k_merge_runs<2>;
    if (lists <= 8) return k_merge_runs<4>;
    if (lists <= 16) return k_merge_runs<8>;
    return k_merge_runs<16>;
}

MergeFn pick(int slots) {
    if (slots <= 64) return k_merge<1>;
    if (slots <= 128) return k_merge<2>;
    if (slots <= 256) return k_merge<4>;
    if (slots <= 512) return k_merge<8>;
    return k_merge<16>;
}

}  // namespace

int merge_run(const MergeArgs& a, int* launches, char* err, size_t errlen) {
    const int k = a.k;
    if (k <= 32 && knob(kKnobMergeNetwork, 0) == 0) {
        const RowMergeFn f = pick_rows(k, a.cand_ids, a.cand_d, a.ids_out, a.dists_out);
        if (a.timer) a.timer->begin(kKMerge, a.stream);
        f<<<static_cast<unsigned>((a.n + 255) / 256), 256, 0, a.stream>>>(
            a.n, k, a.n_trees, a.cand_ids, a.cand_d, a.ids_out, a.dists_out);
        if (a.timer) a.timer->end(kKMerge, a.stream);
        ++*launches;
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            std::snprintf(err, errlen, "merge launch failed: %s", hipGetErrorString(e));
            return kHip;
        }
        return kOk;
    }
    const int64_t blocks = (a.n + 3) / 4;
    constexpr int kMaxSlots = 1024;
    int t = 0;
    bool prev = false;
    const bool runs = k <= 32;  // lists fit runs of 32 slots
    const int unit = runs ? 32 : k;
    while (t < a.n_trees) {
        const int room = kMaxSlots - (prev ? unit : 0);
        int g = room / unit;
        if (g < 1) g = 1;
        const int t1 = t + g < a.n_trees ? t + g : a.n_trees;
        const int slots = (prev ? unit : 0) + (t1 - t) * unit;
        if (slots > kMaxSlots) {
            std::snprintf(err, errlen, "k=%d too large for the merge", k);
            return kUnsupported;
        }
        const MergeFn f = runs ? pick_runs((prev ? 1 : 0) + (t1 - t)) : pick(slots);
        if (a.timer) a.timer->begin(kKMerge, a.stream);
        f<<<static_cast<unsigned>(blocks), 256, 0, a.stream>>>(
            a.n, k, t, t1, a.cand_ids, a.cand_d, a.ids_out, a.dists_out, prev ? 1 : 0);
        if (a.timer) a.timer->end(kKMerge, a.stream);
        ++*launches;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            std::snprintf(err, errlen, "merge launch failed: %s", hipGetErrorString(e));
            return kHip;
        }
        prev = true;
        t = t1;
    }
    return kOk;
}

}  // namespace knng
