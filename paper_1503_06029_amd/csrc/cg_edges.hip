// Edges of the cell graph over the dictionary's cells (Section 2.2), by
// flip-and-look-up (Section 3.2, Algorithm 4) organised around two orders.
//
// A distance-1 pair (u, v), u < v, differs at exactly one bit k, where u has
// 0 and v has 1 (lexicographic order).  With the split s of the dictionary:
//
//  - k >= s: u and v share bits 0 .. s-1, so v lies after u inside u's prefix
//    group (the cells sharing u's first s bits, contiguous in sorted order).
//    The P pass scans that group; when it holds more than group_max cells
//    after u, it looks up u xor e_k for each such k instead (binary search).
//  - k < s: u and v share bits s .. l-1, so they sit in one run of the
//    suffix-grouped order (equal 32-bit suffix hash; collisions are weeded
//    out by the exact distance test).  The S pass scans runs of up to
//    group_max cells, and looks up u xor e_k for k < s in longer runs.
//
// Every edge is found once, from u.  u's neighbours in ascending v are its
// flips in descending k: first its P-neighbours (k >= s) in group order,
// then its S-neighbours (k < s) in run order (ids ascend within a run).
// So edge slots are offsets[u] + rank for P, offsets[u] + cntP[u] + rank for
// S, with offsets = exclusive scan of cntP + cntS.  Each pass runs twice:
// once to count, once to write.
#include "cg_internal.hpp"

namespace cg {

namespace {

// First s bits of a and b equal?
template <typename T>
__device__ __forceinline__ bool same_prefix(const T *a, const T *b, int s) {
    constexpr int B = Bits<T>::B;
    const int full = s / B, rem = s % B;
    for (int w = 0; w < full; ++w)
        if (a[w] != b[w]) return false;
    if (rem) {
        const T m = static_cast<T>(~T(0)) << (B - rem);
        if ((a[full] ^ b[full]) & m) return false;
    }
    return true;
}

__device__ __forceinline__ void emit(uint32_t *uv, uint16_t *bit, int64_t cap, int64_t pos, uint32_t u,
                                     uint32_t v, int k) {
    if (pos < cap) {
        uv[2 * pos] = u;
        uv[2 * pos + 1] = v;
        if (bit) bit[pos] = static_cast<uint16_t>(k);
    }
}

template <typename T, bool WRITE>
__global__ void __launch_bounds__(256) k_p_pass(const T *__restrict__ cells, const int64_t *d_n, int64_t ncap,
                                                int words, int ell, int s, int gmax, uint32_t *__restrict__ cntP,
                                                const int64_t *__restrict__ offsets, uint32_t *__restrict__ uv,
                                                uint16_t *__restrict__ bit, int64_t cap) {
    const int64_t n = load_n(d_n, ncap);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const T *me = cells + i * words;
        const int64_t base = WRITE ? offsets[i] : 0;
        uint32_t c = 0;
        bool big = false;
        for (int64_t j = i + 1; j < n; ++j) {
            const T *o = cells + j * words;
            if (!same_prefix<T>(me, o, s)) break;
            if (j - i > gmax) { big = true; break; }
            int pos;
            if (dist_upto2<T>(me, o, words, &pos) == 1) {
                if (WRITE) emit(uv, bit, cap, base + c, static_cast<uint32_t>(i), static_cast<uint32_t>(j), pos);
                ++c;
            }
        }
        if (big) {
            c = 0;
            for (int k = ell - 1; k >= s; --k) {
                if (get_bit<T>(me, k)) continue;
                const int64_t v = find_row<T>(cells, words, i + 1, n, me, k);
                if (v >= 0) {
                    if (WRITE) emit(uv, bit, cap, base + c, static_cast<uint32_t>(i), static_cast<uint32_t>(v), k);
                    ++c;
                }
            }
        }
        if (!WRITE) cntP[i] = c;
    }
}

template <typename T, bool WRITE>
__global__ void __launch_bounds__(256) k_s_pass(const T *__restrict__ cells, const uint64_t *__restrict__ sfx,
                                                const int64_t *d_n, int64_t ncap, int words, int s, int rmax,
                                                uint32_t *__restrict__ cntS, const uint32_t *__restrict__ cntP,
                                                const int64_t *__restrict__ offsets, uint32_t *__restrict__ uv,
                                                uint16_t *__restrict__ bit, int64_t cap) {
    const int64_t n = load_n(d_n, ncap);
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
         q += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const uint64_t e = sfx[q];
        const uint32_t h = static_cast<uint32_t>(e >> 32);
        const uint32_t id = static_cast<uint32_t>(e);
        int64_t left = 0, right = 0;
        while (left <= rmax && q - left - 1 >= 0 && static_cast<uint32_t>(sfx[q - left - 1] >> 32) == h) ++left;
        while (right <= rmax && q + right + 1 < n && static_cast<uint32_t>(sfx[q + right + 1] >> 32) == h) ++right;
        const T *me = cells + static_cast<int64_t>(id) * words;
        const int64_t base = WRITE ? offsets[id] + cntP[id] : 0;
        uint32_t c = 0;
        if (left + right + 1 > rmax) {
            for (int k = s - 1; k >= 0; --k) {
                if (get_bit<T>(me, k)) continue;
                const int64_t v = find_row<T>(cells, words, static_cast<int64_t>(id) + 1, n, me, k);
                if (v >= 0) {
                    if (WRITE) emit(uv, bit, cap, base + c, id, static_cast<uint32_t>(v), k);
                    ++c;
                }
            }
        } else {
            for (int64_t r = q - left; r <= q + right; ++r) {
                const uint32_t v = static_cast<uint32_t>(sfx[r]);
                if (v <= id) continue;
                int pos;
                if (dist_upto2<T>(me, cells + static_cast<int64_t>(v) * words, words, &pos) == 1 && pos < s) {
                    if (WRITE) emit(uv, bit, cap, base + c, id, v, pos);
                    ++c;
                }
            }
        }
        if (!WRITE) cntS[id] = c;
    }
}

__global__ void k_status(const int64_t *total, int64_t cap, int32_t *status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *status = (*total > cap) ? CG_ECAPACITY : CG_OK;
}

struct EdgesWs {
    uint32_t *cntP, *cntS;
    int64_t *offsets;
    uint64_t *tile_sums;
};

EdgesWs carve_edges(void *base, int64_t ncap, bool need_offsets, size_t *bytes) {
    Carver c(base);
    EdgesWs w{};
    const int64_t n = ncap > 0 ? ncap : 1;
    w.cntP = c.take<uint32_t>(n);
    w.cntS = c.take<uint32_t>(n);
    w.offsets = need_offsets ? c.take<int64_t>(n + 1) : nullptr;
    w.tile_sums = c.take<uint64_t>(scan_tiles(n));
    *bytes = c.bytes();
    return w;
}

template <typename T>
cg_status edges_impl(const cg_dict &d, uint32_t *uv, uint16_t *bit, int64_t cap, int64_t *d_nedges,
                     int64_t *d_offsets, void *ws, int32_t *d_status, hipStream_t s) {
    size_t b;
    EdgesWs w = carve_edges(ws, d.ncells_cap, true, &b);
    int64_t *offsets = d_offsets ? d_offsets : w.offsets;
    const int64_t ncap = d.ncells_cap;
    const T *cells = static_cast<const T *>(d.cells);
    const int words = d.lay.words, ell = d.lay.ell, sp = d.params.split_bit, gmax = d.params.group_max;
    const unsigned grid = blocks_for(ncap, 256, 16384);

    if (ncap == 0) {
        CG_TRY(fill_i64(d_nedges, 0, 1, s));
        if (d_offsets) CG_TRY(fill_i64(d_offsets, 0, 1, s));
        hipLaunchKernelGGL(k_status, dim3(1), dim3(64), 0, s, d_nedges, cap, d_status);
        CG_LAUNCHED("edges_status");
        return CG_OK;
    }
    hipLaunchKernelGGL((k_p_pass<T, false>), dim3(grid), dim3(256), 0, s, cells, d.d_ncells, ncap, words, ell, sp,
                       gmax, w.cntP, static_cast<const int64_t *>(nullptr), uv, bit, cap);
    CG_LAUNCHED("edges_p_count");
    if (sp > 0) {
        hipLaunchKernelGGL((k_s_pass<T, false>), dim3(grid), dim3(256), 0, s, cells, d.sfx, d.d_ncells, ncap, words,
                           sp, gmax, w.cntS, static_cast<const uint32_t *>(nullptr),
                           static_cast<const int64_t *>(nullptr), uv, bit, cap);
        CG_LAUNCHED("edges_s_count");
    } else {
        CG_TRY(fill_u32(w.cntS, 0, ncap, s));
    }
    CG_TRY(scan_pair_to_i64(w.cntP, w.cntS, offsets, ncap, d.d_ncells, w.tile_sums, d_nedges, s));
    hipLaunchKernelGGL(k_status, dim3(1), dim3(64), 0, s, d_nedges, cap, d_status);
    CG_LAUNCHED("edges_status");
    hipLaunchKernelGGL((k_p_pass<T, true>), dim3(grid), dim3(256), 0, s, cells, d.d_ncells, ncap, words, ell, sp,
                       gmax, w.cntP, offsets, uv, bit, cap);
    CG_LAUNCHED("edges_p_write");
    if (sp > 0) {
        hipLaunchKernelGGL((k_s_pass<T, true>), dim3(grid), dim3(256), 0, s, cells, d.sfx, d.d_ncells, ncap, words,
                           sp, gmax, w.cntS, w.cntP, offsets, uv, bit, cap);
        CG_LAUNCHED("edges_s_write");
    }
    return CG_OK;
}

}  // namespace

size_t edges_workspace_bytes(const cg_dict &d, int64_t cap) {
    (void)cap;
    size_t b;
    carve_edges(nullptr, d.ncells_cap, true, &b);
    return b;
}

cg_status run_edges(const cg_dict &d, uint32_t *uv, uint16_t *bit, int64_t cap, int64_t *d_nedges,
                    int64_t *d_offsets, void *ws, size_t ws_bytes, int32_t *d_status, hipStream_t s) {
    (void)ws_bytes;
    if (d.lay.word_bits == 64)
        return edges_impl<uint64_t>(d, uv, bit, cap, d_nedges, d_offsets, ws, d_status, s);
    return edges_impl<uint32_t>(d, uv, bit, cap, d_nedges, d_offsets, ws, d_status, s);
}

}  // namespace cg
