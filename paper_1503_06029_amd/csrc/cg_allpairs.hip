// Edges by the heuristic of Section 3.1: all pairs of cells, pruned with the
// triangle bound (*) of Section 1.1 against h reference cells.
//
// Algorithm 1 (ComputeDist): D[d][j] = dist(ref_d, x_j) for every cell j.
// Algorithm 2 (ParallelHeuristic), corrected: a pair (i, j) can be at
// distance 1 only if every reference distance differs by exactly one
// (|D[d][i] - D[d][j]| = 1 for all d; the printed test has its inequality
// reversed), and only such pairs get the exact XOR-popcount comparison.
// Pairs involving a reference are scanned like all others.
//
// Tiling: one 256-thread block per pair of 256-cell tiles (I <= J); the
// reference distances and rows of tile J sit in LDS, each thread owns one
// cell of tile I.  Found edges set bit k of a per-cell upward-neighbour mask
// and are appended to a list; ranks within a cell (descending k = ascending
// v) come from the mask, so the final placement matches the other paths byte
// for byte.
#include "cg_internal.hpp"

#include <cmath>

namespace cg {

namespace {

constexpr int AP_TILE = 256;
constexpr int AP_MAX_REFS = 8;

template <typename T>
__global__ void __launch_bounds__(256) k_ref_dists(const T *__restrict__ cells, const int64_t *d_n, int64_t ncap,
                                                   int words, int h, uint16_t *__restrict__ D) {
    const int64_t n = load_n(d_n, ncap);
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < n;
         j += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const T *x = cells + j * words;
        for (int d = 0; d < h; ++d) {
            const int64_t r = (static_cast<int64_t>(d) * n) / h;  // references spread over the order
            const T *y = cells + r * words;
            uint32_t c = 0;
            for (int w = 0; w < words; ++w) c += popc<T>(x[w] ^ y[w]);
            D[static_cast<int64_t>(d) * ncap + j] = static_cast<uint16_t>(c);
        }
    }
}

// One block per tile pair (I, J), I <= J.  Tile J's reference distances and
// (WT > 0) its rows, zero-padded to WT words, sit in LDS; thread t owns cell
// i0 + t of tile I with its own distances and row in registers.  All threads
// walk the 256 cells of tile J together, so every LDS read is a broadcast.
// Found edges go to a block stash in LDS and reach the global list with one
// reservation per block (per-edge global atomics would serialise on the
// cursor); a stash that fills up sends the rest one wave-reservation at a
// time.  WT = 0: rows too wide for LDS, read from global memory.
constexpr int AP_STASH = 1024;

template <typename T, int WT>
__global__ void __launch_bounds__(AP_TILE) k_allpairs(const T *__restrict__ cells, const int64_t *d_n, int64_t ncap,
                                                      int words, int h, const uint16_t *__restrict__ D,
                                                      T *__restrict__ mask, uint4 *__restrict__ list,
                                                      unsigned long long *__restrict__ cursor, int64_t list_cap) {
    constexpr int B = Bits<T>::B;
    constexpr int LW = WT + 1;
    extern __shared__ __align__(16) unsigned char smem[];
    T *rj = reinterpret_cast<T *>(smem);  // WT > 0: AP_TILE rows of LW words
    __shared__ uint16_t dj[AP_MAX_REFS][AP_TILE];
    __shared__ uint4 stash[AP_STASH];
    __shared__ uint32_t s_n;
    __shared__ unsigned long long s_base;
    const int64_t n = load_n(d_n, ncap);
    // block -> (I, J), I <= J, from the triangular index b = J (J + 1) / 2 + I
    const int64_t b = blockIdx.x;
    int64_t J = static_cast<int64_t>((std::sqrt(8.0 * static_cast<double>(b) + 1.0) - 1.0) * 0.5);
    while (J * (J + 1) / 2 > b) --J;
    while ((J + 1) * (J + 2) / 2 <= b) ++J;
    const int64_t I = b - J * (J + 1) / 2;
    const int64_t i0 = I * AP_TILE, j0 = J * AP_TILE;
    if (j0 >= n) return;  // the same for the whole block
    const int t = threadIdx.x, lane = t & 63;
    const int jn = static_cast<int>(n - j0 < AP_TILE ? n - j0 : AP_TILE);
    for (int d = 0; d < h; ++d) dj[d][t] = t < jn ? D[static_cast<int64_t>(d) * ncap + j0 + t] : 0;
    if (WT > 0) {
        for (int e = t; e < AP_TILE * WT; e += AP_TILE) {
            const int r = e / WT, w = e % WT;
            rj[r * LW + w] = (r < jn && w < words) ? cells[(j0 + r) * words + w] : T(0);
        }
    }
    if (t == 0) s_n = 0;
    __syncthreads();
    const int64_t i = i0 + t;
    const bool own = i < n;
    uint16_t di[AP_MAX_REFS];
    for (int d = 0; d < AP_MAX_REFS; ++d) di[d] = (own && d < h) ? D[static_cast<int64_t>(d) * ncap + i] : 0;
    T xi[WT > 0 ? WT : 1];
    if (WT > 0) {
#pragma unroll
        for (int w = 0; w < (WT > 0 ? WT : 1); ++w) xi[w] = (own && w < words) ? cells[i * words + w] : T(0);
    }
    const T *xg = cells + (own ? i : 0) * words;
    // j > i: in the diagonal tile only cells after i; lanes past the end idle
    const int jstart = (I == J) ? t + 1 : 0;
    for (int jj = 0; jj < jn; ++jj) {
        bool ok = own && jj >= jstart;
        for (int d = 0; d < h; ++d) {
            const int a = di[d], c = dj[d][jj];
            ok = ok && ((a - c == 1) || (c - a == 1));
        }
        int pos = 0;
        bool hit = false;
        if (ok) {
            if (WT > 0) {
                int dd = 0, first = -1;
#pragma unroll
                for (int w = 0; w < (WT > 0 ? WT : 1); ++w) {
                    const T x = xi[w] ^ rj[jj * LW + w];
                    dd += popc<T>(x);
                    first = (x && first < 0) ? w * B + clz_t<T>(x) : first;
                }
                hit = dd == 1;
                pos = first;
            } else {
                hit = dist_upto2<T>(xg, cells + (j0 + jj) * words, words, &pos) == 1;
            }
        }
        if (hit) {
            if (B == 64)
                atomicOr(reinterpret_cast<unsigned long long *>(mask + i * words + pos / B),
                         static_cast<unsigned long long>(bitmask_of<T>(pos)));
            else
                atomicOr(reinterpret_cast<unsigned int *>(mask + i * words + pos / B),
                         static_cast<unsigned int>(bitmask_of<T>(pos)));
        }
        const uint64_t hm = ballot64(hit);
        if (hm) {  // one LDS counter update per wave; past the stash, one global reservation per wave
            uint32_t rb = 0;
            if (lane == 0) rb = atomicAdd(&s_n, static_cast<uint32_t>(__popcll(hm)));
            rb = __shfl(rb, 0, 64);
            const uint32_t r = rb + static_cast<uint32_t>(__popcll(hm & lanemask_lt()));
            const uint4 e = make_uint4(static_cast<uint32_t>(i), static_cast<uint32_t>(j0 + jj),
                                       static_cast<uint32_t>(pos), 0u);
            const bool in_stash = r < static_cast<uint32_t>(AP_STASH);
            const uint64_t om = ballot64(hit && !in_stash);
            if (hit && in_stash) stash[r] = e;
            if (om) {
                unsigned long long g = 0;
                if (lane == 0) g = atomicAdd(cursor, static_cast<unsigned long long>(__popcll(om)));
                g = shfl_u64(g, 0);
                if (hit && !in_stash) {
                    const unsigned long long k = g + static_cast<unsigned long long>(__popcll(om & lanemask_lt()));
                    if (static_cast<int64_t>(k) < list_cap) list[k] = e;
                }
            }
        }
    }
    __syncthreads();
    const uint32_t m = s_n < static_cast<uint32_t>(AP_STASH) ? s_n : static_cast<uint32_t>(AP_STASH);
    if (t == 0) s_base = m ? atomicAdd(cursor, static_cast<unsigned long long>(m)) : 0ull;
    __syncthreads();
    for (uint32_t r = t; r < m; r += AP_TILE) {
        const unsigned long long k = s_base + r;
        if (static_cast<int64_t>(k) < list_cap) list[k] = stash[r];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_place(const uint4 *__restrict__ list, const unsigned long long *cursor,
                                               int64_t list_cap, const T *__restrict__ mask, int words,
                                               const int64_t *__restrict__ offsets, uint32_t *__restrict__ uv,
                                               uint16_t *__restrict__ bit, int64_t cap) {
    constexpr int B = Bits<T>::B;
    int64_t cnt = static_cast<int64_t>(*cursor);
    if (cnt > list_cap) cnt = list_cap;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < cnt;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const uint4 r = list[e];
        const int k = static_cast<int>(r.z);
        const T *m = mask + static_cast<int64_t>(r.x) * words;
        const int kw = k / B;
        // neighbours of u with a larger position come first (smaller v)
        const T below = static_cast<T>(bitmask_of<T>(k) - T(1));
        int rank = popc<T>(m[kw] & below);
        for (int w = kw + 1; w < words; ++w) rank += popc<T>(m[w]);
        const int64_t pos = offsets[r.x] + rank;
        if (pos < cap) {
            uv[2 * pos] = r.x;
            uv[2 * pos + 1] = r.y;
            if (bit) bit[pos] = static_cast<uint16_t>(k);
        }
    }
}

__global__ void k_status_ap(const int64_t *total, int64_t cap, int32_t *status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *status = (*total > cap) ? CG_ECAPACITY : CG_OK;
}

struct ApWs {
    uint16_t *D;
    void *mask;
    uint4 *list;
    unsigned long long *cursor;
    int64_t *offsets;
    uint64_t *tile_sums;
};

ApWs carve_ap(void *base, const cg_dict &d, int64_t cap, size_t *bytes) {
    Carver c(base);
    ApWs w{};
    const int64_t n = d.ncells_cap > 0 ? d.ncells_cap : 1;
    const int h = d.params.n_refs > 0 ? d.params.n_refs : 1;
    w.D = c.take<uint16_t>(static_cast<size_t>(h) * n);
    w.mask = c.take<char>(static_cast<size_t>(n) * d.lay.words * (d.lay.word_bits / 8));
    w.list = c.take<uint4>(cap > 0 ? cap : 1);
    w.cursor = c.take<unsigned long long>(1);
    w.offsets = c.take<int64_t>(n + 1);
    w.tile_sums = c.take<uint64_t>(scan_tiles(n));
    *bytes = c.bytes();
    return w;
}

template <typename T>
cg_status ap_impl(const cg_dict &d, uint32_t *uv, uint16_t *bit, int64_t cap, int64_t *d_nedges,
                  int64_t *d_offsets, void *ws, int32_t *d_status, hipStream_t s) {
    size_t b;
    ApWs w = carve_ap(ws, d, cap, &b);
    const int64_t ncap = d.ncells_cap;
    const int words = d.lay.words;
    const int h = d.params.n_refs;
    const T *cells = static_cast<const T *>(d.cells);
    int64_t *offsets = d_offsets ? d_offsets : w.offsets;
    const int64_t mask_words = (ncap > 0 ? ncap : 1) * words;
    if (sizeof(T) == 8) CG_TRY(fill_i64(static_cast<int64_t *>(w.mask), 0, mask_words, s));
    else CG_TRY(fill_u32(static_cast<uint32_t *>(w.mask), 0, mask_words, s));
    CG_TRY(fill_i64(reinterpret_cast<int64_t *>(w.cursor), 0, 1, s));
    if (ncap > 0) {
        if (h > 0) {
            hipLaunchKernelGGL((k_ref_dists<T>), dim3(blocks_for(ncap, 256, 16384)), dim3(256), 0, s, cells,
                               d.d_ncells, ncap, words, h, w.D);
            CG_LAUNCHED("allpairs_ref_dists");
        }
        const int64_t tiles = (ncap + AP_TILE - 1) / AP_TILE;
        const int64_t pairs = tiles * (tiles + 1) / 2;
        if (pairs > 0x7fffffffLL) return set_error(CG_EUNSUPPORTED, "all-pairs path: %lld cells is too many", (long long)ncap);
        int wt = 1;
        while (wt < words) wt <<= 1;
        const int wcap = sizeof(T) == 8 ? 16 : 32;  // rows of up to 1024 bits are staged in LDS
        const dim3 grid(static_cast<unsigned>(pairs));
        T *mk = static_cast<T *>(w.mask);
#define CG_AP(WTV)                                                                                                 \
    hipLaunchKernelGGL((k_allpairs<T, WTV>), grid, dim3(AP_TILE), static_cast<size_t>(AP_TILE) * ((WTV) + 1) * sizeof(T), s, \
                       cells, d.d_ncells, ncap, words, h, w.D, mk, w.list, w.cursor, cap)
        if (wt > wcap) {
            CG_AP(0);
        } else {
            switch (wt) {
            case 1: CG_AP(1); break;
            case 2: CG_AP(2); break;
            case 4: CG_AP(4); break;
            case 8: CG_AP(8); break;
            case 16: CG_AP(16); break;
            default: CG_AP(32); break;
            }
        }
#undef CG_AP
        CG_LAUNCHED("allpairs_pairs");
    }
    CG_TRY(scan_rowpop_to_i64(w.mask, d.lay.word_bits, words, offsets, ncap, d.d_ncells, w.tile_sums, d_nedges, s));
    if (ncap == 0) {
        CG_TRY(fill_i64(d_nedges, 0, 1, s));
        CG_TRY(fill_i64(offsets, 0, 1, s));
    }
    hipLaunchKernelGGL(k_status_ap, dim3(1), dim3(64), 0, s, d_nedges, cap, d_status);
    CG_LAUNCHED("allpairs_status");
    if (cap > 0) {
        hipLaunchKernelGGL((k_place<T>), dim3(blocks_for(cap, 256, 16384)), dim3(256), 0, s, w.list, w.cursor, cap,
                           static_cast<const T *>(w.mask), words, offsets, uv, bit, cap);
        CG_LAUNCHED("allpairs_place");
    }
    return CG_OK;
}

}  // namespace

size_t allpairs_workspace_bytes(const cg_dict &d, int64_t cap) {
    size_t b;
    carve_ap(nullptr, d, cap, &b);
    return b;
}

cg_status run_edges_allpairs(const cg_dict &d, uint32_t *uv, uint16_t *bit, int64_t cap, int64_t *d_nedges,
                             int64_t *d_offsets, void *ws, size_t ws_bytes, int32_t *d_status, hipStream_t s) {
    (void)ws_bytes;
    if (d.lay.word_bits == 64) return ap_impl<uint64_t>(d, uv, bit, cap, d_nedges, d_offsets, ws, d_status, s);
    return ap_impl<uint32_t>(d, uv, bit, cap, d_nedges, d_offsets, ws, d_status, s);
}

}  // namespace cg
