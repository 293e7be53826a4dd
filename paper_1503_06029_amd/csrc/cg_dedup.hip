// Dedup: sort the packed rows lexicographically and drop duplicates
// (Section 3.2: radix sort of X with duplicate removal; Section 2.2: X may be
// a multiset).
//
// 1. extract: key = the first 64 bits of each row (x(0) most significant),
//    value = row index;
// 2. LSD radix sort of (key, index) over the key bits that can be nonzero;
// 3. rows with equal keys form segments; when l > 64 each segment of two or
//    more rows is ordered by the full row: segments of up to `smax` rows by
//    one wave each (rank sort in LDS), longer ones by one block each (bitonic
//    network over an index array in global memory);
// 4. a row is a new cell iff it differs from its predecessor; a scan of those
//    flags gives cell ids, and a gather writes the cells and row_to_cell.
#include "cg_internal.hpp"

namespace cg {

namespace {

constexpr uint32_t SENT = 0xFFFFFFFFu;
constexpr int SMALL_WAVES = 4;
constexpr int SMALL_LDS_PER_WAVE = 16384;

template <typename T>
__global__ void __launch_bounds__(256) k_extract(const T *__restrict__ rows, int64_t n, int words,
                                                 uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < n;
         j += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        keys[j] = head64<T>(rows + j * words, words);
        vals[j] = static_cast<uint32_t>(j);
    }
}

// End of the run of keys equal to keys[j] (keys sorted ascending): the first
// index e > j with keys[e] != keys[j], or n.
__device__ __forceinline__ int64_t run_end(const uint64_t *keys, int64_t j, int64_t n) {
    const uint64_t k = keys[j];
    int64_t good = j, bad = j + 1, step = 1;
    while (bad < n && keys[bad] == k) {
        good = bad;
        step <<= 1;
        bad = j + step;
    }
    if (bad > n) bad = n;
    // keys[good] == k, and bad == n or keys[bad] != k
    while (bad - good > 1) {
        const int64_t m = good + ((bad - good) >> 1);
        if (keys[m] == k) good = m; else bad = m;
    }
    return bad;
}

__global__ void __launch_bounds__(256) k_heads(const uint64_t *__restrict__ keys, int64_t n, bool tiefix,
                                               int smax, uint8_t *__restrict__ uniq, uint2 *small_list,
                                               uint2 *large_list, uint32_t *counters) {
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < n;
         j += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const bool head = (j == 0) || keys[j] != keys[j - 1];
        uniq[j] = head ? 1 : 0;
        if (tiefix && head) {
            const int64_t e = run_end(keys, j, n);
            const int64_t len = e - j;
            if (len >= 2) {
                uint2 seg = make_uint2(static_cast<uint32_t>(j), static_cast<uint32_t>(len));
                if (len <= smax) small_list[atomicAdd(&counters[0], 1u)] = seg;
                else large_list[atomicAdd(&counters[1], 1u)] = seg;
            }
        }
    }
}

// One wave per segment of 2..smax rows: rank sort by the full row in LDS.
template <typename T>
__global__ void __launch_bounds__(256) k_tiefix_small(const T *__restrict__ rows, int words, int from,
                                                      int lds_stride, int smax, const uint2 *__restrict__ list,
                                                      const uint32_t *__restrict__ counters,
                                                      uint32_t *__restrict__ vals, uint8_t *__restrict__ uniq) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    T *lds = reinterpret_cast<T *>(smem) + static_cast<size_t>(wave) * smax * lds_stride;
    const uint32_t count = counters[0];
    const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
    for (uint32_t s = blockIdx.x * (blockDim.x >> 6) + wave; s < count; s += nwaves) {
        const uint2 seg = list[s];
        const int64_t a = seg.x;
        const int len = static_cast<int>(seg.y);
        uint32_t myval = lane < len ? vals[a + lane] : 0u;
        // cooperative copy of the segment's rows into LDS (all lanes take part
        // in every shuffle; only in-range slots are stored)
        const int total = len * words;
        for (int i0 = 0; i0 < total; i0 += 64) {
            const int i = i0 + lane;
            const int r = i < total ? i / words : 0;
            const uint32_t src = static_cast<uint32_t>(__shfl(static_cast<int>(myval), r, 64));
            if (i < total) lds[r * lds_stride + (i - r * words)] = rows[static_cast<int64_t>(src) * words + (i - r * words)];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < len) {
            const T *me = lds + lane * lds_stride;
            int rank = 0;
            bool dup = false;
            for (int j = 0; j < len; ++j) {
                if (j == lane) continue;
                const int c = row_cmp<T>(lds + j * lds_stride, me, words, from);
                if (c < 0 || (c == 0 && j < lane)) ++rank;
                if (c == 0 && j < lane) dup = true;
            }
            vals[a + rank] = myval;
            uniq[a + rank] = dup ? 0 : 1;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

template <typename T>
__device__ __forceinline__ bool idx_less(const T *rows, int words, int from, uint32_t x, uint32_t y) {
    if (x == SENT) return false;
    if (y == SENT) return true;
    const int c = row_cmp<T>(rows + static_cast<int64_t>(x) * words, rows + static_cast<int64_t>(y) * words,
                             words, from);
    return c < 0 || (c == 0 && x < y);
}

// One block per long segment: bitonic network over its index array, kept in
// global scratch at [2a, 2a + P), P = next power of two >= len.
template <typename T>
__global__ void __launch_bounds__(256) k_tiefix_large(const T *__restrict__ rows, int words, int from,
                                                      const uint2 *__restrict__ list,
                                                      const uint32_t *__restrict__ counters, uint32_t *vals,
                                                      uint8_t *uniq, uint32_t *scratch) {
    const uint32_t count = counters[1];
    for (uint32_t s = blockIdx.x; s < count; s += gridDim.x) {
        const uint2 seg = list[s];
        const int64_t a = seg.x;
        const int64_t len = seg.y;
        int64_t P = 1;
        while (P < len) P <<= 1;
        uint32_t *scr = scratch + 2 * a;
        for (int64_t i = threadIdx.x; i < P; i += blockDim.x) scr[i] = i < len ? vals[a + i] : SENT;
        __syncthreads();
        for (int64_t k = 2; k <= P; k <<= 1) {
            for (int64_t j = k >> 1; j > 0; j >>= 1) {
                for (int64_t i = threadIdx.x; i < P; i += blockDim.x) {
                    const int64_t p = i ^ j;
                    if (p > i) {
                        const uint32_t x = scr[i], y = scr[p];
                        const bool asc = (i & k) == 0;
                        const bool swap = asc ? idx_less<T>(rows, words, from, y, x)
                                              : idx_less<T>(rows, words, from, x, y);
                        if (swap) { scr[i] = y; scr[p] = x; }
                    }
                }
                __syncthreads();
            }
        }
        for (int64_t i = threadIdx.x; i < len; i += blockDim.x) {
            const uint32_t x = scr[i];
            vals[a + i] = x;
            bool u = true;
            if (i > 0) {
                const uint32_t y = scr[i - 1];
                u = row_cmp<T>(rows + static_cast<int64_t>(x) * words, rows + static_cast<int64_t>(y) * words,
                               words, from) != 0;
            }
            uniq[a + i] = u ? 1 : 0;
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_gather(const T *__restrict__ rows, int64_t n, int words,
                                                const uint32_t *__restrict__ vals, const uint8_t *__restrict__ uniq,
                                                const uint32_t *__restrict__ cidx, T *__restrict__ cells,
                                                uint32_t *__restrict__ row_to_cell) {
    const int64_t total = n * words;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t j = g / words;
        const int w = static_cast<int>(g - j * words);
        const uint32_t u = uniq[j];
        const uint32_t cid = cidx[j] + u - 1;
        const uint32_t src = vals[j];
        if (u) cells[static_cast<int64_t>(cid) * words + w] = rows[static_cast<int64_t>(src) * words + w];
        if (w == 0 && row_to_cell) row_to_cell[src] = cid;
    }
}

struct DedupWs {
    uint64_t *keys[2];
    uint32_t *vals[2];
    uint32_t *hist;
    uint64_t *tile_sums;
    uint8_t *uniq;
    uint32_t *cidx;
    uint2 *small_list, *large_list;
    uint32_t *counters;
    uint32_t *scratch;
};

DedupWs carve_dedup(void *base, int64_t n, cg_layout lay, size_t *bytes) {
    Carver c(base);
    DedupWs w{};
    const int64_t m = n > 0 ? n : 1;
    w.keys[0] = c.take<uint64_t>(m);
    w.keys[1] = c.take<uint64_t>(m);
    w.vals[0] = c.take<uint32_t>(m);
    w.vals[1] = c.take<uint32_t>(m);
    w.hist = c.take<uint32_t>(radix_hist_entries(m));
    int64_t ts = scan_tiles(m);
    int64_t ts2 = scan_tiles(radix_hist_entries(m));
    w.tile_sums = c.take<uint64_t>(ts > ts2 ? ts : ts2);
    w.uniq = c.take<uint8_t>(m);
    w.cidx = c.take<uint32_t>(m);
    w.counters = c.take<uint32_t>(4);
    if (lay.ell > 64) {
        w.small_list = c.take<uint2>(m / 2 + 1);
        w.large_list = c.take<uint2>(m / 2 + 1);
        w.scratch = c.take<uint32_t>(2 * m);
    }
    *bytes = c.bytes();
    return w;
}

template <typename T>
cg_status dedup_impl(const T *rows, int64_t n, cg_layout lay, T *cells, uint32_t *row_to_cell, int64_t *d_ncells,
                     void *ws, hipStream_t s) {
    size_t bytes;
    DedupWs w = carve_dedup(ws, n, lay, &bytes);
    const int words = lay.words;
    if (n == 0) return fill_i64(d_ncells, 0, 1, s);

    hipLaunchKernelGGL((k_extract<T>), dim3(blocks_for(n, 256, 16384)), dim3(256), 0, s, rows, n, words,
                       w.keys[0], w.vals[0]);
    CG_LAUNCHED("dedup_extract");

    const int sig = lay.ell < 64 ? lay.ell : 64;  // key bits that can be nonzero: [64 - sig, 64)
    const int lo = ((64 - sig) / 8) * 8;
    int which = 0;
    CG_TRY(radix_sort_u64(w.keys, w.vals, n, nullptr, lo, 64, w.hist, w.tile_sums, &which, s));
    uint64_t *keys = w.keys[which];
    uint32_t *vals = w.vals[which];

    const bool tiefix = lay.ell > 64;
    const int B = static_cast<int>(sizeof(T) * 8);
    const int from = 64 / B;  // words covered by the sort key
    int lds_stride = words + ((words % 2 == 0) ? 1 : 0);
    int smax = 0;
    if (tiefix) {
        const int64_t per_row = static_cast<int64_t>(lds_stride) * sizeof(T);
        smax = static_cast<int>(SMALL_LDS_PER_WAVE / per_row);
        if (smax > 64) smax = 64;
        CG_TRY(fill_u32(w.counters, 0, 4, s));
    }
    hipLaunchKernelGGL(k_heads, dim3(blocks_for(n, 256, 16384)), dim3(256), 0, s, keys, n, tiefix,
                       smax < 2 ? 1 : smax, w.uniq, w.small_list, w.large_list, w.counters);
    CG_LAUNCHED("dedup_heads");
    if (tiefix) {
        if (smax >= 2) {
            const size_t lds = static_cast<size_t>(SMALL_WAVES) * smax * lds_stride * sizeof(T);
            hipLaunchKernelGGL((k_tiefix_small<T>), dim3(blocks_for(n / 2 + 1, SMALL_WAVES, 2048)),
                               dim3(64 * SMALL_WAVES), lds, s, rows, words, from, lds_stride, smax, w.small_list,
                               w.counters, vals, w.uniq);
            CG_LAUNCHED("dedup_tiefix_small");
        }
        hipLaunchKernelGGL((k_tiefix_large<T>), dim3(256), dim3(256), 0, s, rows, words, from, w.large_list,
                           w.counters, vals, w.uniq, w.scratch);
        CG_LAUNCHED("dedup_tiefix_large");
    }
    CG_TRY(scan_u8_to_u32(w.uniq, w.cidx, n, nullptr, w.tile_sums, d_ncells, s));
    hipLaunchKernelGGL((k_gather<T>), dim3(blocks_for(n * words, 256, 65536)), dim3(256), 0, s, rows, n, words,
                       vals, w.uniq, w.cidx, cells, row_to_cell);
    CG_LAUNCHED("dedup_gather");
    return CG_OK;
}

}  // namespace

size_t dedup_workspace_bytes(int64_t n, cg_layout lay) {
    size_t b;
    carve_dedup(nullptr, n, lay, &b);
    return b;
}

cg_status run_dedup(const void *rows, int64_t n, cg_layout lay, void *cells, uint32_t *row_to_cell,
                    int64_t *d_ncells, void *ws, size_t ws_bytes, hipStream_t s) {
    (void)ws_bytes;
    if (lay.word_bits == 64)
        return dedup_impl<uint64_t>(static_cast<const uint64_t *>(rows), n, lay, static_cast<uint64_t *>(cells),
                                    row_to_cell, d_ncells, ws, s);
    return dedup_impl<uint32_t>(static_cast<const uint32_t *>(rows), n, lay, static_cast<uint32_t *>(cells),
                                row_to_cell, d_ncells, ws, s);
}

}  // namespace cg
