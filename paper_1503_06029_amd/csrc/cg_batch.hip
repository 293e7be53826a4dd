// Batched scenes: many independent scenes packed into one virtual scene
// whose word 0 carries the scene number twice, so the ordinary dedup,
// dictionary and edge passes run on all of them at once; then the result is
// split back into per-scene slices with scene-local ids.
#include "cg_internal.hpp"

namespace cg {

namespace {

constexpr int MAX_SCENES = 65536;

// Index j with rows[j] <= r < rows[j + 1] (rows ascending, rows[0] = 0).
__device__ __forceinline__ int scene_of(const int64_t *rows, int n_scenes, int64_t r) {
    int lo = 0, hi = n_scenes;  // answer in [lo, hi)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rows[mid] <= r) lo = mid; else hi = mid;
    }
    return lo;
}

// Sign bytes -> 32 column bits, MSB first: x holds 4 bytes (lowest address in
// the low byte); the result's top nibble has one bit per byte (set iff the
// byte is nonzero), the lowest-addressed byte most significant.
__device__ __forceinline__ uint32_t nibble_of(uint32_t x) {
    uint32_t y = x | (x >> 4);
    y |= y >> 2;
    y |= y >> 1;
    y &= 0x01010101u;
    return (y * 0x80402010u) >> 28;  // byte b's flag lands on bit 31 - b, nothing carries into 28..31
}

// Sign bytes of one 32-byte column group at LDS byte address A (any
// alignment; lim <= 32 valid bytes) -> the packed word, MSB first.
__device__ __forceinline__ uint32_t pack32_lds(const uint8_t *lds, int A, int lim) {
    const int A4 = A & ~3, off = A & 3;
    uint32_t wd[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) wd[k] = *reinterpret_cast<const uint32_t *>(lds + A4 + 4 * k);
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t x = __builtin_amdgcn_alignbyte(wd[k + 1], wd[k], static_cast<uint32_t>(off));
        v |= nibble_of(x) << (28 - 4 * k);
    }
    return lim < 32 ? v & (~0u << (32 - lim)) : v;
}

// A block packs PR consecutive virtual rows.  Their scenes' sign bytes are
// contiguous per scene (row r of scene j at bits_off[j] + r l_j), so the
// block first copies each scene's share of its rows into LDS with aligned
// 16-byte loads (only the first and last piece of a share, where it may
// reach outside the scene's bytes, go byte by byte), then packs: one thread
// per (row, word), word 0 the scene tag, word w >= 1 columns 32 (w - 1) ..
// 32 w - 1 read from LDS.  Global reads are whole 16-byte pieces of one
// contiguous stream; the scene search is done once per block.  A scene with
// l beyond the layout's RB = 32 (words - 1) bytes (refused by the host
// check) has only its first RB bytes per row copied, byte by byte.
__global__ void __launch_bounds__(256) k_batch_pack(const uint8_t *__restrict__ bits,
                                                    const int64_t *__restrict__ bits_off,
                                                    const int32_t *__restrict__ scene_ell,
                                                    const int64_t *__restrict__ scene_rows, int n_scenes,
                                                    int64_t n_rows, int words, int PR, uint32_t *__restrict__ out) {
    extern __shared__ __align__(16) unsigned char smem[];
    // per segment (one scene's share of the block's rows): first row, l, LDS
    // byte offset of its first row, scene; per row: its segment
    int *seg_row0 = reinterpret_cast<int *>(smem);
    int *seg_ell = seg_row0 + PR;
    int *seg_off = seg_ell + PR;
    int *seg_j = seg_off + PR;
    uint16_t *row_seg = reinterpret_cast<uint16_t *>(seg_j + PR);
    uint8_t *lb = reinterpret_cast<uint8_t *>(smem) + ((16 * PR + 2 * PR + 15) & ~15);
    __shared__ int s_nseg;
    const int RB = 32 * (words - 1);
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * PR;
    const int nr = static_cast<int>(n_rows - r0 < PR ? n_rows - r0 : PR);
    const int t = threadIdx.x;
    if (t == 0) {
        int j = scene_of(scene_rows, n_scenes, r0);
        int ns = 0, off = 0;
        for (; j < n_scenes && scene_rows[j] < r0 + nr; ++j) {
            const int64_t a = scene_rows[j] > r0 ? scene_rows[j] : r0;
            const int64_t b = scene_rows[j + 1] < r0 + nr ? scene_rows[j + 1] : r0 + nr;
            if (b <= a) continue;  // an empty scene
            const int ell = scene_ell[j];
            const int rb = ell < RB ? ell : RB;
            seg_row0[ns] = static_cast<int>(a - r0);
            seg_ell[ns] = ell;
            // keep the global stream's address alignment mod 16 in LDS
            const int64_t g = bits_off[j] + (a - scene_rows[j]) * ell;
            seg_off[ns] = off + static_cast<int>(ell <= RB ? ((reinterpret_cast<uintptr_t>(bits) + g) & 15) : 0);
            seg_j[ns] = j;
            for (int64_t r = a; r < b; ++r) row_seg[r - r0] = static_cast<uint16_t>(ns);
            off += ((static_cast<int>(b - a) * rb + 16 + 15) & ~15) + 16;
            ++ns;
        }
        s_nseg = ns;
    }
    __syncthreads();
    const int nseg = s_nseg;
    for (int q = 0; q < nseg; ++q) {
        const int j = seg_j[q], ell = seg_ell[q];
        const int rs = seg_row0[q];
        const int re = q + 1 < nseg ? seg_row0[q + 1] : nr;
        const int64_t s0 = bits_off[j];
        const int64_t s1 = s0 + (scene_rows[j + 1] - scene_rows[j]) * ell;  // end of the scene's bytes
        const int64_t g0 = s0 + (r0 + rs - scene_rows[j]) * ell;
        uint8_t *dst = lb + seg_off[q];
        if (ell <= RB) {
            const int64_t nb = static_cast<int64_t>(re - rs) * ell;
            const int64_t a16 = g0 - static_cast<int64_t>((reinterpret_cast<uintptr_t>(bits) + g0) & 15);
            const int64_t nchunks = (g0 + nb - a16 + 15) >> 4;
            uint8_t *d16 = dst - (g0 - a16);  // LDS address of the aligned piece start
            for (int64_t c = t; c < nchunks; c += blockDim.x) {
                const int64_t p = a16 + 16 * c;
                if (p >= s0 && p + 16 <= s1) {
                    *reinterpret_cast<uint4 *>(d16 + 16 * c) = *reinterpret_cast<const uint4 *>(bits + p);
                } else {
                    for (int b = 0; b < 16; ++b)
                        if (p + b >= g0 && p + b < g0 + nb) d16[16 * c + b] = bits[p + b];
                }
            }
        } else {
            const int cnt = (re - rs) * RB;
            for (int e = t; e < cnt; e += blockDim.x) {
                const int rr = e / RB, col = e - rr * RB;
                dst[e] = bits[g0 + static_cast<int64_t>(rr) * ell + col];
            }
        }
    }
    __syncthreads();
    const int tot = nr * words;
    for (int e = t; e < tot; e += blockDim.x) {
        const int rr = e / words, w = e - rr * words;
        const int q = row_seg[rr];
        const int j = seg_j[q];
        uint32_t v;
        if (w == 0) {
            v = (static_cast<uint32_t>(j) << 16) | static_cast<uint32_t>(j);
        } else {
            const int ell = seg_ell[q];
            const int rb = ell < RB ? ell : RB;
            const int col0 = (w - 1) * 32;
            v = 0;
            if (col0 < rb) {
                const int lim = rb - col0 < 32 ? rb - col0 : 32;
                v = pack32_lds(lb, seg_off[q] + (rr - seg_row0[q]) * rb + col0, lim);
            }
        }
        out[(r0 + rr) * words + w] = v;
    }
}

// Rows per block of the batch pack and its LDS bytes: about 16 KB of sign
// bytes per block (more blocks per CU than 32 KB: 9.2 against 9.4 ms on the
// widest batch class).
static int batch_pack_rows(int words) {
    const int RB = 32 * (words - 1);
    int pr = 16384 / (RB > 0 ? RB : 32);
    if (pr > 256) pr = 256;
    if (pr < 16) pr = 16;
    return pr;
}
static size_t batch_pack_lds(int words, int pr) {
    const size_t RB = 32 * static_cast<size_t>(words - 1);
    // per-segment tables, then per segment its rows, alignment slack, 16
    // bytes of padding read past its end (at most pr segments)
    return ((16 * static_cast<size_t>(pr) + 2 * pr + 15) & ~size_t(15)) + pr * RB + pr * 48 + 64;
}

// cell_off[j] = first cell whose tag word is >= tag(j); edge_off[j] = its
// first edge.  One thread per scene boundary (j = 0 .. n_scenes).
__global__ void k_batch_bounds(const uint32_t *__restrict__ cells, const int64_t *d_ncells, int64_t ncap,
                               int words, int n_scenes, const int64_t *__restrict__ offsets,
                               int64_t *__restrict__ cell_off, int64_t *__restrict__ edge_off) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > n_scenes) return;
    const int64_t n = load_n(d_ncells, ncap);
    int64_t lo = 0, hi = n;
    if (j == n_scenes) {
        lo = n;
    } else {
        const uint32_t tag = (static_cast<uint32_t>(j) << 16) | static_cast<uint32_t>(j);
        while (lo < hi) {
            const int64_t mid = lo + ((hi - lo) >> 1);
            if (cells[mid * words] < tag) lo = mid + 1; else hi = mid;
        }
    }
    cell_off[j] = lo;
    edge_off[j] = offsets[lo];
}

// Rewrites edges (and bits) to scene-local ids / positions.
__global__ void __launch_bounds__(256) k_batch_local_edges(const int64_t *__restrict__ cell_off, int n_scenes,
                                                           const int64_t *__restrict__ d_nedges, int64_t cap,
                                                           uint32_t *__restrict__ uv, uint16_t *__restrict__ bit) {
    int64_t E = *d_nedges;
    if (E > cap) E = cap;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < E;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const uint32_t u = uv[2 * e];
        const int j = scene_of(cell_off, n_scenes, static_cast<int64_t>(u));
        const uint32_t base = static_cast<uint32_t>(cell_off[j]);
        uv[2 * e] = u - base;
        uv[2 * e + 1] -= base;
        if (bit) bit[e] = static_cast<uint16_t>(bit[e] - 32);
    }
}

__global__ void __launch_bounds__(256) k_batch_local_rows(const int64_t *__restrict__ cell_off,
                                                          const int64_t *__restrict__ scene_rows, int n_scenes,
                                                          int64_t n_rows, uint32_t *__restrict__ r2c) {
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < n_rows;
         r += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int j = scene_of(scene_rows, n_scenes, r);
        r2c[r] -= static_cast<uint32_t>(cell_off[j]);
    }
}

}  // namespace

cg_status batch_layout(int32_t ell_max, cg_layout *lay) {
    if (ell_max < 1 || ell_max > 65535 - 32) return set_error(CG_EINVAL, "cg_batch_layout: ell_max=%d", ell_max);
    const int32_t words = 1 + (ell_max + 31) / 32;
    *lay = cg_layout{32 * words, 32, words};
    return CG_OK;
}

cg_status run_batch_pack(const uint8_t *bits, const int64_t *bits_off, const int32_t *scene_ell,
                         const int64_t *scene_rows, int32_t n_scenes, int64_t n_rows, cg_layout lay, void *out,
                         hipStream_t s) {
    if (n_scenes < 0 || n_scenes > MAX_SCENES)
        return set_error(CG_EINVAL, "cg_batch_pack: n_scenes=%d out of 0..%d", n_scenes, MAX_SCENES);
    if (n_rows == 0) return CG_OK;
    const int pr = batch_pack_rows(lay.words);
    const size_t lds = batch_pack_lds(lay.words, pr);
    CG_TRY(allow_lds(reinterpret_cast<const void *>(&k_batch_pack), lds));
    hipLaunchKernelGGL(k_batch_pack, dim3(blocks_for(n_rows, pr)), dim3(256), lds, s, bits, bits_off, scene_ell,
                       scene_rows, n_scenes, n_rows, lay.words, pr, static_cast<uint32_t *>(out));
    CG_LAUNCHED("batch_pack");
    return CG_OK;
}

cg_status run_batch_split(const cg_dict &d, int32_t n_scenes, const int64_t *offsets, const int64_t *d_nedges,
                          int64_t cap, int64_t *cell_off, int64_t *edge_off, int32_t localize, uint32_t *uv,
                          uint16_t *bit, uint32_t *r2c, const int64_t *scene_rows, int64_t n_rows, hipStream_t s) {
    if (n_scenes < 0 || n_scenes > MAX_SCENES) return set_error(CG_EINVAL, "cg_batch_split: n_scenes=%d", n_scenes);
    hipLaunchKernelGGL(k_batch_bounds, dim3(blocks_for(n_scenes + 1, 256)), dim3(256), 0, s,
                       static_cast<const uint32_t *>(d.cells), d.d_ncells, d.ncells_cap, d.lay.words, n_scenes,
                       offsets, cell_off, edge_off);
    CG_LAUNCHED("batch_bounds");
    if (!localize) return CG_OK;
    if (cap > 0 && uv) {
        hipLaunchKernelGGL(k_batch_local_edges, dim3(blocks_for(cap, 256, 16384)), dim3(256), 0, s, cell_off,
                           n_scenes, d_nedges, cap, uv, bit);
        CG_LAUNCHED("batch_local_edges");
    }
    if (r2c && n_rows > 0) {
        hipLaunchKernelGGL(k_batch_local_rows, dim3(blocks_for(n_rows, 256, 16384)), dim3(256), 0, s, cell_off,
                           scene_rows, n_scenes, n_rows, r2c);
        CG_LAUNCHED("batch_local_rows");
    }
    return CG_OK;
}

}  // namespace cg
