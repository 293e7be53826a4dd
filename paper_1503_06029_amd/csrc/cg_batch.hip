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

// One thread per (virtual row, 32-bit word): word 0 is the scene tag, word w
// >= 1 packs columns 32 (w - 1) .. 32 w - 1 of the scene's row, MSB first.
// The 32 bytes are read as aligned 4-byte words (those lying wholly inside
// the scene's bytes; the others byte by byte) and aligned with alignbyte.
// A block takes one contiguous chunk of (row, word) elements: one binary
// search for the scene of its first row, after which each thread steps its
// own scene index forward as its rows advance (a chunk spans a few scene
// boundaries at most), so no load chain precedes each step's work.
__global__ void __launch_bounds__(256) k_batch_pack(const uint8_t *__restrict__ bits,
                                                    const int64_t *__restrict__ bits_off,
                                                    const int32_t *__restrict__ scene_ell,
                                                    const int64_t *__restrict__ scene_rows, int n_scenes,
                                                    int64_t n_rows, int words, int64_t chunk,
                                                    uint32_t *__restrict__ out) {
    __shared__ int s_j0;
    const int64_t total = n_rows * words;
    const bool aligned = (reinterpret_cast<uintptr_t>(bits) & 3) == 0;
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t c1 = c0 + chunk < total ? c0 + chunk : total;
    if (c0 >= total) return;
    if (threadIdx.x == 0) s_j0 = scene_of(scene_rows, n_scenes, c0 / words);
    __syncthreads();
    int j = s_j0;
    for (int64_t g0 = c0; g0 < c1; g0 += blockDim.x) {
        const int64_t g = g0 + threadIdx.x;
        if (g >= c1) break;
        const int64_t r = g / words;
        const int w = static_cast<int>(g - r * words);
        while (j + 1 < n_scenes && scene_rows[j + 1] <= r) ++j;
        uint32_t v;
        if (w == 0) {
            v = (static_cast<uint32_t>(j) << 16) | static_cast<uint32_t>(j);
        } else {
            const int ell = scene_ell[j];
            const int col0 = (w - 1) * 32;
            v = 0;
            if (col0 < ell) {
                const int64_t s0 = bits_off[j];
                const int64_t s1 = s0 + (scene_rows[j + 1] - scene_rows[j]) * ell;  // end of the scene's bytes
                const int64_t A = s0 + (r - scene_rows[j]) * ell + col0;
                const int lim = ell - col0 < 32 ? ell - col0 : 32;
                if (aligned) {
                    const int64_t A4 = A & ~int64_t(3);
                    const int off = static_cast<int>(A - A4);
                    uint32_t wd[9];
#pragma unroll
                    for (int k = 0; k < 9; ++k) {
                        const int64_t p = A4 + 4 * k;
                        if (p >= A + lim) {
                            wd[k] = 0;
                        } else if (p >= s0 && p + 4 <= s1) {
                            wd[k] = *reinterpret_cast<const uint32_t *>(bits + p);
                        } else {
                            uint32_t x = 0;
                            for (int b = 0; b < 4; ++b)
                                if (p + b >= s0 && p + b < s1) x |= static_cast<uint32_t>(bits[p + b]) << (8 * b);
                            wd[k] = x;
                        }
                    }
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const uint32_t x = __builtin_amdgcn_alignbyte(wd[k + 1], wd[k], static_cast<uint32_t>(off));
                        v |= nibble_of(x) << (28 - 4 * k);
                    }
                    if (lim < 32) v &= ~0u << (32 - lim);
                } else {
                    const uint8_t *src = bits + A;
                    for (int c = 0; c < lim; ++c) v |= static_cast<uint32_t>(src[c] != 0) << (31 - c);
                }
            }
        }
        out[g] = v;
    }
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
    const int64_t total = n_rows * lay.words;
    // chunks of whole 256-element steps, at most 8,192 blocks
    const int64_t nb = blocks_for(total, 256, 8192);
    const int64_t chunk = ((total + nb - 1) / nb + 255) / 256 * 256;
    hipLaunchKernelGGL(k_batch_pack, dim3(blocks_for(total, chunk)), dim3(256), 0, s, bits, bits_off, scene_ell,
                       scene_rows, n_scenes, n_rows, lay.words, chunk, static_cast<uint32_t *>(out));
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
