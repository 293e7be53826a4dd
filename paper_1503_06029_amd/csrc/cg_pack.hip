// Pack: n x l sign bytes -> n packed rows (Section 2.1: bit i of a point's
// vector is 1 iff the point satisfies constraint c_i; a nonzero byte is 1).
//
// One thread per 16-column chunk of a row.  Consecutive threads own
// consecutive chunks, so a wave reads 1 KiB of contiguous sign bytes with
// 16-byte loads when rows are dense (row_stride == l, 16-byte aligned), and
// writes 128 contiguous bytes of packed words as 16-bit pieces.  A chunk's
// 16 bits land most-significant-first: chunk c of a row is the 16-bit piece
// (c mod q) of word c / q (q = word_bits / 16) counted from the top.
#include "cg_internal.hpp"

namespace cg {

namespace {

__device__ __forceinline__ uint32_t nz_bits_be(uint32_t x) {
    // bits (3..0) <- bytes (0..3) nonzero, byte 0 (lowest address) first
    uint32_t r = 0;
    r |= ((x & 0x000000ffu) != 0) << 3;
    r |= ((x & 0x0000ff00u) != 0) << 2;
    r |= ((x & 0x00ff0000u) != 0) << 1;
    r |= ((x & 0xff000000u) != 0) << 0;
    return r;
}

__global__ void __launch_bounds__(256) k_pack(const uint8_t *__restrict__ bits, int64_t n, int64_t row_stride,
                                              int ell, int word_bits, int words, uint16_t *__restrict__ out,
                                              bool vec_ok) {
    const int q = word_bits / 16;
    const int chunks = words * q;
    const int64_t total = n * chunks;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t r = g / chunks;
        const int c = static_cast<int>(g - r * chunks);
        const int col = c * 16;
        uint32_t v = 0;
        if (col < ell) {
            const uint8_t *src = bits + r * row_stride + col;
            if (vec_ok && col + 16 <= ell) {
                uint4 x = *reinterpret_cast<const uint4 *>(src);
                v = (nz_bits_be(x.x) << 12) | (nz_bits_be(x.y) << 8) | (nz_bits_be(x.z) << 4) | nz_bits_be(x.w);
            } else {
                const int lim = ell - col < 16 ? ell - col : 16;
                for (int j = 0; j < lim; ++j) v |= static_cast<uint32_t>(src[j] != 0) << (15 - j);
            }
        }
        // little-endian words: the top 16 bits of a word are its last 16-bit piece
        const int w = c / q, piece = c - w * q;
        const int64_t half = r * (static_cast<int64_t>(words) * q) + static_cast<int64_t>(w) * q + (q - 1 - piece);
        out[half] = static_cast<uint16_t>(v);
    }
}

}  // namespace

cg_status launch_pack(const uint8_t *bits, int64_t n, int64_t row_stride, cg_layout lay, void *out,
                      hipStream_t s) {
    if (n == 0) return CG_OK;
    const bool vec_ok = (row_stride % 16 == 0) && ((reinterpret_cast<uintptr_t>(bits) & 15) == 0);
    const int64_t total = n * static_cast<int64_t>(lay.words) * (lay.word_bits / 16);
    hipLaunchKernelGGL(k_pack, dim3(blocks_for(total, 256, 1 << 20)), dim3(256), 0, s, bits, n, row_stride,
                       lay.ell, lay.word_bits, lay.words, static_cast<uint16_t *>(out), vec_ok);
    CG_LAUNCHED("pack");
    return CG_OK;
}

}  // namespace cg
