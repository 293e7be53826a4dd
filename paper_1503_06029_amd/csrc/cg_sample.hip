// Sampling fused with packing: the step before the path.  Section 2.1: the
// sign vector of a sampled point P has bit i = 1 iff P satisfies constraint
// c_i; here the constraints are half-spaces a_i . p >= c_i of R^3 and the
// points are uniform in a box, drawn from a counter-based generator so that
// point i of a stream is a pure function of (seed, scene, i).  Bits go
// straight into packed words: no sign-byte matrix exists, in HBM or on the
// host.
//
// Generator: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC 2011), block
// i of key (seed, scene) = the point's three coordinates (the fourth word is
// unused).  Float contract, every operation rounded to nearest float64 with
// no fused multiply-add (contraction is switched off in the kernel):
//   u_j = (x_j >> 11) * 2^-53;   p_j = lo_j + (hi_j - lo_j) * u_j;
//   r_i = ((a_i0 * p0 + a_i1 * p1) + a_i2 * p2) - c_i;   bit i = (r_i >= 0).
#include "cg_internal.hpp"

namespace cg {

namespace {

// Ten rounds: words 0 and 2 times the round multipliers (128-bit products),
// halves recombined with words 1 and 3 and the key; the key advances by the
// two Weyl constants after every round.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
        const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

struct Box {
    double lo[3], hi[3];
};

// One thread per point; the planes are read with wave-uniform indices.
template <typename T>
__global__ void __launch_bounds__(256) k_sample_pack(const double *__restrict__ planes, int ell, int64_t n,
                                                     uint64_t seed, uint64_t scene, Box box, int words,
                                                     T *__restrict__ out) {
#pragma clang fp contract(off)
    constexpr int B = static_cast<int>(sizeof(T) * 8);
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t x[4] = {static_cast<uint64_t>(i), 0ull, 0ull, 0ull};
    philox4x64_10(x, seed, scene);
    double p[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double u = static_cast<double>(x[j] >> 11) * 0x1.0p-53;
        p[j] = box.lo[j] + (box.hi[j] - box.lo[j]) * u;
    }
    T *row = out + i * words;
    for (int w = 0; w < words; ++w) {
        const int k0 = w * B;
        const int kn = ell - k0 < B ? ell - k0 : B;
        T acc = 0;
        for (int b = 0; b < kn; ++b) {
            const double *a = planes + 4 * static_cast<int64_t>(k0 + b);
            const double s = (a[0] * p[0] + a[1] * p[1]) + a[2] * p[2];
            const double r = s - a[3];
            acc |= (r >= 0.0 ? T(1) : T(0)) << (B - 1 - b);
        }
        row[w] = acc;
    }
}

// Batched scenes: virtual row r belongs to the scene j with scene_rows[j] <=
// r < scene_rows[j + 1] and is that scene's point r - scene_rows[j], drawn
// with the scene's own key; word 0 is the scene tag (j << 16 | j), words
// 1 .. the scene's bits (32 planes per word, MSB first, zero past its l),
// the layout cg_batch_pack writes.  One block looks its first row's scene up
// by binary search; each thread walks on from there.
__global__ void __launch_bounds__(256) k_batch_sample_pack(const double *__restrict__ planes,
                                                           const int64_t *__restrict__ planes_off,
                                                           const int32_t *__restrict__ scene_ell,
                                                           const int64_t *__restrict__ scene_rows,
                                                           const uint64_t *__restrict__ keys, int n_scenes,
                                                           int64_t n_rows, Box box, int words,
                                                           uint32_t *__restrict__ out) {
#pragma clang fp contract(off)
    __shared__ int s_j0;
    for (int64_t r0 = static_cast<int64_t>(blockIdx.x) * blockDim.x; r0 < n_rows;
         r0 += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        __syncthreads();
        if (threadIdx.x == 0) {
            int lo = 0, hi = n_scenes;  // the scene of row r0: in [lo, hi)
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (scene_rows[mid] <= r0) lo = mid; else hi = mid;
            }
            s_j0 = lo;
        }
        __syncthreads();
        const int64_t r = r0 + threadIdx.x;
        if (r >= n_rows) continue;
        int j = s_j0;
        while (j + 1 < n_scenes && scene_rows[j + 1] <= r) ++j;
        const int64_t i = r - scene_rows[j];
        const int ell = scene_ell[j];
        const double *pl = planes + 4 * planes_off[j];
        uint64_t x[4] = {static_cast<uint64_t>(i), 0ull, 0ull, 0ull};
        philox4x64_10(x, keys[2 * j], keys[2 * j + 1]);
        double p[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double u = static_cast<double>(x[d] >> 11) * 0x1.0p-53;
            p[d] = box.lo[d] + (box.hi[d] - box.lo[d]) * u;
        }
        uint32_t *row = out + r * words;
        row[0] = (static_cast<uint32_t>(j) << 16) | static_cast<uint32_t>(j);
        for (int w = 1; w < words; ++w) {
            const int k0 = (w - 1) * 32;
            const int kn = ell - k0 < 32 ? ell - k0 : 32;
            uint32_t acc = 0;
            for (int b = 0; b < kn; ++b) {
                const double *a = pl + 4 * (k0 + b);
                const double sum = (a[0] * p[0] + a[1] * p[1]) + a[2] * p[2];
                const double res = sum - a[3];
                acc |= (res >= 0.0 ? 1u : 0u) << (31 - b);
            }
            row[w] = acc;
        }
    }
}

}  // namespace

cg_status run_batch_sample_pack(const double *planes, const int64_t *planes_off, const int32_t *scene_ell,
                                const int64_t *scene_rows, const uint64_t *keys, int32_t n_scenes, int64_t n_rows,
                                const double lohi[6], cg_layout lay, void *out, hipStream_t s) {
    if (n_rows == 0 || n_scenes == 0) return CG_OK;
    Box box;
    for (int j = 0; j < 3; ++j) {
        box.lo[j] = lohi[j];
        box.hi[j] = lohi[3 + j];
    }
    hipLaunchKernelGGL(k_batch_sample_pack, dim3(blocks_for(n_rows, 256, 1 << 20)), dim3(256), 0, s, planes,
                       planes_off, scene_ell, scene_rows, keys, n_scenes, n_rows, box, lay.words,
                       static_cast<uint32_t *>(out));
    CG_LAUNCHED("batch_sample_pack");
    return CG_OK;
}

cg_status run_sample_pack(const double *planes, int32_t ell, int64_t n, uint64_t seed, uint64_t scene,
                          const double lohi[6], cg_layout lay, void *out, hipStream_t s) {
    if (n == 0) return CG_OK;
    Box box;
    for (int j = 0; j < 3; ++j) {
        box.lo[j] = lohi[j];
        box.hi[j] = lohi[3 + j];
    }
    const unsigned blocks = blocks_for(n, 256);
    if (lay.word_bits == 64)
        hipLaunchKernelGGL((k_sample_pack<uint64_t>), dim3(blocks), dim3(256), 0, s, planes, ell, n, seed, scene, box,
                           lay.words, static_cast<uint64_t *>(out));
    else
        hipLaunchKernelGGL((k_sample_pack<uint32_t>), dim3(blocks), dim3(256), 0, s, planes, ell, n, seed, scene, box,
                           lay.words, static_cast<uint32_t *>(out));
    CG_LAUNCHED("sample_pack");
    return CG_OK;
}

}  // namespace cg
