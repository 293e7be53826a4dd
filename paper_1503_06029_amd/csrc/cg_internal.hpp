// Internal declarations and device helpers of the cell-graph library.
// Wave64 (CDNA) throughout: every wave-level helper assumes 64 lanes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/cellgraph.h"

namespace cg {

// ------------------------------------------------------------------ errors

// Records an error for cg_last_error() and returns st.
cg_status set_error(cg_status st, const char *fmt, ...);
// Checks hipGetLastError() after a launch; returns CG_OK or CG_EHIP.
cg_status check_launch(const char *what);

#define CG_TRY(expr)                        \
    do {                                    \
        cg_status _st = (expr);             \
        if (_st != CG_OK) return _st;       \
    } while (0)

#define CG_LAUNCHED(what) CG_TRY(::cg::check_launch(what))

// --------------------------------------------------------- workspace carving

// Bump allocator over a caller-provided buffer; with base == nullptr it only
// measures.  Every carve is 256-byte aligned.
struct Carver {
    char *base;
    size_t used;
    explicit Carver(void *b) : base(static_cast<char *>(b)), used(0) {}
    template <typename T> T *take(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        used = off + count * sizeof(T);
        return base ? reinterpret_cast<T *>(base + off) : nullptr;
    }
    size_t bytes() const { return (used + 255) & ~size_t(255); }
};

// Lets `kernel` be launched with `bytes` of dynamic LDS (above 64 KB the
// runtime needs the kernel's limit raised first).  Fails with CG_EUNSUPPORTED
// when the device offers less LDS per block.
cg_status allow_lds(const void *kernel, size_t bytes);

// ------------------------------------------------------------- lane helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ uint32_t shfl_up_u32(uint32_t x, int d) {
    return static_cast<uint32_t>(__shfl_up(static_cast<int>(x), d, 64));
}
__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t x, int d) {
    uint32_t lo = shfl_up_u32(static_cast<uint32_t>(x), d);
    uint32_t hi = shfl_up_u32(static_cast<uint32_t>(x >> 32), d);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_u64(uint64_t x, int src) {
    uint32_t lo = static_cast<uint32_t>(__shfl(static_cast<int>(static_cast<uint32_t>(x)), src, 64));
    uint32_t hi = static_cast<uint32_t>(__shfl(static_cast<int>(static_cast<uint32_t>(x >> 32)), src, 64));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_u64_xor(uint64_t x, int m) {
    uint32_t lo = static_cast<uint32_t>(__shfl_xor(static_cast<int>(static_cast<uint32_t>(x)), m, 64));
    uint32_t hi = static_cast<uint32_t>(__shfl_xor(static_cast<int>(static_cast<uint32_t>(x >> 32)), m, 64));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Inclusive prefix sum across the 64 lanes of a wave, by data-parallel
// primitives (DPP): shifts by 1, 2, 4, 8 lanes inside each 16-lane row, then
// row 0's and row 2's last lanes broadcast into rows 1 and 3, and lane 31
// into rows 2 and 3.  Lanes whose source is out of range, or whose row is
// masked off, add 0.  Six dependent ALU steps, no LDS round trips.
#define CG_DPP(x, ctrl, rmask) \
    static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), (ctrl), (rmask), 0xf, true))
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t x) {
    x += CG_DPP(x, 0x111, 0xf);  // row_shr:1
    x += CG_DPP(x, 0x112, 0xf);  // row_shr:2
    x += CG_DPP(x, 0x114, 0xf);  // row_shr:4
    x += CG_DPP(x, 0x118, 0xf);  // row_shr:8
    x += CG_DPP(x, 0x142, 0xa);  // row_bcast:15 into rows 1 and 3
    x += CG_DPP(x, 0x143, 0xc);  // row_bcast:31 into rows 2 and 3
    return x;
}
// The value of the lane one (xor 1) or two (xor 2) places away within the
// lane's quad of four.
__device__ __forceinline__ uint32_t quad_xor1(uint32_t x) { return CG_DPP(x, 0xB1, 0xf); }  // quad_perm 1,0,3,2
__device__ __forceinline__ uint32_t quad_xor2(uint32_t x) { return CG_DPP(x, 0x4E, 0xf); }  // quad_perm 2,3,0,1

// Sum over each aligned group of G lanes (G a power of two up to 64), in
// every lane of the group: quad permutes for pairs and quads, the
// half-row and row mirrors for 8 and 16 lanes (after the smaller sums a
// lane's mirror holds the other half's sum), lane shuffles beyond.
template <int G>
__device__ __forceinline__ uint64_t group_sum_u64(uint64_t x) {
    static_assert(G >= 1 && G <= 64 && (G & (G - 1)) == 0, "group of a power of two lanes");
    uint32_t lo = static_cast<uint32_t>(x), hi = static_cast<uint32_t>(x >> 32);
    auto add = [&](uint32_t ylo, uint32_t yhi) {
        const uint64_t r = ((static_cast<uint64_t>(hi) << 32) | lo) + ((static_cast<uint64_t>(yhi) << 32) | ylo);
        lo = static_cast<uint32_t>(r);
        hi = static_cast<uint32_t>(r >> 32);
    };
    if constexpr (G >= 2) add(quad_xor1(lo), quad_xor1(hi));
    if constexpr (G >= 4) add(quad_xor2(lo), quad_xor2(hi));
    if constexpr (G >= 8) add(CG_DPP(lo, 0x141, 0xf), CG_DPP(hi, 0x141, 0xf));  // row_half_mirror
    if constexpr (G >= 16) add(CG_DPP(lo, 0x140, 0xf), CG_DPP(hi, 0x140, 0xf)); // row_mirror
    uint64_t r = (static_cast<uint64_t>(hi) << 32) | lo;
    if constexpr (G >= 32) r += shfl_u64_xor(r, 16);
    if constexpr (G >= 64) r += shfl_u64_xor(r, 32);
    return r;
}
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t x) {
    uint32_t lo = static_cast<uint32_t>(x), hi = static_cast<uint32_t>(x >> 32);
    auto step = [&](uint32_t ylo, uint32_t yhi) {
        const uint64_t r = ((static_cast<uint64_t>(hi) << 32) | lo) + ((static_cast<uint64_t>(yhi) << 32) | ylo);
        lo = static_cast<uint32_t>(r);
        hi = static_cast<uint32_t>(r >> 32);
    };
    step(CG_DPP(lo, 0x111, 0xf), CG_DPP(hi, 0x111, 0xf));
    step(CG_DPP(lo, 0x112, 0xf), CG_DPP(hi, 0x112, 0xf));
    step(CG_DPP(lo, 0x114, 0xf), CG_DPP(hi, 0x114, 0xf));
    step(CG_DPP(lo, 0x118, 0xf), CG_DPP(hi, 0x118, 0xf));
    step(CG_DPP(lo, 0x142, 0xa), CG_DPP(hi, 0x142, 0xa));
    step(CG_DPP(lo, 0x143, 0xc), CG_DPP(hi, 0x143, 0xc));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}
#undef CG_DPP
// The value of lane 63 (a wave's total after an inclusive scan), as a
// wave-uniform scalar.
__device__ __forceinline__ uint32_t lane63_u32(uint32_t x) {
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), 63));
}

// Exclusive prefix sum over a 256-thread block (4 waves); returns the
// exclusive value and writes the block total to *total.  `tmp` must hold 4
// entries of LDS.  Contains __syncthreads().
__device__ __forceinline__ uint64_t block256_excl_scan_u64(uint64_t x, uint64_t *tmp, uint64_t *total) {
    int t = threadIdx.x, w = t >> 6, l = t & 63;
    uint64_t inc = wave_incl_scan_u64(x);
    if (l == 63) tmp[w] = inc;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint64_t v = tmp[i];
        if (i < w) pre += v;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return pre + inc - x;
}

// Appends `item` to list[] at a slot taken from *counter with one atomic per
// wave (same-address atomics serialise, so per-lane atomics do not scale).
// Every active lane of the wave must call it; lanes with want == false only
// vote.  Slots at or past cap are counted but not written.
template <typename V>
__device__ __forceinline__ void wave_append(V *list, unsigned long long *counter, int64_t cap, bool want, V item) {
    const uint64_t m = ballot64(want);
    if (m == 0) return;
    const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
    unsigned long long b = 0;
    if (lane_id() == leader) b = atomicAdd(counter, static_cast<unsigned long long>(__popcll(m)));
    b = shfl_u64(b, leader);
    if (want) {
        const unsigned long long k = b + static_cast<unsigned long long>(__popcll(m & lanemask_lt()));
        if (static_cast<int64_t>(k) < cap) list[k] = item;
    }
}

// -------------------------------------------------------------- row helpers

template <typename T> struct Bits;
template <> struct Bits<uint32_t> { static constexpr int B = 32; };
template <> struct Bits<uint64_t> { static constexpr int B = 64; };

// Mask with only vector position k set inside its word (MSB-first layout).
template <typename T> __device__ __forceinline__ T bitmask_of(int k) {
    return T(1) << (Bits<T>::B - 1 - (k % Bits<T>::B));
}

template <typename T> __device__ __forceinline__ int get_bit(const T *row, int k) {
    return static_cast<int>((row[k / Bits<T>::B] >> (Bits<T>::B - 1 - (k % Bits<T>::B))) & T(1));
}

// First 64 vector bits of a row as an unsigned integer, x(0) most significant.
template <typename T> __device__ __forceinline__ uint64_t head64(const T *row, int words);
template <> __device__ __forceinline__ uint64_t head64<uint64_t>(const uint64_t *row, int) { return row[0]; }
template <> __device__ __forceinline__ uint64_t head64<uint32_t>(const uint32_t *row, int words) {
    uint64_t hi = row[0];
    uint64_t lo = words > 1 ? row[1] : 0u;
    return (hi << 32) | lo;
}

// Tile of block b when a grid's tiles are dealt out per XCD: workgroups go
// round-robin over the 8 XCDs (b mod 8), so XCD x is given one contiguous run
// of tiles and neighbouring tiles share that XCD's L2 (their partial lines
// of output are merged there before they reach HBM).  A bijection of
// [0, g) for any grid size g.
__device__ __forceinline__ int xcd_tile(int b, int g) {
    const int x = b & 7, i = b >> 3, q = g >> 3, r = g & 7;
    return x * q + (x < r ? x : r) + i;
}

template <typename T> __device__ __forceinline__ int popc(T x);
template <> __device__ __forceinline__ int popc<uint32_t>(uint32_t x) { return __popc(x); }
template <> __device__ __forceinline__ int popc<uint64_t>(uint64_t x) { return __popcll(x); }

template <typename T> __device__ __forceinline__ int clz_t(T x);
template <> __device__ __forceinline__ int clz_t<uint32_t>(uint32_t x) { return __clz(x); }
template <> __device__ __forceinline__ int clz_t<uint64_t>(uint64_t x) { return __clzll(x); }

// Three-way lexicographic compare of two rows from word `from` on.
template <typename T>
__device__ __forceinline__ int row_cmp(const T *a, const T *b, int words, int from = 0) {
    for (int w = from; w < words; ++w) {
        T x = a[w], y = b[w];
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}

// Same order for rows in global memory: four words of each row are loaded
// together per step, so a comparison waits for one round trip per four
// words instead of one per word.
template <typename T>
__device__ __forceinline__ int row_cmp4(const T *a, const T *b, int words, int from = 0) {
    for (int w0 = from; w0 < words; w0 += 4) {
        T x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int w = w0 + u;
            x[u] = w < words ? a[w] : T(0);
            y[u] = w < words ? b[w] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (x[u] != y[u]) return x[u] < y[u] ? -1 : 1;
    }
    return 0;
}

// Compare cell row `c` with (q xor e_k), k < 0 meaning q itself.
template <typename T>
__device__ __forceinline__ int row_cmp_flip(const T *c, const T *q, int words, int kw, T km) {
    for (int w = 0; w < words; ++w) {
        T y = q[w] ^ (w == kw ? km : T(0));
        T x = c[w];
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}

// Hamming distance of two rows, stopping once it reaches 2.  On distance 1,
// *pos receives the differing position.
template <typename T>
__device__ __forceinline__ int dist_upto2(const T *a, const T *b, int words, int *pos) {
    int d = 0;
    for (int w = 0; w < words; ++w) {
        T x = a[w] ^ b[w];
        if (x) {
            d += popc<T>(x);
            if (d >= 2) return 2;
            *pos = w * Bits<T>::B + clz_t<T>(x);
        }
    }
    return d;
}

// Hamming distance without early exit, loading 8 words per batch so their
// loads are in flight together (what global-memory rows want).  *pos gets
// the first differing position (meaningful when the distance is 1).
template <typename T>
__device__ __forceinline__ int dist_full(const T *a, const T *b, int words, int *pos) {
    int d = 0;
    int first = -1;
    for (int w0 = 0; w0 < words; w0 += 8) {
        T x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int w = w0 + u;
            x[u] = w < words ? (a[w] ^ b[w]) : T(0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            d += popc<T>(x[u]);
            if (x[u] && first < 0) first = (w0 + u) * Bits<T>::B + clz_t<T>(x[u]);
        }
    }
    *pos = first;
    return d;
}

// Hamming distance of two rows of exactly WT words (compile time), without
// branches; *pos gets the first differing position (meaningful at distance 1).
template <typename T, int WT>
__device__ __forceinline__ int dist_t(const T *a, const T *b, int *pos) {
    int d = 0, first = -1;
#pragma unroll
    for (int w = 0; w < WT; ++w) {
        const T x = a[w] ^ b[w];
        d += popc<T>(x);
        first = (x && first < 0) ? w * Bits<T>::B + clz_t<T>(x) : first;
    }
    *pos = first;
    return d;
}

// dist_t in chunks of 4 words with a rolled outer loop: fewer registers
// live at once (for kernels that keep other state in registers).
template <typename T, int WT>
__device__ __forceinline__ int dist_t4(const T *a, const T *b, int *pos) {
    if constexpr (WT <= 4) {
        return dist_t<T, WT>(a, b, pos);
    } else {
        int d = 0, first = -1;
#pragma unroll 1
        for (int w0 = 0; w0 < WT; w0 += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const T x = a[w0 + u] ^ b[w0 + u];
                d += popc<T>(x);
                first = (x && first < 0) ? (w0 + u) * Bits<T>::B + clz_t<T>(x) : first;
            }
        }
        *pos = first;
        return d;
    }
}

// Block-wide copy of nrows contiguous global rows (`words` words each) into
// LDS rows of stride LW, with U loads in flight per thread (a plain loop with
// a run-time trip count would wait for each load before the next).
template <typename T, int NT, int U = 16>
__device__ __forceinline__ void copy_rows_to_lds(T *lds, int LW, const T *__restrict__ src, int nrows, int words) {
    const int tot = nrows * words;
    for (int e0 = threadIdx.x; e0 < tot; e0 += NT * U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * NT;
            v[u] = e < tot ? src[e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * NT;
            if (e < tot) {
                const int r = e / words;
                lds[r * LW + (e - r * words)] = v[u];
            }
        }
    }
}

// Index of the cell equal to (q xor e_k) within the sorted rows [lo, hi), or
// -1.  k < 0 looks up q itself.
template <typename T>
__device__ __forceinline__ int64_t find_row(const T *cells, int words, int64_t lo, int64_t hi,
                                            const T *q, int k) {
    int kw = k >= 0 ? k / Bits<T>::B : -1;
    T km = k >= 0 ? bitmask_of<T>(k) : T(0);
    const int64_t end = hi;
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (row_cmp_flip<T>(cells + mid * words, q, words, kw, km) < 0) lo = mid + 1;
        else hi = mid;
    }
    if (lo < end && row_cmp_flip<T>(cells + lo * words, q, words, kw, km) == 0) return lo;
    return -1;
}

// find_row for q xor e_k, searching only the directory bucket of the flipped
// vector's top p bits (dir[g] = first cell whose top p bits are >= g),
// narrowed to [lo_b, hi_b) when the caller knows the target lies there.
template <typename T>
__device__ __forceinline__ int64_t find_flip_dir(const T *cells, int words, const uint32_t *dir, int p, const T *q,
                                                 int k, int64_t lo_b = 0, int64_t hi_b = INT64_MAX) {
    uint64_t h = head64<T>(q, words);
    if (k < 64) h ^= 1ull << (63 - k);
    const int64_t g = p ? static_cast<int64_t>(h >> (64 - p)) : 0;
    int64_t lo = dir[g], hi = dir[g + 1];
    if (lo < lo_b) lo = lo_b;
    if (hi > hi_b) hi = hi_b;
    return lo < hi ? find_row<T>(cells, words, lo, hi, q, k) : -1;
}

// Wave-cooperative look-ups of q xor e_k for k = khi, khi - 1, ..., klo
// where q has a 0 at k (so the target is larger than q; targets are searched
// in [lo_b, hi_b) of the sorted cells only): each round the
// lanes take 64 consecutive k, descending.  f(v, k, rank) runs on the lane
// that found cell v; rank counts the targets found at larger k (that is,
// smaller v).  Every lane of the wave calls it with the same q; returns the
// number found.
template <typename T, class F>
__device__ __forceinline__ uint32_t wave_flip_lookups(const T *cells, int words, const uint32_t *dir, int p,
                                                      const T *q, int khi, int klo, F f, int64_t lo_b = 0,
                                                      int64_t hi_b = INT64_MAX) {
    const int lane = __lane_id();
    uint32_t c = 0;
    for (int k0 = khi; k0 >= klo; k0 -= 64) {
        const int k = k0 - lane;
        int64_t v = -1;
        if (k >= klo && !get_bit<T>(q, k)) v = find_flip_dir<T>(cells, words, dir, p, q, k, lo_b, hi_b);
        const uint64_t m = __ballot(v >= 0);
        if (v >= 0) {
            const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
            f(static_cast<uint32_t>(v), k, c + static_cast<uint32_t>(__popcll(m & below)));
        }
        c += static_cast<uint32_t>(__popcll(m));
    }
    return c;
}

// 64-bit finaliser (the MurmurHash3 fmix64 mixing function).
__device__ __forceinline__ uint64_t fmix64(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

// 32-bit hash of bits s .. l-1 of a row (the suffix-grouped order of the
// dictionary sorts cells by it; equal suffixes give equal hashes).  It is a
// sum of per-word terms, finished by one mix, so lanes holding different
// words of a row can add their terms and combine them in any order.
template <typename T>
__device__ __forceinline__ uint64_t suffix_term(T x, int w, int s) {
    constexpr int B = Bits<T>::B;
    const int w0 = s / B;
    if (w < w0) return 0;
    if (w == w0 && (s % B)) x &= (T(~T(0)) >> (s % B));
    // one multiply per word by a word-dependent odd constant; the sum is
    // mixed once at the end
    const uint64_t y = static_cast<uint64_t>(x) ^ (static_cast<uint64_t>(x) >> 29);
    return y * (0x9e3779b97f4a7c15ull + 2ull * static_cast<uint64_t>(w)) + static_cast<uint64_t>(w);
}
__device__ __forceinline__ uint32_t suffix_finish(uint64_t sum) {
    return static_cast<uint32_t>(fmix64(sum ^ 0x243f6a8885a308d3ull) >> 32);
}
template <typename T>
__device__ __forceinline__ uint32_t suffix_hash32(const T *row, int words, int s) {
    uint64_t sum = 0;
    for (int w = 0; w < words; ++w) sum += suffix_term<T>(row[w], w, s);
    return suffix_finish(sum);
}

__device__ __forceinline__ int64_t load_n(const int64_t *d_n, int64_t cap) {
    if (!d_n) return cap;
    int64_t n = *d_n;
    return n < cap ? (n < 0 ? 0 : n) : cap;
}

// -------------------------------------------------------- host-side helpers

inline unsigned blocks_for(int64_t items, int64_t per_block, int64_t max_blocks = 1 << 30) {
    int64_t b = (items + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return static_cast<unsigned>(b);
}

// ------------------------------------------------- primitives (cg_prims.hip)

// Device-wide exclusive scan.  Each primitive reads a per-item 32-bit value,
// writes the exclusive prefix to out[i] (i < n) and the total to *total (if
// non-null).  n = min(*d_n, n_cap) (d_n may be null).  tile_sums must hold
// scan_tiles(n_cap) entries.
int64_t scan_tiles(int64_t n_cap);
cg_status scan_u32_to_u32(const uint32_t *in, uint32_t *out, int64_t n_cap, const int64_t *d_n,
                          uint64_t *tile_sums, uint32_t *total, hipStream_t s);
// The byte form takes flags that are 0 or 1 (it counts a word's flags with
// one multiply).
cg_status scan_u8_to_u32(const uint8_t *in, uint32_t *out, int64_t n_cap, const int64_t *d_n,
                         uint64_t *tile_sums, int64_t *total, hipStream_t s);
// out[i] = sum_{j<i} (a[j] + b[j]) as int64; out[n] and *total = the sum.
cg_status scan_pair_to_i64(const uint32_t *a, const uint32_t *b, int64_t *out, int64_t n_cap,
                           const int64_t *d_n, uint64_t *tile_sums, int64_t *total, hipStream_t s);
// out[i] = sum_{j<i} a[j] as int64; out[n] and *total = the sum.
cg_status scan_u32_to_i64(const uint32_t *a, int64_t *out, int64_t n_cap, const int64_t *d_n, uint64_t *tile_sums,
                          int64_t *total, hipStream_t s);
// Same for popcounts of `words` words per row (T-sized words).
cg_status scan_rowpop_to_i64(const void *rows, int word_bits, int words, int64_t *out, int64_t n_cap,
                             const int64_t *d_n, uint64_t *tile_sums, int64_t *total, hipStream_t s);

// LSD radix sort of 64-bit keys (with optional 32-bit values) by key bits
// [bit_lo, bit_hi), 8 bits per pass, stable.  The sorted data ends in
// keys[res] / vals[res], res returned in *which (0 or 1).  keys[1]/vals[1]
// are scratch of the same size.  hist needs radix_hist_entries(n_cap).
int64_t radix_hist_entries(int64_t n_cap);
cg_status radix_sort_u64(uint64_t *keys[2], uint32_t *vals[2], int64_t n_cap, const int64_t *d_n, int bit_lo,
                         int bit_hi, uint32_t *hist, uint64_t *tile_sums, int *which, hipStream_t s,
                         const unsigned long long *skip = nullptr, int skip_below = 0);

// LSD radix sort of a key held as nplanes (1..3) 32-bit planes, planes[0]
// the most significant (for a dedup key: the row's first 32 bits, then the
// next 32, ...), with 32-bit values, by key bits [bit_lo, 32 nplanes)
// counted from the least significant end, 8 bits per pass, stable.
// lower_planes: the planes below the highest are still wanted after the
// sort (they are carried through the passes of the planes above them).
// key32 (two planes only; device flag, may be null): when nonzero the low
// plane's passes do nothing (the key is its high plane, an even number of
// skipped passes, so *which stays right) and the high plane's passes drop
// it.  The sorted planes and values end in [*which].
cg_status radix_sort_k32(uint32_t *planes[3][2], int nplanes, uint32_t *vals[2], int64_t n_cap, const int64_t *d_n,
                         int bit_lo, uint32_t *hist, int *which, hipStream_t s, bool lower_planes,
                         const unsigned long long *key32);

// Fill kernel (graph-capture safe replacement for hipMemsetAsync).
cg_status fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
cg_status fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);

// ------------------------------------------------------------ path pieces

cg_status launch_pack(const uint8_t *bits, int64_t n, int64_t row_stride, cg_layout lay, void *out,
                      hipStream_t s);

size_t dedup_workspace_bytes(int64_t n, cg_layout lay);
// The dedup half of the fused dedup + dictionary build: as run_dedup, plus
// the suffix-order keys of the cells (hash of bits hash_s .. << 32 | id) in
// sfx, and in *view the sorted keys, new-cell flags and exclusive cell
// numbering (device arrays in the workspace, n entries) for the directory.
struct DedupView {
    const uint32_t *khi;  // sorted keys' first 32 bits (the rows' first 32 bits)
    const uint8_t *uniq;
    const uint32_t *cidx;
};
size_t dedup_fused_workspace_bytes(int64_t n, cg_layout lay);
cg_status run_dedup_fused(const void *rows, int64_t n, cg_layout lay, void *cells, uint32_t *row_to_cell,
                          int64_t *d_ncells, void *ws, int hash_s, uint64_t *sfx, DedupView *view, int key_bits,
                          unsigned long long *extra_zero, int n_extra, hipStream_t s);
cg_status run_dedup(const void *rows, int64_t n, cg_layout lay, void *cells, uint32_t *row_to_cell,
                    int64_t *d_ncells, void *ws, size_t ws_bytes, hipStream_t s);

size_t dict_mem_bytes(int64_t ncap, cg_layout lay, const cg_dict_params &p);
cg_dict_params resolve_params(int64_t ncap, cg_layout lay, const cg_dict_params *p);
cg_status run_dict_build(cg_dict &d, hipStream_t s);
cg_status run_dedup_dict(const void *rows, int64_t n, cg_layout lay, void *cells, uint32_t *row_to_cell,
                         int64_t *d_ncells, void *ws, cg_dict &d, hipStream_t s);

cg_status run_neighbors_d1(const cg_dict &d, const void *q, int64_t nq, uint32_t *count, uint32_t *self,
                           void *mask, hipStream_t s);

size_t edges_workspace_bytes(const cg_dict &d, int64_t cap);
cg_status run_edges(const cg_dict &d, uint32_t *uv, uint16_t *bit, int64_t cap, int64_t *d_nedges,
                    int64_t *d_offsets, void *ws, size_t ws_bytes, int32_t *d_status, hipStream_t s);

size_t allpairs_workspace_bytes(const cg_dict &d, int64_t cap);
cg_status run_edges_allpairs(const cg_dict &d, uint32_t *uv, uint16_t *bit, int64_t cap,
                             int64_t *d_nedges, int64_t *d_offsets, void *ws, size_t ws_bytes,
                             int32_t *d_status, hipStream_t s);

size_t hash_workspace_bytes(const cg_dict &d, int64_t cap);
cg_status run_edges_hash(const cg_dict &d, uint32_t *uv, uint16_t *bit, int64_t cap, int64_t *d_nedges,
                         int64_t *d_offsets, void *ws, int32_t *d_status, hipStream_t s);

cg_status batch_layout(int32_t ell_max, cg_layout *lay);
cg_status run_batch_pack(const uint8_t *bits, const int64_t *bits_off, const int32_t *scene_ell,
                         const int64_t *scene_rows, int32_t n_scenes, int64_t n_rows, cg_layout lay, void *out,
                         hipStream_t s);
cg_status run_batch_split(const cg_dict &d, int32_t n_scenes, const int64_t *offsets, const int64_t *d_nedges,
                          int64_t cap, int64_t *cell_off, int64_t *edge_off, int32_t localize, uint32_t *uv,
                          uint16_t *bit, uint32_t *r2c, const int64_t *scene_rows, int64_t n_rows, hipStream_t s);

size_t csr_workspace_bytes(int64_t ncap, int64_t ecap);
cg_status run_graph_csr(const uint32_t *uv, const int64_t *offsets, const int64_t *d_ncells, int64_t ncap,
                        const int64_t *d_nedges, int64_t ecap, int64_t *adj_off, uint32_t *adj, int32_t *status,
                        void *ws, hipStream_t s);
size_t bfs_workspace_bytes(int64_t ncap);
cg_status run_bfs(const int64_t *adj_off, const uint32_t *adj, const int64_t *d_ncells, int64_t ncap,
                  uint32_t source, int32_t max_levels, int32_t resume, uint32_t *dist, uint32_t *parent,
                  int32_t *levels, int32_t *status, void *ws, hipStream_t s);
cg_status run_bfs_path(const uint32_t *dist, const uint32_t *parent, const int64_t *d_ncells, int64_t ncap,
                       uint32_t target, uint32_t *path, int64_t path_cap, int64_t *len, hipStream_t s);

cg_status run_sample_pack(const double *planes, int32_t ell, int64_t n, uint64_t seed, uint64_t scene,
                          const double lohi[6], cg_layout lay, void *out, hipStream_t s);
cg_status run_batch_sample_pack(const double *planes, const int64_t *planes_off, const int32_t *scene_ell,
                                const int64_t *scene_rows, const uint64_t *keys, int32_t n_scenes, int64_t n_rows,
                                const double lohi[6], cg_layout lay, void *out, hipStream_t s);

}  // namespace cg
