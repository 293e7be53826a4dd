// Device-wide primitives: exclusive scans, LSD radix sort, fills.
//
// Scans are three-phase (tile reduce -> one-block scan of tile sums -> tile
// rescan), deterministic and free of inter-block waiting.  The radix sort is
// the classic per-pass histogram / scan / stable scatter; each scatter stages
// its tile in LDS, sorted by digit, so global writes go out in contiguous runs.
#include "cg_internal.hpp"

namespace cg {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;  // 4096

struct U32Arr {
    const uint32_t *p;
    __device__ uint32_t operator()(int64_t i) const { return p[i]; }
};
struct PairSum {
    const uint32_t *a, *b;
    __device__ uint32_t operator()(int64_t i) const { return a[i] + b[i]; }
};
template <typename T> struct RowPop {
    const T *rows;
    int words;
    __device__ uint32_t operator()(int64_t i) const {
        uint32_t c = 0;
        const T *r = rows + i * words;
        for (int w = 0; w < words; ++w) c += popc<T>(r[w]);
        return c;
    }
};

template <class F>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(F f, int64_t n_cap, const int64_t *d_n,
                                                              uint64_t *tile_sums) {
    __shared__ uint64_t tmp[4];
    const int64_t n = load_n(d_n, n_cap);
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE;
    uint64_t acc = 0;
    if (base < n) {
#pragma unroll 4
        for (int j = 0; j < SCAN_ITEMS; ++j) {
            int64_t i = base + j * SCAN_THREADS + threadIdx.x;
            if (i < n) acc += f(i);
        }
    }
    uint64_t total;
    block256_excl_scan_u64(acc, tmp, &total);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// One block: exclusive scan of the tile sums in place; total to the outputs.
template <typename TO>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_tiles(uint64_t *tile_sums, int64_t n_cap,
                                                             const int64_t *d_n, TO *out_end,
                                                             int64_t *total_i64, uint32_t *total_u32) {
    __shared__ uint64_t tmp[4];
    const int64_t n = load_n(d_n, n_cap);
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    uint64_t carry = 0;
    for (int64_t c = 0; c < tiles; c += SCAN_THREADS) {
        int64_t i = c + threadIdx.x;
        uint64_t v = i < tiles ? tile_sums[i] : 0;
        uint64_t tot;
        uint64_t ex = block256_excl_scan_u64(v, tmp, &tot);
        if (i < tiles) tile_sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        if (out_end) out_end[n] = static_cast<TO>(carry);
        if (total_i64) *total_i64 = static_cast<int64_t>(carry);
        if (total_u32) *total_u32 = static_cast<uint32_t>(carry);
    }
}

template <class F, typename TO>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_down(F f, TO *out, int64_t n_cap, const int64_t *d_n,
                                                            const uint64_t *tile_sums) {
    __shared__ uint64_t vals[SCAN_TILE];
    __shared__ uint64_t tmp[4];
    const int64_t n = load_n(d_n, n_cap);
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE;
    if (base >= n) return;
    const int t = threadIdx.x;
#pragma unroll 4
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = base + j * SCAN_THREADS + t;
        vals[j * SCAN_THREADS + t] = i < n ? f(i) : 0;
    }
    __syncthreads();
    uint64_t local[SCAN_ITEMS];
    uint64_t sum = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        local[j] = vals[t * SCAN_ITEMS + j];
        sum += local[j];
    }
    uint64_t tot;
    uint64_t ex = block256_excl_scan_u64(sum, tmp, &tot) + tile_sums[blockIdx.x];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        vals[t * SCAN_ITEMS + j] = ex;
        ex += local[j];
    }
    __syncthreads();
#pragma unroll 4
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = base + j * SCAN_THREADS + t;
        if (i < n) out[i] = static_cast<TO>(vals[j * SCAN_THREADS + t]);
    }
}

// Exclusive scan of 0/1 byte flags into u32: a thread takes 16 consecutive
// flags with one 16-byte load (byte loads at the end of the input or when
// it is not 16-byte aligned) and counts a word's flags by one multiply; the
// down-sweep writes its 16 outputs as four 16-byte stores.
__device__ __forceinline__ void load_flags16(const uint8_t *p, int64_t i, int64_t n, bool vec, uint32_t f[4]) {
    if (vec && i + 16 <= n) {
        const uint4 v = *reinterpret_cast<const uint4 *>(p + i);
        f[0] = v.x; f[1] = v.y; f[2] = v.z; f[3] = v.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            uint32_t x = 0;
            for (int b = 0; b < 4; ++b) {
                const int64_t q = i + 4 * k + b;
                if (q < n) x |= static_cast<uint32_t>(p[q]) << (8 * b);
            }
            f[k] = x;
        }
    }
}
__device__ __forceinline__ uint32_t flags_in_word(uint32_t x) { return (x * 0x01010101u) >> 24; }

__global__ void __launch_bounds__(SCAN_THREADS) k_scan8_reduce(const uint8_t *flags, int64_t n_cap,
                                                               const int64_t *d_n, uint64_t *tile_sums) {
    __shared__ uint64_t tmp[4];
    const int64_t n = load_n(d_n, n_cap);
    const int64_t i = static_cast<int64_t>(blockIdx.x) * SCAN_TILE + 16 * threadIdx.x;
    const bool vec = (reinterpret_cast<uintptr_t>(flags) & 15) == 0;
    uint64_t acc = 0;
    if (i < n) {
        uint32_t f[4];
        load_flags16(flags, i, n, vec, f);
        acc = flags_in_word(f[0]) + flags_in_word(f[1]) + flags_in_word(f[2]) + flags_in_word(f[3]);
    }
    uint64_t total;
    block256_excl_scan_u64(acc, tmp, &total);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan8_down(const uint8_t *flags, uint32_t *out, int64_t n_cap,
                                                             const int64_t *d_n, const uint64_t *tile_sums) {
    __shared__ uint64_t tmp[4];
    const int64_t n = load_n(d_n, n_cap);
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE;
    if (base >= n) return;
    const int64_t i = base + 16 * threadIdx.x;
    const bool vec = (reinterpret_cast<uintptr_t>(flags) & 15) == 0;
    uint32_t f[4] = {0u, 0u, 0u, 0u};
    if (i < n) load_flags16(flags, i, n, vec, f);
    const uint64_t sum = flags_in_word(f[0]) + flags_in_word(f[1]) + flags_in_word(f[2]) + flags_in_word(f[3]);
    uint64_t tot;
    uint32_t ex = static_cast<uint32_t>(block256_excl_scan_u64(sum, tmp, &tot) + tile_sums[blockIdx.x]);
    if (i >= n) return;
    uint32_t o[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        o[k] = ex;
        ex += (f[k >> 2] >> (8 * (k & 3))) & 0xFFu;
    }
    if (i + 16 <= n && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
        uint4 *o4 = reinterpret_cast<uint4 *>(out + i);
#pragma unroll
        for (int k = 0; k < 4; ++k) o4[k] = make_uint4(o[4 * k], o[4 * k + 1], o[4 * k + 2], o[4 * k + 3]);
    } else {
        for (int k = 0; k < 16 && i + k < n; ++k) out[i + k] = o[k];
    }
}

template <class F, typename TO>
cg_status scan_generic(F f, TO *out, int64_t n_cap, const int64_t *d_n, uint64_t *tile_sums, TO *out_end,
                       int64_t *total_i64, uint32_t *total_u32, hipStream_t s) {
    unsigned tiles = blocks_for(n_cap, SCAN_TILE);
    hipLaunchKernelGGL((k_scan_reduce<F>), dim3(tiles), dim3(SCAN_THREADS), 0, s, f, n_cap, d_n, tile_sums);
    CG_LAUNCHED("scan_reduce");
    hipLaunchKernelGGL((k_scan_tiles<TO>), dim3(1), dim3(SCAN_THREADS), 0, s, tile_sums, n_cap, d_n, out_end,
                       total_i64, total_u32);
    CG_LAUNCHED("scan_tiles");
    hipLaunchKernelGGL((k_scan_down<F, TO>), dim3(tiles), dim3(SCAN_THREADS), 0, s, f, out, n_cap, d_n,
                       tile_sums);
    CG_LAUNCHED("scan_down");
    return CG_OK;
}

// ------------------------------------------------------------------ radix

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;  // 2048
constexpr int RADIX = 256;

__global__ void __launch_bounds__(RS_THREADS) k_radix_hist(const uint64_t *keys, int64_t n_cap, const int64_t *d_n,
                                                           int shift, uint32_t *hist, int num_tiles,
                                                           const unsigned long long *skip) {
    if (skip && *skip) return;
    __shared__ uint32_t h[RADIX];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t n = load_n(d_n, n_cap);
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t base = static_cast<int64_t>(tile) * RS_TILE;
    if (base < n) {
        // the tile's loads are issued together, then counted
        uint64_t k[RS_ITEMS];
#pragma unroll
        for (int j = 0; j < RS_ITEMS; ++j) {
            const int64_t i = base + j * RS_THREADS + t;
            k[j] = i < n ? keys[i] : 0;
        }
#pragma unroll
        for (int j = 0; j < RS_ITEMS; ++j)
            if (base + j * RS_THREADS + t < n) atomicAdd(&h[(k[j] >> shift) & (RADIX - 1)], 1u);
    }
    __syncthreads();
    hist[static_cast<int64_t>(t) * num_tiles + tile] = h[t];
}

// Column scan of the digit-major tile histograms hist[d * num_tiles + tile],
// one block per digit: each row is scanned in place (exclusive, from 0) and
// its total goes to dtot[d]; the scatter adds the totals of the smaller
// digits.  The row passes through LDS in chunks of DS_CHUNK entries, loaded
// and stored coalesced; within a chunk thread t scans entries
// [t * DS_PER, (t + 1) * DS_PER), one pad word per DS_PER entries keeping
// the threads on distinct banks.
constexpr int DS_PER = 16;
constexpr int DS_CHUNK = RS_THREADS * DS_PER;

__global__ void __launch_bounds__(RS_THREADS) k_radix_dscan(uint32_t *hist, int num_tiles, uint32_t *dtot,
                                                            const unsigned long long *skip) {
    if (skip && *skip) return;
    __shared__ uint64_t tmp[4];
    __shared__ uint32_t sr[DS_CHUNK + DS_CHUNK / DS_PER];
    const int d = blockIdx.x, t = threadIdx.x;
    uint32_t *row = hist + static_cast<int64_t>(d) * num_tiles;
    auto pad = [](int k) { return k + k / DS_PER; };
    uint64_t carry = 0;
    for (int c0 = 0; c0 < num_tiles; c0 += DS_CHUNK) {
        const int len = num_tiles - c0 < DS_CHUNK ? num_tiles - c0 : DS_CHUNK;
        uint32_t x[DS_PER];
#pragma unroll
        for (int j = 0; j < DS_PER; ++j) {
            const int k = j * RS_THREADS + t;
            x[j] = k < len ? row[c0 + k] : 0u;
        }
#pragma unroll
        for (int j = 0; j < DS_PER; ++j) sr[pad(j * RS_THREADS + t)] = x[j];
        __syncthreads();
        uint64_t sum = 0;
#pragma unroll
        for (int j = 0; j < DS_PER; ++j) {
            x[j] = sr[pad(t * DS_PER + j)];
            sum += x[j];
        }
        uint64_t tot;
        uint64_t run = carry + block256_excl_scan_u64(sum, tmp, &tot);
#pragma unroll
        for (int j = 0; j < DS_PER; ++j) {
            sr[pad(t * DS_PER + j)] = static_cast<uint32_t>(run);
            run += x[j];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < DS_PER; ++j) {
            const int k = j * RS_THREADS + t;
            if (k < len) row[c0 + k] = sr[pad(k)];
        }
        carry += tot;
        __syncthreads();
    }
    if (t == 0) dtot[d] = static_cast<uint32_t>(carry);
}

template <bool HAS_VALS>
__global__ void __launch_bounds__(RS_THREADS) k_radix_scatter(const uint64_t *kin, const uint32_t *vin,
                                                              uint64_t *kout, uint32_t *vout, int64_t n_cap,
                                                              const int64_t *d_n, int shift,
                                                              const uint32_t *hist_off, const uint32_t *dtot,
                                                              int num_tiles, const unsigned long long *skip) {
    if (skip && *skip) return;
    __shared__ uint32_t wcnt[RS_WAVES][RADIX];
    __shared__ uint32_t tile_start[RADIX];
    __shared__ uint32_t gbase[RADIX];
    __shared__ uint64_t sk[RS_TILE];
    __shared__ uint32_t sv[HAS_VALS ? RS_TILE : 1];
    __shared__ uint64_t tmp[4];

    const int64_t n = load_n(d_n, n_cap);
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t base = static_cast<int64_t>(tile) * RS_TILE;
    if (base >= n) return;
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int tile_n = static_cast<int>(n - base < RS_TILE ? n - base : RS_TILE);

    for (int i = t; i < RS_WAVES * RADIX; i += RS_THREADS) (&wcnt[0][0])[i] = 0;
    __syncthreads();

    uint64_t key[RS_ITEMS];
    uint32_t val[RS_ITEMS];
    uint32_t rank[RS_ITEMS];
    const uint64_t lt = lanemask_lt();
    // wave w owns the contiguous sub-tile [w * 64 * ITEMS, (w + 1) * 64 * ITEMS);
    // all of a thread's loads are issued before the ranking (whose wave
    // barriers would otherwise hold each load back until the previous item
    // is ranked)
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int li = (w * RS_ITEMS + j) * 64 + lane;
        const bool valid = li < tile_n;
        key[j] = valid ? kin[base + li] : 0;
        if (HAS_VALS) val[j] = valid ? vin[base + li] : 0;
    }
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        int li = (w * RS_ITEMS + j) * 64 + lane;
        bool valid = li < tile_n;
        int d = static_cast<int>((key[j] >> shift) & (RADIX - 1));
        uint64_t m = ballot64(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = ballot64((d >> b) & 1);
            m &= ((d >> b) & 1) ? bb : ~bb;
        }
        uint32_t before = 0;
        if (valid) before = wcnt[w][d];
        __builtin_amdgcn_wave_barrier();
        if (valid) {
            rank[j] = before + static_cast<uint32_t>(__popcll(m & lt));
            if ((m & lt) == 0) wcnt[w][d] = before + static_cast<uint32_t>(__popcll(m));
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // thread t owns digit t: wave prefix, tile count, tile-local start
    {
        uint32_t c[RS_WAVES], run = 0;
#pragma unroll
        for (int i = 0; i < RS_WAVES; ++i) {
            c[i] = wcnt[i][t];
            wcnt[i][t] = run;
            run += c[i];
        }
        uint64_t tot;
        uint64_t ex = block256_excl_scan_u64(run, tmp, &tot);
        tile_start[t] = static_cast<uint32_t>(ex);
        // first output position of digit t: the totals of the smaller digits
        // plus this digit's count in the tiles before this one
        const uint64_t dbase = block256_excl_scan_u64(dtot[t], tmp, &tot);
        gbase[t] = static_cast<uint32_t>(dbase) + hist_off[static_cast<int64_t>(t) * num_tiles + tile];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        int li = (w * RS_ITEMS + j) * 64 + lane;
        if (li < tile_n) {
            int d = static_cast<int>((key[j] >> shift) & (RADIX - 1));
            uint32_t p = tile_start[d] + wcnt[w][d] + rank[j];
            sk[p] = key[j];
            if (HAS_VALS) sv[p] = val[j];
        }
    }
    __syncthreads();
    for (int i = t; i < tile_n; i += RS_THREADS) {
        uint64_t k = sk[i];
        int d = static_cast<int>((k >> shift) & (RADIX - 1));
        int64_t g = static_cast<int64_t>(gbase[d]) + (i - static_cast<int>(tile_start[d]));
        kout[g] = k;
        if (HAS_VALS) vout[g] = sv[i];
    }
}

// The same passes over 32-bit keys with one or two 32-bit payloads (the
// dedup's sort key kept as two planes, so a pass over the high plane moves 8
// bytes per row when the low plane is no longer needed).  A pass returns at
// once when *skip is set; the second payload moves only when v1in is given
// and *drop_v1 (if given) is clear.
__global__ void __launch_bounds__(RS_THREADS) k_radix32_hist(const uint32_t *keys, int64_t n_cap, const int64_t *d_n,
                                                             int shift, uint32_t *hist, int num_tiles,
                                                             const unsigned long long *skip) {
    if (skip && *skip) return;
    __shared__ uint32_t h[RADIX];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t n = load_n(d_n, n_cap);
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t base = static_cast<int64_t>(tile) * RS_TILE;
    if (base < n) {
        uint32_t k[RS_ITEMS];
#pragma unroll
        for (int j = 0; j < RS_ITEMS; ++j) {
            const int64_t i = base + j * RS_THREADS + t;
            k[j] = i < n ? keys[i] : 0u;
        }
#pragma unroll
        for (int j = 0; j < RS_ITEMS; ++j)
            if (base + j * RS_THREADS + t < n) atomicAdd(&h[(k[j] >> shift) & (RADIX - 1)], 1u);
    }
    __syncthreads();
    hist[static_cast<int64_t>(t) * num_tiles + tile] = h[t];
}

// NP: how many payload planes besides the values the launch may carry (the
// LDS staging is sized for them).
template <int NP>
__global__ void __launch_bounds__(RS_THREADS) k_radix32_scatter(const uint32_t *kin, const uint32_t *v0in,
                                                                const uint32_t *v1in, const uint32_t *v2in,
                                                                uint32_t *kout, uint32_t *v0out, uint32_t *v1out,
                                                                uint32_t *v2out, int64_t n_cap, const int64_t *d_n,
                                                                int shift, const uint32_t *hist_off,
                                                                const uint32_t *dtot, int num_tiles,
                                                                const unsigned long long *skip,
                                                                const unsigned long long *drop_v1) {
    if (skip && *skip) return;
    __shared__ uint32_t wcnt[RS_WAVES][RADIX];
    __shared__ uint32_t tile_start[RADIX];
    __shared__ uint32_t gbase[RADIX];
    __shared__ uint32_t sk[RS_TILE];
    __shared__ uint32_t sv0[RS_TILE];
    __shared__ uint32_t sv1[NP >= 1 ? RS_TILE : 1];
    __shared__ uint32_t sv2[NP >= 2 ? RS_TILE : 1];
    __shared__ uint64_t tmp[4];

    const int64_t n = load_n(d_n, n_cap);
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t base = static_cast<int64_t>(tile) * RS_TILE;
    if (base >= n) return;
    const bool has1 = NP >= 1 && v1in != nullptr && !(drop_v1 && *drop_v1);
    const bool has2 = NP >= 2 && v2in != nullptr;
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int tile_n = static_cast<int>(n - base < RS_TILE ? n - base : RS_TILE);

    for (int i = t; i < RS_WAVES * RADIX; i += RS_THREADS) (&wcnt[0][0])[i] = 0;
    __syncthreads();

    uint32_t key[RS_ITEMS], v0[RS_ITEMS], v1[RS_ITEMS], v2[RS_ITEMS], rank[RS_ITEMS];
    const uint64_t lt = lanemask_lt();
    // wave w owns the contiguous sub-tile [w * 64 * ITEMS, (w + 1) * 64 * ITEMS);
    // every load is issued before the ranking starts
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int li = (w * RS_ITEMS + j) * 64 + lane;
        const bool valid = li < tile_n;
        key[j] = valid ? kin[base + li] : 0u;
        v0[j] = valid ? v0in[base + li] : 0u;
        v1[j] = (valid && has1) ? v1in[base + li] : 0u;
        v2[j] = (valid && has2) ? v2in[base + li] : 0u;
    }
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int li = (w * RS_ITEMS + j) * 64 + lane;
        const bool valid = li < tile_n;
        const int d = static_cast<int>((key[j] >> shift) & (RADIX - 1));
        uint64_t m = ballot64(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = ballot64((d >> b) & 1);
            m &= ((d >> b) & 1) ? bb : ~bb;
        }
        uint32_t before = 0;
        if (valid) before = wcnt[w][d];
        __builtin_amdgcn_wave_barrier();
        if (valid) {
            rank[j] = before + static_cast<uint32_t>(__popcll(m & lt));
            if ((m & lt) == 0) wcnt[w][d] = before + static_cast<uint32_t>(__popcll(m));
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    {
        uint32_t c[RS_WAVES], run = 0;
#pragma unroll
        for (int i = 0; i < RS_WAVES; ++i) {
            c[i] = wcnt[i][t];
            wcnt[i][t] = run;
            run += c[i];
        }
        uint64_t tot;
        const uint64_t ex = block256_excl_scan_u64(run, tmp, &tot);
        tile_start[t] = static_cast<uint32_t>(ex);
        const uint64_t dbase = block256_excl_scan_u64(dtot[t], tmp, &tot);
        gbase[t] = static_cast<uint32_t>(dbase) + hist_off[static_cast<int64_t>(t) * num_tiles + tile];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int li = (w * RS_ITEMS + j) * 64 + lane;
        if (li < tile_n) {
            const int d = static_cast<int>((key[j] >> shift) & (RADIX - 1));
            const uint32_t p = tile_start[d] + wcnt[w][d] + rank[j];
            sk[p] = key[j];
            sv0[p] = v0[j];
            if (has1) sv1[p] = v1[j];
            if (has2) sv2[p] = v2[j];
        }
    }
    __syncthreads();
    for (int i = t; i < tile_n; i += RS_THREADS) {
        const uint32_t k = sk[i];
        const int d = static_cast<int>((k >> shift) & (RADIX - 1));
        const int64_t g = static_cast<int64_t>(gbase[d]) + (i - static_cast<int>(tile_start[d]));
        kout[g] = k;
        v0out[g] = sv0[i];
        if (has1) v1out[g] = sv1[i];
        if (has2) v2out[g] = sv2[i];
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_i64(int64_t *p, int64_t v, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

}  // namespace

int64_t scan_tiles(int64_t n_cap) { return (n_cap + SCAN_TILE - 1) / SCAN_TILE + 1; }

cg_status scan_u32_to_u32(const uint32_t *in, uint32_t *out, int64_t n_cap, const int64_t *d_n,
                          uint64_t *tile_sums, uint32_t *total, hipStream_t s) {
    return scan_generic(U32Arr{in}, out, n_cap, d_n, tile_sums, static_cast<uint32_t *>(nullptr), nullptr,
                        total, s);
}

cg_status scan_u8_to_u32(const uint8_t *in, uint32_t *out, int64_t n_cap, const int64_t *d_n,
                         uint64_t *tile_sums, int64_t *total, hipStream_t s) {
    const unsigned tiles = blocks_for(n_cap, SCAN_TILE);
    hipLaunchKernelGGL(k_scan8_reduce, dim3(tiles), dim3(SCAN_THREADS), 0, s, in, n_cap, d_n, tile_sums);
    CG_LAUNCHED("scan8_reduce");
    hipLaunchKernelGGL((k_scan_tiles<uint32_t>), dim3(1), dim3(SCAN_THREADS), 0, s, tile_sums, n_cap, d_n,
                       static_cast<uint32_t *>(nullptr), total, static_cast<uint32_t *>(nullptr));
    CG_LAUNCHED("scan_tiles");
    hipLaunchKernelGGL(k_scan8_down, dim3(tiles), dim3(SCAN_THREADS), 0, s, in, out, n_cap, d_n, tile_sums);
    CG_LAUNCHED("scan8_down");
    return CG_OK;
}

cg_status scan_pair_to_i64(const uint32_t *a, const uint32_t *b, int64_t *out, int64_t n_cap,
                           const int64_t *d_n, uint64_t *tile_sums, int64_t *total, hipStream_t s) {
    return scan_generic(PairSum{a, b}, out, n_cap, d_n, tile_sums, out, total, nullptr, s);
}

cg_status scan_u32_to_i64(const uint32_t *a, int64_t *out, int64_t n_cap, const int64_t *d_n, uint64_t *tile_sums,
                          int64_t *total, hipStream_t s) {
    return scan_generic(U32Arr{a}, out, n_cap, d_n, tile_sums, out, total, nullptr, s);
}

cg_status scan_rowpop_to_i64(const void *rows, int word_bits, int words, int64_t *out, int64_t n_cap,
                             const int64_t *d_n, uint64_t *tile_sums, int64_t *total, hipStream_t s) {
    if (word_bits == 64)
        return scan_generic(RowPop<uint64_t>{static_cast<const uint64_t *>(rows), words}, out, n_cap, d_n,
                            tile_sums, out, total, nullptr, s);
    return scan_generic(RowPop<uint32_t>{static_cast<const uint32_t *>(rows), words}, out, n_cap, d_n,
                        tile_sums, out, total, nullptr, s);
}

int64_t radix_hist_entries(int64_t n_cap) {
    return static_cast<int64_t>(RADIX) * (blocks_for(n_cap, RS_TILE) + 1);  // tile rows + digit totals
}

cg_status radix_sort_u64(uint64_t *keys[2], uint32_t *vals[2], int64_t n_cap, const int64_t *d_n, int bit_lo,
                         int bit_hi, uint32_t *hist, uint64_t *tile_sums, int *which, hipStream_t s,
                         const unsigned long long *skip, int skip_below) {
    const int num_tiles = static_cast<int>(blocks_for(n_cap, RS_TILE));
    (void)tile_sums;
    int cur = 0;
    for (int shift = bit_lo; shift < bit_hi; shift += 8) {
        // passes below skip_below do nothing when *skip is set; skipping an even
        // number of leading passes leaves the data where the host expects it
        const unsigned long long *sk = shift < skip_below ? skip : nullptr;
        hipLaunchKernelGGL(k_radix_hist, dim3(num_tiles), dim3(RS_THREADS), 0, s, keys[cur], n_cap, d_n, shift,
                           hist, num_tiles, sk);
        CG_LAUNCHED("radix_hist");
        uint32_t *dtot = hist + static_cast<int64_t>(RADIX) * num_tiles;  // digit totals after the rows
        hipLaunchKernelGGL(k_radix_dscan, dim3(RADIX), dim3(RS_THREADS), 0, s, hist, num_tiles, dtot, sk);
        CG_LAUNCHED("radix_dscan");
        if (vals) {
            hipLaunchKernelGGL((k_radix_scatter<true>), dim3(num_tiles), dim3(RS_THREADS), 0, s, keys[cur],
                               vals[cur], keys[cur ^ 1], vals[cur ^ 1], n_cap, d_n, shift, hist, dtot, num_tiles, sk);
        } else {
            hipLaunchKernelGGL((k_radix_scatter<false>), dim3(num_tiles), dim3(RS_THREADS), 0, s, keys[cur],
                               static_cast<const uint32_t *>(nullptr), keys[cur ^ 1], static_cast<uint32_t *>(nullptr),
                               n_cap, d_n, shift, hist, dtot, num_tiles, sk);
        }
        CG_LAUNCHED("radix_scatter");
        cur ^= 1;
    }
    *which = cur;
    return CG_OK;
}

cg_status radix_sort_k32(uint32_t *planes[3][2], int nplanes, uint32_t *vals[2], int64_t n_cap, const int64_t *d_n,
                         int bit_lo, uint32_t *hist, int *which, hipStream_t s, bool lower_planes,
                         const unsigned long long *key32) {
    const int num_tiles = static_cast<int>(blocks_for(n_cap, RS_TILE));
    uint32_t *dtot = hist + static_cast<int64_t>(RADIX) * num_tiles;  // digit totals after the rows
    uint32_t *none[2] = {nullptr, nullptr};
    int cur = 0;
    for (int bit = bit_lo; bit < 32 * nplanes; bit += 8) {
        // the pass's plane (planes[0] most significant) and the other planes,
        // carried as payloads: planes above it always (their passes follow),
        // planes below it while they are wanted after the sort
        const int q = nplanes - 1 - bit / 32;
        uint32_t *const *o1 = none, *const *o2 = none;
        for (int r = 0; r < nplanes; ++r) {
            if (r == q || (r > q && !lower_planes)) continue;
            if (o1 == none) o1 = planes[r]; else o2 = planes[r];
        }
        // with two planes the device may have chosen 32-bit keys: the low
        // plane's passes do nothing, and the high plane's drop it
        const bool low2 = nplanes == 2 && q == 1;
        const unsigned long long *sk = low2 ? key32 : nullptr;
        const unsigned long long *drop = (nplanes == 2 && q == 0) ? key32 : nullptr;
        hipLaunchKernelGGL(k_radix32_hist, dim3(num_tiles), dim3(RS_THREADS), 0, s, planes[q][cur], n_cap, d_n,
                           bit & 31, hist, num_tiles, sk);
        CG_LAUNCHED("radix32_hist");
        hipLaunchKernelGGL(k_radix_dscan, dim3(RADIX), dim3(RS_THREADS), 0, s, hist, num_tiles, dtot, sk);
        CG_LAUNCHED("radix32_dscan");
        const int np = o2 != none ? 2 : (o1 != none ? 1 : 0);
#define CG_SCATTER32(NPV)                                                                                          \
    hipLaunchKernelGGL((k_radix32_scatter<NPV>), dim3(num_tiles), dim3(RS_THREADS), 0, s, planes[q][cur], vals[cur], \
                       o1[cur], o2[cur], planes[q][cur ^ 1], vals[cur ^ 1], o1[cur ^ 1], o2[cur ^ 1], n_cap, d_n,    \
                       bit & 31, hist, dtot, num_tiles, sk, drop)
        if (np == 2) CG_SCATTER32(2);
        else if (np == 1) CG_SCATTER32(1);
        else CG_SCATTER32(0);
#undef CG_SCATTER32
        CG_LAUNCHED("radix32_scatter");
        cur ^= 1;
    }
    *which = cur;
    return CG_OK;
}

cg_status fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return CG_OK;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
    CG_LAUNCHED("fill_u32");
    return CG_OK;
}

cg_status fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return CG_OK;
    hipLaunchKernelGGL(k_fill_i64, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
    CG_LAUNCHED("fill_i64");
    return CG_OK;
}

}  // namespace cg
