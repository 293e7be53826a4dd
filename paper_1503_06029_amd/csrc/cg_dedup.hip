// Dedup: sort the packed rows lexicographically and drop duplicates
// (Section 3.2: radix sort of X with duplicate removal; Section 2.2: X may be
// a multiset).
//
// 1. extract: key = the first 64 bits of each row (x(0) most significant),
//    value = row index;
// 2. LSD radix sort of (key, index) over the key bits that can be nonzero;
// 3. rows with equal keys form segments; when l > 64 each segment of two or
//    more rows is ordered by the full row: segments of up to `smax` rows in
//    the LDS of the block whose tile holds their first position (rank sort),
//    up to LMAX rows by one block each (bitonic network over (next 64 bits,
//    index) pairs in LDS), longer ones by one block each (bitonic network over
//    an index array in global memory);
// 4. a row is a new cell iff it differs from its predecessor; a scan of those
//    flags gives cell ids, and a gather writes the cells and row_to_cell.
#include "cg_internal.hpp"

namespace cg {

namespace {

constexpr uint32_t SENT = 0xFFFFFFFFu;
constexpr int64_t TILE_LDS = 53248;  // three blocks per CU
constexpr int LMAX = 8192;          // longest segment sorted in one block's LDS (96 KB of it)
// Rows longer than 64 bits are sorted on their first 64 bits, or on their
// first 32 when a sample shows those already separate the rows (then the
// four low radix passes are skipped); equal-key segments are finished by
// full-row comparison either way.  counters[2] holds the choice (1: 32).
constexpr int PROBE = 4096;        // sampled rows
constexpr int PROBE_TIES = 128;    // at most this many equal neighbours (about 3 %) for 32-bit keys
constexpr int64_t PROBE_MIN_N = 1 << 20;

// One block: the top 32 bits of PROBE rows spread over the input go into an
// LDS hash set; if at most PROBE_TIES of them were already present, 32-bit
// keys are chosen (counters[2] = 1), else 64-bit keys (0).
constexpr int PROBE_SLOTS = 2 * PROBE;
template <typename T>
__global__ void __launch_bounds__(1024) k_key_probe(const T *__restrict__ rows, int64_t n, int words,
                                                    unsigned long long *__restrict__ counters) {
    __shared__ uint32_t tab[PROBE_SLOTS];
    __shared__ int ties;
    const int t = threadIdx.x;
    if (t == 0) ties = 0;
    for (int i = t; i < PROBE_SLOTS; i += 1024) tab[i] = 0xFFFFFFFFu;
    __syncthreads();
    int local = 0;
    for (int i = t; i < PROBE; i += 1024) {
        const int64_t r = static_cast<int64_t>(i) * n / PROBE;
        uint32_t k = static_cast<uint32_t>(head64<T>(rows + r * words, words) >> 32);
        if (k == 0xFFFFFFFFu) k = 0xFFFFFFFEu;  // the empty mark
        uint32_t h = (k * 0x9E3779B1u) >> 19;   // 13 bits: PROBE_SLOTS = 8192
        for (int step = 0; step < PROBE_SLOTS; ++step) {
            const uint32_t old = atomicCAS(&tab[h], 0xFFFFFFFFu, k);
            if (old == 0xFFFFFFFFu) break;
            if (old == k) { ++local; break; }
            h = (h + 1) & (PROBE_SLOTS - 1);
        }
    }
    if (local) atomicAdd(&ties, local);
    __syncthreads();
    if (t == 0) counters[2] = ties <= PROBE_TIES ? 1ull : 0ull;
}

template <typename T>
__global__ void __launch_bounds__(256) k_extract(const T *__restrict__ rows, int64_t n, int words,
                                                 const unsigned long long *__restrict__ key32,
                                                 uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const uint64_t kmask = (key32 && *key32) ? 0xFFFFFFFF00000000ull : ~0ull;
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < n;
         j += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        keys[j] = head64<T>(rows + j * words, words) & kmask;
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

// l <= 64: the key is the whole row, so a row is a new cell iff its key
// differs from its predecessor's.
__global__ void __launch_bounds__(256) k_heads(const uint64_t *__restrict__ keys, int64_t n,
                                               uint8_t *__restrict__ uniq) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j < n) uniq[j] = ((j == 0) || keys[j] != keys[j - 1]) ? 1 : 0;
}

// One block per tile of PT sorted positions (l > 64).  The tile owns the
// segments (runs of equal keys) whose first position lies in it; a segment of
// 2..smax rows may reach up to smax positions past the tile.  The rows of the
// owned multi-row segments are gathered into LDS (slot = position - tile
// start), every row computes its rank within its segment by comparing the
// remaining words with all others (ties broken by position), and the sorted
// row indices and first-of-equal-run flags are written back.  Singletons are
// flagged unique; longer segments go to the large-segment list (rare, so one
// atomic each is fine).
constexpr int TT = 256;

template <typename T>
__global__ void __launch_bounds__(TT) k_tiefix_tile(const T *__restrict__ rows, const uint64_t *__restrict__ keys,
                                                    int64_t n, int words, int from64, int smax,
                                                    uint32_t *__restrict__ vals, uint8_t *__restrict__ uniq,
                                                    uint2 *__restrict__ large_list,
                                                    unsigned long long *__restrict__ counters) {
    const int from = counters[2] ? from64 / 2 : from64;  // words covered by the sort key
    extern __shared__ __align__(16) unsigned char smem[];
    const int LW = words + ((words & 1) ? 0 : 1);
    const int slots = TT + smax;
    // keys of positions b0 - 1 .. b0 + slots - 1 (index = position - b0 + 1)
    uint64_t *skeys = reinterpret_cast<uint64_t *>(smem);
    T *lrows = reinterpret_cast<T *>(skeys + slots + 1);
    // with smax == 1 no segment is small and the row area is not allocated
    int32_t *segof = reinterpret_cast<int32_t *>(lrows + (smax > 1 ? static_cast<size_t>(slots) * LW : 0));
    int32_t *seglen = segof + slots;
    uint32_t *sval = reinterpret_cast<uint32_t *>(seglen + slots);
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * TT;
    const int t = threadIdx.x;
    const int64_t wend = (b0 + slots < n) ? b0 + slots : n;  // window end (exclusive)
    for (int e0 = t; e0 <= slots; e0 += TT * 4) {
        uint64_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t pos = b0 - 1 + e0 + u * TT;
            v[u] = (e0 + u * TT <= slots && pos >= 0 && pos < wend) ? keys[pos] : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (e0 + u * TT <= slots) skeys[e0 + u * TT] = v[u];
    }
    for (int r = t; r < slots; r += TT) segof[r] = -1;
    __syncthreads();
    const int64_t p = b0 + t;
    bool large = false;
    uint2 seg = make_uint2(0u, 0u);
    if (p < n) {
        const uint64_t k = skeys[t + 1];
        const bool head = (p == 0) || k != skeys[t];
        if (head) {
            int64_t e = p + 1;
            while (e < wend && skeys[e - b0 + 1] == k) ++e;
            if (e == wend && e < n) e = run_end(keys, p, n);  // reaches past the window: long segment
            const int64_t len = e - p;
            if (len == 1) {
                uniq[p] = 1;
            } else if (len <= smax) {
                for (int r = 0; r < len; ++r) {
                    segof[t + r] = t;
                    seglen[t + r] = static_cast<int32_t>(len);
                }
            } else {
                large = true;
                seg = make_uint2(static_cast<uint32_t>(p), static_cast<uint32_t>(len));
            }
        }
    }
    wave_append<uint2>(large_list, &counters[1], n, large, seg);
    __syncthreads();
    for (int r0 = t; r0 < slots; r0 += TT * 4) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = r0 + u * TT;
            v[u] = (r < slots && segof[r] >= 0) ? vals[b0 + r] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = r0 + u * TT;
            if (r < slots && segof[r] >= 0) sval[r] = v[u];
        }
    }
    __syncthreads();
    constexpr int U = 16;
    for (int e0 = t; e0 < slots * words; e0 += TT * U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * TT;
            const int r = e / words;
            v[u] = (e < slots * words && segof[r] >= 0) ? rows[static_cast<int64_t>(sval[r]) * words + (e - r * words)]
                                                        : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * TT;
            const int r = e / words;
            if (e < slots * words && segof[r] >= 0) lrows[r * LW + (e - r * words)] = v[u];
        }
    }
    __syncthreads();
    for (int r = t; r < slots; r += TT) {
        const int a = segof[r];
        if (a < 0) continue;
        const int len = seglen[r];
        const T *me = lrows + r * LW;
        int rank = 0;
        bool dup = false;
        for (int j = a; j < a + len; ++j) {
            if (j == r) continue;
            const int c = row_cmp<T>(lrows + j * LW, me, words, from);
            if (c < 0 || (c == 0 && j < r)) ++rank;
            if (c == 0 && j < r) dup = true;
        }
        vals[b0 + a + rank] = sval[r];
        uniq[b0 + a + rank] = dup ? 0 : 1;
    }
}

// Same, with rows zero-padded to WT words in LDS (WT a power of two fixed at
// compile time): the copy and every comparison are straight-line code.
template <typename T, int WT, int FROM>
__device__ __forceinline__ int lex_cmp_t(const T *a, const T *b) {
    // words before FROM are covered by the sort key
    int res = 0;
#pragma unroll
    for (int w = WT - 1; w >= FROM; --w) {
        const T x = a[w], y = b[w];
        res = (x != y) ? (x < y ? -1 : 1) : res;
    }
    return res;
}

// KB is the sort key's width in bits (32 or 64); the kernel for the width
// not chosen by the probe (counters[2]) returns at once.
template <typename T, int WT, int KB>
__global__ void __launch_bounds__(TT) k_tiefix_t(const T *__restrict__ rows, const uint64_t *__restrict__ keys,
                                                 int64_t n, int words, int smax, uint32_t *__restrict__ vals,
                                                 uint8_t *__restrict__ uniq, uint2 *__restrict__ large_list,
                                                 unsigned long long *__restrict__ counters) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int LW = WT + 1;
    if ((counters[2] != 0) != (KB == 32)) return;
    constexpr int FROM = KB / Bits<T>::B;  // words covered by the sort key
    const int slots = TT + smax;
    uint64_t *skeys = reinterpret_cast<uint64_t *>(smem);  // positions b0 - 1 .. b0 + slots - 1
    T *lrows = reinterpret_cast<T *>(skeys + slots + 1);
    int32_t *segof = reinterpret_cast<int32_t *>(lrows + static_cast<size_t>(slots) * LW);
    int32_t *seglen = segof + slots;
    uint32_t *sval = reinterpret_cast<uint32_t *>(seglen + slots);
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * TT;
    const int t = threadIdx.x;
    const int64_t wend = (b0 + slots < n) ? b0 + slots : n;
    // keys of the window and the row indices of its positions, loaded together
    for (int e0 = t; e0 <= slots; e0 += TT * 4) {
        uint64_t v[4];
        uint32_t x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t pos = b0 - 1 + e0 + u * TT;
            const bool in = e0 + u * TT <= slots && pos >= 0 && pos < wend;
            v[u] = in ? keys[pos] : 0;
            x[u] = (in && pos >= b0) ? vals[pos] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * TT;
            if (e <= slots) skeys[e] = v[u];
            if (e >= 1 && e <= slots) sval[e - 1] = x[u];
        }
    }
    for (int r = t; r < slots; r += TT) segof[r] = -1;
    __syncthreads();
    const int64_t p = b0 + t;
    bool large = false;
    uint2 seg = make_uint2(0u, 0u);
    if (p < n) {
        const uint64_t k = skeys[t + 1];
        if (p == 0 || k != skeys[t]) {
            int64_t e = p + 1;
            while (e < wend && skeys[e - b0 + 1] == k) ++e;
            if (e == wend && e < n) e = run_end(keys, p, n);
            const int64_t len = e - p;
            if (len == 1) {
                uniq[p] = 1;
            } else if (len <= smax) {
                for (int r = 0; r < len; ++r) {
                    segof[t + r] = t;
                    seglen[t + r] = static_cast<int32_t>(len);
                }
            } else {
                large = true;
                seg = make_uint2(static_cast<uint32_t>(p), static_cast<uint32_t>(len));
            }
        }
    }
    wave_append<uint2>(large_list, &counters[1], n, large, seg);
    __syncthreads();

    constexpr int U = 16;
    const int tot = slots * WT;
    for (int e0 = t; e0 < tot; e0 += TT * U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * TT;
            const int r = e / WT, w = e % WT;
            v[u] = (e < tot && w < words && segof[r] >= 0) ? rows[static_cast<int64_t>(sval[r]) * words + w] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * TT;
            if (e < tot) lrows[(e / WT) * LW + (e % WT)] = v[u];
        }
    }
    __syncthreads();
    // Summary of each row against its segment's first row a: the first word
    // f (past the sort key) where they differ (WT if equal), the row's word
    // there and the first row's word there.  Two rows then compare by their
    // summaries alone unless they differ from row a first in the same word
    // with the same value (a tie, settled by comparing the rows).
    uint8_t *sf = reinterpret_cast<uint8_t *>(sval + slots);
    // 8-byte aligned offset from the LDS base (offset arithmetic keeps the
    // pointer in the LDS address space: a round trip through an integer
    // address would turn every access into a flat memory access)
    const ptrdiff_t sv_off = ((sf + slots) - reinterpret_cast<uint8_t *>(smem) + 7) & ~ptrdiff_t(7);
    T *sv = reinterpret_cast<T *>(smem + sv_off);
    T *shv = sv + slots;
    for (int r = t; r < slots; r += TT) {
        const int a = segof[r];
        if (a < 0) continue;
        const T *me = lrows + r * LW, *hd = lrows + a * LW;
        int f = WT;
        T v = 0, h = 0;
#pragma unroll
        for (int w = WT - 1; w >= FROM; --w) {
            const T x = me[w], y = hd[w];
            const bool ne = x != y;
            f = ne ? w : f;
            v = ne ? x : v;
            h = ne ? y : h;
        }
        sf[r] = static_cast<uint8_t>(f);
        sv[r] = v;
        shv[r] = h;
    }
    __syncthreads();
    for (int r = t; r < slots; r += TT) {
        const int a = segof[r];
        if (a < 0) continue;
        const int len = seglen[r];
        const int fm = sf[r];
        const T vm = sv[r], hm = shv[r];
        int rank = 0;
        bool dup = false;
        unsigned long long tie[2] = {0ull, 0ull};  // j - a of tied rows (len <= 128)
#pragma unroll 4
        for (int j = a; j < a + len; ++j) {
            const int fj = sf[j];
            const T vj = sv[j], hj = shv[j];
            // compare row j with row r, branch-free; 2 marks a tie
            const int c_lt = vj < hj ? -1 : 1;   // j leaves the first row first
            const int c_gt = hm < vm ? -1 : 1;   // r leaves it first
            const int c_eq = fj == WT ? 0 : (vj != vm ? (vj < vm ? -1 : 1) : 2);
            const int c = fj < fm ? c_lt : (fj > fm ? c_gt : c_eq);
            const bool before = j < r;
            rank += (c == -1 || (c == 0 && before)) ? 1 : 0;
            dup = dup || (c == 0 && before);
            const int o = j - a;
            if (c == 2 && j != r) tie[o >> 6] |= 1ull << (o & 63);
        }
        // ties: compare the rows themselves
        const T *me = lrows + r * LW;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            unsigned long long m = tie[h];
            while (m) {
                const int j = a + h * 64 + __ffsll(m) - 1;
                m &= m - 1;
                const int c = lex_cmp_t<T, WT, FROM>(lrows + j * LW, me);
                rank += (c < 0 || (c == 0 && j < r)) ? 1 : 0;
                dup = dup || (c == 0 && j < r);
            }
        }
        vals[b0 + a + rank] = sval[r];
        uniq[b0 + a + rank] = dup ? 0 : 1;
    }
}

template <typename T, int WT>
size_t tiefix_t_lds(int smax) {
    const size_t slots = static_cast<size_t>(TT + smax);
    return (slots + 1) * 8 + slots * ((WT + 1) * sizeof(T) + 12) + slots + 8 + 2 * slots * sizeof(T);
}

template <typename T, int WT>
int tiefix_t_smax() {
    const int64_t per = (WT + 3) * static_cast<int64_t>(sizeof(T)) + 21;
    int64_t smax = (TILE_LDS - 16) / per - TT - 1;
    if (smax > 128) smax = 128;  // the rank loop's tie masks cover 128 rows
    return static_cast<int>(smax);
}

template <typename T, int WT>
cg_status tiefix_t_launch(const T *rows, const uint64_t *keys, int64_t n, int words, uint32_t *vals, uint8_t *uniq,
                          uint2 *large_list, unsigned long long *counters, bool probed, hipStream_t s) {
    const int smax = tiefix_t_smax<T, WT>();
    const size_t lds = tiefix_t_lds<T, WT>(smax);
    hipLaunchKernelGGL((k_tiefix_t<T, WT, 64>), dim3(blocks_for(n, TT)), dim3(TT), lds, s, rows, keys, n, words, smax,
                       vals, uniq, large_list, counters);
    CG_LAUNCHED("dedup_tiefix_t");
    if (probed) {  // the probe may have chosen 32-bit keys
        hipLaunchKernelGGL((k_tiefix_t<T, WT, 32>), dim3(blocks_for(n, TT)), dim3(TT), lds, s, rows, keys, n, words,
                           smax, vals, uniq, large_list, counters);
        CG_LAUNCHED("dedup_tiefix_t32");
    }
    return CG_OK;
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
__global__ void __launch_bounds__(1024) k_tiefix_large(const T *__restrict__ rows, int words, int from64,
                                                      const uint2 *__restrict__ list,
                                                      const unsigned long long *__restrict__ counters, uint32_t *vals,
                                                      uint8_t *uniq, uint32_t *scratch) {
    const int from = counters[2] ? from64 / 2 : from64;  // words covered by the sort key
    const uint32_t count = static_cast<uint32_t>(counters[1]);
    for (uint32_t s = blockIdx.x; s < count; s += gridDim.x) {
        const uint2 seg = list[s];
        const int64_t a = seg.x;
        const int64_t len = seg.y;
        if (len <= LMAX) continue;  // k_tiefix_mid took it
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

// Segments longer than the tile kernel takes, up to LMAX rows: one block per
// segment sorts (next 64 bits of the row, row index) pairs by a bitonic
// network in LDS; pairs whose 64-bit values tie compare the rest of the rows
// in global memory.  Then a row is flagged new iff it differs from its
// predecessor in the segment.
template <typename T>
__device__ __forceinline__ uint64_t key2_of(const T *row, int words, int from);
template <>
__device__ __forceinline__ uint64_t key2_of<uint64_t>(const uint64_t *row, int words, int from) {
    return from < words ? row[from] : 0ull;
}
template <>
__device__ __forceinline__ uint64_t key2_of<uint32_t>(const uint32_t *row, int words, int from) {
    const uint64_t hi = from < words ? row[from] : 0u;
    const uint64_t lo = from + 1 < words ? row[from + 1] : 0u;
    return (hi << 32) | lo;
}

template <typename T>
__global__ void __launch_bounds__(1024) k_tiefix_mid(const T *__restrict__ rows, int words, int from64,
                                                     const uint2 *__restrict__ list,
                                                     const unsigned long long *__restrict__ counters,
                                                     uint32_t *__restrict__ vals, uint8_t *__restrict__ uniq) {
    const int from = counters[2] ? from64 / 2 : from64;  // words covered by the sort key
    extern __shared__ __align__(16) unsigned char smem[];  // LMAX keys, then LMAX indices
    uint64_t *sk = reinterpret_cast<uint64_t *>(smem);
    uint32_t *si = reinterpret_cast<uint32_t *>(smem + LMAX * sizeof(uint64_t));
    constexpr int K2 = 64 / Bits<T>::B;  // words covered by the second key
    const int from2 = from + K2;
    const uint32_t count = static_cast<uint32_t>(counters[1]);
    for (uint32_t sgi = blockIdx.x; sgi < count; sgi += gridDim.x) {
        const uint2 seg = list[sgi];
        const int64_t a = seg.x;
        const int len = static_cast<int>(seg.y);
        if (len > LMAX) continue;  // k_tiefix_large takes it
        int P = 1;
        while (P < len) P <<= 1;
        for (int i = threadIdx.x; i < P; i += blockDim.x) {
            if (i < len) {
                const uint32_t v = vals[a + i];
                si[i] = v;
                sk[i] = key2_of<T>(rows + static_cast<int64_t>(v) * words, words, from);
            } else {
                si[i] = SENT;
                sk[i] = ~0ull;
            }
        }
        __syncthreads();
        for (int k = 2; k <= P; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < P; i += blockDim.x) {
                    const int p = i ^ j;
                    if (p > i) {
                        const uint64_t ka = sk[i], kb = sk[p];
                        const uint32_t ia = si[i], ib = si[p];
                        bool a_gt;
                        if (ka != kb) {
                            a_gt = ka > kb;
                        } else if (ia == SENT || ib == SENT) {
                            a_gt = ia == SENT;
                        } else {
                            const int c = row_cmp<T>(rows + static_cast<int64_t>(ia) * words,
                                                     rows + static_cast<int64_t>(ib) * words, words, from2);
                            a_gt = c > 0 || (c == 0 && ia > ib);
                        }
                        if (((i & k) == 0) == a_gt) {
                            sk[i] = kb; sk[p] = ka;
                            si[i] = ib; si[p] = ia;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (int i = threadIdx.x; i < len; i += blockDim.x) {
            const uint32_t x = si[i];
            vals[a + i] = x;
            bool u = true;
            if (i > 0 && sk[i - 1] == sk[i])
                u = row_cmp<T>(rows + static_cast<int64_t>(x) * words, rows + static_cast<int64_t>(si[i - 1]) * words,
                               words, from2) != 0;
            uniq[a + i] = u ? 1 : 0;
        }
        __syncthreads();
    }
}

template <typename V>
__global__ void __launch_bounds__(256) k_gather(const V *__restrict__ rows, int64_t n, int pieces,
                                                const uint32_t *__restrict__ vals, const uint8_t *__restrict__ uniq,
                                                const uint32_t *__restrict__ cidx, V *__restrict__ cells,
                                                uint32_t *__restrict__ row_to_cell) {
    const int64_t total = n * pieces;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t j = g / pieces;
        const int w = static_cast<int>(g - j * pieces);
        const uint32_t u = uniq[j];
        const uint32_t cid = cidx[j] + u - 1;
        const uint32_t src = vals[j];
        if (u) cells[static_cast<int64_t>(cid) * pieces + w] = rows[static_cast<int64_t>(src) * pieces + w];
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
    uint2 *large_list;
    unsigned long long *counters;
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
    w.counters = c.take<unsigned long long>(4);
    if (lay.ell > 64) {
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

    const bool tiefix = lay.ell > 64;
    const bool probe = tiefix && n >= PROBE_MIN_N;
    CG_TRY(fill_i64(reinterpret_cast<int64_t *>(w.counters), 0, 4, s));
    if (probe) {
        hipLaunchKernelGGL((k_key_probe<T>), dim3(1), dim3(1024), 0, s, rows, n, words, w.counters);
        CG_LAUNCHED("dedup_key_probe");
    }
    hipLaunchKernelGGL((k_extract<T>), dim3(blocks_for(n, 256, 16384)), dim3(256), 0, s, rows, n, words,
                       probe ? w.counters + 2 : nullptr, w.keys[0], w.vals[0]);
    CG_LAUNCHED("dedup_extract");

    // key bits that can be nonzero: [64 - sig, 64); with 32-bit keys the four
    // passes below bit 32 find every digit zero and are skipped on the device
    const int sig = tiefix ? 64 : lay.ell;
    const int lo = ((64 - sig) / 8) * 8;
    int which = 0;
    CG_TRY(radix_sort_u64(w.keys, w.vals, n, nullptr, lo, 64, w.hist, w.tile_sums, &which, s,
                          probe ? w.counters + 2 : nullptr, 32));
    uint64_t *keys = w.keys[which];
    uint32_t *vals = w.vals[which];

    const int B = static_cast<int>(sizeof(T) * 8);
    const int from = 64 / B;  // words covered by a 64-bit sort key (the mid pass halves it for 32)
    if (!tiefix) {
        hipLaunchKernelGGL(k_heads, dim3(blocks_for(n, 256)), dim3(256), 0, s, keys, n, w.uniq);
        CG_LAUNCHED("dedup_heads");
    } else {
        const int LW = words + ((words % 2 == 0) ? 1 : 0);
        const int64_t per_slot = static_cast<int64_t>(LW) * sizeof(T) + 20;
        int64_t smax = TILE_LDS / per_slot - TT - 1;
        if (smax > 512) smax = 512;
        size_t lds = static_cast<size_t>(TT + smax) * per_slot + 8;
        if (smax < 2) {  // rows too wide for LDS: every multi-row segment takes the large path
            smax = 1;
            lds = static_cast<size_t>(TT + 1) * 20 + 8;
        }
        int wt = 1;
        while (wt < words) wt <<= 1;
        const int wcap = sizeof(T) == 8 ? 16 : 32;
        if (wt <= wcap) {  // every such width leaves room for segments of 80+ rows
            switch (wt) {
            case 2: CG_TRY((tiefix_t_launch<T, 2>(rows, keys, n, words, vals, w.uniq, w.large_list, w.counters, probe, s))); break;
            case 4: CG_TRY((tiefix_t_launch<T, 4>(rows, keys, n, words, vals, w.uniq, w.large_list, w.counters, probe, s))); break;
            case 8: CG_TRY((tiefix_t_launch<T, 8>(rows, keys, n, words, vals, w.uniq, w.large_list, w.counters, probe, s))); break;
            case 16: CG_TRY((tiefix_t_launch<T, 16>(rows, keys, n, words, vals, w.uniq, w.large_list, w.counters, probe, s))); break;
            default: CG_TRY((tiefix_t_launch<T, 32>(rows, keys, n, words, vals, w.uniq, w.large_list, w.counters, probe, s))); break;
            }
        } else {
            hipLaunchKernelGGL((k_tiefix_tile<T>), dim3(blocks_for(n, TT)), dim3(TT), lds, s, rows, keys, n, words,
                               from, static_cast<int>(smax), vals, w.uniq, w.large_list, w.counters);
            CG_LAUNCHED("dedup_tiefix_tile");
        }
        const size_t mid_lds = static_cast<size_t>(LMAX) * (sizeof(uint64_t) + sizeof(uint32_t));
        CG_TRY(allow_lds(reinterpret_cast<const void *>(&k_tiefix_mid<T>), mid_lds));
        hipLaunchKernelGGL((k_tiefix_mid<T>), dim3(1024), dim3(1024), mid_lds, s, rows, words, from, w.large_list,
                           w.counters, vals, w.uniq);
        CG_LAUNCHED("dedup_tiefix_mid");
        hipLaunchKernelGGL((k_tiefix_large<T>), dim3(256), dim3(1024), 0, s, rows, words, from, w.large_list,
                           w.counters, vals, w.uniq, w.scratch);
        CG_LAUNCHED("dedup_tiefix_large");
    }
    CG_TRY(scan_u8_to_u32(w.uniq, w.cidx, n, nullptr, w.tile_sums, d_ncells, s));
    const size_t rowbytes = static_cast<size_t>(words) * sizeof(T);
    if (rowbytes % 16 == 0) {
        const int pieces = static_cast<int>(rowbytes / 16);
        hipLaunchKernelGGL((k_gather<uint4>), dim3(blocks_for(n * pieces, 256, 65536)), dim3(256), 0, s,
                           reinterpret_cast<const uint4 *>(rows), n, pieces, vals, w.uniq, w.cidx,
                           reinterpret_cast<uint4 *>(cells), row_to_cell);
    } else {
        hipLaunchKernelGGL((k_gather<T>), dim3(blocks_for(n * words, 256, 65536)), dim3(256), 0, s, rows, n, words,
                           vals, w.uniq, w.cidx, cells, row_to_cell);
    }
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
