// Dedup: sort the packed rows lexicographically and drop duplicates
// (Section 3.2: radix sort of X with duplicate removal; Section 2.2: X may be
// a multiset).
//
// 1. extract: key = the first 64 bits of each row (x(0) most significant),
//    value = row index;
// 2. LSD radix sort of (key, index) over the key bits that can be nonzero;
// 3. rows with equal keys form segments; when l > 64 each segment of two or
//    more rows is ordered by the full row: segments of up to 128 rows by the
//    block whose tile holds their first position (rank sort over row
//    summaries taken against the segment's first row), up to LMAX rows by one
//    block each (bitonic network over (next 64 bits, index) pairs in LDS;
//    256-thread blocks up to 2,048 rows, 1,024-thread blocks beyond),
//    longer ones by one block each (bitonic network over an index array in
//    global memory);
// 4. a row is a new cell iff it differs from its predecessor; a scan of those
//    flags gives cell ids, and a gather writes the cells and row_to_cell.
#include "cg_internal.hpp"

namespace cg {

namespace {

constexpr uint32_t SENT = 0xFFFFFFFFu;
constexpr int64_t TILE_LDS = 53248;  // three blocks per CU
constexpr int LMAX = 8192;          // longest segment sorted in one block's LDS (96 KB of it)
// The sort key lives in up to three 32-bit planes: p0 = the row's first 32
// bits, p1 = the next 32, p2 = the 32 after those (absent planes are not
// part of the key).  Read as (first 64 bits, next 32) with absent planes 0.
struct Key96 {
    uint64_t a;
    uint32_t b;
    __device__ __forceinline__ bool operator==(const Key96 &o) const { return a == o.a && b == o.b; }
    __device__ __forceinline__ bool operator!=(const Key96 &o) const { return !(*this == o); }
};
struct KeyPlanes {
    const uint32_t *p0;
    const uint32_t *p1;
    const uint32_t *p2;
    __device__ __forceinline__ Key96 operator[](int64_t i) const {
        return Key96{(static_cast<uint64_t>(p0[i]) << 32) | (p1 ? p1[i] : 0u), p2 ? p2[i] : 0u};
    }
    // the planes of a key of kbits bits
    __device__ __forceinline__ KeyPlanes width(int kbits) const {
        return KeyPlanes{p0, kbits > 32 ? p1 : nullptr, kbits > 64 ? p2 : nullptr};
    }
};

// Key width chosen for this call: 96 when the caller asked for it
// (counters[3]), else 32 when chosen by the caller or the sample
// (counters[2]), else 64.
__device__ __forceinline__ int key_width(const unsigned long long *counters) {
    return counters[3] ? 96 : (counters[2] ? 32 : 64);
}

// Bits 64 .. 95 of a row (0 past its end).
template <typename T> __device__ __forceinline__ uint32_t head_third(const T *row, int words);
template <> __device__ __forceinline__ uint32_t head_third<uint64_t>(const uint64_t *row, int words) {
    return words > 1 ? static_cast<uint32_t>(row[1] >> 32) : 0u;
}
template <> __device__ __forceinline__ uint32_t head_third<uint32_t>(const uint32_t *row, int words) {
    return words > 2 ? row[2] : 0u;
}

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

// The dedup's device counters (long-segment list length, the key-width
// flags: [2] 32-bit keys, [3] 96-bit keys) and, for the fused build, the
// dictionary's gap-list counters: set by block 0 of the key extraction, or
// by a launch of their own before the sample (which sets [2]).
struct DedupInit {
    unsigned long long *counters;  // null: already set
    unsigned long long key32, key96;
    unsigned long long *extra;
    int n_extra;
    __device__ __forceinline__ void run() const {
        const int t = threadIdx.x;
        if (!counters || blockIdx.x != 0) return;
        if (t < 4) counters[t] = t == 2 ? key32 : (t == 3 ? key96 : 0ull);
        if (extra && t < n_extra) extra[t] = 0ull;
    }
};
__global__ void k_dedup_init(DedupInit in) { in.run(); }

template <typename T>
__global__ void __launch_bounds__(256) k_extract(const T *__restrict__ rows, int64_t n, int words,
                                                 const unsigned long long *__restrict__ key32, uint32_t *__restrict__ k0,
                                                 uint32_t *__restrict__ k1, uint32_t *__restrict__ k2,
                                                 uint32_t *__restrict__ vals, DedupInit init) {
    init.run();
    const bool has1 = k1 && !(key32 && *key32);  // the second plane unless the sample chose 32 bits
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < n;
         j += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const T *row = rows + j * words;
        const uint64_t h = head64<T>(row, words);
        k0[j] = static_cast<uint32_t>(h >> 32);
        if (has1) k1[j] = static_cast<uint32_t>(h);
        if (k2) k2[j] = head_third<T>(row, words);
        vals[j] = static_cast<uint32_t>(j);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_hash_rows(const T *__restrict__ rows, int64_t n, int words, int hash_s,
                                                   uint32_t *__restrict__ rhash) {
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < n;
         j += static_cast<int64_t>(gridDim.x) * blockDim.x)
        rhash[j] = suffix_hash32<T>(rows + j * words, words, hash_s);
}

// Key extraction for the fused dedup + dictionary build: a block's 256 rows
// are read whole (coalesced) into LDS, and each thread takes its row's sort
// key and the dictionary's suffix hash of bits hash_s .. from there, so the
// rows' lines are read once for both (the key alone would fetch them anyway).
template <typename T>
__global__ void __launch_bounds__(256) k_extract_hash(const T *__restrict__ rows, int64_t n, int words,
                                                      const unsigned long long *__restrict__ key32,
                                                      uint32_t *__restrict__ k0, uint32_t *__restrict__ k1,
                                                      uint32_t *__restrict__ k2, uint32_t *__restrict__ vals,
                                                      int hash_s, uint32_t *__restrict__ rhash, DedupInit init) {
    init.run();
    extern __shared__ __align__(16) unsigned char smem[];
    T *lrows = reinterpret_cast<T *>(smem);
    const int LW = words | 1;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * 256;
    if (base >= n) return;
    const int tr = static_cast<int>(n - base < 256 ? n - base : 256);
    copy_rows_to_lds<T, 256>(lrows, LW, rows + base * words, tr, words);
    __syncthreads();
    const int t = threadIdx.x;
    if (t >= tr) return;
    const bool has1 = k1 && !(key32 && *key32);
    const T *row = lrows + t * LW;
    const uint64_t h = head64<T>(row, words);
    k0[base + t] = static_cast<uint32_t>(h >> 32);
    if (has1) k1[base + t] = static_cast<uint32_t>(h);
    if (k2) k2[base + t] = head_third<T>(row, words);
    vals[base + t] = static_cast<uint32_t>(base + t);
    rhash[base + t] = suffix_hash32<T>(row, words, hash_s);
}

// End of the run of keys equal to keys[j] (keys sorted ascending): the first
// index e > j with keys[e] != keys[j], or n.
__device__ __forceinline__ int64_t run_end(KeyPlanes keys, int64_t j, int64_t n) {
    const Key96 k = keys[j];
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
__global__ void __launch_bounds__(256) k_heads(KeyPlanes keys, int64_t n, uint8_t *__restrict__ uniq) {
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
__global__ void __launch_bounds__(TT) k_tiefix_tile(const T *__restrict__ rows, KeyPlanes planes, int64_t n,
                                                    int words, int smax,
                                                    uint32_t *__restrict__ vals, uint8_t *__restrict__ uniq,
                                                    uint2 *__restrict__ large_list,
                                                    unsigned long long *__restrict__ counters) {
    const int kbits = key_width(counters);
    const int from = kbits / Bits<T>::B;  // whole words covered by the sort key
    const KeyPlanes keys = planes.width(kbits);
    extern __shared__ __align__(16) unsigned char smem[];
    const int LW = words + ((words & 1) ? 0 : 1);
    const int slots = TT + smax;
    // keys of positions b0 - 1 .. b0 + slots - 1 (index = position - b0 + 1)
    uint64_t *skeys = reinterpret_cast<uint64_t *>(smem);
    uint32_t *skx = reinterpret_cast<uint32_t *>(skeys + slots + 1);  // third planes
    T *lrows = reinterpret_cast<T *>(skx + ((slots + 2) & ~1));
    // with smax == 1 no segment is small and the row area is not allocated
    int32_t *segof = reinterpret_cast<int32_t *>(lrows + (smax > 1 ? static_cast<size_t>(slots) * LW : 0));
    int32_t *seglen = segof + slots;
    uint32_t *sval = reinterpret_cast<uint32_t *>(seglen + slots);
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * TT;
    const int t = threadIdx.x;
    const int64_t wend = (b0 + slots < n) ? b0 + slots : n;  // window end (exclusive)
    for (int e0 = t; e0 <= slots; e0 += TT * 4) {
        Key96 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t pos = b0 - 1 + e0 + u * TT;
            v[u] = (e0 + u * TT <= slots && pos >= 0 && pos < wend) ? keys[pos] : Key96{0, 0};
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (e0 + u * TT <= slots) {
                skeys[e0 + u * TT] = v[u].a;
                skx[e0 + u * TT] = v[u].b;
            }
    }
    for (int r = t; r < slots; r += TT) segof[r] = -1;
    __syncthreads();
    const int64_t p = b0 + t;
    bool large = false;
    uint2 seg = make_uint2(0u, 0u);
    if (p < n) {
        const uint64_t k = skeys[t + 1];
        const uint32_t kx = skx[t + 1];
        const bool head = (p == 0) || k != skeys[t] || kx != skx[t];
        if (head) {
            int64_t e = p + 1;
            while (e < wend && skeys[e - b0 + 1] == k && skx[e - b0 + 1] == kx) ++e;
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

// Segments of 2..WSMAX rows whose first position lies in the block's tile
// of TT positions, ordered by the full row (WT: row words rounded up to a
// power of two, fixed at compile time; KB: the sort key's width in bits, 32
// or 64, and the kernel for the width the probe (counters[2]) did not choose
// returns at once; HB: rows in flight per thread).  Rows stream in with WT
// lanes per row, each lane loading one word of the row and the same word of
// the segment's first row, its head (loaded by every row of the segment, so
// mostly served from cache; no LDS copy of the heads keeps the block near
// 15 KB of LDS), and a ballot over the lanes gives the words where the row and the
// head differ.  Each row keeps an LV-level
// summary against its head (LV = 2 for 64-bit words, 4 for 32-bit words):
//   level c: the (c+1)-th word past the sort key where they differ, as an
//            order code (its index f if the row is below the head there,
//            2 WT - f if above, WT once the rows agree on every word left)
//            and the row's word there;
//   the last level also carries a flag set when they differ in at most LV
//   words.
// Among rows that agree with the head up to some word, the one that leaves
// it there downwards is the smaller, and of two rows leaving it downwards the
// one leaving first is the smaller (upwards: the one leaving last), so rows
// order as their summaries (code, word) level by level do.  Equal summaries
// with both flags set mean equal rows; without, the rows themselves are
// compared (both differ from the head in more than LV words and agree on the
// first LV of them).  A row's rank in its segment (ties broken by position)
// is its sorted position; it is a duplicate iff an equal row precedes it.
// Bits [at, at + nb) of a 192-bit string held most significant first in
// k[0..2] take the nb low bits of v (v < 2^nb; nb <= 64).
__device__ __forceinline__ void put_bits(uint64_t (&k)[3], int at, uint64_t v, int nb) {
    const int w = at >> 6, room = 64 - (at & 63);  // bits left in word w
    if (nb <= room) {
        k[w] |= v << (room - nb);
    } else {
        const int rest = nb - room;  // bits that spill into word w + 1
        k[w] |= v >> rest;
        k[w + 1] |= v << (64 - rest);
    }
}

constexpr int WSMAX = 128;           // longest segment sorted here
constexpr int WSLOTS = TT + WSMAX;   // window: the tile and the longest segment reaching past it

template <typename T, int WT, int KB, int HB = 8>
__global__ void __launch_bounds__(TT) k_tiefix_w(const T *__restrict__ rows, KeyPlanes planes, int64_t n, int words,
                                                 uint32_t *__restrict__ vals,
                                                 uint8_t *__restrict__ uniq, uint2 *__restrict__ large_list,
                                                 unsigned long long *__restrict__ counters) {
    constexpr int FROM = KB / Bits<T>::B;  // words covered by the sort key
    constexpr int NCH = 2 * TT / 64;       // 64-slot chunks of start flags
    constexpr uint32_t GMASK = (WT >= 32) ? 0xFFFFFFFFu : ((1u << WT) - 1u);
    constexpr int RPS = TT / WT;           // rows per TT consecutive elements
    __shared__ uint32_t sval[WSLOTS];
    __shared__ int16_t segof[WSLOTS];       // slot of the row's head, -1 if not sorted here
    __shared__ int16_t seglen[WSLOTS];
    __shared__ int16_t sord[WSLOTS];        // slot of the segment row at each sorted position
    __shared__ uint8_t sfull[WSLOTS];       // per segment head: equal summaries to look at again
    // summary levels per row: 32-bit words keep four for the LDS two 64-bit
    // words take (rows of 32-bit words tend to share more leading words)
    constexpr int LV = sizeof(T) == 4 ? 4 : 2;
    // One pool, used twice: first the window's keys (positions b0 - 1 ..
    // b0 + WSLOTS - 1, with their third planes for 96-bit keys) and the
    // summary levels (per row and level: the code, | flag on the last level,
    // and the row's word there); then each row's summary packed into three
    // 64-bit words for the ranking.
    constexpr size_t P_KEYS = (WSLOTS + 1) * sizeof(uint64_t);
    constexpr size_t P_SV = P_KEYS;
    constexpr size_t P_SKX = P_SV + LV * WSLOTS * sizeof(T);
    constexpr size_t P_SCODE = P_SKX + (WSLOTS + 1) * sizeof(uint32_t);
    constexpr size_t P_END = P_SCODE + LV * WSLOTS;
    constexpr size_t P_PACKED = 3 * WSLOTS * sizeof(uint64_t);
    __shared__ __align__(16) unsigned char pool[P_END > P_PACKED ? P_END : P_PACKED];
    uint64_t *skeys = reinterpret_cast<uint64_t *>(pool);
    T *sv = reinterpret_cast<T *>(pool + P_SV);
    uint32_t *skx = reinterpret_cast<uint32_t *>(pool + P_SKX);
    uint8_t *scode = pool + P_SCODE;
    uint64_t *pk = reinterpret_cast<uint64_t *>(pool);  // pk[3 r .. 3 r + 2]: row r's packed summary
    __shared__ unsigned long long smask[NCH];
    __shared__ int tail_end;                // one past the last row past the tile sorted here
    if (key_width(counters) != KB) return;
    const KeyPlanes keys = planes.width(KB);
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * TT;
    const int t = threadIdx.x, lane = lane_id(), wv = t >> 6;
    const int64_t wend = (b0 + WSLOTS < n) ? b0 + WSLOTS : n;
    const int nw = static_cast<int>(wend - b0);  // slots holding positions
    if (t == 0) tail_end = TT;
    // keys of the window and the row indices of its positions, loaded together
    for (int e0 = t; e0 <= WSLOTS; e0 += TT * 4) {
        Key96 v[4];
        uint32_t x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t pos = b0 - 1 + e0 + u * TT;
            const bool in = e0 + u * TT <= WSLOTS && pos >= 0 && pos < wend;
            v[u] = in ? keys[pos] : Key96{0, 0};
            x[u] = (in && pos >= b0) ? vals[pos] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * TT;
            if (e <= WSLOTS) {
                skeys[e] = v[u].a;
                skx[e] = v[u].b;
            }
            if (e >= 1 && e <= WSLOTS) sval[e - 1] = x[u];
        }
    }
    __syncthreads();
    // a slot starts a segment if its key differs from the previous position's
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int e = t + k * TT;
        const bool st = e < nw && (b0 + e == 0 || skeys[e + 1] != skeys[e] || skx[e + 1] != skx[e]);
        const unsigned long long m = ballot64(st);
        if (lane == 0) smask[wv + k * (TT / 64)] = m;
    }
    __syncthreads();
    // each slot's segment: its head (the last start at or before it) and its
    // end (the next start, the end of the input, or open past the window);
    // summaries start as "equal to the head"
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int e = t + k * TT;
        int16_t so = -1, sl = 0;
        bool large = false;
        uint2 seg = make_uint2(0u, 0u);
        if (e < nw) {
            int st = -1, en = -1;
            int c = e >> 6;
            const unsigned long long upto = (2ull << (e & 63)) - 1ull;  // bits 0 .. e & 63
            unsigned long long m = smask[c] & upto;
            for (;;) {
                if (m) { st = (c << 6) + 63 - __clzll(m); break; }
                if (--c < 0) break;
                m = smask[c];
            }
            c = e >> 6;
            m = smask[c] & ~upto;
            for (;;) {
                if (m) { en = (c << 6) + __ffsll(m) - 1; break; }
                if (++c >= NCH) break;
                m = smask[c];
            }
            if (en < 0 && wend == n) en = nw;
            if (st >= 0 && st < TT) {
                // open (en < 0) only when the window is full, so longer than WSMAX
                const int len = en < 0 ? WSMAX + 1 : en - st;
                if (len == 1) {
                    uniq[b0 + e] = 1;
                } else if (len <= WSMAX) {
                    so = static_cast<int16_t>(st);
                    sl = static_cast<int16_t>(len);
                } else if (e == st) {
                    const int64_t p = b0 + st;
                    const int64_t end = en < 0 ? run_end(keys, p, n) : b0 + en;
                    large = true;
                    seg = make_uint2(static_cast<uint32_t>(p), static_cast<uint32_t>(end - p));
                }
            }
        }
        if (e < WSLOTS) {
            segof[e] = so;
            seglen[e] = sl;
            sfull[e] = 0;
            if (so >= 0) {
#pragma unroll
                for (int c = 0; c < LV; ++c) {
                    scode[LV * e + c] = static_cast<uint8_t>(c == LV - 1 ? (WT | 0x80) : WT);
                    sv[LV * e + c] = T(0);
                }
            }
        }
        if (k == 0) {
            // heads lie in the tile: slot e = t, one wave per 64 slots
            wave_append<uint2>(large_list, &counters[1], n, large, seg);
        } else {
            const unsigned long long tb = ballot64(so >= 0);
            if (tb && lane == 0) atomicMax(&tail_end, (t - lane) + TT + 64 - __clzll(tb));
        }
    }
    __syncthreads();

    // Rows stream in with WT lanes per row: lane w of a row holds word w.
    const int w = t % WT;
    const int rsub = t / WT;
    const int gshift = lane & ~(WT - 1);
    const uint32_t below_w = (1u << w) - 1u;  // the row's words before w
    const bool wload = w < words, wcmp = w >= FROM;
    auto summarize = [&](int r, int a, T x, T y) {
        const bool ne = a >= 0 && wcmp && x != y;
        const uint32_t gm = static_cast<uint32_t>(ballot64(ne) >> gshift) & GMASK;
        const int c = __popc(gm & below_w);  // differing words before this one
        if (ne && c < LV) {
            const int code = (x < y) ? w : 2 * WT - w;
            scode[LV * r + c] = static_cast<uint8_t>(code | ((c == LV - 1 && __popc(gm) <= LV) ? 0x80 : 0));
            sv[LV * r + c] = x;
        }
    };
    {
        constexpr int UT = WT;                  // the tile's TT rows: WT elements per thread
        constexpr int U = UT < HB ? UT : HB;    // rows in flight per thread (and as many head words)
        static_assert(UT % U == 0, "tile batches");
        for (int ub = 0; ub < UT; ub += U) {
            T x[U], y[U];
            int as[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int r = (ub + u) * RPS + rsub;
                const int a = segof[r];
                as[u] = a;
                const bool ld = a >= 0 && wload;
                x[u] = ld ? rows[static_cast<int64_t>(sval[r]) * words + w] : T(0);
                y[u] = ld ? rows[static_cast<int64_t>(sval[a]) * words + w] : T(0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) summarize((ub + u) * RPS + rsub, as[u], x[u], y[u]);
        }
        // rows past the tile that belong to segments starting in it
        const int te = tail_end;
        for (int r0 = TT; r0 < te; r0 += RPS) {
            const int r = r0 + rsub;
            const int a = r < te ? segof[r] : -1;
            const bool ld = a >= 0 && wload;
            const T x = ld ? rows[static_cast<int64_t>(sval[r]) * words + w] : T(0);
            const T y = ld ? rows[static_cast<int64_t>(sval[a]) * words + w] : T(0);
            summarize(r, a, x, y);
        }
    }
    __syncthreads();
    // Each row's summary as one 192-bit string, most significant first: per
    // level the 7-bit code then the word (so strings order as the summaries
    // do); under them the row's slot (bits 1 .. 9 of the last word), which
    // makes a segment's strings distinct and orders equal summaries by
    // position; the flag in the last bit.  Written over the pool once every
    // row's levels are read.
    static_assert(LV * (7 + Bits<T>::B) <= 182 && WSLOTS <= 512, "summary, slot and flag fit 192 bits");
    constexpr uint64_t SLOTM = 0x3FEull;
    uint64_t kp[2][3];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int r = t + h * TT;
        kp[h][0] = kp[h][1] = kp[h][2] = 0;
        if (r < WSLOTS && segof[r] >= 0) {
#pragma unroll
            for (int c = 0; c < LV; ++c) {
                constexpr int B = Bits<T>::B;
                put_bits(kp[h], c * (7 + B), scode[LV * r + c] & 0x7f, 7);
                put_bits(kp[h], c * (7 + B) + 7, static_cast<uint64_t>(sv[LV * r + c]), B);
            }
            kp[h][2] |= (static_cast<uint64_t>(r) << 1) | ((scode[LV * r + LV - 1] & 0x80) ? 1ull : 0ull);
        }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int r = t + h * TT;
        if (r < WSLOTS && segof[r] >= 0) {
            pk[3 * r] = kp[h][0];
            pk[3 * r + 1] = kp[h][1];
            pk[3 * r + 2] = kp[h][2];
        }
    }
    __syncthreads();
    // A row's rank: how many strings of its segment lie below its own (j's
    // string is below r's iff the 192-bit subtraction borrows; the slots
    // differ, so the flag never decides).  The sorted order goes to sord.
    int rk[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int r = t + h * TT;
        const int a = r < WSLOTS ? segof[r] : -1;
        rk[h] = 0;
        if (a < 0) continue;
        const int len = seglen[r];
        const uint64_t m0 = kp[h][0], m1 = kp[h][1], m2 = kp[h][2];
        int rank = 0;
#pragma unroll 2
        for (int j = a; j < a + len; ++j) {
            unsigned long long bw;
            (void)__builtin_subcll(pk[3 * j + 2], m2, 0ull, &bw);
            (void)__builtin_subcll(pk[3 * j + 1], m1, bw, &bw);
            (void)__builtin_subcll(pk[3 * j], m0, bw, &bw);
            rank += static_cast<int>(bw);
        }
        rk[h] = rank;
        sord[a + rank] = static_cast<int16_t>(r);
    }
    __syncthreads();
    // Equal summaries are neighbours in that order, sorted by slot.  A row
    // whose predecessor there has its summary: with both flags set the rows
    // are equal and it is a duplicate; otherwise they may differ past the
    // summary, and the segment is marked for a second look.
    bool dupf[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int r = t + h * TT;
        const int a = r < WSLOTS ? segof[r] : -1;
        dupf[h] = false;
        if (a < 0 || rk[h] == 0) continue;
        const int j = sord[a + rk[h] - 1];
        const uint64_t j2 = pk[3 * j + 2];
        if (pk[3 * j] == kp[h][0] && pk[3 * j + 1] == kp[h][1] && ((j2 ^ kp[h][2]) & ~(SLOTM | 1ull)) == 0) {
            if (j2 & kp[h][2] & 1ull) dupf[h] = true;
            else sfull[a] = 1;
        }
    }
    __syncthreads();
    // In a marked segment each row is ranked again.  32-bit words: the row
    // walks the run of summaries equal to its own on both sides, and for a
    // pair without both flags the rank counted by slot is replaced by a
    // comparison of the rows in full.  64-bit words (equal summaries without
    // flags are rarer there): the whole segment is compared again with the
    // slots left out, such pairs compared in full.
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int r = t + h * TT;
        const int a = r < WSLOTS ? segof[r] : -1;
        if (a < 0) continue;
        int rank = rk[h];
        bool dup = dupf[h];
        if (sfull[a]) {
            const int len = seglen[r];
            auto full_cmp = [&](int j) {
                return row_cmp4<T>(rows + static_cast<int64_t>(sval[j]) * words,
                                   rows + static_cast<int64_t>(sval[r]) * words, words, FROM);
            };
            dup = false;
            if constexpr (sizeof(T) == 4) {
                const int q = a + rank;
                const uint64_t m0 = kp[h][0], m1 = kp[h][1], m2 = kp[h][2];
                auto same_summary = [&](int j) {
                    return pk[3 * j] == m0 && pk[3 * j + 1] == m1 && ((pk[3 * j + 2] ^ m2) & ~(SLOTM | 1ull)) == 0;
                };
                for (int p = q - 1; p >= a; --p) {  // slots below r
                    const int j = sord[p];
                    if (!same_summary(j)) break;
                    if (pk[3 * j + 2] & m2 & 1ull) {
                        dup = true;
                    } else {
                        const int c = full_cmp(j);
                        rank -= c > 0 ? 1 : 0;
                        dup = dup || c == 0;
                    }
                }
                for (int p = q + 1; p < a + len; ++p) {  // slots above r
                    const int j = sord[p];
                    if (!same_summary(j)) break;
                    if (!(pk[3 * j + 2] & m2 & 1ull)) rank += full_cmp(j) < 0 ? 1 : 0;
                }
            } else {
                const uint64_t m0 = kp[h][0], m1 = kp[h][1], m2 = kp[h][2] | SLOTM | 1ull;
                const uint64_t fm = kp[h][2] & 1ull;
                bool anytie = false;
                rank = 0;
                for (int j = a; j < a + len; ++j) {
                    const uint64_t j0 = pk[3 * j], j1 = pk[3 * j + 1], j2r = pk[3 * j + 2];
                    const uint64_t j2 = j2r | SLOTM | 1ull;
                    unsigned long long bw;
                    (void)__builtin_subcll(j2, m2, 0ull, &bw);
                    (void)__builtin_subcll(j1, m1, bw, &bw);
                    (void)__builtin_subcll(j0, m0, bw, &bw);
                    const bool eq = ((j0 ^ m0) | (j1 ^ m1) | (j2 ^ m2)) == 0;
                    const bool same = eq & ((j2r & fm) != 0);
                    const bool sb = same & (j < r);
                    rank += static_cast<int>(bw) + (sb ? 1 : 0);
                    dup = dup | sb;
                    anytie = anytie | (eq & !same & (j != r));
                }
                if (anytie) {
                    for (int j = a; j < a + len; ++j) {
                        const uint64_t j2r = pk[3 * j + 2];
                        const bool eq = pk[3 * j] == m0 && pk[3 * j + 1] == m1 && (j2r | SLOTM | 1ull) == m2;
                        if (!eq || j == r || (j2r & fm)) continue;
                        const int c = full_cmp(j);
                        rank += (c < 0 || (c == 0 && j < r)) ? 1 : 0;
                        dup = dup || (c == 0 && j < r);
                    }
                }
            }
        }
        vals[b0 + a + rank] = sval[r];
        uniq[b0 + a + rank] = dup ? 0 : 1;
    }
}

template <typename T, int WT>
cg_status tiefix_w_launch(const T *rows, KeyPlanes planes, int64_t n, int words, uint32_t *vals, uint8_t *uniq,
                          uint2 *large_list, unsigned long long *counters, bool may32, bool may64, bool may96,
                          hipStream_t s) {
    // one launch per width that may be the chosen one; the others return at once
    if (may64) {
        hipLaunchKernelGGL((k_tiefix_w<T, WT, 64>), dim3(blocks_for(n, TT)), dim3(TT), 0, s, rows, planes, n, words,
                           vals, uniq, large_list, counters);
        CG_LAUNCHED("dedup_tiefix_w");
    }
    if (may32) {
        hipLaunchKernelGGL((k_tiefix_w<T, WT, 32>), dim3(blocks_for(n, TT)), dim3(TT), 0, s, rows, planes, n, words,
                           vals, uniq, large_list, counters);
        CG_LAUNCHED("dedup_tiefix_w32");
    }
    if (may96) {
        hipLaunchKernelGGL((k_tiefix_w<T, WT, 96>), dim3(blocks_for(n, TT)), dim3(TT), 0, s, rows, planes, n, words,
                           vals, uniq, large_list, counters);
        CG_LAUNCHED("dedup_tiefix_w96");
    }
    return CG_OK;
}

template <typename T>
__device__ __forceinline__ bool idx_less(const T *rows, int words, int from, uint32_t x, uint32_t y) {
    if (x == SENT) return false;
    if (y == SENT) return true;
    const int c = row_cmp4<T>(rows + static_cast<int64_t>(x) * words, rows + static_cast<int64_t>(y) * words,
                             words, from);
    return c < 0 || (c == 0 && x < y);
}

// One block per long segment: bitonic network over its index array, kept in
// global scratch at [2a, 2a + P), P = next power of two >= len.
// A segment longer than LMAX rows, by the whole block: bitonic network on
// its index array in global scratch at [2a, 2a + P), P = next power of two
// >= len (slow, met only by heavy-duplicate inputs).
template <typename T>
__device__ void sort_large_segment(const T *__restrict__ rows, int words, int from, int64_t a, int64_t len,
                                   uint32_t *vals, uint8_t *uniq, uint32_t *scratch) {
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
                    const bool swap = asc ? idx_less<T>(rows, words, from, y, x) : idx_less<T>(rows, words, from, x, y);
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
            u = row_cmp4<T>(rows + static_cast<int64_t>(x) * words, rows + static_cast<int64_t>(y) * words, words,
                           from) != 0;
        }
        uniq[a + i] = u ? 1 : 0;
    }
    __syncthreads();
}

// Segments longer than the tile kernel takes, up to LMAX rows: one block per
// segment sorts (next 64 bits of the row, row index) pairs by a bitonic
// network in LDS; pairs whose 64-bit values tie compare the rest of the rows
// in global memory.  Then a row is flagged new iff it differs from its
// predecessor in the segment.  Short segments get small blocks (a bitonic
// stage over P pairs keeps only P / 2 threads busy), so several share a CU.
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

// NT threads and room for LM rows per block; segments of LO < len <= LM
// rows are this launch's (two launches: 256 threads for up to 2,048 rows,
// several blocks per CU; 1,024 threads for the rest up to LMAX).
template <typename T, int NT, int LM, int LO>
__global__ void __launch_bounds__(NT) k_tiefix_mid(const T *__restrict__ rows, int words, int from64,
                                                     const uint2 *__restrict__ list,
                                                     const unsigned long long *__restrict__ counters,
                                                     uint32_t *__restrict__ vals, uint8_t *__restrict__ uniq,
                                                     uint32_t *__restrict__ scratch) {
    (void)from64;
    const int from = key_width(counters) / Bits<T>::B;  // whole words covered by the sort key
    extern __shared__ __align__(16) unsigned char smem[];  // LM keys, then LM indices
    uint64_t *sk = reinterpret_cast<uint64_t *>(smem);
    uint32_t *si = reinterpret_cast<uint32_t *>(smem + LM * sizeof(uint64_t));
    constexpr int K2 = 64 / Bits<T>::B;  // words covered by the second key
    const int from2 = from + K2;
    const uint32_t count = static_cast<uint32_t>(counters[1]);
    for (uint32_t sgi = blockIdx.x; sgi < count; sgi += gridDim.x) {
        const uint2 seg = list[sgi];
        const int64_t a = seg.x;
        const int64_t len64 = seg.y;
        if (len64 > LM) {  // the launch of the longest LDS segments also takes the longer ones
            if (LM == LMAX) sort_large_segment<T>(rows, words, from, a, len64, vals, uniq, scratch);
            continue;
        }
        const int len = static_cast<int>(len64);
        if (len <= LO) continue;  // another launch takes it
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
                            const int c = row_cmp4<T>(rows + static_cast<int64_t>(ia) * words,
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
                u = row_cmp4<T>(rows + static_cast<int64_t>(x) * words, rows + static_cast<int64_t>(si[i - 1]) * words,
                               words, from2) != 0;
            uniq[a + i] = u ? 1 : 0;
        }
        __syncthreads();
    }
}

// Suffix-hash terms of one gathered piece (PW words of type T).
template <typename T, typename V>
__device__ __forceinline__ uint64_t piece_terms(const V &v, int piece, int s) {
    constexpr int PW = static_cast<int>(sizeof(V) / sizeof(T));
    const T *x = reinterpret_cast<const T *>(&v);
    uint64_t sum = 0;
#pragma unroll
    for (int k = 0; k < PW; ++k) sum += suffix_term<T>(x[k], piece * PW + k, s);
    return sum;
}

// sfx (when not null): each cell's suffix-order key (hash << 32 | id).  With
// hash_lanes > 0 (a row's pieces a power of two, at most 64, so a row's
// lanes are adjacent within one wave) the lanes of a row add their pieces'
// hash terms (DPP permutes within the row's lane group); otherwise the hash
// comes from rhash[row].  All lanes of a wave stay in the loop together so
// the permutes see every lane.
//
// PL >= 0: pieces == 1 << PL, so a piece's row and position are a shift and
// a mask (the general form divides a 64-bit index, dozens of instructions).
template <typename T, typename V, int PL>
__global__ void __launch_bounds__(256) k_gather(const V *__restrict__ rows, int64_t n, int pieces,
                                                const uint32_t *__restrict__ vals, const uint8_t *__restrict__ uniq,
                                                const uint32_t *__restrict__ cidx, V *__restrict__ cells,
                                                uint32_t *__restrict__ row_to_cell, const uint32_t *__restrict__ rhash,
                                                uint64_t *__restrict__ sfx, int hash_lanes, int hash_s) {
    // GU pieces per thread per step, each step's pieces a whole number of
    // waves apart, so their loads are in flight together and a row's lanes
    // stay adjacent for the hash sums; the grid is sized so that one step
    // covers every piece
    constexpr int GU = 4;
    const int64_t total = n * pieces;
    const int64_t span = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t g0 = static_cast<int64_t>(blockIdx.x) * blockDim.x; g0 < total; g0 += span * GU) {
        V v[GU];
        uint32_t uu[GU], cid[GU], src[GU];
        int wp[GU];
#pragma unroll
        for (int q = 0; q < GU; ++q) {
            const int64_t g = g0 + q * span + threadIdx.x;
            const bool in = g < total;
            int64_t j;
            if constexpr (PL >= 0) {
                j = in ? (g >> PL) : 0;
                wp[q] = static_cast<int>(g & ((int64_t(1) << PL) - 1));
            } else {
                j = in ? g / pieces : 0;
                wp[q] = static_cast<int>(g - j * pieces);
            }
            uu[q] = in ? uniq[j] : 0u;
            cid[q] = in ? cidx[j] + uu[q] - 1 : 0u;
            src[q] = in ? vals[j] : 0u;
            const int64_t so = PL >= 0 ? (static_cast<int64_t>(src[q]) << (PL >= 0 ? PL : 0))
                                       : static_cast<int64_t>(src[q]) * pieces;
            v[q] = uu[q] ? rows[so + wp[q]] : V{};
        }
#pragma unroll
        for (int q = 0; q < GU; ++q) {
            const int64_t g = g0 + q * span + threadIdx.x;
            const int64_t co = PL >= 0 ? (static_cast<int64_t>(cid[q]) << (PL >= 0 ? PL : 0))
                                       : static_cast<int64_t>(cid[q]) * pieces;
            if (uu[q]) cells[co + wp[q]] = v[q];
            if (g < total && wp[q] == 0 && row_to_cell) row_to_cell[src[q]] = cid[q];
            if (sfx) {
                if (hash_lanes > 0) {
                    uint64_t t = uu[q] ? piece_terms<T, V>(v[q], wp[q], hash_s) : 0ull;
                    if constexpr (PL >= 0) {
                        t = group_sum_u64<(1 << (PL >= 0 ? PL : 0))>(t);  // hash_lanes == 1 << PL
                    } else {
                        for (int d = 1; d < hash_lanes; d <<= 1) t += shfl_u64_xor(t, d);
                    }
                    if (uu[q] && wp[q] == 0) sfx[cid[q]] = (static_cast<uint64_t>(suffix_finish(t)) << 32) | cid[q];
                } else if (uu[q] && wp[q] == 0) {
                    sfx[cid[q]] = (static_cast<uint64_t>(rhash[src[q]]) << 32) | cid[q];
                }
            }
        }
    }
}

struct DedupWs {
    uint32_t *khi[2];
    uint32_t *klo[2];
    uint32_t *kx[2];  // third key plane (96-bit keys, rows longer than 64 bits)
    uint32_t *vals[2];
    uint32_t *hist;
    uint64_t *tile_sums;
    uint8_t *uniq;
    uint32_t *cidx;
    uint2 *large_list;
    unsigned long long *counters;
    uint32_t *scratch;
    uint32_t *rhash;
};

DedupWs carve_dedup(void *base, int64_t n, cg_layout lay, size_t *bytes, bool with_hash = false) {
    Carver c(base);
    DedupWs w{};
    const int64_t m = n > 0 ? n : 1;
    w.khi[0] = c.take<uint32_t>(m);
    w.khi[1] = c.take<uint32_t>(m);
    w.klo[0] = c.take<uint32_t>(m);
    w.klo[1] = c.take<uint32_t>(m);
    if (lay.ell > 64) {
        w.kx[0] = c.take<uint32_t>(m);
        w.kx[1] = c.take<uint32_t>(m);
    }
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
    if (with_hash) w.rhash = c.take<uint32_t>(m);
    *bytes = c.bytes();
    return w;
}

// With hash_s >= 0 (the fused dedup + dictionary build) the suffix hash of
// every row is taken during key extraction and the gather writes each
// cell's suffix-order key to sfx; *view then names the sorted keys, the
// new-cell flags and the cell numbering for the directory.
template <typename T>
cg_status dedup_impl(const T *rows, int64_t n, cg_layout lay, T *cells, uint32_t *row_to_cell, int64_t *d_ncells,
                     void *ws, hipStream_t s, int hash_s = -1, uint64_t *sfx = nullptr, DedupView *view = nullptr,
                     int key_bits = 0, unsigned long long *extra_zero = nullptr, int n_extra = 0) {
    size_t bytes;
    DedupWs w = carve_dedup(ws, n, lay, &bytes, hash_s >= 0);
    // the gather hashes a row from its pieces when they are a power of two
    // (at most 64, so a row's lanes sit together in one wave); otherwise the
    // hashes are taken per row at key extraction
    const size_t rowbytes = static_cast<size_t>(lay.words) * sizeof(T);
    const int pieces = rowbytes % 16 == 0 ? static_cast<int>(rowbytes / 16) : lay.words;
    const int hash_lanes = (hash_s >= 0 && pieces <= 64 && (pieces & (pieces - 1)) == 0) ? pieces : 0;
    uint32_t *rhash = (hash_s >= 0 && hash_lanes == 0) ? w.rhash : nullptr;
    const int words = lay.words;
    if (n == 0) return fill_i64(d_ncells, 0, 1, s);

    const bool tiefix = lay.ell > 64;
    // key width for l > 64: the caller's 32, 64 or 96, or (0) a sample
    // decides between 32 and 64 on the device for long inputs, else 64
    const bool k32 = tiefix && key_bits == 32;
    const bool k96 = tiefix && key_bits == 96;
    const bool probe = tiefix && key_bits == 0 && n >= PROBE_MIN_N;
    DedupInit init{w.counters, k32 ? 1ull : 0ull, k96 ? 1ull : 0ull, extra_zero, n_extra};
    if (probe) {  // the counters are set before the sample; else by the extraction's block 0
        hipLaunchKernelGGL(k_dedup_init, dim3(1), dim3(64), 0, s, init);
        CG_LAUNCHED("dedup_init");
        init.counters = nullptr;
        hipLaunchKernelGGL((k_key_probe<T>), dim3(1), dim3(1024), 0, s, rows, n, words, w.counters);
        CG_LAUNCHED("dedup_key_probe");
    }
    // the sort key: the row's first sig bits in 32-bit planes, sorted by
    // its bits that can be nonzero; with 32-bit keys chosen on the device
    // the second plane's passes are skipped
    const int sig = tiefix ? (k32 ? 32 : (k96 ? 96 : 64)) : lay.ell;
    const int nplanes = (sig + 31) / 32;
    const int bit_lo = ((32 * nplanes - sig) / 8) * 8;
    uint32_t *pl[3][2] = {{w.khi[0], w.khi[1]},
                          {nplanes > 1 ? w.klo[0] : nullptr, nplanes > 1 ? w.klo[1] : nullptr},
                          {nplanes > 2 ? w.kx[0] : nullptr, nplanes > 2 ? w.kx[1] : nullptr}};
    const unsigned long long *key32 = probe ? w.counters + 2 : nullptr;
    const size_t xlds = static_cast<size_t>(256) * (words | 1) * sizeof(T);
    if (rhash && xlds <= 65536) {
        hipLaunchKernelGGL((k_extract_hash<T>), dim3(blocks_for(n, 256)), dim3(256), xlds, s, rows, n, words, key32,
                           pl[0][0], pl[1][0], pl[2][0], w.vals[0], hash_s, rhash, init);
    } else {
        hipLaunchKernelGGL((k_extract<T>), dim3(blocks_for(n, 256, 16384)), dim3(256), 0, s, rows, n, words, key32,
                           pl[0][0], pl[1][0], pl[2][0], w.vals[0], init);
        if (rhash) {  // rows too wide to stage: hash them in place
            hipLaunchKernelGGL((k_hash_rows<T>), dim3(blocks_for(n, 256, 16384)), dim3(256), 0, s, rows, n, words,
                               hash_s, rhash);
            CG_LAUNCHED("dedup_hash_rows");
        }
    }
    CG_LAUNCHED("dedup_extract");

    int which = 0;
    CG_TRY(radix_sort_k32(pl, nplanes, w.vals, n, nullptr, bit_lo, w.hist, &which, s, nplanes > 1, key32));
    const KeyPlanes planes{pl[0][which], pl[1][which], pl[2][which]};
    uint32_t *khi = pl[0][which];
    uint32_t *vals = w.vals[which];

    const int B = static_cast<int>(sizeof(T) * 8);
    const int from = 64 / B;  // unused by the tie-fixes, which take the key width from the device counters
    if (!tiefix) {
        hipLaunchKernelGGL(k_heads, dim3(blocks_for(n, 256)), dim3(256), 0, s, planes, n, w.uniq);
        CG_LAUNCHED("dedup_heads");
    } else {
        const int LW = words + ((words % 2 == 0) ? 1 : 0);
        // per slot: its row, key (8 + 4 bytes), segment, length, row index
        const int64_t per_slot = static_cast<int64_t>(LW) * sizeof(T) + 24;
        int64_t smax = TILE_LDS / per_slot - TT - 1;
        if (smax > 512) smax = 512;
        size_t lds = static_cast<size_t>(TT + smax) * per_slot + 16;
        if (smax < 2) {  // rows too wide for LDS: every multi-row segment takes the large path
            smax = 1;
            lds = static_cast<size_t>(TT + 1) * 24 + 16;
        }
        int wt = 1;
        while (wt < words) wt <<= 1;
        if (wt <= 32) {  // head rows of up to 32 words fit the summary kernel's LDS
            switch (wt) {
            case 2: CG_TRY((tiefix_w_launch<T, 2>(rows, planes, n, words, vals, w.uniq, w.large_list, w.counters, probe || k32, !k32 && !k96, k96, s))); break;
            case 4: CG_TRY((tiefix_w_launch<T, 4>(rows, planes, n, words, vals, w.uniq, w.large_list, w.counters, probe || k32, !k32 && !k96, k96, s))); break;
            case 8: CG_TRY((tiefix_w_launch<T, 8>(rows, planes, n, words, vals, w.uniq, w.large_list, w.counters, probe || k32, !k32 && !k96, k96, s))); break;
            case 16: CG_TRY((tiefix_w_launch<T, 16>(rows, planes, n, words, vals, w.uniq, w.large_list, w.counters, probe || k32, !k32 && !k96, k96, s))); break;
            default: CG_TRY((tiefix_w_launch<T, 32>(rows, planes, n, words, vals, w.uniq, w.large_list, w.counters, probe || k32, !k32 && !k96, k96, s))); break;
            }
        } else {
            hipLaunchKernelGGL((k_tiefix_tile<T>), dim3(blocks_for(n, TT)), dim3(TT), lds, s, rows, planes, n, words,
                               static_cast<int>(smax), vals, w.uniq, w.large_list, w.counters);
            CG_LAUNCHED("dedup_tiefix_tile");
        }
        constexpr int MID_S = 2048;  // segments up to this many rows: 256-thread blocks, 24 KB of LDS each
        const size_t mid_lds_s = static_cast<size_t>(MID_S) * (sizeof(uint64_t) + sizeof(uint32_t));
        hipLaunchKernelGGL((k_tiefix_mid<T, 256, MID_S, 0>), dim3(2048), dim3(256), mid_lds_s, s, rows, words, from,
                           w.large_list, w.counters, vals, w.uniq, w.scratch);
        CG_LAUNCHED("dedup_tiefix_mid_s");
        const size_t mid_lds = static_cast<size_t>(LMAX) * (sizeof(uint64_t) + sizeof(uint32_t));
        CG_TRY(allow_lds(reinterpret_cast<const void *>(&k_tiefix_mid<T, 1024, LMAX, MID_S>), mid_lds));
        hipLaunchKernelGGL((k_tiefix_mid<T, 1024, LMAX, MID_S>), dim3(1024), dim3(1024), mid_lds, s, rows, words, from,
                           w.large_list, w.counters, vals, w.uniq, w.scratch);
        CG_LAUNCHED("dedup_tiefix_mid");
    }
    CG_TRY(scan_u8_to_u32(w.uniq, w.cidx, n, nullptr, w.tile_sums, d_ncells, s));
    if (rowbytes % 16 == 0) {
        // GU pieces per thread, all in flight: the grid covers every piece in one step
        const dim3 g(blocks_for(n * pieces, 256 * 4, 65536));
        const uint4 *r4 = reinterpret_cast<const uint4 *>(rows);
        uint4 *c4 = reinterpret_cast<uint4 *>(cells);
#define CG_GATHER4(PLV)                                                                                            \
    hipLaunchKernelGGL((k_gather<T, uint4, PLV>), g, dim3(256), 0, s, r4, n, pieces, vals, w.uniq, w.cidx, c4,     \
                       row_to_cell, rhash, sfx, hash_lanes, hash_s)
        switch (pieces) {
        case 1: CG_GATHER4(0); break;
        case 2: CG_GATHER4(1); break;
        case 4: CG_GATHER4(2); break;
        case 8: CG_GATHER4(3); break;
        case 16: CG_GATHER4(4); break;
        case 32: CG_GATHER4(5); break;
        case 64: CG_GATHER4(6); break;
        default: CG_GATHER4(-1); break;
        }
#undef CG_GATHER4
    } else {
        const dim3 g(blocks_for(n * words, 256 * 4, 65536));
#define CG_GATHER1(PLV)                                                                                            \
    hipLaunchKernelGGL((k_gather<T, T, PLV>), g, dim3(256), 0, s, rows, n, words, vals, w.uniq, w.cidx, cells,     \
                       row_to_cell, rhash, sfx, hash_lanes, hash_s)
        switch (words) {
        case 1: CG_GATHER1(0); break;
        case 2: CG_GATHER1(1); break;
        default: CG_GATHER1(-1); break;
        }
#undef CG_GATHER1
    }
    CG_LAUNCHED("dedup_gather");
    if (view) {
        view->khi = khi;
        view->uniq = w.uniq;
        view->cidx = w.cidx;
    }
    return CG_OK;
}

}  // namespace

size_t dedup_workspace_bytes(int64_t n, cg_layout lay) {
    size_t b;
    carve_dedup(nullptr, n, lay, &b);
    return b;
}

size_t dedup_fused_workspace_bytes(int64_t n, cg_layout lay) {
    size_t b;
    carve_dedup(nullptr, n, lay, &b, true);
    return b;
}

cg_status run_dedup_fused(const void *rows, int64_t n, cg_layout lay, void *cells, uint32_t *row_to_cell,
                          int64_t *d_ncells, void *ws, int hash_s, uint64_t *sfx, DedupView *view, int key_bits,
                          unsigned long long *extra_zero, int n_extra, hipStream_t s) {
    if (lay.word_bits == 64)
        return dedup_impl<uint64_t>(static_cast<const uint64_t *>(rows), n, lay, static_cast<uint64_t *>(cells),
                                    row_to_cell, d_ncells, ws, s, hash_s, sfx, view, key_bits, extra_zero, n_extra);
    return dedup_impl<uint32_t>(static_cast<const uint32_t *>(rows), n, lay, static_cast<uint32_t *>(cells),
                                row_to_cell, d_ncells, ws, s, hash_s, sfx, view, key_bits, extra_zero, n_extra);
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
