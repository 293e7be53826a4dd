// Dictionary over the sorted distinct cells, and distance-1 queries against it.
//
// Section 3.2 builds a 2^r-ary search tree over the sorted vectors whose
// nodes stand for the index ranges vectors(C, v) and whose leaves hold the
// values.  Here the top of that tree is one flat level: a directory over the
// first p bits (dir[g] = first cell whose top p bits are >= g), i.e. the
// ranges of all 2^p nodes at depth p of a binary tree; below it a range is
// finished by binary search over the sorted keys.  The suffix-grouped order
// (cell ids sorted by a 32-bit hash of bits s .. l-1) is built here too;
// cg_edges uses it for flips below bit s.
//
// Queries (Algorithm 4): for query q and bit k, the target q xor e_k never
// exists as a row; each comparison XORs the flipped bit in on the fly
// (Section 3.2 notes x' need not be materialised).
#include "cg_internal.hpp"

#include <algorithm>

namespace cg {

namespace {

// One block per 256-cell tile.  The tile's rows are read once, coalesced,
// into LDS (when they fit; wide rows are read in place), then each thread
// hashes its cell's suffix and writes the directory entries that point at it:
// those of the empty groups between its predecessor's top p bits and its
// own.  Short gaps are filled in place; a gap longer than GAPMIN entries
// (clustered keys, e.g. batched scenes whose top bits are a scene tag) is
// listed, and k_dir_gaps fills it with a whole block.  Gaps are disjoint, so
// at most (2^p + 1) / (GAPMIN + 1) + 1 are listed.
constexpr int DT = 256;
constexpr int GAPMIN = 64;
constexpr int64_t GAPHUGE = 65536;  // longer gaps are listed apart and filled by every block

__device__ __forceinline__ void push_gap(uint4 *gaps, unsigned long long *gap_n, int64_t cap, bool want,
                                         int64_t lo, int64_t hi, uint32_t v) {
    const uint64_t m = ballot64(want);
    if (m == 0) return;
    const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
    unsigned long long b = 0;
    if (lane_id() == leader) b = atomicAdd(gap_n, static_cast<unsigned long long>(__popcll(m)));
    b = shfl_u64(b, leader);
    if (want) {
        const unsigned long long k = b + static_cast<unsigned long long>(__popcll(m & lanemask_lt()));
        if (static_cast<int64_t>(k) < cap)
            gaps[k] = make_uint4(static_cast<uint32_t>(lo), static_cast<uint32_t>(hi), v, 0u);
    }
}

template <typename T>
__global__ void __launch_bounds__(DT) k_dict_scan(const T *__restrict__ cells, const int64_t *d_n, int64_t ncap,
                                                  int words, int p, int s, uint32_t *__restrict__ dir,
                                                  uint64_t *__restrict__ sfx, bool stage, uint4 *__restrict__ gaps,
                                                  unsigned long long *gap_n, int64_t gap_cap,
                                                  uint4 *__restrict__ huge, int64_t huge_cap) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t n = load_n(d_n, ncap);
    const int64_t G = int64_t(1) << p;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * DT;
    if (n == 0) {
        for (int64_t g = base + threadIdx.x; g <= G; g += static_cast<int64_t>(gridDim.x) * DT) dir[g] = 0;
        return;
    }
    if (base >= n) return;
    const int tr = static_cast<int>(n - base < DT ? n - base : DT);
    const int LW = words | 1;
    T *lrows = reinterpret_cast<T *>(smem);
    if (stage) {
        copy_rows_to_lds<T, DT>(lrows, LW, cells + base * words, tr, words);
        __syncthreads();
    }
    const int t = threadIdx.x;
    if (t >= tr) return;
    const int64_t i = base + t;
    // LDS and global rows take separate code so each access keeps its own
    // address space (a pointer that may point to either becomes a flat access)
    uint64_t hme, hprev = 0;
    uint32_t hsh;
    if (stage) {
        const T *row = lrows + t * LW;
        hme = head64<T>(row, words);
        hsh = suffix_hash32<T>(row, words, s);
    } else {
        const T *row = cells + i * words;
        hme = head64<T>(row, words);
        hsh = suffix_hash32<T>(row, words, s);
    }
    if (i > 0) hprev = (stage && t > 0) ? head64<T>(lrows + (t - 1) * LW, words) : head64<T>(cells + (i - 1) * words, words);
    const int64_t gi = p ? static_cast<int64_t>(hme >> (64 - p)) : 0;
    const int64_t gp = i == 0 ? -1 : (p ? static_cast<int64_t>(hprev >> (64 - p)) : 0);
    // entries gp + 1 .. gi point at cell i
    const bool long_gap = gi - gp > GAPMIN;
    if (long_gap) {
        dir[gi] = static_cast<uint32_t>(i);
    } else {
        for (int64_t g = gp + 1; g <= gi; ++g) dir[g] = static_cast<uint32_t>(i);
    }
    const bool huge_gap = gi - gp > GAPHUGE;
    push_gap(gaps, gap_n, gap_cap, long_gap && !huge_gap, gp + 1, gi - 1, static_cast<uint32_t>(i));
    push_gap(huge, gap_n + 1, huge_cap, huge_gap, gp + 1, gi - 1, static_cast<uint32_t>(i));
    if (i == n - 1) {  // entries gi + 1 .. G point past the end
        if (G - gi > GAPMIN) {
            const bool hg = G - gi > GAPHUGE;
            const unsigned long long k = atomicAdd(hg ? gap_n + 1 : gap_n, 1ull);
            if (static_cast<int64_t>(k) < (hg ? huge_cap : gap_cap))
                (hg ? huge : gaps)[k] = make_uint4(static_cast<uint32_t>(gi + 1), static_cast<uint32_t>(G),
                                                   static_cast<uint32_t>(n), 0u);
        } else {
            for (int64_t g = gi + 1; g <= G; ++g) dir[g] = static_cast<uint32_t>(n);
        }
    }
    sfx[i] = (static_cast<uint64_t>(hsh) << 32) | static_cast<uint64_t>(i);
}

// Fills the listed long gaps: gap (lo, hi, v) sets dir[lo .. hi] = v; one
// block per ordinary gap, and every block takes its share of each huge one.
__global__ void __launch_bounds__(256) k_dir_gaps(uint32_t *__restrict__ dir, const uint4 *__restrict__ gaps,
                                                  const unsigned long long *gap_n, int64_t gap_cap,
                                                  const uint4 *__restrict__ huge, int64_t huge_cap) {
    int64_t cnt = static_cast<int64_t>(gap_n[0]);
    if (cnt > gap_cap) cnt = gap_cap;
    for (int64_t k = blockIdx.x; k < cnt; k += gridDim.x) {
        const uint4 g = gaps[k];
        for (int64_t e = static_cast<int64_t>(g.x) + threadIdx.x; e <= static_cast<int64_t>(g.y); e += blockDim.x)
            dir[e] = g.z;
    }
    int64_t hc = static_cast<int64_t>(gap_n[1]);
    if (hc > huge_cap) hc = huge_cap;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t k = 0; k < hc; ++k) {
        const uint4 g = huge[k];
        for (int64_t e = static_cast<int64_t>(g.x) + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
             e <= static_cast<int64_t>(g.y); e += stride)
            dir[e] = g.z;
    }
}

// One wave per query; lanes take bits k0 + lane for k0 = 0, 64, ...
template <typename T>
__global__ void __launch_bounds__(256) k_d1_query(const T *__restrict__ cells, const int64_t *d_n, int64_t ncap,
                                                  int words, int ell, const uint32_t *__restrict__ dir, int p,
                                                  const T *__restrict__ queries, int64_t nq,
                                                  uint32_t *__restrict__ count, uint32_t *__restrict__ self,
                                                  T *__restrict__ mask) {
    constexpr int B = Bits<T>::B;
    const int lane = threadIdx.x & 63;
    const int64_t wid = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    const int64_t n = load_n(d_n, ncap);
    (void)n;
    for (int64_t qi = wid; qi < nq; qi += nw) {
        const T *q = queries + qi * words;
        const uint64_t qh = head64<T>(q, words);
        uint32_t total = 0;
        for (int k0 = 0; k0 < ell; k0 += 64) {
            const int k = k0 + lane;
            bool found = false;
            if (k < ell) {
                const uint64_t th = qh ^ (k < 64 ? (1ull << (63 - k)) : 0ull);
                const int64_t g = p ? static_cast<int64_t>(th >> (64 - p)) : 0;
                found = find_row<T>(cells, words, dir[g], dir[g + 1], q, k) >= 0;
            }
            const uint64_t m = ballot64(found);
            total += static_cast<uint32_t>(__popcll(m));
            if (mask) {
                T *mrow = mask + qi * words;
                if (B == 64) {
                    if (lane == 0) mrow[k0 / 64] = static_cast<T>(__brevll(m));
                } else {
                    const int w = k0 / 32;
                    if (lane == 0) mrow[w] = static_cast<T>(__brev(static_cast<uint32_t>(m)));
                    if (lane == 1 && w + 1 < words) mrow[w + 1] = static_cast<T>(__brev(static_cast<uint32_t>(m >> 32)));
                }
            }
        }
        if (lane == 0) {
            if (count) count[qi] = total;
            if (self) {
                const int64_t g = p ? static_cast<int64_t>(qh >> (64 - p)) : 0;
                const int64_t id = find_row<T>(cells, words, dir[g], dir[g + 1], q, -1);
                self[qi] = id >= 0 ? static_cast<uint32_t>(id) : 0xFFFFFFFFu;
            }
        }
    }
}

// Queries by the query's own directory bucket.  A flip at k >= p keeps the
// top p bits, so q xor e_k can only be a cell of q's own bucket, and it is
// one exactly when that cell is at distance 1 from q, differing at k.  So
// instead of one search per flip, the wave reads the bucket's cells once
// (one lane per cell) and sets mask bit k for each cell at distance 1 (the
// cell at distance 0 is q itself); only the p flips inside the directory
// bits are searched, each in its own bucket.  Buckets larger than DB_MAX
// cells fall back to per-flip searches for k >= p too.  MW: most words per
// row (the wave's mask is accumulated in LDS).
constexpr int DB_MAX = 256;
constexpr int D1_MW = 64;

template <typename T>
__global__ void __launch_bounds__(256) k_d1_bucket(const T *__restrict__ cells, int words, int ell,
                                                   const uint32_t *__restrict__ dir, int p,
                                                   const T *__restrict__ queries, int64_t nq,
                                                   uint32_t *__restrict__ count, uint32_t *__restrict__ self,
                                                   T *__restrict__ mask) {
    constexpr int B = Bits<T>::B;
    __shared__ T smask[4][D1_MW];
    __shared__ uint32_t sself[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wid = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    T *sm = smask[wv];
    for (int64_t qi = wid; qi < nq; qi += nw) {
        const T *q = queries + qi * words;
        const uint64_t qh = head64<T>(q, words);
        const int64_t g = p ? static_cast<int64_t>(qh >> (64 - p)) : 0;
        const uint32_t lo = dir[g], hi = dir[g + 1];
        for (int w = lane; w < words; w += 64) sm[w] = T(0);
        if (lane == 0) sself[wv] = 0xFFFFFFFFu;
        __builtin_amdgcn_wave_barrier();
        if (hi - lo <= static_cast<uint32_t>(DB_MAX)) {
            // the bucket's cells, one lane each: distance 1 at k sets bit k
            for (uint32_t c = lo + lane; c < hi; c += 64) {
                const T *x = cells + static_cast<int64_t>(c) * words;
                int d = 0, first = -1;
                for (int w = 0; w < words && d < 2; ++w) {
                    const T y = x[w] ^ q[w];
                    if (y) {
                        d += popc<T>(y);
                        if (first < 0) first = w * B + clz_t<T>(y);
                    }
                }
                if (d == 0) sself[wv] = c;
                if (d == 1) {
                    if (B == 64)
                        atomicOr(reinterpret_cast<unsigned long long *>(&sm[first / B]),
                                 static_cast<unsigned long long>(bitmask_of<T>(first)));
                    else
                        atomicOr(reinterpret_cast<unsigned int *>(&sm[first / B]),
                                 static_cast<unsigned int>(bitmask_of<T>(first)));
                }
            }
        } else {
            // a long bucket: search it once per flip at k >= p
            for (int k0 = p; k0 < ell; k0 += 64) {
                const int k = k0 + lane;
                const bool found = k < ell && find_row<T>(cells, words, lo, hi, q, k) >= 0;
                if (found) {
                    if (B == 64)
                        atomicOr(reinterpret_cast<unsigned long long *>(&sm[k / B]),
                                 static_cast<unsigned long long>(bitmask_of<T>(k)));
                    else
                        atomicOr(reinterpret_cast<unsigned int *>(&sm[k / B]), static_cast<unsigned int>(bitmask_of<T>(k)));
                }
            }
            if (lane == 0) {
                const int64_t id = find_row<T>(cells, words, lo, hi, q, -1);
                if (id >= 0) sself[wv] = static_cast<uint32_t>(id);
            }
        }
        // flips inside the directory bits: each in the bucket of its own top p bits
        if (lane < p && lane < ell) {
            const int k = lane;
            const uint64_t th = qh ^ (1ull << (63 - k));
            const int64_t g2 = static_cast<int64_t>(th >> (64 - p));
            if (find_row<T>(cells, words, dir[g2], dir[g2 + 1], q, k) >= 0) {
                if (B == 64)
                    atomicOr(reinterpret_cast<unsigned long long *>(&sm[k / B]),
                             static_cast<unsigned long long>(bitmask_of<T>(k)));
                else
                    atomicOr(reinterpret_cast<unsigned int *>(&sm[k / B]), static_cast<unsigned int>(bitmask_of<T>(k)));
            }
        }
        __builtin_amdgcn_wave_barrier();
        uint32_t c = 0;
        for (int w = lane; w < words; w += 64) {
            const T m = sm[w];
            c += static_cast<uint32_t>(popc<T>(m));
            if (mask) mask[qi * words + w] = m;
        }
        const uint32_t tot = lane63_u32(wave_incl_scan_u32(c));
        if (lane == 0) {
            if (count) count[qi] = tot;
            if (self) self[qi] = sself[wv];
        }
        __builtin_amdgcn_wave_barrier();  // the wave's LDS is cleared for its next query
    }
}

struct DictMem {
    uint32_t *dir;
    uint4 *gaps;
    unsigned long long *gap_n;  // [0]: gaps, [1]: huge gaps
    int64_t gap_cap;
    uint4 *huge;
    int64_t huge_cap;
    uint64_t *sfx[2];
    uint32_t *hist;
    uint64_t *tile_sums;
    uint16_t *tdep;   // tree kind: per cell, the deepest level shared with its predecessor
    uint32_t *tlev;   // tree kind: nodes per level (depth + 1)
    uint32_t *thist;  // tree kind: cells per shared depth (depth entries)
};

int tree_depth_of(int ell, int r) { return (ell + r - 1) / r; }

DictMem carve_dict(void *base, int64_t ncap, int ell, const cg_dict_params &p, size_t *bytes) {
    Carver c(base);
    DictMem m{};
    const int64_t n = ncap > 0 ? ncap : 1;
    m.dir = c.take<uint32_t>((size_t(1) << p.dir_bits) + 1);
    m.gap_cap = (int64_t(1) << p.dir_bits) / (GAPMIN + 1) + 2;
    m.gaps = c.take<uint4>(m.gap_cap);
    m.gap_n = c.take<unsigned long long>(2);
    m.huge_cap = (int64_t(1) << p.dir_bits) / (GAPHUGE + 1) + 2;
    m.huge = c.take<uint4>(m.huge_cap);
    m.sfx[0] = c.take<uint64_t>(n);
    m.sfx[1] = c.take<uint64_t>(n);
    m.hist = c.take<uint32_t>(radix_hist_entries(n));
    int64_t ts = scan_tiles(n), ts2 = scan_tiles(radix_hist_entries(n));
    m.tile_sums = c.take<uint64_t>(std::max(ts, ts2));
    if (p.kind == CG_DICT_TREE) {
        const int depth = tree_depth_of(ell, p.fanout_bits);
        m.tdep = c.take<uint16_t>(n);
        m.tlev = c.take<uint32_t>(depth + 1);
        m.thist = c.take<uint32_t>(depth);
    }
    *bytes = c.bytes();
    return m;
}

int ceil_log2(int64_t x) {
    int b = 0;
    while ((int64_t(1) << b) < x) ++b;
    return b;
}

}  // namespace

cg_dict_params resolve_params(int64_t ncap, cg_layout lay, const cg_dict_params *in) {
    cg_dict_params p;
    cg_dict_params_default(&p);
    if (in) p = *in;
    const int lg = ceil_log2(ncap > 2 ? ncap : 2);
    if (p.dir_bits < 0) p.dir_bits = std::max(1, std::min(lg, 22));
    if (p.dir_bits > lay.ell) p.dir_bits = lay.ell;
    if (p.split_bit < 0) {
        int s = ((lg + 16 + 31) / 32) * 32;
        p.split_bit = std::min(s, lay.ell);
    }
    if (p.group_max < 0) p.group_max = 64;
    if (p.kind == CG_DICT_TREE && p.fanout_bits == 0) p.fanout_bits = 2;
    return p;
}

size_t dict_mem_bytes(int64_t ncap, cg_layout lay, const cg_dict_params &p) {
    size_t b;
    carve_dict(nullptr, ncap, lay.ell, p, &b);
    return b;
}

// Directory from the dedup's sorted keys (the fused dedup + dictionary
// build): entry g is the first cell whose top p bits are >= g; the position
// that starts that cell is the first position whose key's top p bits are
// >= g (the previous position has smaller top bits, so it starts a cell).
// The sort key always keeps the top 32 bits, so no cell row is read.  A
// wave covers 64 positions and the entries from just past its first
// position's predecessor up to its last position: with at most DW of them,
// each lane takes entries 64 apart and finds its position by a binary
// search over the wave's 64 top-bit values in LDS, so writes leave
// coalesced; a wider stretch (sparse keys) is written as k_dict_scan does,
// each cell's entries by its own lane and long gaps listed for k_dir_gaps.
constexpr int DW = 4096;
constexpr int DK = 4;  // position chunks per block of the directory from sorted keys
__global__ void __launch_bounds__(DT) k_dir_from_keys(const uint32_t *__restrict__ keys,
                                                      const uint8_t *__restrict__ uniq,
                                                      const uint32_t *__restrict__ cidx, int64_t n,
                                                      const int64_t *d_ncells, int p, uint32_t *__restrict__ dir,
                                                      uint4 *__restrict__ gaps, unsigned long long *gap_n,
                                                      int64_t gap_cap, uint4 *__restrict__ huge, int64_t huge_cap) {
    __shared__ int64_t sg[DT];
    __shared__ uint32_t sc[DT];
    const int64_t G = int64_t(1) << p;
    const int lane = threadIdx.x & 63, wb = threadIdx.x & ~63;
    const int64_t nc = *d_ncells;
    // DK chunks of DT positions per block, their loads issued together; each
    // wave then handles its 64 positions of each chunk in turn
    uint8_t un[DK];
    uint32_t kk[DK], kq[DK], cc[DK];
#pragma unroll
    for (int k = 0; k < DK; ++k) {
        const int64_t i = (static_cast<int64_t>(blockIdx.x) * DK + k) * DT + threadIdx.x;
        const int64_t ii = i < n ? i : (n > 0 ? n - 1 : 0);
        un[k] = uniq[ii];
        kk[k] = keys[ii];
        kq[k] = keys[ii > 0 ? ii - 1 : 0];
        cc[k] = cidx[ii];
    }
#pragma unroll
    for (int k = 0; k < DK; ++k) {
        const int64_t i = (static_cast<int64_t>(blockIdx.x) * DK + k) * DT + threadIdx.x;
        const int64_t i0 = i - lane;  // the wave's first position
        if (i0 >= n) break;           // whole waves only: the shuffles below see every lane
        const bool valid = i < n;
        const uint32_t k0 = kk[k], c = cc[k];
        const bool act = valid && un[k] != 0;
        const int64_t gi = p ? static_cast<int64_t>(k0 >> (32 - p)) : 0;
        const int64_t gp = i == 0 ? -1 : (p ? static_cast<int64_t>(kq[k] >> (32 - p)) : 0);
        // the wave's stretch of entries: (lane 0's predecessor, last valid lane]
        const int64_t lo = static_cast<int64_t>(shfl_u64(static_cast<uint64_t>(gp), 0)) + 1;
        const int last = static_cast<int>((n - i0 < 64 ? n - i0 : 64) - 1);
        const int64_t hi = static_cast<int64_t>(shfl_u64(static_cast<uint64_t>(gi), last));
        if (hi - lo + 1 <= DW) {
            __builtin_amdgcn_wave_barrier();  // the previous chunk's searches are done with sg, sc
            sg[threadIdx.x] = valid ? gi : INT64_MAX;
            sc[threadIdx.x] = c;
            __builtin_amdgcn_wave_barrier();
            for (int64_t g = lo + lane; g <= hi; g += 64) {
                int a = 0, b = last;  // first lane whose top bits are >= g (lane last's are)
                while (a < b) {
                    const int m = (a + b) >> 1;
                    if (sg[wb + m] < g) a = m + 1; else b = m;
                }
                dir[g] = sc[wb + a];
            }
        } else {
            bool long_gap = false, huge_gap = false;
            if (act) {
                long_gap = gi - gp > GAPMIN;
                huge_gap = gi - gp > GAPHUGE;
                if (long_gap) {
                    dir[gi] = c;
                } else {
                    for (int64_t g = gp + 1; g <= gi; ++g) dir[g] = c;
                }
            }
            push_gap(gaps, gap_n, gap_cap, act && long_gap && !huge_gap, gp + 1, gi - 1, c);
            push_gap(huge, gap_n + 1, huge_cap, act && huge_gap, gp + 1, gi - 1, c);
        }
        if (act && static_cast<int64_t>(c) == nc - 1) {  // entries gi + 1 .. G point past the end
            if (G - gi > GAPMIN) {
                const bool hg = G - gi > GAPHUGE;
                const unsigned long long q = atomicAdd(hg ? gap_n + 1 : gap_n, 1ull);
                if (static_cast<int64_t>(q) < (hg ? huge_cap : gap_cap))
                    (hg ? huge : gaps)[q] = make_uint4(static_cast<uint32_t>(gi + 1), static_cast<uint32_t>(G),
                                                       static_cast<uint32_t>(nc), 0u);
            } else {
                for (int64_t g = gi + 1; g <= G; ++g) dir[g] = static_cast<uint32_t>(nc);
            }
        }
    }
}

// ------------------------------------------------------------ tree kind
// Section 3.2's 2^r-ary tree over the sorted cells, held as index ranges:
// level h has one node per distinct prefix of h digits (digit i = bits
// i r .. i r + r - 1, most significant first, zero past l), a node's cells
// are a contiguous range, and a leaf holds one cell, its id the value.
// Algorithm 3 builds the levels one after another; here they follow from
// each cell's shared depth with its predecessor: cell i >= 1 shares its
// node with cell i - 1 down to level floor(lcp / r) (lcp = their common
// leading bits) and starts a node at every deeper level, so level h holds
// 1 + |{i >= 1 : depth_i < h}| nodes.
constexpr int TREE_HB = 1024;  // shared depths counted in LDS below this, deeper ones in memory

template <typename T>
__global__ void __launch_bounds__(256) k_tree_depth(const T *__restrict__ cells, const int64_t *d_ncells,
                                                    int64_t ncap, int words, int r, int depth,
                                                    uint16_t *__restrict__ tdep, uint32_t *__restrict__ thist) {
    constexpr int B = Bits<T>::B;
    __shared__ uint32_t h[TREE_HB];
    for (int i = threadIdx.x; i < TREE_HB; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int64_t n = load_n(d_ncells, ncap);
    if (blockIdx.x == 0 && threadIdx.x == 0 && n > 0) tdep[0] = 0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x + 1; i < n; i += stride) {
        const T *a = cells + (i - 1) * words;
        const T *b = cells + i * words;
        int w = 0;
        T x = a[0] ^ b[0];
        while (x == T(0) && w + 1 < words) {
            ++w;
            x = a[w] ^ b[w];
        }
        const int lcp = x ? w * B + clz_t<T>(x) : words * B;
        int dl = lcp / r;
        if (dl > depth - 1) dl = depth - 1;  // equal rows (not sorted-distinct input): the deepest level
        tdep[i] = static_cast<uint16_t>(dl);
        if (dl < TREE_HB) atomicAdd(&h[dl], 1u);
        else atomicAdd(&thist[dl], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < TREE_HB && i < depth; i += blockDim.x)
        if (h[i]) atomicAdd(&thist[i], h[i]);
}

// Level sizes from the shared-depth counts: levels[0] = 1 (the root, when
// there are cells), levels[h] = levels[0] + count of depths below h.
__global__ void __launch_bounds__(256) k_tree_levels(const uint32_t *__restrict__ thist, int depth,
                                                     const int64_t *d_ncells, int64_t ncap,
                                                     uint32_t *__restrict__ tlev) {
    __shared__ uint64_t tmp[4];
    const int64_t n = load_n(d_ncells, ncap);
    const uint64_t root = n > 0 ? 1u : 0u;
    if (threadIdx.x == 0) tlev[0] = static_cast<uint32_t>(root);
    uint64_t carry = root;
    for (int c0 = 0; c0 < depth; c0 += 256) {
        const int v = c0 + static_cast<int>(threadIdx.x);
        const uint64_t x = v < depth ? thist[v] : 0u;
        uint64_t tot;
        const uint64_t ex = block256_excl_scan_u64(x, tmp, &tot);
        if (v < depth) tlev[v + 1] = static_cast<uint32_t>(carry + ex + x);
        carry += tot;
        __syncthreads();
    }
}

// Digit h of a row (r bits from bit h r, most significant first).
template <typename T>
__device__ __forceinline__ uint32_t digit_at(const T *row, int words, int r, int h) {
    constexpr int B = Bits<T>::B;
    const int p = h * r, w = p / B, o = p % B;
    if (o + r <= B) return static_cast<uint32_t>((row[w] >> (B - o - r)) & static_cast<T>((1u << r) - 1u));
    const int lo_bits = o + r - B;  // bits taken from the next word
    uint32_t d = static_cast<uint32_t>((row[w] & (static_cast<T>(~T(0)) >> o)) << lo_bits);
    if (w + 1 < words) d |= static_cast<uint32_t>(row[w + 1] >> (B - lo_bits));
    return d;
}

// Algorithm 4's search for q xor e_k (k < 0: q itself) down the tree: at
// level h the node's range narrows to the cells whose digit h is the
// query's (two binary searches over the range, which is sorted on that
// digit); a range of one cell is compared in full.
template <typename T>
__device__ int64_t find_tree(const T *cells, int words, int r, int depth, int64_t n, const T *q, int k) {
    int64_t lo = 0, hi = n;
    for (int h = 0; h < depth && hi - lo > 1; ++h) {
        uint32_t d = digit_at<T>(q, words, r, h);
        if (k >= h * r && k < h * r + r) d ^= 1u << (r - 1 - (k - h * r));
        int64_t a = lo, b = hi;
        while (a < b) {
            const int64_t m = a + ((b - a) >> 1);
            if (digit_at<T>(cells + m * words, words, r, h) < d) a = m + 1; else b = m;
        }
        int64_t c = a, e = hi;
        while (c < e) {
            const int64_t m = c + ((e - c) >> 1);
            if (digit_at<T>(cells + m * words, words, r, h) <= d) c = m + 1; else e = m;
        }
        lo = a;
        hi = c;
    }
    return hi > lo ? find_row<T>(cells, words, lo, hi, q, k) : -1;
}

// Distance-1 queries through the tree: one wave per query, a lane per
// flipped bit (the output is that of k_d1_query).
template <typename T>
__global__ void __launch_bounds__(256) k_d1_tree(const T *__restrict__ cells, const int64_t *d_n, int64_t ncap,
                                                 int words, int ell, int r, int depth,
                                                 const T *__restrict__ queries, int64_t nq,
                                                 uint32_t *__restrict__ count, uint32_t *__restrict__ self,
                                                 T *__restrict__ mask) {
    constexpr int B = Bits<T>::B;
    const int lane = threadIdx.x & 63;
    const int64_t wid = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    const int64_t n = load_n(d_n, ncap);
    for (int64_t qi = wid; qi < nq; qi += nw) {
        const T *q = queries + qi * words;
        uint32_t total = 0;
        for (int k0 = 0; k0 < ell; k0 += 64) {
            const int k = k0 + lane;
            const bool found = k < ell && find_tree<T>(cells, words, r, depth, n, q, k) >= 0;
            const uint64_t m = ballot64(found);
            total += static_cast<uint32_t>(__popcll(m));
            if (mask) {
                T *mrow = mask + qi * words;
                if (B == 64) {
                    if (lane == 0) mrow[k0 / 64] = static_cast<T>(__brevll(m));
                } else {
                    const int w = k0 / 32;
                    if (lane == 0) mrow[w] = static_cast<T>(__brev(static_cast<uint32_t>(m)));
                    if (lane == 1 && w + 1 < words) mrow[w + 1] = static_cast<T>(__brev(static_cast<uint32_t>(m >> 32)));
                }
            }
        }
        if (lane == 0) {
            if (count) count[qi] = total;
            if (self) {
                const int64_t id = find_tree<T>(cells, words, r, depth, n, q, -1);
                self[qi] = id >= 0 ? static_cast<uint32_t>(id) : 0xFFFFFFFFu;
            }
        }
    }
}

// The tree's arrays over d's cells (written by then in stream order).
template <typename T>
static cg_status tree_build(cg_dict &d, const DictMem &m, hipStream_t s) {
    const int r = d.params.fanout_bits;
    const int depth = tree_depth_of(d.lay.ell, r);
    CG_TRY(fill_u32(m.thist, 0u, depth, s));
    hipLaunchKernelGGL((k_tree_depth<T>), dim3(blocks_for(d.ncells_cap, 256, 4096)), dim3(256), 0, s,
                       static_cast<const T *>(d.cells), d.d_ncells, d.ncells_cap, d.lay.words, r, depth, m.tdep,
                       m.thist);
    CG_LAUNCHED("tree_depth");
    hipLaunchKernelGGL(k_tree_levels, dim3(1), dim3(256), 0, s, m.thist, depth, d.d_ncells, d.ncells_cap, m.tlev);
    CG_LAUNCHED("tree_levels");
    d.tree_depth = m.tdep;
    d.tree_levels = m.tlev;
    return CG_OK;
}

// The suffix-grouped order serves only the lookup path's S side (flips at
// k < s); other paths and s = 0 skip its sort.
static bool suffix_order_needed(const cg_dict_params &p) { return p.path == CG_PATH_LOOKUP && p.split_bit > 0; }

template <typename T> static cg_status dict_build_impl(cg_dict &d, hipStream_t s) {
    size_t b;
    DictMem m = carve_dict(d.mem, d.ncells_cap, d.lay.ell, d.params, &b);
    const int64_t ncap = d.ncells_cap;
    const int64_t G = int64_t(1) << d.params.dir_bits;
    const int64_t items = std::max<int64_t>(ncap, G + 1);
    const size_t lds = static_cast<size_t>(DT) * (d.lay.words | 1) * sizeof(T);
    const bool stage = lds <= 65536;
    CG_TRY(fill_i64(reinterpret_cast<int64_t *>(m.gap_n), 0, 2, s));
    hipLaunchKernelGGL((k_dict_scan<T>), dim3(blocks_for(items, DT)), dim3(DT), stage ? lds : 0, s,
                       static_cast<const T *>(d.cells), d.d_ncells, ncap, d.lay.words, d.params.dir_bits,
                       d.params.split_bit, m.dir, m.sfx[0], stage, m.gaps, m.gap_n, m.gap_cap, m.huge, m.huge_cap);
    CG_LAUNCHED("dict_scan");
    hipLaunchKernelGGL(k_dir_gaps, dim3(256), dim3(256), 0, s, m.dir, m.gaps, m.gap_n, m.gap_cap, m.huge, m.huge_cap);
    CG_LAUNCHED("dict_gaps");
    int which = 0;
    if (ncap > 0 && suffix_order_needed(d.params))
        CG_TRY(radix_sort_u64(m.sfx, nullptr, ncap, d.d_ncells, 32, 64, m.hist, m.tile_sums, &which, s));
    d.dir = m.dir;
    d.sfx = m.sfx[which];
    if (d.params.kind == CG_DICT_TREE) CG_TRY(tree_build<T>(d, m, s));
    return CG_OK;
}

// Fused dedup + dictionary build: the same cells, row_to_cell, directory
// and suffix order as cg_dedup followed by cg_dict_build, without reading
// the cells back (suffix hashes come from key extraction, the directory
// from the sorted keys).  d is filled as by cg_dict_build (cells = the
// dedup output, ncells_cap = n).
cg_status run_dedup_dict(const void *rows, int64_t n, cg_layout lay, void *cells, uint32_t *row_to_cell,
                         int64_t *d_ncells, void *ws, cg_dict &d, hipStream_t s) {
    size_t b;
    DictMem m = carve_dict(d.mem, d.ncells_cap, d.lay.ell, d.params, &b);
    const int64_t G = int64_t(1) << d.params.dir_bits;
    d.dir = m.dir;
    d.sfx = m.sfx[0];
    if (n == 0) {
        CG_TRY(fill_i64(d_ncells, 0, 1, s));
        if (d.params.kind == CG_DICT_TREE) {
            CG_TRY(fill_u32(m.tlev, 0u, tree_depth_of(lay.ell, d.params.fanout_bits) + 1, s));
            d.tree_depth = m.tdep;
            d.tree_levels = m.tlev;
        }
        return fill_u32(m.dir, 0u, G + 1, s);
    }
    DedupView v{};
    const bool sfx = suffix_order_needed(d.params);
    // the dedup's init launch also clears the gap-list counters
    CG_TRY(run_dedup_fused(rows, n, lay, cells, row_to_cell, d_ncells, ws, sfx ? d.params.split_bit : -1,
                           sfx ? m.sfx[0] : nullptr, &v, d.params.key_bits, m.gap_n, 2, s));
    hipLaunchKernelGGL(k_dir_from_keys, dim3(blocks_for(n, DT * DK)), dim3(DT), 0, s, v.khi, v.uniq, v.cidx, n, d_ncells,
                       d.params.dir_bits, m.dir, m.gaps, m.gap_n, m.gap_cap, m.huge, m.huge_cap);
    CG_LAUNCHED("dir_from_keys");
    hipLaunchKernelGGL(k_dir_gaps, dim3(256), dim3(256), 0, s, m.dir, m.gaps, m.gap_n, m.gap_cap, m.huge, m.huge_cap);
    CG_LAUNCHED("dict_gaps");
    int which = 0;
    if (sfx) CG_TRY(radix_sort_u64(m.sfx, nullptr, d.ncells_cap, d_ncells, 32, 64, m.hist, m.tile_sums, &which, s));
    d.sfx = m.sfx[which];
    if (d.params.kind == CG_DICT_TREE) {
        if (lay.word_bits == 64) CG_TRY(tree_build<uint64_t>(d, m, s));
        else CG_TRY(tree_build<uint32_t>(d, m, s));
    }
    return CG_OK;
}

cg_status run_dict_build(cg_dict &d, hipStream_t s) {
    if (d.lay.word_bits == 64) return dict_build_impl<uint64_t>(d, s);
    return dict_build_impl<uint32_t>(d, s);
}

template <typename T>
static cg_status d1_impl(const cg_dict &d, const void *q, int64_t nq, uint32_t *count, uint32_t *self, void *mask,
                         hipStream_t s) {
    if (nq == 0) return CG_OK;
    if (d.params.kind == CG_DICT_TREE) {
        hipLaunchKernelGGL((k_d1_tree<T>), dim3(blocks_for(nq, 4, 65536)), dim3(256), 0, s,
                           static_cast<const T *>(d.cells), d.d_ncells, d.ncells_cap, d.lay.words, d.lay.ell,
                           d.params.fanout_bits, tree_depth_of(d.lay.ell, d.params.fanout_bits),
                           static_cast<const T *>(q), nq, count, self, static_cast<T *>(mask));
        CG_LAUNCHED("d1_tree");
        return CG_OK;
    }
    if (d.lay.words <= D1_MW) {
        hipLaunchKernelGGL((k_d1_bucket<T>), dim3(blocks_for(nq, 4, 65536)), dim3(256), 0, s,
                           static_cast<const T *>(d.cells), d.lay.words, d.lay.ell, d.dir, d.params.dir_bits,
                           static_cast<const T *>(q), nq, count, self, static_cast<T *>(mask));
        CG_LAUNCHED("d1_bucket");
        return CG_OK;
    }
    hipLaunchKernelGGL((k_d1_query<T>), dim3(blocks_for(nq, 4, 65536)), dim3(256), 0, s,
                       static_cast<const T *>(d.cells), d.d_ncells, d.ncells_cap, d.lay.words, d.lay.ell, d.dir,
                       d.params.dir_bits, static_cast<const T *>(q), nq, count, self, static_cast<T *>(mask));
    CG_LAUNCHED("d1_query");
    return CG_OK;
}

cg_status run_neighbors_d1(const cg_dict &d, const void *q, int64_t nq, uint32_t *count, uint32_t *self,
                           void *mask, hipStream_t s) {
    if (d.lay.word_bits == 64) return d1_impl<uint64_t>(d, q, nq, count, self, mask, s);
    return d1_impl<uint32_t>(d, q, nq, count, self, mask, s);
}

}  // namespace cg
