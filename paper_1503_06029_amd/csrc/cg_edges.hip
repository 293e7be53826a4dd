// Edges of the cell graph over the dictionary's cells (Section 2.2), by
// flip-and-look-up (Section 3.2, Algorithm 4) organised around two orders.
//
// A distance-1 pair (u, v), u < v, differs at exactly one bit k, where u has
// 0 and v has 1 (lexicographic order).  With the split s of the dictionary:
//
//  - k >= s: u and v share bits 0 .. s-1, so v lies after u inside u's prefix
//    group (the cells sharing u's first s bits, contiguous in sorted order).
//    The P pass scans that group; when it holds more than group_max cells
//    after u, it looks up u xor e_k for each such k instead (binary search).
//  - k < s: u and v share bits s .. l-1, so they sit in one run of the
//    suffix-grouped order (equal 32-bit suffix hash; collisions are weeded
//    out by the exact distance test).  The S pass scans runs of up to
//    group_max cells, and looks up u xor e_k for k < s in longer runs.
//
// Every edge is found once, from u.  u's neighbours in ascending v are its
// flips in descending k: first its P-neighbours (k >= s) in group order,
// then its S-neighbours (k < s) in run order (ids ascend within a run).
// So edge slots are offsets[u] + rank for P, offsets[u] + cntP[u] + rank for
// S, with offsets = exclusive scan of cntP + cntS.
//
// Fast path (rows of at most 1024 bits): the S pass counts each cell's
// S-neighbours from the cells that share a suffix hash; one persistent P
// kernel streams every cell once through LDS (256-cell tiles), counts each
// cell's P-neighbours and stashes them per tile; a scan over tile totals
// gives offsets; placement writes P edges slot by slot, and a second S pass
// writes the S edges.  Pairs inside a group are pre-filtered with the bound
// (*) of Section 1.1 against the zero vector: a distance-1 pair has
// popcounts differing by exactly one.
// Generic path (longer rows): count and write passes over global memory.
#include "cg_internal.hpp"

namespace cg {

namespace {

// First s bits of a and b equal?
template <typename T>
__device__ __forceinline__ bool same_prefix(const T *a, const T *b, int s) {
    constexpr int B = Bits<T>::B;
    const int full = s / B, rem = s % B;
    for (int w = 0; w < full; ++w)
        if (a[w] != b[w]) return false;
    if (rem) {
        const T m = static_cast<T>(~T(0)) << (B - rem);
        if ((a[full] ^ b[full]) & m) return false;
    }
    return true;
}

__device__ __forceinline__ void emit(uint32_t *uv, uint16_t *bit, int64_t cap, int64_t pos, uint32_t u,
                                     uint32_t v, int k) {
    if (pos < cap) {
        uv[2 * pos] = u;
        uv[2 * pos + 1] = v;
        if (bit) bit[pos] = static_cast<uint16_t>(k);
    }
}

template <typename T, bool WRITE>
__global__ void __launch_bounds__(256) k_p_pass(const T *__restrict__ cells, const int64_t *d_n, int64_t ncap,
                                                int words, int ell, int s, int gmax, uint32_t *__restrict__ cntP,
                                                const int64_t *__restrict__ offsets, uint32_t *__restrict__ uv,
                                                uint16_t *__restrict__ bit, int64_t cap) {
    const int64_t n = load_n(d_n, ncap);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const T *me = cells + i * words;
        const int64_t base = WRITE ? offsets[i] : 0;
        uint32_t c = 0;
        bool big = false;
        for (int64_t j = i + 1; j < n; ++j) {
            const T *o = cells + j * words;
            if (!same_prefix<T>(me, o, s)) break;
            if (j - i > gmax) { big = true; break; }
            int pos;
            if (dist_upto2<T>(me, o, words, &pos) == 1) {
                if (WRITE) emit(uv, bit, cap, base + c, static_cast<uint32_t>(i), static_cast<uint32_t>(j), pos);
                ++c;
            }
        }
        if (big) {
            c = 0;
            for (int k = ell - 1; k >= s; --k) {
                if (get_bit<T>(me, k)) continue;
                const int64_t v = find_row<T>(cells, words, i + 1, n, me, k);
                if (v >= 0) {
                    if (WRITE) emit(uv, bit, cap, base + c, static_cast<uint32_t>(i), static_cast<uint32_t>(v), k);
                    ++c;
                }
            }
        }
        if (!WRITE) cntP[i] = c;
    }
}

template <typename T, bool WRITE>
__global__ void __launch_bounds__(256) k_s_pass(const T *__restrict__ cells, const uint64_t *__restrict__ sfx,
                                                const int64_t *d_n, int64_t ncap, int words, int s, int rmax,
                                                uint32_t *__restrict__ cntS, const uint32_t *__restrict__ cntP,
                                                const int64_t *__restrict__ offsets, uint32_t *__restrict__ uv,
                                                uint16_t *__restrict__ bit, int64_t cap) {
    const int64_t n = load_n(d_n, ncap);
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
         q += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const uint64_t e = sfx[q];
        const uint32_t h = static_cast<uint32_t>(e >> 32);
        const uint32_t id = static_cast<uint32_t>(e);
        int64_t left = 0, right = 0;
        while (left <= rmax && q - left - 1 >= 0 && static_cast<uint32_t>(sfx[q - left - 1] >> 32) == h) ++left;
        while (right <= rmax && q + right + 1 < n && static_cast<uint32_t>(sfx[q + right + 1] >> 32) == h) ++right;
        const T *me = cells + static_cast<int64_t>(id) * words;
        const int64_t base = WRITE ? offsets[id] + cntP[id] : 0;
        uint32_t c = 0;
        if (left + right + 1 > rmax) {
            for (int k = s - 1; k >= 0; --k) {
                if (get_bit<T>(me, k)) continue;
                const int64_t v = find_row<T>(cells, words, static_cast<int64_t>(id) + 1, n, me, k);
                if (v >= 0) {
                    if (WRITE) emit(uv, bit, cap, base + c, id, static_cast<uint32_t>(v), k);
                    ++c;
                }
            }
        } else {
            for (int64_t r = q - left; r <= q + right; ++r) {
                const uint32_t v = static_cast<uint32_t>(sfx[r]);
                if (v <= id) continue;
                int pos;
                if (dist_upto2<T>(me, cells + static_cast<int64_t>(v) * words, words, &pos) == 1 && pos < s) {
                    if (WRITE) emit(uv, bit, cap, base + c, id, v, pos);
                    ++c;
                }
            }
        }
        if (!WRITE) cntS[id] = c;
    }
}

__global__ void k_status(const int64_t *total, int64_t cap, int32_t *status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *status = (*total > cap) ? CG_ECAPACITY : CG_OK;
}

// ------------------------------------------------------------- fast path
//
// No inter-block waiting and no contended atomics (same-address device
// atomics serialise at roughly 10 ns each, so tickets and shared cursors do
// not scale).  The P pass keeps what it found in a per-tile stash and adds
// its tile total to one of 64-tile super-tiles; a placement block gets its
// output offset by summing the super-tiles and tiles before it, then copies
// its stash to the final slots.
//
//   E0 init      zero cntS and the super-tile totals
//   E1 S-count   per block of the suffix order: cntS[u] for cells followed by
//                an equal suffix hash, found S edges (with ranks) to the
//                block's S stash; starters of long runs to a list
//   E2 P-find    persistent, per cell tile, rows in LDS: cntP[u], P edges
//                (v - u, k) to the tile's P stash, tile and super-tile totals
//                of cntP + cntS; cells of long groups to a list (flag BIG)
//   E3 look-ups  listed cells of both sides (long S runs, long P groups),
//                one wave each: their counts, added to their tile totals
//   E4 P-place   per cell tile: offsets (the super-tile prefix summed in the
//                block when there are few super-tiles), |E| and status (last
//                tile), P edges from the stash slot by slot; then the listed
//                cells' S and P edges by look-up
//   E5 P-fix     tiles whose P stash overflowed: rescan and write
//   E6 S-place   stashed S edges to next(u) - cntS[u] + rank (blocks whose
//                stash overflowed run the S pass again in write mode)

constexpr int PT = 256;              // items per tile = threads per block
constexpr int P_STASH = 4 * PT;      // P edges kept per cell tile
constexpr uint32_t BIG = 0x80000000u;
constexpr int SUP = 64;              // tiles per super-tile

// Output offset of a cell tile: the exclusive prefix of the super-tile
// totals at its super-tile plus the totals of the tiles before it in that
// super-tile.  With raw_sup the super-tile totals are not scanned (at most
// SUP_INLINE of them) and the block sums those before its own; else they
// hold their exclusive prefix (k_sup_scan).  Block-wide over 256 threads,
// contains barriers.
constexpr int SUP_INLINE = 1024;
__device__ __forceinline__ uint64_t tile_offset(int64_t tile, const uint64_t *__restrict__ tile_tot,
                                                const uint64_t *__restrict__ sup, bool raw_sup, uint64_t *tmp) {
    const int64_t sidx = tile / SUP;
    const int64_t k2 = sidx * SUP + threadIdx.x;
    uint64_t part = (static_cast<int>(threadIdx.x) < SUP && k2 < tile) ? tile_tot[k2] : 0;
    if (raw_sup) {  // the super-tiles before this one join the same block sum
#pragma unroll
        for (int k = 0; k < SUP_INLINE / 256; ++k) {
            const int64_t j = threadIdx.x + 256 * k;
            if (j < sidx) part += sup[j];
        }
    }
    uint64_t tot;
    block256_excl_scan_u64(part, tmp, &tot);
    return (raw_sup ? 0 : sup[sidx]) + tot;
}



__global__ void k_edges_init(uint32_t *cntS, int64_t ncap, int64_t *d_nedges, int64_t *offsets, int32_t *status,
                             unsigned long long *big_n, uint64_t *sup_tot, int64_t nsup) {
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = gid; i < ncap; i += stride) cntS[i] = 0;
    for (int64_t i = gid; i < nsup; i += stride) sup_tot[i] = 0;
    if (gid == 0) {
        big_n[0] = 0;
        big_n[1] = 0;
        big_n[2] = 0;
        big_n[3] = 0;
        *d_nedges = 0;
        if (offsets) offsets[0] = 0;
        *status = CG_OK;
    }
}

// S pass over the suffix order (cells sorted by (32-bit suffix hash, id)).
// Only positions followed by an equal hash can have a later S-neighbour, so a
// block streams SC positions of the order and lists those "starters" in LDS.
// Each starter pairs with the later members of its run (at most rmax; ids
// ascend along a run, so partners come in ascending v); the (starter,
// partner) pairs of the block are numbered by a scan and checked by groups
// of four lanes, each lane taking every fourth word of both rows (so a row's
// words are read in 32-byte runs and 64 pairs are in flight per pass over
// the block; a block takes 1,024 positions so that one round trip of loads
// covers more of the order).  A found edge
// sets bit j - 1 of its starter's mask (j = partner's offset in the run), so
// a starter's rank of an edge is the popcount of its mask below j.  A starter
// followed by more than rmax members looks up u xor e_k for every k < s
// instead.  The count pass writes cntS[u]; the write pass redoes the checks
// and emits at next(u) - cntS[u] + rank.
constexpr int SC = 4 * PT;  // suffix-order positions per block (four per thread)
constexpr int SRMAX = 64;   // most later run members scanned; more use look-ups
constexpr int SG = 4;       // lanes per pair check (two for rows of up to two words)
constexpr int S_STASH = 256;  // S edges kept per block of the suffix order

template <typename T, bool WRITE>
__global__ void __launch_bounds__(PT) k_s_scan(const T *__restrict__ cells, const uint64_t *__restrict__ sfx,
                                               const int64_t *d_n, int64_t ncap, int words, int s, int rmax,
                                               uint32_t *__restrict__ cntS, const int64_t *__restrict__ offsets,
                                               const int64_t *__restrict__ offnext, uint32_t *__restrict__ uv,
                                               uint16_t *__restrict__ bit, int64_t cap, uint32_t *__restrict__ big_list,
                                               unsigned long long *__restrict__ big_n, uint4 *__restrict__ sstash,
                                               uint32_t *__restrict__ sstash_n) {
    constexpr int B = Bits<T>::B;
    constexpr int PER = SC / PT;
    __shared__ uint32_t hs[SC + 1];
    __shared__ uint32_t ids[SC];
    __shared__ uint16_t lst[SC];
    __shared__ uint32_t pofs[SC + 1];  // first pair of each starter; big starters own none
    __shared__ unsigned long long smask[SC];
    __shared__ uint2 sfound[S_STASH];  // (v, starter | j << 10 | pos << 17) of found S edges
    __shared__ uint32_t nfound;
    __shared__ uint64_t tmp[4];
    const int64_t n = load_n(d_n, ncap);
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * SC;
    if (c0 >= n) return;
    // the write pass only redoes blocks whose edges overflowed the stash
    if (WRITE) {
        const uint32_t m = sstash_n[blockIdx.x];
        if (m <= static_cast<uint32_t>(S_STASH)) {  // the stash holds this block's edges: drop them into place
            const uint4 *src = sstash + static_cast<int64_t>(blockIdx.x) * S_STASH;
            for (uint32_t f = threadIdx.x; f < m; f += PT) {
                const uint4 e = src[f];
                const int64_t next = offsets ? offsets[static_cast<int64_t>(e.x) + 1] : offnext[e.x];
                emit(uv, bit, cap, next - cntS[e.x] + (e.z >> 16), e.x, e.y, static_cast<int>(e.z & 0xffffu));
            }
            return;
        }
    }
    const int cl = static_cast<int>(n - c0 < SC ? n - c0 : SC);
    const bool hasnx = c0 + cl < n;  // hs[cl] holds the next position's hash
    const int t = threadIdx.x;
    if (t == 0) nfound = 0;
    {
        uint64_t v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = t + u * PT;
            v[u] = e < cl ? sfx[c0 + e] : 0;
        }
        const uint64_t nx = (t == 0 && hasnx) ? sfx[c0 + cl] : 0;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = t + u * PT;
            if (e < cl) {
                hs[e] = static_cast<uint32_t>(v[u] >> 32);
                ids[e] = static_cast<uint32_t>(v[u]);
            }
        }
        if (t == 0 && hasnx) hs[cl] = static_cast<uint32_t>(nx >> 32);
    }
    __syncthreads();
    auto hash_at = [&](int64_t p) -> uint32_t {
        const int64_t ep = p - c0;
        return (ep < cl || (ep == cl && hasnx)) ? hs[ep] : static_cast<uint32_t>(sfx[p] >> 32);
    };
    auto id_at = [&](int64_t p) -> uint32_t {
        const int64_t ep = p - c0;
        return ep < cl ? ids[ep] : static_cast<uint32_t>(sfx[p]);
    };
    // starters, in position order: thread t looks at positions PER t .. PER t + PER - 1
    uint32_t flags = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int e = t * PER + u;
        const bool st = e < cl && (e + 1 < cl || hasnx) && hs[e + 1] == hs[e];
        flags |= st ? (1u << u) : 0u;
    }
    uint64_t nst64;
    uint32_t k = static_cast<uint32_t>(block256_excl_scan_u64(static_cast<uint64_t>(__popc(flags)), tmp, &nst64));
    const int nst = static_cast<int>(nst64);
    // partners per starter (big: none, looked up below); starters k .. of this thread
    uint32_t np[PER];
    bool bigs[PER];
    uint32_t mine = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        np[u] = 0;
        bigs[u] = false;
        if (flags & (1u << u)) {
            const int e = t * PER + u;
            const int64_t q = c0 + e;
            const uint32_t h = hs[e];
            int L = 1;
            bool big = false;
            while (q + L + 1 < n && hash_at(q + L + 1) == h) {
                if (L == rmax) { big = true; break; }
                ++L;
            }
            bigs[u] = big;
            np[u] = big ? 0u : static_cast<uint32_t>(L);
            mine += np[u];
        }
    }
    uint64_t npairs64;
    uint32_t pf = static_cast<uint32_t>(block256_excl_scan_u64(mine, tmp, &npairs64));
    const uint32_t npairs = static_cast<uint32_t>(npairs64);
    uint32_t kk = k;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        if (flags & (1u << u)) {
            lst[kk] = static_cast<uint16_t>(t * PER + u);
            pofs[kk] = pf;
            smask[kk] = 0;
            pf += np[u];
            ++kk;
        }
    }
    if (t == 0) pofs[nst] = npairs;
    __syncthreads();

    // pair checks: group g of sg lanes takes pairs g, g + PT / sg, ... (sg the
    // same for every lane: two lanes for rows of up to two words, else SG)
    const int sg = words <= 2 ? 2 : SG;
    const int lg = t % sg, g = t / sg, ng = PT / sg;
    auto check_pair = [&](uint32_t pidx, int *li_out, int *j_out, uint32_t *u_out, uint32_t *v_out, int *pos_out) {
        int lo = 0, hi = nst;  // last starter with pofs <= pidx
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pofs[mid] <= pidx) lo = mid; else hi = mid;
        }
        const int j = static_cast<int>(pidx - pofs[lo]) + 1;
        const int e = lst[lo];
        const uint32_t u = ids[e];
        const uint32_t v = id_at(c0 + e + j);
        const T *a = cells + static_cast<int64_t>(u) * words;
        const T *b = cells + static_cast<int64_t>(v) * words;
        int d = 0, first = 0x7fffffff;
        for (int w = lg; w < words; w += sg) {
            const T x = a[w] ^ b[w];
            d += popc<T>(x);
            first = (x && first == 0x7fffffff) ? w * B + clz_t<T>(x) : first;
        }
        // the sg lanes of a pair are one aligned pair or quad: quad permutes
        if (sg == 4) {
            d += static_cast<int>(quad_xor2(static_cast<uint32_t>(d)));
            const int o = static_cast<int>(quad_xor2(static_cast<uint32_t>(first)));
            first = o < first ? o : first;
        }
        {
            d += static_cast<int>(quad_xor1(static_cast<uint32_t>(d)));
            const int o = static_cast<int>(quad_xor1(static_cast<uint32_t>(first)));
            first = o < first ? o : first;
        }
        *li_out = lo;
        *j_out = j;
        *u_out = u;
        *v_out = v;
        *pos_out = first;
        return d;
    };
    for (uint32_t p0 = 0; p0 < npairs; p0 += ng) {
        const uint32_t pidx = p0 + g;
        if (pidx < npairs) {  // uniform across the sg lanes of a group
            int li, j, pos;
            uint32_t u, v;
            const int d = check_pair(pidx, &li, &j, &u, &v, &pos);
            if (lg == 0 && d == 1 && pos < s) {
                atomicOr(&smask[li], 1ull << (j - 1));
                if (!WRITE) {
                    const uint32_t f = atomicAdd(&nfound, 1u);
                    if (f < static_cast<uint32_t>(S_STASH))
                        sfound[f] = make_uint2(v, static_cast<uint32_t>(li) | (static_cast<uint32_t>(j) << 10) |
                                                      (static_cast<uint32_t>(pos) << 17));
                }
            }
        }
    }
    __syncthreads();

    if (!WRITE) {
        kk = k;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            if (flags & (1u << u)) {
                const uint32_t c = static_cast<uint32_t>(__popcll(smask[kk]));
                if (c) cntS[ids[t * PER + u]] = c;
                ++kk;
            }
        }
        // starters of long runs go to k_big_lookup
#pragma unroll
        for (int u = 0; u < PER; ++u)
            wave_append<uint32_t>(big_list, big_n, n, (flags & (1u << u)) && bigs[u], ids[t * PER + u < cl ? t * PER + u : 0]);
        // found edges with their ranks to the block's stash (k_s_place drops them into place)
        const uint32_t nf = nfound;
        if (t == 0) sstash_n[blockIdx.x] = nf;
        if (nf <= static_cast<uint32_t>(S_STASH)) {
            uint4 *out = sstash + static_cast<int64_t>(blockIdx.x) * S_STASH;
            for (uint32_t f = t; f < nf; f += PT) {
                const uint2 e = sfound[f];
                const int li = static_cast<int>(e.y & 1023u), j = static_cast<int>((e.y >> 10) & 127u);
                const uint32_t rank = static_cast<uint32_t>(__popcll(smask[li] & ((1ull << (j - 1)) - 1ull)));
                out[f] = make_uint4(ids[lst[li]], e.x, (e.y >> 17) | (rank << 16), 0u);
            }
        }
        return;
    }
    // write: found pairs again, at next(u) - cntS[u] + rank
    for (uint32_t p0 = 0; p0 < npairs; p0 += ng) {
        const uint32_t pidx = p0 + g;
        if (pidx < npairs) {
            int li, j, pos;
            uint32_t u, v;
            const int d = check_pair(pidx, &li, &j, &u, &v, &pos);
            if (lg == 0 && d == 1 && pos < s) {
                const int64_t next = offsets ? offsets[static_cast<int64_t>(u) + 1] : offnext[u];
                const unsigned long long m = smask[li];
                const int64_t slot = next - cntS[u] + __popcll(m & ((1ull << (j - 1)) - 1ull));
                emit(uv, bit, cap, slot, u, v, pos);
            }
        }
    }
}

// Cells whose group (P) or run (S) is too long to scan are listed by the
// scanning kernels and handled by k_big_lookup, one wave per cell, lanes
// over the bits (wave_flip_lookups).

// One block: exclusive prefix of the super-tile totals, in place.
__global__ void __launch_bounds__(256) k_sup_scan(uint64_t *sup_tot, int64_t nsup) {
    __shared__ uint64_t tmp[4];
    uint64_t carry = 0;
    for (int64_t k0 = 0; k0 < nsup; k0 += 256) {
        const int64_t k = k0 + threadIdx.x;
        const uint64_t x = k < nsup ? sup_tot[k] : 0;
        uint64_t tot;
        const uint64_t ex = block256_excl_scan_u64(x, tmp, &tot);
        if (k < nsup) sup_tot[k] = carry + ex;
        carry += tot;
    }
}

// Listed cells of both sides in one launch: items [0, nS) are S-listed
// cells (k < s), then the P-listed ones (k >= s), one wave each.  Count
// (WRITE = false): cntS[u] or cntP[u] (flagged BIG), and the count is added
// to the cell's tile and super-tile totals (k_p_find has already written
// those, counting these cells as 0).  Write: the edges at their slots.
constexpr int BQ = 128;                 // listed-cell neighbours a wave keeps in LDS
constexpr uint32_t BST_NONE = 0xFFFFFFFFu;

template <typename T, bool WRITE>
__global__ void __launch_bounds__(256) k_big_lookup(const T *__restrict__ cells, const uint32_t *__restrict__ dir,
                                                    int p, int words, int ell, int s,
                                                    const uint32_t *__restrict__ s_list,
                                                    const uint32_t *__restrict__ p_list,
                                                    const unsigned long long *__restrict__ big_n, int64_t list_cap,
                                                    uint32_t *__restrict__ cntS, uint32_t *__restrict__ cntP,
                                                    uint64_t *__restrict__ tile_tot, uint64_t *__restrict__ sup_tot,
                                                    const int64_t *__restrict__ offsets,
                                                    const int64_t *__restrict__ offnext, uint32_t *__restrict__ uv,
                                                    uint16_t *__restrict__ bit, int64_t cap,
                                                    uint2 *__restrict__ bst, unsigned long long *__restrict__ bst_n,
                                                    int64_t bst_cap, uint32_t *__restrict__ bstart) {
    // the count pass keeps each listed cell's neighbours (v, k) in found order
    // (a wave's first BQ in LDS, then a share of bst reserved for them), so
    // the write pass copies them instead of searching again; a cell with more,
    // or past bst's capacity, is searched again (bstart = BST_NONE)
    __shared__ uint2 bq[4][BQ];
    const int wv = threadIdx.x >> 6;
    int64_t ns = static_cast<int64_t>(big_n[0]), np = static_cast<int64_t>(big_n[1]);
    if (ns > list_cap) ns = list_cap;
    if (np > list_cap) np = list_cap;
    const int lane = threadIdx.x & 63;
    const int64_t nw = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
    for (int64_t it = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); it < ns + np;
         it += nw) {
        const bool sside = it < ns;  // the same for the whole wave
        const uint32_t u = sside ? s_list[it] : p_list[it - ns];
        const T *q = cells + static_cast<int64_t>(u) * words;
        const int khi = sside ? s - 1 : ell - 1, klo = sside ? 0 : s;
        // a P-neighbour (k >= s) follows u inside u's prefix group: search
        // [u + 1, end of the group) only (the end found once per cell by a
        // galloping search over the first s bits; dir's last entry is the
        // cell count)
        int64_t lo_b = 0, hi_b = INT64_MAX;
        if (!sside) {
            const int64_t n = dir[static_cast<int64_t>(1) << p];
            int64_t good = u, bad = static_cast<int64_t>(u) + 1, step = 1;
            while (bad < n && same_prefix<T>(cells + bad * words, q, s)) {
                good = bad;
                step <<= 1;
                bad = static_cast<int64_t>(u) + step;
            }
            if (bad > n) bad = n;
            while (bad - good > 1) {
                const int64_t mid = good + ((bad - good) >> 1);
                if (same_prefix<T>(cells + mid * words, q, s)) good = mid; else bad = mid;
            }
            lo_b = static_cast<int64_t>(u) + 1;
            hi_b = bad;
        }
        if (!WRITE) {
            const uint32_t c = wave_flip_lookups<T>(cells, words, dir, p, q, khi, klo, [&](uint32_t v, int k, uint32_t r) {
                if (r < static_cast<uint32_t>(BQ)) bq[wv][r] = make_uint2(v, static_cast<uint32_t>(k));
            }, lo_b, hi_b);
            __builtin_amdgcn_wave_barrier();
            uint32_t st = c == 0 ? 0u : BST_NONE;
            if (c > 0 && c <= static_cast<uint32_t>(BQ)) {
                unsigned long long b0 = 0;
                if (lane == 0) b0 = atomicAdd(bst_n, static_cast<unsigned long long>(c));
                b0 = shfl_u64(b0, 0);
                if (static_cast<int64_t>(b0 + c) <= bst_cap) {
                    st = static_cast<uint32_t>(b0);
                    for (uint32_t r = lane; r < c; r += 64) bst[b0 + r] = bq[wv][r];
                }
            }
            __builtin_amdgcn_wave_barrier();  // bq is free for the wave's next cell
            if (lane == 0) {
                bstart[it] = st;
                if (sside) cntS[u] = c; else cntP[u] = BIG | c;
                atomicAdd(reinterpret_cast<unsigned long long *>(&tile_tot[u / PT]), static_cast<unsigned long long>(c));
                atomicAdd(reinterpret_cast<unsigned long long *>(&sup_tot[(u / PT) / SUP]),
                          static_cast<unsigned long long>(c));
            }
        } else {
            int64_t base;
            if (sside) {
                const uint32_t ct = cntS[u];
                base = (offsets ? offsets[static_cast<int64_t>(u) + 1] : offnext[u]) - ct;
            } else {
                base = offsets ? offsets[u]
                               : offnext[u] - static_cast<int64_t>(cntP[u] & ~BIG) - static_cast<int64_t>(cntS[u]);
            }
            const uint32_t st = bstart[it];
            if (st != BST_NONE) {
                const uint32_t c = sside ? cntS[u] : (cntP[u] & ~BIG);
                for (uint32_t r = lane; r < c; r += 64) {
                    const uint2 e = bst[static_cast<int64_t>(st) + r];
                    emit(uv, bit, cap, base + r, u, e.x, static_cast<int>(e.y));
                }
            } else {
                wave_flip_lookups<T>(cells, words, dir, p, q, khi, klo, [&](uint32_t v, int k, uint32_t r) {
                    emit(uv, bit, cap, base + r, u, v, k);
                }, lo_b, hi_b);
            }
        }
    }
}

// ---------------------------------------------------------------- P tiles
//
// A P tile holds PT cells plus up to HALO following rows (for the prefix
// group that crosses the tile's end) in LDS, each row zero-padded to WT
// words (WT a power of two, fixed at compile time, so every row operation
// is straight-line code; the zero words change neither distances nor order).

constexpr int HALO = 32;       // rows past the tile kept in LDS
constexpr int NB = 12;         // P-neighbours remembered per cell between count and write
constexpr int PROWS = PT + HALO;

template <typename T, int WT> struct PTile {
    static constexpr int LW = WT + 1;  // odd stride: lanes reading different rows spread over banks
    static constexpr size_t rows_bytes = static_cast<size_t>(PROWS) * LW * sizeof(T);
    static constexpr size_t bytes = rows_bytes + PROWS * 4 /* pcs */ + PT * NB * 4 /* nbl */ + PROWS + 4 /* heads */;
};

// Block-wide copy of nrows contiguous global rows into LDS rows padded with
// zero words to WT (stride LW), U loads in flight per thread.
template <typename T, int WT, int NT, int U>
__device__ __forceinline__ void copy_rows_padded(T *lds, const T *__restrict__ src, int nrows, int words) {
    constexpr int LW = WT + 1;
    const int tot = nrows * WT;
    for (int e0 = threadIdx.x; e0 < tot; e0 += NT * U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * NT;
            const int r = e / WT, w = e % WT;
            v[u] = (e < tot && w < words) ? src[r * words + w] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * NT;
            if (e < tot) lds[(e / WT) * LW + (e % WT)] = v[u];
        }
    }
}

// Only the ceil(s / B) words that hold the prefix are read (s is the same
// for every lane, so the per-word tests are uniform branches).
template <typename T, int WT>
__device__ __forceinline__ bool same_prefix_t(const T *a, const T *b, int s) {
    constexpr int B = Bits<T>::B;
    const int full = s / B, rem = s % B;
    T acc = 0;
#pragma unroll
    for (int w = 0; w < WT; ++w)
        if (w < full) acc |= a[w] ^ b[w];
    if (rem && full < WT) acc |= (a[full] ^ b[full]) & (static_cast<T>(~T(0)) << (B - rem));
    return acc == 0;
}

// Loads the tile (tr rows) and its halo (rows after it sharing the last
// row's first s bits, at most HALO) into LDS with popcounts and group heads
// (heads[r] = 1 iff row r starts a prefix group; heads[tr + th] = 0 iff the
// last group may continue past the loaded rows).
template <typename T, int WT>
__device__ __forceinline__ int load_ptile(T *rows, uint32_t *pcs, uint8_t *heads, int *s_th,
                                          const T *__restrict__ cells, int words, int s, int64_t base, int64_t n,
                                          int *th) {
    constexpr int LW = WT + 1;
    const int tr = static_cast<int>(n - base < PT ? n - base : PT);
    copy_rows_padded<T, WT, PT, 16>(rows, cells + base * words, tr, words);
    if (threadIdx.x == 0) *s_th = HALO;
    __syncthreads();
    const int64_t avail = n - base - tr;
    const int hmax = static_cast<int>(avail < HALO ? avail : HALO);
    if (static_cast<int>(threadIdx.x) < hmax) {
        const T *o = cells + (base + tr + threadIdx.x) * words;
        if (!same_prefix<T>(rows + (tr - 1) * LW, o, s)) atomicMin(s_th, static_cast<int>(threadIdx.x));
    }
    __syncthreads();
    const int h = *s_th < hmax ? *s_th : hmax;
    copy_rows_padded<T, WT, PT, 4>(rows + tr * LW, cells + (base + tr) * words, h, words);
    __syncthreads();
    for (int r = threadIdx.x; r < tr + h; r += PT) {
        uint32_t pc = 0;
        const T *me = rows + r * LW;
#pragma unroll
        for (int w = 0; w < WT; ++w) pc += popc<T>(me[w]);
        pcs[r] = pc;
        heads[r] = (r == 0 || !same_prefix_t<T, WT>(rows + (r - 1) * LW, me, s)) ? 1 : 0;
    }
    // past the loaded rows: 0 if the last group may go on (full halo, more cells), else 1
    if (threadIdx.x == 0) heads[tr + h] = (h == HALO && base + tr + h < n) ? 0 : 1;
    __syncthreads();
    *th = h;
    return tr;
}

// P-neighbours of tile cell t (global index i), in ascending v: the rest of
// its prefix group, from LDS, then past the loaded rows in global memory.
// f(delta = v - i, k, rank) per neighbour.  Returns the count, or BIG when
// the group holds more than gmax cells after i (f is then not called).
template <typename T, int WT, class F>
__device__ __forceinline__ uint32_t p_scan_t(const T *rows, const uint32_t *pcs, const uint8_t *heads, int tl,
                                             int t, int64_t i, int64_t base, int64_t n,
                                             const T *__restrict__ cells, int words, int s, int gmax, F f) {
    constexpr int LW = WT + 1;
    const T *me = rows + t * LW;
    const uint32_t pc = pcs[t];
    uint32_t c = 0;
    int jj = t + 1;
    for (; jj < tl; ++jj) {
        if (heads[jj]) return c;
        if (jj - t > gmax) return BIG;
        const uint32_t po = pcs[jj];
        if (po == pc + 1 || po + 1 == pc) {
            int pos;
            if (dist_t<T, WT>(me, rows + jj * LW, &pos) == 1) { f(static_cast<uint32_t>(jj - t), pos, c); ++c; }
        }
    }
    if (!heads[tl]) {
        // loaded rows ended inside the group: it goes on in global memory
        for (int64_t j = base + tl; j < n; ++j) {
            const T *o = cells + j * words;
            if (!same_prefix<T>(me, o, s)) break;
            if (j - i > gmax) return BIG;
            int pos;
            if (dist_full<T>(me, o, words, &pos) == 1) { f(static_cast<uint32_t>(j - i), pos, c); ++c; }
        }
    }
    return c;
}

// Look-up form of the P-neighbours of cell i (all k >= s, descending k).
template <typename T, class F>
__device__ __forceinline__ uint32_t p_lookup(const T *__restrict__ cells, int64_t i, int64_t n, int words, int ell,
                                             int s, F f) {
    const T *me = cells + i * words;
    uint32_t c = 0;
    for (int k = ell - 1; k >= s; --k) {
        if (get_bit<T>(me, k)) continue;
        const int64_t v = find_row<T>(cells, words, i + 1, n, me, k);
        if (v >= 0) { f(static_cast<uint32_t>(v), k, c); ++c; }
    }
    return c;
}

// Count and record the P-neighbours of one tile.  Each wave owns 64 cells of
// the tile and works alone after the tile is in LDS (two block barriers per
// tile: LDS reuse and LDS fill).  A lane walks its cell's prefix group over
// the offset d = j - i, four offsets per step, keeping pairs whose popcounts
// differ by exactly one (the bound (*) of Section 1.1 against the zero
// vector); each step's candidates go straight into the wave's ring queue,
// which is verified (full-row distance in LDS) 64 entries at a time, so the
// row comparisons run on full waves.  A hit sets bit d - 1 of the cell's
// offset mask and is listed with its position; since scans stop at
// d = PSCAN, a cell's rank of an edge is the popcount of its mask below d.
// Row popcounts carry two flags: HEADF (the row starts a prefix group) and
// PASTF (past the loaded rows), so a lane stops at either with one compare.
constexpr int CQ = 128;                // per-wave candidate ring (a power of two, at least 128)
constexpr int PSCAN = 64;              // longest in-tile scan; longer groups use look-ups
constexpr int PWAVES = PT / 64;        // waves per block, 64 cells each
constexpr int WST = P_STASH / PWAVES;  // stash entries per wave
constexpr int PCS = PT + PSCAN + 8;    // popcount entries: rows, then PASTF padding for the scans
constexpr uint32_t HEADF = 0x40000000u;
constexpr uint32_t PASTF = 0x80000000u;

template <typename T, int WT> struct PFind {
    static constexpr int LW = WT + 1;
    static constexpr size_t rows_bytes = static_cast<size_t>(PROWS) * LW * sizeof(T);
    // rows | mask[PT] (u64) | pcs[PCS] | res[P_STASH] | ring[PWAVES][CQ] | sbase[PT]
    static constexpr size_t bytes = rows_bytes + PT * 8 + PCS * 4 + P_STASH * 4 + PWAVES * CQ * 4 + PT * 4;
};

// Distance of two LDS rows of WT words; *pos = the first differing position
// when the distance is 1 (the word index is kept while summing popcounts and
// the word is read once more at the end).
template <typename T, int WT>
__device__ __forceinline__ int dist_lds(const T *a, const T *b, int *pos) {
    constexpr int B = Bits<T>::B;
    int d = 0, wi = 0;
#pragma unroll
    for (int w = 0; w < WT; ++w) {  // unrolled: the LDS loads issue together
        const T x = a[w] ^ b[w];
        d += popc<T>(x);
        wi = x ? w : wi;
    }
    const T x = a[wi] ^ b[wi];
    *pos = wi * B + clz_t<T>(x | T(1));
    return d;
}

// Persistent: each block walks a strided sequence of tiles and, while it
// works on one tile in LDS, already has the next tile's rows (tile plus
// HALO rows) and cntS values in flight in registers, so the stream of rows
// never waits for the comparisons.  Tiles are dealt out per XCD (workgroups
// go round-robin over the 8 XCDs): XCD x takes the x-th eighth of the
// tiles, so a tile and the one after it (whose first rows are the tile's
// halo) are read on the same XCD at about the same time and the halo comes
// from that XCD's L2.  FULLW: rows are exactly WT words, so a tile is one
// contiguous run of words and loads and LDS stores need no index arithmetic.
template <typename T, int WT> constexpr int p_find_blocks() { return (sizeof(T) == 4 && WT == 32) ? 2 : 3; }

template <typename T, int WT, bool FULLW>
__global__ void __launch_bounds__(PT, (p_find_blocks<T, WT>())) k_p_find(const T *__restrict__ cells,
                                               const int64_t *d_n, int64_t ncap, int words, int ell, int s, int gmax,
                                               const uint32_t *__restrict__ cntS, uint32_t *__restrict__ cntP,
                                               uint32_t *__restrict__ stash, uint32_t *__restrict__ stash_n,
                                               uint64_t *__restrict__ tile_tot, uint64_t *__restrict__ sup_tot,
                                               uint32_t *__restrict__ big_list, unsigned long long *__restrict__ big_n,
                                               uint32_t *__restrict__ fix_list, unsigned long long *__restrict__ fix_n) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_nres[PWAVES];
    __shared__ uint64_t s_tot;
    __shared__ uint32_t s_ovf;
    using L = PFind<T, WT>;
    constexpr int LW = L::LW;
    constexpr int NE = (PROWS * WT + PT - 1) / PT;  // prefetched words per thread
    constexpr int RPU = PT / WT;                     // rows per prefetch step (PT is a multiple of WT)
    T *rows = reinterpret_cast<T *>(smem);
    unsigned long long *mask = reinterpret_cast<unsigned long long *>(smem + L::rows_bytes);
    uint32_t *pcs = reinterpret_cast<uint32_t *>(mask + PT);
    uint32_t *res = pcs + PCS;
    uint32_t *ring = res + P_STASH;
    uint32_t *sbase = ring + PWAVES * CQ;
    const int64_t n = load_n(d_n, ncap);
    const int64_t ntiles = (n + PT - 1) / PT;
    const int G8 = static_cast<int>(gridDim.x >> 3);
    const int xcd = static_cast<int>(blockIdx.x & 7), lb = static_cast<int>(blockIdx.x >> 3);
    const int64_t T8 = (ntiles + 7) / 8;
    const int64_t r0 = xcd * T8;
    const int64_t r1 = r0 + T8 < ntiles ? r0 + T8 : ntiles;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    uint32_t *q = ring + wv * CQ;
    uint32_t *wres = res + wv * WST;
    const int gm = gmax < PSCAN ? gmax : PSCAN;

    // FULLW with rows a whole number of 16-byte chunks: the tile moves as
    // 16-byte pieces (half the load instructions of word loads)
    constexpr bool V16 = FULLW && (WT * sizeof(T)) % 16 == 0;
    constexpr int PW = 16 / static_cast<int>(sizeof(T));                // words per piece
    constexpr int NC = (PROWS * WT / PW + PT - 1) / PT;                 // pieces per thread
    constexpr int NPRE = V16 ? NC * PW : NE;
    T pre[NPRE];
    uint32_t pre_cs = 0;
    auto prefetch = [&](int64_t tile) {
        const int64_t base = tile * PT;
        const int64_t av = n - base;
        const int avail = static_cast<int>(av < PROWS ? av : PROWS);
        const T *src = cells + base * words;
        if (V16 && avail == PROWS) {  // the tile and its halo are all there: plain 16-byte loads
            const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
#pragma unroll
            for (int u = 0; u < NC; ++u) {
                const int c = t + u * PT;
                const uint4 v = c < PROWS * WT / PW ? s4[c] : make_uint4(0u, 0u, 0u, 0u);
                const T *pv = reinterpret_cast<const T *>(&v);
#pragma unroll
                for (int k = 0; k < PW; ++k) pre[u * PW + k] = pv[k];
            }
        } else if (FULLW && avail == PROWS) {  // plain word loads
#pragma unroll
            for (int u = 0; u < NE; ++u) {
                const int e = t + u * PT;
                pre[u] = e < PROWS * WT ? src[e] : T(0);
            }
        } else {
            // every load is issued (out-of-range ones read the tile's first
            // word, which exists) and masked when stored to LDS
            const int tot = avail * WT;
#pragma unroll
            for (int u = 0; u < NE; ++u) {
                const int e = t + u * PT;
                const int r = e / WT, w = e % WT;
                const bool ok = e < tot && w < words;
                pre[u] = src[ok ? r * words + w : 0];
            }
        }
        pre_cs = cntS[base + t < n ? base + t : base];
    };

    int64_t tile = r0 + lb;
    int64_t prev = -1;
    if (tile < r1) prefetch(tile);
    if (t == 0) {
        s_tot = 0;
        s_ovf = 0;
    }
    for (; tile < r1; tile += G8) {
        const int64_t base = tile * PT;
        const int tr = static_cast<int>(n - base < PT ? n - base : PT);
        const int tl = static_cast<int>(n - base < PROWS ? n - base : PROWS);  // loaded rows
        __syncthreads();  // the previous tile's LDS is free; its total is complete
        if (t == 0) {
            if (prev >= 0) {
                const uint64_t tot = s_tot;
                tile_tot[prev] = tot;
                atomicAdd(reinterpret_cast<unsigned long long *>(&sup_tot[prev / SUP]),
                          static_cast<unsigned long long>(tot));
            }
            s_tot = 0;
            s_ovf = 0;
        }
        if (V16 && tl == PROWS) {
            // piece c holds words c * PW .. c * PW + PW - 1 of the tile, all in one row
#pragma unroll
            for (int u = 0; u < NC; ++u) {
                const int c = t + u * PT;
                if (c < PROWS * WT / PW) {
                    T *dst = rows + ((c * PW) / WT) * LW + ((c * PW) % WT);
#pragma unroll
                    for (int k = 0; k < PW; ++k) dst[k] = pre[u * PW + k];
                }
            }
        } else {
            const int tot = tl * WT;
            const bool full = FULLW && tl == PROWS;
#pragma unroll
            for (int u = 0; u < NE; ++u) {
                const int e = t + u * PT;
                if (e < PROWS * WT) {
                    // e / WT = t / WT + u * RPU and e % WT = t % WT
                    T *dst = rows + (t / WT + u * RPU) * LW + (t % WT);
                    *dst = (full || (e < tot && (e % WT) < words)) ? pre[u] : T(0);
                }
            }
        }
        const uint32_t cs = base + t < n ? pre_cs : 0u;
        // the registers are free once stored: the next tile's loads go out now,
        // before the barriers, so they are in flight during all of this tile
        if (tile + G8 < r1) prefetch(tile + G8);
        mask[t] = 0;
        if (lane == 0) s_nres[wv] = 0;
        __syncthreads();
        for (int r = t; r < tl; r += PT) {
            const T *me = rows + r * LW;
            uint32_t pc = 0;
#pragma unroll
            for (int w = 0; w < WT; ++w) pc += popc<T>(me[w]);
            const bool hd = r == 0 || !same_prefix_t<T, WT>(me - LW, me, s);
            pcs[r] = pc | (hd ? HEADF : 0u);
        }
        for (int r = tl + t; r < PCS; r += PT) pcs[r] = PASTF;
        __syncthreads();
        const int64_t i = base + t;
        const bool more = base + tl < n;  // cells exist past the loaded rows

        // verify `cnt` ring entries from `from` (one per lane); hits to the
        // mask and the wave's result list (one LDS counter update per wave)
        auto verify = [&](uint32_t from, uint32_t cnt) {
            const bool act = static_cast<uint32_t>(lane) < cnt;
            const uint32_t e = act ? q[(from + lane) & (CQ - 1)] : 0u;
            const int t0 = static_cast<int>(e >> 16), j0 = static_cast<int>(e & 0xffffu);
            int pos;
            const bool hit = act && dist_lds<T, WT>(rows + t0 * LW, rows + j0 * LW, &pos) == 1;
            if (hit) atomicOr(&mask[t0], 1ull << (j0 - t0 - 1));
            const uint64_t hm = ballot64(hit);
            if (hm) {
                uint32_t rb = 0;
                if (lane == 0) rb = atomicAdd(&s_nres[wv], static_cast<uint32_t>(__popcll(hm)));
                rb = __shfl(rb, 0, 64);
                if (hit) {
                    const uint32_t r = rb + static_cast<uint32_t>(__popcll(hm & lanemask_lt()));
                    if (r < static_cast<uint32_t>(WST))
                        wres[r] = (static_cast<uint32_t>(t0) << 24) | (static_cast<uint32_t>(j0 - t0) << 16) |
                                  static_cast<uint32_t>(pos);
                }
            }
        };

        // Each cell's run: the loaded rows after it up to the next group head
        // or the end of the loaded rows (every flag is in a 64-row mask; the
        // wave's three masks cover rows t + 1 .. t + gm + 1).  A run longer
        // than gm rows means look-ups (big); a run that stops at the end of
        // the loaded rows while cells remain is finished in global memory
        // (spill).  Then a lock-step scan over d up to the longest run.
        const uint32_t pcm1 = (pcs[t] & 0x3fffffffu) - 1u;
        int run = 0;
        bool big = false, spill = false;
        {
            unsigned long long hm[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int r = (wv + k) * 64 + lane;
                hm[k] = ballot64(r < PCS && pcs[r] >= HEADF);
            }
            const int r1 = lane + 1;  // row t + 1, counted from the wave's first row
            const unsigned long long a0 = r1 < 64 ? hm[0] & (~0ull << r1) : 0ull;
            const unsigned long long a1 = r1 < 64 ? hm[1] : hm[1] & (~0ull << (r1 - 64));
            const int e = a0 ? __ffsll(a0) - 1 : (a1 ? 64 + __ffsll(a1) - 1 : (hm[2] ? 128 + __ffsll(hm[2]) - 1 : 192));
            const int de = e - lane;  // offset of the first flagged row after t
            if (t < tr) {
                if (de <= gm + 1) {
                    run = de - 1 < gm ? de - 1 : gm;
                    spill = pcs[t + de] >= PASTF && more;
                } else {
                    run = gm;
                    big = true;
                }
            }
        }
        int rmax = run;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int v = __shfl_xor(rmax, o, 64);
            rmax = v > rmax ? v : rmax;
        }
        uint32_t qh = 0, qt = 0;  // ring head and tail (wave-uniform)
        const uint32_t *pp = pcs + t;
        uint32_t xn = pp[1];  // the next offset's entry is read one step ahead
#pragma unroll 1
        for (int d = 1; d <= rmax; ++d) {
            const uint32_t x = xn;
            xn = pp[d + 1];
            const bool cand = d <= run && ((x - pcm1) & ~2u) == 0u;
            const uint64_t m = ballot64(cand);
            if (m) {
                if (cand) q[(qt + static_cast<uint32_t>(__popcll(m & lanemask_lt()))) & (CQ - 1)] =
                    (static_cast<uint32_t>(t) << 16) | static_cast<uint32_t>(t + d);
                qt += static_cast<uint32_t>(__popcll(m));
                if (qt - qh >= 64u) {
                    __builtin_amdgcn_wave_barrier();
                    verify(qh, 64u);
                    qh += 64u;
                }
            }
        }
        if (qt != qh) {
            __builtin_amdgcn_wave_barrier();
            verify(qh, qt - qh);
        }
        if (spill && !big) {
            // the group goes on past the loaded rows: finish it in global memory
            const T *me = rows + t * LW;
            for (int64_t j = base + tl; j < n; ++j) {
                const T *o = cells + j * words;
                if (!same_prefix<T>(me, o, s)) break;
                if (j - i > gm) { big = true; break; }
                int pos;
                if (dist_full<T>(me, o, words, &pos) == 1) {
                    const int d0 = static_cast<int>(j - i);
                    atomicOr(&mask[t], 1ull << (d0 - 1));
                    const uint32_t r = atomicAdd(&s_nres[wv], 1u);
                    if (r < static_cast<uint32_t>(WST))
                        wres[r] = (static_cast<uint32_t>(t) << 24) | (static_cast<uint32_t>(d0) << 16) |
                                  static_cast<uint32_t>(pos);
                }
            }
        }
        // cells of long groups: counted by k_big_lookup, which also adds them to the tile total
        wave_append<uint32_t>(big_list, big_n, n, big && t < tr, static_cast<uint32_t>(i));
        __builtin_amdgcn_wave_barrier();
        uint32_t cp = 0;
        if (t < tr) {
            cp = big ? BIG : static_cast<uint32_t>(__popcll(mask[t]));
            cntP[i] = cp;
        }
        const uint32_t stashed = (cp & BIG) ? 0u : cp;
        const uint32_t inc = wave_incl_scan_u32(stashed);
        const uint32_t tot_stash = lane63_u32(inc);
        const uint32_t all = wave_incl_scan_u32((cp & ~BIG) + (t < tr ? cs : 0u));
        sbase[t] = (cp & BIG) ? 0xffffffffu : inc - stashed;
        const uint32_t wall = lane63_u32(all);
        const uint32_t nres = s_nres[wv];
        const uint32_t m = nres > tot_stash ? nres : tot_stash;
        if (lane == 0) {
            stash_n[tile * PWAVES + wv] = m;
            atomicAdd(reinterpret_cast<unsigned long long *>(&s_tot), static_cast<unsigned long long>(wall));
        }
        __builtin_amdgcn_wave_barrier();
        if (m <= static_cast<uint32_t>(WST)) {
            uint32_t *out = stash + tile * P_STASH + wv * WST;
            for (uint32_t r = lane; r < nres; r += 64) {
                const uint32_t e = wres[r];
                const int t0 = static_cast<int>(e >> 24);
                const int d0 = static_cast<int>((e >> 16) & 0xffu);
                const uint32_t sb = sbase[t0];
                if (sb == 0xffffffffu) continue;  // found by look-up at placement instead
                const uint32_t rank = static_cast<uint32_t>(__popcll(mask[t0] & ((1ull << (d0 - 1)) - 1ull)));
                out[sb + rank] = (static_cast<uint32_t>(d0) << 16) | (e & 0xffffu);
            }
        } else if (lane == 0) {
            // this wave's stash overflowed: k_p_fix rescans the tile (listed
            // once, by the first wave to overflow; the flag is cleared after
            // the next tile's first barrier)
            if (atomicOr(&s_ovf, 1u) == 0u) {
                const unsigned long long k = atomicAdd(fix_n, 1ull);
                if (static_cast<int64_t>(k) < ntiles) fix_list[k] = static_cast<uint32_t>(tile);
            }
        }
        prev = tile;
    }
    __syncthreads();
    if (t == 0 && prev >= 0) {
        const uint64_t tot = s_tot;
        tile_tot[prev] = tot;
        atomicAdd(reinterpret_cast<unsigned long long *>(&sup_tot[prev / SUP]), static_cast<unsigned long long>(tot));
    }
}

// Placement of P edges for tiles whose stash held them; offsets for all.
// The tile's edges fill one contiguous range of slots: thread r takes slots
// r, r + PT, ..., finds the owning cell by binary search over the tile's
// exclusive scan, and copies the P edge from the stash (the cell's S slots
// are left to the S write pass), so the output is written coalesced.
template <typename T>
__global__ void __launch_bounds__(PT) k_p_place(const int64_t *d_n, int64_t ncap,
                                                const uint32_t *__restrict__ cntS, const uint32_t *__restrict__ cntP,
                                                const uint32_t *__restrict__ stash,
                                                const uint32_t *__restrict__ stash_n,
                                                const uint64_t *__restrict__ tile_tot,
                                                const uint64_t *__restrict__ sup_tot, bool raw_sup,
                                                int64_t *__restrict__ offsets, int64_t *__restrict__ offnext,
                                                uint32_t *__restrict__ uv, uint16_t *__restrict__ bit, int64_t cap,
                                                int64_t *__restrict__ d_nedges, int32_t *__restrict__ status) {
    __shared__ uint64_t tmp[4];
    __shared__ uint32_t sx[PT];   // tile-relative first slot of each cell
    __shared__ uint32_t ssb[PT];  // first stash entry of each cell
    __shared__ uint32_t scp[PT];  // P count (BIG flag kept)
    const int64_t n = load_n(d_n, ncap);
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * PT;
    if (base >= n) return;
    const int t = threadIdx.x;
    const int64_t i = base + t;
    const int tr = static_cast<int>(n - base < PT ? n - base : PT);
    uint32_t cp = 0, cs = 0;
    if (t < tr) {
        cp = cntP[i];
        cs = cntS[i];
    }
    const uint64_t t_off = tile_offset(tile, tile_tot, sup_tot, raw_sup, tmp);
    // each wave's 64 cells own one region of WST stash entries (k_p_find)
    bool ovf = false;
#pragma unroll
    for (int w = 0; w < PWAVES; ++w) ovf = ovf || stash_n[tile * PWAVES + w] > static_cast<uint32_t>(WST);
    const uint32_t c = cp & ~BIG;
    const uint32_t stashed = (cp & BIG) ? 0u : cp;
    uint64_t tot_all;
    const uint64_t exa = block256_excl_scan_u64(static_cast<uint64_t>(c) + cs, tmp, &tot_all);
    const uint32_t exs = (t >> 6) * WST + wave_incl_scan_u32(stashed) - stashed;
    const int64_t out0 = static_cast<int64_t>(t_off + exa);
    if (t == 0 && base + tr == n) {  // the last tile: |E|, offsets[n], status
        const int64_t tot = static_cast<int64_t>(t_off + tot_all);
        *d_nedges = tot;
        if (offsets) offsets[n] = tot;
        *status = tot > cap ? CG_ECAPACITY : CG_OK;
    }
    if (t < tr) {
        if (offsets) offsets[i] = out0;
        else if (cs || (cp & BIG)) offnext[i] = out0 + c + cs;
    }
    sx[t] = static_cast<uint32_t>(exa);
    ssb[t] = exs;
    scp[t] = t < tr ? cp : 0u;
    __syncthreads();
    if (ovf) return;  // k_p_fix writes this tile's scanned P edges
    const uint32_t *src = stash + tile * P_STASH;
    for (uint32_t r = t; r < static_cast<uint32_t>(tot_all); r += PT) {
        int lo = 0, hi = tr;  // last cell with sx <= r
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (sx[mid] <= r) lo = mid; else hi = mid;
        }
        const uint32_t k = r - sx[lo];
        const uint32_t cpl = scp[lo];
        if ((cpl & BIG) || k >= cpl) continue;  // looked-up cell, or an S slot
        const uint32_t e = src[ssb[lo] + k];
        const int64_t u = base + lo;
        emit(uv, bit, cap, static_cast<int64_t>(t_off) + r, static_cast<uint32_t>(u),
             static_cast<uint32_t>(u + (e >> 16)), static_cast<int>(e & 0xffffu));
    }
}

// Tiles whose P stash overflowed (listed by k_p_find): reload and write their
// scanned P edges.
template <typename T, int WT>
__global__ void __launch_bounds__(PT) k_p_fix(const T *__restrict__ cells, const int64_t *d_n, int64_t ncap,
                                              int words, int s, int gmax, const uint32_t *__restrict__ cntS,
                                              const uint32_t *__restrict__ cntP,
                                              const uint32_t *__restrict__ fix_list,
                                              const unsigned long long *__restrict__ fix_n,
                                              const uint64_t *__restrict__ tile_tot,
                                              const uint64_t *__restrict__ sup_tot, bool raw_sup,
                                              uint32_t *__restrict__ uv, uint16_t *__restrict__ bit, int64_t cap) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint64_t tmp[4];
    __shared__ int s_th;
    const int64_t n = load_n(d_n, ncap);
    const int64_t ntiles = (n + PT - 1) / PT;
    int64_t nfix = static_cast<int64_t>(*fix_n);
    if (nfix > ntiles) nfix = ntiles;
    using L = PTile<T, WT>;
    T *rows = reinterpret_cast<T *>(smem);
    uint32_t *pcs = reinterpret_cast<uint32_t *>(smem + L::rows_bytes);
    uint32_t *nbl = pcs + PROWS;
    uint8_t *heads = reinterpret_cast<uint8_t *>(nbl + PT * NB);
    const int t = threadIdx.x;
    for (int64_t k = blockIdx.x; k < nfix; k += gridDim.x) {
        const int64_t tile = fix_list[k];
        const int64_t base = tile * PT;
        int th;
        const int tr = load_ptile<T, WT>(rows, pcs, heads, &s_th, cells, words, s, base, n, &th);
        const int64_t i = base + t;
        uint32_t cp = 0, cs = 0;
        if (t < tr) {
            cp = cntP[i];
            cs = cntS[i];
        }
        uint64_t tot;
        const uint64_t exa = block256_excl_scan_u64(static_cast<uint64_t>(cp & ~BIG) + cs, tmp, &tot);
        const uint64_t t_off = tile_offset(tile, tile_tot, sup_tot, raw_sup, tmp);
        if (t < tr && !(cp & BIG) && cp != 0) {
            const int64_t out0 = static_cast<int64_t>(t_off + exa);
            p_scan_t<T, WT>(rows, pcs, heads, tr + th, t, i, base, n, cells, words, s, gmax,
                            [&](uint32_t d, int k, uint32_t r) {
                                emit(uv, bit, cap, out0 + r, static_cast<uint32_t>(i), static_cast<uint32_t>(i + d),
                                     k);
                            });
        }
        __syncthreads();  // LDS is reloaded for the next tile
    }
}

struct EdgesWs {
    uint32_t *cntP, *cntS;
    int64_t *offsets;
    uint64_t *tile_sums;
    uint64_t *tile_tot;
    uint64_t *sup_tot;
    int64_t nsup;
    uint32_t *p_stash, *p_stash_n;
    uint4 *s_stash;              // S edges per block of the suffix order
    uint32_t *s_stash_n;
    uint32_t *s_big, *p_big;     // cells left to k_big_lookup
    uint32_t *p_fix;             // tiles whose P stash overflowed
    unsigned long long *big_n;   // [0]: S list length, [1]: P list length, [2]: overflowed tiles,
                                 // [3]: entries of bst taken
    uint2 *bst;                  // listed cells' neighbours (v, k), count pass to write pass
    int64_t bst_cap;
    uint32_t *bstart;            // per listed cell: its first bst entry, or BST_NONE
};

// Padded row width (power of two) for the P tiles, or 0 when rows are too
// wide for them (u64: up to 16 words, u32: up to 32 words, i.e. l <= 1024).
int tile_width(const cg_dict &d) {
    const int cap = d.lay.word_bits == 64 ? 16 : 32;
    int wt = 1;
    while (wt < d.lay.words) wt <<= 1;
    return wt <= cap ? wt : 0;
}

bool fast_path_ok(const cg_dict &d) { return tile_width(d) > 0 && d.params.group_max < 65536; }

EdgesWs carve_edges(void *base, int64_t ncap, size_t *bytes) {
    Carver c(base);
    EdgesWs w{};
    const int64_t n = ncap > 0 ? ncap : 1;
    const int64_t tiles = (n + PT - 1) / PT;
    w.cntP = c.take<uint32_t>(n);
    w.cntS = c.take<uint32_t>(n);
    w.offsets = c.take<int64_t>(n + 1);
    w.tile_sums = c.take<uint64_t>(scan_tiles(n));
    w.tile_tot = c.take<uint64_t>(tiles);
    w.nsup = (tiles + SUP - 1) / SUP;
    w.sup_tot = c.take<uint64_t>(w.nsup);
    w.p_stash = c.take<uint32_t>(tiles * P_STASH);
    w.p_stash_n = c.take<uint32_t>(tiles * PWAVES);
    const int64_t sblocks = (n + SC - 1) / SC;
    w.s_stash = c.take<uint4>(sblocks * S_STASH);
    w.s_stash_n = c.take<uint32_t>(sblocks);
    w.s_big = c.take<uint32_t>(n);
    w.p_big = c.take<uint32_t>(n);
    w.p_fix = c.take<uint32_t>(tiles);
    w.big_n = c.take<unsigned long long>(4);
    w.bst_cap = n;
    w.bst = c.take<uint2>(w.bst_cap);
    w.bstart = c.take<uint32_t>(2 * n);
    *bytes = c.bytes();
    return w;
}

// Blocks of a persistent kernel: as many as fit on the device at once
// (a multiple of 8, one share per XCD), but no more than there are tiles.
unsigned persistent_blocks(const void *kernel, size_t lds, int64_t ntiles) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, PT, lds) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    int64_t g = static_cast<int64_t>(cus) * per_cu;
    const int64_t need = (ntiles + 7) / 8 * 8;
    if (g > need) g = need;
    g = g / 8 * 8;
    return static_cast<unsigned>(g < 8 ? 8 : g);
}

template <typename T, int WT>
cg_status p_pass_launch(const cg_dict &d, const EdgesWs &w, int64_t cap, int64_t *d_nedges, int64_t *d_offsets,
                        int64_t *offnext, uint32_t *uv, uint16_t *bit, int32_t *d_status, hipStream_t s) {
    const int64_t ncap = d.ncells_cap;
    const T *cells = static_cast<const T *>(d.cells);
    const int words = d.lay.words, ell = d.lay.ell, sp = d.params.split_bit, gmax = d.params.group_max;
    const int pb = d.params.dir_bits;
    const int64_t ntiles = (ncap + PT - 1) / PT;
    const dim3 grid(static_cast<unsigned>(ntiles));
    const dim3 sgrid(static_cast<unsigned>((ncap + SC - 1) / SC));
    const dim3 bgrid(blocks_for(ncap, 4, 256));  // one wave per listed cell
    const size_t lds = PTile<T, WT>::bytes;
    const size_t lds_find = PFind<T, WT>::bytes;
    const int rmax = gmax < SRMAX ? gmax : SRMAX;
    const int64_t *no_off = nullptr;
    if (sp > 0) {
        hipLaunchKernelGGL((k_s_scan<T, false>), sgrid, dim3(PT), 0, s, cells, d.sfx, d.d_ncells, ncap, words, sp,
                           rmax, w.cntS, no_off, no_off, uv, bit, cap, w.s_big, w.big_n, w.s_stash, w.s_stash_n);
        CG_LAUNCHED("edges_s_count");
    }
    if (words == WT) {
        const unsigned pblocks =
            persistent_blocks(reinterpret_cast<const void *>(&k_p_find<T, WT, true>), lds_find, ntiles);
        hipLaunchKernelGGL((k_p_find<T, WT, true>), dim3(pblocks), dim3(PT), lds_find, s, cells, d.d_ncells, ncap,
                           words, ell, sp, gmax, w.cntS, w.cntP, w.p_stash, w.p_stash_n, w.tile_tot, w.sup_tot,
                           w.p_big, w.big_n + 1, w.p_fix, w.big_n + 2);
    } else {
        const unsigned pblocks =
            persistent_blocks(reinterpret_cast<const void *>(&k_p_find<T, WT, false>), lds_find, ntiles);
        hipLaunchKernelGGL((k_p_find<T, WT, false>), dim3(pblocks), dim3(PT), lds_find, s, cells, d.d_ncells, ncap,
                           words, ell, sp, gmax, w.cntS, w.cntP, w.p_stash, w.p_stash_n, w.tile_tot, w.sup_tot,
                           w.p_big, w.big_n + 1, w.p_fix, w.big_n + 2);
    }
    CG_LAUNCHED("edges_p_find");
    // listed cells of both sides: their counts, added to their tile totals
    hipLaunchKernelGGL((k_big_lookup<T, false>), bgrid, dim3(256), 0, s, cells, d.dir, pb, words, ell, sp, w.s_big,
                       w.p_big, w.big_n, ncap, w.cntS, w.cntP, w.tile_tot, w.sup_tot, no_off, no_off, uv, bit, cap,
                       w.bst, w.big_n + 3, w.bst_cap, w.bstart);
    CG_LAUNCHED("edges_big_count");
    // up to SUP_INLINE super-tiles each placement block sums those before
    // its own; more are scanned first
    const bool raw_sup = w.nsup <= SUP_INLINE;
    if (!raw_sup) {
        hipLaunchKernelGGL(k_sup_scan, dim3(1), dim3(256), 0, s, w.sup_tot, w.nsup);
        CG_LAUNCHED("edges_sup_scan");
    }
    hipLaunchKernelGGL((k_p_place<T>), grid, dim3(PT), 0, s, d.d_ncells, ncap, w.cntS, w.cntP, w.p_stash,
                       w.p_stash_n, w.tile_tot, w.sup_tot, raw_sup, d_offsets, offnext, uv, bit, cap, d_nedges,
                       d_status);
    CG_LAUNCHED("edges_p_place");
    hipLaunchKernelGGL((k_big_lookup<T, true>), bgrid, dim3(256), 0, s, cells, d.dir, pb, words, ell, sp, w.s_big,
                       w.p_big, w.big_n, ncap, w.cntS, w.cntP, w.tile_tot, w.sup_tot, d_offsets, offnext, uv, bit,
                       cap, w.bst, w.big_n + 3, w.bst_cap, w.bstart);
    CG_LAUNCHED("edges_big_write");
    const int gm = gmax < PSCAN ? gmax : PSCAN;  // same scan limit as k_p_find
    hipLaunchKernelGGL((k_p_fix<T, WT>), dim3(blocks_for(ntiles, 1, 64)), dim3(PT), lds, s, cells, d.d_ncells, ncap,
                       words, sp, gm, w.cntS, w.cntP, w.p_fix, w.big_n + 2, w.tile_tot, w.sup_tot, raw_sup, uv, bit,
                       cap);
    CG_LAUNCHED("edges_p_fix");
    if (sp > 0) {
        hipLaunchKernelGGL((k_s_scan<T, true>), sgrid, dim3(PT), 0, s, cells, d.sfx, d.d_ncells, ncap, words, sp,
                           rmax, w.cntS, d_offsets, offnext, uv, bit, cap, w.s_big, w.big_n, w.s_stash, w.s_stash_n);
        CG_LAUNCHED("edges_s_write_place");
    }
    return CG_OK;
}

template <typename T>
cg_status edges_fast(const cg_dict &d, uint32_t *uv, uint16_t *bit, int64_t cap, int64_t *d_nedges,
                     int64_t *d_offsets, const EdgesWs &w, int32_t *d_status, hipStream_t s) {
    const int64_t ncap = d.ncells_cap;
    const int64_t ntiles = (ncap + PT - 1) / PT;
    int64_t *offnext = w.offsets;  // sparse next-offsets when the caller wants no offsets
    hipLaunchKernelGGL(k_edges_init, dim3(blocks_for(ncap, 256, 4096)), dim3(256), 0, s, w.cntS, ncap, d_nedges,
                       d_offsets, d_status, w.big_n, w.sup_tot, w.nsup);
    CG_LAUNCHED("edges_init");
    if (ncap == 0) return CG_OK;
    const dim3 grid(static_cast<unsigned>(ntiles));
    switch (tile_width(d)) {
    case 1: CG_TRY((p_pass_launch<T, 1>(d, w, cap, d_nedges, d_offsets, offnext, uv, bit, d_status, s))); break;
    case 2: CG_TRY((p_pass_launch<T, 2>(d, w, cap, d_nedges, d_offsets, offnext, uv, bit, d_status, s))); break;
    case 4: CG_TRY((p_pass_launch<T, 4>(d, w, cap, d_nedges, d_offsets, offnext, uv, bit, d_status, s))); break;
    case 8: CG_TRY((p_pass_launch<T, 8>(d, w, cap, d_nedges, d_offsets, offnext, uv, bit, d_status, s))); break;
    case 16: CG_TRY((p_pass_launch<T, 16>(d, w, cap, d_nedges, d_offsets, offnext, uv, bit, d_status, s))); break;
    default: CG_TRY((p_pass_launch<T, 32>(d, w, cap, d_nedges, d_offsets, offnext, uv, bit, d_status, s))); break;
    }
    return CG_OK;
}

template <typename T>
cg_status edges_generic(const cg_dict &d, uint32_t *uv, uint16_t *bit, int64_t cap, int64_t *d_nedges,
                        int64_t *d_offsets, const EdgesWs &w, int32_t *d_status, hipStream_t s) {
    int64_t *offsets = d_offsets ? d_offsets : w.offsets;
    const int64_t ncap = d.ncells_cap;
    const T *cells = static_cast<const T *>(d.cells);
    const int words = d.lay.words, ell = d.lay.ell, sp = d.params.split_bit, gmax = d.params.group_max;
    const unsigned grid = blocks_for(ncap, 256, 16384);

    if (ncap == 0) {
        CG_TRY(fill_i64(d_nedges, 0, 1, s));
        if (d_offsets) CG_TRY(fill_i64(d_offsets, 0, 1, s));
        hipLaunchKernelGGL(k_status, dim3(1), dim3(64), 0, s, d_nedges, cap, d_status);
        CG_LAUNCHED("edges_status");
        return CG_OK;
    }
    hipLaunchKernelGGL((k_p_pass<T, false>), dim3(grid), dim3(256), 0, s, cells, d.d_ncells, ncap, words, ell, sp,
                       gmax, w.cntP, static_cast<const int64_t *>(nullptr), uv, bit, cap);
    CG_LAUNCHED("edges_p_count");
    if (sp > 0) {
        hipLaunchKernelGGL((k_s_pass<T, false>), dim3(grid), dim3(256), 0, s, cells, d.sfx, d.d_ncells, ncap, words,
                           sp, gmax, w.cntS, static_cast<const uint32_t *>(nullptr),
                           static_cast<const int64_t *>(nullptr), uv, bit, cap);
        CG_LAUNCHED("edges_s_count");
    } else {
        CG_TRY(fill_u32(w.cntS, 0, ncap, s));
    }
    CG_TRY(scan_pair_to_i64(w.cntP, w.cntS, offsets, ncap, d.d_ncells, w.tile_sums, d_nedges, s));
    hipLaunchKernelGGL(k_status, dim3(1), dim3(64), 0, s, d_nedges, cap, d_status);
    CG_LAUNCHED("edges_status");
    hipLaunchKernelGGL((k_p_pass<T, true>), dim3(grid), dim3(256), 0, s, cells, d.d_ncells, ncap, words, ell, sp,
                       gmax, w.cntP, offsets, uv, bit, cap);
    CG_LAUNCHED("edges_p_write");
    if (sp > 0) {
        hipLaunchKernelGGL((k_s_pass<T, true>), dim3(grid), dim3(256), 0, s, cells, d.sfx, d.d_ncells, ncap, words,
                           sp, gmax, w.cntS, w.cntP, offsets, uv, bit, cap);
        CG_LAUNCHED("edges_s_write_place");
    }
    return CG_OK;
}

template <typename T>
cg_status edges_impl(const cg_dict &d, uint32_t *uv, uint16_t *bit, int64_t cap, int64_t *d_nedges,
                     int64_t *d_offsets, void *ws, int32_t *d_status, hipStream_t s) {
    size_t b;
    EdgesWs w = carve_edges(ws, d.ncells_cap, &b);
    if (fast_path_ok(d)) return edges_fast<T>(d, uv, bit, cap, d_nedges, d_offsets, w, d_status, s);
    return edges_generic<T>(d, uv, bit, cap, d_nedges, d_offsets, w, d_status, s);
}

}  // namespace

size_t edges_workspace_bytes(const cg_dict &d, int64_t cap) {
    (void)cap;
    size_t b;
    carve_edges(nullptr, d.ncells_cap, &b);
    return b;
}

cg_status run_edges(const cg_dict &d, uint32_t *uv, uint16_t *bit, int64_t cap, int64_t *d_nedges,
                    int64_t *d_offsets, void *ws, size_t ws_bytes, int32_t *d_status, hipStream_t s) {
    (void)ws_bytes;
    if (d.lay.word_bits == 64)
        return edges_impl<uint64_t>(d, uv, bit, cap, d_nedges, d_offsets, ws, d_status, s);
    return edges_impl<uint32_t>(d, uv, bit, cap, d_nedges, d_offsets, ws, d_status, s);
}

}  // namespace cg
