// Edges in O(n l) probes (Section 6: a construction of the cell graph in
// O(n l) time, the searching step done through an auxiliary structure).  The
// paper does not give that structure; here it is a hash table keyed by an
// additive hash of the whole vector,
//
//     H(x) = sum of r_k over the positions k with x(k) = 1   (mod 2^64),
//
// with r_k a fixed pseudo-random 64-bit weight per position.  Setting bit k
// of x adds r_k, so the key of x xor e_k (for x(k) = 0) is H(x) + r_k,
// obtained in O(1) from H(x): each cell takes l probes in all, one per flip,
// instead of one search per flip.  A probe that finds an equal key is
// checked against the row itself (different vectors may share a key), so the
// edges are exact and the output bytes are those of the other paths.
//
//   H1  H(x) for every cell (thread per cell, set bits one by one)
//   H2  insert (H, id) into an open-addressing table of at least 2n slots
//   H3  count pass: one wave per cell, lanes over positions (descending k);
//       a hit is a cell equal to x xor e_k; per-cell upward counts
//   H4  scan of the counts into offsets, |E| and status
//   H5  write pass: the same probes, hits written at offsets[u] + rank
//       (u's neighbours in ascending v are its flips in descending k)
#include "cg_internal.hpp"

namespace cg {

namespace {

constexpr uint32_t EMPTY_ID = 0xFFFFFFFFu;

// Weight of position k: the 64-bit finaliser of a counter (distinct,
// well-spread values; any fixed choice gives the same edges).
__device__ __forceinline__ uint64_t pos_weight(int k) {
    return fmix64(0x9e3779b97f4a7c15ull * static_cast<uint64_t>(k + 1) + 0x632be59bd9b4e019ull);
}

template <typename T>
__global__ void __launch_bounds__(256) k_hp_keys(const T *__restrict__ cells, const int64_t *d_n, int64_t ncap,
                                                 int words, uint64_t *__restrict__ keys) {
    constexpr int B = Bits<T>::B;
    const int64_t n = load_n(d_n, ncap);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const T *row = cells + i * words;
        uint64_t h = 0;
        for (int w = 0; w < words; ++w) {
            T x = row[w];
            while (x) {  // set bits, most significant first: position w B + leading zeros
                const int lz = clz_t<T>(x);
                h += pos_weight(w * B + lz);
                x &= ~(T(1) << (B - 1 - lz));
            }
        }
        keys[i] = h;
    }
}

__global__ void __launch_bounds__(256) k_hp_insert(const uint64_t *__restrict__ keys, const int64_t *d_n,
                                                   int64_t ncap, uint64_t mask, uint64_t *__restrict__ tkey,
                                                   uint32_t *__restrict__ tid) {
    const int64_t n = load_n(d_n, ncap);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const uint64_t h = keys[i];
        uint64_t slot = h & mask;
        // at most half the slots are taken, so a free one is always found
        for (;;) {
            if (atomicCAS(&tid[slot], EMPTY_ID, static_cast<uint32_t>(i)) == EMPTY_ID) {
                tkey[slot] = h;
                break;
            }
            slot = (slot + 1) & mask;
        }
    }
}

// Cell id equal to (q xor e_k) with key qk, or -1: walk the probe run from
// the key's slot to the first free slot; equal keys are checked row by row.
template <typename T>
__device__ __forceinline__ int64_t hp_find(const T *cells, int words, const uint64_t *tkey, const uint32_t *tid,
                                           uint64_t mask, const T *q, int k, uint64_t qk) {
    const int kw = k / Bits<T>::B;
    const T km = bitmask_of<T>(k);
    uint64_t slot = qk & mask;
    for (;;) {
        const uint32_t id = tid[slot];
        if (id == EMPTY_ID) return -1;
        if (tkey[slot] == qk &&
            row_cmp_flip<T>(cells + static_cast<int64_t>(id) * words, q, words, kw, km) == 0)
            return id;
        slot = (slot + 1) & mask;
    }
}

// One wave per cell u (grid-stride over cells), lanes over positions k in
// descending chunks of 64; a hit at a flip with x(k) = 0 is an edge (u, v).
// WRITE = false: cnt[u] = number of hits; true: edges at offsets[u] + rank.
template <typename T, bool WRITE>
__global__ void __launch_bounds__(256) k_hp_probe(const T *__restrict__ cells, const int64_t *d_n, int64_t ncap,
                                                  int words, int ell, const uint64_t *__restrict__ keys,
                                                  const uint64_t *__restrict__ tkey, const uint32_t *__restrict__ tid,
                                                  uint64_t mask, uint32_t *__restrict__ cnt,
                                                  const int64_t *__restrict__ offsets, uint32_t *__restrict__ uv,
                                                  uint16_t *__restrict__ bit, int64_t cap) {
    const int64_t n = load_n(d_n, ncap);
    const int lane = threadIdx.x & 63;
    const int64_t nw = static_cast<int64_t>(gridDim.x) * (blockDim.x >> 6);
    for (int64_t u = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); u < n; u += nw) {
        const T *q = cells + u * words;
        const uint64_t h = keys[u];
        const int64_t base = WRITE ? offsets[u] : 0;
        uint32_t c = 0;
        for (int k0 = ell - 1; k0 >= 0; k0 -= 64) {
            const int k = k0 - lane;
            int64_t v = -1;
            if (k >= 0 && !get_bit<T>(q, k)) v = hp_find<T>(cells, words, tkey, tid, mask, q, k, h + pos_weight(k));
            const uint64_t m = ballot64(v >= 0);
            if (WRITE && v >= 0) {
                const int64_t pos = base + c + static_cast<int64_t>(__popcll(m & lanemask_lt()));
                if (pos < cap) {
                    uv[2 * pos] = static_cast<uint32_t>(u);
                    uv[2 * pos + 1] = static_cast<uint32_t>(v);
                    if (bit) bit[pos] = static_cast<uint16_t>(k);
                }
            }
            c += static_cast<uint32_t>(__popcll(m));
        }
        if (!WRITE && lane == 0) cnt[u] = c;
    }
}

__global__ void k_hp_status(const int64_t *total, int64_t cap, int32_t *status) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *status = (*total > cap) ? CG_ECAPACITY : CG_OK;
}

struct HashWs {
    uint64_t *keys;
    uint64_t *tkey;
    uint32_t *tid;
    uint32_t *cnt;
    int64_t *offsets;
    uint64_t *tile_sums;
    uint64_t slots;
};

uint64_t table_slots(int64_t ncap) {
    uint64_t s = 64;
    while (s < 2ull * static_cast<uint64_t>(ncap > 0 ? ncap : 1)) s <<= 1;
    return s;
}

HashWs carve_hash(void *base, const cg_dict &d, size_t *bytes) {
    Carver c(base);
    HashWs w{};
    const int64_t n = d.ncells_cap > 0 ? d.ncells_cap : 1;
    w.slots = table_slots(d.ncells_cap);
    w.keys = c.take<uint64_t>(n);
    w.tkey = c.take<uint64_t>(w.slots);
    w.tid = c.take<uint32_t>(w.slots);
    w.cnt = c.take<uint32_t>(n);
    w.offsets = c.take<int64_t>(n + 1);
    w.tile_sums = c.take<uint64_t>(scan_tiles(n));
    *bytes = c.bytes();
    return w;
}

template <typename T>
cg_status hash_impl(const cg_dict &d, uint32_t *uv, uint16_t *bit, int64_t cap, int64_t *d_nedges,
                    int64_t *d_offsets, void *ws, int32_t *d_status, hipStream_t s) {
    size_t b;
    HashWs w = carve_hash(ws, d, &b);
    const int64_t ncap = d.ncells_cap;
    const int words = d.lay.words, ell = d.lay.ell;
    const T *cells = static_cast<const T *>(d.cells);
    int64_t *offsets = d_offsets ? d_offsets : w.offsets;
    if (ncap == 0) {
        CG_TRY(fill_i64(d_nedges, 0, 1, s));
        CG_TRY(fill_i64(offsets, 0, 1, s));
        hipLaunchKernelGGL(k_hp_status, dim3(1), dim3(64), 0, s, d_nedges, cap, d_status);
        CG_LAUNCHED("hash_status");
        return CG_OK;
    }
    const uint64_t mask = w.slots - 1;
    CG_TRY(fill_u32(w.tid, EMPTY_ID, static_cast<int64_t>(w.slots), s));
    const dim3 g(blocks_for(ncap, 256, 16384));
    hipLaunchKernelGGL((k_hp_keys<T>), g, dim3(256), 0, s, cells, d.d_ncells, ncap, words, w.keys);
    CG_LAUNCHED("hash_keys");
    hipLaunchKernelGGL(k_hp_insert, g, dim3(256), 0, s, w.keys, d.d_ncells, ncap, mask, w.tkey, w.tid);
    CG_LAUNCHED("hash_insert");
    const dim3 wg(blocks_for(ncap, 4, 16384));  // one wave per cell
    hipLaunchKernelGGL((k_hp_probe<T, false>), wg, dim3(256), 0, s, cells, d.d_ncells, ncap, words, ell, w.keys,
                       w.tkey, w.tid, mask, w.cnt, static_cast<const int64_t *>(nullptr), uv, bit, cap);
    CG_LAUNCHED("hash_count");
    CG_TRY(scan_u32_to_i64(w.cnt, offsets, ncap, d.d_ncells, w.tile_sums, d_nedges, s));
    hipLaunchKernelGGL(k_hp_status, dim3(1), dim3(64), 0, s, d_nedges, cap, d_status);
    CG_LAUNCHED("hash_status");
    if (cap > 0) {
        hipLaunchKernelGGL((k_hp_probe<T, true>), wg, dim3(256), 0, s, cells, d.d_ncells, ncap, words, ell, w.keys,
                           w.tkey, w.tid, mask, w.cnt, offsets, uv, bit, cap);
        CG_LAUNCHED("hash_write");
    }
    return CG_OK;
}

}  // namespace

size_t hash_workspace_bytes(const cg_dict &d, int64_t cap) {
    (void)cap;
    size_t b;
    carve_hash(nullptr, d, &b);
    return b;
}

cg_status run_edges_hash(const cg_dict &d, uint32_t *uv, uint16_t *bit, int64_t cap, int64_t *d_nedges,
                         int64_t *d_offsets, void *ws, int32_t *d_status, hipStream_t s) {
    if (d.lay.word_bits == 64) return hash_impl<uint64_t>(d, uv, bit, cap, d_nedges, d_offsets, ws, d_status, s);
    return hash_impl<uint32_t>(d, uv, bit, cap, d_nedges, d_offsets, ws, d_status, s);
}

}  // namespace cg
