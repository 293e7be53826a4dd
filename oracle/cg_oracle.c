/*
 * CPU oracle for the cell-graph construction path of
 *   K. Kaczmarski, P. Rzazewski, A. Wolant,
 *   "Massively Parallel Construction of the Cell Graph" (arXiv:1503.06029).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package's smoke check
 * and the benchmark's CPU-baseline leg load this file's shared object.  The
 * HIP library never includes, links or calls it, and this file includes no
 * header of that library: the two implementations share nothing but the
 * seeded input generators.
 *
 * Plain, slow and meant to be checked by eye.  The method reaches exactly the
 * plain definitions below, so the oracle is those definitions written out:
 *
 *   - a vector x in [2]^l has bits x(0) .. x(l-1), zero-based (Section 1.1);
 *   - dist(x, y) = #{ i : x(i) != y(i) } (Section 1.1, Hamming distance);
 *   - the input is a multiset of such vectors (Section 2.2, last paragraphs);
 *     the cells are its distinct members, and the cell graph joins two cells
 *     iff their distance is 1 (Section 2.2, definition of G_X);
 *   - sorting and duplicate removal come first (Section 3.2, the radix-sort
 *     step); the order is lexicographic with x(0) most significant, the only
 *     order under which the sets vectors(C, v) of Section 3.2 are contiguous
 *     index ranges.
 *
 * Packed-row layout handled here (the library boundary's layout, restated
 * independently): a row is `words` machine words of `word_bits` bits
 * (32 or 64); bit i of the vector sits in word i / word_bits at bit position
 * word_bits - 1 - (i mod word_bits), so x(0) is the most significant bit of
 * word 0; positions >= l hold 0.
 *
 * Every count that can exceed 2^31 is an int64_t.  Parallel loops use
 * OpenMP over independent outer indices only; each output slot is computed
 * by one iteration, so results do not depend on the thread count.
 */
#define _GNU_SOURCE
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- */
/* Bit access on a packed row (Section 1.1: x(i), zero-based).             */
/* ---------------------------------------------------------------------- */

static int get_bit(const void *row, int word_bits, int64_t i)
{
    if (word_bits == 64) {
        const uint64_t *w = (const uint64_t *)row;
        return (int)((w[i / 64] >> (63 - (i % 64))) & 1u);
    } else {
        const uint32_t *w = (const uint32_t *)row;
        return (int)((w[i / 32] >> (31 - (i % 32))) & 1u);
    }
}

static const void *row_ptr(const void *base, int words, int word_bits, int64_t r)
{
    return (const char *)base + (size_t)r * (size_t)words * (size_t)(word_bits / 8);
}

int cgo_version(void) { return 1; }

int cgo_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads used by the parallel loops from now on (timing runs only; the
 * results do not depend on it). */
void cgo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------------- */
/* O1: bits -> packed words.                                               */
/* Section 2.1: bit i of v_P is 1 iff P satisfies constraint c_i; a byte   */
/* of the 0/1 sign matrix is taken as 1 iff it is nonzero.                 */
/* ---------------------------------------------------------------------- */

int cgo_pack(const uint8_t *bits, int64_t n, int64_t row_stride, int ell,
             int word_bits, int words, void *out)
{
    if (word_bits != 32 && word_bits != 64) return -1;
    if ((int64_t)words * word_bits < ell) return -1;
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        const uint8_t *src = bits + r * row_stride;
        for (int w = 0; w < words; ++w) {
            uint64_t acc = 0;
            for (int t = 0; t < word_bits; ++t) {
                int64_t i = (int64_t)w * word_bits + t;
                int b = (i < ell) ? (src[i] != 0) : 0;
                acc |= (uint64_t)b << (word_bits - 1 - t);
            }
            if (word_bits == 64)
                ((uint64_t *)out)[r * words + w] = acc;
            else
                ((uint32_t *)out)[r * words + w] = (uint32_t)acc;
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Lexicographic comparison, x(0) most significant, bit by bit.            */
/* ---------------------------------------------------------------------- */

struct cmp_ctx {
    const void *rows;
    int ell, word_bits, words;
};

static int lex_compare(const void *a, const void *b, int ell, int word_bits)
{
    for (int64_t i = 0; i < ell; ++i) {
        int x = get_bit(a, word_bits, i), y = get_bit(b, word_bits, i);
        if (x != y) return x < y ? -1 : 1;
    }
    return 0;
}

static int cmp_rows_by_index(const void *pa, const void *pb, void *vctx)
{
    const struct cmp_ctx *c = (const struct cmp_ctx *)vctx;
    int64_t ia = *(const int64_t *)pa, ib = *(const int64_t *)pb;
    int r = lex_compare(row_ptr(c->rows, c->words, c->word_bits, ia),
                        row_ptr(c->rows, c->words, c->word_bits, ib),
                        c->ell, c->word_bits);
    if (r) return r;
    return (ia > ib) - (ia < ib);
}

/* ---------------------------------------------------------------------- */
/* O2: multiset of rows -> sorted distinct cells + row_to_cell.            */
/* Section 2.2 (X may be a multiset; output only unique pairs) and         */
/* Section 3.2 (sort X, removing duplicates).  Cell id = rank in the       */
/* lexicographic order.  `cells` must hold n rows; returns the number of   */
/* cells, or -1 on bad arguments / allocation failure.                     */
/* ---------------------------------------------------------------------- */

int64_t cgo_dedup(const void *rows, int64_t n, int ell, int word_bits, int words,
                  void *cells, uint32_t *row_to_cell)
{
    if (word_bits != 32 && word_bits != 64) return -1;
    if (n == 0) return 0;
    int64_t *order = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!order) return -1;
    for (int64_t i = 0; i < n; ++i) order[i] = i;
    struct cmp_ctx ctx = { rows, ell, word_bits, words };
    qsort_r(order, (size_t)n, sizeof(int64_t), cmp_rows_by_index, &ctx);

    size_t rb = (size_t)words * (size_t)(word_bits / 8);
    int64_t nc = 0;
    for (int64_t j = 0; j < n; ++j) {
        const void *cur = row_ptr(rows, words, word_bits, order[j]);
        if (j == 0 || lex_compare(cur, row_ptr(rows, words, word_bits, order[j - 1]),
                                  ell, word_bits) != 0) {
            memcpy((char *)cells + (size_t)nc * rb, cur, rb);
            ++nc;
        }
        if (row_to_cell) row_to_cell[order[j]] = (uint32_t)(nc - 1);
    }
    free(order);
    return nc;
}

/* ---------------------------------------------------------------------- */
/* dist(x, y) (Section 1.1).  The count of differing bits is the popcount  */
/* of the XOR of the packed words: positions >= l are 0 in both rows.      */
/* Stops counting once `stop_at` is reached (0 = never).  *first_diff gets */
/* the smallest differing position, or -1.                                 */
/* ---------------------------------------------------------------------- */

static int64_t hamming(const void *a, const void *b, int word_bits, int words,
                       int64_t stop_at, int64_t *first_diff)
{
    int64_t d = 0;
    if (first_diff) *first_diff = -1;
    for (int w = 0; w < words; ++w) {
        uint64_t x;
        if (word_bits == 64)
            x = ((const uint64_t *)a)[w] ^ ((const uint64_t *)b)[w];
        else
            x = (uint64_t)(((const uint32_t *)a)[w] ^ ((const uint32_t *)b)[w]);
        if (!x) continue;
        if (first_diff && *first_diff < 0) {
            int lead = (word_bits == 64) ? __builtin_clzll(x)
                                         : __builtin_clz((uint32_t)x);
            *first_diff = (int64_t)w * word_bits + lead;
        }
        d += __builtin_popcountll(x);
        if (stop_at && d >= stop_at) return d;
    }
    return d;
}

int64_t cgo_dist(const void *a, const void *b, int word_bits, int words)
{
    return hamming(a, b, word_bits, words, 0, 0);
}

/* Bit-by-bit distance, straight from the definition; used by the tests to
 * pin the popcount form above. */
int64_t cgo_dist_bitwise(const void *a, const void *b, int ell, int word_bits)
{
    int64_t d = 0;
    for (int64_t i = 0; i < ell; ++i)
        d += get_bit(a, word_bits, i) != get_bit(b, word_bits, i);
    return d;
}

/* ---------------------------------------------------------------------- */
/* O3/O4: edges of the cell graph by comparing all pairs (Section 3.1,     */
/* the naive O(n^2 l) method; Section 2.2 definition of G_X).              */
/* Edges (u, v), u < v, dist = 1, in ascending (u, v) order; bit[e] is the */
/* differing position.  deg_up[u] = #{v > u adjacent to u}; offsets is the */
/* exclusive prefix sum of deg_up with offsets[n] = |E|.  At most `cap`    */
/* edges are written; the return value is |E| (or -1 on bad arguments).    */
/* Any of uv / bit / offsets / deg_up may be NULL.                         */
/* ---------------------------------------------------------------------- */

int64_t cgo_edges(const void *cells, int64_t nc, int word_bits, int words,
                  int64_t cap, uint32_t *uv, uint16_t *bit, int64_t *offsets,
                  uint32_t *deg_up)
{
    if (word_bits != 32 && word_bits != 64) return -1;
    uint32_t *deg = (uint32_t *)calloc((size_t)(nc > 0 ? nc : 1), sizeof(uint32_t));
    int64_t *off = (int64_t *)malloc((size_t)(nc + 1) * sizeof(int64_t));
    if (!deg || !off) { free(deg); free(off); return -1; }

    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t u = 0; u < nc; ++u) {
        const void *ru = row_ptr(cells, words, word_bits, u);
        uint32_t c = 0;
        for (int64_t v = u + 1; v < nc; ++v)
            if (hamming(ru, row_ptr(cells, words, word_bits, v), word_bits, words, 2, 0) == 1)
                ++c;
        deg[u] = c;
    }
    off[0] = 0;
    for (int64_t u = 0; u < nc; ++u) off[u + 1] = off[u] + deg[u];
    int64_t E = off[nc];

    if (uv || bit) {
        #pragma omp parallel for schedule(dynamic, 64)
        for (int64_t u = 0; u < nc; ++u) {
            if (!deg[u]) continue;
            const void *ru = row_ptr(cells, words, word_bits, u);
            int64_t pos = off[u];
            for (int64_t v = u + 1; v < nc && pos < off[u + 1]; ++v) {
                int64_t fd;
                if (hamming(ru, row_ptr(cells, words, word_bits, v), word_bits, words, 2, &fd) == 1) {
                    if (pos < cap) {
                        if (uv) { uv[2 * pos] = (uint32_t)u; uv[2 * pos + 1] = (uint32_t)v; }
                        if (bit) bit[pos] = (uint16_t)fd;
                    }
                    ++pos;
                }
            }
        }
    }
    if (offsets) memcpy(offsets, off, (size_t)(nc + 1) * sizeof(int64_t));
    if (deg_up && nc) memcpy(deg_up, deg, (size_t)nc * sizeof(uint32_t));
    free(deg);
    free(off);
    return E;
}

/* ---------------------------------------------------------------------- */
/* O3/O4 by the search of Section 3.2 (Algorithm 4): for every cell x and   */
/* every position k, the vector x' = x with bit k negated is looked up in   */
/* the dictionary of cells; (x, x') is an edge iff x' is a cell.  Only      */
/* positions with x(k) = 0 are searched, so x' > x and each edge is found   */
/* once, from its smaller end (the paper's loop would report it from both   */
/* ends).  The dictionary is the sorted cell array searched with the C      */
/* library's bsearch: the tree T of Section 3.2 is built over the same      */
/* lexicographic order, and a leaf's value (the cell id) is the rank found  */
/* here.  With the packed layout (x(0) = most significant bit of word 0),   */
/* comparing words as unsigned integers from word 0 up is that order.       */
/* Cells must be sorted and distinct (as cgo_dedup writes them).            */
/* For cell u, the found v ascend as k descends, so u's edges are written   */
/* in ascending (u, v).  Output arguments and return value as cgo_edges.    */
/* ---------------------------------------------------------------------- */

struct search_key {
    const void *row;
    int word_bits, words;
};

static int cmp_key_with_cell(const void *pk, const void *pcell)
{
    const struct search_key *k = (const struct search_key *)pk;
    for (int w = 0; w < k->words; ++w) {
        uint64_t a, b;
        if (k->word_bits == 64) {
            a = ((const uint64_t *)k->row)[w];
            b = ((const uint64_t *)pcell)[w];
        } else {
            a = ((const uint32_t *)k->row)[w];
            b = ((const uint32_t *)pcell)[w];
        }
        if (a != b) return a < b ? -1 : 1;
    }
    return 0;
}

/* Id of the cell equal to `row` with position k negated, or -1. */
static int64_t search_flip(const void *cells, int64_t nc, int word_bits, int words,
                           const void *row, int64_t k, void *tmp)
{
    size_t rb = (size_t)words * (size_t)(word_bits / 8);
    memcpy(tmp, row, rb);
    if (word_bits == 64)
        ((uint64_t *)tmp)[k / 64] ^= (uint64_t)1 << (63 - k % 64);
    else
        ((uint32_t *)tmp)[k / 32] ^= (uint32_t)1 << (31 - k % 32);
    struct search_key key = { tmp, word_bits, words };
    const char *hit = (const char *)bsearch(&key, cells, (size_t)nc, rb, cmp_key_with_cell);
    return hit ? (int64_t)((hit - (const char *)cells) / (ptrdiff_t)rb) : -1;
}

int64_t cgo_edges_search(const void *cells, int64_t nc, int ell, int word_bits, int words,
                         int64_t cap, uint32_t *uv, uint16_t *bit, int64_t *offsets,
                         uint32_t *deg_up)
{
    if (word_bits != 32 && word_bits != 64) return -1;
    if (ell < 1 || (int64_t)words * word_bits < ell) return -1;
    uint32_t *deg = (uint32_t *)calloc((size_t)(nc > 0 ? nc : 1), sizeof(uint32_t));
    int64_t *off = (int64_t *)malloc((size_t)(nc + 1) * sizeof(int64_t));
    if (!deg || !off) { free(deg); free(off); return -1; }
    size_t rb = (size_t)words * (size_t)(word_bits / 8);

    #pragma omp parallel
    {
        uint64_t tmp[(65536 + 63) / 64];
        #pragma omp for schedule(dynamic, 256)
        for (int64_t u = 0; u < nc; ++u) {
            const void *ru = row_ptr(cells, words, word_bits, u);
            uint32_t c = 0;
            for (int64_t k = ell - 1; k >= 0; --k)
                if (!get_bit(ru, word_bits, k) && search_flip(cells, nc, word_bits, words, ru, k, tmp) >= 0)
                    ++c;
            deg[u] = c;
        }
    }
    off[0] = 0;
    for (int64_t u = 0; u < nc; ++u) off[u + 1] = off[u] + deg[u];
    int64_t E = off[nc];

    if (uv || bit) {
        #pragma omp parallel
        {
            uint64_t tmp[(65536 + 63) / 64];
            #pragma omp for schedule(dynamic, 256)
            for (int64_t u = 0; u < nc; ++u) {
                if (!deg[u]) continue;
                const void *ru = row_ptr(cells, words, word_bits, u);
                int64_t pos = off[u];
                for (int64_t k = ell - 1; k >= 0 && pos < off[u + 1]; --k) {
                    if (get_bit(ru, word_bits, k)) continue;
                    int64_t v = search_flip(cells, nc, word_bits, words, ru, k, tmp);
                    if (v < 0) continue;
                    if (pos < cap) {
                        if (uv) { uv[2 * pos] = (uint32_t)u; uv[2 * pos + 1] = (uint32_t)v; }
                        if (bit) bit[pos] = (uint16_t)k;
                    }
                    ++pos;
                }
            }
        }
    }
    (void)rb;
    if (offsets) memcpy(offsets, off, (size_t)(nc + 1) * sizeof(int64_t));
    if (deg_up && nc) memcpy(deg_up, deg, (size_t)nc * sizeof(uint32_t));
    free(deg);
    free(off);
    return E;
}

/* ---------------------------------------------------------------------- */
/* All neighbors (both directions) of selected cells, by comparing each    */
/* selected cell with every cell (Section 2.2 definition).  For sampled    */
/* parity at sizes where the full pair scan is too slow.  For sample s,    */
/* out_count[s] = degree; the neighbor ids are written, ascending, to      */
/* out_ids[s * max_deg ...] (at most max_deg of them).                     */
/* ---------------------------------------------------------------------- */

int cgo_neighbors_of(const void *cells, int64_t nc, int word_bits, int words,
                     const int64_t *sample, int64_t ns, int max_deg,
                     uint32_t *out_count, uint32_t *out_ids)
{
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < ns; ++s) {
        int64_t u = sample[s];
        const void *ru = row_ptr(cells, words, word_bits, u);
        uint32_t c = 0;
        for (int64_t v = 0; v < nc; ++v) {
            if (v == u) continue;
            if (hamming(ru, row_ptr(cells, words, word_bits, v), word_bits, words, 2, 0) == 1) {
                if ((int)c < max_deg) out_ids[s * max_deg + c] = (uint32_t)v;
                ++c;
            }
        }
        out_count[s] = c;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* O5: distance-1 queries against the set of cells, for arbitrary query    */
/* vectors (Section 3.2, the search step: for every bit k, is x with bit   */
/* k negated a member?).  Written as a comparison with every cell:         */
/*   mask bit k set  <=>  some cell c has dist(q, c) = 1 and differs at k; */
/*   self = id of the cell equal to q, or 0xFFFFFFFF;                      */
/*   count = number of set mask bits.                                      */
/* mask uses the packed-row layout; any output may be NULL.                */
/* ---------------------------------------------------------------------- */

int cgo_d1_queries(const void *cells, int64_t nc, const void *queries, int64_t nq,
                   int word_bits, int words, uint32_t *count, uint32_t *self,
                   void *mask)
{
    size_t rb = (size_t)words * (size_t)(word_bits / 8);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < nq; ++q) {
        const void *rq = row_ptr(queries, words, word_bits, q);
        uint32_t c = 0, me = 0xFFFFFFFFu;
        char *mrow = mask ? (char *)mask + (size_t)q * rb : 0;
        if (mrow) memset(mrow, 0, rb);
        for (int64_t v = 0; v < nc; ++v) {
            int64_t fd;
            int64_t d = hamming(rq, row_ptr(cells, words, word_bits, v), word_bits, words, 2, &fd);
            if (d == 0) me = (uint32_t)v;
            else if (d == 1) {
                ++c;
                if (mrow) {
                    if (word_bits == 64)
                        ((uint64_t *)mrow)[fd / 64] |= (uint64_t)1 << (63 - fd % 64);
                    else
                        ((uint32_t *)mrow)[fd / 32] |= (uint32_t)1 << (31 - fd % 32);
                }
            }
        }
        if (count) count[q] = c;
        if (self) self[q] = me;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Algorithm 1 (ComputeDist): distances of every cell to each reference    */
/* vector, D[d * nc + j] = dist(ref_d, x_j), for the heuristic of          */
/* Section 3.1.                                                            */
/* ---------------------------------------------------------------------- */

int cgo_ref_dists(const void *cells, int64_t nc, const void *refs, int h,
                  int word_bits, int words, uint32_t *D)
{
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nc; ++j)
        for (int d = 0; d < h; ++d)
            D[(int64_t)d * nc + j] = (uint32_t)hamming(row_ptr(refs, words, word_bits, d),
                                                       row_ptr(cells, words, word_bits, j),
                                                       word_bits, words, 0, 0);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Algorithm 2 (ParallelHeuristic) over the distinct cells, sequential:    */
/* pairs are compared only when the triangle bound (*) of Section 1.1      */
/* allows distance 1 for every reference d, i.e.                           */
/* |dist(x_i, r_d) - dist(x_j, r_d)| = 1 (a distance-1 pair moves every    */
/* distance by exactly one; the printed filter has its inequality          */
/* reversed).  References are given cells; all pairs i < j are scanned,    */
/* including those involving a reference.  Output as cgo_edges.            */
/* ---------------------------------------------------------------------- */

int64_t cgo_edges_heuristic(const void *cells, int64_t nc, int word_bits, int words,
                            const int64_t *ref_ids, int h, int64_t cap,
                            uint32_t *uv, uint16_t *bit)
{
    uint32_t *D = (uint32_t *)malloc((size_t)(h > 0 ? h : 1) * (size_t)(nc > 0 ? nc : 1) * sizeof(uint32_t));
    if (!D) return -1;
    for (int d = 0; d < h; ++d)
        for (int64_t j = 0; j < nc; ++j)
            D[(int64_t)d * nc + j] = (uint32_t)hamming(row_ptr(cells, words, word_bits, ref_ids[d]),
                                                       row_ptr(cells, words, word_bits, j),
                                                       word_bits, words, 0, 0);
    int64_t E = 0;
    for (int64_t i = 0; i < nc; ++i) {
        for (int64_t j = i + 1; j < nc; ++j) {
            int ok = 1;
            for (int d = 0; d < h && ok; ++d) {
                int64_t a = D[(int64_t)d * nc + i], b = D[(int64_t)d * nc + j];
                if ((a > b ? a - b : b - a) != 1) ok = 0;
            }
            if (!ok) continue;
            int64_t fd;
            if (hamming(row_ptr(cells, words, word_bits, i), row_ptr(cells, words, word_bits, j),
                        word_bits, words, 2, &fd) == 1) {
                if (E < cap) {
                    if (uv) { uv[2 * E] = (uint32_t)i; uv[2 * E + 1] = (uint32_t)j; }
                    if (bit) bit[E] = (uint16_t)fd;
                }
                ++E;
            }
        }
    }
    free(D);
    return E;
}

/* ---------------------------------------------------------------------- */
/* Section 3.2: the 2^r-ary search tree T over sorted distinct cells,      */
/* built level by level as in Algorithm 3 (ConstructTree), with each node  */
/* held as the index range [first, last] of the cells below it.            */
/*                                                                         */
/* digit(x, i) = the r bits x(i*r) .. x(i*r + r - 1), read most            */
/* significant first (Figure 2: 001001 -> 0,2,1); bits past l read as 0.   */
/*                                                                         */
/* Level 0 is the root, covering all cells.  Level h (1 <= h <= depth)     */
/* holds one node per v-child created: for every node C on level h-1 and   */
/* every v in [2^r] whose set vectors(C, v) is non-empty.  depth =         */
/* ceil(l / r); the last level holds the leaves, one per cell, the value   */
/* of a leaf being its cell id.                                            */
/*                                                                         */
/* level_sizes[h] = number of nodes on level h, h = 0 .. depth.            */
/* If node_first / node_last / node_digit are non-NULL they receive, level */
/* after level, every node's range and the digit on the edge into it       */
/* (root digit = -1); they must hold sum(level_sizes) entries.  Returns    */
/* the total number of nodes, or -1.                                       */
/* ---------------------------------------------------------------------- */

static int digit_of(const void *row, int word_bits, int ell, int r, int64_t i)
{
    int v = 0;
    for (int t = 0; t < r; ++t) {
        int64_t pos = i * r + t;
        int b = pos < ell ? get_bit(row, word_bits, pos) : 0;
        v = (v << 1) | b;
    }
    return v;
}

int64_t cgo_tree_levels(const void *cells, int64_t nc, int ell, int word_bits, int words,
                        int r, int64_t *level_sizes, int64_t *node_first,
                        int64_t *node_last, int32_t *node_digit)
{
    if (r < 1 || r > 16) return -1;
    int depth = (ell + r - 1) / r;
    /* current level's ranges */
    int64_t *cf = (int64_t *)malloc((size_t)(nc + 1) * sizeof(int64_t));
    int64_t *cl = (int64_t *)malloc((size_t)(nc + 1) * sizeof(int64_t));
    int64_t *nf = (int64_t *)malloc((size_t)(nc + 1) * sizeof(int64_t));
    int64_t *nl = (int64_t *)malloc((size_t)(nc + 1) * sizeof(int64_t));
    int32_t *nd = (int32_t *)malloc((size_t)(nc + 1) * sizeof(int32_t));
    if (!cf || !cl || !nf || !nl || !nd) { free(cf); free(cl); free(nf); free(nl); free(nd); return -1; }

    int64_t total = 0, cur = 0;
    if (nc > 0) { cf[0] = 0; cl[0] = nc - 1; cur = 1; }
    level_sizes[0] = cur;
    if (node_first && cur) { node_first[0] = 0; node_last[0] = nc - 1; node_digit[0] = -1; }
    total = cur;

    for (int h = 1; h <= depth; ++h) {
        int64_t nxt = 0;
        /* vectors(C, v) for every node C of level h-1: the sub-range of C
         * whose digit h-1 equals v; it is contiguous because the cells are
         * sorted.  A child exists iff that range is non-empty. */
        for (int64_t c = 0; c < cur; ++c) {
            int64_t a = cf[c];
            while (a <= cl[c]) {
                int v = digit_of(row_ptr(cells, words, word_bits, a), word_bits, ell, r, h - 1);
                int64_t b = a;
                while (b + 1 <= cl[c] &&
                       digit_of(row_ptr(cells, words, word_bits, b + 1), word_bits, ell, r, h - 1) == v)
                    ++b;
                nf[nxt] = a; nl[nxt] = b; nd[nxt] = v; ++nxt;
                a = b + 1;
            }
        }
        level_sizes[h] = nxt;
        if (node_first) {
            memcpy(node_first + total, nf, (size_t)nxt * sizeof(int64_t));
            memcpy(node_last + total, nl, (size_t)nxt * sizeof(int64_t));
            memcpy(node_digit + total, nd, (size_t)nxt * sizeof(int32_t));
        }
        total += nxt;
        memcpy(cf, nf, (size_t)nxt * sizeof(int64_t));
        memcpy(cl, nl, (size_t)nxt * sizeof(int64_t));
        cur = nxt;
    }
    free(cf); free(cl); free(nf); free(nl); free(nd);
    return total;
}

/* Digits of one packed row (for the Figure 2 table). */
int cgo_digits(const void *row, int ell, int word_bits, int r, int32_t *out)
{
    int depth = (ell + r - 1) / r;
    for (int i = 0; i < depth; ++i) out[i] = digit_of(row, word_bits, ell, r, i);
    return depth;
}

/* ---------------------------------------------------------------------- */
/* O6: search on the cell graph.  Section 2.1: once the cells and their    */
/* neighbours are known, a graph algorithm finds the route; Section 6: a   */
/* path in the cell graph is an approximate solution of the motion-        */
/* planning problem.                                                       */
/*                                                                         */
/* cgo_adjacency: the undirected graph of the edge list uv[0..E) (pairs of */
/* cell ids < n) as adjacency lists: cell u's neighbours are              */
/* adj[adj_off[u] .. adj_off[u+1]), ascending.  Degrees are counted, each  */
/* edge is placed in both lists, and each list is sorted.  Returns 0, or   */
/* -1 on bad arguments.                                                    */
/* ---------------------------------------------------------------------- */
static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

int cgo_adjacency(int64_t n, int64_t E, const uint32_t *uv, int64_t *adj_off, uint32_t *adj)
{
    if (n < 0 || E < 0 || !adj_off || (E > 0 && (!uv || !adj))) return -1;
    for (int64_t u = 0; u <= n; ++u) adj_off[u] = 0;
    for (int64_t e = 0; e < E; ++e) {
        if (uv[2 * e] >= (uint64_t)n || uv[2 * e + 1] >= (uint64_t)n) return -1;
        adj_off[uv[2 * e] + 1] += 1;
        adj_off[uv[2 * e + 1] + 1] += 1;
    }
    for (int64_t u = 0; u < n; ++u) adj_off[u + 1] += adj_off[u];
    int64_t *fill = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!fill) return -1;
    for (int64_t u = 0; u < n; ++u) fill[u] = adj_off[u];
    for (int64_t e = 0; e < E; ++e) {
        uint32_t a = uv[2 * e], b = uv[2 * e + 1];
        adj[fill[a]++] = b;
        adj[fill[b]++] = a;
    }
    for (int64_t u = 0; u < n; ++u)
        qsort(adj + adj_off[u], (size_t)(adj_off[u + 1] - adj_off[u]), sizeof(uint32_t), cmp_u32);
    free(fill);
    return 0;
}

/* cgo_bfs: breadth-first search from `source` over such lists.            */
/* dist[v] = the fewest edges on a path from the source to v, or           */
/* 0xFFFFFFFF if there is none (a FIFO queue visits the cells in order of  */
/* distance).  parent[v] = the smallest neighbour w of v with              */
/* dist[w] = dist[v] - 1 (the source is its own parent; unreached cells    */
/* get 0xFFFFFFFF), chosen after the search from that definition.         */
/* Returns the largest distance, or -1 on bad arguments.                   */
int64_t cgo_bfs(int64_t n, const int64_t *adj_off, const uint32_t *adj, uint32_t source, uint32_t *dist,
                uint32_t *parent)
{
    const uint32_t NONE = 0xFFFFFFFFu;
    if (n <= 0 || (int64_t)source >= n || !adj_off || !dist) return -1;
    uint32_t *queue = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    if (!queue) return -1;
    for (int64_t v = 0; v < n; ++v) dist[v] = NONE;
    int64_t head = 0, tail = 0, far = 0;
    dist[source] = 0;
    queue[tail++] = source;
    while (head < tail) {
        uint32_t u = queue[head++];
        if ((int64_t)dist[u] > far) far = dist[u];
        for (int64_t j = adj_off[u]; j < adj_off[u + 1]; ++j) {
            uint32_t v = adj[j];
            if (dist[v] == NONE) {
                dist[v] = dist[u] + 1;
                queue[tail++] = v;
            }
        }
    }
    free(queue);
    if (parent) {
        for (int64_t v = 0; v < n; ++v) {
            parent[v] = NONE;
            if (dist[v] == NONE) continue;
            if (v == (int64_t)source) { parent[v] = source; continue; }
            for (int64_t j = adj_off[v]; j < adj_off[v + 1]; ++j) {
                uint32_t w = adj[j];
                if (dist[w] + 1 == dist[v] && (parent[v] == NONE || w < parent[v])) parent[v] = w;
            }
        }
    }
    return far;
}

/* ---------------------------------------------------------------------- */
/* O7: sampled points -> sign vectors (Section 2.1: bit i of v_P is 1 iff  */
/* the point P satisfies constraint c_i; the paper samples the             */
/* configuration space, Section 2.1 and Section 5).  Constraints are       */
/* half-spaces a_i . p >= c_i of R^3; points are uniform in a box.        */
/*                                                                         */
/* Random numbers: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel */
/* random numbers: as easy as 1, 2, 3", SC 2011), written here from its    */
/* definition: ten rounds, each multiplying words 0 and 2 by the two round */
/* constants into 128-bit products and recombining the halves with words   */
/* 1 and 3 and the key, the key advancing by the two Weyl constants        */
/* between rounds.                                                         */
/* Float contract (every operation rounded to nearest float64, no fused    */
/* multiply-add -- this file is compiled with -ffp-contract=off):          */
/*   x = philox(counter = (i, 0, 0, 0), key = (seed, scene));              */
/*   u_j = (x_j >> 11) * 2^-53;  p_j = lo_j + (hi_j - lo_j) * u_j;          */
/*   r_i = ((a_i0 * p0 + a_i1 * p1) + a_i2 * p2) - c_i;  bit i = r_i >= 0.  */
/* ---------------------------------------------------------------------- */
void cgo_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        unsigned __int128 p0 = (unsigned __int128)M0 * c0, p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Point i of stream (seed, scene) in the box lohi = (lo0, lo1, lo2, hi0,  */
/* hi1, hi2). */
void cgo_sample_point(int64_t i, uint64_t seed, uint64_t scene, const double lohi[6], double p[3])
{
    uint64_t ctr[4] = {(uint64_t)i, 0, 0, 0}, key[2] = {seed, scene}, x[4];
    cgo_philox4x64(ctr, key, x);
    for (int j = 0; j < 3; ++j) {
        double u = (double)(x[j] >> 11) * 0x1.0p-53;
        double d = lohi[3 + j] - lohi[j];
        double m = d * u;
        p[j] = lohi[j] + m;
    }
}

/* Sign bytes (n x ell, row-major) of n sampled points against ell planes  */
/* given as (a0, a1, a2, c) rows.  Returns 0, or -1 on bad arguments.      */
int cgo_sample_signs(const double *planes, int ell, int64_t n, uint64_t seed, uint64_t scene,
                     const double lohi[6], uint8_t *bits)
{
    if (ell < 1 || n < 0 || !planes || !lohi || (n > 0 && !bits)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double p[3];
        cgo_sample_point(i, seed, scene, lohi, p);
        for (int k = 0; k < ell; ++k) {
            const double *a = planes + 4 * (int64_t)k;
            double t0 = a[0] * p[0], t1 = a[1] * p[1], t2 = a[2] * p[2];
            double s = t0 + t1;
            s = s + t2;
            double r = s - a[3];
            bits[i * ell + k] = r >= 0.0 ? 1 : 0;
        }
    }
    return 0;
}
