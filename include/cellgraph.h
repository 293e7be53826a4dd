/*
 * cellgraph.h -- C ABI of the MI355X (gfx950) cell-graph construction library.
 *
 * The library builds the cell graph of Kaczmarski, Rzazewski and Wolant,
 * "Massively Parallel Construction of the Cell Graph" (arXiv:1503.06029):
 * given a multiset X of binary vectors of length l (one constraint-sign
 * vector per sampled point, Section 2.1), it deduplicates X into cells and
 * emits every pair of cells at Hamming distance 1 (the graph G_X of
 * Section 2.2).  The path is: pack (sign bytes -> words), dedup (radix sort
 * + unique, Section 3.2), dictionary build (sorted keys + prefix directory
 * + suffix-grouped order), distance-1 queries (Section 3.2, Algorithm 4's
 * flip-and-look-up), and edge emission (prefix sum + compaction).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every d_* pointer is a DEVICE pointer owned by the caller.  The library
 *   never allocates or frees device memory; scratch space is passed in as a
 *   workspace whose size the matching *_workspace / *_size call reports.
 * - `stream` is a hipStream_t (NULL = the default stream).  Calls only
 *   enqueue work on it and return; none synchronises with the host.  Values
 *   that depend on the data (cell count, edge count, overflow) are written to
 *   device scalars.
 * - Synchronous return codes report argument validation and launch
 *   failures only.  On any error nothing is enqueued after the failing
 *   launch; cg_last_error() gives the text (per host thread).
 * - No global mutable device state: concurrent calls on different streams
 *   with disjoint buffers are safe.
 *
 * Packed-row layout (cg_layout)
 * -----------------------------
 * A vector x(0) .. x(l-1) (zero-based, Section 1.1) is stored as `words`
 * unsigned machine words of `word_bits` bits (32 or 64), words = ceil(l /
 * word_bits).  Bit i sits in word i / word_bits at bit position
 * word_bits - 1 - (i mod word_bits): x(0) is the most significant bit of
 * word 0.  Positions >= l must be 0 (cg_pack guarantees it; other producers
 * must too).  Rows are contiguous, row r starting at word r * words.
 * With this layout, comparing rows word by word as unsigned integers from
 * word 0 is the lexicographic order with x(0) most significant, which is
 * the order of the sorted cells and of the sets vectors(C, v) of Section 3.2.
 *
 * Output order
 * ------------
 * Cells are the distinct input rows in ascending lexicographic order; a
 * cell's id is its rank.  Edges are the pairs (u, v), u < v, of cells at
 * distance 1, in ascending (u, v) order; bit[e] is the one position where
 * they differ (cell u has 0 there, cell v has 1).  The output is unique: the
 * same input gives the same bytes whatever the parameters.
 */
#ifndef CELLGRAPH_H
#define CELLGRAPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *cg_stream_t; /* same type as hipStream_t */

typedef int32_t cg_status;
#define CG_OK            0
#define CG_EINVAL       -1  /* bad argument: null pointer, bad layout, size out of range */
#define CG_EWORKSPACE   -2  /* workspace / dictionary memory smaller than reported size   */
#define CG_ECAPACITY    -3  /* (device status only) more edges than the output capacity  */
#define CG_EHIP         -4  /* HIP launch or runtime error; see cg_last_error()           */
#define CG_EUNSUPPORTED -5  /* valid request the library does not implement             */

typedef struct cg_layout {
    int32_t ell;       /* vector length l, 1 <= l <= 65535                    */
    int32_t word_bits; /* 32 or 64                                             */
    int32_t words;     /* ceil(ell / word_bits)                                */
} cg_layout;

/* Library version, (major << 16) | minor. */
int32_t cg_version(void);

/* Static text for a status code. */
const char *cg_status_string(cg_status st);

/* Copies the calling thread's last error text (NUL-terminated, truncated to
 * len) into buf; returns the status that produced it (CG_OK if none). */
cg_status cg_last_error(char *buf, size_t len);

/* Fills *lay for a vector length and word size; CG_EINVAL if out of range. */
cg_status cg_make_layout(int32_t ell, int32_t word_bits, cg_layout *lay);

/* ------------------------------------------------------------------ pack
 * Section 2.1: bit i of a point's vector is 1 iff the point satisfies
 * constraint c_i.  Packs an n x l byte matrix (row r at d_bits + r *
 * row_stride, byte != 0 means 1) into n packed rows (layout above), writing
 * n * lay.words words to d_packed and zeroing positions >= l.
 * Errors: CG_EINVAL if n < 0, row_stride < l, or a required pointer is NULL
 * while n > 0.  d_bits and d_packed must not overlap.                       */
cg_status cg_pack(const uint8_t *d_bits, int64_t n, int64_t row_stride,
                  cg_layout lay, void *d_packed, cg_stream_t stream);

/* ----------------------------------------------------------------- dedup
 * Section 2.2 (X may be a multiset; only unique pairs are wanted) and
 * Section 3.2 (sort X by radix sort, removing duplicates).  Sorts the n
 * packed rows lexicographically and removes duplicates:
 *   d_cells      (capacity n rows) <- the distinct rows, ascending;
 *   d_row_to_cell (nullable, n)    <- id of the cell equal to each row;
 *   *d_ncells    (device int64)    <- number of cells.
 * The input is not modified and must not overlap the outputs.  Requires
 * n < 2^32.  Workspace: cg_dedup_workspace(n, lay) bytes, any alignment >= 256.
 * Errors: CG_EINVAL (bad layout, n out of range, NULL pointers),
 * CG_EWORKSPACE (ws_bytes too small).                                       */
cg_status cg_dedup_workspace(int64_t n, cg_layout lay, size_t *bytes);
cg_status cg_dedup(const void *d_packed, int64_t n, cg_layout lay, void *d_cells,
                   uint32_t *d_row_to_cell, int64_t *d_ncells, void *d_ws,
                   size_t ws_bytes, cg_stream_t stream);

/* ------------------------------------------------------------ dictionary
 * A device dictionary over the sorted distinct cells (Section 3.2: the
 * sorted set makes every vectors(C, v) a contiguous index range; the paper's
 * tree stores its values, the cell ids, in the leaves).  The library keeps:
 *   - the sorted cells themselves (borrowed, not copied);
 *   - a directory over the first p bits: dir[g] = first cell whose first p
 *     bits are >= g, for g = 0 .. 2^p (the top levels of a 2^p-ary tree of
 *     Section 3.2, held as ranges);
 *   - a suffix-grouped order: the cell ids sorted by a 32-bit hash of bits
 *     s .. l-1, so cells that agree on all bits past s sit together (built
 *     only for the flip-and-look-up edge path with s > 0, the one reader).
 * A distance-1 pair that differs at bit k >= s shares its first s bits and
 * is adjacent in the sorted order; one that differs at k < s shares bits
 * s .. l-1 and is adjacent in the suffix-grouped order.                     */
#define CG_DICT_SORTED 0        /* sorted keys + prefix directory + suffix order */
#define CG_DICT_TREE 1          /* the same, plus Section 3.2's leaf-valued 2^r-ary
                                   tree held as index ranges (Algorithm 3: level h
                                   has one node per distinct h-digit prefix of r-bit
                                   digits); distance-1 queries descend it digit by
                                   digit (Algorithm 4); edges use the directory,
                                   whose ranges are the tree's top levels           */
#define CG_PATH_LOOKUP 0        /* edges by flip-and-look-up over the two orders */
#define CG_PATH_ALLPAIRS 1      /* edges by the (*)-filtered all-pairs scan       */
#define CG_PATH_HASH 2          /* edges in O(n l) probes of an additive-hash table
                                   (Section 6: the O(n l) construction); each flip
                                   updates the key in O(1), hits are checked row by
                                   row, so the output is the same                  */

typedef struct cg_dict_params {
    int32_t kind;       /* CG_DICT_SORTED or CG_DICT_TREE                         */
    int32_t dir_bits;   /* p, 0..24; -1 = automatic (about log2 of the capacity)  */
    int32_t split_bit;  /* s, 0..l; -1 = automatic                                */
    int32_t path;       /* CG_PATH_LOOKUP, _ALLPAIRS or _HASH (used by cg_edges)  */
    int32_t n_refs;     /* h, 0..8: reference vectors of the all-pairs path       */
    int32_t group_max;  /* groups larger than this are searched, not scanned;
                           1..1024, -1 = automatic                                */
    int32_t key_bits;   /* sort-key width of cg_dedup_dict when l > 64: 32, 64 or
                           96 bits of each row; 0 = automatic (for 2^20 rows
                           or more a sample of rows decides between 32 and 64
                           on the device, else 64).  Rows sharing the key are
                           ordered by full-row comparison either way, so only
                           speed changes                                    */
    int32_t fanout_bits; /* r, bits per digit of the CG_DICT_TREE tree (fan-out
                           2^r): 1..8, 0 = 2 (the paper's Figure 2); must be 0
                           for CG_DICT_SORTED                               */
} cg_dict_params;

/* The automatic parameters (all -1, kind/path 0, n_refs 4). */
cg_status cg_dict_params_default(cg_dict_params *p);

/* One entry of an autotuner table: the parameters measured fastest for
 * rows of `words` words and about 2^log2_rows rows. */
typedef struct cg_tune_entry {
    int32_t words;
    int32_t log2_rows;
    cg_dict_params params;
} cg_tune_entry;

/* Parameters from an autotuner table (read only; the caller owns it): the
 * entry with lay.words words whose log2_rows is nearest to log2(ncells_cap)
 * (ties: the smaller), or the automatic parameters when no entry has these
 * words.  Every choice gives the same output bytes; the table only decides
 * speed.  Errors: CG_EINVAL (NULL out, NULL table with n_entries > 0,
 * n_entries < 0, an entry whose parameters cg_dict_size would reject). */
cg_status cg_dict_params_tuned(const cg_tune_entry *table, int32_t n_entries, int64_t ncells_cap, cg_layout lay,
                               cg_dict_params *out);

/* Host-side handle of device pointers.  It BORROWS d_cells, d_ncells and
 * d_mem, which must outlive it; it needs no destroy call.  Fields are
 * filled by cg_dict_build (parameters with their automatic values resolved)
 * and are read-only for the caller. */
typedef struct cg_dict {
    uint32_t magic;
    cg_layout lay;
    cg_dict_params params;      /* resolved */
    int64_t ncells_cap;
    const void *cells;          /* ncells_cap rows, first *d_ncells valid   */
    const int64_t *d_ncells;
    uint32_t *dir;              /* 2^dir_bits + 1 entries                    */
    uint64_t *sfx;              /* ncells_cap entries: (hash << 32) | id      */
    void *mem;
    size_t mem_bytes;
    /* CG_DICT_TREE only (else NULL), depth = ceil(l / r) levels below the root: */
    uint16_t *tree_depth;       /* ncells_cap entries: for cell i >= 1, the deepest
                                   level whose node holds both cell i - 1 and cell
                                   i (their common leading bits / r); cell i starts
                                   a node at every level below it                */
    uint32_t *tree_levels;      /* depth + 1 entries: nodes per level, level 0 the
                                   root (Algorithm 3's level sizes)              */
} cg_dict;

/* Bytes of dictionary memory for up to ncells_cap cells. */
cg_status cg_dict_size(int64_t ncells_cap, cg_layout lay, const cg_dict_params *p,
                       size_t *bytes);

/* Builds the dictionary over d_cells[0 .. *d_ncells), which must be sorted
 * and distinct (as written by cg_dedup; not checked).  p may be NULL for the
 * defaults.  Errors: CG_EINVAL, CG_EWORKSPACE, CG_EUNSUPPORTED (kind). */
cg_status cg_dict_build(const void *d_cells, const int64_t *d_ncells, int64_t ncells_cap,
                        cg_layout lay, const cg_dict_params *p, void *d_mem,
                        size_t mem_bytes, cg_dict *out, cg_stream_t stream);

/* Fused dedup + dictionary build: the same cells, row_to_cell, cell count
 * and dictionary as cg_dedup followed by cg_dict_build(d_cells, d_ncells,
 * n, lay, p, ...), in fewer passes over the rows: suffix hashes are taken
 * while the sort keys are extracted and the directory comes from the sorted
 * keys, so the cells are not read back.  Arguments as for the two calls
 * (the dictionary's ncells_cap is n; d_mem needs cg_dict_size(n, lay, p));
 * the workspace needs cg_dedup_dict_workspace(n, lay) bytes.  *out is a
 * dictionary handle exactly like cg_dict_build's.
 * Errors: CG_EINVAL, CG_EWORKSPACE. */
cg_status cg_dedup_dict_workspace(int64_t n, cg_layout lay, size_t *bytes);
cg_status cg_dedup_dict(const void *d_packed, int64_t n, cg_layout lay, void *d_cells, uint32_t *d_row_to_cell,
                        int64_t *d_ncells, void *d_ws, size_t ws_bytes, const cg_dict_params *p, void *d_mem,
                        size_t mem_bytes, cg_dict *out, cg_stream_t stream);

/* ----------------------------------------------------- distance-1 queries
 * Section 3.2 (Algorithm 4): for every query vector q and every bit k, is
 * q with bit k negated a cell?  For each of the nq rows at d_queries (same
 * layout as the dictionary):
 *   d_mask  (nullable, nq rows)  <- bit k set iff q xor e_k is a cell;
 *   d_count (nullable, nq)       <- number of set mask bits;
 *   d_self  (nullable, nq)       <- id of the cell equal to q, or 0xFFFFFFFF.
 * Errors: CG_EINVAL (bad dictionary handle, nq < 0, NULL queries with nq > 0). */
cg_status cg_neighbors_d1(const cg_dict *dict, const void *d_queries, int64_t nq,
                          uint32_t *d_count, uint32_t *d_self, void *d_mask,
                          cg_stream_t stream);

/* ------------------------------------------------------------------ edges
 * Section 2.2 (edges of G_X) over the dictionary's own cells, emitted in
 * ascending (u, v) order by a prefix sum over the per-cell counts of upward
 * neighbours (u < v):
 *   d_uv      (cap x 2 uint32)    <- (u, v) pairs;
 *   d_bit     (nullable, cap)     <- differing position of each pair;
 *   *d_nedges (device int64)      <- |E|, always exact;
 *   d_offsets (nullable, ncells_cap + 1 int64) <- offsets[u] = index of u's
 *              first edge, offsets[*d_ncells] = |E|;
 *   *d_status (device int32)      <- CG_OK, or CG_ECAPACITY if |E| > cap, in
 *              which case nothing is written at or past index cap, the
 *              contents below cap are unspecified, and the caller re-calls
 *              with cap >= *d_nedges and the same dictionary.
 * The dictionary's path parameter picks the method (flip-and-look-up, the
 * (*)-filtered all-pairs scan of Section 3.1, or the O(n l) hash probes of
 * Section 6); the output bytes are the same.
 * Workspace: cg_edges_workspace(dict, cap) bytes.
 * Errors: CG_EINVAL, CG_EWORKSPACE.                                         */
cg_status cg_edges_workspace(const cg_dict *dict, int64_t cap, size_t *bytes);
/* The same size before any dictionary exists (for planning device memory):
 * the workspace cg_edges will need for a dictionary of up to ncells_cap cells
 * in layout lay built with parameters p (NULL = defaults).
 * Errors: CG_EINVAL, CG_EUNSUPPORTED (as cg_dict_size). */
cg_status cg_edges_workspace_size(int64_t ncells_cap, cg_layout lay, const cg_dict_params *p, int64_t cap,
                                  size_t *bytes);
cg_status cg_edges(const cg_dict *dict, uint32_t *d_uv, uint16_t *d_bit, int64_t cap,
                   int64_t *d_nedges, int64_t *d_offsets, void *d_ws, size_t ws_bytes,
                   int32_t *d_status, cg_stream_t stream);

/* ------------------------------------------------- edges, no allocation
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that forbid
 * it): cg_edges with the same arguments and output bytes, minus the
 * workspace.  The scratch lives in a static device array of
 * CG_NOALLOC_SCRATCH_BYTES per GPU, held from the first call on that GPU
 * until the process ends (64 MiB: the edge passes of about one million
 * cells; cg_edges_workspace(dict, cap) reports what a call needs).  Nothing
 * is allocated or freed.  Every call on a GPU shares that GPU's array, so
 * calls that overlap on one GPU (other streams, other host threads) race;
 * calls on one stream are ordered and safe.
 * Errors: as cg_edges; CG_EWORKSPACE when the call needs more scratch than
 * the array holds (use cg_edges with a workspace then); CG_EHIP if the
 * array's device address cannot be taken. */
#define CG_NOALLOC_SCRATCH_BYTES (64u << 20)
cg_status cg_edges_noalloc(const cg_dict *dict, uint32_t *d_uv, uint16_t *d_bit, int64_t cap,
                           int64_t *d_nedges, int64_t *d_offsets, int32_t *d_status,
                           cg_stream_t stream);

/* --------------------------------------------------------- batched scenes
 * Many independent scenes (each its own multiset of sign vectors, with its
 * own l, Section 2.2) in one pass.  The scenes of a batch are packed into one
 * virtual scene whose rows are 32-bit words: word 0 holds the scene number
 * twice ((j << 16) | j), so rows of different scenes differ in at least two
 * bits and are never neighbours; words 1.. hold the scene's vector (MSB
 * first, zero beyond its l).  cg_dedup / cg_dict_build / cg_edges then run
 * unchanged on the virtual scene: cells come out grouped by scene (word 0 is
 * most significant), each scene's cells in lexicographic order, and its
 * edges form a contiguous slice of the edge list.  cg_batch_split finds
 * those slices and rewrites ids and bit positions to scene-local values.
 * At most 65536 scenes per batch. */

/* Layout of the virtual scene for scenes of length at most ell_max: 32-bit
 * words, 1 + ceil(ell_max / 32) of them (l = 32 + 32 * that). */
cg_status cg_batch_layout(int32_t ell_max, cg_layout *lay);

/* Packs the scenes into virtual rows.  Scene j (0 <= j < n_scenes) has
 * scene_rows[j+1] - scene_rows[j] rows of scene_ell[j] sign bytes each,
 * row r at d_bits + bits_off[j] + r * scene_ell[j]; it becomes virtual rows
 * scene_rows[j] .. scene_rows[j+1]-1.  d_scene_rows (n_scenes + 1 entries,
 * exclusive prefix sums, first 0), d_bits_off and d_scene_ell are device
 * arrays.  Writes scene_rows[n_scenes] * lay.words words to d_packed.
 * Errors: CG_EINVAL (lay not from cg_batch_layout, scene l > the layout's,
 * n_scenes out of 0..65536, NULL pointers). */
cg_status cg_batch_pack(const uint8_t *d_bits, const int64_t *d_bits_off, const int32_t *d_scene_ell,
                        const int64_t *d_scene_rows, int32_t n_scenes, int64_t n_rows, cg_layout lay,
                        void *d_packed, cg_stream_t stream);

/* After cg_edges on the virtual scene's dictionary (with d_offsets):
 *   d_cell_off (n_scenes + 1 int64) <- first virtual cell of each scene;
 *   d_edge_off (n_scenes + 1 int64) <- first edge of each scene;
 * and, if localize != 0, rewrites d_uv[0 .. min(|E|, cap)) to scene-local
 * cell ids and d_bit (nullable) to scene-local positions (minus 32), and
 * d_row_to_cell (nullable, n_rows) to scene-local cell ids.
 * Errors: CG_EINVAL. */
cg_status cg_batch_split(const cg_dict *dict, int32_t n_scenes, const int64_t *d_offsets,
                         const int64_t *d_nedges, int64_t cap, int64_t *d_cell_off, int64_t *d_edge_off,
                         int32_t localize, uint32_t *d_uv, uint16_t *d_bit, uint32_t *d_row_to_cell,
                         const int64_t *d_scene_rows, int64_t n_rows, cg_stream_t stream);

/* ------------------------------------------------------- cell graph search
 * Section 2.1: once the cells and their neighbours are known, a graph
 * algorithm finds the route; Section 6: a path in the cell graph is an
 * approximate solution of the motion-planning problem, and traversing the
 * graph on the GPU is the next problem.  These calls work on the output of
 * cg_edges (with d_offsets) for one scene.
 *
 * cg_graph_csr: the undirected adjacency of G_X in CSR form.
 *   d_uv, d_offsets, d_nedges, d_ncells: as written by cg_edges (and the
 *              dictionary's cell count); nedges_cap = the cap given to it.
 *   d_adj_off (ncells_cap + 1 int64) <- adj_off[u] = first entry of cell u's
 *              list, adj_off[*d_ncells] = 2 |E|;
 *   d_adj     (2 x nedges_cap uint32) <- each cell's neighbours, ascending;
 *   *d_status (device int32) <- CG_OK, or CG_ECAPACITY if *d_nedges >
 *              nedges_cap (the edge list was cut short: the lists then hold
 *              only the edges below the cap).
 * Workspace: cg_graph_csr_workspace(ncells_cap, nedges_cap, &bytes).
 * Errors: CG_EINVAL (NULL buffers, capacities out of 0 .. 2^32-1),
 * CG_EWORKSPACE. */
cg_status cg_graph_csr_workspace(int64_t ncells_cap, int64_t nedges_cap, size_t *bytes);
cg_status cg_graph_csr(const uint32_t *d_uv, const int64_t *d_offsets, const int64_t *d_ncells, int64_t ncells_cap,
                       const int64_t *d_nedges, int64_t nedges_cap, int64_t *d_adj_off, uint32_t *d_adj,
                       int32_t *d_status, void *d_ws, size_t ws_bytes, cg_stream_t stream);

/* cg_bfs: breadth-first search over a cg_graph_csr adjacency from cell
 * `source`, one level per launch, max_levels levels per call:
 *   d_dist   (ncells_cap uint32)           <- hops from the source, or
 *            0xFFFFFFFF if not reached;
 *   d_parent (nullable, ncells_cap uint32) <- the smallest neighbour one hop
 *            closer to the source (the source is its own parent), or
 *            0xFFFFFFFF; with it, every shortest path is the parent chain;
 *   *d_levels (nullable, device int32)     <- the largest distance found;
 *   *d_status (device int32) <- CG_OK when the search is complete,
 *            CG_ECAPACITY when cells remain on the frontier after
 *            max_levels levels (cells on that frontier have their distance
 *            but not yet their parent), CG_EINVAL if source >= *d_ncells.
 * After CG_ECAPACITY, calling again with resume = 1 and the same buffers and
 * workspace continues the search; resume = 0 starts a new one.  Levels past
 * the end of the search cost one empty launch each, so the call never waits
 * for the device.  The workspace holds the search state between calls.
 * Workspace: cg_bfs_workspace(ncells_cap, &bytes).
 * Errors: CG_EINVAL (NULL buffers, max_levels outside 1 .. 65536),
 * CG_EWORKSPACE. */
cg_status cg_bfs_workspace(int64_t ncells_cap, size_t *bytes);
cg_status cg_bfs(const int64_t *d_adj_off, const uint32_t *d_adj, const int64_t *d_ncells, int64_t ncells_cap,
                 uint32_t source, int32_t max_levels, int32_t resume, uint32_t *d_dist, uint32_t *d_parent,
                 int32_t *d_levels, int32_t *d_status, void *d_ws, size_t ws_bytes, cg_stream_t stream);

/* cg_bfs_path: after a complete cg_bfs with parents, the shortest path from
 * the source to `target` by the parent chain: *d_len <- its number of cells
 * (0 if the target is unreached or out of range), and, if it fits in
 * path_cap, d_path[0 .. len) <- source .. target.
 * Errors: CG_EINVAL (NULL buffers, path_cap < 0). */
cg_status cg_bfs_path(const uint32_t *d_dist, const uint32_t *d_parent, const int64_t *d_ncells, int64_t ncells_cap,
                      uint32_t target, uint32_t *d_path, int64_t path_cap, int64_t *d_len, cg_stream_t stream);

/* --------------------------------------------------- sampling + packing
 * The step before the path (Section 2.1: bit i of a sampled point's vector
 * is 1 iff the point satisfies constraint c_i).  Constraints are the
 * half-spaces a_i . p >= c_i of R^3, d_planes = lay.ell rows of four
 * float64 (a_i0, a_i1, a_i2, c_i), device memory.  Point i (0 <= i < n) of
 * the stream (seed, scene) is uniform in the box lo .. hi, box = host array
 * (lo0, lo1, lo2, hi0, hi1, hi2), drawn from Philox4x64-10 (Salmon et al.,
 * SC 2011) with counter (i, 0, 0, 0) and key (seed, scene).  Float
 * contract, each operation rounded to nearest float64, no fused
 * multiply-add:
 *   u_j = (x_j >> 11) * 2^-53 for the block's words x_0, x_1, x_2;
 *   p_j = lo_j + (hi_j - lo_j) * u_j;
 *   r_i = ((a_i0 * p0 + a_i1 * p1) + a_i2 * p2) - c_i;  bit i = (r_i >= 0).
 * Writes n packed rows (layout lay, as cg_pack) to d_packed; no sign bytes
 * are formed.
 * Errors: CG_EINVAL (bad layout, n out of 0 .. 2^32-1, NULL pointers, a box
 * with lo > hi). */
cg_status cg_sample_pack(const double *d_planes, int64_t n, uint64_t seed, uint64_t scene, const double *box,
                         cg_layout lay, void *d_packed, cg_stream_t stream);

/* Batched sampling: cg_batch_pack's virtual rows made from scene
 * descriptions instead of sign bytes.  Scene j (0 <= j < n_scenes) has
 * d_scene_ell[j] planes at d_planes + 4 * d_planes_off[j] (rows of (a0, a1,
 * a2, c) float64) and d_scene_rows[j+1] - d_scene_rows[j] points; its point
 * i is the one cg_sample_pack draws with seed = d_scene_key[2j] and scene =
 * d_scene_key[2j+1], in the box shared by all scenes (host array as for
 * cg_sample_pack); it becomes virtual row d_scene_rows[j] + i (word 0 the
 * scene tag, words 1.. its bits).  All d_* arrays are device memory.  Scene
 * l above the layout's is not checked (extra planes are dropped).
 * Errors: CG_EINVAL (layout not from cg_batch_layout, n_scenes out of
 * 0 .. 65536, n_rows out of range, NULL pointers, lo > hi). */
cg_status cg_batch_sample_pack(const double *d_planes, const int64_t *d_planes_off, const int32_t *d_scene_ell,
                               const int64_t *d_scene_rows, const uint64_t *d_scene_key, int32_t n_scenes,
                               int64_t n_rows, const double *box, cg_layout lay, void *d_packed, cg_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* CELLGRAPH_H */
