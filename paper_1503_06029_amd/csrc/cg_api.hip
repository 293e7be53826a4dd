// C ABI entry points: argument validation, status codes, dispatch.
#include "cg_internal.hpp"

#include <cstdarg>
#include <cstdio>
#include <cstring>

namespace cg {

cg_status allow_lds(const void *kernel, size_t bytes) {
    int dev = 0, cap = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return set_error(CG_EHIP, "cannot query the LDS size per block");
    if (bytes > static_cast<size_t>(cap))
        return set_error(CG_EUNSUPPORTED, "kernel needs %zu bytes of LDS per block, device offers %d", bytes, cap);
    if (bytes > 65536 &&
        hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes)) != hipSuccess)
        return set_error(CG_EHIP, "cannot raise the LDS limit of a kernel to %zu bytes", bytes);
    return CG_OK;
}

namespace {
thread_local char g_err[512] = {0};
thread_local cg_status g_err_status = CG_OK;
constexpr uint32_t DICT_MAGIC = 0x43474431u;  // "CGD1"
}  // namespace

cg_status set_error(cg_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    g_err_status = st;
    return st;
}

cg_status check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(CG_EHIP, "%s: %s", what, hipGetErrorString(e));
    return CG_OK;
}

static cg_status check_layout(const cg_layout &lay) {
    if (lay.ell < 1 || lay.ell > 65535) return set_error(CG_EINVAL, "layout: ell=%d out of range 1..65535", lay.ell);
    if (lay.word_bits != 32 && lay.word_bits != 64)
        return set_error(CG_EINVAL, "layout: word_bits=%d (must be 32 or 64)", lay.word_bits);
    const int32_t want = (lay.ell + lay.word_bits - 1) / lay.word_bits;
    if (lay.words != want) return set_error(CG_EINVAL, "layout: words=%d, expected %d", lay.words, want);
    return CG_OK;
}

static cg_status check_dict(const cg_dict *d) {
    if (!d || d->magic != DICT_MAGIC) return set_error(CG_EINVAL, "dictionary handle not built by cg_dict_build");
    return CG_OK;
}

}  // namespace cg

using namespace cg;

extern "C" {

int32_t cg_version(void) { return (1 << 16) | 0; }

const char *cg_status_string(cg_status st) {
    switch (st) {
    case CG_OK: return "ok";
    case CG_EINVAL: return "invalid argument";
    case CG_EWORKSPACE: return "workspace too small";
    case CG_ECAPACITY: return "edge capacity exceeded";
    case CG_EHIP: return "HIP error";
    case CG_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

cg_status cg_last_error(char *buf, size_t len) {
    if (buf && len) {
        strncpy(buf, g_err, len - 1);
        buf[len - 1] = 0;
    }
    return g_err_status;
}

cg_status cg_make_layout(int32_t ell, int32_t word_bits, cg_layout *lay) {
    if (!lay) return set_error(CG_EINVAL, "cg_make_layout: lay is NULL");
    cg_layout l{ell, word_bits, word_bits > 0 ? (ell + word_bits - 1) / word_bits : 0};
    CG_TRY(check_layout(l));
    *lay = l;
    return CG_OK;
}

cg_status cg_pack(const uint8_t *d_bits, int64_t n, int64_t row_stride, cg_layout lay, void *d_packed,
                  cg_stream_t stream) {
    CG_TRY(check_layout(lay));
    if (n < 0) return set_error(CG_EINVAL, "cg_pack: n=%lld < 0", (long long)n);
    if (row_stride < lay.ell) return set_error(CG_EINVAL, "cg_pack: row_stride=%lld < ell=%d", (long long)row_stride, lay.ell);
    if (n > 0 && (!d_bits || !d_packed)) return set_error(CG_EINVAL, "cg_pack: NULL buffer");
    return launch_pack(d_bits, n, row_stride, lay, d_packed, reinterpret_cast<hipStream_t>(stream));
}

cg_status cg_dedup_workspace(int64_t n, cg_layout lay, size_t *bytes) {
    CG_TRY(check_layout(lay));
    if (n < 0 || n >= (int64_t(1) << 32)) return set_error(CG_EINVAL, "cg_dedup: n=%lld out of range", (long long)n);
    if (!bytes) return set_error(CG_EINVAL, "cg_dedup_workspace: bytes is NULL");
    *bytes = dedup_workspace_bytes(n, lay);
    return CG_OK;
}

cg_status cg_dedup(const void *d_packed, int64_t n, cg_layout lay, void *d_cells, uint32_t *d_row_to_cell,
                   int64_t *d_ncells, void *d_ws, size_t ws_bytes, cg_stream_t stream) {
    CG_TRY(check_layout(lay));
    if (n < 0 || n >= (int64_t(1) << 32)) return set_error(CG_EINVAL, "cg_dedup: n=%lld out of range", (long long)n);
    if (!d_ncells) return set_error(CG_EINVAL, "cg_dedup: d_ncells is NULL");
    if (n > 0 && (!d_packed || !d_cells)) return set_error(CG_EINVAL, "cg_dedup: NULL buffer");
    const size_t need = dedup_workspace_bytes(n, lay);
    if (!d_ws || ws_bytes < need)
        return set_error(CG_EWORKSPACE, "cg_dedup: workspace %zu < %zu bytes", ws_bytes, need);
    return run_dedup(d_packed, n, lay, d_cells, d_row_to_cell, d_ncells, d_ws, ws_bytes,
                     reinterpret_cast<hipStream_t>(stream));
}

cg_status cg_dict_params_default(cg_dict_params *p) {
    if (!p) return set_error(CG_EINVAL, "cg_dict_params_default: NULL");
    memset(p, 0, sizeof(*p));
    p->kind = CG_DICT_SORTED;
    p->dir_bits = -1;
    p->split_bit = -1;
    p->path = CG_PATH_LOOKUP;
    p->n_refs = 4;
    p->group_max = -1;
    return CG_OK;
}

static cg_status check_params(const cg_dict_params *p, const cg_layout &lay) {
    if (!p) return CG_OK;
    if (p->kind != CG_DICT_SORTED && p->kind != CG_DICT_TREE)
        return set_error(CG_EUNSUPPORTED, "dictionary kind %d not supported", p->kind);
    if (p->dir_bits < -1 || p->dir_bits > 24) return set_error(CG_EINVAL, "dir_bits=%d out of range -1..24", p->dir_bits);
    if (p->split_bit < -1 || p->split_bit > lay.ell)
        return set_error(CG_EINVAL, "split_bit=%d out of range -1..ell", p->split_bit);
    if (p->path != CG_PATH_LOOKUP && p->path != CG_PATH_ALLPAIRS && p->path != CG_PATH_HASH)
        return set_error(CG_EINVAL, "path=%d", p->path);
    if (p->n_refs < 0 || p->n_refs > 8) return set_error(CG_EINVAL, "n_refs=%d out of range 0..8", p->n_refs);
    if (p->group_max != -1 && (p->group_max < 1 || p->group_max > 1024))
        return set_error(CG_EINVAL, "group_max=%d out of range 1..1024", p->group_max);
    if (p->key_bits != 0 && p->key_bits != 32 && p->key_bits != 64 && p->key_bits != 96)
        return set_error(CG_EINVAL, "key_bits=%d: 0, 32, 64 or 96", p->key_bits);
    if (p->kind == CG_DICT_SORTED && p->fanout_bits)
        return set_error(CG_EINVAL, "fanout_bits=%d: must be 0 for the sorted kind", p->fanout_bits);
    if (p->fanout_bits < 0 || p->fanout_bits > 8)
        return set_error(CG_EINVAL, "fanout_bits=%d out of range 0..8", p->fanout_bits);
    return CG_OK;
}

cg_status cg_dict_params_tuned(const cg_tune_entry *table, int32_t n_entries, int64_t ncells_cap, cg_layout lay,
                               cg_dict_params *out) {
    if (!out) return set_error(CG_EINVAL, "cg_dict_params_tuned: out is NULL");
    if (n_entries < 0 || (n_entries > 0 && !table)) return set_error(CG_EINVAL, "cg_dict_params_tuned: bad table");
    CG_TRY(check_layout(lay));
    int lg = 0;
    while (lg < 62 && (int64_t(2) << lg) <= ncells_cap) ++lg;  // floor(log2(ncells_cap)), 0 for < 2
    int best = -1, best_d = 0;
    for (int32_t i = 0; i < n_entries; ++i) {
        if (table[i].words != lay.words) continue;
        const int dd = table[i].log2_rows > lg ? table[i].log2_rows - lg : lg - table[i].log2_rows;
        if (best < 0 || dd < best_d || (dd == best_d && table[i].log2_rows < table[best].log2_rows)) {
            best = i;
            best_d = dd;
        }
    }
    if (best < 0) return cg_dict_params_default(out);
    CG_TRY(check_params(&table[best].params, lay));
    *out = table[best].params;
    return CG_OK;
}

cg_status cg_dict_size(int64_t ncells_cap, cg_layout lay, const cg_dict_params *p, size_t *bytes) {
    CG_TRY(check_layout(lay));
    CG_TRY(check_params(p, lay));
    if (ncells_cap < 0 || ncells_cap >= (int64_t(1) << 32))
        return set_error(CG_EINVAL, "ncells_cap=%lld out of range", (long long)ncells_cap);
    if (!bytes) return set_error(CG_EINVAL, "cg_dict_size: bytes is NULL");
    *bytes = dict_mem_bytes(ncells_cap, lay, resolve_params(ncells_cap, lay, p));
    return CG_OK;
}

cg_status cg_dict_build(const void *d_cells, const int64_t *d_ncells, int64_t ncells_cap, cg_layout lay,
                        const cg_dict_params *p, void *d_mem, size_t mem_bytes, cg_dict *out, cg_stream_t stream) {
    CG_TRY(check_layout(lay));
    CG_TRY(check_params(p, lay));
    if (!out) return set_error(CG_EINVAL, "cg_dict_build: out is NULL");
    if (ncells_cap < 0 || ncells_cap >= (int64_t(1) << 32))
        return set_error(CG_EINVAL, "ncells_cap=%lld out of range", (long long)ncells_cap);
    if (!d_ncells) return set_error(CG_EINVAL, "cg_dict_build: d_ncells is NULL");
    if (ncells_cap > 0 && !d_cells) return set_error(CG_EINVAL, "cg_dict_build: d_cells is NULL");
    cg_dict d;
    memset(&d, 0, sizeof(d));
    d.params = resolve_params(ncells_cap, lay, p);
    const size_t need = dict_mem_bytes(ncells_cap, lay, d.params);
    if (!d_mem || mem_bytes < need) return set_error(CG_EWORKSPACE, "cg_dict_build: memory %zu < %zu bytes", mem_bytes, need);
    d.magic = DICT_MAGIC;
    d.lay = lay;
    d.ncells_cap = ncells_cap;
    d.cells = d_cells;
    d.d_ncells = d_ncells;
    d.mem = d_mem;
    d.mem_bytes = mem_bytes;
    CG_TRY(run_dict_build(d, reinterpret_cast<hipStream_t>(stream)));
    *out = d;
    return CG_OK;
}

cg_status cg_neighbors_d1(const cg_dict *dict, const void *d_queries, int64_t nq, uint32_t *d_count,
                          uint32_t *d_self, void *d_mask, cg_stream_t stream) {
    CG_TRY(check_dict(dict));
    if (nq < 0) return set_error(CG_EINVAL, "cg_neighbors_d1: nq=%lld < 0", (long long)nq);
    if (nq > 0 && !d_queries) return set_error(CG_EINVAL, "cg_neighbors_d1: d_queries is NULL");
    return run_neighbors_d1(*dict, d_queries, nq, d_count, d_self, d_mask, reinterpret_cast<hipStream_t>(stream));
}

cg_status cg_edges_workspace(const cg_dict *dict, int64_t cap, size_t *bytes) {
    CG_TRY(check_dict(dict));
    if (cap < 0) return set_error(CG_EINVAL, "cg_edges_workspace: cap < 0");
    if (!bytes) return set_error(CG_EINVAL, "cg_edges_workspace: bytes is NULL");
    switch (dict->params.path) {
    case CG_PATH_ALLPAIRS: *bytes = allpairs_workspace_bytes(*dict, cap); break;
    case CG_PATH_HASH: *bytes = hash_workspace_bytes(*dict, cap); break;
    default: *bytes = edges_workspace_bytes(*dict, cap); break;
    }
    return CG_OK;
}

cg_status cg_edges_workspace_size(int64_t ncells_cap, cg_layout lay, const cg_dict_params *p, int64_t cap,
                                  size_t *bytes) {
    CG_TRY(check_layout(lay));
    CG_TRY(check_params(p, lay));
    if (ncells_cap < 0 || ncells_cap >= (int64_t(1) << 32))
        return set_error(CG_EINVAL, "ncells_cap=%lld out of range", (long long)ncells_cap);
    if (cap < 0) return set_error(CG_EINVAL, "cg_edges_workspace_size: cap < 0");
    if (!bytes) return set_error(CG_EINVAL, "cg_edges_workspace_size: bytes is NULL");
    cg_dict d;
    memset(&d, 0, sizeof(d));
    d.magic = DICT_MAGIC;
    d.lay = lay;
    d.ncells_cap = ncells_cap;
    d.params = resolve_params(ncells_cap, lay, p);
    return cg_edges_workspace(&d, cap, bytes);
}

cg_status cg_edges(const cg_dict *dict, uint32_t *d_uv, uint16_t *d_bit, int64_t cap, int64_t *d_nedges,
                   int64_t *d_offsets, void *d_ws, size_t ws_bytes, int32_t *d_status, cg_stream_t stream) {
    CG_TRY(check_dict(dict));
    if (cap < 0) return set_error(CG_EINVAL, "cg_edges: cap=%lld < 0", (long long)cap);
    if (cap > 0 && !d_uv) return set_error(CG_EINVAL, "cg_edges: d_uv is NULL");
    if (!d_nedges || !d_status) return set_error(CG_EINVAL, "cg_edges: d_nedges / d_status is NULL");
    size_t need = 0;
    CG_TRY(cg_edges_workspace(dict, cap, &need));
    if (!d_ws || ws_bytes < need) return set_error(CG_EWORKSPACE, "cg_edges: workspace %zu < %zu bytes", ws_bytes, need);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (dict->params.path == CG_PATH_ALLPAIRS)
        return run_edges_allpairs(*dict, d_uv, d_bit, cap, d_nedges, d_offsets, d_ws, ws_bytes, d_status, s);
    if (dict->params.path == CG_PATH_HASH)
        return run_edges_hash(*dict, d_uv, d_bit, cap, d_nedges, d_offsets, d_ws, d_status, s);
    return run_edges(*dict, d_uv, d_bit, cap, d_nedges, d_offsets, d_ws, ws_bytes, d_status, s);
}

cg_status cg_batch_layout(int32_t ell_max, cg_layout *lay) {
    if (!lay) return set_error(CG_EINVAL, "cg_batch_layout: lay is NULL");
    return batch_layout(ell_max, lay);
}

cg_status cg_batch_pack(const uint8_t *d_bits, const int64_t *d_bits_off, const int32_t *d_scene_ell,
                        const int64_t *d_scene_rows, int32_t n_scenes, int64_t n_rows, cg_layout lay,
                        void *d_packed, cg_stream_t stream) {
    CG_TRY(check_layout(lay));
    if (lay.word_bits != 32 || lay.ell != 32 * lay.words || lay.words < 2)
        return set_error(CG_EINVAL, "cg_batch_pack: layout not made by cg_batch_layout");
    if (n_rows < 0 || n_rows >= (int64_t(1) << 32)) return set_error(CG_EINVAL, "cg_batch_pack: n_rows out of range");
    if (n_rows > 0 && (!d_bits || !d_bits_off || !d_scene_ell || !d_scene_rows || !d_packed))
        return set_error(CG_EINVAL, "cg_batch_pack: NULL buffer");
    return run_batch_pack(d_bits, d_bits_off, d_scene_ell, d_scene_rows, n_scenes, n_rows, lay, d_packed,
                          reinterpret_cast<hipStream_t>(stream));
}

cg_status cg_batch_split(const cg_dict *dict, int32_t n_scenes, const int64_t *d_offsets, const int64_t *d_nedges,
                         int64_t cap, int64_t *d_cell_off, int64_t *d_edge_off, int32_t localize, uint32_t *d_uv,
                         uint16_t *d_bit, uint32_t *d_row_to_cell, const int64_t *d_scene_rows, int64_t n_rows,
                         cg_stream_t stream) {
    CG_TRY(check_dict(dict));
    if (dict->lay.word_bits != 32 || dict->lay.words < 2)
        return set_error(CG_EINVAL, "cg_batch_split: dictionary is not over a batched layout");
    if (!d_offsets || !d_nedges || !d_cell_off || !d_edge_off) return set_error(CG_EINVAL, "cg_batch_split: NULL buffer");
    if (localize && d_row_to_cell && n_rows > 0 && !d_scene_rows)
        return set_error(CG_EINVAL, "cg_batch_split: d_scene_rows is NULL");
    if (cap < 0) return set_error(CG_EINVAL, "cg_batch_split: cap < 0");
    return run_batch_split(*dict, n_scenes, d_offsets, d_nedges, cap, d_cell_off, d_edge_off, localize, d_uv, d_bit,
                           d_row_to_cell, d_scene_rows, n_rows, reinterpret_cast<hipStream_t>(stream));
}

cg_status cg_graph_csr_workspace(int64_t ncells_cap, int64_t nedges_cap, size_t *bytes) {
    if (ncells_cap < 0 || ncells_cap >= (int64_t(1) << 32) || nedges_cap < 0 || nedges_cap >= (int64_t(1) << 32))
        return set_error(CG_EINVAL, "cg_graph_csr_workspace: capacity out of range");
    if (!bytes) return set_error(CG_EINVAL, "cg_graph_csr_workspace: bytes is NULL");
    *bytes = csr_workspace_bytes(ncells_cap, nedges_cap);
    return CG_OK;
}

cg_status cg_graph_csr(const uint32_t *d_uv, const int64_t *d_offsets, const int64_t *d_ncells, int64_t ncells_cap,
                       const int64_t *d_nedges, int64_t nedges_cap, int64_t *d_adj_off, uint32_t *d_adj,
                       int32_t *d_status, void *d_ws, size_t ws_bytes, cg_stream_t stream) {
    size_t need = 0;
    CG_TRY(cg_graph_csr_workspace(ncells_cap, nedges_cap, &need));
    if (!d_offsets || !d_ncells || !d_nedges || !d_adj_off || !d_status)
        return set_error(CG_EINVAL, "cg_graph_csr: NULL buffer");
    if (nedges_cap > 0 && (!d_uv || !d_adj)) return set_error(CG_EINVAL, "cg_graph_csr: d_uv / d_adj is NULL");
    if (!d_ws || ws_bytes < need) return set_error(CG_EWORKSPACE, "cg_graph_csr: workspace %zu < %zu bytes", ws_bytes, need);
    return run_graph_csr(d_uv, d_offsets, d_ncells, ncells_cap, d_nedges, nedges_cap, d_adj_off, d_adj, d_status, d_ws,
                         reinterpret_cast<hipStream_t>(stream));
}

cg_status cg_bfs_workspace(int64_t ncells_cap, size_t *bytes) {
    if (ncells_cap < 0 || ncells_cap >= (int64_t(1) << 32))
        return set_error(CG_EINVAL, "cg_bfs_workspace: ncells_cap out of range");
    if (!bytes) return set_error(CG_EINVAL, "cg_bfs_workspace: bytes is NULL");
    *bytes = bfs_workspace_bytes(ncells_cap);
    return CG_OK;
}

cg_status cg_bfs(const int64_t *d_adj_off, const uint32_t *d_adj, const int64_t *d_ncells, int64_t ncells_cap,
                 uint32_t source, int32_t max_levels, int32_t resume, uint32_t *d_dist, uint32_t *d_parent,
                 int32_t *d_levels, int32_t *d_status, void *d_ws, size_t ws_bytes, cg_stream_t stream) {
    size_t need = 0;
    CG_TRY(cg_bfs_workspace(ncells_cap, &need));
    if (!d_adj_off || !d_adj || !d_ncells || !d_dist || !d_status) return set_error(CG_EINVAL, "cg_bfs: NULL buffer");
    if (max_levels < 1 || max_levels > 65536) return set_error(CG_EINVAL, "cg_bfs: max_levels=%d out of 1..65536", max_levels);
    if (!d_ws || ws_bytes < need) return set_error(CG_EWORKSPACE, "cg_bfs: workspace %zu < %zu bytes", ws_bytes, need);
    return run_bfs(d_adj_off, d_adj, d_ncells, ncells_cap, source, max_levels, resume, d_dist, d_parent, d_levels,
                   d_status, d_ws, reinterpret_cast<hipStream_t>(stream));
}

cg_status cg_bfs_path(const uint32_t *d_dist, const uint32_t *d_parent, const int64_t *d_ncells, int64_t ncells_cap,
                      uint32_t target, uint32_t *d_path, int64_t path_cap, int64_t *d_len, cg_stream_t stream) {
    if (!d_dist || !d_parent || !d_ncells || !d_len) return set_error(CG_EINVAL, "cg_bfs_path: NULL buffer");
    if (path_cap < 0 || (path_cap > 0 && !d_path)) return set_error(CG_EINVAL, "cg_bfs_path: bad path buffer");
    return run_bfs_path(d_dist, d_parent, d_ncells, ncells_cap, target, d_path, path_cap, d_len,
                        reinterpret_cast<hipStream_t>(stream));
}

cg_status cg_sample_pack(const double *d_planes, int64_t n, uint64_t seed, uint64_t scene, const double *box,
                         cg_layout lay, void *d_packed, cg_stream_t stream) {
    CG_TRY(check_layout(lay));
    if (n < 0 || n >= (int64_t(1) << 32)) return set_error(CG_EINVAL, "cg_sample_pack: n=%lld out of range", (long long)n);
    if (!box) return set_error(CG_EINVAL, "cg_sample_pack: box is NULL");
    if (n > 0 && (!d_planes || !d_packed)) return set_error(CG_EINVAL, "cg_sample_pack: NULL buffer");
    for (int j = 0; j < 3; ++j)
        if (!(box[j] <= box[3 + j])) return set_error(CG_EINVAL, "cg_sample_pack: box lo > hi in axis %d", j);
    return run_sample_pack(d_planes, lay.ell, n, seed, scene, box, lay, d_packed,
                           reinterpret_cast<hipStream_t>(stream));
}

cg_status cg_batch_sample_pack(const double *d_planes, const int64_t *d_planes_off, const int32_t *d_scene_ell,
                               const int64_t *d_scene_rows, const uint64_t *d_scene_key, int32_t n_scenes,
                               int64_t n_rows, const double *box, cg_layout lay, void *d_packed, cg_stream_t stream) {
    CG_TRY(check_layout(lay));
    if (lay.word_bits != 32 || lay.ell != 32 * lay.words || lay.words < 2)
        return set_error(CG_EINVAL, "cg_batch_sample_pack: layout not made by cg_batch_layout");
    if (n_scenes < 0 || n_scenes > 65536) return set_error(CG_EINVAL, "cg_batch_sample_pack: n_scenes=%d", n_scenes);
    if (n_rows < 0 || n_rows >= (int64_t(1) << 32)) return set_error(CG_EINVAL, "cg_batch_sample_pack: n_rows out of range");
    if (!box) return set_error(CG_EINVAL, "cg_batch_sample_pack: box is NULL");
    for (int j = 0; j < 3; ++j)
        if (!(box[j] <= box[3 + j])) return set_error(CG_EINVAL, "cg_batch_sample_pack: box lo > hi in axis %d", j);
    if (n_rows > 0 && (!d_planes || !d_planes_off || !d_scene_ell || !d_scene_rows || !d_scene_key || !d_packed))
        return set_error(CG_EINVAL, "cg_batch_sample_pack: NULL buffer");
    return run_batch_sample_pack(d_planes, d_planes_off, d_scene_ell, d_scene_rows, d_scene_key, n_scenes, n_rows, box,
                                 lay, d_packed, reinterpret_cast<hipStream_t>(stream));
}

cg_status cg_dedup_dict_workspace(int64_t n, cg_layout lay, size_t *bytes) {
    CG_TRY(check_layout(lay));
    if (n < 0 || n >= (int64_t(1) << 32)) return set_error(CG_EINVAL, "cg_dedup_dict_workspace: n out of range");
    if (!bytes) return set_error(CG_EINVAL, "cg_dedup_dict_workspace: bytes is NULL");
    *bytes = dedup_fused_workspace_bytes(n, lay);
    return CG_OK;
}

cg_status cg_dedup_dict(const void *d_packed, int64_t n, cg_layout lay, void *d_cells, uint32_t *d_row_to_cell,
                        int64_t *d_ncells, void *d_ws, size_t ws_bytes, const cg_dict_params *p, void *d_mem,
                        size_t mem_bytes, cg_dict *out, cg_stream_t stream) {
    CG_TRY(check_layout(lay));
    CG_TRY(check_params(p, lay));
    if (n < 0 || n >= (int64_t(1) << 32)) return set_error(CG_EINVAL, "cg_dedup_dict: n=%lld out of range", (long long)n);
    if (!d_ncells || !out || (n > 0 && (!d_packed || !d_cells)))
        return set_error(CG_EINVAL, "cg_dedup_dict: NULL buffer");
    size_t need = 0;
    CG_TRY(cg_dedup_dict_workspace(n, lay, &need));
    if (!d_ws || ws_bytes < need) return set_error(CG_EWORKSPACE, "cg_dedup_dict: workspace %zu < %zu bytes", ws_bytes, need);
    cg_dict d;
    memset(&d, 0, sizeof(d));
    d.params = resolve_params(n, lay, p);
    const size_t mneed = dict_mem_bytes(n, lay, d.params);
    if (!d_mem || mem_bytes < mneed)
        return set_error(CG_EWORKSPACE, "cg_dedup_dict: dictionary memory %zu < %zu bytes", mem_bytes, mneed);
    d.magic = DICT_MAGIC;
    d.lay = lay;
    d.ncells_cap = n;
    d.cells = d_cells;
    d.d_ncells = d_ncells;
    d.mem = d_mem;
    d.mem_bytes = mem_bytes;
    CG_TRY(run_dedup_dict(d_packed, n, lay, d_cells, d_row_to_cell, d_ncells, d_ws, d,
                          reinterpret_cast<hipStream_t>(stream)));
    *out = d;
    return CG_OK;
}

}  // extern "C"
