// Search on the cell graph (Section 2.1: once the cells and their neighbours
// are known, a graph algorithm finds the robot's route; Section 6: a path in
// the cell graph is an approximate solution of the motion-planning problem,
// and traversing the graph on the GPU is the next problem).
//
// 1. Undirected adjacency in CSR form from the edge list (u < v, ascending):
//    each edge (u, v) is keyed by v << 32 | u and radix-sorted on v (stable,
//    so each v's lower neighbours come out ascending); cell u's list is its
//    lower neighbours followed by its upper ones (the edge list's own run),
//    so every list is ascending.
// 2. Breadth-first search from one cell, one launch per level over the
//    current frontier (two frontier arrays, three rotating counters: level L
//    reads counter L mod 3, appends to (L + 1) mod 3 and clears (L + 2) mod
//    3).  A level whose frontier is empty returns at once, so the host
//    enqueues a fixed number of levels without waiting; the search state
//    stays in the workspace and a later call can resume it.  A cell's parent
//    is its smallest neighbour one level closer to the source, taken when
//    the cell is expanded (its list is ascending and that level is final by
//    then), so the parent array is unique.
#include "cg_internal.hpp"

namespace cg {

namespace {

constexpr uint32_t UNREACHED = 0xFFFFFFFFu;
constexpr int ST = 256;  // threads per block

struct BfsState {
    unsigned long long cnt[3];  // frontier sizes, rotating by level
    int32_t base;               // first level of the next call
    int32_t levels;             // last non-empty level so far
};

__global__ void __launch_bounds__(ST) k_csr_keys(const uint32_t *__restrict__ uv, const int64_t *d_ne, int64_t cap,
                                                 uint64_t *__restrict__ keys, int32_t *status) {
    const int64_t E = load_n(d_ne, cap);
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * ST + threadIdx.x;
    if (gid == 0) *status = (*d_ne > cap) ? CG_ECAPACITY : CG_OK;
    for (int64_t e = gid; e < E; e += static_cast<int64_t>(gridDim.x) * ST)
        keys[e] = (static_cast<uint64_t>(uv[2 * e + 1]) << 32) | uv[2 * e];
}

// Runs of equal v in the sorted keys: [dstart[v], dend[v]) (both 0 if none).
__global__ void __launch_bounds__(ST) k_csr_runs(const uint64_t *__restrict__ keys, const int64_t *d_ne, int64_t cap,
                                                 uint32_t *__restrict__ dstart, uint32_t *__restrict__ dend) {
    const int64_t E = load_n(d_ne, cap);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * ST + threadIdx.x; i < E;
         i += static_cast<int64_t>(gridDim.x) * ST) {
        const uint32_t v = static_cast<uint32_t>(keys[i] >> 32);
        if (i == 0 || static_cast<uint32_t>(keys[i - 1] >> 32) != v) dstart[v] = static_cast<uint32_t>(i);
        if (i == E - 1 || static_cast<uint32_t>(keys[i + 1] >> 32) != v) dend[v] = static_cast<uint32_t>(i + 1);
    }
}

// Degrees: upper neighbours from the edge offsets (only edges below the
// capacity, which are the ones in the list), lower ones from the runs.
__global__ void __launch_bounds__(ST) k_csr_deg(const int64_t *__restrict__ off, const int64_t *d_n, int64_t ncap,
                                                int64_t ecap, const uint32_t *__restrict__ dstart,
                                                const uint32_t *__restrict__ dend, uint32_t *__restrict__ updeg,
                                                uint32_t *__restrict__ downdeg) {
    const int64_t n = load_n(d_n, ncap);
    for (int64_t u = static_cast<int64_t>(blockIdx.x) * ST + threadIdx.x; u < n;
         u += static_cast<int64_t>(gridDim.x) * ST) {
        const int64_t a = off[u] < ecap ? off[u] : ecap, b = off[u + 1] < ecap ? off[u + 1] : ecap;
        updeg[u] = static_cast<uint32_t>(b - a);
        downdeg[u] = dend[u] - dstart[u];
    }
}

// Lower neighbours: sorted key i = (v, u) goes to v's list at i - dstart[v].
__global__ void __launch_bounds__(ST) k_csr_down(const uint64_t *__restrict__ keys, const int64_t *d_ne, int64_t cap,
                                                 const int64_t *__restrict__ adj_off,
                                                 const uint32_t *__restrict__ dstart, uint32_t *__restrict__ adj) {
    const int64_t E = load_n(d_ne, cap);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * ST + threadIdx.x; i < E;
         i += static_cast<int64_t>(gridDim.x) * ST) {
        const uint64_t k = keys[i];
        const uint32_t v = static_cast<uint32_t>(k >> 32);
        adj[adj_off[v] + (i - dstart[v])] = static_cast<uint32_t>(k);
    }
}

// Upper neighbours: edge e = (u, v) goes to u's list after its lower ones.
__global__ void __launch_bounds__(ST) k_csr_up(const uint32_t *__restrict__ uv, const int64_t *d_ne, int64_t cap,
                                               const int64_t *__restrict__ off, const int64_t *__restrict__ adj_off,
                                               const uint32_t *__restrict__ downdeg, uint32_t *__restrict__ adj) {
    const int64_t E = load_n(d_ne, cap);
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * ST + threadIdx.x; e < E;
         e += static_cast<int64_t>(gridDim.x) * ST) {
        const uint32_t u = uv[2 * e], v = uv[2 * e + 1];
        adj[adj_off[u] + downdeg[u] + (e - off[u])] = v;
    }
}

__global__ void __launch_bounds__(ST) k_bfs_clear(const int64_t *d_n, int64_t ncap, uint32_t *__restrict__ dist,
                                                  uint32_t *__restrict__ parent) {
    const int64_t n = load_n(d_n, ncap);
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * ST + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * ST) {
        dist[i] = UNREACHED;
        if (parent) parent[i] = UNREACHED;
    }
}

__global__ void k_bfs_source(const int64_t *d_n, int64_t ncap, uint32_t source, uint32_t *dist, uint32_t *parent,
                             uint32_t *frontier, BfsState *st, int32_t *status) {
    const int64_t n = load_n(d_n, ncap);
    st->base = 0;
    st->levels = 0;
    st->cnt[1] = 0;
    st->cnt[2] = 0;
    if (static_cast<int64_t>(source) >= n) {
        st->cnt[0] = 0;
        *status = CG_EINVAL;
        return;
    }
    st->cnt[0] = 1;
    frontier[0] = source;
    dist[source] = 0;
    if (parent) parent[source] = source;
    *status = CG_OK;
}

// Level base + step: expand the frontier, claim unreached neighbours with a
// compare-and-swap on their distance, append the claimed ones (one counter
// update per wave), and record each expanded cell's parent.  A wave takes 64
// frontier cells and flattens their lists: entry k of the wave's
// concatenated lists goes to lane k mod 64, which finds the owning cell by
// binary search over the lists' starts, so every (cell, neighbour) pair of
// the wave is read in parallel rather than list by list.
__global__ void __launch_bounds__(ST) k_bfs_level(const int64_t *__restrict__ adj_off, const uint32_t *__restrict__ adj,
                                                  int64_t ncap, uint32_t *__restrict__ dist,
                                                  uint32_t *__restrict__ parent, uint32_t *fa, uint32_t *fb,
                                                  BfsState *st, int step) {
    __shared__ uint32_t s_start[ST];  // per wave: exclusive scan of the 64 list lengths
    __shared__ int64_t s_first[ST];   // per wave: each cell's first list entry
    __shared__ uint32_t s_par[ST];    // per wave: smallest neighbour one level closer
    const int level = st->base + step;
    const unsigned long long cur = st->cnt[level % 3];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->cnt[(level + 2) % 3] = 0;  // the previous level's input; the next level's output
        if (cur) st->levels = level;
    }
    if (cur == 0) return;
    const uint32_t *in = (level & 1) ? fb : fa;
    uint32_t *out = (level & 1) ? fa : fb;
    unsigned long long *ocnt = &st->cnt[(level + 1) % 3];
    const uint32_t prev = static_cast<uint32_t>(level - 1), next = static_cast<uint32_t>(level + 1);
    const int lane = lane_id(), wbase = threadIdx.x & ~63;
    for (int64_t b = static_cast<int64_t>(blockIdx.x) * ST; b < static_cast<int64_t>(cur);
         b += static_cast<int64_t>(gridDim.x) * ST) {
        const int64_t f = b + threadIdx.x;
        const bool act = f < static_cast<int64_t>(cur);
        const uint32_t u = act ? in[f] : 0u;
        const int64_t j0 = act ? adj_off[u] : 0;
        const uint32_t deg = act ? static_cast<uint32_t>(adj_off[u + 1] - j0) : 0u;
        const uint32_t incl = wave_incl_scan_u32(deg);
        const uint32_t tot = static_cast<uint32_t>(__shfl(static_cast<int>(incl), 63, 64));
        s_start[threadIdx.x] = incl - deg;
        s_first[threadIdx.x] = j0;
        s_par[threadIdx.x] = UNREACHED;
        __builtin_amdgcn_wave_barrier();
        for (uint32_t k0 = 0; k0 < tot; k0 += 64) {
            const uint32_t k = k0 + static_cast<uint32_t>(lane);
            bool claim = false;
            uint32_t v = 0;
            if (k < tot) {
                // owner: the last lane whose list starts at or before k
                int lo = 0, hi = 63;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_start[wbase + mid] <= k) lo = mid; else hi = mid - 1;
                }
                v = adj[s_first[wbase + lo] + (k - s_start[wbase + lo])];
                const uint32_t d = dist[v];
                if (level > 0 && d == prev) atomicMin(&s_par[wbase + lo], v);
                if (d == UNREACHED) claim = atomicCAS(&dist[v], UNREACHED, next) == UNREACHED;
            }
            wave_append<uint32_t>(out, ocnt, ncap, claim, v);
        }
        __builtin_amdgcn_wave_barrier();
        if (act && parent && level > 0) parent[u] = s_par[threadIdx.x];
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ void k_bfs_finish(BfsState *st, int max_levels, int32_t *levels, int32_t *status) {
    st->base += max_levels;
    if (st->cnt[st->base % 3] > 0) *status = CG_ECAPACITY;  // cells remain on the frontier
    else if (*status != CG_EINVAL) *status = CG_OK;
    if (levels) *levels = st->levels;
}

// One thread: follow parents from the target back to the source and write
// the path source .. target (cell at distance d goes to path[d]).
__global__ void k_bfs_path(const uint32_t *dist, const uint32_t *parent, const int64_t *d_n, int64_t ncap,
                           uint32_t target, uint32_t *path, int64_t path_cap, int64_t *len) {
    const int64_t n = load_n(d_n, ncap);
    if (static_cast<int64_t>(target) >= n || dist[target] == UNREACHED) {
        *len = 0;
        return;
    }
    const int64_t L = static_cast<int64_t>(dist[target]) + 1;
    *len = L;
    if (L > path_cap) return;
    uint32_t v = target;
    for (int64_t d = L - 1; d >= 0; --d) {
        if (static_cast<int64_t>(v) >= n) {  // chain broken: the search was not complete
            *len = 0;
            return;
        }
        path[d] = v;
        v = parent[v];
    }
}

struct CsrWs {
    uint64_t *keys[2];
    uint32_t *hist, *dstart, *dend, *updeg, *downdeg;
    uint64_t *tile_sums;
};

CsrWs carve_csr(void *base, int64_t ncap, int64_t ecap, size_t *bytes) {
    Carver c(base);
    CsrWs w;
    const int64_t e = ecap > 0 ? ecap : 1;
    w.keys[0] = c.take<uint64_t>(e);
    w.keys[1] = c.take<uint64_t>(e);
    w.hist = c.take<uint32_t>(radix_hist_entries(e));
    w.dstart = c.take<uint32_t>(ncap + 1);
    w.dend = c.take<uint32_t>(ncap + 1);
    w.updeg = c.take<uint32_t>(ncap + 1);
    w.downdeg = c.take<uint32_t>(ncap + 1);
    w.tile_sums = c.take<uint64_t>(scan_tiles(ncap + 1));
    *bytes = c.bytes();
    return w;
}

struct BfsWs {
    BfsState *st;
    uint32_t *fa, *fb;
};

BfsWs carve_bfs(void *base, int64_t ncap, size_t *bytes) {
    Carver c(base);
    BfsWs w;
    w.st = c.take<BfsState>(1);
    w.fa = c.take<uint32_t>(ncap + 1);
    w.fb = c.take<uint32_t>(ncap + 1);
    *bytes = c.bytes();
    return w;
}

}  // namespace

size_t csr_workspace_bytes(int64_t ncap, int64_t ecap) {
    size_t b;
    carve_csr(nullptr, ncap, ecap, &b);
    return b;
}

cg_status run_graph_csr(const uint32_t *uv, const int64_t *offsets, const int64_t *d_ncells, int64_t ncap,
                        const int64_t *d_nedges, int64_t ecap, int64_t *adj_off, uint32_t *adj, int32_t *status,
                        void *ws, hipStream_t s) {
    size_t bytes;
    CsrWs w = carve_csr(ws, ncap, ecap, &bytes);
    const unsigned gb_e = blocks_for(ecap, ST, 4096), gb_n = blocks_for(ncap, ST, 4096);
    hipLaunchKernelGGL(k_csr_keys, dim3(gb_e), dim3(ST), 0, s, uv, d_nedges, ecap, w.keys[0], status);
    CG_LAUNCHED("csr_keys");
    int bits = 1;
    while (bits < 32 && (int64_t(1) << bits) < ncap) ++bits;
    const int passes = (bits + 7) / 8;
    int which = 0;
    CG_TRY(radix_sort_u64(w.keys, nullptr, ecap, d_nedges, 32, 32 + 8 * passes, w.hist, w.tile_sums, &which, s));
    const uint64_t *keys = w.keys[which];
    CG_TRY(fill_u32(w.dstart, 0u, ncap + 1, s));
    CG_TRY(fill_u32(w.dend, 0u, ncap + 1, s));
    hipLaunchKernelGGL(k_csr_runs, dim3(gb_e), dim3(ST), 0, s, keys, d_nedges, ecap, w.dstart, w.dend);
    CG_LAUNCHED("csr_runs");
    hipLaunchKernelGGL(k_csr_deg, dim3(gb_n), dim3(ST), 0, s, offsets, d_ncells, ncap, ecap, w.dstart, w.dend,
                       w.updeg, w.downdeg);
    CG_LAUNCHED("csr_deg");
    CG_TRY(scan_pair_to_i64(w.updeg, w.downdeg, adj_off, ncap, d_ncells, w.tile_sums, nullptr, s));
    hipLaunchKernelGGL(k_csr_down, dim3(gb_e), dim3(ST), 0, s, keys, d_nedges, ecap, adj_off, w.dstart, adj);
    CG_LAUNCHED("csr_down");
    hipLaunchKernelGGL(k_csr_up, dim3(gb_e), dim3(ST), 0, s, uv, d_nedges, ecap, offsets, adj_off, w.downdeg, adj);
    CG_LAUNCHED("csr_up");
    return CG_OK;
}

size_t bfs_workspace_bytes(int64_t ncap) {
    size_t b;
    carve_bfs(nullptr, ncap, &b);
    return b;
}

cg_status run_bfs(const int64_t *adj_off, const uint32_t *adj, const int64_t *d_ncells, int64_t ncap,
                  uint32_t source, int32_t max_levels, int32_t resume, uint32_t *dist, uint32_t *parent,
                  int32_t *levels, int32_t *status, void *ws, hipStream_t s) {
    size_t bytes;
    BfsWs w = carve_bfs(ws, ncap, &bytes);
    if (!resume) {
        hipLaunchKernelGGL(k_bfs_clear, dim3(blocks_for(ncap, ST, 4096)), dim3(ST), 0, s, d_ncells, ncap, dist,
                           parent);
        CG_LAUNCHED("bfs_clear");
        hipLaunchKernelGGL(k_bfs_source, dim3(1), dim3(1), 0, s, d_ncells, ncap, source, dist, parent, w.fa, w.st,
                           status);
        CG_LAUNCHED("bfs_source");
    }
    // one block per CU at most: a level's grid-stride loop covers any
    // frontier, and small frontiers (most levels) waste few empty blocks
    const unsigned gb = blocks_for(ncap, ST, 256);
    for (int step = 0; step < max_levels; ++step) {
        hipLaunchKernelGGL(k_bfs_level, dim3(gb), dim3(ST), 0, s, adj_off, adj, ncap, dist, parent, w.fa, w.fb, w.st,
                           step);
        CG_LAUNCHED("bfs_level");
    }
    hipLaunchKernelGGL(k_bfs_finish, dim3(1), dim3(1), 0, s, w.st, max_levels, levels, status);
    CG_LAUNCHED("bfs_finish");
    return CG_OK;
}

cg_status run_bfs_path(const uint32_t *dist, const uint32_t *parent, const int64_t *d_ncells, int64_t ncap,
                       uint32_t target, uint32_t *path, int64_t path_cap, int64_t *len, hipStream_t s) {
    hipLaunchKernelGGL(k_bfs_path, dim3(1), dim3(1), 0, s, dist, parent, d_ncells, ncap, target, path, path_cap,
                       len);
    CG_LAUNCHED("bfs_path");
    return CG_OK;
}

}  // namespace cg
