// cg_edges_noalloc: cg_edges for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  The edge passes' scratch (per-cell counts and offsets, per-tile
// stashes and totals, lists of long groups and runs) lives in one file-scope
// device array instead of a caller workspace.  Each GPU the library runs on
// holds its own copy of the array until the process ends.
//
// The array's name is a host-side stand-in in host code; its device address
// is taken once per device with hipGetSymbolAddress and only that address is
// passed to kernels.  Every call on a GPU shares that GPU's array and leaves
// its contents behind; the edge kernels clear what must start at zero
// themselves (with fill kernels, not memsets).  Calls that overlap on one
// GPU (two streams, or two host threads) race on the array.
#include "cg_internal.hpp"

#include <mutex>

namespace cg {

namespace {

static __device__ __align__(256) unsigned char scratch[CG_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES] = {};

// Device address of the current device's array, taken on the first call on
// that device (with it current) and kept.
cg_status scratch_address(void **out) {
    int dev = -1;
    const hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) return set_error(CG_EHIP, "cg_edges_noalloc: hipGetDevice: %s", hipGetErrorString(ge));
    if (dev < 0 || dev >= MAX_DEVICES)
        return set_error(CG_EUNSUPPORTED, "cg_edges_noalloc: device %d beyond the %d devices served", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(CG_EHIP, "cg_edges_noalloc: hipGetSymbolAddress on device %d: %s", dev,
                             hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return CG_OK;
}

}  // namespace

}  // namespace cg

using namespace cg;

extern "C" cg_status cg_edges_noalloc(const cg_dict *dict, uint32_t *d_uv, uint16_t *d_bit, int64_t cap,
                                      int64_t *d_nedges, int64_t *d_offsets, int32_t *d_status, cg_stream_t stream) {
    size_t need = 0;
    CG_TRY(cg_edges_workspace(dict, cap, &need));  // also validates the dictionary handle and cap
    if (need > static_cast<size_t>(CG_NOALLOC_SCRATCH_BYTES))
        return set_error(CG_EWORKSPACE,
                         "cg_edges_noalloc: %lld cells need %zu bytes of scratch, more than the %zu held per device; "
                         "use cg_edges with a workspace",
                         static_cast<long long>(dict->ncells_cap), need,
                         static_cast<size_t>(CG_NOALLOC_SCRATCH_BYTES));
    void *ws = nullptr;
    CG_TRY(scratch_address(&ws));
    return cg_edges(dict, d_uv, d_bit, cap, d_nedges, d_offsets, ws, static_cast<size_t>(CG_NOALLOC_SCRATCH_BYTES),
                    d_status, stream);
}
