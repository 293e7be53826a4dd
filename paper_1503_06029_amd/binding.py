"""Python binding of ``libcellgraph.so`` (ctypes).

The functions below carry the C ABI's names and only marshal arguments:
torch tensors supply device memory, ``torch.cuda.current_stream()`` supplies
the stream, and every step of the path runs in the library's HIP kernels.
There is no fallback: if the shared library is missing or fails to load,
importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcellgraph.so")

CG_OK, CG_EINVAL, CG_EWORKSPACE, CG_ECAPACITY, CG_EHIP, CG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
CG_DICT_SORTED = 0
CG_DICT_TREE = 1
CG_PATH_LOOKUP, CG_PATH_ALLPAIRS, CG_PATH_HASH = 0, 1, 2

c_i32, c_i64, c_vp, c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t


class Layout(ctypes.Structure):
    _fields_ = [("ell", c_i32), ("word_bits", c_i32), ("words", c_i32)]


class DictParams(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("dir_bits", c_i32), ("split_bit", c_i32), ("path", c_i32),
                ("n_refs", c_i32), ("group_max", c_i32), ("key_bits", c_i32), ("fanout_bits", c_i32)]


class Dict(ctypes.Structure):
    _fields_ = [("magic", ctypes.c_uint32), ("lay", Layout), ("params", DictParams),
                ("ncells_cap", c_i64), ("cells", c_vp), ("d_ncells", c_vp), ("dir", c_vp),
                ("sfx", c_vp), ("mem", c_vp), ("mem_bytes", c_sz), ("tree_depth", c_vp),
                ("tree_levels", c_vp)]


class CellGraphError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"cellgraph status {status}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(or python paper_1503_06029_amd/build.py) first")

_lib = ctypes.CDLL(LIB_PATH)


def _sig(name, args, res=c_i32):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("cg_version", [])
_sig("cg_status_string", [c_i32], ctypes.c_char_p)
_sig("cg_last_error", [ctypes.c_char_p, c_sz])
_sig("cg_make_layout", [c_i32, c_i32, ctypes.POINTER(Layout)])
_sig("cg_pack", [c_vp, c_i64, c_i64, Layout, c_vp, c_vp])
_sig("cg_dedup_workspace", [c_i64, Layout, ctypes.POINTER(c_sz)])
_sig("cg_dedup", [c_vp, c_i64, Layout, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp])
_sig("cg_dict_params_default", [ctypes.POINTER(DictParams)])
_sig("cg_dict_size", [c_i64, Layout, ctypes.POINTER(DictParams), ctypes.POINTER(c_sz)])
_sig("cg_dict_params_tuned", [c_vp, c_i32, c_i64, Layout, ctypes.POINTER(DictParams)])
_sig("cg_dict_build", [c_vp, c_vp, c_i64, Layout, ctypes.POINTER(DictParams), c_vp, c_sz,
                       ctypes.POINTER(Dict), c_vp])
_sig("cg_dedup_dict_workspace", [c_i64, Layout, ctypes.POINTER(c_sz)])
_sig("cg_dedup_dict", [c_vp, c_i64, Layout, c_vp, c_vp, c_vp, c_vp, c_sz, ctypes.POINTER(DictParams), c_vp, c_sz,
                       ctypes.POINTER(Dict), c_vp])
_sig("cg_neighbors_d1", [ctypes.POINTER(Dict), c_vp, c_i64, c_vp, c_vp, c_vp, c_vp])
_sig("cg_edges_workspace", [ctypes.POINTER(Dict), c_i64, ctypes.POINTER(c_sz)])
_sig("cg_edges_workspace_size", [c_i64, Layout, ctypes.POINTER(DictParams), c_i64, ctypes.POINTER(c_sz)])
_sig("cg_edges", [ctypes.POINTER(Dict), c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_sz, c_vp, c_vp])
_sig("cg_edges_noalloc", [ctypes.POINTER(Dict), c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp])
_sig("cg_batch_layout", [c_i32, ctypes.POINTER(Layout)])
_sig("cg_batch_pack", [c_vp, c_vp, c_vp, c_vp, c_i32, c_i64, Layout, c_vp, c_vp])
_sig("cg_batch_split", [ctypes.POINTER(Dict), c_i32, c_vp, c_vp, c_i64, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp,
                        c_i64, c_vp])
_sig("cg_graph_csr_workspace", [c_i64, c_i64, ctypes.POINTER(c_sz)])
_sig("cg_graph_csr", [c_vp, c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp])
_sig("cg_bfs_workspace", [c_i64, ctypes.POINTER(c_sz)])
_sig("cg_bfs", [c_vp, c_vp, c_vp, c_i64, ctypes.c_uint32, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp])
_sig("cg_bfs_path", [c_vp, c_vp, c_vp, c_i64, ctypes.c_uint32, c_vp, c_i64, c_vp, c_vp])
_sig("cg_sample_pack", [c_vp, c_i64, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double), Layout,
                        c_vp, c_vp])
_sig("cg_batch_sample_pack", [c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_i64, ctypes.POINTER(ctypes.c_double), Layout,
                              c_vp, c_vp])

EXPORTS = ("cg_version", "cg_status_string", "cg_last_error", "cg_make_layout", "cg_pack",
           "cg_dedup_workspace", "cg_dedup", "cg_dict_params_default", "cg_dict_size",
           "cg_dict_build", "cg_neighbors_d1", "cg_edges_workspace", "cg_edges_workspace_size", "cg_edges",
           "cg_batch_layout", "cg_batch_pack", "cg_batch_split", "cg_graph_csr_workspace", "cg_graph_csr",
           "cg_bfs_workspace", "cg_bfs", "cg_bfs_path", "cg_sample_pack",
           "cg_batch_sample_pack", "cg_dedup_dict_workspace", "cg_dedup_dict", "cg_edges_noalloc",
           "cg_dict_params_tuned")


def lib():
    return _lib


def _check(st: int):
    if st != CG_OK:
        buf = ctypes.create_string_buffer(512)
        _lib.cg_last_error(buf, 512)
        raise CellGraphError(st, buf.value.decode(errors="replace"))


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def version() -> int:
    return _lib.cg_version()


def make_layout(ell: int, word_bits: int = 64) -> Layout:
    lay = Layout()
    _check(_lib.cg_make_layout(ell, word_bits, ctypes.byref(lay)))
    return lay


def word_dtype(word_bits: int):
    return torch.int64 if word_bits == 64 else torch.int32


# ------------------------------------------------------------ the C calls

def cg_pack(d_bits, n: int, row_stride: int, lay: Layout, d_packed, stream=None):
    _check(_lib.cg_pack(_ptr(d_bits), n, row_stride, lay, _ptr(d_packed), _stream(stream)))


def cg_dedup_workspace(n: int, lay: Layout) -> int:
    b = c_sz()
    _check(_lib.cg_dedup_workspace(n, lay, ctypes.byref(b)))
    return b.value


def cg_dedup(d_packed, n: int, lay: Layout, d_cells, d_row_to_cell, d_ncells, d_ws, ws_bytes: int,
             stream=None):
    _check(_lib.cg_dedup(_ptr(d_packed), n, lay, _ptr(d_cells), _ptr(d_row_to_cell), _ptr(d_ncells),
                         _ptr(d_ws), ws_bytes, _stream(stream)))


def cg_dict_params_default(**overrides) -> DictParams:
    p = DictParams()
    _check(_lib.cg_dict_params_default(ctypes.byref(p)))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


class TuneEntry(ctypes.Structure):
    _fields_ = [("words", c_i32), ("log2_rows", c_i32), ("params", DictParams)]


def cg_dict_params_tuned(entries, ncells_cap: int, lay: Layout) -> DictParams:
    """entries: [(words, log2_rows, DictParams)]."""
    arr = (TuneEntry * max(len(entries), 1))()
    for i, (w, lg, prm) in enumerate(entries):
        arr[i].words, arr[i].log2_rows, arr[i].params = w, lg, prm
    out = DictParams()
    _check(_lib.cg_dict_params_tuned(ctypes.cast(arr, c_vp) if entries else None, len(entries), ncells_cap, lay,
                                     ctypes.byref(out)))
    return out


def cg_dict_size(ncells_cap: int, lay: Layout, params: DictParams | None = None) -> int:
    b = c_sz()
    _check(_lib.cg_dict_size(ncells_cap, lay, ctypes.byref(params) if params is not None else None,
                             ctypes.byref(b)))
    return b.value


def cg_dict_build(d_cells, d_ncells, ncells_cap: int, lay: Layout, params: DictParams | None, d_mem,
                  mem_bytes: int, stream=None) -> Dict:
    out = Dict()
    _check(_lib.cg_dict_build(_ptr(d_cells), _ptr(d_ncells), ncells_cap, lay,
                              ctypes.byref(params) if params is not None else None, _ptr(d_mem), mem_bytes,
                              ctypes.byref(out), _stream(stream)))
    return out


def cg_dedup_dict_workspace(n: int, lay: Layout) -> int:
    b = c_sz()
    _check(_lib.cg_dedup_dict_workspace(n, lay, ctypes.byref(b)))
    return b.value


def cg_dedup_dict(d_packed, n: int, lay: Layout, d_cells, d_row_to_cell, d_ncells, d_ws, ws_bytes: int,
                  params: DictParams | None, d_mem, mem_bytes: int, stream=None) -> Dict:
    out = Dict()
    _check(_lib.cg_dedup_dict(_ptr(d_packed), n, lay, _ptr(d_cells), _ptr(d_row_to_cell), _ptr(d_ncells),
                              _ptr(d_ws), ws_bytes, ctypes.byref(params) if params is not None else None,
                              _ptr(d_mem), mem_bytes, ctypes.byref(out), _stream(stream)))
    return out


def cg_neighbors_d1(d: Dict, d_queries, nq: int, d_count=None, d_self=None, d_mask=None, stream=None):
    _check(_lib.cg_neighbors_d1(ctypes.byref(d), _ptr(d_queries), nq, _ptr(d_count), _ptr(d_self),
                                _ptr(d_mask), _stream(stream)))


def cg_edges_workspace(d: Dict, cap: int) -> int:
    b = c_sz()
    _check(_lib.cg_edges_workspace(ctypes.byref(d), cap, ctypes.byref(b)))
    return b.value


def cg_edges_workspace_for(ncells_cap: int, lay: Layout, params: DictParams | None, cap: int) -> int:
    """cg_edges_workspace_size: the edges workspace before a dictionary exists."""
    b = c_sz()
    _check(_lib.cg_edges_workspace_size(ncells_cap, lay, ctypes.byref(params) if params is not None else None, cap,
                                        ctypes.byref(b)))
    return b.value


def cg_edges(d: Dict, d_uv, d_bit, cap: int, d_nedges, d_offsets, d_ws, ws_bytes: int, d_status,
             stream=None):
    _check(_lib.cg_edges(ctypes.byref(d), _ptr(d_uv), _ptr(d_bit), cap, _ptr(d_nedges), _ptr(d_offsets),
                         _ptr(d_ws), ws_bytes, _ptr(d_status), _stream(stream)))


def cg_edges_noalloc(d: Dict, d_uv, d_bit, cap: int, d_nedges, d_offsets, d_status, stream=None):
    _check(_lib.cg_edges_noalloc(ctypes.byref(d), _ptr(d_uv), _ptr(d_bit), cap, _ptr(d_nedges), _ptr(d_offsets),
                                 _ptr(d_status), _stream(stream)))


# Bytes of the static scratch cg_edges_noalloc uses per device (CG_NOALLOC_SCRATCH_BYTES).
NOALLOC_SCRATCH_BYTES = 64 << 20


def cg_batch_layout(ell_max: int) -> Layout:
    lay = Layout()
    _check(_lib.cg_batch_layout(ell_max, ctypes.byref(lay)))
    return lay


def cg_batch_pack(d_bits, d_bits_off, d_scene_ell, d_scene_rows, n_scenes: int, n_rows: int, lay: Layout,
                  d_packed, stream=None):
    _check(_lib.cg_batch_pack(_ptr(d_bits), _ptr(d_bits_off), _ptr(d_scene_ell), _ptr(d_scene_rows), n_scenes,
                              n_rows, lay, _ptr(d_packed), _stream(stream)))


def cg_batch_split(d: Dict, n_scenes: int, d_offsets, d_nedges, cap: int, d_cell_off, d_edge_off,
                   localize: bool, d_uv=None, d_bit=None, d_row_to_cell=None, d_scene_rows=None, n_rows: int = 0,
                   stream=None):
    _check(_lib.cg_batch_split(ctypes.byref(d), n_scenes, _ptr(d_offsets), _ptr(d_nedges), cap, _ptr(d_cell_off),
                               _ptr(d_edge_off), 1 if localize else 0, _ptr(d_uv), _ptr(d_bit),
                               _ptr(d_row_to_cell), _ptr(d_scene_rows), n_rows, _stream(stream)))


def cg_graph_csr_workspace(ncells_cap: int, nedges_cap: int) -> int:
    b = c_sz()
    _check(_lib.cg_graph_csr_workspace(ncells_cap, nedges_cap, ctypes.byref(b)))
    return b.value


def cg_graph_csr(d_uv, d_offsets, d_ncells, ncells_cap: int, d_nedges, nedges_cap: int, d_adj_off, d_adj,
                 d_status, d_ws, ws_bytes: int, stream=None):
    _check(_lib.cg_graph_csr(_ptr(d_uv), _ptr(d_offsets), _ptr(d_ncells), ncells_cap, _ptr(d_nedges), nedges_cap,
                             _ptr(d_adj_off), _ptr(d_adj), _ptr(d_status), _ptr(d_ws), ws_bytes, _stream(stream)))


def cg_bfs_workspace(ncells_cap: int) -> int:
    b = c_sz()
    _check(_lib.cg_bfs_workspace(ncells_cap, ctypes.byref(b)))
    return b.value


def cg_bfs(d_adj_off, d_adj, d_ncells, ncells_cap: int, source: int, max_levels: int, resume: bool, d_dist,
           d_parent, d_levels, d_status, d_ws, ws_bytes: int, stream=None):
    _check(_lib.cg_bfs(_ptr(d_adj_off), _ptr(d_adj), _ptr(d_ncells), ncells_cap, source, max_levels,
                       1 if resume else 0, _ptr(d_dist), _ptr(d_parent), _ptr(d_levels), _ptr(d_status),
                       _ptr(d_ws), ws_bytes, _stream(stream)))


def cg_bfs_path(d_dist, d_parent, d_ncells, ncells_cap: int, target: int, d_path, path_cap: int, d_len,
                stream=None):
    _check(_lib.cg_bfs_path(_ptr(d_dist), _ptr(d_parent), _ptr(d_ncells), ncells_cap, target, _ptr(d_path),
                            path_cap, _ptr(d_len), _stream(stream)))


def cg_sample_pack(d_planes, n: int, seed: int, scene: int, box, lay: Layout, d_packed, stream=None):
    """box: (lo0, lo1, lo2, hi0, hi1, hi2) on the host."""
    b = (ctypes.c_double * 6)(*[float(v) for v in box])
    _check(_lib.cg_sample_pack(_ptr(d_planes), n, seed, scene, b, lay, _ptr(d_packed), _stream(stream)))


def cg_batch_sample_pack(d_planes, d_planes_off, d_scene_ell, d_scene_rows, d_scene_key, n_scenes: int,
                         n_rows: int, box, lay: Layout, d_packed, stream=None):
    b = (ctypes.c_double * 6)(*[float(v) for v in box])
    _check(_lib.cg_batch_sample_pack(_ptr(d_planes), _ptr(d_planes_off), _ptr(d_scene_ell), _ptr(d_scene_rows),
                                     _ptr(d_scene_key), n_scenes, n_rows, b, lay, _ptr(d_packed), _stream(stream)))
