"""The C-ABI library loads, exports every declared symbol, and validates its
arguments on the host (no kernel is launched by these tests)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cellgraph.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_five_calls():
    names = declared_functions()
    for call in ("cg_pack", "cg_dedup", "cg_dict_build", "cg_neighbors_d1", "cg_edges"):
        assert call in names


def test_library_exports_every_declared_symbol():
    from paper_1503_06029_amd import binding as B
    lib = B.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(B.EXPORTS) == set(declared_functions())
    assert B.version() >> 16 == 1


def test_status_strings():
    from paper_1503_06029_amd import binding as B
    assert B.lib().cg_status_string(0) == b"ok"
    assert B.lib().cg_status_string(-3) == b"edge capacity exceeded"


def test_layout_validation():
    from paper_1503_06029_amd import binding as B
    lay = B.make_layout(130, 64)
    assert (lay.ell, lay.word_bits, lay.words) == (130, 64, 3)
    lay = B.make_layout(130, 32)
    assert lay.words == 5
    for bad in ((0, 64), (70000, 64), (10, 16)):
        with pytest.raises(B.CellGraphError) as e:
            B.make_layout(*bad)
        assert e.value.status == B.CG_EINVAL


def test_argument_validation_without_gpu():
    from paper_1503_06029_amd import binding as B
    lay = B.make_layout(100, 64)
    with pytest.raises(B.CellGraphError) as e:
        B.cg_dedup_workspace(-1, lay)
    assert e.value.status == B.CG_EINVAL
    with pytest.raises(B.CellGraphError) as e:
        B.cg_dedup_workspace(1 << 32, lay)
    assert e.value.status == B.CG_EINVAL
    # workspace smaller than reported: rejected before any launch
    need = B.cg_dedup_workspace(1000, lay)
    assert need > 0
    with pytest.raises(B.CellGraphError) as e:
        B.cg_dedup(1 << 20, 1000, lay, 1 << 21, None, 1 << 22, 1 << 23, need - 1, stream=0)
    assert e.value.status == B.CG_EWORKSPACE
    with pytest.raises(B.CellGraphError) as e:
        B.cg_dedup(1 << 20, 1000, lay, 1 << 21, None, None, 1 << 23, need, stream=0)
    assert e.value.status == B.CG_EINVAL
    # pack: row stride shorter than a row
    with pytest.raises(B.CellGraphError) as e:
        B.cg_pack(1 << 20, 10, 50, lay, 1 << 21, stream=0)
    assert e.value.status == B.CG_EINVAL
    # dictionary parameters
    p = B.cg_dict_params_default()
    assert (p.dir_bits, p.split_bit, p.group_max, p.path) == (-1, -1, -1, 0)
    assert B.cg_dict_size(1000, lay, p) > 0
    for kb in (0, 32, 64, 96):
        assert B.cg_dict_size(1000, lay, B.cg_dict_params_default(key_bits=kb)) > 0
    # the tree kind: fan-out bits 0 (automatic: 2) to 8; its arrays add to the size
    sorted_bytes = B.cg_dict_size(1000, lay, B.cg_dict_params_default())
    for r in range(0, 9):
        assert B.cg_dict_size(1000, lay, B.cg_dict_params_default(kind=B.CG_DICT_TREE, fanout_bits=r)) > sorted_bytes
    for r in (-1, 9):
        with pytest.raises(B.CellGraphError):
            B.cg_dict_size(1000, lay, B.cg_dict_params_default(kind=B.CG_DICT_TREE, fanout_bits=r))
    for field, val in (("dir_bits", 30), ("split_bit", 101), ("n_refs", 9), ("group_max", 0), ("kind", 7),
                       ("key_bits", 48), ("key_bits", -1), ("fanout_bits", 1)):
        q = B.cg_dict_params_default(**{field: val})
        with pytest.raises(B.CellGraphError) as e:
            B.cg_dict_size(1000, lay, q)
        assert e.value.status in (B.CG_EINVAL, B.CG_EUNSUPPORTED)
    # a dictionary handle not made by cg_dict_build
    with pytest.raises(B.CellGraphError) as e:
        B.cg_edges_workspace(B.Dict(), 10)
    assert e.value.status == B.CG_EINVAL


def test_product_has_no_cpu_fallback():
    # the package never imports the oracle
    pkg = os.path.join(ROOT, "paper_1503_06029_amd")
    for f in os.listdir(pkg):
        if f.endswith(".py"):
            src = open(os.path.join(pkg, f)).read()
            assert "import oracle" not in src and "from oracle" not in src, f


def test_tuned_params_pick_nearest_entry():
    """cg_dict_params_tuned: the entry with the layout's words and the
    nearest log2 size (ties to the smaller), defaults without such words."""
    from paper_1503_06029_amd import binding as B
    lay = B.cg_batch_layout(224)  # 8 words
    mk = lambda s: B.cg_dict_params_default(split_bit=s)
    table = [(8, 10, mk(40)), (8, 14, mk(48)), (8, 20, mk(64)), (16, 14, mk(96))]
    assert B.cg_dict_params_tuned(table, 1 << 14, lay).split_bit == 48
    assert B.cg_dict_params_tuned(table, 1 << 12, lay).split_bit == 40   # 12: 2 from 10 and 14 -> the smaller
    assert B.cg_dict_params_tuned(table, (1 << 18) + 5, lay).split_bit == 64
    assert B.cg_dict_params_tuned(table, 1, lay).split_bit == 40
    other = B.cg_batch_layout(480)  # 16 words
    assert B.cg_dict_params_tuned(table, 1 << 3, other).split_bit == 96
    d = B.cg_dict_params_tuned(table, 1 << 14, B.cg_batch_layout(32))  # 2 words: none -> defaults
    assert (d.split_bit, d.dir_bits, d.path) == (-1, -1, 0)
    assert B.cg_dict_params_tuned([], 100, lay).split_bit == -1
    with pytest.raises(B.CellGraphError) as e:
        B.cg_dict_params_tuned([(8, 10, B.cg_dict_params_default(path=7))], 1 << 10, lay)
    assert e.value.status == B.CG_EINVAL


def test_tuner_table_round_trip(tmp_path):
    """The tuner's JSON table comes back through the library's pick."""
    from paper_1503_06029_amd import binding as B, tuner
    p = tmp_path / "t.json"
    tn = tuner.Tuner(str(p))
    tn.table[tuner.key_of(4, 5000)] = dict(split_bit=48, dir_bits=12, group_max=32)
    tn.table[tuner.key_of(4, 300000)] = dict(path=B.CG_PATH_HASH, split_bit=0, dir_bits=18)
    tn.save()
    tn2 = tuner.Tuner(str(p))
    a = tn2.params_for(4, 6000)
    assert (a.split_bit, a.dir_bits, a.group_max, a.path) == (48, 12, 32, 0)
    b = tn2.params_for(4, 250000)
    assert (b.path, b.split_bit) == (B.CG_PATH_HASH, 0)
    assert tn2.params_for(8, 5000) is None
