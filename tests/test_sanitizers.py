"""Host code under AddressSanitizer + UndefinedBehaviorSanitizer (CPU only).

* The oracle's C code, built with gcc -fsanitize=address,undefined, runs
  every function on small inputs in a child process (the sanitizer runtime
  preloaded, since the Python interpreter is not instrumented).
* The library's host code (argument validation, size queries, error text),
  built with the sanitizers on the host side only (-Xarch_host), is driven
  from plain C by tests/abi_host_check.c; no kernel is launched.

Any sanitizer report makes the child exit non-zero."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
ENV_SAN = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}

DRIVER = textwrap.dedent("""
    import os
    import numpy as np
    import oracle
    from paper_1503_06029_amd import inputs
    assert oracle.lib()._name == os.environ["CG_ORACLE_LIB"]
    rng = np.random.default_rng(5)
    for ell, wb in ((3, 32), (40, 32), (70, 64), (200, 64), (1024, 64)):
        R = inputs.clustered_multiset(rng, 60, ell, 4, 30)
        rows = oracle.pack(R, wb)
        cells, r2c = oracle.dedup(rows, ell, wb)
        uv, bit, off = oracle.edges(cells, wb)
        uv2, bit2, off2 = oracle.edges_search(cells, ell, wb)
        assert np.array_equal(uv, uv2) and np.array_equal(bit, bit2) and np.array_equal(off, off2)
        nb, cnt = oracle.neighbors_of(cells, np.arange(min(10, len(cells))), wb, max_deg=3)
        q = np.concatenate([cells[:5], rows[:5]])
        oracle.d1_queries(cells, q, wb)
        refs = cells[:3]
        oracle.ref_dists(cells, refs, wb)
        oracle.edges_heuristic(cells, [0, 1, 2], wb)
        if ell % 2 == 0 and ell <= 200:
            oracle.tree_levels(cells, ell, 2, wb, nodes=True)
            oracle.digits(cells[0], ell, 2, wb)
        oracle.dist(cells[0], cells[-1], wb)
        oracle.dist_bitwise(cells[0], cells[-1], ell, wb)
        A = oracle.adjacency(len(cells), uv)
        oracle.bfs(len(cells), uv, 0)
    planes = rng.normal(size=(33, 4))
    oracle.sample_signs(planes, 200, 7, 3, (-1.0, -1.0, -1.0, 1.0, 1.0, 1.0))
    oracle.philox4x64((1, 2, 3, 4), (5, 6))
    # empty inputs
    e = np.zeros((0, 2), dtype=np.uint64)
    oracle.edges(e, 64)
    print("oracle ok")
""")


def _run(cmd, env=None, cwd=ROOT, timeout=600):
    r = subprocess.run(cmd, cwd=cwd, env=env, capture_output=True, text=True, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


@pytest.mark.slow
def test_oracle_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "libcg_oracle_san.so")
    rc, out = _run(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-ffp-contract=off", *SAN,
                    "-o", lib, os.path.join(ROOT, "oracle", "cg_oracle.c")])
    assert rc == 0, out
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    env = dict(os.environ, CG_ORACLE_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}", OMP_NUM_THREADS="2", **ENV_SAN)
    env["PYTHONPATH"] = ROOT
    rc, out = _run([sys.executable, "-c", DRIVER], env=env)
    assert rc == 0 and "oracle ok" in out, out[-4000:]
    assert "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out[-4000:]


@pytest.mark.slow
def test_library_host_code_under_asan_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_1503_06029_amd import build as hb
    lib = str(tmp_path / "libcellgraph_san.so")
    hb.build(out=lib, build_dir=str(tmp_path / "obj"), host_flags=SAN)
    exe = str(tmp_path / "abi_host_check")
    clang = "/opt/rocm/lib/llvm/bin/clang"
    rc, out = _run([clang, *SAN, "-I", os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "abi_host_check.c"),
                    lib, f"-Wl,-rpath,{tmp_path}", "-o", exe])
    assert rc == 0, out
    env = dict(os.environ, **ENV_SAN)
    rc, out = _run([exe], env=env, timeout=300)
    assert rc == 0 and out.strip().endswith("ok"), out[-4000:]
    assert "runtime error" not in out and "ERROR: AddressSanitizer" not in out, out[-4000:]
