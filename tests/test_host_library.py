"""CPU-only checks of the HIP library's host side: the shared object loads,
every entry point declared in include/pivco.h is exported, and the host tree
builder (package-merge, written independently of the oracle) agrees with the
oracle.  No kernel is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pivco.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pivco_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2606_05765_amd import pivco as P
    lib = ctypes.CDLL(P.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_host_tree_builder_matches_oracle():
    from paper_2606_05765_amd import pivco as P
    rng = np.random.default_rng(30)
    for trial in range(400):
        m = int(rng.integers(2, 257))
        c = np.zeros(256, np.uint64)
        syms = rng.choice(256, size=m, replace=False)
        kind = trial % 4
        if kind == 0:
            c[syms] = rng.integers(1, 1 << 20, size=m)
        elif kind == 1:
            c[syms] = rng.integers(1, 4, size=m)           # many ties
        elif kind == 2:
            c[syms] = (2.0 ** rng.uniform(0, 40, size=m)).astype(np.uint64) + 1  # skewed
        else:
            c[syms] = 7                                      # all equal
        for L in (11, 12, 15):
            if (1 << L) < m:
                continue
            assert np.array_equal(P.pivco_build_tree(c, L), O.lengths(c, L)), (trial, L)


def test_host_tree_builder_rejects_bad_input():
    from paper_2606_05765_amd import pivco as P
    with pytest.raises(P.PivcoError):
        P.pivco_build_tree(np.zeros(256, np.uint64))
    c = np.zeros(256, np.uint64)
    c[3] = 5
    with pytest.raises(P.PivcoError):
        P.pivco_build_tree(c)                                # one symbol
    c[:] = 1
    with pytest.raises(P.PivcoError):
        P.pivco_build_tree(c, 7)                             # 256 symbols need 8 bits


def test_stream_info_on_oracle_stream():
    from paper_2606_05765_amd import pivco as P
    x = (np.arange(100_000) % 13).astype(np.uint8)
    st = O.encode(x, 4096, ans_mode=1)
    info = P.pivco_stream_info(st.tobytes())
    assert info == O.stream_info(st)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: any --gpus other than 1 exits with status 2
    and says so, before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""
