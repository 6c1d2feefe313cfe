"""The C ABI library loads and exports every function include/nnpot.h
declares; host-side argument checks work without a GPU (no compute calls)."""
import ctypes as C
import json
import os
import re

import numpy as np
import pytest

from paper_2305_11805_amd import nnpot, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "nnpot.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nn_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    return nnpot.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(nnpot.EXPORTS)


def test_descriptor_dim_matches_paper_sizes(L):
    with open(os.path.join(ROOT, "tests", "golden", "descriptor_sizes.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        p = synth.mbp_params(c["n_species"], 5.0, c["n_rad"], c["n_theta"], c["n_rs_ang"])
        s, keep = nnpot.make_params(p)
        assert nnpot.nn_descriptor_dim(s) == c["dim"], c["cite"]


def test_host_side_errors(L):
    p = synth.mbp_params(2, 5.0, 16, 8, 4)
    s, keep = nnpot.make_params(p)
    assert nnpot.nn_workspace_size(100, 1, 1000, s) > 0
    bad = synth.mbp_params(2, 5.0, 16, 5, 4)  # 5 angle bins: no kernel compiled
    sb, keep2 = nnpot.make_params(bad)
    assert nnpot.nn_descriptor_dim(sb) == -1
    with pytest.raises(nnpot.NNError) as e:
        nnpot.nn_workspace_size(100, 1, 1000, sb)
    assert e.value.status == 5
    z = synth.mbp_params(1, 5.0, 16, 8, 4, zeta=2.5)
    sz, keep3 = nnpot.make_params(z)
    assert nnpot.nn_descriptor_dim(sz) == -1
    # null system / negative sizes are rejected before any device work
    out = C.c_size_t(0)
    assert L.nn_workspace_size(-1, 1, 0, None, None, 0, 0, C.byref(out)) == 1
    assert L.nn_build_neighbors(None, 5.0, 0.0, None, None, 0, None) == 1
    assert "sys is NULL" in nnpot.nn_last_error()
    sysd = nnpot.nn_system(10, 1, None, None, None, None, None)
    n = C.c_int64(0)
    assert L.nn_count_neighbors(C.byref(sysd), 5.0, C.byref(n), None, 0, None) == 1
