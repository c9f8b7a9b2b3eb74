"""The C-ABI library loads and exports every function include/vor.h declares (CPU only: no
compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "vor.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|void|const char \*)\s*(vor_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("vor_create", "vor_destroy", "vor_compute", "vor_compute_batch", "vor_submit",
                 "vor_poll", "vor_result_free", "vor_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1212_1095_amd as vor
    lib = ctypes.CDLL(vor.lib_path())
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror_and_version_without_gpu():
    import paper_1212_1095_amd as vor
    assert vor.vor_strerror(vor.VOR_E_DUPLICATE) == "duplicate sites"
    assert vor.vor_strerror(12345) == "unknown status"
    assert "gfx950" in vor.vor_version()


def test_create_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import paper_1212_1095_amd as vor
    with pytest.raises(vor.VorError):
        vor.Context()


def test_no_fallback_when_library_missing(tmp_path, monkeypatch):
    import paper_1212_1095_amd._binding as b
    monkeypatch.setattr(b, "_LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(b, "_lib", None)
    with pytest.raises(ImportError):
        b.lib()


def test_autotune_table_lookup(tmp_path):
    """The autotuner's table maps (distribution, nearest log2 n) to Context.tune arguments."""
    import json
    from paper_1212_1095_amd import autotune
    table = {"uniform": {"10": {"sites_per_bucket": 2.0, "block": 256, "block_halfwidth": 0,
                                "leaf_halfwidth": 0, "scan_path": 1, "ms": 0.3},
                         "20": {"sites_per_bucket": 1.0, "block": 128, "block_halfwidth": 2,
                                "ms": 2.0}}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(table))
    assert autotune.best_params(1000, "uniform", path=str(p)) == (2.0, 256, 0, 0, 1)
    assert autotune.best_params(900000, "uniform", path=str(p)) == (1.0, 128, 2, 0, 0)
    assert autotune.best_params(1000, "clustered", path=str(p)) is None


def test_autotune_size_table(tmp_path):
    """The batch section of the table becomes the per-set size classes of Context.size_tuning."""
    import json
    from paper_1212_1095_amd import autotune
    table = {"uniform_batch": {"12": {"sites_per_bucket": 1.5, "block_halfwidth": 2,
                                      "leaf_halfwidth": 0, "ms": 3.0},
                               "5": {"sites_per_bucket": 2.0, "block_halfwidth": 1, "ms": 9.0}}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(table))
    assert autotune.size_table("uniform", path=str(p)) == [(5, 2.0, 1, 0), (12, 1.5, 2, 0)]
    assert autotune.size_table("clustered", path=str(p)) == []
    for e in json.load(open(autotune.TABLE)).get("uniform", {}).values():
        rho, h, ht, path = (e["sites_per_bucket"], e["block_halfwidth"], e["leaf_halfwidth"],
                            e["scan_path"])
        assert (rho, h, ht, path) in autotune.DEFAULT_GRID, "shipped entry outside the sweep grid"


def test_result_layout_of_null_results_without_gpu():
    """vor_result_layout: a NULL result gives a row of zeros; a NULL table is refused."""
    import numpy as np
    import paper_1212_1095_amd as vor
    from paper_1212_1095_amd import _binding as b
    outs = (ctypes.POINTER(b.vor_result) * 3)()
    tab = np.full((3, 8), 7, np.uint64)
    rc = b.lib().vor_result_layout(outs, 3, tab.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    assert rc == vor.VOR_OK and not tab.any()
    assert b.lib().vor_result_layout(outs, 3, None) == vor.VOR_E_INVAL
