"""CPU-side checks of the boundary: the library loads and exports every entry
point the header declares; size queries are pure host arithmetic."""
from __future__ import annotations

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bcinc.h")
LIB = os.path.join(ROOT, "paper_1311_2147_amd", "libbcinc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(bc_[a-z_]+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def lib_built():
    if not os.path.exists(LIB):
        from paper_1311_2147_amd import build

        build.build()
    return LIB


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("bc_load_graph", "bc_update_edge", "bc_update_vertex", "bc_scores", "bc_submit", "bc_recompute",
                     "bc_get_rows", "bc_get_dag"):
        assert required in names


def test_library_exports_every_declared_symbol(lib_built):
    out = subprocess.run(["nm", "-D", "--defined-only", lib_built], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (bc_[a-z_]+)\b", out))
    missing = declared_functions() - exported
    assert not missing, f"declared but not exported: {sorted(missing)}"


def test_binding_loads_and_covers_the_header(lib_built):
    from paper_1311_2147_amd import bcinc

    assert set(bcinc.EXPORTED) == declared_functions()


def test_size_queries(lib_built):
    from paper_1311_2147_amd import bcinc

    n = 1000
    b = bcinc.bc_graph_bytes(n, 8000, 0)
    # D (int32), sigma (uint64) and the stored predecessors (int32) dominate
    assert b >= 16 * n * n
    assert b < 16 * n * n + 8000 * 64 + n * 400
    assert bcinc.bc_graph_bytes(0, 10, 0) == 0
    s1 = bcinc.bc_scratch_bytes(n, 10)
    s2 = bcinc.bc_scratch_bytes(n, 20)
    assert s2 > s1 > 0


def test_status_strings(lib_built):
    from paper_1311_2147_amd import bcinc

    for code in bcinc.STATUS_NAMES:
        assert bcinc._lib.bc_status_string(code)


def test_create_without_device_fails_cleanly(lib_built):
    import ctypes

    import torch

    from paper_1311_2147_amd import bcinc

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    cfg = bcinc.bc_config(0, 0, None, None, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    rc = bcinc._lib.bc_create(ctypes.byref(h), ctypes.byref(cfg))
    assert rc in (-12, -1)


def test_checkpoint_file_holds_plain_arrays(lib_built, tmp_path):
    """save_checkpoint writes the arcs as plain arrays; load_checkpoint reads
    them without pickles and hands load_graph exactly what was saved."""
    import numpy as np

    from paper_1311_2147_amd import bcinc

    arcs = bcinc.Arcs(6, False, np.array([0, 1, 4], np.int32), np.array([2, 3, 5], np.int32),
                      np.array([7, 9, 11], np.int64))

    class Saved:
        def arcs(self):
            return arcs

    class Loader:
        def load_graph(self, g, **kw):
            self.g = g
            return "loaded"

    path = str(tmp_path / "graph.npz")
    bcinc.save_checkpoint(Saved(), path)
    with np.load(path, allow_pickle=False) as z:
        assert set(z.files) == {"n", "directed", "src", "dst", "w"}
    ld = Loader()
    assert bcinc.load_checkpoint(ld, path) == "loaded"
    g = ld.g
    assert g.n == 6 and g.directed is False and g.m == 3
    assert np.array_equal(g.src, arcs.src) and np.array_equal(g.dst, arcs.dst) and np.array_equal(g.w, arcs.w)


def _header_defines(prefix):
    text = open(HEADER).read()
    return {m.group(1): int(m.group(2)) for m in re.finditer(rf"#define ({prefix}\w+)\s+(-?\d+)", text)}


def test_binding_constants_match_the_header(lib_built):
    """Status codes, config flags, check kinds and the stats struct's fields
    of the binding are the header's."""
    from paper_1311_2147_amd import bcinc

    text = open(HEADER).read()
    codes = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(BC_(?:OK|ERR_\w+))\s*=\s*(-?\d+)", text)}
    assert codes == {name: code for code, name in bcinc.STATUS_NAMES.items()}
    flags = _header_defines("BC_FLAG_")
    assert flags == {"BC_FLAG_TIMING": bcinc.BC_FLAG_TIMING, "BC_FLAG_FULL_SEARCH": bcinc.BC_FLAG_FULL_SEARCH,
                     "BC_FLAG_CHECK": bcinc.BC_FLAG_CHECK}
    kinds = _header_defines("BC_CHECK_")
    assert {v: k[len("BC_CHECK_"):].lower() for k, v in kinds.items()} == bcinc.CHECK_KINDS
    body = text[:text.index("} bc_update_stats;")].rsplit("typedef struct {", 1)[1]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"int64_t\s+(\w+);", body)
    assert fields == [f for f, _ in bcinc.bc_update_stats._fields_]


def test_requests_marshal_once_into_a_batch(lib_built):
    """Context._requests fills bc_request entries (edge: kind 0 with u, v, w;
    vertex: kind 1 with v and its edge array) and passes a Batch through
    untouched, so a batch marshalled before a timed region is not redone."""
    from paper_1311_2147_amd import bcinc
    from paper_1311_2147_amd import workloads as W

    class G:
        gid = 3

    ups = [W.Update("edge", u=1, v=2, w=7), W.Update("vertex", v=4, edges=[(4, 5, 2), (6, 4, 9)])]
    reqs, keep = bcinc.Context._requests([(G(), up) for up in ups])
    assert (reqs[0].graph, reqs[0].kind, reqs[0].u, reqs[0].v, reqs[0].w) == (3, 0, 1, 2, 7)
    assert (reqs[1].graph, reqs[1].kind, reqs[1].v, reqs[1].k) == (3, 1, 4, 2)
    assert [(reqs[1].edges[i].a, reqs[1].edges[i].b, reqs[1].edges[i].w) for i in range(2)] == [(4, 5, 2), (6, 4, 9)]
    batch = bcinc.Batch(reqs, keep, len(ups))
    again, kept = bcinc.Context._requests(batch)
    assert again is reqs and kept is keep and len(batch) == 2


def test_check_kinds_of_the_kernels_are_the_headers():
    """The device's CK_* kinds (bc_check.hip) carry the public BC_CHECK_* values."""
    src = open(os.path.join(ROOT, "paper_1311_2147_amd", "csrc", "bc_check.hip")).read()
    device = {m.group(1): int(m.group(2)) for m in re.finditer(r"\bCK_(\w+)\s*=\s*(\d+)", src)}
    public = {k[len("BC_CHECK_"):]: v for k, v in _header_defines("BC_CHECK_").items()}
    assert device == public
