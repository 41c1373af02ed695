"""C-ABI contract checks that need no GPU: the library loads, exports every function the
header declares, and rejects bad input on the host before any device work."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1301_1247_amd", "libqpscatter.so")
HDR = os.path.join(ROOT, "include", "qpscatter.h")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "return")))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("hbs_build", "hbs_apply", "qp_solve", "qp_solve_many", "hbs_free", "hbs_last_error", "hbs_stats"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    for n in _declared():
        assert hasattr(lib, n), n


def test_binding_covers_every_declared_symbol():
    from paper_1301_1247_amd import binding
    assert set(_declared()) <= set(binding.EXPORTED)


def _geom(N=256):
    import qpinputs
    from paper_1301_1247_amd.geometry import discretize
    return discretize(qpinputs.star(), N)


def _build(nodes, w, nrm, N, omega=10.0, tol=1e-10, **kw):
    from paper_1301_1247_amd import binding as B
    o = B.hbs_opts(**kw)
    h = C.c_void_p()
    rc = B._lib.hbs_build(nodes.ctypes.data, w.ctypes.data, nrm.ctypes.data, N, omega, tol, C.byref(o), C.byref(h))
    return rc, B._lib.hbs_last_error().decode()


def test_nonfinite_geometry_rejected_on_host():
    nodes, w, nrm, _ = _geom()
    nodes = nodes.copy()
    nodes[3, 0] = np.nan
    rc, msg = _build(nodes, w, nrm, 256)
    assert rc == -2 and "non-finite" in msg


def test_non_unit_normals_rejected():
    nodes, w, nrm, _ = _geom()
    rc, msg = _build(nodes, w, 1.5 * nrm, 256)
    assert rc == -1 and "unit" in msg


def test_bad_sizes_and_tolerance_rejected():
    nodes, w, nrm, _ = _geom()
    assert _build(nodes, w, nrm, 256, tol=1e-20)[0] == -1
    assert _build(nodes, w, nrm, 256, omega=-1.0)[0] == -1
    assert _build(nodes, w, nrm, 100, leaf_size=64)[0] == -1          # N < 2 leaf
    assert _build(nodes, w, nrm, 256, quad=1)[0] == -1                # Kress without curvature
    rc, msg = _build(nodes, w, nrm, 256, quad=1, curvature=w.ctypes.data)
    assert rc == -1 and "EXACT" in msg                                # Kress needs exact compression


def test_negative_weights_rejected():
    nodes, w, nrm, _ = _geom()
    w2 = w.copy()
    w2[0] = -w2[0]
    assert _build(nodes, w2, nrm, 256)[0] == -1


def test_free_null_is_noop_and_error_is_thread_local():
    from paper_1301_1247_amd import binding as B
    B._lib.hbs_free(None)
    nodes, w, nrm, _ = _geom()
    rc, msg = _build(nodes, w, nrm, 256, tol=1.0)
    assert rc == -1 and msg
    import threading
    seen = []
    t = threading.Thread(target=lambda: seen.append(B._lib.hbs_last_error().decode()))
    t.start()
    t.join()
    assert seen == [""]


def test_max_modes_counts_propagating_orders():
    from paper_1301_1247_amd import binding as B
    om, d = 40.0, 2 * math.pi
    mm = B._lib.qp_max_modes(om, d)
    for th in np.linspace(-3.1, -0.05, 50):
        kap = om * math.cos(th)
        n = sum(1 for j in range(-200, 201) if abs(kap + 2 * math.pi * j / d) <= om)
        assert n <= mm


def test_kr6_corrections_match_oracle_derivation():
    """Library (long double, host) and oracle (50-digit mpmath) derive the same corrections."""
    from paper_1301_1247_amd import binding as B
    from oracle import quadrature
    g_lib = B.kr6_corrections()
    g_or = quadrature.kr6_corrections()
    assert np.abs(g_lib - g_or).max() < 1e-12 * np.abs(g_or).max()


# ---------------------------------------------------------------- GEMM tile tuning table (host logic)

def _clog2(x):
    x = max(1, int(x))
    return (x - 1).bit_length()


@pytest.mark.parametrize("c64,m,n,k,cnt", [(0, 1, 1, 1, 1), (0, 64, 64, 16, 1), (0, 65, 200, 97, 1024),
                                           (1, 808, 200, 808, 1), (0, 0, 0, 0, 0), (1, 4097, 3, 20011, 7)])
def test_gemm_class_key_packing(c64, m, n, k, cnt):
    from paper_1301_1247_amd import binding as B
    key = B.gemm_class(m, n, k, cnt, complex64=bool(c64))
    assert key == (c64 << 24 | _clog2(m) << 18 | _clog2(n) << 12 | _clog2(k) << 6 | _clog2(cnt))
    assert B.gemm_class_fields(key) == (c64, _clog2(m), _clog2(n), _clog2(k), _clog2(cnt))


def test_gemm_tune_table_roundtrip_and_builtin():
    import json
    from paper_1301_1247_amd import binding as B
    builtin = B.gemm_tune_get()
    path = os.path.join(ROOT, "paper_1301_1247_amd", "gemm_tune_default.json")
    if os.path.exists(path):
        want = {int(e["key"]): int(e["cfg"]) for e in json.load(open(path))["table"]}
        assert builtin == want  # the library embeds the committed table
    try:
        k1, k2 = B.gemm_class(100, 200, 50, 1000), B.gemm_class(808, 200, 808, 1, complex64=True)
        B.gemm_tune_set({k1: 1, k2: 3})
        assert B.gemm_tune_get() == {k1: 1, k2: 3}
        assert B.gemm_tune_lookup(k1) == 1 and B.gemm_tune_lookup(k2) == 3
        assert B.gemm_tune_lookup(k1 + 1) == -1
        with pytest.raises(B.HBSError):
            B.gemm_tune_set({k1: 4})
        assert B.gemm_tune_get() == {k1: 1, k2: 3}  # a rejected table leaves the active one
        B.gemm_tune_set({})
        assert B.gemm_tune_get() == {}
    finally:
        B.gemm_tune_set(None)
    assert B.gemm_tune_get() == builtin


def test_gemm_tune_sweep_bounds():
    from paper_1301_1247_amd import binding as B
    for bad in (-1, 4):
        with pytest.raises(B.HBSError):
            B.gemm_tune_begin(bad)
    B.gemm_tune_begin(2)
    assert B.gemm_tune_end() == {}  # nothing launched: no classes timed


def test_gemm_tune_choose_keeps_default_within_margin():
    """The sweep's rule: a class leaves 64 x 64 tiles only for a configuration more than the
    margin faster; classes missing under configuration 0 keep it."""
    from paper_1301_1247_amd.tune_gemm import choose
    times = {0: {1: (10.0, 3), 2: (5.0, 3), 3: (1.0, 1)},
             1: {1: (9.0, 3), 2: (4.9, 3), 3: (2.0, 1)},
             2: {1: (9.8, 3), 2: (4.0, 3)},
             3: {1: (11.0, 3), 2: (6.0, 3), 4: (0.5, 1)}}
    table, rows = choose(times, margin=0.03)
    assert table == {1: 1, 2: 2}          # 10% and 20% faster; class 3: 64 x 64 is fastest
    assert 4 not in table                 # never timed with 64 x 64: stays on the default
    assert [r["key"] for r in rows] == [1, 2, 3, 4]
    assert rows[0]["ms"] == {"0": 10.0, "1": 9.0, "2": 9.8, "3": 11.0}
    table_strict, _ = choose(times, margin=0.15)
    assert table_strict == {2: 2}


def test_mem_limit_refused_before_any_device_allocation():
    """hbs_opts.mem_limit is checked on the host: a budget smaller than the geometry upload fails
    with HBS_E_OOM and an error text naming the limit, without touching the device (this runs on
    a host with no GPU)."""
    nodes, w, nrm, _ = _geom()
    rc, msg = _build(nodes, w, nrm, 256, mem_limit=4096)
    assert rc == -3, (rc, msg)
    assert "mem_limit of 4096 device bytes exceeded" in msg


def test_image_period_needs_far_radius():
    """Neighbour-image columns need the far-field circle (it represents the images beyond
    far_radius): the combination is refused on the host, as is a negative period."""
    nodes, w, nrm, _ = _geom()
    rc, msg = _build(nodes, w, nrm, 256, image_period=1.0)
    assert rc == -1 and "far_radius" in msg, (rc, msg)
    rc, msg = _build(nodes, w, nrm, 256, image_period=-1.0, far_radius=2.0)
    assert rc == -1 and "image_period" in msg, (rc, msg)


def test_transmission_options_are_checked_on_the_host():
    """index > 0 (the transmission problem of Sec. 5) is built on the Kapur-Rokhlin operator without
    the Dirichlet-trained rank model, and its image columns need the far-field circle like the
    Dirichlet ones: each combination is refused before any GPU work, as is a negative or
    non-finite index."""
    nodes, w, nrm, _ = _geom()
    for kw, word in ((dict(index=-1.0), "index"), (dict(index=float("nan")), "index"),
                     (dict(index=1.5, quad=1), "KR6"), (dict(index=1.5, quad=2), "KR6"),
                     (dict(index=1.5, image_period=1.0), "far_radius"),
                     (dict(index=1.5, rank_predictor=1), "rank_predictor"),
                     (dict(index=1.5, leaf_size=512), "leaf_size")):
        rc, msg = _build(nodes, w, nrm, 256, **kw)
        assert rc == -1 and word in msg, (kw, rc, msg)


def test_opts_struct_size_matches_binding():
    from paper_1301_1247_amd import binding as B
    o = B.hbs_opts()
    assert o.struct_size == C.sizeof(B.HbsOpts)
    assert o.mem_limit == 0 and o.image_period == 0.0 and o.index == 0.0
    q = B.qp_opts()
    assert q.struct_size == C.sizeof(B.QpOpts)


def test_alpert_rule_derived_by_the_library_matches_oracle():
    """The library derives Alpert's nodes and weights itself (long double Newton); the oracle does
    it independently in 50-digit arithmetic.  One set of numbers, so they must agree."""
    from oracle import alpert as al
    from paper_1301_1247_amd import binding as B
    for m, a in ((2, 2), (3, 3), (5, 6)):
        x, w = B.alpert_rule(m, a)
        xo, wo = al.rule(m, a)
        assert np.abs(x - xo).max() < 1e-13 and np.abs(w - wo).max() < 1e-13


def test_alpert_needs_room_for_its_band():
    nodes, w, nrm, _ = _geom(256)
    rc, msg = _build(nodes, w, nrm, 256, quad=2, leaf_size=8)
    assert rc == -1 and "leaf_size" in msg


def test_struct_layouts_match_the_header(tmp_path):
    """Every field the binding declares sits at the header's offset with the header's size (a C
    program built against include/qpscatter.h prints offsetof and sizeof of each)."""
    import shutil
    import subprocess
    from paper_1301_1247_amd import binding as B
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = (("hbs_opts", B.HbsOpts), ("qp_opts", B.QpOpts), ("hbs_stats_t", B.HbsStats))
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "qpscatter.h"', "int main(void) {"]
    for cname, py in structs:
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("%zu %zu\\n", offsetof({cname}, {fname}), sizeof((({cname} *)0)->{fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True,
                   capture_output=True, text=True)
    out = iter(subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n"))
    for cname, py in structs:
        assert int(next(out)) == C.sizeof(py), cname
        for fname, _ in py._fields_:
            off, size = map(int, next(out).split())
            fld = getattr(py, fname)
            assert (off, size) == (fld.offset, fld.size), (cname, fname)
