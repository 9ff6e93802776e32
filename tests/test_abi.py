"""The C-ABI library loads on the CPU and exports every function include/richards.h declares."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "richards.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rich_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_binding_surface():
    import paper_2112_05051_amd as rich
    assert declared() == sorted(rich.EXPORTS)


def test_library_exports_every_declared_symbol():
    import paper_2112_05051_amd as rich
    if not os.path.exists(rich.LIB_PATH):
        pytest.fail("librichards.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(rich.LIB_PATH)
    missing = [name for name in declared() if not hasattr(lib, name)]
    assert not missing, missing


def test_status_strings_without_gpu():
    import paper_2112_05051_amd as rich
    lib = rich.load()
    assert lib.rich_status_string(0) == b"ok"
    assert b"fresh Jacobian" in lib.rich_status_string(-6)


def test_argument_validation_without_gpu():
    """Invalid problems are rejected on the host before any device work."""
    import ctypes as C

    import paper_2112_05051_amd as rich
    from paper_2112_05051_amd import _lib
    import synth
    lib = rich.load()
    P = synth.cube_problem(8, synth.ARITH, 1.0)
    O = synth.Options()
    b = C.c_size_t()
    assert lib.rich_query_bytes(C.byref(_lib.make_problem(P)), C.byref(_lib.make_opts(O)), C.byref(b)) == 0
    assert b.value > 8 ** 3 * 8 * 30
    for field, bad in (("dt", 0.0), ("hx", -1.0), ("nx", 0), ("mean", 7)):
        Q = synth.cube_problem(8, synth.ARITH, 1.0)
        setattr(Q, field, bad)
        assert lib.rich_query_bytes(C.byref(_lib.make_problem(Q)), C.byref(_lib.make_opts(O)), C.byref(b)) == -1
    O2 = synth.Options(gmres_restart=65)
    assert lib.rich_query_bytes(C.byref(_lib.make_problem(P)), C.byref(_lib.make_opts(O2)), C.byref(b)) == -1
    O3 = synth.Options(amg_smoothed=17)
    assert lib.rich_query_bytes(C.byref(_lib.make_problem(P)), C.byref(_lib.make_opts(O3)), C.byref(b)) == -1
    # the smoothed hierarchy plans for its prolongators and denser coarse levels
    b_sa = C.c_size_t()
    O4 = synth.Options(amg_smoothed=1)
    assert lib.rich_query_bytes(C.byref(_lib.make_problem(P)), C.byref(_lib.make_opts(O4)), C.byref(b_sa)) == 0
    assert b_sa.value > b.value
    h = C.c_void_p()
    assert lib.rich_create(C.byref(_lib.make_problem(P)), C.byref(_lib.make_opts(O)), None, None, C.byref(h)) == -1


def test_server_rejects_over_budget_without_gpu():
    import numpy as np

    import paper_2112_05051_amd as rich
    import synth
    srv = rich.Server(1 << 20, 2)  # 1 MiB
    rec = synth.recipe("c1", n=8)
    with pytest.raises(rich.RichError) as e:
        srv.submit(rec.problem, rec.options, rec.ks(), rec.p0(), 1)
    assert e.value.status == -3
    srv.close()


def test_option_domains_without_gpu():
    """The smoother, aggregation, strength and GMRES round options are checked on the host."""
    import ctypes as C

    import paper_2112_05051_amd as rich
    from paper_2112_05051_amd import _lib
    import synth
    lib = rich.load()
    P = synth.cube_problem(8, synth.ARITH, 1.0)
    b = C.c_size_t()
    for kw, ok in (({"smoother": 1}, True), ({"smoother": 2}, False), ({"amg_aggregation": 1}, True),
                   ({"amg_aggregation": 2}, False), ({"amg_aggregation": 1, "amg_theta": 1.5}, False),
                   ({"amg_aggregation": 1, "amg_block": 0}, False), ({"amg_aggregation": 1, "amg_theta": 0.25}, True),
                   ({"gmres_block": 0}, False), ({"gmres_block": 1}, True), ({"gmres_block": 10}, True),
                   ({"gmres_block": 11}, False), ({"gmres_shift": float("nan")}, False),
                   ({"gmres_shift": 0.0}, True), ({"gmres_shift_span": -0.1}, False),
                   ({"gmres_shift_span": 0.0}, True), ({"gmres_shift_span": float("inf")}, False)):
        O = synth.Options(**kw)
        rc = lib.rich_query_bytes(C.byref(_lib.make_problem(P)), C.byref(_lib.make_opts(O)), C.byref(b))
        assert (rc == 0) == ok, (kw, rc)


def test_server_batching_set_only_before_submissions():
    import numpy as np

    import paper_2112_05051_amd as rich
    import synth
    lib = rich.load()
    srv = rich.Server(1 << 30, 1, fused=True)
    rec = synth.recipe("c1", n=6)
    srv.submit(rec.problem, rec.options, rec.ks(), rec.p0(), 1)
    assert lib.rich_server_set_batching(srv._s, 0) == -11  # RICH_ESTATE
    assert srv.batch_stats() == (0, 0)
    srv.close()
