"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every function declared in include/pou.h, and the ctypes structures match."""
import ctypes
import os

import pytest

import paper_1510_07230_amd as pk


def _built():
    return os.path.exists(pk.LIB_PATH)


@pytest.mark.skipif(not _built(), reason="libpou.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    L = pk.lib()
    declared = pk.header_symbols()
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(pk._SIGNATURES)


@pytest.mark.skipif(not _built(), reason="libpou.so not built")
def test_default_params_are_the_papers_constants():
    p = pk.default_params()
    assert (p.rho1, p.delta, p.eta) == (1e-4, 0.1, 0.85)
    assert p.s_max == 10 and p.terms == 15 and p.cg_precond == 1


def test_struct_layouts_match_header():
    """Field order of the structs in include/pou.h matches the ctypes mirror."""
    import re
    txt = open(pk.HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    for cls, tag in ((pk.Params, "pou_params"), (pk.StepInfo, "pou_step_info"),
                     (pk.EnergyTerms, "pou_energy_terms"), (pk.Grid, "pou_grid")):
        body = txt[:txt.index("} " + tag + ";")]
        body = body[body.rindex("typedef struct {") + len("typedef struct {"):]
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            parts = decl.split(None, 1)
            names += [v.strip() for v in parts[1].split(",")]
        assert names == [f for f, _ in cls._fields_], (tag, names)
    assert ctypes.sizeof(pk.Grid) == 16


@pytest.mark.skipif(not _built(), reason="libpou.so not built")
def test_null_arguments_rejected_on_host():
    L = pk.lib()
    assert L.pou_create(None, 0, None) == -1
    assert L.pou_destroy(None) == -1
    assert L.pou_reset_history(None) == -1
    assert L.pou_energy(None, None, None) == -1
