"""The C ABI library loads and exports every function include/gis.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gis.h")
LIB = os.path.join(ROOT, "paper_2202_06111_amd", "libgis.so")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int32_t|void|const char\*)\s+(gis_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        from paper_2202_06111_amd import build
        build.build()
    return LIB


def test_header_declares_the_four_entry_points():
    names = _declared()
    for n in ("gis_build_graph", "gis_prune", "gis_subdivide", "gis_solve"):
        assert n in names


def test_library_exports_every_declared_symbol(built):
    out = subprocess.run(["nm", "-D", "--defined-only", built], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (gis_\w+)$", out, re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(built)
    for n in _declared():
        getattr(lib, n)


def test_binding_declares_the_same_symbols(built):
    from paper_2202_06111_amd import gis
    assert sorted(gis.EXPORTED) == _declared()
    assert gis.lib().gis_version().startswith(b"gis-mi355x")


def test_struct_layouts_match_the_header(built, tmp_path):
    """ctypes mirrors of the ABI structs have the sizes the C compiler gives them."""
    from paper_2202_06111_amd import gis
    src = str(tmp_path / "sizeof.c")
    exe = str(tmp_path / "sizeof")
    with open(src, "w") as f:
        f.write('#include <stdio.h>\n#include "gis.h"\nint main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n",'
                'sizeof(gis_system),sizeof(gis_grid),sizeof(gis_opts),sizeof(gis_cells),'
                'sizeof(gis_graph),sizeof(gis_round_stats),sizeof(gis_solve_info),'
                'sizeof(gis_tuning));return 0;}\n')
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, src], check=True)
    sizes = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                            check=True).stdout.split()]
    mirrors = [gis.SystemT, gis.GridT, gis.OptsT, gis.CellsT, gis.GraphT, gis.RoundStatsT,
               gis.SolveInfoT, gis.TuningT]
    assert sizes == [ctypes.sizeof(m) for m in mirrors]
