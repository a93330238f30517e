"""The C-ABI library loads and exports every symbol include/crkfr.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

from paper_2502_07517_amd import crkfr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "crkfr.h")).read()
    return sorted(set(re.findall(r"\b(crkfr_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(crkfr.SYMBOLS) == declared_symbols()


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(crkfr.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_config_struct_matches_header_field_count():
    text = open(os.path.join(ROOT, "include", "crkfr.h")).read()
    body = re.search(r"typedef struct \{(.*?)\} crkfr_config;", text, re.S).group(1)
    decls = [l.split("/*")[0].strip() for l in body.splitlines()]
    names = []
    for d in decls:
        if not d:
            continue
        names += [n.strip().split("[")[0] for n in d.rstrip(";").split(None, 1)[1].split(",")]
    assert names == [f for f, _ in crkfr.Config._fields_]


def test_create_rejects_grids_beyond_32bit_indices():
    """Nodes and face points are indexed with 32-bit integers in the kernels;
    larger grids are refused before any device call."""
    import pytest
    for eq, N, nx, ny in [(crkfr.EULER2D, 3, 11586, 11586), (crkfr.EULER2D, 1, 1, 2 ** 29),
                          (crkfr.EULER1D, 4, 2 ** 29, 1)]:
        with pytest.raises(crkfr.CrkfrError) as e:
            crkfr.Solver(eq, N, nx, ny)
        assert e.value.code == -1 and "2^31" in str(e.value)      # CRKFR_EINVAL
