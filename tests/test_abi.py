"""The C-ABI library loads and exports every symbol include/otip.h declares
(no compute: these run without a GPU)."""
import ctypes
import os
import re

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "otip.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(otip_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["otip_version", "otip_params_default", "otip_create", "otip_destroy",
                 "otip_last_error", "otip_solve", "otip_solve_batch", "otip_result_info",
                 "otip_result_copy", "otip_result_free", "otip_price", "otip_rmin",
                 "otip_kron_apply", "otip_kron_apply_t", "otip_schur"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2206_11009_amd import _abi
    lib = _abi.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(_abi.SIGNATURES)


def test_version_and_defaults_without_gpu():
    import paper_2206_11009_amd as otip
    assert otip.otip_version() == 4
    p = otip.otip_params_default()
    # the paper's stated parameters (Section 5.2, Section 3.3, Section 4.3)
    assert p.tol == 1e-6 and p.cg_tol_pred == 1e-6 and p.cg_tol_corr == 1e-3
    assert p.max_iter == 200 and p.cg_max_iter == 1000 and p.max_corr == 3
    assert p.step_scale == 0.995 and p.switch_window == 5


def test_struct_layouts_match_header_field_order():
    """Field names of the ctypes mirrors appear in the header in the same order."""
    from paper_2206_11009_amd import _abi
    txt = open(HEADER).read()
    for st, cname in [(_abi.otip_params, "otip_params"), (_abi.otip_problem, "otip_problem"),
                      (_abi.otip_info, "otip_info")]:
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (cname, cname), txt, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = re.findall(r"\b([a-z_0-9]+)\s*(?:,|;)", body)
        # declarations like "double mcc_beta_min;" or "int32_t m;"
        assert [f for f, _ in st._fields_] == fields, cname


def test_product_path_needs_a_gpu():
    import torch
    import paper_2206_11009_amd as otip
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(otip.OtipError):
        otip.Context(0)


def test_library_was_built_from_these_sources():
    """The loaded library carries the hash of the sources beside it (a stale
    build is refused at load time rather than tested in place of them)."""
    from paper_2206_11009_amd import _abi
    from paper_2206_11009_amd.build import source_id
    assert _abi.load().otip_source_id().decode() == source_id()
