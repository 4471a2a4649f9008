"""The C-ABI library loads and exports every entry point its header declares
(CPU only: no compute calls)."""
import ctypes

import pytest

from paper_1605_08021_amd import acp


def test_library_exports_header_symbols():
    lib = acp.load_library()
    syms = acp.header_symbols()
    assert len(syms) >= 15
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def test_default_options_and_version():
    lib = acp.load_library()
    o = acp.AcpOpts()
    lib.acp_default_opts(ctypes.byref(o))
    assert o.tol == 1e-8 and o.n_cheb == 8 and o.solver == acp.SOLVER_CG
    assert o.precision == acp.PREC_FP64 and o.dyson_max_iter == 4
    assert lib.acp_version().startswith(b"acp-gfx950")


def test_struct_layouts_match_header():
    """Field order and count of the ctypes mirrors follow include/acp.h."""
    import re
    text = re.sub(r"/\*.*?\*/", "", open(acp.HEADER).read(), flags=re.S)
    for cname, py in (("acp_opts", acp.AcpOpts), ("acp_stats", acp.AcpStats),
                      ("acp_grid", acp.AcpGrid), ("acp_eig_opts", acp.AcpEigOpts),
                      ("acp_scf_opts", acp.AcpScfOpts)):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + r";", text).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            parts = decl.replace("*", " ").split(None, 1)[1]
            for n in parts.split(","):
                names.append(re.sub(r"\[.*\]", "", n).strip())
        assert names == [f for f, _ in py._fields_], (cname, names)


def test_null_context_calls_are_rejected():
    lib = acp.load_library()
    assert lib.acp_apply_chi0(None, None, 0, None) == acp.ACP_EINVAL
    lib.acp_destroy(None)
    # calls without a context report through acp_last_error(NULL)
    assert lib.acp_lowest_eigenpairs(None, None, None, None, None, None, None, None, None) == acp.ACP_EINVAL
    assert lib.acp_last_error(None) == b"null argument"


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(acp, "_lib", None)
    with pytest.raises(RuntimeError):
        acp.load_library(str(tmp_path / "missing.so"))
