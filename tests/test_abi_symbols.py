"""The C-ABI library loads and exports every function include/pnof.h declares (no GPU needed).

Also exercises the host-only validation of pnof_check_problem, which runs before anything is
enqueued and so needs no device.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pnof.h")

P = pytest.importorskip("paper_2004_06142_amd")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+(pnof_[A-Za-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.library_path()):
        pytest.fail(f"{P.library_path()} is not built")
    return P.lib()


def test_header_parses():
    names = declared_functions()
    assert "pnof_lagrangian" in names and "pnof_orbital_step" in names and len(names) >= 20


def test_every_declared_symbol_is_exported(lib):
    raw = ctypes.CDLL(P.library_path())
    missing = [n for n in declared_functions() if not hasattr(raw, n)]
    assert not missing, f"declared in pnof.h but not exported: {missing}"


def test_binding_names_match_header():
    assert set(P.EXPORTS) <= set(declared_functions())


def test_abi_version(lib):
    m = re.search(r"#define\s+PNOF_ABI_VERSION\s+(\d+)", open(HEADER).read())
    assert lib.pnof_abi_version() == int(m.group(1))


def _check(lib, **kw):
    base = dict(nbf=40, naux=160, npairs=4, ncwo=3, functional=P.PNOF7, precision=P.FP64, ints=P.INTS_DF_F64, flags=0)
    base.update(kw)
    prob = P.Problem(**base)
    return lib.pnof_check_problem(ctypes.byref(prob)), lib.pnof_last_error(None).decode()


@pytest.mark.parametrize("kw,status", [
    ({}, 0),
    ({"precision": P.BF16_SPLIT, "ints": P.INTS_DF_BF16}, 0),
    ({"nbf": 0}, 2),
    ({"npairs": 11}, 2),                       # 11 * 4 > 40
    ({"ncwo": 0}, 2),
    ({"functional": 6}, 1),
    ({"precision": P.FP32}, 0),
    ({"precision": P.FP32, "ints": P.INTS_DF_BF16}, 0),
    ({"precision": 4}, 1),
    ({"ints": 9}, 1),
    ({"flags": 4}, 1),
    ({"naux": 0}, 2),                          # density fitting needs naux > 0
    ({"ints": P.INTS_ERI4_F64, "naux": 0}, 0),
    ({"ints": P.INTS_ERI4_F64, "naux": 8}, 2),
    ({"ints": P.INTS_ERI4_F64, "naux": 0, "nbf": 65, "npairs": 4}, 2),
    ({"ints": P.INTS_ERI4_F64, "naux": 0, "precision": P.BF16_SPLIT}, 3),
    ({"ints": P.INTS_ERI4_F64, "naux": 0, "precision": P.FP32}, 3),
])
def test_check_problem(lib, kw, status):
    st, msg = _check(lib, **kw)
    assert st == status, msg
    if status:
        assert msg


def test_null_problem(lib):
    assert lib.pnof_check_problem(None) == 1
