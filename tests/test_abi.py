"""CPU-side checks of the C ABI: the library loads and exports every entry
point include/ldrop.h declares, and the binding's struct layouts match the
header's field order.  No compute call is made (no GPU here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ldrop.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:ld_status|void|int64_t|const char\s*\*)\s+(ld_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libldrop():
    from paper_2501_04456_amd import ldrop
    if not os.path.exists(ldrop.LIB_PATH):
        from paper_2501_04456_amd import build
        build.build()
    return ldrop.lib()


def test_every_declared_symbol_is_exported(libldrop):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(libldrop, n), f"{n} declared in ldrop.h but not exported"


def test_binding_covers_header():
    from paper_2501_04456_amd import ldrop
    assert sorted(ldrop.SYMBOLS) == declared_functions()


def test_struct_layouts_match_header():
    from paper_2501_04456_amd import ldrop
    txt = open(HEADER).read()
    for cname, py in (("ld_params", ldrop.ld_params), ("ld_radius", ldrop.ld_radius),
                      ("ld_tuning", ldrop.ld_tuning), ("ld_ff_config", ldrop.ld_ff_config),
                      ("ld_ff_train_cfg", ldrop.ld_ff_train_cfg),
                      ("ld_ff_train_report", ldrop.ld_ff_train_report),
                      ("ld_paper_config", ldrop.ld_paper_config), ("ld_diag", ldrop.ld_diag)):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + ";", txt).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            decl = re.sub(r"^(int32_t|int64_t|uint64_t|double)\s+", "", decl)
            for f in decl.split(","):
                fields.append(re.sub(r"\[.*\]", "", f).strip())
        assert [f[0] for f in py._fields_] == fields, cname
    assert C.sizeof(ldrop.ld_params) == 8 + 6 * 8 * 8 + 64 * 8 + 4 * 8 + 3 * 8 + 8 + 16 + 8
    assert C.sizeof(ldrop.ld_radius) == 48 + 2 * 16 * 8
    assert C.sizeof(ldrop.ld_ff_config) == 40
    assert C.sizeof(ldrop.ld_paper_config) == 16 + 8 * 8


def test_no_torch_in_signatures():
    txt = open(HEADER).read()
    assert "torch" not in txt.lower().replace("pytorch", "")


def test_error_text_without_gpu(libldrop):
    # ld_last_error is callable without a device and starts empty
    libldrop.ld_last_error.restype = C.c_char_p
    assert libldrop.ld_last_error() is not None


def test_oracle_exports_every_declared_function():
    """The checker's shared library, as built, carries every function its
    header declares (a build step that compiled only part of its sources
    would leave tests failing with missing symbols)."""
    import oracle
    txt = open(os.path.join(ROOT, "oracle", "ldo.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = sorted(set(re.findall(r"^\s*(?:void|int64_t|double)\s+(ldo_\w+)\s*\(", txt, flags=re.M)))
    assert len(names) >= 25
    if not os.path.exists(oracle._LIB_PATH):
        oracle.build()
    L = C.CDLL(oracle._LIB_PATH)
    for n in names:
        assert hasattr(L, n), f"{n} declared in ldo.h but not in {oracle._LIB_PATH}"
