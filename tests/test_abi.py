"""C-ABI checks that need no GPU: the library loads, exports every function
include/xab.h declares, and its host-only logic (class table, status names,
argument checks that fail before any device call) behaves as documented."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xab.h")


def _lib_path():
    import paper_2405_01599_amd as xab
    if not os.path.exists(xab.LIB_PATH):
        pytest.skip("libxab.so not built")
    return xab.LIB_PATH


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(xab_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("xab_spmv_csr", "xab_spmv_sym", "xab_select", "xab_gmres", "xab_bicgstab", "xab_init",
                     "xab_matrix_csr", "xab_plan_fixed", "xab_features", "xab_selector_train"):
        assert required in names


def test_library_exports_every_declared_symbol():
    path = _lib_path()
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_library_loads_and_binds():
    import paper_2405_01599_amd as xab
    _lib_path()
    L = xab.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) <= set(xab.SIGNATURES)


def test_class_table():
    import paper_2405_01599_amd as xab
    _lib_path()
    seen = []
    for k in range(xab.NCLASSES):
        v, p = xab.class_params(k)
        seen.append((v, p.lanes_per_row, p.tile_nnz, p.j_per_lane, p.col_block))
    assert [s[0] for s in seen[:3]] == [xab.ROW] * 3
    assert [s[1] for s in seen[:3]] == [1, 8, 64]
    assert [s[0] for s in seen[3:5]] == [xab.NNZ] * 2 and [s[2] for s in seen[3:5]] == [2048, 8192]
    assert [s[0] for s in seen[5:9]] == [xab.BSS] * 4 and [s[3] for s in seen[5:9]] == [4, 8, 16, 32]
    assert seen[9][0] == xab.SYM_ATOMIC and seen[10][0] == seen[11][0] == xab.SYM_S3
    assert seen[12][0] == xab.XCB and seen[12][3] == 0  # entries per lane chosen from the size
    assert seen[13][0] == xab.SELL and xab.class_params(13)[1].tile_rows == 1024
    assert seen[14][0] == xab.BCSR
    with pytest.raises(xab.XabError):
        xab.class_params(15)


def test_status_strings_and_null_checks():
    import paper_2405_01599_amd as xab
    L = xab.lib()
    assert L.xab_status_str(0) == b"ok"
    assert L.xab_status_str(-4) == b"invalid CSR structure"
    assert L.xab_status_str(2) == b"breakdown"
    # null handles are rejected before any device work
    assert L.xab_init(None, None) == -1
    assert L.xab_matrix_csr(None, 1, 1, 1, None, None, None, 0, 0, None) == -1
    assert L.xab_spmv_csr(None, None, None, 0, None, 0, 0) == -1
    assert L.xab_select(None, None, 0, None, None) == -1
    assert L.xab_gmres(None, None, None, None, None, None) == -1
    assert L.xab_bicgstab(None, None, None, None, None, None, None) == -1
    assert L.xab_features(None, None, None, None) == -1
    assert L.xab_class_params(0, None, None) == -1
    assert xab.MLP_NPARAMS == 64 * 12 + 64 + 64 * 64 + 64 + 15 * 64 + 15


def test_product_path_has_no_oracle_dependency():
    """The HIP library and its binding never reach the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_2405_01599_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower().replace("oracles", ""), f
    import paper_2405_01599_amd as xab
    path = _lib_path()
    out = subprocess.run(["nm", "-D", path], capture_output=True, text=True, check=True).stdout
    assert "orc_" not in out


STRUCTS = {"Params": "xab_params", "InitOpts": "xab_init_opts", "SelectInfo": "xab_select_info",
           "TrainOpts": "xab_train_opts", "TrainInfo": "xab_train_info", "KrylovOpts": "xab_krylov_opts",
           "KrylovInfo": "xab_krylov_info", "EigOpts": "xab_eig_opts", "EigInfo": "xab_eig_info"}


def test_header_is_strict_c99(tmp_path):
    """The boundary header stands alone as ISO C99 (no C++ in it)."""
    src = tmp_path / "h.c"
    src.write_text('#include "xab.h"\nint main(void) { return 0; }\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                    "-I", os.path.join(ROOT, "include"), str(src)], check=True)


def test_binding_struct_layouts_match_the_header(tmp_path):
    """Every ctypes mirror of a header struct has the C compiler's size and
    the same offset and size for every field (a field added on one side
    only, or out of order, fails here)."""
    import ctypes

    import paper_2405_01599_amd as xab
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "xab.h"', "int main(void) {"]
    for py, c in STRUCTS.items():
        cls = getattr(xab, py)
        lines.append(f'    printf("{py} %zu\\n", sizeof({c}));')
        for f in cls._fields_:
            name = f[0]
            lines.append(f'    printf("{py}.{name} %zu %zu\\n", offsetof({c}, {name}), sizeof((({c} *)0)->{name}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if line.strip():
            key, *vals = line.split()
            got[key] = [int(v) for v in vals]
    for py in STRUCTS:
        cls = getattr(xab, py)
        assert got[f"{py}"] == [ctypes.sizeof(cls)], py
        for f in cls._fields_:
            d = getattr(cls, f[0])
            assert got[f"{py}.{f[0]}"] == [d.offset, d.size], (py, f[0])
