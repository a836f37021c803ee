"""The C ABI library loads and exports every entry point include/deflan.h declares (CPU only:
no compute call is made without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "deflan.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    names = re.findall(r"\b(dl_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_solver_calls():
    names = declared_functions()
    for must in ("dl_solve_first", "dl_solve_next", "dl_apply", "dl_op_create", "dl_ctx_create", "dl_eig_info"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_0901_3163_amd import deflan
    lib = ctypes.CDLL(deflan.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(deflan.EXPORTED) == declared_functions()
    assert deflan.lib.dl_version() >= 200
    assert deflan.lib.dl_last_error() == b""


def test_invalid_arguments_are_rejected_without_a_device():
    from paper_0901_3163_amd import deflan
    import ctypes as C
    rc = deflan.lib.dl_ctx_create(0, None, None)
    assert rc == deflan.DL_E_INVALID
    assert b"NULL" in deflan.lib.dl_last_error()
    rc = deflan.lib.dl_solve_first(None, None, None, 0, 10, 5, 1e-10, None, None, None)
    assert rc == deflan.DL_E_INVALID
    rc = deflan.lib.dl_solve_next(None, None, 0, None, None, 0, 1e-10, None, None)
    assert rc == deflan.DL_E_INVALID  # op is NULL
    assert deflan.lib.dl_eig_save(None, b"/nonexistent/x") == deflan.DL_E_INVALID
    assert deflan.lib.dl_eig_load(None, b"/nonexistent/x", None) == deflan.DL_E_INVALID
    assert deflan.lib.dl_op_fingerprint(None, None) == deflan.DL_E_INVALID
    assert deflan.lib.dl_tune_tsk(None, deflan.DL_TSK_DOTS16, 1024, 8, 4, 3, None, None, None) == deflan.DL_E_INVALID


def test_binding_structs_match_the_header(tmp_path):
    """Every option / statistics struct of the binding has the size and field offsets that a
    C compiler gives the header's declaration (a field added on one side only fails here)."""
    import shutil
    import subprocess
    import pytest
    from paper_0901_3163_amd import deflan
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = [deflan.dl_first_opts, deflan.dl_next_opts, deflan.dl_stats, deflan.dl_batch_item]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "deflan.h"', "int main(void) {"]
    for s in structs:
        n = s.__name__
        lines.append(f'  printf("{n} size %zu\\n", sizeof({n}));')
        for f, _ in s._fields_:
            lines.append(f'  printf("{n} {f} %zu\\n", offsetof({n}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                         text=True).stdout.splitlines())
    for s in structs:
        n = s.__name__
        assert int(got[f"{n} size"]) == ctypes.sizeof(s), n
        for f, _ in s._fields_:
            assert int(got[f"{n} {f}"]) == getattr(s, f).offset, (n, f)


def test_binding_fails_loudly_without_the_library(tmp_path):
    """The package copied without libdeflan.so cannot be imported: there is no CPU fallback."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_0901_3163_amd"
    pkg.mkdir()
    src = os.path.join(ROOT, "paper_0901_3163_amd")
    for f in ("__init__.py", "deflan.py"):
        shutil.copy(os.path.join(src, f), pkg / f)
    p = subprocess.run([sys.executable, "-c", "import paper_0901_3163_amd"], cwd=tmp_path, capture_output=True,
                       text=True, timeout=120, env=dict(os.environ, PYTHONPATH=str(tmp_path)))
    assert p.returncode != 0
    assert "ImportError" in p.stderr and "libdeflan.so is missing" in p.stderr
