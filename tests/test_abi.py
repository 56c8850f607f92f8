"""The C-ABI library loads without a GPU and exports every symbol that
include/tdvp.h declares."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "tdvp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tdvp_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("tdvp_heff_apply", "tdvp_krylov_expm", "tdvp_env_update", "tdvp_sweep"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2606_04771_amd as T
    for name in declared_functions():
        assert hasattr(T.lib, name), f"{name} declared in tdvp.h but not exported"
    out = subprocess.run(["nm", "-D", "--defined-only", T.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (tdvp_[a-z0-9_]+)", out))
    assert set(declared_functions()) <= exported
    # nothing beyond the declared C ABI is exported under the tdvp_ prefix
    assert exported <= set(declared_functions())


def test_context_creation_reports_missing_gpu_cleanly():
    import paper_2606_04771_amd as T
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        pytest.skip("a GPU is present")
    with pytest.raises(T.TdvpError) as e:
        T.Context(0)
    assert e.value.code in (-5, -1)


def test_context_setters_reject_a_null_context():
    """Calls on a null context return INVALID (-1) and leave a message, on any machine."""
    import paper_2606_04771_amd as T
    assert T.lib.tdvp_ctx_set_graphs(None, 1) == -1
    assert T.lib.tdvp_ctx_set_precision(None, 0) == -1
    assert T.lib.tdvp_ctx_synchronize(None) == -1
    assert b"null ctx" in T.lib.tdvp_last_error(None)


def test_package_and_build_module_import_without_the_library(tmp_path):
    """In a checkout where libtdvp.so has not been built yet, the package and
    its build module import (the library is loaded at first use), and the
    first call into the library fails loudly instead of falling back."""
    import shutil
    import sys
    pkg = os.path.join(ROOT, "paper_2606_04771_amd")
    dst = tmp_path / "paper_2606_04771_amd"
    shutil.copytree(pkg, dst, ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__"))
    code = ("import paper_2606_04771_amd as T, paper_2606_04771_amd.build as B\n"
            "assert callable(B.build)\n"
            "try:\n"
            "    T.lib.tdvp_ctx_create\n"
            "except ImportError as e:\n"
            "    print('missing:', e)\n"
            "else:\n"
            "    raise SystemExit('library loaded from nowhere')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "missing:" in r.stdout
