"""The C-ABI library loads and exports every entry point include/dcg.h
declares; the Python binding exposes each under the same name (no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w]*\s*\**\s+\**(dcg_\w+)\s*\(", text, re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("dcg_setup", "dcg_solve", "dcg_apply", "dcg_destroy", "dcg_strerror",
                     "dcg_last_error", "dcg_host_assemble"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = pytest.importorskip("paper_2606_13429_amd._binding")
    cdll = ctypes.CDLL(lib.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(cdll, n)]
    assert not missing, missing
    unbound = [n for n in _declared() if not hasattr(lib, n)]
    assert not unbound, unbound


def test_status_strings_and_defaults():
    lib = pytest.importorskip("paper_2606_13429_amd._binding")
    assert lib.dcg_strerror(lib.DCG_EINVAL) == "invalid argument"
    mesh, opt = lib.dcg_defaults()
    assert (mesh.n, mesh.penalty, mesh.pre, mesh.post) == (512, 10.0, 2, 2)
    assert opt.prec == lib.DCG_MIXED and abs(opt.c_F - 0.01) < 1e-15 and opt.max_inner == 100


def test_setup_rejects_bad_arguments_before_touching_the_device():
    lib = pytest.importorskip("paper_2606_13429_amd._binding")
    mesh, opt = lib.dcg_defaults()
    mesh.n = 48
    with pytest.raises(lib.DCGError) as ei:
        lib.dcg_setup(mesh, 1e-3, 1.0, opt)
    assert ei.value.status == lib.DCG_EINVAL and "16" in str(ei.value)
    mesh.n = 32
    for dt, nu in ((0.0, 1.0), (-1.0, 1.0), (1e-3, 0.0), (float("nan"), 1.0)):
        with pytest.raises(lib.DCGError):
            lib.dcg_setup(mesh, dt, nu, opt)
