"""The C-ABI boundary: libefm.so loads without a GPU and exports every
function that include/ec.h declares, and the Python binding (argument
marshalling only) names each of them with the same name."""
import ctypes
import os
import re

import pytest

E = pytest.importorskip("paper_1704_07369_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ec.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)      # drop comments
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(ec_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("ec_setup_kernel", "ec_batch_create", "ec_collide", "ec_entropy_prod",
                     "ec_step_graph", "ec_surrogate_train", "ec_surrogate_collide",
                     "ec_plan_destroy", "ec_batch_destroy", "ec_last_error"):
        assert required in names, required


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(E.binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_function():
    missing = [n for n in declared_functions() if n not in E.binding._SIGS]
    assert not missing, missing
    extra = [n for n in E.binding._SIGS if n not in declared_functions()]
    assert not extra, extra
