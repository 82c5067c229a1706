"""The C-ABI library loads and exports every symbol include/pacim.h declares
(no compute calls: these tests run without a GPU)."""
import os
import re

from paper_2311_07554_amd import pacim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pacim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(im_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("im_build_sketches", "im_select_seeds", "im_select_seeds_from", "im_graph_upload",
                     "im_ctx_create", "im_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = pacim.load()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert sorted(pacim._SIGS) == _declared()
