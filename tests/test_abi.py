"""The C ABI library loads and exports every symbol include/spade.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "spade.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spade_[a-z_]+)\s*\(", src)))


def test_header_declares_query_calls():
    names = _declared()
    for n in ("spade_select", "spade_join_count", "spade_join_pairs"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2203_14362_amd import spade
    lib = ctypes.CDLL(spade.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(_declared()) == sorted(spade.EXPORTS)


def test_binding_refuses_without_device():
    import torch
    if torch.cuda.is_available():
        return
    from paper_2203_14362_amd import Context
    try:
        Context(0)
    except RuntimeError as e:
        assert "device" in str(e)
    else:
        raise AssertionError("Context() must fail loudly without a HIP device")
