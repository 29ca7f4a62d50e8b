"""The C ABI library loads and exports every entry point include/vr.h
declares; host-side error paths that need no GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    src = open(os.path.join(ROOT, "include", "vr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vr_[a-z0-9_]+)\s*\(", src)))


def test_header_matches_binding():
    from paper_1902_01010_amd import vr
    assert sorted(vr.ENTRY_POINTS) == declared_entry_points()


def test_library_exports_every_entry_point():
    from paper_1902_01010_amd import vr
    lib = vr.load_library()
    missing = [s for s in declared_entry_points() if not hasattr(lib, s)]
    assert not missing, missing


def test_create_without_device_reports_no_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_1902_01010_amd import vr
    with pytest.raises(vr.VrError) as e:
        vr.Context(0)
    assert e.value.code == vr.VR_ERR_NO_DEVICE
