"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/hisalog.h declares, and fails cleanly without a GPU."""

import os
import re

import pytest

import paper_2311_02206_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hisalog.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hl_[a-z_]+)\s*\(", text)))


def test_header_symbols_are_exported():
    syms = declared_symbols()
    assert len(syms) >= 19
    L = pkg.lib()
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(pkg.EXPORTS) == syms


def test_strerror_is_static_text():
    L = pkg.lib()
    assert L.hl_strerror(0) == b"ok"
    assert L.hl_strerror(-6) == b"unsupported"
    assert L.hl_strerror(-99) == b"unknown error"


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(pkg.HlError) as ei:
        pkg.Engine()
    assert ei.value.code == pkg.hisalog.HL_E_DEVICE
