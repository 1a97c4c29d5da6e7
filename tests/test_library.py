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


STRUCTS = {"hl_options": "Options", "hl_stats": "Stats", "hl_tuning": "Tuning"}


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the option, statistics and tuning structs have
    the header's size and field offsets (checked by compiling the header
    with the host C compiler)."""
    import ctypes
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hisalog.h"',
             "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        py = getattr(pkg.hisalog, pyname)
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    want = {}
    for line in out.splitlines():
        s, f, v = line.split()
        want[(s, f)] = int(v)
    for cname, pyname in STRUCTS.items():
        py = getattr(pkg.hisalog, pyname)
        assert ctypes.sizeof(py) == want[(cname, "size")], cname
        for f, _ in py._fields_:
            assert getattr(py, f).offset == want[(cname, f)], (cname, f)


def test_fused_flags_and_capacity_are_checked_on_a_planning_engine():
    """hl_create rejects a fused capacity that is not a power of two of at
    least 1,024, and accepts the fused flags (a planning-only engine needs
    no GPU)."""
    import ctypes
    h = pkg.hisalog
    L = pkg.lib()

    def create(flags, cap):
        opt = h.Options()
        L.hl_options_init(ctypes.byref(opt))
        opt.device = -1
        opt.flags = flags
        opt.fused_capacity = cap
        e = ctypes.c_void_p()
        rc = L.hl_create(ctypes.byref(opt), ctypes.byref(e))
        if rc == 0:
            L.hl_destroy(e)
        return rc

    assert create(h.HL_FLAG_FUSED | h.HL_FLAG_HIP_GRAPH, 0) == 0
    assert create(h.HL_FLAG_FUSED, 4096) == 0
    assert create(h.HL_FLAG_FUSED, 1000) == h.HL_E_INVALID
    assert create(h.HL_FLAG_FUSED, 512) == h.HL_E_INVALID


def test_expand_tile_option_is_checked():
    """hl_options.expand_tile takes 0 (default), 1024, 2048 or 4096."""
    import ctypes
    h = pkg.hisalog
    L = pkg.lib()
    for tile, want in ((0, 0), (1024, 0), (2048, 0), (4096, 0), (512, h.HL_E_INVALID),
                       (3000, h.HL_E_INVALID), (8192, h.HL_E_INVALID)):
        opt = h.Options()
        L.hl_options_init(ctypes.byref(opt))
        opt.device = -1
        opt.expand_tile = tile
        e = ctypes.c_void_p()
        rc = L.hl_create(ctypes.byref(opt), ctypes.byref(e))
        if rc == 0:
            L.hl_destroy(e)
        assert rc == want, tile
