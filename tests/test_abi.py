"""Boundary checks that need no GPU: the C-ABI library loads, exports every entry
point include/kpsi.h declares, and fails cleanly when no device is present."""
import os
import re

import pytest

from paper_2007_14931_amd import kpsi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "kpsi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kpsi_[a-z_]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert sorted(kpsi.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    L = kpsi.lib()
    for name in _declared():
        assert hasattr(L, name), name


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device error path")
def test_create_without_device_reports_hip_error():
    st, msg = kpsi.create_status(0, kpsi.FP64)
    assert st == kpsi.KPSI_E_HIP
    assert "device" in msg


def test_create_rejects_bad_precision():
    st, msg = kpsi.create_status(0, 7)
    assert st in (kpsi.KPSI_E_ARG, kpsi.KPSI_E_HIP)


STRUCTS = [("kpsi_kinematics", "Kinematics"), ("kpsi_resonance", "Resonance"),
           ("kpsi_fit_options", "FitOptions"), ("kpsi_fit_result", "FitResult"), ("kpsi_peaks", "Peaks"),
           ("kpsi_mlp_options", "MlpOptions")]


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct the binding passes by pointer has the size and field offsets the header
    gives it (a C program compiled against include/kpsi.h prints them)."""
    import ctypes as C
    import subprocess
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "kpsi.h"', "int main(void) {"]
    for cname, pyname in STRUCTS:
        py = getattr(kpsi, pyname)
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (l.split() for l in out if l)}
    for cname, pyname in STRUCTS:
        py = getattr(kpsi, pyname)
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
