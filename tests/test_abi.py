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
