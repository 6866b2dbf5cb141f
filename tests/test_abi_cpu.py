"""CPU checks of the C ABI: the library loads without a GPU and exports every
entry point include/vhpd.h declares; the binding's signature table matches."""

import os
import re

import pytest

from paper_2405_12484_amd import vhpd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vhpd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vh_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("vh_ctx_create", "vh_mesh_create", "vh_mesh_set_params", "vh_mesh_prefactor",
                 "vh_mesh_step", "vh_mesh_read_state", "vh_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = vhpd.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_header():
    assert sorted(vhpd.SIGNATURES) == _declared()


def test_no_device_is_reported_as_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(vhpd.VHError) as ei:
        vhpd.Context(0)
    assert ei.value.code in (vhpd.VH_EDEVICE, vhpd.VH_EINVAL)
