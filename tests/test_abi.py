"""The C-ABI library loads and exports every entry point its header declares (no GPU;
no compute calls).  The binding rejects host tensors before any call reaches HIP."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mjh.h")
LIB = os.path.join(ROOT, "paper_2502_08844_amd", "libmjh.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mjh_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mjh_model_upload", "mjh_world_alloc", "mjh_step", "mjh_rollout_fwd",
                     "mjh_rollout_bwd", "mjh_graph_capture", "mjh_autotune"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmjh.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmjh.so not built")
def test_binding_rejects_host_tensors():
    import torch
    from paper_2502_08844_amd import mjh
    with pytest.raises(ValueError):
        mjh._ptr(torch.zeros(3))
    with pytest.raises(ValueError):
        mjh._ptr(torch.zeros(3, dtype=torch.float64))


def test_reference_exports():
    import oracle
    lib = ctypes.CDLL(oracle.lib_path())
    for n in ("mjo_load", "mjo_step", "mjo_forward", "mjo_rollout_loss", "mjo_rollout_jvp",
              "mjo_count_flops"):
        assert hasattr(lib, n)
