"""The warm-start network's C ABI (include/ibm_unet.h): every declared entry
point is exported, the parameter layout matches the network the oracle
defines, and shapes and workspaces are validated on the host before any GPU
call (no compute call, no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from oracle import unet as OU
from paper_2402_17337_amd import ibm
from paper_2402_17337_amd import unet as U

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibm_unet.h")


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(ibm.LIB_PATH):
        from paper_2402_17337_amd import build
        build.build(force=True)
    yield


def test_every_declared_symbol_is_exported():
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(ibm_unet_[a-z0-9_]+)\s*\(", txt)))
    assert len(names) == len(U.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", ibm.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(ibm_unet_\w+)", out))
    assert not [n for n in names if n not in exported]
    assert set(U.EXPORTED) == set(names)


def test_layers_and_parameter_count_match_the_oracle_network():
    specs = [(n, ci, co, r) for n, ci, co, r in OU.layer_specs()]
    assert specs == U.LAYERS
    p = OU.init_params(0)
    n = sum(v.size for v in p.values())
    assert U.param_count() == n
    vec = U.flatten_params(p)
    assert vec.size == n
    back = U.unflatten_params(vec)
    for k in p:
        assert back[k].shape == p[k].shape


def test_workspace_bytes_validates_shapes():
    L = U.lib()
    assert L.ibm_unet_workspace_bytes(1, 768, 1024) > 0
    assert L.ibm_unet_workspace_bytes(16, 256, 256) % 256 == 0
    for b, h, w in ((0, 64, 64), (1, 60, 64), (1, 64, 96), (1, 4, 64), (1, 64, 32)):
        assert L.ibm_unet_workspace_bytes(b, h, w) == 0
    # about 120 bf16 activations per pixel at level 0, plus gradients
    b = L.ibm_unet_workspace_bytes(1, 768, 1024)
    assert 300 * 768 * 1024 < b < 1500 * 768 * 1024


def test_create_rejects_bad_workspaces_before_any_gpu_call():
    L = U.lib()
    h = C.c_void_p()
    need = L.ibm_unet_workspace_bytes(1, 64, 64)
    assert L.ibm_unet_create(1, 64, 64, None, need, None, C.byref(h)) == ibm.ERR_INVALID
    assert L.ibm_unet_create(1, 64, 64, C.c_void_p(256), need - 1, None, C.byref(h)) == ibm.ERR_INVALID
    assert L.ibm_unet_create(1, 64, 64, C.c_void_p(257), need, None, C.byref(h)) == ibm.ERR_INVALID
    assert L.ibm_unet_create(1, 64, 48, C.c_void_p(256), need, None, C.byref(h)) == ibm.ERR_INVALID
    assert not h.value


def test_conv_layer_validation():
    L = U.lib()
    assert L.ibm_unet_conv_workspace_bytes(1, 5, 8, 3, 1) > 0
    assert L.ibm_unet_conv_workspace_bytes(1, 5, 12, 3, 1) == 0
    assert L.ibm_unet_conv_workspace_bytes(1, 5, 8, 0, 1) == 0
    assert L.ibm_unet_conv_workspace_bytes(1, 5, 8, 3, 257) == 0
    need = L.ibm_unet_conv_workspace_bytes(1, 5, 8, 3, 1)
    # missing operands are rejected before anything is enqueued
    assert L.ibm_unet_conv3x3(0, 1, 5, 8, 3, 1, None, C.c_void_p(256), None, None, C.c_void_p(256),
                              C.c_void_p(256), need, None) == ibm.ERR_INVALID
    assert L.ibm_unet_conv3x3(3, 1, 5, 8, 3, 1, C.c_void_p(256), C.c_void_p(256), None, C.c_void_p(256),
                              C.c_void_p(256), C.c_void_p(256), need, None) == ibm.ERR_INVALID
