"""The C-ABI library: it loads, exports every entry point include/ibm.h
declares, and validates arguments on the host before any GPU call (these tests
make no compute call and need no GPU)."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2402_17337_amd import ibm
from paper_2402_17337_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibm.h")


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(ibm.LIB_PATH):
        from paper_2402_17337_amd import build
        build.build(force=True)
    yield


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ibm_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", ibm.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(ibm_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = ibm.lib()
    for n in names:
        assert hasattr(L, n)
    assert set(ibm.EXPORTED) == set(names)


def test_library_is_built_for_gfx950():
    # the offload bundle of the device code names its target
    data = open(ibm.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


def test_struct_layouts_match_header():
    # field order and sizes of the mirrored structs (the header is the contract)
    import ctypes as C
    assert C.sizeof(ibm.Params) == 4 * 4 + 10 * 8 + 4 * 4 + 4 * 8 + 2 * 4 + 8 + 2 * 4
    assert C.sizeof(ibm.StepStats) == 8 * 4 + 7 * 8
    assert C.sizeof(ibm.SolveOpts) == 4 * 4 + 2 * 8
    assert C.sizeof(ibm.SolveStats) == 4 * 4 + 3 * 8


def test_workspace_bytes_is_pure_and_scales():
    a = ibm.workspace_bytes(128, 96)
    b = ibm.workspace_bytes(1024, 768)
    assert a > 0 and b > 50 * a
    assert b % 256 == 0
    # about 33 doubles per cell at the plunging 1024x768 workload (fields,
    # solver vectors, split copies, network maps)
    assert 25 * 8 * 1024 * 768 < b < 40 * 8 * 1024 * 768
    assert ibm.workspace_bytes(127, 96) == 0
    assert ibm.workspace_bytes(6, 96) == 0


def test_status_strings():
    for s in (ibm.OK, ibm.NOT_CONVERGED, ibm.ERR_INVALID, ibm.ERR_HIP, ibm.ERR_NAN):
        assert ibm.status_string(s) and ibm.status_string(s) != "unknown status"
    assert ibm.status_string(12345) == "unknown status"


@pytest.mark.parametrize("bad", [
    dict(nx=127),                       # odd
    dict(dt=0.0), dict(re=-1.0),
    dict(p_omega=2.0), dict(uv_omega=0.0),
    dict(p_max_iter=0), dict(p_check=0),
    dict(bc=1),                         # periodic mode takes no body
    dict(bc=1, body=0, p_method=2),     # ... and no mixed-precision sweeps
    dict(bc=2),                         # unknown boundary mode
    dict(y0=0.1),                       # body outside the interior
    dict(amp=5.9),                      # plunge range leaves the domain
    dict(p_method=7),
])
def test_init_rejects_invalid_parameters_before_any_gpu_call(bad):
    nx = bad.pop("nx", 128)
    ny = 96
    xf, yf = W.uniform_faces(nx, 16.0), W.uniform_faces(ny, 12.0)
    # a NULL workspace: validation of the parameters comes first either way
    assert ibm.init_status(nx, ny, xf, yf, workspace_ptr=0, **bad) == ibm.ERR_INVALID


def test_init_rejects_non_increasing_faces():
    xf, yf = W.uniform_faces(64, 8.0), W.uniform_faces(48, 6.0)
    xf[10] = xf[9]
    assert ibm.init_status(64, 48, xf, yf, workspace_ptr=0, x0=4.0, y0=3.0) == ibm.ERR_INVALID


def test_init_rejects_small_or_misaligned_workspace():
    xf, yf = W.uniform_faces(64, 8.0), W.uniform_faces(48, 6.0)
    need = ibm.workspace_bytes(64, 48)
    assert ibm.init_status(64, 48, xf, yf, workspace_ptr=0, x0=4.0, y0=3.0) == ibm.ERR_INVALID
    assert ibm.init_status(64, 48, xf, yf, workspace_ptr=1 << 20, workspace_bytes_=need - 256,
                           x0=4.0, y0=3.0) == ibm.ERR_INVALID
    assert ibm.init_status(64, 48, xf, yf, workspace_ptr=(1 << 20) + 8, workspace_bytes_=need,
                           x0=4.0, y0=3.0) == ibm.ERR_INVALID


def test_binding_refuses_to_run_without_a_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    c = W.small_plunging()
    with pytest.raises(RuntimeError):
        ibm.Solver(c["nx"], c["ny"], c["xf"], c["yf"], **c["params"])


def test_batched_workload_recipe():
    # the many-case workload: seeded, 64 cases, sizes and parameters in range,
    # core spacing whole in both directions, about 21 M cells in all
    a = W.batched_plunging(8, 0)
    b = W.batched_plunging(8, 0)
    assert [c["nx"] for c in a] == [c["nx"] for c in b]
    for c in a:
        assert c["nx"] % 32 == 0 and 256 <= c["nx"] <= 1024 and c["ny"] == 3 * c["nx"] // 4
        p = c["params"]
        assert 0.2 <= p["amp"] <= 0.8 and 0.2 <= p["freq"] <= 0.6 and p["re"] in (100.0, 300.0, 500.0)
        assert len(c["xf"]) == c["nx"] + 1 and np.all(np.diff(c["xf"]) > 0)
        assert ibm.workspace_bytes(c["nx"], c["ny"]) > 0


def test_batch_entry_points_reject_null_handles():
    import ctypes as C
    L = ibm.lib()
    assert L.ibm_batch_set_graph(None, 2) == ibm.ERR_INVALID
    assert L.ibm_batch_step(None, 1, None) == ibm.ERR_INVALID
    out = C.c_void_p()
    assert L.ibm_batch_create(0, None, C.byref(out)) == ibm.ERR_INVALID and not out.value


def test_benchmark_refuses_more_than_one_gpu():
    # one GPU only: the refusal comes before anything touches a device
    r = subprocess.run(["python", os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stdout
