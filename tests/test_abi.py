"""The C-ABI library loads and exports every function include/tcm.h declares (no GPU
needed: nothing is computed), the binding's request record matches the C layout, and the
build compiles every HIP source for gfx950."""
import ctypes as C
import os

import pytest

from paper_0704_1672_amd import tcm


def test_library_exports_every_header_symbol():
    lib = C.CDLL(tcm.LIB_PATH)
    names = tcm.header_symbols()
    assert "tcm_moments" in names and "tcm_pair_energy" in names and "tcm_batch_energy" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    assert set(tcm.header_symbols()) <= set(tcm._SIGS), set(tcm.header_symbols()) - set(tcm._SIGS)


def test_request_layout():
    assert C.sizeof(tcm.tcm_pair_req) == 8 + 8 + 24 + 32 + 4 + 4
    assert tcm.PAIR_REQ_DTYPE.itemsize == C.sizeof(tcm.tcm_pair_req)


def test_strerror_without_device():
    assert tcm.tcm_strerror(tcm.TCM_EDOMAIN).startswith("separation condition")
    assert tcm.tcm_strerror(12345) == "unknown status"


def test_create_rejects_missing_device():
    # no GPU in a CPU-only container: context creation reports a device error, never crashes
    if os.environ.get("HIP_VISIBLE_DEVICES", None) == "" or not os.path.exists("/dev/kfd"):
        with pytest.raises(tcm.TCMError) as e:
            tcm.tcm_create(0)
        assert e.value.code in (tcm.TCM_EDEVICE,)
    with pytest.raises(tcm.TCMError):
        tcm.tcm_create(10_000)


def test_make_requests_broadcasts_scalars_and_rows():
    import numpy as np
    R = np.arange(48, dtype=float).reshape(16, 3)
    req = tcm.make_requests(7, 9, R, 12)                       # one pair of molecules, many R
    assert len(req) == 16 and np.all(req["a"] == 7) and np.all(req["b"] == 9)
    assert np.array_equal(req["R"], R) and np.all(req["L"] == 12) and np.all(req["quat_b"][:, 0] == 1.0)
    q = np.tile([0.5, 0.5, 0.5, 0.5], (5, 1))
    req = tcm.make_requests([1, 2, 3, 4, 5], 0, [1.0, 2.0, 3.0], [8, 8, 16, 16, 20], q, flags=tcm.TCM_REUSE)
    assert len(req) == 5 and np.all(req["R"] == [1.0, 2.0, 3.0]) and np.array_equal(req["quat_b"], q)
    assert np.all(req["flags"] == tcm.TCM_REUSE) and list(req["L"]) == [8, 8, 16, 16, 20]
    with pytest.raises(ValueError):
        tcm.make_requests([1, 2, 3], 0, np.zeros((2, 3)), 8)  # incompatible lengths


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU: asked for more it says so and exits non-zero, before
    touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU only" in (r.stdout + r.stderr)
