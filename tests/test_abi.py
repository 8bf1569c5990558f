"""Host-side checks of the C ABI: the library loads, exports every declared
entry point, and rejects invalid grids before touching the GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tc.h")
LIB = os.path.join(ROOT, "paper_1311_2481_amd", "libtc.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(tc_[a-z_]+)\s*\(", text)))


needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libtc.so not built")


@needs_lib
def test_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (tc_\w+)", out))
    missing = [s for s in declared() if s not in exported]
    assert not missing, missing
    assert len(declared()) >= 15


@needs_lib
def test_binding_covers_header():
    import paper_1311_2481_amd as pkg
    assert sorted(pkg.EXPORTS) == declared()


@needs_lib
@pytest.mark.parametrize("field,value,msg", [
    ("m_z", 31, "even m_z"),
    ("n_s", 7, "n_s = 9"),
    ("p_theta", 40, "3/2 rule"),
    ("p_z", 24, "3/2 rule"),
    ("n_r", 5, "n_r"),
    ("precision", 7, "precision"),
])
def test_init_rejects_invalid_grid(field, value, msg):
    import paper_1311_2481_amd as pkg
    lib = pkg.load_library()
    g = pkg._Grid(32, 16, 32, 0, 0, 1.0, 1.0, 0.0, 9, 0)
    setattr(g, field, value)
    ctx = ctypes.c_void_p()
    st = lib.tc_init(ctypes.byref(g), 0.5, 100.0, 0.0, 1e-3, None, ctypes.byref(ctx))
    assert st == pkg.TC_EINVAL
    assert ctx.value is None
    assert msg in lib.tc_last_error(None).decode()


@needs_lib
def test_init_rejects_unsupported_transform_length():
    import paper_1311_2481_amd as pkg
    lib = pkg.load_library()
    g = pkg._Grid(32, 16, 32, 49, 0, 1.0, 1.0, 0.0, 9, 0)
    ctx = ctypes.c_void_p()
    assert lib.tc_init(ctypes.byref(g), 0.5, 100.0, 0.0, 1e-3, None, ctypes.byref(ctx)) == pkg.TC_EINVAL
    for bad in (dict(eta=1.5), dict(dt=0.0)):
        args = dict(eta=0.5, dt=1e-3)
        args.update(bad)
        g = pkg._Grid(32, 16, 32, 0, 0, 1.0, 1.0, 0.0, 9, 0)
        assert lib.tc_init(ctypes.byref(g), args["eta"], 100.0, 0.0, args["dt"], None, ctypes.byref(ctx)) == pkg.TC_EINVAL


@needs_lib
def test_solver_needs_gpu_and_fails_loudly():
    import torch
    import paper_1311_2481_amd as pkg
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError, match="GPU"):
        pkg.Solver(32, 16, 32, 0.5, 100.0, 0.0, 1e-3)
