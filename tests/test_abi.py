"""CPU checks of the C-ABI library: it loads, exports every entry point the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2501_12349_amd import fpts
    if not os.path.exists(fpts.LIB_PATH):
        from paper_2501_12349_amd import build
        build.build()
    return fpts, fpts.load_library()


def _declared(header="fpts.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fpts_\w+)\s*\(", src)))


def test_header_declares_the_binding_exports():
    fpts, _ = _lib()
    assert _declared() == sorted(fpts.EXPORTS)
    assert _declared("fpts_serve.h") == sorted(fpts.SERVE_EXPORTS)
    assert _declared("fpts_lpt.h") == sorted(fpts.LPT_EXPORTS)


def test_library_exports_every_declared_symbol():
    _, L = _lib()
    for name in _declared() + _declared("fpts_serve.h") + _declared("fpts_lpt.h"):
        assert hasattr(L, name), name


def test_defaults_and_status_strings():
    fpts, L = _lib()
    p = fpts.Params()
    L.fpts_params_default(ctypes.byref(p), 3, 3, 8, 1000)
    assert (p.dim, p.ref_dim, p.nodes_1d, p.n_elem) == (3, 3, 8, 1000)
    assert p.bbox_tol == 0.1 and p.max_iter == 50 and p.newton_tol == 1e-10
    assert p.mixed_max_iter == 10 and p.mixed_tol == 1e-3
    assert p.surf_eps_d == 1e-10 and p.hash_n == 0
    assert L.fpts_status_string(0) == b"ok"
    assert L.fpts_status_string(-1) == b"invalid argument"


@pytest.mark.parametrize("dim,ref_dim,N,nel", [(1, 1, 4, 10), (3, 4, 4, 10), (2, 3, 4, 10),
                                               (3, 3, 1, 10), (3, 3, 11, 10), (3, 3, 4, 0)])
def test_setup_rejects_bad_params_without_device(dim, ref_dim, N, nel):
    fpts, L = _lib()
    p = fpts.Params()
    L.fpts_params_default(ctypes.byref(p), dim, ref_dim, N, nel)
    buf = (ctypes.c_double * 16)()
    h = ctypes.c_void_p()
    assert L.fpts_setup(ctypes.byref(p), buf, None, ctypes.byref(h)) == -1
    assert not h.value


def test_null_handles_are_rejected():
    _, L = _lib()
    assert L.fpts_find(None, 10, None, None, None, None, None, 0, None, 0, None) == -1
    assert L.fpts_eval(None, 10, None, None, None, 1, None, None, None, 0, None) == -1
    assert L.fpts_find_workspace_size(None, 10) == 0
    assert L.fpts_destroy(None) == 0


@pytest.mark.parametrize("budget,streams,maxb", [(1 << 10, 2, 1000), (1 << 30, 0, 1000),
                                                 (1 << 30, 17, 1000), (1 << 30, 2, 0)])
def test_server_rejects_bad_arguments_without_device(budget, streams, maxb):
    _, L = _lib()
    h = ctypes.c_void_p()
    assert L.fpts_server_create(budget, streams, maxb, ctypes.byref(h)) == -1
    assert not h.value
    assert L.fpts_server_destroy(None) == 0
    assert L.fpts_server_submit(None, 0, 10, None, None, None, None, None, None, 0, None,
                                None) == -1


def test_lpt_rejects_bad_arguments_without_device():
    fpts, L = _lib()
    p = fpts.LptParams()
    p.tau, p.dt = 5.0, 1e-3
    assert L.fpts_lpt_workspace_size(None, 10) == 0
    args = [1, None, None, None, None, None, None, None, None, 0, None, 0, None]
    assert L.fpts_lpt_step(None, ctypes.byref(p), 10, *args) == -1
    assert L.fpts_lpt_step(None, None, 10, *args) == -1
