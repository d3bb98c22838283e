"""CPU checks of the boundary: the HIP library loads and exports every symbol
its header declares; host-side argument validation (no device work)."""
import ctypes
import os
import re

import pytest

from paper_2602_14667_amd import rrmhd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", fn)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(rrmhd_\w+)\s*\(", txt):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_symbols()
    for core in ("rrmhd_create", "rrmhd_init", "rrmhd_step", "rrmhd_moments",
                 "rrmhd_diagnostics"):
        assert core in names


def test_library_exports_every_declared_symbol():
    L = rrmhd.lib()
    missing = [n for n in declared_symbols() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    assert set(declared_symbols()) <= set(rrmhd.EXPORTED) | {
        n for n in declared_symbols() if n.startswith("rrmhd_batch")
        or n.startswith("rrmhd_closure") or n.startswith("rrmhd_tune")}


def test_strerror_without_device():
    L = rrmhd.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.rrmhd_strerror(code)
    assert L.rrmhd_strerror(-6) != L.rrmhd_strerror(-99)


@pytest.mark.parametrize("args", [
    dict(nx=0, ny=4, tau_f=0.6, tau_m=0.6),
    dict(nx=4, ny=4, tau_f=0.5, tau_m=0.6),
    dict(nx=4, ny=4, tau_f=0.6, tau_m=0.4),
    dict(nx=4, ny=4, tau_f=float("nan"), tau_m=0.6),
    dict(nx=4, ny=1, tau_f=0.6, tau_m=0.6, walls=True),
])
def test_create_rejects_bad_arguments_before_touching_the_device(args):
    L = rrmhd.lib()
    g = rrmhd.Grid(args["nx"], args["ny"], 0, 0.0)
    bc = rrmhd.BC(1 if args.get("walls") else 0)
    h = ctypes.c_void_p(1234)
    rc = L.rrmhd_create(ctypes.byref(g), args["tau_f"], args["tau_m"],
                        ctypes.byref(bc), None, ctypes.byref(h))
    assert rc == rrmhd.EINVAL
    assert not h.value


@pytest.mark.parametrize("nx,ny,storage", [(32768, 32768, 0), (65536, 16384, 0),
                                            (65536, 32768, 1), (46341, 46341, 1)])
def test_create_rejects_planes_of_4_gib(nx, ny, storage):
    """In-plane offsets are 32-bit byte offsets: a plane of 2^32 bytes or
    more is refused before any allocation."""
    L = rrmhd.lib()
    g = rrmhd.Grid(nx, ny, storage, 0.0)
    h = ctypes.c_void_p(1234)
    assert L.rrmhd_create(ctypes.byref(g), 0.6, 0.6, None, None,
                          ctypes.byref(h)) == rrmhd.EINVAL
    assert not h.value


def test_create_rejects_non_power_of_two_scale():
    L = rrmhd.lib()
    g = rrmhd.Grid(4, 4, 1, 3.0)
    h = ctypes.c_void_p()
    assert L.rrmhd_create(ctypes.byref(g), 0.6, 0.6, None, None,
                          ctypes.byref(h)) == rrmhd.EINVAL


def test_null_handle_calls_are_rejected():
    L = rrmhd.lib()
    assert L.rrmhd_step(None, 1) == rrmhd.EINVAL
    assert L.rrmhd_init(None, None, None) == rrmhd.EINVAL
    assert L.rrmhd_destroy(None) == rrmhd.OK
    assert L.rrmhd_batch_set_fetch(None, 1) == rrmhd.EINVAL
    assert L.rrmhd_batch_set_shape(None, -1, 0, 0, -1) == rrmhd.EINVAL
    assert L.rrmhd_batch_step(None, 1) == rrmhd.EINVAL
    # training entry points: argument checks come before any device work
    assert L.rrmhd_train_onestep_samples(None, None, None, None, None, None, 64, 4,
                                         0.55, None, None, None, None, None) == rrmhd.EINVAL
    assert L.rrmhd_train_onestep_loss_grad(None, None, None, None, None, 1, 16, 0.55,
                                           1.0, 0, None, None) == rrmhd.EINVAL
    assert L.rrmhd_train_samples(None, None, None, 64, 4, 0.55, None, None, None,
                                 None) == rrmhd.EINVAL
    assert L.rrmhd_closure_enable(None, 1) == rrmhd.EINVAL
    assert L.rrmhd_autotune(None, None, 3, None, None, None, None) == rrmhd.EINVAL
    assert L.rrmhd_save(None, b"/nonexistent/x.ck") == rrmhd.EINVAL
    assert L.rrmhd_load(None, b"/nonexistent/x.ck") == rrmhd.EINVAL


def test_create_rejects_unknown_storage_flags():
    L = rrmhd.lib()
    for storage in (0x400, 0x101 | 0x400, 3, 0x104, 0x800 | 0x200):  # 0x104: unknown kind with one buffer
        g = rrmhd.Grid(4, 4, storage, 0.0)
        h = ctypes.c_void_p()
        assert L.rrmhd_create(ctypes.byref(g), 0.6, 0.6, None, None,
                              ctypes.byref(h)) == rrmhd.EINVAL
        assert not h.value


@pytest.mark.parametrize("args", [
    (0, 4, 4, 0), (4, 4, 0, 0), (4, 70000, 2, 0), (4, 2, 70000, 0), (4, 4, 4, 2),
    (4, 4, 4, 0x200), (4, 4, 4, 0x102), (2048, 2048, 256, 0x100),
    (2048, 2048, 256, 0),  # 2^30 nodes x 4 B does not fit 32-bit offsets
])
def test_create3d_rejects_bad_arguments_before_touching_the_device(args):
    L = rrmhd.lib()
    nx, ny, nz, storage = args
    h = ctypes.c_void_p(1234)
    rc = L.rrmhd3d_create(nx, ny, nz, storage, 0.6, 0.6, None, ctypes.byref(h))
    assert rc == rrmhd.EINVAL
    assert not h.value


def test_create3d_rejects_bad_relaxation_times():
    L = rrmhd.lib()
    for tf, tm in ((0.5, 0.6), (0.6, 0.5), (float("nan"), 0.6)):
        h = ctypes.c_void_p()
        assert L.rrmhd3d_create(4, 4, 4, 0, tf, tm, None, ctypes.byref(h)) == rrmhd.EINVAL


def test_null_3d_handle_calls_are_rejected():
    L = rrmhd.lib()
    assert L.rrmhd3d_step(None, 1) == rrmhd.EINVAL
    assert L.rrmhd3d_init(None, None, None) == rrmhd.EINVAL
    assert L.rrmhd3d_moments(None, None, None, None) == rrmhd.EINVAL
    assert L.rrmhd3d_set_launch(None, 64, 4, 0) == rrmhd.EINVAL
    assert L.rrmhd3d_destroy(None) == rrmhd.OK
