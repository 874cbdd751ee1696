"""Host-side checks of libpic.so that need no GPU: the library loads and exports
every function include/pic.h declares, and the host-only paths (argument
validation, sizes, the c_att calibration) behave."""
import ctypes as C
import os
import re

import pytest

from paper_1502_07722_amd import binding as B
from paper_1502_07722_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(pic_\w+)\s*\(", txt, flags=re.M))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("pic_init", "pic_deposit", "pic_force", "pic_push", "pic_step", "pic_workspace_bytes",
                 "pic_destroy", "pic_last_error", "pic_sync", "pic_kick", "pic_calibrate_catt"):
        assert must in names


@pytest.mark.parametrize("name", declared_functions())
def test_library_exports_every_declared_symbol(name):
    assert hasattr(B.lib, name), name


def test_sizes():
    g = W.Grid(ndim=2, n=(64, 64), h=(2e-9, 2e-9), bc=(0, 1))
    assert B.pic_num_nodes(g) == 64 * 65
    g3 = W.Grid(ndim=3, n=(8, 9, 10), h=(2e-9,) * 3, bc=(0, 0, 1))
    assert B.pic_num_nodes(g3) == 8 * 9 * 11
    assert B.pic_workspace_bytes(g, 1000) > 64 * 65 * 12
    assert B.pic_workspace_bytes(g, 2_000_000) > B.pic_workspace_bytes(g, 1000)


def test_invalid_grids_are_rejected():
    bad = [W.Grid(ndim=4, n=(4, 4), h=(1e-9, 1e-9), bc=(0, 0)),
           W.Grid(ndim=2, n=(0, 4), h=(1e-9, 1e-9), bc=(0, 0)),
           W.Grid(ndim=2, n=(4, 4), h=(-1e-9, 1e-9), bc=(0, 0)),
           W.Grid(ndim=2, n=(4, 4), h=(1e-9, 1e-9), bc=(2, 0)),
           W.Grid(ndim=2, n=(1 << 16, 1 << 16), h=(1e-9, 1e-9), bc=(0, 0))]
    for g in bad:
        assert B.pic_num_nodes(g) == 0
        assert B.pic_workspace_bytes(g, 10) == 0


def _init(grid, pot, dt=1e-15, max_n=10, ws=None, nbytes=0):
    ctx = C.c_void_p()
    rc = B.lib.pic_init(C.byref(ctx), C.byref(B.grid_t(grid)), C.byref(B.potential_t(pot)), dt, max_n,
                        C.c_void_p(ws) if ws else None, nbytes, None)
    return rc, ctx


def test_pic_init_rejects_bad_arguments_before_touching_the_device():
    g = W.Grid(ndim=2, n=(8, 8), h=(2e-9, 2e-9), bc=(0, 1))
    pot = W.Potential()
    assert _init(W.Grid(ndim=2, n=(0, 8), h=(2e-9, 2e-9), bc=(0, 1)), pot)[0] == B.PIC_EINVAL
    assert _init(g, W.Potential(g_clamp=2.5))[0] == B.PIC_EINVAL
    assert _init(g, W.Potential(D=-1.0))[0] == B.PIC_EINVAL
    assert _init(g, pot, dt=0.0)[0] == B.PIC_EINVAL
    assert _init(g, pot, max_n=-1)[0] == B.PIC_EINVAL
    assert _init(g, pot)[0] == B.PIC_ENOSPACE                      # no workspace
    assert _init(g, pot, ws=4096, nbytes=16)[0] == B.PIC_ENOSPACE  # too small
    n = B.pic_workspace_bytes(g, 10)
    assert _init(g, pot, ws=4096 + 8, nbytes=n)[0] == B.PIC_EINVAL  # misaligned


def test_null_context_calls_fail_cleanly():
    s = B.pic_particles_t(0, None, None, None, None)
    assert B.lib.pic_deposit(None, C.byref(s), None) == B.PIC_EINVAL
    assert B.lib.pic_step(None, C.byref(s), 1, None, 0) == B.PIC_EINVAL
    assert B.lib.pic_sync(None) == B.PIC_EINVAL
    assert B.lib.pic_set_record_states(None, 1) == B.PIC_EINVAL
    assert B.lib.pic_record_bytes(None, 10, 2) == 0
    assert B.lib.pic_backward_bytes(None, 2) == 0
    assert B.lib.pic_last_error(None) == b"context is NULL"


@pytest.mark.parametrize("h_nm,layers", [(2.0, 8), (2.0, 12), (1.0, 8), (4.0, 6)])
def test_library_calibration_matches_oracle(oracle_lib, h_nm, layers):
    """Two independent implementations of the correction-factor calibration
    (library: analytic lattice profile + adaptive Simpson; oracle: literal
    lattice deposit + adaptive Gauss-Legendre) must agree."""
    O = oracle_lib
    g = W.Grid(ndim=2, n=(8, 8), h=(h_nm * 1e-9,) * 3, bc=(0, 1))
    pot = W.Potential(s_rep=1.5)
    c_lib, w_lib = B.pic_calibrate_catt(g, pot, W.N_SOLID, layers)
    c_orc, w_orc, _ = O.calibrate_catt(g, pot, W.N_SOLID, slab_layers=layers, lattice_k=2)
    assert c_lib == pytest.approx(c_orc, rel=1e-9, abs=0)
    assert w_lib == pytest.approx(w_orc, rel=1e-9, abs=0)
