"""The C-ABI library loads and exports every symbol its header declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "microcosm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_[a-z_0-9]+)\s*\(", text)))


def _lib():
    from paper_2607_02954_amd import sim
    if not os.path.exists(sim.LIB_PATH):
        pytest.skip("libmicrocosm.so not built")
    return sim


def test_every_declared_symbol_is_exported():
    sim = _lib()
    L = sim.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(sim.EXPORTS)


def test_host_only_queries():
    sim = _lib()
    L = sim.lib()
    p = sim.SimParams()
    L.sim_params_default(ctypes.byref(p), 64, 48)
    assert (p.nx, p.ny, p.pbd_iters, p.repulse_radius) == (64, 48, 4, 4)
    assert abs(p.tau - 1.0) < 1e-7 and abs(p.trt_magic - 0.25) < 1e-7
    n = ctypes.c_size_t()
    assert L.sim_workspace_size(ctypes.byref(p), 3, 40, ctypes.byref(n)) == 0
    assert n.value >= 9 * 64 * 48 * 4
    p.flags = sim.SIM_SPLAT_SORTED
    m = ctypes.c_size_t()
    assert L.sim_workspace_size(ctypes.byref(p), 3, 40, ctypes.byref(m)) == 0
    bad = sim.SimParams()
    L.sim_params_default(ctypes.byref(bad), 64, 48)
    bad.tau = 0.4
    assert L.sim_workspace_size(ctypes.byref(bad), 3, 40, ctypes.byref(n)) == sim.SIM_E_INVALID
    assert b"tau" in L.sim_last_error()
    bad.tau = 1.0
    bad.repulse_radius = 9
    assert L.sim_workspace_size(ctypes.byref(bad), 3, 40, ctypes.byref(n)) == sim.SIM_E_INVALID
    w = ctypes.c_size_t()
    L.sim_params_default(ctypes.byref(p), 128, 128)
    assert L.sim_batch_world_bytes(ctypes.byref(p), 4, 100, ctypes.byref(w)) == 0
    assert w.value > 9 * 2 * 128 * 128 * 4


def test_params_mirror_matches_header_defaults():
    sim = _lib()
    L = sim.lib()
    p = sim.SimParams()
    L.sim_params_default(ctypes.byref(p), 32, 32)
    q = sim.Params(nx=32, ny=32).c()
    for name, _ in sim.SimParams._fields_:
        assert abs(getattr(p, name) - getattr(q, name)) < 1e-7, name


def test_noalloc_size_limit_checked_on_host():
    """sim_step_noalloc refuses a world larger than its static scratch before
    touching the device (the pointers are never dereferenced)."""
    sim = _lib()
    L = sim.lib()
    p = sim.SimParams()
    L.sim_params_default(ctypes.byref(p), 2048, 2048)
    fake = ctypes.c_void_p(256)
    a = sim.SimArrays(1, 16, fake, fake, fake, fake, fake, fake, fake, fake, fake, fake)
    st = L.sim_step_noalloc(ctypes.byref(p), ctypes.byref(a), 0, None, None)
    assert st == sim.SIM_E_WORKSPACE
    assert b"scratch" in L.sim_last_error()
    p.tau = 0.4
    assert L.sim_step_noalloc(ctypes.byref(p), ctypes.byref(a), 0, None, None) == sim.SIM_E_INVALID
