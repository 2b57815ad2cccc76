"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/nbody.h declares, rejects bad arguments with the
documented codes before touching a device, and its host copy of the block
step rule is bit-exact against the oracle's integer rule."""
import json
import math
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_0707_0438_amd as nb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")
GRAPE_HEADER = os.path.join(ROOT, "include", "nbody_grape.h")


def declared_functions(header=None):
    names = set()
    for h in ([header] if header else [HEADER, GRAPE_HEADER]):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(nbody_[a-z_0-9]+|GPU[A-Za-z_0-9]*)\s*\(", src))
    return sorted(names)


def test_header_declarations_match_binding_list():
    assert declared_functions(HEADER) == sorted(nb.EXPORTS)
    assert declared_functions(GRAPE_HEADER) == sorted(nb.GRAPE_EXPORTS)


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", nb.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [f for f in declared_functions() if f not in syms]
    assert not missing, missing
    L = nb.lib()
    for f in declared_functions():
        assert hasattr(L, f)
    assert L.nbody_abi_version() == 1


@pytest.fixture()
def hostctx():
    c = nb.Context(-1)
    yield c
    c.close()


def _src(p=8):
    return nb.Src(*([p] * 7))


def _out(p=8):
    return nb.Out(*([p] * 7))


def test_force_argument_errors(hostctx):
    L = nb.lib()
    h = hostctx.handle
    call = lambda **kw: L.nbody_force(h, None, kw.get("prec", 1), kw.get("G", 1.0), kw.get("eps", 0.1),
                                      kw.get("ni", 10), kw.get("I", _src()), kw.get("iself"),
                                      kw.get("nj", 10), kw.get("J", _src()), kw.get("out", _out()))
    assert call(ni=-1) == -1
    assert call(nj=-1) == -1
    assert call(ni=1 << 31) == -1
    assert call(eps=-0.5) == -1
    assert call(eps=float("nan")) == -1
    assert call(eps=float("inf")) == -1
    assert call(G=float("inf")) == -1
    assert call(prec=7) == -1
    bad = _src(); bad.vz = None
    assert call(I=bad) == -1
    assert "row 5 is NULL" in hostctx.last_error()
    mis = _src(); mis.y = 12
    assert call(J=mis) == -1
    assert "aligned" in hostctx.last_error()
    nom = _src(); nom.m = None
    assert call(J=nom) == -1                  # j masses are required
    assert call(I=nom) == -4                  # i masses are not: reaches the device check
    o = _out(); o.pot = None
    assert call(out=o) == -1
    assert call(ni=3, nj=0, iself=8) == -1    # self indices into an empty j set
    # well-formed call on a context without a device
    assert call() == -4
    assert "no device" in hostctx.last_error()


def test_force_acc_nn_leapfrog_argument_errors(hostctx):
    L = nb.lib()
    h = hostctx.handle
    novel = nb.Src(8, 8, 8, None, None, None, 8)
    out3 = nb.Out(8, 8, 8, None, None, None, 8)
    acc = lambda **kw: L.nbody_force_acc(h, None, 1, 1.0, kw.get("eps", 0.1), kw.get("ni", 10),
                                         kw.get("I", novel), None, 10, kw.get("J", novel),
                                         kw.get("out", out3))
    # the force-only evaluation needs neither velocities nor jerk rows
    assert acc() == -4
    assert acc(eps=-1.0) == -1 and acc(ni=-2) == -1
    nom = nb.Src(8, 8, 8, None, None, None, None)
    assert acc(J=nom) == -1
    o = nb.Out(8, 8, 8, None, None, None, None)
    assert acc(out=o) == -1
    nn = lambda **kw: L.nbody_force_nn(h, None, 1, 1.0, 0.1, 10, kw.get("I", _src()), None, 10, _src(),
                                       _out(), kw.get("nn", 8), kw.get("r2", None))
    assert nn() == -4
    assert nn(nn=None) == -1 and "nn is NULL" in hostctx.last_error()
    assert nn(r2=12) == -1
    assert nn(I=novel) == -1                  # the jerk needs velocities
    lf = lambda **kw: L.nbody_leapfrog(h, None, 1, 1.0, kw.get("eps", 0.1), kw.get("dt", 0.01),
                                       kw.get("steps", 3), kw.get("n", 10), kw.get("x", 8), 8, 8,
                                       kw.get("a", 8), kw.get("pot", None), 0)
    assert lf() == -4
    assert lf(steps=-1) == -1 and lf(dt=float("nan")) == -1 and lf(n=-1) == -1
    assert lf(x=None) == -1 and lf(a=None) == -1 and lf(pot=4) == -1
    assert lf(n=0, x=None) == -4              # nothing to move: reaches the device check


@pytest.mark.timeout(60)
def test_reserve_sizing_terminates(hostctx):
    """nbody_reserve sizes the split partials on the host (before it needs a
    device) over max_i and the powers of two below it; the walk must end for
    every max_i, powers of two included (a host context then reports the
    missing device)."""
    L = nb.lib()
    h = hostctx.handle
    for ni in (0, 1, 2, 3, 4, 1000, 3000, 4096, 65536, 1 << 20, (1 << 31) - 1):
        assert L.nbody_reserve(h, ni, 4096) == -4, ni


def test_force_tile_environment_override(monkeypatch):
    """NBODY_FORCE_TILE pins the launch shape of every precision that
    compiles it (read at nbody_create, before any device work); a shape no
    precision has makes nbody_create fail with NBODY_ERR_ARG."""
    monkeypatch.setenv("NBODY_FORCE_TILE", "256,2,256,0,0,101")
    c = nb.Context(-1)
    try:
        for prec in ("ds", "fp32"):
            t = c.get_tile(1 << 20, 1 << 20, prec)
            assert (t["tile_j"], t["ipt"], t["wg"], t["unroll"]) == (256, 2, 256, 101), (prec, t)
    finally:
        c.close()
    monkeypatch.setenv("NBODY_FORCE_TILE", "64,1,128,3")
    c = nb.Context(-1)
    try:
        t = c.get_tile(5000, 5000, "ds")
        assert (t["tile_j"], t["ipt"], t["wg"], t["split"]) == (64, 1, 128, 3)
    finally:
        c.close()
    for bad in ("100,2,256", "256,3,256", "nonsense", "64,1,128,-1"):
        monkeypatch.setenv("NBODY_FORCE_TILE", bad)
        with pytest.raises(nb.NBodyError) as e:
            nb.Context(-1)
        assert e.value.code == -1, bad


def test_other_entry_points_validate(hostctx):
    L = nb.lib()
    h = hostctx.handle
    import ctypes as C
    na, tn = C.c_int64(), C.c_int64()
    assert L.nbody_select_active(h, None, -1, 8, 8, 8, C.byref(na), C.byref(tn)) == -1
    assert L.nbody_select_active(h, None, 5, None, 8, 8, C.byref(na), C.byref(tn)) == -1
    assert L.nbody_select_active(h, None, 5, 8, 8, 8, None, C.byref(tn)) == -1
    assert L.nbody_reserve(h, -5, 1) == -1
    t = nb.Tile(100, 2, 256, 0, 0, 0, 0)
    assert L.nbody_set_tile(h, 1, C.byref(t)) == -1
    t = nb.Tile(128, 3, 256, 0, 0, 0, 0)
    assert L.nbody_set_tile(h, 1, C.byref(t)) == -1
    t = nb.Tile(64, 2, 256, 0, 1, 0, 0)          # scalar-cache path exists with tile 128 only
    assert L.nbody_set_tile(h, 1, C.byref(t)) == -1
    t = nb.Tile(128, 2, 64, 0, 1, 0, 0)
    assert L.nbody_set_tile(h, 1, C.byref(t)) == 0
    t = nb.Tile(128, 2, 256, 0, 0, 0, 0)
    assert L.nbody_set_tile(h, 1, C.byref(t)) == 0
    got = hostctx.get_tile(1000, 1000)
    assert (got["tile_j"], got["ipt"], got["wg"], got["jsrc"]) == (128, 2, 256, 0)
    assert L.nbody_set_tile(h, 1, None) == 0
    hp = C.c_void_p()
    o = nb.HermiteOpts(1.0, 0.01, 0.02, 0.01, -20, -3, 0, 1)
    assert L.nbody_hermite_create(h, C.byref(hp), 0, C.byref(o)) == -1
    o2 = nb.HermiteOpts(1.0, 0.01, 0.02, 0.01, -3, -20, 0, 1)
    assert L.nbody_hermite_create(h, C.byref(hp), 100, C.byref(o2)) == -1
    o3 = nb.HermiteOpts(1.0, 0.01, -1.0, 0.01, -20, -3, 0, 1)
    assert L.nbody_hermite_create(h, C.byref(hp), 100, C.byref(o3)) == -1
    o4 = nb.HermiteOpts(1.0, 0.01, 0.02, 0.01, -20, -3, 5, 1)
    assert L.nbody_hermite_create(h, C.byref(hp), 100, C.byref(o4)) == -1
    assert L.nbody_hermite_create(h, C.byref(hp), 100, C.byref(o)) == -4
    assert L.nbody_hermite_step(None, None, None, None) == -1
    # the differentiable run indexes [3][n] rows in int32: n <= (2^31 - 1) / 3
    assert L.nbody_shared_ckpt_bytes(715827882, 8, 8) == 12 * 8 * 715827882
    assert L.nbody_shared_ckpt_bytes(715827883, 8, 8) == -1
    P = nb.Src(*([None] * 7))
    assert L.nbody_shared_run(h, None, 1, 1.0, 0.01, 0.01, 4, 715827883, P, None, None, None, 1) == -1
    assert "715827882" in hostctx.last_error()
    assert L.nbody_destroy(None) == 0


def test_grape_interface_validates_without_a_device():
    L = nb.lib()
    import ctypes as C
    v = (C.c_double * 3)(0.0, 0.0, 0.0)
    assert L.GPU_open(-1) == -1 and L.GPU_open(16) == -1
    assert L.GPU_close(-1) == -1 and L.GPU_close(3) == 0          # closing a closed cluster
    # every call on a cluster that is not open is an argument error
    assert L.GPU_set_j_particle(3, 0, 0, 0.0, 1.0, v, v, v, v) == -1
    assert L.GPU_set_ti(3, 0.0) == -1
    assert L.GPUcalc_firsthalf(3, 0, 0, None, None, None, 0.0) == -1
    assert L.GPUcalc_lasthalf(3, 0, None, None, None) == -1
    assert L.GPU_set_nn(3, 1) == -1 and L.GPU_set_precision(3, 1) == -1
    assert L.GPU_last_error(99) == b"cluster id out of range"
    assert L.GPU_npipes() > 0


def test_create_rejects_bad_device():
    import ctypes as C
    L = nb.lib()
    h = C.c_void_p(1)
    assert L.nbody_create(C.byref(h), -2, None) == -1
    assert not h.value
    assert L.nbody_create(None, 0, None) == -1


def test_block_level_matches_oracle_golden_cases():
    with open(os.path.join(ROOT, "tests", "golden", "quantise_cases.json")) as f:
        cases = json.load(f)["cases"]
    for crit, dt_old, t_new, lmin, lmax, want, why in cases:
        assert nb.block_level(float(crit), dt_old, t_new, lmin, lmax) == want, why


def test_block_level_matches_oracle_random():
    g = np.random.default_rng(0)
    for _ in range(3000):
        lmin = int(g.integers(-20, -5)); lmax = int(g.integers(lmin, 0))
        crit = float(2.0 ** g.uniform(-24, 2)) * (1 if g.random() > 0.05 else -1)
        dt_old = 0 if g.random() < 0.2 else int(1 << int(g.integers(lmin + 20, lmax + 21)))
        t_new = int(g.integers(0, 1 << 22)) * max(dt_old, 1)
        assert nb.block_level(crit, dt_old, t_new, lmin, lmax) == \
            oracle.quantise_dt(crit, dt_old, t_new, lmin, lmax)
    assert nb.block_level(0.1, 0, 0, -3, -20) == -1


def test_single_hip_runtime_in_process():
    # libnbody must bind to the HIP runtime PyTorch already loaded, never a
    # second copy (two runtimes in one process cannot share streams).
    nb.lib()
    import torch  # noqa: F401
    maps = open("/proc/self/maps").read()
    libs = set(re.findall(r"/\S*libamdhip64\S*", maps))
    assert len(libs) == 1, libs
