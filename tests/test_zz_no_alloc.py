"""The allocation-free evaluation (nbody_force_noalloc) through the C ABI:
its outputs against nbody_force's on the same inputs, for two calls in a
row on one context, the second with a smaller input (the device array it
works in keeps the first call's contents), in both precisions.  The
context is created with NBODY_DEBUG_FAIL_ALLOC=1, so any device allocation
the library made would fail: the allocation-free calls must succeed
before and after nbody_force (whose own first allocation is then refused
and retried)."""
import ctypes as C

import numpy as np
import pytest

import nbody_inputs as ics
from gpu_util import dev, host, rel_err_stats

pytestmark = pytest.mark.gpu


def _call(fn, ctx, prec, eps, xi, vi, xj, vj, mj, iself):
    import torch
    import paper_0707_0438_amd as nb
    ni, nj = xi.shape[1], xj.shape[1]
    acc = torch.full((3, ni), float("nan"), dtype=torch.float64, device="cuda")
    jerk = torch.full((3, ni), float("nan"), dtype=torch.float64, device="cuda")
    pot = torch.full((ni,), float("nan"), dtype=torch.float64, device="cuda")
    ptr = lambda t: C.c_void_p(t.data_ptr())
    I = nb.Src(ptr(xi[0]), ptr(xi[1]), ptr(xi[2]), ptr(vi[0]), ptr(vi[1]), ptr(vi[2]), None)
    J = nb.Src(ptr(xj[0]), ptr(xj[1]), ptr(xj[2]), ptr(vj[0]), ptr(vj[1]), ptr(vj[2]), ptr(mj))
    O = nb.Out(ptr(acc[0]), ptr(acc[1]), ptr(acc[2]), ptr(jerk[0]), ptr(jerk[1]), ptr(jerk[2]), ptr(pot))
    sp = ptr(iself) if iself is not None else None
    torch.cuda.synchronize()
    rc = fn(ctx.handle, None, nb.PREC[prec], 1.0, eps, ni, I, sp, nj, J, O)
    torch.cuda.synchronize()
    return rc, host(acc), host(jerk), host(pot)


BARS = {"ds": (1e-5, 1e-4, 1e-6), "fp32": (1e-5, 1e-4, 1e-6)}


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_noalloc_matches_force_two_calls(prec, monkeypatch):
    import torch
    import paper_0707_0438_amd as nb
    L = nb.lib()
    monkeypatch.setenv("NBODY_DEBUG_FAIL_ALLOC", "1")
    ctx = nb.Context(0)
    monkeypatch.delenv("NBODY_DEBUG_FAIL_ALLOC")
    try:
        # call 1: a self-gravitating set (i = j, self pairs by index), large
        # enough for a split with partials; call 2: a smaller i-list against
        # a different, smaller j set with a ragged tail
        big = ics.plummer(20000, 4242, "equal")
        small_j = ics.plummer(3001, 4243, "salpeter")
        small_i = ics.plummer(777, 4244, "equal")
        X, V, M = dev(big.pos), dev(big.vel), dev(big.mass)
        S = torch.arange(big.n, dtype=torch.int32, device="cuda")
        cases = [
            (X, V, X, V, M, S, 1e-3),
            (dev(small_i.pos), dev(small_i.vel), dev(small_j.pos), dev(small_j.vel), dev(small_j.mass),
             None, 1.0 / 256),
        ]
        results = []
        for k, (xi, vi, xj, vj, mj, iself, eps) in enumerate(cases):
            print(f"[noalloc] {prec} call {k + 1}: n_i={xi.shape[1]} n_j={xj.shape[1]}", flush=True)
            rc, a0, j0, p0 = _call(L.nbody_force_noalloc, ctx, prec, eps, xi, vi, xj, vj, mj, iself)
            assert rc == 0, ctx.last_error()
            results.append((a0, j0, p0))
        # the reference calls come after, so that the allocation-free calls
        # ran on a context that had not allocated anything
        for k, (xi, vi, xj, vj, mj, iself, eps) in enumerate(cases):
            rc, a1, j1, p1 = _call(L.nbody_force, ctx, prec, eps, xi, vi, xj, vj, mj, iself)
            if rc == -2:   # the injected first-allocation failure, once
                rc, a1, j1, p1 = _call(L.nbody_force, ctx, prec, eps, xi, vi, xj, vj, mj, iself)
            assert rc == 0, ctx.last_error()
            a0, j0, p0 = results[k]
            for got in (a0, j0, p0):
                assert np.all(np.isfinite(got))
            ea, ej, ep = rel_err_stats(a0, a1), rel_err_stats(j0, j1), rel_err_stats(p0, p1)
            print(f"[noalloc] {prec} call {k + 1}: acc {ea} jerk {ej} pot {ep}", flush=True)
            ba, bj, bp = BARS[prec]
            assert ea["p99"] <= ba and ej["p99"] <= bj and ep["p99"] <= bp
        # the second call again, after the larger one: identical bits
        xi, vi, xj, vj, mj, iself, eps = cases[1]
        rc, a2, j2, p2 = _call(L.nbody_force_noalloc, ctx, prec, eps, xi, vi, xj, vj, mj, iself)
        assert rc == 0, ctx.last_error()
        assert np.array_equal(a2, results[1][0]) and np.array_equal(j2, results[1][1])
        assert np.array_equal(p2, results[1][2])
    finally:
        ctx.close()


def test_noalloc_rejects_beyond_its_scratch():
    """Sizes whose packed records exceed the 64 MiB array are refused before
    anything is launched, with the sizes in the message."""
    import torch
    import paper_0707_0438_amd as nb
    L = nb.lib()
    ctx = nb.Context(0)
    try:
        x = torch.zeros(8, dtype=torch.float64, device="cuda")
        p = C.c_void_p(x.data_ptr())
        src = nb.Src(p, p, p, p, p, p, p)
        out = nb.Out(p, p, p, p, p, p, p)
        n = (64 << 20) // 48 + 1   # one DS record more than fits
        rc = L.nbody_force_noalloc(ctx.handle, None, 1, 1.0, 0.01, 1, src, None, n, src, out)
        assert rc == -1
        assert "beyond its" in ctx.last_error()
    finally:
        ctx.close()
