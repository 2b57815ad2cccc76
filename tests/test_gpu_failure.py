"""Failure handling through the C ABI, forced from the host: an injected
device-allocation failure (NBODY_DEBUG_FAIL_ALLOC=k fails the k-th
allocation a context makes) must surface as NBODY_ERR_NOMEM before anything
is launched, leave the context and the integrator usable, and a retried call
must continue exactly as if nothing had failed.  No kernel is made to fault."""
import numpy as np
import pytest

import nbody_inputs as ics
from gpu_util import dev, host

pytestmark = pytest.mark.gpu

NOMEM = -2


def _with_retry(fn, counter):
    import paper_0707_0438_amd as nb
    try:
        return fn()
    except nb.NBodyError as e:
        assert e.code == NOMEM, e
        counter.append(str(e))
        return fn()


def _hermite_sequence(c, p, eps, counter):
    """create, set_state, two advances, energy; every call retried once on
    NOMEM.  Returns the final state and energies."""
    X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
    h = _with_retry(lambda: c.hermite(p.n, eps=eps, eta=0.02, prec="ds"), counter)
    try:
        _with_retry(lambda: h.set_state(X, V, M), counter)
        _with_retry(lambda: h.advance(1 << 12), counter)
        e1 = _with_retry(lambda: h.energy(), counter)
        _with_retry(lambda: h.advance(1 << 13), counter)
        st = h.get_state()
        return {k: host(v) for k, v in st.items()}, e1
    finally:
        h.close()


def test_injected_allocation_failure_hermite(monkeypatch):
    """Block steps on a small Salpeter set: with the k-th allocation failing
    (k = 1 .. 8, which covers every allocation of the sequence), each failing
    call returns NBODY_ERR_NOMEM and its retry continues; the final state and
    the energy are bit-identical to a run without failures."""
    import torch
    import paper_0707_0438_amd as nb
    p = ics.plummer(2048, 901, "salpeter")
    eps = 1e-3
    monkeypatch.delenv("NBODY_DEBUG_FAIL_ALLOC", raising=False)
    c = nb.Context(0)
    try:
        ref, eref = _hermite_sequence(c, p, eps, [])
    finally:
        c.close()
    failed_at = []
    for k in range(1, 9):
        monkeypatch.setenv("NBODY_DEBUG_FAIL_ALLOC", str(k))
        c = nb.Context(0)
        try:
            hits = []
            got, e = _hermite_sequence(c, p, eps, hits)
            torch.cuda.synchronize()
        finally:
            c.close()
        if hits:
            failed_at.append(k)
            assert "injected" in hits[0]
        for key in ("x", "v", "a", "jerk", "t", "dt"):
            assert np.array_equal(got[key], ref[key]), (k, key)
        assert e == eref, k
    print("allocations that failed and were retried:", failed_at, flush=True)
    assert len(failed_at) >= 3


def test_injected_allocation_failure_force(monkeypatch):
    """nbody_force with its first allocation failing: NBODY_ERR_NOMEM, the
    output rows untouched, and the next call on the same context correct."""
    import torch
    import paper_0707_0438_amd as nb
    monkeypatch.setenv("NBODY_DEBUG_FAIL_ALLOC", "1")
    c = nb.Context(0)
    try:
        p = ics.plummer(1500, 902)
        X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
        S = torch.arange(p.n, dtype=torch.int32, device="cuda")
        out = (torch.full((3, p.n), 7.0, dtype=torch.float64, device="cuda"),
               torch.full((3, p.n), 7.0, dtype=torch.float64, device="cuda"),
               torch.full((p.n,), 7.0, dtype=torch.float64, device="cuda"))
        with pytest.raises(nb.NBodyError) as ei:
            c.force(X, V, X, V, M, 0.01, i_self=S, out=out)
        assert ei.value.code == NOMEM and "injected" in str(ei.value)
        torch.cuda.synchronize()
        assert all(bool((t == 7.0).all()) for t in out)
        a, j, pt = c.force(X, V, X, V, M, 0.01, i_self=S)
        monkeypatch.delenv("NBODY_DEBUG_FAIL_ALLOC")
        c2 = nb.Context(0)
        try:
            b = c2.force(X, V, X, V, M, 0.01, i_self=S)
        finally:
            c2.close()
        torch.cuda.synchronize()
        for u, w in zip((a, j, pt), b):
            assert torch.equal(u, w)
    finally:
        c.close()


def test_reserve_covers_later_calls(monkeypatch):
    """After nbody_reserve(max_i, max_j) the calls it covers allocate
    nothing: with the allocation after the reserve's own ones set to fail,
    DS and FP32 evaluations of every size up to the reserved one (including
    split partial sums) succeed, and only a larger j set hits the injected
    failure."""
    import torch
    import paper_0707_0438_amd as nb
    n = 3000
    # the reserve makes three allocations here (i records, j records, split
    # partial sums): the fourth is the first one after it
    monkeypatch.setenv("NBODY_DEBUG_FAIL_ALLOC", "4")
    c = nb.Context(0)
    try:
        c.reserve(n, n)
        p = ics.plummer(n, 903)
        X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
        for prec in ("ds", "fp32"):
            for ni in (n, 1000, 100, 7):
                tile = c.get_tile(ni, n, prec)
                sel = np.sort(np.random.default_rng(ni).choice(n, ni, replace=False))
                if ni == n:
                    c.force(X, V, X, V, M, 0.01, prec=prec, i_self=torch.arange(n, dtype=torch.int32,
                                                                                 device="cuda"))
                else:
                    c.force(X[:, sel].contiguous(), V[:, sel].contiguous(), X, V, M, 0.01, prec=prec,
                            i_self=dev(sel.astype(np.int32)))
                assert tile["split"] >= 1
        torch.cuda.synchronize()
        q = ics.plummer(n + 1000, 904)
        with pytest.raises(nb.NBodyError) as ei:
            c.force(X, V, dev(q.pos), dev(q.vel), dev(q.mass), 0.01)
        assert ei.value.code == NOMEM
    finally:
        c.close()
