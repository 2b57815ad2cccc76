"""GPU parity of nbody_force against the float64 oracle (element by element
on the same seeded inputs)."""
import numpy as np
import pytest

import nbody_inputs as ics
import oracle
from gpu_util import BARS, dev, host, rel_err_stats

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_0707_0438_amd as nb
    c = nb.Context(0)
    yield c
    c.close()


def run(ctx, xi, vi, xj, vj, mj, eps, prec, iself=None, G=1.0):
    import torch
    s = None if iself is None else dev(np.asarray(iself, dtype=np.int32))
    a, j, p = ctx.force(dev(xi), dev(vi), dev(xj), dev(vj), dev(mj), eps, G=G, prec=prec, i_self=s)
    torch.cuda.synchronize()
    return host(a), host(j), host(p)


def check(got, ref, prec, label=""):
    bars = BARS[prec]
    stats = {k: rel_err_stats(g, r) for k, g, r in zip(("acc", "jerk", "pot"), got, ref)}
    print(label, prec, {k: f"p99={v['p99']:.2e} max={v['max']:.2e}" for k, v in stats.items()}, flush=True)
    for k in ("acc", "jerk", "pot"):
        assert stats[k]["p99"] <= bars[k], (k, stats[k])
    return stats


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_self_set_ragged(ctx, prec):
    p = ics.plummer(3001, 101)
    eps = 1.0 / 256
    ref = oracle.force(p.pos, p.vel, p.pos, p.vel, p.mass, eps, iself=np.arange(p.n))
    got = run(ctx, p.pos, p.vel, p.pos, p.vel, p.mass, eps, prec, iself=np.arange(p.n))
    check(got, ref, prec, "self-set n=3001")


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_i_subset_and_disjoint_sets(ctx, prec):
    p = ics.plummer(2500, 102)
    eps = 0.01
    g = np.random.default_rng(0)
    sel = np.sort(g.choice(p.n, 777, replace=False))
    ref = oracle.force(p.pos[:, sel], p.vel[:, sel], p.pos, p.vel, p.mass, eps, iself=sel)
    got = run(ctx, p.pos[:, sel], p.vel[:, sel], p.pos, p.vel, p.mass, eps, prec, iself=sel)
    check(got, ref, prec, "subset")
    q = ics.plummer(333, 103)
    ref = oracle.force(q.pos, q.vel, p.pos, p.vel, p.mass, eps)
    got = run(ctx, q.pos, q.vel, p.pos, p.vel, p.mass, eps, prec)
    check(got, ref, prec, "disjoint")


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_every_launch_shape_and_split(ctx, prec):
    import torch
    p = ics.plummer(1500, 104)
    eps = 1.0 / 256
    ref = oracle.force(p.pos, p.vel, p.pos, p.vel, p.mass, eps, iself=np.arange(p.n))
    X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
    S = dev(np.arange(p.n, dtype=np.int32))
    shapes = [(tj, ipt, wg, 0, 0, 0) for tj in (64, 128, 256) for ipt in (1, 2, 4) for wg in (128, 256)]
    shapes += [(128, ipt, wg, 1, 0, 0) for ipt in (1, 2, 4) for wg in (64, 256)]
    # short tiles for small sets
    shapes += [(tj, 1, wg, 0, 0, 0) for tj in (16, 32) for wg in (64, 128)]
    # unroll / occupancy / software-pipelined variants
    shapes += [(256, 1, 256, 0, 2, 0), (256, 1, 256, 0, 8, 0), (256, 1, 256, 0, 4, 6), (256, 1, 256, 0, 4, 8),
               (256, 2, 256, 0, 1, 0), (256, 2, 256, 0, 2, 0), (256, 2, 256, 0, 2, 5), (128, 2, 256, 0, 2, 4),
               (256, 1, 256, 0, 102, 0), (256, 1, 256, 0, 104, 0), (256, 2, 256, 0, 101, 0)]
    if prec == "ds":
        shapes += [(128, 1, 256, 0, 102, 0), (256, 1, 128, 0, 102, 0)]
    try:
        for tj, ipt, wg, js, unr, wpe in shapes:
            for split in (1, 5):
                ctx.set_tile(prec, tile_j=tj, ipt=ipt, wg=wg, split=split, jsrc=js, unroll=unr, waves=wpe)
                r1 = ctx.force(X, V, X, V, M, eps, prec=prec, i_self=S)
                r2 = ctx.force(X, V, X, V, M, eps, prec=prec, i_self=S)
                torch.cuda.synchronize()
                for u, w in zip(r1, r2):
                    assert torch.equal(u, w), (tj, ipt, wg, js, unr, wpe, split)
                check(tuple(host(t) for t in r1), ref, prec,
                      f"tj={tj} ipt={ipt} wg={wg} js={js} unr={unr} wpe={wpe} S={split}")
    finally:
        ctx.set_tile(prec)


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_zero_softening_and_coincident_particles(ctx, prec):
    p = ics.plummer(700, 105)
    x = p.pos.copy()
    x[:, 5] = x[:, 9]          # two distinct particles at one point
    v = p.vel.copy()
    ref = oracle.force(x, v, x, v, p.mass, 0.0, iself=np.arange(p.n))
    got = run(ctx, x, v, x, v, p.mass, 0.0, prec, iself=np.arange(p.n))
    for q in got:
        assert np.all(np.isfinite(q))
    mask = np.ones(p.n, bool); mask[[5, 9]] = False
    check(tuple(q[..., mask] for q in got), tuple(q[..., mask] for q in ref), prec, "eps=0")
    # softened: the coincident pair interacts in the potential (-m/eps)
    eps = 0.05
    ref = oracle.force(x, v, x, v, p.mass, eps, iself=np.arange(p.n))
    got = run(ctx, x, v, x, v, p.mass, eps, prec, iself=np.arange(p.n))
    check(got, ref, prec, "coincident eps>0")


def test_edge_sizes(ctx):
    import torch
    p = ics.plummer(5, 106)
    # empty i list: nothing to do
    e = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    a, j, pt = ctx.force(e, e, dev(p.pos), dev(p.vel), dev(p.mass), 0.1)
    assert a.shape == (3, 0)
    # empty j set: zero output
    e1 = torch.empty((0,), dtype=torch.float64, device="cuda")
    a, j, pt = ctx.force(dev(p.pos), dev(p.vel), e, e, e1, 0.1)
    torch.cuda.synchronize()
    assert torch.count_nonzero(a) == 0 and torch.count_nonzero(pt) == 0
    # one particle against itself: zero force, zero potential
    one = ics.plummer(1, 107)
    for prec in ("ds", "fp32"):
        got = run(ctx, one.pos, one.vel, one.pos, one.vel, one.mass, 0.1, prec, iself=[0])
        assert np.all(got[0] == 0) and np.all(got[1] == 0) and abs(got[2][0]) < 1e-6
    # two particles: closed form through the library
    x = np.array([[0.0, 0.3], [0.0, 0.4], [0.0, 0.0]])
    v = np.zeros((3, 2)); m = np.array([0.25, 0.75])
    got = run(ctx, x, v, x, v, m, 0.0, "ds", iself=[0, 1], G=2.0)
    assert got[0][0, 0] == pytest.approx(2.0 * 0.75 * 0.3 / 0.5 ** 3, rel=1e-6)
    assert got[2][1] == pytest.approx(-2.0 * 0.25 / 0.5, rel=1e-6)


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_plummer1k_full(ctx, prec):
    p = ics.workload("plummer1k_hermite")
    eps = 1.0 / 256
    ref = oracle.force(p.pos, p.vel, p.pos, p.vel, p.mass, eps, iself=np.arange(p.n))
    got = run(ctx, p.pos, p.vel, p.pos, p.vel, p.mass, eps, prec, iself=np.arange(p.n))
    check(got, ref, prec, "N=1024")


def test_plummer1m_sampled(ctx):
    """N = 2^20, eps = 1e-4, all particles evaluated in the benchmark's launch
    shape; 4096 seeded rows checked against the oracle."""
    import torch
    p = ics.workload("plummer1m_force")
    eps = 1e-4
    g = np.random.default_rng(2)
    sel = np.sort(g.choice(p.n, 4096, replace=False))
    ref = oracle.force(p.pos[:, sel], p.vel[:, sel], p.pos, p.vel, p.mass, eps, iself=sel)
    X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
    S = torch.arange(p.n, dtype=torch.int32, device="cuda")
    out = {}
    for prec in ("ds", "fp32"):
        a, j, pt = ctx.force(X, V, X, V, M, eps, prec=prec, i_self=S)
        torch.cuda.synchronize()
        got = (host(a)[:, sel], host(j)[:, sel], host(pt)[sel])
        out[prec] = check(got, ref, prec, "N=2^20 sampled")
    assert out["ds"]["acc"]["p99"] < out["fp32"]["acc"]["p99"]


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_small_blocks_many_splits(ctx, prec):
    """Small i-lists against a large, ragged j set: many j-ranges, so the
    partials go through the wave-per-row float64 reduce."""
    import torch
    p = ics.plummer(70001, 107)
    eps = 1e-3
    X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
    for ni in (1, 7, 100, 1000):
        sel = np.sort(np.random.default_rng(ni).choice(p.n, ni, replace=False))
        tile = ctx.get_tile(ni, p.n, prec)
        assert tile["split"] >= 32 or ni == 1000, tile
        ref = oracle.force(p.pos[:, sel], p.vel[:, sel], p.pos, p.vel, p.mass, eps, iself=sel)
        a, j, pt = ctx.force(X[:, sel].contiguous(), V[:, sel].contiguous(), X, V, M, eps, prec=prec,
                             i_self=dev(sel.astype(np.int32)))
        torch.cuda.synchronize()
        check((host(a), host(j), host(pt)), ref, prec, f"ni={ni} split={tile['split']}")


def test_large_j_set(ctx):
    """A j set of 2^25 + 77 particles (beyond 2^24, so record offsets and j
    indices need more than float or 24-bit range) against 42 i-particles,
    37 of them members of the set (including the last one) and 5 outside:
    force in both precisions and the nearest neighbour against the oracle."""
    import torch
    nj = (1 << 25) + 77
    g = np.random.default_rng(11)
    xj = g.normal(size=(3, nj)); vj = 0.3 * g.normal(size=(3, nj)); mj = np.full(nj, 1.0 / nj)
    members = np.sort(np.concatenate([g.choice(nj - 1, 36, replace=False), [nj - 1]]))
    outside = g.normal(size=(3, 5)); vout = g.normal(size=(3, 5))
    xi = np.concatenate([xj[:, members], outside], 1); vi = np.concatenate([vj[:, members], vout], 1)
    iself = np.concatenate([members, -np.ones(5, dtype=np.int64)])
    eps = 1e-3
    ref = oracle.force(xi, vi, xj, vj, mj, eps, iself=iself)
    ref_nn, _ = oracle.nearest(xi, xj, iself=iself)
    X, V, M = dev(xj), dev(vj), dev(mj)
    S = dev(iself.astype(np.int32))
    for prec in ("ds", "fp32"):
        a, j, pt = ctx.force(dev(xi), dev(vi), X, V, M, eps, prec=prec, i_self=S)
        torch.cuda.synchronize()
        check((host(a), host(j), host(pt)), ref, prec, "nj=2^25+77")
    _, _, _, nn, _ = ctx.force_nn(dev(xi), dev(vi), X, V, M, eps, prec="ds", i_self=S)
    torch.cuda.synchronize()
    nn = host(nn)
    d = ((xj[:, nn] - xi) ** 2).sum(0)
    dref = ((xj[:, ref_nn] - xi) ** 2).sum(0)
    assert np.all(d <= dref * (1 + 2e-6))
    assert np.mean(nn == ref_nn) > 0.95


def test_debug_self_check(monkeypatch):
    """With NBODY_DEBUG_SELF_CHECK=1 the library verifies that every i row
    named by i_self equals its j row bit for bit (and lies in the j set)."""
    import torch
    import paper_0707_0438_amd as nb
    monkeypatch.setenv("NBODY_DEBUG_SELF_CHECK", "1")
    c = nb.Context(0)
    try:
        p = ics.plummer(300, 108)
        X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
        sel = np.arange(0, 300, 7)
        XI, VI = X[:, sel].contiguous(), V[:, sel].contiguous()
        S = dev(sel.astype(np.int32))
        for prec in ("ds", "fp32"):
            c.force(XI, VI, X, V, M, 0.01, prec=prec, i_self=S)
            c.force_acc(XI, X, M, 0.01, prec=prec, i_self=S)
        torch.cuda.synchronize()
        XI[0, 3] += 1e-3                    # i row 3 no longer equals j row 21
        with pytest.raises(nb.NBodyError, match="i_self"):
            c.force(XI, VI, X, V, M, 0.01, i_self=S)
        with pytest.raises(nb.NBodyError, match="i_self"):
            c.force_acc(XI, X, M, 0.01, prec="fp32", i_self=S)
        XI[0, 3] = X[0, sel[3]]             # restored
        bad = S.clone()
        bad[1] = 5000                       # beyond the j set
        with pytest.raises(nb.NBodyError, match="i_self"):
            c.force(XI, VI, X, V, M, 0.01, i_self=bad)
        c.force(XI, VI, X, V, M, 0.01, i_self=S)
    finally:
        c.close()


def test_autotune_cache_timing_and_reserve(tmp_path):
    """The autotuner picks a compiled shape, stores it in the JSON-lines cache
    and a new context reading that cache uses it for the same size bucket;
    results in the tuned shape still meet the bars; per-launch kernel timing
    counts launches; nbody_reserve pre-sizes scratch."""
    import json
    import torch
    import paper_0707_0438_amd as nb
    cache = str(tmp_path / "tune.jsonl")
    p = ics.plummer(3000, 109)
    X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
    c = nb.Context(0, tune_cache=cache)
    try:
        c.reserve(4096, 4096)
        tile, ms = c.autotune(X, V, X, V, M, 0.01, prec="ds", reps=1)
        assert ms > 0 and tile["tile_j"] in (16, 32, 64, 128, 256) and tile["ipt"] in (1, 2, 4)
        lines = [json.loads(ln) for ln in open(cache) if ln.strip()]
        assert len(lines) >= 1
        got = c.get_tile(3000, 3000, "ds")
        assert (got["tile_j"], got["ipt"], got["wg"]) == (tile["tile_j"], tile["ipt"], tile["wg"])
        c.kernel_timing(True)
        S = torch.arange(p.n, dtype=torch.int32, device="cuda")
        for _ in range(3):
            a, j, pt = c.force(X, V, X, V, M, 0.01, prec="ds", i_self=S)
        kms, launches = c.kernel_time()
        c.kernel_timing(False)
        assert launches == 3 and kms > 0
        ref = oracle.force(p.pos, p.vel, p.pos, p.vel, p.mass, 0.01, iself=np.arange(p.n))
        check((host(a), host(j), host(pt)), ref, "ds", "tuned shape")
    finally:
        c.close()
    c2 = nb.Context(0, tune_cache=cache)
    try:
        got = c2.get_tile(3000, 3000, "ds")
        assert (got["tile_j"], got["ipt"], got["wg"]) == (tile["tile_j"], tile["ipt"], tile["wg"])
    finally:
        c2.close()


def test_work_on_a_caller_stream(ctx):
    """Every call enqueues on the stream it is given: a force evaluation, a
    block-step advance and the fused adjoint on a side stream (default
    priority) give the same bits as on the current stream."""
    import torch
    p = ics.plummer(2500, 110, "salpeter")
    X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
    S = torch.arange(p.n, dtype=torch.int32, device="cuda")
    ga = dev(np.random.default_rng(3).normal(size=(3, p.n)))
    base = ctx.force(X, V, X, V, M, 1e-3, i_self=S)
    gbase = ctx.force_vjp_self(X, V, M, 1e-3, ga)
    h0 = ctx.hermite(p.n, eps=1e-3, eta=0.02, prec="ds")
    h0.set_state(X, V, M)
    h0.advance(1 << 12)
    x0 = h0.get_state()["x"].clone()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        Xs, Vs, Ms, Ss = X.clone(), V.clone(), M.clone(), S.clone()
    got = ctx.force(Xs, Vs, Xs, Vs, Ms, 1e-3, i_self=Ss, stream=side)
    ggot = ctx.force_vjp_self(Xs, Vs, Ms, 1e-3, ga, stream=side)
    h1 = ctx.hermite(p.n, eps=1e-3, eta=0.02, prec="ds")
    h1.set_state(Xs, Vs, Ms, stream=side)
    h1.advance(1 << 12, stream=side)
    x1 = h1.get_state(stream=side)["x"]
    side.synchronize()
    for u, w in zip(base, got):
        assert torch.equal(u, w)
    for u, w in zip(gbase, ggot):
        assert torch.equal(u, w)
    assert torch.equal(x0, x1)
    h0.close(); h1.close()
