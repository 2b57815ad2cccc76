"""GPU parity of the batched (many independent clusters) path: bitwise
agreement with per-cluster nbody_force in the same launch shape, parity with
the oracle on the 512-cluster workload, graph replay against eager steps,
and the degenerate cluster layouts."""
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


def small_clusters(seed, sizes):
    def one(s, k):
        if s == 0:
            return ics.Particles(np.zeros((3, 0)), np.zeros((3, 0)), np.zeros(0))
        return ics.plummer(int(s), seed * 100 + k)
    parts = [one(s, k) for k, s in enumerate(sizes)]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    pos = np.concatenate([p.pos for p in parts], axis=1)
    vel = np.concatenate([p.vel for p in parts], axis=1)
    m = np.concatenate([p.mass for p in parts])
    eps = 1.0 / (4.0 * np.maximum(np.asarray(sizes, dtype=np.float64), 1.0) ** (1.0 / 3.0))
    return off, eps, pos, vel, m


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_batched_equals_per_cluster_bitwise(ctx, prec):
    import torch
    sizes = [1, 700, 64, 129, 5, 300, 2, 1000, 77]
    off, eps, pos, vel, m = small_clusters(7, sizes)
    X, V, M = dev(pos), dev(vel), dev(m)
    O, E = dev(off), dev(eps)
    try:
        for tj, ipt, wg in ((128, 2, 256), (64, 1, 128), (256, 4, 256)):
            ctx.set_tile(prec, tile_j=tj, ipt=ipt, wg=wg, split=1)
            a, j, p = ctx.force_batched(X, V, M, O, E, prec=prec)
            for c in range(len(sizes)):
                lo, hi = int(off[c]), int(off[c + 1])
                xc, vc, mc = X[:, lo:hi].contiguous(), V[:, lo:hi].contiguous(), M[lo:hi].contiguous()
                ac, jc, pc = ctx.force(xc, vc, xc, vc, mc, float(eps[c]), prec=prec,
                                       i_self=torch.arange(hi - lo, dtype=torch.int32, device="cuda"))
                torch.cuda.synchronize()
                assert torch.equal(ac, a[:, lo:hi]) and torch.equal(jc, j[:, lo:hi]), (tj, ipt, wg, c)
                assert torch.equal(pc, p[lo:hi]), (tj, ipt, wg, c)
    finally:
        ctx.set_tile(prec)


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_batched_512_clusters_against_oracle(ctx, prec):
    """The 512-cluster workload (N_c log-uniform in [64, 8192], eps_c =
    1/(4 N_c^(1/3))): every row of 40 seeded clusters against the oracle."""
    import torch
    off, eps, p = ics.clusters(512, ics.seed_for(4))
    a, j, pt = ctx.force_batched(dev(p.pos), dev(p.vel), dev(p.mass), dev(off), dev(eps), prec=prec)
    torch.cuda.synchronize()
    a, j, pt = host(a), host(j), host(pt)
    picks = np.random.default_rng(3).choice(512, 40, replace=False)
    got_a, got_j, got_p, ref_a, ref_j, ref_p = [], [], [], [], [], []
    for c in picks:
        lo, hi = int(off[c]), int(off[c + 1])
        ra, rj, rp = oracle.force(p.pos[:, lo:hi], p.vel[:, lo:hi], p.pos[:, lo:hi], p.vel[:, lo:hi],
                                  p.mass[lo:hi], float(eps[c]), iself=np.arange(hi - lo))
        ref_a.append(ra); ref_j.append(rj); ref_p.append(rp)
        got_a.append(a[:, lo:hi]); got_j.append(j[:, lo:hi]); got_p.append(pt[lo:hi])
    st = {"acc": rel_err_stats(np.concatenate(got_a, 1), np.concatenate(ref_a, 1)),
          "jerk": rel_err_stats(np.concatenate(got_j, 1), np.concatenate(ref_j, 1)),
          "pot": rel_err_stats(np.concatenate(got_p), np.concatenate(ref_p))}
    print(prec, {k: f"p99={v['p99']:.2e} max={v['max']:.2e}" for k, v in st.items()}, flush=True)
    for k in st:
        assert st[k]["p99"] <= BARS[prec][k], (k, st[k])


def test_degenerate_layouts(ctx):
    import torch
    off, eps, pos, vel, m = small_clusters(9, [3, 0, 1, 4])
    n = pos.shape[1]
    # one extra particle after the last cluster belongs to no cluster
    pos = np.concatenate([pos, np.zeros((3, 1))], 1); vel = np.concatenate([vel, np.zeros((3, 1))], 1)
    m = np.concatenate([m, [0.5]])
    a, j, p = ctx.force_batched(dev(pos), dev(vel), dev(m), dev(off), dev(eps))
    torch.cuda.synchronize()
    a, p = host(a), host(p)
    assert np.all(a[:, n] == 0) and p[n] == 0            # outside every cluster
    assert np.all(a[:, 3] == 0) and p[3] == 0             # the one-particle cluster
    ra, _, rp = oracle.force(pos[:, 4:8], vel[:, 4:8], pos[:, 4:8], vel[:, 4:8], m[4:8], float(eps[3]),
                             iself=np.arange(4))
    assert rel_err_stats(a[:, 4:8], ra)["max"] < 1e-5
    # offsets beyond the particle count are clamped, not followed
    bad = np.array([0, 2, 10 ** 9], dtype=np.int64)
    a2, _, _ = ctx.force_batched(dev(pos), dev(vel), dev(m), dev(bad), dev(np.array([0.1, 0.1])))
    torch.cuda.synchronize()
    assert np.all(np.isfinite(host(a2)))
    # no clusters at all
    a3, _, _ = ctx.force_batched(dev(pos), dev(vel), dev(m), dev(np.zeros(1, np.int64)),
                                 torch.empty((0,), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert torch.count_nonzero(a3) == 0


def test_batch_hermite_graph_equals_eager_and_oracle(ctx):
    import torch
    sizes = [64, 500, 129, 2000, 90]
    off, eps, pos, vel, m = small_clusters(11, sizes)
    n = pos.shape[1]
    dt, steps = 1.0 / 256, 32
    X, V, M, O, E = dev(pos), dev(vel), dev(m), dev(off), dev(eps)
    a0, j0, _ = ctx.force_batched(X, V, M, O, E)
    states = {}
    for mode in ("eager", "graph"):
        x, v, a, j = X.clone(), V.clone(), a0.clone(), j0.clone()
        ctx.batch_hermite(x, v, a, j, M, O, E, dt, steps, use_graph=(mode == "graph"))
        torch.cuda.synchronize()
        states[mode] = (x, v, a, j)
    for u, w in zip(states["eager"], states["graph"]):
        assert torch.equal(u, w)
    # replays of the captured graph with eager work in between: each replay
    # advances the same way as eager steps
    x, v, a, j = X.clone(), V.clone(), a0.clone(), j0.clone()
    xe, ve, ae, je = X.clone(), V.clone(), a0.clone(), j0.clone()
    for rep in range(3):
        ctx.batch_hermite(x, v, a, j, M, O, E, dt, steps, use_graph=True)
        ctx.batch_hermite(xe, ve, ae, je, M, O, E, dt, steps, use_graph=False)
        torch.cuda.synchronize()
        assert torch.equal(x, xe) and torch.equal(v, ve), rep
    # against the oracle, cluster by cluster
    xg = host(states["graph"][0])
    for c in (0, 3):
        lo, hi = int(off[c]), int(off[c + 1])
        xr, _ = oracle.hermite_shared_forward(pos[:, lo:hi], vel[:, lo:hi], m[lo:hi], float(eps[c]), dt, steps)
        assert np.abs(xg[:, lo:hi] - xr).max() < 1e-7


def test_clusters512_graph_run_against_oracle(ctx):
    """The full batched workload: 512 clusters (N_c log-uniform in
    [64, 8192], eps_c = 1/(4 N_c^(1/3))) advanced 32 shared Hermite steps of
    1/256 through one captured hipGraph; 12 seeded clusters (including the
    largest and the smallest) against the oracle's shared-step run."""
    import torch
    off, eps, p = ics.clusters(512, ics.seed_for(4))
    sizes = np.diff(off)
    X, V, M, O, E = dev(p.pos), dev(p.vel), dev(p.mass), dev(off), dev(eps)
    a, j, _ = ctx.force_batched(X, V, M, O, E)
    x, v = X.clone(), V.clone()
    ctx.batch_hermite(x, v, a, j, M, O, E, 1.0 / 256, 32, use_graph=True)
    torch.cuda.synchronize()
    xg, vg = host(x), host(v)
    g = np.random.default_rng(6)
    picks = set(g.choice(512, 10, replace=False).tolist()) | {int(np.argmax(sizes)), int(np.argmin(sizes))}
    worst = 0.0
    for c in sorted(picks):
        lo, hi = int(off[c]), int(off[c + 1])
        xr, vr = oracle.hermite_shared_forward(p.pos[:, lo:hi], p.vel[:, lo:hi], p.mass[lo:hi], float(eps[c]),
                                               1.0 / 256, 32)
        dx = np.abs(xg[:, lo:hi] - xr).max()
        worst = max(worst, dx)
        assert dx < 1e-7 and np.abs(vg[:, lo:hi] - vr).max() < 1e-6, (c, hi - lo, dx)
    print("512 clusters, 32 graph steps: worst max|dx| over", len(picks), "clusters", worst, flush=True)
