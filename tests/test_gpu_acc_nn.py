"""GPU parity of the force-only evaluation (nbody_force_acc), the
nearest-neighbour evaluation (nbody_force_nn) and the leapfrog driver
(nbody_leapfrog) against the float64 oracle."""
import numpy as np
import pytest

import nbody_inputs as ics
import oracle
from gpu_util import BARS, dev, host, rel_err_stats

pytestmark = pytest.mark.gpu

# relative slack of a float32 distance comparison: where two candidates are
# closer than this (relative), either may be reported
NN_TOL = {"ds": 2e-6, "fp32": 2e-4}


@pytest.fixture(scope="module")
def ctx():
    import paper_0707_0438_amd as nb
    c = nb.Context(0)
    yield c
    c.close()


def check_acc(a, pot, ref_a, ref_p, prec, label):
    sa, sp = rel_err_stats(a, ref_a), rel_err_stats(pot, ref_p)
    print(label, prec, f"acc p99={sa['p99']:.2e} max={sa['max']:.2e} pot p99={sp['p99']:.2e}", flush=True)
    assert sa["p99"] <= BARS[prec]["acc"] and sp["p99"] <= BARS[prec]["pot"]


def check_nn(nn, r2, xi, xj, iself, prec, label):
    """The reported j must be a nearest one up to float32 rounding; where the
    nearest is clear by more than that, it must be the oracle's; the
    reported distance must be the distance of the reported j."""
    ref_nn, ref_r2 = oracle.nearest(xi, xj, iself=iself)
    tol = NN_TOL[prec]
    ok = nn >= 0
    assert np.array_equal(ok, ref_nn >= 0), label
    d = ((xj[:, nn[ok]] - xi[:, ok]) ** 2).sum(0)
    assert np.all(d <= ref_r2[ok] * (1 + tol) + 1e-300), label
    np.testing.assert_allclose(r2[ok], d, rtol=4 * tol)
    assert np.all(np.isinf(r2[~ok]))
    # second-nearest distance of every i, in float64
    ni = xi.shape[1]
    second = np.empty(ni)
    for b in range(0, ni, 512):
        D = ((xj[:, None, :] - xi[:, b:b + 512, None]) ** 2).sum(0)
        if iself is not None:
            rows = np.arange(D.shape[0])
            s = np.asarray(iself[b:b + 512])
            D[rows[s >= 0], s[s >= 0]] = np.inf
        part = np.partition(D, 1, axis=1) if D.shape[1] > 1 else np.full((D.shape[0], 2), np.inf)
        second[b:b + 512] = part[:, 1]
    clear = ok & (second > ref_r2 * (1 + 4 * tol))
    same = np.mean(nn[clear] == ref_nn[clear])
    print(label, prec, f"nn: {clear.sum()} clear cases, agreement {same:.6f}", flush=True)
    assert np.array_equal(nn[clear], ref_nn[clear]), label


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_force_acc_against_oracle_and_full_kernel(ctx, prec):
    import torch
    p = ics.plummer(3001, 601)
    eps = 1.0 / 256
    X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
    S = torch.arange(p.n, dtype=torch.int32, device="cuda")
    a, pot = ctx.force_acc(X, X, M, eps, prec=prec, i_self=S)
    af, _, pf = ctx.force(X, V, X, V, M, eps, prec=prec, i_self=S)
    torch.cuda.synchronize()
    ref_a, ref_p = oracle.force_acc(p.pos, p.pos, p.mass, eps, iself=np.arange(p.n))
    check_acc(host(a), host(pot), ref_a, ref_p, prec, "acc self set")
    # the same launch shape and the same arithmetic as the full kernel
    assert torch.equal(a, af) and torch.equal(pot, pf)
    # i subset (split j ranges) and disjoint sets
    sel = np.sort(np.random.default_rng(1).choice(p.n, 77, replace=False))
    a, pot = ctx.force_acc(X[:, sel].contiguous(), X, M, eps, prec=prec, i_self=dev(sel.astype(np.int32)))
    torch.cuda.synchronize()
    ref_a, ref_p = oracle.force_acc(p.pos[:, sel], p.pos, p.mass, eps, iself=sel)
    check_acc(host(a), host(pot), ref_a, ref_p, prec, "acc subset")
    q = ics.plummer(500, 602)
    a, pot = ctx.force_acc(dev(q.pos), X, M, eps, prec=prec)
    torch.cuda.synchronize()
    ref_a, ref_p = oracle.force_acc(q.pos, p.pos, p.mass, eps)
    check_acc(host(a), host(pot), ref_a, ref_p, prec, "acc disjoint")


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_force_acc_unsoftened_and_edges(ctx, prec):
    import torch
    p = ics.plummer(1500, 603)
    X, M = dev(p.pos), dev(p.mass)
    a, pot = ctx.force_acc(X, X, M, 0.0, prec=prec, i_self=torch.arange(p.n, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    ref_a, ref_p = oracle.force_acc(p.pos, p.pos, p.mass, 0.0, iself=np.arange(p.n))
    check_acc(host(a), host(pot), ref_a, ref_p, prec, "acc eps=0")
    e = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    a, pot = ctx.force_acc(X[:, :5].contiguous(), e, torch.empty((0,), dtype=torch.float64, device="cuda"), 0.1,
                           prec=prec)
    torch.cuda.synchronize()
    assert torch.count_nonzero(a) == 0 and torch.count_nonzero(pot) == 0
    a, pot = ctx.force_acc(e, X, M, 0.1, prec=prec)
    assert a.shape == (3, 0)


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_force_nn_against_oracle(ctx, prec):
    import torch
    p = ics.plummer(3001, 604)
    eps = 1.0 / 256
    X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
    a, j, pt, nn, r2 = ctx.force_nn(X, V, X, V, M, eps, prec=prec,
                                    i_self=torch.arange(p.n, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    ref = oracle.force(p.pos, p.vel, p.pos, p.vel, p.mass, eps, iself=np.arange(p.n))
    for k, g, r in zip(("acc", "jerk", "pot"), (a, j, pt), ref):
        st = rel_err_stats(host(g), r)
        assert st["p99"] <= BARS[prec][k], (k, st)
    check_nn(host(nn), host(r2), p.pos, p.pos, np.arange(p.n), prec, "nn self set")
    # small i-lists: many j ranges, reduced per range
    for ni in (1, 50, 900):
        sel = np.sort(np.random.default_rng(ni).choice(p.n, ni, replace=False))
        _, _, _, nn, r2 = ctx.force_nn(X[:, sel].contiguous(), V[:, sel].contiguous(), X, V, M, eps, prec=prec,
                                       i_self=dev(sel.astype(np.int32)))
        torch.cuda.synchronize()
        check_nn(host(nn), host(r2), p.pos[:, sel], p.pos, sel, prec, f"nn subset {ni}")
    # disjoint i set, no self
    q = ics.plummer(400, 605)
    _, _, _, nn, r2 = ctx.force_nn(dev(q.pos), dev(q.vel), X, V, M, eps, prec=prec)
    torch.cuda.synchronize()
    check_nn(host(nn), host(r2), q.pos, p.pos, None, prec, "nn disjoint")


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_force_nn_exact_ties_take_lowest_index(ctx, prec):
    """Integer lattice points in shuffled order: distances are exact in
    float32, every interior point has six neighbours at distance 1, and the
    reported one must be the lowest index among them (bit-exact with the
    oracle), across j ranges as well."""
    import torch
    g = np.random.default_rng(7)
    L = 16
    grid = np.stack(np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij"), 0).reshape(3, -1)
    pos = grid[:, g.permutation(grid.shape[1])].astype(np.float64) - L / 2
    n = pos.shape[1]
    vel = np.zeros_like(pos)
    m = np.full(n, 1.0 / n)
    X, V, M = dev(pos), dev(vel), dev(m)
    for sel in (np.arange(n), np.sort(g.choice(n, 60, replace=False))):
        ref_nn, ref_r2 = oracle.nearest(pos[:, sel], pos, iself=sel)
        for eps in (0.1, 0.0):   # the softened and the unsoftened (eps = 0) kernels
            a, _, pt, nn, r2 = ctx.force_nn(X[:, sel].contiguous(), V[:, sel].contiguous(), X, V, M, eps,
                                            prec=prec, i_self=dev(sel.astype(np.int32)))
            torch.cuda.synchronize()
            assert np.array_equal(host(nn), ref_nn), eps
            assert np.array_equal(host(r2), ref_r2), eps
            assert np.all(np.isfinite(host(a))) and np.all(np.isfinite(host(pt)))


def test_force_nn_degenerate(ctx):
    import torch
    # the only j is i itself: no candidate
    x = dev(np.ones((3, 1))); v = dev(np.zeros((3, 1))); m = dev(np.ones(1))
    _, _, pt, nn, r2 = ctx.force_nn(x, v, x, v, m, 0.1, i_self=torch.zeros(1, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    assert host(nn).tolist() == [-1] and np.isinf(host(r2)[0]) and host(pt)[0] == 0.0
    # coincident distinct particles are neighbours at distance 0
    pos = np.array([[0.0, 0.0, 5.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    X, V = dev(pos), dev(np.zeros((3, 3)))
    _, _, _, nn, r2 = ctx.force_nn(X, V, X, V, dev(np.ones(3)), 0.1,
                                   i_self=torch.arange(3, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    assert host(nn).tolist() == [1, 0, 0] and host(r2).tolist() == [0.0, 0.0, 25.0]
    # empty j set
    e = torch.empty((3, 0), dtype=torch.float64, device="cuda")
    _, _, _, nn, r2 = ctx.force_nn(X, V, e, e, torch.empty((0,), dtype=torch.float64, device="cuda"), 0.1)
    torch.cuda.synchronize()
    assert host(nn).tolist() == [-1, -1, -1]


def test_plummer1m_acc_and_nn_sampled(ctx):
    """N = 2^20, eps = 1e-4, all particles evaluated (large launch shape);
    2048 seeded rows of the force-only and nearest-neighbour outputs against
    the oracle."""
    import torch
    p = ics.workload("plummer1m_force")
    eps = 1e-4
    sel = np.sort(np.random.default_rng(5).choice(p.n, 2048, replace=False))
    X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
    S = torch.arange(p.n, dtype=torch.int32, device="cuda")
    ref_a, ref_p = oracle.force_acc(p.pos[:, sel], p.pos, p.mass, eps, iself=sel)
    for prec in ("ds", "fp32"):
        a, pot = ctx.force_acc(X, X, M, eps, prec=prec, i_self=S)
        torch.cuda.synchronize()
        check_acc(host(a)[:, sel], host(pot)[sel], ref_a, ref_p, prec, "acc N=2^20 sampled")
        del a, pot
    _, _, _, nn, r2 = ctx.force_nn(X, V, X, V, M, eps, prec="ds", i_self=S)
    torch.cuda.synchronize()
    ref_nn, ref_r2 = oracle.nearest(p.pos[:, sel], p.pos, iself=sel)
    nn, r2 = host(nn)[sel], host(r2)[sel]
    d = ((p.pos[:, nn] - p.pos[:, sel]) ** 2).sum(0)
    assert np.all(d <= ref_r2 * (1 + NN_TOL["ds"]))
    agree = np.mean(nn == ref_nn)
    print("nn N=2^20 sampled agreement", agree, flush=True)
    assert agree > 0.99


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_leapfrog_against_oracle(ctx, prec):
    """N = 1024 Plummer, eps = 1/256, 32 kick-drift-kick steps of 1/256."""
    import torch
    p = ics.workload("plummer1k_hermite")
    eps, dt = 1.0 / 256, 1.0 / 256
    xr, vr, ar, pr = oracle.leapfrog(p.pos, p.vel, p.mass, eps, dt, 32)
    X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
    acc, pot = ctx.leapfrog(X, V, M, eps, dt, 32, prec=prec)
    torch.cuda.synchronize()
    dx, dv = np.abs(host(X) - xr).max(), np.abs(host(V) - vr).max()
    print(prec, "leapfrog max|dx|", dx, "max|dv|", dv, flush=True)
    assert dx < (1e-7 if prec == "ds" else 1e-5) and dv < (1e-6 if prec == "ds" else 1e-4)
    check_acc(host(acc), host(pot), ar, pr, prec, "leapfrog end")
    # two chained runs of 16 equal one run of 32, bit for bit
    X2, V2 = dev(p.pos), dev(p.vel)
    a2, _ = ctx.leapfrog(X2, V2, M, eps, dt, 16, prec=prec, want_pot=False)
    a2, pot2 = ctx.leapfrog(X2, V2, M, eps, dt, 16, acc=a2, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(X2, X) and torch.equal(V2, V) and torch.equal(a2, acc) and torch.equal(pot2, pot)
    # no steps: positions, velocities and the given acceleration stay; the potential is produced
    a3 = acc.clone()
    a3, pot3 = ctx.leapfrog(X2, V2, M, eps, dt, 0, acc=a3, prec=prec)
    torch.cuda.synchronize()
    assert torch.equal(a3, acc) and torch.equal(X2, X) and torch.equal(pot3, pot)
