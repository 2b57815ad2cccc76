"""GPU parity of the differentiable shared-step Hermite run: forward against
the oracle's run, gradient against the oracle's adjoint and against central
finite differences of the float64 oracle, autograd plumbing, and the
translation / boost identities at the full differentiation workload."""
import numpy as np
import pytest

import nbody_inputs as ics
import oracle
from gpu_util import dev, elem_err_stats, host, mass_grad_scale, rel_err_stats, scaled_err_stats

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_0707_0438_amd as nb
    c = nb.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_shared_run_matches_oracle(ctx, prec):
    import torch
    p = ics.plummer(700, 401)
    eps, dt, steps = 1e-3, 1.0 / 128, 16
    xr, vr = oracle.hermite_shared_forward(p.pos, p.vel, p.mass, eps, dt, steps)
    xT, vT, _ = ctx.shared_run(dev(p.pos), dev(p.vel), dev(p.mass), eps, dt, steps, prec=prec,
                               checkpoints=False)
    torch.cuda.synchronize()
    dx = np.abs(host(xT) - xr).max()
    dv = np.abs(host(vT) - vr).max()
    print(prec, "shared run max|dx|", dx, "max|dv|", dv, flush=True)
    assert dx < (1e-7 if prec == "ds" else 1e-4)
    assert dv < (1e-6 if prec == "ds" else 1e-3)


@pytest.mark.parametrize("prec,every", [("ds", 5), ("ds", 16), ("fp32", 3)])
def test_shared_adjoint_matches_oracle(ctx, prec, every):
    import torch
    p = ics.plummer(400, 402)
    eps, dt, steps = 1e-2, 1.0 / 128, 13
    w = np.random.default_rng(8).normal(size=(3, p.n))
    rx, rv, rm = oracle.hermite_shared_adjoint(p.pos, p.vel, p.mass, eps, dt, steps, w)
    X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
    _, _, ck = ctx.shared_run(X, V, M, eps, dt, steps, prec=prec, ckpt_every=every)
    gx, gv, gm = ctx.shared_adjoint(X, V, M, eps, dt, steps, ck, dev(w), prec=prec, ckpt_every=every)
    torch.cuda.synchronize()
    st = {"gx0": rel_err_stats(host(gx), rx), "gv0": rel_err_stats(host(gv), rv),
          "gm": scaled_err_stats(host(gm), rm)}
    print(prec, every, {k: f"p99={v['p99']:.2e} max={v['max']:.2e}" for k, v in st.items()}, flush=True)
    bar = 1e-4 if prec == "ds" else 1e-2
    for k in st:
        assert st[k]["p99"] <= bar, (k, st[k])


def test_gradient_against_oracle_finite_differences(ctx):
    """The differentiation recipe (eps = 1e-3, dt = 1/128, 64 steps,
    checkpoints every 8, L = sum w.x(T)) at N = 1024: GPU gradient against
    central differences (h = 1e-6) of the float64 oracle run on 32 seeded
    coordinates (>= 8 each from x, v, m)."""
    import torch
    p = ics.plummer(1024, ics.seed_for(3))
    eps, dt, steps = 1e-3, 1.0 / 128, 64
    w = ics.rng(ics.seed_for(3), 9).normal(size=(3, p.n))
    X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
    _, _, ck = ctx.shared_run(X, V, M, eps, dt, steps, ckpt_every=8)
    gx, gv, gm = ctx.shared_adjoint(X, V, M, eps, dt, steps, ck, dev(w), ckpt_every=8)
    torch.cuda.synchronize()
    gx, gv, gm = host(gx), host(gv), host(gm)

    def L(x0, v0, m):
        x, _ = oracle.hermite_shared_forward(x0, v0, m, eps, dt, steps)
        return float((w * x).sum())

    g = np.random.default_rng(11)
    h = 1e-6
    worst = 0.0
    picks = [("x", int(g.integers(p.n)), int(g.integers(3))) for _ in range(11)] + \
            [("v", int(g.integers(p.n)), int(g.integers(3))) for _ in range(11)] + \
            [("m", int(g.integers(p.n)), 0) for _ in range(10)]
    for kind, i, c in picks:
        x0, v0, m = p.pos.copy(), p.vel.copy(), p.mass.copy()
        xp, vp, mp = x0.copy(), v0.copy(), m.copy()
        xm, vm, mm = x0.copy(), v0.copy(), m.copy()
        if kind == "x":
            xp[c, i] += h; xm[c, i] -= h; ana = gx[c, i]
        elif kind == "v":
            vp[c, i] += h; vm[c, i] -= h; ana = gv[c, i]
        else:
            mp[i] += h; mm[i] -= h; ana = gm[i]
        fd = (L(xp, vp, mp) - L(xm, vm, mm)) / (2 * h)
        err = abs(ana - fd) / max(abs(fd), 1e-3)
        worst = max(worst, err)
        assert err < 1e-3, (kind, i, c, ana, fd)
    print("worst relative FD mismatch", worst, flush=True)


def test_autograd_functions(ctx):
    import torch
    from paper_0707_0438_amd.autograd import HermiteShared, NBodyForce
    p = ics.plummer(300, 403)
    X = dev(p.pos).requires_grad_(True)
    V = dev(p.vel).requires_grad_(True)
    M = dev(p.mass).requires_grad_(True)
    w = dev(np.random.default_rng(12).normal(size=(3, p.n)))
    xT, vT = HermiteShared.apply(ctx, X, V, M, 1e-2, 1.0 / 64, 10, 4)
    (w * xT).sum().backward()
    rx, rv, rm = oracle.hermite_shared_adjoint(p.pos, p.vel, p.mass, 1e-2, 1.0 / 64, 10, host(w))
    assert rel_err_stats(host(X.grad), rx)["p99"] < 1e-4
    assert scaled_err_stats(host(M.grad), rm)["p99"] < 1e-4
    X.grad = None; V.grad = None; M.grad = None
    a, j, pt = NBodyForce.apply(ctx, X, V, M, 0.05)
    ga = np.random.default_rng(13).normal(size=(3, p.n))
    (dev(ga) * a).sum().backward()
    ref = oracle.force_vjp(p.pos, p.vel, p.pos, p.vel, p.mass, 0.05, ga, iself=np.arange(p.n))
    assert rel_err_stats(host(X.grad), ref[0] + ref[2])["p99"] < 1e-5
    sc = mass_grad_scale(p.pos, p.vel, p.pos, p.vel, 0.05, ga, iself=np.arange(p.n))
    assert elem_err_stats(host(M.grad), ref[4], sc)["p99"] < 1e-5


def test_plummer16k_gradient_identities(ctx):
    """Full differentiation workload (N = 16384, eps = 1e-3, 64 steps of
    1/128, checkpoints every 8): shifting every x0 by c shifts x(T) by c and
    boosting every v0 by u shifts x(T) by u T, so sum_k gx0_k = sum_i w_i
    and sum_k gv0_k = T sum_i w_i, at any size."""
    import torch
    p = ics.workload("plummer16k_adjoint")
    eps, dt, steps = 1e-3, 1.0 / 128, 64
    w = ics.rng(ics.seed_for(3), 9).normal(size=(3, p.n))
    X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
    _, _, ck = ctx.shared_run(X, V, M, eps, dt, steps, ckpt_every=8)
    gx, gv, gm = ctx.shared_adjoint(X, V, M, eps, dt, steps, ck, dev(w), ckpt_every=8)
    torch.cuda.synchronize()
    gx, gv = host(gx), host(gv)
    sw = w.sum(axis=1)
    ex = np.abs(gx.sum(axis=1) - sw).max() / np.abs(w).sum()
    ev = np.abs(gv.sum(axis=1) - steps * dt * sw).max() / (steps * dt * np.abs(w).sum())
    print("translation", ex, "boost", ev, flush=True)
    assert ex < 1e-6 and ev < 1e-6
    assert np.all(np.isfinite(host(gm)))


def test_plummer16k_gradient_against_oracle_adjoint(ctx):
    """The full differentiation workload (N = 16384, eps = 1e-3, 64 steps of
    1/128, checkpoints every 8, L = sum w.x(T)): every gradient component
    against the float64 oracle's adjoint of the same run, and 32 seeded
    components (11 of x0, 11 of v0, 10 masses) against central finite
    differences (h = 1e-6) of the float64 oracle's run, stored in
    tests/golden/adjoint16k_fd.json by make_adjoint16k_fd.py (oracle only).
    About a minute of host time for the oracle adjoint."""
    import json
    import os
    import torch
    p = ics.workload("plummer16k_adjoint")
    eps, dt, steps = 1e-3, 1.0 / 128, 64
    w = ics.rng(ics.seed_for(3), 9).normal(size=(3, p.n))
    with open(os.path.join(os.path.dirname(__file__), "golden", "adjoint16k_fd.json")) as f:
        fd = json.load(f)
    assert fd["recipe"]["n"] == p.n and fd["h"] == 1e-6 and len(fd["entries"]) == 32
    rx, rv, rm = oracle.hermite_shared_adjoint(p.pos, p.vel, p.mass, eps, dt, steps, w)
    X, V, M, W = dev(p.pos), dev(p.vel), dev(p.mass), dev(w)
    for prec, bar in (("ds", 1e-4), ("fp32", 1e-3)):
        _, _, ck = ctx.shared_run(X, V, M, eps, dt, steps, prec=prec, ckpt_every=8)
        gx, gv, gm = ctx.shared_adjoint(X, V, M, eps, dt, steps, ck, W, prec=prec, ckpt_every=8)
        torch.cuda.synchronize()
        gx, gv, gm = host(gx), host(gv), host(gm)
        st = {"gx0": rel_err_stats(gx, rx), "gv0": rel_err_stats(gv, rv),
              "gm": scaled_err_stats(gm, rm)}
        print(prec, "N=16384", {k: f"p99={v['p99']:.2e} max={v['max']:.2e}" for k, v in st.items()}, flush=True)
        for k in st:
            assert st[k]["p99"] <= bar, (prec, k, st[k])
        # against the oracle's central differences, element by element
        worst = 0.0
        for e in fd["entries"]:
            ana = {"x": gx, "v": gv}[e["kind"]][e["c"], e["i"]] if e["kind"] != "m" else gm[e["i"]]
            err = abs(ana - e["fd"]) / max(abs(e["fd"]), 1e-3)
            worst = max(worst, err)
            if prec == "ds":
                assert err <= 1e-3, (e, ana)
        print(prec, "N=16384 worst relative mismatch against finite differences", f"{worst:.2e}", flush=True)
