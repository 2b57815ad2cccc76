"""GPU parity of the GRAPE-6-style interface (include/nbody_grape.h): j
particles set one by one with their own times, predicted on the device,
force, jerk, potential and nearest neighbour of i groups against the float64
oracle, identities distinct from addresses, i-particles outside the j set,
partial j sets, updates between steps and the call-order errors."""
import numpy as np
import pytest

import nbody_inputs as ics
import oracle
from gpu_util import BARS, rel_err_stats

pytestmark = pytest.mark.gpu


def system(n, seed):
    p = ics.plummer(n, seed)
    a, j, _ = oracle.force(p.pos, p.vel, p.pos, p.vel, p.mass, 0.01, iself=np.arange(n))
    g = np.random.default_rng(seed)
    tj = g.integers(0, 8, n) / 256.0          # each particle at its own time
    ident = 1000 + g.permutation(n)            # identities differ from addresses
    return p, a, j, tj, ident


def predicted(p, a, j, tj, ti):
    xp = np.empty_like(p.pos); vp = np.empty_like(p.vel)
    for k in range(p.n):
        xp[:, k], vp[:, k] = oracle.predict(p.pos[:, k], p.vel[:, k], a[:, k], j[:, k], ti - tj[k])
    return xp, vp


@pytest.fixture(scope="module")
def grape():
    import paper_0707_0438_amd as nb
    g = nb.Grape(0)
    yield g
    g.close()


def load(g, p, a, j, tj, ident, order):
    for k in order:
        g.set_j_particle(k, ident[k], tj[k], p.mass[k], p.pos[:, k], p.vel[:, k], a[:, k], j[:, k])


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_grape_sequence_against_oracle(grape, prec):
    n, eps = 2000, 0.01
    p, a, j, tj, ident = system(n, 701)
    grape.set_precision(prec)
    load(grape, p, a, j, tj, ident, np.random.default_rng(1).permutation(n))
    ti = 8 / 256.0
    grape.set_ti(ti)
    xp, vp = predicted(p, a, j, tj, ti)
    sel = np.sort(np.random.default_rng(2).choice(n, 300, replace=False))
    grape.calc_firsthalf(n, ident[sel], xp[:, sel].T, vp[:, sel].T, eps * eps)
    acc, jerk, pot, nnb = grape.calc_lasthalf(sel.size, nn=True)
    ra, rj, rp = oracle.force(xp[:, sel], vp[:, sel], xp, vp, p.mass, eps, iself=sel)
    for k, g_, r in (("acc", acc.T, ra), ("jerk", jerk.T, rj), ("pot", pot, rp)):
        st = rel_err_stats(g_, r)
        print(prec, k, f"p99={st['p99']:.2e}", flush=True)
        assert st["p99"] <= BARS[prec][k], (k, st)
    nn_ref, _ = oracle.nearest(xp[:, sel], xp, iself=sel)
    agree = np.mean(nnb == ident[nn_ref])
    print(prec, "nearest-neighbour agreement", agree, flush=True)
    assert agree > 0.99
    # i-particles outside the j set: the given positions, nothing excluded
    q = ics.plummer(50, 702)
    grape.calc_firsthalf(n, np.arange(50) + 10 ** 6, q.pos.T, q.vel.T, eps * eps)
    acc, jerk, pot = grape.calc_lasthalf(50)
    ra, rj, rp = oracle.force(q.pos, q.vel, xp, vp, p.mass, eps)
    assert rel_err_stats(acc.T, ra)["p99"] <= BARS[prec]["acc"]
    assert rel_err_stats(pot, rp)["p99"] <= BARS[prec]["pot"]
    # the first nj addresses only
    nj = 1200
    sub = sel[sel < nj]
    grape.calc_firsthalf(nj, ident[sub], xp[:, sub].T, vp[:, sub].T, eps * eps)
    acc, _, pot = grape.calc_lasthalf(sub.size)
    ra, _, rp = oracle.force(xp[:, sub], vp[:, sub], xp[:, :nj], vp[:, :nj], p.mass[:nj], eps, iself=sub)
    assert rel_err_stats(acc.T, ra)["p99"] <= BARS[prec]["acc"]
    grape.set_precision("ds")


def test_grape_updates_and_call_order(grape):
    import paper_0707_0438_amd as nb
    n, eps = 800, 0.02
    p, a, j, tj, ident = system(n, 703)
    load(grape, p, a, j, tj, ident, range(n))
    grape.set_ti(0.05)
    # move ten particles to a later time and state, then step again
    moved = np.arange(0, n, 80)
    p2 = ics.plummer(n, 704)
    for k in moved:
        p.pos[:, k] = p2.pos[:, k]; p.vel[:, k] = p2.vel[:, k]; tj[k] = 0.0625
        grape.set_j_particle(k, ident[k], tj[k], p.mass[k], p.pos[:, k], p.vel[:, k], a[:, k], j[:, k])
    with pytest.raises(nb.NBodyError):   # j data changed since the last set_ti
        grape.calc_firsthalf(n, ident[:5], np.zeros((5, 3)), np.zeros((5, 3)), eps * eps)
    ti = 0.0625
    grape.set_ti(ti)
    xp, vp = predicted(p, a, j, tj, ti)
    grape.set_nn(False)
    grape.calc_firsthalf(n, ident[moved], xp[:, moved].T, vp[:, moved].T, eps * eps)
    with pytest.raises(nb.NBodyError):   # nearest neighbour was not enabled
        grape.calc_lasthalf(moved.size, nn=True)
    with pytest.raises(nb.NBodyError):   # a calculation is still pending
        grape.calc_firsthalf(n, ident[moved], xp[:, moved].T, vp[:, moved].T, eps * eps)
    with pytest.raises(nb.NBodyError):   # ni differs from the pending call
        grape.calc_lasthalf(moved.size + 1)
    acc, jerk, pot = grape.calc_lasthalf(moved.size)
    ra, rj, rp = oracle.force(xp[:, moved], vp[:, moved], xp, vp, p.mass, eps, iself=moved)
    assert rel_err_stats(acc.T, ra)["p99"] <= BARS["ds"]["acc"]
    assert rel_err_stats(jerk.T, rj)["p99"] <= BARS["ds"]["jerk"]
    with pytest.raises(nb.NBodyError):   # nothing pending
        grape.calc_lasthalf(moved.size)
    grape.set_nn(True)
