"""Pins of the oracle's nearest-neighbour search (Section 3.3) and of the
force-only evaluation with its kick-drift-kick leapfrog (the acceleration-only
integration of Section 4): a k-d tree from scipy, exact ties on a lattice,
the self / empty cases, time reversibility, second-order convergence on an
analytic Kepler orbit, and chaining of runs."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import nbody_inputs as ics
import oracle
from test_oracle_hermite import kepler_state


def test_nearest_against_kdtree_self_set():
    p = ics.plummer(3000, 501)
    nn, r2 = oracle.nearest(p.pos, p.pos, iself=np.arange(p.n))
    d, k = cKDTree(p.pos.T).query(p.pos.T, k=2)
    # k-d tree column 0 is the point itself at distance 0 (no duplicates here)
    assert np.all(k[:, 0] == np.arange(p.n)) and np.all(d[:, 0] == 0)
    assert np.array_equal(nn, k[:, 1])
    np.testing.assert_allclose(r2, d[:, 1] ** 2, rtol=1e-12)


def test_nearest_against_kdtree_disjoint_and_subset():
    p = ics.plummer(2000, 502)
    q = ics.plummer(500, 503)
    nn, r2 = oracle.nearest(q.pos, p.pos)
    d, k = cKDTree(p.pos.T).query(q.pos.T, k=1)
    assert np.array_equal(nn, k)
    np.testing.assert_allclose(r2, d ** 2, rtol=1e-12)
    sel = np.sort(np.random.default_rng(1).choice(p.n, 300, replace=False))
    nn, _ = oracle.nearest(p.pos[:, sel], p.pos, iself=sel)
    _, k = cKDTree(p.pos.T).query(p.pos[:, sel].T, k=2)
    assert np.array_equal(nn, k[:, 1])


def test_nearest_ties_take_lowest_index():
    # i at the origin, six lattice neighbours at distance 1 given in a
    # shuffled order, plus farther points: the lowest index among the six
    g = np.random.default_rng(2)
    pts = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1), (2, 0, 0), (0, 3, 0)]
    order = g.permutation(len(pts))
    xj = np.array([pts[o] for o in order], dtype=float).T
    nn, r2 = oracle.nearest(np.zeros((3, 1)), xj)
    near = [k for k, o in enumerate(order) if o < 6]
    assert nn[0] == min(near) and r2[0] == 1.0
    # coincident distinct particles are neighbours at distance 0; self is not
    x = np.array([[0.0, 0.0, 5.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    nn, r2 = oracle.nearest(x, x, iself=np.arange(3))
    assert nn.tolist() == [1, 0, 0] and r2.tolist() == [0.0, 0.0, 25.0]


def test_nearest_without_candidates():
    x = np.ones((3, 1))
    nn, r2 = oracle.nearest(x, x, iself=np.array([0]))
    assert nn[0] == -1 and r2[0] == np.inf
    nn, r2 = oracle.nearest(x, np.zeros((3, 0)))
    assert nn[0] == -1 and r2[0] == np.inf


def test_force_acc_ignores_velocities():
    p = ics.plummer(400, 504)
    a, ph = oracle.force_acc(p.pos, p.pos, p.mass, 0.01, iself=np.arange(p.n))
    a2, _, ph2 = oracle.force(p.pos, p.vel, p.pos, p.vel, p.mass, 0.01, iself=np.arange(p.n))
    assert np.array_equal(a, a2) and np.array_equal(ph, ph2)


def test_leapfrog_time_reversible():
    p = ics.plummer(64, 505)
    x, v, a, _ = oracle.leapfrog(p.pos, p.vel, p.mass, 0.05, 1.0 / 256, 50)
    xb, vb, _, _ = oracle.leapfrog(x, -v, p.mass, 0.05, 1.0 / 256, 50, acc=a)
    assert np.abs(xb - p.pos).max() < 1e-12
    assert np.abs(vb + p.vel).max() < 1e-12


def kepler_lf_error(log2dt, t_end=1.0):
    m = np.array([0.6, 0.4])
    x0, v0 = kepler_state(0.6, 0.4, 1.0, 0.5, 0.0)
    dt = 2.0 ** log2dt
    x, v, _, _ = oracle.leapfrog(x0, v0, m, 0.0, dt, int(round(t_end / dt)))
    xe, _ = kepler_state(0.6, 0.4, 1.0, 0.5, t_end)
    return np.abs(x - xe).max()


def test_leapfrog_second_order_on_kepler():
    e8, e9, e10 = kepler_lf_error(-8), kepler_lf_error(-9), kepler_lf_error(-10)
    assert e10 < 1e-4
    assert 3.5 < e8 / e9 < 4.5 and 3.5 < e9 / e10 < 4.5


def test_leapfrog_energy_bounded_and_chaining():
    p = ics.plummer(256, 506)
    eps, dt = 0.05, 1.0 / 512
    e0 = sum(oracle.energy(p.pos, p.vel, p.mass, eps))
    x, v, a, pot = oracle.leapfrog(p.pos, p.vel, p.mass, eps, dt, 256)
    e1 = 0.5 * (p.mass * (v * v).sum(0)).sum() + 0.5 * (p.mass * pot).sum()
    assert e1 == pytest.approx(sum(oracle.energy(x, v, p.mass, eps)), rel=1e-13)
    assert abs((e1 - e0) / e0) < 1e-4
    # two runs of 128 steps chained through the returned acceleration equal one of 256
    xa, va, aa, _ = oracle.leapfrog(p.pos, p.vel, p.mass, eps, dt, 128)
    xb, vb, ab, potb = oracle.leapfrog(xa, va, p.mass, eps, dt, 128, acc=aa)
    assert np.array_equal(xb, x) and np.array_equal(vb, v) and np.array_equal(potb, pot)
