"""Pins of the FP64 oracle's force, jerk and potential against facts that do
not come from the oracle itself: two-body closed forms, Newton's third law,
a = -grad(phi), jerk = da/dt along the motion, the analytic Plummer mean
field, and the exclusion rules of Section 3.1 / 3.3.

Each test is chosen so that a plausible slip in the oracle (a dropped jerk
term, a wrong sign or index, a transposed row) fails at least one of them.
"""
import math

import numpy as np
import pytest

import nbody_inputs as ics
import oracle


def rand_system(n, seed, spread=1.0):
    g = np.random.default_rng(seed)
    x = g.normal(0, spread, (3, n))
    v = g.normal(0, 0.5, (3, n))
    m = g.uniform(0.5, 1.5, n) / n
    return x, v, m


# ---- two-body closed forms ----------------------------------------------------

@pytest.mark.parametrize("eps", [0.0, 0.1, 1.0 / 256])
def test_two_body_static_closed_form(eps):
    # particle 0 at origin, particle 1 (mass M) at distance d on the y axis:
    # softened attraction G M d / (d^2 + eps^2)^(3/2) toward particle 1,
    # potential -G M / sqrt(d^2 + eps^2).
    d, M, G = 0.7, 0.3, 2.0
    x = np.array([[0.0, 0.0], [0.0, d], [0.0, 0.0]])
    v = np.zeros((3, 2))
    m = np.array([0.5, M])
    acc, jerk, pot = oracle.force(x, v, x, v, m, eps, G=G, iself=[0, 1])
    s = d * d + eps * eps
    assert acc[1, 0] == pytest.approx(G * M * d / s ** 1.5, rel=1e-15)
    assert acc[0, 0] == 0.0 and acc[2, 0] == 0.0
    assert acc[1, 1] == pytest.approx(-G * 0.5 * d / s ** 1.5, rel=1e-15)
    assert pot[0] == pytest.approx(-G * M / math.sqrt(s), rel=1e-15)
    assert pot[1] == pytest.approx(-G * 0.5 / math.sqrt(s), rel=1e-15)
    assert np.all(jerk == 0.0)


def test_two_body_jerk_radial_and_tangential():
    # Unsoftened: for separation d and relative velocity u,
    #  radial u: d/dt (G M / d^2) = -2 G M u / d^3 (along the line)
    #  tangential u: the direction turns, |jerk| = G M u / d^3 along u.
    d, M, u = 1.3, 0.8, 0.25
    x = np.array([[0.0, d], [0.0, 0.0], [0.0, 0.0]])
    m = np.array([1.0, M])
    vr = np.array([[0.0, u], [0.0, 0.0], [0.0, 0.0]])  # particle 1 recedes along +x
    _, jr, _ = oracle.force(x, vr, x, vr, m, 0.0, iself=[0, 1])
    # a_0 = +G M / d^2 x-hat; receding: magnitude falls
    assert jr[0, 0] == pytest.approx(-2.0 * M * u / d ** 3, rel=1e-14)
    assert abs(jr[1, 0]) < 1e-18 and abs(jr[2, 0]) < 1e-18
    vt = np.array([[0.0, 0.0], [0.0, u], [0.0, 0.0]])  # particle 1 moves along +y
    _, jt, _ = oracle.force(x, vt, x, vt, m, 0.0, iself=[0, 1])
    assert jt[1, 0] == pytest.approx(M * u / d ** 3, rel=1e-14)
    assert abs(jt[0, 0]) < 1e-18 and abs(jt[2, 0]) < 1e-18


# ---- invariants ---------------------------------------------------------------

@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_newton_third_law(eps):
    x, v, m = rand_system(300, 1)
    acc, jerk, _ = oracle.force(x, v, x, v, m, eps, iself=np.arange(300))
    for q in (acc, jerk):
        tot = (q * m).sum(axis=1)
        scale = (np.abs(q) * m).sum()
        assert np.all(np.abs(tot) <= 1e-13 * scale)


def test_acc_is_minus_grad_potential():
    x, v, m = rand_system(40, 2)
    eps = 0.01
    acc, _, _ = oracle.force(x, v, x, v, m, eps, iself=np.arange(40))
    h = 1e-6
    for i in (0, 7, 39):
        for k in range(3):
            xp = x.copy(); xp[k, i] += h
            xm = x.copy(); xm[k, i] -= h
            _, _, pp = oracle.force(xp[:, i:i + 1], v[:, i:i + 1], xp, v, m, eps, iself=[i])
            _, _, pm = oracle.force(xm[:, i:i + 1], v[:, i:i + 1], xm, v, m, eps, iself=[i])
            g = (pp[0] - pm[0]) / (2 * h)
            assert -g == pytest.approx(acc[k, i], rel=1e-7, abs=1e-9 * np.abs(acc[:, i]).max())


def test_jerk_is_time_derivative_of_acc():
    x, v, m = rand_system(50, 3)
    eps = 0.02
    n = 50
    _, jerk, _ = oracle.force(x, v, x, v, m, eps, iself=np.arange(n))
    h = 1e-6
    ap, _, _ = oracle.force(x + h * v, v, x + h * v, v, m, eps, iself=np.arange(n))
    am, _, _ = oracle.force(x - h * v, v, x - h * v, v, m, eps, iself=np.arange(n))
    fd = (ap - am) / (2 * h)
    scale = np.abs(jerk).max(axis=0)
    assert np.all(np.abs(fd - jerk) <= 1e-7 * scale + 1e-12)


def test_i_list_subset_matches_full_rows():
    # An i-list evaluated against all j equals the matching rows of the
    # full evaluation (self excluded by index).
    x, v, m = rand_system(64, 4)
    sel = np.array([5, 0, 63, 17])
    af, jf, pf = oracle.force(x, v, x, v, m, 0.01, iself=np.arange(64))
    a, j, p = oracle.force(x[:, sel], v[:, sel], x, v, m, 0.01, iself=sel)
    assert np.array_equal(a, af[:, sel]) and np.array_equal(j, jf[:, sel])
    assert np.array_equal(p, pf[sel])


def test_self_excluded_by_index_not_distance():
    # Two distinct particles at the same point with eps > 0 do interact in
    # the potential (-m/eps each), while the self term is removed.
    eps = 0.1
    x = np.zeros((3, 3)); x[0, 2] = 0.5
    v = np.zeros((3, 3))
    m = np.array([0.2, 0.3, 0.5])
    _, _, pot = oracle.force(x, v, x, v, m, eps, iself=[0, 1, 2])
    assert pot[0] == pytest.approx(-0.3 / eps - 0.5 / math.sqrt(0.25 + eps * eps), rel=1e-15)
    _, _, pot_noself = oracle.force(x, v, x, v, m, eps, iself=None)
    assert pot_noself[0] == pytest.approx(pot[0] - 0.2 / eps, rel=1e-15)


def test_zero_softening_skips_coincident_pair():
    x = np.zeros((3, 3)); x[0, 2] = 2.0
    v = np.zeros((3, 3))
    m = np.array([1.0, 1.0, 1.0])
    acc, _, pot = oracle.force(x, v, x, v, m, 0.0, iself=None)
    assert np.all(np.isfinite(acc)) and np.all(np.isfinite(pot))
    assert acc[0, 0] == pytest.approx(1.0 / 4.0)
    assert pot[0] == pytest.approx(-0.5)


def test_linear_in_masses_and_G():
    x, v, m = rand_system(30, 5)
    a1, j1, p1 = oracle.force(x, v, x, v, m, 0.03, iself=np.arange(30))
    a2, j2, p2 = oracle.force(x, v, x, v, 2.0 * m, 0.03, G=3.0, iself=np.arange(30))
    np.testing.assert_allclose(a2, 6.0 * a1, rtol=1e-14)
    np.testing.assert_allclose(j2, 6.0 * j1, rtol=1e-14, atol=1e-14 * np.abs(j1).max())
    np.testing.assert_allclose(p2, 6.0 * p1, rtol=1e-14)


# ---- Plummer mean field (pins the sampler and the force together) ------------

def test_plummer_mean_field_and_virial():
    n = 1 << 15
    p = ics.plummer(n, 12345)
    b = ics.PLUMMER_B
    g = np.random.default_rng(0)
    sel = np.sort(g.choice(n, 3000, replace=False))
    acc, _, pot = oracle.force(p.pos[:, sel], p.vel[:, sel], p.pos, p.vel, p.mass, 1e-4,
                               iself=sel)
    r = np.linalg.norm(p.pos[:, sel], axis=0)
    ar = (acc * p.pos[:, sel]).sum(axis=0) / r          # radial component
    # analytic Plummer (M = 1, G = 1): a_r = -r / (r^2 + b^2)^(3/2)
    ana = -r / (r * r + b * b) ** 1.5
    bins = np.quantile(r, np.linspace(0.05, 0.9, 8))
    for lo, hi in zip(bins[:-1], bins[1:]):
        w = (r >= lo) & (r < hi)
        assert abs(ar[w].mean() / ana[w].mean() - 1.0) < 0.03
    # potential: phi = -1 / sqrt(r^2 + b^2)
    np.testing.assert_allclose(pot.mean(), (-1 / np.sqrt(r * r + b * b)).mean(), rtol=0.02)
    # virial equilibrium and E = -1/4 in N-body units
    ek, ep = oracle.energy(p.pos, p.vel, p.mass, 1e-4)
    assert abs(2 * ek / abs(ep) - 1.0) < 0.05
    assert abs((ek + ep) / -0.25 - 1.0) < 0.05


def test_tiny_n_brute_force_high_precision():
    # Independent evaluation at 40 digits (mpmath) on tiny N: the FP64 oracle
    # must agree to rounding level.
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    x, v, m = rand_system(9, 6)
    eps = 0.05
    acc, jerk, pot = oracle.force(x, v, x, v, m, eps, iself=np.arange(9))
    for i in range(9):
        A = [mp.mpf(0)] * 3; J = [mp.mpf(0)] * 3; P = mp.mpf(0)
        for j in range(9):
            if j == i:
                continue
            r = [mp.mpf(x[k, j]) - mp.mpf(x[k, i]) for k in range(3)]
            u = [mp.mpf(v[k, j]) - mp.mpf(v[k, i]) for k in range(3)]
            s = sum(q * q for q in r) + mp.mpf(eps) ** 2
            ru = sum(r[k] * u[k] for k in range(3))
            for k in range(3):
                A[k] += mp.mpf(m[j]) * r[k] / s ** 1.5
                J[k] += mp.mpf(m[j]) * (u[k] / s ** 1.5 - 3 * ru * r[k] / s ** 2.5)
            P -= mp.mpf(m[j]) / mp.sqrt(s)
        for k in range(3):
            assert abs(float(A[k]) - acc[k, i]) <= 1e-14 * abs(float(A[k])) + 1e-300
            assert abs(float(J[k]) - jerk[k, i]) <= 1e-13 * max(abs(float(J[k])), 1e-12)
        assert abs(float(P) - pot[i]) <= 1e-14 * abs(float(P))
