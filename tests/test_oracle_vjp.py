"""Pins of the oracle's force adjoint (vector-Jacobian product) against
finite differences, symmetry identities and homogeneity (Euler) identities.
None of them re-derives the adjoint formula."""
import numpy as np
import pytest

import oracle


def system(n, seed):
    g = np.random.default_rng(seed)
    return g.normal(0, 1, (3, n)), g.normal(0, 0.5, (3, n)), g.uniform(0.5, 1.5, n) / n


def loss(x, v, m, eps, ga, gj, gp, xi=None, vi=None, iself=None):
    xi = x if xi is None else xi
    vi = v if vi is None else vi
    a, j, p = oracle.force(xi, vi, x, v, m, eps, iself=iself)
    return (ga * a).sum() + (gj * j).sum() + (gp * p).sum()


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_vjp_directional_derivatives(eps):
    # <cotangent, directional FD> = <gradient, direction> for x, v and m.
    n = 24
    x, v, m = system(n, 1)
    g = np.random.default_rng(2)
    ga, gj, gp = g.normal(size=(3, n)), g.normal(size=(3, n)), g.normal(size=n)
    iself = np.arange(n)
    gxi, gvi, gxj, gvj, gmj = oracle.force_vjp(x, v, x, v, m, eps, ga, gj, gp, iself=iself)
    gx, gv = gxi + gxj, gvi + gvj
    h = 1e-6
    for name, grad in (("x", gx), ("v", gv), ("m", gmj)):
        d = g.normal(size=grad.shape)
        def f(t):
            xx, vv, mm = x.copy(), v.copy(), m.copy()
            if name == "x":
                xx += t * d
            elif name == "v":
                vv += t * d
            else:
                mm += t * d
            return loss(xx, vv, mm, eps, ga, gj, gp, iself=iself)
        fd = (f(h) - f(-h)) / (2 * h)
        assert fd == pytest.approx((grad * d).sum(), rel=2e-7, abs=1e-9)


def test_vjp_i_and_j_sides_separately():
    # Distinct i and j sets: the i-side and j-side cotangents each match FD.
    g = np.random.default_rng(3)
    xi, vi = g.normal(0, 1, (3, 7)), g.normal(0, 1, (3, 7))
    xj, vj, mj = g.normal(0, 1, (3, 11)), g.normal(0, 1, (3, 11)), g.uniform(0.1, 1, 11)
    ga, gj, gp = g.normal(size=(3, 7)), g.normal(size=(3, 7)), g.normal(size=7)
    eps = 0.1
    gxi, gvi, gxj, gvj, gmj = oracle.force_vjp(xi, vi, xj, vj, mj, eps, ga, gj, gp)
    h = 1e-6

    def L(xi_, vi_, xj_, vj_, mj_):
        a, j, p = oracle.force(xi_, vi_, xj_, vj_, mj_, eps)
        return (ga * a).sum() + (gj * j).sum() + (gp * p).sum()

    args = [xi, vi, xj, vj, mj]
    for k, grad in enumerate((gxi, gvi, gxj, gvj, gmj)):
        d = g.normal(size=grad.shape)
        up = [a.copy() for a in args]; dn = [a.copy() for a in args]
        up[k] += h * d; dn[k] -= h * d
        fd = (L(*up) - L(*dn)) / (2 * h)
        assert fd == pytest.approx((grad * d).sum(), rel=2e-7, abs=1e-9)


def test_vjp_translation_and_galilean_invariance():
    n = 40
    x, v, m = system(n, 4)
    g = np.random.default_rng(5)
    ga, gj, gp = g.normal(size=(3, n)), g.normal(size=(3, n)), g.normal(size=n)
    gxi, gvi, gxj, gvj, _ = oracle.force_vjp(x, v, x, v, m, 0.02, ga, gj, gp,
                                             iself=np.arange(n))
    sx = (gxi + gxj).sum(axis=1); sv = (gvi + gvj).sum(axis=1)
    scale = np.abs(gxi).sum()
    assert np.all(np.abs(sx) < 1e-12 * scale)
    assert np.all(np.abs(sv) < 1e-12 * np.abs(gvi).sum())


def test_vjp_euler_homogeneity():
    # Outputs are linear in the masses: sum_k m_k dL/dm_k = L.
    # With eps = 0 they are homogeneous in (x, v) -> (l x, l v) of degree -2
    # (a, jerk) and -1 (phi); in v alone, jerk has degree 1 and a, phi 0.
    n = 30
    x, v, m = system(n, 6)
    g = np.random.default_rng(7)
    ga, gj, gp = g.normal(size=(3, n)), g.normal(size=(3, n)), g.normal(size=n)
    iself = np.arange(n)
    a, j, p = oracle.force(x, v, x, v, m, 0.0, iself=iself)
    La, Lj, Lp = (ga * a).sum(), (gj * j).sum(), (gp * p).sum()
    gxi, gvi, gxj, gvj, gmj = oracle.force_vjp(x, v, x, v, m, 0.0, ga, gj, gp, iself=iself)
    assert (m * gmj).sum() == pytest.approx(La + Lj + Lp, rel=1e-12)
    gx, gv = gxi + gxj, gvi + gvj
    assert (x * gx).sum() + (v * gv).sum() == pytest.approx(-2 * La - 2 * Lj - Lp, rel=1e-11)
    assert (v * gv).sum() == pytest.approx(Lj, rel=1e-11)


def test_vjp_null_cotangents_equal_zero_cotangents():
    n = 12
    x, v, m = system(n, 8)
    ga = np.random.default_rng(9).normal(size=(3, n))
    r1 = oracle.force_vjp(x, v, x, v, m, 0.1, ga, None, None, iself=np.arange(n))
    r2 = oracle.force_vjp(x, v, x, v, m, 0.1, ga, np.zeros((3, n)), np.zeros(n),
                          iself=np.arange(n))
    for a, b in zip(r1, r2):
        np.testing.assert_array_equal(a, b)


def test_stored_central_differences_match_adjoint_at_full_size():
    """tests/golden/adjoint16k_fd.json (written from the oracle alone by
    make_adjoint16k_fd.py): at the full differentiation recipe (N = 16384,
    eps = 1e-3, 64 Hermite steps of 1/128, L = sum w.x(T)), central differences
    of L with h = 1e-6 agree with the oracle's adjoint of the same run, 32
    seeded coordinates.  Positions and velocities: the difference is set by
    the rounding noise of L over 2h, about 1e-6 of the gradients' rms.
    Masses (m = 1/16384): h moves a mass by 1.6 %, so the O(h^2) truncation
    of the central difference dominates; the bar is 1e-3 of the rms."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "adjoint16k_fd.json")) as f:
        d = json.load(f)
    assert d["recipe"]["n"] == 16384 and d["h"] == 1e-6
    kinds = {k: [e for e in d["entries"] if e["kind"] == k] for k in "xvm"}
    assert len(kinds["x"]) >= 8 and len(kinds["v"]) >= 8 and len(kinds["m"]) >= 8
    for k, bar in (("x", 5e-6), ("v", 5e-6), ("m", 1e-3)):
        fd = np.array([e["fd"] for e in kinds[k]])
        ad = np.array([e["oracle_adjoint"] for e in kinds[k]])
        rms = np.sqrt(np.mean(fd * fd))
        err = np.abs(fd - ad) / rms
        assert err.max() <= bar, (k, err.max())
        assert np.median(np.abs(fd - ad) / np.abs(fd)) <= 1e-5, k
