"""Pins of the oracle's Hermite integrator (Section 3, after Makino & Aarseth
1992) and block time steps (Section 3.1): corrector exactness on a cubic
acceleration, fourth-order convergence on an analytic Kepler orbit, the
integer block-selection and step-level rules, energy conservation, and the
shared-step adjoint against finite differences."""
import json
import math
import os

import numpy as np
import pytest

import nbody_inputs as ics
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TICK = 2.0 ** -20


def test_corrector_exact_on_cubic_acceleration():
    # a(t) = c0 + c1 t + c2 t^2/2 + c3 t^3/6 exactly: the interpolated second
    # and third derivatives and the corrected x, v equal the exact integrals.
    g = np.random.default_rng(0)
    c0, c1, c2, c3 = (g.normal(size=3) for _ in range(4))
    x0, v0 = g.normal(size=3), g.normal(size=3)
    D = 0.37
    a1 = c0 + c1 * D + c2 * D ** 2 / 2 + c3 * D ** 3 / 6
    j1 = c1 + c2 * D + c3 * D ** 2 / 2
    xp, vp = oracle.predict(x0, v0, c0, c1, D)
    np.testing.assert_allclose(xp, x0 + v0 * D + c0 * D ** 2 / 2 + c1 * D ** 3 / 6, rtol=1e-15)
    x1, v1, a2, a3 = oracle.correct(xp, vp, c0, c1, a1, j1, D)
    np.testing.assert_allclose(a2, c2, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(a3, c3, rtol=1e-11, atol=1e-11)
    xe = x0 + v0 * D + c0 * D ** 2 / 2 + c1 * D ** 3 / 6 + c2 * D ** 4 / 24 + c3 * D ** 5 / 120
    ve = v0 + c0 * D + c1 * D ** 2 / 2 + c2 * D ** 3 / 6 + c3 * D ** 4 / 24
    np.testing.assert_allclose(x1, xe, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(v1, ve, rtol=1e-14, atol=1e-15)


def kepler_state(m1, m2, a, e, t):
    """Two-body positions/velocities about the centre of mass, pericentre at
    t = 0 on +x, solved from Kepler's equation M = E - e sin E."""
    M = m1 + m2
    n = math.sqrt(M / a ** 3)
    Mean = n * t
    E = Mean
    for _ in range(60):
        E -= (E - e * math.sin(E) - Mean) / (1 - e * math.cos(E))
    rel = np.array([a * (math.cos(E) - e), a * math.sqrt(1 - e * e) * math.sin(E), 0.0])
    Edot = n / (1 - e * math.cos(E))
    relv = np.array([-a * math.sin(E) * Edot, a * math.sqrt(1 - e * e) * math.cos(E) * Edot, 0.0])
    x = np.stack([-m2 / M * rel, m1 / M * rel], axis=1)
    v = np.stack([-m2 / M * relv, m1 / M * relv], axis=1)
    return x, v


def kepler_error(log2dt, t_end=1.0):
    m = np.array([0.6, 0.4])
    x0, v0 = kepler_state(0.6, 0.4, 1.0, 0.5, 0.0)
    st = oracle.HermiteState(x0, v0, m)
    oracle.hermite_run(st, int(t_end / TICK), eps=0.0, shared_log2=log2dt, init=True)
    xe, ve = kepler_state(0.6, 0.4, 1.0, 0.5, t_end)
    assert np.all(st.t == int(t_end / TICK))
    return np.abs(st.x - xe).max(), st


def test_kepler_fourth_order_convergence():
    e6, _ = kepler_error(-6)
    e7, _ = kepler_error(-7)
    e8, _ = kepler_error(-8)
    assert e8 < 1e-7
    assert 11.0 < e6 / e7 < 22.0
    assert 11.0 < e7 / e8 < 22.0


def test_kepler_energy_and_angular_momentum():
    _, st = kepler_error(-8, t_end=2.0)
    m = st.m
    def E(x, v):
        r = np.linalg.norm(x[:, 1] - x[:, 0])
        return 0.5 * (m * (v * v).sum(axis=0)).sum() - m[0] * m[1] / r
    def L(x, v):
        return (m * np.cross(x.T, v.T).T).sum(axis=1)
    x0, v0 = kepler_state(0.6, 0.4, 1.0, 0.5, 0.0)
    assert abs(E(st.x, st.v) / E(x0, v0) - 1) < 1e-8
    assert abs(L(st.x, st.v)[2] / L(x0, v0)[2] - 1) < 1e-8


def test_quantise_golden_cases():
    with open(os.path.join(GOLDEN, "quantise_cases.json")) as f:
        cases = json.load(f)["cases"]
    for crit, dt_old, t_new, lmin, lmax, want, why in cases:
        c = float(crit) if not isinstance(crit, str) else float(crit)
        got = oracle.quantise_dt(c, dt_old, t_new, lmin, lmax)
        assert got == want, why


def test_select_active_brute_force():
    g = np.random.default_rng(1)
    for trial in range(50):
        n = int(g.integers(1, 400))
        lv = g.integers(0, 8, n)
        dt = (1 << (10 + lv)).astype(np.int64)
        t = (g.integers(0, 64, n) * dt).astype(np.int64)
        idx, tn = oracle.select_active(t, dt)
        want_tn = min(int(a) + int(b) for a, b in zip(t, dt))
        want = [k for k in range(n) if int(t[k]) + int(dt[k]) == want_tn]
        assert tn == want_tn and idx.tolist() == want


def test_block_steps_single_level_equals_shared_steps():
    # With the level range pinned to one value the block scheme must take the
    # same steps as the shared scheme, bit for bit.
    p = ics.plummer(128, 11)
    a = oracle.HermiteState(p.pos, p.vel, p.mass)
    b = oracle.HermiteState(p.pos, p.vel, p.mass)
    t_end = 1 << 17  # 0.125
    oracle.hermite_run(a, t_end, eps=1 / 256, lmin=-8, lmax=-8, init=True)
    oracle.hermite_run(b, t_end, eps=1 / 256, shared_log2=-8, init=True)
    assert a.steps == b.steps == 32
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.v, b.v)


def test_block_steps_invariants_and_energy():
    p = ics.plummer(256, 12)
    st = oracle.HermiteState(p.pos, p.vel, p.mass)
    eps = 1 / 256
    e0 = sum(oracle.energy(st.x, st.v, st.m, eps))
    oracle.hermite_run(st, 0, eps=eps, eta=0.02, init=True)   # first steps only
    assert np.all(st.dt >= 1) and np.all(st.dt <= 1 << 17)
    assert np.all((st.dt & (st.dt - 1)) == 0)
    t_end = 1 << 17
    oracle.hermite_run(st, t_end, eps=eps, eta=0.02)
    assert np.all(st.t == t_end)                 # synchronised at a 2^-3 boundary
    assert np.all(st.t % st.dt == 0)             # commensurability
    assert st.sum_active > 256 and st.steps > 8  # genuinely hierarchical
    e1 = sum(oracle.energy(st.x, st.v, st.m, eps))
    assert abs((e1 - e0) / e0) < 1e-5


def test_shared_plummer_energy_scale():
    # The 1024-body, eps = 1/256, dt = 1/256 run to t = 0.125: energy error
    # at the ~1e-7 level of Table 2 or below (sanity, not a bound from the
    # paper).
    p = ics.workload("plummer1k_hermite")
    st = oracle.HermiteState(p.pos, p.vel, p.mass)
    eps = 1 / 256
    e0 = sum(oracle.energy(st.x, st.v, st.m, eps))
    oracle.hermite_run(st, 1 << 17, eps=eps, shared_log2=-8, init=True)
    e1 = sum(oracle.energy(st.x, st.v, st.m, eps))
    assert st.steps == 32
    assert abs((e1 - e0) / e0) < 1e-5


def test_shared_adjoint_against_finite_differences():
    n, steps, D, eps = 12, 6, 1.0 / 64, 0.05
    p = ics.plummer(n, 13)
    w = np.random.default_rng(3).normal(size=(3, n))
    gx0, gv0, gm = oracle.hermite_shared_adjoint(p.pos, p.vel, p.mass, eps, D, steps, w)

    def L(x0, v0, m):
        x, _ = oracle.hermite_shared_forward(x0, v0, m, eps, D, steps)
        return (w * x).sum()

    h = 1e-6
    g = np.random.default_rng(4)
    for k in range(6):
        i, c = int(g.integers(n)), int(g.integers(3))
        for which, grad in (("x", gx0), ("v", gv0)):
            xp, vp = p.pos.copy(), p.vel.copy()
            xm, vm = p.pos.copy(), p.vel.copy()
            if which == "x":
                xp[c, i] += h; xm[c, i] -= h
            else:
                vp[c, i] += h; vm[c, i] -= h
            fd = (L(xp, vp, p.mass) - L(xm, vm, p.mass)) / (2 * h)
            assert fd == pytest.approx(grad[c, i], rel=1e-6, abs=1e-8)
        mp_, mm_ = p.mass.copy(), p.mass.copy()
        mp_[i] += h; mm_[i] -= h
        fd = (L(p.pos, p.vel, mp_) - L(p.pos, p.vel, mm_)) / (2 * h)
        assert fd == pytest.approx(gm[i], rel=1e-6, abs=1e-8)


def test_shared_adjoint_translation_and_boost():
    # Shifting every x0 by c shifts x(T) by c; boosting every v0 by u shifts
    # x(T) by u T.  So sum_k gx0_k = sum_i w_i and sum_k gv0_k = T sum_i w_i.
    n, steps, D, eps = 16, 8, 1.0 / 32, 0.05
    p = ics.plummer(n, 14)
    w = np.random.default_rng(5).normal(size=(3, n))
    gx0, gv0, _ = oracle.hermite_shared_adjoint(p.pos, p.vel, p.mass, eps, D, steps, w)
    np.testing.assert_allclose(gx0.sum(axis=1), w.sum(axis=1), rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(gv0.sum(axis=1), steps * D * w.sum(axis=1), rtol=1e-9, atol=1e-9)


def test_aarseth_criterion_on_circular_orbit():
    """On a circular orbit of angular frequency w every derivative of the
    acceleration has magnitude |a| w^k and successive ones are orthogonal,
    so the criterion sqrt(eta (|a||a2| + |j|^2) / (|j||a3| + |a2|^2))
    reduces to sqrt(eta) / w whatever |a| is.  The second derivative is the
    one carried to the new time, a2 + a3 D."""
    g = np.random.default_rng(5)
    for _ in range(20):
        A, w, eta = g.uniform(0.1, 10), g.uniform(0.1, 10), g.uniform(0.001, 0.1)
        ph = g.uniform(0, 2 * math.pi)
        e1 = np.array([math.cos(ph), math.sin(ph), 0.0])
        e2 = np.array([-math.sin(ph), math.cos(ph), 0.0])
        a1, j1 = -A * e1, -A * w * e2
        a2_new, a3 = A * w * w * e1, A * w ** 3 * e2
        for D in (0.0, 1e-3, 0.25):
            dt = oracle.aarseth_dt(a1, j1, a2_new - a3 * D, a3, D, eta)
            assert dt == pytest.approx(math.sqrt(eta) / w, rel=1e-12), (A, w, eta, D)


def test_first_step_on_circular_orbit():
    """The first step eta_s |a| / |j| is 1 / w on a circular orbit (each
    body's acceleration turns at the orbital frequency), so the initial level
    is the largest power of two not above eta_s / w."""
    for a, eta_s in ((1.0, 0.01), (0.3, 0.02), (2.5, 0.005)):
        m = np.array([0.6, 0.4])
        x0, v0 = kepler_state(0.6, 0.4, a, 0.0, 0.0)
        w = math.sqrt(1.0 / a ** 3)
        st = oracle.HermiteState(x0, v0, m)
        oracle.hermite_run(st, 0, eps=0.0, eta_s=eta_s, init=True)
        want = 2.0 ** math.floor(math.log2(eta_s / w))
        assert np.all(st.dt == int(round(want / TICK))), (a, eta_s, st.dt)
