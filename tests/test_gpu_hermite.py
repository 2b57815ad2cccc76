"""GPU parity of the block-step selection and the Hermite driver against the
float64 oracle."""
import numpy as np
import pytest

import nbody_inputs as ics
import oracle
from gpu_util import dev, host

pytestmark = pytest.mark.gpu

TICKS = 1 << 20


@pytest.fixture(scope="module")
def ctx():
    import paper_0707_0438_amd as nb
    c = nb.Context(0)
    yield c
    c.close()


def test_select_active_bit_exact(ctx):
    g = np.random.default_rng(0)
    for n in (1, 2, 63, 64, 65, 4095, 4096, 4097, 20000, 65536, 1 << 20):
        lv = g.integers(0, 10, n)
        dt = (1 << (3 + lv)).astype(np.int64)
        t = (g.integers(0, 50, n) * dt).astype(np.int64)
        want, tn = oracle.select_active(t, dt)
        idx, gtn = ctx.select_active(dev(t), dev(dt))
        assert gtn == tn, n
        assert np.array_equal(host(idx), want), n
    # every particle due at once (shared steps) and exactly one due
    n = 1 << 20
    t = np.zeros(n, np.int64); dt = np.full(n, 4096, np.int64)
    idx, tn = ctx.select_active(dev(t), dev(dt))
    assert tn == 4096 and np.array_equal(host(idx), np.arange(n, dtype=np.int32))
    dt[777777] = 1
    idx, tn = ctx.select_active(dev(t), dev(dt))
    assert tn == 1 and host(idx).tolist() == [777777]
    idx, tn = ctx.select_active(dev(np.zeros(0, np.int64)), dev(np.zeros(0, np.int64)))
    assert idx.numel() == 0


def gpu_state(h):
    s = h.get_state()
    return {k: host(v) for k, v in s.items()}


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_shared_steps_plummer1k(ctx, prec):
    """N = 1024, eps = 1/256, dt = 1/256 to t = 0.125 (32 steps)."""
    p = ics.workload("plummer1k_hermite")
    eps = 1.0 / 256
    ref = oracle.HermiteState(p.pos, p.vel, p.mass)
    e0 = sum(oracle.energy(ref.x, ref.v, ref.m, eps))
    oracle.hermite_run(ref, TICKS // 8, eps=eps, shared_log2=-8, init=True)
    h = ctx.hermite(p.n, eps=eps, shared_dt_log2=-8, prec=prec)
    h.set_state(dev(p.pos), dev(p.vel), dev(p.mass))
    ek0, ep0 = h.energy()
    assert ek0 + ep0 == pytest.approx(e0, rel=1e-6)
    st = h.advance(TICKS // 8)
    assert st["steps"] == 32 and st["sum_active"] == 32 * p.n and st["t_ticks"] == TICKS // 8
    s = gpu_state(h)
    assert np.all(s["t"] == TICKS // 8) and np.all(s["dt"] == TICKS // 256)
    dx = np.abs(s["x"] - ref.x).max()
    dv = np.abs(s["v"] - ref.v).max()
    print(prec, "max|dx|", dx, "max|dv|", dv, flush=True)
    if prec == "ds":
        assert dx <= 1e-7 and dv <= 1e-6
    else:
        assert dx <= 1e-5 and dv <= 1e-4
    ek, ep = h.energy()
    e1 = sum(oracle.energy(ref.x, ref.v, ref.m, eps))
    print(prec, "dE/E gpu", (ek + ep - e0) / e0, "oracle", (e1 - e0) / e0, flush=True)
    assert abs((ek + ep - e0) / e0) < 1e-5


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_block_steps_salpeter_reduced(ctx, prec):
    """Salpeter recipe at N = 2048, eps = 1e-3, eta = 0.02, levels 2^-3..2^-20,
    to t = 1/32: block structure and energy against the oracle.  Trajectories
    of such runs may part once a step criterion lands within rounding of a
    power of two; the comparison is statistical after the first mismatch."""
    p = ics.plummer(2048, ics.seed_for(1), "salpeter")
    eps = 1e-3
    t_end = TICKS // 32
    ref = oracle.HermiteState(p.pos, p.vel, p.mass)
    e0 = sum(oracle.energy(ref.x, ref.v, ref.m, eps))
    oracle.hermite_run(ref, 0, eps=eps, eta=0.02, init=True)
    h = ctx.hermite(p.n, eps=eps, eta=0.02, dt_min_log2=-20, dt_max_log2=-3, prec=prec)
    h.set_state(dev(p.pos), dev(p.vel), dev(p.mass))
    s0 = gpu_state(h)
    same_first = np.mean(s0["dt"] == ref.dt)
    assert same_first > 0.99
    # step in lockstep while the active sets agree
    first_diff = None
    for k in range(400):
        idx_ref, tn_ref = oracle.select_active(ref.t, ref.dt)
        if tn_ref > t_end:
            break
        na, tt = h.step()
        s = gpu_state(h)
        oracle.hermite_run(ref, tn_ref, eps=eps, eta=0.02, max_steps=1)
        if first_diff is None and (tt != tn_ref or na != idx_ref.size):
            first_diff = k
            break
    print(prec, "first block step whose active set differs:", first_diff, flush=True)
    h.advance(t_end)
    oracle.hermite_run(ref, t_end, eps=eps, eta=0.02)
    s = gpu_state(h)
    assert np.all(s["t"] % s["dt"] == 0)
    assert np.all(s["t"] <= t_end)
    ek, ep = h.energy()
    e_ref = sum(oracle.energy(ref.x, ref.v, ref.m, eps))
    drift_gpu = abs((ek + ep - e0) / e0)
    drift_ref = abs((e_ref - e0) / e0)
    print(prec, "energy drift gpu", drift_gpu, "oracle", drift_ref, flush=True)
    assert drift_gpu < max(1e-5, 10 * drift_ref)


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_shared_steps_survive_interleaved_calls(ctx, prec):
    """Shared steps keep the next step's records from the fused corrector.
    Energy evaluations, direct force calls on the same context, state reads,
    a save/load into a new driver and a fresh set_state between steps must
    not change a bit of the trajectory (N = 700, a ragged size)."""
    p = ics.plummer(700, 204)
    eps, T = 1.0 / 128, TICKS // 16     # 16 steps of 2^-8
    X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
    h = ctx.hermite(p.n, eps=eps, shared_dt_log2=-8, prec=prec)
    h.set_state(X, V, M)
    h.advance(T)
    ref = gpu_state(h)
    # the same run with other work between the steps
    h.set_state(X, V, M)                # records of the old run are stale now
    S = dev(np.arange(p.n, dtype=np.int32))
    for _ in range(8):
        h.step()
        h.energy()
        ctx.force(X, V, X, V, M, eps, prec=prec, i_self=S)
        gpu_state(h)
    blob = h.save()
    h2 = ctx.hermite(p.n, eps=eps, shared_dt_log2=-8, prec=prec)
    h2.load(blob)
    for _ in range(8):
        h2.step()
        ctx.force(X, V, X, V, M, eps, prec=prec, i_self=S)
    got = gpu_state(h2)
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_shared_steps_without_split(ctx, prec):
    """The same kind of run with the pairwise kernel forced to one j-range
    (the corrector then reads the forces directly, no split reduce) against
    the oracle."""
    p = ics.plummer(600, 205)
    eps, T = 1.0 / 128, TICKS // 16
    ref = oracle.HermiteState(p.pos, p.vel, p.mass)
    oracle.hermite_run(ref, T, eps=eps, shared_log2=-8, init=True)
    ctx.set_tile(prec, tile_j=64, ipt=1, wg=128, split=1)
    try:
        assert ctx.get_tile(p.n, p.n, prec)["split"] == 1
        h = ctx.hermite(p.n, eps=eps, shared_dt_log2=-8, prec=prec)
        h.set_state(dev(p.pos), dev(p.vel), dev(p.mass))
        st = h.advance(T)
        s = gpu_state(h)
    finally:
        ctx.set_tile(prec)
    assert st["steps"] == 16
    dx = np.abs(s["x"] - ref.x).max()
    dv = np.abs(s["v"] - ref.v).max()
    print(prec, "split 1: max|dx|", dx, "max|dv|", dv, flush=True)
    if prec == "ds":
        assert dx <= 1e-8 and dv <= 1e-7
    else:
        assert dx <= 1e-6 and dv <= 1e-5


def test_save_load_continues_bit_identically(ctx):
    p = ics.plummer(1500, 201, "salpeter")
    h = ctx.hermite(p.n, eps=1e-3, eta=0.02, prec="ds")
    h.set_state(dev(p.pos), dev(p.vel), dev(p.mass))
    for _ in range(20):
        h.step()
    blob = h.save()
    for _ in range(30):
        h.step()
    a = gpu_state(h)
    h2 = ctx.hermite(p.n, eps=1e-3, eta=0.02, prec="ds")
    h2.load(blob)
    for _ in range(30):
        h2.step()
    b = gpu_state(h2)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_energy_matches_oracle(ctx):
    p = ics.plummer(4096, 202)
    for prec in ("ds", "fp32"):
        h = ctx.hermite(p.n, eps=0.01, shared_dt_log2=-8, prec=prec)
        h.set_state(dev(p.pos), dev(p.vel), dev(p.mass))
        ek, ep = h.energy()
        rk, rp = oracle.energy(p.pos, p.vel, p.mass, 0.01)
        assert ek == pytest.approx(rk, rel=1e-13)
        assert ep == pytest.approx(rp, rel=1e-6 if prec == "ds" else 1e-4)


def test_block_advance_in_pieces_equals_one_advance(ctx):
    """The device-resident block stepping enqueues steps in chunks; where the
    chunks and the advance calls fall must not change a single bit."""
    p = ics.plummer(3000, 203, "salpeter")
    T = TICKS // 64
    runs = []
    for pieces in ((T,), (T // 4, T // 2, T), (T // 8, T // 8, 3 * T // 4, T)):
        h = ctx.hermite(p.n, eps=1e-3, eta=0.02, prec="ds")
        h.set_state(dev(p.pos), dev(p.vel), dev(p.mass))
        for t in pieces:
            st = h.advance(t)
        runs.append((st, gpu_state(h)))
        h.close()
    for st, s in runs[1:]:
        assert st == runs[0][0]
        for k in s:
            assert np.array_equal(s[k], runs[0][1][k]), k
    st0 = runs[0][0]
    assert st0["steps"] > 10 and st0["sum_active"] > st0["steps"]


def test_block_steps_unsoftened_kepler(ctx):
    """Two bodies on an e = 0.5 orbit with eps = 0 in block mode (the
    zero-softening path): the orbit and its energy against the oracle."""
    from test_oracle_hermite import kepler_state
    m = np.array([0.6, 0.4])
    x0, v0 = kepler_state(0.6, 0.4, 1.0, 0.5, 0.0)
    ref = oracle.HermiteState(x0, v0, m)
    oracle.hermite_run(ref, TICKS // 2, eps=0.0, eta=0.01, lmin=-20, lmax=-6, init=True)
    h = ctx.hermite(2, eps=0.0, eta=0.01, dt_min_log2=-20, dt_max_log2=-6, prec="ds")
    h.set_state(dev(x0), dev(v0), dev(m))
    st = h.advance(TICKS // 2)
    s = gpu_state(h)
    assert np.all(s["t"] == TICKS // 2) and st["t_ticks"] == TICKS // 2
    print("kepler block steps gpu", st["steps"], "oracle", ref.steps, "max|dx|", np.abs(s["x"] - ref.x).max(),
          flush=True)
    assert np.abs(s["x"] - ref.x).max() < 1e-6
    assert abs(st["steps"] - ref.steps) <= max(2, ref.steps // 20)


def test_salpeter64k_full_size_short_interval(ctx):
    """The block-step workload at full size (N = 65536, Salpeter masses,
    eps = 1e-3, eta = 0.02, levels 2^-3..2^-20) through the same driver the
    benchmark times, t = 0 -> 1/512: in lockstep with the oracle until the
    first block whose active set differs, then both to the end; block
    structure, positions and energy compared."""
    p = ics.workload("salpeter64k_block")
    eps = 1e-3
    t_end = TICKS // 512
    ref = oracle.HermiteState(p.pos, p.vel, p.mass)
    oracle.hermite_run(ref, 0, eps=eps, eta=0.02, init=True)
    h = ctx.hermite(p.n, eps=eps, eta=0.02, dt_min_log2=-20, dt_max_log2=-3, prec="ds")
    h.set_state(dev(p.pos), dev(p.vel), dev(p.mass))
    e0 = sum(h.energy())
    s0 = gpu_state(h)
    assert np.mean(s0["dt"] == ref.dt) > 0.999
    first_diff, k = None, 0
    while True:
        idx_ref, tn_ref = oracle.select_active(ref.t, ref.dt)
        if tn_ref > t_end:
            break
        na, tt = h.step()
        oracle.hermite_run(ref, tn_ref, eps=eps, eta=0.02, max_steps=1)
        if tt != tn_ref or na != idx_ref.size:
            first_diff = k
            break
        k += 1
    st = h.advance(t_end)
    oracle.hermite_run(ref, t_end, eps=eps, eta=0.02)
    s = gpu_state(h)
    dx = np.sort(np.abs(s["x"] - ref.x).max(axis=0))
    print("salpeter64k to t=1/512: lockstep blocks", k, "first differing", first_diff, "steps gpu", st["steps"],
          "oracle", ref.steps, "|dx| p99", dx[int(0.99 * dx.size)], "max", dx[-1], flush=True)
    assert np.all(s["t"] <= t_end) and np.all(s["t"] % s["dt"] == 0)
    assert abs(st["steps"] - ref.steps) <= max(2, ref.steps // 20)
    if first_diff is None:
        assert st["steps"] == ref.steps and st["sum_active"] == ref.sum_active
        assert np.array_equal(s["t"], ref.t) and np.array_equal(s["dt"], ref.dt)
    assert dx[int(0.99 * dx.size)] < 1e-9
    ek, ep = h.energy()
    print("salpeter64k energy drift gpu", abs((ek + ep - e0) / e0), flush=True)
    assert abs((ek + ep - e0) / e0) < 1e-6


def test_salpeter64k_statistics_against_oracle(ctx):
    """The block-step workload at full size to t = 1/8 (about 3700 block
    steps) against the float64 oracle's run of the same interval, whose
    statistics tests/golden/make_salpeter64k_stats.py stored (the oracle takes
    minutes).  Trajectories of two correct integrators part, so the DS run is
    held to the oracle's block count, active count, energy error, census of
    step levels and conservation of momentum and angular momentum; plain FP32
    is reported beside it (its rounding noise changes the step choices)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "salpeter64k_oracle_stats.json")) as f:
        g = json.load(f)
    p = ics.workload("salpeter64k_block")
    T = g["t_end_ticks"]
    ref_levels = {int(k): v for k, v in g["end"]["levels"].items()}
    L0 = np.array(g["angular_momentum_0"])
    dL_ref = np.linalg.norm(np.array(g["end"]["angular_momentum"]) - L0)
    for prec in ("ds", "fp32"):
        h = ctx.hermite(p.n, eps=1e-3, eta=0.02, dt_min_log2=-20, dt_max_log2=-3, prec=prec)
        h.set_state(dev(p.pos), dev(p.vel), dev(p.mass))
        ek, ep = h.energy()
        e0 = ek + ep
        assert e0 == pytest.approx(g["E0"], rel=1e-6)
        st = h.advance(T)
        s = gpu_state(h)
        ek, ep = h.energy()
        de = (ek + ep - e0) / e0
        assert np.all(s["t"] == T)
        lv, cnt = np.unique(np.log2(s["dt"] / TICKS).astype(int), return_counts=True)
        levels = dict(zip(lv.tolist(), cnt.tolist()))
        tv = sum(abs(levels.get(k, 0) - ref_levels.get(k, 0)) for k in set(levels) | set(ref_levels)) / 2 / p.n
        P = np.linalg.norm((p.mass * s["v"]).sum(axis=1))
        L = (p.mass * np.cross(s["x"].T, s["v"].T).T).sum(axis=1)
        dL = np.linalg.norm(L - L0)
        print(f"{prec}: steps {st['steps']} (oracle {g['block_steps']}), active {st['sum_active']} "
              f"(oracle {g['sum_active']}), dE/E {de:.3e} (oracle {g['end']['dE_over_E']:.3e}), "
              f"level census distance {tv:.4f}, |P| {P:.2e} (oracle {g['end']['momentum']:.2e}), "
              f"|dL| {dL:.2e} (oracle {dL_ref:.2e})", flush=True)
        assert abs(de) < 1e-6
        if prec == "ds":
            assert abs(st["steps"] - g["block_steps"]) <= 0.03 * g["block_steps"]
            assert abs(st["sum_active"] - g["sum_active"]) <= 0.03 * g["sum_active"]
            assert abs(de - g["end"]["dE_over_E"]) < 1e-7
            assert tv < 0.03
            assert P < 5 * g["end"]["momentum"]
            assert dL < 5 * dL_ref
        h.close()


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_shared_steps_unsoftened_kepler(ctx, prec):
    """The e = 0.5 two-body orbit with eps = 0 and shared steps of 2^-8 to
    t = 1/2 (the unsoftened kernel through the shared-step driver) against
    the oracle."""
    from test_oracle_hermite import kepler_state
    m = np.array([0.6, 0.4])
    x0, v0 = kepler_state(0.6, 0.4, 1.0, 0.5, 0.0)
    ref = oracle.HermiteState(x0, v0, m)
    oracle.hermite_run(ref, TICKS // 2, eps=0.0, shared_log2=-8, init=True)
    h = ctx.hermite(2, eps=0.0, shared_dt_log2=-8, prec=prec)
    h.set_state(dev(x0), dev(v0), dev(m))
    st = h.advance(TICKS // 2)
    s = gpu_state(h)
    assert st["steps"] == 128 and np.all(s["t"] == TICKS // 2)
    dx = np.abs(s["x"] - ref.x).max()
    print(prec, "kepler shared max|dx|", dx, flush=True)
    assert dx < (1e-6 if prec == "ds" else 1e-4)


def test_single_particle_block_steps(ctx):
    """One particle: no force, a step criterion of 0/0, hence the smallest
    level (a zero or non-finite criterion gives 2^lmin); it drifts in a
    straight line, step after step, with only kinetic energy."""
    x0 = np.array([[0.25], [-0.5], [1.0]])
    v0 = np.array([[0.125], [0.0], [-0.25]])
    m = np.array([0.75])
    h = ctx.hermite(1, eps=1e-2, eta=0.02, dt_min_log2=-12, dt_max_log2=-3, prec="ds")
    h.set_state(dev(x0), dev(v0), dev(m))
    for k in range(1, 4):
        na, tt = h.step()
        assert na == 1 and tt == k * (TICKS >> 12)
    s = gpu_state(h)
    assert np.all(s["dt"] == TICKS >> 12)
    np.testing.assert_allclose(s["x"], x0 + v0 * 3 * 2.0 ** -12, rtol=0, atol=1e-15)
    assert np.array_equal(s["v"], v0)
    ek, ep = h.energy()
    assert ek == pytest.approx(0.5 * 0.75 * (0.125 ** 2 + 0.25 ** 2), rel=1e-14) and ep == 0.0


def test_salpeter64k_energy_drift_per_time_unit(ctx):
    """The block-step workload over its whole span (N = 65536 Salpeter,
    eps = 1e-3, eta = 0.02, levels 2^-3 .. 2^-20, t = 0 -> 1): the energy
    drift |E(t) - E(0)| / |E(0)| / t stays below 1e-6 per N-body time unit at
    t = 1, in both precisions.  The bar is taken over the full unit: over
    t = 1/8 the float64 oracle itself drifts 1.8e-6 per unit, as the
    integrator's error at eta = 0.02 is not spread evenly in time.  The
    energy is also reported at t = 1/4, 1/2 and 3/4."""
    p = ics.workload("salpeter64k_block")
    for prec in ("ds", "fp32"):
        h = ctx.hermite(p.n, eps=1e-3, eta=0.02, dt_min_log2=-20, dt_max_log2=-3, prec=prec)
        h.set_state(dev(p.pos), dev(p.vel), dev(p.mass))
        ek, ep = h.energy()
        e0 = ek + ep
        marks = []
        for q in (1, 2, 3, 4):
            st = h.advance(q * TICKS // 4)
            ek, ep = h.energy()
            marks.append((st["t_ticks"] / TICKS, (ek + ep - e0) / e0))
        t1, de = marks[-1]
        print(prec, "steps", st["steps"], "dE/E at t = 1/4 .. 1:", ", ".join(f"{d:.2e}" for _, d in marks),
              f"drift per unit at t = 1: {abs(de) / t1:.2e}", flush=True)
        assert t1 == 1.0
        assert abs(de) / t1 < 1e-6, (prec, de)
        h.close()


@pytest.mark.parametrize("prec", ["ds", "fp32"])
@pytest.mark.parametrize("levels", [(-20, -3), (-8, -8)])
def test_block_step_forces_per_step(ctx, prec, levels):
    """Block steps of the Salpeter recipe at N = 4096 (eps = 1e-3): after every
    step, the new acceleration and jerk of the block's particles (the
    pairwise sums of the step, reduced over the j-ranges) against the
    oracle's forces on the same predicted state, particle by particle.  The
    state before the step is read back, every particle is predicted to the
    block time by the oracle's predictor, and the oracle evaluates the block
    against all of them; so the check does not depend on the GPU and oracle
    trajectories staying in lockstep (their step criteria are differences of
    nearly equal accelerations and part within a few dozen steps).  The
    block list and time are checked against the oracle's selection on the
    same ticks.  Levels 2^-20..2^-3 give blocks of every size below 2048
    (the j-parallel launch shape: single particles, partial groups) and a few
    larger; one level 2^-8 makes every block the whole set (LDS tiles)."""
    from gpu_util import BARS, rel_err_stats
    p = ics.plummer(4096, 4711, "salpeter")
    eps = 1e-3
    lmin, lmax = levels
    h = ctx.hermite(p.n, eps=eps, eta=0.02, dt_min_log2=lmin, dt_max_log2=lmax, prec=prec)
    h.set_state(dev(p.pos), dev(p.vel), dev(p.mass))
    bar_a, bar_j = BARS[prec]["acc"], BARS[prec]["jerk"]
    sizes, worst = [], [0.0, 0.0]
    s = gpu_state(h)
    for k in range(100 if lmin < lmax else 6):
        idx, tn = oracle.select_active(s["t"], s["dt"])
        D = (tn - s["t"]) / TICKS
        xp, vp = np.empty((3, p.n)), np.empty((3, p.n))
        for q in range(p.n):
            xp[:, q], vp[:, q] = oracle.predict(s["x"][:, q], s["v"][:, q], s["a"][:, q], s["jerk"][:, q], D[q])
        ra, rj, _ = oracle.force(xp[:, idx], vp[:, idx], xp, vp, s["m"], eps, iself=idx)
        na, tt = h.step()
        assert (na, tt) == (idx.size, tn), k
        s = gpu_state(h)
        ea = rel_err_stats(s["a"][:, idx], ra)
        ej = rel_err_stats(s["jerk"][:, idx], rj)
        assert np.array_equal(s["t"][idx], np.full(idx.size, tn))
        worst = [max(worst[0], ea["p99"]), max(worst[1], ej["p99"])]
        assert ea["p99"] <= bar_a and ej["p99"] <= bar_j, (k, na, ea, ej)
        sizes.append(na)
    print(prec, levels, "blocks", len(sizes), "sizes min/median/max", min(sizes), int(np.median(sizes)),
          max(sizes), "worst acc p99 %.2e jerk p99 %.2e" % tuple(worst), flush=True)
    if lmin < lmax:
        assert min(sizes) == 1 and any(1 < z < 2048 and z % 2 for z in sizes)
    else:
        assert min(sizes) == p.n


def test_trace_lines_match_statistics(tmp_path, monkeypatch):
    """NBODY_TRACE=<path>: one JSON line per step, block and shared; the
    block lines' count, active sum and times agree with the integrator's own
    statistics and with the oracle's block selection at the first step."""
    import json
    import paper_0707_0438_amd as nb
    path = tmp_path / "trace.jsonl"
    monkeypatch.setenv("NBODY_TRACE", str(path))
    c = nb.Context(0)
    monkeypatch.delenv("NBODY_TRACE")
    try:
        p = ics.plummer(3000, 4712, "salpeter")
        h = c.hermite(p.n, eps=1e-3, eta=0.02, prec="ds")
        h.set_state(dev(p.pos), dev(p.vel), dev(p.mass))
        s0 = gpu_state(h)
        idx0, tn0 = oracle.select_active(s0["t"], s0["dt"])
        st = h.advance(TICKS // 128)
        h.close()
        hs = c.hermite(1024, eps=1.0 / 256, shared_dt_log2=-8, prec="fp32")
        q = ics.workload("plummer1k_hermite")
        hs.set_state(dev(q.pos), dev(q.vel), dev(q.mass))
        hs.advance(3 * 4096)
        hs.close()
    finally:
        c.close()
    lines = [json.loads(ln) for ln in open(path)]
    blk = [r for r in lines if r["mode"] == "block"]
    sh = [r for r in lines if r["mode"] == "shared"]
    assert len(blk) == st["steps"] and [r["step"] for r in blk] == list(range(1, st["steps"] + 1))
    assert sum(r["n_act"] for r in blk) == st["sum_active"]
    assert blk[0]["t_ticks"] == tn0 and blk[0]["n_act"] == idx0.size
    t = [r["t_ticks"] for r in blk]
    assert all(b > a for a, b in zip(t, t[1:])) and t[-1] <= TICKS // 128
    assert all(r["shape"] in ("small", "large") and r["ranges"] >= 1 and r["groups"] >= 1 for r in blk)
    assert [r["t_ticks"] for r in sh] == [4096, 8192, 12288] and all(r["n_act"] == 1024 for r in sh)


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_block_graph_replay_equals_eager(ctx, prec, monkeypatch):
    """With NBODY_BLOCK_GRAPH=1 long block-step advances replay chunks of 64
    steps from a captured hipGraph; with NBODY_BLOCK_GRAPH=0 (the default)
    the same steps are launched one by one.  Salpeter N = 4096 to t = 1/16 (several graph replays, the last
    one partly past the end time), then a second advance that reuses the
    captured graph: states, block statistics and energies are
    bit-identical."""
    import paper_0707_0438_amd as nb
    p = ics.plummer(4096, 4713, "salpeter")
    eps = 1e-3
    out = []
    for graph in ("1", "0"):
        monkeypatch.setenv("NBODY_BLOCK_GRAPH", graph)
        h = ctx.hermite(p.n, eps=eps, eta=0.02, prec=prec)
        monkeypatch.delenv("NBODY_BLOCK_GRAPH")
        h.set_state(dev(p.pos), dev(p.vel), dev(p.mass))
        st1 = h.advance(TICKS // 16)
        st2 = h.advance(TICKS // 8)
        out.append((gpu_state(h), st1, st2, h.energy()))
        h.close()
    (sa, a1, a2, ea), (sb, b1, b2, eb) = out
    print(prec, "steps", a1["steps"], a2["steps"], flush=True)
    assert a1["steps"] > 3 * 64 and a2["steps"] > a1["steps"] + 64
    assert (a1["steps"], a1["sum_active"], a2["steps"], a2["sum_active"]) == \
        (b1["steps"], b1["sum_active"], b2["steps"], b2["sum_active"])
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    assert ea == eb


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_shared_step_one_launch_equals_two(ctx, prec, monkeypatch):
    """Shared steps of small sets run as one launch: each work-group sweeps
    all j for its group of particles and corrects them, writing the next
    step's records to a second buffer.  With NBODY_FUSED_CORRECT=0 the same
    sums (one j-range) and the same corrector run as two launches.  The
    states and energies are bit-identical: N = 1024, a ragged N = 301, the
    eps = 0 two-body orbit, and a run with energy evaluations and direct
    force calls between its steps (the records alternate between the two
    buffers)."""
    cases = [(ics.plummer(1024, 4715), 1.0 / 256), (ics.plummer(301, 4716), 1.0 / 64)]
    for p, eps in cases:
        out = []
        for fuse in ("1", "0"):
            monkeypatch.setenv("NBODY_FUSED_CORRECT", fuse)
            h = ctx.hermite(p.n, eps=eps, shared_dt_log2=-8, prec=prec)
            monkeypatch.delenv("NBODY_FUSED_CORRECT")
            X, V, M = dev(p.pos), dev(p.vel), dev(p.mass)
            h.set_state(X, V, M)
            st = h.advance(TICKS // 16)
            mid = gpu_state(h)
            for _ in range(5):
                h.step()
                h.energy()
                ctx.force(X, V, X, V, M, eps, prec=prec)
            out.append((mid, gpu_state(h), st, h.energy()))
            h.close()
        (ma, sa, a, ea), (mb, sb, b, eb) = out
        print(prec, p.n, "steps", a["steps"], flush=True)
        assert a["steps"] == b["steps"] == 16
        for k in sa:
            assert np.array_equal(ma[k], mb[k]), (p.n, k)
            assert np.array_equal(sa[k], sb[k]), (p.n, k)
        assert ea == eb
    # eps = 0: the e = 0.5 two-body orbit
    from test_oracle_hermite import kepler_state
    m = np.array([0.6, 0.4])
    x, v = kepler_state(0.6, 0.4, 1.0, 0.5, 0.0)
    res = []
    for fuse in ("1", "0"):
        monkeypatch.setenv("NBODY_FUSED_CORRECT", fuse)
        h = ctx.hermite(2, eps=0.0, shared_dt_log2=-8, prec=prec)
        monkeypatch.delenv("NBODY_FUSED_CORRECT")
        h.set_state(dev(x), dev(v), dev(m))
        h.advance(TICKS // 8)
        res.append(gpu_state(h))
        h.close()
    for k in res[0]:
        assert np.array_equal(res[0][k], res[1][k]), k
    # one particle (a group with an empty slot, no force) and three (a full
    # group and a partial one)
    g = np.random.default_rng(4717)
    for n in (1, 3):
        x = g.standard_normal((3, n)) * 0.3
        v = g.standard_normal((3, n)) * 0.2
        m = np.full(n, 1.0 / n)
        res = []
        for fuse in ("1", "0"):
            monkeypatch.setenv("NBODY_FUSED_CORRECT", fuse)
            h = ctx.hermite(n, eps=0.05, shared_dt_log2=-8, prec=prec)
            monkeypatch.delenv("NBODY_FUSED_CORRECT")
            h.set_state(dev(x), dev(v), dev(m))
            st = h.advance(TICKS // 16)
            res.append((gpu_state(h), st["steps"]))
            h.close()
        assert res[0][1] == res[1][1] == 16
        for k in res[0][0]:
            assert np.array_equal(res[0][0][k], res[1][0][k]), (n, k)
        if n == 1:
            # no force: a straight line
            assert np.allclose(res[0][0]["x"], x + v * (1.0 / 16), rtol=0, atol=1e-15)


@pytest.mark.parametrize("prec", ["ds", "fp32"])
def test_shared_steps_wide_sweep_against_oracle(ctx, prec):
    """Shared steps of more than 1536 particles run the one-launch form with
    4 j records per lane per sweep (a different float32 summation order from
    the two-launch form).  N = 2048, eps = 1/256, 16 steps of 2^-8, against
    the float64 oracle's run with the bars of the N = 1024 shared-step test;
    and the unsoftened instance (eps = 0) on the same set scaled by 10 (no
    close pairs), 16 steps of 2^-6."""
    p = ics.plummer(2048, 4718)
    for eps, scale, lg in ((1.0 / 256, 1.0, -8), (0.0, 10.0, -6)):
        x0, v0 = p.pos * scale, p.vel / np.sqrt(scale)
        ref = oracle.HermiteState(x0, v0, p.mass)
        T = 16 << (20 + lg)
        oracle.hermite_run(ref, T, eps=eps, shared_log2=lg, init=True)
        h = ctx.hermite(p.n, eps=eps, shared_dt_log2=lg, prec=prec)
        h.set_state(dev(x0), dev(v0), dev(p.mass))
        st = h.advance(T)
        s = gpu_state(h)
        h.close()
        assert st["steps"] == 16
        dx = np.abs(s["x"] - ref.x).max() / scale
        dv = np.abs(s["v"] - ref.v).max() * np.sqrt(scale)
        print(prec, "N = 2048 eps", eps, "max|dx|", dx, "max|dv|", dv, flush=True)
        if prec == "ds":
            assert dx <= 1e-7 and dv <= 1e-6
        else:
            assert dx <= 1e-5 and dv <= 1e-4
