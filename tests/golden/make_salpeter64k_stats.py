"""Write salpeter64k_oracle_stats.json: statistics of the float64 oracle's
block-step run of the Salpeter workload at full size (N = 65536, Plummer
positions and velocities, Salpeter masses on [0.1, 100] normalised to 1,
eps = 1e-3, Aarseth eta = 0.02, levels 2^-3 .. 2^-20) from t = 0 to 1/8.

Calls only the oracle and the input generator.  Block-step trajectories of
two correct integrators part after a while (a criterion within rounding of a
power of two picks another level), so the GPU run is compared with these
statistics rather than particle by particle: block steps, active particles,
energy error, the census of time-step levels at the end, and the
conservation of momentum and angular momentum.

Run from the repository root:  python tests/golden/make_salpeter64k_stats.py
(about ten minutes on eight cores).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import nbody_inputs as ics  # noqa: E402
import oracle  # noqa: E402

TICKS = 1 << 20
T_END = TICKS // 8
EPS, ETA = 1e-3, 0.02


def stats(x, v, m, t, dt, e0, eps):
    ek, ep = oracle.energy(x, v, m, eps)
    p = (m * v).sum(axis=1)
    L = (m * np.cross(x.T, v.T).T).sum(axis=1)
    levels, counts = np.unique(np.log2(dt / TICKS).astype(int), return_counts=True)
    return {
        "dE_over_E": (ek + ep - e0) / e0,
        "momentum": float(np.linalg.norm(p)),
        "angular_momentum": L.tolist(),
        "levels": {str(int(k)): int(c) for k, c in zip(levels, counts)},
        "all_at_t_end": bool(np.all(t == T_END)),
    }


def main():
    p = ics.workload("salpeter64k_block")
    s = oracle.HermiteState(p.pos, p.vel, p.mass)
    t0 = time.time()
    oracle.hermite_run(s, 0, eps=EPS, eta=ETA, init=True)
    ek0, ep0 = oracle.energy(s.x, s.v, s.m, EPS)
    e0 = ek0 + ep0
    L0 = (s.m * np.cross(s.x.T, s.v.T).T).sum(axis=1)
    oracle.hermite_run(s, T_END, eps=EPS, eta=ETA)
    # t = 1/8 is a multiple of every level's step, so every particle is due
    # there and the state is synchronised without prediction
    assert np.all(s.t == T_END)
    out = {
        "workload": "salpeter64k_block (N = 65536), eps = 1e-3, eta = 0.02, levels 2^-3..2^-20, t = 0 -> 1/8",
        "t_end_ticks": T_END,
        "block_steps": s.steps,
        "sum_active": s.sum_active,
        "E0": e0,
        "angular_momentum_0": L0.tolist(),
        "end": stats(s.x, s.v, s.m, s.t, s.dt, e0, EPS),
        "oracle_seconds": round(time.time() - t0, 1),
        "oracle_threads": oracle.num_threads(),
    }
    with open(os.path.join(HERE, "salpeter64k_oracle_stats.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
