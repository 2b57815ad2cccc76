"""Central finite differences of the differentiation workload's loss, from the
float64 oracle alone (no GPU code is imported), for the GPU gradient test.

Recipe (the differentiation workload): N = 16384 equal-mass Plummer sphere
(seeded inputs of ``nbody_inputs``), eps = 1e-3, 64 shared fourth-order
Hermite steps of 1/128 (T = 1/2), loss L = sum_i w_i . x_i(T) with w ~ N(0, 1)
seeded; 32 seeded coordinates: 11 of the initial positions, 11 of the initial
velocities and 10 masses; central differences (L(q + h) - L(q - h)) / 2h with
h = 1e-6.  The oracle's own adjoint of the same run is stored beside them, at
the same coordinates.  Writes ``adjoint16k_fd.json`` next to this file.  About
20 minutes on 8 cores.

Run: python tests/golden/make_adjoint16k_fd.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import nbody_inputs as ics  # noqa: E402
import oracle  # noqa: E402

EPS, DT, STEPS, H = 1e-3, 1.0 / 128, 64, 1e-6


def picks(n):
    """11 (x, particle, component), 11 (v, ...), 10 (m, particle, 0), seeded."""
    g = ics.rng(ics.seed_for(3), 10)
    out = []
    for kind, k in (("x", 11), ("v", 11)):
        idx = g.choice(n, k, replace=False)
        comp = g.integers(0, 3, k)
        out += [(kind, int(i), int(c)) for i, c in zip(idx, comp)]
    out += [("m", int(i), 0) for i in g.choice(n, 10, replace=False)]
    return out


def main():
    p = ics.workload("plummer16k_adjoint")
    w = ics.rng(ics.seed_for(3), 9).normal(size=(3, p.n))

    def loss(x0, v0, m):
        x, _ = oracle.hermite_shared_forward(x0, v0, m, EPS, DT, STEPS)
        return float((w * x).sum())

    t0 = time.time()
    gx, gv, gm = oracle.hermite_shared_adjoint(p.pos, p.vel, p.mass, EPS, DT, STEPS, w)
    print(f"oracle adjoint: {time.time() - t0:.0f} s", flush=True)
    entries = []
    for kind, i, c in picks(p.n):
        vals = []
        for sgn in (+1.0, -1.0):
            x0, v0, m = p.pos.copy(), p.vel.copy(), p.mass.copy()
            if kind == "x":
                x0[c, i] += sgn * H
            elif kind == "v":
                v0[c, i] += sgn * H
            else:
                m[i] += sgn * H
            vals.append(loss(x0, v0, m))
        fd = (vals[0] - vals[1]) / (2.0 * H)
        adj = float({"x": gx, "v": gv}[kind][c, i]) if kind != "m" else float(gm[i])
        entries.append({"kind": kind, "i": i, "c": c, "fd": fd, "oracle_adjoint": adj,
                        "L_plus": vals[0], "L_minus": vals[1]})
        print(f"{kind} i={i} c={c} fd={fd:.10e} adjoint={adj:.10e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    doc = {
        "what": "central finite differences (float64 oracle) of L = sum_i w_i . x_i(T)",
        "recipe": {"workload": "plummer16k_adjoint", "n": p.n, "eps": EPS, "dt": DT, "steps": STEPS,
                   "w": "nbody_inputs.rng(seed_for(3), 9).normal(size=(3, n))",
                   "coordinates": "nbody_inputs.rng(seed_for(3), 10): 11 x, 11 v, 10 m"},
        "h": H,
        "entries": entries,
    }
    with open(os.path.join(HERE, "adjoint16k_fd.json"), "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote adjoint16k_fd.json", flush=True)


if __name__ == "__main__":
    main()
