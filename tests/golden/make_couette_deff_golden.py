"""Write the float64 oracle reference for the Taylor/Couette dispersion
check at reduced size (calls only the oracle and the seeded workloads).

taylor_couette_64x24x12_600.json: the ternary Couette workload's physics
  (sigma 2, 3, 4; packing 0.25; eps/kT = 0.3 with cutoff 2.5 sigma; walls at
  y = 0 and 23 moving at -+0.05; Gaussian tracer band of species 3, width 8,
  centred in x) on 64x24x12, 600 oracle steps (direct attractive sum).
  Every 10 steps the amplitude of the tracer's section-averaged mode
  |sum_r n_3 exp(-i 2 pi x / 64)|, whose decay rate is D_eff (2 pi / 64)^2
  (Sec. 5.2, eq. c99), and the least-squares D_eff over t >= 100.

    python tests/golden/make_couette_deff_golden.py [--threads 8]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--steps", type=int, default=600)
    args = ap.parse_args()
    oracle.set_threads(args.threads)
    m, n0, u0 = W.config_taylor_couette(64, 24, 12)
    o = oracle.Oracle(m)
    f = o.init(n0, u0)
    k = 2 * math.pi / m.nx
    x = np.arange(m.nx)
    ts, amps = [], []
    t0 = time.time()
    for t in range(0, args.steps + 1, 10):
        prof = o.densities(f)[2].sum(axis=(0, 1))
        amps.append(float(abs(np.sum(prof * np.exp(-1j * k * x)))))
        ts.append(float(t))
        if t < args.steps:
            f = o.step(f, 10)
    ts, amps = np.array(ts), np.array(amps)
    sel = ts >= 100
    D = float(-np.polyfit(ts[sel], np.log(amps[sel]), 1)[0] / k ** 2)
    print(f"couette 64x24x12: {args.steps} steps in {time.time() - t0:.0f}s, D_eff {D:.6f}", flush=True)
    out = {"workload": m.name, "shape": list(m.shape()), "steps": args.steps, "every": 10, "t": ts.tolist(),
           "amplitude": amps.tolist(), "fit_t_min": 100.0, "D_eff": D,
           "mass": [float(v) for v in o.densities(f).sum(axis=(1, 2, 3))]}
    with open(os.path.join(HERE, f"taylor_couette_64x24x12_{args.steps}.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
