"""Write the float64 oracle reference of the bulk-diffusion workload.

Bulk mutual diffusion, binary (sigma = 3, 4.5; packing 0.3; x1 = 0.5;
eps/kT = 0.5, cutoff 2.5 sigma_ab) on a periodic 128x32x32 D3Q19 lattice,
initial composition mode of amplitude 0.05 plus 1 % noise (workloads,
seed 2024).  Calls only the oracle (attractive field by float64 FFT, pinned
to the ordered direct sum by the tests).  Records:
  - species densities at 4096 seeded sample sites after 100 steps, with the
    per-species max norm of the full field;
  - the amplitude of the (n_0 - n_1) mode at k = 2 pi / 128 every 10 steps
    up to 2000 steps, and D_12 from the least-squares slope of ln A over
    t >= 200 (1/tau = D q^2, Sec. 5.1).

    python tests/golden/make_bulk_diffusion_golden.py [--steps 2000] [--threads 6]
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


def mode_amplitude(n, nx):
    k = 2 * math.pi / nx
    dn = (n[0] - n[1]).sum(axis=(0, 1))
    return float(abs(np.sum(dn * np.exp(-1j * k * np.arange(nx)))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--threads", type=int, default=6)
    ap.add_argument("--every", type=int, default=10)
    args = ap.parse_args()
    oracle.set_threads(args.threads)
    m, n0, u0 = W.config_bulk_diffusion()
    o = oracle.Oracle(m)
    f = o.init(n0, u0)
    rng = np.random.Generator(np.random.PCG64(77))
    sites = np.sort(rng.choice(m.N, size=4096, replace=False))
    ts, amps = [], []
    out = {"workload": m.name, "shape": list(m.shape()), "sigma": list(m.sigma), "seed": 2024,
           "sample_sites": sites.tolist(), "every": args.every}
    t0 = time.time()
    t = 0
    while True:
        n = o.densities(f)
        ts.append(t)
        amps.append(mode_amplitude(n, m.nx))
        if t == 100:
            out["n100_sample"] = [n[a].ravel()[sites].tolist() for a in range(m.M)]
            out["n100_maxnorm"] = [float(np.abs(n[a]).max()) for a in range(m.M)]
            out["n100_mass"] = [float(n[a].sum()) for a in range(m.M)]
        if t >= args.steps:
            break
        f = o.step_fft(f, args.every)
        t += args.every
        if t % 100 == 0:
            print(f"step {t}  A={amps[-1]:.6e}  elapsed {time.time() - t0:.0f}s", flush=True)
    ts, amps = np.array(ts), np.array(amps)
    sel = ts >= 200
    slope = np.polyfit(ts[sel], np.log(amps[sel]), 1)[0]
    k = 2 * math.pi / m.nx
    out["t"] = ts.tolist()
    out["amplitude"] = amps.tolist()
    out["D12"] = float(-slope / k ** 2)
    out["fit_t_min"] = 200
    out["oracle_threads"] = args.threads
    path = os.path.join(HERE, f"bulk_diffusion_128x32x32_{args.steps}.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"D12 = {out['D12']:.6f}  written {path}", flush=True)


if __name__ == "__main__":
    main()
