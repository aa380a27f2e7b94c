"""Write the float64 oracle's mode-decay D_12 for six members of the
64-system ensemble (calls only the oracle and the seeded workloads).

ensemble_d12_members.json: the ensemble of periodic binaries (seed 4242,
edges from {32, 48, 64, 96}, x1 ~ U[0.1, 0.9], packing ~ U[0.1, 0.35],
sigma_22 = 2 U[1, 2], composition mode of amplitude 0.05 along x).  Each
member's initial state does not vary across y and z, and in a periodic box
the stencil sums then see the same values for any cross-section, so the
oracle runs every member on nx x 1 x 1 (the mode's amplitude only scales by
ny nz).  1000 steps, the amplitude |sum_r (n_1 - n_2) exp(-i 2 pi x / nx)|
every 10 steps, and the least-squares D_12 = -slope(ln A, t) / (2 pi / nx)^2
over t >= 200 (Sec. 5.1).

A member is kept when its fit is well-conditioned with margin: R^2 >= 0.9999
and the amplitude at the last sample at least 1e-3 of the first (well above
the float32 rounding floor of the densities).  Of those, the six with the
fewest lattice sites in their real box are stored with their series.

For all 64 members the file also holds the fit under the library's
documented window and quality rule (mlb_fit_series_ex, mode kind) applied to
the float64 series: the window starts at min(t_min, the first t with
A <= 0.1 A_first) and keeps samples with A >= 1e-6 A_first; the fit is
well-conditioned when it has at least five samples, R^2 >= 0.98 and every
windowed amplitude is at least 1e-4 A_first.

    python tests/golden/make_ensemble_d12_golden.py [--threads 8]
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

STEPS, EVERY, T_MIN = 1000, 10, 200.0


def mode_series(mem, steps=STEPS, every=EVERY):
    """(t, A) of the composition mode of ensemble member `mem` on nx x 1 x 1."""
    m0 = mem.mixture
    m = W.Mixture(m0.nx, 1, 1, sigma=m0.sigma, tau=m0.tau, name=m0.name + "_line")
    n0 = np.ascontiguousarray(mem.n0[:, :1, :1, :])
    u0 = np.ascontiguousarray(mem.u0[:, :, :1, :1, :])
    o = oracle.Oracle(m)
    f = o.init(n0, u0)
    k = 2 * math.pi / m.nx
    x = np.arange(m.nx)
    ts, amps = [], []
    for t in range(0, steps + 1, every):
        n = o.densities(f)
        amps.append(float(abs(np.sum((n[0] - n[1]).sum(axis=(0, 1)) * np.exp(-1j * k * x)))))
        ts.append(float(t))
        if t < steps:
            f = o.step(f, every)
    return np.array(ts), np.array(amps)


def fit(ts, amps, nx, t_min=T_MIN):
    k = 2 * math.pi / nx
    sel = ts >= t_min
    y = np.log(amps[sel])
    slope, icpt = np.polyfit(ts[sel], y, 1)
    resid = y - (icpt + slope * ts[sel])
    r2 = 1.0 - float(np.sum(resid ** 2)) / float(np.sum((y - y.mean()) ** 2))
    return float(-slope / k ** 2), r2


def library_rule(ts, amps, nx, t_min=T_MIN):
    """(D, R^2, samples, smallest windowed A / A_first, flag) under the
    window and quality rule stated for the library's mode fit."""
    a0 = amps[0]
    t_lo = t_min
    below = np.nonzero(amps <= 0.1 * a0)[0]
    if below.size:
        t_lo = min(t_min, ts[below[0]])
    sel = (ts >= t_lo) & (amps >= 1e-6 * a0)
    n = int(sel.sum())
    if n < 2:
        return float("nan"), 0.0, n, float("nan"), False
    D, r2 = fit(ts[sel], amps[sel], nx, t_min=-math.inf)
    vmin = float(amps[sel].min() / a0)
    return D, r2, n, vmin, bool(n >= 5 and r2 >= 0.98 and vmin >= 1e-4)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--keep", type=int, default=6)
    args = ap.parse_args()
    oracle.set_threads(args.threads)
    members = W.config_ensemble()
    rows, rule = [], []
    t0 = time.time()
    for idx, mem in enumerate(members):
        m = mem.mixture
        ts, amps = mode_series(mem)
        D, r2 = fit(ts, amps, m.nx)
        tail = amps[-1] / amps[0]
        ok = r2 >= 0.9999 and tail >= 1e-3
        print(f"member {idx:2d} {m.nx}x{m.ny}x{m.nz} x1 {mem.x1:.3f} packing {mem.packing:.3f} "
              f"sigma2 {m.sigma[1]:.3f}: D {D:.6f} R2 {r2:.6f} A_end/A_0 {tail:.2e} {'keep' if ok else ''}",
              flush=True)
        Dr, r2r, nr, vmin, flag = library_rule(ts, amps, m.nx)
        rule.append({"member": idx, "d12": Dr, "r2": r2r, "samples": nr, "min_ratio": vmin, "well_conditioned": flag})
        if ok:
            rows.append({"member": idx, "shape": [m.nx, m.ny, m.nz], "sites": m.N, "x1": mem.x1,
                         "packing": mem.packing, "sigma": list(m.sigma), "d12": D, "r2": r2,
                         "amplitude_ratio_end": float(tail), "t": ts.tolist(), "amplitude": amps.tolist()})
    rows.sort(key=lambda r: (r["sites"], r["member"]))
    keep = sorted(rows[:args.keep], key=lambda r: r["member"])
    print(f"{len(rows)} of {len(members)} well-conditioned with margin; kept members "
          f"{[r['member'] for r in keep]}; {sum(r['well_conditioned'] for r in rule)} of {len(members)} "
          f"well-conditioned under the library's rule ({time.time() - t0:.0f}s)", flush=True)
    out = {"ensemble": {"count": len(members), "seed": 4242}, "steps": STEPS, "every": EVERY, "fit_t_min": T_MIN,
           "members": keep, "library_rule": rule}
    with open(os.path.join(HERE, "ensemble_d12_members.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
