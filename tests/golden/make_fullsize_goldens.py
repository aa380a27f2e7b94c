"""Write float64 oracle references for the full-size Taylor/Couette and
ensemble workloads (calls only the oracle and the seeded workloads).

taylor_couette_256x64x16_5.json: the ternary mixture between moving walls
  (256x64x16, sigma 2, 3, 4, packing 0.25, eps/kT = 0.3 with cutoff 2.5
  sigma, walls at y = 0 and 63 moving at -+0.05, tracer band of species 3)
  advanced by the ordered oracle step (direct attractive sum; beyond a wall
  the hard-core stencils see the mirrored fluid moving with the wall, the
  attractive field sees nothing); species densities at 4096 seeded sites,
  the field max norms and the species masses.
closure_physics_192x64x64_5.json: the learned-closure workload's plain
  path (binary, sigma 2 and 3, packing 0.2, composition mode along x,
  192x64x64), 5 oracle steps; densities at 4096 seeded sites.
ensemble_64_members_20.json: the 64-system ensemble of the batched
  workload (seed 4242); the three smallest systems advanced 20 steps by the
  oracle; densities at 1024 seeded sites of each, max norms and masses.

    python tests/golden/make_fullsize_goldens.py [--threads 8]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def sample(n, sites):
    return [n[a].ravel()[sites].tolist() for a in range(n.shape[0])]


def taylor(steps):
    m, n0, u0 = W.config_taylor_couette()
    o = oracle.Oracle(m)
    f = o.init(n0, u0)
    t0 = time.time()
    f = o.step(f, steps)
    n = o.densities(f)
    rng = np.random.Generator(np.random.PCG64(91))
    sites = np.sort(rng.choice(m.N, size=4096, replace=False))
    print(f"taylor: {steps} steps in {time.time() - t0:.0f}s", flush=True)
    return {"workload": m.name, "shape": list(m.shape()), "steps": steps, "sample_sites": sites.tolist(),
            "n_sample": sample(n, sites), "maxnorm": [float(np.abs(n[a]).max()) for a in range(m.M)],
            "mass": [float(n[a].sum()) for a in range(m.M)]}


def closure_physics(steps):
    m, n0, u0 = W.config_closure_physics()
    o = oracle.Oracle(m)
    t0 = time.time()
    f = o.step(o.init(n0, u0), steps)
    n = o.densities(f)
    rng = np.random.Generator(np.random.PCG64(93))
    sites = np.sort(rng.choice(m.N, size=4096, replace=False))
    print(f"closure physics: {steps} steps in {time.time() - t0:.0f}s", flush=True)
    return {"workload": m.name, "shape": list(m.shape()), "steps": steps, "sample_sites": sites.tolist(),
            "n_sample": sample(n, sites), "maxnorm": [float(np.abs(n[a]).max()) for a in range(m.M)],
            "mass": [float(n[a].sum()) for a in range(m.M)]}


def ensemble(steps, pick=3):
    members = W.config_ensemble()
    order = sorted(range(len(members)), key=lambda k: (members[k].mixture.N, k))[:pick]
    out = {"count": len(members), "steps": steps, "systems": []}
    rng = np.random.Generator(np.random.PCG64(92))
    for k in order:
        mem = members[k]
        m = mem.mixture
        o = oracle.Oracle(m)
        f = o.step(o.init(mem.n0, mem.u0), steps)
        n = o.densities(f)
        sites = np.sort(rng.choice(m.N, size=min(1024, m.N), replace=False))
        out["systems"].append({"index": k, "shape": list(m.shape()), "sigma": list(m.sigma),
                               "sample_sites": sites.tolist(), "n_sample": sample(n, sites),
                               "maxnorm": [float(np.abs(n[a]).max()) for a in range(m.M)],
                               "mass": [float(n[a].sum()) for a in range(m.M)]})
        print(f"ensemble system {k} {m.shape()} done", flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=8)
    ap.add_argument("--taylor-steps", type=int, default=5)
    ap.add_argument("--ensemble-steps", type=int, default=20)
    ap.add_argument("--only", default="taylor,closure,ensemble")
    args = ap.parse_args()
    oracle.set_threads(args.threads)
    todo = args.only.split(",")
    if "closure" in todo:
        c = closure_physics(5)
        with open(os.path.join(HERE, "closure_physics_192x64x64_5.json"), "w") as fh:
            json.dump(c, fh)
    if "taylor" not in todo:
        if "ensemble" in todo:
            e = ensemble(args.ensemble_steps)
            with open(os.path.join(HERE, f"ensemble_64_members_{args.ensemble_steps}.json"), "w") as fh:
                json.dump(e, fh)
        return
    t = taylor(args.taylor_steps)
    with open(os.path.join(HERE, f"taylor_couette_256x64x16_{args.taylor_steps}.json"), "w") as fh:
        json.dump(t, fh)
    e = ensemble(args.ensemble_steps)
    with open(os.path.join(HERE, f"ensemble_64_members_{args.ensemble_steps}.json"), "w") as fh:
        json.dump(e, fh)


if __name__ == "__main__":
    main()
