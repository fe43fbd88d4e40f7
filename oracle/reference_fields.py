"""Oracle reference fields for long horizons (test infrastructure).

Runs the FP64 oracle on one of the benchmark workloads and saves the
force-shifted velocity (and density) of the fluid cells after each requested
number of steps, so that GPU runs of the same workload can state their error
against the oracle at horizons too long to recompute on the GPU machine.
Only this oracle package and the seeded input generators are used; nothing
here reads a value produced by the GPU path.

    python -m oracle.reference_fields channel --steps 1000,5000 --out ref/channel.npz

Output (numpy .npz, float32 values of the FP64 fields):
  steps      the horizons, in order
  fluid      flat indices (x fastest) of the fluid cells
  u_<n>      (3, n_fluid) velocity after n steps
  rho_<n>    (n_fluid,) density after n steps
  meta       JSON text describing the workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402


def workload(name):
    from paper_2307_11752_amd import workloads as W

    if name == "channel":
        return W.channel_spheres()
    if name == "tgv3d":
        return W.tgv3d()
    raise ValueError(name)


def run(name, horizons, out, nthreads=0):
    wl = workload(name)
    ref = oracle.Lattice(wl.descriptor, wl.material, wl.periodic, wl.tau, g=wl.g,
                         u_wall=wl.u_wall, nthreads=nthreads)
    ref.init_equilibrium(None, wl.u0)
    fluid = np.flatnonzero(wl.material.ravel() == 1).astype(np.int64)
    arrays = {"steps": np.asarray(horizons, np.int64), "fluid": fluid}
    done = 0
    t0 = time.perf_counter()
    for h in horizons:
        while done < h:
            n = min(100, h - done)
            ref.step(n)
            done += n
            print(f"[oracle {name}] {done}/{horizons[-1]} steps, {time.perf_counter() - t0:.0f} s",
                  flush=True)
        rho, u = ref.moments()
        arrays[f"u_{h}"] = u.reshape(3, -1)[:, fluid].astype(np.float32)
        arrays[f"rho_{h}"] = rho.ravel()[fluid].astype(np.float32)
    arrays["meta"] = np.array(json.dumps({
        "workload": wl.name, "shape": list(wl.shape), "tau": wl.tau, "g": list(wl.g),
        "periodic": wl.periodic, "oracle_threads": oracle.num_threads() if not nthreads else nthreads,
        "seconds": round(time.perf_counter() - t0, 1)}))
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    np.savez(out, **arrays)
    print(f"wrote {out}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["channel", "tgv3d"])
    ap.add_argument("--steps", default="1000,5000")
    ap.add_argument("--out", required=True)
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    horizons = sorted(int(s) for s in a.steps.split(","))
    run(a.workload, horizons, a.out, a.threads)


if __name__ == "__main__":
    main()
