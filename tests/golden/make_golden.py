"""Writes tests/golden/workloads.json: per synthetic workload, the number of kept
frequencies and the absolute Wiener regularisation eps_abs = eps_rel * max |Y^B|^2,
both computed by the FP64 oracle alone (they need every kept frequency, which is
slow in the oracle at full size).  Run: python tests/golden/make_golden.py"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle.wdd as O  # noqa: E402
import synth  # noqa: E402


def main():
    out = {"source": "tests/golden/make_golden.py (FP64 oracle only)", "workloads": {}}
    for name in ("small", "medium", "defocus", "large"):
        wl = synth.WORKLOADS[name]
        plan = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.k, amplitude=wl.aperture_amplitude(),
                           defocus_edge=wl.defocus_edge, step=wl.step)
        out["workloads"][name] = {"n_freq": int(plan.n_hat), "eps_abs": float(plan.eps_abs),
                                  "amplitude": float(plan.amplitude)}
        print(name, plan.n_hat, plan.eps_abs, flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "workloads.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
