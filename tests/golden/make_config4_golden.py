"""Writes tests/golden/config4_oracle.json: CPU-oracle values for the 30-qubit
alternating-layer workload (3-regular graph, 4 rounds, G = 330, S = 510).

Calls only the oracle.  Stored per trajectory: its fired error sites, its
fidelity against the error-free state, and its amplitudes at 1024 fixed
random indices; plus the error-free state's amplitudes at those indices.
Trajectories: t = 0 at p = 1e-5, and the first two trajectories with at least
one fired site at p = 1e-4 and at p = 1e-3 (seed 0, circuit id 0).

With --xonly it writes tests/golden/config4_oracle_xonly.json instead: the
first two trajectories with at least one fired site at p = 1e-3 under the
X-only model (p_x = p, p_y = p_z = 0).  A single Z or Y error sends this
circuit's state to the sector orthogonal to the error-free one (F ~ 0), while
X errors leave intermediate fidelities, so these exercise the scoring of
the 30-qubit workload away from F in {0, 1}.

Needs about 40 GB of host memory (two FP64 states of 2^30 amplitudes) and
takes roughly an hour on 8 cores.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    xonly = "--xonly" in sys.argv[1:]
    c = W.config4()
    n = c.n
    rng = np.random.default_rng(1234)
    idx = np.sort(rng.choice(1 << n, 1024, replace=False))

    def model(p):
        return (p, 0.0, 0.0) if xonly else (p / 3, p / 3, p / 3)

    picks = [] if xonly else [(1e-5, 0)]
    for p in ((1e-3,) if xonly else (1e-4, 1e-3)):
        found = 0
        t = 0
        while found < 2:
            s, _ = oracle.sample_trajectory(0, 0, t, c.S, *model(p))
            if len(s):
                picks.append((p, t))
                found += 1
            t += 1
    t0 = time.time()
    ref = oracle.final_state_pattern(c, [], [])
    print(f"reference state: {time.time() - t0:.0f} s", flush=True)
    out = {"workload": c.name, "n": n, "G": c.G, "S": c.S, "seed": 0, "cid": 0,
           "model": "x" if xonly else "uniform",
           "indices": idx.tolist(),
           "reference": {"re": ref[idx].real.tolist(), "im": ref[idx].imag.tolist(),
                         "norm": float(np.vdot(ref, ref).real)},
           "trajectories": []}
    for p, t in picks:
        t0 = time.time()
        s, pa = oracle.sample_trajectory(0, 0, t, c.S, *model(p))
        psi = oracle.final_state(c, *model(p), 0, t)
        F = oracle.fidelity(ref, psi, n)
        out["trajectories"].append({"p": p, "t": t, "sites": s.tolist(), "paulis": pa.tolist(), "F": F,
                                    "re": psi[idx].real.tolist(), "im": psi[idx].imag.tolist()})
        print(f"p={p} t={t} sites={s.tolist()} F={F:.15f} ({time.time() - t0:.0f} s)", flush=True)
        del psi
    name = "config4_oracle_xonly.json" if xonly else "config4_oracle.json"
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
