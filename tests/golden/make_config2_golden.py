"""Writes tests/golden/config2_oracle_large.json: CPU-oracle fidelities of
the batched workload's 19- and 20-qubit instances among circuit seeds 0..31
(random rotation + CNOT layers), trajectories [0, 2) at p = 1e-3 (p/3 per
Pauli), seed 0, circuit id = circuit seed.  Calls only the oracle.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

P_ERR = 1e-3
N_TRAJ = 2


def main():
    out = {"p": P_ERR, "seed": 0, "n_traj": N_TRAJ, "instances": []}
    for s in range(32):
        c = W.config2(s)
        if c.n < 19:
            continue
        t0 = time.time()
        fid, cnt = oracle.run(c, P_ERR / 3, P_ERR / 3, P_ERR / 3, 0, 0, N_TRAJ, 0.9, cid=s)
        fired = [int(len(oracle.sample_trajectory(0, s, t, c.S, P_ERR / 3, P_ERR / 3, P_ERR / 3)[0]))
                 for t in range(N_TRAJ)]
        out["instances"].append({"circuit_seed": s, "n": c.n, "G": c.G, "S": c.S, "F": [float(x) for x in fid],
                                 "fired": fired})
        print(f"seed {s}: n={c.n} G={c.G} F={list(fid)} fired={fired} ({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(HERE, "config2_oracle_large.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
