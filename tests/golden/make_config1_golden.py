"""Writes tests/golden/config1_oracle.json: CPU-oracle values for the
24-qubit workload (GHZ preparation, full QFT, 50 random layers; G = 2136,
S = 3047) at its 13 uniform rates 10^(-5 + j/4), seed 0, circuit id 0.

Calls only the oracle.  Stored per rate:
  * a digest of the fired error sites of trajectories [0, 10^4): SHA-256 of
    the CSR arrays offsets (uint64, 10^4 + 1), sites (int32) and paulis
    (uint8, 1 = X, 2 = Y, 3 = Z), concatenated in that order, and the total
    fired count;
  * the fidelity F of trajectories [0, 16) against the error-free state, and
    each one's fired-site count.
A trajectory without a fired site runs the error-free circuit, so its state
is the reference state itself; its stored F is the oracle's fidelity of that
state with itself.  The others are run with the oracle's final_state.

Takes about an hour on 8 cores (each 24-qubit trajectory is 2136 gates over
2^24 amplitudes).
"""
import hashlib
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

N_SITES = 10_000
N_STATES = 16


def site_digest(c, p, n_traj):
    offs = np.zeros(n_traj + 1, np.uint64)
    sites, paulis = [], []
    for t in range(n_traj):
        s, pa = oracle.sample_trajectory(0, 0, t, c.S, p / 3, p / 3, p / 3)
        sites.append(s.astype(np.int32))
        paulis.append(pa.astype(np.uint8))
        offs[t + 1] = offs[t] + len(s)
    s = np.concatenate(sites) if sites else np.zeros(0, np.int32)
    pa = np.concatenate(paulis) if paulis else np.zeros(0, np.uint8)
    h = hashlib.sha256(offs.tobytes() + s.tobytes() + pa.tobytes()).hexdigest()
    return h, int(offs[-1])


def main():
    c = W.config1()
    n = c.n
    rates = W.rates_config1()
    t0 = time.time()
    ref = oracle.final_state_pattern(c, [], [])
    f_ref = oracle.fidelity(ref, ref, n)
    print(f"reference state: {time.time() - t0:.0f} s, F(R, R) = {f_ref!r}", flush=True)
    out = {"workload": c.name, "n": n, "G": c.G, "S": c.S, "seed": 0, "cid": 0,
           "n_site_traj": N_SITES, "n_state_traj": N_STATES, "rates": [], "ref_norm": float(np.vdot(ref, ref).real)}
    for j, p in enumerate(rates):
        t1 = time.time()
        dig, tot = site_digest(c, p, N_SITES)
        rec = {"j": j, "p": float(p), "site_sha256": dig, "fired_total": tot, "F": [], "fired": []}
        for t in range(N_STATES):
            s, pa = oracle.sample_trajectory(0, 0, t, c.S, p / 3, p / 3, p / 3)
            if len(s) == 0:
                F = f_ref
            else:
                psi = oracle.final_state(c, p / 3, p / 3, p / 3, 0, t)
                F = oracle.fidelity(ref, psi, n)
                del psi
            rec["F"].append(F)
            rec["fired"].append(int(len(s)))
        out["rates"].append(rec)
        print(f"rate {j} p={p:.3e}: {tot} fired sites over {N_SITES} trajectories; "
              f"fired {rec['fired']}; {time.time() - t1:.0f} s", flush=True)
        with open(os.path.join(HERE, "config1_oracle.json"), "w") as f:
            json.dump(out, f)


if __name__ == "__main__":
    main()
