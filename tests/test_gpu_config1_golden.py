"""GPU parity on the 24-qubit headline workload (GHZ preparation, full QFT,
50 random rotation + CNOT layers; G = 2136, S = 3047) at all 13 of its
uniform rates 10^(-5 + j/4), against stored CPU-oracle values
(tests/golden/config1_oracle.json, written by
tests/golden/make_config1_golden.py, which calls only the oracle).

Checked, seed 0, circuit id 0, in the plan the benchmark runs:
  * the fired error sites of trajectories [0, 10^4) at every rate, bit for
    bit (SHA-256 of the CSR arrays offsets / sites / paulis);
  * the fidelities of trajectories [0, 16) at every rate (208 values), in
    complex64 (within 2e-5) and complex128 (within 1e-12), and the two GPU
    precisions against each other (within 2e-5);
  * equal success counts (F >= 0.9) outside the margin |F_oracle - tau| <
    the precision's bar; any trajectory inside the margin is listed.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "config1_oracle.json")
TAU = 0.9


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as f:
        g = json.load(f)
    assert len(g["rates"]) == 13
    return g


@pytest.fixture(scope="module")
def P():
    import paper_2301_07264_amd as P
    P.lib()
    return P


def test_config1_sites_all_rates(P, gold):
    c = W.config1()
    assert (c.n, c.G, c.S) == (gold["n"], gold["G"], gold["S"])
    ctx = P.nt_create(0)
    h = P.nt_circuit_load(ctx, c)
    try:
        N = gold["n_site_traj"]
        for rec in gold["rates"]:
            p = rec["p"]
            P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
            off, sites, paulis = P.nt_sample_sites(ctx, h, 0, 0, N)
            k = int(off[-1])
            dig = hashlib.sha256(np.ascontiguousarray(off, np.uint64).tobytes()
                                 + np.ascontiguousarray(sites[:k], np.int32).tobytes()
                                 + np.ascontiguousarray(paulis[:k], np.uint8).tobytes()).hexdigest()
            _say(f"config1 sites: rate {rec['j']} p={p:.3e}: {k} fired")
            assert k == rec["fired_total"]
            assert dig == rec["site_sha256"]
    finally:
        P.nt_circuit_free(h)
        P.nt_destroy(ctx)


def test_config1_fidelities_all_rates(P, gold):
    c = W.config1()
    ctx = P.nt_create(0)
    h = P.nt_circuit_load(ctx, c)
    try:
        n = gold["n_state_traj"]
        got = {}
        for prec, bar in (("c64", 2e-5), ("c128", 1e-12)):
            P.nt_set_precision(ctx, P.NT_C64 if prec == "c64" else P.NT_C128)
            flips = []
            worst = 0.0
            for rec in gold["rates"]:
                p = rec["p"]
                P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
                f = np.zeros(n)
                cnt, _ = P.nt_run(ctx, h, 0, 0, n, TAU, f)
                fo = np.asarray(rec["F"])
                d = np.abs(f - fo)
                worst = max(worst, float(d.max()))
                assert d.max() <= bar, (prec, rec["j"], float(d.max()))
                margin = np.abs(fo - TAU) < bar
                flips += [(rec["j"], int(t)) for t in np.flatnonzero(margin)]
                succ_o = fo >= TAU
                assert int(((f >= TAU) != succ_o)[~margin].sum()) == 0
                if not margin.any():
                    assert cnt == int(succ_o.sum())
                got[(prec, rec["j"])] = f
            _say(f"config1 fidelities {prec}: 208 values, max |F - F_oracle| = {worst:.2e}, "
                 f"margin trajectories {flips}")
        for rec in gold["rates"]:
            assert np.abs(got[("c64", rec["j"])] - got[("c128", rec["j"])]).max() <= 2e-5
    finally:
        P.nt_circuit_free(h)
        P.nt_destroy(ctx)


@pytest.mark.parametrize("width", [1, 3, 4])
def test_config1_fidelities_other_fusion_widths(P, gold, width):
    """The same 208 stored values in complex64 under the other fusion widths
    (none; blocks and layers only; diagonal runs only): every fused-op path
    at the headline size, errors inside fused ops included."""
    c = W.config1()
    ctx = P.nt_create(0)
    h = P.nt_circuit_load(ctx, c)
    try:
        P.nt_set_precision(ctx, P.NT_C64)
        P.nt_circuit_set_fusion(h, P.NT_C64, width)
        n = gold["n_state_traj"]
        worst = 0.0
        for rec in gold["rates"]:
            p = rec["p"]
            P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
            f = np.zeros(n)
            P.nt_run(ctx, h, 0, 0, n, TAU, f)
            d = np.abs(f - np.asarray(rec["F"]))
            worst = max(worst, float(d.max()))
            assert d.max() <= 2e-5, (width, rec["j"], float(d.max()))
        _say(f"config1 fidelities c64, fusion width {width}: max |F - F_oracle| = {worst:.2e}")
    finally:
        P.nt_circuit_free(h)
        P.nt_destroy(ctx)
