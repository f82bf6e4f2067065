"""Pins of the oracle's large-state branch.

From 20 qubits up the oracle applies gates and Pauli errors with loops that
are parallel over amplitudes, and from 22 qubits its Monte Carlo and
exhaustive runs take that branch.  Every full-size expected value of the
24- and 30-qubit workloads comes from it, so it is pinned here against
closed forms (GHZ, QFT = sqrt(N) ifft, QFT of GHZ, GHZ chains with every site
fired) and against an independent tensor-contraction simulator
(``pinlib.tn_simulate``), at 20-22 qubits.
"""
import math

import numpy as np
import pytest

import pinlib
import workloads as W


def _rand_circuit(n, rng, depth):
    """U / CNOT / CP / SWAP / RZZ / CZ / RX mix between random pairs."""
    gates = []
    for _ in range(depth):
        a, b = (int(x) for x in rng.choice(n, 2, replace=False))
        kind = rng.integers(0, 6)
        if kind == 0:
            gates.append(W.Gate("U", (a,), tuple(rng.uniform(0, 2 * math.pi, 3))))
        elif kind == 1:
            gates.append(W.Gate("CNOT", (a, b)))
        elif kind == 2:
            gates.append(W.Gate("CP", (a, b), (float(rng.uniform(0, 2 * math.pi)),)))
        elif kind == 3:
            gates.append(W.Gate("SWAP", (a, b)))
        elif kind == 4:
            gates.append(W.Gate("RZZ", (a, b), (float(rng.uniform(0, 2 * math.pi)),)))
        else:
            gates.append(W.Gate("RX", (a,), (float(rng.uniform(0, 2 * math.pi)),)))
    return W.Circuit(n, gates)


@pytest.mark.parametrize("n", [20, 21])
def test_ghz_large(orc, n):
    psi = orc.final_state_pattern(W.ghz(n), [], [])
    h = 1 / math.sqrt(2)
    assert abs(psi[0] - h) < 1e-15 and abs(psi[-1] - h) < 1e-15
    rest = psi[1:-1]
    assert np.count_nonzero(rest) == 0


def test_qft_basis_state_large_vs_fft(orc):
    n = 20
    N = 1 << n
    for x in (1, 12345, N - 3):
        psi = orc.final_state_pattern(W.qft(n), [], [], init_index=x)
        e = np.zeros(N, complex)
        e[x] = 1
        ref = math.sqrt(N) * np.fft.ifft(e)
        assert np.abs(psi - ref).max() < 1e-12


def test_qft_of_ghz_large_closed_form(orc):
    n = 20
    N = 1 << n
    c = W.Circuit(n, W.ghz(n).gates + W.qft(n).gates)
    psi = orc.final_state_pattern(c, [], [])
    k = np.arange(N)
    amp = (1 + np.exp(-2j * math.pi * k / N)) / math.sqrt(2 * N)
    assert np.abs(psi - amp).max() < 1e-12
    np.testing.assert_allclose(np.abs(psi) ** 2, (1 + np.cos(2 * math.pi * k / N)) / N, atol=1e-15)


@pytest.mark.parametrize("pauli,code", [("X", (1.0, 0.0, 0.0)), ("Z", (0.0, 0.0, 1.0))])
def test_ghz_chain_every_site_fired_22(orc, pauli, code):
    # error model "always X" / "always Z": every site fires, through the
    # sampler and the parallel gate and Pauli loops
    n = 22
    psi = orc.final_state(W.ghz(n), *code, seed=0, traj=0)
    want = pinlib.ghz_chain_all_fired(n, pauli)
    idx = np.flatnonzero(np.abs(psi) > 1e-12)
    assert sorted(idx.tolist()) == sorted(want)
    for k, v in want.items():
        assert abs(psi[k] - v) < 1e-14


@pytest.mark.parametrize("n,seed", [(20, 3), (21, 4)])
def test_random_circuit_fixed_pattern_vs_tensor_sim(orc, n, seed):
    rng = np.random.default_rng(seed)
    c = _rand_circuit(n, rng, 36)
    S = c.S
    sites = np.sort(rng.choice(S, 9, replace=False)).astype(np.int32)
    paulis = rng.integers(1, 4, size=sites.size).astype(np.uint8)
    got = orc.final_state_pattern(c, sites, paulis)
    want = pinlib.tn_simulate(c, dict(zip(sites.tolist(), paulis.tolist())))
    assert np.linalg.norm(got - want) < 1e-12
    assert abs(np.linalg.norm(got) - 1) < 1e-13


def test_mc_run_large_branch_vs_tensor_sim(orc):
    # orc.run takes its large-state branch at n >= 22: reference, per
    # trajectory state and the sequential fidelity sums
    n = 22
    rng = np.random.default_rng(7)
    c = _rand_circuit(n, rng, 24)
    p = 0.05
    fid, cnt = orc.run(c, p / 3, p / 3, p / 3, seed=11, t0=0, N=3, tau=0.9)
    ref = pinlib.tn_simulate(c)
    want = []
    for t in range(3):
        s, pa = orc.sample_trajectory(11, 0, t, c.S, p / 3, p / 3, p / 3)
        psi = pinlib.tn_simulate(c, dict(zip(s.tolist(), pa.tolist())))
        want.append(pinlib.fid(ref, psi))
    np.testing.assert_allclose(fid, want, rtol=0, atol=1e-12)
    assert cnt == sum(1 for f in want if f >= 0.9)
    assert any(len(orc.sample_trajectory(11, 0, t, c.S, p / 3, p / 3, p / 3)[0]) for t in range(3))


def test_exhaustive_large_branch_vs_tensor_sim(orc):
    n = 22
    c = W.Circuit(n, [W.Gate("H", (0,)), W.Gate("CNOT", (0, 21)), W.Gate("RX", (21,), (0.7,)),
                      W.Gate("CP", (21, 5), (1.1,))])
    out = orc.exhaustive(c)
    ref = pinlib.tn_simulate(c)
    for s in range(c.S):
        for e in (1, 2, 3):
            psi = pinlib.tn_simulate(c, {s: e})
            assert abs(out[s, e - 1] - pinlib.fid(ref, psi)) < 1e-12


def test_tensor_sim_vs_kron_small():
    # the tensor simulator itself against full Kronecker operators
    rng = np.random.default_rng(5)
    c = _rand_circuit(5, rng, 30)
    sites = sorted(rng.choice(c.S, 6, replace=False).tolist())
    pat = [0] * c.S
    fired = {}
    for s in sites:
        pat[s] = int(rng.integers(1, 4))
        fired[s] = pat[s]
    want = pinlib.simulate_pattern(c, pat)
    got = pinlib.tn_simulate(c, fired)
    assert np.abs(got - want).max() < 1e-13
