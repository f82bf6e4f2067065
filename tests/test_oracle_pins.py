"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks it against a
printed worked example, a closed form, an independent construction (expm of
generators, Kronecker products, exact density matrices, full enumeration of
error patterns) or a published reference implementation (numpy's Philox).
"""
import json
import math
import os

import numpy as np
import pytest

import pinlib
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rand_state(rng, n):
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


# --------------------------------------------------------------------------
# Q-1: Pauli actions (Sec. II, Eq. 2 and the XX example).

def _cmat(rows):
    return np.array([[complex(re, im) for re, im in row] for row in rows])


def test_eq2_worked_actions(orc):
    gold = json.load(open(os.path.join(GOLD, "eq2_pauli_actions.json")))
    rng = np.random.default_rng(1)
    for code, name in ((1, "X"), (2, "Y"), (3, "Z")):
        a = rand_state(rng, 1)
        out = orc.apply_pauli(a, 1, 0, code)
        np.testing.assert_allclose(out, _cmat(gold[name]) @ a, atol=1e-15)
    # XX on |psi> = a0|00> + a1|01> + a2|10> + a3|11> (paper's printed order:
    # leftmost label = qubit 1, so index = 2*b1 + b0 matches k's bits).
    a = rand_state(rng, 2)
    out = orc.apply_pauli(orc.apply_pauli(a, 2, 0, 1), 2, 1, 1)
    np.testing.assert_allclose(out, _cmat(gold["XX"]) @ a, atol=1e-15)


def test_pauli_identities(orc):
    rng = np.random.default_rng(2)
    n = 3
    a = rand_state(rng, n)
    for q in range(n):
        for code in (1, 2, 3):        # X^2 = Y^2 = Z^2 = I
            b = orc.apply_pauli(orc.apply_pauli(a, n, q, code), n, q, code)
            np.testing.assert_allclose(b, a, atol=1e-15)
        # XY = iZ  (apply Y first, then X)
        xy = orc.apply_pauli(orc.apply_pauli(a, n, q, 2), n, q, 1)
        np.testing.assert_allclose(xy, 1j * orc.apply_pauli(a, n, q, 3), atol=1e-15)
        # Y = i X Z
        y = orc.apply_pauli(a, n, q, 2)
        xz = orc.apply_pauli(orc.apply_pauli(a, n, q, 3), n, q, 1)
        np.testing.assert_allclose(y, 1j * xz, atol=1e-15)


# --------------------------------------------------------------------------
# Q-2: gate matrices and gate application.

GATES_1Q = [("H", ()), ("X", ()), ("Y", ()), ("Z", ()), ("S", ()), ("T", ()),
            ("RX", (0.731,)), ("RY", (-1.913,)), ("RZ", (2.417,)), ("U", (0.3, 1.1, 5.9))]
GATES_2Q = [("CNOT", ()), ("CZ", ()), ("CP", (0.4321,)), ("SWAP", ()), ("RZZ", (1.234,))]


@pytest.mark.parametrize("name,params", GATES_1Q + GATES_2Q)
def test_gate_matrix_vs_generators(orc, name, params):
    np.testing.assert_allclose(orc.gate_matrix(name, params),
                               pinlib.gate_unitary(name, params), atol=1e-14)


def test_u_is_rz_ry_rz_order(orc):
    # Rz(c) must act first: U(a,b,c) != Rz(c) Ry(b) Rz(a) for generic angles.
    a, b, c = 0.3, 1.1, 2.0
    U = orc.gate_matrix("U", (a, b, c))
    wrong = pinlib.rot(pinlib.PZ, c) @ pinlib.rot(pinlib.PY, b) @ pinlib.rot(pinlib.PZ, a)
    assert np.abs(U - wrong).max() > 1e-3


def _random_unitary(rng, d):
    z = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_gate_application_vs_kron(orc, n):
    rng = np.random.default_rng(10 + n)
    for trial in range(12):
        a = rand_state(rng, n)
        if n >= 2 and trial % 2:
            name, params = GATES_2Q[trial % len(GATES_2Q)]
            qa, qb = (int(x) for x in rng.choice(n, 2, replace=False))
            qs = [qa, qb]
            mat = None
            if trial % 5 == 0:
                name, params, mat = "U2Q", (), _random_unitary(rng, 4)
        else:
            name, params = GATES_1Q[trial % len(GATES_1Q)]
            qs = [int(rng.integers(n))]
            mat = None
            if trial % 4 == 0:
                name, params, mat = "U1Q", (), _random_unitary(rng, 2)
        full = pinlib.embed(n, qs, pinlib.gate_unitary(name, params, mat))
        got = orc.apply_gate(a, n, name, qs, params, mat)
        np.testing.assert_allclose(got, full @ a, atol=1e-14)
        assert abs(np.linalg.norm(got) - 1) < 1e-14


def test_cnot_control_target_orientation(orc):
    # CNOT(0 -> 1) on |01> (qubit 0 set) gives |11>; on |10> it does nothing.
    e = np.zeros(4, complex)
    e[1] = 1
    out = orc.apply_gate(e, 2, "CNOT", [0, 1])
    assert abs(out[3] - 1) < 1e-15
    e = np.zeros(4, complex)
    e[2] = 1
    out = orc.apply_gate(e, 2, "CNOT", [0, 1])
    assert abs(out[2] - 1) < 1e-15


# --------------------------------------------------------------------------
# Q-3: closed forms.

@pytest.mark.parametrize("n", [2, 5, 9])
def test_ghz_closed_form(orc, n):
    psi = orc.final_state_pattern(W.ghz(n), [], [])
    want = np.zeros(1 << n, complex)
    want[0] = want[-1] = 1 / math.sqrt(2)
    np.testing.assert_allclose(psi, want, atol=1e-15)
    assert np.count_nonzero(np.abs(psi) > 0) == 2


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("pauli", ["X", "Z"])
def test_ghz_chain_every_site_fired(orc, n, pauli):
    """Every site fires one Pauli (p = 1 of one type): the oracle's sampled
    run, a brute-force simulation of the pattern and the propagation
    argument of pinlib.ghz_chain_all_fired agree."""
    c = W.ghz(n)
    want = np.zeros(1 << n, complex)
    for k, a in pinlib.ghz_chain_all_fired(n, pauli).items():
        want[k] = a
    code = {"X": 1, "Z": 3}[pauli]
    np.testing.assert_allclose(pinlib.simulate_pattern(c, [code] * c.S), want, atol=1e-14)
    model = (1.0, 0.0, 0.0) if pauli == "X" else (0.0, 0.0, 1.0)
    np.testing.assert_allclose(orc.final_state(c, *model, 3, 0), want, atol=1e-15)


@pytest.mark.parametrize("n", [3, 5, 8])
def test_qft_basis_states_vs_fft(orc, n):
    N = 1 << n
    c = W.qft(n)
    for x in (0, 1, N // 3, N - 1):
        psi = orc.final_state_pattern(c, [], [], init_index=x)
        e = np.zeros(N, complex)
        e[x] = 1
        np.testing.assert_allclose(psi, math.sqrt(N) * np.fft.ifft(e), atol=1e-13)


@pytest.mark.parametrize("n", [4, 7])
def test_qft_of_ghz_closed_form(orc, n):
    N = 1 << n
    psi = orc.final_state_pattern(W.ghz(n) + W.qft(n), [], [])
    k = np.arange(N)
    np.testing.assert_allclose(np.abs(psi) ** 2, (1 + np.cos(2 * np.pi * k / N)) / N, atol=1e-14)
    np.testing.assert_allclose(psi, (1 + np.exp(-2j * np.pi * k / N)) / math.sqrt(2 * N), atol=1e-13)


def test_norm_preserved_random_circuit(orc):
    c = W.random_layers(10, 12, np.random.default_rng(3))
    psi = orc.final_state_pattern(c, [], [])
    assert abs(np.vdot(psi, psi).real - 1) < 1e-13


# --------------------------------------------------------------------------
# Q-4: Philox4x64-10 against numpy's implementation (counter is pre-incremented
# by numpy before each block, so start it one below the wanted counter).

def _numpy_philox_block(counter, key):
    c = [int(x) for x in counter]
    # subtract one with borrow across the 256-bit counter
    for i in range(4):          # wraps to all-ones when the counter is zero
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = (1 << 64) - 1
    bg = np.random.Philox(counter=np.array(c, np.uint64), key=np.array(key, np.uint64))
    return bg.random_raw(4)


def test_philox_matches_numpy(orc):
    rng = np.random.default_rng(4)
    cases = [([0, 0, 0, 0], [0, 0]), ([1, 0, 0, 0], [5, 7]),
             ([(1 << 64) - 1, (1 << 64) - 1, (1 << 64) - 1, (1 << 64) - 1], [(1 << 64) - 1, (1 << 64) - 1]),
             ([3046, 9999, 0, 0], [0, 0])]
    for _ in range(40):
        cases.append((list(rng.integers(0, 1 << 63, 4, dtype=np.uint64) * 2 + 1),
                      list(rng.integers(0, 1 << 63, 2, dtype=np.uint64))))
    for ctr, key in cases:
        np.testing.assert_array_equal(orc.philox4x64_10(ctr, key), _numpy_philox_block(ctr, key))


def test_thresholds(orc):
    th, alw = orc.thresholds(0.25, 0.25, 0.0)
    assert int(th[0]) == 1 << 63 and not alw[0]          # 0.5 * 2^64
    assert int(th[1]) == 1 << 63                         # X share 1/2
    assert alw[2]                                        # X or Y share = 1
    th, alw = orc.thresholds(0.0, 0.0, 0.0)
    assert int(th[0]) == 0 and not alw[0]
    th, alw = orc.thresholds(0.5, 0.25, 0.25)
    assert alw[0]                                        # total 1 => always
    p = 1e-3
    th, alw = orc.thresholds(p / 3, p / 3, p / 3)
    assert int(th[0]) == math.floor(math.ldexp((p / 3 + p / 3) + p / 3, 64))
    # uniform model: the type split is thr(1/3), thr(2/3) at every rate, also
    # where (p/3) / (p/3 + p/3 + p/3) rounds away from 1/3
    third = math.floor(math.ldexp(1.0 / 3.0, 64))
    two_thirds = math.floor(math.ldexp(2.0 / 3.0, 64))
    drifts = 0
    for p in (6.8e-5, 1e-4, 1.4318e-4, 2.7e-4, 1e-3, 0.3):
        th, alw = orc.thresholds(p / 3, p / 3, p / 3)
        assert (int(th[1]), int(th[2])) == (third, two_thirds)
        x = p / 3
        drifts += math.floor(math.ldexp(x / (x + x + x), 64)) != third
    assert drifts > 0   # the plain quotient would move the split with the rate


# --------------------------------------------------------------------------
# Q-5: sampling statistics, nesting (common random numbers).

def test_sampling_binomial_and_types(orc):
    S, N, p = 500, 400, 0.02
    tot = 0
    types = np.zeros(4)
    for t in range(N):
        s, pa = orc.sample_trajectory(0, 0, t, S, p / 3, p / 3, p / 3)
        assert np.all(np.diff(s) > 0)
        tot += len(s)
        types += np.bincount(pa, minlength=4)
    mean, var = N * S * p, N * S * p * (1 - p)
    assert abs(tot - mean) / math.sqrt(var) < 5
    for k in (1, 2, 3):
        f = types[k] / tot
        assert abs(f - 1 / 3) < 5 * math.sqrt((1 / 3) * (2 / 3) / tot)


def test_sampling_nested_across_rates(orc):
    S = 800
    for t in range(50):
        lo_s, lo_p = orc.sample_trajectory(7, 3, t, S, 1e-3 / 3, 1e-3 / 3, 1e-3 / 3)
        hi_s, hi_p = orc.sample_trajectory(7, 3, t, S, 3e-2 / 3, 3e-2 / 3, 3e-2 / 3)
        hi = dict(zip(hi_s.tolist(), hi_p.tolist()))
        for s, pa in zip(lo_s.tolist(), lo_p.tolist()):
            assert s in hi and hi[s] == pa


def test_sampling_is_philox_threshold_rule(orc):
    # Brute force: recompute the rule from numpy's Philox for a few sites.
    p = 0.3
    th, _ = orc.thresholds(p / 3, p / 3, p / 3)
    s_list, p_list = orc.sample_trajectory(11, 2, 5, 64, p / 3, p / 3, p / 3)
    got = dict(zip(s_list.tolist(), p_list.tolist()))
    for s in range(64):
        w = _numpy_philox_block([s, 5, 0, 0], [11, 2])
        if int(w[0]) < int(th[0]):
            want = 1 if int(w[1]) < int(th[1]) else (2 if int(w[1]) < int(th[2]) else 3)
            assert got.get(s) == want
        else:
            assert s not in got


# --------------------------------------------------------------------------
# Site order and error placement: the oracle's own sampler + run equals an
# independent simulation of the same pattern (Sec. IV-B.2: after each gate,
# independently on each of its qubits).

def test_errors_applied_at_sites(orc):
    rng = np.random.default_rng(5)
    c = W.random_layers(4, 3, rng) + W.qft(4)
    S = c.S
    ops = pinlib.circuit_unitaries(c)
    for t in range(6):
        p = 0.3
        s_list, p_list = orc.sample_trajectory(9, 0, t, S, p / 3, p / 3, p / 3)
        pat = [0] * S
        for s, pa in zip(s_list, p_list):
            pat[int(s)] = int(pa)
        want = pinlib.simulate_pattern(c, pat, ops)
        got = orc.final_state(c, p / 3, p / 3, p / 3, 9, t)
        np.testing.assert_allclose(got, want, atol=1e-13)


# --------------------------------------------------------------------------
# Q-6: trajectory mean of linear criteria -> exact density matrix.

@pytest.mark.parametrize("n,layers", [(3, 3), (5, 2)])
def test_mc_mean_converges_to_density_matrix(orc, n, layers):
    c = W.random_layers(n, layers, np.random.default_rng(20 + n))
    p = 0.05
    rho = pinlib.density_depolarizing(c, p / 3, p / 3, p / 3)
    ref = pinlib.simulate_pattern(c, [0] * c.S)
    exact_F = np.vdot(ref, rho @ ref).real
    N = 6000
    fid, _ = orc.run(c, p / 3, p / 3, p / 3, 1, 0, N, 0.9)
    se = fid.std() / math.sqrt(N)
    assert abs(fid.mean() - exact_F) < 5 * se + 1e-12
    # diagonal of rho from the trajectories' |a_k|^2
    probs = np.zeros(1 << n)
    M = 1500
    acc = []
    for t in range(M):
        psi = orc.final_state(c, p / 3, p / 3, p / 3, 1, t)
        acc.append(np.abs(psi) ** 2)
    acc = np.array(acc)
    probs = acc.mean(0)
    se = acc.std(0) / math.sqrt(M)
    assert np.all(np.abs(probs - np.diag(rho).real) < 5 * se + 1e-9)


# --------------------------------------------------------------------------
# Q-7 / Q-9: success probability (indicator criterion) vs exact enumeration of
# every Pauli pattern, and the tolerable-rate search vs the exact root.

@pytest.fixture(scope="module")
def tiny():
    rng = np.random.default_rng(30)
    # n = 3, 5 gates, S = 7 -> 4^7 = 16384 patterns
    g = W.random_layers(3, 1, rng).gates[:4] + [W.Gate("RZZ", (0, 2), (0.7,))]
    c = W.Circuit(3, g, "tiny")
    assert c.S == 7
    coeff = pinlib.enumerate_success_weights(c, 0.9)
    return c, coeff


def test_success_probability_vs_enumeration(orc, tiny):
    c, coeff = tiny
    S = c.S
    assert coeff[0] == 1
    for p in (0.02, 0.1, 0.3):
        exact = pinlib.success_poly(coeff, S, p)
        N = 20000
        _, cnt = orc.run(c, p / 3, p / 3, p / 3, 3, 0, N, 0.9)
        phat = cnt / N
        sigma = math.sqrt(exact * (1 - exact) / N)
        assert abs(phat - exact) < 5 * sigma + 1e-12, (p, phat, exact)


def test_tolerable_rate_vs_exact_root(orc, tiny):
    from scipy.optimize import brentq
    c, coeff = tiny
    S = c.S
    Pt = 0.66
    pstar = brentq(lambda p: pinlib.success_poly(coeff, S, p) - Pt, 1e-6, 0.75)
    N = 20000
    rc, phat, probes = orc.tolerable_rate(c, Pt, 0.01, 1e-3, 0.7, 5, N, 0.9)
    assert rc == 0 and probes >= 3
    mc_err = 5 * math.sqrt(Pt * (1 - Pt) / N)
    assert abs(pinlib.success_poly(coeff, S, phat) - Pt) <= 0.01 + mc_err
    assert abs(math.log10(phat) - math.log10(pstar)) < 0.5
    # not bracketed
    rc, _, _ = orc.tolerable_rate(c, Pt, 0.01, 0.5, 0.7, 5, 2000, 0.9)
    assert rc == 1


# --------------------------------------------------------------------------
# Q-8: exhaustive single errors (Sec. IV-B.1, Eq. 3) and Eq. 4 / Eq. 5.

def test_exhaustive_matches_first_order_coefficient(orc, tiny):
    c, coeff = tiny
    F = orc.exhaustive(c)
    assert F.shape == (c.S, 3)
    # weight-1 successes of the enumeration = exhaustive successes
    assert int((F >= 0.9).sum()) == int(coeff[1])
    # each single-error state equals the independent simulation
    ops = pinlib.circuit_unitaries(c)
    ref = pinlib.simulate_pattern(c, [0] * c.S, ops)
    for s in range(c.S):
        for e in (1, 2, 3):
            pat = [0] * c.S
            pat[s] = e
            assert abs(F[s, e - 1] - pinlib.fid(ref, pinlib.simulate_pattern(c, pat, ops))) < 1e-12


def test_eq4_is_first_order_of_exact_success(orc, tiny):
    c, coeff = tiny
    S = c.S
    F = orc.exhaustive(c)
    succ = (F >= 0.9).astype(float)
    P_e = succ.mean(0)                      # per-type single-error success
    P_R = 1.0
    for p in (1e-4, 1e-3):
        E_e = [S * p / 3] * 3               # expected errors counted over sites
        eq4 = orc.eq4(P_e, P_R, E_e)
        exact = pinlib.success_poly(coeff, S, p)
        assert abs(eq4 - exact) < 3 * (S * p) ** 2    # agree to first order in p
    # Eq. 5 inverts Eq. 4 at a target
    Pt = 0.9
    p5 = orc.eq5(Pt, P_e, P_R, S)
    E_e = [S * p5 / 3] * 3
    assert abs(orc.eq4(P_e, P_R, E_e) - Pt) < 1e-12
    # p < 1/units whenever the target exceeds the one-error success (Sec. IV-D)
    assert P_e.mean() < Pt and p5 < 1.0 / S


# --------------------------------------------------------------------------
# Other criteria (Sec. II): correct-outcome probability and heavy output.

def test_criteria_vs_bruteforce(orc):
    c = W.random_layers(4, 3, np.random.default_rng(40))
    p = 0.05
    ops = pinlib.circuit_unitaries(c)
    ref = pinlib.simulate_pattern(c, [0] * c.S, ops)
    pr = np.abs(ref) ** 2
    med = np.median(pr)
    assert abs(orc.median_prob(ref, c.n) - med) < 1e-15
    heavy = pr > med
    target = int(np.argmax(pr))
    v1 = orc.run_criterion(c, p / 3, p / 3, p / 3, 2, 0, 8, 1, target)
    v2 = orc.run_criterion(c, p / 3, p / 3, p / 3, 2, 0, 8, 2)
    for t in range(8):
        s_list, p_list = orc.sample_trajectory(2, 0, t, c.S, p / 3, p / 3, p / 3)
        pat = [0] * c.S
        for s, pa in zip(s_list, p_list):
            pat[int(s)] = int(pa)
        psi = pinlib.simulate_pattern(c, pat, ops)
        pp = np.abs(psi) ** 2
        assert abs(v1[t] - pp[target] / pp.sum()) < 1e-13
        assert abs(v2[t] - pp[heavy].sum() / pp.sum()) < 1e-13


def test_fidelity_definition(orc):
    rng = np.random.default_rng(6)
    a = rand_state(rng, 4) * 1.7
    b = rand_state(rng, 4) * 0.3
    want = abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)
    assert abs(orc.fidelity(a, b, 4) - want) < 1e-15
    assert orc.fidelity(a, a, 4) == pytest.approx(1.0, abs=1e-15)


# Exhaustive branch under the measurement criteria (Sec. IV-B.1 with Sec. II):
# each single-error state against a brute-force statevector.
def test_exhaustive_criteria_vs_bruteforce(orc):
    c = W.random_layers(4, 3, np.random.default_rng(41))
    ops = pinlib.circuit_unitaries(c)
    ref = pinlib.simulate_pattern(c, [0] * c.S, ops)
    pr = np.abs(ref) ** 2
    heavy = pr > np.median(pr)
    target = int(np.argmax(pr))
    v1, r1 = orc.exhaustive_criterion(c, 1, target)
    v2, r2 = orc.exhaustive_criterion(c, 2)
    v0, r0 = orc.exhaustive_criterion(c, 0)
    assert abs(r1 - pr[target] / pr.sum()) < 1e-14
    assert abs(r2 - pr[heavy].sum() / pr.sum()) < 1e-14
    assert abs(r0 - 1.0) < 1e-14
    for s in range(c.S):
        for e in range(3):
            pat = [0] * c.S
            pat[s] = e + 1
            psi = pinlib.simulate_pattern(c, pat, ops)
            pp = np.abs(psi) ** 2
            assert abs(v1[s, e] - pp[target] / pp.sum()) < 1e-13
            assert abs(v2[s, e] - pp[heavy].sum() / pp.sum()) < 1e-13
            fid = abs(np.vdot(ref, psi)) ** 2 / (np.vdot(ref, ref).real * pp.sum())
            assert abs(v0[s, e] - fid) < 1e-13


# An error on a qubit's last site acts after every gate on that qubit: Z leaves
# every measurement probability unchanged, X and Y move the target's
# probability to the index with that bit flipped.
def test_criteria_last_site_pauli_invariants(orc):
    c = W.random_layers(5, 4, np.random.default_rng(42))
    last = {}
    s = 0
    for g in c.gates:
        for q in g.qubits:
            last[q] = s
            s += 1
    ref = orc.final_state_pattern(c, [], [])
    pr = np.abs(ref) ** 2 / np.vdot(ref, ref).real
    target = 11
    v1, r1 = orc.exhaustive_criterion(c, 1, target)
    v2, r2 = orc.exhaustive_criterion(c, 2)
    for q, site in last.items():
        assert abs(v1[site, 2] - r1) < 1e-13          # Z
        assert abs(v2[site, 2] - r2) < 1e-13
        for e in (0, 1):                               # X, Y
            assert abs(v1[site, e] - pr[target ^ (1 << q)]) < 1e-13


# Heavy-output probability of a Haar-like state: for Porter-Thomas distributed
# probabilities the mass above the median tends to (1 + ln 2) / 2 ~ 0.847.
def test_heavy_output_porter_thomas(orc):
    c = W.random_layers(12, 24, np.random.default_rng(43))
    # |0...0>: median 0, the heavy set is {0} and holds all the mass
    _, r2 = orc.exhaustive_criterion(W.Circuit(c.n, c.gates[:0]), 2)
    assert r2 == 1.0
    vals = orc.run_criterion(c, 0.0, 0.0, 0.0, 0, 0, 1, 2)
    assert abs(vals[0] - (1 + math.log(2)) / 2) < 0.02


# Quantum-volume model circuits (general U2Q): the noiseless heavy-output
# probability of a square model circuit approaches (1 + ln 2) / 2, and the
# Pauli-twirled depolarizing limit (p -> 3/4 per touched qubit, uniform Paulis)
# gives the uniform distribution, whose heavy mass is exactly 1/2.
def test_heavy_output_quantum_volume(orc):
    vals = []
    for s in range(6):
        c = W.quantum_volume(10, 10, np.random.default_rng(500 + s))
        vals.append(orc.run_criterion(c, 0.0, 0.0, 0.0, 0, 0, 1, 2)[0])
    assert abs(np.mean(vals) - (1 + math.log(2)) / 2) < 0.03
    c = W.quantum_volume(6, 6, np.random.default_rng(7))
    v = orc.run_criterion(c, 0.25, 0.25, 0.25, 0, 0, 400, 2)
    # 400 trajectories of a fully scrambled state: mean 1/2 within ~5 sigma
    assert abs(v.mean() - 0.5) < 0.05


# --------------------------------------------------------------------------
# The paper's tolerable-rate steps (Sec. IV-D, Fig. 3): exhaustive simulation
# first, Eq. 5 when at most one error is tolerable, else Monte Carlo at
# increasing rates.

def _single_error_success(circ, tau):
    """P_e (X, Y, Z) from brute-force single-error states (Kronecker sims)."""
    ops = pinlib.circuit_unitaries(circ)
    S = len(pinlib.site_list(circ))
    ref = pinlib.simulate_pattern(circ, [0] * S, ops)
    P = []
    for e in (1, 2, 3):
        ok = 0
        for s in range(S):
            pat = [0] * S
            pat[s] = e
            ok += pinlib.fid(ref, pinlib.simulate_pattern(circ, pat, ops)) >= tau
        P.append(ok / S)
    return np.array(P), S


def test_fig3_eq5_branch_vs_bruteforce(orc):
    rng = np.random.default_rng(21)
    c = W.random_layers(3, 2, rng)
    tau, Pt = 0.9, 0.66
    P_e, S = _single_error_success(c, tau)
    P1 = P_e.mean()
    assert P1 <= Pt            # this circuit tolerates at most one error on average
    rc, p, method, probes, p4 = orc.tolerable_rate_fig3(c, Pt, 0.01, 0, 1000, tau)
    assert rc == 0 and method == 0 and probes == 0
    np.testing.assert_array_equal(p4[:3], P_e)
    assert p4[3] == 1.0
    want = (Pt - 1.0) / (P1 - 1.0) / S          # Eq. 5 with S error locations
    assert abs(p - want) <= 1e-15 * want
    assert p <= 1.0 / S                          # the corollary of Eq. 5 (Sec. IV-D)


def test_fig3_monte_carlo_branch_vs_exact_root(orc):
    from scipy.optimize import brentq
    # Two qubits, each prepared with Bloch vector (1, 1, 1)/sqrt(3), then
    # identity rotations (more error sites, no change of state): any Pauli
    # on one qubit leaves F = 1/3, on both F = 1/9.  With tau = 0.3 every
    # single error is tolerated (P1 = 1), so the steps go to Monte Carlo.
    th = math.acos(1 / math.sqrt(3))
    g = []
    for q in (0, 1):
        g.append(W.Gate("U", (q,), (math.pi / 4, th, 0.0)))
        g += [W.Gate("RZ", (q,), (0.0,)) for _ in range(3)]
    c = W.Circuit(2, g)
    tau, Pt, tol, N = 0.3, 0.66, 0.01, 20000
    P_e, S = _single_error_success(c, tau)
    assert P_e.tolist() == [1.0, 1.0, 1.0]
    rc, p, method, probes, p4 = orc.tolerable_rate_fig3(c, Pt, tol, 5, N, tau)
    assert rc == 0 and method == 1 and probes >= 2
    assert p4.tolist() == [1.0, 1.0, 1.0, 1.0]
    cw = pinlib.enumerate_success_weights(c, tau)
    P_exact = pinlib.success_poly(cw, S, p)
    sigma = math.sqrt(Pt * (1 - Pt) / N)
    assert abs(P_exact - Pt) <= tol + 5 * sigma
    root = brentq(lambda x: pinlib.success_poly(cw, S, x) - Pt, 1e-6, 0.5)
    assert root > 1.0 / S          # more than one error on average is tolerable
    assert abs(math.log10(p / root)) < 0.05
