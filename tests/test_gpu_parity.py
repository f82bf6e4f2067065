"""GPU parity: the HIP library against the CPU oracle on identical inputs.

Bar (for identical Philox seeds):
  * fired error sites: bit-exact (site index and Pauli);
  * final amplitudes: L2 distance <= 1e-12 (complex128) / 1e-5 (complex64)
    per unit-norm trajectory state;
  * fidelities: |F_gpu - F_oracle| <= 1e-12 (complex128) / 2e-5 (complex64);
  * success counts: equal, except for trajectories whose oracle fidelity lies
    within the precision's fidelity error of tau (reported by id).
"""
import math
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TAU = 0.9


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2301_07264_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def ctx(P):
    c = P.nt_create(0)
    yield c
    P.nt_destroy(c)


def _load(P, circ, cid=0):
    h = P.nt_circuit_load(None, circ)
    if cid:
        P.nt_circuit_set_id(h, cid)
    return h


def _l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.complex128) - np.asarray(b, np.complex128)))


def _all_gates_circuit(n, layers, seed):
    rng = np.random.default_rng(seed)
    gates = []
    names1 = ["H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "U", "U1Q"]
    names2 = ["CNOT", "CZ", "CP", "SWAP", "RZZ", "U2Q"]
    for _ in range(layers):
        for q in range(n):
            nm = names1[int(rng.integers(len(names1)))]
            if nm in ("RX", "RY", "RZ"):
                gates.append(W.Gate(nm, (q,), (float(rng.uniform(0, 2 * math.pi)),)))
            elif nm == "U":
                gates.append(W.Gate(nm, (q,), tuple(float(x) for x in rng.uniform(0, 2 * math.pi, 3))))
            elif nm == "U1Q":
                z = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
                qm, r = np.linalg.qr(z)
                gates.append(W.Gate(nm, (q,), (), qm * (np.diag(r) / np.abs(np.diag(r)))))
            else:
                gates.append(W.Gate(nm, (q,)))
        perm = rng.permutation(n)
        for i in range(n // 2):
            a, b = int(perm[2 * i]), int(perm[2 * i + 1])
            nm = names2[int(rng.integers(len(names2)))]
            if nm in ("CP", "RZZ"):
                gates.append(W.Gate(nm, (a, b), (float(rng.uniform(0, 2 * math.pi)),)))
            elif nm == "U2Q":
                z = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
                qm, r = np.linalg.qr(z)
                gates.append(W.Gate(nm, (a, b), (), qm * (np.diag(r) / np.abs(np.diag(r)))))
            else:
                gates.append(W.Gate(nm, (a, b)))
    return W.Circuit(n, gates, f"allgates{n}")


# ---------------------------------------------------------------------------
# Error sites: bit-exact.

@pytest.mark.parametrize("p", [1e-3, 0.05])
def test_sites_bitexact_config0(P, ctx, orc, p):
    c = W.config0()
    h = _load(P, c)
    P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
    N = 1000
    off, sites, paulis = P.nt_sample_sites(ctx, h, 0, 0, N)
    for t in range(N):
        s_o, p_o = orc.sample_trajectory(0, 0, t, c.S, p / 3, p / 3, p / 3)
        a, b = int(off[t]), int(off[t + 1])
        np.testing.assert_array_equal(sites[a:b], s_o)
        np.testing.assert_array_equal(paulis[a:b], p_o)
    P.nt_circuit_free(h)


def test_sites_bitexact_config1_sample(P, ctx, orc):
    c = W.config1()
    h = _load(P, c, cid=5)
    p = 1e-2
    P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
    t0, N = 9000, 300
    off, sites, paulis = P.nt_sample_sites(ctx, h, 17, t0, N)
    for t in range(N):
        s_o, p_o = orc.sample_trajectory(17, 5, t0 + t, c.S, p / 3, p / 3, p / 3)
        a, b = int(off[t]), int(off[t + 1])
        np.testing.assert_array_equal(sites[a:b], s_o)
        np.testing.assert_array_equal(paulis[a:b], p_o)
    P.nt_circuit_free(h)


def test_sites_uneven_model(P, ctx, orc):
    c = W.config0()
    h = _load(P, c)
    for model in [(0.02, 0.0, 0.0), (0.0, 0.03, 0.01), (0.0, 0.0, 0.05), (0.5, 0.3, 0.2), (0, 0, 0)]:
        P.nt_set_error_model(ctx, *model)
        off, sites, paulis = P.nt_sample_sites(ctx, h, 3, 100, 50)
        for t in range(50):
            s_o, p_o = orc.sample_trajectory(3, 0, 100 + t, c.S, *model)
            a, b = int(off[t]), int(off[t + 1])
            np.testing.assert_array_equal(sites[a:b], s_o)
            np.testing.assert_array_equal(paulis[a:b], p_o)
    P.nt_circuit_free(h)


# ---------------------------------------------------------------------------
# The 8-qubit workload: every trajectory, complex128.

def test_config0_full_parity_c128(P, ctx, orc):
    c = W.config0()
    h = _load(P, c)
    p = 1e-3
    P.nt_set_precision(ctx, P.NT_C128)
    P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
    N = 1000
    fid = np.zeros(N)
    cnt, phat = P.nt_run(ctx, h, 0, 0, N, TAU, fid)
    f_o, c_o = orc.run(c, p / 3, p / 3, p / 3, 0, 0, N, TAU)
    _say("config0 c128 count", cnt, "oracle", c_o, "max |dF|", np.abs(fid - f_o).max())
    assert np.abs(fid - f_o).max() <= 1e-12
    assert cnt == c_o
    assert phat == c_o / N
    for t in (0, 1, 2, 5, 17, 999):
        g = P.nt_final_state(ctx, h, 0, t, P.NT_C128)
        o = orc.final_state(c, p / 3, p / 3, p / 3, 0, t)
        assert _l2(g, o) <= 1e-12, t
    P.nt_circuit_free(h)


# ---------------------------------------------------------------------------
# Every gate kind, single- and multi-pass plans, heavy error rates (many
# frame updates), both precisions.

CASES = [(3, 4), (6, 3), (9, 3), (12, 2), (14, 2), (16, 2)]


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("n,layers", CASES)
def test_all_gates_states(P, ctx, orc, prec, n, layers):
    c = _all_gates_circuit(n, layers, 100 + n)
    h = _load(P, c, cid=3)
    pr = P.NT_C128 if prec == "c128" else P.NT_C64
    tol = 1e-12 if prec == "c128" else 1e-5
    P.nt_set_precision(ctx, pr)
    npass, nseg, L = P.nt_plan_info(h, pr)
    _say(f"all-gates n={n} G={c.G} prec={prec} passes={npass} segments={nseg} L={L}")
    ref = P.nt_reference_state(ctx, h, pr)
    ref_o = orc.final_state_pattern(c, [], [])
    assert _l2(ref, ref_o) <= tol
    for p in (0.0, 0.02, 0.3):
        P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
        for t in range(4):
            g = P.nt_final_state(ctx, h, 11, t, pr)
            o = orc.final_state(c, p / 3, p / 3, p / 3, 11, t, cid=3)
            assert _l2(g, o) <= tol, (p, t, _l2(g, o))
        N = 64
        fid = np.zeros(N)
        cnt, _ = P.nt_run(ctx, h, 11, 0, N, TAU, fid)
        f_o, c_o = orc.run(c, p / 3, p / 3, p / 3, 11, 0, N, TAU, cid=3)
        ftol = 1e-12 if prec == "c128" else 2e-5
        assert np.abs(fid - f_o).max() <= ftol, (p, np.abs(fid - f_o).max())
        margin = np.abs(f_o - TAU) < ftol
        assert int(((fid >= TAU) != (f_o >= TAU))[~margin].sum()) == 0
        if not margin.any():
            assert cnt == c_o
    P.nt_circuit_free(h)


def test_uneven_error_models_states(P, ctx, orc):
    c = _all_gates_circuit(14, 2, 7)
    h = _load(P, c)
    P.nt_set_precision(ctx, P.NT_C128)
    for model in [(0.2, 0.0, 0.0), (0.0, 0.2, 0.0), (0.0, 0.0, 0.2), (0.6, 0.2, 0.2)]:
        P.nt_set_error_model(ctx, *model)
        for t in range(3):
            g = P.nt_final_state(ctx, h, 5, t, P.NT_C128)
            o = orc.final_state(c, *model, 5, t)
            assert _l2(g, o) <= 1e-12, (model, t)
    P.nt_circuit_free(h)


# ---------------------------------------------------------------------------
# Register-heavy circuits: many CNOTs and two-qubit diagonals between random
# pairs, so that the register-permutation CNOT (every target / control
# register-bit pair), the per-lane CNOT, and the diagonal bodies with one or
# both qubits in the registers all run, under error models that flip the
# control value through the frame (X and Y errors) as well as its sign (Z).

def _register_heavy_circuit(n, layers, seed):
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(layers):
        for q in range(n):
            nm = ["U", "H", "RX", "RZ", "RY"][int(rng.integers(5))]
            if nm == "U":
                gates.append(W.Gate(nm, (q,), tuple(float(x) for x in rng.uniform(0, 2 * math.pi, 3))))
            elif nm == "H":
                gates.append(W.Gate(nm, (q,)))
            else:
                gates.append(W.Gate(nm, (q,), (float(rng.uniform(0, 2 * math.pi)),)))
        for _ in range(2 * n):
            a, b = (int(x) for x in rng.choice(n, 2, replace=False))
            nm = ["CNOT", "CNOT", "CZ", "CP", "RZZ"][int(rng.integers(5))]
            if nm in ("CP", "RZZ"):
                gates.append(W.Gate(nm, (a, b), (float(rng.uniform(0, 2 * math.pi)),)))
            else:
                gates.append(W.Gate(nm, (a, b)))
    return W.Circuit(n, gates, f"regheavy{n}")


@pytest.mark.parametrize("prec", ["c64", "c128"])
@pytest.mark.parametrize("n,layers", [(6, 4), (11, 3), (16, 2)])
def test_register_heavy_states(P, ctx, orc, prec, n, layers):
    c = _register_heavy_circuit(n, layers, 300 + n)
    h = _load(P, c, cid=9)
    pr = P.NT_C128 if prec == "c128" else P.NT_C64
    tol = 1e-12 if prec == "c128" else 1e-5
    ftol = 1e-12 if prec == "c128" else 2e-5
    P.nt_set_precision(ctx, pr)
    npass, nseg, L = P.nt_plan_info(h, pr)
    _say(f"register-heavy n={n} G={c.G} prec={prec} passes={npass} segments={nseg} L={L}")
    for model in [(0.0, 0.0, 0.0), (0.2, 0.0, 0.0), (0.0, 0.1, 0.1), (0.1, 0.1, 0.1)]:
        P.nt_set_error_model(ctx, *model)
        for t in range(3):
            g = P.nt_final_state(ctx, h, 21, t, pr)
            o = orc.final_state(c, *model, 21, t, cid=9)
            assert _l2(g, o) <= tol, (model, t, _l2(g, o))
        N = 32
        fid = np.zeros(N)
        P.nt_run(ctx, h, 21, 0, N, TAU, fid)
        f_o, _ = orc.run(c, *model, 21, 0, N, TAU, cid=9)
        assert np.abs(fid - f_o).max() <= ftol, (model, np.abs(fid - f_o).max())
    P.nt_circuit_free(h)


# ---------------------------------------------------------------------------
# Closed forms on the GPU path.

@pytest.mark.parametrize("n", [5, 14, 17])
def test_gpu_ghz_qft_closed_form(P, ctx, n):
    N = 1 << n
    h = _load(P, W.ghz(n) + W.qft(n))
    for pr, tol in ((P.NT_C128, 1e-12), (P.NT_C64, 2e-6)):
        P.nt_set_precision(ctx, pr)
        psi = P.nt_reference_state(ctx, h, pr).astype(np.complex128)
        k = np.arange(N)
        want = (1 + np.exp(-2j * np.pi * k / N)) / math.sqrt(2 * N)
        assert _l2(psi, want) <= tol
    P.nt_circuit_free(h)


# ---------------------------------------------------------------------------
# Results do not depend on batching; runs repeat bit-exactly.

def test_batch_independence_and_determinism(P, ctx):
    c = _all_gates_circuit(15, 2, 9)
    h = _load(P, c)
    P.nt_set_precision(ctx, P.NT_C64)
    P.nt_set_error_model(ctx, 0.01, 0.01, 0.01)
    N = 40
    runs = []
    for mb in (0, 1, 7):
        P.nt_set_max_batch(ctx, mb)
        f = np.zeros(N)
        P.nt_run(ctx, h, 2, 10, N, TAU, f)
        runs.append(f)
    P.nt_set_max_batch(ctx, 0)
    for f in runs[1:]:
        np.testing.assert_array_equal(f.view(np.uint64), runs[0].view(np.uint64))
    # a range split in two gives the same values
    f1 = np.zeros(15)
    f2 = np.zeros(25)
    P.nt_run(ctx, h, 2, 10, 15, TAU, f1)
    P.nt_run(ctx, h, 2, 25, 25, TAU, f2)
    np.testing.assert_array_equal(np.concatenate([f1, f2]).view(np.uint64), runs[0].view(np.uint64))
    P.nt_circuit_free(h)


def test_zero_error_trajectories_score_exactly_one(P, ctx):
    c = W.config1(n=16, layers=6)
    h = _load(P, c)
    for pr in (P.NT_C64, P.NT_C128):
        P.nt_set_precision(ctx, pr)
        P.nt_set_error_model(ctx, 0, 0, 0)
        f = np.zeros(8)
        cnt, _ = P.nt_run(ctx, h, 0, 0, 8, 1.0, f)
        assert np.all(f == 1.0) and cnt == 8
    P.nt_circuit_free(h)


# ---------------------------------------------------------------------------
# Sweep and tolerable-rate search match the oracle exactly (same counts).

def test_sweep_and_tolerable_rate_vs_oracle(P, ctx, orc):
    c = W.config0()
    h = _load(P, c)
    P.nt_set_precision(ctx, P.NT_C128)
    rates = [1e-4, 1e-3, 3e-3, 1e-2]
    N = 500
    got = P.nt_sweep(ctx, h, rates, 0, N, TAU)
    want = orc.sweep(c, rates, 0, N, TAU)
    np.testing.assert_array_equal(got, want)
    ps, probes = P.nt_tolerable_rate(ctx, h, 0.66, 0.01, 1e-4, 1e-1, 0, N, TAU)
    rc, ps_o, probes_o = orc.tolerable_rate(c, 0.66, 0.01, 1e-4, 1e-1, 0, N, TAU)
    assert rc == 0 and ps == ps_o and probes == probes_o
    assert ps < 1.0 / c.G          # tolerable rate below 1/G (Sec. IV-D)
    with pytest.raises(P.NtError) as ei:
        P.nt_tolerable_rate(ctx, h, 0.66, 0.01, 0.05, 0.1, 0, 200, TAU)
    assert ei.value.status == P.NT_ERR_NOT_BRACKETED
    P.nt_circuit_free(h)


@pytest.mark.parametrize("name,maker,N", [
    ("8 qubits", lambda: W.config0(), 1000),
    ("16 qubits, 20 layers", lambda: W.config1(n=16, layers=20), 2000),
])
def test_tolerable_rate_auto(P, ctx, orc, name, maker, N):
    """The two-stage search without a caller's bracket: its answer meets the
    criterion on all N trajectories (checked with the oracle's sweep at that
    rate where the oracle finishes quickly, else with an independent library
    run), with and without the exact short-cuts, and both agree."""
    c = maker()
    h = _load(P, c)
    P.nt_set_precision(ctx, P.NT_C128 if c.n <= 8 else P.NT_C64)
    answers = []
    for sc in (0, P.NT_SHORTCUT_ZERO_FIRED | P.NT_SHORTCUT_CHECKPOINT | P.NT_SHORTCUT_REUSE):
        P.nt_set_shortcuts(ctx, sc)
        _say(f"auto search, {name}, short-cuts {sc}")
        p, kc, kf, br = P.nt_tolerable_rate_auto(ctx, h, 0.66, 0.01, 0, N, TAU)
        assert kc >= 2 and kf >= 1 and br[0] <= p <= br[1]
        answers.append((p, kc, kf))
    P.nt_set_shortcuts(ctx, 0)
    # bit-identical short-cuts: the same probes, the same answer
    assert answers[0] == answers[1]
    p = answers[0][0]
    if c.n <= 8:
        Pm = float(orc.sweep(c, [p], 0, N, TAU)[0])
    else:
        Pm = float(P.nt_sweep(ctx, h, [p], 0, N, TAU)[0])
    assert abs(Pm - 0.66) <= 0.01 + 1e-12
    assert p < 1.0 / c.G          # below 1/G (Sec. IV-D)
    P.nt_circuit_free(h)


def test_tolerable_rate_auto_arguments(P, ctx):
    h = _load(P, W.config0())
    for bad in ((0.0, 0.01), (1.0, 0.01), (0.66, -1.0)):
        with pytest.raises(P.NtError) as ei:
            P.nt_tolerable_rate_auto(ctx, h, bad[0], bad[1], 0, 100, TAU)
        assert ei.value.status == P.NT_ERR_INVALID_ARG
    with pytest.raises(P.NtError):
        P.nt_tolerable_rate_auto(ctx, h, 0.66, 0.01, 0, 0, TAU)
    P.nt_circuit_free(h)


# ---------------------------------------------------------------------------
# The 24-qubit workload at full size: reference state vs the oracle, and a
# few trajectories' fidelities, in the precision and launch shape the
# benchmark times.

def test_config1_full_size_sampled(P, ctx, orc):
    c = W.config1()
    h = _load(P, c)
    ref_o = orc.final_state_pattern(c, [], [])
    rng = np.random.default_rng(0)
    idx = rng.choice(1 << c.n, 4096, replace=False)
    for pr, tol in ((P.NT_C64, 1e-5), (P.NT_C128, 1e-12)):
        P.nt_set_precision(ctx, pr)
        ref = P.nt_reference_state(ctx, h, pr)
        d = _l2(ref, ref_o)
        _say("config1 reference L2", pr, d)
        assert d <= tol
        assert np.abs(ref[idx] - ref_o[idx]).max() <= tol
    # trajectories with errors at the highest rate
    p = 1e-2
    P.nt_set_precision(ctx, P.NT_C64)
    P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
    g = P.nt_final_state(ctx, h, 0, 0, P.NT_C64)
    o = orc.final_state(c, p / 3, p / 3, p / 3, 0, 0)
    _say("config1 t=0 p=1e-2 L2", _l2(g, o))
    assert _l2(g, o) <= 1e-5
    f = np.zeros(2)
    P.nt_run(ctx, h, 0, 0, 2, TAU, f)
    assert abs(f[0] - orc.fidelity(ref_o, o, c.n)) <= 2e-5
    P.nt_circuit_free(h)


# ---------------------------------------------------------------------------
# Argument errors on the GPU side.

def test_gpu_error_paths(P, ctx):
    c = W.config0()
    h = _load(P, c)
    with pytest.raises(P.NtError) as ei:
        P.nt_set_error_model(ctx, 0.5, 0.5, 0.5)
    assert ei.value.status == P.NT_ERR_INVALID_ARG
    with pytest.raises(P.NtError):
        P.nt_set_precision(ctx, 7)
    P.nt_set_error_model(ctx, 0.3, 0.3, 0.3)
    offs, s, pa = P.nt_sample_sites(ctx, h, 0, 0, 10, cap=1)   # retried with the needed size
    assert int(offs[-1]) == s.size
    P.nt_circuit_free(h)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_degenerate_circuits(P, ctx, orc, prec):
    """Degenerate inputs: a circuit without gates (no sites, every
    trajectory is |0..0>, the tolerable rate does not exist), one-qubit
    circuits under no errors, some errors and every site fired, and a single
    trajectory, against the oracle."""
    pr = P.NT_C64 if prec == "c64" else P.NT_C128
    tol_f = 2e-5 if prec == "c64" else 1e-12
    tol_a = 1e-5 if prec == "c64" else 1e-12
    P.nt_set_precision(ctx, pr)
    # no gates
    h = _load(P, W.Circuit(3, []))
    P.nt_set_error_model(ctx, 0.1, 0.1, 0.1)
    f = np.zeros(5)
    cnt, pv = P.nt_run(ctx, h, 0, 0, 5, TAU, f)
    assert cnt == 5 and pv == 1.0
    np.testing.assert_array_equal(f, np.ones(5))
    psi = P.nt_final_state(ctx, h, 0, 0, pr)
    assert psi[0] == 1 and np.count_nonzero(psi) == 1
    with pytest.raises(P.NtError) as ei:
        P.nt_tolerable_rate(ctx, h, 0.66, 0.01, 1e-4, 1e-1, 0, 20, TAU)
    assert ei.value.status == P.NT_ERR_NOT_BRACKETED
    P.nt_circuit_free(h)
    # one qubit, every one-qubit kind
    rng = np.random.default_rng(8)
    gates = []
    for name in ("H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "U", "H", "RX"):
        npar = W.GATE_NPARAM[name]
        gates.append(W.Gate(name, (0,), tuple(float(x) for x in rng.uniform(0, 2 * np.pi, npar))))
    c = W.Circuit(1, gates)
    h = _load(P, c, cid=5)
    for model in ((0.0, 0.0, 0.0), (0.1, 0.05, 0.15), (1 / 3, 1 / 3, 1 / 3)):
        _say(f"one qubit, {prec}, model {model}")
        P.nt_set_error_model(ctx, *model)
        N = 40
        f = np.zeros(N)
        cnt, _ = P.nt_run(ctx, h, 2, 0, N, TAU, f)
        f_o, c_o = orc.run(c, *model, 2, 0, N, TAU, cid=5)
        assert float(np.abs(f - f_o).max()) <= tol_f
        margin = np.abs(f_o - TAU) < tol_f
        assert cnt == c_o or margin.any()
        for t in (0, 1, 7):
            psi = P.nt_final_state(ctx, h, 2, t, pr).astype(np.complex128)
            assert _l2(psi, orc.final_state(c, *model, 2, t, cid=5)) <= tol_a
        # a single trajectory
        f1 = np.zeros(1)
        P.nt_run(ctx, h, 2, 7, 1, TAU, f1)
        assert abs(f1[0] - f_o[7]) <= tol_f
    P.nt_circuit_free(h)


# ---------------------------------------------------------------------------
# Exact short-cuts (zero-fired trajectories, error-free checkpoints) give
# bit-identical results to the plain run.

@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_shortcuts_bit_identical(P, ctx, prec):
    pr = P.NT_C64 if prec == "c64" else P.NT_C128
    for c in (_all_gates_circuit(16, 3, 21), W.config0()):
        h = _load(P, c)
        P.nt_set_precision(ctx, pr)
        for p in (1e-3, 2e-2):
            P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
            N = 96
            base = np.zeros(N)
            P.nt_set_shortcuts(ctx, 0)
            c0, _ = P.nt_run(ctx, h, 4, 7, N, TAU, base)
            for flags in (1, 2, 3):
                P.nt_set_shortcuts(ctx, flags)
                f = np.zeros(N)
                c1, _ = P.nt_run(ctx, h, 4, 7, N, TAU, f)
                np.testing.assert_array_equal(f.view(np.uint64), base.view(np.uint64))
                assert c1 == c0
        P.nt_set_shortcuts(ctx, 0)
        P.nt_circuit_free(h)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_reuse_bit_identical(P, ctx, prec):
    """NT_SHORTCUT_REUSE: values reused across rates (repeats, nearby rates,
    a changed seed, circuit id and criterion in between) equal those of
    runs without it, bit for bit; so does a tolerable-rate search."""
    pr = P.NT_C64 if prec == "c64" else P.NT_C128
    c = _all_gates_circuit(16, 3, 22)
    h = _load(P, c)
    P.nt_set_precision(ctx, pr)
    base_flags = P.NT_SHORTCUT_ZERO_FIRED | P.NT_SHORTCUT_CHECKPOINT | P.NT_SHORTCUT_LAST_ERROR
    N = 96
    steps = [(4, 2e-3), (4, 1e-3), (4, 2e-3), (4, 1.05e-3), (5, 1.05e-3), (4, 5e-3), (4, 1e-3)]

    def runs(flags):
        P.nt_set_shortcuts(ctx, flags)
        out = []
        for k, (seed, p) in enumerate(steps):
            P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
            if k == 3:
                P.nt_circuit_set_id(h, 2)      # new errors for the same (seed, trajectory)
            f = np.zeros(N)
            cnt, _ = P.nt_run(ctx, h, seed, 7, N, TAU, f)
            out.append((cnt, f))
        P.nt_circuit_set_id(h, 0)
        return out

    plain = runs(base_flags)
    reused = runs(base_flags | P.NT_SHORTCUT_REUSE)
    for (c0, f0), (c1, f1) in zip(plain, reused):
        np.testing.assert_array_equal(f1.view(np.uint64), f0.view(np.uint64))
        assert c1 == c0
    P.nt_set_shortcuts(ctx, base_flags)
    s0 = P.nt_tolerable_rate(ctx, h, 0.66, 0.01, 1e-4, 0.2, 3, 256, TAU)
    P.nt_set_shortcuts(ctx, base_flags | P.NT_SHORTCUT_REUSE)
    s1 = P.nt_tolerable_rate(ctx, h, 0.66, 0.01, 1e-4, 0.2, 3, 256, TAU)
    assert s1 == s0
    P.nt_set_shortcuts(ctx, 0)
    P.nt_circuit_free(h)


# ---------------------------------------------------------------------------
# Exhaustive single-error branch (Sec. IV-B.1, Eq. 3), Eq. 4, Eq. 5 and the
# method switch of Fig. 2, against the oracle.

@pytest.mark.parametrize("n,layers", [(6, 3), (15, 2)])
def test_exhaustive_vs_oracle(P, ctx, orc, n, layers):
    c = W.random_layers(n, layers, np.random.default_rng(50 + n))
    h = _load(P, c)
    P.nt_set_precision(ctx, P.NT_C128)
    fid, pe, pr = P.nt_exhaustive(ctx, h, TAU)
    f_o = orc.exhaustive(c)
    assert np.abs(fid - f_o).max() <= 1e-12
    margin = np.abs(f_o - TAU) < 1e-12
    want = np.where(margin, fid >= TAU, f_o >= TAU).mean(0)
    np.testing.assert_array_equal(pe, want)
    assert pr == 1.0
    p = 1e-3
    E = [c.S * p / 3] * 3
    assert abs(P.nt_eq4(pe, pr, E) - orc.eq4(pe, pr, E)) < 1e-15
    if pe.mean() != pr:
        assert abs(P.nt_eq5(0.66, pe, pr, c.S) - orc.eq5(0.66, pe, pr, c.S)) < 1e-15
    # method switch: E(N) = S p
    P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
    Pm, method = P.nt_success_probability(ctx, h, 0, 200, TAU)
    if c.S * p <= 1:
        assert method == 0 and abs(Pm - orc.eq4(pe, pr, E)) < 1e-15
    big = 3.0 / c.S
    P.nt_set_error_model(ctx, big / 3, big / 3, big / 3)
    Pm, method = P.nt_success_probability(ctx, h, 0, 200, TAU)
    cnt, _ = P.nt_run(ctx, h, 0, 0, 200, TAU)
    assert method == 1 and Pm == cnt / 200
    P.nt_circuit_free(h)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_last_error_shortcut(P, ctx, prec):
    """Scoring right after the last error (the unitary suffix keeps the
    overlap) agrees with the full run to rounding."""
    pr = P.NT_C64 if prec == "c64" else P.NT_C128
    ftol = 2e-5 if prec == "c64" else 1e-12
    c = _all_gates_circuit(16, 4, 33)
    h = _load(P, c)
    P.nt_set_precision(ctx, pr)
    for p in (2e-3, 3e-2):
        P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
        N = 128
        base = np.zeros(N)
        P.nt_set_shortcuts(ctx, 0)
        c0, _ = P.nt_run(ctx, h, 9, 0, N, TAU, base)
        f = np.zeros(N)
        P.nt_set_shortcuts(ctx, P.NT_SHORTCUT_ZERO_FIRED | P.NT_SHORTCUT_CHECKPOINT | P.NT_SHORTCUT_LAST_ERROR)
        c1, _ = P.nt_run(ctx, h, 9, 0, N, TAU, f)
        P.nt_set_shortcuts(ctx, 0)
        assert np.abs(f - base).max() <= ftol
        margin = np.abs(base - TAU) < ftol
        assert int(((f >= TAU) != (base >= TAU))[~margin].sum()) == 0
    P.nt_circuit_free(h)


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_shortcuts_single_pass_plans(P, ctx, prec):
    """Short-cuts on circuits whose plan is one pass (n <= tile width): the
    last-error short-cut reduces to scoring at the only pass."""
    pr = P.NT_C64 if prec == "c64" else P.NT_C128
    ftol = 2e-5 if prec == "c64" else 1e-12
    P.nt_set_precision(ctx, pr)
    for c in (W.config0(), W.config3_circuit(100003), _all_gates_circuit(11, 3, 5)):
        h = _load(P, c)
        npass, _, _ = P.nt_plan_info(h, pr)
        assert npass == 1
        for p in (1e-3, 3e-2):
            P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
            N = 64
            base = np.zeros(N)
            P.nt_set_shortcuts(ctx, 0)
            c0, _ = P.nt_run(ctx, h, 2, 0, N, TAU, base)
            for flags in (3, 7):
                _say(f"single-pass short-cuts: n={c.n} p={p} flags={flags} prec={prec}")
                P.nt_set_shortcuts(ctx, flags)
                f = np.zeros(N)
                c1, _ = P.nt_run(ctx, h, 2, 0, N, TAU, f)
                if flags == 3:
                    np.testing.assert_array_equal(f.view(np.uint64), base.view(np.uint64))
                else:
                    assert np.abs(f - base).max() <= ftol
        P.nt_set_shortcuts(ctx, 0)
        P.nt_circuit_free(h)


def test_tile_widths_and_autotune(P, ctx, orc):
    """Every allowed tile width gives the oracle's fidelities (to the
    precision's bar); the autotuner picks one of the candidates it timed and
    runs are reproducible under the chosen width."""
    c = W.random_layers(17, 8, np.random.default_rng(77))
    h = _load(P, c)
    P.nt_set_precision(ctx, P.NT_C64)
    p = 0.02
    P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
    N = 8
    want, _ = orc.run(c, p / 3, p / 3, p / 3, 6, 0, N, TAU)
    for L in (10, 11, 12, 13):
        _say(f"tile width {L}")
        P.nt_circuit_set_tile(h, P.NT_C64, L)
        assert P.nt_plan_info(h, P.NT_C64)[2] == L
        f = np.zeros(N)
        P.nt_run(ctx, h, 6, 0, N, TAU, f)
        assert np.abs(f - want).max() <= 2e-5
    P.nt_circuit_set_tile(h, P.NT_C64, 0)
    _say("autotune")
    L, ms = P.nt_autotune(ctx, h, 1, 64)
    assert L in (11, 12, 13) and np.all(ms > 0)
    assert P.nt_plan_info(h, P.NT_C64)[2] == L
    a = np.zeros(N)
    b = np.zeros(N)
    P.nt_run(ctx, h, 6, 0, N, TAU, a)
    P.nt_run(ctx, h, 6, 0, N, TAU, b)
    np.testing.assert_array_equal(a.view(np.uint64), b.view(np.uint64))
    assert np.abs(a - want).max() <= 2e-5
    P.nt_circuit_free(h)
