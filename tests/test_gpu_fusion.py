"""GPU parity of fused two-qubit blocks against the CPU oracle.

A fused block applies a two-qubit gate and the one-qubit gates around it as
one dense 4x4; an error inside it (a later gate of the block acts on its
qubit) must still act right after its own gate (Sec. IV-B).  Exhaustive
single-error simulation puts one error at every site with every Pauli, so it
reaches every position inside every block; the Monte Carlo runs at high rates
and with every site fired put several errors into one block.  Bars as in the
other parity tests: fidelities within 1e-12 (complex128) / 2e-5 (complex64),
states within L2 1e-12 / 1e-5.
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


def _l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.complex128) - np.asarray(b, np.complex128)))


def _mixed_circuit(n, layers, seed):
    # random layers with every two-qubit kind and runs of one-qubit gates
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(layers):
        for q in range(n):
            for _ in range(1 + int(rng.integers(2))):
                nm = ["U", "H", "RX", "T"][int(rng.integers(4))]
                if nm == "U":
                    gates.append(W.Gate(nm, (q,), tuple(float(x) for x in rng.uniform(0, 2 * math.pi, 3))))
                elif nm == "RX":
                    gates.append(W.Gate(nm, (q,), (float(rng.uniform(0, 2 * math.pi)),)))
                else:
                    gates.append(W.Gate(nm, (q,)))
        perm = rng.permutation(n)
        for i in range(n // 2):
            a, b = int(perm[2 * i]), int(perm[2 * i + 1])
            nm = ["CNOT", "CNOT", "CZ", "CP", "RZZ", "SWAP"][int(rng.integers(6))]
            if nm in ("CP", "RZZ"):
                gates.append(W.Gate(nm, (a, b), (float(rng.uniform(0, 2 * math.pi)),)))
            else:
                gates.append(W.Gate(nm, (a, b)))
    return W.Circuit(n, gates, f"mixed{n}")


def _diag_circuit(n, layers, seed):
    # one-qubit layers, then long stretches of diagonal gates (one- and
    # two-qubit, phases of every kind) on random qubits: runs whose qubits sit
    # in the registers, in the tile, and outside it, with one or several
    # register qubits per run
    rng = np.random.default_rng(seed)
    gates = []
    for _ in range(layers):
        for q in range(n):
            if rng.integers(2):
                gates.append(W.Gate("H", (q,)))
            else:
                gates.append(W.Gate("RX", (q,), (float(rng.uniform(0, 2 * math.pi)),)))
        for _ in range(3 * n):
            nm = ["RZ", "T", "S", "Z", "CP", "CZ", "RZZ"][int(rng.integers(7))]
            if nm in ("RZ", "T", "S", "Z"):
                q = int(rng.integers(n))
                par = (float(rng.uniform(-4 * math.pi, 4 * math.pi)),) if nm == "RZ" else ()
                gates.append(W.Gate(nm, (q,), par))
            else:
                a, b = (int(x) for x in rng.choice(n, 2, replace=False))
                par = (float(rng.uniform(-4 * math.pi, 4 * math.pi)),) if nm in ("CP", "RZZ") else ()
                gates.append(W.Gate(nm, (a, b), par))
    return W.Circuit(n, gates, f"diag{n}")


CIRCUITS = [
    ("layers8", lambda: W.random_layers(8, 6, np.random.default_rng(81))),
    ("layers15", lambda: W.random_layers(15, 3, np.random.default_rng(82))),   # several passes
    ("mixed9", lambda: _mixed_circuit(9, 3, 83)),
    # the 24-qubit workload's structure at 12 qubits: QFT runs of controlled
    # phases (diagonal runs) and random layers (blocks)
    ("ghzqft12", lambda: W.config1(n=12, layers=3)),
    # rounds of RZZ on a 3-regular graph and RX (diagonal runs)
    ("qaoa12", lambda: W.config4(n=12, rounds=2)),
    # long diagonal runs (up to 31 gates, errors at every stage inside them)
    ("diag12", lambda: _diag_circuit(12, 2, 92)),
    # Haar-random two-qubit gates, each a block of its own on two register
    # qubits (errors before a block pick its frame variant)
    ("qv10", lambda: W.quantum_volume(10, 6, np.random.default_rng(93))),
]


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("name,make", CIRCUITS)
def test_blocks_every_single_error(P, ctx, orc, prec, name, make):
    c = make()
    h = P.nt_circuit_load(None, c)
    pr = P.NT_C128 if prec == "c128" else P.NT_C64
    n_ops, n_blocks = P.nt_plan_ops(h, pr)
    _say(f"{name} G={c.G} S={c.S} prec={prec}: {n_ops} ops, {n_blocks} fused blocks")
    assert n_blocks > 0
    P.nt_set_precision(ctx, pr)
    fid, pe, _ = P.nt_exhaustive(ctx, h, TAU)
    f_o = orc.exhaustive(c)
    tol = 1e-12 if prec == "c128" else 2e-5
    err = float(np.abs(fid - f_o).max())
    _say(f"  exhaustive: 3S = {3 * c.S} states, max |dF| = {err:.2e}")
    assert err <= tol
    P.nt_circuit_free(h)


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("name,make", CIRCUITS)
def test_blocks_many_errors(P, ctx, orc, prec, name, make):
    c = make()
    pr = P.NT_C128 if prec == "c128" else P.NT_C64
    tol = 1e-12 if prec == "c128" else 1e-5
    ftol = 1e-12 if prec == "c128" else 2e-5
    h = P.nt_circuit_load(None, c)
    P.nt_circuit_set_id(h, 5)
    P.nt_set_precision(ctx, pr)
    # every site fired (uniform types), a high rate, and X-only errors
    for model in [(1 / 3, 1 / 3, 1 / 3), (0.1, 0.1, 0.1), (0.25, 0.0, 0.0)]:
        P.nt_set_error_model(ctx, *model)
        for t in range(3):
            g = P.nt_final_state(ctx, h, 13, t, pr)
            o = orc.final_state(c, *model, 13, t, cid=5)
            assert _l2(g, o) <= tol, (model, t, _l2(g, o))
        N = 48
        fid = np.zeros(N)
        P.nt_run(ctx, h, 13, 0, N, TAU, fid)
        f_o, _ = orc.run(c, *model, 13, 0, N, TAU, cid=5)
        assert np.abs(fid - f_o).max() <= ftol, (model, np.abs(fid - f_o).max())
    P.nt_circuit_free(h)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_fusion_modes_agree_with_oracle(P, ctx, orc, prec):
    # the same trajectories under every fusion width (blocks and runs,
    # blocks, runs, none) against the oracle, on a circuit with both
    c = W.config1(n=14, layers=6)
    pr = P.NT_C128 if prec == "c128" else P.NT_C64
    ftol = 1e-12 if prec == "c128" else 2e-5
    P.nt_set_precision(ctx, pr)
    p = 0.02
    P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
    want, _ = orc.run(c, p / 3, p / 3, p / 3, 3, 0, 64, TAU)
    for width in (2, 3, 4, 1):
        h = P.nt_circuit_load(None, c)
        P.nt_circuit_set_fusion(h, pr, width)
        n_ops, n_fused = P.nt_plan_ops(h, pr)
        fid = np.zeros(64)
        P.nt_run(ctx, h, 3, 0, 64, TAU, fid)
        err = float(np.abs(fid - want).max())
        _say(f"fusion width {width}: {n_ops} ops, {n_fused} fused, max |dF| = {err:.2e}")
        assert err <= ftol
        assert (n_fused == 0) == (width == 1)
        P.nt_circuit_free(h)


def test_plan_autotuner(P, ctx, orc):
    """The plan autotuner times every (tile width, fusion width) pair, keeps
    one it timed, and the chosen plan gives the oracle's values and
    reproducible runs."""
    c = W.config1(n=16, layers=8)
    h = P.nt_circuit_load(None, c)
    P.nt_set_precision(ctx, P.NT_C64)
    p = 0.01
    P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
    L, fw, ms = P.nt_autotune_plan(ctx, h, 1, 32)
    _say(f"autotune: tile {L}, fusion {fw}, ms {np.round(ms, 2)}")
    assert fw in (1, 2, 3, 4) and L in (11, 12, 13) and np.all(ms > 0)
    assert P.nt_plan_info(h, P.NT_C64)[2] == L
    N = 16
    want, _ = orc.run(c, p / 3, p / 3, p / 3, 6, 0, N, TAU)
    a = np.zeros(N)
    b = np.zeros(N)
    P.nt_run(ctx, h, 6, 0, N, TAU, a)
    P.nt_run(ctx, h, 6, 0, N, TAU, b)
    np.testing.assert_array_equal(a.view(np.uint64), b.view(np.uint64))
    assert np.abs(a - want).max() <= 2e-5
    P.nt_circuit_free(h)


DIAG_CIRCUITS = [
    ("ghzqft16", lambda: W.config1(n=16, layers=0)),
    ("diag17", lambda: _diag_circuit(17, 3, 91)),
    ("qaoa16", lambda: W.config4(n=16, rounds=2)),
]


@pytest.mark.parametrize("name,make", DIAG_CIRCUITS)
def test_diagonal_runs(P, ctx, orc, name, make):
    """Diagonal runs at complex64 over 2^12-amplitude tiles (several passes,
    qubits outside the tile): a run with no error inside it is one phase per
    amplitude from fixed-point angle sums, one with an error inside it is
    applied gate by gate.  Error-free states take the first form for every
    run; the error models put errors inside and outside runs."""
    c = make()
    pr = P.NT_C64
    P.nt_set_precision(ctx, pr)
    for width in (4, 2):
        h = P.nt_circuit_load(None, c)
        P.nt_circuit_set_id(h, 7)
        P.nt_circuit_set_tile(h, pr, 12)
        P.nt_circuit_set_fusion(h, pr, width)
        n_ops, n_fused = P.nt_plan_ops(h, pr)
        _say(f"{name} G={c.G} fusion {width}: {n_ops} ops, {n_fused} fused")
        assert n_fused > 0
        for model in [(0.0, 0.0, 0.0), (0.004, 0.004, 0.004), (0.1, 0.0, 0.0), (1 / 3, 1 / 3, 1 / 3)]:
            P.nt_set_error_model(ctx, *model)
            for t in range(3):
                g = P.nt_final_state(ctx, h, 21, t, pr)
                o = orc.final_state(c, *model, 21, t, cid=7)
                err = _l2(g, o)
                assert err <= 1e-5, (model, t, err)
        p = 0.01
        P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
        N = 64
        fid = np.zeros(N)
        P.nt_run(ctx, h, 21, 0, N, TAU, fid)
        f_o, _ = orc.run(c, p / 3, p / 3, p / 3, 21, 0, N, TAU, cid=7)
        assert np.abs(fid - f_o).max() <= 2e-5
        P.nt_circuit_free(h)
