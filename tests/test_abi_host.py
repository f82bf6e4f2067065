"""Host-side checks of libnisqtol: exported symbols, argument validation,
the text format, and the gate-pass planner.  No GPU is needed: circuits and
plans are host objects, and no compute call is made."""
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_2301_07264_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_2301_07264_amd import build
        build.build()
    P.lib()
    return P


def test_exports_every_declared_symbol(P):
    hdr = open(os.path.join(ROOT, "include", "nisqtol.h")).read()
    declared = set(re.findall(r"\b(nt_[a-z0-9_]+)\s*\(", hdr))
    assert declared, "no declarations found"
    L = P.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(P.EXPORTED)


def test_version_and_last_error(P):
    assert "nisqtol" in P.nt_version()
    with pytest.raises(P.NtError):
        P.nt_circuit_load(None, W.Circuit(0, []))
    assert "n_qubits" in P.nt_last_error()


def test_create_without_gpu_fails_cleanly(P):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(P.NtError) as ei:
        P.nt_create(0)
    assert ei.value.status == P.NT_ERR_DEVICE


def _expect(P, status, fn, *a):
    with pytest.raises(P.NtError) as ei:
        fn(*a)
    assert ei.value.status == status, str(ei.value)


def test_circuit_validation(P):
    bad = [
        W.Circuit(3, [W.Gate("H", (3,))]),                 # qubit out of range
        W.Circuit(3, [W.Gate("CNOT", (1, 1))]),            # duplicate qubits
        W.Circuit(33, [W.Gate("H", (0,))]),                # too many qubits
        W.Circuit(2, [W.Gate("RX", (0,), (float("nan"),))]),
        W.Circuit(2, [W.Gate("U1Q", (0,), (), np.array([[1, 1], [0, 1]]))]),  # not unitary
    ]
    for c in bad:
        _expect(P, P.NT_ERR_INVALID_ARG, P.nt_circuit_load, None, c)


def test_unknown_kind_and_arity(P):
    import ctypes as C
    g = (P.nt_gate * 1)()
    g[0].kind = 99
    g[0].nq = 1
    h = C.c_void_p()
    assert P.lib().nt_circuit_load(None, 2, C.cast(g, C.c_void_p), 1, C.byref(h)) == P.NT_ERR_INVALID_ARG
    g[0].kind = P.GATE_KIND["CNOT"]
    g[0].nq = 1
    assert P.lib().nt_circuit_load(None, 2, C.cast(g, C.c_void_p), 1, C.byref(h)) == P.NT_ERR_INVALID_ARG
    assert P.lib().nt_circuit_load(None, 2, None, 1, C.byref(h)) == P.NT_ERR_INVALID_ARG


def test_gate_count_limit(P):
    # event words carry the op index in 20 bits; the loader caps G at 2^19
    # (a plan may add up to one no-op per gate) before it reads any gate
    import ctypes as C
    g = (P.nt_gate * 1)()
    g[0].kind = P.GATE_KIND["H"]
    g[0].nq = 1
    h = C.c_void_p()
    rc = P.lib().nt_circuit_load(None, 2, C.cast(g, C.c_void_p), (1 << 19) + 1, C.byref(h))
    assert rc == P.NT_ERR_UNSUPPORTED
    assert "2^19" in P.nt_last_error()


def test_null_handles(P):
    import ctypes as C
    L = P.lib()
    assert L.nt_set_error_model(None, 0.1, 0, 0) == P.NT_ERR_INVALID_ARG
    assert L.nt_set_precision(None, 1) == P.NT_ERR_INVALID_ARG
    assert L.nt_run(None, None, 0, 0, 1, 0.9, None, None, None) == P.NT_ERR_INVALID_ARG
    assert L.nt_run_batch(None, None, 1, 0, 0, 1, 0.9, None, None, None) == P.NT_ERR_INVALID_ARG
    assert L.nt_set_criterion(None, 0, 0) == P.NT_ERR_INVALID_ARG
    assert L.nt_circuit_info(None, None, None, None) == P.NT_ERR_INVALID_ARG
    L.nt_destroy(None)
    L.nt_circuit_free(None)


def test_info_and_text_roundtrip(P, tmp_path):
    for c in (W.config0(), W.config1(n=10, layers=3), W.config4(n=12, rounds=2)):
        h = P.nt_circuit_load(None, c)
        assert P.nt_circuit_info(h) == (c.n, c.G, c.S)
        path = str(tmp_path / "c.txt")
        W.write_text(c, path)
        h2 = P.nt_circuit_load_text(None, path)
        assert P.nt_circuit_info(h2) == (c.n, c.G, c.S)
        assert W.from_text(W.to_text(c)).gates == c.gates
        P.nt_circuit_free(h)
        P.nt_circuit_free(h2)
    with open(tmp_path / "bad.txt", "w") as f:
        f.write("qubits 2\nFOO 0\n")
    _expect(P, P.NT_ERR_INVALID_ARG, P.nt_circuit_load_text, None, str(tmp_path / "bad.txt"))
    _expect(P, P.NT_ERR_INVALID_ARG, P.nt_circuit_load_text, None, str(tmp_path / "missing.txt"))


# ---------------------------------------------------------------------------
# Planner invariants (host logic).

DIAG = {"Z", "S", "T", "RZ", "CZ", "CP", "RZZ"}


def _needs(g):
    if g.name in DIAG:
        return set()
    if g.name == "CNOT":
        return {g.qubits[1]}
    return set(g.qubits)


def _check_plan(P, c, prec):
    h = P.nt_circuit_load(None, c)
    npass, nseg, L = P.nt_plan_info(h, prec)
    ex = P.nt_plan_export(h, prec)
    og = ex["op_gate"]
    assert sorted(og.tolist()) == list(range(c.G))            # every gate once
    # per-qubit order preserved
    last = {}
    for o, g in enumerate(og.tolist()):
        for q in c.gates[g].qubits:
            assert last.get(q, -1) < g
            last[q] = g
    cfix = min(c.n, 4 if prec == P.NT_C64 else 3)
    for pm in ex["pass_local_mask"].tolist():
        assert bin(pm).count("1") == L
        assert pm & ((1 << cfix) - 1) == (1 << cfix) - 1       # coalescing qubits local
    for o, g in enumerate(og.tolist()):
        need = _needs(c.gates[g])
        pm = int(ex["pass_local_mask"][ex["op_pass"][o]])
        sm = int(ex["segment_reg_mask"][ex["op_segment"][o]])
        dense2 = c.gates[g].name == "U2Q"                 # applied in LDS, not registers
        for q in need:
            assert (pm >> q) & 1
            assert dense2 or (sm >> q) & 1
    assert np.all(np.diff(ex["op_pass"]) >= 0) and np.all(np.diff(ex["op_segment"]) >= 0)
    P.nt_circuit_free(h)
    return npass, og


@pytest.mark.parametrize("which", ["c0", "c1small", "c4small", "c1", "c4"])
def test_plan_invariants(P, which):
    c = {"c0": W.config0(), "c1small": W.config1(n=15, layers=4), "c4small": W.config4(n=16, rounds=2),
         "c1": W.config1(), "c4": W.config4()}[which]
    for prec in (P.NT_C64, P.NT_C128):
        npass, _ = _check_plan(P, c, prec)
        if c.n <= 12:
            assert npass == 1


@pytest.mark.parametrize("width", [1, 2, 3, 4])
def test_plan_invariants_every_fusion_width(P, width):
    """Every fusion width (blocks, diagonal runs, one-qubit layers, none)
    keeps each gate once, the order of the gates on every qubit, and the
    locality and register needs of every gate."""
    for c in (W.config1(n=15, layers=4), W.config4(n=16, rounds=2), W.config1(n=13, layers=2)):
        for prec in (P.NT_C64, P.NT_C128):
            h = P.nt_circuit_load(None, c)
            P.nt_circuit_set_fusion(h, prec, width)
            n_ops, n_fused = P.nt_plan_ops(h, prec)
            if width == 1:
                assert n_fused == 0 and n_ops == c.G
            npass, nseg, L = P.nt_plan_info(h, prec)
            ex = P.nt_plan_export(h, prec)
            og = ex["op_gate"].tolist()
            assert sorted(og) == list(range(c.G))
            last = {}
            for o, g in enumerate(og):
                for q in c.gates[g].qubits:
                    assert last.get(q, -1) < g
                    last[q] = g
                pm = int(ex["pass_local_mask"][ex["op_pass"][o]])
                sm = int(ex["segment_reg_mask"][ex["op_segment"][o]])
                for q in _needs(c.gates[g]):
                    assert (pm >> q) & 1 and (sm >> q) & 1
            P.nt_circuit_free(h)


def test_plan_order_is_same_unitary(P, orc):
    """Gates applied in plan order give the circuit's own final state."""
    c = W.config1(n=14, layers=3) + W.Circuit(14, [W.Gate("SWAP", (0, 13)), W.Gate("U2Q", (2, 9), (),
                                                                                       np.eye(4)[[1, 0, 3, 2]])])
    for prec in (P.NT_C64, P.NT_C128):
        _, og = _check_plan(P, c, prec)
        reordered = W.Circuit(c.n, [c.gates[g] for g in og.tolist()])
        a = orc.final_state_pattern(c, [], [])
        b = orc.final_state_pattern(reordered, [], [])
        assert np.abs(a - b).max() < 1e-12


def test_workload_sizes():
    assert (W.config0().G, W.config0().S) == (240, 320)
    assert (W.config1().G, W.config1().S) == (2136, 3047)
    assert (W.config4().G, W.config4().S) == (330, 510)
    assert len(W.rates_config1()) == 13 and abs(W.rates_config1()[-1] - 1e-2) < 1e-15


def test_tile_override_host(P):
    c = W.config1(n=20, layers=4)
    h = P.nt_circuit_load(None, c)
    _, _, L0 = P.nt_plan_info(h, P.NT_C64)
    assert L0 in (12, 13)
    for L in (10, 11, 12, 13):
        P.nt_circuit_set_tile(h, P.NT_C64, L)
        npass, nseg, Lp = P.nt_plan_info(h, P.NT_C64)
        assert Lp == L and npass >= 1
    with pytest.raises(P.NtError):
        P.nt_circuit_set_tile(h, P.NT_C64, 14)
    with pytest.raises(P.NtError):
        P.nt_circuit_set_tile(h, P.NT_C128, 13)
    with pytest.raises(P.NtError):
        P.nt_circuit_set_tile(h, P.NT_C64, 9)
    P.nt_circuit_set_tile(h, P.NT_C64, 0)
    assert P.nt_plan_info(h, P.NT_C64)[2] == L0
    P.nt_circuit_free(h)
    small = P.nt_circuit_load(None, W.config0())          # n = 8: the only width is 8
    P.nt_circuit_set_tile(small, P.NT_C64, 8)
    assert P.nt_plan_info(small, P.NT_C64)[2] == 8
    P.nt_circuit_free(small)
