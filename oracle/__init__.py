"""CPU oracle for Monte Carlo Pauli-error state-vector simulation.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg.  The GPU library never imports, links or
calls anything here, and this package never imports the GPU library.

The arithmetic lives in ``nisq_oracle.c`` (plain FP64 C, OpenMP over
trajectories).  This module only marshals arguments.  Every function cites
the paper passage it follows in the C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nisq_oracle.c")
LIB = os.path.join(HERE, "libnisq_oracle.so")

# The oracle's own gate numbering (matches the enum in nisq_oracle.c).
KIND = {
    "H": 0, "X": 1, "Y": 2, "Z": 3, "S": 4, "T": 5, "RX": 6, "RY": 7, "RZ": 8,
    "U": 9, "U1Q": 10, "CNOT": 11, "CZ": 12, "CP": 13, "SWAP": 14, "RZZ": 15,
    "U2Q": 16,
}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-D_GNU_SOURCE", SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        i32, i64, u64, dbl = C.c_int, C.c_int64, C.c_uint64, C.c_double
        L.orc_gate_matrix.argtypes = [i32, P, P, P]
        L.orc_gate_matrix.restype = i32
        L.orc_philox4x64_10.argtypes = [P, P, P]
        L.orc_philox4x64_10.restype = None
        L.orc_thresholds.argtypes = [dbl, dbl, dbl, P, P]
        L.orc_thresholds.restype = None
        L.orc_sample_trajectory.argtypes = [u64, u64, u64, i64, dbl, dbl, dbl, P, P, i64]
        L.orc_sample_trajectory.restype = i64
        L.orc_apply_gate.argtypes = [i32, P, i32, i32, i32, P, P]
        L.orc_apply_gate.restype = i32
        L.orc_apply_pauli.argtypes = [i32, P, i32, i32]
        L.orc_apply_pauli.restype = None
        L.orc_fidelity.argtypes = [i32, P, P]
        L.orc_fidelity.restype = dbl
        circ = [i32, i64, P, P, P, P, P]
        L.orc_final_state_pattern.argtypes = circ + [u64, P, P, i64, P]
        L.orc_final_state_pattern.restype = i32
        L.orc_final_state.argtypes = circ + [dbl, dbl, dbl, u64, u64, u64, P]
        L.orc_final_state.restype = i32
        L.orc_run.argtypes = circ + [dbl, dbl, dbl, u64, u64, u64, u64, dbl, i32, P, P, P]
        L.orc_run.restype = i32
        L.orc_sweep.argtypes = circ + [P, i32, u64, u64, u64, dbl, i32, P]
        L.orc_sweep.restype = i32
        L.orc_tolerable_rate.argtypes = circ + [dbl, dbl, dbl, dbl, u64, u64, u64, dbl, i32, P, P]
        L.orc_tolerable_rate.restype = i32
        L.orc_exhaustive.argtypes = circ + [i32, P]
        L.orc_exhaustive.restype = i32
        L.orc_tolerable_rate_fig3.argtypes = circ + [dbl, dbl, u64, u64, u64, dbl, i32, P, P, P, P]
        L.orc_tolerable_rate_fig3.restype = i32
        L.orc_eq4.argtypes = [P, dbl, P]
        L.orc_eq4.restype = dbl
        L.orc_eq5.argtypes = [dbl, P, dbl, dbl]
        L.orc_eq5.restype = dbl
        L.orc_median_prob.argtypes = [i32, P]
        L.orc_median_prob.restype = dbl
        L.orc_run_criterion.argtypes = circ + [dbl, dbl, dbl, u64, u64, u64, u64, i32, u64, i32, P]
        L.orc_run_criterion.restype = i32
        L.orc_exhaustive_criterion.argtypes = circ + [i32, u64, i32, P, P]
        L.orc_exhaustive_criterion.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class OCircuit:
    """A circuit marshalled into the oracle's flat arrays."""

    def __init__(self, circuit):
        G = len(circuit.gates)
        self.n = circuit.n
        self.G = G
        self.kind = np.array([KIND[g.name] for g in circuit.gates], np.int32)
        self.q0 = np.array([g.qubits[0] for g in circuit.gates], np.int32)
        self.q1 = np.array([g.qubits[1] if len(g.qubits) > 1 else -1 for g in circuit.gates], np.int32)
        self.params = np.zeros((max(G, 1), 3), np.float64)
        self.umats = np.zeros((max(G, 1), 32), np.float64)
        for i, g in enumerate(circuit.gates):
            for j, v in enumerate(g.params):
                self.params[i, j] = v
            if g.matrix is not None:
                m = np.asarray(g.matrix, np.complex128).ravel()
                self.umats[i, 0:2 * m.size:2] = m.real
                self.umats[i, 1:2 * m.size:2] = m.imag
        self.S = int(sum(len(g.qubits) for g in circuit.gates))

    def args(self):
        return (self.n, self.G, _p(self.kind), _p(self.q0), _p(self.q1),
                _p(self.params), _p(self.umats))


def gate_matrix(name: str, params: Sequence[float] = (), matrix=None) -> np.ndarray:
    p = np.zeros(3, np.float64)
    p[:len(params)] = params
    um = np.zeros(32, np.float64)
    if matrix is not None:
        m = np.asarray(matrix, np.complex128).ravel()
        um[0:2 * m.size:2] = m.real
        um[1:2 * m.size:2] = m.imag
    out = np.zeros(32, np.float64)
    ar = lib().orc_gate_matrix(KIND[name], _p(p), _p(um), _p(out))
    dim = 2 if ar == 1 else 4
    c = out[0::2] + 1j * out[1::2]
    return c[:dim * dim].reshape(dim, dim)


def philox4x64_10(counter, key) -> np.ndarray:
    ctr = np.asarray(counter, np.uint64)
    k = np.asarray(key, np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_p(ctr), _p(k), _p(out))
    return out


def thresholds(px, py, pz):
    out = np.zeros(3, np.uint64)
    alw = np.zeros(3, np.int32)
    lib().orc_thresholds(px, py, pz, _p(out), _p(alw))
    return out, alw


def sample_trajectory(seed, cid, traj, S, px, py, pz):
    sites = np.zeros(max(S, 1), np.int32)
    paulis = np.zeros(max(S, 1), np.uint8)
    cnt = lib().orc_sample_trajectory(seed, cid, traj, S, px, py, pz, _p(sites), _p(paulis), S)
    return sites[:cnt].copy(), paulis[:cnt].copy()


def apply_gate(psi: np.ndarray, n: int, name: str, qubits, params=(), matrix=None) -> np.ndarray:
    st = np.ascontiguousarray(psi, np.complex128).copy()
    p = np.zeros(3, np.float64)
    p[:len(params)] = params
    um = np.zeros(32, np.float64)
    if matrix is not None:
        m = np.asarray(matrix, np.complex128).ravel()
        um[0:2 * m.size:2] = m.real
        um[1:2 * m.size:2] = m.imag
    q1 = qubits[1] if len(qubits) > 1 else -1
    rc = lib().orc_apply_gate(n, _p(st), KIND[name], qubits[0], q1, _p(p), _p(um))
    assert rc == 0
    return st


def apply_pauli(psi: np.ndarray, n: int, q: int, pauli: int) -> np.ndarray:
    st = np.ascontiguousarray(psi, np.complex128).copy()
    lib().orc_apply_pauli(n, _p(st), q, pauli)
    return st


def fidelity(ref: np.ndarray, psi: np.ndarray, n: int) -> float:
    a = np.ascontiguousarray(ref, np.complex128)
    b = np.ascontiguousarray(psi, np.complex128)
    return lib().orc_fidelity(n, _p(a), _p(b))


def final_state_pattern(circuit, sites, paulis, init_index: int = 0) -> np.ndarray:
    oc = OCircuit(circuit)
    s = np.ascontiguousarray(sites, np.int32)
    pa = np.ascontiguousarray(paulis, np.uint8)
    out = np.zeros(1 << circuit.n, np.complex128)
    rc = lib().orc_final_state_pattern(*oc.args(), init_index, _p(s), _p(pa), len(s), _p(out))
    assert rc == 0
    return out


def final_state(circuit, px, py, pz, seed, traj, cid: int = 0) -> np.ndarray:
    oc = OCircuit(circuit)
    out = np.zeros(1 << circuit.n, np.complex128)
    rc = lib().orc_final_state(*oc.args(), px, py, pz, seed, cid, traj, _p(out))
    assert rc == 0
    return out


def run(circuit, px, py, pz, seed, t0, N, tau, cid: int = 0, nthreads: int = 0,
        return_threads: bool = False):
    """Monte Carlo run: returns (fid[N], count[, threads])."""
    oc = OCircuit(circuit)
    fid = np.zeros(max(N, 1), np.float64)
    cnt = np.zeros(1, np.uint64)
    thr = np.zeros(1, np.int32)
    rc = lib().orc_run(*oc.args(), px, py, pz, seed, cid, t0, N, tau, nthreads,
                       _p(fid), _p(cnt), _p(thr))
    if rc:
        raise RuntimeError(f"orc_run failed: {rc}")
    if return_threads:
        return fid[:N], int(cnt[0]), int(thr[0])
    return fid[:N], int(cnt[0])


def sweep(circuit, rates, seed, N, tau, cid: int = 0, nthreads: int = 0) -> np.ndarray:
    oc = OCircuit(circuit)
    r = np.ascontiguousarray(rates, np.float64)
    out = np.zeros(len(r), np.float64)
    rc = lib().orc_sweep(*oc.args(), _p(r), len(r), seed, cid, N, tau, nthreads, _p(out))
    assert rc == 0
    return out


def tolerable_rate(circuit, P_target, tol, p_lo, p_hi, seed, N, tau, cid: int = 0,
                   nthreads: int = 0):
    """Returns (status, p_star, n_probes); status 1 = not bracketed."""
    oc = OCircuit(circuit)
    ps = np.zeros(1, np.float64)
    npb = np.zeros(1, np.int32)
    rc = lib().orc_tolerable_rate(*oc.args(), P_target, tol, p_lo, p_hi, seed, cid, N, tau,
                                  nthreads, _p(ps), _p(npb))
    return rc, float(ps[0]), int(npb[0])


def tolerable_rate_fig3(circuit, P_target, tol, seed, N, tau, cid: int = 0, nthreads: int = 0):
    """The paper's steps (exhaustive first, Eq. 5 or Monte Carlo at increasing
    rates).  Returns (status, p_star, method, n_probes, [P_X, P_Y, P_Z, P_R]);
    status 1 = not bracketed, method 0 = Eq. 5, 1 = Monte Carlo."""
    oc = OCircuit(circuit)
    ps = np.zeros(1, np.float64)
    meth = np.zeros(1, np.int32)
    npb = np.zeros(1, np.int32)
    p4 = np.zeros(4, np.float64)
    rc = lib().orc_tolerable_rate_fig3(*oc.args(), P_target, tol, seed, cid, N, tau, nthreads,
                                       _p(ps), _p(meth), _p(npb), _p(p4))
    return rc, float(ps[0]), int(meth[0]), int(npb[0]), p4


def exhaustive(circuit, nthreads: int = 0) -> np.ndarray:
    """Fidelity of every single-error state, shape [S, 3] (X, Y, Z)."""
    oc = OCircuit(circuit)
    out = np.zeros((max(oc.S, 1), 3), np.float64)
    rc = lib().orc_exhaustive(*oc.args(), nthreads, _p(out))
    assert rc == 0
    return out[:oc.S]


def exhaustive_criterion(circuit, crit: int, target: int = 0, nthreads: int = 0):
    """Criterion value of every single-error state, shape [S, 3] (X, Y, Z),
    and of the reference state."""
    oc = OCircuit(circuit)
    out = np.zeros((max(oc.S, 1), 3), np.float64)
    rv = C.c_double(0.0)
    rc = lib().orc_exhaustive_criterion(*oc.args(), crit, target, nthreads, _p(out), C.byref(rv))
    assert rc == 0
    return out[:oc.S], rv.value


def eq4(P_e, P_R, E_e) -> float:
    a = np.ascontiguousarray(P_e, np.float64)
    b = np.ascontiguousarray(E_e, np.float64)
    return lib().orc_eq4(_p(a), P_R, _p(b))


def eq5(P_target, P_e, P_R, units) -> float:
    a = np.ascontiguousarray(P_e, np.float64)
    return lib().orc_eq5(P_target, _p(a), P_R, units)


def median_prob(psi: np.ndarray, n: int) -> float:
    a = np.ascontiguousarray(psi, np.complex128)
    return lib().orc_median_prob(n, _p(a))


def run_criterion(circuit, px, py, pz, seed, t0, N, crit, target=0, cid=0, nthreads=0):
    """Per-trajectory criterion values: crit 1 = |a_target|^2, 2 = heavy output."""
    oc = OCircuit(circuit)
    out = np.zeros(max(N, 1), np.float64)
    rc = lib().orc_run_criterion(*oc.args(), px, py, pz, seed, cid, t0, N, crit, target,
                                 nthreads, _p(out))
    assert rc == 0
    return out[:N]
