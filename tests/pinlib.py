"""Independent constructions used to pin the oracle.

Nothing here is shared with the oracle's C code: gate unitaries are built from
their defining generators with ``scipy.linalg.expm`` or from projectors, full
2^n x 2^n operators with ``numpy.kron``, noisy averages by exact density-matrix
evolution or by enumerating every Pauli error pattern.  A mistake in the
oracle (a transposed matrix, a wrong sign or phase, a wrong qubit order, a
dropped error term) shows up as a mismatch against these.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.linalg import expm

I2 = np.eye(2, dtype=complex)
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
PAULI = {1: PX, 2: PY, 3: PZ}
P0 = np.array([[1, 0], [0, 0]], dtype=complex)   # |0><0|
P1 = np.array([[0, 0], [0, 1]], dtype=complex)   # |1><1|


def rot(P, theta):
    """exp(-i theta P / 2) from the generator."""
    return expm(-1j * theta * P / 2)


def gate_unitary(name, params=(), matrix=None):
    """Local unitary; 2q operators act on local index b_q0 + 2 b_q1, i.e. the
    operator is kron(op_on_q1, op_on_q0)."""
    if name == "H":
        return (PX + PZ) / math.sqrt(2)
    if name == "X":
        return PX.copy()
    if name == "Y":
        return PY.copy()
    if name == "Z":
        return PZ.copy()
    if name == "S":
        return expm(1j * math.pi / 4 * (I2 - PZ))       # diag(1, i)
    if name == "T":
        return expm(1j * math.pi / 8 * (I2 - PZ))       # diag(1, e^{i pi/4})
    if name == "RX":
        return rot(PX, params[0])
    if name == "RY":
        return rot(PY, params[0])
    if name == "RZ":
        return rot(PZ, params[0])
    if name == "U":
        a, b, c = params
        return rot(PZ, a) @ rot(PY, b) @ rot(PZ, c)
    if name == "U1Q":
        return np.asarray(matrix, complex)
    # two-qubit: first listed qubit = local bit 0 -> right factor of kron
    if name == "CNOT":      # control q0, target q1
        return np.kron(I2, P0) + np.kron(PX, P1)
    if name == "CZ":
        return np.kron(I2, P0) + np.kron(PZ, P1)
    if name == "CP":
        return np.kron(I2, I2) + (np.exp(1j * params[0]) - 1) * np.kron(P1, P1)
    if name == "SWAP":
        return 0.5 * (np.kron(I2, I2) + np.kron(PX, PX) + np.kron(PY, PY) + np.kron(PZ, PZ))
    if name == "RZZ":
        return expm(-1j * params[0] / 2 * np.kron(PZ, PZ))
    if name == "U2Q":
        return np.asarray(matrix, complex)
    raise ValueError(name)


def embed(n, qubits, U):
    """Full 2^n operator of a local operator on `qubits` (qubit 0 = LSB).

    Built as a sum over matrix units with numpy.kron, independent of any
    index-bit arithmetic used by the simulators."""
    k = len(qubits)
    full = np.zeros((1 << n, 1 << n), dtype=complex)
    for r in range(1 << k):
        for c in range(1 << k):
            if U[r, c] == 0:
                continue
            # |r><c| on the listed qubits, identity elsewhere
            ops = []
            for q in range(n):
                if q in qubits:
                    j = qubits.index(q)
                    rb, cb = (r >> j) & 1, (c >> j) & 1
                    E = np.zeros((2, 2), complex)
                    E[rb, cb] = 1
                    ops.append(E)
                else:
                    ops.append(I2)
            term = np.array([[1.0 + 0j]])
            for q in range(n - 1, -1, -1):      # kron(op_{n-1}, ..., op_0)
                term = np.kron(term, ops[q])
            full += U[r, c] * term
    return full


def circuit_unitaries(circuit):
    return [embed(circuit.n, list(g.qubits), gate_unitary(g.name, g.params, g.matrix))
            for g in circuit.gates]


def site_list(circuit):
    """(gate index, qubit) per error site, in gate order then listed order."""
    out = []
    for gi, g in enumerate(circuit.gates):
        for q in g.qubits:
            out.append((gi, q))
    return out


def simulate_pattern(circuit, pattern, full_ops=None, init_index=0):
    """Independent simulation with errors: pattern[s] in {0,1,2,3}."""
    n = circuit.n
    if full_ops is None:
        full_ops = circuit_unitaries(circuit)
    paulis = {}
    for s, (gi, q) in enumerate(site_list(circuit)):
        if pattern[s]:
            paulis.setdefault(gi, []).append(embed(n, [q], PAULI[pattern[s]]))
    psi = np.zeros(1 << n, complex)
    psi[init_index] = 1
    for gi, U in enumerate(full_ops):
        psi = U @ psi
        for E in paulis.get(gi, []):
            psi = E @ psi
    return psi


def fid(a, b):
    return abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)


def density_depolarizing(circuit, px, py, pz):
    """Exact density-matrix evolution: after each gate, on each touched qubit,
    rho -> (1-sum) rho + px X rho X + py Y rho Y + pz Z rho Z."""
    n = circuit.n
    rho = np.zeros((1 << n, 1 << n), complex)
    rho[0, 0] = 1
    ps = 1 - px - py - pz
    for g in circuit.gates:
        U = embed(n, list(g.qubits), gate_unitary(g.name, g.params, g.matrix))
        rho = U @ rho @ U.conj().T
        for q in g.qubits:
            X = embed(n, [q], PX)
            Y = embed(n, [q], PY)
            Z = embed(n, [q], PZ)
            rho = ps * rho + px * X @ rho @ X + py * Y @ rho @ Y + pz * Z @ rho @ Z
    return rho


def enumerate_success_weights(circuit, tau):
    """Exact success polynomial coefficients for uniform p/3 errors.

    Returns c[w] = number of weight-w error patterns (w non-identity sites,
    each X/Y/Z) whose final state has fidelity >= tau, so that
    P(p) = sum_w c[w] (1-p)^(S-w) (p/3)^w."""
    ops = circuit_unitaries(circuit)
    ref = simulate_pattern(circuit, [0] * 64, ops)
    S = len(site_list(circuit))
    c = np.zeros(S + 1, dtype=np.int64)
    for pat in itertools.product(range(4), repeat=S):
        psi = simulate_pattern(circuit, pat, ops)
        w = sum(1 for v in pat if v)
        if fid(ref, psi) >= tau:
            c[w] += 1
    return c


def success_poly(c, S, p):
    w = np.arange(len(c))
    return float(np.sum(c * (1 - p) ** (S - w) * (p / 3) ** w))


def ghz_chain_all_fired(n, pauli):
    """Nonzero amplitudes {index: value} of the GHZ circuit H(0), CNOT(j ->
    j+1) for j < n-1, with `pauli` ('X' or 'Z') fired at every site.

    Each error is moved to the end through the later CNOTs, which map X on a
    control to X on control and target and Z on a target to Z on control and
    target and leave the rest alone.  X: qubit j ends with j + 2 flips for
    j <= n-2 (one from the H error, one from the error on j as a control, j
    from the errors on the targets 1..j carried down the chain) and n for
    j = n-1, so X acts on the odd j <= n-2 and on n-1 when n is odd.  Z: the
    errors stay where they fire; every qubit but the last collects two, the
    last one, so the result is Z on qubit n-1."""
    full = (1 << n) - 1
    h = 1 / math.sqrt(2)
    if pauli == "X":
        mask = sum(1 << j for j in range(n - 1) if j % 2 == 1)
        if n % 2 == 1:
            mask |= 1 << (n - 1)
        return {mask: h, mask ^ full: h}
    if pauli == "Z":
        return {0: h, full: -h}
    raise ValueError(pauli)


# ---------------------------------------------------------------------------
# Tensor-network simulator for large states (n ~ 20-22), independent of the
# oracle's index-bit loops: the state is an n-axis array of shape (2,)*n
# (numpy's C order puts qubit n-1 on axis 0, so qubit q is axis n-1-q), and a
# gate is a tensordot of its local unitary with the axes of its qubits.

def _axis(n, q):
    return n - 1 - q


def tn_apply(psi, n, qubits, U):
    """Apply a local unitary (2x2, or 4x4 on local index b_q0 + 2 b_q1)."""
    t = psi.reshape((2,) * n)
    if len(qubits) == 1:
        ax = _axis(n, qubits[0])
        out = np.tensordot(U, t, axes=([1], [ax]))
        out = np.moveaxis(out, 0, ax)
    else:
        a, b = _axis(n, qubits[0]), _axis(n, qubits[1])
        # local index i = b_q0 + 2 b_q1 -> reshaped U4[b1_out, b0_out, b1_in, b0_in]
        U4 = np.asarray(U).reshape(2, 2, 2, 2)
        out = np.tensordot(U4, t, axes=([2, 3], [b, a]))
        out = np.moveaxis(out, [0, 1], [b, a])
    return np.ascontiguousarray(out).reshape(-1)


def tn_simulate(circuit, fired=None, init_index=0):
    """Final state; fired: {site: pauli code} with sites in gate order, then
    listed-qubit order."""
    n = circuit.n
    psi = np.zeros(1 << n, complex)
    psi[init_index] = 1
    s = 0
    for g in circuit.gates:
        psi = tn_apply(psi, n, list(g.qubits), gate_unitary(g.name, g.params, g.matrix))
        for q in g.qubits:
            if fired and s in fired:
                psi = tn_apply(psi, n, [q], PAULI[fired[s]])
            s += 1
    return psi
