"""Circuit generators for the synthetic workloads.

Conventions (shared interface, not arithmetic):
  * qubit 0 is the least-significant bit of a basis-state index;
  * a gate is (name, qubits, params); two-qubit gates list their qubits in the
    order that defines their error sites (one site per listed qubit, in order);
  * CNOT lists (control, target).

Workloads (all seeded with ``numpy.random.default_rng``):
  * random rotation layers: per layer, for q = 0..n-1 one U(a, b, c) with
    a, b, c uniform in [0, 2*pi) (U = Rz(a) Ry(b) Rz(c), one gate, one site),
    then a random disjoint pairing perm = rng.permutation(n) with
    CNOT(perm[2i] -> perm[2i+1]); for odd n the last qubit of perm is unpaired;
  * GHZ preparation: H(0), CNOT(i -> i+1) for i = 0..n-2;
  * QFT: for j = n-1 down to 0: H(j), then for m = j-1 down to 0 a controlled
    phase CP(pi / 2**(j-m)) on (m, j); finally SWAP(q, n-1-q) for q < n//2;
  * quantum-volume model circuits: per layer a random pairing with a
    Haar-random U(4) on every pair;
  * alternating-layer circuit on a random 3-regular graph: H on every qubit,
    then R rounds of RZZ(gamma_r) on the edges (lexicographic, i < j) followed by
    RX(beta_r) on every qubit, gamma_r and beta_r uniform in [0, pi).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

# Gate vocabulary: name -> number of qubits / number of real parameters.
GATE_ARITY = {
    "H": 1, "X": 1, "Y": 1, "Z": 1, "S": 1, "T": 1,
    "RX": 1, "RY": 1, "RZ": 1, "U": 1, "U1Q": 1,
    "CNOT": 2, "CZ": 2, "CP": 2, "SWAP": 2, "RZZ": 2, "U2Q": 2,
}
GATE_NPARAM = {
    "H": 0, "X": 0, "Y": 0, "Z": 0, "S": 0, "T": 0,
    "RX": 1, "RY": 1, "RZ": 1, "U": 3, "U1Q": 0,
    "CNOT": 0, "CZ": 0, "CP": 1, "SWAP": 0, "RZZ": 1, "U2Q": 0,
}


@dataclass
class Gate:
    name: str
    qubits: Tuple[int, ...]
    params: Tuple[float, ...] = ()
    # Row-major complex matrix for U1Q (2x2) / U2Q (4x4); None otherwise.
    matrix: object = None


@dataclass
class Circuit:
    n: int
    gates: List[Gate] = field(default_factory=list)
    name: str = ""

    @property
    def G(self) -> int:
        return len(self.gates)

    @property
    def S(self) -> int:
        """Number of error sites: one per qubit a gate touches."""
        return sum(len(g.qubits) for g in self.gates)

    def __add__(self, other: "Circuit") -> "Circuit":
        assert self.n == other.n
        return Circuit(self.n, list(self.gates) + list(other.gates),
                       self.name + "+" + other.name)

    def arrays(self):
        """Flat arrays (names, q0, q1, params[G,3], matrices) for C callers."""
        G = len(self.gates)
        names = [g.name for g in self.gates]
        q0 = np.zeros(G, np.int32)
        q1 = np.full(G, -1, np.int32)
        par = np.zeros((G, 3), np.float64)
        for i, g in enumerate(self.gates):
            q0[i] = g.qubits[0]
            if len(g.qubits) > 1:
                q1[i] = g.qubits[1]
            for j, v in enumerate(g.params):
                par[i, j] = v
        return names, q0, q1, par


def random_layers(n: int, layers: int, rng: np.random.Generator) -> Circuit:
    gates: List[Gate] = []
    for _ in range(layers):
        ang = rng.uniform(0.0, 2.0 * math.pi, size=(n, 3))
        for q in range(n):
            gates.append(Gate("U", (q,), tuple(float(v) for v in ang[q])))
        perm = rng.permutation(n)
        for i in range(n // 2):
            gates.append(Gate("CNOT", (int(perm[2 * i]), int(perm[2 * i + 1]))))
    return Circuit(n, gates, f"layers{layers}")


def ghz(n: int) -> Circuit:
    gates = [Gate("H", (0,))]
    gates += [Gate("CNOT", (i, i + 1)) for i in range(n - 1)]
    return Circuit(n, gates, "ghz")


def qft(n: int) -> Circuit:
    gates: List[Gate] = []
    for j in range(n - 1, -1, -1):
        gates.append(Gate("H", (j,)))
        for m in range(j - 1, -1, -1):
            gates.append(Gate("CP", (m, j), (math.pi / float(2 ** (j - m)),)))
    for q in range(n // 2):
        gates.append(Gate("SWAP", (q, n - 1 - q)))
    return Circuit(n, gates, "qft")


def haar_unitary(dim: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random dim x dim unitary: QR of a complex Gaussian matrix with the
    phases of R's diagonal moved into Q (Mezzadri's recipe)."""
    z = (rng.normal(size=(dim, dim)) + 1j * rng.normal(size=(dim, dim))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


def quantum_volume(n: int, depth: int, rng: np.random.Generator) -> Circuit:
    """Quantum-volume-style model circuit: depth layers, each a random pairing
    perm = rng.permutation(n) with a Haar-random U(4) (one U2Q gate) on
    (perm[2i], perm[2i+1]); for odd n the last qubit of perm idles."""
    gates: List[Gate] = []
    for _ in range(depth):
        perm = rng.permutation(n)
        for i in range(n // 2):
            gates.append(Gate("U2Q", (int(perm[2 * i]), int(perm[2 * i + 1])), (), haar_unitary(4, rng)))
    return Circuit(n, gates, f"qv{n}x{depth}")


def random_regular_graph(n: int, d: int, rng: np.random.Generator):
    """Configuration model with rejection: simple d-regular graph, sorted edges."""
    assert (n * d) % 2 == 0
    while True:
        stubs = np.repeat(np.arange(n), d)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        edges = set()
        ok = True
        for a, b in pairs:
            a, b = int(a), int(b)
            if a == b:
                ok = False
                break
            e = (min(a, b), max(a, b))
            if e in edges:
                ok = False
                break
            edges.add(e)
        if ok:
            return sorted(edges)


def qaoa_3regular(n: int, rounds: int, rng: np.random.Generator) -> Circuit:
    edges = random_regular_graph(n, 3, rng)
    gates = [Gate("H", (q,)) for q in range(n)]
    for _ in range(rounds):
        gamma = float(rng.uniform(0.0, math.pi))
        beta = float(rng.uniform(0.0, math.pi))
        for a, b in edges:
            gates.append(Gate("RZZ", (a, b), (gamma,)))
        for q in range(n):
            gates.append(Gate("RX", (q,), (beta,)))
    return Circuit(n, gates, f"qaoa3reg_r{rounds}")


# ---------------------------------------------------------------------------
# The five synthetic workloads.

def config0(seed: int = 0) -> Circuit:
    """8 qubits, 20 random rotation + CNOT layers (G=240, S=320)."""
    c = random_layers(8, 20, np.random.default_rng(seed))
    c.name = "layers8x20"
    return c


def config1(seed: int = 0, n: int = 24, layers: int = 50) -> Circuit:
    """GHZ preparation, full QFT, then random layers (n=24: G=2136, S=3047)."""
    c = ghz(n) + qft(n) + random_layers(n, layers, np.random.default_rng(seed))
    c.name = f"ghz_qft_layers{n}x{layers}"
    return c


def config2(circuit_seed: int) -> Circuit:
    """One batched-workload instance: n ~ U{10..20}, layers ~ U{10..100}."""
    rng = np.random.default_rng(circuit_seed)
    n = int(rng.integers(10, 21))
    layers = int(rng.integers(10, 101))
    c = random_layers(n, layers, rng)
    c.name = f"batch{circuit_seed}_n{n}_l{layers}"
    return c


def config3_circuit(circuit_seed: int) -> Circuit:
    """One surrogate-training instance: n ~ U{8..16}, layers ~ U{5..80}."""
    rng = np.random.default_rng(circuit_seed)
    n = int(rng.integers(8, 17))
    layers = int(rng.integers(5, 81))
    c = random_layers(n, layers, rng)
    c.name = f"surr{circuit_seed}_n{n}_l{layers}"
    return c


def config4(seed: int = 0, n: int = 30, rounds: int = 4) -> Circuit:
    """30-qubit alternating layers on a 3-regular graph (G=330, S=510)."""
    c = qaoa_3regular(n, rounds, np.random.default_rng(seed))
    c.name = f"qaoa3reg{n}x{rounds}"
    return c


def rates_config1() -> np.ndarray:
    """13 log-spaced per-gate rates 10**(-5 + j/4), j = 0..12."""
    return np.array([10.0 ** (-5.0 + j / 4.0) for j in range(13)])


def rates_config4() -> np.ndarray:
    """7 log-spaced rates 10**(-5 + j/3), j = 0..6."""
    return np.array([10.0 ** (-5.0 + j / 3.0) for j in range(7)])


# ---------------------------------------------------------------------------
# Text format: first line "qubits <n>", then one gate per line:
#   NAME q0 [q1] [p0 p1 p2]            (angles written with repr: exact round trip)
#   U1Q q re00 im00 re01 im01 ...     (row-major complex entries)
# Lines starting with '#' are comments.

def to_text(c: Circuit) -> str:
    out = [f"# circuit {c.name}", f"qubits {c.n}"]
    for g in c.gates:
        parts = [g.name] + [str(q) for q in g.qubits]
        if g.matrix is not None:
            m = np.asarray(g.matrix, dtype=np.complex128).ravel()
            for v in m:
                parts += [repr(float(v.real)), repr(float(v.imag))]
        else:
            parts += [repr(float(p)) for p in g.params]
        out.append(" ".join(parts))
    return "\n".join(out) + "\n"


def from_text(text: str) -> Circuit:
    n = None
    gates: List[Gate] = []
    name = ""
    for raw in text.splitlines():
        line = raw.strip()
        if not line:
            continue
        if line.startswith("#"):
            if line.startswith("# circuit "):
                name = line[len("# circuit "):]
            continue
        tok = line.split()
        if tok[0] == "qubits":
            n = int(tok[1])
            continue
        gname = tok[0]
        if gname not in GATE_ARITY:
            raise ValueError(f"unknown gate {gname!r}")
        k = GATE_ARITY[gname]
        qs = tuple(int(t) for t in tok[1:1 + k])
        rest = [float(t) for t in tok[1 + k:]]
        if gname in ("U1Q", "U2Q"):
            dim = 2 ** k
            vals = np.array(rest, dtype=np.float64)
            if vals.size != 2 * dim * dim:
                raise ValueError("bad matrix size")
            m = (vals[0::2] + 1j * vals[1::2]).reshape(dim, dim)
            gates.append(Gate(gname, qs, (), m))
        else:
            gates.append(Gate(gname, qs, tuple(rest)))
    if n is None:
        raise ValueError("missing 'qubits' line")
    return Circuit(n, gates, name)


def write_text(c: Circuit, path: str) -> None:
    with open(path, "w") as f:
        f.write(to_text(c))


def read_text(path: str) -> Circuit:
    with open(path) as f:
        return from_text(f.read())
