"""Seeded synthetic circuit generators and the text circuit format.

This module produces gate lists only (gate name, qubits, angles, and the
random matrices of U2Q gates, which are inputs).  It holds none of the
simulation arithmetic: no named-gate matrices, no random error draws, no
scoring.  Both the CPU oracle tests and the GPU library's binding read
circuits from here, so parity never depends on how a circuit was made.
"""
from .circuits import (  # noqa: F401
    Gate, Circuit, GATE_ARITY, GATE_NPARAM,
    random_layers, ghz, qft, qaoa_3regular, random_regular_graph, quantum_volume, haar_unitary,
    config0, config1, config2, config3_circuit, config4,
    rates_config1, rates_config4,
    write_text, read_text, to_text, from_text,
)
