"""Host-side checks of the surrogate: the library's gate graph against the
definition written out independently in tests/gnn_ref.py, and argument
validation of the surrogate entry points (no GPU needed)."""
import ctypes as C

import numpy as np
import pytest

import gnn_ref
import workloads as W


@pytest.fixture(scope="module")
def P():
    import paper_2301_07264_amd as P
    P.lib()
    return P


@pytest.mark.parametrize("maker", [
    lambda: W.config3_circuit(5),
    lambda: W.qft(5),
    lambda: W.qaoa_3regular(6, 2, np.random.default_rng(3)),
    lambda: W.quantum_volume(4, 3, np.random.default_rng(4)),
])
def test_graph_matches_definition(P, maker):
    c = maker()
    h = P.nt_circuit_load(None, c)
    x, rp, col, glob = P.nt_gnn_graph(h)
    P.nt_circuit_free(h)
    xr, nbr, gr = gnn_ref.graph(c)
    np.testing.assert_allclose(x, xr, rtol=0, atol=1e-6)
    np.testing.assert_allclose(glob, gr, rtol=1e-7)
    assert len(rp) == len(nbr) + 1
    for v, ns in enumerate(nbr):
        assert sorted(col[rp[v]:rp[v + 1]].tolist()) == sorted(ns)


def test_graph_small_by_hand(P):
    # H(0); CNOT(0 -> 1); RZ(0.5) on 1: layers 0, 1, 2; edges H-CNOT (qubit 0),
    # CNOT-RZ (qubit 1)
    c = W.Circuit(2, [W.Gate("H", (0,)), W.Gate("CNOT", (0, 1)), W.Gate("RZ", (1,), (0.5,))])
    h = P.nt_circuit_load(None, c)
    x, rp, col, glob = P.nt_gnn_graph(h)
    P.nt_circuit_free(h)
    assert x.shape == (3, 32)
    assert x[0, 0] == 1 and x[1, 11] == 1 and x[2, 8] == 1
    assert x[2, 17] == pytest.approx(np.sin(0.5)) and x[2, 18] == pytest.approx(np.cos(0.5))
    assert x[0, 17] == 0 and x[0, 18] == 0                 # no angle: zeros, not cos(0)
    np.testing.assert_allclose(x[:, 23], [0, 1 / 3, 2 / 3], rtol=1e-6)
    np.testing.assert_allclose(x[:, 24], [0, 1, 0])
    assert rp.tolist() == [0, 1, 3, 4]
    assert sorted(col[1:3].tolist()) == [0, 2] and col[0] == 1 and col[3] == 1
    np.testing.assert_allclose(glob, [2 / 16, 3 / 2048, 4 / 4096, 1], rtol=1e-7)


def test_surrogate_argument_errors(P):
    L = P.lib()
    assert L.nt_gnn_create(None, 0, C.byref(C.c_void_p())) == P.NT_ERR_INVALID_ARG
    assert L.nt_gnn_graph(None, None, None, None, None, None, None) == P.NT_ERR_INVALID_ARG
    assert L.nt_gnn_train(None, 1, 1, 0.1, 0, None) == P.NT_ERR_INVALID_ARG
    assert L.nt_gnn_predict(None, None, 0, 0, None) == P.NT_ERR_INVALID_ARG
    L.nt_gnn_destroy(None)


def test_reference_gradient_by_finite_differences():
    """The FP64 reference itself against central differences."""
    rng = np.random.default_rng(0)
    circs = [W.config3_circuit(s) for s in (1, 2)]
    circs = [W.Circuit(c.n, c.gates[:40]) for c in circs]
    _, total = gnn_ref.layout()
    params = rng.normal(scale=0.2, size=total)
    labels = rng.uniform(size=(2, 13))
    l0, g, _ = gnn_ref.loss_and_grad(params, circs, labels)
    for i in rng.choice(total, 12, replace=False):
        e = np.zeros(total)
        e[i] = 1e-6
        lp, _, _ = gnn_ref.loss_and_grad(params + e, circs, labels)
        lm, _, _ = gnn_ref.loss_and_grad(params - e, circs, labels)
        assert abs((lp - lm) / 2e-6 - g[i]) <= 1e-6 + 1e-4 * abs(g[i])
