"""GPU checks of the surrogate network's kernels against the FP64 reference
(tests/gnn_ref.py): loss and gradient of the plain FP32 path within 1e-4
(relative, per parameter block), the bf16 MFMA path within bf16 rounding
(loss 2e-2 relative, gradient cosine >= 0.99 per block); predictions; a
training run that lowers the loss and is bit-for-bit repeatable."""
import sys

import numpy as np
import pytest

import gnn_ref
import workloads as W

pytestmark = pytest.mark.gpu


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


def _small_set(n=6):
    out = []
    for s in range(n):
        c = W.config3_circuit(100 + s)
        out.append(W.Circuit(c.n, c.gates[:min(len(c.gates), 120 + 37 * s)]))
    return out


def _blocks(v):
    off, _ = gnn_ref.layout()
    return {k: v[o:o + s] for k, (o, s) in off.items()}


@pytest.fixture(scope="module")
def model_and_data(P, ctx):
    circs = _small_set()
    hs = [P.nt_circuit_load(None, c) for c in circs]
    rng = np.random.default_rng(1)
    labels = rng.uniform(0.05, 0.95, size=(len(circs), 13)).astype(np.float32)
    m = P.nt_gnn_create(ctx, 7)
    P.nt_gnn_set_data(m, hs, labels)
    yield m, circs, hs, labels
    P.nt_gnn_destroy(m)
    for h in hs:
        P.nt_circuit_free(h)


def test_gnn_fp32_gradient_vs_fp64(P, model_and_data):
    m, circs, hs, labels = model_and_data
    params = P.nt_gnn_params(m)
    _say("surrogate: FP32 loss and gradient vs FP64 reference")
    loss, grad = P.nt_gnn_loss_grad(m, 0, len(circs), exact=True)
    lr, gr, _ = gnn_ref.loss_and_grad(params.astype(np.float64), circs, labels.astype(np.float64))
    assert abs(loss - lr) <= 1e-5 * abs(lr)
    gb, rb = _blocks(grad), _blocks(gr)
    for k in rb:
        den = np.linalg.norm(rb[k])
        assert np.linalg.norm(gb[k] - rb[k]) <= 1e-4 * den + 1e-9, k


def test_gnn_bf16_gradient_close(P, model_and_data):
    m, circs, hs, labels = model_and_data
    params = P.nt_gnn_params(m)
    _say("surrogate: bf16 MFMA loss and gradient vs FP64 reference")
    loss, grad = P.nt_gnn_loss_grad(m, 0, len(circs), exact=False)
    lr, gr, _ = gnn_ref.loss_and_grad(params.astype(np.float64), circs, labels.astype(np.float64))
    assert abs(loss - lr) <= 2e-2 * abs(lr)
    gb, rb = _blocks(grad), _blocks(gr)
    for k in rb:
        a, b = gb[k].astype(np.float64), rb[k]
        if np.linalg.norm(b) < 1e-8:
            continue
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
        assert cos >= 0.99, (k, cos)


def test_gnn_predict_vs_fp64(P, model_and_data):
    m, circs, hs, labels = model_and_data
    params = P.nt_gnn_params(m)
    _, _, out = gnn_ref.loss_and_grad(params.astype(np.float64), circs, labels.astype(np.float64))
    pe = P.nt_gnn_predict(m, hs, exact=True)
    assert np.abs(pe - out).max() <= 1e-5
    pb = P.nt_gnn_predict(m, hs, exact=False)
    assert np.abs(pb - out).max() <= 2e-2


def test_gnn_training_lowers_loss_and_repeats(P, ctx):
    circs = [W.config3_circuit(200 + s) for s in range(48)]
    hs = [P.nt_circuit_load(None, c) for c in circs]
    # a smooth synthetic target: exp(-S p) at the 13 rates
    lab = np.array([[np.exp(-c.S * r) for r in P.GNN_RATES] for c in circs], np.float32)
    runs = []
    for rep in range(2):
        m = P.nt_gnn_create(ctx, 11)
        P.nt_gnn_set_data(m, hs, lab)
        _say(f"surrogate: training run {rep}")
        losses = P.nt_gnn_train(m, 40, 8, 3e-3, seed=5)
        runs.append((losses, P.nt_gnn_params(m)))
        P.nt_gnn_destroy(m)
    (l0, p0), (l1, p1) = runs
    assert l0[-1] < 0.25 * l0[0]
    np.testing.assert_array_equal(p0.view(np.uint32), p1.view(np.uint32))
    np.testing.assert_array_equal(l0, l1)
    for h in hs:
        P.nt_circuit_free(h)
