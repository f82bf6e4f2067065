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


def test_labels_match_oracle_sweep(P, ctx, orc):
    """Labels are the library's batched Monte Carlo success probabilities;
    spot-check them against the oracle's sweep (complex128: equal counts)."""
    from paper_2301_07264_amd import surrogate as SG
    circs = [W.config3_circuit(s) for s in (300, 301, 302, 303)]
    circs = [c for c in circs if c.n <= 12][:3]
    hs = [P.nt_circuit_load(None, c) for c in circs]
    P.nt_set_precision(ctx, P.NT_C128)
    N = 96
    _say("surrogate labels vs oracle sweep")
    lab = SG.make_labels(ctx, hs, N, seed=4)
    for i, c in enumerate(circs):
        want = orc.sweep(c, P.GNN_RATES, 4, N, 0.9, cid=i)
        np.testing.assert_allclose(lab[i], want, rtol=0, atol=1e-6)
    P.nt_set_precision(ctx, P.NT_C64)
    for h in hs:
        P.nt_circuit_free(h)


def test_surrogate_bracket_saves_probes(P, ctx):
    """Trained on Monte Carlo labels, the surrogate predicts held-out curves
    well, and its guided search reaches the same tolerance with less Monte
    Carlo work than the search over the whole grid; it is compared with the
    best route without a model (the two-stage search from the zero-error
    bound, nt_tolerable_rate_auto) in units of full-sample probes."""
    from paper_2301_07264_amd import surrogate as SG
    P.nt_set_precision(ctx, P.NT_C64)
    train_c = [W.config3_circuit(s) for s in range(512)]
    held_c = [W.config3_circuit(100000 + s) for s in range(48)]
    th = [P.nt_circuit_load(None, c) for c in train_c]
    hh = [P.nt_circuit_load(None, c) for c in held_c]
    _say("surrogate gain: labels")
    lab_tr = SG.make_labels(ctx, th, 256, seed=1)
    lab_ho = SG.make_labels(ctx, hh, 256, seed=1)
    _say("surrogate gain: training")
    m, losses = SG.train(ctx, th, lab_tr, epochs=60)
    assert losses[-1] < 0.2 * losses[0]
    pred = P.nt_gnn_predict(m, hh)
    mse = float(((pred - lab_ho) ** 2).mean())
    base = float(((lab_tr.mean(0)[None, :] - lab_ho) ** 2).mean())
    _say(f"  held-out mse {mse:.3g} vs {base:.3g} for the training mean")
    assert mse < 0.1 * base
    ev = [i for i in range(len(hh)) if lab_ho[i, 0] >= 0.66 > lab_ho[i, -1]][:6]
    assert len(ev) >= 4
    work = {"full": [], "auto": [], "surrogate": []}
    N = 1024
    for i in ev:
        _say(f"surrogate gain: searches on held-out circuit {i}")
        r = SG.tolerable_rate_searches(ctx, hh[i], m, n_traj=N, seed=3)
        # every route stops on the same criterion over the same trajectories:
        # the success probability at its rate is within the tolerance
        for name in work:
            p = r[name]["p_star"]
            P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
            _, Pm = P.nt_run(ctx, hh[i], 3, 0, N, 0.9)
            assert abs(Pm - 0.66) <= 0.01 + 1e-12, (name, p, Pm)
            work[name].append(r[name]["work"])
    mean = {k: float(np.mean(v)) for k, v in work.items()}
    _say(f"  Monte Carlo work (full-sample probes): {mean}")
    assert mean["surrogate"] < mean["full"]
    assert mean["surrogate"] <= mean["auto"]
    P.nt_gnn_destroy(m)
    for h in th + hh:
        P.nt_circuit_free(h)
