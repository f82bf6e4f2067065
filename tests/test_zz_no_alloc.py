"""GPU test of nt_run_noalloc, the entry point that allocates no device
memory (its buffers live in a static scratch array per device).

Its values must equal nt_run's (short-cuts off) bit for bit: same plan, same
kernels, same trajectories.  Two calls in a row, the second with a smaller
input, so that the second runs on what the first left in the shared array;
a multi-pass circuit (trajectory states in the array); the measurement
criteria; and a request too large for the array, refused before any launch.
"""
import sys

import numpy as np
import pytest

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


def _both(P, ctx, h, seed, t0, N, tau):
    f_ref = np.zeros(N)
    c_ref, p_ref = P.nt_run(ctx, h, seed, t0, N, tau, f_ref)
    f_na = np.full(N, np.nan)
    c_na, p_na = P.nt_run_noalloc(ctx, h, seed, t0, N, tau, f_na)
    np.testing.assert_array_equal(f_na.view(np.uint64), f_ref.view(np.uint64))
    assert c_na == c_ref and p_na == p_ref
    return f_ref


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_noalloc_equals_run_two_calls(P, prec):
    pr = P.NT_C64 if prec == "c64" else P.NT_C128
    ctx = P.nt_create(0)
    try:
        P.nt_set_precision(ctx, pr)
        big, small = W.config0(), W.random_layers(5, 6, np.random.default_rng(3))
        hb, hs = P.nt_circuit_load(ctx, big), P.nt_circuit_load(ctx, small)
        P.nt_set_error_model(ctx, 1e-3 / 3, 1e-3 / 3, 1e-3 / 3)
        _say(f"noalloc {prec}: 8 qubits, 300 trajectories")
        f1 = _both(P, ctx, hb, 7, 0, 300, 0.9)
        P.nt_set_error_model(ctx, 0.05 / 3, 0.05 / 3, 0.05 / 3)
        _say(f"noalloc {prec}: 5 qubits, 40 trajectories (second, smaller call)")
        f2 = _both(P, ctx, hs, 7, 11, 40, 0.9)
        # both runs see failing and succeeding trajectories
        assert f1.min() < 0.9 <= f1.max() and f2.min() < 0.9
        P.nt_circuit_free(hb)
        P.nt_circuit_free(hs)
    finally:
        P.nt_destroy(ctx)


def test_noalloc_multi_pass_and_criteria(P):
    ctx = P.nt_create(0)
    try:
        P.nt_set_precision(ctx, P.NT_C64)
        c = W.random_layers(16, 4, np.random.default_rng(5))
        h = P.nt_circuit_load(ctx, c)
        assert P.nt_plan_info(h, P.NT_C64)[0] > 1
        p = 0.01
        P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
        _say("noalloc: 16 qubits, multi-pass, 24 trajectories")
        _both(P, ctx, h, 2, 0, 24, 0.9)
        for crit in (P.NT_CRIT_HEAVY, P.NT_CRIT_TARGET_PROB):
            _say(f"noalloc: criterion {crit}")
            P.nt_set_criterion(ctx, crit, 5)
            _both(P, ctx, h, 2, 0, 12, 0.5)
        P.nt_set_criterion(ctx, P.NT_CRIT_FIDELITY, 0)
        P.nt_circuit_free(h)
    finally:
        P.nt_destroy(ctx)


def test_noalloc_rejects_oversized(P):
    ctx = P.nt_create(0)
    try:
        P.nt_set_precision(ctx, P.NT_C64)
        h = P.nt_circuit_load(ctx, W.ghz(24))     # a 128 MiB state
        with pytest.raises(P.NtError) as e:
            P.nt_run_noalloc(ctx, h, 0, 0, 1, 0.9)
        assert e.value.status == P.NT_ERR_UNSUPPORTED
        assert "scratch" in str(e.value)
        # the context still works afterwards
        _both(P, ctx, P.nt_circuit_load(ctx, W.config0()), 1, 0, 8, 0.9)
    finally:
        P.nt_destroy(ctx)
