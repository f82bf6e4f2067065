"""The largest state the library accepts (32 qubits: 32 GiB per complex64
state) and long CNOT chains with every error site fired, against the closed
forms of pinlib.ghz_chain_all_fired (themselves checked against the oracle
and a brute-force simulation in test_oracle_pins.py).

At 32 qubits the final state goes to a device buffer and is checked at its
two nonzero entries plus a count of nonzero components over all 2^33 floats;
smaller sizes compare the whole state on the host."""
import ctypes as C
import sys

import numpy as np
import pytest

import pinlib
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


@pytest.mark.parametrize("n", [7, 20, 32])
def test_ghz_chain_every_site_fired(P, n):
    import torch
    ctx = P.nt_create(0)
    h = P.nt_circuit_load(None, W.ghz(n))
    try:
        precs = [(P.NT_C64, 1e-6)] + ([(P.NT_C128, 1e-13)] if n <= 20 else [])
        for pr, tol in precs:
            P.nt_set_precision(ctx, pr)
            for pauli, model in (("X", (1.0, 0.0, 0.0)), ("Z", (0.0, 0.0, 1.0))):
                _say(f"ghz chain n={n} prec={pr} every site {pauli}")
                P.nt_set_error_model(ctx, *model)
                want = pinlib.ghz_chain_all_fired(n, pauli)
                # fidelity with the error-free GHZ state: the supports are
                # disjoint (X) or the two terms cancel exactly (Z)
                f = np.full(2, -1.0)
                cnt, p = P.nt_run(ctx, h, 0, 0, 2, TAU, f)
                full = (1 << n) - 1
                same = set(want) == {0, full} and want[0] == want[full]
                np.testing.assert_array_equal(f, np.full(2, 1.0 if same else 0.0))
                assert cnt == (2 if same else 0)
                if n <= 20:
                    psi = P.nt_final_state(ctx, h, 0, 1, pr).astype(np.complex128)
                    ref = np.zeros(1 << n, complex)
                    for k, a in want.items():
                        ref[k] = a
                    assert float(np.abs(psi - ref).max()) <= tol
                else:
                    t = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
                    st = P.lib().nt_final_state(ctx, h, C.c_uint64(0), C.c_uint64(1), C.c_void_p(t.data_ptr()),
                                                C.c_int64(t.numel()))
                    assert st == P.NT_OK, P.nt_last_error()
                    torch.cuda.synchronize()
                    idx = sorted(want)
                    got = t[torch.tensor(idx, device="cuda")].cpu().numpy().astype(np.complex128)
                    assert float(np.abs(got - np.array([want[k] for k in idx])).max()) <= tol
                    # the amplitudes are real: exactly two nonzero components
                    assert int(torch.count_nonzero(torch.view_as_real(t))) == len(idx)
                    del t
                    torch.cuda.empty_cache()
    finally:
        P.nt_circuit_free(h)
        P.nt_destroy(ctx)
