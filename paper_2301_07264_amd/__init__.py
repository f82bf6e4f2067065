"""Python binding of libnisqtol (MI355X / gfx950).

Argument marshalling only: every step of the simulation runs in the HIP
library, which must have been built (``paper_2301_07264_amd.build.build()``).
Importing this package does not load the library; the first call does, and
fails loudly when it is missing.  There is no CPU fallback.

The functions keep the C names (``nt_create``, ``nt_run``, ...) and signatures
of include/nisqtol.h, with numpy arrays in place of pointers and exceptions in
place of status codes.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libnisqtol.so")

NT_OK = 0
NT_ERR_INVALID_ARG = 1
NT_ERR_UNSUPPORTED = 2
NT_ERR_OUT_OF_MEMORY = 3
NT_ERR_DEVICE = 4
NT_ERR_BUFFER_TOO_SMALL = 5
NT_ERR_NOT_BRACKETED = 6
STATUS_NAMES = {0: "NT_OK", 1: "NT_ERR_INVALID_ARG", 2: "NT_ERR_UNSUPPORTED", 3: "NT_ERR_OUT_OF_MEMORY",
                4: "NT_ERR_DEVICE", 5: "NT_ERR_BUFFER_TOO_SMALL", 6: "NT_ERR_NOT_BRACKETED"}

NT_C64 = 1
NT_C128 = 2

GATE_KIND = {
    "H": 0, "X": 1, "Y": 2, "Z": 3, "S": 4, "T": 5, "RX": 6, "RY": 7, "RZ": 8, "U": 9,
    "U1Q": 10, "CNOT": 11, "CZ": 12, "CP": 13, "SWAP": 14, "RZZ": 15, "U2Q": 16,
}

# Symbols declared in include/nisqtol.h.
EXPORTED = [
    "nt_create", "nt_destroy", "nt_set_error_model", "nt_set_precision", "nt_set_max_batch",
    "nt_circuit_load", "nt_circuit_load_text", "nt_circuit_free", "nt_circuit_info",
    "nt_circuit_set_id", "nt_plan_info", "nt_plan_export", "nt_run", "nt_run_noalloc", "nt_sweep", "nt_sweep_crossing", "nt_tolerable_rate",
    "nt_tolerable_rate_auto", "nt_tolerable_rate_fig3",
    "nt_sample_sites", "nt_final_state", "nt_reference_state", "nt_timing_enable",
    "nt_timing_reset", "nt_timing_read", "nt_last_error", "nt_version",
    "nt_set_shortcuts", "nt_exhaustive", "nt_eq4", "nt_eq5", "nt_success_probability",
    "nt_set_criterion", "nt_run_batch",
    "nt_gnn_create", "nt_gnn_destroy", "nt_gnn_graph", "nt_gnn_params", "nt_gnn_set_params",
    "nt_gnn_set_data", "nt_gnn_loss_grad", "nt_gnn_train", "nt_gnn_predict", "nt_tolerable_rate_guided",
    "nt_circuit_set_tile", "nt_circuit_set_fusion", "nt_autotune", "nt_autotune_plan", "nt_plan_ops",
]

GNN_RATES = [10.0 ** (-5.0 + j / 4.0) for j in range(13)]

NT_CRIT_FIDELITY = 0
NT_CRIT_TARGET_PROB = 1
NT_CRIT_HEAVY = 2
NT_SHORTCUT_ZERO_FIRED = 1
NT_SHORTCUT_CHECKPOINT = 2
NT_SHORTCUT_LAST_ERROR = 4
NT_SHORTCUT_REUSE = 8


class nt_gate(C.Structure):
    _fields_ = [("kind", C.c_uint16), ("nq", C.c_uint8), ("pad", C.c_uint8),
                ("q", C.c_int32 * 2), ("param", C.c_double * 3), ("matrix", C.POINTER(C.c_double))]


class NtError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib() -> C.CDLL:
    """Load libnisqtol.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libnisqtol.so not built ({LIB_PATH}); run paper_2301_07264_amd.build.build()")
    # PyTorch ships its own HIP runtime under the same soname.  Loaded first,
    # it is the one the library binds to, so torch's device pointers and
    # streams are valid here and the process holds a single runtime; loaded
    # after the library, it would bring a second runtime that sees no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P, i32, i64, u64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_uint64, C.c_double
    PP = C.POINTER(C.c_void_p)
    sig = {
        "nt_create": ([PP, i32, P], i32),
        "nt_destroy": ([P], None),
        "nt_set_error_model": ([P, dbl, dbl, dbl], i32),
        "nt_set_precision": ([P, i32], i32),
        "nt_set_max_batch": ([P, u64], i32),
        "nt_circuit_load": ([P, i32, P, i64, PP], i32),
        "nt_circuit_load_text": ([P, C.c_char_p, PP], i32),
        "nt_circuit_free": ([P], None),
        "nt_circuit_info": ([P, P, P, P], i32),
        "nt_circuit_set_id": ([P, u64], i32),
        "nt_plan_info": ([P, i32, P, P, P], i32),
        "nt_plan_export": ([P, i32, P, P, P, P, P], i32),
        "nt_run": ([P, P, u64, u64, u64, dbl, P, P, P], i32),
        "nt_run_noalloc": ([P, P, u64, u64, u64, dbl, P, P, P], i32),
        "nt_sweep": ([P, P, P, i32, u64, u64, dbl, P], i32),
        "nt_sweep_crossing": ([P, P, P, i32, u64, u64, dbl, dbl, P, P], i32),
        "nt_tolerable_rate": ([P, P, dbl, dbl, dbl, dbl, u64, u64, dbl, P, P], i32),
        "nt_tolerable_rate_auto": ([P, P, dbl, dbl, u64, u64, dbl, P, P, P, P], i32),
        "nt_tolerable_rate_fig3": ([P, P, dbl, dbl, u64, u64, dbl, P, P, P, P], i32),
        "nt_sample_sites": ([P, P, u64, u64, u64, P, P, P, i64, P], i32),
        "nt_final_state": ([P, P, u64, u64, P, i64], i32),
        "nt_reference_state": ([P, P, P, i64], i32),
        "nt_timing_enable": ([P, i32], i32),
        "nt_timing_reset": ([P], i32),
        "nt_timing_read": ([P, P, P, P, P, P], i32),
        "nt_set_shortcuts": ([P, i32], i32),
        "nt_set_criterion": ([P, i32, u64], i32),
        "nt_run_batch": ([P, P, i32, u64, u64, u64, dbl, P, P, P], i32),
        "nt_gnn_create": ([P, u64, PP], i32),
        "nt_gnn_destroy": ([P], None),
        "nt_gnn_graph": ([P, P, P, P, P, P, P], i32),
        "nt_gnn_params": ([P, P, P], i32),
        "nt_gnn_set_params": ([P, P, i64], i32),
        "nt_gnn_set_data": ([P, P, i32, P], i32),
        "nt_gnn_loss_grad": ([P, i32, i32, i32, P, P], i32),
        "nt_gnn_train": ([P, i32, i32, dbl, u64, P], i32),
        "nt_gnn_predict": ([P, P, i32, i32, P], i32),
        "nt_tolerable_rate_guided": ([P, P, P, dbl, dbl, u64, u64, dbl, P, P, P], i32),
        "nt_circuit_set_tile": ([P, i32, i32], i32),
        "nt_circuit_set_fusion": ([P, i32, i32], i32),
        "nt_plan_ops": ([P, i32, P, P], i32),
        "nt_autotune": ([P, P, u64, u64, P, P], i32),
        "nt_autotune_plan": ([P, P, u64, u64, P, P, P, i32], i32),
        "nt_exhaustive": ([P, P, dbl, P, P, P], i32),
        "nt_eq4": ([P, dbl, P, P], i32),
        "nt_eq5": ([dbl, P, dbl, dbl, P], i32),
        "nt_success_probability": ([P, P, u64, u64, dbl, P, P], i32),
        "nt_last_error": ([], C.c_char_p),
        "nt_version": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(status: int) -> None:
    if status != NT_OK:
        msg = lib().nt_last_error().decode(errors="replace")
        raise NtError(status, msg)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def nt_last_error() -> str:
    return lib().nt_last_error().decode(errors="replace")


def nt_version() -> str:
    return lib().nt_version().decode()


# ---- context -----------------------------------------------------------------

def nt_create(device: int = 0, hip_stream: Optional[int] = None) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().nt_create(C.byref(h), device, C.c_void_p(hip_stream) if hip_stream else None))
    return h


def nt_destroy(ctx) -> None:
    lib().nt_destroy(ctx)


def nt_set_error_model(ctx, p_x: float, p_y: float, p_z: float) -> None:
    _check(lib().nt_set_error_model(ctx, p_x, p_y, p_z))


def nt_set_precision(ctx, prec: int) -> None:
    _check(lib().nt_set_precision(ctx, prec))


def nt_set_max_batch(ctx, max_batch: int) -> None:
    _check(lib().nt_set_max_batch(ctx, max_batch))


# ---- circuits ------------------------------------------------------------------

class _GateArray:
    """Keeps the nt_gate array and the matrices it points to alive."""

    def __init__(self, circuit):
        G = len(circuit.gates)
        self.arr = (nt_gate * max(G, 1))()
        self.mats = []
        for i, g in enumerate(circuit.gates):
            e = self.arr[i]
            e.kind = GATE_KIND[g.name]
            e.nq = len(g.qubits)
            e.q[0] = g.qubits[0]
            e.q[1] = g.qubits[1] if len(g.qubits) > 1 else -1
            for j, v in enumerate(g.params):
                e.param[j] = float(v)
            if g.matrix is not None:
                m = np.asarray(g.matrix, np.complex128).ravel()
                buf = np.empty(2 * m.size, np.float64)
                buf[0::2] = m.real
                buf[1::2] = m.imag
                self.mats.append(buf)
                e.matrix = buf.ctypes.data_as(C.POINTER(C.c_double))
        self.G = G


def nt_circuit_load(ctx, circuit) -> C.c_void_p:
    """Load a ``workloads.Circuit`` (gate list) into the library."""
    ga = _GateArray(circuit)
    h = C.c_void_p()
    _check(lib().nt_circuit_load(ctx, circuit.n, C.cast(ga.arr, C.c_void_p), ga.G, C.byref(h)))
    return h


def nt_circuit_load_text(ctx, path: str) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().nt_circuit_load_text(ctx, path.encode(), C.byref(h)))
    return h


def nt_circuit_free(circ) -> None:
    lib().nt_circuit_free(circ)


def nt_circuit_info(circ) -> Tuple[int, int, int]:
    n, G, S = C.c_int(), C.c_int64(), C.c_int64()
    _check(lib().nt_circuit_info(circ, C.byref(n), C.byref(G), C.byref(S)))
    return n.value, G.value, S.value


def nt_circuit_set_id(circ, cid: int) -> None:
    _check(lib().nt_circuit_set_id(circ, cid))


def nt_plan_info(circ, prec: int) -> Tuple[int, int, int]:
    a, b, c = C.c_int(), C.c_int(), C.c_int()
    _check(lib().nt_plan_info(circ, prec, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def nt_plan_export(circ, prec: int):
    """Dict with op_gate, op_pass, op_segment, pass_local_mask, segment_reg_mask."""
    npass, nseg, _ = nt_plan_info(circ, prec)
    _, G, _ = nt_circuit_info(circ)
    og = np.zeros(max(G, 1), np.int32)
    op = np.zeros(max(G, 1), np.int32)
    osg = np.zeros(max(G, 1), np.int32)
    pm = np.zeros(max(npass, 1), np.uint64)
    sm = np.zeros(max(nseg, 1), np.uint64)
    _check(lib().nt_plan_export(circ, prec, _ptr(og), _ptr(op), _ptr(osg), _ptr(pm), _ptr(sm)))
    return {"op_gate": og[:G], "op_pass": op[:G], "op_segment": osg[:G],
            "pass_local_mask": pm[:npass], "segment_reg_mask": sm[:nseg]}


# ---- runs ----------------------------------------------------------------------

def nt_run(ctx, circ, seed: int, traj_begin: int, n_traj: int, tau: float,
           fid_out: Optional[np.ndarray] = None, fid_out_ptr: Optional[int] = None):
    """Returns (count, p).  fid_out: host float64 array of n_traj, or
    fid_out_ptr: a device pointer (e.g. torch tensor data_ptr())."""
    cnt = C.c_uint64()
    p = C.c_double()
    if fid_out is not None:
        assert fid_out.dtype == np.float64 and fid_out.size >= n_traj and fid_out.flags.c_contiguous
        fp = _ptr(fid_out)
    elif fid_out_ptr is not None:
        fp = C.c_void_p(fid_out_ptr)
    else:
        fp = None
    _check(lib().nt_run(ctx, circ, seed, traj_begin, n_traj, tau, fp, C.byref(cnt), C.byref(p)))
    return cnt.value, p.value



def nt_run_noalloc(ctx, circ, seed: int, traj_begin: int, n_traj: int, tau: float,
           fid_out: Optional[np.ndarray] = None, fid_out_ptr: Optional[int] = None):
    """nt_run without device allocation (static scratch array).  Returns (count, p).  fid_out: host float64 array of n_traj, or
    fid_out_ptr: a device pointer (e.g. torch tensor data_ptr())."""
    cnt = C.c_uint64()
    p = C.c_double()
    if fid_out is not None:
        assert fid_out.dtype == np.float64 and fid_out.size >= n_traj and fid_out.flags.c_contiguous
        fp = _ptr(fid_out)
    elif fid_out_ptr is not None:
        fp = C.c_void_p(fid_out_ptr)
    else:
        fp = None
    _check(lib().nt_run_noalloc(ctx, circ, seed, traj_begin, n_traj, tau, fp, C.byref(cnt), C.byref(p)))
    return cnt.value, p.value

def nt_run_batch(ctx, circs, seed: int, traj_begin: int, n_traj: int, tau: float,
                 vals_out: Optional[np.ndarray] = None, vals_out_ptr: Optional[int] = None):
    """Many circuits at once.  Returns (counts[n_circ], p[n_circ]).  vals_out:
    host float64 array [n_circ, n_traj], or vals_out_ptr: a device pointer."""
    k = len(circs)
    arr = (C.c_void_p * k)(*[C.c_void_p(h.value if isinstance(h, C.c_void_p) else h) for h in circs])
    cnt = np.zeros(k, np.uint64)
    p = np.zeros(k, np.float64)
    if vals_out is not None:
        assert vals_out.dtype == np.float64 and vals_out.size == k * n_traj and vals_out.flags.c_contiguous
        vp = _ptr(vals_out)
    else:
        vp = C.c_void_p(vals_out_ptr) if vals_out_ptr else None
    _check(lib().nt_run_batch(ctx, arr, k, seed, traj_begin, n_traj, tau, vp, _ptr(cnt), _ptr(p)))
    return cnt, p


def nt_sweep(ctx, circ, rates: Sequence[float], seed: int, n_traj: int, tau: float) -> np.ndarray:
    r = np.ascontiguousarray(rates, np.float64)
    out = np.zeros(len(r), np.float64)
    _check(lib().nt_sweep(ctx, circ, _ptr(r), len(r), seed, n_traj, tau, _ptr(out)))
    return out


def nt_sweep_crossing(ctx, circ, rates: Sequence[float], seed: int, n_traj: int, tau: float, P_target: float):
    """The sweep route: (success probabilities at the rates, the rate where the
    curve, linear in log10 p, first falls below P_target)."""
    r = np.ascontiguousarray(rates, np.float64)
    out = np.zeros(len(r), np.float64)
    ps = C.c_double()
    _check(lib().nt_sweep_crossing(ctx, circ, _ptr(r), len(r), seed, n_traj, tau, P_target, _ptr(out),
                                   C.byref(ps)))
    return out, ps.value


def nt_tolerable_rate(ctx, circ, P_target: float, tol: float, p_lo: float, p_hi: float, seed: int,
                      n_traj: int, tau: float) -> Tuple[float, int]:
    ps = C.c_double()
    npb = C.c_int()
    _check(lib().nt_tolerable_rate(ctx, circ, P_target, tol, p_lo, p_hi, seed, n_traj, tau,
                                   C.byref(ps), C.byref(npb)))
    return ps.value, npb.value


def nt_tolerable_rate_auto(ctx, circ, P_target: float, tol: float, seed: int, n_traj: int, tau: float):
    """Returns (p_star, coarse evaluations, full evaluations, (lo, hi) of the last bracket)."""
    ps = C.c_double()
    kc = C.c_int()
    kf = C.c_int()
    br = (C.c_double * 2)()
    _check(lib().nt_tolerable_rate_auto(ctx, circ, P_target, tol, seed, n_traj, tau, C.byref(ps), C.byref(kc),
                                        C.byref(kf), br))
    return ps.value, kc.value, kf.value, (br[0], br[1])


def nt_tolerable_rate_fig3(ctx, circ, P_target: float, tol: float, seed: int, n_traj: int, tau: float):
    """The paper's steps: exhaustive simulation, then Eq. 5 or Monte Carlo at
    increasing rates.  Returns (p_star, method, Monte Carlo evaluations,
    [P_X, P_Y, P_Z, P_R]); method 0 = Eq. 5, 1 = Monte Carlo."""
    ps = C.c_double()
    meth = C.c_int()
    k = C.c_int()
    p4 = np.zeros(4, np.float64)
    _check(lib().nt_tolerable_rate_fig3(ctx, circ, P_target, tol, seed, n_traj, tau, C.byref(ps), C.byref(meth),
                                        C.byref(k), _ptr(p4)))
    return ps.value, meth.value, k.value, p4


def nt_sample_sites(ctx, circ, seed: int, traj_begin: int, n_traj: int, cap: Optional[int] = None):
    """Returns (offsets[n_traj+1], sites, paulis) drawn on the device."""
    offsets = np.zeros(n_traj + 1, np.uint64)
    n_out = C.c_int64()
    if cap is None:
        _, _, S = nt_circuit_info(circ)
        cap = max(16, n_traj * 4 + 64)
    sites = np.zeros(max(cap, 1), np.int32)
    paulis = np.zeros(max(cap, 1), np.uint8)
    st = lib().nt_sample_sites(ctx, circ, seed, traj_begin, n_traj, _ptr(offsets), _ptr(sites),
                               _ptr(paulis), cap, C.byref(n_out))
    if st == NT_ERR_BUFFER_TOO_SMALL:
        need = n_out.value
        sites = np.zeros(max(need, 1), np.int32)
        paulis = np.zeros(max(need, 1), np.uint8)
        st = lib().nt_sample_sites(ctx, circ, seed, traj_begin, n_traj, _ptr(offsets), _ptr(sites),
                                   _ptr(paulis), need, C.byref(n_out))
    _check(st)
    return offsets, sites[:n_out.value].copy(), paulis[:n_out.value].copy()


def _state_buffer(circ, prec):
    n, _, _ = nt_circuit_info(circ)
    dt = np.complex64 if prec == NT_C64 else np.complex128
    return np.zeros(1 << n, dt)


def nt_final_state(ctx, circ, seed: int, traj: int, prec: int) -> np.ndarray:
    out = _state_buffer(circ, prec)
    _check(lib().nt_final_state(ctx, circ, seed, traj, _ptr(out), out.size))
    return out


def nt_reference_state(ctx, circ, prec: int) -> np.ndarray:
    out = _state_buffer(circ, prec)
    _check(lib().nt_reference_state(ctx, circ, _ptr(out), out.size))
    return out


def nt_set_shortcuts(ctx, flags: int) -> None:
    _check(lib().nt_set_shortcuts(ctx, flags))


def nt_set_criterion(ctx, criterion: int, target: int = 0) -> None:
    _check(lib().nt_set_criterion(ctx, criterion, target))


def nt_exhaustive(ctx, circ, tau: float):
    """Returns (fid[S, 3], P_e[3] (X, Y, Z), P_R)."""
    _, _, S = nt_circuit_info(circ)
    fid = np.zeros((max(S, 1), 3), np.float64)
    pe = np.zeros(3, np.float64)
    pr = C.c_double()
    _check(lib().nt_exhaustive(ctx, circ, tau, _ptr(fid), _ptr(pe), C.byref(pr)))
    return fid[:S], pe, pr.value


def nt_eq4(P_e, P_R: float, E_e) -> float:
    a = np.ascontiguousarray(P_e, np.float64)
    b = np.ascontiguousarray(E_e, np.float64)
    out = C.c_double()
    _check(lib().nt_eq4(_ptr(a), P_R, _ptr(b), C.byref(out)))
    return out.value


def nt_eq5(P_target: float, P_e, P_R: float, units: float) -> float:
    a = np.ascontiguousarray(P_e, np.float64)
    out = C.c_double()
    _check(lib().nt_eq5(P_target, _ptr(a), P_R, units, C.byref(out)))
    return out.value


def nt_success_probability(ctx, circ, seed: int, n_traj: int, tau: float):
    """Returns (P, method) with method 0 = exhaustive + Eq. 4, 1 = Monte Carlo."""
    P = C.c_double()
    m = C.c_int()
    _check(lib().nt_success_probability(ctx, circ, seed, n_traj, tau, C.byref(P), C.byref(m)))
    return P.value, m.value


def nt_timing_enable(ctx, enable: bool) -> None:
    _check(lib().nt_timing_enable(ctx, 1 if enable else 0))


def nt_timing_reset(ctx) -> None:
    _check(lib().nt_timing_reset(ctx))


def nt_timing_read(ctx):
    """(launches, ms_total, algorithmic_bytes_total, updates_total, flops_total)."""
    n = C.c_int64()
    ms, by, up, fl = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    _check(lib().nt_timing_read(ctx, C.byref(n), C.byref(ms), C.byref(by), C.byref(up), C.byref(fl)))
    return n.value, ms.value, by.value, up.value, fl.value


# ---- learned surrogate ------------------------------------------------------------

def _handles(circs):
    return (C.c_void_p * len(circs))(*[C.c_void_p(h.value if isinstance(h, C.c_void_p) else h) for h in circs])


def nt_gnn_create(ctx, seed: int = 0) -> C.c_void_p:
    m = C.c_void_p()
    _check(lib().nt_gnn_create(ctx, seed, C.byref(m)))
    return m


def nt_gnn_destroy(m) -> None:
    lib().nt_gnn_destroy(m)


def nt_gnn_graph(circ):
    """Host graph of a circuit: (x[G, 32], row_ptr[G+1], col[E], glob[4])."""
    nn = C.c_int64()
    ne = C.c_int64()
    _check(lib().nt_gnn_graph(circ, None, None, None, None, C.byref(nn), C.byref(ne)))
    x = np.zeros((nn.value, 32), np.float32)
    rp = np.zeros(nn.value + 1, np.int32)
    col = np.zeros(max(ne.value, 1), np.int32)
    glob = np.zeros(4, np.float32)
    _check(lib().nt_gnn_graph(circ, _ptr(x), _ptr(rp), _ptr(col), _ptr(glob), C.byref(nn), C.byref(ne)))
    return x, rp, col[:ne.value], glob


def nt_gnn_params(m) -> np.ndarray:
    n = C.c_int64()
    _check(lib().nt_gnn_params(m, None, C.byref(n)))
    out = np.zeros(n.value, np.float32)
    _check(lib().nt_gnn_params(m, _ptr(out), C.byref(n)))
    return out


def nt_gnn_set_params(m, params) -> None:
    p = np.ascontiguousarray(params, np.float32)
    _check(lib().nt_gnn_set_params(m, _ptr(p), p.size))


def nt_gnn_set_data(m, circs, labels=None) -> None:
    lab = None if labels is None else np.ascontiguousarray(labels, np.float32)
    if lab is not None:
        assert lab.shape == (len(circs), 13)
    _check(lib().nt_gnn_set_data(m, _handles(circs), len(circs), _ptr(lab)))


def nt_gnn_loss_grad(m, g0: int, g1: int, exact: bool):
    loss = C.c_double()
    n = C.c_int64()
    _check(lib().nt_gnn_params(m, None, C.byref(n)))
    grad = np.zeros(n.value, np.float32)
    _check(lib().nt_gnn_loss_grad(m, g0, g1, int(exact), C.byref(loss), _ptr(grad)))
    return loss.value, grad


def nt_gnn_train(m, epochs: int, batch_graphs: int, lr: float, seed: int = 0) -> np.ndarray:
    out = np.zeros(max(epochs, 1), np.float64)
    _check(lib().nt_gnn_train(m, epochs, batch_graphs, lr, seed, _ptr(out)))
    return out[:epochs]


def nt_gnn_predict(m, circs, exact: bool = False) -> np.ndarray:
    out = np.zeros((len(circs), 13), np.float32)
    _check(lib().nt_gnn_predict(m, _handles(circs), len(circs), int(exact), _ptr(out)))
    return out


def nt_tolerable_rate_guided(ctx, circ, m, P_target: float, tol: float, seed: int, n_traj: int, tau: float):
    """Returns (p_star, n_probes, (p_lo, p_hi))."""
    p = C.c_double()
    k = C.c_int()
    br = np.zeros(2, np.float64)
    _check(lib().nt_tolerable_rate_guided(ctx, circ, m, P_target, tol, seed, n_traj, tau, C.byref(p), C.byref(k),
                                          _ptr(br)))
    return p.value, k.value, (float(br[0]), float(br[1]))


def nt_circuit_set_tile(circ, prec: int, tile_qubits: int) -> None:
    _check(lib().nt_circuit_set_tile(circ, prec, tile_qubits))


def nt_plan_ops(circ, prec: int):
    """Returns (ops run per error-free trajectory, fused blocks)."""
    a, b = C.c_int64(), C.c_int64()
    _check(lib().nt_plan_ops(circ, prec, C.byref(a), C.byref(b)))
    return a.value, b.value


def nt_circuit_set_fusion(circ, prec: int, width: int) -> None:
    _check(lib().nt_circuit_set_fusion(circ, prec, width))


def nt_autotune(ctx, circ, seed: int, n_traj: int):
    """Returns (chosen tile width, milliseconds per candidate)."""
    t = C.c_int()
    ms = np.zeros(3, np.float64)
    _check(lib().nt_autotune(ctx, circ, seed, n_traj, C.byref(t), _ptr(ms)))
    return t.value, ms


def nt_autotune_plan(ctx, circ, seed: int, n_traj: int):
    """Returns (chosen tile width, chosen fusion width, milliseconds per
    candidate, tile-major over fusion widths 2, 3, 4, 1)."""
    t = C.c_int()
    f = C.c_int()
    ms = np.zeros(12, np.float64)
    _check(lib().nt_autotune_plan(ctx, circ, seed, n_traj, C.byref(t), C.byref(f), _ptr(ms), 12))
    return t.value, f.value, ms
