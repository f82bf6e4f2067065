"""Surrogate pipeline: Monte Carlo labels for many circuits, training, and the
tolerable-rate search with and without the surrogate's bracket.  Argument
marshalling and sequencing only; every step runs in libnisqtol.

Labels: the success probability (fidelity >= tau) at the 13 rates
10^(-5 + j/4) from n_traj trajectories per circuit and rate, all circuits of
a rate in one batched call, zero-fired trajectories not simulated (F = 1
exactly either way).  Circuit i uses circuit id i, so every circuit draws its
own errors; the rates share trajectories (nested fired sets).
"""
from __future__ import annotations

import math
import time
from typing import Dict, List, Sequence

import numpy as np

from . import (GNN_RATES, NT_CRIT_FIDELITY, NT_ERR_NOT_BRACKETED, NT_SHORTCUT_CHECKPOINT,
               NT_SHORTCUT_LAST_ERROR, NT_SHORTCUT_REUSE, NT_SHORTCUT_ZERO_FIRED, NtError, nt_circuit_info, nt_circuit_set_id,
               nt_exhaustive, nt_eq5, nt_gnn_create, nt_gnn_predict, nt_gnn_set_data, nt_gnn_train,
               nt_run_batch, nt_set_criterion, nt_set_error_model, nt_set_shortcuts, nt_sweep,
               nt_tolerable_rate, nt_tolerable_rate_guided)

GRID_LO, GRID_HI = GNN_RATES[0], GNN_RATES[-1]


def make_labels(ctx, handles: Sequence, n_traj: int, seed: int = 0, tau: float = 0.9) -> np.ndarray:
    """[n, 13] success probabilities at the surrogate's rates."""
    for i, h in enumerate(handles):
        nt_circuit_set_id(h, i)
    nt_set_criterion(ctx, NT_CRIT_FIDELITY, 0)
    nt_set_shortcuts(ctx, NT_SHORTCUT_ZERO_FIRED)
    out = np.zeros((len(handles), len(GNN_RATES)), np.float32)
    try:
        for j, p in enumerate(GNN_RATES):
            nt_set_error_model(ctx, p / 3, p / 3, p / 3)
            _, pj = nt_run_batch(ctx, list(handles), seed, 0, n_traj, tau)
            out[:, j] = pj
    finally:
        nt_set_shortcuts(ctx, 0)
    return out


def train(ctx, handles: Sequence, labels: np.ndarray, epochs: int = 60, batch_graphs: int = 32,
          lr: float = 2e-3, seed: int = 0):
    """A trained model and its per-epoch training loss."""
    m = nt_gnn_create(ctx, seed)
    nt_gnn_set_data(m, list(handles), labels)
    losses = nt_gnn_train(m, epochs, batch_graphs, lr, seed)
    return m, losses


def _interp_crossing(rates: Sequence[float], P: Sequence[float], target: float) -> float:
    """Rate where the piecewise-linear (in log10 p) curve first falls below
    target; the grid end when it never does."""
    for k in range(len(rates) - 1):
        if P[k] >= target > P[k + 1]:
            x0, x1 = math.log10(rates[k]), math.log10(rates[k + 1])
            t = (P[k] - target) / (P[k] - P[k + 1])
            return 10.0 ** (x0 + t * (x1 - x0))
    return rates[0] if P[0] < target else rates[-1]


def tolerable_rate_searches(ctx, h, model, P_target: float = 0.66, tol: float = 0.01, n_traj: int = 2048,
                            seed: int = 0, tau: float = 0.9) -> Dict[str, dict]:
    """Time to the tolerable rate of one circuit by five routes:
    'sweep'     the plain 13-point Monte Carlo sweep, crossing interpolated;
    'full'      the regula-falsi search over the whole grid [1e-5, 1e-2];
    'eq5'       exhaustive single errors, Eq. 5's rate, search in [p/3, 3p]
                (whole grid when that fails);
    'surrogate' one probe at the surrogate's predicted crossing, then the
                search in brackets around it (whole grid fallback);
    'bound'     no model: the bracket [p0/2, 2 p0] from the zero-error bound
                p0 = 1 - P*^(1/S) (P(p) >= (1 - p)^S), then [p0/2, 1/G],
                then the whole grid.
    Short-cuts (zero-fired, checkpoint, last error) are on for every route;
    values are reused only within a route (the store is cleared before each),
    so no route profits from another's probes."""
    flags = NT_SHORTCUT_ZERO_FIRED | NT_SHORTCUT_CHECKPOINT | NT_SHORTCUT_LAST_ERROR | NT_SHORTCUT_REUSE

    def fresh():
        nt_set_shortcuts(ctx, flags)   # also empties the reuse store

    res = {}
    try:
        fresh()
        t0 = time.perf_counter()
        P = nt_sweep(ctx, h, GNN_RATES, seed, n_traj, tau)
        res["sweep"] = {"seconds": time.perf_counter() - t0, "probes": len(GNN_RATES),
                        "p_star": _interp_crossing(GNN_RATES, P, P_target)}

        def search(lo, hi):
            return nt_tolerable_rate(ctx, h, P_target, tol, lo, hi, seed, n_traj, tau)

        fresh()
        t0 = time.perf_counter()
        try:
            p, k = search(GRID_LO, GRID_HI)
        except NtError as e:
            if e.status != NT_ERR_NOT_BRACKETED:
                raise
            p, k = float("nan"), -1
        res["full"] = {"seconds": time.perf_counter() - t0, "probes": k, "p_star": p}

        fresh()
        t0 = time.perf_counter()
        _, _, S = nt_circuit_info(h)
        _, pe, pr = nt_exhaustive(ctx, h, tau)
        probes = 0
        try:
            p5 = nt_eq5(P_target, pe, pr, S)
        except NtError:
            p5 = float("nan")
        p = float("nan")
        done = False
        if math.isfinite(p5) and p5 > 0:
            lo, hi = max(GRID_LO, p5 / 3), min(GRID_HI, p5 * 3)
            if lo < hi:
                try:
                    p, k = search(lo, hi)
                    probes += k
                    done = True
                except NtError as e:
                    if e.status != NT_ERR_NOT_BRACKETED:
                        raise
                    probes += 2
        if not done:
            try:
                p, k = search(GRID_LO, GRID_HI)
                probes += k
            except NtError as e:
                if e.status != NT_ERR_NOT_BRACKETED:
                    raise
        res["eq5"] = {"seconds": time.perf_counter() - t0, "probes": probes, "p_star": p, "p_eq5": p5}

        fresh()
        t0 = time.perf_counter()
        try:
            p, k, br = nt_tolerable_rate_guided(ctx, h, model, P_target, tol, seed, n_traj, tau)
        except NtError as e:
            if e.status != NT_ERR_NOT_BRACKETED:
                raise
            p, k, br = float("nan"), -1, (GRID_LO, GRID_HI)
        res["surrogate"] = {"seconds": time.perf_counter() - t0, "probes": k, "p_star": p, "bracket": br}

        fresh()
        t0 = time.perf_counter()
        _, G, S = nt_circuit_info(h)
        p0 = 1.0 - P_target ** (1.0 / max(S, 1))
        lo0 = max(GRID_LO, p0 / 2)
        tries = [[lo0, min(2 * p0, 1.0 / max(G, 1), GRID_HI)], [lo0, min(1.0 / max(G, 1), GRID_HI)],
                 [GRID_LO, GRID_HI]]
        tries = [t for i, t in enumerate(tries) if t[0] < t[1] and t not in tries[:i]]
        p, probes, br = float("nan"), 0, tries[-1]
        for br in tries:
            try:
                p, k = search(br[0], br[1])
                probes += k
                break
            except NtError as e:
                if e.status != NT_ERR_NOT_BRACKETED:
                    raise
                probes += 2
        res["bound"] = {"seconds": time.perf_counter() - t0, "probes": probes, "p_star": p, "bracket": br, "p0": p0}
    finally:
        nt_set_shortcuts(ctx, 0)
    return res
