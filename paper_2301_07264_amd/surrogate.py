"""Surrogate pipeline: Monte Carlo labels for many circuits, training, and the
tolerable-rate search with and without the surrogate's bracket.  Argument
marshalling and sequencing only; every step runs in libnisqtol.

Labels: the success probability (fidelity >= tau) at the 13 rates
10^(-5 + j/4) from n_traj trajectories per circuit and rate, a chunk of
circuits of a rate in one batched call, zero-fired trajectories not simulated
(F = 1 exactly either way).  Every circuit has its own circuit id, so every
circuit draws its own errors; the rates share trajectories (nested fired
sets).
"""
from __future__ import annotations

import time
from typing import Dict, List, Sequence

import numpy as np

from . import (GNN_RATES, NT_CRIT_FIDELITY, NT_ERR_NOT_BRACKETED, NT_SHORTCUT_CHECKPOINT, NT_SHORTCUT_REUSE,
               NT_SHORTCUT_ZERO_FIRED, NtError, nt_circuit_set_id, nt_gnn_create, nt_gnn_set_data, nt_gnn_train,
               nt_run_batch, nt_set_criterion, nt_set_error_model, nt_set_shortcuts, nt_sweep_crossing,
               nt_tolerable_rate, nt_tolerable_rate_auto, nt_tolerable_rate_fig3, nt_tolerable_rate_guided)

GRID_LO, GRID_HI = GNN_RATES[0], GNN_RATES[-1]


def make_labels(ctx, handles: Sequence, n_traj: int, seed: int = 0, tau: float = 0.9, chunk: int = 2048,
                id_base: int = 0, progress=None) -> np.ndarray:
    """[n, 13] success probabilities at the surrogate's rates.  Circuits run
    in chunks, every rate for one chunk before the next, so each circuit's
    plan and reference state are built once (the library caches a few
    thousand plans).  Circuit i draws with circuit id id_base + i.
    progress(done, total) is called after each chunk."""
    for i, h in enumerate(handles):
        nt_circuit_set_id(h, id_base + i)
    nt_set_criterion(ctx, NT_CRIT_FIDELITY, 0)
    nt_set_shortcuts(ctx, NT_SHORTCUT_ZERO_FIRED)
    out = np.zeros((len(handles), len(GNN_RATES)), np.float32)
    try:
        for c0 in range(0, len(handles), chunk):
            part = list(handles[c0:c0 + chunk])
            for j, p in enumerate(GNN_RATES):
                nt_set_error_model(ctx, p / 3, p / 3, p / 3)
                _, pj = nt_run_batch(ctx, part, seed, 0, n_traj, tau)
                out[c0:c0 + len(part), j] = pj
            if progress:
                progress(c0 + len(part), len(handles))
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


ROUTES = ("sweep", "full", "paper", "auto", "surrogate")


def tolerable_rate_searches(ctx, h, model, P_target: float = 0.66, tol: float = 0.01, n_traj: int = 2048,
                            seed: int = 0, tau: float = 0.9, routes: Sequence[str] = ROUTES) -> Dict[str, dict]:
    """Time to the tolerable rate of one circuit by five routes, each one
    library call:
    'sweep'     the plain 13-point Monte Carlo sweep, crossing interpolated
                (nt_sweep_crossing);
    'full'      the regula-falsi search over the whole grid [1e-5, 1e-2]
                (nt_tolerable_rate);
    'paper'     the paper's steps: exhaustive single errors, Eq. 5 when at
                most one error is tolerable, else Monte Carlo at increasing
                rates (nt_tolerable_rate_fig3);
    'auto'      no model: brackets from the zero-error bound, on a fifth of
                the trajectories, then all of them (nt_tolerable_rate_auto);
    'surrogate' one probe at the surrogate's predicted crossing, then the
                search in brackets around it (nt_tolerable_rate_guided).
    Only the bit-identical short-cuts are on (zero-fired, checkpoint, reuse);
    the reuse store is emptied before each route, so no route profits from
    another's probes.  'probes' counts Monte Carlo evaluations; 'work' counts
    them in units of n_traj trajectories (the auto route's first stage runs
    a fifth of them)."""
    flags = NT_SHORTCUT_ZERO_FIRED | NT_SHORTCUT_CHECKPOINT | NT_SHORTCUT_REUSE

    def fresh():
        nt_set_shortcuts(ctx, flags)   # also empties the reuse store

    def timed(name, fn):
        fresh()
        t0 = time.perf_counter()
        try:
            r = fn()
        except NtError as e:
            if e.status != NT_ERR_NOT_BRACKETED:
                raise
            r = {"p_star": float("nan"), "probes": -1, "work": float("nan")}
        r["seconds"] = time.perf_counter() - t0
        res[name] = r

    res = {}
    try:
        def sweep():
            _, p = nt_sweep_crossing(ctx, h, GNN_RATES, seed, n_traj, tau, P_target)
            return {"p_star": p, "probes": len(GNN_RATES), "work": float(len(GNN_RATES))}

        def full():
            p, k = nt_tolerable_rate(ctx, h, P_target, tol, GRID_LO, GRID_HI, seed, n_traj, tau)
            return {"p_star": p, "probes": k, "work": float(k)}

        def paper():
            p, method, k, _ = nt_tolerable_rate_fig3(ctx, h, P_target, tol, seed, n_traj, tau)
            return {"p_star": p, "probes": k, "work": float(k), "method": method}

        def auto():
            p, kc, kf, br = nt_tolerable_rate_auto(ctx, h, P_target, tol, seed, n_traj, tau)
            return {"p_star": p, "probes": kc + kf, "work": kf + kc * max(1, n_traj // 5) / n_traj,
                    "bracket": br}

        def guided():
            p, k, br = nt_tolerable_rate_guided(ctx, h, model, P_target, tol, seed, n_traj, tau)
            return {"p_star": p, "probes": k, "work": float(k), "bracket": br}

        for name, fn in (("sweep", sweep), ("full", full), ("paper", paper), ("auto", auto),
                         ("surrogate", guided)):
            if name in routes:
                timed(name, fn)
    finally:
        nt_set_shortcuts(ctx, 0)
    return res
