"""Benchmark: trajectory amplitude-updates/s of the Monte Carlo Pauli-error
simulation on one MI355X, with the roofline of the gate-pass kernel and the
CPU oracle timed beside it.

Workload (default, --workload ghz_qft_layers24): the 24-qubit circuit (GHZ
preparation, full QFT, 50 random rotation + CNOT layers; G = 2136 gates,
S = 3047 error sites), complex64 amplitudes with FP64 overlaps / norms /
counts, uniform Pauli error rate cycling over the 13 rates 10^(-5 + j/4).
--workload qaoa3reg30: the 30-qubit alternating-layer circuit on a random
3-regular graph (G = 330, S = 510, 8 GiB complex64 state), rates 10^(-5+j/3).
--workload batch512: 512 independent random-layer instances (n uniform in
10..20, 10..100 layers, circuit id = instance seed), 256 trajectories each at
p = 1e-3, all in one batched call per step.
One step = one batch of B trajectories through the whole path: Philox
error-site sampling, every gate pass, fused fidelity scoring and the success
count.  Inputs (circuit plan and reference state) are resident in HBM before
the timed region.

Unit of work: one amplitude-update = one gate applied to one amplitude of one
trajectory (N * G * 2^n per run); Pauli errors are folded and not counted.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
# Vector ALU peaks (published, MI355X): FP32 157.3 TFLOP/s, FP64 78.6 TFLOP/s
# (256 CUs x 4 SIMDs x 2.4 GHz; a wave64 FP32 FMA with VGPR operands issues
# about every 2 cycles per SIMD, an FP64 FMA every 4).  Complex64 amplitudes
# are FP32 arithmetic, complex128 FP64.
ALU_PEAK_TFLOPS = {"c64": 157.3, "c128": 78.6}

# HBM bytes per gate-pass launch from rocprofv3 FETCH_SIZE / WRITE_SIZE
# (calibrated against a device copy), per workload, valid for the kernel
# source and the plan (tile width, ops per trajectory, passes) they were
# taken on (profiles/hbm_traffic_*.md).
MEASURED_TRAFFIC = {
    ("ghz_qft_layers24", "c64", 32): {
        "bytes_per_launch": 8.416e9,
        "passes": 43, "tile_qubits": 12, "ops": 984,
        "kernel_sha256": "1b7fccad597628a0698696c8efcee173ef29e1ce4d28f31bc485044d7e684b7e",
    },
    ("qaoa3reg30", "c64", 4): {
        "bytes_per_launch": 6.560e10,
        "passes": 11, "tile_qubits": 12, "ops": 216,
        "kernel_sha256": "1b7fccad597628a0698696c8efcee173ef29e1ce4d28f31bc485044d7e684b7e",
    },
}


_COPY_GBS = None


def device_copy_gbs(nbytes: int = 4 << 30) -> float:
    """Practical HBM rate of this machine: a device-to-device copy of nbytes
    (read + write bytes over the best of five, HIP events), measured once per
    process after the timed region."""
    global _COPY_GBS
    if _COPY_GBS is None:
        import torch
        x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        y.copy_(x)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = float("inf")
        for _ in range(5):
            e0.record()
            y.copy_(x)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        del x, y
        torch.cuda.empty_cache()
        _COPY_GBS = 2.0 * nbytes / (best / 1e3) / 1e9
    return _COPY_GBS


def kernel_sha256():
    import hashlib
    path = os.path.join(ROOT, "paper_2301_07264_amd", "csrc", "kernels.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["ghz_qft_layers24", "qaoa3reg30", "batch512", "surrogate"],
                    default="ghz_qft_layers24")
    ap.add_argument("--train-circuits", type=int, default=2048)
    ap.add_argument("--heldout-circuits", type=int, default=256)
    ap.add_argument("--label-traj", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=80)
    ap.add_argument("--eval-circuits", type=int, default=16)
    ap.add_argument("--routes", type=str, default="sweep,full,paper,auto,surrogate",
                    help="surrogate workload: tolerable-rate routes timed on the held-out circuits")
    ap.add_argument("--labels-out", type=str, default=None,
                    help="surrogate workload: write the labels (npz) and stop after labelling")
    ap.add_argument("--labels-in", type=str, default=None,
                    help="surrogate workload: read labels written by --labels-out instead of labelling "
                         "(several files, comma-separated, for the parts of --label-part)")
    ap.add_argument("--label-part", type=str, default=None,
                    help="surrogate workload with --labels-out: label only part K of M (K/M) of the circuits "
                         "(training then held-out, in order)")
    ap.add_argument("--batch", type=int, default=0, help="trajectories per step (0: 32 for 24 qubits, 4 for 30)")
    ap.add_argument("--prec", choices=["c64", "c128"], default="c64")
    ap.add_argument("--fusion", type=int, choices=[0, 1, 2, 3, 4], default=0,
                    help="gate fusion of the plan: 0 automatic, 1 none, 2 two-qubit blocks and diagonal "
                         "runs, 3 blocks only, 4 diagonal runs only")
    ap.add_argument("--no-autotune", action="store_true",
                    help="with --fusion 0: keep the library's default plan instead of the plan autotuner's "
                         "choice of tile width and fusion (nt_autotune_plan, run before the timed region)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-traj", type=int, default=1, help="oracle trajectories timed on the host")
    ap.add_argument("--traffic", type=str, default=None,
                    help="JSON file with measured HBM bytes per pass launch (rocprofv3 counters)")
    ap.add_argument("--ttr", dest="ttr", action="store_true", default=None,
                    help="time the tolerable-rate search (P* = 0.66 +- 0.01, 10^4 trajectories per probe, "
                         "exact short-cuts on); default on for the 24-qubit workload")
    ap.add_argument("--no-ttr", dest="ttr", action="store_false", help="skip the tolerable-rate search")
    ap.add_argument("--ttr-traj", type=int, default=10000)
    ap.add_argument("--sweep-traj", type=int, default=1000,
                    help="trajectories of the timed 13-point sweep baseline (0: skip)")
    ap.add_argument("--no-sub", action="store_true",
                    help="skip the 30-qubit sub-record of the default run")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a device copy of this many bytes (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.ttr is None:
        args.ttr = args.workload == "ghz_qft_layers24"
    if args.copy_bytes:
        import torch
        x = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: one GPU only; --gpus {args.gpus} is not supported "
              f"(trajectories would shard by range with one count all-reduce; not built).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2301_07264_amd as P
    import workloads as W

    P.lib()
    if args.workload == "batch512":
        return bench_batch(args, P, W)
    if args.workload == "surrogate":
        return bench_surrogate(args, P, W)
    out = bench_single(args, P, W, args.workload, False)
    if args.workload == "ghz_qft_layers24" and not args.no_sub:
        # the 30-qubit workload beside it (8 GiB states, HBM-bound): its own
        # amplitude-update rate and roofline, no search and no CPU leg
        print("bench: 30-qubit workload (sub-record) ...", file=sys.stderr, flush=True)
        sub = bench_single(args, P, W, "qaoa3reg30", True)
        out["sub_records"] = {"qaoa3reg30": {k: sub[k] for k in ("value", "unit", "ms_per_step", "steps", "warmup",
                                                               "config", "roofline")}}
        # the 512 batched uneven instances (n 10..20) beside them
        print("bench: batched workload (sub-record) ...", file=sys.stderr, flush=True)
        bsub = bench_batch(args, P, W, sub=True)
        out["sub_records"]["batch512"] = {k: bsub[k] for k in ("value", "unit", "ms_per_step", "steps", "warmup",
                                                              "config", "roofline")}
    print(json.dumps(out), flush=True)


def bench_single(args, P, W, workload, sub):
    """One gate-pass workload: `steps` timed batches of trajectories after
    `warmup` untimed ones; sub: a sub-record (5 steps, 1 warmup, default
    batch, no search and no CPU leg)."""
    import numpy as np
    import torch

    steps, warmup = (5, 1) if sub else (args.steps, args.warmup)
    if workload == "ghz_qft_layers24":
        circ = W.config1()
        rates = W.rates_config1()
        wl = "ghz+qft+50 random layers, 24 qubits, G=2136, S=3047, 13 rates 1e-5..1e-2 cycled per step"
        B = (0 if sub else args.batch) or 32
    else:
        circ = W.config4()
        rates = W.rates_config4()
        wl = "alternating layers on a random 3-regular graph, 30 qubits, G=330, S=510, 7 rates 1e-5..1e-3 cycled per step"
        B = (0 if sub else args.batch) or 4
    n, G, S = circ.n, circ.G, circ.S
    prec = P.NT_C64 if args.prec == "c64" else P.NT_C128
    tau = 0.9

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = P.nt_create(0, stream.cuda_stream)
    h = P.nt_circuit_load(ctx, circ)
    P.nt_circuit_set_fusion(h, prec, args.fusion)
    P.nt_set_precision(ctx, prec)
    P.nt_set_max_batch(ctx, B)
    tuned = None
    if args.fusion == 0 and not args.no_autotune:
        # the plan autotuner picks tile width and fusion on one batch at the
        # middle rate (untimed set-up, like the plan upload)
        pm = float(rates[len(rates) // 2])
        P.nt_set_error_model(ctx, pm / 3, pm / 3, pm / 3)
        tL, tf, tms = P.nt_autotune_plan(ctx, h, 0, B)
        tuned = {"tile_qubits": tL, "fusion": tf, "rate": pm, "trajectories": B,
                 "ms_per_candidate": [round(float(x), 3) for x in tms],
                 "candidates": "tile widths from the largest down, each with fusion 2, 3, 4, 1"}
        print(f"bench: plan autotuner chose tile {tL}, fusion {tf}", file=sys.stderr, flush=True)
    n_pass, n_seg, L = P.nt_plan_info(h, prec)
    n_ops, n_blocks = P.nt_plan_ops(h, prec)

    fid_dev = torch.empty(B, dtype=torch.float64, device="cuda:0")
    state = {"t": 0, "step": 0, "count": 0}

    def step():
        p = float(rates[state["step"] % len(rates)])
        P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
        cnt, _ = P.nt_run(ctx, h, 0, state["t"], B, tau, fid_out_ptr=fid_dev.data_ptr())
        state["t"] += B
        state["step"] += 1
        state["count"] += cnt

    # resident inputs: plan upload + reference state happen here
    P.nt_set_error_model(ctx, 0, 0, 0)
    P.nt_run(ctx, h, 0, 0, 1, tau)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()

    state["count"] = 0
    P.nt_timing_enable(ctx, True)
    P.nt_timing_reset(ctx)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    launches, pass_ms, pass_bytes, pass_updates, pass_flops = P.nt_timing_read(ctx)
    P.nt_timing_enable(ctx, False)

    n_traj = steps * B
    updates = float(n_traj) * G * (1 << n)
    value = updates / (ms / 1e3)
    amp = 8 if prec == P.NT_C64 else 16
    # algorithmic bytes of one pass launch: B states read + written once
    bytes_per_launch = pass_bytes / max(launches, 1)
    avg_launch_ms = pass_ms / max(launches, 1)
    achieved = bytes_per_launch / (avg_launch_ms / 1e3) / 1e9
    flops_per_launch = pass_flops / max(launches, 1)
    achieved_tf = flops_per_launch / (avg_launch_ms / 1e3) / 1e12
    traffic = None
    if args.traffic and os.path.exists(args.traffic):
        with open(args.traffic) as f:
            traffic = json.load(f).get("bytes_per_launch")
    else:
        m = MEASURED_TRAFFIC.get((workload, args.prec, B))
        if (m and m["kernel_sha256"] == kernel_sha256() and m["passes"] == n_pass and m["tile_qubits"] == L
                and m["ops"] == n_ops):
            traffic = m["bytes_per_launch"]

    ttr = None
    sweep = None
    if args.ttr and not sub:
        # Time-to-tolerable-rate with the bit-identical short-cuts: zero-fired
        # trajectories are not simulated, a trajectory starts at the error-free
        # checkpoint before its first error, and a trajectory whose fired set
        # at a probe equals one it had at an earlier probe (same count: the
        # sets are nested across rates) reuses that value.
        flags = P.NT_SHORTCUT_ZERO_FIRED | P.NT_SHORTCUT_CHECKPOINT | P.NT_SHORTCUT_REUSE
        P.nt_set_shortcuts(ctx, flags)
        P.nt_set_max_batch(ctx, 0)
        print("bench: timing the tolerable-rate search ...", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # nt_tolerable_rate_auto: Illinois regula falsi in log10 p, first on
        # N/5 of the trajectories in brackets from the zero-error bound
        # p0 = 1 - P*^(1/S) (P(p) >= (1 - p)^S: error-free trajectories
        # succeed) and 1/G (Sec. IV-D), then on all N from the coarse answer
        # (one probe, one Newton step, then a bracket between them).
        S = circ.S
        p0 = 1.0 - 0.66 ** (1.0 / S)
        N_full = args.ttr_traj
        N_coarse = max(1, N_full // 5)
        p_star, k_c, k_f, bracket = P.nt_tolerable_rate_auto(ctx, h, 0.66, 0.01, 0, N_full, tau)
        probes = k_c + k_f
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ttr = {"seconds": dt, "p_star": p_star, "probes": probes,
               "probes_by_stage": {f"{N_coarse} trajectories": k_c, f"{N_full} trajectories": k_f},
               "P_target": 0.66, "tol": 0.01, "trajectories_per_probe": N_full, "bracket": bracket,
               "search": "Illinois in log10 p; N/5 trajectories, then all N from the coarse answer",
               "shortcuts": "bit-identical only: zero-fired trajectories skipped, start at the first-error "
                            "checkpoint, values of fired sets already simulated at an earlier probe reused",
               "one_over_G": 1.0 / G, "zero_error_bound": p0}
        # The baseline beside it: the plain 13-point Monte Carlo sweep with the
        # same short-cuts (store emptied first), crossing interpolated in
        # log10 p.  Timed on the first args.sweep_traj trajectories; every
        # trajectory costs the same in expectation, so the time at N_full
        # trajectories is that time scaled by N_full / args.sweep_traj.
        if args.sweep_traj > 0:
            P.nt_set_shortcuts(ctx, flags)          # empties the reuse store
            print(f"bench: timing the 13-point sweep on {args.sweep_traj} trajectories ...", file=sys.stderr,
                  flush=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Psw, p_sw = P.nt_sweep_crossing(ctx, h, rates, 0, args.sweep_traj, tau, 0.66)
            torch.cuda.synchronize()
            dts = time.perf_counter() - t0
            sweep = {"seconds_measured": dts, "trajectories_measured": args.sweep_traj,
                     "seconds_at_ttr_trajectories": dts * N_full / args.sweep_traj,
                     "scaled": args.sweep_traj != N_full, "rates": len(rates),
                     "p_star_interpolated": p_sw, "P": [float(x) for x in Psw],
                     "ttr_speedup": (dts * N_full / args.sweep_traj) / dt if dt > 0 else None}
        # The same search with the last-error short-cut added (a trajectory
        # is scored right after the pass of its last error, against the
        # error-free state there): exact in arithmetic, not bit for bit, so
        # it is reported apart from the number above.
        P.nt_set_shortcuts(ctx, flags | P.NT_SHORTCUT_LAST_ERROR)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p_le, kc_le, kf_le, _ = P.nt_tolerable_rate_auto(ctx, h, 0.66, 0.01, 0, N_full, tau)
        torch.cuda.synchronize()
        ttr["with_last_error_shortcut"] = {"seconds": time.perf_counter() - t0, "p_star": p_le,
                                           "probes": kc_le + kf_le,
                                           "note": "exact in arithmetic only: fidelities differ from the full "
                                                   "run by rounding"}
        P.nt_set_shortcuts(ctx, 0)

    cpu = None
    if not args.no_cpu_baseline and not sub:
        import oracle
        p = float(rates[len(rates) // 2])
        if n <= 26:
            t0 = time.perf_counter()
            _, _, threads = oracle.run(circ, p / 3, p / 3, p / 3, 0, 0, args.cpu_traj, tau, return_threads=True)
            dt = time.perf_counter() - t0
            # the oracle simulates the error-free reference and then each trajectory
            cpu = {"value": (args.cpu_traj + 1) * G * (1 << n) / dt, "unit": "amplitude-updates/s",
                   "cores": threads, "kind": "oracle",
                   "sample": f"error-free reference + {args.cpu_traj} trajectory of the same {n}-qubit circuit "
                             f"at p={p:.3g}, FP64, OpenMP inside each gate, {dt:.1f} s wall"}
        else:
            # a full 2^30-amplitude FP64 trajectory takes tens of minutes on the
            # host: time the oracle on the circuit's first gates instead
            k = 12
            prefix = W.Circuit(n, circ.gates[:k], circ.name + "_prefix")
            t0 = time.perf_counter()
            oracle.final_state_pattern(prefix, [], [])
            dt = time.perf_counter() - t0
            import os as _os
            cpu = {"value": k * (1 << n) / dt, "unit": "amplitude-updates/s",
                   "cores": _os.cpu_count(), "kind": "oracle",
                   "sample": f"first {k} gates of the {n}-qubit circuit, one FP64 state, OpenMP inside "
                             f"each gate, {dt:.1f} s wall"}

    hbm_frac = achieved / HBM_PEAK_GBS
    alu_peak = ALU_PEAK_TFLOPS[args.prec]
    alu_frac = achieved_tf / alu_peak
    copy_gbs = device_copy_gbs()
    hbm_view = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": hbm_frac, "traffic": traffic,
                "device_copy_GBps": copy_gbs, "frac_of_device_copy": achieved / copy_gbs}
    alu_view = {"bound": "alu", "achieved": achieved_tf, "peak": alu_peak, "unit": "TFLOP/s",
                "frac": alu_frac, "traffic": traffic}
    # the binding roofline is the one the kernel is closest to
    roofline = dict(alu_view if alu_frac >= hbm_frac else hbm_view)
    roofline.update({"kernel": "k_pass", "launches": launches, "avg_launch_ms": avg_launch_ms,
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "algorithmic_flops_per_launch": flops_per_launch,
                     "pass_kernel_share_of_step": pass_ms / ms if ms > 0 else None,
                     "hbm_view": hbm_view, "alu_view": alu_view})
    out = {
        "metric": "trajectory amplitude-updates/s (% HBM peak); time-to-tolerable-error-rate ±0.01",
        "value": value,
        "unit": "amplitude-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64" if prec == P.NT_C64 else "c128",
        "data": "synthetic",
        "config": {"workload": wl,
                   "trajectories_per_step": B, "n_qubits": n, "gates": G, "sites": S,
                   "amplitudes": args.prec, "passes_per_trajectory": n_pass, "segments": n_seg,
                   "tile_qubits": L, "ops_per_trajectory": n_ops, "fused_ops": n_blocks,
                   "plan_autotune": tuned,
                   "parallelism": "single GPU, trajectory batch"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_tolerable_rate": ttr,
        "sweep_baseline": sweep,
        "successes": state["count"],
        "trajectories": n_traj,
    }
    P.nt_circuit_free(h)
    P.nt_destroy(ctx)
    return out


def bench_surrogate(args, P, W):
    """Learned surrogate: labels for the training circuits (n 8..16, 5..80
    layers), training, held-out accuracy, and the time to the tolerable rate
    (P* = 0.66 +- 0.01) of held-out circuits with and without its bracket."""
    import numpy as np
    import torch
    from paper_2301_07264_amd import surrogate as SG

    torch.cuda.set_device(0)
    ctx = P.nt_create(0)
    P.nt_set_precision(ctx, P.NT_C64)
    ntr, nho = args.train_circuits, args.heldout_circuits
    t0 = time.perf_counter()
    train_c, held_c, th, hh = [], [], [], []
    for s in range(ntr + nho):
        c = W.config3_circuit(s) if s < ntr else W.config3_circuit(100000 + s - ntr)
        (train_c if s < ntr else held_c).append(c)
        (th if s < ntr else hh).append(P.nt_circuit_load(ctx, c))
        if (s + 1) % 2000 == 0:
            print(f"bench: {s + 1}/{ntr + nho} circuits generated, {time.perf_counter() - t0:.0f} s",
                  file=sys.stderr, flush=True)
    upd = sum(c.G * (1 << c.n) for c in train_c + held_c) * args.label_traj * 13
    t_label = None
    if args.labels_in:
        lab = np.full((ntr + nho, 13), np.nan, np.float32)
        t_label = 0.0
        for path in args.labels_in.split(","):
            z = np.load(path)
            assert (int(z["train_circuits"]), int(z["heldout_circuits"]), int(z["label_traj"])) == (
                ntr, nho, args.label_traj), path
            a, b = int(z["first"]), int(z["end"])
            lab[a:b] = z["labels"]
            t_label += float(z["seconds"])
        assert not np.isnan(lab).any(), "labels missing for some circuits"
        lab_tr, lab_ho = lab[:ntr], lab[ntr:]
        # circuit ids as labelling set them
        for i, h in enumerate(th + hh):
            P.nt_circuit_set_id(h, i)
    else:
        first, end = 0, ntr + nho
        if args.label_part:
            k, m = (int(x) for x in args.label_part.split("/"))
            first, end = (ntr + nho) * k // m, (ntr + nho) * (k + 1) // m
        print(f"bench: labels for circuits [{first}, {end}) of {ntr} + {nho} ...", file=sys.stderr, flush=True)

        def prog(done, total):
            print(f"bench: labelled {done}/{total} circuits, {time.perf_counter() - t0:.0f} s",
                  file=sys.stderr, flush=True)

        t0 = time.perf_counter()
        lab = SG.make_labels(ctx, (th + hh)[first:end], args.label_traj, seed=1, id_base=first, progress=prog,
                             chunk=1024)
        t_label = time.perf_counter() - t0
        if args.labels_out:
            np.savez(args.labels_out, labels=lab, first=first, end=end, seconds=t_label, train_circuits=ntr,
                     heldout_circuits=nho, label_traj=args.label_traj)
            print(json.dumps({"labels": args.labels_out, "seconds": t_label, "circuits": [first, end],
                              "train_circuits": ntr, "heldout_circuits": nho, "label_traj": args.label_traj,
                              "amplitude_updates_logical": sum(c.G * (1 << c.n) for c in (train_c + held_c)[first:end])
                              * args.label_traj * 13}), flush=True)
            return
        lab_tr, lab_ho = lab[:ntr], lab[ntr:]
    print(f"bench: training ({args.epochs} epochs) ...", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    model, losses = SG.train(ctx, th, lab_tr, epochs=args.epochs)
    t_train = time.perf_counter() - t0
    pred = P.nt_gnn_predict(model, hh)
    mse_ho = float(((pred - lab_ho) ** 2).mean())
    base_ho = float(((lab_tr.mean(0)[None, :] - lab_ho) ** 2).mean())
    # evaluation on held-out circuits whose tolerable rate lies inside the grid
    ev = [i for i in range(nho) if lab_ho[i, 0] >= 0.66 > lab_ho[i, -1]][:args.eval_circuits]
    routes = {}
    routes_on = tuple(args.routes.split(","))
    t0 = time.perf_counter()
    for k, i in enumerate(ev):
        if k % 25 == 0:
            print(f"bench: tolerable-rate routes, held-out circuit {k + 1}/{len(ev)}, "
                  f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
        r = SG.tolerable_rate_searches(ctx, hh[i], model, n_traj=2048, seed=3, routes=routes_on)
        for name, v in r.items():
            routes.setdefault(name, []).append(v)
    summary = {name: {"mean_seconds": float(np.mean([x["seconds"] for x in v])),
                      "mean_probes": float(np.mean([x["probes"] for x in v])),
                      "p_star_median": float(np.median([x["p_star"] for x in v]))}
               for name, v in routes.items()}
    for name, v in routes.items():
        summary[name]["mean_work"] = float(np.mean([x["work"] for x in v]))
        summary[name]["not_bracketed"] = int(sum(1 for x in v if x["probes"] < 0))
        if name != "sweep" and "sweep" in routes:
            d = [abs(np.log10(x["p_star"]) - np.log10(y["p_star"])) for x, y in zip(v, routes["sweep"])
                 if x["p_star"] > 0 and y["p_star"] > 0]
            summary[name]["median_abs_log10_ratio_to_sweep"] = float(np.median(d)) if d else None
    sp = summary.get("surrogate", {}).get("mean_seconds")
    if sp:
        for base in ("sweep", "auto", "full", "paper"):
            if base in summary:
                summary["surrogate"][f"speedup_vs_{base}"] = summary[base]["mean_seconds"] / sp
    out = {
        "metric": "time-to-tolerable-error-rate ±0.01 (held-out circuits, mean)",
        "value": sp, "unit": "s", "n_gpus": 1, "steps": len(ev), "warmup": 0,
        "ms_per_step": sp * 1e3 if sp else None, "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "c64 (simulation), bf16/fp32 (network)", "data": "synthetic",
        "config": {"workload": f"surrogate: {ntr} training + {nho} held-out random-layer circuits, n 8..16, "
                               f"5..80 layers; labels from {args.label_traj} trajectories at 13 rates; "
                               f"searches with 2048 trajectories per probe",
                   "parallelism": "single GPU"},
        "labels": {"seconds": t_label, "amplitude_updates_logical": upd},
        "training": {"seconds": t_train, "epochs": args.epochs, "loss_first": float(losses[0]),
                     "loss_last": float(losses[-1])},
        "heldout": {"mse": mse_ho, "mse_predicting_training_mean": base_ho},
        "routes": summary, "eval_circuits": len(ev),
    }
    print(json.dumps(out), flush=True)
    P.nt_gnn_destroy(model)
    for h in th + hh:
        P.nt_circuit_free(h)
    P.nt_destroy(ctx)


def bench_batch(args, P, W, sub=False):
    """Batched uneven instances: one nt_run_batch call over all 512 circuits
    per step (inputs resident: plans and reference states built before the
    timed region).  sub: a sub-record of the default run (2 steps after 1
    warmup, no CPU leg), returned instead of printed."""
    import numpy as np
    import torch

    n_circ, N, p, tau = 512, 256, 1e-3, 0.9
    circs = [W.config2(s) for s in range(n_circ)]
    prec = P.NT_C64 if args.prec == "c64" else P.NT_C128
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    ctx = P.nt_create(0, stream.cuda_stream)
    P.nt_set_precision(ctx, prec)
    hs = []
    for s, c in enumerate(circs):
        h = P.nt_circuit_load(ctx, c)
        P.nt_circuit_set_id(h, s)
        P.nt_circuit_set_fusion(h, prec, args.fusion)
        hs.append(h)
    P.nt_set_error_model(ctx, p / 3, p / 3, p / 3)
    vals = torch.empty(n_circ, N, dtype=torch.float64, device="cuda:0")
    P.nt_run_batch(ctx, hs, 0, 0, 1, tau)          # plans + reference states
    steps, warmup = (2, 1) if sub else (args.steps, args.warmup)
    for _ in range(warmup):
        P.nt_run_batch(ctx, hs, 0, 0, N, tau, vals_out_ptr=vals.data_ptr())
    torch.cuda.synchronize()
    P.nt_timing_enable(ctx, True)
    P.nt_timing_reset(ctx)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    succ = 0
    e0.record(stream)
    for k in range(steps):
        cnt, _ = P.nt_run_batch(ctx, hs, 0, k * N, N, tau, vals_out_ptr=vals.data_ptr())
        succ += int(cnt.sum())
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    launches, pass_ms, pass_bytes, pass_updates, pass_flops = P.nt_timing_read(ctx)
    P.nt_timing_enable(ctx, False)
    updates = float(steps) * N * sum(c.G * (1 << c.n) for c in circs)
    value = updates / (ms / 1e3)
    achieved_tf = pass_flops / (pass_ms / 1e3) / 1e12
    achieved_gbs = pass_bytes / (pass_ms / 1e3) / 1e9
    alu_peak = ALU_PEAK_TFLOPS[args.prec]
    alu_view = {"bound": "alu", "achieved": achieved_tf, "peak": alu_peak, "unit": "TFLOP/s",
                "frac": achieved_tf / alu_peak, "traffic": None}
    copy_gbs = device_copy_gbs()
    hbm_view = {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": None,
                "device_copy_GBps": copy_gbs, "frac_of_device_copy": achieved_gbs / copy_gbs}
    roofline = dict(alu_view if alu_view["frac"] >= hbm_view["frac"] else hbm_view)
    roofline.update({"kernel": "k_pass (all launch shapes, time-weighted)", "launches": launches,
                     "avg_launch_ms": pass_ms / max(launches, 1),
                     "pass_kernel_share_of_step": pass_ms / ms if ms > 0 else None,
                     "hbm_view": hbm_view, "alu_view": alu_view})
    cpu = None
    if not args.no_cpu_baseline and not sub:
        import oracle
        sample = [(s, c) for s, c in enumerate(circs) if c.n <= 15][:6]
        t0 = time.perf_counter()
        upd = 0
        threads = 0
        for s, c in sample:
            _, _, threads = oracle.run(c, p / 3, p / 3, p / 3, 0, 0, 96, tau, cid=s, return_threads=True)
            upd += 97 * c.G * (1 << c.n)
        dt = time.perf_counter() - t0
        cpu = {"value": upd / dt, "unit": "amplitude-updates/s", "cores": threads, "kind": "oracle",
               "sample": f"instances {[s for s, _ in sample]} (n <= 15), error-free reference + 96 trajectories "
                         f"each, FP64, one trajectory per thread, {dt:.1f} s wall"}
    ns = [c.n for c in circs]
    out = {
        "metric": "trajectory amplitude-updates/s (% HBM peak); time-to-tolerable-error-rate ±0.01",
        "value": value, "unit": "amplitude-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": ms / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.prec, "data": "synthetic",
        "config": {"workload": "512 random-layer instances, n 10..20, 10..100 layers, 256 trajectories each, "
                               "p=1e-3, one batched call per step",
                   "circuits": n_circ, "trajectories_per_circuit": N, "n_min": min(ns), "n_max": max(ns),
                   "gates_total": sum(c.G for c in circs), "amplitudes": args.prec,
                   "parallelism": "single GPU, circuits x trajectories"},
        "roofline": roofline, "cpu_baseline": cpu, "successes": succ,
        "trajectories": steps * N * n_circ,
    }
    for h in hs:
        P.nt_circuit_free(h)
    P.nt_destroy(ctx)
    if sub:
        return out
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
