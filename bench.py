"""Benchmark of the HEOM-2DVS hot path on one MI355X.

Workload (default): the water-like three-mode model (4x4x5 = 80 states,
K=2 Pade terms per mode, depth L=6: 5005 ADOs), 128 trajectories -- the t1
samples of the 128x128 grid -- propagated together in FP32 by fixed-step RK4:
the batched t2/t3 propagation that dominates a 2D spectrum.  One "step" is one
RK4 step of the whole batch (4 fused RHS launches).  value = ADO-updates/s =
trajectories x ADOs x steps / wall time.

Also reported: seconds per 2D spectrum (full 128x128 grid, FP32 propagation
with FP64 pairing) measured end to end for t2 = 0 and for the t2 set {0, 50 fs}
(the batched t2 propagation in the timed region), the FP32 error of the t2 = 0
spectrum against the FP64 path, the equilibration with its convergence flag, a
short FP64 propagation leg with its own roofline, the roofline of the dominant
kernel from HIP-event timings of its launches inside the timed region, the
uneven multi-instance batch in each launch form, the reverse-mode gradient of
the gradient workload's depth-6 model (one t1 / t3 sample, two t2 values), and the CPU oracle's
rate on a bounded sample (all cores and one core).

The whole run keeps to a wall-clock budget (--wall-budget, counted from the
start of the process, imports included): the spectrum legs always run; the CPU
baseline, the gradient and the multi-instance legs, in that order, run only if
their usual duration still fits, and are otherwise reported as skipped.
"""

from __future__ import annotations

import time

_T_START = time.time()

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# HBM traffic of the matrix-core kernel per launch at the default workload, from
# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs (profiles/rhs_mfma_kernel_3mode_L6_b128_fp32.md),
# scaled by the counters' readings for kernels of known size.  Keyed by the
# kernel source hash: a changed kernel reports traffic null until re-profiled.
PROFILED_TRAFFIC = {  # source hash -> kernel choice -> bytes per launch
    "6619fa0244e5ed0b": {  # FP32 at this shape: both choices run the runtime-shape kernel
        "mfma": {"read_GB": 328.9, "write_GB": 32.8, "batch": 128, "precision": "fp32"},
        "mfma_dyn": {"read_GB": 328.9, "write_GB": 32.8, "batch": 128, "precision": "fp32"},
        # the FP64 leg: 32 trajectories
        "fp64:mfma": {"read_GB": 154.7, "write_GB": 16.4, "batch": 32, "precision": "fp64"},
    },
}

PEAKS = {  # MI355X published dense peaks
    "fp32_tflops": 157.3,
    "fp64_tflops": 78.6,
    "hbm_gbs": 8000.0,
}


def algorithmic_flops_per_rhs(model):
    """Flops of one RHS evaluation of every ADO of one trajectory.

    Per ADO: H commutator 8 d^3 (complex x real, both sides); V_s products
    8 d^2 sum_s d_s; neighbour combination 2 d^2 per upper neighbour (unit
    coefficient, shared by both sides) and 16 d^2 per lower neighbour (complex
    coefficient, two sides); damping 2 d^2; RK4 stage update 4 d^2.
    """
    ops = model.operators()
    n = ops["ado_n"]
    d = model.d
    depth = n.sum(1)
    n_up = np.where(depth < model.depth, n.shape[1], 0).sum()
    n_down = int((n > 0).sum())
    per_ado = 8 * d ** 3 + 8 * d * d * sum(model.dims) + 6 * d * d
    return per_ado * model.n_ado + d * d * (2 * n_up + 16 * n_down)


KERNEL_FILES = {"generic": ("kernels.hip", "rhs_generic_kernel"), "mfma": ("mfma_rhs.hip", "rhs_mfma_kernel"),
                "mfma_dyn": ("mfma_rhs.hip", "rhs_mfma_kernel"), "kron": ("kron_rhs.hip", "rhs_kron_kernel"),
                "mfma_gh": ("mfma_rhs.hip", "rhs_mfma_gh_kernel")}


def kernel_source_hash(kernel="mfma"):
    import hashlib
    path = os.path.join(ROOT, "paper_2601_20550_amd", "csrc", KERNEL_FILES[kernel][0])
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def cpu_baseline(params, budget_s=30.0):
    """Oracle rate on a bounded sample: RHS evaluations of one trajectory, with
    the BLAS thread pool at its default size (all host cores it uses) and
    limited to one thread."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import heom as oh
    from oracle import model as om
    import workloads as w
    cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    o = om.build(params)
    x = w.random_hierarchy(1, len(o.hier), o.d, seed=1)[0]

    def rate(limit_s, max_rhs):
        t0 = time.perf_counter()
        n_rhs = 0
        while True:
            oh.rhs(o, x)
            n_rhs += 1
            if time.perf_counter() - t0 > limit_s or n_rhs >= max_rhs:
                break
        dt = (time.perf_counter() - t0) / n_rhs
        return len(o.hier) / (4.0 * dt), n_rhs, dt  # one ADO-update = one RK4 step = 4 RHS

    r_all, n_all, dt_all = rate(budget_s / 3, 2)
    with threadpool_limits(1):
        r_one, n_one, dt_one = rate(budget_s / 3, 1)
    return {"value": r_all, "unit": "ADO-updates/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{n_all} oracle RHS evaluation(s) of one trajectory of the "
                      f"{len(o.hier)}-ADO model ({dt_all:.1f} s each); 4 RHS = 1 RK4 step",
            "single_core": {"value": r_one, "unit": "ADO-updates/s", "cores": 1,
                            "sample": f"{n_one} RHS evaluation(s) with the BLAS pool limited to one "
                                      f"thread ({dt_one:.1f} s each)"}}


def batch_forms(P, torch, b, models, precision, n_traj=8, steps=5):
    """RK4 steps of the whole batch with n_traj trajectories per instance (the
    shape of the batched t2 propagation): the autotuner's choice, then ms per
    step of per-class launches, one launch per stage, and the autotuned form
    replayed from a captured graph."""
    states = []
    for m in models:
        s = P.State(m, n_traj, precision)
        s.set_ground()
        states.append(s)
    chosen, tune_ms = P.heom_batch_autotune(b, precision, n_traj=n_traj, reps=3)
    shapes = {}
    for nb in sorted({(m.d + 15) // 16 for m in models}):
        wg, lds = P.heom_batch_get_class_shape(b, nb)
        shapes[f"d<={16 * nb}"] = {"workgroups_per_cu": wg,
                                   "neighbour_sums": {1: "lds", 0: "registers", -1: "default"}[lds]}
    out = {"trajectories_per_instance": n_traj, "steps": steps, "autotune_choice": chosen,
           "autotune_ms_per_step": tune_ms, "class_shapes": shapes}
    items = n_traj * sum(m.n_ado for m in models)
    for form, graph in (("per_class", 0), ("single", 0), (chosen, steps)):
        P.heom_batch_set_launch(b, form)
        P.heom_batch_set_graph_steps(b, graph)
        P.heom_batch_propagate(b, states, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.heom_batch_propagate(b, states, steps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        key = form + ("_graph" if graph else "")
        out[key] = {"ms_per_step": dt * 1e3, "ado_updates_per_s": items / dt}
    P.heom_batch_set_launch(b, "auto")
    P.heom_batch_set_graph_steps(b, 0)
    return out


def multi_instance(P, torch, precision, stream, compare=False):
    """The uneven 64-instance batch (d = 6, 25, 80; 35..5005 ADOs; t2 = 0):
    batched RK4 steps of 8 trajectories per instance in each launch form, then
    seconds for all 64 responses batched (the autotuned form; 16 x 16 samples
    of the workload's 64 x 64 grid spacing) and, with compare, one instance
    after another, and their agreement."""
    import workloads as w
    insts = w.cfg4_instances()
    models = [P.heom_model_build(p, stream=stream) for p, _ in insts]
    # the 64 x 64 grid of the workload, reduced to 16 x 16 samples at the
    # same spacing to keep the default run short (the scans are 150 instead
    # of 630 RK4 steps)
    grid = dict(insts[0][1])
    grid["n1"] = grid["n3"] = 16
    rhos = []
    for m in models:
        r = P.State(m, 1, "fp64")
        r.set_ground()
        rhos.append(r)
    b = P.heom_batch_create(models)
    forms = batch_forms(P, torch, b, models, precision)
    tiny = {"n1": 2, "n3": 2, "steps_per_sample": 1, "t2_steps": [0]}
    P.heom_batch_response_2d(b, rhos, tiny, precision)          # warm-up (code objects)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Rb = P.heom_batch_response_2d(b, rhos, grid, precision)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    n1, sps = grid["n1"], grid["steps_per_sample"]
    # single-trajectory RK4 steps: t3 scan (adjoint) + one t1 scan per pathway
    ado_steps = sum(m.n_ado for m in models) * 3 * (n1 - 1) * sps
    out = {"instances": len(models), "grid": [n1, grid["n3"]], "t2": 0, "precision": precision,
           "d_classes": sorted({m.d for m in models}), "launch_form": P.heom_batch_get_launch(b),
           "s_batched": t_batch, "ado_updates_per_s_batched": ado_steps / t_batch,
           "rho_eq": "ground state (timing only)", "batched_trajectories": forms}
    if compare:
        t0 = time.perf_counter()
        Rs = [P.heom_response_2d(m, r, grid, precision, "adjoint") for m, r in zip(models, rhos)]
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        out["s_one_by_one"] = t_seq
        out["speedup"] = t_seq / t_batch
        out["max_rel_diff_vs_one_by_one"] = max(
            float(np.max(np.abs(a - c)) / max(np.max(np.abs(c)), 1e-300)) for a, c in zip(Rb, Rs))
    return out


def gradient_timing(P, torch, stream):
    """Reverse-mode gradient (FP64) of a random linear functional of the
    responses of the gradient workload's model (three modes, depth 6: 5005 ADOs
    of 80 x 80; t2 in {0, 100 fs}), rho held fixed (200 RK4 steps from the
    ground state): seconds for the forward responses, for the vjp (operator
    gradients) and for the chain to the 12 fitted parameters.  One t1 and one
    t3 sample (t1 = t3 = 0), so the cost is
    the t2 propagation of both pathways and its adjoint sweep; the 64 x 64 grid
    propagates 64 trajectories per pathway through t2 instead of one."""
    import workloads as w
    params, g5, _ = w.cfg5()
    grid = {"n1": 1, "n3": 1, "steps_per_sample": 10, "t2_steps": list(g5["t2_steps"])}
    m = P.heom_model_build(params, stream=stream)
    rho = P.State(m, 1, "fp64")
    rho.set_ground()
    P.heom_propagate(m, rho, 200)
    P.heom_response_2d(m, rho, {"n1": 2, "n3": 2, "steps_per_sample": 1, "t2_steps": [0]}, "fp64",
                       "adjoint")
    P.heom_model_set_progress(m, lambda ph, done, tot: print(f"gradient leg, {ph}: {done}/{tot} RK4 steps",
                                                             file=sys.stderr, flush=True), 200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    R = P.heom_response_2d(m, rho, grid, "fp64", "adjoint")
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    W = np.random.default_rng(0).standard_normal(R.shape) + 0j
    t0 = time.perf_counter()
    g = P.heom_response_2d_vjp(m, rho, grid, W, stationary=False)
    torch.cuda.synchronize()
    t_vjp = time.perf_counter() - t0
    P.heom_model_set_progress(m, None)
    t0 = time.perf_counter()
    gt = P.heom_params_vjp(params, w.theta_directions(params), g)
    t_chain = time.perf_counter() - t0
    return {"model": "3-mode, depth 6 (5005 ADOs), d = 80, 12 parameters", "grid": [1, 1],
            "t2_steps": grid["t2_steps"], "precision": "fp64", "s_forward_responses": t_fwd, "s_vjp": t_vjp,
            "s_parameter_chain": t_chain, "vjp_over_forward": t_vjp / t_fwd,
            "finite": bool(np.isfinite(gt).all())}


def fp64_leg(P, torch, m, steps, flops_per_traj):
    """The plain FP64 propagation of the same model: 32 trajectories (the FP64
    batch is chunked by memory in the response path), its own HIP-event roofline
    against the FP64 peak."""
    B = 32
    prev = P.heom_model_get_kernel(m, "fp64")
    s = P.State(m, B, "fp64")
    s.set_ground()
    P.heom_propagate(m, s, 1)
    torch.cuda.synchronize()
    P.heom_timing_enable(m, True)
    t0 = time.perf_counter()
    P.heom_propagate(m, s, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_ms, n_launch, _ = P.heom_timing_read(m)
    P.heom_timing_enable(m, False)
    del s
    avg = k_ms / 1e3 / max(n_launch, 1)
    achieved = flops_per_traj * B / avg / 1e12
    out = {"value": B * m.n_ado * steps / wall, "unit": "ADO-updates/s", "trajectories": B, "steps": steps,
           "ms_per_step": wall / steps * 1e3, "kernel_choice": prev,
           "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAKS["fp64_tflops"], "unit": "TFLOP/s",
                        "frac": achieved / PEAKS["fp64_tflops"], "traffic": None, "avg_launch_ms": avg * 1e3,
                        "launches": n_launch}}
    prof = PROFILED_TRAFFIC.get(kernel_source_hash(prev), {}).get("fp64:" + prev) if prev in KERNEL_FILES else None
    if prof and prof["batch"] == B and m.n_ado == 5005 and m.d == 80:
        out["roofline"]["traffic"] = (prof["read_GB"] + prof["write_GB"]) * 1e9
        out["roofline"]["traffic_unit"] = "bytes per launch (HBM, calibrated rocprofv3 counters)"
    return out


def spectrum_legs(P, torch, w, m, params, grid, args):
    """rho_eq by GMRES (FP64), then 2D spectra of the full 128 x 128 grid: the
    t2 = 0 spectrum alone, the first --spectrum-t2 t2 values in one call (the
    batched t2 propagation of 2 x 128 trajectories in the timed region), and
    the FP32 error of the t2 = 0 spectrum against the FP64 path."""
    out = {}
    progress = lambda ph, done, tot: print(f"{ph}: {done}/{tot} RK4 steps", file=sys.stderr,  # noqa: E731
                                           flush=True)
    # rho_eq: 100 RK4 steps from |0><0|, then GMRES corrections, each call one
    # restart cycle of --eq-chunk applications of 500 steps, until the residual
    # reaches --eq-tol or --eq-seconds have passed (progress on stderr)
    torch.cuda.synchronize()
    t_eq = time.perf_counter()
    rho = P.State(m, 1, "fp64")
    rho.set_ground()
    P.heom_propagate(m, rho, 100)
    eq_applies, eq_res = 0, float("inf")
    P.heom_model_set_progress(m, progress, 5000)
    while True:
        a, eq_res = P.heom_stationary_refine(m, rho, tol=args.eq_tol, max_applies=args.eq_chunk,
                                             restart=args.eq_chunk)
        eq_applies += a
        print(f"equilibration: {eq_applies} applications, residual {eq_res:.3e}", file=sys.stderr, flush=True)
        if eq_res <= args.eq_tol or time.perf_counter() - t_eq > args.eq_seconds or a == 0:
            break
    P.heom_model_set_progress(m, None)
    torch.cuda.synchronize()
    t_eq = time.perf_counter() - t_eq
    converged = bool(eq_res <= args.eq_tol)
    out["equilibration"] = {"method": "GMRES on I - Phi^500 (FP64)", "s": t_eq,
                            "rk4_steps": 100 + 500 * eq_applies, "residual": eq_res, "tol": args.eq_tol,
                            "converged": converged}
    dt_s = grid["steps_per_sample"] * params["dt"]
    all_t2 = list(grid["t2_steps"])
    dt_fs = params["dt"] * w.FS_PER_TIME_UNIT
    # the first --spectrum-t2 t2 values in one call: the t1 snapshots of both
    # pathways are propagated through t2 as one 128-trajectory batch per
    # pathway (the batched t2 propagation is in the timed region)
    g2 = dict(grid)
    g2["t2_steps"] = all_t2[:max(1, args.spectrum_t2)]
    P.heom_model_set_progress(m, progress, 100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    R = P.heom_response_2d(m, rho, g2, args.precision, "adjoint")
    S = [P.heom_spectrum_2d(R[q, 0], R[q, 1], dt_s) for q in range(R.shape[0])]
    torch.cuda.synchronize()
    t_set = time.perf_counter() - t0
    P.heom_model_set_progress(m, None)
    n_t2 = len(g2["t2_steps"])
    out["s_per_2d_spectrum"] = t_set / n_t2
    out["s_2d_spectra_t2_set"] = {
        "t2_fs": [round(x * dt_fs, 1) for x in g2["t2_steps"]], "s": t_set, "s_per_2d_spectrum": t_set / n_t2,
        "grid": [g2["n1"], g2["n3"]], "precision": args.precision,
        "method": "adjoint (t3 by the transposed propagation of the detection functional)",
        "rho_eq_converged": converged, "finite": bool(all(np.isfinite(x).all() for x in S))}
    if args.eps_spec and args.precision == "fp32":
        # FP32 error of the t2 = 0 spectrum against the FP64 GPU path
        g1 = dict(grid)
        g1["t2_steps"] = [all_t2[0]]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R64 = P.heom_response_2d(m, rho, g1, "fp64", "adjoint")
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        S64 = P.heom_spectrum_2d(R64[0, 0], R64[0, 1], dt_s)
        out["eps_spec"] = {"t2_fs": 0.0, "grid": [g1["n1"], g1["n3"]],
                           "value": float(np.max(np.abs(S[0] - S64)) / np.max(np.abs(S64))),
                           "R_rel": float(np.max(np.abs(R[0] - R64[0])) / np.max(np.abs(R64[0]))),
                           "reference": "FP64 GPU path", "target": 1e-4, "s_fp64_t2_0": t64}
    return out


def leg_skip_reason(elapsed_s, usual_s, budget_s):
    """None if an optional leg of usual duration usual_s (MI355X, default
    sizes) still fits the wall-clock budget after elapsed_s, else the reason
    recorded in its place."""
    if elapsed_s + usual_s <= budget_s:
        return None
    return (f"wall-clock budget: {elapsed_s:.0f} s elapsed, leg takes about {usual_s:.0f} s, "
            f"budget {budget_s:.0f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--depth", type=int, default=6)
    ap.add_argument("--spectrum", type=int, default=1, help="also time one full 2D spectrum")
    ap.add_argument("--spectrum-t2", type=int, default=2,
                    help="number of the workload's t2 values in the timed response call "
                         "(1: t2 = 0 only; cfg3 has 0, 50, 100, 200 fs)")
    ap.add_argument("--eq-tol", type=float, default=1e-7)
    ap.add_argument("--eq-seconds", type=float, default=200.0)
    ap.add_argument("--eq-chunk", type=int, default=100,
                    help="GMRES applications per refinement call; each call is one restart cycle "
                         "(restarts every 10 applications stagnate on the slow population modes)")
    ap.add_argument("--fp64-steps", type=int, default=3,
                    help="RK4 steps of a 32-trajectory FP64 leg with its own roofline (0: skip)")
    ap.add_argument("--eps-spec", type=int, default=1,
                    help="also compute the t2 = 0 spectrum in FP64 and report the FP32 error")
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--multi", type=int, default=1,
                    help="1: also time the 64-instance uneven batch; 2: and one instance at a time")
    ap.add_argument("--grad", type=int, default=1, help="also time the reverse-mode gradient")
    ap.add_argument("--workload", default="cfg3", choices=["cfg3", "paper", "brownian"],
                    help="cfg3: 3-mode, 80 states, depth 6 (5005 ADOs); paper: the paper's hierarchy "
                         "scale, 3 x 4 levels, K = 4 Pade, depth 5 (15,504 ADOs), 300 K assumed; "
                         "brownian: cfg3's modes with Brownian baths (complex rate pairs), "
                         "12 terms, depth 5 (6188 ADOs)")
    ap.add_argument("--kernel", default="auto", choices=["auto", "generic", "mfma", "mfma_dyn", "kron", "mfma_gh"])
    ap.add_argument("--wall-budget", type=float, default=570.0,
                    help="seconds from process start within which the optional legs must finish")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the path shards into independent "
              "trajectory batches; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2601_20550_amd as P
    import workloads as w

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "paper":
        params, grid = w.paper_scale()
    elif args.workload == "brownian":
        params, grid = w.cfg3_brownian()
    else:
        params, grid = w.cfg3(depth=args.depth)
    stream = torch.cuda.current_stream()
    m = P.heom_model_build(params, stream=stream.cuda_stream)
    B = args.batch
    tune = None
    if args.kernel == "auto":
        best, ms = P.heom_autotune(m, min(B, 8), args.precision, reps=3)
        tune = {"chosen": best, "ms_per_step_8traj": ms}
    else:
        P.heom_model_set_kernel(m, args.precision, args.kernel)
    kernel = P.heom_model_get_kernel(m, args.precision)
    s = P.State(m, B, args.precision)
    s.set_ground()
    P.heom_propagate(m, s, args.warmup)
    torch.cuda.synchronize()

    P.heom_timing_enable(m, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.heom_propagate(m, s, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_ms, n_launch, upd = P.heom_timing_read(m)
    P.heom_timing_enable(m, False)

    ado_updates = B * m.n_ado * args.steps
    value = ado_updates / wall
    avg_launch_s = k_ms / 1e3 / max(n_launch, 1)
    flops_launch = algorithmic_flops_per_rhs(m) * B
    achieved = flops_launch / avg_launch_s / 1e12
    peak = PEAKS["fp32_tflops"] if args.precision == "fp32" else PEAKS["fp64_tflops"]

    line = {
        "metric": "ADO-updates/s + s per 2D spectrum (3-mode, L=6); FP32/batched vs FP64",
        "value": value,
        "unit": "ADO-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic (seeded water-like 3-mode model; no trained inputs)",
        "config": {"workload": ({"cfg3": f"3-mode MAB HEOM, 80 states, K=2 Pade x3, depth {args.depth} ",
                                 "paper": "3-mode MAB HEOM at the paper's scale, 64 states, K=4 Pade x3, "
                                          f"depth {params['depth']}, 300 K assumed ",
                                 "brownian": "3-mode MAB HEOM, 80 states, Brownian baths (omega_b 0.25, "
                                             f"K=2 Pade) x3, depth {params['depth']} "}[args.workload])
                               + f"({m.n_ado} ADOs), {B} trajectories batched, RK4 dt=0.1",
                   "n_ado": m.n_ado, "d": m.d, "trajectories": B},
        "roofline": {"bound": "alu" if kernel == "generic" else "mfma", "achieved": achieved,
                     "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "kernel": KERNEL_FILES[kernel][1] + " (fused RHS + RK4 stage)",
                     "avg_launch_ms": avg_launch_s * 1e3, "launches": n_launch},
        "kernel_choice": kernel,
        "kernel_source": kernel_source_hash(kernel),
        "autotune": tune,
    }

    prof = PROFILED_TRAFFIC.get(kernel_source_hash(kernel), {}).get(kernel)
    if (prof and prof["batch"] == B
            and prof["precision"] == args.precision and args.depth == 6 and args.workload == "cfg3"):
        line["roofline"]["traffic"] = (prof["read_GB"] + prof["write_GB"]) * 1e9
        line["roofline"]["traffic_unit"] = "bytes per launch (HBM, calibrated rocprofv3 counters)"
        line["roofline"]["hbm_GBs_at_traffic"] = line["roofline"]["traffic"] / avg_launch_s / 1e9

    t_leg = time.perf_counter()

    def leg_done(name):
        nonlocal t_leg
        print(f"{name} leg done in {time.perf_counter() - t_leg:.1f} s", file=sys.stderr, flush=True)
        t_leg = time.perf_counter()

    if args.fp64_steps > 0 and args.precision == "fp32":
        line["fp64"] = fp64_leg(P, torch, m, args.fp64_steps, algorithmic_flops_per_rhs(m))
        leg_done("fp64")
    if args.spectrum:
        line.update(spectrum_legs(P, torch, w, m, params, grid, args))
        leg_done("spectrum")
    del s

    def fits(name, usual_s):
        why = leg_skip_reason(time.time() - _T_START, usual_s, args.wall_budget)
        if why is None:
            return True
        line[name] = {"skipped": why}
        print(f"{name} leg skipped (budget)", file=sys.stderr, flush=True)
        return False

    if args.cpu_baseline and fits("cpu_baseline", 25.0):
        line["cpu_baseline"] = cpu_baseline(params)
        leg_done("cpu baseline")
    if args.grad and fits("gradient", 55.0):
        line["gradient"] = gradient_timing(P, torch, stream.cuda_stream)
        leg_done("gradient")
    if args.multi and fits("multi_instance", 25.0 if args.multi == 1 else 120.0):
        line["multi_instance"] = multi_instance(P, torch, args.precision, stream.cuda_stream,
                                                compare=args.multi > 1)
        leg_done("multi-instance")
    line["wall_s"] = time.time() - _T_START
    print(json.dumps(line))


if __name__ == "__main__":
    main()
