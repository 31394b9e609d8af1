"""Benchmark: logL + gradient evaluations per second on one MI355X.

Default workload: GTR 4-state model, 3 epochs, 512-taxon coalescent tree,
100,000 site patterns simulated under the epoch model, 4 discrete-gamma
categories; one step = transition matrices + post-order partials + root
log-likelihood + pre-order adjoint with all 1,022 branch-length gradients,
in FP32 with FP64 reductions.  Inputs are resident on the device before the
timed region; the step returns logL and the gradient to the host.

Prints one JSON line (see the design doc for the roofline accounting).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6

WORKLOADS = {
    1: "HKY 4-state, 2 epochs (boundary 0.5), 16-taxon coalescent tree, 1000 patterns, 4 gamma categories",
    2: "GTR 4-state, 3 epochs, 512-taxon coalescent tree, 100000 patterns, 4 gamma categories, "
       "logL + 1022 branch-length gradients",
    3: "GY94 61-state codon (padded 64), 4 epochs, 128-taxon tree, 10000 patterns, 1 category, "
       "logL + branch-length and rate-matrix gradients",
    4: "40-state asymmetric CTMC, 12 processes over 48 intervals, 2000-taxon tree, 1 pattern, "
       "logL + branch-length and rate-matrix gradients",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(prob, precision):
    """Algorithmic HBM bytes of one evaluation, per phase."""
    N = prob.n_tips
    P = prob.n_patterns
    C = len(prob.cat_rates)
    K = prob.n_states
    Kp = 4 if K <= 4 else (8 if K <= 8 else (K + 15) // 16 * 16)
    b = 8 if precision == "fp64" else 4
    V = P * C * Kp * b          # one partial (or outside) vector set of a node
    T = P                       # u8 tip states of one tip
    s = 4 * P                   # int32 cumulative scale exponents of one node
    post = (2 * N - 3) * V + N * T + (2 * N - 3) * s   # write N-1, read N-2 internal children
    pre = (3 * N - 6) * V + N * T                          # read q_u (N-2), read internal p (N-2), write q (N-2)
    return {"post_order": post, "pre_order_dP": pre}


def run_cpu_baseline(prob, sample_patterns, want_Q):
    """The FP64 oracle on a pattern subsample, scaled to evaluations/s of the full problem."""
    import copy
    from threadpoolctl import threadpool_limits

    from oracle import epoch_oracle as O
    sub = copy.copy(prob)
    sub.tips = prob.tips[:, :sample_patterns].copy()
    sub.weights = prob.weights[:sample_patterns].copy()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        logL = O.log_likelihood(sub)
        d_branch, d_Q = O.gradient(sub, wrt=("branch", "Q") if want_Q else ("branch",))
        dt = time.perf_counter() - t0
    full = dt * prob.n_patterns / sample_patterns
    return sub, logL, d_branch, d_Q, {
        "value": 1.0 / full, "unit": "evals/s", "cores": 1, "kind": "oracle",
        "sample": f"{sample_patterns} of {prob.n_patterns} patterns, full tree; {dt:.2f} s measured, "
                  f"scaled linearly in patterns (FP64 numpy/scipy, 1 BLAS thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--kernel", default="auto", choices=["auto", "generic"])
    ap.add_argument("--patterns", type=int, default=None, help="override the pattern count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=None)
    ap.add_argument("--grad-q", action="store_true", help="also form dlogL/dQ (default for configs 3, 4)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported "
                                   "(the multi-GPU pattern-sharded design is described in DESIGN.md)"}))
        sys.exit(2)

    import torch
    from paper_1309_3075_amd import workloads as W
    from paper_1309_3075_amd.likelihood import from_problem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    want_Q = args.grad_q or args.config in (3, 4)
    log(f"bench: generating config C{args.config} ...")
    t0 = time.perf_counter()
    prob = W.make_config(args.config, n_patterns=args.patterns)
    log(f"bench: generated in {time.perf_counter() - t0:.1f} s: N={prob.n_tips} P={prob.n_patterns} "
        f"K={prob.n_states} C={len(prob.cat_rates)} S={prob.n_processes} M={prob.n_intervals}")
    lik = from_problem(prob, args.precision, grad_branch=True, grad_Q=want_Q, kernel=args.kernel,
                       use_pi=args.config != 4)

    def step():
        lik.update_transition_matrices()
        lik.update_partials()
        lL = lik.root_log_likelihood()
        db, dq = lik.gradient(branch=True, Q=want_Q)
        return lL, db, dq

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("bench: warmup done")
    lik.set_timing(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        logL, db, dq = step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = lik.timing()
    ms_per_step = wall * 1000.0 / args.steps
    value = args.steps / wall
    log(f"bench: {ms_per_step:.3f} ms/step, phases {phases}")

    abytes = algorithmic_bytes(prob, args.precision)
    # dominant kernel: the phase with the largest device time among the pruning passes
    dom = max(("post_order", "pre_order_dP"), key=lambda k: phases[k][0])
    dom_ms = phases[dom][0] / args.steps
    launches = {"post_order": "nuc_post_level", "pre_order_dP": "nuc_pre_level"}[dom] \
        if prob.n_states == 4 and args.kernel == "auto" else \
        {"post_order": "post_level_generic", "pre_order_dP": "pre_level_generic + grad_G_generic"}[dom]
    achieved = abytes[dom] / (dom_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": launches, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "algorithmic_bytes_per_eval": abytes[dom], "ms_per_eval": round(dom_ms, 4)}
    total_bytes = sum(abytes.values())
    result = {
        "metric": "logL+gradient evals/sec", "value": round(value, 3), "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic (seeded coalescent tree, patterns simulated under the epoch model)",
        "config": {"workload": WORKLOADS[args.config], "config_index": args.config, "n_tips": prob.n_tips,
                   "n_patterns": prob.n_patterns, "n_states": prob.n_states,
                   "n_categories": len(prob.cat_rates), "precision": args.precision, "kernel": args.kernel,
                   "grad_Q": want_Q},
        "roofline": roofline,
        "whole_step_hbm_fraction": round(total_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "phases_ms_per_eval": {k: round(v[0] / args.steps, 4) for k, v in phases.items()},
        "logL": logL,
    }

    from paper_1309_3075_amd import _abi
    probe = {k: round(_abi.bandwidth_probe(1 << 31, k, 20), 1) for k in ("copy", "read", "write")}
    result["measured_hbm_GBps"] = probe
    result["roofline"]["frac_of_measured_copy"] = round(achieved / probe["copy"], 4)
    log(f"bench: bandwidth probe {probe}")

    if not args.no_cpu_baseline:
        sample = args.cpu_sample or min(prob.n_patterns, {1: 1000, 2: 2000, 3: 500, 4: 1}.get(args.config, 1000))
        log(f"bench: cpu baseline on {sample} patterns ...")
        sub, ref_logL, ref_b, ref_q, cpu = run_cpu_baseline(prob, sample, want_Q)
        result["cpu_baseline"] = cpu
        # parity of the same GPU path on the same subsample
        with from_problem(sub, args.precision, grad_branch=True, grad_Q=want_Q, kernel=args.kernel,
                          use_pi=args.config != 4) as small:
            g_logL = small.log_likelihood()
            g_b, g_q = small.gradient(branch=True, Q=want_Q)
        parity = {"sample_patterns": sample, "logL_rel_err": abs(g_logL - ref_logL) / abs(ref_logL),
                  "grad_branch_rel_err": float(np.linalg.norm(g_b - ref_b) / np.linalg.norm(ref_b))}
        if want_Q:
            parity["grad_Q_rel_err"] = float(np.linalg.norm(g_q - ref_q) / np.linalg.norm(ref_q))
        result["parity_vs_oracle"] = parity
    lik.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
