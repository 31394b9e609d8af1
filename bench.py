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


def algorithmic_flops(prob):
    """Algorithmic flops of one logL+gradient evaluation: internal-child
    matrix-vector products 2K^2 per (pattern, category); tip children are lookups;
    pre-order products and gradient outer products (N-2) 2K^2 P C each; epoch products
    (2m-1) 2K^3 per (branch, category); the dlogL/dQ adjoint chain three K x K products
    (6K^3) per segment term (W = R V^-T, Y = U^T W, the update of R); padding never counted."""
    from paper_1309_3075_amd import _abi  # the library's host planner gives the segment counts
    N, P, K, C = prob.n_tips, prob.n_patterns, prob.n_states, len(prob.cat_rates)
    n_int_children = N - 2
    post = n_int_children * 2 * K * K * P * C
    pre = 2 * (N - 2) * 2 * K * K * P * C
    off, _, _ = _abi.plan_segments(prob.parent, prob.height, prob.boundaries, prob.interval_process,
                                   prob.n_processes)
    m = np.diff(off)
    chain = int(np.sum(np.maximum(2 * m - 1, 0))) * 2 * K ** 3 * C
    adjoint = int(np.sum(m)) * C * 6 * K ** 3
    return {"post_order": post, "pre_order_dP": pre, "transition_matrices": chain, "grad_Q": adjoint}


def fp64_reconstruction(prob, use_pi):
    """Whether the library forms exp(tQ) in FP64 for this problem: it does so in FP32 instances when
    some eigenvector matrix has infinity-norm condition number above 32 (the same rule, evaluated here
    on the eigensystems the binding hands over)."""
    from paper_1309_3075_amd.eigen import eigensystem
    for s, Q in enumerate(prob.Q):
        e = eigensystem(Q, prob.pi_process[s] if use_pi else None)
        cond = np.abs(e.V).sum(axis=1).max() * np.abs(e.Vinv).sum(axis=1).max()
        if cond > 32.0:
            return True
    return False


def committed_traffic(name, kernel):
    """HBM bytes per evaluation of `kernel` from a committed counter summary under profiles/,
    or None when the summary is missing or the kernel source has changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split(None, 1)
        vals[k] = v.strip()
    src = os.path.join(ROOT, vals.get("source", ""))
    if not os.path.isfile(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != vals.get("source_sha256"):
        return None
    try:
        return int(vals[f"{kernel}_read_bytes_per_eval"]) + int(vals[f"{kernel}_write_bytes_per_eval"])
    except KeyError:
        return None


def run_cpu_baseline(prob, sample_patterns, want_Q, want_grad=True):
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
        d_branch, d_Q = (O.gradient(sub, wrt=("branch", "Q") if want_Q else ("branch",)) if want_grad
                         else (None, None))
        dt = time.perf_counter() - t0
    full = dt * prob.n_patterns / sample_patterns
    return sub, logL, d_branch, d_Q, {
        "value": 1.0 / full, "unit": "evals/s", "cores": 1, "kind": "oracle",
        "sample": f"{sample_patterns} of {prob.n_patterns} patterns, full tree; {dt:.2f} s measured, "
                  f"scaled linearly in patterns (FP64 numpy/scipy, 1 BLAS thread)"}


def run_batch(args):
    """Batched codon workload: independent 64-state problems in one replayed HIP graph."""
    import torch
    from paper_1309_3075_amd import _abi
    from paper_1309_3075_amd import workloads as W
    from paper_1309_3075_amd.likelihood import EpochBatchEvaluator, from_problem

    n = args.batch or 64
    log(f"bench: generating {n} batched codon problems ...")
    t0 = time.perf_counter()
    probs = W.make_batch(n, scale=args.batch_scale)
    log(f"bench: generated in {time.perf_counter() - t0:.1f} s; patterns {sum(p.n_patterns for p in probs)}")
    members = [from_problem(p, args.precision, grad_branch=True, grad_Q=args.grad_q) for p in probs]
    tune = os.path.join(ROOT, "paper_1309_3075_amd", "tune_cache.json")
    batch = EpochBatchEvaluator(members, tune_cache=tune)
    for _ in range(args.warmup):
        batch.evaluate(grad_branch=True, grad_Q=args.grad_q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        logL = batch.evaluate(grad_branch=True, grad_Q=args.grad_q)
    wall = time.perf_counter() - t0
    ms = wall * 1000 / args.steps
    flops = sum(sum(v for k, v in algorithmic_flops(p).items()) for p in probs)
    achieved = flops / (ms * 1e-3) / 1e12
    result = {
        "metric": "logL+gradient evals/sec", "value": round(n * args.steps / wall, 3), "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic (seeded coalescent trees, codon patterns simulated under the epoch model)",
        "config": {"workload": f"{n} batched GY94 codon problems (61 states padded to 64, 4 epochs), "
                               f"64-256 taxa and 1000-20000 patterns each (x{args.batch_scale}), one replayed "
                               "hipGraph per step, logL + branch gradients",
                   "config_index": 5, "n_problems": n, "precision": args.precision,
                   "tuned_target_blocks": batch.target_blocks()},
        "roofline": {"bound": "mfma", "kernel": "whole batched graph (codon_post/pre_level dominant)",
                     "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": None,
                     "algorithmic_flops_per_step": flops},
        "logL_first": float(logL[0]),
    }
    batch.close()
    for m in members:
        m.close()
    print(json.dumps(result), flush=True)


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
    ap.add_argument("--batch", type=int, default=None, help="number of problems for config 5 (default 64)")
    ap.add_argument("--batch-scale", type=float, default=1.0, help="shrink factor of the config-5 problems")
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
    if args.config == 5:
        return run_batch(args)
    want_Q = args.grad_q or args.config in (3, 4)
    want_grad = args.config != 1  # the 16-taxon workload is a plain log-likelihood
    log(f"bench: generating config C{args.config} ...")
    t0 = time.perf_counter()
    prob = W.make_config(args.config, n_patterns=args.patterns)
    log(f"bench: generated in {time.perf_counter() - t0:.1f} s: N={prob.n_tips} P={prob.n_patterns} "
        f"K={prob.n_states} C={len(prob.cat_rates)} S={prob.n_processes} M={prob.n_intervals}")
    lik = from_problem(prob, args.precision, grad_branch=want_grad, grad_Q=want_Q, kernel=args.kernel,
                       use_pi=args.config != 4)

    def step():
        # the whole path (P stage, pruning, root log-likelihood, gradients) with one host sync
        lL, _, db, dq = lik.evaluate(branch=want_grad, Q=want_Q)
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
    aflops = algorithmic_flops(prob)
    # dominant kernel: the phase with the largest device time
    dom = max(("post_order", "pre_order_dP", "transition_matrices") + (("grad_Q",) if want_Q else ()),
              key=lambda k: phases[k][0])
    dom_ms = phases[dom][0] / args.steps
    path = ("nuc" if prob.n_states == 4 else ("codon" if prob.n_states > 48 and args.precision == "fp32"
                                               and len(prob.cat_rates) == 1 else "generic"))
    if args.kernel == "generic":
        path = "generic"
    # the library takes the tree walk for FP32 4-state instances of at most 1024 tiles of 16 patterns
    cp = 1 if len(prob.cat_rates) <= 1 else (2 if len(prob.cat_rates) <= 2 else (4 if len(prob.cat_rates) <= 4 else 8))
    walk = args.precision == "fp32" and -(-prob.n_patterns // (64 // cp)) <= 1024
    names = {"nuc": {"post_order": "nuc_walk_mfma (post-order program)" if walk else "nuc_post_level",
                     "pre_order_dP": "nuc_walk_mfma (pre-order program)" if walk else "nuc_pre_level"},
             "codon": {"post_order": "codon_post_level", "pre_order_dP": "codon_pre_level + codon_pre_split"},
             "generic": {"post_order": "post_level_generic", "pre_order_dP": "pre_level_generic + grad_G_generic"}}
    Kp = 4 if prob.n_states <= 4 else (8 if prob.n_states <= 8 else (prob.n_states + 15) // 16 * 16)
    mfma_pstage = args.kernel == "auto" and Kp >= 16
    if dom == "grad_Q":
        kname = "qgrad_chain + qgrad_h + qgrad_final" if mfma_pstage else "qgrad_segments + qgrad_reduce"
    else:
        kname = names[path].get(dom, "pstage_mfma (+ split-chain combine)" if mfma_pstage else "pstage_generic")
    if path == "codon" or dom in ("transition_matrices", "grad_Q"):
        achieved = aflops[dom] / (dom_ms * 1e-3) / 1e12
        # the chains run in FP64 when the instance forms exp(tQ) in FP64 (ill-conditioned eigenvectors)
        peak = FP64_PEAK_TFLOPS if (args.precision == "fp64" or dom in ("transition_matrices", "grad_Q")
                                    and fp64_reconstruction(prob, args.config != 4)) \
            else FP32_PEAK_TFLOPS
        roofline = {"bound": "mfma", "kernel": kname, "achieved": round(achieved, 3), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                    "algorithmic_flops_per_eval": aflops[dom], "ms_per_eval": round(dom_ms, 4),
                    "hbm_GBps_same_kernel": round(abytes.get(dom, 0) / (dom_ms * 1e-3) / 1e9, 1)}
    else:
        achieved = abytes[dom] / (dom_ms * 1e-3) / 1e9
        traffic = None
        if path == "nuc" and args.precision == "fp32" and args.config == 2 and args.patterns is None:
            traffic = committed_traffic("nuc_C2_hbm_traffic.txt", kname)
        roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "traffic_unit": "bytes per evaluation (all launches of the kernel)",
                    "algorithmic_bytes_per_eval": abytes[dom], "ms_per_eval": round(dom_ms, 4)}
    total_bytes = sum(abytes.values())
    result = {
        "metric": "logL+gradient evals/sec" if want_grad else "logL evals/sec", "value": round(value, 3),
        "unit": "evals/s", "n_gpus": 1,
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
    if result["roofline"]["unit"] == "GB/s":
        result["roofline"]["frac_of_measured_copy"] = round(achieved / probe["copy"], 4)
    result["algorithmic_flops_per_eval"] = aflops
    log(f"bench: bandwidth probe {probe}")

    if not args.no_cpu_baseline:
        sample = args.cpu_sample or min(prob.n_patterns, {1: 1000, 2: 30000, 3: 3000, 4: 1}.get(args.config, 1000))
        log(f"bench: cpu baseline on {sample} patterns ...")
        sub, ref_logL, ref_b, ref_q, cpu = run_cpu_baseline(prob, sample, want_Q, want_grad)
        result["cpu_baseline"] = cpu
        # parity of the same GPU path on the same subsample
        with from_problem(sub, args.precision, grad_branch=want_grad, grad_Q=want_Q, kernel=args.kernel,
                          use_pi=args.config != 4) as small:
            g_logL = small.log_likelihood()
            if want_grad:
                g_b, g_q = small.gradient(branch=True, Q=want_Q)
        parity = {"sample_patterns": sample, "logL_rel_err": abs(g_logL - ref_logL) / abs(ref_logL)}
        if want_grad:
            parity["grad_branch_rel_err"] = float(np.linalg.norm(g_b - ref_b) / np.linalg.norm(ref_b))
        if want_Q:
            parity["grad_Q_rel_err"] = float(np.linalg.norm(g_q - ref_q) / np.linalg.norm(ref_q))
        result["parity_vs_oracle"] = parity
    lik.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
