"""Benchmark: logL + gradient evaluations per second on one MI355X.

Headline workload: GTR 4-state model, 3 epochs, 512-taxon coalescent tree,
100,000 site patterns simulated under the epoch model, 4 discrete-gamma
categories; one step = transition matrices + post-order partials + root
log-likelihood + pre-order adjoint with all 1,022 branch-length gradients,
in FP32 with FP64 reductions.  Inputs are resident on the device before the
timed region; the step returns logL and the gradient to the host.

The same JSON line also carries the metric's other legs, each timed here:
the same workload in FP64 (fast kernels and the plain generic FP64 kernels),
the 128-taxon GY94 codon workload and the 64-problem batched codon workload,
each with its own roofline, and the FP64 oracle timed on one host core and on
all of them.  `--config N` benchmarks one workload alone.

Prints one JSON line (the design doc gives the roofline accounting).
"""
import argparse
import json
import os
import platform
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
    6: "20-state reversible model (amino-acid-sized; padded to 32 on the matrix cores), 4 epochs, 128-taxon tree, "
       "10000 patterns, 1 category, logL + branch-length and rate-matrix gradients",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def padded(K):
    return 4 if K <= 4 else (8 if K <= 8 else (K + 15) // 16 * 16)


def algorithmic_bytes(prob, precision):
    """Algorithmic HBM bytes of one evaluation, per phase."""
    N = prob.n_tips
    P = prob.n_patterns
    C = len(prob.cat_rates)
    Kp = padded(prob.n_states)
    b = 8 if precision == "fp64" else 4
    V = P * C * Kp * b          # one partial (or outside) vector set of a node
    T = P                       # u8 tip states of one tip
    s = 4 * P                   # int32 cumulative scale exponents of one node
    post = (2 * N - 3) * V + N * T + 2 * (N - 1) * s   # write N-1, read N-2 internal children; scales
    pre = (3 * N - 6) * V + N * T + 2 * (N - 2) * s     # read q_u, read internal p, write q; scales
    return {"post_order": post, "pre_order_dP": pre}


def algorithmic_flops(prob):
    """Algorithmic flops of one logL+gradient evaluation: internal-child
    matrix-vector products 2K^2 per (pattern, category); tip children are lookups;
    pre-order products and gradient outer products (N-2) 2K^2 P C each; epoch products
    (2m-1) 2K^3 per (branch, category); the dlogL/dQ adjoint chain three K x K products
    (6K^3) per segment term (W = R V^-T, Y = U^T W, the update of R); padding never counted."""
    from paper_1309_3075_amd import _abi  # the library's host planner gives the segment counts
    N, P, K, C = prob.n_tips, prob.n_patterns, prob.n_states, len(prob.cat_rates)
    post = (N - 2) * 2 * K * K * P * C
    pre = 2 * (N - 2) * 2 * K * K * P * C
    off, _, _ = _abi.plan_segments(prob.parent, prob.height, prob.boundaries, prob.interval_process,
                                   prob.n_processes)
    m = np.diff(off)
    chain = int(np.sum(np.maximum(2 * m - 1, 0))) * 2 * K ** 3 * C
    adjoint = int(np.sum(m)) * C * 6 * K ** 3
    return {"post_order": post, "pre_order_dP": pre, "transition_matrices": chain, "grad_Q": adjoint}


def fp64_reconstruction(prob, use_pi, mode=0):
    """Whether the library forms exp(tQ) in FP64 for this problem in an FP32 instance: with the default
    eigen_precision 0 it does so when some eigenvector matrix has infinity-norm condition number above
    32 (the same rule, evaluated here on the eigensystems the binding hands over); 1 never, 2 always."""
    if mode:
        return mode == 2
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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def host_threads():
    """Threads the host offers this process (the GPU machine limits it through OMP_NUM_THREADS)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    return min(avail, int(env)) if env and env.isdigit() else avail


def oracle_timed(prob, want_grad, want_Q, threads):
    from threadpoolctl import threadpool_limits

    from oracle import epoch_oracle as O
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        logL = O.log_likelihood(prob)
        d_branch, d_Q = (O.gradient(prob, wrt=("branch", "Q") if want_Q else ("branch",)) if want_grad
                         else (None, None))
        dt = time.perf_counter() - t0
    return logL, d_branch, d_Q, dt


def pattern_subset(prob, n):
    import copy
    sub = copy.copy(prob)
    sub.tips = prob.tips[:, :n].copy()
    sub.weights = prob.weights[:n].copy()
    return sub


def _oracle_chunk(job):
    """One worker's share of the all-cores oracle timing: the oracle, unchanged, on a slice of
    the patterns (sites are independent given the tree, so the slices' results add up)."""
    prob, lo, hi, want_grad, want_Q = job
    import copy
    sub = copy.copy(prob)
    sub.tips = prob.tips[:, lo:hi].copy()
    sub.weights = prob.weights[lo:hi].copy()
    logL, d_branch, d_Q, _ = oracle_timed(sub, want_grad, want_Q, 1)
    return logL, d_branch, d_Q


def oracle_all_cores(sub, want_grad, want_Q, n_workers):
    """Wall time of the oracle over the sample split into n_workers pattern slices run by as many
    processes (one BLAS thread each); the pool is started before the clock."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    P = sub.n_patterns
    cuts = [P * k // n_workers for k in range(n_workers + 1)]
    jobs = [(sub, cuts[k], cuts[k + 1], want_grad, want_Q) for k in range(n_workers) if cuts[k + 1] > cuts[k]]
    with ProcessPoolExecutor(max_workers=len(jobs), mp_context=multiprocessing.get_context("spawn")) as ex:
        list(ex.map(_oracle_chunk, [(pattern_subset(sub, 1), 0, 1, False, False)] * len(jobs)))  # start-up
        t0 = time.perf_counter()
        parts = list(ex.map(_oracle_chunk, jobs))
        dt = time.perf_counter() - t0
    logL = sum(p[0] for p in parts)
    return logL, dt


def run_cpu_baseline(prob, sample_patterns, want_Q, want_grad=True):
    """The FP64 oracle on a pattern subsample, on one host thread and on every thread the host
    offers (one process per pattern slice), scaled to evaluations/s of the full problem (linear
    in patterns)."""
    sub = pattern_subset(prob, sample_patterns)
    logL, d_branch, d_Q, dt1 = oracle_timed(sub, want_grad, want_Q, 1)
    n_all = host_threads()
    logL_all, dtn = oracle_all_cores(sub, want_grad, want_Q, n_all)
    assert abs(logL_all - logL) <= 1e-9 * abs(logL), (logL_all, logL)
    scale = prob.n_patterns / sample_patterns
    sample = (f"{sample_patterns} of {prob.n_patterns} patterns, full tree; scaled linearly in patterns "
              f"(FP64 numpy/scipy oracle)")
    return sub, logL, d_branch, d_Q, {
        "value": 1.0 / (dt1 * scale), "unit": "evals/s", "cores": 1, "kind": "oracle",
        "sample": sample + f"; {dt1:.2f} s measured on 1 thread",
        "all_cores": {"value": 1.0 / (dtn * scale), "cores": n_all, "seconds_measured": round(dtn, 3),
                      "how": f"{n_all} processes, one pattern slice and one BLAS thread each"},
        "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def time_instance(lik, steps, warmup, want_grad, want_Q):
    """Evaluations/s of one instance through epoch_evaluate, with per-phase device times.  Every
    step is a whole evaluation: incremental re-evaluation is switched off."""
    import torch
    lik.set_option("incremental", 0)

    def step():
        lL, _, db, dq = lik.evaluate(branch=want_grad, Q=want_Q)
        return lL, db, dq

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    lik.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = lik.timing()
    lik.set_timing(False)
    return steps / wall, wall * 1000.0 / steps, phases, out


def roofline(prob, precision, kernel, phases, steps, want_Q, config, traffic_ok):
    """Roofline of the phase with the largest device time."""
    abytes = algorithmic_bytes(prob, precision)
    aflops = algorithmic_flops(prob)
    dom = max(("post_order", "pre_order_dP", "transition_matrices") + (("grad_Q",) if want_Q else ()),
              key=lambda k: phases[k][0])
    dom_ms = phases[dom][0] / steps
    path = ("nuc" if prob.n_states == 4 else ("codon" if (prob.n_states > 48 or 16 < prob.n_states <= 32)
                                               and precision == "fp32" and len(prob.cat_rates) == 1 else "generic"))
    if kernel == "generic":
        path = "generic"
    cp = 1 if len(prob.cat_rates) <= 1 else (2 if len(prob.cat_rates) <= 2 else (4 if len(prob.cat_rates) <= 4 else 8))
    walk = precision == "fp32" and -(-prob.n_patterns // (64 // cp)) <= 1024
    names = {"nuc": {"post_order": "nuc_walk_mfma (post-order program)" if walk else "nuc_post_level",
                     "pre_order_dP": "nuc_walk_mfma (pre-order program)" if walk else "nuc_pre_level"},
             "codon": {"post_order": "codon_post_level", "pre_order_dP": "codon_pre_level + codon_pre_split"},
             "generic": {"post_order": "post_level_generic", "pre_order_dP": "pre_level_generic + grad_G_generic"}}
    mfma_pstage = kernel == "auto" and padded(prob.n_states) >= 16
    if dom == "grad_Q":
        kname = "qgrad_chain + qgrad_h + qgrad_final" if mfma_pstage else "qgrad_segments + qgrad_reduce"
    else:
        kname = names[path].get(dom, "pstage_mfma (+ split-chain combine)" if mfma_pstage else "pstage_generic")
    if path == "codon" or dom in ("transition_matrices", "grad_Q"):
        achieved = aflops[dom] / (dom_ms * 1e-3) / 1e12
        # the chains run in FP64 when the instance forms exp(tQ) in FP64 (ill-conditioned eigenvectors)
        peak = FP64_PEAK_TFLOPS if (precision == "fp64" or dom in ("transition_matrices", "grad_Q")
                                    and fp64_reconstruction(prob, config != 4)) else FP32_PEAK_TFLOPS
        return {"bound": "mfma", "kernel": kname, "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                "algorithmic_flops_per_eval": aflops[dom], "ms_per_eval": round(dom_ms, 4),
                "hbm_GBps_algorithmic_same_kernel": round(abytes.get(dom, 0) / (dom_ms * 1e-3) / 1e9, 1)}
    achieved = abytes[dom] / (dom_ms * 1e-3) / 1e9
    traffic = None
    if traffic_ok and path == "nuc" and precision == "fp32" and config == 2 and not walk:
        traffic = committed_traffic("nuc_C2_hbm_traffic.txt", kname)
    r = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
         "traffic_unit": "bytes per evaluation (all launches of the kernel)",
         "achieved_is": "algorithmic bytes / kernel time",
         "algorithmic_bytes_per_eval": abytes[dom], "ms_per_eval": round(dom_ms, 4)}
    if traffic:
        r["counter_GBps"] = round(traffic / (dom_ms * 1e-3) / 1e9, 1)
        r["counter_frac"] = round(traffic / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return r


def gpu_parity(sub, precision, kernel, use_pi, ref_logL, ref_b, ref_q, want_grad, want_Q, options=None):
    from paper_1309_3075_amd.likelihood import from_problem
    with from_problem(sub, precision, grad_branch=want_grad, grad_Q=want_Q, kernel=kernel, use_pi=use_pi,
                      options=options) as small:
        g_logL, _, g_b, g_q = small.evaluate(branch=want_grad, Q=want_Q)
    out = {"sample_patterns": sub.n_patterns, "logL_rel_err": abs(g_logL - ref_logL) / abs(ref_logL)}
    for key, g, r in (("grad_branch", g_b, ref_b), ("grad_Q", g_q, ref_q)):
        if g is None or r is None:
            continue
        err = np.abs(g - r).ravel()
        floor = 1e-3 * np.abs(r).max()
        out[f"{key}_rel_err"] = float(np.linalg.norm(g - r) / np.linalg.norm(r))
        out[f"{key}_max_componentwise"] = float(np.max(err / np.maximum(np.abs(r).ravel(), floor)))
    return out


def proposal_leg(prob, steps, use_pi=True):
    """MCMC-style proposals on an FP32 log-likelihood-only instance: each step moves the rate of one
    random branch and evaluates the log-likelihood, re-forming only that branch's transition
    matrices and the partials on its path to the root; timed against full evaluations of the
    same instance (incremental re-evaluation switched off)."""
    import torch
    from paper_1309_3075_amd.likelihood import from_problem
    rng = np.random.default_rng(17)
    n = prob.parent.shape[0]
    branches = [v for v in range(n) if prob.parent[v] >= 0]
    out = {}
    with from_problem(prob, "fp32", use_pi=use_pi) as lik:
        for mode in ("full", "incremental"):
            lik.set_option("incremental", 1 if mode == "incremental" else 0)
            lik.log_likelihood()
            rates = prob.branch_rate.copy()
            work = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(steps):
                v = int(branches[rng.integers(len(branches))])
                rates[v] *= 1.01 if k % 2 == 0 else 1 / 1.01
                lik.set_branch_rates([v], [rates[v]])
                lik.evaluate()
                work.append(lik.work_counts()[1])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            out[mode] = {"proposals_per_s": round(steps / dt, 2), "ms_per_proposal": round(dt * 1000 / steps, 4),
                         "mean_partials_formed": round(float(np.mean(work)), 2)}
    out["speedup_incremental_over_full"] = round(out["incremental"]["proposals_per_s"] / out["full"]["proposals_per_s"], 3)
    out["what"] = "one random branch rate changed per step, then logL (FP32, no gradient)"
    return out


def rate_matrix_step_leg(prob, steps):
    """Steps whose rate matrices change on every call, as in gradient-based fitting of the
    substitution model: (a) every process's Q handed to an FP32 instance (host eigendecomposition,
    asynchronous upload) followed by one evaluation with branch and rate-matrix gradients, with and
    without the reconstruction-residual check; (b) the torch.autograd step: GY94 Q_s(kappa, omega_s)
    built in torch, forward through the library, backward to kappa, omega_s and the branch lengths."""
    import torch
    from paper_1309_3075_amd.autograd import EpochLogLikelihood, EpochModel, gy94_q
    from paper_1309_3075_amd.eigen import eigensystem
    from paper_1309_3075_amd.likelihood import from_problem
    out = {}
    with from_problem(prob, "fp32", grad_branch=True, grad_Q=True) as lik:
        lik.set_option("incremental", 0)
        for check in (True, False):
            for k in range(steps + 2):
                if k == 2:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                for s, Q in enumerate(prob.Q):
                    lik.set_rate_matrix(s, Q * (1 + 1e-6 * (k % 3)), prob.pi_process[s], check_residual=check)
                lik.evaluate(branch=True, Q=True)
            torch.cuda.synchronize()
            out["set_Q_then_eval_ms" + ("_residual_check" if check else "")] = \
                round((time.perf_counter() - t0) * 1e3 / steps, 4)
    t0 = time.perf_counter()
    for _ in range(steps):
        for s, Q in enumerate(prob.Q):
            eigensystem(Q, prob.pi_process[s])
    out["host_eigendecompositions_ms"] = round((time.perf_counter() - t0) * 1e3 / steps, 4)
    model = EpochModel(prob, "fp32", reversible_pi=prob.pi_process)
    try:
        pi = torch.tensor(prob.pi_process[0])
        kappa = torch.tensor(2.0, dtype=torch.float64, requires_grad=True)
        omegas = [torch.tensor(0.3 + 0.1 * s, dtype=torch.float64, requires_grad=True)
                  for s in range(prob.n_processes)]
        ell = model.branch_lengths().requires_grad_(True)
        for k in range(steps + 2):
            if k == 2:
                t0 = time.perf_counter()
            with torch.no_grad():
                kappa.add_(0.01 if k % 2 else -0.01)
            EpochLogLikelihood.apply(model, ell, *[gy94_q(kappa, om, pi) for om in omegas]).backward()
        torch.cuda.synchronize()
        out["autograd_step_ms"] = round((time.perf_counter() - t0) * 1e3 / steps, 4)
    finally:
        model.close()
    out["what"] = (f"{prob.n_processes} rate matrices changed per step; FP32 instance; the host part is "
                   "numpy's eigendecomposition of each Q")
    return out


def precision_leg(prob, config, steps, want_grad, want_Q, use_pi, parity):
    """The other arithmetics of the same workload, each with its parity against the oracle on the
    CPU-baseline sample when one was drawn: the transition matrices and dlogL/dQ chains of the FP32
    instance formed the other way (FP32 products where the conditioning rule picks FP64, FP64 where it
    picks FP32), and the FP64 instance."""
    from paper_1309_3075_amd import _abi
    from paper_1309_3075_amd.likelihood import from_problem
    out = {}
    if fp64_reconstruction(prob, use_pi):
        variants = [("fp32_products", "fp32", {"eigen_precision": 1})]
    else:
        variants = [("fp64_reconstruction", "fp32", {"eigen_precision": 2})]
    variants.append(("fp64_instance", "fp64", {}))
    for name, precision, options in variants:
        leg = {"options": options}
        try:
            with from_problem(prob, precision, grad_branch=want_grad, grad_Q=want_Q, use_pi=use_pi,
                              options=options) as lik:
                v, ms, _, _ = time_instance(lik, steps, 2, want_grad, want_Q)
            leg.update({"evals_per_s": round(v, 3), "ms_per_eval": round(ms, 4)})
            if parity is not None:
                sub, ref_logL, ref_b, ref_q = parity
                leg["parity_vs_oracle"] = gpu_parity(sub, precision, "auto", use_pi, ref_logL, ref_b, ref_q,
                                                     want_grad, want_Q, options)
        except _abi.EpochError as e:  # e.g. a NaN log-likelihood from FP32 products of ill-conditioned systems
            leg["error"] = str(e)
        out[name] = leg
    return out


def run_codon_leg(steps, warmup, with_parity):
    """The 128-taxon GY94 codon workload (FP32, branch and rate-matrix gradients)."""
    from paper_1309_3075_amd import workloads as W
    from paper_1309_3075_amd.likelihood import from_problem
    prob = W.make_config(3)
    lik = from_problem(prob, "fp32", grad_branch=True, grad_Q=True)
    eps, ms, phases, _ = time_instance(lik, steps, warmup, True, True)
    lik.close()
    # the same evaluation in FP64: on the FP64 matrix cores, and on the plain generic FP64 kernels
    with from_problem(prob, "fp64", grad_branch=True, grad_Q=True) as l64:
        e64, ms64, _, _ = time_instance(l64, max(3, steps // 2), 2, True, True)
    with from_problem(prob, "fp64", grad_branch=True, grad_Q=True, kernel="generic") as lg:
        eg, msg, _, _ = time_instance(lg, 3, 1, True, True)
    proposals = proposal_leg(prob, 4 * steps)
    q_steps = rate_matrix_step_leg(prob, steps)
    aflops = algorithmic_flops(prob)
    total = sum(aflops.values())
    leg = {"workload": WORKLOADS[3], "evals_per_s": round(eps, 2), "ms_per_eval": round(ms, 4),
           "roofline": roofline(prob, "fp32", "auto", phases, steps, True, 3, False),
           "whole_eval_TFLOPs": round(total / (ms * 1e-3) / 1e12, 3),
           "whole_eval_frac_fp32_peak": round(total / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS, 4),
           "phases_ms_per_eval": {k: round(v[0] / steps, 4) for k, v in phases.items()},
           "fp64": {"evals_per_s": round(e64, 2), "ms_per_eval": round(ms64, 4),
                    "generic_fp64_evals_per_s": round(eg, 2), "generic_fp64_ms_per_eval": round(msg, 4),
                    "speedup_fp32_over_fp64": round(eps / e64, 3),
                    "speedup_fp32_over_generic_fp64": round(eps / eg, 3)},
           "one_branch_proposals": proposals, "rate_matrix_steps": q_steps}
    if with_parity:
        sub = pattern_subset(prob, 1000)
        ref_logL, ref_b, ref_q, _ = oracle_timed(sub, True, True, host_threads())
        leg["parity_vs_oracle"] = gpu_parity(sub, "fp32", "auto", True, ref_logL, ref_b, ref_q, True, True)
    return leg


def run_batch_leg(n, scale, steps, warmup, precision="fp32", grad_q=False, tune=None):
    """Batched codon workload: independent 64-state problems in one replayed HIP graph."""
    import torch
    from paper_1309_3075_amd import workloads as W
    from paper_1309_3075_amd.likelihood import EpochBatchEvaluator, from_problem

    log(f"bench: generating {n} batched codon problems ...")
    t0 = time.perf_counter()
    probs = W.make_batch(n, scale=scale)
    log(f"bench: generated in {time.perf_counter() - t0:.1f} s; patterns {sum(p.n_patterns for p in probs)}")
    members = [from_problem(p, precision, grad_branch=True, grad_Q=grad_q) for p in probs]
    batch = EpochBatchEvaluator(members, tune_cache=tune)
    for _ in range(warmup):
        batch.evaluate(grad_branch=True, grad_Q=grad_q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        logL = batch.evaluate(grad_branch=True, grad_Q=grad_q)
    wall = time.perf_counter() - t0
    ms = wall * 1000 / steps
    flops = 0
    for p in probs:
        f = algorithmic_flops(p)
        flops += f["post_order"] + f["pre_order_dP"] + f["transition_matrices"] + (f["grad_Q"] if grad_q else 0)
    achieved = flops / (ms * 1e-3) / 1e12
    leg = {"workload": f"{n} batched GY94 codon problems (61 states padded to 64, 4 epochs), 64-256 taxa and "
                       f"1000-20000 patterns each (x{scale}), one replayed hipGraph per step, logL + branch gradients"
                       + (" + rate-matrix gradients" if grad_q else ""),
           "problems_per_s": round(n * steps / wall, 3), "ms_per_batch": round(ms, 4),
           "tuned_target_blocks": batch.target_blocks(), "tuned_split_blocks": batch.split_blocks(),
           "roofline": {"bound": "mfma", "kernel": "whole batched graph (codon_post/pre_level dominant)",
                        "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": None,
                        "algorithmic_flops_per_batch": flops},
           "logL_first": float(logL[0])}
    batch.close()
    for m in members:
        m.close()
    return leg


def run_nuc_batch_leg(n, steps):
    """Batch of small 4-state problems (16-64 taxa, 300-3,000 patterns, FP32, branch gradients): each member
    runs its own launches, spread over concurrent branches of one replayed graph; timed against the same
    members evaluated one after another."""
    import torch
    from paper_1309_3075_amd import workloads as W
    from paper_1309_3075_amd.likelihood import EpochBatchEvaluator, from_problem
    rng = np.random.default_rng(5)
    probs = [W.make_config(1, replicate=i, n_tips=int(rng.integers(16, 65)), n_patterns=int(rng.integers(300, 3001)))
             for i in range(n)]
    members = [from_problem(p, "fp32", grad_branch=True) for p in probs]
    try:
        for m in members:
            m.evaluate(branch=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for m in members:
                m.evaluate(branch=True)
        torch.cuda.synchronize()
        serial = n * steps / (time.perf_counter() - t0)
        batch = EpochBatchEvaluator(members)
        batch.evaluate(grad_branch=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            batch.evaluate(grad_branch=True)
        wall = time.perf_counter() - t0
        batch.close()
    finally:
        for m in members:
            m.close()
    return {"workload": f"{n} small 4-state problems (C1 model, 16-64 taxa, 300-3000 patterns), FP32, logL + branch "
                        "gradients, one replayed hipGraph per step",
            "problems_per_s": round(n * steps / wall, 1), "ms_per_batch": round(wall * 1000 / steps, 4),
            "serial_single_instances_problems_per_s": round(serial, 1)}


def run_batch(args):
    leg = run_batch_leg(args.batch or 64, args.batch_scale, args.steps, args.warmup, args.precision, args.grad_q,
                        os.path.join(ROOT, "paper_1309_3075_amd", "tune_cache.json"))
    result = {
        "metric": "logL+gradient evals/sec", "value": leg["problems_per_s"], "unit": "evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": leg["ms_per_batch"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic (seeded coalescent trees, codon patterns simulated under the epoch model)",
        "config": {"workload": leg["workload"], "config_index": 5, "n_problems": args.batch or 64,
                   "precision": args.precision, "tuned_target_blocks": leg["tuned_target_blocks"]},
        "roofline": leg["roofline"], "logL_first": leg["logL_first"],
    }
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=None,
                    help="benchmark one workload alone (1-5); default: the headline workload with every leg")
    ap.add_argument("--precision", default=None, choices=["fp32", "fp64"],
                    help="default: FP64 for the 16-taxon workload (as it is stated), FP32 otherwise")
    ap.add_argument("--kernel", default="auto", choices=["auto", "generic"])
    ap.add_argument("--patterns", type=int, default=None, help="override the pattern count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-legs", action="store_true",
                    help="time the workload only (no other-precision legs): for profiling one configuration")
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
    headline = args.config is None
    config = 2 if headline else args.config
    if args.precision is None:
        args.precision = "fp64" if config == 1 else "fp32"
    if config == 5:
        return run_batch(args)
    want_Q = args.grad_q or config in (3, 4, 6)
    want_grad = config != 1  # the 16-taxon workload is a plain log-likelihood
    use_pi = config != 4
    log(f"bench: generating config C{config} ...")
    t0 = time.perf_counter()
    prob = W.make_config(config, n_patterns=args.patterns)
    log(f"bench: generated in {time.perf_counter() - t0:.1f} s: N={prob.n_tips} P={prob.n_patterns} "
        f"K={prob.n_states} C={len(prob.cat_rates)} S={prob.n_processes} M={prob.n_intervals}")
    lik = from_problem(prob, args.precision, grad_branch=want_grad, grad_Q=want_Q, kernel=args.kernel,
                       use_pi=use_pi)
    # the timed region: K whole evaluations, each with one host synchronisation
    value, ms_per_step, phases, (logL, _, _) = time_instance(lik, args.steps, args.warmup, want_grad, want_Q)
    log(f"bench: {ms_per_step:.3f} ms/step, phases {phases}")
    lik.close()
    roof = roofline(prob, args.precision, args.kernel, phases, args.steps, want_Q, config,
                    args.patterns is None)
    abytes = algorithmic_bytes(prob, args.precision)
    result = {
        "metric": "logL+gradient evals/sec" if want_grad else "logL evals/sec", "value": round(value, 3),
        "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic (seeded coalescent tree, patterns simulated under the epoch model)",
        "config": {"workload": WORKLOADS[config], "config_index": config, "n_tips": prob.n_tips,
                   "n_patterns": prob.n_patterns, "n_states": prob.n_states,
                   "n_categories": len(prob.cat_rates), "precision": args.precision, "kernel": args.kernel,
                   "grad_Q": want_Q},
        "roofline": roof,
        "whole_step_hbm_fraction": round(sum(abytes.values()) / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "phases_ms_per_eval": {k: round(v[0] / args.steps, 4) for k, v in phases.items()},
        "logL": logL,
    }

    from paper_1309_3075_amd import _abi
    probe = {k: round(_abi.bandwidth_probe(1 << 31, k, 20), 1) for k in ("copy", "read", "write")}
    result["measured_hbm_GBps"] = probe
    if roof["unit"] == "GB/s":
        roof["frac_of_measured_copy"] = round(roof["achieved"] / probe["copy"], 4)
    aflops = algorithmic_flops(prob)
    result["algorithmic_flops_per_eval"] = aflops
    # the metric's "partials GFLOP/s": algorithmic flops of the post-order pass (partials) and of the pre-order
    # pass with dlogL/dP, each over its own device time
    result["partials_GFLOP_per_s"] = {
        k: round(aflops[k] / (phases[k][0] / args.steps * 1e-3) / 1e9, 1)
        for k in ("post_order", "pre_order_dP") if k in phases and phases[k][0] > 0}
    log(f"bench: bandwidth probe {probe}")

    sample = None
    if not args.no_cpu_baseline:
        sample = args.cpu_sample or min(prob.n_patterns, {1: 1000, 2: 30000, 3: 3000, 4: 1, 6: 3000}.get(config, 1000))
        log(f"bench: cpu baseline on {sample} patterns ...")
        sub, ref_logL, ref_b, ref_q, cpu = run_cpu_baseline(prob, sample, want_Q, want_grad)
        result["cpu_baseline"] = cpu
        result["parity_vs_oracle"] = gpu_parity(sub, args.precision, args.kernel, use_pi, ref_logL, ref_b, ref_q,
                                                want_grad, want_Q)
    if not headline and config in (3, 4, 6) and args.precision == "fp32" and args.kernel == "auto" \
            and args.patterns is None and not args.no_extra_legs:
        log("bench: FP32-products and FP64 legs ...")
        result["fp64_reconstruction_default"] = fp64_reconstruction(prob, use_pi)
        result["other_precisions"] = precision_leg(prob, config, max(3, args.steps // 2), want_grad, want_Q, use_pi,
                                                   (sub, ref_logL, ref_b, ref_q) if sample else None)

    if headline and args.precision == "fp32" and args.kernel == "auto" and args.patterns is None:
        # the metric's FP64 half on the same workload: the fast kernels and the plain generic FP64 path
        log("bench: FP64 leg ...")
        steps64 = max(3, args.steps // 2)
        with from_problem(prob, "fp64", grad_branch=True) as l64:
            v64, ms64, ph64, _ = time_instance(l64, steps64, 2, True, False)
        with from_problem(prob, "fp64", grad_branch=True, kernel="generic") as lg:
            vg, msg, _, _ = time_instance(lg, 3, 1, True, False)
        fp64 = {"evals_per_s": round(v64, 3), "ms_per_eval": round(ms64, 4),
                "roofline": roofline(prob, "fp64", "auto", ph64, steps64, False, 2, False),
                "generic_fp64_evals_per_s": round(vg, 3), "generic_fp64_ms_per_eval": round(msg, 4),
                "speedup_fp32_over_fp64": round(value / v64, 3),
                "speedup_fp32_over_generic_fp64": round(value / vg, 3)}
        if sample:
            fp64["parity_vs_oracle"] = gpu_parity(sub, "fp64", "auto", True, ref_logL, ref_b, None, True, False)
        result["fp64"] = fp64
        log("bench: proposal leg ...")
        result["one_branch_proposals"] = proposal_leg(prob, 100)
        log("bench: codon leg ...")
        result["codon_C3"] = run_codon_leg(max(5, args.steps), 2, sample is not None)
        log("bench: batched codon leg ...")
        result["batch_C5"] = run_batch_leg(64, 1.0, max(3, args.steps // 4), 1,
                                           tune=os.path.join(ROOT, "paper_1309_3075_amd", "tune_cache.json"))
        log("bench: batched small 4-state leg ...")
        result["batch_small_nucleotide"] = run_nuc_batch_leg(64, max(5, args.steps))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
