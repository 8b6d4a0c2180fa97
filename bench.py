#!/usr/bin/env python
"""Branch-gradient evaluations per second on one MI355X.

One step = one full evaluation of the hot path on the 1000-taxon, 10,000-
pattern HKY+Gamma4 workload (Yule tree, b ~ Exp(mean 0.01), 5% ambiguous tip
entries, pattern weights 1+Poisson(3)): P(t) and dP/dt for every branch and
category, post-order partials, root log-likelihood, pre-order partials fused
with the per-branch gradient contraction, and the final float64 sums -- logL
plus all 1998 branch derivatives.  Inputs are resident in HBM before timing
starts.  Two timed regions, each bracketed by device synchronisation: K
back-to-back asynchronous evaluations launched on one stream, and K replays
of one evaluation captured as a HIP graph; the value is the faster, and the
JSON names it and gives both.  Neither region records profiling events.

Also reported: p50/p99 latency of synchronous requests (new branch lengths
in, logL + gradient back in host memory), the live per-kernel-class device
time from HIP events in a separate K-evaluation run (roofline of the
dominant kernel), the float64 path's
throughput, accuracy against the FP64 oracle on a pattern sample, and the
oracle's own throughput on the host CPU (cpu_baseline).

    python bench.py [--gpus 1] [--steps 50] [--warmup 5]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "branch-gradient evals/s at 1000 taxa x 10k patterns; p50/p99 request latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2303_04390_amd", "csrc", "phg_kernels.hip")

# HBM bytes per evaluation by kernel class on the hky1000 FP32 workload under the
# work-queue schedule, from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE;
# scaled by a plain 1 GiB copy: x2.0 and x1.0; profiles/queue_kernels_hky1000_fp32.md),
# recorded with the kernel source whose SHA-256 is given.  When the kernel
# source or the schedule differs the figure no longer applies and traffic is null.
MEASURED_TRAFFIC = {
    "kernel_source_sha256": "ee041b382291f30531def3f9dfaea3b65f3421f8e40605f49b529227136e9728",
    "schedule": "queue",
    "bytes_per_eval": {"pre_grad": 720013824, "post": 493579571},
}


def kernel_source_sha256():
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def algorithmic_bytes(parent, n_tips, C, R, S, tsz):
    """Bytes each pass must move per evaluation under the level schedule.

    post: read each internal child's partial (R*S*tsz) and int32 exponent,
          each tip child's 1-byte code; write each non-root internal partial
          and exponent; at the root read W_c and write the float64 log site
          likelihood.
    pre+grad: read q of each non-root parent, read p and write q of each
          internal child, read each tip child's code, read W_c once per
          level, write one float64 gradient partial per branch and tile.
    All per pattern, times C (the partials per tile, times the tile count).
    """
    n = parent.shape[0]
    root = n - 1
    vec = R * S * tsz
    post = pre = 0
    pre_levels = set()
    depth = node_depths(parent)
    for k in range(n_tips, n):
        kids = np.nonzero(parent == k)[0]
        for x in kids:
            if x >= n_tips:
                post += vec + 4
                pre += 2 * vec
            else:
                post += 1
                pre += 1
        if k != root:
            post += vec + 4
            pre += vec
        else:
            post += 16
        pre_levels.add(depth[k])
    pre += 8 * len(pre_levels)
    tiles = -(-C // 64)
    return post * C, pre * C + 8 * (n - 1) * tiles


def algorithmic_bytes_blocked(parent, n_tips, C, R, S, tsz, block_depth=3):
    """Bytes each pass must move per evaluation under the blocked schedule.

    Block roots are the internal nodes at depths 0, 3, 6, ...; a workgroup
    keeps everything inside its block in registers, so HBM sees only the
    block roots' vectors and the tips' codes.
    post: each tip's code once; each non-root block root's partial and
          exponent written once (by its own block) and read once (by the
          block above); at the root W_c read and the log site likelihood
          written.
    pre+grad: each tip's code once; for each non-root block root, its
          partial read and its q written by the block above, and that q
          read by its own block; W_c read once per block; one float64
          gradient partial per branch and tile.
    """
    n = parent.shape[0]
    root = n - 1
    vec = R * S * tsz
    depth = node_depths(parent)
    roots = [v for v in range(n_tips, n) if depth[v] % block_depth == 0]
    nb = len(roots) - 1                       # non-root block roots
    post = n_tips + nb * 2 * (vec + 4) + 16
    pre = n_tips + nb * 3 * vec + 8 * len(roots)
    tiles = -(-C // 64)
    return post * C, pre * C + 8 * (n - 1) * tiles


def node_depths(parent):
    n = parent.shape[0]
    depth = np.full(n, -1, np.int64)
    depth[n - 1] = 0
    stack = [n - 1]
    kids = [[] for _ in range(n)]
    for x in range(n - 1):
        kids[parent[x]].append(x)
    while stack:
        v = stack.pop()
        for x in kids[v]:
            depth[x] = depth[v] + 1
            stack.append(x)
    return depth


def _yule_parents(args):
    """Worker: fresh Yule topologies for (n_tips, seed) pairs."""
    from paper_2303_04390_amd import synth
    return [synth.yule_topology(int(n), np.random.default_rng(int(sd))) for n, sd in args]


def serving_measurement(args, B, synth):
    """Poisson stream of likelihood+gradient requests through the server.

    Requests arrive at args.serving_rate per second for args.serving_seconds.
    Half are branch-length perturbations b * exp(N(0, 0.05)) of a registered
    tree (an HMC step); the other half bring a new tree: a freshly drawn Yule
    topology with taxa ~ round(LogUniform[64, 4096]), branch lengths ~
    Exp(0.01), HKY+Gamma4 drawn as in the 1000-taxon workload (kappa ~
    U[1,5], alpha ~ U[0.2,2], pi ~ Dir(10^4)), and patterns ~
    round(LogUniform[500, 20000]) whose tip states are a block of one
    alignment simulated beforehand on a 4096-taxon tree (not re-simulated
    per tree, which would take seconds each).  A new tree is registered when
    its request arrives, by a pool of host threads, so registration (host
    copy and validation) is inside that request's latency; its upload and
    first evaluation follow on the GPU.  The 32 most recently registered
    trees stay registered.  Latency = results in host memory minus arrival.
    Also reported: the GPU-busy fraction (serving kernels' device time over
    the stream's wall time).
    """
    import math
    import multiprocessing as mp
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.default_rng(args.seed + 1000)
    t0 = time.perf_counter()
    n_req = int(args.serving_rate * args.serving_seconds)
    arrivals = np.cumsum(rng.exponential(1.0 / args.serving_rate, n_req))
    is_step = rng.random(n_req) < 0.5
    is_step[0] = False
    new_idx = np.nonzero(~is_step)[0]
    n_new = len(new_idx)
    sizes_N = np.round(np.exp(rng.uniform(math.log(64), math.log(4096), n_new))).astype(int)
    sizes_C = np.round(np.exp(rng.uniform(math.log(500), math.log(20000), n_new))).astype(int)
    seeds = rng.integers(0, 1 << 30, n_new)
    # fresh topologies, drawn in worker processes
    jobs = [list(zip(sizes_N[k::args.cpu_workers], seeds[k::args.cpu_workers])) for k in range(args.cpu_workers)]
    with mp.get_context("spawn").Pool(args.cpu_workers) as pool:
        parts = pool.map(_yule_parents, jobs)
    parents = [None] * n_new
    for k in range(args.cpu_workers):
        parents[k::args.cpu_workers] = parts[k]
    base = synth.config_problem("hky1000", seed=args.seed + 77, n_tips=4096, n_patterns=20000)
    gen_s = time.perf_counter() - t0

    def new_problem(k):
        r = np.random.default_rng(int(seeds[k]) + 1)
        N, C = int(sizes_N[k]), int(sizes_C[k])
        pi = r.dirichlet([10.0] * 4)
        Q = synth.hky_model(r.uniform(1.0, 5.0), pi)
        rates, w = synth.discrete_gamma(r.uniform(0.2, 2.0), 4)
        V, Vinv, lam = synth.eigensystem(Q, pi)
        r0 = int(r.integers(0, 4096 - N + 1))
        c0 = int(r.integers(0, 20000 - C + 1))
        return synth.Problem(parent=parents[k], b=r.exponential(0.01, 2 * N - 2), V=V, Vinv=Vinv, lam=lam,
                             pi=pi, rates=rates, weights=w,
                             codes=np.ascontiguousarray(base.codes[r0:r0 + N, c0:c0 + C], np.int32),
                             pattern_weights=np.ones(C), Q=Q)

    budget = 96 << 30
    srv = B.phg_server_create(0, budget, 32)
    regs = ThreadPoolExecutor(max_workers=8)
    window = []                 # (tree id, b, n_branches), most recent last
    submitted = []              # (req id, n_branches, kind, host seconds from arrival to submit)
    futs = {}
    reg_s = []

    def register(k, i):
        # on a host thread at the request's arrival: build, register, submit
        prob = new_problem(k)
        ta = time.perf_counter()
        tid = B.phg_server_register_tree(srv, prob, B.PHG_FP32_SCALED)
        rs = time.perf_counter() - ta
        rid = B.phg_server_submit(srv, tid, prob.b)
        return tid, prob.b, 2 * prob.n_tips - 2, rid, rs, time.perf_counter() - start - arrivals[i]

    nrng = np.random.default_rng(args.seed + 5)
    try:
        busy0, wall0 = B.phg_server_busy(srv)
        start = time.perf_counter()
        knew = 0
        for i in range(n_req):
            while True:
                dt = arrivals[i] - (time.perf_counter() - start)
                if dt <= 0:
                    break
                time.sleep(min(dt, 0.0005))
            # new trees whose registration and submission finished join the window
            for j in sorted(futs):
                if futs[j].done():
                    tid, b, E, rid, rs, pre_s = futs.pop(j).result()
                    reg_s.append(rs)
                    submitted.append((rid, E, "new", pre_s))
                    window.append((tid, b, E))
                    if len(window) > 32:
                        B.phg_server_release_tree(srv, window.pop(0)[0])
            if is_step[i] and not window:
                # no tree registered yet: wait for the first one
                j = min(futs)
                tid, b, E, rid, rs, pre_s = futs.pop(j).result()
                reg_s.append(rs)
                submitted.append((rid, E, "new", pre_s))
                window.append((tid, b, E))
            if is_step[i]:
                tid, b, E = window[int(nrng.integers(len(window)))]
                b2 = b * np.exp(nrng.normal(0.0, 0.05, E))
                rid = B.phg_server_submit(srv, tid, b2)
                submitted.append((rid, E, "step", time.perf_counter() - start - arrivals[i]))
            else:
                futs[i] = regs.submit(register, knew, i)
                knew += 1
        for j in sorted(futs):
            tid, b, E, rid, rs, pre_s = futs[j].result()
            reg_s.append(rs)
            submitted.append((rid, E, "new", pre_s))
        lat = {"step": [], "new": []}
        t_last = None
        for rid, E, kind, pre_s in submitted:
            while True:
                done, logl, grad, ts, td = B.phg_server_poll_timed(srv, rid, E)
                if done:
                    break
                time.sleep(0.0002)
            lat[kind].append(pre_s * 1e3 + (td - ts) * 1e-6)
        span = time.perf_counter() - start
        busy1, wall1 = B.phg_server_busy(srv)
        stats = B.phg_server_stats(srv)
    finally:
        regs.shutdown(wait=True)
        B.phg_server_destroy(srv)
    allv = np.array(lat["step"] + lat["new"])

    def pct(v):
        v = np.asarray(v)
        return {"p50": round(float(np.percentile(v, 50)), 3), "p99": round(float(np.percentile(v, 99)), 3),
                "max": round(float(v.max()), 3), "requests": int(v.size)}

    return {
        "workload": "Poisson arrivals; half branch-length perturbations x exp(N(0,0.05)) of registered trees, "
                    "half new trees (fresh Yule topology, taxa LogUniform[64,4096], b~Exp(0.01), HKY+Gamma4 "
                    "as the 1000-taxon workload, patterns LogUniform[500,20000] from a pre-simulated "
                    "alignment), FP32 + rescaling, registration inside the latency window",
        "rate_req_per_s": args.serving_rate, "seconds": args.serving_seconds, "requests": n_req,
        "new_trees": int(n_new), "mean_taxa_x_patterns_new": float(np.mean(sizes_N * sizes_C)),
        "latency_ms": pct(allv), "latency_ms_steps": pct(lat["step"]), "latency_ms_new_trees": pct(lat["new"]),
        "registration_ms": pct(np.array(reg_s) * 1e3),
        "throughput_req_per_s": round(n_req / span, 1),
        "gpu_busy_fraction": round((busy1 - busy0) / max(wall1 - wall0, 1), 4),
        "server_stats": stats, "slots": 32, "budget_bytes": budget,
        "generation_s": round(gen_s, 1),
    }


MFMA_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}      # MI355X dense MFMA peaks
# MI355X vector-ALU peaks (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz x 2 flops
# per FMA, FP64 at full rate; the FP32 figure counts packed FMAs, which
# this build does not emit, so its issue-limited FP32 rate is the FP64 one)
VALU_PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
VALU_UNPACKED_TFLOPS = 78.6


def kernel_family(B, S, R, fp32):
    """The library's level-kernel family for these sizes ('valu', 'mfma', ...)."""
    prec = B.PHG_FP32_SCALED if fp32 else B.PHG_FP64
    return B.KERNEL_FAMILY_NAMES[B.phg_kernel_family_of(S, R, prec)]


def accuracy(logl, grad, ref, n_sample):
    """Error against the oracle: log-likelihood relative error; per gradient
    component the scaled error |g-g*| / max(|g*|, 1e-2 A) (A = sum_c W_c |d_c|),
    the pure relative error |g-g*| / |g*|, how many components relied on the
    1e-2 A floor, and how many exceed 1e-4 in pure relative terms."""
    g, gs, A = np.asarray(grad), ref["grad"], ref["absgrad"]
    err = np.abs(g - gs)
    denom = np.maximum(np.abs(gs), 1e-2 * A)
    pure = err / np.maximum(np.abs(gs), 1e-300)
    return {"sample_patterns": int(n_sample),
            "logl_rel_err": float(abs(logl - ref["logl"]) / abs(ref["logl"])),
            "grad_max_scaled_err": float(np.max(err / denom)),
            "grad_max_pure_rel_err": float(np.max(pure)),
            "grad_components": int(g.size),
            "grad_floor_used": int(np.sum(1e-2 * A > np.abs(gs))),
            "grad_pure_rel_err_above_1e-4": int(np.sum(pure > 1e-4))}


def algorithmic_flops(n_tips, C, R, S):
    """The method's own flops per evaluation at S states (2 S^2 per S x S
    matrix-vector product, per pattern and category): the post-order forms
    P_x p_x once per internal child (N-2 of them; a tip child's P e_y is a
    column of P, no product); the pre-order forms P_x' p_x' for the sibling
    vector, dP_x p_x and q_x = P_x^T u_x once per internal child (eq:preorder,
    eq:gradient).  4 (N-2) products in all; the per-pattern dot products are
    lower order and not counted."""
    return 4.0 * (n_tips - 2) * 2.0 * S * S * C * R


def executed_flops(parent, n_tips, C, R, S, family):
    """Products the kernels issue per evaluation, at S padded to the 16-state
    MFMA tile (MFMA kernels) or to 20, 24 or 32 states (vector-ALU kernels).
    A tip child given by its code is a gather from the P(t) tables, not a
    product, so the kernels issue P_x p_x in the post-order and P_x p_x,
    dP_x p_x and P_x^T u_x in the pre-order for internal children only: the
    method's 4 (N-2) products, padded."""
    n = parent.shape[0]
    internal_children = int(np.sum(np.arange(n - 1) >= n_tips))
    if family == "valu":
        Sp = 20 if S <= 20 else (24 if S <= 24 else 32)
    else:
        Sp = -(-S // 16) * 16
    return 4 * internal_children * 2.0 * Sp * Sp * C * R


def state_space_measurement(args, B, synth, stream, out):
    """Throughput and arithmetic-unit utilisation of the larger state spaces: the
    500-taxon amino-acid and 128-taxon codon workloads, a 122-state
    (Markov-modulated size) case and a 240-state case (the largest state
    count of byte tip codes, near the paper's 256-state phylogeographic
    models), in FP32 and FP64."""
    import torch
    import oracle
    res = {}
    cases = [(w, synth.config_problem(w, seed=args.seed)) for w in args.states.split(",")]
    for name, prob in cases:
        N, C, S, R = prob.n_tips, prob.n_patterns, prob.n_states, prob.n_categories
        alg_f = algorithmic_flops(N, C, R, S)
        # accuracy against the oracle on a pattern sample of the same workload
        # (not for the 10,000-taxon 256-state shape: the oracle's P(t) alone
        # would take minutes there; its per-chunk tables are checked against
        # full tables bit for bit in the parity tests)
        sample = prob.subset_patterns(np.arange(min(args.state_sample_patterns, C)))
        ref = (oracle.evaluate_problem(sample) if args.state_sample_patterns > 0 and name != "s256big"
               else None)
        for prec, tag in ((B.PHG_FP32_SCALED, "f32"), (B.PHG_FP64, "f64")):
            if tag not in args.state_precisions.split(","):
                continue
            family = kernel_family(B, S, R, tag == "f32")
            exe_f = executed_flops(prob.parent, N, C, R, S, family)
            # the vector-ALU kernels run their work-queue traversal (one launch
            # per pass) unless --state-schedule levels
            sched = (B.PHG_SCHEDULE_QUEUE if family == "valu" and args.state_schedule == "queue"
                     else B.PHG_SCHEDULE_AUTO)
            h = B.phg_create(N, C, S, R, prec, 0)
            try:
                if sched != B.PHG_SCHEDULE_AUTO:
                    B.phg_set_schedule(h, sched)
                B.phg_bind_stream(h, stream.cuda_stream)
                B.set_problem(h, prob)
                B.phg_prepare(h)
                for _ in range(2):
                    B.phg_gradient_async(h, out.data_ptr(), out.data_ptr() + 8)
                torch.cuda.synchronize()
                B.phg_profile_enable(h, True)
                k = args.state_steps
                t0 = time.perf_counter()
                for _ in range(k):
                    B.phg_gradient_async(h, out.data_ptr(), out.data_ptr() + 8)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / k
                ms_cls, n_prof, _ = B.phg_profile_read(h)
                slots = B.phg_table_slots(h)
                sched_name = {B.PHG_SCHEDULE_LEVELS: "levels", B.PHG_SCHEDULE_BLOCKS: "blocks",
                              B.PHG_SCHEDULE_QUEUE: "queue"}[B.phg_get_schedule(h)]
                ws = B.phg_workspace_size(N, C, S, R, prec)
            finally:
                B.phg_destroy(h)
            cls = dict(zip(B.PROF_NAMES, (ms_cls / max(n_prof, 1)).tolist()))
            t_mm = (cls["post"] + cls["pre_grad"]) * 1e-3
            tflops = alg_f / t_mm / 1e12
            peak = (VALU_PEAK_TFLOPS if family == "valu" else MFMA_PEAK_TFLOPS)[tag]
            entry = {
                "n_tips": N, "n_patterns": C, "n_states": S, "n_categories": R,
                "kernels": family, "schedule": sched_name,
                "evals_per_s": round(1.0 / dt, 1), "ms_per_eval": round(dt * 1e3, 4),
                "ms_per_class": {k2: round(v, 4) for k2, v in cls.items()},
                "algorithmic_gflop_per_eval": round(alg_f / 1e9, 2),
                "tflops": round(tflops, 2), "peak_tflops": peak, "frac": round(tflops / peak, 4),
                # the same method flops against the dense MFMA peak, whichever
                # unit ran them (comparable across kernel families)
                "mfma_peak_frac": round(tflops / MFMA_PEAK_TFLOPS[tag], 4),
                "executed_gflop_per_eval": round(exe_f / 1e9, 2),
                "executed_tflops": round(exe_f / t_mm / 1e12, 2),
                "table_slots": slots, "workspace_bytes": ws}
            if family == "valu" and tag == "f32":
                entry["frac_unpacked_valu"] = round(tflops / VALU_UNPACKED_TFLOPS, 4)
            if ref is not None:
                with B.Context.for_problem(sample, prec, schedule=sched) as ctx:
                    logl, grad = ctx.gradient()
                entry["accuracy_vs_oracle"] = accuracy(logl, grad, ref, sample.n_patterns)
            res[f"{name}_{tag}"] = entry
            print(f"[bench] {name} {tag}: {1.0 / dt:.1f} evals/s, {tflops:.1f} TFLOP/s", file=sys.stderr,
                  flush=True)
    return res


def batched_vs_fp64(args, B, prob, fp64_evals_per_s):
    """k chains of the 1000-taxon workload evaluated concurrently through the
    server in FP32 (each chain resubmits as soon as its result returns, with
    perturbed branch lengths), against the plain FP64 single-context rate."""
    import threading
    E = 2 * prob.n_tips - 2
    srv = B.phg_server_create(0, 48 << 30, max(args.batched_chains, 1))
    counts = [0] * args.batched_chains
    stop = threading.Event()
    errors = []
    try:
        tids = [B.phg_server_register_tree(srv, prob, B.PHG_FP32_SCALED) for _ in range(args.batched_chains)]
        # warm: make every tree resident
        for t in tids:
            B.phg_server_wait(srv, B.phg_server_submit(srv, t, prob.b), E)

        def chain(k):
            rng = np.random.default_rng(k)
            try:
                while not stop.is_set():
                    b = prob.b * np.exp(rng.normal(0.0, 0.05, E))
                    B.phg_server_wait(srv, B.phg_server_submit(srv, tids[k], b), E)
                    counts[k] += 1
            except Exception as ex:  # noqa: BLE001
                errors.append(repr(ex))

        th = [threading.Thread(target=chain, args=(k,)) for k in range(args.batched_chains)]
        t0 = time.perf_counter()
        for t in th:
            t.start()
        time.sleep(args.batched_seconds)
        stop.set()
        for t in th:
            t.join(timeout=60)
        dt = time.perf_counter() - t0
        stats = B.phg_server_stats(srv)
    finally:
        B.phg_server_destroy(srv)
    if errors:
        raise RuntimeError(errors[0])
    rate = sum(counts) / dt
    return {"chains": args.batched_chains, "fp32_batched_evals_per_s": round(rate, 1),
            "fp64_single_evals_per_s": round(fp64_evals_per_s, 1),
            "speedup": round(rate / fp64_evals_per_s, 2), "server_launches": stats["launches"],
            "server_steps": stats["steps"]}


def _oracle_block(prob):
    """One pattern block through the unchanged oracle, one BLAS thread."""
    import oracle
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        r = oracle.evaluate_problem(prob)
    return r["logl"], r["grad"]


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(prob, args):
    """The FP64 oracle as it stands, on the host: one thread on a pattern
    sample, and every available core (at most --cpu-workers processes) on the
    whole workload split into contiguous pattern blocks whose log-likelihoods
    and gradients are summed in block order -- the paper's CPU scheme of
    column blocks.  Each: one warm-up run, then the median of three."""
    import multiprocessing as mp
    import statistics
    import oracle
    from threadpoolctl import threadpool_limits
    C = prob.n_patterns
    Cs = min(args.cpu_sample_patterns, C)
    s1 = prob.subset_patterns(np.arange(Cs))
    print(f"[bench] oracle, 1 thread, {Cs} patterns: warm-up + 3 runs", file=sys.stderr, flush=True)
    t1 = []
    with threadpool_limits(limits=1):
        for _ in range(4):
            t0 = time.perf_counter()
            oracle.evaluate_problem(s1)
            t1.append(time.perf_counter() - t0)
    t1 = statistics.median(t1[1:])
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    workers = max(1, min(args.cpu_workers, avail))
    blocks = [prob.subset_patterns(ix) for ix in np.array_split(np.arange(C), workers)]
    print(f"[bench] oracle, {workers} processes, {C} patterns: warm-up + 3 runs", file=sys.stderr, flush=True)
    tall = []
    with mp.get_context("spawn").Pool(workers) as pool:
        for _ in range(4):
            t0 = time.perf_counter()
            parts = pool.map(_oracle_block, blocks, chunksize=1)
            logl = 0.0
            grad = np.zeros_like(parts[0][1])
            for ll, g in parts:          # fixed block order
                logl += ll
                grad += g
            tall.append(time.perf_counter() - t0)
    tall = statistics.median(tall[1:])
    return {"value": round(1.0 / tall, 4), "unit": "evals/s", "cores": workers, "kind": "oracle",
            "sample": f"the whole 1000-taxon workload ({C} patterns) in {workers} contiguous pattern blocks, "
                      f"one process each, block results summed in order; median of 3 after 1 warm-up: "
                      f"{tall:.2f} s per evaluation",
            "one_thread": {"value": round((Cs / C) / t1, 5), "unit": "evals/s",
                           "sample": f"first {Cs} of {C} patterns, median of 3 after 1 warm-up: {t1:.2f} s, "
                                     f"scaled by {C}/{Cs} (cost is linear in patterns)"},
            "host": {"cpu_model": _cpu_model(), "nproc": os.cpu_count(), "available_cpus": avail},
            "logl_all_cores": logl}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--latency-requests", type=int, default=50)
    ap.add_argument("--fp64-steps", type=int, default=10)
    ap.add_argument("--cpu-sample-patterns", type=int, default=1000,
                    help="patterns of the one-thread oracle timing")
    ap.add_argument("--accuracy-sample-patterns", type=int, default=3000,
                    help="patterns of the 1000-taxon workload checked against the oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--schedule", choices=("auto", "levels", "blocks", "queue"), default="queue",
                    help="traversal schedule of the FP32 4-state path (default: the work-queue traversal; "
                         "FP64 contexts take auto, i.e. blocks)")
    ap.add_argument("--quick", action="store_true",
                    help="throughput and kernel-class times only (for profiler runs)")
    ap.add_argument("--serving-seconds", type=float, default=60.0,
                    help="length of the Poisson request stream for the serving measurement")
    ap.add_argument("--serving-rate", type=float, default=500.0, help="mean arrivals per second")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-states", action="store_true", help="skip the 20/61/122/240-state measurements")
    ap.add_argument("--state-steps", type=int, default=10)
    ap.add_argument("--states", default="aa500,codon128,s122,s240,s256big",
                    help="state-space workloads to measure (comma-separated)")
    ap.add_argument("--state-precisions", default="f32,f64")
    ap.add_argument("--state-schedule", choices=("queue", "levels"), default="queue",
                    help="schedule of the vector-ALU (17..32-state) entries")
    ap.add_argument("--only-states", action="store_true",
                    help="measure the state-space workloads only (for profiler runs)")
    ap.add_argument("--state-sample-patterns", type=int, default=200,
                    help="patterns of each state-space workload checked against the oracle (0: none)")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="most processes of the all-cores oracle timing (the box's CPU share per GPU)")
    ap.add_argument("--batched-chains", type=int, default=8)
    ap.add_argument("--batched-seconds", type=float, default=3.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (read + write) three times, "
                         "a known-size reference for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path shards over "
              "site patterns across GPUs by design but this build runs and reports a single GPU.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2303_04390_amd import binding as B
    from paper_2303_04390_amd import synth

    if args.only_states:
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        stream = torch.cuda.Stream(device=dev)
        out = torch.empty(1 << 16, dtype=torch.float64, device=dev)
        print(json.dumps({"state_spaces": state_space_measurement(args, B, synth, stream, out)}), flush=True)
        return
    prob = synth.config_problem("hky1000", seed=args.seed)
    N, C, S, R = prob.n_tips, prob.n_patterns, prob.n_states, prob.n_categories
    E = 2 * N - 2
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)
    out = torch.empty(1 + E, dtype=torch.float64, device=dev)

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {args.calibrate_copy} MiB read + written, 3 times",
              file=sys.stderr, flush=True)
        del src, dst

    sched = {"auto": B.PHG_SCHEDULE_AUTO, "levels": B.PHG_SCHEDULE_LEVELS,
             "blocks": B.PHG_SCHEDULE_BLOCKS, "queue": B.PHG_SCHEDULE_QUEUE}[args.schedule]
    SCHED_NAMES = {B.PHG_SCHEDULE_LEVELS: "levels", B.PHG_SCHEDULE_BLOCKS: "blocks",
                   B.PHG_SCHEDULE_QUEUE: "queue"}

    def open_ctx(prec, schedule=None):
        schedule = sched if schedule is None else schedule
        h = B.phg_create(N, C, S, R, prec, 0)
        # the work-queue traversal is FP32-only: FP64 contexts keep AUTO
        if schedule != B.PHG_SCHEDULE_AUTO and not (schedule == B.PHG_SCHEDULE_QUEUE and prec != B.PHG_FP32_SCALED):
            B.phg_set_schedule(h, schedule)
        B.phg_bind_stream(h, stream.cuda_stream)
        B.set_problem(h, prob)
        B.phg_prepare(h)
        return h

    def run_async(h, k):
        for _ in range(k):
            B.phg_gradient_async(h, out.data_ptr(), out.data_ptr() + 8)

    # ------------------------------------------------ throughput (FP32 path)
    h = open_ctx(B.PHG_FP32_SCALED)
    print(f"[bench] workload hky1000 N={N} C={C} S={S} R={R}; warmup {args.warmup}", file=sys.stderr, flush=True)
    run_async(h, args.warmup)
    torch.cuda.synchronize()
    # K evaluations launched on the stream
    t0 = time.perf_counter()
    run_async(h, args.steps)
    torch.cuda.synchronize()
    stream_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # K replays of one evaluation captured as a HIP graph (inputs resident;
    # the graph holds only the kernel launches)
    graph_ms, graph_note = None, None
    try:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            B.phg_bind_stream(h, torch.cuda.current_stream().cuda_stream)
            B.phg_gradient_async(h, out.data_ptr(), out.data_ptr() + 8)
        B.phg_bind_stream(h, stream.cuda_stream)
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        del graph
    except Exception as e:
        B.phg_bind_stream(h, stream.cuda_stream)
        graph_note = f"graph capture failed: {e}"
    # value: the faster of the two ways to run the same K evaluations
    if graph_ms is not None and graph_ms < stream_ms:
        ms_per_step, timing = graph_ms, "hip graph replay"
    else:
        ms_per_step, timing = stream_ms, "stream launches"
    value = 1e3 / ms_per_step
    print(f"[bench] fp32 {ms_per_step:.3f} ms/eval ({value:.1f} evals/s, {timing}); stream "
          f"{stream_ms:.3f}, graph {graph_ms if graph_ms is None else round(graph_ms, 3)} ms/eval",
          file=sys.stderr, flush=True)
    # kernel-class device times from HIP events, in a separate run
    B.phg_profile_enable(h, True)
    run_async(h, args.steps)
    torch.cuda.synchronize()
    ms_cls, n_prof, launches = B.phg_profile_read(h)
    B.phg_profile_enable(h, False)

    # ------------------------------------------------ live kernel-class times
    per_eval_ms = ms_cls / max(n_prof, 1)
    sched_name = SCHED_NAMES[B.phg_get_schedule(h)]
    blocked = sched_name in ("blocks", "queue")
    post_bytes, pre_bytes = (algorithmic_bytes_blocked if blocked else algorithmic_bytes)(
        prob.parent, N, C, R, S, 4)
    cls = dict(zip(B.PROF_NAMES, per_eval_ms.tolist()))
    dominant = max(("post", "pre_grad"), key=lambda k: cls[k])
    dom_bytes = pre_bytes if dominant == "pre_grad" else post_bytes
    dom_ms = cls[dominant]
    n_launch = int(launches[B.PROF_NAMES.index(dominant)])
    # per launch: algorithmic bytes / average launch duration (= per-eval totals)
    achieved = (dom_bytes / n_launch) / (dom_ms * 1e-3 / n_launch) / 1e9
    traffic = None
    if (MEASURED_TRAFFIC["kernel_source_sha256"] == kernel_source_sha256()
            and MEASURED_TRAFFIC["schedule"] == sched_name
            and dominant in MEASURED_TRAFFIC["bytes_per_eval"]):
        traffic = int(MEASURED_TRAFFIC["bytes_per_eval"][dominant] / n_launch)
    # the dominant kernel's share of the method minimum M0 (every internal
    # partial written once and read once, tip codes twice, exponents once):
    # the pre-order reads each non-root internal partial and each tip code
    # once, the post-order does the rest
    vec = R * S * 4
    m0 = (2 * N - 3) * vec + 2 * N + (N - 1)
    m0_pre = ((N - 2) * vec + N) * C
    m0_share = m0_pre if dominant == "pre_grad" else m0 * C - m0_pre
    m0_achieved = (m0_share / n_launch) / (dom_ms * 1e-3 / n_launch) / 1e9
    roofline = {
        "bound": "hbm",
        # the class: the work-queue kernel's pass (<R, 1> post-order, <R, 2>
        # pre-order), or the level kernels (wide launches take <R, false>,
        # narrow, latency-bound ones <R, true>)
        "kernel": (f"queue_bmf_kernel<{R}, {2 if dominant == 'pre_grad' else 1}>" if sched_name == "queue"
                   else f"{'pre' if dominant == 'pre_grad' else 'post'}_bmf_kernel<{R}, *>"
                   if blocked and R & (R - 1) == 0
                   else f"{'pre' if dominant == 'pre_grad' else 'post'}_{'blk' if blocked else 's4'}_kernel<float,{R}>"),
        "schedule": sched_name,
        "achieved": round(m0_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(m0_achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "algorithmic_bytes_per_launch": int(m0_share / n_launch),
        "algorithmic_bytes": "the kernel's share of the method minimum M0 per launch",
        "launches_per_eval": n_launch,
        "launch_avg_us": round(dom_ms * 1e3 / n_launch, 3),
        "schedule_bytes_per_launch": int(dom_bytes / n_launch),
        "schedule_achieved": round(achieved, 1),
        "schedule_frac": round(achieved / HBM_PEAK_GBS, 4),
        "schedule_bytes": "bytes the schedule itself must move per launch (block roots' vectors, codes)",
    }
    path = {"ms_per_class": {k: round(v, 4) for k, v in cls.items()},
            "launches_per_class": dict(zip(B.PROF_NAMES, launches.tolist())),
            "m0_bytes_per_eval": int(m0 * C),
            "m0_ceiling_evals_per_s": round(HBM_PEAK_GBS * 1e9 / (m0 * C), 1),
            "frac_of_m0_ceiling": round(value / (HBM_PEAK_GBS * 1e9 / (m0 * C)), 4)}

    if args.quick:
        B.phg_destroy(h)
        rec = {"metric": METRIC, "value": round(value, 2), "unit": "evals/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
               "quick": True, "timing": {"method": timing, "stream_launches_ms_per_step": round(stream_ms, 4),
                   "graph_replay_ms_per_step": None if graph_ms is None else round(graph_ms, 4),
                   "note": graph_note},
               "roofline": roofline, "path": path}
        print(json.dumps(rec), flush=True)
        return

    # ------------------------------------------------ request latency (sync)
    rng = np.random.default_rng(123)
    lat = []
    for i in range(args.latency_requests):
        b = prob.b * np.exp(rng.normal(0.0, 0.05, E))
        ta = time.perf_counter()
        B.phg_set_branch_lengths(h, b)
        B.phg_gradient(h, E)
        lat.append((time.perf_counter() - ta) * 1e3)
    B.phg_set_branch_lengths(h, prob.b)
    lat = np.array(lat)
    B.phg_destroy(h)

    # ------------------------------------------------ the other FP32 schedules
    sched_ms = {sched_name: round(stream_ms, 4)}
    for other, code in (("blocks", B.PHG_SCHEDULE_BLOCKS), ("levels", B.PHG_SCHEDULE_LEVELS),
                        ("queue", B.PHG_SCHEDULE_QUEUE)):
        if other in sched_ms:
            continue
        ho = open_ctx(B.PHG_FP32_SCALED, code)
        run_async(ho, args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_async(ho, args.steps)
        torch.cuda.synchronize()
        sched_ms[other] = round((time.perf_counter() - t0) * 1e3 / args.steps, 4)
        B.phg_destroy(ho)
    print(f"[bench] fp32 schedules, stream launches, ms/eval: {sched_ms}", file=sys.stderr, flush=True)

    # ------------------------------------------------ plain FP64 path
    h64 = open_ctx(B.PHG_FP64)
    run_async(h64, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_async(h64, args.fp64_steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    B.phg_destroy(h64)
    fp64_ms = (t1 - t0) * 1e3 / args.fp64_steps

    serving = None
    batched = None
    states = None
    if not args.no_states:
        print("[bench] 20-, 61-, 122- and 240-state workloads", file=sys.stderr, flush=True)
        states = state_space_measurement(args, B, synth, stream, out)
    if not args.no_serving:
        print("[bench] batched FP32 chains vs plain FP64", file=sys.stderr, flush=True)
        batched = batched_vs_fp64(args, B, prob, 1e3 / fp64_ms)
        print(f"[bench] serving stream {args.serving_rate}/s for {args.serving_seconds}s", file=sys.stderr,
              flush=True)
        serving = serving_measurement(args, B, synth)

    rec = {
        "metric": METRIC, "value": round(value, 2), "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "hky1000: 1000-taxon Yule tree (b~Exp(0.01)), HKY+Gamma4, 10,000 "
                               "simulated patterns (weights 1+Poisson(3), 5% ambiguous tip entries); "
                               "FP32 partials with power-of-two rescaling, FP64 P(t) and reductions",
                   "n_tips": N, "n_patterns": C, "n_states": S, "n_categories": R, "seed": args.seed,
                   "schedule": sched_name},
        "branch_derivatives_per_s": round(value * E, 1),
        "timing": {"method": timing, "stream_launches_ms_per_step": round(stream_ms, 4),
                   "graph_replay_ms_per_step": None if graph_ms is None else round(graph_ms, 4),
                   "note": graph_note},
        "latency_ms": ({"p50": serving["latency_ms"]["p50"], "p99": serving["latency_ms"]["p99"],
                        "what": "serving stream (see serving): arrival to logL + gradient in host memory"}
                       if serving else None),
        "sync_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                            "p99": round(float(np.percentile(lat, 99)), 4),
                            "requests": int(lat.size),
                            "what": "one synchronous request on the 1000-taxon workload: new branch lengths "
                                    "in, logL + 1998 derivatives in host memory"},
        "roofline": roofline,
        "path": path,
        "fp64_path": {"ms_per_step": round(fp64_ms, 4), "evals_per_s": round(1e3 / fp64_ms, 2)},
        "fp32_schedules_ms_per_step": dict(sched_ms, what="the same FP32 evaluation under each 4-state "
                                           "schedule, stream launches (the value's schedule is in config)"),
        "batched_fp32_vs_fp64": batched,
        "state_spaces": states,
        "serving": serving,
    }

    # ------------------------------------------------ oracle: CPU baseline + accuracy
    if not args.no_cpu_baseline:
        import oracle
        rec["cpu_baseline"] = cpu_baseline(prob, args)
        Cs = min(args.accuracy_sample_patterns, C)
        sample = prob.subset_patterns(np.arange(Cs))
        print(f"[bench] accuracy against the oracle on {Cs} patterns", file=sys.stderr, flush=True)
        ref = oracle.evaluate_problem(sample)
        acc = {}
        for prec, name in ((B.PHG_FP32_SCALED, "fp32"), (B.PHG_FP64, "fp64")):
            with B.Context.for_problem(sample, prec) as ctx:
                logl, grad = ctx.gradient()
                ran = B.phg_last_precision(ctx.handle)
                sat = B.phg_fp32_saturation(ctx.handle)
            acc[name] = accuracy(logl, grad, ref, Cs)
            acc[name]["ran_in"] = "fp64" if ran == B.PHG_FP64 else "fp32"
        acc["fp32_guard_saturation"] = round(sat, 4)
        acc["rule"] = "scaled: |g-g*| / max(|g*|, 1e-2 * sum_c W_c |d_c|); pure: |g-g*| / |g*|"
        rec["accuracy_vs_oracle"] = acc
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
