"""Throughput of the LMEP hot path on one MI355X.

Default workload: viscous Burgers u_t + u u_x = nu u_xx, N = 65536 nodes,
Dirichlet ends with one-sided edge stencils, n = 7, ETD1 with the phi1 weights
of the augmented local matrix rebuilt every step from the frozen local
velocity (one FP64 Pade scaling-and-squaring exponential of an 8x8 local
matrix per node per step), 1000 steps.  A "step" is one time step of the whole
hot path: weight build for every node + banded apply.

Prints one JSON line: node-steps/s of the timed K steps (inputs resident in
HBM), the roofline of the dominant kernel (the weight build, FP64 vector ALU)
from HIP events recorded around each build launch in a second, profiled pass
over the same K steps, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 64 lanes x 2 flop x 2.4 GHz
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E


def pade_flops(m: int, matrices: int, squarings: int) -> float:
    """Algorithmic flops of degree-13 Pade scaling-and-squaring on m x m
    matrices, 2 flops per multiply-add: 6 products for U and V, one LU solve
    with m right-hand sides (8 m^3 / 3), and one product per squaring."""
    return matrices * (2.0 * 6 * m ** 3 + 8.0 * m ** 3 / 3.0) + squarings * 2.0 * m ** 3


def _moment_terms(n: int):
    """Per order K = 1..n-1 of the unshifted, dispersion-free moment recursion:
    (entries, terms) -- the theta-degrees m that can be non-zero
    (ceil(K/2) <= m <= K) and the recursion terms that feed them (a mu[K-1][m-1]
    and 2 b (K-1) mu[K-2][m-1], each only where that moment can be non-zero)."""
    lo = lambda k: (k + 1) // 2
    out = []
    for K in range(1, n):
        k = K - 1
        ms = range(lo(K), K + 1)
        terms = 0
        for m in ms:
            terms += (m >= 1 and m - 1 >= lo(k))
            terms += (k >= 1 and m >= 1 and m - 1 >= lo(k - 1) and m <= k)
        out.append((len(ms), terms))
    return out


def taylor_flops(n: int, fused: bool) -> float:
    """Algorithmic flops of one node of the finite-Taylor build (multiply-add =
    2, a product into a zero sum = 1), in the unshifted, dispersion-free case:
    the moment recursion over the moments that can be non-zero (_moment_terms;
    plus the scaled diffusion coefficient per order from order 2), the two
    moment sums per order (exponential: adds; phi1: multiply-adds), the
    contraction with the table rows (2 n multiply-adds per order), the
    scaling of W1 (by dt, or with fusion by -g dt), and with fusion the
    derivative at the node (n multiplies + n multiply-adds) and the stencil sum
    W0.u + W1.N' with N'_j = (u_j - u_i) d_j (6 per position)."""
    f = 0.0
    for K, (c, t) in enumerate(_moment_terms(n), start=1):
        f += 2 * t - c + (1 if K >= 2 else 0)   # every entry's first term is a product
        f += (c - 1) + (2 * c - 1)               # the exponential and phi1 sums
        f += 4.0 * n                             # contraction
    f += n
    if fused:
        f += 3.0 * n + 6.0 * n
    return f


def stationary_flops(p: dict) -> float:
    """Algorithmic flops of one node-step of the banded apply with stationary
    weights (multiply-add = 2): W0.u (+ W1.N) over the n-window, N itself
    (Allen-Cahn g(u - u^3): 4; KdV -(g/2) D1.(u u): 3n + 2), and for ETD2RK with
    a nonlinearity N(a) plus a + W2.(N(a) - N(u)) (2n + 1)."""
    n = p["n"]
    rk2 = p["scheme"] == "etd2rk"
    nl = p.get("nonlin", "none")
    has_n = p["scheme"] != "linear" and nl != "none"
    n_cost = {"allen_cahn": 4.0, "kdv": 3.0 * n + 2.0}.get(nl, 0.0)
    if p["scheme"] == "etdrk4":
        # E2.u once, P2.N(u), P2.N(a), E2.a + P2.(2N(b) - N(u)), E.u + A.N(u) +
        # B.(N(a) + N(b)) + C.N(c): nine n-term sums, three pointwise combinations,
        # four evaluations of N; without N only E.u
        return 2.0 * n * 9 + 3.0 + 4.0 * n_cost if has_n else 2.0 * n
    f = 2.0 * n
    if has_n:
        f += 2.0 * n + n_cost
        if rk2:
            f += n_cost + 2.0 * n + 1.0
    return f


PEAK_LDS_GBS = 256 * 128 * 2.4  # 128 B per clock per CU
SCHEME_ID = {"linear": 0, "etd1": 1, "etd2rk": 2, "etdrk4": 3}
KINDS = {"linear": 1, "etd1": 2, "etd2rk": 3, "etdrk4": 6}
NONLIN_ID = {"none": 0, "burgers_frozen": 1, "kdv": 2, "allen_cahn": 3}


def measured_traffic(kernels, workload):
    """HBM bytes per launch of the named kernels (summed) on this workload, from
    the byte-counter summaries under profiles/ (FETCH_SIZE and WRITE_SIZE
    scaled by a copy probe).  Lines read
      traffic-bytes-per-launch <kernel> <bytes> workload <name> sources-sha256 <hash> <files...>
    None unless every kernel has a line for this workload whose recorded sha256
    of the kernel's sources still matches the sources in this tree."""
    import glob
    import hashlib
    table = {}
    for f in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(f):
            t = line.split()
            if len(t) >= 8 and t[0] == "traffic-bytes-per-launch" and t[3] == "workload" and t[5] == "sources-sha256":
                table[(t[1], t[4])] = (float(t[2]), t[6], t[7:])
    total = 0.0
    for k in kernels:
        if (k, workload) not in table:
            return None
        val, digest, files = table[(k, workload)]
        h = hashlib.sha256()
        for rel in files:
            path = os.path.join(ROOT, rel)
            if not os.path.exists(path):
                return None
            h.update(open(path, "rb").read())
        if h.hexdigest()[:16] != digest:
            return None
        total += val
    return total


def make_workload(name: str):
    import workloads
    if name == "burgers":
        p, u0 = workloads.burgers()
        return [p], [u0], "viscous Burgers N=65536 n=7 Dirichlet, frozen-velocity ETD1, weights rebuilt every step"
    if name == "kdv":
        p, u0 = workloads.kdv()
        return [p], [u0], "periodic KdV N=1048576 n=9 ETD2RK, dispersive number 4/pi^3, stationary weights"
    if name == "allen_cahn_batch":
        ps, us = workloads.allen_cahn_batch()
        return ps, us, "4096 Allen-Cahn instances N_k in [512,65536], n_k in {5,7,9,11}, ETD1, stationary weights"
    if name == "burgers_etdrk4":
        p, u0 = workloads.burgers_etdrk4()
        return [p], [u0], ("the paper's Burgers run: periodic N=1048576 n=13, nu=0.03, stationary L = nu D2, "
                           "N = -u u_x, ETDRK4")
    if name == "burgers_upwind":
        p, u0 = workloads.burgers_upwind()
        return [p], [u0], ("viscous Burgers N=65536 n=7 periodic on fully one-sided (upwind) stencils at "
                           "CFL 3.5, frozen-velocity ETD1, weights rebuilt every step")
    if name == "allen_cahn_chebyshev_batch":
        ps, us = workloads.allen_cahn_chebyshev_batch()
        return ps, us, ("8192 Allen-Cahn instances on the paper's Chebyshev grid (N=64, n=21), nu ~ U[0.005,0.01], "
                        "Dirichlet -1/1, ETD1, per-node stationary weights")
    if name == "allen_cahn_chebyshev":
        p, u0 = workloads.allen_cahn_chebyshev()
        return [p], [u0], "the paper's Allen-Cahn run: Chebyshev N=64, n=21, nu=0.01, dt=1e-4, ETD1"
    if name == "advection_diffusion":
        p, u0 = workloads.advection_diffusion()
        return [p], [u0], "periodic advection-diffusion N=256 n=5 CFL 2, LINEAR"
    if name == "burgers_batch":
        p, pt, u0s = workloads.burgers_adjoint_batch()
        return ([p] * len(u0s), u0s,
                "64 Burgers trajectories N=262144 n=9 Dirichlet (the adjoint workload's forward), frozen-velocity "
                "ETD1, weights rebuilt every step")
    if name == "burgers_adjoint":
        p, pt, u0s = workloads.burgers_adjoint_batch()
        return ([p] * len(u0s), u0s,
                "adjoint: 64 Burgers trajectories N=262144 n=9, ETD1 frozen velocity, forward + checkpointed reverse")
    raise SystemExit(f"unknown workload {name}")


def plain_forward(problems, states, steps, max_instances=None):
    """The plain path the batched and adjoint paths are compared with: the
    single-instance forward, each instance on its own (one lmep_step call per
    instance, per-step eager launches, default tiles), one after another.
    Weights of stationary instances are built before the clock starts.
    Returns (node-steps/s, instances timed)."""
    import torch
    import paper_2603_15964_amd as lmep
    k = len(problems) if max_instances is None else min(len(problems), max_instances)
    runs = []
    for p, u in zip(problems[:k], states[:k]):
        b = lmep.Batch([p], device="cuda:0")
        w = b.empty_weights()
        u0 = b.pack([u])
        if p.get("nonlin") != "burgers_frozen":
            b.build_weights(w, u0)
        runs.append((b, w, u0, b.empty_state()))
    for b, w, u0, out in runs:  # warm-up: plans, code objects
        b.step(w, u0, 1, 0, u_out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b, w, u0, out in runs:
        b.step(w, u0, steps, 0, u_out=out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return sum(int(p["N"]) for p in problems[:k]) * steps / el, k


def bench_adjoint(problems, states, steps, every=None):
    """Forward with checkpoints + reverse through lmep_adjoint_step; returns
    (seconds, node-steps, checkpoint interval) with node-steps = nodes x steps.
    every=None: autograd's choice (every state when they fit in half the free
    device memory)."""
    import torch
    import paper_2603_15964_amd as lmep
    from paper_2603_15964_amd import autograd as lad
    batch = lmep.Batch(problems, device="cuda:0")
    u0 = batch.pack(states).requires_grad_(True)
    nu = torch.tensor([p["nu"] for p in problems], dtype=torch.float64, device="cuda:0", requires_grad=True)
    target = torch.zeros_like(u0)
    if every is None:
        every = lad.auto_checkpoint_every(batch, steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    uT = lad.solve(batch, u0, steps, nu=nu, checkpoint_every=every)
    loss = 0.5 * torch.sum((uT - target) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, batch.state_size * steps, every


def pair_pade_flops(m: int, squarings: float) -> float:
    """Algorithmic flops of one Frechet derivative by degree-13 Pade on the
    block-triangular pair [[A, E], [0, A]] of order-m blocks (2 per
    multiply-add): a pair product is three m x m products; 6 pair products for
    U and V (36 m^3), the pair solve (LU of Q 2m^3/3, m right-hand sides for X
    2m^3, the correction Q_E X 2m^3, m right-hand sides for the E part 2m^3),
    and one pair product per squaring (6 m^3)."""
    return 36.0 * m ** 3 + (2.0 / 3.0 + 6.0) * m ** 3 + 6.0 * m ** 3 * squarings


def adj_taylor_flops(n: int, p: int) -> float:
    """Algorithmic flops of one node of the finite-Taylor reverse-step kernel
    (2 per multiply-add; unshifted, dispersion-free): the moment recursion over
    the moments that can be non-zero (_moment_terms; plus one coefficient
    multiply per order), the three moment sums per order (M(1), its integral
    and its first moment: 5c - 3 for c entries), the contractions per order
    with the table row (W0 and tau, and for ETD1 W1 and nu: 2n each), the
    three derivative terms per order (5 each, 2.5 for LINEAR), the window's N
    values (3 per position, ETD1), and the scaled outputs."""
    mt = _moment_terms(n)
    rec = sum(2 * t - c + 1 for c, t in mt)
    sums = sum(5 * c - 3 for c, t in mt)
    con = (n - 1) * (2 * n) * (4 if p >= 1 else 2)
    der = (n - 1) * 3 * (5 if p >= 1 else 2.5)
    nval = 3 * n if p >= 1 else 0
    out = (n if p >= 1 else 0) + 9
    return float(rec + sums + con + der + nval + out)


def adj_fused_flops(n: int, p: int) -> float:
    """Algorithmic flops per node of the fused reverse-step kernel: the
    per-node part (adj_taylor_flops) and the two gathers over the n stencils
    containing the node -- ghat (5 per term) and lambda (4 per term, the own
    window's n multiply-adds, and 3 per ghat term) -- halo recomputation not
    counted."""
    return adj_taylor_flops(n, p) + (5 + 4 + 2 + 3) * n


def adjoint_roofline(problems, states, reps: int = 5):
    """Roofline of the per-node kernel of the reverse step (finite Taylor
    series, or the Frechet derivative by the block-triangular Pade exponential
    with LMEP_EXP_PADE): HIP events around that kernel
    (LMEP_OPT_PROFILE_ADJOINT) over `reps` reverse steps at u0; for Pade its
    squarings come from a counting forward step at the same state (the pair's
    scaling is chosen from the same local matrix)."""
    import torch
    import paper_2603_15964_amd as lmep
    batch = lmep.Batch(problems, device="cuda:0")
    u0 = batch.pack(states)
    lam = torch.sin(torch.arange(batch.state_size, dtype=torch.float64, device="cuda:0"))
    w = batch.empty_weights()
    batch.step(w, u0, 1, lmep.LMEP_F_COUNT)
    cnt = lmep.lmep_profile_last()
    mean_s = cnt["squarings"] / max(1, cnt["matrices"])
    batch.adjoint_step(u0, lam)  # warm-up
    lmep.lmep_set_option(lmep.LMEP_OPT_PROFILE_ADJOINT, 1)
    fre_ms, launches, rest_ms = 0.0, 0, 0.0
    try:
        for _ in range(reps):
            batch.adjoint_step(u0, lam)
            prof = lmep.lmep_profile_last()
            fre_ms += prof["build_ms"]
            launches += prof["build_launches"]
            rest_ms += prof["apply_ms"]
    finally:
        lmep.lmep_set_option(lmep.LMEP_OPT_PROFILE_ADJOINT, 0)
    p0 = problems[0]
    m = p0["n"] + {"linear": 0, "etd1": 1}[p0["scheme"]]
    taylor = (lmep.lmep_get_option(lmep.LMEP_OPT_EXP_METHOD) == lmep.LMEP_EXP_AUTO and
              all(p.get("react", 0.0) == 0.0 for p in problems))
    if taylor:
        # the whole reverse step of a tile in one kernel (per-node part and gathers)
        flops = batch.state_size * adj_fused_flops(p0["n"], m - p0["n"]) * reps
        kname = f"adj_fused_kernel<{p0['n']},{m - p0['n']}>"
        mean_s = 0.0
    else:
        flops = batch.state_size * pair_pade_flops(m, mean_s) * reps
        kname = f"adj_frechet_kernel<{p0['n']},{m - p0['n']}>"
    tf = flops / (fre_ms / 1e3) / 1e12
    return {"bound": "alu", "achieved": tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / PEAK_FP64_TFLOPS, "traffic": measured_traffic([kname], "burgers_adjoint"), "kernel": kname,
            "avg_launch_us": fre_ms * 1e3 / max(1, launches), "flops_per_launch": flops / max(1, launches),
            "mean_squarings": mean_s, "rest_of_reverse_step_us": rest_ms * 1e3 / reps}


def cpu_baseline(problem, u0, budget_s: float = 15.0):
    """The oracle as it stands, on a bounded number of steps of the same workload."""
    import oracle
    t = time.perf_counter()
    u = oracle.run(problem, u0, 1)
    one = time.perf_counter() - t
    steps = max(1, min(1000, int(budget_s / max(one, 1e-6))))
    t = time.perf_counter()
    oracle.run(problem, u, steps)
    el = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": problem["N"] * steps / el, "unit": "node-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} steps of the same workload (N={problem['N']}) after 1 warm step"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed steps first (brings the clocks up; the timed region of the default run is short)")
    ap.add_argument("--workload", default="burgers")
    ap.add_argument("--graph", action="store_true", help="replay the step loop from a hipGraph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain single-instance comparison runs (and the Pade comparison run)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (calibrates byte counters)")
    ap.add_argument("--persistent", action="store_true",
                    help="advance several steps per launch (LMEP_F_PERSISTENT)")
    ap.add_argument("--launch", choices=("auto", "one-step", "persistent"), default="auto",
                    help="auto: several steps per launch for frozen-velocity workloads the multi-step kernel covers "
                         "whose batch is under 2^20 nodes (too small to fill the GPU in one step), one step "
                         "otherwise; --persistent is the same as --launch persistent")
    ap.add_argument("--steps-per-launch", type=int, default=None, choices=(1, 2, 4, 8),
                    help="steps per launch of the multi-step path (default 8; for --launch auto on frozen "
                         "velocity the deepest whose largest region (512 positions) keeps 128 written nodes)")
    ap.add_argument("--tune", action="store_true",
                    help="let the autotuner pick fusion / steps per launch / apply tile (cached per GPU and shape)")
    ap.add_argument("--exp-method", choices=("auto", "pade"), default="auto",
                    help="exponential of the frozen-velocity rebuild: finite Taylor series where it applies (auto) "
                         "or Pade scaling-and-squaring everywhere")
    ap.add_argument("--skip-count", action="store_true",
                    help="skip the squaring-count pass (its atomics would show up in a kernel trace)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}), flush=True)
        raise SystemExit(2)

    import torch
    import paper_2603_15964_amd as lmep

    if args.copy_probe:
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": a.numel() * 8, "copies": 3}), flush=True)
        return

    problems, states, desc = make_workload(args.workload)
    dev = "cuda:0"
    if args.launch == "persistent":
        args.persistent = True
    elif args.launch == "auto" and not args.persistent and not args.tune:
        frozen_all = all(p.get("nonlin") == "burgers_frozen" for p in problems)
        covered = all(p["bc"] != "neumann" and p.get("react", 0.0) == 0.0 for p in problems)
        small = sum(int(p["N"]) for p in problems) < (1 << 20)
        args.persistent = frozen_all and covered and small and args.exp_method == "auto"
        if args.persistent and args.steps_per_launch is None:
            # deepest launch whose largest region (512 positions; the library sizes
            # regions per CU up to that) still writes 128 nodes per block (the halo
            # grows by n - 1 per step, 2 (n - 1) for one-sided windows)
            reach = max((2 if p.get("window", "centred") == "upwind" else 1) * (int(p["n"]) - 1) for p in problems)
            args.steps_per_launch = next((kb for kb in (8, 4, 2) if 512 - 2 * kb * reach >= 128), 1)
    if args.steps_per_launch is None:
        args.steps_per_launch = 8
    lmep.lmep_set_option(lmep.LMEP_OPT_EXP_METHOD,
                         lmep.LMEP_EXP_PADE if args.exp_method == "pade" else lmep.LMEP_EXP_AUTO)
    if args.workload == "burgers_adjoint":
        wu = max(1, min(args.warmup, 10))  # a short warm-up: its checkpoint segment holds every state
        bench_adjoint(problems, states, wu, every=wu)
        secs, node_steps, every = bench_adjoint(problems, states, args.steps)
        out = {"metric": "node-steps/s (weight build+apply, FP64), adjoint: forward + checkpointed reverse",
               "value": node_steps / secs, "unit": "node-steps/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": secs * 1e3 / args.steps, "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
               "config": {"workload": desc, "instances": len(problems), "nodes": sum(p["N"] for p in problems),
                          "checkpoint_every": every},
               "roofline": adjoint_roofline(problems, states)}
        if not args.no_plain:
            pv, pk = plain_forward(problems, states, min(args.steps, 50))
            out["plain"] = {"value": pv, "unit": "node-steps/s", "instances": pk,
                            "kind": "single-instance forward only, instances one at a time, per-step eager launches",
                            "ratio": out["value"] / pv}
        print(json.dumps(out), flush=True)
        return
    batch = lmep.Batch(problems, device=dev)
    w = batch.empty_weights()
    u0 = batch.pack(states)
    ua, ub = batch.empty_state(), batch.empty_state()
    frozen = any(p.get("nonlin") == "burgers_frozen" for p in problems)
    if not all(p.get("nonlin") == "burgers_frozen" for p in problems):
        batch.build_weights(w, u0)
    flags = lmep.LMEP_F_GRAPH if args.graph else 0
    kb = 1
    tuned = None
    if args.tune:
        from paper_2603_15964_amd import tune as lt
        tuned = lt.tune(batch, w, u0, steps=max(4, min(args.steps, 50)))
        opts = dict(tuned.choice.options)
        for o, v in opts.items():
            lmep.lmep_set_option(o, v)
        flags |= tuned.choice.flags
        args.persistent = bool(tuned.choice.flags & lmep.LMEP_F_PERSISTENT)
        if args.persistent:
            kb = opts[lmep.LMEP_OPT_STEPS_PER_LAUNCH]
    elif args.persistent:
        flags |= lmep.LMEP_F_PERSISTENT
        kb = args.steps_per_launch
        lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, kb)

    if args.warmup > 0:
        batch.step(w, u0, args.warmup, flags, u_out=ua)
    else:
        ua.copy_(u0)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    batch.step(w, ua, args.steps, flags, u_out=ub)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = start.elapsed_time(stop)
    node_steps = batch.state_size * args.steps
    value = node_steps / wall

    # profiled pass: HIP events around every build / apply launch, same K steps
    # from the same state; then an untimed pass over the same steps that counts
    # the squarings each local exponential took (for the algorithmic flops)
    batch.step(w, ua, args.steps, lmep.LMEP_F_PROFILE | (flags & lmep.LMEP_F_PERSISTENT), u_out=ub)
    if frozen and not args.skip_count:
        batch.step(w, ua, args.steps, lmep.LMEP_F_COUNT, u_out=ub)
    prof = lmep.lmep_profile_last()
    roof = None
    extra = {"gpu_event_ms": gpu_ms, "wall_ms": wall * 1e3}
    apply_bytes = {"burgers": 128.0, "burgers_upwind": 128.0, "kdv": 16.0, "allen_cahn_batch": 16.0, "advection_diffusion": 16.0}
    taylor = frozen and args.exp_method == "auto" and all(p.get("react", 0.0) == 0.0 for p in problems)
    if frozen and prof["build_launches"] > 0 and prof["matrices"] > 0:
        p0 = problems[0]
        m = p0["n"] + {"linear": 0, "etd1": 1, "etd2rk": 2}[p0["scheme"]]
        fused = lmep.lmep_get_option(lmep.LMEP_OPT_FUSE_FROZEN) == 1
        if taylor and args.persistent:
            # node-steps of the launches (the halo each block recomputes is not counted)
            flops = taylor_flops(p0["n"], True) * prof["matrices"]
            kname = f"taylor_stepk_kernel<{p0['n']}>"
        elif taylor:
            flops = taylor_flops(p0["n"], fused) * prof["matrices"]
            kname = f"build_taylor_kernel<{p0['n']},{'true' if fused else 'false'}>"
        else:
            flops = pade_flops(m, prof["matrices"], prof["squarings"])
            kname = f"build_pade_kernel<{p0['n']},{m - p0['n']},{'true' if fused else 'false'}>"
        # When every launch of the timed region is this kernel (fused steps, one
        # stencil size, no separate apply launches), its average duration is the
        # timed region's GPU event time over its launches (back-to-back gaps
        # included); otherwise the profiled pass's events around each launch,
        # which add their own overhead to every launch.
        only = prof["apply_launches"] == 0 and len({p["n"] for p in problems}) == 1
        build_s = gpu_ms / 1e3 if only else prof["build_ms"] / 1e3
        achieved = flops / build_s / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": measured_traffic([kname], args.workload),
                "kernel": kname,
                "avg_launch_us": build_s * 1e6 / prof["build_launches"],
                "duration_from": "timed region events" if only else "events around each launch",
                "avg_launch_us_events_each": prof["build_ms"] * 1e3 / prof["build_launches"],
                "flops_per_launch": flops / prof["build_launches"],
                "mean_squarings": prof["squarings"] / max(1, prof["matrices"])}
    nonuniform = any(p.get("x") is not None for p in problems)
    if prof["apply_launches"] > 0:
        apply_s = prof["apply_ms"] / 1e3
        avg_us = prof["apply_ms"] * 1e3 / prof["apply_launches"]
        # algorithmic HBM bytes: per node and launch, u in + u out (16 B), plus
        # the per-node weights of the frozen-velocity path (read every step) or
        # of a non-uniform grid (read once per launch)
        if nonuniform:
            per_node = sum(p["N"] * (16.0 + 8.0 * KINDS[p["scheme"]] * p["n"]) for p in problems) / batch.state_size
            if args.persistent:  # whole instances per block: every step of the call in one launch
                kb = args.steps
            ab = per_node * node_steps / kb
        else:
            ab = apply_bytes.get(args.workload, 16.0) * node_steps / kb
        gbs = ab / apply_s / 1e9
        extra["apply"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": gbs / PEAK_HBM_GBS, "avg_launch_us": avg_us, "steps_per_launch": kb,
                          "bytes_per_launch": ab / prof["apply_launches"]}
        if not frozen:
            fl = sum(stationary_flops(p) * p["N"] for p in problems) * args.steps
            tf = fl / apply_s / 1e12
            extra["apply_alu"] = {"bound": "alu", "achieved": tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                                  "frac": tf / PEAK_FP64_TFLOPS, "flops_per_launch": fl / prof["apply_launches"]}
        if roof is None:
            # one step per launch: HBM-bound; several: the traffic is paid once
            # per launch and the FP64 work of the steps bounds the kernel
            def kname(p):
                nl = NONLIN_ID[p.get("nonlin", "none")] if p["scheme"] != "linear" else 0
                if p.get("x") is not None:
                    return f"resident_kernel<{p['n']},{SCHEME_ID[p['scheme']]},{nl}>"
                if p["scheme"] == "etdrk4":
                    return f"stepk_rk4_kernel<{p['n']},{nl},{kb}>"
                return f"stepk_kernel<{p['n']},{SCHEME_ID[p['scheme']]},{nl},{kb}>"
            if kb > 1 or any(p["scheme"] == "etdrk4" for p in problems) or (nonuniform and args.persistent):
                names = sorted({kname(p) for p in problems})
            elif nonuniform and all(p["N"] <= 64 for p in problems):
                names = sorted({f"apply_kernel<{p['n']},{SCHEME_ID[p['scheme']]},"
                                f"{NONLIN_ID[p.get('nonlin', 'none')] if p['scheme'] != 'linear' else 0},true,64>"
                                for p in problems})
            else:
                names = ["apply_kernel"]
            if nonuniform and args.persistent:
                # one block holds an instance: per node-step the kernel reads its
                # window of u from LDS (N is formed from it), and for ETD2RK with
                # a nonlinearity the windows of N(a) and N(u) as well
                def lds_reads(p):
                    has_n = p["scheme"] != "linear" and p.get("nonlin", "none") != "none"
                    return p["n"] * (1 + (2 if has_n and p["scheme"] == "etd2rk" else 0))
                lb = sum(p["N"] * 8.0 * lds_reads(p) for p in problems) * args.steps
                gbs_lds = lb / apply_s / 1e9
                extra["lds"] = {"bound": "lds", "achieved": gbs_lds, "peak": PEAK_LDS_GBS, "unit": "GB/s",
                                "frac": gbs_lds / PEAK_LDS_GBS, "bytes_per_launch": lb / prof["apply_launches"]}
            roof = dict(extra["lds"] if (nonuniform and args.persistent) else
                        (extra["apply_alu"] if kb > 1 else extra["apply"]),
                        traffic=measured_traffic(names, args.workload) if (kb > 1 or nonuniform) else None,
                        kernel=" + ".join(names), avg_launch_us=avg_us)
    out = {
        "metric": "node-steps/s (weight build+apply, FP64)",
        "value": value,
        "unit": "node-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "instances": batch.count, "nodes": batch.state_size,
                   "graph": bool(args.graph), "steps_per_launch": kb,
                   "exponential": ("finite Taylor" if taylor else "Pade") if frozen else "Pade (weights built once)",
                   "tuned": (dict(tuned.choice.describe(), from_cache=tuned.from_cache) if tuned else None)},
        "roofline": roof,
        "detail": extra,
    }
    if taylor and not args.no_plain:
        # the same steps through the Pade build, for comparison
        lmep.lmep_set_option(lmep.LMEP_OPT_EXP_METHOD, lmep.LMEP_EXP_PADE)
        pflags = flags & ~lmep.LMEP_F_PERSISTENT  # the Pade build runs one step per launch
        batch.step(w, ua, 2, pflags, u_out=ub)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        batch.step(w, ua, args.steps, pflags, u_out=ub)
        torch.cuda.synchronize()
        pw = time.perf_counter() - t1
        lmep.lmep_set_option(lmep.LMEP_OPT_EXP_METHOD, lmep.LMEP_EXP_AUTO)
        out["pade_path"] = {"value": node_steps / pw, "unit": "node-steps/s",
                            "kind": "same steps, frozen-velocity weights by Pade scaling-and-squaring",
                            "ratio": value / (node_steps / pw)}
    if len(problems) > 1 and not args.no_plain:
        pv, pk = plain_forward(problems, states, min(args.steps, 20))
        out["plain"] = {"value": pv, "unit": "node-steps/s", "instances": pk,
                        "kind": "single-instance forward, instances one at a time, per-step eager launches",
                        "ratio": value / pv}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(problems[0], states[0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
