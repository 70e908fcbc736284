"""Throughput of the LMEP hot path on one MI355X.

Default workload: the batched path -- 4096 independent Allen-Cahn instances
(N_k uniform in [512, 65536], stencil n_k in {5, 7, 9, 11}, periodic or Neumann
ends, ETD1 with phi1 weights of the augmented local matrix built once per
instance) advanced 16 steps per launch, every stencil size in one launch.  A "step" is one time step of the whole
hot path for every instance: the weights are stationary, so after the first
build a step is the banded apply.

Printed, one JSON line:
  value     node-steps/s of the timed K steps of the batch (inputs resident in
            HBM, wall clock between synchronisations);
  roofline  the dominant kernel of those steps: algorithmic work per launch
            over its average launch duration, from HIP events recorded around
            each of its launches on the library's stream in a profiled pass
            over the same K steps;
  plain     the same instances one at a time through the single-instance
            forward (one lmep_step per instance, one step per launch);
  adjoint   the adjoint workload (64 Burgers trajectories of 262144 nodes,
            500 steps, a checkpoint every 50, loss against the state reached
            with nu * 1.1): forward + checkpointed reverse, beside its own
            plain single-instance forward, with the roofline of the reverse
            kernel;
  upwind_sweep  linear advection on one-sided stencils of n = 7 .. 15 at
            Courant number n/2 to a fixed final time (the time taken should
            not grow with n);
  single_instance  the viscous-Burgers workload (N = 65536, n = 7, weights
            rebuilt every step from the frozen velocity), 1000 steps;
  cpu_baseline  the oracle on a bounded sample of the batch, on the host's
            cores and on one thread.
Other workloads: --workload NAME (see make_workload).
"""
from __future__ import annotations

import argparse
import json
import math
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


def taylor_dd_flops(n: int, fused: bool) -> float:
    """Algorithmic flops of one node of the double-double finite-Taylor build
    (one-sided windows), each double-double operation counted by the FP64
    flops it takes (fma = 2; two-sum 6, add 20, multiply 10, multiply by a
    double 8, division by a double about 28 with the division counted as
    one, fma 30): per order K = 1 .. n-1 the K + 1 moments (four products and
    three adds each, the dispersion term carried too), their exponential and
    phi1 sums, and the contraction of both rows with the table; then the
    scaling and rounding of the rows, and with fusion the FP64 derivative and
    stencil sum."""
    add, mul, mul_d, div_d, fma = 20, 10, 8, 28, 30
    f = 0.0
    for K in range(1, n):
        moments = K + 1
        f += moments * (mul + (mul_d + add) + 2 * (mul + add))  # the recursion's terms
        f += moments * (add + div_d + add)                       # E and F sums
        f += 2 * n * fma                                         # W0, W1 contraction
    f += 2 * n * (mul_d + 1)                                     # scaling and rounding
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
        return [p], [u0], ("the paper's Burgers run: periodic N=1048576 n=19, nu=0.03, stationary L = nu D2, "
                           "N = -u u_x, ETDRK4")
    if name == "burgers_upwind":
        p, u0 = workloads.burgers_upwind()
        return [p], [u0], ("viscous Burgers N=65536 n=7 periodic on fully one-sided (upwind) stencils at "
                           "CFL 3.5, frozen-velocity ETD1, weights rebuilt every step")
    if name == "burgers_upwind15":
        p, u0 = workloads.burgers_upwind(n=15, cfl=7.5, amp=1e-4)
        return [p], [u0], ("viscous Burgers N=65536 n=15 periodic on one-sided stencils at CFL 7.5 (velocity 1 +- 1e-4), "
                           "frozen-velocity ETD1 with the weights in double-double, rebuilt every step")
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
    if name.startswith("upwind_advection"):
        n = int(name[len("upwind_advection"):] or 15)
        p, u0 = workloads.upwind_advection(n=n)
        return [p], [u0], f"linear advection N=1048576 periodic on one-sided stencils, n={n}, Courant {n / 2}"
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


def bench_adjoint(problems, states, steps, every, target=None):
    """Forward with a checkpoint every `every` steps + reverse through
    lmep_adjoint_step, loss 0.5 ||u(T) - target||^2 (target: the state the
    same u0 reaches with nu * 1.1, or zeros); gradients w.r.t. u0 and nu.
    Returns the wall seconds of forward + backward."""
    import torch
    import paper_2603_15964_amd as lmep
    from paper_2603_15964_amd import autograd as lad
    batch = lmep.Batch(problems, device="cuda:0")
    u0 = batch.pack(states).requires_grad_(True)
    nu = torch.tensor([p["nu"] for p in problems], dtype=torch.float64, device="cuda:0", requires_grad=True)
    if target is None:
        target = torch.zeros_like(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    uT = lad.solve(batch, u0, steps, nu=nu, checkpoint_every=every)
    loss = 0.5 * torch.sum((uT - target) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def adjoint_target(problems, target_problems, states, steps):
    """The state the same u0 reaches after `steps` steps with the target
    problems (nu * 1.1)."""
    import torch
    import paper_2603_15964_amd as lmep
    tb = lmep.Batch(target_problems, device="cuda:0")
    w = tb.empty_weights()
    with torch.no_grad():
        out = tb.step(w, tb.pack(states), steps)
    torch.cuda.synchronize()
    return out


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
    fre_ms, launches, rest_ms, name = 0.0, 0, 0.0, None
    try:
        pb = lmep.Batch(problems, device="cuda:0")  # a plan made with the profiling option
        for _ in range(reps):
            pb.adjoint_step(u0, lam)
            prof = lmep.lmep_profile_last()
            fre_ms += prof["build_ms"]
            launches += prof["build_launches"]
            rest_ms += prof["apply_ms"]
            name = lmep.lmep_profile_kernels()[0][0]
    finally:
        lmep.lmep_set_option(lmep.LMEP_OPT_PROFILE_ADJOINT, 0)
    p0 = problems[0]
    m = p0["n"] + {"linear": 0, "etd1": 1}[p0["scheme"]]
    if name.startswith("adj_fused_kernel"):
        # the whole reverse step of a tile in one kernel (per-node part and gathers)
        flops = batch.state_size * adj_fused_flops(p0["n"], m - p0["n"]) * reps
        mean_s = 0.0
    else:
        flops = batch.state_size * pair_pade_flops(m, mean_s) * reps
    tf = flops / (fre_ms / 1e3) / 1e12
    return {"bound": "alu", "achieved": tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / PEAK_FP64_TFLOPS, "traffic": measured_traffic([name], "burgers_adjoint"), "kernel": name,
            "avg_launch_us": fre_ms * 1e3 / max(1, launches), "flops_per_launch": flops / max(1, launches),
            "duration_from": "HIP events around each launch of the kernel",
            "mean_squarings": mean_s, "rest_of_reverse_step_us": rest_ms * 1e3 / reps}


def _cpu_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


def _omp_threads(k=None):
    """OpenMP threads of the oracle's runtime (libgomp), set to k if given."""
    import ctypes
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None
    if k is not None:
        gomp.omp_set_num_threads(int(k))
    return int(gomp.omp_get_max_threads())


def cpu_baseline(problems, states, budget_s: float = 12.0, one_thread_s: float = 6.0):
    """The oracle as it stands, on a bounded sample of the workload: the first
    instances of the batch (whole instances, weights built and applied by the
    oracle's own run) for as many steps as fit the budget, on all the threads
    its OpenMP runtime uses, then on one thread."""
    import oracle

    def sample(budget, steps=50):
        # the first instance, timed at one and at three steps, gives the
        # oracle's cost per node of its weight build and of a step
        t = time.perf_counter()
        oracle.run(problems[0], states[0], 1)
        t1 = time.perf_counter() - t
        t = time.perf_counter()
        oracle.run(problems[0], states[0], 3)
        t3 = time.perf_counter() - t
        n0 = problems[0]["N"]
        step_pn = max((t3 - t1) / 2, 1e-9) / n0
        build_pn = max(t1 - (t3 - t1) / 2, 0.0) / n0
        per_node = build_pn + steps * step_pn
        k, nodes = 0, 0
        while k < len(problems) and (nodes + problems[k]["N"]) * per_node <= budget:
            nodes += problems[k]["N"]
            k += 1
        k = max(k, 1)
        nodes = sum(int(p["N"]) for p in problems[:k])
        t = time.perf_counter()
        for p, u in zip(problems[:k], states[:k]):
            oracle.run(p, u, steps)
        el = time.perf_counter() - t
        return nodes * steps / el, k, steps, nodes

    model, nproc, usable = _cpu_info()
    threads = _omp_threads()
    v, k, steps, nodes = sample(budget_s)
    out = {"value": v, "unit": "node-steps/s", "cores": threads or usable, "kind": "oracle",
           "sample": f"first {k} of {len(problems)} instances ({nodes} nodes), {steps} steps each (weights built "
                     f"by the oracle's own run)",
           "cpu_model": model, "nproc": nproc, "usable_cpus": usable, "omp_threads": threads}
    if threads and threads > 1:
        _omp_threads(1)
        try:
            v1, k1, s1, n1 = sample(one_thread_s)
        finally:
            _omp_threads(threads)
        out["one_thread"] = {"value": v1, "unit": "node-steps/s",
                             "sample": f"first {k1} instances ({n1} nodes), {s1} steps each"}
    return out


def _parse_kernel(name):
    """(base name, [template integers or booleans]) of a kernel name."""
    if "<" not in name:
        return name, []
    base, args = name.split("<", 1)
    vals = []
    for t in args.rstrip(">").split(","):
        t = t.strip()
        vals.append(t == "true" if t in ("true", "false") else int(t))
    return base, vals


def kernel_work(name, problems, steps):
    """(bound, algorithmic work over `steps` steps, unit of work) of a kernel:
    FP64 flops for the builds and the multi-step kernels, HBM bytes for the
    one-step apply, LDS bytes for the resident kernel; None if unknown."""
    base, v = _parse_kernel(name)

    def group(pred):
        return [p for p in problems if pred(p)]

    def nl_id(p):
        return NONLIN_ID[p.get("nonlin", "none")] if p["scheme"] != "linear" else 0

    frozen = lambda p: p.get("nonlin") == "burgers_frozen"
    if base == "taylor_stepk_kernel":
        g = group(lambda p: frozen(p) and p["n"] == v[0])
        return "alu", taylor_flops(v[0], True) * sum(p["N"] for p in g) * steps, "flop"
    if base == "build_taylor_dd_kernel":
        g = group(lambda p: frozen(p) and p["n"] == v[0])
        return "alu", taylor_dd_flops(v[0], v[1]) * sum(p["N"] for p in g) * steps, "flop"
    if base == "build_taylor_kernel":
        g = group(lambda p: frozen(p) and p["n"] == v[0])
        return "alu", taylor_flops(v[0], v[1]) * sum(p["N"] for p in g) * steps, "flop"
    if base == "stepk_mixed_kernel":  # every size of one scheme and nonlinearity, more than 512 nodes
        # nonlinearity code 4: Allen-Cahn with coefficient 1 in every instance
        want = NONLIN_ID["allen_cahn"] if v[1] == 4 else v[1]
        g = group(lambda p: SCHEME_ID[p["scheme"]] == v[0] and nl_id(p) == want and not frozen(p)
                  and p.get("x") is None and p.get("window", "centred") == "centred" and p["N"] > 512)
        return "alu", sum(stationary_flops(p) * p["N"] for p in g) * steps, "flop"
    if base in ("stepk_kernel", "stepk_upwind_kernel", "stepk_rk4_kernel"):
        def side(p):
            if p.get("window", "centred") != "upwind" or p.get("c", 0.0) == 0.0:
                return 0
            return 1 if p["c"] > 0 else 2
        if base != "stepk_rk4_kernel":
            want = v[4] if base == "stepk_upwind_kernel" else 0
            g = group(lambda p: p["n"] == v[0] and SCHEME_ID[p["scheme"]] == v[1] and nl_id(p) == v[2]
                      and not frozen(p) and p.get("x") is None and side(p) == want)
        else:
            g = group(lambda p: p["n"] == v[0] and p["scheme"] == "etdrk4")
        return "alu", sum(stationary_flops(p) * p["N"] for p in g) * steps, "flop"
    if base == "apply_kernel":
        g = group(lambda p: p["n"] == v[0] and SCHEME_ID[p["scheme"]] == v[1] and nl_id(p) == v[2])
        per = 0.0
        for p in g:
            if p.get("x") is not None:
                per += p["N"] * (16.0 + 8.0 * KINDS[p["scheme"]] * p["n"])
            elif frozen(p):
                per += p["N"] * (16.0 + 16.0 * p["n"])
            else:
                per += p["N"] * 16.0
        return "hbm", per * steps, "byte"
    if base == "resident_kernel":
        g = group(lambda p: p["n"] == v[0] and SCHEME_ID[p["scheme"]] == v[1] and (p.get("x") is None) == v[3])

        def lds_reads(p):
            has_n = p["scheme"] != "linear" and p.get("nonlin", "none") != "none"
            return p["n"] * (1 + (2 if has_n and p["scheme"] == "etd2rk" else 0))
        return "lds", sum(p["N"] * 8.0 * lds_reads(p) for p in g) * steps, "byte"
    return None


def kernel_rooflines(batch, w, u, steps, flags, problems, workload):
    """A profiled pass over the same `steps` steps (HIP events around every
    launch, per kernel): per kernel its average launch time and algorithmic
    rate against its roofline; the dominant kernel (largest total time)
    first."""
    import paper_2603_15964_amd as lmep
    out = batch.empty_state()
    batch.step(w, u, steps, lmep.LMEP_F_PROFILE | (flags & lmep.LMEP_F_PERSISTENT), u_out=out)
    rows = []
    for name, ms, launches in sorted(lmep.lmep_profile_kernels(), key=lambda t: -t[1]):
        row = {"kernel": name, "launches": launches, "avg_launch_us": ms * 1e3 / max(1, launches),
               "total_ms": ms}
        wk = kernel_work(name, problems, steps)
        if wk is not None and ms > 0:
            bound, work, unit = wk
            rate = work / (ms / 1e3)
            if bound == "alu":
                row.update(bound="alu", achieved=rate / 1e12, peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                           frac=rate / 1e12 / PEAK_FP64_TFLOPS, flops_per_launch=work / launches)
            else:
                peak = PEAK_HBM_GBS if bound == "hbm" else PEAK_LDS_GBS
                row.update(bound=bound, achieved=rate / 1e9, peak=peak, unit="GB/s", frac=rate / 1e9 / peak,
                           bytes_per_launch=work / launches)
        rows.append(row)
    dom = dict(rows[0]) if rows else {}
    if dom:
        dom["traffic"] = measured_traffic([dom["kernel"]], workload)
        dom["duration_from"] = ("HIP events on the library's stream around each launch of this kernel (one pair "
                                "around all of them when a step runs this kernel alone), profiled pass over the "
                                "timed steps")
    return dom, rows


def forward_line(problems, states, steps, warmup, flags, kb=None):
    """Times `steps` steps of the batch after `warmup` untimed ones.  Returns
    (result dict, batch, weights, state the timed steps started from)."""
    import torch
    import paper_2603_15964_amd as lmep
    if kb is not None:
        lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, kb)
    batch = lmep.Batch(problems, device="cuda:0")
    w = batch.empty_weights()
    u0 = batch.pack(states)
    ua, ub = batch.empty_state(), batch.empty_state()
    if not all(p.get("nonlin") == "burgers_frozen" for p in problems):
        batch.build_weights(w, u0)
    if warmup > 0:
        batch.step(w, u0, warmup, flags, u_out=ua)
    else:
        ua.copy_(u0)
    # plans (and, with LMEP_F_GRAPH, the graph) of the timed call's shape
    batch.step(w, ua, steps if flags & lmep.LMEP_F_GRAPH else min(steps, 2 * (kb or 1)), flags, u_out=ub)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    batch.step(w, ua, steps, flags, u_out=ub)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    node_steps = batch.state_size * steps
    res = {"value": node_steps / wall, "unit": "node-steps/s", "steps": steps, "warmup": warmup,
           "ms_per_step": wall * 1e3 / steps, "gpu_event_ms": start.elapsed_time(stop), "wall_ms": wall * 1e3,
           "instances": batch.count, "nodes": batch.state_size}
    return res, batch, w, ua


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed steps of the headline workload")
    ap.add_argument("--warmup", type=int, default=200, help="untimed steps first (brings the clocks up)")
    ap.add_argument("--workload", default="allen_cahn_batch")
    ap.add_argument("--graph", action="store_true", help="replay the step loop from a hipGraph (cached by the plan)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain single-instance comparison runs")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint workload")
    ap.add_argument("--no-single", action="store_true", help="skip the single-instance Burgers workload")
    ap.add_argument("--separate-groups", action="store_true",
                    help="one multi-step launch per stencil size instead of one over every size "
                         "(LMEP_OPT_MERGE_GROUPS = 0)")
    ap.add_argument("--no-upwind-sweep", action="store_true",
                    help="skip the one-sided advection runs over stencil sizes")
    ap.add_argument("--adjoint-steps", type=int, default=500)
    ap.add_argument("--adjoint-every", type=int, default=50, help="checkpoint interval of the adjoint run")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (calibrates byte counters)")
    ap.add_argument("--launch", choices=("auto", "one-step", "persistent"), default="auto",
                    help="auto: several steps per launch wherever the multi-step kernels cover the workload; "
                         "--persistent is the same as --launch persistent")
    ap.add_argument("--persistent", action="store_true", help="advance several steps per launch")
    ap.add_argument("--steps-per-launch", type=int, default=None, choices=(1, 2, 4, 8, 16))
    ap.add_argument("--tune", action="store_true",
                    help="let the autotuner pick the launch configuration (cached per GPU and shape)")
    ap.add_argument("--exp-method", choices=("auto", "pade"), default="auto",
                    help="exponential of the frozen-velocity rebuild: finite Taylor series where it applies (auto) "
                         "or Pade scaling-and-squaring everywhere")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: the batch is one GPU's share (multi-GPU sharding is a design, not code); --gpus must be 1"}), flush=True)
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

    lmep.lmep_set_option(lmep.LMEP_OPT_EXP_METHOD,
                         lmep.LMEP_EXP_PADE if args.exp_method == "pade" else lmep.LMEP_EXP_AUTO)
    # the batch's stencil sizes share one multi-step launch (largest n first)
    lmep.lmep_set_option(lmep.LMEP_OPT_MERGE_GROUPS, 0 if args.separate_groups else 1)
    if args.workload == "burgers_adjoint":
        args.no_adjoint = False
    problems, states, desc = make_workload(args.workload)
    flags, kb = launch_choice(problems, args)
    if args.graph:
        flags |= lmep.LMEP_F_GRAPH
    tuned = None
    if args.tune:
        from paper_2603_15964_amd import tune as lt
        b0 = lmep.Batch(problems, device="cuda:0")
        w0 = b0.empty_weights()
        u00 = b0.pack(states)
        if not all(p.get("nonlin") == "burgers_frozen" for p in problems):
            b0.build_weights(w0, u00)
        tuned = lt.tune(b0, w0, u00, steps=max(4, min(args.steps, 50)))
        for o, v in tuned.choice.options.items():
            lmep.lmep_set_option(o, v)
        flags = (flags & lmep.LMEP_F_GRAPH) | tuned.choice.flags
        kb = tuned.choice.options.get(lmep.LMEP_OPT_STEPS_PER_LAUNCH, 1) if flags & lmep.LMEP_F_PERSISTENT else 1

    out = {"metric": "node-steps/s (weight build+apply, FP64) batched/adjoint vs plain @1e-10 err"}
    if args.workload == "burgers_adjoint":
        res = adjoint_line(problems, states, args)
        out.update(value=res.pop("value"), unit="node-steps/s", n_gpus=1, steps=args.adjoint_steps,
                   warmup=0, ms_per_step=res.pop("ms_per_step"), higher_is_better=True, scaling="weak",
                   vs_baseline=None, dtype="f64", data="synthetic",
                   config={"workload": desc, **res.pop("config")}, roofline=res.pop("roofline"))
        out.update(res)
    else:
        # the plain path first: the timed steps then run at the clocks a
        # sustained load holds, whatever the step counts asked for
        plain = None
        if len(problems) > 1 and not args.no_plain:
            plain = plain_forward(problems, states, min(args.steps, 20))
        res, batch, w, ua = forward_line(problems, states, args.steps, args.warmup, flags, kb)
        roof, rows = kernel_rooflines(batch, w, ua, args.steps, flags, problems, args.workload)
        frozen = any(p.get("nonlin") == "burgers_frozen" for p in problems)
        out.update(value=res["value"], unit="node-steps/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
                   ms_per_step=res["ms_per_step"], higher_is_better=True, scaling="weak", vs_baseline=None,
                   dtype="f64", data="synthetic",
                   config={"workload": desc, "path": "batched" if len(problems) > 1 else "single instance",
                           "instances": res["instances"], "nodes": res["nodes"],
                           "steps_per_launch": kb, "graph": bool(flags & lmep.LMEP_F_GRAPH),
                           "exponential": ("finite Taylor" if args.exp_method == "auto" else "Pade") if frozen
                           else "Pade (weights built once)",
                           "tuned": (dict(tuned.choice.describe(), from_cache=tuned.from_cache) if tuned else None)},
                   roofline=roof, kernels=rows,
                   detail={"gpu_event_ms": res["gpu_event_ms"], "wall_ms": res["wall_ms"]})
        if plain is not None:
            pv, pk = plain
            out["plain"] = {"value": pv, "unit": "node-steps/s", "instances": pk, "steps": min(args.steps, 20),
                            "kind": "single-instance forward: instances one at a time, one lmep_step call each, "
                                    "one step per launch",
                            "ratio": res["value"] / pv}
        if args.workload == "allen_cahn_batch":
            lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, 8)
            if not args.no_adjoint:
                ap_, as_, _ = make_workload("burgers_adjoint")
                out["adjoint"] = adjoint_line(ap_, as_, args)
            if not args.no_upwind_sweep:
                out["upwind_sweep"] = upwind_sweep()
            if not args.no_single:
                sp, ss, sdesc = make_workload("burgers")
                sflags, skb = launch_choice(sp, argparse.Namespace(launch="auto", persistent=False,
                                                                   steps_per_launch=None, exp_method="auto"))
                sres, sb, sw, su = forward_line(sp, ss, 1000, 100, sflags, skb)
                sroof, _ = kernel_rooflines(sb, sw, su, 1000, sflags, sp, "burgers")
                out["single_instance"] = {"workload": sdesc, "value": sres["value"], "unit": "node-steps/s",
                                          "steps": 1000, "warmup": 100, "ms_per_step": sres["ms_per_step"],
                                          "steps_per_launch": skb, "roofline": sroof}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(problems, states)
    print(json.dumps(out), flush=True)


def launch_choice(problems, args):
    """(flags, steps per launch): several steps per launch wherever the
    multi-step kernels cover every instance (stationary weights, centred or
    one-sided windows, 16 or 8 per launch;
    frozen velocity by the finite-Taylor kernel on Dirichlet or periodic grids
    under 2^20 nodes -- larger batches fill the GPU in one step), else one."""
    import paper_2603_15964_amd as lmep
    if args.launch == "one-step" and not args.persistent:
        return 0, 1
    frozen = [p.get("nonlin") == "burgers_frozen" for p in problems]
    if all(frozen):
        covered = all(p["bc"] != "neumann" and p.get("react", 0.0) == 0.0 for p in problems) and \
            args.exp_method == "auto"
        small = sum(int(p["N"]) for p in problems) < (1 << 20)
        multi = covered and (small or args.persistent or args.launch == "persistent")
        if not multi:
            return 0, 1
        kb = args.steps_per_launch
        if kb is None:
            # deepest launch whose largest region (512 positions) still writes
            # 128 nodes per block (the halo grows by n - 1 per step, 2 (n - 1)
            # for one-sided windows)
            reach = max((2 if p.get("window", "centred") == "upwind" else 1) * (int(p["n"]) - 1) for p in problems)
            kb = next((k for k in (8, 4, 2) if 512 - 2 * k * reach >= 128), 1)
        return lmep.LMEP_F_PERSISTENT, kb
    if any(frozen):
        return 0, 1
    nonuniform_small = all(p.get("x") is None or p["N"] <= 512 for p in problems)
    if nonuniform_small:
        # the deepest launch whose recomputed halo stays within 1/8 of the
        # 2048-position region: 16 steps for ETD1 Allen-Cahn up to n = 15 (the
        # launch's HBM pass costs about two steps of the n = 11 kernel), 8 for
        # KdV's two stencil passes per stage (ETDRK4 groups take at most 8)
        def halo(p, kb):
            nl = p.get("nonlin", "none")
            apps = (4 if p["scheme"] == "etdrk4" else 2) if (p["scheme"] in ("etd2rk", "etdrk4") and nl != "none") \
                else 1
            apps *= 2 if (p["scheme"] != "linear" and nl == "kdv") else 1
            return kb * apps * ((int(p["n"]) - 1) // 2)
        kb = args.steps_per_launch or next(k for k in (16, 8) if k == 8 or
                                           all(2 * halo(p, k) <= 2048 // 8 for p in problems if p.get("x") is None))
        return lmep.LMEP_F_PERSISTENT, kb
    return 0, 1


def upwind_sweep(stencils=(7, 9, 11, 13, 15), N=2 ** 20, transit=1.0 / 8.0, kb=16):
    """Sec. 4.1's efficiency claim for one-sided stencils: advection over a
    fixed time (the signal crosses `transit` of the periodic domain) at
    Courant number n/2, kb steps per launch.  The steps needed fall like 1/n
    while the work per step grows like n, so the time to the final time
    should not grow with n.  One warm-up run per n, then one timed run."""
    import torch
    import paper_2603_15964_amd as lmep
    import workloads
    lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, kb)
    rows = []
    for n in stencils:
        p, u0 = workloads.upwind_advection(n=n, N=N)
        steps = int(math.ceil(transit / p["dt"]))
        b = lmep.Batch([p], device="cuda:0")
        w = b.empty_weights()
        u = b.pack([u0])
        out = b.empty_state()
        b.build_weights(w, u)
        b.step(w, u, steps, lmep.LMEP_F_PERSISTENT, u_out=out)  # warm-up, plans
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(w, u, steps, lmep.LMEP_F_PERSISTENT, u_out=out)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        rows.append({"n": n, "courant": p["dt"] / p["h"], "steps": steps, "ms": secs * 1e3,
                     "us_per_step": secs * 1e6 / steps, "node_steps_per_s": N * steps / secs})
    for r in rows:
        r["time_vs_first"] = r["ms"] / rows[0]["ms"]
    lmep.lmep_set_option(lmep.LMEP_OPT_STEPS_PER_LAUNCH, 8)
    return {"workload": f"linear advection N={N} periodic, one-sided stencils at Courant n/2, final time "
                        f"{transit} of a transit, {kb} steps per launch",
            "rows": rows}


def adjoint_line(problems, states, args):
    """The adjoint workload: forward + checkpointed reverse, against the plain
    single-instance forward of the same trajectories."""
    import torch
    import paper_2603_15964_amd as lmep
    import workloads
    _, pt, _ = workloads.burgers_adjoint_batch()
    tprobs = [dict(pt)] * len(problems)
    steps, every = args.adjoint_steps, args.adjoint_every
    target = adjoint_target(problems, tprobs, states, steps)
    bench_adjoint(problems, states, min(steps, 10), min(steps, 10), target=None)  # warm-up: plans, code objects
    secs = bench_adjoint(problems, states, steps, every, target=target)
    nodes = sum(int(p["N"]) for p in problems)
    res = {"workload": "64 Burgers trajectories N=262144 n=9, ETD1 frozen velocity, forward + checkpointed reverse, "
                       "loss against the state reached with nu*1.1",
           "value": 2.0 * nodes * steps / secs, "unit": "node-steps/s",
           "node_steps": "forward and reverse steps, sum N x steps each (recomputation not counted)",
           "steps": steps, "ms_per_step": secs * 1e3 / steps, "wall_s": secs,
           "config": {"instances": len(problems), "nodes": nodes, "checkpoint_every": every},
           "roofline": adjoint_roofline(problems, states)}
    if not args.no_plain:
        pv, pk = plain_forward(problems, states, min(steps, 20))
        res["plain"] = {"value": pv, "unit": "node-steps/s", "instances": pk, "steps": min(steps, 20),
                        "kind": "single-instance forward only: trajectories one at a time, one step per launch"}
        res["ratio"] = res["value"] / pv
    torch.cuda.synchronize()
    return res


if __name__ == "__main__":
    main()
