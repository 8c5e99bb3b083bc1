"""Benchmark: KKT solves/s (refactor + FGMRES-IR to NRBE <= 1e-12) on one MI355X.

Workload (default): the largest single-GPU instance, a sequence of 5 same-pattern KKT systems
of 2,000,000 unknowns (n = 1,150,000, m = 850,000, 10.55 M nonzeros; D log-uniform in
[1e-12, 1e12], 1 % perturbation of H/J values per step, fresh right-hand side), FGMRES(50),
plain FP64 path.  `--config 2` runs the 60,000-unknown sequence of 20 systems (FGMRES(10)),
`--config 3` the 500,000-unknown one (FGMRES(30)).  The host analysis runs once (timed
separately); a timed step is one refactorization plus one FGMRES-IR solve of the next
system of the sequence, with every system's values and right-hand side already resident in
HBM.  The same steps are also run with FP32 factors as the preconditioner (mixed).

Prints ONE JSON line (see the keys below): solves/s, per-solve latency percentiles, the
HBM roofline of the dominant kernel (algorithmic bytes over its average launch time, from
HIP events recorded inside the library around that kernel's launches in the timed region;
an untimed pass before it times every kernel class to find the dominant one and to report the
per-class breakdown) and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E nameplate


def algorithmic_bytes(cls: str, ai: dict) -> float:
    """Bytes a kernel class must move per launch, each array counted once (FP64 factors, 4-byte
    indices), as the per-stage table of the method's data movement gives them:
      SpTRSV (one triangle): nnz_T (8 + 4) + (N + 1) 4 + 2 N 8    (values + indices, row
                             pointers, right-hand side read, solution written)
      refactorization:       f 8 (read) + f 4 (pattern) + f 8 (write) + 4 per precomputed
                             update position (the update list)
      SpMV:                  nnz_K 12 + (N + 1) 4 + 3 N 8"""
    n, nnz, lnz, unz, upd = ai["n"], ai["nnz"], ai["nnz_l"], ai["nnz_u"], ai["updates"]
    f = lnz + unz
    if cls == "trsv_l":
        return lnz * 12 + (n + 1) * 4 + 2 * n * 8
    if cls == "trsv_u":
        return unz * 12 + (n + 1) * 4 + 2 * n * 8
    if cls == "refactor":
        return f * (8 + 4 + 8) + upd * 4
    if cls == "spmv":
        return nnz * 12 + (n + 1) * 4 + 3 * n * 8
    raise KeyError(cls)


ROOT = os.path.dirname(os.path.abspath(__file__))
PROFILES = os.path.join(ROOT, "profiles")
# kernel-name prefixes of each class in the counter summary (the solve kernels carry a second
# template flag: dense segments on or off)
KERNEL_NAMES = {"trsv_l": "kkt::k_trsv<double,true", "trsv_u": "kkt::k_trsv<double,false",
                "refactor": "kkt::k_refactor<double", "spmv": "kkt::k_spmv_dots"}


def source_digest() -> str:
    """sha256 over the library's kernel and analysis sources (names and contents)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2401_13926_amd", "csrc")
    for fn in sorted(os.listdir(d)):
        if fn.endswith((".hip", ".cpp", ".hpp")):
            h.update(fn.encode())
            with open(os.path.join(d, fn), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def measured_traffic(cls: str, workload: str):
    """HBM bytes (read + written) per launch of a kernel class, from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary of this workload; None when there is none or the library
    sources changed since the counters were taken."""
    name = KERNEL_NAMES.get(cls)
    path = os.path.join(PROFILES, workload + "_hbm_counters.txt")
    if not name or not os.path.exists(path):
        return None
    digest = source_digest()
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) == 5 and parts[0] == "traffic" and parts[1].startswith(name) and parts[4] == digest:
                return float(parts[2]) + float(parts[3])
    return None


def copy_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy rate of this GPU (bytes read + bytes written per second, GB/s):
    the measured counterpart of the nameplate HBM peak."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    return 2.0 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9


def _cpu_worker(cfg, rank, procs, seconds, q):
    """One process of cpu_all_cores: regenerates the sequence (CPU only, no GPU use) and runs
    the oracle's direct method on systems rank, rank + procs, ... for about `seconds`."""
    sys.path.insert(0, ROOT)
    import kkt_synth as ks
    import oracle
    pattern = ks.make_pattern(cfg)
    nsys = ks.WORKLOAD_SHAPES[cfg]["steps"]
    Q = oracle.order(pattern.rowptr, pattern.colidx)
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        v, b = pattern.system(1 + (rank + done * procs) % nsys)
        oracle.direct_solve(pattern.rowptr, pattern.colidx, v, b, Q=Q)
        done += 1
    q.put((done, time.perf_counter() - t0))


def cpu_all_cores(cfg, seconds, procs):
    """The oracle's direct method in `procs` fresh processes (spawned, so none inherits this
    process's GPU state), each solving its share of the sequence's systems for about
    `seconds`: throughput for independent systems, which a sequence whose next system
    depends on this solution cannot use.  Returns (solves, wall seconds of the slowest)."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    q = ctx.Queue()
    ps = [ctx.Process(target=_cpu_worker, args=(cfg, r, procs, seconds, q)) for r in range(procs)]
    for p_ in ps:
        p_.start()
    res = [q.get() for _ in ps]
    for p_ in ps:
        p_.join()
    return sum(d for d, _ in res), max(t for _, t in res)


def host_cpu() -> dict:
    """Logical CPUs this process may run on, and the CPU model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"nproc": avail, "cpu_count": os.cpu_count(), "model": model}


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo, hi = int(np.floor(k)), int(np.ceil(k))
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


# workload name and FGMRES restart of each configuration
WORKLOADS = {1: ("kkt_single_7k", 10), 2: ("kkt_sequence_60k", 10), 3: ("kkt_sequence_500k", 30),
             5: ("kkt_sequence_2m", 50)}


def run_gpu(P, torch, pattern, systems, steps, warmup, precision, profile, restart=10, gram_schmidt=0,
            tile_lds_kib=0, cold_steps=0):
    dev = torch.device("cuda:0")
    v1, _ = systems[0]
    t0 = time.perf_counter()
    s = P.Solver(pattern.rowptr, pattern.colidx, v1, precision=precision, restart=restart,
                 gram_schmidt=gram_schmidt, tile_lds_kib=tile_lds_kib)
    analysis_s = time.perf_counter() - t0
    s.bind(dev)
    vals = [torch.as_tensor(v, device=dev) for v, _ in systems]
    rhs = [torch.as_tensor(b, device=dev) for _, b in systems]
    x = torch.empty_like(rhs[0])
    M = len(systems)
    for i in range(warmup):
        s.refactor(vals[i % M])
        s.solve(rhs[i % M], x, allow_noconv=True)
    torch.cuda.synchronize()
    # Untimed breakdown pass with every kernel class timed (two events per launch cost about
    # 10 % of a step); it names the dominant class, whose launches alone carry events in the
    # timed region below.
    times, breakdown, dom = None, None, None
    if profile:
        s.set_profiling(True)
        for i in range(min(steps, 20)):
            k = (warmup + i) % M
            s.refactor(vals[k])
            s.solve(rhs[k], x, allow_noconv=True)
        breakdown = s.kernel_times()
        cands = [c for c in ("refactor", "trsv_l", "trsv_u", "spmv") if breakdown[c][0] > 0]
        dom = max(cands, key=lambda c: breakdown[c][1])
        s.set_profiling(True, classes=[dom])
    lat = []
    infos = []
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        k = (warmup + i) % M
        ev[i][0].record()
        s.refactor(vals[k])
        _, info = s.solve(rhs[k], x, allow_noconv=True)
        ev[i][1].record()
        infos.append(info)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = [a.elapsed_time(b) for a, b in ev]
    if profile:
        times = s.kernel_times()
        s.set_profiling(False)
    # cold-cache leg (not part of `value`): before each step a 1 GiB device copy evicts the
    # 4 MiB L2s and the 256 MiB MALL; the step itself is timed with events as above
    cold = None
    if cold_steps > 0:
        flush_src = torch.ones((1 << 30) // 8, dtype=torch.float64, device=dev)
        flush_dst = torch.empty_like(flush_src)
        cold = []
        for i in range(cold_steps):
            k = (warmup + i) % M
            flush_dst.copy_(flush_src)
            a, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            s.refactor(vals[k])
            s.solve(rhs[k], x, allow_noconv=True)
            b_.record()
            b_.synchronize()
            cold.append(a.elapsed_time(b_))
        del flush_src, flush_dst
    # solutions of every system of the sequence, after the timed region (for the comparison
    # with the CPU baseline's solutions)
    xs, nrbe_all = [], []
    for k in range(M):
        s.refactor(vals[k])
        _, info = s.solve(rhs[k], x, allow_noconv=True)
        xs.append(x.cpu().numpy().copy())
        nrbe_all.append(info["nrbe"])
    return dict(nrbe_all=nrbe_all, solver=s, analysis_s=analysis_s, wall=wall, lat=lat, infos=infos, times=times,
                breakdown=breakdown, dominant=dom, xs=xs, cold=cold)


def cpu_baseline(pattern, systems, budget_s, gpu_xs=None):
    """The oracle's plain direct method (ordering reused, fresh threshold-pivoted LU and
    triangular solves per system) on the first systems of the sequence, single-threaded,
    until about budget_s seconds of work.  On the first pass over the sequence its solutions
    are compared with the GPU's (relative difference in the infinity norm, against the bound
    1e-8 times the condition estimate of that system); the condition estimates are not timed."""
    import oracle
    Q = oracle.order(pattern.rowptr, pattern.colidx)
    done = 0
    el = 0.0
    cmp = []
    while True:
        v, b = systems[done % len(systems)]
        t0 = time.perf_counter()
        x_o, f = oracle.direct_solve(pattern.rowptr, pattern.colidx, v, b, Q=Q)
        el += time.perf_counter() - t0
        if gpu_xs is not None and done < len(systems):
            rel = float(np.max(np.abs(gpu_xs[done] - x_o)) / np.max(np.abs(x_o)))
            cmp.append((rel, f.condest(pattern.rowptr, v)))
        done += 1
        if el >= budget_s or done >= 200:
            break
    return done, el, cmp


def run_serving(P, torch, args):
    """Serving workload: requests of 8 patterns (dims 7,000..500,000) arrive as a Poisson
    process; each is the next system of its pattern (refactor + FGMRES-IR).  Then the same
    requests all at once (saturation).  Latency = completion - arrival, from the library."""
    import threading
    import kkt_synth as ks
    dev = torch.device("cuda:0")
    npat = len(ks.SERVING_DIMS)
    steps = max(1, args.serve_steps)
    pats, vals, rhs = [], [], []
    t0 = time.perf_counter()
    for k in range(npat):
        p = ks.make_pattern(4, k)
        pats.append(p)
        sys_k = [p.system(s) for s in range(1, steps + 1)]
        vals.append([torch.as_tensor(v, device=dev) for v, _ in sys_k])
        rhs.append([torch.as_tensor(b, device=dev) for _, b in sys_k])
    gen_s = time.perf_counter() - t0
    srv = P.Server(int(args.pool_gb * (1 << 30)), workers=args.workers, device=dev, max_batch=args.max_batch,
                   graphs=not args.no_graphs)
    t0 = time.perf_counter()
    pids = [srv.add_pattern(p.rowptr, p.colidx, p.system(1)[0]) for p in pats]
    analysis_s = time.perf_counter() - t0
    print("serving: %d patterns analysed in %.1f s (inputs %.1f s)" % (npat, analysis_s, gen_s),
          file=sys.stderr, flush=True)
    rng = np.random.default_rng([2401, 4])
    pat_of = rng.integers(0, npat, size=args.requests)
    gaps = rng.exponential(1.0 / args.rate, size=args.requests)

    def one_run(saturate):
        nxt = [0] * npat
        res = [None] * args.requests
        tickets = [None] * args.requests
        ready = threading.Semaphore(0)

        def collector():
            for i in range(args.requests):
                ready.acquire()
                res[i] = srv.wait(tickets[i])
        th = threading.Thread(target=collector)
        th.start()
        start = time.perf_counter()
        t_arr = start
        for i in range(args.requests):
            if not saturate:
                t_arr += gaps[i]
                dt = t_arr - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
            k = int(pat_of[i])
            j = nxt[k] % steps
            nxt[k] += 1
            x = torch.empty_like(rhs[k][j])
            tickets[i] = srv.submit(pids[k], vals[k][j], rhs[k][j], x)
            ready.release()
        th.join()
        wall = time.perf_counter() - start
        lat = [r[2]["latency_ms"] for r in res]
        svc = [r[2]["service_ms"] for r in res]
        conv = [r[1]["converged"] == 1 for r in res]
        return {"solves_per_s": args.requests / wall, "wall_s": wall,
                "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
                "service_p50_ms": percentile(svc, 50), "service_p99_ms": percentile(svc, 99),
                "all_converged": all(conv), "repivots": int(sum(r[1]["repivoted"] for r in res)),
                "max_nrbe": max(r[1]["nrbe"] for r in res)}

    poisson = one_run(False)
    print("poisson run done", file=sys.stderr, flush=True)
    sat = one_run(True)
    st = srv.stats()
    srv.close()
    out = {
        "metric": "KKT solves/s served (refactor+FGMRES-IR to NRBE<=1e-12), p50/p99 latency ms",
        "value": poisson["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.requests,
        "warmup": 0, "ms_per_step": 1e3 * poisson["wall_s"] / args.requests, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded KKT generator, %d systems per pattern cycled)" % steps,
        "config": {"workload": "kkt_serving_8_patterns", "dims": list(ks.SERVING_DIMS), "requests": args.requests,
                   "rate_per_s": args.rate, "workers": args.workers, "pool_gb": args.pool_gb,
                   "max_batch": args.max_batch, "graphs": not args.no_graphs},
        "poisson": poisson, "saturation": sat, "server": st, "analysis_s": analysis_s,
    }
    print(json.dumps(out), flush=True)


def run_hykkt(P, torch, args):
    """HyKKT on the same workload with a zero (2,2) block: per step, the refactorization of
    H_gamma and the CG solve of the next system; the FGMRES-IR path is timed on the same
    systems for comparison (its (2,2) block is exactly zero as well)."""
    import kkt_synth as ks
    dev = torch.device("cuda:0")
    cfg = args.config
    pattern = ks.make_pattern(cfg, delta=0.0)
    nsys = ks.WORKLOAD_SHAPES[cfg]["steps"]
    systems = [pattern.system(k) for k in range(1, nsys + 1)]
    vals = [torch.as_tensor(v, device=dev) for v, _ in systems]
    rhs = [torch.as_tensor(b, device=dev) for _, b in systems]
    t0 = time.perf_counter()
    h = P.HyKKT(pattern.rowptr, pattern.colidx, systems[0][0], n_primal=pattern.n).bind(dev)
    analysis_s = time.perf_counter() - t0
    print("hykkt: analysis %.1f s" % analysis_s, file=sys.stderr, flush=True)
    steps = max(1, args.steps)
    infos, lat = [], []
    for i in range(args.warmup + steps):
        k = i % nsys
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        h.refactor(vals[k])
        _, info = h.solve(rhs[k], allow_noconv=True)
        torch.cuda.synchronize()
        if i >= args.warmup:
            lat.append(1e3 * (time.perf_counter() - s0))
            infos.append(info)
        print("hykkt step %d: %.1f ms, CG %d" % (i, 1e3 * (time.perf_counter() - s0), info["cg_iterations"]),
              file=sys.stderr, flush=True)
    wall = 1e-3 * sum(lat)
    wname, restart = WORKLOADS[cfg]
    r64 = run_gpu(P, torch, pattern, systems, min(steps, 10), 1, P.PREC_FP64, False, restart)
    out = {
        "metric": "KKT solves/s by HyKKT (H_gamma refactor + CG on the Schur complement, NRBE<=1e-12)",
        "value": steps / wall, "unit": "solves/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded KKT generator with a zero (2,2) block)",
        "config": {"workload": wname + "_delta0", "N": pattern.N, "nnz": pattern.nnz, "systems": nsys,
                   "gamma": infos[0]["gamma"], "cg_tol": 1e-12},
        "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
        "cg_iterations": [int(i["cg_iterations"]) for i in infos],
        "all_converged": all(i["converged"] == 1 for i in infos),
        "max_nrbe": max(i["nrbe"] for i in infos), "analysis_s": analysis_s,
        "hgamma_nnz_and_factor": list(h.sizes()),
        "fgmres_ir_same_systems": {"solves_per_s": min(steps, 10) / r64["wall"],
                                   "iterations": [int(i["iterations"]) for i in r64["infos"]],
                                   "max_nrbe": max(i["nrbe"] for i in r64["infos"])},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=5, choices=sorted(WORKLOADS),
                    help="workload: 1 (7k, one system), 2 (60k x 20), 3 (500k x 10), 5 (2M x 5, "
                         "the largest single-GPU instance; default)")
    ap.add_argument("--mixed-steps", type=int, default=10)
    ap.add_argument("--gram-schmidt", choices=["cgs2", "dcgs2"], default="cgs2",
                    help="Arnoldi orthogonalization: CGS2 (default) or delayed CGS2 (one reduction per step)")
    ap.add_argument("--cold-steps", type=int, default=10,
                    help="steps timed after a 1 GiB cache flush each (reported apart from value)")
    ap.add_argument("--cpu-procs", type=int, default=min(16, os.cpu_count() or 1),
                    help="also time the oracle in this many independent processes (0: skip)")
    ap.add_argument("--tile-lds-kib", type=int, default=0,
                    help="LDS budget of a triangular-solve tile in KiB (0: the library default)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--serve", action="store_true",
                    help="serving workload: Poisson arrivals over 8 patterns, then saturation")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--workers", type=int, default=8,
                    help="serving worker threads, one stream each (4: 187 solves/s, 8: 206, 16: 199 "
                         "at 200/s offered)")
    ap.add_argument("--pool-gb", type=float, default=32.0)
    ap.add_argument("--max-batch", type=int, default=4,
                    help="serving: most same-pattern requests refactored in one launch (1: no batching)")
    ap.add_argument("--no-graphs", action="store_true",
                    help="serving: launch batched refactorizations directly instead of from HIP graphs")
    ap.add_argument("--hykkt", action="store_true",
                    help="HyKKT on the workload with a zero (2,2) block, FGMRES-IR on the same systems")
    ap.add_argument("--serve-steps", type=int, default=3)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 256 MiB device buffer 4 times (reference kernel for the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this solver has no multi-GPU path "
              "(a single KKT sequence is solved on one device); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import kkt_synth as ks
    import paper_2401_13926_amd as P
    try:
        P.lib()
    except ImportError:
        from paper_2401_13926_amd import build
        build.build(force=True)
        P.lib()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.serve:
        run_serving(P, torch, args)
        return
    if args.hykkt:
        run_hykkt(P, torch, args)
        return
    if args.calibrate_copy:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": nbytes, "copy_bytes_written_per_launch": nbytes,
                          "launches": 4}), flush=True)
        return

    cfg = args.config
    pattern = ks.make_pattern(cfg)
    nsys = ks.WORKLOAD_SHAPES[cfg]["steps"]
    systems = [pattern.system(k) for k in range(1, nsys + 1)]
    print("workload config %d: N=%d nnz=%d systems=%d" % (cfg, pattern.N, pattern.nnz, nsys),
          file=sys.stderr, flush=True)

    wname, restart = WORKLOADS[cfg]
    gs = P.GS_DCGS2 if args.gram_schmidt == "dcgs2" else P.GS_CGS2
    r64 = run_gpu(P, torch, pattern, systems, args.steps, args.warmup, P.PREC_FP64, not args.no_profile, restart, gs,
                  args.tile_lds_kib, args.cold_steps)
    copy_gbs = copy_bandwidth(torch)
    ai = r64["solver"].info()
    print("fp64 done: %.1f ms/step" % (1e3 * r64["wall"] / args.steps), file=sys.stderr, flush=True)
    rmx = None
    if args.mixed_steps > 0:
        rmx = run_gpu(P, torch, pattern, systems, args.mixed_steps, 1, P.PREC_MIXED, False, restart, gs,
                      args.tile_lds_kib)
        print("mixed done: %.1f ms/step" % (1e3 * rmx["wall"] / args.mixed_steps), file=sys.stderr, flush=True)

    infos = r64["infos"]
    value = args.steps / r64["wall"]
    out = {
        "metric": "KKT solves/s (refactor+FGMRES-IR to NRBE<=1e-12), FP32-LU vs FP64; p50/p99 ms",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r64["wall"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded KKT generator; the paper's ACTIVSg sequences are not available)",
        "config": {"workload": wname, "N": pattern.N,
                   "nnz": pattern.nnz, "systems": nsys, "restart": restart, "delta_tol": 1e-14,
                   "nrbe_target": 1e-12, "precision": "fp64", "gram_schmidt": args.gram_schmidt,
                   "tile_lds_kib": args.tile_lds_kib},
        "p50_ms": percentile(r64["lat"], 50),
        "p99_ms": percentile(r64["lat"], 99),
        "cold_cache": None if not r64["cold"] else {
            "steps": len(r64["cold"]), "p50_ms": percentile(r64["cold"], 50), "p99_ms": percentile(r64["cold"], 99),
            "solves_per_s_from_mean": 1e3 / float(np.mean(r64["cold"])),
            "flush": "1 GiB device copy before each step (L2s and MALL evicted)"},
        "max_nrbe": max(i["nrbe"] for i in infos),
        "all_converged": all(i["converged"] == 1 for i in infos),
        "mean_iterations": float(np.mean([i["iterations"] for i in infos])),
        "analysis_s": r64["analysis_s"],
        "factor": {k: ai[k] for k in ("nnz_l", "nnz_u", "levels_refactor", "levels_l", "levels_u", "updates")},
    }
    if rmx is not None:
        mi = rmx["infos"]
        out["mixed"] = {
            "value": args.mixed_steps / rmx["wall"], "unit": "solves/s",
            "p50_ms": percentile(rmx["lat"], 50), "p99_ms": percentile(rmx["lat"], 99),
            "fallback_fraction": float(np.mean([i["fallback"] for i in mi])),
            "max_nrbe": max(i["nrbe"] for i in mi),
            "all_converged": all(i["converged"] == 1 for i in mi),
        }
    t = r64["times"]
    if t:
        bd = r64["breakdown"]
        out["kernel_ms"] = {k: {"launches": n, "total_ms": ms} for k, (n, ms) in bd.items()}
        out["kernel_ms_note"] = ("every class timed, %d untimed steps before the timed region; in the "
                                 "timed region only the dominant class carries events" % min(args.steps, 20))
        dom = r64["dominant"]
        n_l, ms = t[dom]
        avg_s = ms / n_l / 1e3
        bytes_per = algorithmic_bytes(dom, ai)
        achieved = bytes_per / avg_s / 1e9
        traffic = measured_traffic(dom, wname)
        out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                           "avg_launch_us": avg_s * 1e6, "algorithmic_bytes_per_launch": bytes_per,
                           "measured_copy_peak": copy_gbs, "frac_of_measured_copy": achieved / copy_gbs}
        # every class of the breakdown pass against the same peak (SpMV and refactorization
        # separately, as well as the dominant class above)
        per = {}
        for c in ("refactor", "trsv_l", "trsv_u", "spmv"):
            if bd[c][0] > 0:
                us = bd[c][1] / bd[c][0] * 1e3
                by = algorithmic_bytes(c, ai)
                per[c] = {"avg_launch_us": us, "algorithmic_bytes_per_launch": by,
                          "achieved_gbs": by / us / 1e3, "frac": by / us / 1e3 / HBM_PEAK_GBS}
        out["roofline_per_kernel"] = per
        # the second floor: dependent levels, each paid in sequence whatever the bandwidth
        lv = {"refactor": ai["levels_refactor"], "trsv_l": ai["levels_l"], "trsv_u": ai["levels_u"]}
        out["dependency_floor"] = {
            "levels": lv,
            "us_per_level": {c: bd[c][1] / max(1, bd[c][0]) * 1e3 / lv[c] for c in lv if bd[c][0] > 0},
            "note": "average launch time / DAG levels of that launch; the solves and the refactorization are "
                    "bound by this chain, not by HBM bandwidth"}
    if not args.no_cpu and args.cpu_procs > 0:
        done_p, wall_p = cpu_all_cores(cfg, args.cpu_seconds / 2, args.cpu_procs)
        out["cpu_all_cores"] = {"value": done_p / wall_p, "unit": "solves/s", "processes": args.cpu_procs,
                                "kind": "oracle", "note": "independent systems, one per process at a time; "
                                "a sequence whose next system needs this solution cannot use it"}
    if not args.no_cpu:
        done, el, cmp = cpu_baseline(pattern, systems, args.cpu_seconds, r64["xs"])
        out["cpu_baseline"] = {"value": done / el, "unit": "solves/s", "cores": 1, "kind": "oracle",
                               "host": host_cpu(),
                               "sample": "%d systems of the same sequence, plain direct method (reused "
                                         "ordering, fresh threshold-pivoted LU + triangular solves), "
                                         "single thread, %.1f s" % (done, el)}
        if cmp:
            out["vs_oracle"] = {
                "systems": len(cmp),
                "max_rel_diff": max(r for r, _ in cmp),
                "max_condest": max(c for _, c in cmp),
                "all_within_1e-8_condest": all(r <= 1e-8 * c for r, c in cmp),
                "max_ratio_to_bound": max(r / (1e-8 * c) for r, c in cmp),
                "per_system": [{"system": k + 1, "rel_diff": r, "condest": c, "nrbe": n_}
                               for k, ((r, c), n_) in enumerate(zip(cmp, r64["nrbe_all"]))],
                "note": "rel_diff = ||x_gpu - x_oracle||_inf / ||x_oracle||_inf against the oracle's plain "
                        "direct method; condest = the oracle's 1-norm condition estimate of that system",
            }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
