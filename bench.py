"""Benchmark of the space-time DG slab residual on one MI355X.

Workload: PEC unit-cube cavity, 32^3 axis-aligned hexahedra, p = 4, q = 3,
two materials (eps = 1 for x < 0.5, else 4; mu = 1), dt = 0.01; inputs are
seeded N(0, 1) coefficient vectors, resident in HBM before timing starts.

A step is one residual apply over the whole mesh (the operator the slab's
GMRES applies every iteration: mass, curl, centred fluxes, P^{-1} fused),
in FP32 (the apply used inside FP64 iterative refinement).  The same apply in
FP64 (the plain FP64 path) is timed right after, on the same inputs, and the
FP32+refinement and plain-FP64 slab solves are timed on the first slab of the
workload's mode-superposition initial field.

Prints one JSON line.  value = trial degrees of freedom 6 (q+1)(p+1)^3 n_el per
apply / seconds per apply, in GDoF/s.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    # enough untimed applies (~0.1 s) for the GPU to reach steady clocks: with
    # 10 the timed applies still ran ~10% slower than in steady state
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--settle-s", type=float, default=1.0,
                    help="seconds of untimed applies before the warm-up steps, so that the GPU's clocks "
                         "have settled whatever --warmup is (a few warm-up steps alone leave the timed "
                         "applies ~20%% slower)")
    ap.add_argument("--dist-steps", type=int, default=50,
                    help="extra applies timed one by one (an event pair each) after the timed region, "
                         "for the p10/p50/p90 of the launch duration (0 = skip)")
    ap.add_argument("--n", type=int, default=32, help="mesh is n^3 elements")
    ap.add_argument("--p", type=int, default=4)
    ap.add_argument("--q", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-march", action="store_true",
                    help="skip the 64-slab marches of the solve leg and the march of the local-time leg")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="elements in the oracle's timed sample (0 = sized to ~15 s)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--no-graded", action="store_true", help="skip the graded trilinear 24^3 leg")
    ap.add_argument("--no-large", action="store_true", help="skip the 48^3 p=6 q=4 leg")
    ap.add_argument("--no-local-time", action="store_true",
                    help="skip the leg with local time steps (32^3 two-material cavity, 4/2/1 sub-intervals)")
    ap.add_argument("--no-diss", action="store_true", help="skip the dissipative (D_h, c = 1) leg")
    ap.add_argument("--no-reoriented", action="store_true",
                    help="skip the leg with every element's vertices relabelled by a random cube rotation")
    ap.add_argument("--serve-requests", type=int, default=256,
                    help="requests of the Poisson serving stream (0 = skip the serving leg)")
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--serve-max-active", type=int, default=16)
    ap.add_argument("--serve-krylov", choices=("fp32", "fp64"), default="fp32",
                    help="storage of the serving solver's Krylov basis (sums are FP64 either way)")
    ap.add_argument("--serve-batch", type=int, default=1,
                    help="1: requests of one kernel group run their restart cycles batched")
    ap.add_argument("--serve-graph", type=int, default=1,
                    help="1: the serving solvers replay Arnoldi iterations as captured HIP graphs")
    ap.add_argument("--serve-eta-rel", type=float, default=1e-3,
                    help="also run the stream with inexact solves, eta_it <= this * sqrt(2 E(0)) per "
                         "request (0 = skip)")
    return ap.parse_args()


def settle(stdg, torch, mh, dt, prec, mode, x, y, seconds):
    """Untimed applies for `seconds` of wall time (clock ramp-up)."""
    if seconds <= 0:
        return 0
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    n = 0
    while time.perf_counter() - t0 < seconds:
        for _ in range(20):
            stdg.stdg_residual_apply(mh, dt, prec, mode, x, None, y, stream)
        n += 20
        torch.cuda.synchronize()
    return n


def launch_distribution(stdg, torch, mh, dt, prec, mode, x, y, steps):
    """p10 / p50 / p90 of the launch duration (ms), one event pair per apply,
    measured after the timed region (the events themselves add a little)."""
    if steps <= 0:
        return None
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        stdg.stdg_residual_apply(mh, dt, prec, mode, x, None, y, stream)
        b.record(stream)
    torch.cuda.synchronize()
    d = np.array([a.elapsed_time(b) for a, b in ev])
    return {"p10_ms": round(float(np.percentile(d, 10)), 5), "p50_ms": round(float(np.percentile(d, 50)), 5),
            "p90_ms": round(float(np.percentile(d, 90)), 5), "launches": steps}


def time_applies(stdg, torch, mh, dt, prec, mode, x, y, steps, warmup, settle_s=0.0):
    """Wall time of `steps` applies after `warmup` untimed ones (preceded by
    `settle_s` seconds of untimed applies), and the average launch duration
    from one pair of HIP events on the launch stream bracketing the timed
    launches (one kernel per apply on this mesh; the average includes the
    short gaps between launches).  Events between the launches would
    themselves add 1-3% to each step."""
    stream = torch.cuda.current_stream()
    settle(stdg, torch, mh, dt, prec, mode, x, y, settle_s)
    for _ in range(warmup):
        stdg.stdg_residual_apply(mh, dt, prec, mode, x, None, y, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        stdg.stdg_residual_apply(mh, dt, prec, mode, x, None, y, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.full(steps, e0.elapsed_time(e1) / steps)  # ms per launch
    return wall, per


def practical_ceiling(stdg, torch, mib=2048, reps=20):
    """HBM bytes per second of the library's streaming copy (16-byte
    non-temporal loads and stores over the whole chip): `mib` MiB read and
    written per launch, averaged over `reps` launches after 5 untimed ones."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(5):
        stdg.stdg_stream_copy(src, dst, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        stdg.stdg_stream_copy(src, dst, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(src[:1 << 20], dst[:1 << 20])) and bool(torch.equal(src[-1024:], dst[-1024:]))
    del src, dst
    if not ok:
        raise RuntimeError("streaming copy produced wrong data")
    return {"mib": mib, "ms": ms, "gb_per_s": 2 * mib * (1 << 20) / (ms * 1e-3) / 1e9}


def measured_traffic(prec, variant=""):
    """HBM bytes per launch of the timed kernel (variant "dissipative_": the
    kernel with D_h) from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, if it was taken on the current kernel source (else None)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("residual_kernel.h", "residual_inst.hip"):
        with open(os.path.join(ROOT, "paper_1307_5310_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    path = os.path.join(ROOT, "profiles", "residual_apply_cavity32_p4q3_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if ("sha256[:16] (residual_kernel.h + residual_inst.hip): " + h.hexdigest()[:16]) not in text:
        return None
    key = "traffic_bytes_%s%s = " % (variant, "fp32" if prec == 1 else "fp64")
    for line in text.splitlines():
        if line.startswith(key):
            return float(line[len(key):])
    return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def oracle_small():
    """The oracle on the small cavity (4^3, p = 2, q = 1, dt = 0.05) in full:
    one residual apply and the direct solve of its first slab from TE101."""
    import synth
    from oracle import fields
    from oracle.dg import Discretisation
    cfg = synth.cavity_small()
    m = cfg["mesh"]
    d = Discretisation(m.vertices, m.hexes, m.p, m.q, m.eps, m.mu)
    U = synth.random_vector(d.trial_off[-1], 0)
    d.residual(U, cfg["dt"])  # reference matrices cached outside the timing
    t = time.perf_counter()
    d.residual(U, cfg["dt"])
    t_apply = time.perf_counter() - t
    s0 = fields.project(d, fields.te101, 0.0)
    t = time.perf_counter()
    d.solve_direct(s0, cfg["dt"])
    t_solve = time.perf_counter() - t
    return {"apply_s": round(t_apply, 4), "slab_solve_direct_s": round(t_solve, 4),
            "trial_dof": int(d.trial_off[-1])}


def cpu_baseline(cfg, sample_n):
    """The oracle as it stands, on a bounded sample of the workload's elements."""
    from oracle.dg import Discretisation
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    m = cfg["mesh"]
    d = Discretisation(m.vertices, m.hexes, m.p, m.q, m.eps, m.mu)
    import synth
    x = synth.random_vector(m.unknown_size(), 0)
    U = d.embed_unknowns(x)
    rng = np.random.default_rng(7)
    # warm the oracle's caches (reference matrices) outside the timing
    d.apply_rows(U, cfg["dt"], [0])
    if sample_n <= 0:
        t = time.perf_counter()
        d.apply_rows(U, cfg["dt"], list(rng.choice(m.n_elements, 16, replace=False)))
        per = (time.perf_counter() - t) / 16
        sample_n = int(min(m.n_elements, max(16, 15.0 / max(per, 1e-6))))
    sample = list(rng.choice(m.n_elements, sample_n, replace=False))
    t = time.perf_counter()
    d.apply_rows(U, cfg["dt"], sample)
    el = time.perf_counter() - t
    a = int(m.p[0]) + 1
    q = int(m.q[0])
    dof = 6 * (q + 1) * a ** 3 * sample_n
    small = oracle_small()
    return {"value": dof / el / 1e9, "unit": "GDoF/s", "cores": int(threads), "cpu_model": cpu_model(),
            "small_cavity": small,
            "kind": "oracle",
            "sample": "%d random elements of the %d-element mesh, operator apply (dense local blocks), %.1f s"
                      % (sample_n, m.n_elements, el)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1307_5310_amd as stdg
    import synth

    cfg = synth.cavity_two_material(n=args.n, p=args.p, q=args.q)
    m = cfg["mesh"]
    dt = cfg["dt"]
    a, q, ne = args.p + 1, args.q, m.n_elements
    trial_dof = 6 * (q + 1) * a ** 3 * ne
    log("workload %s: %d elements, %.1f M trial DoF" % (cfg["name"], ne, trial_dof / 1e6))
    ctx = stdg.stdg_init(0, 0)
    mh = stdg.stdg_mesh_upload(ctx, m.vertices, m.hexes, m.p, m.q, m.eps, m.mu)
    # element order of the kernels' work lists: the library's autotuner (timed
    # here, outside the timed region)
    tuned = stdg.stdg_mesh_autotune(mh, stdg.STDG_FP32, dt, reps=10)
    order = tuned["order"]
    log("autotuned work-list order: %s, launch variants %s"
        % ("Morton" if order == 0 else "columns of %d" % order, tuned["variants"]))
    info = stdg.stdg_mesh_info(mh)
    nu = info["unknown_size"]
    x64 = torch.from_numpy(synth.random_vector(nu, 0)).cuda()
    x32 = x64.float()
    y32 = torch.empty(nu, dtype=torch.float32, device="cuda")
    y64 = torch.empty(nu, dtype=torch.float64, device="cuda")
    mode = stdg.STDG_OPERATOR_PRECOND

    if args.calib_copy_mib > 0:
        # counter calibration: the library's streaming copy, which reads and
        # writes exactly this many MiB
        nbytes = args.calib_copy_mib * (1 << 20)
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").normal_()
        dst = torch.empty_like(src)
        for _ in range(3):
            stdg.stdg_stream_copy(src, dst, torch.cuda.current_stream())
        torch.cuda.synchronize()
        log("calibration copy of %d MiB done" % args.calib_copy_mib)
        del src, dst
    ceiling = practical_ceiling(stdg, torch)
    log("practical ceiling: streaming copy of %d MiB at %.0f GB/s" % (ceiling["mib"], ceiling["gb_per_s"]))

    log("FP32 apply: %.1f s settle + %d warmup + %d timed" % (args.settle_s, args.warmup, args.steps))
    torch.cuda.synchronize()
    wall32, per32 = time_applies(stdg, torch, mh, dt, stdg.STDG_FP32, mode, x32, y32, args.steps, args.warmup,
                                 args.settle_s)
    dist32 = launch_distribution(stdg, torch, mh, dt, stdg.STDG_FP32, mode, x32, y32, args.dist_steps)
    log("FP64 apply: %.1f s settle + %d warmup + %d timed" % (args.settle_s, args.warmup, args.steps))
    wall64, per64 = time_applies(stdg, torch, mh, dt, stdg.STDG_FP64, mode, x64, y64, args.steps, args.warmup,
                                 args.settle_s)
    dist64 = launch_distribution(stdg, torch, mh, dt, stdg.STDG_FP64, mode, x64, y64, args.dist_steps)
    ms32 = wall32 * 1e3 / args.steps
    ms64 = wall64 * 1e3 / args.steps
    k32 = float(per32.mean())
    k64 = float(per64.mean())
    bytes32 = 12 * q * a ** 3 * 4 * ne
    bytes64 = 12 * q * a ** 3 * 8 * ne
    achieved = bytes32 / (k32 * 1e-3) / 1e9
    gdofs32 = trial_dof / (ms32 * 1e-3) / 1e9
    gdofs64 = trial_dof / (ms64 * 1e-3) / 1e9
    log("FP32 %.3f ms/apply (kernel %.3f ms), FP64 %.3f ms/apply (kernel %.3f ms)" % (ms32, k32, ms64, k64))

    solve = None
    if not args.no_solve:
        try:
            solve = time_solves(stdg, torch, mh, m, cfg, march=not args.no_march)
        except Exception as e:  # solver reported separately; the apply line still prints
            log("slab solve skipped: %s" % e)

    diss = None
    if not args.no_diss:
        log("dissipative stabilisation D_h, c = 1")
        diss = time_dissipative(stdg, torch, mh, cfg, args, (("fp32", stdg.STDG_FP32, x32, y32),
                                                            ("fp64", stdg.STDG_FP64, x64, y64)))

    reoriented = None
    if not args.no_reoriented:
        log("reoriented numbering of the same cavity")
        reoriented = time_reoriented(stdg, torch, ctx, mh, cfg, args, (("fp32", stdg.STDG_FP32, x32, y32),
                                                                      ("fp64", stdg.STDG_FP64, x64, y64)))

    local_time = None
    if not args.no_local_time:
        log("local time steps: two-material 32^3 cavity, 4/2/1 sub-intervals")
        local_time = time_local_time(stdg, torch, ctx, 20, 5, march=not args.no_march)

    graded = large = None
    if not args.no_graded:
        log("graded trilinear 24^3")
        graded = time_graded(stdg, torch, ctx, 20, 5)
    if not args.no_large:
        log("large cavity 48^3 p=6 q=4")
        large = time_large(stdg, torch, ctx, 10, 3)

    serving = None
    if args.serve_requests > 0:
        log("serving stream: %d requests" % args.serve_requests)
        serving = time_serving(stdg, ctx, args.serve_requests, args.serve_budget_gb, args.serve_max_active,
                               args.serve_krylov, graph=bool(args.serve_graph), batch=bool(args.serve_batch))
        log("serving: %.2f solves/s, p50 %.3f s, p99 %.3f s" % (serving["solves_per_s"], serving["p50_latency_s"],
                                                               serving["p99_latency_s"]))
        if args.serve_eta_rel > 0:
            log("serving stream, inexact solves")
            serving["inexact"] = time_serving(stdg, ctx, args.serve_requests, args.serve_budget_gb,
                                              args.serve_max_active, args.serve_krylov, args.serve_eta_rel,
                                              graph=bool(args.serve_graph), batch=bool(args.serve_batch))
            log("serving inexact: %.2f solves/s, p50 %.3f s, p99 %.3f s" % (
                serving["inexact"]["solves_per_s"], serving["inexact"]["p50_latency_s"],
                serving["inexact"]["p99_latency_s"]))

    cpu = None
    if not args.no_cpu_baseline:
        log("oracle CPU baseline on a bounded sample")
        cpu = cpu_baseline(cfg, args.cpu_sample)

    out = {
        "metric": "Residual GDoF/s at p=4,q=3 (FP32+refine vs FP64); slab solves/s, p99 latency",
        "value": round(gdofs32, 2),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "PEC cavity %d^3 affine hex, p=%d q=%d, eps 1|4 split at x=0.5, dt=%g; "
                               "preconditioned operator apply on N(0,1) coefficients (seed 0)"
                               % (args.n, args.p, args.q, dt),
                   "elements": ne, "trial_dof": trial_dof, "unknowns": nu,
                   "work_order": "Morton" if order == 0 else "columns of %d" % order,
                   "launch_variants": tuned["variants"]},
        "settle_s": args.settle_s,
        "launch_ms_fp32": dist32,
        "fp64": {"value": round(gdofs64, 2), "unit": "GDoF/s", "ms_per_step": round(ms64, 5),
                 "kernel_ms": round(k64, 5), "launch_ms": dist64,
                 "hbm_frac": round(bytes64 / (k64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "fp32_over_fp64": round(gdofs32 / gdofs64, 3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(1) if (args.n, args.p, args.q) == (32, 4, 3) else None,
                     "kernel": "residual_kernel<float,%d,%d,2,true,false,%d>" % (a, q, tuned["variants"][0]),
                     "kernel_ms": round(k32, 5), "algorithmic_bytes": bytes32,
                     "practical_peak": round(ceiling["gb_per_s"], 1),
                     "frac_practical": round(achieved / ceiling["gb_per_s"], 4),
                     "practical_peak_kernel": "stdg_stream_copy, %d MiB copied (read + write counted)"
                                              % ceiling["mib"]},
        "cpu_baseline": cpu,
    }
    if solve is not None:
        out["slab_solve"] = solve
    if diss is not None:
        out["dissipative"] = diss
    if reoriented is not None:
        out["reoriented"] = reoriented
    if local_time is not None:
        out["local_time_steps"] = local_time
    if graded is not None:
        out["graded_trilinear"] = graded
    if large is not None:
        out["large_cavity"] = large
    if serving is not None:
        out["serving"] = serving
    print(json.dumps(out), flush=True)
    stdg.stdg_mesh_free(mh)
    stdg.stdg_finalize(ctx)


def time_serving(stdg, ctx, n_requests, budget_gb, max_active, krylov, eta_rel=0.0, graph=False, batch=True):
    """The serving stream: independent PEC cavity solves (n^3, n in {4,..,16},
    p in 2..6, q = p - 1, eps in {1,2,4} per element, 20 slabs, dt = h/(2p+1))
    arriving as a Poisson process at 50 per second, submitted at their arrival
    times; FP32 applies inside FP64 refinement to rtol 1e-10 per slab."""
    import synth
    reqs = synth.serving_stream(n_requests=n_requests)
    dofs = [r["mesh"].trial_size() * r["n_slabs"] for r in reqs]
    srv = stdg.stdg_serve_start(ctx, hbm_budget=int(budget_gb * (1 << 30)), max_active=max_active,
                                inner_prec=stdg.STDG_FP32, rtol=1e-10, max_iters=3000, max_refine=300,
                                krylov_prec=stdg.STDG_FP32 if krylov == "fp32" else stdg.STDG_FP64,
                                eta_rel=eta_rel, use_graph=graph, batch_cycles=batch)
    results = {}
    try:
        c0 = stdg.stdg_serve_clock(srv)
        tickets = []
        k = 0
        last_log = 0.0
        while len(results) < len(reqs):
            now = stdg.stdg_serve_clock(srv) - c0
            while k < len(reqs) and reqs[k]["arrival"] <= now:
                m = reqs[k]["mesh"]
                tickets.append(stdg.stdg_serve_submit(srv, m.vertices, m.hexes, m.p, m.q, m.eps, m.mu, 0.0,
                                                      reqs[k]["dt"], reqs[k]["n_slabs"], mnl=reqs[k]["init"].mnl,
                                                      abc=reqs[k]["init"].abc))
                k += 1
            for i, t in enumerate(tickets):
                if i not in results:
                    r = stdg.stdg_serve_poll(srv, t)
                    if r is not None:
                        results[i] = r
            if now - last_log > 5.0:
                log("serving: %d submitted, %d done at %.1f s" % (k, len(results), now))
                last_log = now
            time.sleep(0.0005)
    finally:
        stdg.stdg_serve_stop(srv)
    res = [results[i] for i in range(len(reqs))]
    lat = np.array([r["t_done"] - r["t_submit"] for r in res])
    span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
    bad = [i for i, r in enumerate(res) if r["status"] != 0]
    return {"requests": len(res), "rate_per_s": 50.0, "slabs_per_request": reqs[0]["n_slabs"],
            "solves_per_s": round(len(res) / span, 3), "slab_solves_per_s": round(sum(r["slabs_done"] for r in res) / span, 2),
            "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
            "mean_latency_s": round(float(lat.mean()), 4), "span_s": round(span, 3),
            "gdof_per_s_trial_x_slabs": round(sum(dofs) / span / 1e9, 3),
            "iters_per_slab": round(sum(r["iters"] for r in res) / sum(r["slabs_done"] for r in res), 2),
            "max_rel_res": max(r["max_rel_res"] for r in res), "failed": bad,
            "hbm_budget_gb": budget_gb, "max_active": max_active, "krylov_basis": krylov, "graphs": bool(graph),
            "batch_cycles": bool(batch), "batched_cycles": int(sum(r["batched_cycles"] for r in res)),
            "requests_batched": int(sum(1 for r in res if r["batched_cycles"] > 0)),
            "stop": ("eta_it <= %g sqrt(2 E(0)) per request" % eta_rel) if eta_rel > 0 else "rtol 1e-10 per slab",
            "max_eta_it_rel": (max(r["eta_it"] / np.sqrt(2 * r["energy_start"]) for r in res if r["energy_start"] > 0)
                               if eta_rel > 0 else None),
            "max_energy_drift": max(abs(r["energy_end"] - r["energy_start"]) / max(r["energy_start"], 1e-300)
                                    for r in res)}


def _time_mode(stdg, torch, mh, dt, prec, mode, x, y, steps, warmup):
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        stdg.stdg_residual_apply(mh, dt, prec, mode, x, None, y, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        stdg.stdg_residual_apply(mh, dt, prec, mode, x, None, y, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _slab_with_source(stdg, torch, mh, info, cfg, inner, krylov):
    """One slab from a zero field driven by the workload's current, from the
    middle of its time window (load assembly included in the time)."""
    src = cfg["source"]
    t0 = src.t0 - cfg["dt"]
    state = torch.zeros(info["state_size"], dtype=torch.float64, device="cuda")
    load = torch.zeros(info["unknown_size"], dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t = time.perf_counter()
    stdg.stdg_load_assemble(mh, src, t0, cfg["dt"], load)
    r = stdg.stdg_slab_solve(mh, t0, cfg["dt"], load, state, inner_prec=inner, krylov_prec=krylov, rtol=1e-10,
                             max_iters=4000, max_refine=400)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    return {"s_per_slab": round(el, 4), "iters": r["iters"], "rel_res": r["rel_res"], "status": r["status"],
            "energy_end": r["energy_end"]}


def time_dissipative(stdg, torch, mh, cfg, args, vecs, c=1.0):
    """The headline workload with the dissipative stabilisation D_h switched on
    (c = 1): the preconditioned apply in both precisions next to the plain one
    (timed the same way, back to back), and one slab solve (FP32 applies with
    FP64 refinement, FP32 basis) from the projected modes with its energy loss."""
    a, q = args.p + 1, args.q
    ne = cfg["mesh"].n_elements
    trial = 6 * (q + 1) * a ** 3 * ne
    dt = cfg["dt"]
    mode = stdg.STDG_OPERATOR_PRECOND
    out = {"c": c}
    plain = {name: _time_mode(stdg, torch, mh, dt, prec, mode, x, y, args.steps, args.warmup)
             for name, prec, x, y in vecs}
    stdg.stdg_mesh_set_dissipation(mh, c)
    try:
        for name, prec, x, y in vecs:
            ms = _time_mode(stdg, torch, mh, dt, prec, mode, x, y, args.steps, args.warmup)
            sz = 4 if prec == stdg.STDG_FP32 else 8
            bytes_ = (12 * q * a ** 3 + 24) * sz * ne  # + the 24 face coefficients per element
            out[name] = {"apply_ms": round(ms, 5), "plain_apply_ms": round(plain[name], 5),
                         "over_plain": round(ms / plain[name], 3),
                         "gdof_per_s": round(trial / (ms * 1e-3) / 1e9, 2),
                         "hbm_frac": round(bytes_ / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "algorithmic_bytes": bytes_,
                         "traffic": measured_traffic(prec, "dissipative_")
                         if (args.n, args.p, args.q) == (32, 4, 3) else None}
            log("dissipative %s: apply %.3f ms (plain %.3f ms)" % (name, ms, plain[name]))
        info = stdg.stdg_mesh_info(mh)
        modes = cfg["init"]
        state = torch.zeros(info["state_size"], dtype=torch.float64, device="cuda")
        stdg.stdg_project_modes(mh, modes.mnl, modes.abc, state)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = stdg.stdg_slab_solve(mh, 0.0, dt, None, state, inner_prec=stdg.STDG_FP32, rtol=1e-10, max_iters=3000,
                                 max_refine=300, krylov_prec=stdg.STDG_FP32)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out["slab_fp32_refine_fp32_basis"] = {
            "s_per_solve": round(el, 4), "iters": r["iters"], "rel_res": r["rel_res"], "status": r["status"],
            "energy_loss_rel": (r["energy_start"] - r["energy_end"]) / max(r["energy_start"], 1e-300)}
        log("dissipative slab solve: %.3f s, %d iters" % (el, r["iters"]))
    finally:
        stdg.stdg_mesh_set_dissipation(mh, 0.0)
    return out


def time_reoriented(stdg, torch, ctx, mh, cfg, args, vecs):
    """The headline cavity with every element's vertices relabelled by a
    seeded random cube rotation: the same physical mesh whose neighbours meet
    in all eight face orientations.  The preconditioned apply (same input
    vector, which is a different field on this numbering) next to the
    canonical numbering, timed back to back."""
    import synth
    m = cfg["mesh"]
    hexes = synth.reorient(m.hexes, seed=0)
    a, q, ne = args.p + 1, args.q, m.n_elements
    trial = 6 * (q + 1) * a ** 3 * ne
    dt = cfg["dt"]
    mode = stdg.STDG_OPERATOR_PRECOND
    plain = {name: _time_mode(stdg, torch, mh, dt, prec, mode, x, y, args.steps, args.warmup)
             for name, prec, x, y in vecs}
    mr = stdg.stdg_mesh_upload(ctx, m.vertices, hexes, m.p, m.q, m.eps, m.mu)
    out = {"relabelled_elements": int((hexes != m.hexes).any(axis=1).sum()), "elements": ne}
    try:
        for name, prec, x, y in vecs:
            ms = _time_mode(stdg, torch, mr, dt, prec, mode, x, y, args.steps, args.warmup)
            out[name] = {"apply_ms": round(ms, 5), "canonical_apply_ms": round(plain[name], 5),
                         "over_canonical": round(ms / plain[name], 3),
                         "gdof_per_s": round(trial / (ms * 1e-3) / 1e9, 2)}
            log("reoriented %s: apply %.3f ms (canonical %.3f ms)" % (name, ms, plain[name]))
    finally:
        stdg.stdg_mesh_free(mr)
    return out


def time_graded(stdg, torch, ctx, steps, warmup):
    """Graded trilinear 24^3 mesh (p = 3..6 by ring, q = p - 2, interior
    vertices perturbed by 10% of h): the operator apply (quadrature mass) and
    one source-driven slab."""
    import synth
    cfg = synth.graded_nonaffine()
    m = cfg["mesh"]
    mh = stdg.stdg_mesh_upload(ctx, m.vertices, m.hexes, m.p, m.q, m.eps, m.mu)
    info = stdg.stdg_mesh_info(mh)
    a = m.p.astype(np.int64) + 1
    q = m.q.astype(np.int64)
    G = a + 1
    trial = int((6 * (q + 1) * a ** 3).sum())
    mass_qp = 2 * q * (3 * 2 * 2 * (a ** 3 * G + a ** 2 * G ** 2 + a * G ** 3) + 15 * G ** 3) + 80 * G ** 3
    flops = float((174 * q * a ** 3 + 24 * q * a ** 2 * (a ** 2 // 4) - 6 * q * a ** 3 + mass_qp).sum())
    out = {"workload": cfg["name"] + ", eps = mu = 1, dt = %g" % cfg["dt"], "elements": m.n_elements,
           "trial_dof": trial}
    nu = info["unknown_size"]
    x64 = torch.from_numpy(synth.random_vector(nu, 0)).cuda()
    for name, prec, x in (("fp32", stdg.STDG_FP32, x64.float()), ("fp64", stdg.STDG_FP64, x64)):
        y = torch.empty_like(x)
        ms = _time_mode(stdg, torch, mh, cfg["dt"], prec, stdg.STDG_OPERATOR, x, y, steps, warmup)
        ms_pre = _time_mode(stdg, torch, mh, cfg["dt"], prec, stdg.STDG_OPERATOR_PRECOND, x, y, steps, warmup)
        sz = 4 if prec == stdg.STDG_FP32 else 8
        bytes_ = float((12 * q * a ** 3).sum() * sz)
        peak_tf = 157.3 if prec == stdg.STDG_FP32 else 78.6
        out[name] = {"operator_ms": round(ms, 5), "gdof_per_s": round(trial / (ms * 1e-3) / 1e9, 2),
                     "precond_operator_ms": round(ms_pre, 5),
                     "hbm_frac": round(bytes_ / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "compute_frac": round(flops / (ms * 1e-3) / 1e12 / peak_tf, 4),
                     "algorithmic_bytes": bytes_, "algorithmic_flops": flops}
        log("graded %s: operator %.3f ms (%.1f GDoF/s)" % (name, ms, trial / (ms * 1e-3) / 1e9))
    out["slab_fp32_refine_fp32_basis"] = _slab_with_source(stdg, torch, mh, info, cfg, stdg.STDG_FP32, stdg.STDG_FP32)
    out["slab_fp64"] = _slab_with_source(stdg, torch, mh, info, cfg, stdg.STDG_FP64, stdg.STDG_FP64)
    stdg.stdg_mesh_free(mh)
    return out


def time_large(stdg, torch, ctx, steps, warmup):
    """48^3 affine cavity, p = 6, q = 4 (1.14e9 trial DoF), eps ~ U[1, 4]:
    the preconditioned operator apply and one source-driven slab."""
    import synth
    cfg = synth.large_cavity()
    m = cfg["mesh"]
    t = time.perf_counter()
    mh = stdg.stdg_mesh_upload(ctx, m.vertices, m.hexes, m.p, m.q, m.eps, m.mu)
    log("large: mesh upload %.1f s" % (time.perf_counter() - t))
    info = stdg.stdg_mesh_info(mh)
    a, q, ne = 7, 4, m.n_elements
    trial = 6 * (q + 1) * a ** 3 * ne
    out = {"workload": cfg["name"] + ", eps ~ U[1,4], dt = h/13", "elements": ne, "trial_dof": trial}
    nu = info["unknown_size"]
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    x64 = torch.randn(nu, dtype=torch.float64, device="cuda", generator=g)
    for name, prec, x in (("fp32", stdg.STDG_FP32, x64.float()), ("fp64", stdg.STDG_FP64, x64)):
        y = torch.empty_like(x)
        ms = _time_mode(stdg, torch, mh, cfg["dt"], prec, stdg.STDG_OPERATOR_PRECOND, x, y, steps, warmup)
        sz = 4 if prec == stdg.STDG_FP32 else 8
        bytes_ = 12 * q * a ** 3 * sz * ne
        out[name] = {"apply_ms": round(ms, 4), "gdof_per_s": round(trial / (ms * 1e-3) / 1e9, 2),
                     "hbm_frac": round(bytes_ / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        log("large %s: apply %.3f ms (%.1f GDoF/s)" % (name, ms, trial / (ms * 1e-3) / 1e9))
        del y
    del x64
    torch.cuda.empty_cache()
    out["slab_fp32_refine_fp32_basis"] = _slab_with_source(stdg, torch, mh, info, cfg, stdg.STDG_FP32, stdg.STDG_FP32)
    log("large: one slab %.2f s" % out["slab_fp32_refine_fp32_basis"]["s_per_slab"])
    stdg.stdg_mesh_free(mh)
    return out


def time_local_time(stdg, torch, ctx, steps, warmup, march=True):
    """Local time steps: the two-material 32^3 cavity (p = 4, q = 3) with 4 /
    2 / 1 sub-intervals per slab by region.  Operator and preconditioned
    applies (the rows of elements with sub-intervals and of their neighbours
    run in the local-time kernel, the rest in the kernel groups), the same
    mesh without sub-intervals for comparison, and a march of slabs with the
    energy drift (Thm 4.1: conserved without a source)."""
    import synth
    cfg = synth.local_time_cavity()
    m = cfg["mesh"]
    a = m.p.astype(np.int64) + 1
    nt = m.q.astype(np.int64) * m.nsub.astype(np.int64)
    out = {"workload": cfg["name"] + ", dt = %g" % cfg["dt"], "elements": m.n_elements,
           "sub_intervals": {str(k): int((m.nsub == k).sum()) for k in (1, 2, 4)},
           "trial_dof": int((6 * (nt + 1) * a ** 3).sum())}
    res = {}
    for label, nsub in (("local", m.nsub), ("uniform", None)):
        mh = stdg.stdg_mesh_upload(ctx, m.vertices, m.hexes, m.p, m.q, m.eps, m.mu, nsub)
        info = stdg.stdg_mesh_info(mh)
        x64 = torch.from_numpy(synth.random_vector(info["unknown_size"], 0)).cuda()
        lev = nt if nsub is not None else m.q.astype(np.int64)
        for name, prec, x in (("fp32", stdg.STDG_FP32, x64.float()), ("fp64", stdg.STDG_FP64, x64)):
            y = torch.empty_like(x)
            ms = _time_mode(stdg, torch, mh, cfg["dt"], prec, stdg.STDG_OPERATOR, x, y, steps, warmup)
            ms_pre = _time_mode(stdg, torch, mh, cfg["dt"], prec, stdg.STDG_OPERATOR_PRECOND, x, y, steps, warmup)
            sz = 4 if prec == stdg.STDG_FP32 else 8
            bytes_ = float((12 * lev * a ** 3).sum() * sz)
            trial = float((6 * (lev + 1) * a ** 3).sum())
            res.setdefault(label, {})[name] = {
                "operator_ms": round(ms, 4), "precond_operator_ms": round(ms_pre, 4),
                "gdof_per_s": round(trial / (ms * 1e-3) / 1e9, 2),
                "hbm_frac": round(bytes_ / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "algorithmic_bytes": bytes_}
            log("local time (%s) %s: operator %.3f ms, preconditioned %.3f ms" % (label, name, ms, ms_pre))
        if nsub is not None and march:
            out["march_fp32_refine"] = _march(stdg, torch, mh, cfg, info, cfg["n_slabs"],
                                              inner_prec=stdg.STDG_FP32, krylov_prec=stdg.STDG_FP32, rtol=1e-10,
                                              max_iters=3000, max_refine=300, use_graph=1)
            log("local time march: %.2f slab solves/s, drift %.2e" % (
                out["march_fp32_refine"]["slab_solves_per_s"], out["march_fp32_refine"]["energy_drift"]))
        stdg.stdg_mesh_free(mh)
    out.update(res)
    return out


def _march(stdg, torch, mh, cfg, info, n_slabs, **opts):
    """The workload's march of n_slabs slabs from the projected modes; wall
    time, iterations and the energy drift (Thm 3.1: conserved without a
    source)."""
    modes = cfg["init"]
    state = torch.zeros(info["state_size"], dtype=torch.float64, device="cuda")
    stdg.stdg_project_modes(mh, modes.mnl, modes.abc, state)
    e0 = stdg.stdg_energy(mh, state)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, eta2, worst = 0, 0.0, 0.0
    for n in range(n_slabs):
        r = stdg.stdg_slab_solve(mh, n * cfg["dt"], cfg["dt"], None, state, **opts)
        iters += r["iters"]
        eta2 += r["eta2"]
        worst = max(worst, r["rel_res"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"s": round(el, 3), "slab_solves_per_s": round(n_slabs / el, 2), "iters_per_slab": round(iters / n_slabs, 2),
            "max_rel_res": worst, "energy_drift": (r["energy_end"] - e0) / e0, "eta2": eta2, "e0": e0}


def time_solves(stdg, torch, mh, m, cfg, march=True):
    """FP32-apply + FP64 refinement vs plain FP64: one slab from the projected
    mode superposition to rtol 1e-10 (whole restart cycles replayed as
    graphs), and the workload's 64-slab march in both paths."""
    info = stdg.stdg_mesh_info(mh)
    modes = cfg["init"]
    res = {}
    paths = (("fp32_refine", stdg.STDG_FP32, stdg.STDG_FP32), ("fp32_refine_fp64_basis", stdg.STDG_FP32, stdg.STDG_FP64),
             ("fp64", stdg.STDG_FP64, stdg.STDG_FP64))
    for name, inner, krylov in paths:
        # the first solve of a path allocates its solver and captures its graph: untimed
        for rep in range(2):
            state = torch.zeros(info["state_size"], dtype=torch.float64, device="cuda")
            stdg.stdg_project_modes(mh, modes.mnl, modes.abc, state)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = stdg.stdg_slab_solve(mh, 0.0, cfg["dt"], None, state, inner_prec=inner, rtol=1e-10,
                                     max_iters=3000, max_refine=300, krylov_prec=krylov, use_graph=1)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
        res[name] = {"s_per_solve": round(el, 4), "solves_per_s": round(1.0 / el, 3), "iters": r["iters"],
                     "refinements": r["refinements"], "rel_res": r["rel_res"],
                     "energy_drift": (r["energy_end"] - r["energy_start"]) / max(r["energy_start"], 1e-300)}
        log("slab solve %s: %.3f s, %d iters" % (name, el, r["iters"]))
    res["speedup_fp32_refine"] = round(res["fp64"]["s_per_solve"] / res["fp32_refine"]["s_per_solve"], 3)
    res["speedup_fp32_refine_fp64_basis"] = round(
        res["fp64"]["s_per_solve"] / res["fp32_refine_fp64_basis"]["s_per_solve"], 3)
    n_slabs = cfg["n_slabs"]
    if march:
        # metric 2 of the workload: its 64 slabs solved exactly (rtol 1e-10 per slab) in both paths
        for name, inner, krylov in (paths[0], paths[2]):
            mr = _march(stdg, torch, mh, cfg, info, n_slabs, inner_prec=inner, krylov_prec=krylov, rtol=1e-10,
                        max_iters=3000, max_refine=300, use_graph=1)
            mr.pop("eta2")
            mr.pop("e0")
            res["march_%d_slabs_%s" % (n_slabs, name)] = mr
            log("%d-slab march %s: %.2f s (%.1f slab solves/s)" % (n_slabs, name, mr["s"], mr["slab_solves_per_s"]))
        res["march_speedup_fp32_refine"] = round(res["march_%d_slabs_fp64" % n_slabs]["s"] /
                                                 res["march_%d_slabs_fp32_refine" % n_slabs]["s"], 3)
    # inexact solve (Section 5.3): stop at the iteration-error bound, with a
    # budget of eta_it <= 1e-3 sqrt(2 E(0)) over the workload's 64 slabs
    state = torch.zeros(info["state_size"], dtype=torch.float64, device="cuda")
    stdg.stdg_project_modes(mh, modes.mnl, modes.abc, state)
    e0 = stdg.stdg_energy(mh, state)
    eta_tol = 1e-3 * np.sqrt(2.0 * e0) / np.sqrt(n_slabs)
    opts = dict(inner_prec=stdg.STDG_FP32, rtol=1e-10, max_iters=3000, max_refine=300, krylov_prec=stdg.STDG_FP32,
                eta_tol=eta_tol, eta_t_final=n_slabs * cfg["dt"], use_graph=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = stdg.stdg_slab_solve(mh, 0.0, cfg["dt"], None, state, **opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res["inexact_fp32_refine"] = {"s_per_solve": round(el, 4), "solves_per_s": round(1.0 / el, 3),
                                  "iters": r["iters"], "eta_it_term": float(np.sqrt(r["eta2"])),
                                  "eta_tol": float(eta_tol), "rel_res": r["rel_res"]}
    log("slab solve inexact: %.3f s, %d iters" % (el, r["iters"]))
    if march:
        mr = _march(stdg, torch, mh, cfg, info, n_slabs, **opts)
        mr["eta_it_rel"] = float(np.sqrt(mr.pop("eta2")) / np.sqrt(2.0 * mr.pop("e0")))
        res["march_%d_slabs_inexact" % n_slabs] = mr
        log("%d-slab inexact march: %.2f s (%.1f slab solves/s)" % (n_slabs, mr["s"], mr["slab_solves_per_s"]))
    return res


if __name__ == "__main__":
    main()
