#!/usr/bin/env python3
"""Throughput of the fused collide-and-stream step on one MI355X.

Workload (the bandwidth sweep of the coupled DDF model): a fully periodic
8192 x 8192 D2Q9 grid, total-energy form with viscous heating and the
correction term, tau_f = 0.8, Pr = 0.71, b = 3, seeded Gaussian perturbations
(sigma = 1e-3) of rho, u and T.  One step = one fused launch over every node
(gather 18 populations, moments, correction term, MRT f, BGK h with coupling,
store 18 populations).  value = MLUPS (million node updates per second) with
FP32 population storage; the 16-bit storage run and the smaller grids are
reported beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_NODE = {"f32": 144, "f16": 72, "bf16": 72}  # 18 loads + 18 stores per node-update


def kernel_source_hash() -> str:
    """Hash of the device code (everything above the host-side section of
    lbddf.hip): a profile stays valid while the kernels are unchanged."""
    with open(os.path.join(ROOT, "paper_1109_6672_amd", "csrc", "lbddf.hip"), "rb") as fh:
        src = fh.read()
    cut = src.find(b"// ------------------------------------------------------------- host side")
    return hashlib.sha256(src if cut < 0 else src[:cut]).hexdigest()[:16]


def measured_traffic(key: str, nodes: int):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it was
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(key)
    if not e or e.get("kernel_source_sha") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def bounded_case(kind: str, storage: str):
    """The bounded configurations: the large-dT cavity at 512^2 and 2048^2
    (walls on all sides, Sutherland viscosity) and the acoustic channel
    2048 x 256 (inlet, outlet, periodic in y)."""
    from paper_1109_6672_amd import workloads as W

    if kind in ("cavity512", "cavity2048"):
        p = W.cavity(int(kind[6:]), 1e5, 1.2, 0.06, sutherland=True, storage=storage)
        p.update(s_e=1.5, s_zeta=1.5)
        return p, W.conduction_fields(p)
    p = W.channel(2048, 256, U0=0.01, period=200.0, storage=storage)
    return p, W.rest_fields(p)


def time_gpu(n: int, storage: str, steps: int, warmup: int, strip_rows: int = 0, case=None, arith: str = "f32"):
    import torch

    from paper_1109_6672_amd import lbddf, workloads as W

    if case is None:
        p = W.periodic(n, storage=storage)
        fields = W.gaussian_fields(p, sigma=1e-3)
    else:
        p, fields = bounded_case(case, storage)
    n_nodes = p["nx"] * p["ny"]
    s = lbddf.Solver(p, device=0, arith=arith)
    s.init(*fields)
    del fields
    if strip_rows:
        s.set_strip_rows(strip_rows)
    s.step(warmup)
    stream = s.stream
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    s.step(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    d = s.diag(check=False)
    nodes = n_nodes
    out = dict(n=n if case is None else f"{p['nx']}x{p['ny']}", storage=storage, steps=steps, ms_total=ms, ms_per_step=ms / steps, wall_s=wall,
               mlups=nodes * steps / (ms * 1e-3) / 1e6, strip_rows=s.strip_rows, bad_nodes=d["bad"])
    out["gbs"] = BYTES_PER_NODE[storage] * nodes / (out["ms_per_step"] * 1e-3) / 1e9
    s.close()
    del s
    torch.cuda.empty_cache()
    return out


def copy_bandwidth(reps: int = 5, probe: bool = True):
    """A plain device copy of 2 GiB timed with HIP events: with probe, the
    library's STREAM-like copy (lb_copy_probe), the practical memory ceiling
    beside the nominal 8 TB/s; else torch's copy, the calibration run of the
    FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    from paper_1109_6672_amd import lbddf

    x = torch.empty(1 << 29, dtype=torch.float32, device="cuda")
    x.fill_(1.0)
    y = torch.empty_like(x)
    run = (lambda: lbddf.copy_probe(x, y)) if probe else (lambda: y.copy_(x))
    run()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(reps):
        run()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    if probe and not torch.equal(x, y):
        raise RuntimeError("copy probe: destination differs from the source")
    out = {"copy_kernel": "lb_copy_probe" if probe else "torch copy_", "copy_bytes_read": x.numel() * 4,
           "copy_bytes_written": x.numel() * 4, "copy_GBs": 2 * x.numel() * 4 / (ms * 1e-3) / 1e9}
    del x, y
    torch.cuda.empty_cache()
    return out


def _cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            return next(line.split(":", 1)[1].strip() for line in fh if line.startswith("model name"))
    except (OSError, StopIteration):
        return "unknown"


def _oracle_mlups(p, fields, seconds, chunk):
    """Oracle MLUPS on one workload: steps in chunks until `seconds` pass
    (initialisation and a first chunk excluded)."""
    from oracle import oracle as O

    o = O.Oracle(p).init(*fields)
    o.step(chunk)
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        o.step(chunk)
        steps += chunk
    t = time.perf_counter() - t0
    o.close()
    return p["nx"] * p["ny"] * steps / t / 1e6, steps, t


def cpu_baseline(seconds: float):
    """The FP64 oracle as it stands on the host cores: the headline recipe on
    a bounded sample (periodic 512 x 512) with all cores and with one thread,
    then short samples of the Couette, small-dT cavity, large-dT 64^2 cavity
    and acoustic-channel workloads (the oracle runs grids below 8192 nodes on
    one thread)."""
    from oracle import oracle as O
    from paper_1109_6672_amd import workloads as W

    # the host's CPU share: OMP_NUM_THREADS when set, else the cores this
    # process may run on
    want = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0)) or 1
    O.set_threads(want)
    cores = O.threads()
    p = W.periodic(512)
    f = W.gaussian_fields(p, sigma=1e-3)
    all_cores, steps, t = _oracle_mlups(p, f, 0.4 * seconds, 2)
    O.set_threads(1)
    one, steps1, t1 = _oracle_mlups(p, f, 0.2 * seconds, 1)
    samples = [dict(workload="periodic 512x512, headline recipe", threads=cores, mlups=all_cores),
               dict(workload="periodic 512x512, headline recipe", threads=1, mlups=one)]
    O.set_threads(cores)
    extra = [("Couette 4x64 (config 1)", W.couette(), W.rest_fields, 2000),
             ("small-dT cavity 128x128 (config 2)", W.cavity(128, 1e4, 0.02, 0.02), W.noisy_temperature_fields, 20),
             ("large-dT cavity 64x64 (config 3 downscale)", W.cavity(64, 1e5, 1.2, 0.06, sutherland=True),
              W.conduction_fields, 50),
             ("acoustic channel 2048x256 (config 4b)", W.channel(), W.rest_fields, 2)]
    for name, q, make, chunk in extra:
        m, _, _ = _oracle_mlups(q, make(q), 0.1 * seconds, chunk)
        samples.append(dict(workload=name, threads=cores if q["nx"] * q["ny"] >= 8192 else 1, mlups=m))
    return dict(value=all_cores, unit="MLUPS", cores=cores, kind="oracle",
                sample=f"periodic 512x512, same recipe as the headline, {steps} steps in {t:.1f} s on {cores} "
                       f"threads (FP64, OpenMP over rows); single thread {one:.2f} MLUPS ({steps1} steps in "
                       f"{t1:.1f} s)", single_thread=one, samples=samples, cpu=_cpu_model())


def serving_compare(n_requests: int = 24, sizes=(64, 128, 256), k_steps: int = 1000, tol: float = 1e-8,
                    cap: int = 100_000, modes=("packed", "f16", "seq"), progress: float = 0.0):
    """The continuous-batching server against one solve per launch, on the
    same seeded stream of cavity requests (Poisson arrivals, 50 per second).
    modes picks the runs: packed (FP32), f16 (packed, FP16 storage), seq (one
    solve per launch, FP32)."""
    from paper_1109_6672_amd import lbddf, serving as SV, workloads as W

    keep = ("p50_s", "p99_s", "converged_p50_s", "converged_p99_s", "solves_per_s", "mlups", "wall_s", "states",
            "median_steps", "states_by_edge")
    out = {
        "workload": f"{n_requests} differentially heated cavity requests, edges {'/'.join(map(str, sizes))}, "
                    "Poisson arrivals 50/s, Ra log-uniform 1e3..1e6, dT/T0 uniform 0.02..1.2, FP32, "
                    f"residual = relative change of T over {k_steps} steps, tol {tol:g}, plateau test, "
                    f"cap {cap} steps; one at a time = lb_step (graph replays) and one residual per check",
    }
    reqs = W.serving_mix(n_requests, sizes=sizes, rate=50.0)
    if "packed" in modes:
        pool = lbddf.load().lbs_pool_overhead() + sum(lbddf.state_bytes(r["params"]) + 256 for r in reqs)
        packed, srv, _ = SV.run_server(reqs, pool, k_steps=k_steps, tol=tol, max_steps=cap, progress=progress)
        srv.close()
        out["packed"] = {k: packed[k] for k in keep}
    if "f16" in modes:
        reqs16 = W.serving_mix(n_requests, sizes=sizes, rate=50.0, storage="f16")
        pool16 = lbddf.load().lbs_pool_overhead() + sum(lbddf.state_bytes(r["params"]) + 256 for r in reqs16)
        packed16, srv, _ = SV.run_server(reqs16, pool16, storage="f16", k_steps=k_steps, tol=tol, max_steps=cap,
                                         progress=progress)
        srv.close()
        del reqs16
        out["packed_f16_storage"] = {k: packed16[k] for k in keep}
    if "seq" in modes:
        seq = SV.run_sequential(reqs, k_steps=k_steps, tol=tol, max_steps=cap, progress=progress)
        out["one_at_a_time"] = {k: seq[k] for k in keep}
    if "packed" in out and "one_at_a_time" in out:
        out["solves_per_s_ratio"] = out["packed"]["solves_per_s"] / out["one_at_a_time"]["solves_per_s"]
        out["p99_ratio"] = out["one_at_a_time"]["p99_s"] / out["packed"]["p99_s"]
    return out


def pmc_summary(run_dir: str, n: int = 8192) -> dict:
    """HBM bytes per launch of the headline step from rocprofv3 PMC runs under
    run_dir ({f32,f16}fetch and {f32,f16}write with FETCH_SIZE / WRITE_SIZE,
    the FP16 pair optional; cfetch and cwrite on --copy-only, whose k_copy
    dispatches each copy 2 GiB).  The scales come from the copy: bytes it
    moved over the KiB each counter reports for it.  Returns the entries of
    profiles/traffic.json for the current device code."""
    import csv

    def values(sub, counter, match):
        with open(os.path.join(run_dir, sub, "c_counter_collection.csv")) as fh:
            return [float(r["Counter_Value"]) for r in csv.DictReader(fh)
                    if r["Counter_Name"] == counter and match(r["Kernel_Name"])]

    def mean(v):
        if not v:
            raise ValueError("no matching dispatches")
        return sum(v) / len(v)

    copy = lambda k: "k_copy" in k  # the library's copy probe: every dispatch copies 2 GiB
    copied_kib = 2 * 2**30 / 1024
    fetch_scale = round(copied_kib / mean(values("cfetch", "FETCH_SIZE", copy)), 2)
    write_scale = round(copied_kib / mean(values("cwrite", "WRITE_SIZE", copy)), 2)
    sha, out = kernel_source_hash(), {}
    for st, code in (("f32", 0), ("f16", 1)):
        if st != "f32" and not os.path.isdir(os.path.join(run_dir, f"{st}fetch")):
            continue  # the FP16 runs are optional
        step = lambda k, code=code: f"k_step<{code}, false" in k
        f = mean(values(f"{st}fetch", "FETCH_SIZE", step))
        w = mean(values(f"{st}write", "WRITE_SIZE", step))
        out[f"lb_step_periodic{n}_{st}"] = dict(
            kernel=f"k_step<{st.upper()}, periodic> (void (anonymous namespace)::k_step<{code}, false, "
                   "(anonymous namespace)::Head>)",
            kernel_source_sha=sha, fetch_kib_per_launch_raw=round(f, 1), write_kib_per_launch_raw=round(w, 1),
            fetch_scale=fetch_scale, write_scale=write_scale,
            bytes_per_launch=int(round(1024 * (f * fetch_scale + w * write_scale))),
            algorithmic_bytes_per_launch=BYTES_PER_NODE[st] * n * n,
            source=f"profiles/lb_step_periodic{n}_{st}.md")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=8192, help="grid edge of the headline workload")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the 16-bit and smaller-grid runs")
    ap.add_argument("--no-serving", action="store_true", help="skip the packed-server comparison")
    ap.add_argument("--serving-requests", type=int, default=16, help="requests in the serving mix")
    ap.add_argument("--serving-sizes", default="64,128", help="grid edges of the serving mix")
    ap.add_argument("--serving-only", action="store_true",
                    help="only the serving comparison, with progress lines on stderr")
    ap.add_argument("--serving-modes", default="packed,f16,seq",
                    help="runs of the serving comparison: packed, f16, seq (one solve per launch)")
    ap.add_argument("--serving-cap", type=int, default=400_000, help="step cap per request")
    ap.add_argument("--serving-k", type=int, default=1000,
                    help="steps per batch and between residual checks (the residual is the change over them)")
    ap.add_argument("--only", default="", help="storage of a single run (profiling): f32 | f16 | bf16")
    ap.add_argument("--workload", default="periodic",
                    help="workload of an --only run: periodic (n x n) | cavity512 | cavity2048 | channel2048x256")
    ap.add_argument("--copy-only", action="store_true",
                    help="HBM counter calibration and copy ceiling: the library's copy probe over 2 GiB")
    ap.add_argument("--pmc-summary", metavar="DIR", default="",
                    help="no GPU: write profiles/traffic.json from the rocprofv3 PMC runs under DIR")
    args = ap.parse_args()
    if args.pmc_summary:
        t = pmc_summary(args.pmc_summary, args.n)
        with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
            json.dump(t, fh, indent=2)
            fh.write("\n")
        print(json.dumps(t, indent=2))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU halo-exchange design is described, not built).", file=sys.stderr)
        sys.exit(2)

    if args.copy_only:
        print(json.dumps(copy_bandwidth()), flush=True)
        return

    if args.serving_only:
        print(json.dumps(serving_compare(args.serving_requests,
                                         tuple(int(v) for v in args.serving_sizes.split(",")),
                                         k_steps=args.serving_k,
                                         cap=args.serving_cap, modes=tuple(args.serving_modes.split(",")),
                                         progress=20.0)), flush=True)
        return

    if args.only:
        case = None if args.workload == "periodic" else args.workload
        r = time_gpu(args.n, args.only, args.steps, args.warmup, case=case)
        print(json.dumps(r), flush=True)
        return

    head = time_gpu(args.n, "f32", args.steps, args.warmup)
    print(f"# f32 {args.n}^2: {head['mlups']:.0f} MLUPS, {head['gbs']:.0f} GB/s algorithmic", file=sys.stderr,
          flush=True)
    extra = {}
    if not args.no_extra:
        for storage, n in (("f16", args.n), ("bf16", args.n), ("f32", 4096), ("f16", 4096), ("f32", 1024)):
            if n > args.n:
                continue
            r = time_gpu(n, storage, args.steps, args.warmup)
            extra[f"{storage}_{n}"] = {k: r[k] for k in ("mlups", "gbs", "ms_per_step", "strip_rows")}
            print(f"# {storage} {n}^2: {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        # the library with the step's arithmetic in FP64 (FP32 storage)
        r = time_gpu(args.n, "f32", args.steps, args.warmup, arith="f64")
        extra[f"f32_{args.n}_fp64_arith"] = {k: r[k] for k in ("mlups", "gbs", "ms_per_step", "strip_rows")}
        print(f"# f32 storage, FP64 arithmetic {args.n}^2: {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        # the bounded grids take ~20 us per step: time whole graph batches
        # (2048 steps, 64 replays of 32) after as many warm-up steps
        for case, storage in (("cavity512", "f32"), ("cavity512", "f16"), ("channel2048x256", "f32"),
                              ("cavity2048", "f32")):
            steps = max(args.steps, 2048) if case != "cavity2048" else max(args.steps, 256)
            r = time_gpu(0, storage, steps, max(args.warmup, 64), case=case)
            extra[f"{storage}_{case}"] = {k: r[k] for k in ("mlups", "gbs", "ms_per_step", "strip_rows")}
            print(f"# {storage} {case}: {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    nodes = args.n * args.n
    alg = BYTES_PER_NODE["f32"] * nodes
    achieved = alg / (head["ms_per_step"] * 1e-3) / 1e9
    traffic = measured_traffic(f"lb_step_periodic{args.n}_f32", nodes)
    copy = copy_bandwidth()
    line = {
        "metric": "MLUPS (FP32 storage) + % HBM roofline",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"coupled DDF D2Q9, periodic {args.n}x{args.n}, Gaussian sigma=1e-3 on rho,u,T, "
                               "total energy + heating + correction, MRT, FP32 storage",
                   "nodes": nodes, "strip_rows": head["strip_rows"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "bytes_per_node": BYTES_PER_NODE["f32"], "kernel": "k_step<F32, periodic>",
                     "copy_GBs": round(copy["copy_GBs"], 1), "frac_of_copy": round(achieved / copy["copy_GBs"], 4)},
        "extra": extra,
        "bad_nodes": head["bad_nodes"],
    }
    if not args.no_serving:
        line["serving"] = serving_compare(args.serving_requests,
                                          tuple(int(v) for v in args.serving_sizes.split(",")),
                                          cap=args.serving_cap)
        print(f"# serving: {line['serving']['packed']['solves_per_s']:.1f} solves/s packed, "
              f"{line['serving']['one_at_a_time']['solves_per_s']:.1f} one at a time", file=sys.stderr, flush=True)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
