"""Throughput of the batched IPC Newton step on one MI355X.

Workload (default): 256 grasp environments stepped together in every launch --
soft superquadric objects (tet count lognormal, median 5k, clipped to
[1k, 20k]) squeezed by a two-slab soft gripper, dt = 0.01 s, dhat = 1e-3 m,
100-step horizon (closing 60 steps, then lifting 40).  A bench "step" is one
time step of every environment (the timed steps are one ipc_step_batch call);
the metric is converged environment-steps per second.  Inputs are seeded synthetic scenes shaped like the paper's grasp
validations (Sec. III-D); they are resident in device memory before timing.

The same scenes are run with FP64 PCG and with mixed precision (FP32 PCG
matrix/vectors, FP64 dot products; everything else FP64).  `value` is the
mixed-precision throughput; the FP64 figure is reported beside it.  The
paper's speedup notion (N environments batched vs the same N run one after
another, Sec. IV-A) is reported as context from a sequential single-environment
run on the same GPU.

Serving (`serving` object): a bounded sample of the request stream -- sphere
grasps (tet count lognormal, median 10k, clipped to [2k, 50k], 100 steps each)
arriving as a Poisson process at 50 requests/s -- submitted at their arrival
times to the library's continuous-batching server (200 GB budget, slot cap
tuned by the server), mixed precision; p50/p99 latency is completion time
minus arrival time, throughput is converged steps over the span from the first
arrival to the last completion.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

# At least five hardware queues for this process (read by the HIP runtime
# when it starts, so before any GPU call): four library lanes plus the null
# stream; the library's lane count defaults to the queues minus one, at most 4.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 5:
    os.environ["GPU_MAX_HW_QUEUES"] = "5"

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2503_05020_amd import ipc as G  # noqa: E402
from paper_2503_05020_amd import scenes as S  # noqa: E402

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_scene(workload: str, i: int):
    if workload == "superquadric_batch":
        return S.superquadric_grasp(i)
    if workload == "sphere_grasp":
        return S.parallel_jaw_sphere(seed=i)
    if workload == "cube_drop":
        return S.soft_cube_drop(seed=i)
    raise SystemExit(f"unknown workload {workload}")


def make_scenes(workload: str, n_envs: int):
    return [make_scene(workload, i) for i in range(n_envs)]


def run_gpu(scs, precision, warmup, steps, pcg_tol, label, count_all=False, autotune=None, **overrides):
    import torch
    t0 = time.time()
    gs = [G.ipc_create_scene(sc, precision=precision, pcg_rel_tol=pcg_tol, **overrides) for sc in scs]
    log(f"[{label}] created {len(gs)} scenes in {time.time() - t0:.1f}s")
    for k in range(warmup):
        rc, infos = G.ipc_step_batch(gs, 1)
        log(f"[{label}] warmup step {k}: newton(max)={max(i['max_newton_iters'] for i in infos)}")
    if autotune:
        # per-workload choice of the scheduling knobs (untimed; changes no result)
        t1 = time.time()
        log(f"[{label}] autotune: {G.ipc_autotune(gs, 3, autotune)} in {time.time() - t1:.1f}s")
    torch.cuda.synchronize()
    if not count_all:
        G.ipc_prof_reset()
    # the timed steps in one call: each lane of the library then runs through
    # them at its own pace instead of waiting for the slowest lane every step
    t0 = time.perf_counter()
    rc, infos = G.ipc_step_batch(gs, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    converged = sum(i["steps_done"] for i in infos)
    newton = sum(i["newton_iters"] for i in infos)
    pcg = sum(i["pcg_iters"] for i in infos)
    log(f"[{label}] {steps} timed steps: converged {converged}/{len(gs) * steps} env-steps")
    prof = G.ipc_prof_read()
    pairs = G.ipc_prof_pairs()
    failed = sum(1 for g in gs if G.ipc_scene_sizes(g)[6])
    for g in gs:
        G.ipc_destroy_scene(g)
    return dict(wall=wall, converged=converged, newton=newton, pcg=pcg, prof=prof, pairs=pairs, failed=failed,
                value=converged / wall, ms_per_step=1e3 * wall / steps)


def contact_rates(r):
    """Contact work per second of the timed window (all lanes): candidate pairs classified and barrier /
    friction elements evaluated (gradient + projected Hessian) by the assembly passes."""
    w = r["wall"]
    p = r["pairs"]
    return {"candidates_classified_per_s": round(p["candidates"] / w), "barrier_elems_per_s": round(p["barrier_elems"] / w),
            "friction_elems_per_s": round(p["friction_elems"] / w),
            "contact_pair_evals_per_s": round((p["barrier_elems"] + p["friction_elems"]) / w)}


def sequential_gpu(scs, precision, warmup, steps, pcg_tol, n):
    """The same environments run one after another (the paper's baseline for its speedup)."""
    done = 0
    wall = 0.0
    for sc in scs[:n]:
        g = G.ipc_create_scene(sc, precision=precision, pcg_rel_tol=pcg_tol)
        G.ipc_step(g, warmup)
        t0 = time.perf_counter()
        rc, info = G.ipc_step(g, steps)
        wall += time.perf_counter() - t0
        done += info["steps_done"]
        G.ipc_destroy_scene(g)
    return dict(value=done / wall, envs=n)


def _oracle_worker(args):
    """One host process: the oracle on environments envs, each stepped `warmup` steps untimed and then
    through the timed window (at most `steps` steps) until `budget_s` of timed stepping is spent."""
    workload, n_envs, envs, warmup, steps, budget_s = args
    import oracle as O
    done, timed = 0, 0.0
    used = []
    for e in envs:
        if timed >= budget_s:
            break
        o = O.Scene(make_scene(workload, e), pcg_rel_tol=1e-4)
        rc, _ = o.step(warmup)
        if rc != 0:
            continue
        used.append(e)
        for _ in range(steps):
            t0 = time.perf_counter()
            rc, _ = o.step(1)
            timed += time.perf_counter() - t0
            if rc != 0:
                break
            done += 1
            if timed >= budget_s:
                break
    return done, timed, used


def cpu_baseline(workload, n_envs, warmup, steps, budget_s=15.0):
    """The oracle (single-threaded per environment, FP64, PCG tolerance 1e-4 as the GPU run) timed on the
    host cores: one process per core, each taking environments spread over the whole batch, every
    environment stepped to the GPU's first timed step untimed and then timed through the GPU's window;
    throughput = timed converged env-steps over the timed seconds per process, summed over processes."""
    import multiprocessing as mp
    import platform
    import subprocess
    ncpu = os.cpu_count() or 1
    try:
        aff = len(os.sched_getaffinity(0))
    except AttributeError:
        aff = ncpu
    procs = max(1, min(16, aff))
    stride = max(1, n_envs // (procs * 4))
    order = list(range(0, n_envs, stride))
    jobs = [(workload, n_envs, order[k::procs], warmup, steps, budget_s) for k in range(procs)]
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_oracle_worker, jobs)
    per_proc = [d / t for d, t, _ in res if t > 0]
    done = sum(d for d, _, _ in res)
    envs = sorted(e for _, _, u in res for e in u)
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        model = next((ln.split(":", 1)[1].strip() for ln in out.splitlines() if ln.startswith("Model name")), "")
    except Exception:
        pass
    return dict(value=round(sum(per_proc), 3), unit="converged env-steps/s", cores=procs, kind="oracle",
                single_core=round(sum(d for d, _, _ in res) / max(1e-9, sum(t for _, t, _ in res)), 3),
                nproc=ncpu, cpus_allowed=aff, lscpu_model=model or platform.processor(),
                sample=f"{done} timed env-steps of {len(envs)} environments spread over the batch "
                       f"({envs[:6]}...), each from step {warmup} (untimed before) through at most {steps} steps, "
                       f"{procs} processes of one thread, about {budget_s:.0f} s of timed stepping each")


def serving(n_req, rate, budget, slots, precision, n_steps=100):
    reqs = S.serving_requests(n_req, rate=rate, seed=1)
    scs = [S.serving_scene(r) for r in reqs]
    log(f"[serving] {n_req} requests, {sum(len(sc['tets']) for sc in scs)} tets in total")
    srv = G.ipc_server_create(budget, slots)
    try:
        t0 = time.perf_counter()
        ids = []
        for r, sc in zip(reqs, scs):
            dt = t0 + r["arrival"] - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            ids.append(G.ipc_server_submit(srv, sc, n_steps, precision))
        infos = []
        for k, i in enumerate(ids):
            infos.append(G.ipc_server_wait(srv, i, 3600.0))
            if k % 8 == 7:
                st = G.ipc_server_stats(srv)
                log(f"[serving] {k + 1} done, running {st['running']:.0f}, queued {st['queued']:.0f}, "
                    f"cap {st['slot_cap']:.0f}")
        st = G.ipc_server_stats(srv)
    finally:
        G.ipc_server_destroy(srv)
    lat = sorted(i["t_done"] - i["t_submit"] for i in infos)
    span = max(i["t_done"] for i in infos) - min(i["t_submit"] for i in infos)
    steps = sum(i["steps_done"] for i in infos)

    def pct(q):
        return lat[min(len(lat) - 1, int(round(q * (len(lat) - 1))))]
    return {"requests": n_req, "arrival_rate_per_s": rate, "steps_per_request": n_steps,
            "p50_latency_s": round(pct(0.5), 3), "p99_latency_s": round(pct(0.99), 3),
            "converged_steps_per_s": round(steps / span, 2), "failed": sum(i["status"] == G.IPC_REQ_FAILED for i in infos),
            "slot_cap": int(st["slot_cap"]), "budget_bytes": budget,
            "tets_total": int(sum(len(sc["tets"]) for sc in scs))}


def measured_traffic(precision):
    """HBM bytes per k_spmv launch from the committed rocprofv3 counter runs (FETCH_SIZE + WRITE_SIZE,
    scaled by the same counters on a plain copy of known size), or None when the kernel source has
    changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "spmv_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    src = os.path.join(ROOT, "paper_2503_05020_amd", "csrc", "ipc_kernels.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != d.get("kernel_source_sha256"):
            return None
    v = d.get("bytes_per_launch", {}).get(precision)
    return None if v is None else int(v)


def pmc_summary(d, copy_mib):
    """Write profiles/spmv_traffic.json from rocprofv3 --pmc csv runs under directory d:
    pmc_copy_<C> (this script with --copy-probe copy_mib) and pmc_spmv_<prec>_<C> (this script with
    --precision <prec> --count-all-bytes, its output in pmc_spmv_<prec>_<C>.log), for C in FETCH_SIZE,
    WRITE_SIZE (KiB per dispatch)."""
    import csv
    import glob
    import hashlib

    def rows(sub):
        out = []
        for f in glob.glob(os.path.join(d, sub, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                out += list(csv.DictReader(fh))
        return out

    def per_dispatch(rs, counter, pick):
        v = {}
        for r in rs:
            if r["Counter_Name"] == counter and pick(r["Kernel_Name"]):
                k = r.get("Dispatch_Id") or r.get("Correlation_Id")
                v[k] = v.get(k, 0.0) + float(r["Counter_Value"])
        return list(v.values())

    res = {"copy_probe_bytes": copy_mib << 20}
    factor = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        rs = rows(f"pmc_copy_{c}")
        vals = per_dispatch(rs, c, lambda n: "copy" in n.lower())
        kib = max(vals)  # the copy dispatches (the fill before them reads nothing)
        factor[c] = (copy_mib << 20) / (kib * 1024.0)
        res[f"copy_{c}_kib_per_dispatch"] = kib
        res[f"factor_{c}"] = round(factor[c], 4)
    res["bytes_per_launch"] = {}
    for prec in ("fp64", "mixed"):
        tot = 0.0
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            vals = per_dispatch(rows(f"pmc_spmv_{prec}_{c}"), c, lambda n: "k_spmv" in n)
            if not vals:
                tot = None
                break
            mean = sum(vals) / len(vals)
            res[f"spmv_{prec}_{c}_kib_mean"] = round(mean, 1)
            res[f"spmv_{prec}_{c}_dispatches"] = len(vals)
            tot += mean * 1024.0 * factor[c]
        if tot is not None:
            res["bytes_per_launch"][prec] = int(tot)
        # the algorithmic bytes of the same launches (the counter runs use --count-all-bytes)
        log_path = os.path.join(d, f"pmc_spmv_{prec}_FETCH_SIZE.log")
        if os.path.exists(log_path):
            with open(log_path) as fh:
                for line in fh:
                    if line.startswith("{") and "algorithmic_bytes_per_launch" in line:
                        alg = json.loads(line)["algorithmic_bytes_per_launch"][prec]
                        res.setdefault("algorithmic_bytes_per_launch", {})[prec] = alg
                        if tot:
                            res.setdefault("traffic_over_algorithmic", {})[prec] = round(tot / alg, 3)
    with open(os.path.join(ROOT, "paper_2503_05020_amd", "csrc", "ipc_kernels.hip"), "rb") as f:
        res["kernel_source_sha256"] = hashlib.sha256(f.read()).hexdigest()
    out = os.path.join(ROOT, "profiles", "spmv_traffic.json")
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


def _bw(bytes_, ms):
    return bytes_ / (ms * 1e-3) / 1e9


def roofline(prof, precision):
    """k_spmv (the dominant kernel): the event-timed launches' algorithmic bytes over their time (the bytes
    are counted by a separate launch, so no counting runs inside the timed kernel); beside it the whole PCG
    iteration (product + update) and the assembly pass against the same HBM peak."""
    if prof["spmv_launches"] <= 0 or prof["spmv_ms"] <= 0:
        return None
    avg_ms = prof["spmv_ms"] / prof["spmv_launches"]
    bytes_per_launch = prof["spmv_bytes"] / prof["spmv_launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(precision), "kernel": "k_spmv",
           "avg_launch_us": round(avg_ms * 1e3, 2), "bytes_per_launch": int(bytes_per_launch),
           "launches_timed": int(prof["spmv_launches"])}
    if prof["big_launches"] > 0 and prof["big_ms"] > 0:
        # the same, restricted to the launches over more than 64 tiles (the
        # rest are the latency-bound tails of the last environments' solves)
        bms = prof["big_ms"] / prof["big_launches"]
        bb = prof["big_bytes"] / prof["big_launches"]
        out["large_launches"] = {"achieved": round(bb / (bms * 1e-3) / 1e9, 1), "frac": round(bb / (bms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "avg_launch_us": round(bms * 1e3, 2), "bytes_per_launch": int(bb),
                                 "launches_timed": int(prof["big_launches"])}
    if prof["iters"] > 0 and prof["iter_ms"] > 0:
        a = _bw(prof["iter_bytes"], prof["iter_ms"])
        out["pcg_iteration"] = {"achieved": round(a, 1), "frac": round(a / HBM_PEAK_GBS, 4),
                                "avg_us": round(1e3 * prof["iter_ms"] / prof["iters"], 2),
                                "bytes_per_iteration": int(prof["iter_bytes"] / prof["iters"]),
                                "kernels": ["k_spmv", "k_pcg_update"], "iterations_timed": prof["iters"]}
    if prof["asm_passes"] > 0 and prof["asm_ms"] > 0:
        a = _bw(prof["asm_bytes"], prof["asm_ms"])
        out["assembly"] = {"achieved": round(a, 1), "frac": round(a / HBM_PEAK_GBS, 4),
                           "avg_us": round(1e3 * prof["asm_ms"] / prof["asm_passes"], 2),
                           "bytes_per_pass": int(prof["asm_bytes"] / prof["asm_passes"]),
                           "kernels": ["k_elastic", "k_assemble_rows", "k_assemble_sell"],
                           "passes_timed": prof["asm_passes"]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=12)
    ap.add_argument("--envs", type=int, default=256)
    ap.add_argument("--workload", default="superquadric_batch")
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="both")
    ap.add_argument("--pcg-tol", type=float, default=1e-4)
    ap.add_argument("--sequential-envs", type=int, default=8)
    ap.add_argument("--full-horizon", type=int, default=100,
                    help="also time this many steps from step 0 (the whole grasp) per precision; 0 skips")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", default="",
                    help="tune the scheduling knobs per workload before timing, caching the choice in this file")
    ap.add_argument("--relative-stop", type=float, default=1e-3,
                    help="also time the mixed window with the paper's relative Newton stop (eps_r; 0 skips)")
    ap.add_argument("--serve-requests", type=int, default=48, help="0 skips the serving run")
    ap.add_argument("--serve-slots", type=int, default=0, help="0 = slot cap tuned by the server")
    ap.add_argument("--serve-rate", type=float, default=50.0, help="request arrivals per second")
    ap.add_argument("--serve-only", action="store_true",
                    help="only run the serving sample (--serve-requests at --serve-rate) and print its JSON object")
    ap.add_argument("--count-all-bytes", action="store_true",
                    help="count the algorithmic bytes of every PCG product launch (warm-up included), time none")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many MiB, 5 times (calibrates HBM counters)")
    ap.add_argument("--pmc-summary", default="",
                    help="only summarise rocprofv3 --pmc csv runs under this directory into profiles/spmv_traffic.json")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary, args.copy_probe or 512)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: environments are independent and would be sharded across GPUs "
              "without any collective; only --gpus 1 is supported.", file=sys.stderr)
        sys.exit(2)
    import torch  # device selection only
    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    if args.copy_probe > 0:
        n = args.copy_probe << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n, "copy_probe_bytes_written": n, "launches": 5}), flush=True)
        return
    if args.serve_only:
        serve = serving(args.serve_requests, args.serve_rate, 200 << 30, args.serve_slots, G.IPC_MIXED)
        print(json.dumps({"serving": serve}), flush=True)
        return
    scs = make_scenes(args.workload, args.envs)
    ntets = sum(len(sc["E"]) for sc in scs)
    log(f"workload {args.workload}: {len(scs)} envs, {ntets} tets")
    G.ipc_prof_enable(2 if args.count_all_bytes else 1)
    results = {}
    precs = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    for p in precs:
        results[p] = run_gpu(scs, G.IPC_MIXED if p == "mixed" else G.IPC_FP64, args.warmup, args.steps,
                             args.pcg_tol, p, args.count_all_bytes, autotune=args.autotune or None)
        if args.count_all_bytes:
            pr = results[p]["prof"]
            # algorithmic bytes per product launch over the whole run, the
            # launches a counter run of the same command sees
            print(json.dumps({"algorithmic_bytes_per_launch": {p: int(pr["spmv_bytes"] / max(1, pr["spmv_launches"]))},
                              "launches": pr["spmv_launches"]}), flush=True)
        log(f"[{p}] {results[p]['value']:.1f} converged env-steps/s, {results[p]['ms_per_step']:.1f} ms/step")
    main_p = "mixed" if "mixed" in results else precs[0]
    r = results[main_p]
    seq = None
    if args.sequential_envs > 0:
        seq = sequential_gpu(scs, G.IPC_MIXED if main_p == "mixed" else G.IPC_FP64, args.warmup, args.steps,
                             args.pcg_tol, min(args.sequential_envs, len(scs)))
        log(f"sequential single-env: {seq['value']:.2f} env-steps/s")
    serve = None
    if args.serve_requests > 0:
        serve = serving(args.serve_requests, args.serve_rate, 200 << 30, args.serve_slots, G.IPC_MIXED)
        log(f"[serving] {serve}")
    rel = None
    if args.relative_stop > 0 and "mixed" in results:
        # the same window under the relative reading of the Newton stop (eps_r L h)
        h = run_gpu(scs, G.IPC_MIXED, args.warmup, args.steps, args.pcg_tol, "mixed relative stop",
                    newton_rel_tol=args.relative_stop)
        rel = {"eps_r": args.relative_stop, "value": round(h["value"], 2), "ms_per_step": round(h["ms_per_step"], 2),
               "failed_envs": h["failed"], "newton_iters": h["newton"], "pcg_iters": h["pcg"]}
        log(f"[mixed relative stop] {h['value']:.1f} converged env-steps/s, {h['failed']} failed")
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.workload, len(scs), args.warmup, args.steps)
    horizon = None
    if args.full_horizon > 0:
        # the whole grasp (closing with gravity off, gravity from step 60), both precisions
        horizon = {}
        for p in precs:
            h = run_gpu(scs, G.IPC_MIXED if p == "mixed" else G.IPC_FP64, 0, args.full_horizon, args.pcg_tol,
                        f"{p} horizon")
            horizon[p] = {"value": round(h["value"], 2), "steps": args.full_horizon, "failed_envs": h["failed"],
                          "wall_s": round(h["wall"], 2)}
            log(f"[{p}] full horizon: {h['value']:.1f} converged env-steps/s over steps 0..{args.full_horizon - 1}")
    out = {
        "metric": "converged sim steps/s over batched scenes",
        "value": round(r["value"], 2),
        "unit": "converged env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32pcg" if main_p == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "envs": len(scs), "tets": ntets, "precision": main_p,
                   "pcg_rel_tol": args.pcg_tol, "first_timed_step": args.warmup,
                   "pcg_preconditioner": "two-level (block Jacobi + rigid-body coarse space)"
                   if G.ipc_get_tuning(G.IPC_TUNE_COARSE) else "block Jacobi"},
        "newton_iters": r["newton"],
        "pcg_iters": r["pcg"],
        "failed_envs": r["failed"],
        "roofline": roofline(r["prof"], main_p),
        "contact": contact_rates(r),
        "cpu_baseline": cpu,
        "serving": serve,
    }
    if "fp64" in results and main_p != "fp64":
        f = results["fp64"]
        out["fp64"] = {"value": round(f["value"], 2), "ms_per_step": round(f["ms_per_step"], 2),
                       "failed_envs": f["failed"], "roofline": roofline(f["prof"], "fp64"),
                       "contact": contact_rates(f)}
    if horizon:
        out["full_horizon"] = horizon
    if rel:
        out["relative_newton_stop"] = rel
    if seq:
        out["sequential_single_env"] = {"value": round(seq["value"], 3), "envs": seq["envs"],
                                        "speedup_batched_vs_sequential": round(r["value"] / seq["value"], 2)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
