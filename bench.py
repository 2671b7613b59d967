"""Benchmark of the WADG sweep on one MI355X.

One step = one pass of the whole hot path over one batch: every slice of the
workload advanced by its LSRK steps (5 fused stage launches per step: trace
gathers, volume term, flux and lift, WADG mass inverse, stage update), then
the per-slice reductions (norms, finite check).  Default workload: wadg128
(128 x 128 curvilinear elements of degree 3, i.e. 512 x 512 nodes per field,
heterogeneous c^2, 256 time slices of 10 steps, FP64: 4.8 GB of state and
workspace, far beyond the memory-side cache).

Prints one JSON line.  ``value`` = grid-point-steps/s: slices x nodes per
slice (one node carries p, u, v) x LSRK steps per slice / seconds per step.

``--path`` selects another part of the library, each also one JSON line:
fp32 (FP32-bulk sweep, with its error against the FP64 sweep), batch (the
1000-problem batch, one 4-step sweep per step), adjoint (forward sweep with
checkpoints plus the reverse sweep on the 128 x 128 sensitivity problem),
parareal (the wadg64 trajectory by parareal, against the serial fine sweep).
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# wadg_kernel_in_use value -> kernel name (WADG_KERNEL_STREAMED .. _PIPE)
KERNEL_NAMES = {1: "stage_kernel", 2: "resident_kernel", 3: "split_kernel", 4: "pipe_kernel"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--path", choices=("fp64", "fp32", "batch", "adjoint", "parareal"),
                    default="fp64", help="what to measure (default: the FP64 sweep)")
    ap.add_argument("--workload", default="wadg128")
    ap.add_argument("--tile-groups", type=int, default=None,
                    help="schedule: element groups per tile (default: library default)")
    ap.add_argument("--tile-slices", type=int, default=0)
    ap.add_argument("--kernel", choices=("auto", "streamed", "resident", "split", "pipe"),
                    default="auto",
                    help="stage-kernel variant (default: the library's choice)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this size before the timed "
                         "region, as the known-size reference for HBM byte counters")
    ap.add_argument("--cpu-baseline-seconds", type=float, default=15.0,
                    help="approximate CPU seconds for the oracle baseline (0: skip)")
    return ap.parse_args()


def kernel_choice(W, name):
    """--kernel value -> WADG_KERNEL_* constant."""
    return {"auto": W.WADG_KERNEL_AUTO, "streamed": W.WADG_KERNEL_STREAMED,
            "resident": W.WADG_KERNEL_RESIDENT, "split": W.WADG_KERNEL_SPLIT,
            "pipe": W.WADG_KERNEL_PIPE}[name]


def stage_bytes(K, S, N, nq1, word=8):
    """Algorithmic HBM bytes of one stage launch, averaged over the 5 stages:
    per element and slice, read Q_in and write Q_out (3 (N+1)^2 values
    each), read the residual in stages 2-5 (stage 1 has A = 0) and write it
    in stages 1-4 (stage 5's is never read: the next step starts with A =
    0); per element, read the geometry once (6 nq1^2 volume + 12 nq1 face
    values, 8 int32 offsets).  word: bytes per value (8 FP64, 4 FP32-bulk)."""
    Np = (N + 1) ** 2
    per_elem_slice = 3 * Np * word * (2 + 8 / 5)
    per_elem = (6 * nq1 * nq1 + 12 * nq1) * word + 8 * 4
    return K * (S * per_elem_slice + per_elem)


def stage_bytes_4(K, S, N, nq1, word=8):
    """The coarser count of the hot-path scope table: four state arrays per
    element and slice in every stage (read Q_in and the residual, write
    Q_out and the residual) and the geometry's values once per element."""
    Np = (N + 1) ** 2
    return K * (S * 3 * Np * word * 4 + (6 * nq1 * nq1 + 12 * nq1) * word)


def measured_traffic(kernel, workload):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) from the
    rocprofv3 counter runs recorded in profiles/hbm_traffic.json, or None when
    there is no record for this kernel and workload or the code of the
    kernel's sources has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    for rec in json.load(open(path))["records"]:
        if rec["kernel"] != kernel or rec["workload"] != workload:
            continue
        if sources_digest(rec["sources"]) == rec["sources_sha1"]:
            return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    return None


def sources_digest(sources):
    """SHA-1 of the code of the listed source files with their comments and
    white space removed, so that a counter record stays valid across
    comment-only edits and lapses with any change to the code."""
    import hashlib
    import re
    h = hashlib.sha1()
    for src in sources:
        with open(os.path.join(ROOT, src)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(re.sub(r"\s+", "", text).encode())
    return h.hexdigest()


def cpu_baseline(prob, seconds):
    """The oracle, as it stands, on a bounded sample: whole slices of the same
    workload, one after another, on one host thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import WADGOracle
    with threadpool_limits(1):
        o = WADGOracle(prob.mesh, nq1=prob.nq1, c2=prob.c2, tau_p=prob.tau_p, tau_u=prob.tau_u)
        # size the sample from one timed step of one slice
        t0 = time.perf_counter()
        o.integrate(prob.Q0[0], prob.dt, 1)
        one = time.perf_counter() - t0
        steps = max(1, min(prob.nsteps, int(seconds / max(one, 1e-6))))
        nsl = max(1, min(len(prob.Q0), int(seconds / max(one * prob.nsteps, 1e-6))))
        if nsl > 1:
            steps = prob.nsteps
        t0 = time.perf_counter()
        for s in range(nsl):
            o.integrate(prob.Q0[s], prob.dt, steps)
        el = time.perf_counter() - t0
    nodes = prob.K * (prob.N + 1) ** 2
    return {"value": nsl * nodes * steps / el, "unit": "grid-point-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{nsl} slice(s) x {steps} LSRK steps of {prob.name} "
                      f"({prob.K} elements, N={prob.N}), numpy FP64, 1 thread, {el:.1f} s"}


def common(args, value, ms_per_step, dtype, config):
    return {"metric": "grid-point-steps/sec", "value": value, "unit": "grid-point-steps/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


# Floating-point operations per element and LSRK stage, sum-factorised, at
# N = 3 with 5 Gauss points per direction: volume 3,180, mass inverse
# 2,235, surface 2,224, update 192 (the volume and inverse parts follow
# from the operation counts of the kernels' contractions; FMA = 2).
FLOPS_PER_ELEMENT_STAGE = {(3, 5): 7831}
PEAK_FP32_TFLOPS = 157.3


def roofline_alu(flops_launch, stage_ms, peak_tflops):
    """The FP32 path's arithmetic roofline: its kernels issue no packed
    (two-wide) FP32 instructions, so half the peak is their ceiling."""
    achieved = flops_launch / (stage_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": peak_tflops, "unit": "TFLOP/s",
            "frac": achieved / peak_tflops, "flops_per_launch": flops_launch,
            "frac_of_unpacked_rate": achieved / (peak_tflops / 2)}


def roofline(kname, bytes_launch, stage_ms, traffic=None, bytes_4=None):
    achieved = bytes_launch / (stage_ms * 1e-3) / 1e9
    r = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
         "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
         # measured HBM bytes (the counters) at this run's launch time
         "traffic_frac": (None if traffic is None else
                          traffic / (stage_ms * 1e-3) / 1e9 / PEAK_HBM_GBS),
         "kernel": kname, "avg_launch_us": stage_ms * 1e3,
         "algorithmic_bytes_per_launch": bytes_launch}
    if bytes_4 is not None:
        # the same launch time against the four-array count
        r["algorithmic_bytes_4_state_arrays"] = bytes_4
        r["frac_4_state_arrays"] = bytes_4 / (stage_ms * 1e-3) / 1e9 / PEAK_HBM_GBS
    return r


def calibrate(args, torch):
    """The known-size device copy that HBM byte counters are scaled by."""
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst


def timed(args, torch, stream, body):
    """warmup untimed calls of body(), then args.steps timed ones bracketed by
    synchronisations; returns (wall seconds, [HIP-event ms of each call])."""
    for _ in range(args.warmup):
        body()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        body()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, [a.elapsed_time(b) for a, b in ev]


def run_fp32(args):
    """FP32-bulk sweep (state, residual and geometry FP32 inside the sweep,
    FP64 in and out) of the whole workload; error against the FP64 sweep of
    the same start states."""
    import numpy as np
    import torch
    import paper_1608_03836_amd as W
    from workloads import make_problem
    prob = make_problem(args.workload)
    sol = W.Solver.from_problem(prob)
    sol.set_kernel(kernel_choice(W, args.kernel))
    S, K, N = prob.S, prob.K, prob.N
    stream = torch.cuda.current_stream()
    Q64 = sol.upload(prob.Q0)
    sol.integrate(Q64, S, prob.dt, prob.nsteps, stream=stream)
    Q = sol.upload(prob.Q0)
    work = sol.workspace_fp32(S)
    sol.integrate_fp32(Q, S, prob.dt, prob.nsteps, work=work, stream=stream)
    torch.cuda.synchronize()
    d = (Q - Q64).reshape(S, -1)
    rel = float(torch.max(torch.linalg.norm(d, dim=1) /
                          torch.linalg.norm(Q64.reshape(S, -1), dim=1)).item())
    l2 = sol.l2_norms(Q, Q64, S)        # L2 with the Jacobian, per slice
    rel_l2 = float(np.max(l2[:, 0] / l2[:, 1]))
    del Q64
    calibrate(args, torch)
    elapsed, ev = timed(args, torch, stream,
                        lambda: sol.integrate_fp32(Q, S, prob.dt, prob.nsteps, work=work,
                                                   stream=stream))
    norms = sol.norms(Q, None, S)
    assert np.all(norms[:, 3] == 1.0), "non-finite state"
    nodes = K * (N + 1) ** 2
    line = common(args, S * nodes * prob.nsteps / (elapsed / args.steps),
                  1e3 * elapsed / args.steps, "f32",
                  {"workload": prob.name, "path": "fp32-bulk", "elements": K, "degree": N,
                   "nq1": prob.nq1, "slices": S, "lsrk_steps_per_slice": prob.nsteps,
                   "parallelism": "single-gpu"})
    k = KERNEL_NAMES[sol.kernel_in_use(fp32=True)]
    # the events bracket the whole call: 5 nsteps stage launches plus the two
    # FP64<->FP32 conversions at the ends of the sweep
    kname = f"{k}<float,{N},{prob.nq1}>"
    stage_ms = sum(ev) / (args.steps * 5 * prob.nsteps)
    line["roofline"] = roofline(kname, stage_bytes(K, S, N, prob.nq1, word=4), stage_ms,
                                measured_traffic(kname, prob.name),
                                stage_bytes_4(K, S, N, prob.nq1, word=4))
    fl = FLOPS_PER_ELEMENT_STAGE.get((N, prob.nq1))
    if fl is not None:
        # the arithmetic bound of this path (the HBM one above is not reached)
        line["roofline_alu"] = roofline_alu(fl * K * S, stage_ms, PEAK_FP32_TFLOPS)
    line["max_rel_err_vs_fp64_sweep"] = rel
    line["max_rel_l2_err_vs_fp64_sweep"] = rel_l2
    if args.cpu_baseline_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_baseline_seconds)
    print(json.dumps(line), flush=True)


def run_batch(args):
    """The 1000-problem batch: one 4-step sweep of every problem per step,
    as a replay of the HIP graph the library captured for the sweep, on the
    schedule its autotuner chose."""
    import numpy as np
    import torch
    import paper_1608_03836_amd as W
    from threadpoolctl import threadpool_limits
    from workloads import make_batch
    from oracle import WADGOracle
    probs = make_batch()
    batch = W.Batch([p.mesh for p in probs], [p.S for p in probs])
    dts = [p.dt for p in probs]
    nsteps = probs[0].nsteps
    stream = torch.cuda.current_stream()
    Q = batch.upload([p.Q0 for p in probs])
    work = batch.workspace()
    wg, order, runs, tuned_us = batch.tune(Q, dts, work=work, reps=3, stream=stream)
    batch.capture(Q, work, dts, nsteps)
    calibrate(args, torch)
    elapsed, ev = timed(args, torch, stream, lambda: batch.replay(stream=stream))
    batch.release_graph()
    N, nq1 = batch.N, batch.nq1
    gps = sum(p.S * p.mesh.K * (N + 1) ** 2 for p in probs) * nsteps
    line = common(args, gps / (elapsed / args.steps), 1e3 * elapsed / args.steps, "f64",
                  {"workload": "batch1000", "problems": len(probs),
                   "elements": int(sum(p.mesh.K for p in probs)),
                   "slices": int(sum(p.S for p in probs)), "degree": N, "nq1": nq1,
                   "lsrk_steps_per_slice": nsteps, "launch": "hip-graph replay",
                   "schedule": {"run_slices": runs, "wg_per_cu": wg, "order": order,
                                "tuned_stage_us": tuned_us},
                   "parallelism": "single-gpu"})
    kind = ("batch_pipe_kernel" if runs > 0 else
            "batch_split_kernel" if wg == 0 else "batch_stage_kernel")
    kname = f"{kind}<{N},{nq1}>"
    line["roofline"] = roofline(kname, sum(stage_bytes(p.mesh.K, p.S, N, nq1) for p in probs),
                                sum(ev) / (args.steps * 5 * nsteps),
                                measured_traffic(kname, "batch1000"),
                                sum(stage_bytes_4(p.mesh.K, p.S, N, nq1) for p in probs))
    if args.cpu_baseline_seconds > 0:
        # the oracle on the first problems of the list, whole problems, until
        # about the requested time
        with threadpool_limits(1):
            done, el, npb = 0, 0.0, 0
            for p in probs:
                o = WADGOracle(p.mesh)
                t0 = time.perf_counter()
                for s in range(p.S):
                    o.integrate(p.Q0[s], p.dt, p.nsteps)
                el += time.perf_counter() - t0
                done += p.S * p.mesh.K * (N + 1) ** 2 * p.nsteps
                npb += 1
                if el >= args.cpu_baseline_seconds:
                    break
        line["cpu_baseline"] = {"value": done / el, "unit": "grid-point-steps/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"the first {npb} problems of the batch, every slice, "
                                          f"{nsteps} LSRK steps, numpy FP64, 1 thread, {el:.1f} s"}
    print(json.dumps(line), flush=True)


def run_adjoint(args):
    """Forward sweep with checkpoints plus the reverse (adjoint) sweep: one
    gradient of the terminal objective with respect to the start state and
    the c^2 scale, on the 128 x 128 sensitivity problem."""
    import numpy as np
    import torch
    import paper_1608_03836_amd as W
    from workloads import make_sensitivity_problem
    from paper_1608_03836_amd.autograd import pressure_mask
    prob = make_sensitivity_problem("adj128")
    sol = W.Solver(prob.mesh, nq1=prob.nq1, c2=prob.c0, tau_p=prob.tau_p, tau_u=prob.tau_u)
    sol.set_c2_scale(prob.gamma)
    stream = torch.cuda.current_stream()
    y0 = sol.upload(prob.y0[None])
    work = sol.adjoint_workspace(prob.nsteps)
    target = np.zeros((1, 3) + prob.p_target.shape)
    target[0, 0] = prob.p_target
    target = sol.upload(target)
    mask = pressure_mask(sol)
    n1 = sol.slice_doubles
    fw, rv = [], []

    def body():
        a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        a.record(stream)
        chk = sol.forward_checkpoints(y0, prob.S, prob.dt, prob.nsteps, work=work, stream=stream)
        b.record(stream)
        seed = (2.0 * mask * (chk[prob.S * n1:] - target)).contiguous()
        sol.adjoint(chk, seed, prob.S, prob.dt, prob.nsteps, work=work, stream=stream)
        c.record(stream)
        fw.append((a, b))
        rv.append((b, c))

    elapsed, _ = timed(args, torch, stream, body)
    fwd = sum(a.elapsed_time(b) for a, b in fw[-args.steps:]) / args.steps
    rev = sum(a.elapsed_time(b) for a, b in rv[-args.steps:]) / args.steps
    nodes = prob.mesh.K * (prob.mesh.N + 1) ** 2
    line = common(args, prob.S * prob.nsteps * nodes / (elapsed / args.steps),
                  1e3 * elapsed / args.steps, "f64",
                  {"workload": prob.name, "path": "forward + adjoint",
                   "elements": prob.mesh.K, "degree": prob.mesh.N, "nq1": prob.nq1,
                   "checkpointed_slices": prob.S, "lsrk_steps_per_slice": prob.nsteps,
                   "parallelism": "single-gpu"})
    line["forward_ms"] = fwd
    line["adjoint_ms"] = rev
    # one-slice launches (6.3 MB of state each) are cache-resident: no roofline point
    line["roofline"] = None
    if args.cpu_baseline_seconds > 0:
        from workloads import make_problem
        from types import SimpleNamespace
        p = SimpleNamespace(mesh=prob.mesh, nq1=prob.nq1, c2=lambda x, y: prob.gamma * prob.c0(x, y),
                            tau_p=prob.tau_p, tau_u=prob.tau_u, Q0=prob.y0[None], dt=prob.dt,
                            nsteps=prob.nsteps, K=prob.mesh.K, N=prob.mesh.N, name=prob.name)
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_baseline_seconds)
        line["cpu_baseline"]["sample"] += " (forward sweep only)"
    print(json.dumps(line), flush=True)


def run_parareal(args):
    """The wadg64 trajectory (slice 0's start state, 64 slices of 32 steps)
    by parareal with a 17-step coarse sweep (the fewest coarse steps whose
    CFL number, 1.20, is inside the library's coarse-step bound of 1.25),
    against the serial fine sweep."""
    import numpy as np
    import torch
    import paper_1608_03836_amd as W
    from workloads import make_problem
    prob = make_problem("wadg64", slices=[0])
    sol = W.Solver.from_problem(prob)
    S, nf, nc = 64, prob.nsteps, 17
    stream = torch.cuda.current_stream()
    y0 = sol.upload(prob.Q0[:1])
    work1 = sol.workspace(1)
    q = y0.clone()
    sol.integrate(q, 1, prob.dt, 1, work=work1, stream=stream)
    torch.cuda.synchronize()
    q = y0.clone()
    t0 = time.perf_counter()
    for _ in range(S):
        sol.integrate(q, 1, prob.dt, nf, work=work1, stream=stream)
    torch.cuda.synchronize()
    serial = time.perf_counter() - t0
    res = {}

    def body():
        res["out"] = sol.parareal(y0, S, prob.dt, nf, nc, max_iter=12, tol=1e-8, stream=stream)

    elapsed, _ = timed(args, torch, stream, body)
    U, it, ch = res["out"]
    err = float(torch.linalg.norm(U[S * sol.slice_doubles:] - q) / torch.linalg.norm(q))
    nodes = prob.K * (prob.N + 1) ** 2
    line = common(args, S * nf * nodes / (elapsed / args.steps), 1e3 * elapsed / args.steps,
                  "f64", {"workload": "wadg64-trajectory", "path": "parareal",
                          "elements": prob.K, "degree": prob.N, "slices": S,
                          "fine_steps_per_slice": nf, "coarse_steps_per_slice": nc,
                          "parallelism": "single-gpu"})
    line.update({"iterations": it, "last_change": ch, "rel_err_vs_serial_fine": err,
                 "serial_fine_ms": serial * 1e3,
                 "speedup_vs_serial_fine": serial / (elapsed / args.steps), "roofline": None})
    if args.cpu_baseline_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_baseline_seconds)
    print(json.dumps(line), flush=True)


def _oracle_worker(task):
    """One process of the all-cores baseline: whole slices of the workload,
    one after another, on one thread.  Returns (grid-point-steps, seconds)."""
    workload, slices = task
    from threadpoolctl import threadpool_limits
    from workloads import make_problem
    from oracle import WADGOracle
    prob = make_problem(workload, slices=slices)    # only this worker's start states
    with threadpool_limits(1):
        o = WADGOracle(prob.mesh, nq1=prob.nq1, c2=prob.c2, tau_p=prob.tau_p, tau_u=prob.tau_u)
        t0 = time.perf_counter()
        for i in range(len(slices)):
            o.integrate(prob.Q0[i], prob.dt, prob.nsteps)
        el = time.perf_counter() - t0
    return len(slices) * prob.K * (prob.N + 1) ** 2 * prob.nsteps, el


def _host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_all_cores(workload, slices_per_worker=2):
    """The same oracle on the host cores this run may use (at most 16 worker
    processes; slices are independent, so each worker takes whole slices),
    started before this process touches the GPU.  Rate: all workers' work
    over the slowest worker's compute time."""
    import multiprocessing as mp
    from workloads.configs import CONFIGS
    S = CONFIGS[workload]["S"]
    workers = max(1, min(16, os.cpu_count() or 1, S // slices_per_worker))
    tasks = [(workload, list(range(w * slices_per_worker, (w + 1) * slices_per_worker)))
             for w in range(workers)]
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_worker, tasks)
    work = sum(r[0] for r in res)
    wall = max(r[1] for r in res)
    return {"value": work / wall, "unit": "grid-point-steps/s", "cores": workers,
            "kind": "oracle", "host_cpu": _host_cpu(), "nproc": os.cpu_count(),
            "sample": f"{workers} processes x {slices_per_worker} slice(s) x all LSRK steps of "
                      f"{workload}, numpy FP64, 1 thread each, slowest {wall:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the sweep shards "
              "over slices with no communication, so N GPUs would each advance S/N slices",
              file=sys.stderr)
        sys.exit(2)
    other = {"fp32": run_fp32, "batch": run_batch, "adjoint": run_adjoint,
             "parareal": run_parareal}
    if args.path in other:
        return other[args.path](args)
    # the oracle on all host cores first, while this process has not touched
    # the GPU (its workers are fresh processes)
    allcores = (cpu_baseline_all_cores(args.workload) if args.cpu_baseline_seconds > 0
                else None)
    import numpy as np
    import torch
    import paper_1608_03836_amd as W
    from workloads import make_problem

    prob = make_problem(args.workload)
    sol = W.Solver.from_problem(prob)
    if args.tile_groups:
        sol.set_schedule(args.tile_groups, args.tile_slices)
    sol.set_kernel(kernel_choice(W, args.kernel))
    kname = KERNEL_NAMES[sol.kernel_in_use()]
    kname += f"<double,{prob.N},{prob.nq1}>"
    S, K, N = prob.S, prob.K, prob.N
    Q = sol.upload(prob.Q0)
    work = sol.workspace(S)
    stream = torch.cuda.current_stream()

    def step():
        sol.integrate(Q, S, prob.dt, prob.nsteps, work=work, stream=stream)
        out = sol.norms(Q, None, S, stream=stream)
        return out

    calibrate(args, torch)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        sol.integrate(Q, S, prob.dt, prob.nsteps, work=work, stream=stream)
        ev[i][1].record(stream)
        norms = sol.norms(Q, None, S, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert np.all(norms[:, 3] == 1.0), "non-finite state"

    ms_per_step = 1e3 * elapsed / args.steps
    launches = 5 * prob.nsteps
    stage_ms = sum(a.elapsed_time(b) for a, b in ev) / (args.steps * launches)
    nodes = K * (N + 1) ** 2
    value = S * nodes * prob.nsteps / (elapsed / args.steps)
    bytes_launch = stage_bytes(K, S, N, prob.nq1)

    traffic = measured_traffic(kname, prob.name)
    line = {
        "metric": "grid-point-steps/sec",
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": prob.name, "elements": K, "degree": N, "nq1": prob.nq1,
                   "nodes_per_slice": nodes, "slices": S, "lsrk_steps_per_slice": prob.nsteps,
                   "unknowns_per_slice": 3 * nodes, "parallelism": "single-gpu"},
        "roofline": roofline(kname, bytes_launch, stage_ms, traffic,
                             stage_bytes_4(K, S, N, prob.nq1)),
    }
    # the paper's own stage rate, quoted with its hardware (context only: a
    # different device, precision, element type and mesh); this run in the
    # same unit, scalar unknowns x RK stages per second
    line["paper_context"] = {
        "value": 9.15e8, "unit": "dof-stages/s",
        "what": "strong-weak WADG stage rate at N=3 (Section 6.5.1, time per unknown and stage)",
        "hardware": "one NVIDIA GTX 980, FP32 (inferred), 3D curvilinear tetrahedra",
        "this_run": 3 * nodes * S * 5 * prob.nsteps / (elapsed / args.steps)}
    if args.cpu_baseline_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_baseline_seconds)
        line["cpu_baseline_all_cores"] = allcores
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
