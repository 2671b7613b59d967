"""Benchmark of the WADG sweep on one MI355X.

One step = one pass of the whole hot path over one batch: every slice of the
workload advanced by its LSRK steps (5 fused stage launches per step: trace
gathers, volume term, flux and lift, WADG mass inverse, stage update), then
the per-slice reductions (norms, finite check).  Default workload: wadg64
(64 x 64 curvilinear elements of degree 3, i.e. 256 x 256 nodes per field,
64 time slices of 32 steps, FP64).

Prints one JSON line.  ``value`` = grid-point-steps/s: slices x nodes per
slice (one node carries p, u, v) x LSRK steps per slice / seconds per step.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="wadg64")
    ap.add_argument("--tile-groups", type=int, default=None,
                    help="schedule: element groups per tile (default: library default)")
    ap.add_argument("--tile-slices", type=int, default=0)
    ap.add_argument("--kernel", choices=("auto", "streamed", "resident", "split"), default="auto",
                    help="stage-kernel variant (default: the library's choice)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one device-to-device copy of this size before the timed "
                         "region, as the known-size reference for HBM byte counters")
    ap.add_argument("--cpu-baseline-seconds", type=float, default=15.0,
                    help="approximate CPU seconds for the oracle baseline (0: skip)")
    return ap.parse_args()


def stage_bytes(K, S, N, nq1):
    """Algorithmic HBM bytes of one stage launch, averaged over the 5 stages:
    per element and slice, read Q_in and write Q_out and res (3 (N+1)^2
    doubles each) and read res in 4 of the 5 stages; per element, read the
    geometry once (6 nq1^2 volume + 12 nq1 face doubles, 8 int32 offsets)."""
    Np = (N + 1) ** 2
    per_elem_slice = 3 * Np * 8 * (3 + 4 / 5)
    per_elem = (6 * nq1 * nq1 + 12 * nq1) * 8 + 8 * 4
    return K * (S * per_elem_slice + per_elem)


def measured_traffic(kernel, workload):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) from the
    rocprofv3 counter runs recorded in profiles/hbm_traffic.json, or None when
    there is no record for this kernel and workload or the kernel's sources
    have changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    for rec in json.load(open(path))["records"]:
        if rec["kernel"] != kernel or rec["workload"] != workload:
            continue
        h = hashlib.sha1()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() == rec["sources_sha1"]:
            return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    return None


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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the sweep shards "
              "over slices with no communication, so N GPUs would each advance S/N slices",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1608_03836_amd as W
    from workloads import make_problem

    prob = make_problem(args.workload)
    sol = W.Solver.from_problem(prob)
    if args.tile_groups:
        sol.set_schedule(args.tile_groups, args.tile_slices)
    sol.set_kernel({"auto": W.WADG_KERNEL_AUTO, "streamed": W.WADG_KERNEL_STREAMED,
                    "resident": W.WADG_KERNEL_RESIDENT, "split": W.WADG_KERNEL_SPLIT}[args.kernel])
    kname = {W.WADG_KERNEL_STREAMED: "stage_kernel", W.WADG_KERNEL_RESIDENT: "resident_kernel",
             W.WADG_KERNEL_SPLIT: "split_kernel"}[sol.kernel_in_use()]
    kname += f"<double,{prob.N},{prob.nq1},false>"
    S, K, N = prob.S, prob.K, prob.N
    Q = sol.upload(prob.Q0)
    work = sol.workspace(S)
    stream = torch.cuda.current_stream()

    def step():
        sol.integrate(Q, S, prob.dt, prob.nsteps, work=work, stream=stream)
        out = sol.norms(Q, None, S, stream=stream)
        return out

    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=sol.device)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

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
    achieved = bytes_launch / (stage_ms * 1e-3) / 1e9

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
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     # measured HBM bytes (the counters) at this run's launch time
                     "traffic_frac": (None if traffic is None else
                                      traffic / (stage_ms * 1e-3) / 1e9 / PEAK_HBM_GBS),
                     "kernel": kname,
                     "avg_launch_us": stage_ms * 1e3,
                     "algorithmic_bytes_per_launch": bytes_launch},
    }
    if args.cpu_baseline_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_baseline_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
