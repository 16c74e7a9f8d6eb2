"""Benchmark of the MOMMS FP64 GEMM family on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--member NAME] [--size N]

A step is one C := A B + C product in FP64 at m = n = k = 8192 (uniform
[-1, 1] entries, beta = 1 with random C) by the selected family member
(default: the autotuned pick), with inputs resident in HBM.  The JSON line
reports whole-job TFLOP/s, the dominant kernel's roofline position against
the FP64 MFMA peak, the model's byte prediction, and the CPU oracle timed on
a bounded sample of the same product.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--member", default="AUTO")
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target length of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline leg")
    ap.add_argument("--profile", action="store_true", help="few steps, no CPU leg (for rocprofv3 runs)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic_f64_8192.json"))
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (3 times): the reference for HBM byte counters")
    ap.add_argument("--profile-members", action="store_true",
                    help="run every family member once at --size, separated by marker fills (for rocprofv3)")
    return ap.parse_args()


def copy_calibration():
    """A plain device-to-device copy of 2**27 doubles (1 GiB) three times.

    Under rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE its dispatches must read
    and write 1 GiB each; the ratio counter/known is the scale applied to the
    GEMM kernels' counters.
    """
    import torch

    n = 1 << 27
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": 8 * n, "bytes_written": 8 * n, "repeats": 3}}),
          flush=True)


def profile_members(size):
    """Each member once (after one warm-up) with a 1-element fill between members."""
    import torch

    import paper_1904_05717_amd as mm
    import workloads

    m = n = k = size
    A, B, C = workloads.gemm_operands(m, n, k)
    Ad, Bd, Cd = (torch.from_numpy(x).to("cuda:0") for x in (A, B, C))
    del A, B, C
    marker = torch.empty(1, dtype=torch.float64, device="cuda:0")
    order = []
    for member in mm.FAMILY:
        wsb = mm.workspace_size(m, n, k, member)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda:0") if wsb else None
        mm.gemm(Ad, Bd, Cd, 1.0, 1.0, member=member, workspace=ws)
        marker.fill_(1.0)
        t0 = time.perf_counter()
        mm.gemm(Ad, Bd, Cd, 1.0, 1.0, member=member, workspace=ws)
        marker.fill_(2.0)
        torch.cuda.synchronize()
        order.append({"member": member, "launches": mm.member_plan(member, m, n, k)["launches"],
                      "packed": ws is not None, "s": round(time.perf_counter() - t0, 4)})
        print(json.dumps({"profiled": order[-1]}), flush=True)
    print(json.dumps({"profile_members": order, "size": size}), flush=True)


def cpu_baseline(m, n, k, target_s):
    """Time the oracle on a bounded sample of the same product: full rows of C."""
    import numpy as np

    import oracle
    import workloads

    A, B, C = workloads.gemm_operands(m, n, k)
    # calibrate on one row, then size the sample to about target_s
    rows = np.zeros(n, dtype=np.int64)
    cols = np.arange(n, dtype=np.int64)
    t0 = time.perf_counter()
    oracle.gemm_entries(A, B, rows, cols, C, 1.0, 1.0)
    per_row = max(time.perf_counter() - t0, 1e-6)
    nrows = int(max(1, min(m, target_s / per_row)))
    rr = np.repeat(np.arange(nrows, dtype=np.int64), n)
    cc = np.tile(np.arange(n, dtype=np.int64), nrows)
    t0 = time.perf_counter()
    oracle.gemm_entries(A, B, rr, cc, C, 1.0, 1.0)
    dt = time.perf_counter() - t0
    flops = 2.0 * nrows * n * k
    return {"value": round(flops / dt / 1e12, 6), "unit": "TFLOP/s", "cores": oracle.num_threads(),
            "kind": "oracle", "sample": f"{nrows} full rows of C ({nrows * n} entries, k={k}) of the "
                                        f"{m}x{n}x{k} product, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.profile_members:
        profile_members(args.size)
        return
    import torch

    import paper_1904_05717_amd as mm
    import workloads

    m = n = k = args.size
    member = args.member
    if member == "AUTO":
        member = mm.select_member(m, n, k)
    plan = mm.member_plan(member, m, n, k)
    dev = "cuda:0"
    A, B, C = workloads.gemm_operands(m, n, k)
    Ad = torch.from_numpy(A).to(dev)
    Bd = torch.from_numpy(B).to(dev)
    Cd = torch.from_numpy(C).to(dev)
    del A, B, C
    ws = None
    wsb = mm.workspace_size(m, n, k, member)
    if wsb:
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        mm.gemm(Ad, Bd, Cd, alpha=1.0, beta=1.0, member=member, workspace=ws, stream=stream)

    steps = 3 if args.profile else args.steps
    warm = 1 if args.profile else args.warmup
    for _ in range(warm):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / steps
    flops = 2.0 * m * n * k
    tflops = flops / (ms * 1e-3) / 1e12
    # dominant kernel: the member's main kernel; one launch per step unless the
    # plan splits k or the C region over several launches
    compute_launches = plan["launches"] // (2 if plan["pack"] and ws is not None else 1)
    launch_ms = ms / max(1, compute_launches)
    achieved = (flops / max(1, compute_launches)) / (launch_ms * 1e-3) / 1e12
    model = mm.model_bytes(member, m, n, k, beta=1.0, packed=ws is not None)
    traffic = None
    if os.path.exists(args.traffic_json):
        try:
            tj = json.load(open(args.traffic_json))
            if tj.get("member") == member and tj.get("size") == m:
                traffic = tj.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None
    out = {
        "metric": "FP64 GEMM TFLOP/s + % MFMA peak; HBM bytes vs model; split-prec speedup",
        "value": round(tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"fp64 gemm C+=A*B m=n=k={m} row-major, U[-1,1], beta=1", "member": member,
                   "m": m, "n": n, "k": k},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4),
                     "traffic": traffic},
        "frac_fp64_mfma_peak": round(tflops / FP64_MFMA_PEAK_TFLOPS, 4),
        "model_bytes": {"l2_read": model["l2_read"], "l2_write": model["l2_write"],
                        "hbm_read": model["hbm_read"], "hbm_write": model["hbm_write"],
                        "compulsory": model["compulsory"]},
        "wall_s_timed": round(wall, 3),
    }
    if not args.no_cpu and not args.profile:
        out["cpu_baseline"] = cpu_baseline(m, n, k, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
