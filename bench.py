"""Benchmark of the MOMMS FP64 GEMM family on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--member NAME] [--size N]
                    [--only fp64|split|batch|backward|members|tiled|syrk|tri|ooc|sweep|lowbw]

A step is one C := A B + C product in FP64 at m = n = k = 8192 (uniform
[-1, 1] entries, beta = 1 with random C) by the selected family member
(default: the member the library's selector picks), inputs resident in HBM.
`value` is that product's TFLOP/s.  The same JSON line carries the dominant
kernel's roofline position against the FP64 MFMA peak, the model's byte
prediction next to the rocprofv3-measured traffic, the CPU oracle timed on a
bounded sample, and the other forms of the method measured on their own
workloads: the split-precision product (m = n = k = 8192, 16-decade data,
speedup over the FP64 product and its error), 512 batched uneven problems,
forward + hand-written backward at m = 4096, k = 8192, n = 2048, every
family member over square and shaped problems, tile-major storage, SYRK,
TRSM/TRMM/Cholesky, the out-of-core level, and every member beside a kernel
that takes HBM bandwidth (the varying-bandwidth experiments).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6
LOWP_MFMA_PEAK_TOPS = {"bf16": 2500.0, "fp8": 5000.0, "int8": 5000.0, "crt": 5000.0}   # dense, per the MI355X specification
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic_f64_8192.json")
TILED_MEMBERS = ["C0", "C3C0", "B3C0", "A3C0", "A2C0", "B3A2C0", "A3B2C0", "C3A2C0", "C4A2C0"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--member", default="AUTO")
    ap.add_argument("--size", type=int, default=8192)
    ap.add_argument("--shape", default=None,
                    help="m,n,k for --profile-members / --summarize (default: the square --size)")
    ap.add_argument("--only", default="all",
                    choices=["all", "fp64", "split", "batch", "backward", "members", "tiled", "syrk", "tri",
                             "ooc", "sweep", "lowbw"])
    ap.add_argument("--split", default="crt:14,crt:15,crt:16,int8:8,int8:9,bf16:3,bf16:4,bf16:5,bf16:6,bf16:7,"
                    "fp8:3,fp8:4,fp8:5,fp8:6,fp8:7,fp8:8",
                    help="split-precision configurations to time, as type:slices[,type:slices...]")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="length of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline leg")
    ap.add_argument("--full-json", metavar="PATH", default=None,
                    help="also write every section's full results to PATH as one JSON object")
    ap.add_argument("--profile", action="store_true", help="few steps, FP64 product only (for rocprofv3)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (3 times): the reference for HBM byte counters")
    ap.add_argument("--profile-members", action="store_true",
                    help="run every family member once at --size, separated by marker fills (for rocprofv3)")
    ap.add_argument("--summarize", metavar="DIR",
                    help="turn the rocprofv3 CSV output of a profiling pass in DIR into profiles/ summaries")
    return ap.parse_args()


def events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def copy_calibration():
    """A plain device-to-device copy of 2**27 doubles (1 GiB) three times.

    Under rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE its dispatches must read
    and write 1 GiB each; the ratio known/counter is the scale applied to
    the GEMM kernels' counters.
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


def shape_of(args):
    if args.shape:
        m, n, k = (int(x) for x in args.shape.split(","))
        return m, n, k
    return args.size, args.size, args.size


def shape_tag(m, n, k):
    return str(m) if m == n == k else f"{m}x{n}x{k}"


def profile_members(m, n, k):
    """Each member once (after one warm-up) with a 1-element fill between members."""
    import torch

    import paper_1904_05717_amd as mm
    import workloads

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
        mm.gemm(Ad, Bd, Cd, 1.0, 1.0, member=member, workspace=ws)
        marker.fill_(2.0)
        torch.cuda.synchronize()
        order.append({"member": member, "launches": mm.member_plan(member, m, n, k)["launches"],
                      "packed": ws is not None})
        print(json.dumps({"profiled": order[-1]}), flush=True)
    # the register-resident members again on tile-major ("prepacked") operands
    At, Bt = mm.to_tiled(Ad, "A"), mm.to_tiled(Bd, "B")
    torch.cuda.synchronize()
    marker.fill_(3.0)
    for member in TILED_MEMBERS:
        mm.gemm_tiled(At, Bt, m, n, k, Cd, 1.0, 1.0, member=member)
        marker.fill_(1.0)
        mm.gemm_tiled(At, Bt, m, n, k, Cd, 1.0, 1.0, member=member)
        marker.fill_(2.0)
        torch.cuda.synchronize()
        order.append({"member": member + "/tiled", "launches": mm.member_plan(member, m, n, k)["launches"],
                      "packed": False})
        print(json.dumps({"profiled": order[-1]}), flush=True)
    print(json.dumps({"profile_members": order, "shape": [m, n, k]}), flush=True)


def cpu_baseline(m, n, k, target_s):
    """The oracle timed on a bounded sample of the same product: full rows of C."""
    import numpy as np

    import oracle
    import workloads

    A, B, C = workloads.gemm_operands(m, n, k)
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


def bench_fp64(args):
    import torch

    import paper_1904_05717_amd as mm
    import workloads

    m = n = k = args.size
    member = args.member if args.member != "AUTO" else mm.select_member(m, n, k)
    plan = mm.member_plan(member, m, n, k)
    A, B, C = workloads.gemm_operands(m, n, k)
    Ad, Bd, Cd = (torch.from_numpy(x).to("cuda:0") for x in (A, B, C))
    wsb = mm.workspace_size(m, n, k, member)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda:0") if wsb else None
    stream = torch.cuda.current_stream()

    def step():
        mm.gemm(Ad, Bd, Cd, alpha=1.0, beta=1.0, member=member, workspace=ws, stream=stream)

    steps = 3 if args.profile else args.steps
    warm = 1 if args.profile else args.warmup
    for _ in range(warm):
        step()
    torch.cuda.synchronize()
    e0, e1 = events()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    flops = 2.0 * m * n * k
    # accuracy of the same call, untimed: one product into a fresh copy of C
    # against the oracle on sampled entries, as error / bound (<= 1 passes);
    # skipped under --profile so the traces hold only the timed calls
    err_over_bound = None
    if not args.profile:
        import numpy as np

        import oracle
        C1 = torch.from_numpy(C).to("cuda:0")
        mm.gemm(Ad, Bd, C1, alpha=1.0, beta=1.0, member=member, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        rng = np.random.Generator(np.random.PCG64(31))
        rows = np.concatenate([rng.integers(0, m, 256), [0, 0, m - 1, m - 1]])
        cols = np.concatenate([rng.integers(0, n, 256), [0, n - 1, 0, n - 1]])
        want = oracle.gemm_entries(A, B, rows, cols, C, 1.0, 1.0)
        absab = np.einsum("ij,ji->i", np.abs(A[rows]), np.abs(B[:, cols]))
        bound = 2.0 * (k + 2) * 2.0 ** -53 * (absab + np.abs(C[rows, cols]))
        got = C1.cpu().numpy()[rows, cols]
        err_over_bound = round(float(np.max(np.abs(got - want) / bound)), 4)
        del C1
    del A, B, C
    # The dominant kernel is the member's main kernel; a step is
    # plan["launches"] back-to-back launches of it (plus packing launches for
    # members that pack), so one launch takes ms / compute_launches.
    compute_launches = max(1, plan["launches"] // (2 if plan["pack"] and ws is not None else 1))
    launch_ms = ms / compute_launches
    achieved = (flops / compute_launches) / (launch_ms * 1e-3) / 1e12
    model = mm.model_bytes(member, m, n, k, beta=1.0, packed=ws is not None)
    traffic = None
    measured = None
    if os.path.exists(TRAFFIC_JSON):
        try:
            tj = json.load(open(TRAFFIC_JSON))
            rec = tj.get("members", {}).get(member)
            if rec and tj.get("size") == m and tj.get("kernel_source_sha") == kernel_source_sha():
                traffic = rec["bytes_per_launch"]
                measured = rec
        except (OSError, ValueError, KeyError):
            traffic = None
    res = {
        "value": round(flops / (ms * 1e-3) / 1e12, 3),
        "ms_per_step": round(ms, 4),
        "steps": steps,
        "warmup": warm,
        "wall_s_timed": round(wall, 3),
        "member": member,
        "launches_per_step": compute_launches,
        "max_err_over_bound_260_entries": err_over_bound,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_MFMA_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4), "traffic": traffic,
                     "model_bytes_per_launch": round((model["l2_read"] + model["l2_write"]) / compute_launches),
                     "launch_ms": round(launch_ms, 4), "flops_per_launch": flops / compute_launches},
        "model_bytes": {"l2_read": model["l2_read"], "l2_write": model["l2_write"], "hbm_read": model["hbm_read"],
                        "hbm_write": model["hbm_write"], "compulsory": model["compulsory"]},
    }
    if measured:
        res["measured_vs_model"] = {"measured_bytes": measured["bytes_per_call"],
                                    "model_bytes": model["l2_read"] + model["l2_write"],
                                    "ratio": round(measured["bytes_per_call"] /
                                                   (model["l2_read"] + model["l2_write"]), 3),
                                    "source": os.path.relpath(TRAFFIC_JSON, ROOT)}
    return res


def kernel_source_sha():
    """Hash of the FP64 kernel and planner sources (row-major and tiled)
    without their comments: stored traffic is only used while it matches."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("kernels_f64.hip", "gemm_f64.hip", "sched.h", "tiled.hip", "plan.cpp", "plan_internal.h"):
        with open(os.path.join(ROOT, "paper_1904_05717_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update(text.encode())
    return h.hexdigest()[:16]


def bench_split(args, fp64_ms=None):
    """Split-precision product at m = n = k = size on 16-decade data, for each
    configuration in --split: time, speedup over the FP64 product, rate of
    the low-precision slice products against their MFMA peak, and the error
    against the oracle on 256 sampled entries relative to (|A||B|)_ij."""
    import numpy as np
    import torch

    import oracle
    import paper_1904_05717_amd as mm
    import workloads

    m = n = k = args.size
    configs = [(c.split(":")[0], int(c.split(":")[1])) for c in args.split.split(",") if c]
    A, B, _ = workloads.gemm_operands(m, n, k, kind="loguniform", with_c=False)
    Ad, Bd = torch.from_numpy(A).to("cuda:0"), torch.from_numpy(B).to("cuda:0")
    C = torch.empty((m, n), dtype=torch.float64, device="cuda:0")
    ws_bytes = max(mm.split_workspace_size(m, n, k, S, t) for t, S in configs)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda:0")
    reps = 1 if args.profile else 3

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = events()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    if fp64_ms is None:
        member = mm.select_member(m, n, k)
        fp64_ms = timed(lambda: mm.gemm(Ad, Bd, C, member=member))
    rng = np.random.Generator(np.random.PCG64(2024))
    rows, cols = rng.integers(0, m, 256), rng.integers(0, n, 256)
    exact = oracle.gemm_entries(A, B, rows, cols)
    absab = np.einsum("ij,ji->i", np.abs(A[rows]), np.abs(B[:, cols]))
    runs = []
    for t, S in configs:
        ms = timed(lambda: mm.gemm_split(Ad, Bd, C, slices=S, slice_type=t, workspace=ws))
        got = C.cpu().numpy()[rows, cols]
        rel = np.abs(got - exact) / absab
        pairs = S if t == "crt" else S * (S + 1) // 2   # INT8 products: one per modulus, or the slice pairs
        lowp = pairs * 2.0 * m * n * k / (ms * 1e-3) / 1e12
        runs.append({"slice_type": t, "slices": S, "ms": round(ms, 3),
                     "speedup_vs_fp64": round(fp64_ms / ms, 3),
                     "fp64_equivalent_tflops": round(2.0 * m * n * k / (ms * 1e-3) / 1e12, 3),
                     "slice_products": pairs, "lowp_tops": round(lowp, 1),
                     "lowp_frac_of_peak": round(lowp / LOWP_MFMA_PEAK_TOPS[t], 4),
                     "max_rel_err_vs_absAB": float(rel.max()), "median_rel_err_vs_absAB": float(np.median(rel))})
    # Every entry, not a sample: against the 16-moduli modular product (t = 55
    # at k = 8192; its own error, sampled against the oracle above, is near
    # 1e-16 of |A||B|) with |A||B| from the FP64 product of the absolute values.
    full = None
    if not args.profile and mm.crt_bits(k, 16)[0] is not None:
        wsr = torch.empty(mm.split_workspace_size(m, n, k, 16, "crt"), dtype=torch.uint8, device="cuda:0")
        ref = mm.gemm_split(Ad, Bd, torch.empty_like(C), slices=16, slice_type="crt", workspace=wsr)
        del wsr
        absab_d = mm.gemm(Ad.abs(), Bd.abs(), torch.empty_like(C))
        ref_err = float((np.abs(ref[rows, cols].cpu().numpy() - exact) / absab).max())
        for r in runs:
            mm.gemm_split(Ad, Bd, C, slices=r["slices"], slice_type=r["slice_type"], workspace=ws)
            diff = (C - ref).abs_()
            r["max_rel_err_all_entries"] = float(torch.where(absab_d > 0, diff / absab_d, diff).max().item())
            del diff
        full = {"entries": m * n, "reference": "16-moduli modular product",
                "reference_max_rel_err_on_sample": ref_err}
        del ref, absab_d
    ok = [r for r in runs if r["max_rel_err_vs_absAB"] <= 1e-13 and r.get("max_rel_err_all_entries", 0.0) <= 1e-13]
    best = min(ok, key=lambda r: r["ms"]) if ok else None
    return {"workload": f"m=n=k={m}, sign uniform, magnitude 10^U(-8,8), beta=0",
            "fp64_ms": round(fp64_ms, 3), "runs": runs,
            "fastest_within_1e-13": None if best is None else {key: best[key] for key in (
                "slice_type", "slices", "ms", "speedup_vs_fp64", "max_rel_err_vs_absAB") + (
                ("max_rel_err_all_entries",) if "max_rel_err_all_entries" in best else ())},
            "error_sample": "256 entries against the compensated FP64 oracle",
            "error_all_entries": full}


def bench_tiled(args):
    """The register-resident members on tile-major ("prepacked") operands
    against the same members on row-major operands (bit-identical results),
    and the one-time conversion cost."""
    import torch

    import paper_1904_05717_amd as mm
    import workloads

    m = n = k = args.size
    A, B, C = workloads.gemm_operands(m, n, k)
    Ad, Bd, Cd = (torch.from_numpy(x).to("cuda:0") for x in (A, B, C))
    reps = 1 if args.profile else 5

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = events()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    At, Bt = mm.to_tiled(Ad, "A"), mm.to_tiled(Bd, "B")
    conv = timed(lambda: (mm.to_tiled(Ad, "A", out=At), mm.to_tiled(Bd, "B", out=Bt)))
    out = {"conversion_ms": round(conv, 3), "members": {}}
    for member in TILED_MEMBERS:
        wsb = mm.workspace_size(m, n, k, member)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda:0") if wsb else None
        row = timed(lambda: mm.gemm(Ad, Bd, Cd, 1.0, 1.0, member=member, workspace=ws))
        til = timed(lambda: mm.gemm_tiled(At, Bt, m, n, k, Cd, 1.0, 1.0, member=member))
        out["members"][member] = {"row_major_tflops": round(2.0 * m * n * k / row / 1e9, 2),
                                  "tiled_tflops": round(2.0 * m * n * k / til / 1e9, 2)}
    return out


def bench_syrk(args):
    """Symmetric rank-k update C := X X^T on the lower triangle at n = k = size
    (C3C0 order, tiles above the diagonal skipped) against the full product
    X X^T by the same member; rate in n (n + 1) k flops per second."""
    import torch

    import paper_1904_05717_amd as mm
    import workloads

    n = k = args.size
    X = torch.from_numpy(workloads.uniform((n, k), 26)).to("cuda:0")
    Xt = X.t().contiguous()
    C = torch.zeros((n, n), dtype=torch.float64, device="cuda:0")
    reps = 1 if args.profile else 5

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = events()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_syrk = timed(lambda: mm.syrk(X, C, 1.0, 0.0, uplo="L", member="C3C0"))
    t_gemm = timed(lambda: mm.gemm(X, Xt, C, 1.0, 0.0, member="C3C0"))
    return {"n": n, "k": k, "syrk_ms": round(t_syrk, 3),
            "syrk_tflops": round(n * (n + 1) * k / t_syrk / 1e9, 2),
            "full_product_ms": round(t_gemm, 3), "full_product_tflops": round(2.0 * n * n * k / t_gemm / 1e9, 2),
            "time_ratio": round(t_syrk / t_gemm, 3)}


def bench_ooc(args):
    """Out-of-core product at m = n = k = 2 * size with A, B, C in pinned host
    memory: Resident C blocks in device memory, A and B panels over PCIe.
    Wall time around the whole call (copies in both directions included),
    rate in 2mnk flops per second, the host traffic of the Resident C count
    and the rate it moves at, and the plain pinned host-to-device copy rate
    for context."""
    import time

    import numpy as np
    import torch

    import oracle
    import paper_1904_05717_amd as mm
    import workloads

    m = n = k = 2 * args.size
    A, B, C = workloads.gemm_operands(m, n, k)
    Ah, Bh = torch.from_numpy(A).pin_memory(), torch.from_numpy(B).pin_memory()
    C0 = torch.from_numpy(C).pin_memory()
    del A, B, C
    Ch = torch.empty_like(C0).pin_memory()
    probe = torch.empty(1 << 28, dtype=torch.float64, device="cuda:0")
    src = torch.empty(1 << 28, dtype=torch.float64).pin_memory()
    probe.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    probe.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    h2d = src.numel() * 8 / (time.perf_counter() - t0) / 1e9
    del probe, src
    runs = []
    for block in ((m, n, 2048), (m // 2, n, 2048), (m // 2, n // 2, 2048)):
        mb, nb, kb = block
        ws = torch.empty(mm.ooc_workspace_size(mb, nb, kb), dtype=torch.uint8, device="cuda:0")
        cs = torch.cuda.Stream()
        times = []
        for _ in range(1 if args.profile else 2):
            Ch.copy_(C0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mm.gemm_ooc(Ah, Bh, Ch, alpha=1.0, beta=1.0, block=block, workspace=ws, copy_stream=cs)
            times.append(time.perf_counter() - t0)
        t = min(times)
        host_bytes = 8 * (2 * m * n + m * k * -(-n // nb) + k * n * -(-m // mb))
        runs.append({"block": list(block), "workspace_gib": round(ws.numel() / 2 ** 30, 2), "s": round(t, 4),
                     "tflops_pcie_inclusive": round(2.0 * m * n * k / t / 1e12, 2),
                     "host_gb": round(host_bytes / 1e9, 2), "host_gb_per_s": round(host_bytes / t / 1e9, 1)})
        del ws
    rng = np.random.Generator(np.random.PCG64(12))
    rows, cols = rng.integers(0, m, 32), rng.integers(0, n, 32)
    want = oracle.gemm_entries(Ah.numpy(), Bh.numpy(), rows, cols, C0.numpy(), 1.0, 1.0)
    absab = np.einsum("ij,ji->i", np.abs(Ah.numpy()[rows]), np.abs(Bh.numpy()[:, cols]))
    err = np.abs(Ch.numpy()[rows, cols] - want) / (absab + np.abs(C0.numpy()[rows, cols]))
    return {"m": m, "n": n, "k": k, "operands": "pinned host memory", "runs": runs,
            "pinned_h2d_copy_gb_per_s": round(h2d, 1), "max_rel_err_32_entries": float(err.max())}


def bench_tri(args):
    """Triangular solve and multiply with m = n = size (lower triangle, no
    transposition, well-conditioned T), rate in m^2 n flops per second; the
    Cholesky factorization of an SPD matrix of order size (n^3 / 3 flops);
    the full product of the same shape beside them."""
    import numpy as np
    import torch

    import paper_1904_05717_amd as mm
    import workloads

    m = n = args.size
    A = workloads.uniform((m, m), 27) / np.sqrt(m)
    A[np.diag_indices(m)] = 1.5
    Ad = torch.from_numpy(A).to("cuda:0")
    B0 = torch.from_numpy(workloads.uniform((m, n), 28)).to("cuda:0")
    B = torch.empty_like(B0)
    C = torch.empty_like(B0)
    reps = 1 if args.profile else 5

    def timed(fn, prep=None):
        if prep:
            prep()
        fn()
        torch.cuda.synchronize()
        total = 0.0
        for _ in range(reps):
            if prep:
                prep()
            e0, e1 = events()
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            total += e0.elapsed_time(e1)
        return total / reps

    S0 = torch.from_numpy(workloads.uniform((m, m), 29) / np.sqrt(m)).to("cuda:0")
    S0 = S0 @ S0.t() + torch.eye(m, dtype=torch.float64, device="cuda:0")   # SPD, well conditioned
    S = torch.empty_like(S0)
    t_potrf = timed(lambda: mm.potrf(S), prep=lambda: S.copy_(S0))
    del S, S0
    t_trsm = timed(lambda: mm.trsm(Ad, B, uplo="L"), prep=lambda: B.copy_(B0))
    t_trmm = timed(lambda: mm.trmm(Ad, B0, C, uplo="L"))
    t_gemm = timed(lambda: mm.gemm(Ad, B0, C))
    flops = float(m) * m * n
    return {"m": m, "n": n, "trsm_ms": round(t_trsm, 3), "trsm_tflops": round(flops / t_trsm / 1e9, 2),
            "trmm_ms": round(t_trmm, 3), "trmm_tflops": round(flops / t_trmm / 1e9, 2),
            "potrf_ms": round(t_potrf, 3), "potrf_tflops": round(m ** 3 / 3.0 / t_potrf / 1e9, 2),
            "full_product_ms": round(t_gemm, 3), "full_product_tflops": round(2 * flops / t_gemm / 1e9, 2)}


def bench_batch(args):
    """512 uneven problems (config 4) in one persistent hipGraph-replayed
    launch: the planner's per-problem choice (AUTO) against fixed choices of
    member and register tile for the whole batch.  Median of the replays;
    padding = flops of the padded tiles / algorithmic flops."""
    import torch

    import paper_1904_05717_amd as mm
    import workloads

    shapes = workloads.batch_shapes(512)
    dev = []
    for i, (m, n, k) in enumerate(shapes):
        dev.append((torch.from_numpy(workloads.uniform((m, k), 3 * i)).to("cuda:0"),
                    torch.from_numpy(workloads.uniform((k, n), 3 * i + 1)).to("cuda:0"),
                    torch.from_numpy(workloads.uniform((m, n), 3 * i + 2)).to("cuda:0")))
    probs = [(A, B, C, 1.0, 1.0) for (A, B, C) in dev]
    reps = 2 if args.profile else 20
    choices = [("AUTO", None, None), ("C0", "C0", None), ("C3C0", "C3C0", None), ("C0/128", "C0", 128),
               ("C0/64", "C0", 64), ("B3C0", "B3C0", None), ("A3C0", "A3C0", None)]
    runs = {}
    auto_info = None
    for label, member, tile in (choices[:1] if args.profile else choices):
        plan = mm.BatchPlan(probs, members=member, tiles=tile)
        info = plan.info()
        plan.run()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            e0, e1 = events()
            e0.record()
            plan.run()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        plan.close()
        ms = sorted(times)[len(times) // 2]
        runs[label] = {"ms_per_replay": round(ms, 3), "tflops": round(info["flops"] / (ms * 1e-3) / 1e12, 3),
                       "padding_ratio": round(info["padded_flops"] / info["flops"], 3),
                       "split_problems": sum(1 for c in info["chunks"] if c > 1)}
        if label == "AUTO":
            auto_info = info
    auto = runs["AUTO"]
    fixed = {key: v for key, v in runs.items() if key != "AUTO"}
    best_fixed = min(fixed, key=lambda key: fixed[key]["ms_per_replay"]) if fixed else None
    counts = {}
    for mem, t, c in zip(auto_info["members"], auto_info["tiles"], auto_info["chunks"]):
        key = f"{mem}/{t}" + ("/split" if c > 1 else "")
        counts[key] = counts.get(key, 0) + 1
    return {"problems": 512, "ms_per_replay": auto["ms_per_replay"], "tflops": auto["tflops"],
            "frac_fp64_peak": round(auto["tflops"] / FP64_MFMA_PEAK_TFLOPS, 4),
            "padding_ratio": auto["padding_ratio"], "members": counts,
            "items": auto_info["items"], "persistent_workgroups": auto_info["workgroups"],
            "best_fixed_choice": best_fixed,
            "auto_over_best_fixed": (round(auto["ms_per_replay"] / fixed[best_fixed]["ms_per_replay"], 3)
                                     if best_fixed else None),
            "choices": runs, "graph": "hipGraph replay", "timing": f"median of {reps} replays",
            "shapes": "m, n, k each round(exp(U(ln 32, ln 2048)))"}


def bench_backward(args):
    import torch

    import workloads
    from paper_1904_05717_amd.autograd import matmul

    m, k, n = 4096, 8192, 2048
    out = {}
    for dt in (torch.float64, torch.float32):
        A = torch.from_numpy(workloads.uniform((m, k), workloads.SEED_A)).to("cuda:0", dt).requires_grad_()
        B = torch.from_numpy(workloads.uniform((k, n), workloads.SEED_B)).to("cuda:0", dt).requires_grad_()
        dC = torch.from_numpy(workloads.normal((m, n), workloads.SEED_DC)).to("cuda:0", dt)
        C = matmul(A, B)
        C.backward(dC)
        torch.cuda.synchronize()
        reps = 1 if args.profile else 3
        f0, f1 = events()
        b1 = torch.cuda.Event(enable_timing=True)
        tot = [0.0, 0.0]
        for _ in range(reps):
            A.grad = None
            B.grad = None
            f0.record()
            C = matmul(A, B)
            f1.record()
            C.backward(dC)
            b1.record()
            torch.cuda.synchronize()
            tot[0] += f0.elapsed_time(f1)
            tot[1] += f1.elapsed_time(b1)
        fwd, bwd = tot[0] / reps, tot[1] / reps
        flops = 2.0 * m * n * k
        out["f64" if dt == torch.float64 else "f32_split3"] = {
            "fwd_ms": round(fwd, 3), "bwd_ms": round(bwd, 3),
            "tflops_fwd_bwd": round(3 * flops / ((fwd + bwd) * 1e-3) / 1e12, 3)}
    out["shape"] = {"m": m, "k": k, "n": n}
    return out


def bench_members(args):
    import torch

    import paper_1904_05717_amd as mm
    import workloads

    m = n = k = args.size
    A, B, C = workloads.gemm_operands(m, n, k)
    Ad, Bd, Cd = (torch.from_numpy(x).to("cuda:0") for x in (A, B, C))
    del A, B, C
    res = {}
    for member in mm.FAMILY:
        wsb = mm.workspace_size(m, n, k, member)
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda:0") if wsb else None
        mm.gemm(Ad, Bd, Cd, 1.0, 1.0, member=member, workspace=ws)
        torch.cuda.synchronize()
        e0, e1 = events()
        e0.record()
        mm.gemm(Ad, Bd, Cd, 1.0, 1.0, member=member, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        res[member] = {"ms": round(ms, 3), "tflops": round(2.0 * m * n * k / (ms * 1e-3) / 1e12, 2)}
    return res


LOWBW_SHAPES = [(4096, 4096, 4096), (8192, 8192, 8192), (16384, 16384, 256), (16384, 256, 16384)]
LOWBW_WIDTHS = [32, 64, 128]
LOWBW_CURVE = {"size": 8192, "members": ["A2C0", "B3A2C0", "C4A2C0", "C3C0"], "widths": [16, 48, 96, 160, 192]}


def bench_lowbw(args):
    """Low-bandwidth emulation (the varying-bandwidth experiments of Sec. 5).
    Every family member runs alone, beside the streaming kernel on G whole
    compute units, and beside its sleeping control on the same G compute
    units (G = 32, 64, 128; both reserve the units the same way).  The
    control's time is the member on 256 - G compute units at full bandwidth;
    stream / sleep is what the bandwidth taken costs it.  The streamer's own
    rate is measured alone (20 ms) and over each run.  Best of two calls per
    condition; hipEvents on the product's stream.  `curve`: Goto, B3A2C0,
    C4A2C0 and C3C0 at 8192^3 over more streamer widths (one streaming call
    each at the extra widths), the analogue of the paper's performance
    against bandwidth."""
    import time

    import torch

    import paper_1904_05717_amd as mm
    import workloads

    dev = torch.device("cuda:0")
    hog_stream = torch.cuda.Stream(device=dev)
    reps = 1 if args.profile else 2
    hogs = {}
    alone_rate = {}
    for g in LOWBW_WIDTHS:
        hogs[(g, "sleep")] = mm.BandwidthHog(g, "sleep", device=dev, stream=hog_stream)
        hogs[(g, "stream")] = mm.BandwidthHog(g, "stream", nbytes=4 << 30, device=dev, stream=hog_stream)
    s = hogs[(LOWBW_WIDTHS[0], "sleep")].concurrent_stream()   # a product stream on another hardware queue
    for g in LOWBW_WIDTHS:
        h = hogs[(g, "stream")]
        h.start(max_seconds=5.0)
        time.sleep(0.02)
        h.stop(s)
        alone_rate[g] = round(h.report()["GBps"], 1)

    def run(member, A, B, C, ws, hog):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if hog is not None:
            hog.start(max_seconds=2.0)
            time.sleep(0.005)
        try:
            with torch.cuda.stream(s):
                if hog is not None:
                    hog.mark(s)
                e0.record(s)
                mm.gemm(A, B, C, 1.0, 1.0, member=member, workspace=ws, stream=s)
                e1.record(s)
        finally:
            if hog is not None:
                hog.stop(s)
        rep = hog.report() if hog is not None else None
        s.synchronize()
        if rep is not None and not (rep["covered"] and not rep["timed_out"]):
            # the streamer did not run beside the product: stop here rather than wait out its clock every run
            raise RuntimeError(f"streamer and product did not overlap: {rep}")
        return e0.elapsed_time(e1), rep

    out = {"widths": LOWBW_WIDTHS, "streamer_alone_GBps": alone_rate, "shapes": []}
    curve = {}   # member -> width -> (sleep_ms, stream_ms, streamer GB/s), filled at the curve's size
    for (m, n, k) in LOWBW_SHAPES:
        A, B, C = workloads.gemm_operands(m, n, k)
        Ad, Bd, Cd = (torch.from_numpy(x).to(dev) for x in (A, B, C))
        del A, B, C
        flops = 2.0 * m * n * k
        rows = {}
        for member in mm.FAMILY:
            wsb = mm.workspace_size(m, n, k, member)
            ws = torch.empty(wsb, dtype=torch.uint8, device=dev) if wsb else None
            run(member, Ad, Bd, Cd, ws, None)
            row = {"alone_ms": round(min(run(member, Ad, Bd, Cd, ws, None)[0] for _ in range(reps)), 3)}
            for g in LOWBW_WIDTHS:
                t_sleep = min(run(member, Ad, Bd, Cd, ws, hogs[(g, "sleep")])[0] for _ in range(reps))
                best, rate, covered = None, None, True
                for _ in range(reps):
                    t, rep = run(member, Ad, Bd, Cd, ws, hogs[(g, "stream")])
                    covered = covered and rep["covered"] and not rep["timed_out"]
                    if best is None or t < best:
                        best, rate = t, rep["GBps"]
                row[str(g)] = {"sleep_ms": round(t_sleep, 3), "stream_ms": round(best, 3),
                               "slowdown": round(best / t_sleep, 3),
                               "tflops_stream": round(flops / (best * 1e-3) / 1e12, 2),
                               "streamer_GBps": round(rate, 1), "covered": covered}
            if (m, n, k) == (LOWBW_CURVE["size"],) * 3 and member in LOWBW_CURVE["members"]:
                pts = {}
                for g in LOWBW_CURVE["widths"]:
                    hs = mm.BandwidthHog(g, "sleep", device=dev, stream=hog_stream)
                    hr = mm.BandwidthHog(g, "stream", nbytes=4 << 30, device=dev, stream=hog_stream)
                    t_sleep = min(run(member, Ad, Bd, Cd, ws, hs)[0] for _ in range(reps))
                    t, rep = run(member, Ad, Bd, Cd, ws, hr)
                    pts[str(g)] = {"sleep_ms": round(t_sleep, 3), "stream_ms": round(t, 3),
                                   "slowdown": round(t / t_sleep, 3), "streamer_GBps": round(rep["GBps"], 1),
                                   "covered": rep["covered"] and not rep["timed_out"]}
                    del hs, hr
                for g in LOWBW_WIDTHS:
                    pts[str(g)] = {key: row[str(g)][key] for key in ("sleep_ms", "stream_ms", "slowdown",
                                                                      "streamer_GBps", "covered")}
                curve[member] = {str(g): pts[str(g)] for g in sorted(int(x) for x in pts)}
            mb = mm.model_bytes(member, m, n, k, beta=1.0)
            row["model_hbm_gb"] = round((mb["hbm_read"] + mb["hbm_write"]) / 1e9, 2)
            row["model_l2_gb"] = round((mb["l2_read"] + mb["l2_write"]) / 1e9, 2)
            rows[member] = row
            del ws
        order = {"alone": sorted(rows, key=lambda x: rows[x]["alone_ms"])[:3]}
        for g in LOWBW_WIDTHS:
            order[f"sleep_{g}"] = sorted(rows, key=lambda x: rows[x][str(g)]["sleep_ms"])[:3]
            order[f"stream_{g}"] = sorted(rows, key=lambda x: rows[x][str(g)]["stream_ms"])[:3]
        out["shapes"].append({"m": m, "n": n, "k": k, "members": rows, "fastest_three": order})
        if curve and "curve" not in out:
            out["curve"] = {"m": m, "n": n, "k": k, "members": curve}
        del Ad, Bd, Cd
        torch.cuda.empty_cache()
    return out


SWEEP_SHAPES = [(1024, 1024, 1024), (2048, 2048, 2048), (4096, 4096, 4096), (8192, 8192, 8192),
                (16384, 16384, 16384), (16384, 16384, 256), (16384, 256, 16384)]


def bench_sweep(args):
    """The FP64 sweep: square sizes 1024 .. 16384, the rank-k update
    16384 x 16384 x 256 and the panel-panel product 16384 x 256 x 16384
    (U[-1,1], beta = 1).  Every member timed as the member tuner times it
    (the fastest of three batch means, batches of back-to-back calls at least
    2 ms long, the rounds visiting the members in turn); the member AUTO
    picks; measured L2 traffic against the model where a stored traffic
    profile of the same shape and kernels exists."""
    import torch

    import paper_1904_05717_amd as mm
    import workloads
    from paper_1904_05717_amd import tuner

    out = []
    for (m, n, k) in SWEEP_SHAPES:
        A, B, C = workloads.gemm_operands(m, n, k)
        Ad, Bd, Cd = (torch.from_numpy(x).to("cuda:0") for x in (A, B, C))
        del A, B, C
        traffic = {}
        tj_path = os.path.join(ROOT, "profiles", f"traffic_f64_{shape_tag(m, n, k)}.json")
        try:
            tj = json.load(open(tj_path))
            if tj.get("kernel_source_sha") == kernel_source_sha():
                traffic = {mem: round(r["ratio"], 3) for mem, r in tj["members"].items()}
        except (OSError, ValueError, KeyError):
            pass
        members = {}
        for member, ms in tuner.time_members(mm, Ad, Bd, Cd, mm.FAMILY).items():
            members[member] = {"ms": round(ms, 4), "tflops": round(2.0 * m * n * k / (ms * 1e-3) / 1e12, 2)}
            if member in traffic:
                members[member]["traffic_vs_model"] = traffic[member]
        best = max(members, key=lambda x: members[x]["tflops"])
        out.append({"m": m, "n": n, "k": k, "auto": mm.select_member(m, n, k), "best": best,
                    "best_tflops": members[best]["tflops"], "members": members})
        del Ad, Bd, Cd
        torch.cuda.empty_cache()
    return out


def _csv_rows(path):
    import csv
    with open(path) as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def summarize(d, m=8192, n=8192, k=8192):
    """Profiles from a pass with these rocprofv3 runs (all from /tmp, TMPDIR=/tmp):
      kt_bench:      rocprofv3 --kernel-trace --stats -- python3 bench.py --profile
      fetch_members: rocprofv3 --pmc FETCH_SIZE -- python3 bench.py --profile-members
      write_members: rocprofv3 --pmc WRITE_SIZE -- python3 bench.py --profile-members
      fetch_copy / write_copy: the same counters for bench.py --copy-calibration
    Each member runs once after a warm-up, between two marker fills; the
    dispatches between the first and second fill are its measured call.
    """
    import paper_1904_05717_amd as mm

    def segments(rows):
        segs, cur = [], []
        for r in rows:
            if "FillFunctor" in r["Kernel_Name"]:
                segs.append(cur)
                cur = []
            else:
                cur.append(r)
        segs.append(cur)
        return segs

    def copy_scale(sub, counter):
        rows = [r for r in _csv_rows(os.path.join(d, sub, "run_counter_collection.csv"))
                if "copyBuffer" in r["Kernel_Name"] or "elementwise" in r["Kernel_Name"] and "copy" in
                r["Kernel_Name"].lower()]
        vals = [float(r["Counter_Value"]) * 1024.0 for r in rows if r["Counter_Name"] == counter]
        known = 8.0 * (1 << 27)
        return known / (sum(vals) / len(vals)), vals

    fscale, fvals = copy_scale("fetch_copy", "FETCH_SIZE")
    wscale, wvals = copy_scale("write_copy", "WRITE_SIZE")
    F = segments(_csv_rows(os.path.join(d, "fetch_members", "run_counter_collection.csv")))
    W = segments(_csv_rows(os.path.join(d, "write_members", "run_counter_collection.csv")))
    members = {}
    for i, member in enumerate(mm.FAMILY):
        fr = [r for r in F[2 * i + 1] if "momms" in r["Kernel_Name"]]
        wr = [r for r in W[2 * i + 1] if "momms" in r["Kernel_Name"]]
        fb = sum(float(r["Counter_Value"]) for r in fr) * 1024.0 * fscale
        wb = sum(float(r["Counter_Value"]) for r in wr) * 1024.0 * wscale
        plan = mm.member_plan(member, m, n, k)
        launches = len([r for r in fr if "k_pack" not in r["Kernel_Name"]])
        model = mm.model_bytes(member, m, n, k, beta=1.0, packed=plan["pack"] == 1)
        mb = model["l2_read"] + model["l2_write"] + model["pack"]
        members[member] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_call": fb + wb,
                           "launches": launches, "bytes_per_launch": (fb + wb) / max(1, launches),
                           "model_bytes": mb, "ratio": (fb + wb) / mb}
    # tiled runs follow after one more marker fill: segments 2 * len(FAMILY) + 1 + 2 i + 1
    base = 2 * len(mm.FAMILY) + 1
    for i, member in enumerate(TILED_MEMBERS):
        if base + 2 * i + 1 >= min(len(F), len(W)):
            break
        fr = [r for r in F[base + 2 * i + 1] if "momms" in r["Kernel_Name"]]
        wr = [r for r in W[base + 2 * i + 1] if "momms" in r["Kernel_Name"]]
        fb = sum(float(r["Counter_Value"]) for r in fr) * 1024.0 * fscale
        wb = sum(float(r["Counter_Value"]) for r in wr) * 1024.0 * wscale
        model = mm.model_bytes(member, m, n, k, beta=1.0, packed=False)
        mb = model["l2_read"] + model["l2_write"]
        members[member + "/tiled"] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_call": fb + wb,
                                      "launches": len(fr), "bytes_per_launch": (fb + wb) / max(1, len(fr)),
                                      "model_bytes": mb, "ratio": (fb + wb) / mb}
    tag = shape_tag(m, n, k)
    sel = f"--size {m}" if m == n == k else f"--shape {m},{n},{k}"
    out = {"size": m if m == n == k else None, "shape": [m, n, k], "kernel_source_sha": kernel_source_sha(),
           "fetch_scale": fscale, "write_scale": wscale,
           "copy_fetch_bytes": fvals, "copy_write_bytes": wvals, "members": members}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"traffic_f64_{tag}.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    lines = [f"# L2-to-fabric traffic of every family member, FP64 m={m}, n={n}, k={k}", "",
             "Commands (run from /tmp with TMPDIR=/tmp; repo at /root/repo):", "",
             "    rocprofv3 --pmc FETCH_SIZE -d <dir>/fetch_members -o run --output-format csv -- "
             f"python3 /root/repo/bench.py --profile-members {sel}",
             "    rocprofv3 --pmc WRITE_SIZE -d <dir>/write_members -o run --output-format csv -- "
             f"python3 /root/repo/bench.py --profile-members {sel}",
             "    rocprofv3 --pmc FETCH_SIZE -d <dir>/fetch_copy -o run --output-format csv -- "
             "python3 /root/repo/bench.py --copy-calibration",
             "    rocprofv3 --pmc WRITE_SIZE -d <dir>/write_copy -o run --output-format csv -- "
             "python3 /root/repo/bench.py --copy-calibration",
             f"    python3 bench.py --summarize <dir> {sel}", "",
             f"Calibration on a plain 1 GiB device copy: FETCH_SIZE reads {1/fscale:.4f} of the bytes copied "
             f"(scale {fscale:.4f}), WRITE_SIZE {1/wscale:.4f} (scale {wscale:.4f}).", "",
             "| member | launches | fetch GB | write GB | measured GB | model GB | measured / model |",
             "|---|---|---|---|---|---|---|"]
    for member, r in members.items():
        lines.append(f"| {member} | {r['launches']} | {r['fetch_bytes']/1e9:.2f} | {r['write_bytes']/1e9:.2f} | "
                     f"{r['bytes_per_call']/1e9:.2f} | {r['model_bytes']/1e9:.2f} | {r['ratio']:.2f} |")
    lines += ["", "Model: the library's momms_model_bytes (ideal residency at the boundary between the "
              "per-XCD L2s and the fabric; packing included for members that pack).  `/tiled` rows run the "
              "member on tile-major (\"prepacked\") operands (momms_gemm_tiled); the conversion is outside the "
              "measured call.", ""]
    with open(os.path.join(ROOT, "profiles", f"traffic_f64_{tag}.md"), "w") as fh:
        fh.write("\n".join(lines))
    ks = os.path.join(d, "kt_bench", "run_kernel_stats.csv")
    if os.path.exists(ks) and m == n == k:
        size = m
        import csv
        with open(ks) as fh:
            rows = list(csv.DictReader(fh))
        lines = [f"# Kernel trace of the FP64 benchmark step (m=n=k={size}, selected member)", "",
                 "    rocprofv3 --kernel-trace --stats -d <dir>/kt_bench -o run --output-format csv -- "
                 "python3 /root/repo/bench.py --profile", "",
                 "| kernel | calls | average ns | min ns | max ns | share |", "|---|---|---|---|---|---|"]
        for r in rows:
            name = r["Name"].split("(")[0][:90]
            lines.append(f"| {name} | {r['Calls']} | {float(r['AverageNs']):.0f} | {r['MinNs']} | {r['MaxNs']} | "
                         f"{float(r['Percentage']):.1f} % |")
        with open(os.path.join(ROOT, "profiles", f"kernel_stats_f64_{size}.md"), "w") as fh:
            fh.write("\n".join(lines) + "\n")
    print(json.dumps({"summarized": d, "members": {k: round(v["ratio"], 3) for k, v in members.items()}}))


def _split_summary(sp):
    """Fastest split configuration within 1e-13 of |A||B|, and per slice type
    the fastest such configuration (else the most accurate one)."""
    runs = sp.get("runs", [])

    def ok(r):
        return r["max_rel_err_vs_absAB"] <= 1e-13 and r.get("max_rel_err_all_entries", 0.0) <= 1e-13

    def short(r):
        return {"slices": r["slices"], "ms": r["ms"], "speedup_vs_fp64": r["speedup_vs_fp64"],
                "max_rel_err": float(f"{max(r['max_rel_err_vs_absAB'], r.get('max_rel_err_all_entries', 0.0)):.3g}"),
                "lowp_frac_of_peak": r["lowp_frac_of_peak"], "within_1e-13": ok(r)}

    out = {"fp64_ms": sp.get("fp64_ms")}
    best = sp.get("fastest_within_1e-13")
    out["fastest_within_1e-13"] = None if best is None else {
        "slice_type": best["slice_type"], "slices": best["slices"], "ms": best["ms"],
        "speedup_vs_fp64": best["speedup_vs_fp64"]}
    for t in ("crt", "int8", "bf16", "fp8"):
        rs = [r for r in runs if r["slice_type"] == t]
        if not rs:
            continue
        good = [r for r in rs if ok(r)]
        r = min(good, key=lambda x: x["ms"]) if good else min(rs, key=lambda x: x["max_rel_err_vs_absAB"])
        out[t] = short(r)
    return out


def compact_line(out):
    """The final stdout line: the headline and a short summary of every
    section (the full sections are printed on earlier lines, and written to
    --full-json when given)."""
    keep = ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
            "vs_baseline", "dtype", "data", "config", "roofline", "max_err_over_bound_260_entries",
            "measured_vs_model", "cpu_baseline"]
    line = {k: out[k] for k in keep if k in out}
    if "split_precision" in out:
        line["split"] = _split_summary(out["split_precision"])
    if "batched" in out:
        b = out["batched"]
        line["batched"] = {key: b[key] for key in ("ms_per_replay", "tflops", "frac_fp64_peak", "padding_ratio",
                                                   "members", "best_fixed_choice", "auto_over_best_fixed")
                           if key in b}
    if "backward" in out:
        line["backward_tflops"] = {key: v["tflops_fwd_bwd"] for key, v in out["backward"].items()
                                   if isinstance(v, dict) and "tflops_fwd_bwd" in v}
    if "sweep" in out:
        line["sweep_best_tflops"] = {f"{r['m']}x{r['n']}x{r['k']}": [r["best"], r["best_tflops"], r["auto"]]
                                     for r in out["sweep"]}
    return line


def main():
    args = parse()
    if args.summarize:
        summarize(args.summarize, *shape_of(args))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.profile_members:
        profile_members(*shape_of(args))
        return
    only = "fp64" if (args.profile and args.only == "all") else args.only
    if only in ("split", "batch", "backward", "members", "tiled", "syrk", "tri", "ooc", "sweep", "lowbw"):
        fn = {"split": bench_split, "batch": bench_batch, "backward": bench_backward, "members": bench_members,
              "tiled": bench_tiled, "syrk": bench_syrk, "tri": bench_tri, "ooc": bench_ooc,
              "sweep": bench_sweep, "lowbw": bench_lowbw}[only]
        print(json.dumps({only: fn(args)}), flush=True)
        return
    f = bench_fp64(args)
    out = {
        "metric": "FP64 GEMM TFLOP/s + % MFMA peak; HBM bytes vs model; split-prec speedup",
        "value": f["value"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": f["steps"],
        "warmup": f["warmup"],
        "ms_per_step": f["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"fp64 gemm C+=A*B m=n=k={args.size} row-major, U[-1,1] entries, beta=1",
                   "member": f["member"], "m": args.size, "n": args.size, "k": args.size},
        "roofline": f["roofline"],
        "frac_fp64_mfma_peak": round(f["value"] / FP64_MFMA_PEAK_TFLOPS, 4),
        "model_bytes": f["model_bytes"],
        "wall_s_timed": f["wall_s_timed"],
    }
    if "measured_vs_model" in f:
        out["measured_vs_model"] = f["measured_vs_model"]
    out["max_err_over_bound_260_entries"] = f["max_err_over_bound_260_entries"]
    print(json.dumps({"section": "fp64", "result": f}), flush=True)
    if only == "all":
        sections = [("split_precision", lambda: bench_split(args, fp64_ms=f["ms_per_step"])),
                    ("batched", lambda: bench_batch(args)), ("backward", lambda: bench_backward(args)),
                    ("sweep", lambda: bench_sweep(args)), ("tiled_storage", lambda: bench_tiled(args)),
                    ("syrk", lambda: bench_syrk(args)), ("triangular", lambda: bench_tri(args)),
                    ("out_of_core", lambda: bench_ooc(args)), ("low_bandwidth", lambda: bench_lowbw(args))]
        for name, fn in sections:
            try:
                out[name] = fn()
            except Exception as exc:   # a failed section reports itself; the headline still stands
                if name != "low_bandwidth":
                    raise
                out[name] = {"error": repr(exc)}
            print(json.dumps({"section": name, "result": out[name]}), flush=True)
    if not args.no_cpu and not args.profile:
        out["cpu_baseline"] = cpu_baseline(args.size, args.size, args.size, args.cpu_seconds)
    if args.full_json:
        with open(args.full_json, "w") as fh:
            json.dump(out, fh)
    print(json.dumps(compact_line(out)), flush=True)


if __name__ == "__main__":
    main()
