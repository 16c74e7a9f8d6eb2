"""Measured half of the member autotuner.

`sweep` times every family member on the device for a list of shapes and
returns, per shape bucket (rounded log2 of m, n, k), the fastest member.
`save` writes that table as JSON, with a hash of the FP64 kernel and planner
sources it was measured on; `install` loads a table into the library
(momms_set_member_table), after which MOMMS_AUTO uses it before the analytic
prior, but only while that hash matches the sources next to the built
library (otherwise the prior decides).  The package installs
tuned_members.json (next to this file) at import when it exists.

    python -c "from paper_1904_05717_amd import tuner; tuner.main()"   # on the GPU
"""
import ctypes
import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuned_members.json")
# The sources whose code decides a member's speed: its kernels, its launch
# sequence and its plan.
SOURCES = ("kernels_f64.hip", "gemm_f64.hip", "sched.h", "plan.cpp", "plan_internal.h")


def source_sha(files=SOURCES):
    """Hash of the given csrc files with their comments stripped."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update(text.encode())
    return h.hexdigest()[:16]

SWEEP_SHAPES = [(1024, 1024, 1024), (2048, 2048, 2048), (4096, 4096, 4096), (8192, 8192, 8192),
                (16384, 16384, 256), (16384, 256, 16384), (4096, 8192, 2048), (4096, 2048, 4096),
                (8192, 2048, 4096)]


def bucket(m, n, k):
    return tuple(0 if x <= 1 else int(round(math.log2(x))) for x in (m, n, k))


def time_member(mm, A, B, C, member, reps=3):
    import torch
    m, k = A.shape
    n = B.shape[1]
    wsb = mm.workspace_size(m, n, k, member)
    ws = torch.empty(wsb, dtype=torch.uint8, device=A.device) if wsb else None
    mm.gemm(A, B, C, 1.0, 1.0, member=member, workspace=ws)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        mm.gemm(A, B, C, 1.0, 1.0, member=member, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def time_members(mm, A, B, C, members, min_ms=2.0, rounds=3):
    """Milliseconds per call of each member: the fastest of `rounds` batch
    means, a batch being enough back-to-back calls to last about min_ms (one
    call when a call is longer).  The rounds visit the members in turn, so a
    drift of the clock or of the other load on the device touches every
    member alike, and short calls are timed over many launches."""
    import torch
    m, k = A.shape
    n = B.shape[1]
    ws, reps, best = {}, {}, {}
    for mem in members:
        wsb = mm.workspace_size(m, n, k, mem)
        ws[mem] = torch.empty(wsb, dtype=torch.uint8, device=A.device) if wsb else None
        mm.gemm(A, B, C, 1.0, 1.0, member=mem, workspace=ws[mem])   # warm-up
        torch.cuda.synchronize()
        one = _batch(mm, A, B, C, mem, ws[mem], 1)
        reps[mem] = max(1, min(200, int(math.ceil(min_ms / max(one, 1e-3)))))
        best[mem] = float("inf")
    for _ in range(rounds):
        for mem in members:
            best[mem] = min(best[mem], _batch(mm, A, B, C, mem, ws[mem], reps[mem]))
    return best


def _batch(mm, A, B, C, member, ws, reps):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        mm.gemm(A, B, C, 1.0, 1.0, member=member, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


TIE = 0.01


def pick(mm, m, n, k, times):
    """Fastest member; members within 1% of it tie.  A tie goes to the
    analytic prior's choice when it is among the tied members, else to fewer
    model bytes, then the lower member id."""
    fastest = min(times.values())
    tied = [mem for mem, t in times.items() if t <= fastest * (1.0 + TIE)]
    prior = mm.MEMBER_NAMES[mm._lib.momms_select_member_prior(m, n, k)]
    if prior in tied:
        return prior

    def key(mem):
        b = mm.model_bytes(mem, m, n, k, beta=1.0)
        return (b["l2_read"] + b["l2_write"], mm.MEMBERS[mem])

    return min(tied, key=key)


def repick(path=TABLE):
    """Recompute `best` of a saved table from its stored timings (keeps the
    table's source hash: the timings still belong to those sources)."""
    import paper_1904_05717_amd as mm
    with open(path) as fh:
        table = json.load(fh)
    for e in table["entries"]:
        e["best"] = pick(mm, *e["shape"], e["ms"])
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1)
    return table["entries"]


def sweep(shapes=SWEEP_SHAPES, members=None):
    import torch

    import paper_1904_05717_amd as mm
    import workloads

    members = members or mm.FAMILY
    entries = []
    for (m, n, k) in shapes:
        A, B, C = workloads.gemm_operands(m, n, k)
        Ad, Bd, Cd = (torch.from_numpy(x).to("cuda:0") for x in (A, B, C))
        del A, B, C
        times = time_members(mm, Ad, Bd, Cd, members)
        best = pick(mm, m, n, k, times)
        entries.append({"shape": [m, n, k], "bucket": list(bucket(m, n, k)), "best": best,
                        "ms": {k2: round(v, 4) for k2, v in times.items()},
                        "prior": mm.MEMBER_NAMES[mm._lib.momms_select_member_prior(m, n, k)]})
        print(json.dumps(entries[-1]), flush=True)
        del Ad, Bd, Cd
        torch.cuda.empty_cache()
    return entries


def save(entries, path=TABLE):
    with open(path, "w") as fh:
        json.dump({"source_sha": source_sha(), "entries": entries}, fh, indent=1)


def install(path=TABLE):
    """Load a saved table into the library; returns the number of entries
    (0, leaving the analytic prior in charge, when there is no table or it
    was measured on other kernel or planner sources)."""
    from . import MEMBERS, _lib
    if not os.path.exists(path):
        return 0
    with open(path) as fh:
        table = json.load(fh)
    if table.get("source_sha") != source_sha():
        _lib.momms_set_member_table(0, None, None, None, None)
        return 0
    entries = table["entries"]
    rows = [(e["bucket"], MEMBERS[e["best"]]) for e in entries]
    n = len(rows)
    arr = ctypes.c_int * max(n, 1)
    st = _lib.momms_set_member_table(n, arr(*[r[0][0] for r in rows]), arr(*[r[0][1] for r in rows]),
                                     arr(*[r[0][2] for r in rows]), arr(*[r[1] for r in rows]))
    if st != 0:
        raise RuntimeError(f"momms_set_member_table failed: {st}")
    return n


def main():
    save(sweep())
    print(json.dumps({"saved": TABLE}))


if __name__ == "__main__":
    main()
