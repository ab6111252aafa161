#!/usr/bin/env python3
"""Benchmark of the batched 2x2 SVD on one MI355X.

Headline (one JSON line on stdout): complex FP64 batched SVD, n = 2^24 matrices
whose real and imaginary parts are +-m 2^e (m ~ U[1,2), e ~ U{-1000..1000})
with 1 % special lanes, in SoA layout resident in HBM.  One step = one
zsvd2_batch call over the whole batch.  value = SVDs per second.

The same line carries the other forms of the metric, one entry each
([SVDs/s, fraction of 8 TB/s, fraction of the VALU issue peak]): real FP64;
the singular-values-only and sine-form variants; real and complex FP32
without a rescue and with each FP64 rescue -- the FP64 tail, the sigma
quotient and the FP64 triangle -- at n = 2^24 and at n = 2^26, with the
fraction of lanes each rescue took.  Then the Kogbetliantz solver (sweeps/s of
each driver, a full solve, the SVD with U and V) and the uneven batch, the
roofline of the dominant kernel measured with HIP events on the launch
stream, and the CPU oracle timed on this host as a baseline, together with a
comparison of the GPU's outputs with the oracle's on a sample of lanes.  The
line stays under 4 KB; the full result (every launch figure, every problem of
the uneven batch) goes to stderr before it, and to --detail-out.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2×2 SVDs/s at n=2^24 (FP64, FP32) + % HBM roofline; Kogbetliantz sweeps/s"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per SVD: SoA inputs read once + U, V, smax, smin, s written once
BYTES_PER_SVD = {"d": 120, "z": 216, "s": 60, "c": 108}
# singular values only (SVD2_NO_UV): inputs + smax, smin, s
BYTES_PER_SVD_NOUV = {"d": 56, "z": 88, "s": 28, "c": 44}
# launch shape (threads per block, matrices per lane) used by the benchmark
DEFAULT_LAUNCH = {"d": (256, 1), "z": (64, 2), "s": (256, 1), "c": (256, 1),
                  "d_nouv": (256, 1), "z_nouv": (256, 1), "s_nouv": (256, 1), "c_nouv": (256, 1)}
WARM_S = 0.1  # minimum warm-up per timed variant, seconds
KERNEL_SOURCES = ["paper_2005_07403_amd/csrc/svd2_batch.hip", "paper_2005_07403_amd/csrc/svd2_lane.hpp"]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_inputs(variant: str, n: int, seed_off: int = 1):
    from workloads import SEED_BASE, scaled_law, to_trains
    cplx = variant in ("z", "c")
    dtype = np.float64 if variant in ("d", "z") else np.float32
    A = scaled_law(n, SEED_BASE + seed_off, cplx, dtype=dtype)
    return to_trains(A, dtype)


def time_variant(variant: str, trains_np, steps: int, warmup: int, flagsets, sample=None, urv=False):
    """Time `steps` batched calls on inputs resident in HBM, once per flag set
    in `flagsets` (same inputs).  Returns {flags: dict} with the wall-clock
    time of the timed region and the per-launch kernel time from HIP events
    recorded on the launch stream; the memory-pattern probe (same loads and
    stores, no arithmetic) is timed the same way under key 'pattern', and
    under 'pattern_nouv' for the singular-values-only pattern when a flag set
    has SVD2_NO_UV.  FP32 flag sets with a rescue also get the count of
    rescued lanes (one extra call); with `sample` (lane indices) the outputs
    of the first flag set on those lanes come back as host arrays.  With urv
    the call with the phase outputs (R, U_+, V_+; default flags) is timed as
    well, under key 'urv'."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    S.svd2_set_launch_kind(variant, *DEFAULT_LAUNCH[variant])
    S.svd2_set_launch_kind(variant + "_nouv", *DEFAULT_LAUNCH[variant + "_nouv"])
    dev = [torch.from_numpy(t).cuda() for t in trains_np]
    n = dev[0].numel()
    nout = 19 if len(dev) == 8 else 11
    out = [torch.empty(n, dtype=dev[0].dtype, device="cuda") for _ in range(nout)]
    sig = out[nout - 3:]
    stream = torch.cuda.current_stream()
    res = {}

    def timed(fn):
        # W warm-up steps, and at least WARM_S of warm-up in all, so that the
        # GPU's clocks have left the idle state they drop to while the host
        # generates inputs (otherwise whichever variant is timed first reads
        # several percent slow)
        t0 = time.perf_counter()
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        while time.perf_counter() - t0 < WARM_S:
            for _ in range(8):
                fn()
            torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return dict(n=n, wall_s=t1 - t0, kernel_ms=[a.elapsed_time(b) for a, b in ev])

    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    for flags in flagsets:
        ws = None
        wsb = S.svd2_workspace_bytes(n, flags) if dev[0].dtype == torch.float32 else 0
        if wsb:
            ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        o = sig if flags & S.SVD2_NO_UV else out
        res[flags] = timed(lambda: S.svd2(dev, flags=flags, out=o, ws=ws))
        if flags & S.SVD2_RESCUE_FP64:
            # one more call, outside the timed region, counting the rescued lanes
            cnt.zero_()
            S.svd2(dev, flags=flags, out=o, ws=ws, nrescued=cnt)
            res[flags]["rescued"] = int(cnt.item())
    if urv:
        f = [torch.empty(n, dtype=dev[0].dtype, device="cuda") for _ in range(nout)]
        res["urv"] = timed(lambda: S.svd2(dev, flags=0, out=out, urv=f))
        del f
    if sample is not None:
        # outputs of the default call on a sample of lanes, for the comparison
        # with the oracle in the CPU-baseline leg
        wsb = S.svd2_workspace_bytes(n, flagsets[0]) if dev[0].dtype == torch.float32 else 0
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda") if wsb else None
        S.svd2(dev, flags=flagsets[0], out=out, ws=ws)
        idx = torch.from_numpy(sample).cuda()
        res["sample_out"] = [o.index_select(0, idx).cpu().numpy() for o in out]
        res["sample_flags"] = flagsets[0]
    res["pattern"] = timed(lambda: S.svd2_stream_probe(variant, dev, out))
    if any(f & S.SVD2_NO_UV for f in flagsets):
        res["pattern_nouv"] = timed(lambda: S.svd2_stream_probe(variant + "_nouv", dev, sig))
    del dev, out, cnt
    torch.cuda.empty_cache()
    return res


def cpu_baseline(variant: str, trains_np, budget_s: float = 12.0):
    """The oracle (MIRROR policy, OpenMP over matrices) on this host."""
    import oracle.oracle as O
    cplx = len(trains_np) == 8
    dtype = trains_np[0].dtype
    nthreads = host_threads()
    n = trains_np[0].shape[0]
    reps, t_total = 0, 0.0
    while t_total < budget_s and reps < 50:
        t0 = time.perf_counter()
        O.run_trains(trains_np, cplx, dtype, policy="mirror", rescue=(dtype == np.float32),
                     nthreads=nthreads)
        t_total += time.perf_counter() - t0
        reps += 1
    return dict(value=reps * n / t_total, unit="SVDs/s", cores=nthreads, kind="oracle",
                sample=f"{reps} pass(es) over the same {n}-matrix batch "
                       f"({'complex' if cplx else 'real'} {dtype.name}), {t_total:.1f} s")


def host_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def rescue_mode(flags: int) -> int:
    """the oracle's rescue argument for an FP32 flag set: 0 none, 1 the FP64
    tail, 2 the sigma quotient, 3 the FP64 triangle"""
    if not flags & 4:
        return 0
    return 2 if flags & 16 else (3 if flags & 128 else 1)


def oracle_check(ins, gpu_out, flags: int) -> dict:
    """The GPU's outputs on a sample of lanes beside the oracle's on the same
    lanes: s compared bitwise, sigma'_max and sigma'_min in ulps, U and V in
    eps (absolute; their entries are bounded by one), the count of lanes equal
    in every bit, and the accuracy of the GPU's results by eqs. (33)-(35)
    (rho, delta, eta computed by the oracle in binary128; maxima in eps of the
    element type)."""
    import oracle.oracle as O
    cplx = len(ins) == 8
    dtype = ins[0].dtype
    it = np.int64 if dtype == np.float64 else np.int32
    outs, _ = O.run_trains(ins, cplx, dtype, policy="mirror", rescue=rescue_mode(flags),
                           nthreads=host_threads())
    k = 16 if cplx else 8
    eps = float(np.finfo(dtype).eps)

    def ulps(a, b):
        ia, ib = a.view(it).astype(np.int64), b.view(it).astype(np.int64)
        m = np.int64((1 << (8 * a.itemsize - 1)) - 1)
        ia = np.where(ia < 0, -(ia & m), ia)
        ib = np.where(ib < 0, -(ib & m), ib)
        return int(np.max(np.abs(ia - ib), initial=0))

    same = np.ones(ins[0].shape[0], dtype=bool)
    for g, o in zip(gpu_out, outs):
        same &= (g.view(it) == o.view(it)) | ((g == 0) & (o == 0))
    met = O.metrics(ins, gpu_out, cplx, nthreads=host_threads())
    uv = max(float(np.max(np.abs(gpu_out[i].astype(np.float64) - outs[i]))) for i in range(k))
    return {"lanes": int(ins[0].shape[0]), "bitwise_lanes": int(same.sum()),
            "s_equal": bool(np.array_equal(gpu_out[k + 2].view(it), outs[k + 2].view(it))),
            "smax_ulp": ulps(gpu_out[k], outs[k]), "smin_ulp": ulps(gpu_out[k + 1], outs[k + 1]),
            "uv_max_abs_eps": uv / eps,
            "rho_eps": float(np.nanmax(met["rho"])) / eps, "delta_eps": float(np.nanmax(met["delta"])) / eps,
            "eta_eps": float(np.nanmax(met["eta"])) / eps}


def cpu_upcast(trains32, budget_s: float = 1.5) -> dict:
    """The FP64 oracle on the exact FP64 upcast of an FP32 batch (a leading
    sample), on every host core: what a CPU would take to reach the FP32
    form's results through FP64."""
    import oracle.oracle as O
    cplx = len(trains32) == 8
    n = min(trains32[0].shape[0], 1 << 20)
    sub = [t[:n].astype(np.float64) for t in trains32]
    th = host_threads()
    reps, el = 0, 0.0
    while el < budget_s and reps < 50:
        t0 = time.perf_counter()
        O.run_trains(sub, cplx, np.float64, policy="mirror", nthreads=th)
        el += time.perf_counter() - t0
        reps += 1
    return {"SVDs_per_s": reps * n / el, "sample": f"{reps} x {n} matrices", "threads": th}


def cpu_details(trains_z, trains_d, nthreads, budget_s: float = 1.5):
    """Further oracle timings for context: one thread and all threads, real
    and complex FP64, the MIRROR policy (what the GPU computes) and the REF
    policy (hypot and 1/sqrt through binary128), each on a leading sample of
    the batch repeated for about budget_s."""
    import oracle.oracle as O
    out = {}
    for name, tr, cplx in (("z", trains_z, True), ("d", trains_d, False)):
        for pol in ("mirror", "ref"):
            for th in (1, nthreads):
                if pol == "ref" and th == 1:
                    continue
                n = min(tr[0].shape[0], (1 << 20) if th > 1 else (1 << 17))
                sub = [t[:n] for t in tr]
                reps, el = 0, 0.0
                while el < budget_s and reps < 50:
                    t0 = time.perf_counter()
                    O.run_trains(sub, cplx, np.float64, policy=pol, nthreads=th)
                    el += time.perf_counter() - t0
                    reps += 1
                out[f"{name}_{pol}_{th}t"] = {"SVDs_per_s": reps * n / el, "sample": f"{reps} x {n} matrices"}
    return out


def cpu_kog(order: int = 4096, steps: int = 4, small: int = 256):
    """The oracle's Kogbetliantz (single-threaded plain loops) on the host:
    seconds per step at the benchmark order over a few steps, extrapolated to
    a sweep of order - 1 steps (an extrapolation, stated as such), and a full
    solve at a small order, timed beside the GPU's two-step solve of it."""
    import torch
    import oracle.oracle as O
    from paper_2005_07403_amd import svd2 as S
    from workloads import SEED_BASE, kog_matrix
    A = np.asfortranarray(kog_matrix(order, SEED_BASE + 3, cond=1e12))
    t0 = time.perf_counter()
    for t in range(steps):
        O.kog_step(A, t)
    per_step = (time.perf_counter() - t0) / steps
    B = np.asfortranarray(kog_matrix(small, SEED_BASE + 5, cond=1e12))
    G = torch.from_numpy(B.copy(order="F")).cuda()
    t0 = time.perf_counter()
    ro = O.kog_solve(B, tol=1e-14)
    cpu_s = time.perf_counter() - t0
    S.kog_solve(G.clone(memory_format=torch.preserve_format), tol=1e-14, flags=S.SVD2_KOG_TWO_STEP)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rg = S.kog_solve(G, tol=1e-14, flags=S.SVD2_KOG_TWO_STEP)
    torch.cuda.synchronize()
    gpu_s = time.perf_counter() - t0
    return {"cores": 1, "kind": "oracle", "order": order, "seconds_per_step": per_step,
            "seconds_per_sweep_extrapolated": per_step * (order - 1),
            "sample": f"{steps} steps at order {order}",
            "full_solve": {"order": small, "sweeps": ro["sweeps"], "cpu_seconds": cpu_s,
                           "gpu_two_step_seconds": gpu_s, "gpu_sweeps": rg["sweeps"]}}


def read_traffic(kernel_key: str):
    """HBM bytes per dispatch from the committed rocprofv3 --pmc summary, or
    None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel_key}_pmc.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha:\s*(\w+)", txt)
    b = re.search(r"hbm_bytes_per_dispatch:\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != source_hash():
        return None
    return float(b.group(1))


# issue rate of the vector ALUs: a wave64 instruction occupies a 16-lane SIMD
# for 4 cycles; 256 CUs x 4 SIMDs at 2.4 GHz
VALU_SIMDS, VALU_CLOCK_HZ, VALU_CYCLES_PER_INSTR = 1024, 2.4e9, 4


def read_valu_table():
    """VALU instructions per matrix for each variant, from the committed
    rocprofv3 --pmc summary (SQ_INSTS_VALU per launch x 64 / n), or {} when
    the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "svd2_valu.md")
    if not os.path.exists(path):
        return {}
    txt = open(path).read()
    m = re.search(r"kernel_source_sha:\s*(\w+)", txt)
    t = re.search(r"valu_instr_per_matrix:\s*(\{.*\})", txt)
    if not m or not t or m.group(1) != source_hash():
        return {}
    return json.loads(t.group(1))


def valu_frac(instr_per_matrix, n: int, kernel_ms: float):
    """fraction of the VALU issue peak a launch of n matrices used"""
    if instr_per_matrix is None:
        return None
    cycles = instr_per_matrix * n / 64 * VALU_CYCLES_PER_INSTR
    return cycles / (kernel_ms * 1e-3 * VALU_CLOCK_HZ * VALU_SIMDS)


def kog_bench(order: int, sweeps: int = 2, solve: bool = True, only=None):
    """Kogbetliantz on the one-problem workload: real FP64, A = Q1 diag(s) Q2^T
    with s geometric from 1 to 1e-12.  Sweeps/s of each driver, timed over
    `sweeps` sweeps from the same matrix: the fused persistent kernel, the
    unfused gather -> SVD -> update chain, its hipGraph replay, and two or
    three steps per pass over the matrix; then a full solve with the fastest."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    from workloads import SEED_BASE, kog_matrix
    A, s = kog_matrix(order, SEED_BASE + 3, cond=1e12, return_sigma=True)
    G0 = torch.from_numpy(A).cuda()
    mat = order * order * 8
    steps = order - 1
    # HBM bytes of the matrix per sweep: one read and one write per step for
    # the single-step drivers; one per pass of two steps (plus the odd last
    # step) for the two-step driver
    passes = (steps - 1) // 2 if steps > 1 else 0
    passes3 = steps // 3  # three-step passes, then a two-step pass or a single step for the rest
    hbm_sweep = {"fused": 2 * mat * steps, "unfused": 2 * mat * steps, "graph": 2 * mat * steps,
                 "two_step": 2 * mat * (passes + (steps - 2 * passes)),
                 "three_step": 2 * mat * (passes3 + (1 if steps % 3 else 0))}
    out = {"order": order, "dtype": "f64", "steps_per_sweep": steps,
           "algorithmic_bytes_per_step": 2 * mat}
    modes = {"fused": 0, "unfused": S.SVD2_KOG_UNFUSED, "graph": S.SVD2_KOG_UNFUSED | S.SVD2_KOG_GRAPH,
             "two_step": S.SVD2_KOG_TWO_STEP, "three_step": S.SVD2_KOG_THREE_STEP}
    if only:
        modes = {m: modes[m] for m in only}
    for name, fl in modes.items():
        G = G0.clone(memory_format=torch.preserve_format)
        ws = S.kog_workspace(G, fl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.kog_solve(G, tol=0.0, max_sweeps=sweeps, ws=ws, flags=fl)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"sweeps_per_s": sweeps / el, "us_per_step": el / sweeps / steps * 1e6,
                     "hbm_GBs": hbm_sweep[name] * sweeps / el / 1e9}
        log(f"[bench] kog {name}: {json.dumps(out[name])}")
        del G, ws
    if solve:
        best = max(modes, key=lambda m: out[m]["sweeps_per_s"])
        G = G0.clone(memory_format=torch.preserve_format)
        ws = S.kog_workspace(G, modes[best])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = S.kog_solve(G, tol=1e-14, max_sweeps=60, ws=ws, flags=modes[best])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        sig = S.kog_sigma(G).cpu().numpy()  # the diagonal, sorted on the device
        out["solve"] = {"mode": best, "status": r["status"], "sweeps": r["sweeps"],
                        "off_rel": r["off_rel"], "seconds": el, "sweeps_per_s": r["sweeps"] / el,
                        "sigma_max_abs_err_rel": float(np.max(np.abs(sig - s)) / s[0])}
        log(f"[bench] kog solve: {json.dumps(out['solve'])}")
        del G, ws
    if solve:
        out["svd"] = kog_svd_bench(A, s, G0, mat, steps, passes)
    del G0
    torch.cuda.empty_cache()
    return out


def barrier_bench():
    """What a grid barrier of the fused Kogbetliantz kernel costs: cooperative
    launches of 1, 2 and 4 workgroups per CU that pass 0 or 1000 barriers and
    do nothing else (median of HIP-event times on the launch stream), beside
    the cost of a plain kernel launch (100 back-to-back launches of the small
    memory-pattern probe)."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    ws = torch.empty(256 + 4096 * 64, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def median_ms(fn, reps=15):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {"cus": cus, "workgroup_threads": 256}
    for per in (1, 2, 4):
        blocks = per * cus
        t0 = median_ms(lambda: S.kog_barrier_probe(0, blocks, ws))
        t1 = median_ms(lambda: S.kog_barrier_probe(1000, blocks, ws))
        out[f"blocks_{blocks}"] = {"empty_launch_us": t0 * 1e3, "us_per_barrier": (t1 - t0)}
        log(f"[bench] barrier, {blocks} workgroups: {json.dumps(out[f'blocks_{blocks}'])}")
    x = [torch.ones(256, dtype=torch.float64, device="cuda") for _ in range(8)]
    y = [torch.empty(256, dtype=torch.float64, device="cuda") for _ in range(19)]
    t2 = median_ms(lambda: [S.svd2_stream_probe("z", x, y) for _ in range(100)])
    out["plain_launch_us"] = t2 / 100 * 1e3
    log(f"[bench] plain launch: {out['plain_launch_us']:.2f} us")
    return out


def kog_svd_bench(A, s, G0, mat, steps, passes, full: bool = True):
    """The full SVD A_0 = U diag(sigma) V^* (transformations accumulated,
    three steps per pass) on the one-problem workload: one sweep and a full
    solve, sigma against the known singular values, and the residuals
    ||A_0 - U S V^T||_F / ||A_0||_F and ||U^T U - I||_F computed on the GPU."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    N = A.shape[0]
    fl = S.SVD2_KOG_THREE_STEP
    ws = torch.empty(S.kog_svd_workspace_bytes(N, "d", fl), dtype=torch.uint8, device="cuda")
    # per sweep: the iterate read and written once per pass of three steps
    # (and once for the two-step pass or single step that ends a sweep when 3
    # does not divide its steps); U and V once per six steps (pairs of passes),
    # once for an unpaired last pass and once for that end
    p3 = steps // 3
    rest = 1 if steps % 3 else 0
    hbm = 2 * mat * (p3 + rest) + 2 * 2 * mat * (p3 // 2 + p3 % 2 + rest)
    res = {"mode": "three_step", "algorithmic_bytes_per_sweep": hbm}
    G = G0.clone(memory_format=torch.preserve_format)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.kog_svd(G, tol=0.0, max_sweeps=1, ws=ws, flags=fl)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    res["one_sweep_s"] = el
    res["hbm_GBs"] = hbm / el / 1e9
    if not full:
        del G, ws
        return res
    G = G0.clone(memory_format=torch.preserve_format)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = S.kog_svd(G, tol=1e-14, max_sweeps=60, ws=ws, flags=fl)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    U, V, sig = r["U"], r["V"], r["sigma"]
    A0 = G0
    rec = torch.linalg.norm(A0 - (U * sig) @ V.t().contiguous()) / torch.linalg.norm(A0)
    orth = torch.linalg.norm(U.t().contiguous() @ U - torch.eye(N, dtype=U.dtype, device="cuda"))
    res.update({"status": r["status"], "sweeps": r["sweeps"], "seconds": el, "sweeps_per_s": r["sweeps"] / el,
                "sigma_max_abs_err_rel": float(np.max(np.abs(sig.cpu().numpy() - s)) / s[0]),
                "residual_rel": float(rec), "orthogonality": float(orth)})
    log(f"[bench] kog svd: {json.dumps(res)}")
    del G, ws, U, V
    torch.cuda.empty_cache()
    return res


def kog_batch_bench(nprob: int = 256):
    """The uneven batch: nprob problems of order 32..2048 (log-uniform), half
    complex FP64 (tol 1e-14), half real FP32 (tol 1e-7), condition numbers
    1e2..1e12, solved together by kog_batch_solve with hipGraph replay, three
    steps per pass (the reported run), and one and two steps per pass (for
    comparison, from copies of the same matrices)."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    from workloads import SEED_BASE, kog_problem_set_device
    t0 = time.perf_counter()
    probs = kog_problem_set_device(nprob, SEED_BASE + 5)
    torch.cuda.synchronize()
    log(f"[bench] kog batch: {nprob} problems built in {time.perf_counter() - t0:.1f} s")
    mats = [p["A"] for p in probs]
    tols = [1e-14 if p["cplx"] else 1e-7 for p in probs]
    def on_copies(flags):
        copies = [A.clone(memory_format=torch.preserve_format) for A in mats]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = S.kog_batch_solve(copies, tols, max_sweeps=40, flags=flags)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        del copies
        torch.cuda.empty_cache()
        return r, el

    res1, el1 = on_copies(S.SVD2_KOG_GRAPH)
    res2, el2 = on_copies(S.SVD2_KOG_GRAPH | S.SVD2_KOG_TWO_STEP)
    t0 = time.perf_counter()
    res = S.kog_batch_solve(mats, tols, max_sweeps=40, flags=S.SVD2_KOG_GRAPH | S.SVD2_KOG_THREE_STEP)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    single = {"seconds": el1, "problem_sweeps_per_s": sum(r["sweeps"] for r in res1) / el1,
              "same_sweeps_as_three_step": all(a["sweeps"] == b["sweeps"] for a, b in zip(res, res1))}
    two = {"seconds": el2, "problem_sweeps_per_s": sum(r["sweeps"] for r in res2) / el2,
           "same_sweeps_as_three_step": all(a["sweeps"] == b["sweeps"] for a, b in zip(res, res2))}
    log(f"[bench] kog batch, one step per pass: {json.dumps(single)}; two: {json.dumps(two)}")
    per = []
    for p, r in zip(probs, res):
        d = torch.diagonal(p["A"]).real.double().cpu().numpy()
        sig = np.sort(np.abs(d))[::-1]
        per.append({"order": p["order"], "dtype": "c128" if p["cplx"] else "f32",
                    "cond": float(p["cond"]), "status": r["status"], "sweeps": r["sweeps"],
                    "off_rel": r["off_rel"],
                    "sigma_err_rel": float(np.max(np.abs(sig - p["sigma"])) / p["sigma"][0])})
    total_sweeps = sum(r["sweeps"] for r in res)
    bytes_moved = sum(2 * p["order"] ** 2 * (16 if p["cplx"] else 4) * (p["order"] - 1) * r["sweeps"]
                      for p, r in zip(probs, res))
    out = {"nprob": nprob, "mode": "three_step", "seconds": el, "converged": sum(r["status"] == 0 for r in res),
           "one_step_per_pass": single, "two_steps_per_pass": two,
           "problem_sweeps_per_s": total_sweeps / el, "algorithmic_GBs": bytes_moved / el / 1e9,
           "max_sweeps": max(r["sweeps"] for r in res),
           "max_sigma_err_rel_c128": max(q["sigma_err_rel"] for q in per if q["dtype"] == "c128"),
           "max_sigma_err_rel_f32": max(q["sigma_err_rel"] for q in per if q["dtype"] == "f32"),
           "max_off_rel_c128": max(q["off_rel"] for q in per if q["dtype"] == "c128"),
           "max_off_rel_f32": max(q["off_rel"] for q in per if q["dtype"] == "f32"),
           "problems": per}
    log(f"[bench] kog batch: {json.dumps({k: v for k, v in out.items() if k != 'problems'})}")
    del probs, mats
    torch.cuda.empty_cache()
    return out


def summarize(variant, r, pattern, flags_desc="", nouv=False, valu_per_matrix=None, bps=None):
    n = r["n"]
    if bps is None:
        bps = (BYTES_PER_SVD_NOUV if nouv else BYTES_PER_SVD)[variant]
    kms = float(np.mean(r["kernel_ms"]))
    wall_ms = r["wall_s"] * 1e3 / len(r["kernel_ms"])
    gbs = bps * n / (kms * 1e-3) / 1e9
    pgbs = None
    if pattern is not None:
        pms = float(np.mean(pattern["kernel_ms"]))
        pgbs = bps * n / (pms * 1e-3) / 1e9
    vf = valu_frac(valu_per_matrix, n, kms)
    hf = gbs / HBM_PEAK_GBS
    out = dict(n=n, svds_per_s=n / (wall_ms * 1e-3), ms_per_step=wall_ms, kernel_ms=kms,
               kernel_ms_min=float(np.min(r["kernel_ms"])), kernel_ms_median=float(np.median(r["kernel_ms"])),
               algorithmic_GBs=gbs,
               hbm_frac=hf, bytes_per_svd=bps, valu_instr_per_matrix=valu_per_matrix, valu_frac=vf,
               bound="valu" if vf is not None and vf > hf else "hbm",
               pattern_ceiling_GBs=pgbs, frac_of_pattern_ceiling=None if pgbs is None else gbs / pgbs,
               flags=flags_desc)
    if "rescued" in r:
        out["rescued"] = r["rescued"]
        out["rescued_frac"] = r["rescued"] / n
    return out


def r4(x):
    """four significant digits (None stays None)"""
    if x is None:
        return None
    if isinstance(x, bool) or isinstance(x, int):
        return x
    return float(f"{x:.4g}")


def headline(full: dict) -> dict:
    """The one JSON line bench.py prints last on stdout, kept under 4 KB: the
    headline metric with its roofline and CPU baseline, one entry per variant
    ([SVDs/s, fraction of 8 TB/s, fraction of the VALU issue peak or null]),
    the rescued-lane fraction of each FP32 rescue variant, and the
    Kogbetliantz figures.  Per-problem and per-launch detail stays in `full`."""
    h = full["variants"][full["head"]]
    line = {k: full[k] for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                                  "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config")}
    line["value"] = r4(line["value"])
    line["ms_per_step"] = r4(line["ms_per_step"])
    rl = dict(full["roofline"])
    line["roofline"] = {k: (r4(v) if isinstance(v, float) else v) for k, v in rl.items()}
    cpu = full.get("cpu_baseline")
    if cpu is not None:
        c = {k: cpu[k] for k in ("unit", "cores", "kind", "sample")}
        c["value"] = r4(cpu["value"])
        if "upcast" in cpu:
            c["fp32_via_fp64_upcast_SVDs_per_s"] = {k: r4(v["SVDs_per_s"]) for k, v in cpu["upcast"].items()}
        if "check" in cpu:
            c["gpu_vs_oracle_sample"] = {k: {kk: r4(vv) for kk, vv in v.items()} for k, v in cpu["check"].items()}
        line["cpu_baseline"] = c
    else:
        line["cpu_baseline"] = None
    line["variants_fields"] = ["SVDs/s", "hbm_frac", "valu_frac"]
    line["variants"] = {k: [r4(v["svds_per_s"]), r4(v["hbm_frac"]), r4(v.get("valu_frac"))]
                        for k, v in full["variants"].items()}
    # rescued-lane fractions: one entry per base variant (s, c, s26, c26) when
    # its rescue variants agree, as they should (which lanes are flagged does
    # not depend on how they are rescued), else one per variant
    groups = {}
    for k, v in full["variants"].items():
        if "rescued_frac" in v:
            groups.setdefault(k.split("_")[0], {})[k] = r4(v["rescued_frac"])
    resc = {}
    for base, d in groups.items():
        if len(set(d.values())) == 1:
            resc[base] = next(iter(d.values()))
        else:
            resc.update(d)
    if resc:
        line["rescued_frac"] = resc
    kog = full.get("kogbetliantz")
    if kog:
        k = {"order": kog["order"], "sweeps_per_s": {m: r4(kog[m]["sweeps_per_s"]) for m in
                                                      ("three_step", "two_step", "unfused", "graph", "fused") if m in kog}}
        if "solve" in kog:
            s = kog["solve"]
            k["solve"] = {"mode": s["mode"], "sweeps": s["sweeps"], "seconds": r4(s["seconds"]),
                          "off_rel": r4(s["off_rel"]), "sigma_err_rel": r4(s["sigma_max_abs_err_rel"])}
        if "svd" in kog and "seconds" in kog["svd"]:
            s = kog["svd"]
            k["svd"] = {"sweeps": s["sweeps"], "seconds": r4(s["seconds"]), "residual_rel": r4(s["residual_rel"]),
                        "orthogonality": r4(s["orthogonality"])}
        if "cpu_baseline" in kog:
            k["cpu_oracle_s_per_sweep_extrapolated"] = r4(kog["cpu_baseline"]["seconds_per_sweep_extrapolated"])
        line["kogbetliantz"] = k
    kb = full.get("kogbetliantz_batch")
    if kb:
        line["kogbetliantz_batch"] = {
            "nprob": kb["nprob"], "seconds": r4(kb["seconds"]), "converged": kb["converged"],
            "problem_sweeps_per_s": r4(kb["problem_sweeps_per_s"]),
            "one_step_per_pass_seconds": r4(kb["one_step_per_pass"]["seconds"]),
            "two_steps_per_pass_seconds": r4(kb["two_steps_per_pass"]["seconds"]),
            "max_sigma_err_rel_c128": r4(kb["max_sigma_err_rel_c128"]),
            "max_sigma_err_rel_f32": r4(kb["max_sigma_err_rel_f32"])}
    line["kernel_source_sha"] = full["kernel_source_sha"]
    return line


def emit(full: dict, detail_out=None) -> None:
    """Everything, per launch and per problem, as one line on stderr (and in
    detail_out if given); then the compact headline as the last line on
    stdout."""
    detail = json.dumps(full)
    log(f"[bench] detail: {detail}")
    if detail_out:
        with open(detail_out, "w") as fh:
            fh.write(detail + "\n")
    print(json.dumps(headline(full), separators=(",", ":")), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--only", choices=["d", "z", "s", "c"], default=None,
                    help="time one variant only (for profiling runs)")
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--n32", type=int, default=1 << 26,
                    help="batch size of the FP32 precision-form runs (reported as s26/c26; 0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kog", action="store_true", help="skip the Kogbetliantz measurement")
    ap.add_argument("--kog-order", type=int, default=4096)
    ap.add_argument("--kog-sweeps", type=int, default=1,
                    help="sweeps timed per driver with --kog-only (from the same starting matrix)")
    ap.add_argument("--kog-fused-per-cu", type=int, default=None,
                    help="workgroups per CU of the fused Kogbetliantz kernel (1-16; default: the library's)")
    ap.add_argument("--no-kog-batch", action="store_true", help="skip the uneven Kogbetliantz batch")
    ap.add_argument("--kog-batch", type=int, default=256, help="problems in the uneven batch")
    ap.add_argument("--kog-batch-only", action="store_true",
                    help="run only the uneven Kogbetliantz batch; prints its JSON (for profiling runs)")
    ap.add_argument("--kog-only", default=None, metavar="MODES",
                    help="run only the Kogbetliantz drivers named (comma list of fused, unfused, graph, "
                         "two_step), one sweep each, no solve; prints their JSON (for profiling runs)")
    ap.add_argument("--uv", choices=["both", "full", "nouv"], default="both",
                    help="batched SVD: time only the default kernels (full), only the singular-values-only "
                         "ones (nouv), or every variant (both)")
    ap.add_argument("--kog-svd-only", action="store_true",
                    help="run only one sweep of the Kogbetliantz SVD with U and V (two steps per pass); "
                         "prints its JSON (for profiling runs)")
    ap.add_argument("--detail-out", default=None, metavar="PATH",
                    help="also write the full result (every launch figure, every uneven-batch problem) to PATH")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy (for HBM counter calibration)")
    ap.add_argument("--barrier-probe", action="store_true",
                    help="time the fused Kogbetliantz kernel's grid barrier alone; prints its JSON")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: measures one GPU only; --gpus {args.gpus} is not supported (the batched SVD "
              "would shard by contiguous chunks of the batch, one per GPU, with no exchange)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_07403_amd import svd2 as S
    S.lib()
    tuning = S.apply_tuning()
    if tuning:
        for k, v in tuning.get("svd2_launch", {}).items():
            DEFAULT_LAUNCH[k] = tuple(v)
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(3)

    if args.copy_calibration:
        x = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of 1 GiB done")
        return

    if args.kog_fused_per_cu is not None and S._kog().kog_set_fused_blocks_per_cu(args.kog_fused_per_cu) != 0:
        print(f"bench.py: --kog-fused-per-cu {args.kog_fused_per_cu} is out of range (1-16)", file=sys.stderr)
        sys.exit(2)
    if args.barrier_probe:
        print(json.dumps(barrier_bench()), flush=True)
        return
    if args.kog_only:
        out = kog_bench(args.kog_order, sweeps=args.kog_sweeps, solve=False, only=args.kog_only.split(","))
        print(json.dumps(out), flush=True)
        return
    if args.kog_svd_only:
        from workloads import SEED_BASE, kog_matrix
        A, sig = kog_matrix(args.kog_order, SEED_BASE + 3, cond=1e12, return_sigma=True)
        steps = args.kog_order - 1
        out = kog_svd_bench(A, sig, torch.from_numpy(A).cuda(), args.kog_order ** 2 * 8, steps,
                            (steps - 1) // 2, full=False)
        print(json.dumps(out), flush=True)
        return
    if args.kog_batch_only:
        out = kog_batch_bench(args.kog_batch)
        print(json.dumps({k: v for k, v in out.items() if k != "problems"}), flush=True)
        return

    variants = [args.only] if args.only else ["z", "d", "s", "c"]
    F, NU = S.SVD2_RESCUE_FP64, S.SVD2_NO_UV
    fp32 = {"RESCUE_FP64": F, "RESCUE_FP64|SIGMA": F | S.SVD2_RESCUE_SIGMA,
            "RESCUE_FP64|TRI": F | S.SVD2_RESCUE_TRI, "none": 0,
            "RESCUE_FP64|SIGMA|NO_UV": F | S.SVD2_RESCUE_SIGMA | NU}
    SF = S.SVD2_SINE_FORM
    flagsets = {"d": {"": 0, "NO_UV": NU, "SINE_FORM": SF}, "z": {"": 0, "NO_UV": NU, "SINE_FORM": SF},
                "s": fp32, "c": dict(fp32)}
    if args.uv != "both":  # one kernel per run (profiling): the default form, or singular values only
        keep_nouv = args.uv == "nouv"
        flagsets = {v: {d: f for d, f in fs.items() if ("NO_UV" in d) == keep_nouv and "SINE" not in d}
                    for v, fs in flagsets.items()}
    results, inputs_z, inputs_d = {}, None, None
    checks_in, checks_out, lead32 = {}, {}, {}
    valu_tab = read_valu_table()
    do_cpu = not args.no_cpu_baseline
    # FP32 also at the precision form's own size (2^26: its inputs exceed the
    # 256 MB Infinity Cache, so they come from HBM on every launch)
    runs = [(v, args.n, "") for v in variants]
    if args.n32 and not args.only:
        runs += [(v, args.n32, "26") for v in ("s", "c")]
    for v, n, tag in runs:
        log(f"[bench] generating {v} inputs n={n}")
        tr = make_inputs(v, n)
        # lanes compared with the oracle in the CPU-baseline leg: a seeded
        # sample of the timed batch (special lanes included at their rate)
        sample = None
        if do_cpu and not tag:
            sample = np.sort(np.random.default_rng(20050740).choice(n, size=min(n, 1 << 16), replace=False))
        log(f"[bench] timing {v}{tag}: warmup {args.warmup}, steps {args.steps}")
        urv = v in ("z", "d") and not tag and args.uv == "both"
        r = time_variant(v, tr, args.steps, args.warmup, list(flagsets[v].values()), sample=sample, urv=urv)
        if urv:
            # the phase outputs add R, U_+ and V_+: 11 (real) or 19 (complex) arrays
            results[f"{v}_urv"] = summarize(v, r["urv"], None, "phase outputs R, U+, V+", False, None,
                                            bps=BYTES_PER_SVD[v] + 8 * (19 if v == "z" else 11))
            log(f"[bench] {v}_urv: {json.dumps(results[v + '_urv'])}")
        if sample is not None:
            checks_in[v] = [np.ascontiguousarray(t[sample]) for t in tr]
            checks_out[v] = (r["sample_out"], r["sample_flags"])
            if v in ("s", "c"):
                lead32[v] = [t[: 1 << 20].copy() for t in tr]
        for desc, fl in flagsets[v].items():
            nouv = "NO_UV" in desc
            if desc in ("", "RESCUE_FP64"):
                key = v + tag
            elif nouv:
                key = f"{v}{tag}_nouv"
            elif desc == "SINE_FORM":
                key = f"{v}{tag}_sine"
            elif "TRI" in desc:
                key = f"{v}{tag}_tri"
            else:
                key = f"{v}{tag}_{'sigma' if 'SIGMA' in desc else 'norescue'}"
            results[key] = summarize(v, r[fl], r["pattern_nouv" if nouv else "pattern"], desc, nouv,
                                     valu_tab.get(key.replace("26", "")))
            log(f"[bench] {key}: {json.dumps(results[key])}")
        if v == "z" and not tag:
            inputs_z = tr
        elif v == "d" and not tag:
            inputs_d = tr
        else:
            del tr

    kog = None
    if not args.no_kog and not args.only:
        log(f"[bench] Kogbetliantz, order {args.kog_order}")
        kog = kog_bench(args.kog_order)
    kog_batch = None
    if not args.no_kog_batch and not args.only:
        log(f"[bench] uneven Kogbetliantz batch of {args.kog_batch}")
        kog_batch = kog_batch_bench(args.kog_batch)

    head = "z" if "z" in results else next(iter(results))
    h = results[head]
    steps = args.steps
    cpu = None
    if do_cpu and inputs_z is not None:
        log("[bench] CPU baseline (oracle) ...")
        cpu = cpu_baseline("z", inputs_z)
        log(f"[bench] cpu: {json.dumps(cpu)}")
        if inputs_d is not None:
            cpu["details"] = cpu_details(inputs_z, inputs_d, cpu["cores"])
            log(f"[bench] cpu details: {json.dumps(cpu['details'])}")
        cpu["upcast"] = {v: cpu_upcast(tr) for v, tr in lead32.items()}
        log(f"[bench] cpu, FP32 batches through the FP64 oracle on the upcast: {json.dumps(cpu['upcast'])}")
        cpu["check"] = {v: oracle_check(checks_in[v], *checks_out[v]) for v in checks_in}
        log(f"[bench] GPU against the oracle on sampled lanes: {json.dumps(cpu['check'])}")
        if kog is not None:
            kog["cpu_baseline"] = cpu_kog(args.kog_order)
            log(f"[bench] kog cpu: {json.dumps(kog['cpu_baseline'])}")
    del inputs_z, inputs_d, checks_in, checks_out, lead32
    traffic = read_traffic(f"svd2_{head}")
    dtype_name = {"d": "f64", "z": "f64", "s": "f32", "c": "f32"}[head[0]]
    full = {
        "head": head,
        "metric": METRIC,
        "value": h["svds_per_s"],
        "unit": "SVDs/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype_name,
        "data": "synthetic (seeded +-m 2^e law with 1% special lanes; stands in for the "
                "paper's private random-bit file)",
        "config": {"workload": {"z": "complex FP64 batched 2x2 SVD",
                                "d": "real FP64 batched 2x2 SVD",
                                "s": "real FP32 batched 2x2 SVD + FP64 rescue",
                                "c": "complex FP32 batched 2x2 SVD + FP64 rescue"}[head[0]] +
                   (", singular values only" if head.endswith("_nouv") else ""),
                   "n": h["n"], "layout": "SoA", "exponents": "e in [-1000,1000]" if head[0] in "dz"
                   else "e in [-120,120]", "special_lanes": 0.01,
                   "launch": list(DEFAULT_LAUNCH[head[0] + ("_nouv" if head.endswith("_nouv") else "")])},
        "roofline": {"bound": "hbm", "achieved": h["algorithmic_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": h["hbm_frac"],
                     "traffic": traffic, "traffic_unit": "bytes per launch",
                     "algorithmic_bytes_per_launch": h["bytes_per_svd"] * h["n"],
                     "kernel_ms": h["kernel_ms"], "valu_frac": h["valu_frac"],
                     "pattern_ceiling_GBs": h["pattern_ceiling_GBs"],
                     "frac_of_pattern_ceiling": h["frac_of_pattern_ceiling"]},
        "cpu_baseline": cpu,
        "variants": results,
        "kogbetliantz": kog,
        "kogbetliantz_batch": kog_batch,
        "kernel_source_sha": source_hash(),
    }
    del results, kog, kog_batch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    emit(full, args.detail_out)


def child_processes() -> int:
    """processes this one started that are still there (there should be none)"""
    try:
        import psutil
        return len(psutil.Process().children(recursive=True))
    except Exception:
        return -1


if __name__ == "__main__":
    main()
    log(f"[bench] child processes left: {child_processes()}")
