"""Autotuner: measures launch shapes on the GPU and writes tuning.json.

Tuned:
* the batched 2x2 SVD kernels: threads per workgroup (64/128/256) and
  matrices per lane (1/2), per element type, at n = 2^24 on the +-m 2^e law;
* the Kogbetliantz update tile: row pairs per workgroup kc (64/128/256) and
  column pairs per tile lc, per order bucket, timing unfused steps of a real
  FP64 and a complex FP64 matrix of that order;
* the two-step Kogbetliantz kernel: wavefronts per workgroup (1/2/4) and
  column pairs per wavefront, per order bucket, timing two-step sweeps of the
  same two matrices.

Run:  python -m paper_2005_07403_amd.autotune [--quick]
The binding applies the table with svd2.apply_tuning().
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def _median_ms(fn, reps: int) -> float:
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def _pick(res: dict, tiles) -> tuple:
    """The fastest shape, except that among shapes within 3 % of it the one
    with the fewest tiles wins (small orders are launch-bound and their
    timings differ by noise; fewer, larger tiles are the safer choice when
    the kernel also runs inside a batch)."""
    best = min(res.values())
    near = [k for k, v in res.items() if v <= 1.03 * best]
    return min(near, key=lambda k: (tiles(k), res[k]))


SVD2_KINDS = ["d", "z", "s", "c", "d_nouv", "z_nouv", "s_nouv", "c_nouv"]


def tune_svd2(n: int, reps: int, rounds: int = 3, kinds=SVD2_KINDS) -> dict:
    """Launch shape per element type (and per singular-values-only kernel,
    kinds "*_nouv"), timed at the batch size of interest with `rounds`
    interleaved passes over the candidates (the median of `reps` launches
    each); the best minimum over rounds wins."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    from workloads import SEED_BASE, scaled_law, to_trains
    best = {}
    shapes = [(64, 1), (64, 2), (128, 1), (128, 2), (256, 1), (256, 2)]
    for kind in kinds:
        cplx, nouv = kind[0] in "zc", kind.endswith("_nouv")
        dt = np.float64 if kind[0] in "dz" else np.float32
        dev = [torch.from_numpy(t).cuda() for t in to_trains(scaled_law(n, SEED_BASE + 7, cplx, dtype=dt), dt)]
        out = [torch.empty(n, dtype=dev[0].dtype, device="cuda") for _ in range(3 if nouv else (19 if cplx else 11))]
        flags = 0 if kind[0] in "dz" else S.SVD2_RESCUE_FP64
        if nouv:
            flags |= S.SVD2_NO_UV | (S.SVD2_RESCUE_SIGMA if flags else 0)
        res = {sh: [] for sh in shapes}
        for _ in range(rounds):
            for block, pt in shapes:
                S.svd2_set_launch_kind(kind, block, pt)
                for _ in range(2):
                    S.svd2(dev, flags=flags, out=out)
                res[(block, pt)].append(_median_ms(lambda: S.svd2(dev, flags=flags, out=out), reps))
        b = min(res, key=lambda k: min(res[k]))
        best[kind] = list(b)
        print(f"svd2 {kind}: " + ", ".join(f"{k}={min(v):.4f}ms" for k, v in sorted(res.items())) + f" -> {b}",
              flush=True)
        S.svd2_set_launch_kind(kind, *b)
        del dev, out
        torch.cuda.empty_cache()
    return best


def tune_kog(orders, steps: int) -> list:
    import torch
    from paper_2005_07403_amd import svd2 as S
    rules = []
    rng = np.random.default_rng(11)
    for N in orders:
        n = N // 2
        mats = {"d": np.asfortranarray(rng.standard_normal((N, N))),
                "z": np.asfortranarray(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))}
        res = {}
        for kc in (64, 128, 256):
            if kc > 2 * max(n, 64):
                continue
            for lc in (2, 4, 8, 16, 32):
                if lc > n:
                    continue
                S.kog_set_tile_rules([(1 << 19, kc, lc)])
                tot = 0.0
                for kind, A in mats.items():
                    G = torch.from_numpy(A).cuda()
                    ws = S.kog_workspace(G)
                    S.kog_step(G, 0, ws=ws, flags=S.SVD2_KOG_UNFUSED)
                    tot += _median_ms(lambda: S.kog_step(G, 1, ws=ws, flags=S.SVD2_KOG_UNFUSED), steps)
                    del G, ws
                res[(kc, lc)] = tot
        b = _pick(res, lambda k: -(-n // k[0]) * -(-n // k[1]))
        print(f"kog N={N}: " + ", ".join(f"{k}={v:.3f}ms" for k, v in sorted(res.items())) + f" -> {b}",
              flush=True)
        rules.append([N, b[0], b[1]])
    rules[-1][0] = 1 << 19  # the last rule covers every larger order
    S.kog_set_tile_rules([tuple(r) for r in rules])
    return rules


def tune_kog_two_step(orders, reps: int) -> list:
    """Workgroup shape of the two-step kernel per order: wavefronts per
    workgroup x column pairs per wavefront, timed on one two-step sweep of a
    real and a complex FP64 matrix."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    rules = []
    rng = np.random.default_rng(12)
    fl = S.SVD2_KOG_TWO_STEP
    for N in orders:
        n = N // 2
        mats = {"d": np.asfortranarray(rng.standard_normal((N, N))),
                "z": np.asfortranarray(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))}
        res = {}
        for wpg in (1, 2, 4):
            for lc in (2, 4, 8, 16, 32):
                if wpg * lc > 2 * max(n, 8):
                    continue
                S.kog_set_two_step_tiles([(1 << 19, wpg, lc)])
                tot = 0.0
                for kind, A in mats.items():
                    G = torch.from_numpy(A).cuda()
                    ws = S.kog_workspace(G, fl)
                    S.kog_sweep(G, ws=ws, flags=fl)
                    tot += _median_ms(lambda: S.kog_sweep(G, ws=ws, flags=fl), reps)
                    del G, ws
                res[(wpg, lc)] = tot
        b = _pick(res, lambda k: -(-n // (k[0] * k[1])))
        print(f"kog two-step N={N}: " + ", ".join(f"{k}={v:.3f}ms" for k, v in sorted(res.items())) +
              f" -> {b}", flush=True)
        rules.append([N, b[0], b[1]])
    rules[-1][0] = 1 << 19
    S.kog_set_two_step_tiles([tuple(r) for r in rules])
    return rules


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.json"))
    ap.add_argument("--svd2-only", default=None, metavar="KINDS",
                    help="tune only these batched-SVD kinds (comma list of " + ", ".join(SVD2_KINDS) +
                         ") and merge them into the existing table")
    args = ap.parse_args()
    import torch
    from paper_2005_07403_amd import svd2 as S
    S.lib()
    assert torch.cuda.is_available()
    t0 = time.time()
    if args.svd2_only:
        kinds = args.svd2_only.split(",")
        bad = [k for k in kinds if k not in SVD2_KINDS]
        if bad:
            raise SystemExit(f"unknown kinds {bad}")
        tab = {}
        if os.path.exists(args.out):
            with open(args.out) as fh:
                tab = json.load(fh)
        tab.setdefault("svd2_launch", {}).update(tune_svd2(1 << 24, 20, kinds=kinds))
        with open(args.out, "w") as fh:
            json.dump(tab, fh, indent=1)
        print(json.dumps(tab), flush=True)
        return
    launch = tune_svd2(1 << (22 if args.quick else 24), 10 if args.quick else 20)
    orders = [64, 256, 1024, 4096] if args.quick else [32, 64, 128, 256, 512, 1024, 2048, 4096]
    rules = tune_kog(orders, 5 if args.quick else 10)
    rules2 = tune_kog_two_step(orders, 2 if args.quick else 3)
    tab = {"device": torch.cuda.get_device_name(0), "svd2_launch": launch, "kog_tile_rules": rules,
           "kog_two_step_tiles": rules2, "seconds": round(time.time() - t0, 1)}
    with open(args.out, "w") as fh:
        json.dump(tab, fh, indent=1)
    print(json.dumps(tab), flush=True)


if __name__ == "__main__":
    main()
