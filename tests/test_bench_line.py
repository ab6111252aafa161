"""bench.py's output on the CPU: the headline JSON line built from a result of
the full shape (every variant, the Kogbetliantz sections, an uneven batch of
256 problems, the CPU baseline with its sampled comparison) stays under 4 KB,
is the last line on stdout, and carries the metric, its roofline and the CPU
baseline; the bulky detail goes to stderr and to the --detail-out file."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def fake_run(n, kernel_ms, rescued=None):
    r = {"n": n, "wall_s": kernel_ms * 20 * 1.01e-3, "kernel_ms": [kernel_ms * (1 + 0.001 * i) for i in range(20)]}
    if rescued is not None:
        r["rescued"] = rescued
    return r


def fake_full():
    variants = {}
    n24, n26 = 1 << 24, 1 << 26
    for v in "zd":
        for suf, nouv in (("", False), ("_nouv", True), ("_sine", False)):
            variants[v + suf] = bench.summarize(v, fake_run(n24, 0.6543219), fake_run(n24, 0.63), suf, nouv, 790.123)
    for v in "sc":
        for tag, n in (("", n24), ("26", n26)):
            for suf in ("", "_sigma", "_tri", "_norescue", "_nouv"):
                resc = None if suf == "_norescue" else int(0.83 * n)
                variants[v + tag + suf] = bench.summarize(v, fake_run(n, 0.2345678, resc), fake_run(n, 0.2),
                                                          suf, suf == "_nouv", 402.5)
    h = variants["z"]
    check = {"lanes": 65536, "bitwise_lanes": 65536, "s_equal": True, "smax_ulp": 0, "smin_ulp": 0,
             "uv_max_abs_eps": 0.0, "rho_eps": 3.987654321, "delta_eps": 5.4321, "eta_eps": 4.123456}
    problems = [{"order": 2 * (16 + i), "dtype": "c128" if i < 128 else "f32", "cond": 1.234567e7,
                 "status": 0, "sweeps": 11, "off_rel": 1.23456789e-15, "sigma_err_rel": 2.3456789e-15}
                for i in range(256)]
    kog = {"order": 4096, "dtype": "f64", "steps_per_sweep": 4095, "algorithmic_bytes_per_step": 268435456}
    for m in ("fused", "unfused", "graph", "two_step"):
        kog[m] = {"sweeps_per_s": 7.4912345, "us_per_step": 32.61234, "hbm_GBs": 4123.456}
    kog["solve"] = {"mode": "two_step", "status": 0, "sweeps": 26, "off_rel": 9.87654321e-15, "seconds": 3.4567,
                    "sweeps_per_s": 7.5123, "sigma_max_abs_err_rel": 5.0123456e-13}
    kog["svd"] = {"mode": "two_step", "algorithmic_bytes_per_sweep": 1.0e12, "one_step_s": 0.28, "hbm_GBs": 3900.0,
                  "status": 0, "sweeps": 26, "seconds": 7.3123, "sweeps_per_s": 3.55,
                  "sigma_max_abs_err_rel": 5.04e-13, "residual_rel": 2.403e-12, "orthogonality": 2.2958e-10}
    kog["cpu_baseline"] = {"cores": 1, "kind": "oracle", "order": 4096, "seconds_per_step": 0.101234,
                           "seconds_per_sweep_extrapolated": 414.567, "sample": "4 steps at order 4096",
                           "full_solve": {"order": 256, "sweeps": 12, "cpu_seconds": 0.9,
                                          "gpu_two_step_seconds": 0.037, "gpu_sweeps": 12}}
    batch = {"nprob": 256, "mode": "three_step", "seconds": 7.6123456, "converged": 256,
             "one_step_per_pass": {"seconds": 15.123456, "problem_sweeps_per_s": 250.1, "same_sweeps_as_three_step": True},
             "two_steps_per_pass": {"seconds": 9.323456, "problem_sweeps_per_s": 398.1, "same_sweeps_as_three_step": True},
             "problem_sweeps_per_s": 398.123, "algorithmic_GBs": 2345.6, "max_sweeps": 14,
             "max_sigma_err_rel_c128": 1.2345e-14, "max_sigma_err_rel_f32": 3.456e-6,
             "max_off_rel_c128": 9.1e-15, "max_off_rel_f32": 8.2e-8, "problems": problems}
    cpu = {"value": 5.6123456e7, "unit": "SVDs/s", "cores": 16, "kind": "oracle",
           "sample": "12 pass(es) over the same 16777216-matrix batch (complex float64), 12.3 s",
           "details": {f"z_mirror_{t}t": {"SVDs_per_s": 1.0e6, "sample": "x"} for t in (1, 16)},
           "upcast": {"s": {"SVDs_per_s": 1.01234e8, "sample": "3 x 1048576 matrices", "threads": 16},
                      "c": {"SVDs_per_s": 5.01234e7, "sample": "2 x 1048576 matrices", "threads": 16}},
           "check": {v: dict(check) for v in "zdsc"}}
    return {"head": "z", "metric": bench.METRIC, "value": h["svds_per_s"], "unit": "SVDs/s", "n_gpus": 1,
            "steps": 20, "warmup": 3, "ms_per_step": h["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic (seeded +-m 2^e law with 1% special lanes; stands in for the paper's "
                    "private random-bit file)",
            "config": {"workload": "complex FP64 batched 2x2 SVD", "n": n24, "layout": "SoA",
                       "exponents": "e in [-1000,1000]", "special_lanes": 0.01, "launch": [128, 2]},
            "roofline": {"bound": "hbm", "achieved": h["algorithmic_GBs"], "peak": bench.HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": h["hbm_frac"], "traffic": 3.624939e9,
                         "traffic_unit": "bytes per launch", "algorithmic_bytes_per_launch": 216 * n24,
                         "kernel_ms": h["kernel_ms"], "valu_frac": h["valu_frac"],
                         "pattern_ceiling_GBs": h["pattern_ceiling_GBs"],
                         "frac_of_pattern_ceiling": h["frac_of_pattern_ceiling"]},
            "cpu_baseline": cpu, "variants": variants, "kogbetliantz": kog, "kogbetliantz_batch": batch,
            "kernel_source_sha": "0123456789abcdef"}


def test_headline_is_compact_and_last_on_stdout(capsys, tmp_path):
    full = fake_full()
    path = tmp_path / "detail.json"
    bench.emit(full, str(path))
    out, err = capsys.readouterr()
    lines = out.strip().splitlines()
    last = lines[-1]
    assert len(last.encode()) < 3600, len(last.encode())  # the driver keeps 8000 characters
    line = json.loads(last)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in line, k
    rl = line["roofline"]
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0 and rl["traffic"] > 0
    assert abs(rl["frac"] - rl["achieved"] / rl["peak"]) < 1e-3
    assert set(line["cpu_baseline"]) >= {"value", "unit", "cores", "kind", "sample"}
    assert line["cpu_baseline"]["kind"] == "oracle"
    assert line["cpu_baseline"]["gpu_vs_oracle_sample"]["z"]["s_equal"] is True
    # one entry per variant; one rescued-lane fraction per base variant (its rescue variants agree)
    assert len(line["variants"]) == 26 and all(len(v) == 3 for v in line["variants"].values())
    assert line["rescued_frac"] == {"s": 0.83, "c": 0.83, "s26": 0.83, "c26": 0.83}
    assert line["kogbetliantz"]["sweeps_per_s"]["two_step"] > 0
    assert line["kogbetliantz_batch"]["nprob"] == 256 and "problems" not in line["kogbetliantz_batch"]
    # the detail keeps what the headline leaves out
    det = json.loads(path.read_text())
    assert len(det["kogbetliantz_batch"]["problems"]) == 256
    assert "[bench] detail: " in err


def test_valu_fraction_and_bound():
    # one wave instruction serves 64 matrices and holds a SIMD for 4 cycles;
    # 1024 SIMDs at 2.4 GHz: 400 instructions per matrix over 2^24 matrices
    # need 0.17 ms of issue time, more than the 0.1 ms given
    f = bench.valu_frac(400, 1 << 24, 0.1)
    assert abs(f - 400 * (1 << 24) / 64 * 4 / (0.1e-3 * 2.4e9 * 1024)) < 1e-12
    s = bench.summarize("s", fake_run(1 << 24, 0.1), fake_run(1 << 24, 0.1), "", False, 400)
    assert s["bound"] == "valu" and s["valu_frac"] > s["hbm_frac"]
    s = bench.summarize("z", fake_run(1 << 24, 0.66), fake_run(1 << 24, 0.63), "", False, None)
    assert s["bound"] == "hbm" and s["valu_frac"] is None


def test_rescue_mode_mapping():
    assert bench.rescue_mode(0) == 0
    assert bench.rescue_mode(4) == 1
    assert bench.rescue_mode(4 | 16) == 2
    assert bench.rescue_mode(4 | 128) == 3
    assert bench.rescue_mode(4 | 8 | 16) == 2
    assert np.isclose(bench.r4(1.234567e10), 1.235e10)
