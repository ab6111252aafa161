"""GPU parity of the batched 2x2 SVD (HIP path through the C ABI) against the
CPU oracle, on seeded inputs.  Bar: s exact, sigma' within 4 ulp, U/V within
4 eps, and rho, delta, eta (eqs. (33)-(35)) at most 16 eps in binary128.  The
kernels follow the oracle's operation order, so the lanes are expected to be
bitwise identical; the count is reported and required to be all lanes."""
import numpy as np
import pytest

import oracle.oracle as O
from tests.gpu_util import compare, oracle_outs, run_gpu, same_bits
from workloads import SEED_BASE, random_bits, scaled_law, to_trains, uniform_real

pytestmark = pytest.mark.gpu

EPS = {np.float64: 2.0 ** -52, np.float32: 2.0 ** -23}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2005_07403_amd import svd2 as S
    S.lib()
    yield
    S.svd2_set_launch(256, 1)


def _set_launch(block, pt):
    from paper_2005_07403_amd import svd2 as S
    S.svd2_set_launch(block, pt)


def _check(A, dtype, flags=0, rescue=False, backscale="none", expect_bitwise=True, metrics=True):
    cplx = bool(np.iscomplexobj(A))
    tr = to_trains(A, dtype)
    from paper_2005_07403_amd import svd2 as S
    if dtype == np.float32:
        gpu, nres = run_gpu(tr, flags=flags, nrescued=True)
    else:
        gpu, nres = run_gpu(tr, flags=flags), None
    ora, flagged = oracle_outs(tr, cplx, dtype, rescue=rescue, backscale=backscale)
    st = compare(gpu, ora, cplx, EPS[dtype])
    if expect_bitwise:
        assert st["bitwise_lanes"] == st["lanes"], st
    if rescue:
        assert nres == int(flagged.sum()), (nres, int(flagged.sum()))
    if metrics:
        met = O.metrics(tr, gpu, cplx)
        for key in ("rho", "delta", "eta"):
            assert np.nanmax(met[key]) <= 16 * EPS[dtype], (key, np.nanmax(met[key]) / EPS[dtype])
    del S
    return st


# ---------------------------------------------------------------------------
# T0: the device primitives are the IEEE-754 operations the oracle uses
# ---------------------------------------------------------------------------

def _rand_f64(rng, n):
    bits = rng.integers(0, 2 ** 63, size=n, dtype=np.int64).view(np.float64)
    return np.where(np.isfinite(bits), bits, 1.0)


def _fraction_round(fr, dtype):
    """Correctly rounded Fraction -> dtype (ties to even)."""
    from fractions import Fraction
    f = np.array(float(fr), dtype=dtype)
    best = None
    for c in (np.nextafter(f, -np.inf, dtype=dtype), f, np.nextafter(f, np.inf, dtype=dtype)):
        if not np.isfinite(c):
            continue
        d = abs(Fraction(float(c)) - fr)
        if best is None or d < best[0] or (d == best[0] and (int(np.array(c).view(
                np.int64 if dtype == np.float64 else np.int32)) % 2 == 0)):
            best = (d, c)
    return best[1]


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_primitives_correctly_rounded(dtype):
    import torch
    from fractions import Fraction
    from paper_2005_07403_amd import svd2 as S
    rng = np.random.default_rng(SEED_BASE + 100)
    n = 1 << 20
    if dtype == np.float64:
        x, y, z = _rand_f64(rng, n), _rand_f64(rng, n), _rand_f64(rng, n)
        # plus values near 1 and in [1,3] (the invsqrt arguments), and subnormals
        x[: n // 8] = rng.uniform(1, 3, n // 8)
        y[n // 8: n // 4] = np.ldexp(rng.integers(1, 2 ** 52, n // 8).astype(np.float64), -1074)
    else:
        x = (rng.standard_normal(n) * np.exp2(rng.integers(-140, 120, n))).astype(np.float32)
        y = (rng.standard_normal(n) * np.exp2(rng.integers(-140, 120, n))).astype(np.float32)
        z = (rng.standard_normal(n) * np.exp2(rng.integers(-140, 120, n))).astype(np.float32)
    dt = torch.float64 if dtype == np.float64 else torch.float32
    tx, ty, tz = (torch.from_numpy(a).cuda() for a in (x, y, z))
    out = torch.empty_like(tx)

    def run(op, a=tx, b=ty, c=tz):
        S.svd2_probe(op, a, b, c, out)
        torch.cuda.synchronize()
        return out.cpu().numpy().copy()

    with np.errstate(all="ignore"):
        assert np.array_equal(run(0), x / y, equal_nan=True), "division"
        ax = np.abs(x)
        tax = torch.from_numpy(ax).cuda()
        assert np.array_equal(run(1, tax), np.sqrt(ax)), "sqrt"
        # ldexp with subnormal results, including s = -1, -2 on huge values
        e = rng.integers(-1200 if dtype == np.float64 else -300, 60, n).astype(dtype)
        te = torch.from_numpy(e).cuda()
        assert np.array_equal(run(3, tx, te), np.ldexp(x, e.astype(np.int64)).astype(dtype)), "ldexp"
        fe = np.frexp(x)[1].astype(dtype)
        got = run(4)
        nz = x != 0
        assert np.array_equal(got[nz], fe[nz]), "frexp exponent"
    # fma: exact rational reference on a sample
    got = run(2)
    idx = rng.choice(n, 4000, replace=False)
    for i in idx:
        exact = Fraction(float(x[i])) * Fraction(float(y[i])) + Fraction(float(z[i]))
        if abs(exact) >= Fraction(float(np.finfo(dtype).max)):
            continue
        want = _fraction_round(exact, dtype)
        assert same_bits(np.array([got[i]], dtype=dtype), np.array([want], dtype=dtype))[0], i
    # relaxed min/max: a NaN first argument yields the second
    nan = np.full(8, np.nan, dtype=dtype)
    two = np.full(8, 2.0, dtype=dtype)
    tn, tt = torch.from_numpy(nan).cuda(), torch.from_numpy(two).cuda()
    o8 = torch.empty_like(tn)
    S.svd2_probe(5, tn, tt, None, o8)
    torch.cuda.synchronize()
    assert np.all(o8.cpu().numpy() == 2.0)
    S.svd2_probe(6, tn, tt, None, o8)
    torch.cuda.synchronize()
    assert np.all(o8.cpu().numpy() == 2.0)


def _bits_equal_dev(a, b):
    import torch
    ia = a.view(torch.int32 if a.dtype == torch.float32 else torch.int64)
    ib = b.view(torch.int32 if b.dtype == torch.float32 else torch.int64)
    return bool(torch.equal(ia, ib))


def test_sqrt_and_reciprocal_on_their_domain_fp32_every_argument():
    """The kernels' square root (every x in [1, FLT_MAX]) and reciprocal (every
    x in [1, 2^126), where 1/x is normal) are bitwise the correctly rounded
    sqrt and division of the same device (themselves checked against numpy
    above), on every FP32 argument of those domains."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    chunk = 1 << 26
    for op, ref_op, lo, hi in ((7, 1, 0x3F800000, 0x7F7FFFFF), (8, 0, 0x3F800000, 0x7E7FFFFF)):
        base = lo
        while base <= hi:
            m = min(chunk, hi - base + 1)
            x = torch.arange(base, base + m, dtype=torch.int64, device="cuda").to(torch.int32).view(torch.float32)
            got, want = torch.empty_like(x), torch.empty_like(x)
            S.svd2_probe(op, x, None, None, got)
            if ref_op == 1:
                S.svd2_probe(1, x, None, None, want)
            else:
                S.svd2_probe(0, torch.ones_like(x), x, None, want)
            torch.cuda.synchronize()
            assert _bits_equal_dev(got, want), (op, hex(base))
            base += m
    # and against numpy on a sample of each domain
    rng = np.random.default_rng(SEED_BASE + 77)
    xs = rng.integers(0x3F800000, 0x7F7FFFFF, 1 << 16, dtype=np.int64).astype(np.int32).view(np.float32)
    tx = torch.from_numpy(xs).cuda()
    out = torch.empty_like(tx)
    S.svd2_probe(7, tx, None, None, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), np.sqrt(xs))
    xr = rng.integers(0x3F800000, 0x7E7FFFFF, 1 << 16, dtype=np.int64).astype(np.int32).view(np.float32)
    tx = torch.from_numpy(xr).cuda()
    S.svd2_probe(8, tx, None, None, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), np.float32(1) / xr)


def test_sqrt_and_reciprocal_on_their_domain_fp64_sampled():
    """The FP64 square root on x >= 1 and reciprocal on [1, 2^1022] against
    the device's correctly rounded sqrt and division and numpy: random
    exponents and mantissas, the neighbourhoods of exact squares (where the
    rounding of sqrt is decided), powers of two and their neighbours."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    rng = np.random.default_rng(SEED_BASE + 78)
    n = 1 << 22
    m = rng.integers(0, 1 << 52, n, dtype=np.int64)
    e = rng.integers(1023, 2046, n, dtype=np.int64)           # exponents 0 .. 1022
    x = ((e << 52) | m).view(np.float64)
    r = rng.integers(1 << 26, 1 << 27, n // 4, dtype=np.int64).astype(np.float64)
    sq = r * r                                                 # exact squares (< 2^54)
    sq = sq[sq < 2.0 ** 53]
    near = np.concatenate([np.nextafter(sq, 0), sq, np.nextafter(sq, np.inf)])
    p2 = np.ldexp(1.0, np.arange(0, 1023))
    x = np.concatenate([x, near, p2, np.nextafter(p2, np.inf), np.nextafter(p2[1:], 0),
                        1.0 + np.arange(1, 4096) * np.finfo(np.float64).eps])
    tx = torch.from_numpy(x).cuda()
    got, want = torch.empty_like(tx), torch.empty_like(tx)
    S.svd2_probe(7, tx, None, None, got)
    S.svd2_probe(1, tx, None, None, want)
    torch.cuda.synchronize()
    assert _bits_equal_dev(got, want)
    assert np.array_equal(got.cpu().numpy(), np.sqrt(x))
    xr = x[x <= 2.0 ** 1022]
    tx = torch.from_numpy(xr).cuda()
    got, want = torch.empty_like(tx), torch.empty_like(tx)
    S.svd2_probe(8, tx, None, None, got)
    S.svd2_probe(0, torch.ones_like(tx), tx, None, want)
    torch.cuda.synchronize()
    assert _bits_equal_dev(got, want)
    assert np.array_equal(got.cpu().numpy(), 1.0 / xr)


# ---------------------------------------------------------------------------
# FP64 parity
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("block,pt", [(256, 1), (256, 2), (64, 1), (128, 2)])
def test_real_uniform_65536(block, pt):
    """Real FP64, n = 65536, entries U[-1, 1] (the small parity workload)."""
    _set_launch(block, pt)
    _check(uniform_real(65536, SEED_BASE + 0), np.float64)


@pytest.mark.parametrize("pt", [1, 2])
def test_complex_scaled_law_ragged(pt):
    """Complex FP64 with the +-m 2^e law and 1 % special lanes, ragged n."""
    _set_launch(256, pt)
    A, kinds = scaled_law((1 << 18) + 37, SEED_BASE + 1, True, return_kinds=True)
    st = _check(A, np.float64)
    assert (kinds >= 0).sum() > 2000
    del st


@pytest.mark.parametrize("cplx", [False, True])
def test_random_bits(cplx):
    """The paper's own input law: random 64-bit patterns, finite only."""
    _set_launch(256, 2)
    _check(random_bits(200003, SEED_BASE + 5, cplx), np.float64)


@pytest.mark.parametrize("kind", range(6))
@pytest.mark.parametrize("cplx", [False, True])
def test_special_lanes_only(kind, cplx):
    A, kinds = scaled_law(30000, SEED_BASE + 10 + kind, cplx, special_frac=1.0, return_kinds=True)
    sel = kinds == kind
    _check(A[:, sel], np.float64)


@pytest.mark.parametrize("mode", ["safe", "all"])
@pytest.mark.parametrize("cplx", [False, True])
def test_backscale_modes(mode, cplx):
    from paper_2005_07403_amd import svd2 as S
    flags = S.SVD2_BACKSCALE_SAFE if mode == "safe" else S.SVD2_BACKSCALE_ALL
    A = scaled_law(50000, SEED_BASE + 20, cplx)
    _check(A, np.float64, flags=flags, backscale=mode, metrics=(mode == "safe"))


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 255, 257, 1023])
def test_small_and_ragged_sizes(n):
    for pt in (1, 2):
        _set_launch(64, pt)
        _check(scaled_law(n, SEED_BASE + 30 + n, True), np.float64, metrics=False)
        _check(scaled_law(n, SEED_BASE + 31 + n, False), np.float64, metrics=False)


def test_unaligned_falls_back_and_matches():
    """Arrays offset by one element (8-byte aligned only) take the scalar
    path and still match."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    _set_launch(256, 2)
    n = 10001
    A = scaled_law(n, SEED_BASE + 40, False)
    tr = to_trains(A)
    big = [torch.zeros(n + 1, dtype=torch.float64, device="cuda") for _ in range(4)]
    ins = []
    for b, t in zip(big, tr):
        b[1:] = torch.from_numpy(t).cuda()
        ins.append(b[1:])
    outs = [torch.empty(n + 1, dtype=torch.float64, device="cuda")[1:] for _ in range(11)]
    S.dsvd2_batch(n, [t.data_ptr() for t in ins], [t.data_ptr() for t in outs])
    torch.cuda.synchronize()
    gpu = [o.cpu().numpy() for o in outs]
    ora, _ = oracle_outs(tr, False, np.float64)
    st = compare(gpu, ora, False, EPS[np.float64])
    assert st["bitwise_lanes"] == n


@pytest.mark.parametrize("kind", ["d", "z", "s", "c"])
def test_stream_probe(kind):
    """The memory-pattern probe touches exactly the batched kernel's arrays."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    n = 10007
    dt = torch.float64 if kind in "dz" else torch.float32
    nin, nout = (8, 19) if kind in "zc" else (4, 11)
    ins = [torch.full((n,), float(i + 1), dtype=dt, device="cuda") for i in range(nin)]
    outs = [torch.zeros(n, dtype=dt, device="cuda") for _ in range(nout)]
    S.svd2_stream_probe(kind, ins, outs)
    torch.cuda.synchronize()
    tot = nin * (nin + 1) / 2
    for i, o in enumerate(outs):
        assert torch.all(o == tot + i)


def test_lane_isolation_nonfinite():
    """A lane with Inf/NaN input must not disturb the other lanes."""
    A = scaled_law(4096, SEED_BASE + 41, True)
    A[0, 5] = np.inf
    A[2, 77] = complex(np.nan, 1.0)
    tr = to_trains(A)
    gpu = run_gpu(tr)
    ora, _ = oracle_outs(tr, True, np.float64)
    ok = np.ones(4096, dtype=bool)
    ok[[5, 77]] = False
    compare(gpu, ora, True, EPS[np.float64], lanes=ok)


def _bench_shape(kind):
    """Set and return the launch shape the benchmark times for `kind`: the
    autotuner's table when present (bench.py loads it), else its default."""
    from bench import DEFAULT_LAUNCH
    from paper_2005_07403_amd import svd2 as S
    tab = S.apply_tuning() or {}
    shape = tuple(int(x) for x in tab.get("svd2_launch", {}).get(kind, DEFAULT_LAUNCH[kind]))
    S.svd2_set_launch_kind(kind, *shape)
    assert tuple(S.svd2_get_launch_kind(kind)) == shape
    return shape


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["z", "d"])
def test_full_size_2_24_in_the_benchmark_shape(kind):
    """The full FP64 workloads the benchmark times: n = 2^24 matrices, +-m 2^e,
    e in [-1000, 1000], 1 % special lanes, complex (the headline) and real,
    in the launch shape the benchmark uses.  Every lane is compared with the
    oracle."""
    shape = _bench_shape(kind)
    A = scaled_law(1 << 24, SEED_BASE + 1, kind == "z")
    st = _check(A, np.float64, metrics=False)
    assert st["lanes"] == 1 << 24
    print(f"{kind} n=2^24 shape {shape}: {st}")


# ---------------------------------------------------------------------------
# FP32 form and the FP64 rescue
# ---------------------------------------------------------------------------

RESCUE_MODES = ["plain", "inplace", "queue", "sigma", "sigma_queue", "tri", "tri_queue"]


def _fp32_flags(mode):
    from paper_2005_07403_amd import svd2 as S
    return {"plain": 0, "inplace": S.SVD2_RESCUE_FP64,
            "queue": S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_QUEUE,
            "sigma": S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_SIGMA,
            "sigma_queue": S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_SIGMA | S.SVD2_RESCUE_QUEUE,
            "tri": S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_TRI,
            "tri_queue": S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_TRI | S.SVD2_RESCUE_QUEUE}[mode]


def _oracle_rescue(mode):
    if mode == "plain":
        return 0
    return 2 if mode.startswith("sigma") else (3 if mode.startswith("tri") else 1)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("mode", RESCUE_MODES)
def test_fp32_modes(cplx, mode):
    _set_launch(256, 2)
    A = scaled_law((1 << 17) + 5, SEED_BASE + 2, cplx, dtype=np.float32)
    _check(A, np.float32, flags=_fp32_flags(mode), rescue=_oracle_rescue(mode),
           metrics=(mode != "plain"))


@pytest.mark.parametrize("cplx", [False, True])
def test_fp32_rescue_near_singular(cplx):
    from paper_2005_07403_amd import svd2 as S
    rng = np.random.default_rng(SEED_BASE + 50)
    n = 20000
    u = rng.standard_normal((2, n)) + (1j * rng.standard_normal((2, n)) if cplx else 0)
    v = rng.standard_normal((2, n)) + (1j * rng.standard_normal((2, n)) if cplx else 0)
    A = np.stack([u[0] * np.conj(v[0]), u[1] * np.conj(v[0]), u[0] * np.conj(v[1]),
                  u[1] * np.conj(v[1])]) + 3e-8 * rng.standard_normal((4, n))
    A = A.astype(np.complex64 if cplx else np.float32)
    for mode in RESCUE_MODES[1:]:
        _check(A, np.float32, flags=_fp32_flags(mode), rescue=_oracle_rescue(mode))


@pytest.mark.parametrize("cplx", [False, True])
def test_fp32_caller_workspace(cplx):
    """A workspace the caller passes in is checked at the size it really has:
    one byte short of svd2_workspace_bytes is refused before anything runs,
    and a buffer of exactly that size in another dtype gives the same bits as
    the one the binding allocates."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    from tests.gpu_util import to_dev
    n = 4099
    dev = to_dev(to_trains(scaled_law(n, SEED_BASE + 51, cplx, dtype=np.float32), np.float32))
    fl = _fp32_flags("queue")
    need = S.svd2_workspace_bytes(n, fl)
    assert need % 4 == 0
    ref = [o.cpu() for o in S.svd2(dev, flags=fl)]
    short = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(S.Svd2Error) as err:
        S.svd2(dev, flags=fl, ws=short)
    assert err.value.status == 6
    exact = torch.empty(need // 4, dtype=torch.int32, device="cuda")
    got = [o.cpu() for o in S.svd2(dev, flags=fl, ws=exact)]
    for a, b in zip(ref, got):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))


@pytest.mark.slow
@pytest.mark.parametrize("cplx", [False, True])
def test_fp32_full_size_2_26_sampled(cplx):
    """The FP32 workload at n = 2^26 with the FP64 rescue; the oracle checks
    a random sample of 2^20 lanes of the full-size run."""
    import torch
    from bench import DEFAULT_LAUNCH
    from paper_2005_07403_amd import svd2 as S
    _set_launch(*DEFAULT_LAUNCH["c" if cplx else "s"])
    n = 1 << 26
    A = scaled_law(n, SEED_BASE + 2, cplx, dtype=np.float32)
    tr = to_trains(A)
    del A
    dev = [torch.from_numpy(t).cuda() for t in tr]
    out = S.svd2(dev, flags=S.SVD2_RESCUE_FP64)
    torch.cuda.synchronize()
    rng = np.random.default_rng(SEED_BASE + 60)
    idx = np.sort(rng.choice(n, 1 << 20, replace=False))
    tidx = torch.from_numpy(idx).cuda()
    gpu = [o[tidx].cpu().numpy() for o in out]
    sub = [np.ascontiguousarray(t[idx]) for t in tr]
    ora, _ = oracle_outs(sub, cplx, np.float32, rescue=True)
    st = compare(gpu, ora, cplx, EPS[np.float32])
    assert st["bitwise_lanes"] == st["lanes"]


@pytest.mark.slow
def test_fp32_batch_over_several_launches():
    """A batch longer than one launch's span (2^30 bytes per array, 2^28
    FP32 matrices): n = 2^28 + 3 real FP32 matrices, two matrices per lane
    with a one-matrix tail.  The lanes around the boundary between launches
    and a random sample elsewhere are bitwise the oracle's; the queued rescue
    (whole-batch queue indices) gives byte for byte the in-place rescue's
    outputs and the same rescued-lane count."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    S.svd2_set_launch_kind("s", 256, 2)
    n = (1 << 28) + 3
    A = scaled_law(n, SEED_BASE + 61, False, dtype=np.float32)
    tr = to_trains(A)
    del A
    dev = [torch.from_numpy(t).cuda() for t in tr]
    cnt1 = torch.zeros(1, dtype=torch.int32, device="cuda")
    cnt2 = torch.zeros(1, dtype=torch.int32, device="cuda")
    out1 = S.svd2(dev, flags=S.SVD2_RESCUE_FP64, nrescued=cnt1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(SEED_BASE + 62)
    idx = np.unique(np.concatenate([np.arange((1 << 28) - 300, n), np.arange(0, 64),
                                    rng.choice(n, 1 << 18, replace=False)]))
    tidx = torch.from_numpy(idx).cuda()
    gpu = [o[tidx].cpu().numpy() for o in out1]
    sub = [np.ascontiguousarray(t[idx]) for t in tr]
    ora, _ = oracle_outs(sub, False, np.float32, rescue=True)
    st = compare(gpu, ora, False, EPS[np.float32])
    assert st["bitwise_lanes"] == st["lanes"], st
    del gpu
    ws = torch.empty(S.svd2_workspace_bytes(n, S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_QUEUE), dtype=torch.uint8,
                     device="cuda")
    out2 = S.svd2(dev, flags=S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_QUEUE, ws=ws, nrescued=cnt2)
    torch.cuda.synchronize()
    assert int(cnt1.item()) == int(cnt2.item()) > 0
    for a, b in zip(out1, out2):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    S.svd2_set_launch(256, 1)


# ---------------------------------------------------------------------------
# singular values only (SVD2_NO_UV)
# ---------------------------------------------------------------------------

def _raw(a):
    return np.ascontiguousarray(a).view(np.uint8)


@pytest.mark.parametrize("pt", [1, 2])
@pytest.mark.parametrize("kind,mode", [("d", "none"), ("d", "safe"), ("d", "all"), ("z", "none"),
                                       ("z", "safe"), ("z", "all")] +
                         [(k, m) for k in "sc" for m in RESCUE_MODES])
def test_singular_values_only(kind, mode, pt):
    """smax, smin and s of a NO_UV call are byte for byte those of the full
    call (signed zeros included) and bitwise the oracle's; the rescued-lane
    count is unchanged; U and V are not written (NULL pointers)."""
    import torch
    from paper_2005_07403_amd import svd2 as S
    _set_launch(256, pt)
    cplx, dtype = kind in "zc", np.float64 if kind in "dz" else np.float32
    A = scaled_law((1 << 17) + 5, SEED_BASE + 60, cplx, dtype=dtype)
    tr = to_trains(A, dtype)
    dev = [torch.from_numpy(t).cuda() for t in tr]
    if dtype == np.float64:
        flags = {"none": 0, "safe": S.SVD2_BACKSCALE_SAFE, "all": S.SVD2_BACKSCALE_ALL}[mode]
        rescue, backscale = False, mode
    else:
        flags, rescue, backscale = _fp32_flags(mode), _oracle_rescue(mode), "none"
    c1 = torch.zeros(1, dtype=torch.int32, device="cuda")
    c2 = torch.zeros(1, dtype=torch.int32, device="cuda")
    full = S.svd2(dev, flags=flags, nrescued=c1 if dtype == np.float32 else None)
    sig = S.svd2(dev, flags=flags | S.SVD2_NO_UV, nrescued=c2 if dtype == np.float32 else None)
    torch.cuda.synchronize()
    assert len(sig) == 3
    k = 16 if cplx else 8
    ora, flagged = oracle_outs(tr, cplx, dtype, rescue=rescue, backscale=backscale)
    for j in range(3):
        g, f = sig[j].cpu().numpy(), full[k + j].cpu().numpy()
        assert np.array_equal(_raw(g), _raw(f)), (kind, mode, j)
        assert same_bits(g, ora[k + j]).all(), (kind, mode, j)
    if dtype == np.float32:
        assert int(c1.item()) == int(c2.item()) == (int(flagged.sum()) if rescue else 0)


# ---------------------------------------------------------------------------
# sine form of the assembly (SVD2_SINE_FORM, eq. (31))
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("pt", [1, 2])
@pytest.mark.parametrize("kind,mode", [("d", "none"), ("z", "none"), ("d", "safe"), ("z", "all")] +
                         [(k, m) for k in "sc" for m in RESCUE_MODES])
def test_sine_form_bitwise(kind, mode, pt):
    """Every output of an SVD2_SINE_FORM call is bitwise the oracle's sine
    form, in every backscale and rescue mode (the FP64 tail rescue assembles
    in FP64 by the same form), both launch shapes."""
    from paper_2005_07403_amd import svd2 as S
    _set_launch(256, pt)
    cplx, dtype = kind in "zc", np.float64 if kind in "dz" else np.float32
    A = scaled_law((1 << 16) + 3, SEED_BASE + 65, cplx, dtype=dtype)
    tr = to_trains(A, dtype)
    if dtype == np.float64:
        flags = {"none": 0, "safe": S.SVD2_BACKSCALE_SAFE, "all": S.SVD2_BACKSCALE_ALL}[mode]
        rescue, backscale = False, mode
        gpu = run_gpu(tr, flags=flags | S.SVD2_SINE_FORM)
    else:
        flags, rescue, backscale = _fp32_flags(mode), _oracle_rescue(mode), "none"
        gpu, nres = run_gpu(tr, flags=flags | S.SVD2_SINE_FORM, nrescued=True)
    ora, flagged = O.run_trains(tr, cplx, dtype, policy="mirror", backscale=backscale, rescue=rescue,
                                form="sine")
    for i, (g, o) in enumerate(zip(gpu, ora)):
        assert same_bits(g, o).all(), (kind, mode, i, int((~same_bits(g, o)).sum()))
