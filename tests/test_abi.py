"""C-ABI contract of libsvd2.so on the CPU: the library loads without a GPU,
exports every symbol include/svd2.h declares, and rejects bad arguments with
status codes before any HIP call is made (no compute call is made here)."""
import ctypes
import os
import re

import pytest

from paper_2005_07403_amd import svd2 as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "svd2.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(\w+)\s*\([^;{]*\)\s*;", txt)) - {"if", "return"})


def test_library_exports_every_declared_symbol():
    L = S.lib()
    names = _header_functions()
    assert "dsvd2_batch" in names and "csvd2_batch" in names
    for name in names:
        assert hasattr(L, name), name
    for name in S.EXPORTS:
        assert name in names, name


FAKE = 1 << 40  # host-side fake "device" addresses: never dereferenced


def _ptrs(count, base=FAKE, stride=1 << 30):
    return [base + i * stride for i in range(count)]


def _call(fn, n, ins, outs, flags=0, **kw):
    try:
        fn(n, ins, outs, flags, stream=0, **kw) if not kw else fn(n, ins, outs, flags, stream=0, **kw)
    except S.Svd2Error as e:
        return e.status
    return 0


@pytest.mark.parametrize("fn,nin,nout", [(S.dsvd2_batch, 4, 11), (S.zsvd2_batch, 8, 19),
                                         (S.ssvd2_batch, 4, 11), (S.csvd2_batch, 8, 19)])
def test_argument_errors(fn, nin, nout):
    ins, outs = _ptrs(nin), _ptrs(nout, base=FAKE + (64 << 30))
    # n == 0 with valid pointers: no-op, no HIP call
    assert _call(fn, 0, ins, outs) == 0
    # NULL pointer
    bad = list(outs)
    bad[3] = 0
    assert _call(fn, 10, ins, bad) == 1
    # misaligned pointer
    bad = list(ins)
    bad[1] += 1
    assert _call(fn, 10, bad, outs) == 2
    # output overlapping another output
    bad = list(outs)
    bad[2] = bad[1] + 8
    assert _call(fn, 10, ins, bad) == 3
    # output overlapping an input
    bad = list(outs)
    bad[0] = ins[2]
    assert _call(fn, 10, ins, bad) == 3
    # adjacent but disjoint ranges are fine (n = 0 avoids any launch)
    ok = [FAKE + i * 80 for i in range(nin + nout)]
    assert _call(fn, 0, ok[:nin], ok[nin:]) == 0
    # the sine form of the assembly and singular values only are valid flags
    assert _call(fn, 0, ins, outs, flags=S.SVD2_SINE_FORM) == 0
    assert _call(fn, 0, ins, outs, flags=S.SVD2_SINE_FORM | S.SVD2_NO_UV) == 0
    # contradictory backscale flags
    assert _call(fn, 10, ins, outs, flags=3) == 4
    # unknown flag bits
    assert _call(fn, 10, ins, outs, flags=1 << 12) == 4


@pytest.mark.parametrize("fn,nin,nuv", [(S.dsvd2_batch, 4, 8), (S.zsvd2_batch, 8, 16),
                                        (S.ssvd2_batch, 4, 8), (S.csvd2_batch, 8, 16)])
def test_singular_values_only_arguments(fn, nin, nuv):
    """SVD2_NO_UV: U and V pointers may be NULL (or anything: they are neither
    checked nor written); smax, smin, s are checked as without the flag."""
    ins = _ptrs(nin)
    sig = _ptrs(3, base=FAKE + (64 << 30))
    f = S.SVD2_NO_UV
    assert _call(fn, 0, ins, [0] * nuv + sig, flags=f) == 0
    junk = [ins[0] + 1] * nuv  # misaligned and overlapping an input: ignored
    assert _call(fn, 0, ins, junk + sig, flags=f) == 0
    assert _call(fn, 10, ins, [0] * nuv + sig) == 1  # without the flag U and V are needed
    assert _call(fn, 10, ins, [0] * nuv + [sig[0], 0, sig[2]], flags=f) == 1
    assert _call(fn, 10, ins, [0] * nuv + [sig[0], sig[0] + 8, sig[2]], flags=f) == 3
    assert _call(fn, 10, ins, [0] * nuv + [sig[0], sig[1] + 1, sig[2]], flags=f) == 2
    assert _call(fn, 10, ins, [0] * nuv + [sig[0], ins[1], sig[2]], flags=f) == 3


def _call_urv(fn, n, ins, outs, f, flags=0, **kw):
    try:
        fn(n, ins, outs, f, flags, stream=0, **kw)
    except S.Svd2Error as e:
        return e.status
    return 0


@pytest.mark.parametrize("fn,nin,nout", [(S.dsvd2_batch_urv, 4, 11), (S.zsvd2_batch_urv, 8, 19),
                                         (S.ssvd2_batch_urv, 4, 11), (S.csvd2_batch_urv, 8, 19)])
def test_phase_output_arguments(fn, nin, nout):
    """The *_batch_urv entry points: R required, U_+ and V_+ all or none,
    no backscale, the phase outputs in the alias and alignment checks."""
    ins, outs = _ptrs(nin), _ptrs(nout, base=FAKE + (64 << 30))
    f = _ptrs(nout, base=FAKE + (128 << 30))
    r_only = f[:3] + [0] * (nout - 3)
    assert _call_urv(fn, 0, ins, outs, f) == 0
    assert _call_urv(fn, 0, ins, outs, r_only) == 0
    assert _call_urv(fn, 0, ins, [0] * (nout - 3) + outs[-3:], r_only, flags=S.SVD2_NO_UV) == 0
    assert _call_urv(fn, 0, ins, outs, f, flags=S.SVD2_SINE_FORM) == 0
    for i in range(3):  # R is required
        bad = list(f)
        bad[i] = 0
        assert _call_urv(fn, 10, ins, outs, bad) == 1
    bad = list(f)
    bad[5] = 0  # U_+ / V_+ partly given
    assert _call_urv(fn, 10, ins, outs, bad) == 1
    # the backscale flags are refused: R, U_+ and V_+ belong to 2^s A
    assert _call_urv(fn, 10, ins, outs, f, flags=S.SVD2_BACKSCALE_SAFE) == 4
    assert _call_urv(fn, 10, ins, outs, f, flags=S.SVD2_BACKSCALE_ALL) == 4
    assert _call_urv(fn, 10, ins, outs, f, flags=1 << 12) == 4
    bad = list(f)
    bad[1] += 1  # misaligned R
    assert _call_urv(fn, 10, ins, outs, bad) == 2
    bad = list(f)
    bad[nout - 1] = ins[0]  # V_+ over an input
    assert _call_urv(fn, 10, ins, outs, bad) == 3
    bad = list(f)
    bad[2] = outs[4] + 8  # R over an output
    assert _call_urv(fn, 10, ins, outs, bad) == 3
    bad = r_only[:]
    bad[0] = bad[1]  # two phase outputs on one array
    assert _call_urv(fn, 10, ins, outs, bad) == 3
    # NULL structs
    L = S.lib()
    raw = getattr(L, fn.__name__)
    args = (10, None, None, 0, None) if fn.__name__[0] in "dz" else (10, None, None, 0, None, 0, None)
    assert raw(*args) == 1


def test_singular_values_only_launch_kinds():
    old = S.svd2_get_launch_kind("z_nouv")
    S.svd2_set_launch_kind("z_nouv", 128, 2)
    assert S.svd2_get_launch_kind("z_nouv") == (128, 2)
    S.svd2_set_launch_kind("z_nouv", *old)
    assert S.lib().svd2_set_launch_kind(8, 256, 1) == 4


def test_fp64_rejects_fp32_flags():
    ins, outs = _ptrs(4), _ptrs(11, base=FAKE + (64 << 30))
    assert _call(S.dsvd2_batch, 10, ins, outs, flags=S.SVD2_RESCUE_FP64) == 4


def test_fp32_queue_needs_rescue_and_workspace():
    ins, outs = _ptrs(4), _ptrs(11, base=FAKE + (64 << 30))
    assert _call(S.ssvd2_batch, 10, ins, outs, flags=S.SVD2_RESCUE_QUEUE) == 4
    assert _call(S.ssvd2_batch, 10, ins, outs, flags=S.SVD2_RESCUE_SIGMA) == 4
    assert _call(S.dsvd2_batch, 10, ins, outs, flags=S.SVD2_RESCUE_SIGMA) == 4
    # the middle rescue: needs RESCUE_FP64, excludes RESCUE_SIGMA, FP32 only
    assert _call(S.ssvd2_batch, 10, ins, outs, flags=S.SVD2_RESCUE_TRI) == 4
    assert _call(S.ssvd2_batch, 10, ins, outs,
                 flags=S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_SIGMA | S.SVD2_RESCUE_TRI) == 4
    assert _call(S.dsvd2_batch, 10, ins, outs, flags=S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_TRI) == 4
    # queue without workspace
    assert _call(S.ssvd2_batch, 10, ins, outs,
                 flags=S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_QUEUE) == 1
    # too-small workspace
    assert _call(S.ssvd2_batch, 10, ins, outs, flags=S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_QUEUE,
                 ws=FAKE + (200 << 30), ws_bytes=16) == 6


def test_workspace_size_and_launch_shape():
    assert S.svd2_workspace_bytes(1000, 0) == 0
    assert S.svd2_workspace_bytes(1000, S.SVD2_RESCUE_FP64) == 0
    assert S.svd2_workspace_bytes(1000, S.SVD2_RESCUE_FP64 | S.SVD2_RESCUE_QUEUE) >= 4000
    old = S.svd2_get_launch()
    with pytest.raises(S.Svd2Error):
        S.svd2_set_launch(100, 1)
    with pytest.raises(S.Svd2Error):
        S.svd2_set_launch(256, 3)
    S.svd2_set_launch(128, 2)
    assert S.svd2_get_launch() == (128, 2)
    S.svd2_set_launch(*old)


def test_status_strings():
    L = S.lib()
    for code in range(8):
        assert L.svd2_status_string(code)
    assert L.svd2_status_string(3) == b"output overlaps an input or another output"


def test_binding_raises_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(S, "_lib", None)
    monkeypatch.setattr(S, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        S.lib()


def test_kog_argument_errors():
    """Kogbetliantz entry points validate before any HIP call."""
    import ctypes
    L = S._kog()
    A, ws = FAKE, FAKE + (64 << 30)
    wsb = S.kog_workspace_bytes(64, "d")
    assert wsb > 0 and S.kog_workspace_bytes(63, "d") == 0
    call = lambda N, a, lda, t, w, b, f: L.dkog_step(N, a, lda, t, w, b, f, None)
    assert call(64, 0, 64, 0, ws, wsb, 0) == 1          # NULL matrix
    assert call(64, A, 64, 0, 0, wsb, 0) == 1           # NULL workspace
    assert call(63, A, 64, 0, ws, wsb, 0) == 6          # odd order
    assert call(64, A, 63, 0, ws, wsb, 0) == 6          # lda < N
    assert call(64, A, 64, 0, ws, wsb - 8, 0) == 6      # workspace too small
    assert call(64, A + 4, 64, 0, ws, wsb, 0) == 2      # misaligned matrix
    assert call(64, A, 64, 0, ws + 8, wsb, 0) == 2      # misaligned workspace
    assert call(64, A, 64, 0, A + 256, wsb, 0) == 3     # workspace overlaps A
    assert call(64, A, 64, 0, ws, wsb, 16) == 4         # unknown flag
    assert call(64, A, 64, 0, ws, wsb, 2) == 4          # GRAPH without UNFUSED
    assert call(64, A, 64, 0, ws, wsb, 3) == 4          # GRAPH is solve-only
    assert L.dkog_sweep(64, A, 64, ws, wsb, 3, None) == 4
    assert call(64, A, 64, 0, ws, wsb, 4) == 6          # TWO_STEP step: no room for the matrix buffer
    assert call(64, A, 64, 0, ws, wsb, 5) == 4          # TWO_STEP with UNFUSED
    assert L.dkog_sweep(64, A, 64, ws, wsb, 5, None) == 4   # TWO_STEP with UNFUSED
    assert L.dkog_sweep(64, A, 64, ws, wsb, 4, None) == 6   # too small for the matrix buffer
    ws2 = S.kog_workspace_bytes(64, "d", S.SVD2_KOG_TWO_STEP)
    assert ws2 >= wsb + 64 * 64 * 8
    assert S.kog_workspace_bytes(64, "z", S.SVD2_KOG_TWO_STEP) >= 64 * 64 * 16
    assert L.dkog_sweep(64, A, 64, A + 512, ws2, 4, None) == 3  # overlap
    assert call(64, A, 64, 62, ws, ws2, 4) == 6         # two steps from t = N-2 run past the sweep
    assert call(64, A, 64, -1, ws, ws2, 4) == 6
    assert call(64, A, 64, 63, ws, wsb, 0) == 6         # step out of range
    # three steps per pass: alone, a third rotation set beyond the two-step workspace
    ws3 = S.kog_workspace_bytes(64, "d", S.SVD2_KOG_THREE_STEP)
    assert ws3 > ws2
    assert S.kog_workspace_bytes(64, "c", S.SVD2_KOG_THREE_STEP) > S.kog_workspace_bytes(64, "c", 4)
    assert call(64, A, 64, 0, ws, ws3, 8 | 4) == 4      # THREE_STEP with TWO_STEP
    assert call(64, A, 64, 0, ws, ws3, 8 | 1) == 4      # THREE_STEP with UNFUSED
    assert L.dkog_sweep(64, A, 64, ws, ws3, 8 | 3, None) == 4
    assert call(64, A, 64, 0, ws, ws2, 8) == 6          # too small for the third rotation set
    assert L.dkog_sweep(64, A, 64, ws, ws3 - 8, 8, None) == 6
    assert call(64, A, 64, 61, ws, ws3, 8) == 6         # three steps from t = N-3 run past the sweep
    assert call(64, A, 64, -1, ws, ws3, 8) == 6
    assert L.dkog_sweep(64, A, 64, A + 512, ws3, 8, None) == 3  # overlap
    sw, off = ctypes.c_int(), ctypes.c_double()
    assert L.dkog_solve(64, A, 64, 1e-14, -1, ctypes.byref(sw), ctypes.byref(off), ws, wsb, 0,
                        None) == 6                      # negative max_sweeps


def test_kog_solve_noalloc_argument_errors():
    """The solve on the library's fixed workspace checks its arguments before
    any HIP call: NULL matrix, modes that would need an allocation, and
    orders whose workspace exceeds the fixed 2 MiB."""
    import ctypes
    L = S._kog()
    A = FAKE
    sw, off = ctypes.c_int(), ctypes.c_double()
    call = lambda N, a, lda, f: L.dkog_solve_noalloc(N, a, lda, 1e-14, 40, ctypes.byref(sw),
                                                     ctypes.byref(off), f, None)
    assert call(64, 0, 64, 0) == 1                      # NULL matrix
    for f in (2, 3, 4, 5, 8):                           # GRAPH, TWO_STEP, unknown
        assert call(64, A, 64, f) == 4, f
    assert call(63, A, 64, 0) == 6                      # odd order
    assert call(64, A, 63, 0) == 6                      # lda < N
    lim = max(N for N in range(30000, 30600, 2) if S.kog_workspace_bytes(N, "d") <= 2 << 20)
    assert lim == 30272                                 # the limit the header states
    assert call(lim + 2, A, lim + 2, 0) == 6            # workspace beyond the fixed array
    assert call(1 << 20, A, 1 << 20, 1) == 6


def test_kog_barrier_probe_argument_errors():
    """The barrier probe checks its arguments before any HIP call."""
    L = S._kog()
    ws, wsb = FAKE, 256 + 4096 * 64
    assert L.kog_barrier_probe(10, 256, None, 0, wsb, None) == 1       # NULL workspace
    assert L.kog_barrier_probe(-1, 256, None, ws, wsb, None) == 6      # negative count
    assert L.kog_barrier_probe(10, 0, None, ws, wsb, None) == 6        # no workgroups
    assert L.kog_barrier_probe(10, 4097, None, ws, wsb, None) == 6     # beyond the barrier's slots
    assert L.kog_barrier_probe(10, 256, None, ws, wsb - 1, None) == 6  # short workspace
    assert L.kog_barrier_probe(10, 256, None, ws + 8, wsb, None) == 2  # misaligned workspace


def test_kog_svd_argument_errors():
    """The SVD entry points validate every pointer, size, flag and overlap
    before any HIP call."""
    import ctypes
    L = S._kog()
    N = 64
    A, U, V, sig, ws = (FAKE + (i << 30) for i in range(5))
    wsb = S.kog_svd_workspace_bytes(N, "z")
    assert wsb >= S.kog_workspace_bytes(N, "z", S.SVD2_KOG_TWO_STEP) + 2 * N * N * 16
    assert S.kog_svd_workspace_bytes(N, "z", S.SVD2_KOG_TWO_STEP) == wsb  # 0 means two steps per pass
    assert S.kog_svd_workspace_bytes(N, "z", S.SVD2_KOG_UNFUSED) < wsb
    assert S.kog_svd_workspace_bytes(63, "z") == 0
    sw, off = ctypes.c_int(), ctypes.c_double()

    def call(a=A, lda=N, u=U, ldu=N, v=V, ldv=N, s=sig, ms=40, w=ws, b=wsb, f=0):
        return L.zkog_svd(N, a, lda, u, ldu, v, ldv, s, 1e-14, ms, ctypes.byref(sw), ctypes.byref(off), w, b,
                          f, None)

    assert call(u=0) == 1 and call(v=0) == 1 and call(s=0) == 1 and call(a=0) == 1
    assert call(ldu=N - 1) == 6 and call(ldv=N - 1) == 6 and call(lda=N - 1) == 6
    assert call(ms=0) == 6                               # at least one sweep
    assert call(b=wsb - 1) == 6                          # workspace too small
    assert call(u=U + 8) == 2 and call(s=sig + 4) == 2   # misaligned
    assert call(v=U + 16) == 3                           # V overlaps U
    assert call(s=A + 64) == 3                           # sigma inside A
    assert call(u=ws + wsb - 64) == 3                    # U overlaps the workspace
    assert call(f=S.SVD2_KOG_GRAPH) == 4                 # GRAPH without UNFUSED
    assert call(f=S.SVD2_KOG_TWO_STEP | S.SVD2_KOG_UNFUSED) == 4
    assert call(f=16) == 4                               # unknown flag
    assert call(f=8) == 6                                # three steps per pass: a larger workspace
    assert call(f=8, b=S.kog_svd_workspace_bytes(N, "z", 8), u=0) == 1  # accepted: on to the pointer checks
    assert call(f=8 | 4) == 4


def test_kog_batch_argument_errors():
    import ctypes
    L = S._batch()
    P = (S.kog_problem * 2)()
    for i in range(2):
        P[i].dtype, P[i].N, P[i].lda, P[i].A = 0, 64, 64, FAKE + i * (1 << 30)
        P[i].tol, P[i].max_sweeps = 1e-14, 10
    wsb = L.kog_batch_workspace_bytes(2, P)
    assert wsb > 0
    ws = FAKE + (64 << 30)
    assert L.kog_batch_solve(0, P, 0, 0, 0, None) == 0           # nothing to do
    assert L.kog_batch_solve(2, P, 0, wsb, 0, None) == 1         # NULL workspace
    assert L.kog_batch_solve(2, P, ws, wsb - 1, 0, None) == 6    # too small
    assert L.kog_batch_solve(2, P, ws + 8, wsb, 0, None) == 2    # misaligned
    assert L.kog_batch_solve(2, P, ws, wsb, 1, None) == 4        # UNFUSED is not a batch flag
    wf = L.kog_batch_workspace_bytes_flags
    w2, w3 = wf(2, P, S.SVD2_KOG_TWO_STEP), wf(2, P, S.SVD2_KOG_THREE_STEP)
    assert wsb < w2 < w3                     # a second matrix; two, then three rotation sets
    assert wf(2, P, S.SVD2_KOG_GRAPH) == wsb
    assert wf(2, P, S.SVD2_KOG_TWO_STEP | S.SVD2_KOG_THREE_STEP) == 0
    assert wf(2, P, 1) == 0
    assert L.kog_batch_solve(2, P, ws, w3, S.SVD2_KOG_TWO_STEP | S.SVD2_KOG_THREE_STEP, None) == 4
    assert L.kog_batch_solve(2, P, ws, w3 - 1, S.SVD2_KOG_THREE_STEP, None) == 6
    P[1].N = 63
    assert L.kog_batch_workspace_bytes(2, P) == 0
    assert L.kog_batch_solve(2, P, ws, wsb, 0, None) == 6        # odd order
    P[1].N, P[1].dtype = 64, 9
    assert L.kog_batch_solve(2, P, ws, wsb, 0, None) == 4        # unknown dtype
    P[1].dtype, P[1].A = 0, 0
    assert L.kog_batch_solve(2, P, ws, wsb, 0, None) == 1        # NULL matrix
    P[1].A = ws + 4096
    assert L.kog_batch_solve(2, P, ws, wsb, 0, None) == 3        # matrix inside the workspace
    assert S.lib().kog_set_tile_rules(1, (ctypes.c_int * 1)(100), (ctypes.c_int * 1)(100),
                                      (ctypes.c_int * 1)(8)) == 6  # kc must be 64/128/256


def test_kog_two_step_tile_rules():
    """Shape table of the two-step kernel: wavefronts per workgroup in {1, 2,
    4}; lc in [2, 64] (fixed) or [-3, 0] (fill whole rounds)."""
    import ctypes
    L = S.lib()
    one = lambda x: (ctypes.c_int * 1)(x)
    assert L.kog_set_two_step_tiles(1, one(1 << 20), one(3), one(8)) == 6
    assert L.kog_set_two_step_tiles(1, one(1 << 20), one(4), one(1)) == 6
    assert L.kog_set_two_step_tiles(1, one(1 << 20), one(4), one(65)) == 6
    assert L.kog_set_two_step_tiles(1, one(1 << 20), one(4), one(-4)) == 6
    assert L.kog_set_two_step_tiles(1, one(1 << 20), one(4), one(0)) == 0
    assert L.kog_set_two_step_tiles(2, (ctypes.c_int * 2)(64, 32), (ctypes.c_int * 2)(4, 4),
                                    (ctypes.c_int * 2)(8, 8)) == 6   # max_order must increase
    assert L.kog_set_two_step_tiles(1, None, None, None) == 1
    assert L.kog_set_two_step_tiles(0, None, None, None) == 0      # back to the default


def test_kog_three_step_tile_rules():
    """Shape table of the three-step kernel: wavefronts per workgroup in {1,
    2, 4}; lc in [2, 128] (fixed) or [-3, 0] (fill whole rounds); the SVD
    workspace query takes the three-step flag alone."""
    import ctypes
    L = S.lib()
    one = lambda x: (ctypes.c_int * 1)(x)
    assert L.kog_set_three_step_tiles(1, one(1 << 20), one(3), one(8)) == 6
    assert L.kog_set_three_step_tiles(1, one(1 << 20), one(4), one(1)) == 6
    assert L.kog_set_three_step_tiles(1, one(1 << 20), one(4), one(129)) == 6
    assert L.kog_set_three_step_tiles(1, one(1 << 20), one(1), one(2)) == 0
    assert L.kog_set_three_step_tiles(1, one(1 << 20), one(1), one(-4)) == 6
    assert L.kog_set_three_step_tiles(1, one(1 << 20), one(2), one(-1)) == 0
    assert L.kog_set_three_step_tiles(2, (ctypes.c_int * 2)(64, 32), (ctypes.c_int * 2)(4, 4),
                                      (ctypes.c_int * 2)(8, 8)) == 6   # max_order must increase
    assert L.kog_set_three_step_tiles(1, None, None, None) == 1
    assert L.kog_set_three_step_tiles(0, None, None, None) == 0      # back to the default
    assert S.kog_svd_workspace_bytes(64, "d", S.SVD2_KOG_THREE_STEP) > S.kog_svd_workspace_bytes(64, "d", 4)
    assert S.kog_svd_workspace_bytes(64, "d", S.SVD2_KOG_THREE_STEP | S.SVD2_KOG_TWO_STEP) == 0


def test_kog_sigma_argument_errors():
    """Sorted-diagonal extraction validates before any HIP call."""
    L = S._kog()
    A, out, ws = FAKE, FAKE + (64 << 30), FAKE + (128 << 30)
    wsb = L.kog_sigma_workspace_bytes(100, 0)
    assert wsb == 1024 and L.kog_sigma_workspace_bytes(100, 2) == 512   # 128 keys, 256-byte rounded
    assert L.kog_sigma_workspace_bytes(0, 0) == 0 and L.kog_sigma_workspace_bytes(4, 9) == 0
    call = lambda N, a, lda, o, w, b: L.dkog_sigma(N, a, lda, o, w, b, None)
    assert call(100, 0, 100, out, ws, wsb) == 1           # NULL matrix
    assert call(100, A, 100, 0, ws, wsb) == 1             # NULL output
    assert call(100, A, 99, out, ws, wsb) == 6            # lda < N
    assert call(0, A, 100, out, ws, wsb) == 6             # empty
    assert call(100, A, 100, out, ws, wsb - 8) == 6       # workspace too small
    assert call(100, A + 4, 100, out, ws, wsb) == 2       # misaligned matrix
    assert call(100, A, 100, out, ws + 8, wsb) == 2       # misaligned workspace
    assert call(100, A, 100, A + 800, ws, wsb) == 3       # output inside the matrix
    assert call(100, A, 100, out, out + 256, wsb) == 3    # workspace overlaps the output


def test_binding_refuses_host_tensors():
    """The binding only hands device addresses to the library: host matrices,
    trains and workspaces are refused before any library call."""
    import torch
    A = torch.zeros((8, 8), dtype=torch.float64).t()
    for call in (lambda: S.kog_solve(A), lambda: S.kog_svd(A), lambda: S.kog_sigma(A),
                 lambda: S.kog_batch_solve([A], 1e-14)):
        with pytest.raises(ValueError, match="device tensor"):
            call()
    with pytest.raises(ValueError, match="device tensors"):
        S.svd2([torch.zeros(16, dtype=torch.float64) for _ in range(4)])
    with pytest.raises(ValueError, match="device tensors"):
        S._nbytes(torch.zeros(16, dtype=torch.uint8))


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is present: the launch would run on it")
def test_launch_without_a_device_reports_the_hip_error():
    """With no GPU, a well-formed call passes every argument check, its launch
    fails, and the entry point returns SVD2_ERR_HIP with the HIP error
    (hipErrorNoDevice) kept for svd2_last_hip_error; nothing is dereferenced
    on the host (the addresses are fake device addresses)."""
    L = S.lib()
    for fn, nin, nout in ((S.dsvd2_batch, 4, 11), (S.zsvd2_batch, 8, 19), (S.csvd2_batch, 8, 19)):
        ins, outs = _ptrs(nin), _ptrs(nout, base=FAKE + (64 << 30))
        with pytest.raises(S.Svd2Error) as ei:
            fn(10, ins, outs, 0, stream=0)
        assert ei.value.status == 5
        assert L.svd2_last_hip_error() == 100  # hipErrorNoDevice
        assert "hipError 100" in str(ei.value)
