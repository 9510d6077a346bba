"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, and rejects bad arguments before any device work (no GPU needed)."""
import ctypes
import os

import pytest

from paper_2210_09196_amd import pusch

# Non-null but never dereferenced: every call below fails validation first.
FAKE = ctypes.c_void_p(0x10000)
FAKE2 = ctypes.c_void_p(0x90000000)
EINVAL, EUNSUP, ENOMEM = -1, -2, -4


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pusch.LIB_PATH):
        from paper_2210_09196_amd.build import build
        build()
    return pusch.lib()


def test_exports_every_declared_symbol(lib):
    names = pusch.header_symbols()
    assert len(names) == 29
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(pusch._SIG)


def test_strerror(lib):
    assert pusch.strerror(0) == "success"
    assert "invalid" in pusch.strerror(EINVAL)
    assert pusch.strerror(12345) == "unknown error code"


def test_fft_validation(lib):
    f = lib.pusch_fft
    assert f(None, FAKE2, 4096, 0, 1, None) == EINVAL
    assert f(FAKE, FAKE2, 100, 0, 1, None) == EUNSUP
    assert f(FAKE, FAKE2, 4096, 4097, 1, None) == EINVAL
    assert f(FAKE, FAKE2, 4096, -1, 1, None) == EINVAL
    assert f(FAKE, FAKE2, 4096, 0, -1, None) == EINVAL
    assert f(FAKE, FAKE, 4096, 3300, 1, None) == EINVAL  # in place needs the full output
    assert f(FAKE, ctypes.c_void_p(0x10000 + 8), 64, 0, 2, None) == EINVAL  # partial overlap
    assert f(FAKE, FAKE2, 4096, 0, 0, None) == 0  # empty batch: no-op, no device touched


def test_beamform_validation(lib):
    f = lib.pusch_beamform
    assert f(None, None, FAKE2, 32, 64, 3300, 3300, 1, None) == EINVAL
    assert f(None, FAKE, FAKE2, 65, 64, 3300, 3300, 1, None) == EINVAL  # too many beams
    assert f(None, FAKE, FAKE2, 0, 64, 3300, 3300, 1, None) == EINVAL
    assert f(None, FAKE, FAKE2, 32, 16, 100, 100, 1, None) == EINVAL  # built-in DFT needs beams <= antennas
    assert f(None, FAKE, FAKE2, 32, 64, 3300, 3000, 1, None) == EINVAL  # ld_x < n_re
    assert f(FAKE2, FAKE, FAKE2, 32, 64, 3300, 3300, 1, None) == EINVAL  # W overlaps Y
    assert f(None, FAKE, FAKE2, 32, 64, 0, 1, 5, None) == 0


def test_chest_validation(lib):
    f = lib.pusch_chest
    assert f(FAKE, None, FAKE2, 32, 16, 3300, 2, 1, None) == EINVAL
    assert f(FAKE, FAKE, FAKE2, 32, 16, 3300, 5, 1, None) == EINVAL  # too many pilot symbols
    assert f(FAKE, FAKE, FAKE2, 8, 16, 3300, 2, 1, None) == EINVAL  # more UEs than beams
    assert f(FAKE, FAKE, FAKE2, 32, 16, 15, 2, 1, None) == EINVAL  # a UE without pilots
    assert f(FAKE, FAKE, FAKE2, 64, 33, 3300, 2, 1, None) == EINVAL
    assert f(FAKE, FAKE, FAKE2, 32, 16, 3300, 2, 0, None) == 0


def test_mmse_validation(lib):
    f = lib.pusch_mmse_solve
    assert f(FAKE, FAKE, -1.0, FAKE2, 32, 16, 3300, 12, 1, None, None) == EINVAL
    assert f(FAKE, FAKE, float("nan"), FAKE2, 32, 16, 3300, 12, 1, None, None) == EINVAL
    assert f(FAKE, FAKE, float("inf"), FAKE2, 32, 16, 3300, 12, 1, None, None) == EINVAL
    assert f(FAKE, FAKE, 0.1, FAKE2, 32, 16, 3300, 0, 1, None, None) == EINVAL
    assert f(FAKE, FAKE, 0.1, FAKE2, 8, 16, 3300, 12, 1, None, None) == EINVAL
    assert f(FAKE, FAKE, 0.1, FAKE, 32, 16, 3300, 12, 1, None, None) == EINVAL  # output overlaps input
    assert f(FAKE, FAKE, 0.1, FAKE2, 32, 16, 3300, 12, 0, None, None) == 0


def _desc(**kw):
    d = pusch.SlotDesc()
    vals = dict(n_ant=64, n_fft=4096, n_sc=3300, n_symb=14, n_beams=32, n_ue=16, n_pilot=2, sigma2=0.01)
    vals.update(kw)
    for k, v in vals.items():
        setattr(d, k, v)
    ps = kw.get("pilot_symb", (2, 11))
    for j, s in enumerate(ps):
        d.pilot_symb[j] = s
    d.pilots = kw.get("pilots", 0x20000)
    return d


def test_slot_workspace_bytes(lib):
    d = _desc()
    n = 16
    # active-bin rows padded to a multiple of 16 subcarriers (3300 -> 3312)
    xa = n * 14 * 64 * 3312 * 8
    y = n * 14 * 3300 * 32 * 8
    h = n * 3300 * 16 * 32 * 8
    a = lambda v: (v + 255) // 256 * 256
    # noise estimation scratch: 256 partial sums (8 B) and one estimate per slot
    ne = a(n * 256 * 8 + n * 4)
    # 16 UEs: the channel is estimated inside the detection kernel, no stored
    # estimate (its interpolation taps are a per-geometry table of the library)
    assert lib.pusch_slot_workspace_bytes(ctypes.byref(d), n) == a(xa) + a(y) + ne
    # refinement reads a stored estimate: the fused geometry gains the H region
    dr = _desc(refine=1)
    assert lib.pusch_slot_workspace_bytes(ctypes.byref(dr), n) == a(xa) + a(y) + a(h) + ne
    d32 = _desc(n_ue=32, n_beams=64)
    xa, y, h = n * 14 * 64 * 3312 * 8, n * 14 * 3300 * 64 * 8, n * 3300 * 32 * 64 * 8
    assert lib.pusch_slot_workspace_bytes(ctypes.byref(d32), n) == a(xa) + a(y) + a(h) + ne
    # odd number of beams: separate estimation kernel, stored estimate
    d31 = _desc(n_beams=31)
    xa, y, h = n * 14 * 64 * 3312 * 8, n * 14 * 3300 * 31 * 8, n * 3300 * 16 * 31 * 8
    assert lib.pusch_slot_workspace_bytes(ctypes.byref(d31), n) == a(xa) + a(y) + a(h) + ne
    # one UE: fused detection as well
    d1 = _desc(n_ue=1)
    y = n * 14 * 3300 * 32 * 8
    assert lib.pusch_slot_workspace_bytes(ctypes.byref(d1), n) == a(n * 14 * 64 * 3312 * 8) + a(y) + ne
    assert lib.pusch_slot_workspace_bytes(ctypes.byref(_desc(n_fft=1000)), n) == 0
    assert lib.pusch_slot_workspace_bytes(ctypes.byref(_desc(pilot_symb=(11, 2))), n) == 0


@pytest.mark.parametrize("kw,code", [
    (dict(n_fft=3000), EUNSUP),
    (dict(n_sc=4097), EINVAL),
    (dict(n_sc=8), EINVAL),  # fewer subcarriers than UEs
    (dict(n_symb=17), EINVAL),
    (dict(n_pilot=0), EINVAL),
    (dict(pilot_symb=(2, 2)), EINVAL),
    (dict(pilot_symb=(2, 14)), EINVAL),
    (dict(sigma2=-0.5), EINVAL),
    (dict(n_ue=33, n_beams=64), EINVAL),
    (dict(n_beams=70), EINVAL),
    (dict(pilots=0), EINVAL),
])
def test_slot_validation(lib, kw, code):
    d = _desc(**kw)
    ws = ctypes.c_void_p(0x4000000000)
    assert lib.pusch_slot(ctypes.byref(d), 1, FAKE, FAKE2, None, ws, 1 << 40, None) == code


def test_slot_workspace_errors(lib):
    d = _desc()
    need = lib.pusch_slot_workspace_bytes(ctypes.byref(d), 2)
    ws = ctypes.c_void_p(0x4000000000)
    assert lib.pusch_slot(ctypes.byref(d), 2, FAKE, FAKE2, None, ws, need - 1, None) == ENOMEM
    assert lib.pusch_slot(ctypes.byref(d), 2, FAKE, FAKE2, None, ctypes.c_void_p(0x4000000010), need, None) == EINVAL
    assert lib.pusch_slot(ctypes.byref(d), 0, FAKE, FAKE2, None, ws, need, None) == 0


def test_noise_est_validation(lib):
    # 256 partial sums (8 B) per item; the neighbour table is the library's, per geometry
    assert lib.pusch_noise_est_workspace_bytes(16) == 16 * 256 * 8
    assert lib.pusch_noise_est_workspace_bytes(-1) == 0
    need = lib.pusch_noise_est_workspace_bytes(2)
    f = lib.pusch_noise_est
    ws = ctypes.c_void_p(0x4000000000)
    S = ctypes.c_void_p(0x70000000)
    big = 1 << 30
    assert f(None, FAKE2, S, 32, 16, 3300, 2, 1, ws, big, None) == EINVAL
    assert f(FAKE, FAKE2, None, 32, 16, 3300, 2, 1, ws, big, None) == EINVAL
    assert f(FAKE, FAKE2, S, 32, 16, 31, 2, 1, ws, big, None) == EINVAL  # a UE with one pilot position
    assert f(FAKE, FAKE2, S, 32, 16, 3300, 5, 1, ws, big, None) == EINVAL  # too many pilot symbols
    assert f(FAKE, FAKE2, S, 8, 16, 3300, 2, 1, ws, big, None) == EINVAL  # more UEs than beams
    assert f(FAKE, FAKE2, S, 32, 16, 3300, 2, 2, ws, need - 1, None) == ENOMEM
    assert f(FAKE, FAKE2, S, 32, 16, 3300, 2, 1, None, big, None) == EINVAL
    assert f(FAKE, FAKE2, S, 32, 16, 3300, 2, 1, ctypes.c_void_p(0x4000000004), big, None) == EINVAL
    assert f(FAKE, FAKE2, S, 32, 16, 5000, 2, 1, ws, big, None) == EINVAL  # beyond 4096 subcarriers
    assert f(FAKE, FAKE2, ctypes.c_void_p(0x20000), 32, 16, 3300, 2, 1, ws, big, None) == EINVAL  # inside Yp
    assert f(FAKE, FAKE2, S, 32, 16, 3300, 2, 1, ctypes.c_void_p(0x90000100), big, None) == EINVAL  # ws on pilots
    assert f(FAKE, FAKE2, S, 32, 16, 3300, 2, 0, None, 0, None) == 0  # empty batch


def test_noise_est_static_validation(lib):
    # the allocation-free variant: same checks, no workspace, at most 1024 items per call
    f = lib.pusch_noise_est_static
    f.restype, f.argtypes = ctypes.c_int, [ctypes.c_void_p] * 3 + [ctypes.c_int] * 4 + [ctypes.c_longlong,
                                                                                      ctypes.c_void_p]
    S = ctypes.c_void_p(0x70000000)
    assert f(None, FAKE2, S, 32, 16, 3300, 2, 1, None) == EINVAL
    assert f(FAKE, FAKE2, None, 32, 16, 3300, 2, 1, None) == EINVAL
    assert f(FAKE, FAKE2, S, 32, 16, 31, 2, 1, None) == EINVAL  # a UE with one pilot position
    assert f(FAKE, FAKE2, S, 32, 16, 3300, 5, 1, None) == EINVAL  # too many pilot symbols
    assert f(FAKE, FAKE2, S, 8, 16, 3300, 2, 1, None) == EINVAL  # more UEs than beams
    assert f(FAKE, FAKE2, S, 32, 16, 5000, 2, 1, None) == EINVAL  # beyond 4096 subcarriers
    assert f(FAKE, FAKE2, S, 32, 16, 3300, 2, 1025, None) == EUNSUP  # beyond the scratch's items
    assert f(FAKE, FAKE2, ctypes.c_void_p(0x20000), 32, 16, 3300, 2, 1, None) == EINVAL  # inside Yp
    assert f(FAKE, FAKE2, S, 32, 16, 3300, 2, 0, None) == 0  # empty batch


def test_slot_noise_est_validation(lib):
    ws = ctypes.c_void_p(0x4000000000)
    # estimation needs two pilot positions per UE (n_sc >= 2 n_ue)
    d = _desc(n_fft=64, n_sc=31, noise_est=1)
    assert lib.pusch_slot(ctypes.byref(d), 1, FAKE, FAKE2, None, ws, 1 << 40, None) == EINVAL
    # the given sigma2 is not used, so not checked, when it is estimated
    d = _desc(sigma2=-1.0, noise_est=1)
    need = lib.pusch_slot_workspace_bytes(ctypes.byref(d), 2)
    assert need == lib.pusch_slot_workspace_bytes(ctypes.byref(_desc()), 2)
    assert lib.pusch_slot(ctypes.byref(d), 0, FAKE, FAKE2, None, ws, need, None) == 0
    # the estimates may not overlap the output, the input or the workspace
    for where in (0x90000040, 0x10040, 0x4000000100):
        d = _desc(noise_est=1, sigma2_est=where)
        assert lib.pusch_slot(ctypes.byref(d), 2, FAKE, FAKE2, None, ws, need, None) == EINVAL, hex(where)
    # ignored without noise_est
    d = _desc(sigma2_est=0x90000040)
    assert lib.pusch_slot(ctypes.byref(d), 0, FAKE, FAKE2, None, ws, need, None) == 0


def test_slot_time_varying_needs_the_fused_detection(lib):
    ws = ctypes.c_void_p(0x4000000000)
    ok = _desc(time_varying=1)
    need = lib.pusch_slot_workspace_bytes(ctypes.byref(ok), 2)
    assert need == lib.pusch_slot_workspace_bytes(ctypes.byref(_desc()), 2)
    assert lib.pusch_slot(ctypes.byref(ok), 0, FAKE, FAKE2, None, ws, need, None) == 0
    for kw in (dict(n_beams=31), dict(n_ue=32, n_beams=64), dict(refine=1)):
        d = _desc(time_varying=1, **kw)
        assert lib.pusch_slot(ctypes.byref(d), 0, FAKE, FAKE2, None, ws, 1 << 40, None) == EUNSUP, kw


def test_profile_arguments(lib):
    assert lib.pusch_profile_begin(0) == EINVAL
    assert lib.pusch_profile_end(None, 0) == EINVAL  # not active


def _cell_arrays(descs, n_slot):
    n = len(descs)
    return (pusch.SlotDesc * n)(*descs), (ctypes.c_longlong * n)(*n_slot)


def test_cells_workspace_bytes(lib):
    a = lambda v: (v + 255) // 256 * 256
    big = _desc()
    small = _desc(n_ant=16, n_fft=1024, n_sc=825, n_beams=8, n_ue=4, pilot_symb=(2,), n_pilot=1)
    ws = lambda d, n: lib.pusch_slot_workspace_bytes(ctypes.byref(d), n)
    descs, ns = _cell_arrays([big, small, small], [2, 1, 3])
    # one slice per cell, each that cell's pusch_slot workspace rounded up to 256 bytes
    assert lib.pusch_cells_workspace_bytes(descs, 3, ns, 0) == a(ws(big, 2)) + a(ws(small, 1)) + a(ws(small, 3))
    descs6, ns6 = _cell_arrays([small] * 6, [1] * 6)
    assert lib.pusch_cells_workspace_bytes(descs6, 6, ns6, 0) == 6 * a(ws(small, 1))
    # the streams-only flag does not change the layout
    assert lib.pusch_cells_workspace_bytes(descs6, 6, ns6, 2) == 6 * a(ws(small, 1))
    bad, nsb = _cell_arrays([big, _desc(n_fft=1000)], [1, 1])
    assert lib.pusch_cells_workspace_bytes(bad, 2, nsb, 0) == 0
    assert lib.pusch_cells_workspace_bytes(descs, 0, ns, 0) == 0
    assert lib.pusch_cells_workspace_bytes(None, 1, ns, 0) == 0
    # mixed precision: the FP16 grids need n_ant <= 64 in every cell
    many, nsm = _cell_arrays([small, _desc(n_ant=65)], [1, 1])
    assert lib.pusch_cells_workspace_bytes(many, 2, nsm, 1) == 0
    mws = lambda d, n: lib.pusch_slot_mixed_workspace_bytes(ctypes.byref(d), n)
    assert lib.pusch_cells_workspace_bytes(descs, 3, ns, 1) == a(mws(big, 2)) + a(mws(small, 1)) + a(mws(small, 3))


def test_cells_validation(lib):
    small = _desc(n_ant=16, n_fft=1024, n_sc=825, n_beams=8, n_ue=4, pilot_symb=(2,), n_pilot=1)
    descs, ns = _cell_arrays([small, small], [1, 1])
    need = lib.pusch_cells_workspace_bytes(descs, 2, ns, 0)
    ws = ctypes.c_void_p(0x4000000000)
    P = ctypes.c_void_p
    x = (P * 2)(0x10000, 0x800000)
    o = (P * 2)(0x90000000, 0x98000000)
    f = lib.pusch_cells
    assert f(descs, 0, ns, x, o, None, ws, need, 0, None) == EINVAL
    assert f(None, 2, ns, x, o, None, ws, need, 0, None) == EINVAL
    assert f(descs, 2, ns, x, o, None, ws, need - 1, 0, None) == ENOMEM
    assert f(descs, 2, ns, x, o, None, ctypes.c_void_p(0x4000000010), need, 0, None) == EINVAL  # unaligned
    assert f(descs, 2, ns, x, o, None, None, need, 0, None) == EINVAL
    assert f(descs, 2, ns, x, o, None, ws, need, 1 << 6, None) == EINVAL  # unknown flag
    # the tuner: repetitions and the times array checked before anything runs
    plan = pusch.CellsPlan()
    us = (ctypes.c_float * 8)()
    tune = lib.pusch_cells_tune
    assert tune(descs, 2, ns, x, o, None, ws, need, 0, 0, ctypes.byref(plan), us, 8, None) == EINVAL
    assert tune(descs, 2, ns, x, o, None, ws, need, 0, 1001, ctypes.byref(plan), us, 8, None) == EINVAL
    assert tune(descs, 2, ns, x, o, None, ws, need, 0, 3, ctypes.byref(plan), None, 8, None) == EINVAL
    assert tune(None, 2, ns, x, o, None, ws, need, 0, 3, ctypes.byref(plan), us, 8, None) == EINVAL
    assert lib.pusch_cells_plan_get(descs, 2, ns, 0, None) == EINVAL
    assert lib.pusch_cells_plan_get(descs, 0, ns, 0, ctypes.byref(plan)) == EINVAL
    # one invalid cell rejects the whole call
    bad, nsb = _cell_arrays([small, _desc(sigma2=-1.0)], [1, 1])
    assert f(bad, 2, nsb, x, o, None, ws, 1 << 40, 0, None) == EINVAL
    # a cell's noise estimates over another cell's output
    est = _desc(n_ant=16, n_fft=1024, n_sc=825, n_beams=8, n_ue=4, pilot_symb=(2,), n_pilot=1, noise_est=1,
                sigma2_est=0x98000000 + 64)
    clash, nsc = _cell_arrays([est, small], [1, 1])
    assert f(clash, 2, nsc, x, o, None, ws, need, 0, None) == EINVAL
    # two cells writing the same output
    same = (P * 2)(0x90000000, 0x90000000)
    assert f(descs, 2, ns, x, same, None, ws, need, 0, None) == EINVAL
    # a cell's output inside another cell's workspace slice
    inside = (P * 2)(0x90000000, 0x4000000000 + need - 4096)
    assert f(descs, 2, ns, x, inside, None, ws, need, 0, None) == EINVAL
    # a cell's output over another cell's input
    over = (P * 2)(0x800000, 0x98000000)
    assert f(descs, 2, ns, x, over, None, ws, need, 0, None) == EINVAL


def test_slot_mixed_workspace_and_validation(lib):
    a = lambda v: (v + 255) // 256 * 256
    d = _desc()
    n = 16
    # FP16 active-bin grids (4 B per value, rows padded to 32: 3300 -> 3328),
    # 64 exponent bytes per slot symbol, then as pusch_slot
    xa, ex = n * 14 * 64 * 3328 * 4, n * 14 * 64
    y = n * 14 * 3300 * 32 * 8
    ne = a(n * 256 * 8 + n * 4)
    assert lib.pusch_slot_mixed_workspace_bytes(ctypes.byref(d), n) == a(xa) + a(ex) + a(y) + ne
    many = _desc(n_ant=65, n_beams=32)
    assert lib.pusch_slot_mixed_workspace_bytes(ctypes.byref(many), n) == 0  # FP16 path: up to 64 antennas
    ws = ctypes.c_void_p(0x4000000000)
    f = lib.pusch_slot_mixed
    assert f(ctypes.byref(many), 1, FAKE, FAKE2, None, ws, 1 << 40, None) == EUNSUP
    assert f(ctypes.byref(_desc(sigma2=-1.0)), 1, FAKE, FAKE2, None, ws, 1 << 40, None) == EINVAL
    need = lib.pusch_slot_mixed_workspace_bytes(ctypes.byref(d), 2)
    assert f(ctypes.byref(d), 2, FAKE, FAKE2, None, ws, need - 1, None) == ENOMEM
    assert f(ctypes.byref(d), 0, FAKE, FAKE2, None, ws, need, None) == 0


def test_fft_mfma_is_for_the_reduced_precision_4096_point_slots(lib):
    ws = ctypes.c_void_p(0x4000000000)
    d = _desc()
    d.fft_mfma = 1
    # the FP32 chain has no matrix-core FFT
    assert lib.pusch_slot(ctypes.byref(d), 1, FAKE, FAKE2, None, ws, 1 << 40, None) == EUNSUP
    small = _desc(n_fft=2048, n_sc=1650)
    small.fft_mfma = 1
    for f in (lib.pusch_slot_mixed, lib.pusch_slot_bf16):
        assert f(ctypes.byref(small), 1, FAKE, FAKE2, None, ws, 1 << 40, None) == EUNSUP
        need = lib.pusch_slot_mixed_workspace_bytes(ctypes.byref(d), 2)
        assert f(ctypes.byref(d), 2, FAKE, FAKE2, None, ws, need - 1, None) == ENOMEM  # accepted up to the size check
        assert f(ctypes.byref(d), 0, FAKE, FAKE2, None, ws, need, None) == 0


def test_slot_bf16_workspace_and_validation(lib):
    # the bfloat16 form uses the mixed layout (its exponent table unused)
    d = _desc()
    for n in (1, 16):
        assert lib.pusch_slot_bf16_workspace_bytes(ctypes.byref(d), n) == \
            lib.pusch_slot_mixed_workspace_bytes(ctypes.byref(d), n)
    many = _desc(n_ant=65, n_beams=32)
    assert lib.pusch_slot_bf16_workspace_bytes(ctypes.byref(many), 4) == 0
    ws = ctypes.c_void_p(0x4000000000)
    f = lib.pusch_slot_bf16
    assert f(ctypes.byref(many), 1, FAKE, FAKE2, None, ws, 1 << 40, None) == EUNSUP
    assert f(ctypes.byref(_desc(sigma2=-1.0)), 1, FAKE, FAKE2, None, ws, 1 << 40, None) == EINVAL
    assert f(ctypes.byref(d), 1, None, FAKE2, None, ws, 1 << 40, None) == EINVAL
    need = lib.pusch_slot_bf16_workspace_bytes(ctypes.byref(d), 2)
    assert f(ctypes.byref(d), 2, FAKE, FAKE2, None, ws, need - 1, None) == ENOMEM
    assert f(ctypes.byref(d), 0, FAKE, FAKE2, None, ws, need, None) == 0


def test_denoiser_workspace_and_validation(lib):
    a = lambda v: (v + 255) // 256 * 256
    n, S, K = 64, 14, 256
    P = n * S * K
    # three bfloat16 activations of 32 channels, two FP32 gradient buffers, 1024 x 9248 partial sums, loss parts
    assert lib.pusch_dn_workspace_bytes(S, K, n) == 3 * a(P * 64) + 2 * a(P * 128) + a(1024 * 9248 * 4) + a(1024)
    assert lib.pusch_dn_workspace_bytes(0, K, n) == 0 and lib.pusch_dn_workspace_bytes(17, K, n) == 0
    assert lib.pusch_dn_workspace_bytes(S, 4097, n) == 0 and lib.pusch_dn_workspace_bytes(S, K, -1) == 0
    ws = ctypes.c_void_p(0x4000000000)
    big = 1 << 40
    Pm = ctypes.c_void_p(0x300000)
    fw = lib.pusch_dn_forward
    assert fw(None, FAKE, FAKE2, 1.0, S, K, n, ws, big, None) == EINVAL
    assert fw(Pm, FAKE, FAKE2, 1.0, S, K, n, ctypes.c_void_p(0x4000000010), big, None) == EINVAL
    assert fw(Pm, FAKE, FAKE2, 1.0, S, K, n, ws, 1024, None) == ENOMEM
    assert fw(Pm, FAKE, ctypes.c_void_p(0x10008), 1.0, S, K, n, ws, big, None) == EINVAL  # out on grid
    assert fw(Pm, FAKE, FAKE2, 0.0, S, K, n, ws, big, None) == EINVAL  # the noise unit must be positive
    assert fw(Pm, FAKE, FAKE2, float("nan"), S, K, n, ws, big, None) == EINVAL
    assert fw(Pm, FAKE, FAKE2, 1.0, S, K, 0, ws, big, None) == 0  # no grids
    assert lib.pusch_dn_backward(Pm, FAKE, FAKE2, ctypes.c_void_p(0x500000), S, K, 0, ws, big, None) == EINVAL
    assert lib.pusch_dn_backward(Pm, FAKE, FAKE2, Pm, S, K, n, ws, big, None) == EINVAL  # grads on params
    assert lib.pusch_dn_loss(FAKE, FAKE2, None, ctypes.c_void_p(0x90000008), ctypes.c_void_p(0x700000), S, K, n, ws,
                             big, None) == EINVAL  # dout on the target
    assert lib.pusch_dn_loss(FAKE, FAKE2, ctypes.c_void_p(0x800008), ctypes.c_void_p(0x800000), ctypes.c_void_p(0x700000),
                             S, K, n, ws, big, None) == EINVAL  # weights on dout
    g = ctypes.c_void_p(0x500000)
    m = ctypes.c_void_p(0x600000)
    v = ctypes.c_void_p(0x700000)
    f = lib.pusch_dn_adam
    assert f(Pm, g, m, v, 0, 1e-3, 0.9, 0.999, 1e-8, None) == EINVAL  # steps count from 1
    assert f(Pm, g, m, v, 1, 0.0, 0.9, 0.999, 1e-8, None) == EINVAL
    assert f(Pm, g, m, v, 1, 1e-3, 1.0, 0.999, 1e-8, None) == EINVAL
    assert f(Pm, g, m, m, 1, 1e-3, 0.9, 0.999, 1e-8, None) == EINVAL  # m and v overlap
    ps = (ctypes.c_int * 1)(2)
    lg = lib.pusch_dn_ls_grid
    assert lg(FAKE, FAKE2, ws, 16, 4, 3, 14, 1, ps, 2, None) == EINVAL  # a UE without a pilot position
    assert lg(FAKE, FAKE2, ws, 16, 4, 256, 2, 1, ps, 2, None) == EINVAL  # pilot symbol outside the slot
    assert lg(FAKE, FAKE2, ws, 16, 4, 256, 14, 1, None, 2, None) == EINVAL
    assert lg(FAKE, FAKE2, ws, 16, 4, 256, 14, 1, ps, 0, None) == 0  # empty batch


def test_slot_denoised_workspace_and_validation(lib):
    d = _desc(n_ant=16, n_fft=256, n_sc=256, n_beams=16, n_ue=4, n_pilot=1, pilot_symb=(2,))
    need = lib.pusch_slot_denoised_workspace_bytes(ctypes.byref(d), 2)
    assert need > 0
    assert lib.pusch_slot_denoised_workspace_bytes(ctypes.byref(_desc(refine=1)), 2) == 0
    assert lib.pusch_slot_denoised_workspace_bytes(ctypes.byref(_desc(time_varying=1)), 2) == 0
    assert lib.pusch_slot_denoised_workspace_bytes(ctypes.byref(_desc(noise_est=1)), 2) == 0
    assert lib.pusch_slot_denoised_workspace_bytes(ctypes.byref(_desc(sigma2=0.0)), 2) == 0  # the network's unit
    ws = ctypes.c_void_p(0x4000000000)
    Pm = ctypes.c_void_p(0x300000)
    f = lib.pusch_slot_denoised
    assert f(ctypes.byref(d), 2, FAKE, None, FAKE2, None, None, ws, need, None) == EINVAL  # no parameters
    assert f(ctypes.byref(d), 2, FAKE, Pm, FAKE2, None, None, ws, need - 1, None) == ENOMEM
    assert f(ctypes.byref(d), 2, FAKE, Pm, FAKE2, None, None, ctypes.c_void_p(0x4000000010), need, None) == EINVAL
    assert f(ctypes.byref(d), 2, FAKE, Pm, FAKE2, None, ctypes.c_void_p(0x90000004), ws, need, None) == EINVAL
    assert f(ctypes.byref(d), 0, FAKE, Pm, FAKE2, None, None, ws, need, None) == 0
