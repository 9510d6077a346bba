"""GPU checks of the FFT with its radix-16 passes on the matrix cores (slot
option fft_mfma, 4096 points, reduced-precision slots) against the FP64
oracle: the demodulated grid itself (read from the slot workspace, where the
beamforming stage takes it from) and the detected symbols.

Tolerance: every pass rounds its inputs to the operand format (FP16: u =
2^-11, bfloat16: u = 2^-9 per component) and the DFT matrix entries are
rounded once; the 16-point DFT preserves the RMS relative error, so three
passes plus the rounding of the stored grid give an RMS error of about
sqrt(4) u / sqrt(3) ~ 1.2 u, against 0.6 u for the vector-unit FFT that
rounds only its output.  The grid must stay within NRMSE 2 u-bounds of 2e-3
(FP16) and 8e-3 (bfloat16), the bounds the reduced-precision forms already
use for the detected symbols; the detected symbols within twice those (the
grid error passes through beamforming and detection as in those forms) and
the EVM within 0.1 dB of the FP32 chain.
"""
import numpy as np
import pytest
import torch

from oracle import metrics as M
from checks import assert_xhat
from oracle import pusch_oracle as O
from paper_2210_09196_amd import pusch, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"
TOL_GRID = {"mixed": 2e-3, "bf16": 8e-3}
TOL_X = {"mixed": 4e-3, "bf16": 1.6e-2}
EVM_GAP_DB = 0.1


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def slot_for(cfg, n, precision, sigma2, fft_mfma=True):
    return pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb, sigma2, n,
                      precision=precision, fft_mfma=fft_mfma)


def grid_from_workspace(slot, cfg, n, precision):
    """The FFT output the slot left in its workspace: [n][S][R][n_sc] complex, scale undone."""
    S, R, K = cfg.n_symb, cfg.n_ant, cfg.n_sc
    kp = (K + 31) // 32 * 32
    nbytes = n * S * R * kp * 4
    torch.cuda.synchronize()
    raw = slot.ws[:nbytes].view(torch.float16 if precision == "mixed" else torch.bfloat16)
    g = raw.float().cpu().numpy().reshape(n * S, R, kp, 2)[:, :, :K]
    X = (g[..., 0] + 1j * g[..., 1]).astype(np.complex128)
    if precision == "mixed":
        off = (nbytes + 255) // 256 * 256
        ex = slot.ws[off:off + n * S * 64].view(torch.int8).cpu().numpy().reshape(n * S, 64).astype(np.int64)
        a = np.arange(R)
        X = X * np.ldexp(1.0, -ex[:, (a & 3) * 16 + (a >> 2)])[:, :, None]
    return X.reshape(n, S, R, K)


@pytest.mark.parametrize("precision", ["mixed", "bf16"])
def test_fft_mfma_grid_matches_oracle(precision):
    cfg = synth.CFG2.replace(snr_db=20.0)
    b = synth.make_batch(cfg, [4100, 4101])
    n = 2
    got = {}
    for mf in (True, False):
        slot = slot_for(cfg, n, precision, b["sigma2"], mf)
        slot(dev(b["x_td"]), dev(b["pilots"]))
        got[mf] = grid_from_workspace(slot, cfg, n, precision)
    ref = O.ofdm_demodulate(b["x_td"], cfg.n_sc)
    e_mf, e_valu = M.nrmse(got[True], ref), M.nrmse(got[False], ref)
    rel = np.max(np.abs(got[True] - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2))
    print(f"[fft_mfma] {precision} grid NRMSE {e_mf:.3e} (vector-unit FFT {e_valu:.3e}), max-rel {rel:.3e}", flush=True)
    assert e_mf <= TOL_GRID[precision] and rel <= 10 * TOL_GRID[precision]
    assert e_valu <= e_mf  # the vector-unit FFT rounds once, the matrix-core one per pass


@pytest.mark.parametrize("precision,snr_db", [("mixed", 10.0), ("mixed", 30.0), ("bf16", 10.0), ("bf16", 30.0)])
def test_fft_mfma_slot_evm_gap_and_oracle(precision, snr_db):
    cfg = synth.CFG2.replace(snr_db=snr_db)
    b = synth.make_batch(cfg, [4200, 4201])
    x, p = dev(b["x_td"]), dev(b["pilots"])
    x32, st32 = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb,
                           b["sigma2"], 2)(x, p)
    xm, stm = slot_for(cfg, 2, precision, b["sigma2"])(x, p)
    torch.cuda.synchronize()
    x32, xm = x32.cpu().numpy(), xm.cpu().numpy()
    assert int(st32.sum()) == 0 and int(stm.sum()) == 0
    data = b["data"].transpose(0, 1, 3, 2)
    gap = M.evm_db(xm, data) - M.evm_db(x32, data)
    print(f"[fft_mfma] {precision} {snr_db} dB: EVM FP32 {M.evm_db(x32, data):.3f} dB, gap {gap:.4f} dB", flush=True)
    assert abs(gap) <= EVM_GAP_DB
    for k in range(2):
        ref = O.receive_slot(b["x_td"][k], b["pilots"][k], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                             n_beams=cfg.n_beams)
        assert_xhat(xm[k], ref["x_hat"], TOL_X[precision], f"{precision} fft_mfma")


def test_fft_mfma_every_bin_and_row_scaling():
    # all 4096 bins (the output shift wraps), and inputs scaled by 2^40 with
    # sigma2 by 2^80: the FP16 row scaling keeps every pass in range
    cfg = synth.CFG2.replace(n_sc=4096, n_ant=16, n_beams=16, n_ue=8, snr_db=25.0)
    b = synth.make_batch(cfg, [4300])
    x, p = dev(b["x_td"]), dev(b["pilots"])
    base_slot = slot_for(cfg, 1, "mixed", b["sigma2"])
    base, st = base_slot(x, p)
    grid = grid_from_workspace(base_slot, cfg, 1, "mixed")
    ref = O.ofdm_demodulate(b["x_td"], cfg.n_sc)
    assert M.nrmse(grid, ref) <= TOL_GRID["mixed"]
    a = 2.0 ** 40
    big, st2 = slot_for(cfg, 1, "mixed", b["sigma2"] * a * a)((x * a).contiguous(), p)
    torch.cuda.synchronize()
    assert int(st.sum()) == 0 and int(st2.sum()) == 0
    base, big = base.cpu().numpy(), big.cpu().numpy()
    assert np.all(np.isfinite(big)) and M.nrmse(big, base) <= 1e-6
    xref = O.receive_slot(b["x_td"][0], b["pilots"][0], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                          n_beams=cfg.n_beams)
    assert_xhat(base[0], xref["x_hat"], TOL_X["mixed"])
