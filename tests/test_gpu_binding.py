"""The Python binding rejects output buffers of the wrong size, dtype or
device before anything is launched: the C ABI takes plain pointers and
cannot see a buffer's size, so every output tensor is checked in Python
(a short buffer would otherwise be written past its end)."""
import pytest
import torch

from paper_2210_09196_amd import pusch, synth

pytestmark = pytest.mark.gpu

DEV = "cuda"
C64 = torch.complex64


def z(*shape, dtype=C64, device=DEV):
    return torch.zeros(*shape, dtype=dtype, device=device)


def test_stand_alone_outputs_are_checked():
    X = z(2, 8, 32)
    with pytest.raises(pusch.PuschError, match="elements"):
        pusch.beamform(X, 4, out=z(2, 32, 3))
    Yp = z(2, 1, 64, 8)
    p = z(2, 1, 64)
    with pytest.raises(pusch.PuschError, match="elements"):
        pusch.chest(Yp, p, 4, out=z(2, 64, 4, 7))
    with pytest.raises(pusch.PuschError, match="CUDA"):
        pusch.noise_est(Yp, p, 4, out=torch.zeros(2, dtype=torch.float32))
    with pytest.raises(pusch.PuschError, match="elements"):
        pusch.noise_est(Yp, p, 4, out=z(1, dtype=torch.float32))
    H = z(2, 64, 4, 8)
    Yd = z(2, 3, 64, 8)
    with pytest.raises(pusch.PuschError, match="elements"):
        pusch.mmse_solve(H, Yd, 0.1, out=z(2, 3, 64, 3))
    with pytest.raises(pusch.PuschError, match="int32"):
        pusch.mmse_solve(H, Yd, 0.1, status=z(2, 64, dtype=torch.int64))
    with pytest.raises(pusch.PuschError, match="elements"):
        pusch.mmse_solve(H, Yd, 0.1, status=z(2, 63, dtype=torch.int32))
    torch.cuda.synchronize()


def test_slot_and_cells_outputs_are_checked():
    cfg = synth.CFG1
    slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb, 0.01, 2)
    n_data = cfg.n_symb - len(cfg.pilot_symb)
    x = z(2, cfg.n_symb, cfg.n_ant, cfg.n_fft)
    p = z(2, len(cfg.pilot_symb), cfg.n_sc)
    with pytest.raises(pusch.PuschError, match="x_hat"):
        slot(x, p, z(1, n_data, cfg.n_sc, cfg.n_ue))
    with pytest.raises(pusch.PuschError, match="int32"):
        slot(x, p, z(2, n_data, cfg.n_sc, cfg.n_ue), z(2, cfg.n_sc, dtype=torch.float32))
    with pytest.raises(pusch.PuschError, match="elements"):
        slot(x, p, z(2, n_data, cfg.n_sc, cfg.n_ue), z(2, cfg.n_sc - 1, dtype=torch.int32))

    geom = dict(n_ant=cfg.n_ant, n_fft=cfg.n_fft, n_sc=cfg.n_sc, n_symb=cfg.n_symb, n_beams=cfg.n_beams,
                n_ue=cfg.n_ue, pilot_symb=cfg.pilot_symb, sigma2=0.01, n_slot=1)
    cells = pusch.Cells([geom, geom])
    xs, ps = [z(1, cfg.n_symb, cfg.n_ant, cfg.n_fft)] * 2, [z(1, len(cfg.pilot_symb), cfg.n_sc)] * 2
    outs, sts = cells.outputs()
    with pytest.raises(pusch.PuschError, match="cell 1: status"):
        cells(xs, ps, outs, [sts[0], z(1, cfg.n_sc // 2, dtype=torch.int32)])
    with pytest.raises(pusch.PuschError, match="expected"):
        cells(xs, ps, outs[:1], sts[:1])
    torch.cuda.synchronize()


def test_slot_and_cells_reject_a_beamformer_of_the_wrong_shape():
    # the chain reads n_beams * n_ant values of W: a short one would be read past its end
    cfg = synth.CFG1
    for bad in (z(cfg.n_beams, cfg.n_ant - 1), z(cfg.n_beams - 1, cfg.n_ant), z(cfg.n_beams * cfg.n_ant)):
        with pytest.raises(pusch.PuschError, match="W must be"):
            pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb, 0.01, 1,
                       W=bad)
        geom = dict(n_ant=cfg.n_ant, n_fft=cfg.n_fft, n_sc=cfg.n_sc, n_symb=cfg.n_symb, n_beams=cfg.n_beams,
                    n_ue=cfg.n_ue, pilot_symb=cfg.pilot_symb, sigma2=0.01, n_slot=1)
        with pytest.raises(pusch.PuschError, match="cell 1: W must be"):
            pusch.Cells([geom, dict(geom, W=bad)])
    ok = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb, 0.01, 1,
                    W=z(cfg.n_beams, cfg.n_ant))
    assert ok.W.shape == (cfg.n_beams, cfg.n_ant)
    torch.cuda.synchronize()
