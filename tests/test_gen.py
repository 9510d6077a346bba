"""Statistics and structure of the seeded synthetic slot generator."""
import math

import numpy as np
import pytest

from paper_2210_09196_amd import synth


@pytest.mark.parametrize("bits", [2, 4, 6, 8])
def test_qam_unit_energy_and_gray_neighbours(bits):
    pts, lab = synth.qam_table(bits)
    assert len(set(np.round(pts, 12).tolist())) == 1 << bits
    assert abs(np.mean(np.abs(pts) ** 2) - 1.0) < 1e-12
    # Gray: nearest neighbours (horizontal/vertical) differ in exactly one bit
    dmin = min(abs(a - b) for i, a in enumerate(pts) for b in pts[i + 1:])
    for i in range(len(pts)):
        for j in range(len(pts)):
            if i != j and abs(abs(pts[i] - pts[j]) - dmin) < 1e-9:
                assert int(np.sum(lab[i] != lab[j])) == 1


def test_qam_16_matches_standard_corner():
    pts, lab = synth.qam_table(4)
    # bits 0000 -> (1 + 1j)/sqrt(10); bits 0011 -> (3 + 3j)/sqrt(10)
    assert abs(pts[0] - (1 + 1j) / math.sqrt(10)) < 1e-15
    assert abs(pts[0b0011] - (3 + 3j) / math.sqrt(10)) < 1e-15


def test_tdl_profile_sums_to_one_and_hits_rms_spread():
    p, tau = synth.tdl_profile(8, 300e-9)
    assert abs(p.sum() - 1) < 1e-15
    mean = (p * tau).sum()
    rms = math.sqrt((p * tau * tau).sum() - mean * mean)
    assert abs(rms - 300e-9) < 1e-15
    assert abs(tau[1] - 316.37e-9) < 0.01e-9


def test_pilot_comb_covers_every_ue():
    for n_ue, n_pilot in [(4, 1), (16, 2), (3, 2), (1, 2)]:
        for j in range(n_pilot):
            own = synth.pilot_owner(40, j, n_ue, n_pilot)
            assert set(own.tolist()) == set(range(n_ue))


def test_slot_shapes_and_noise_variance():
    cfg = synth.CFG1
    a = synth.make_slot(cfg, 5)
    b = synth.make_slot(cfg.replace(snr_db=None), 5)
    assert a["x_td"].shape == (14, 16, 256) and a["x_td"].dtype == np.complex64
    assert a["pilots"].shape == (1, 256)
    assert a["data"].shape == (13, 4, 256)
    # same seed: same signal; the difference is the noise, CN(0, sigma^2/N) per sample
    diff = a["x_td"].astype(complex) - b["x_td"].astype(complex)
    var = np.mean(np.abs(diff) ** 2) * cfg.n_fft
    assert abs(var / a["sigma2"] - 1) < 5 / math.sqrt(diff.size)


def test_time_domain_is_inverse_fft_of_grid():
    cfg = synth.CFG1.replace(snr_db=None, n_sc=200)
    s = synth.make_slot(cfg, 3)
    full = np.fft.fft(s["x_td"].astype(complex), axis=-1)
    bins = (np.arange(200) - 100) % 256
    assert np.max(np.abs(full[..., bins] - s["grid"])) < 1e-5
    inactive = np.setdiff1d(np.arange(256), bins)
    assert np.max(np.abs(full[..., inactive])) < 1e-5


def test_generator_is_deterministic():
    a = synth.make_slot(synth.CFG1, 11)
    b = synth.make_slot(synth.CFG1, 11)
    assert np.array_equal(a["x_td"], b["x_td"])
    c = synth.make_slot(synth.CFG1, 12)
    assert not np.array_equal(a["x_td"], c["x_td"])
