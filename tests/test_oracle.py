"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each stage of the chain is checked against something other than the oracle's
own formula: hand-derived worked examples (tests/golden), brute-force sums on
tiny inputs, closed forms, independent library routines and invariants.  The
mutation tests at the end plant plausible mistakes in a copy of the oracle and
check that one of these pins catches each of them.
"""
import math
import types

import numpy as np
import pytest

from oracle import pusch_oracle as O
from oracle import metrics as M
from paper_2210_09196_amd import synth

RNG = np.random.default_rng(1234)


def crandn(*shape, rng=RNG):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def naive_dft(x):
    """Brute-force O(N^2) DFT written as explicit sums (definition of Sec. II's FFT)."""
    n = len(x)
    out = []
    for f in range(n):
        acc = 0j
        for t in range(n):
            ang = -2.0 * math.pi * ((f * t) % n) / n
            acc += x[t] * complex(math.cos(ang), math.sin(ang))
        out.append(acc)
    return np.array(out)


# ----------------------------------------------------------------------------- OFDM demodulation (FFT)

@pytest.mark.parametrize("n", [4, 16, 64, 256])
def test_fft_matches_bruteforce_dft(n):
    x = crandn(n)
    X = O.ofdm_demodulate(x)
    ref = naive_dft(x)
    assert np.max(np.abs(X - ref)) <= 1e-12 * n * np.max(np.abs(ref))


def test_fft_golden(golden):
    g = golden("dft_small.txt")
    np.testing.assert_allclose(O.ofdm_demodulate(np.array(g["x1"], complex)), g["X1"], atol=1e-13)
    np.testing.assert_allclose(O.ofdm_demodulate(np.array(g["x2"], complex)), g["X2"], atol=1e-13)
    X3 = O.ofdm_demodulate(np.array(g["x3"], complex))
    np.testing.assert_allclose(X3[0::2], g["X3_even"], atol=1e-13)


@pytest.mark.parametrize("n", [64, 4096])
def test_fft_parseval_impulse_tone_linearity(n):
    x = crandn(3, n)
    X = O.ofdm_demodulate(x)
    np.testing.assert_allclose(np.sum(np.abs(X) ** 2, -1), n * np.sum(np.abs(x) ** 2, -1), rtol=1e-12)
    imp = np.zeros(n, complex)
    imp[0] = 1.0
    np.testing.assert_allclose(O.ofdm_demodulate(imp), np.ones(n), atol=1e-13)
    f0 = 5
    tone = np.exp(2j * np.pi * f0 * np.arange(n) / n)
    expect = np.zeros(n, complex)
    expect[f0] = n
    np.testing.assert_allclose(O.ofdm_demodulate(tone), expect, atol=1e-9)
    a, b = 0.3 - 1.1j, 2.0 + 0.5j
    np.testing.assert_allclose(O.ofdm_demodulate(a * x[0] + b * x[1]), a * X[0] + b * X[1], atol=1e-10)
    g = crandn(n)
    np.testing.assert_allclose(O.ofdm_demodulate(np.fft.ifft(g)), g, atol=1e-12)


@pytest.mark.parametrize("n_fft,n_sc", [(4096, 3300), (256, 256), (64, 63), (1024, 1)])
def test_active_bin_map(n_fft, n_sc):
    bins = O.active_bins(n_fft, n_sc)
    assert len(set(bins.tolist())) == n_sc  # distinct bins
    assert bins[n_sc // 2] == 0  # DC sits at the centre subcarrier
    # a tone on bin f lands on subcarrier (f + n_sc//2) mod N when that is < n_sc
    for f in (0, 1, n_fft - 1, 7):
        k = (f + n_sc // 2) % n_fft
        tone = np.exp(2j * np.pi * f * np.arange(n_fft) / n_fft)
        Xa = O.ofdm_demodulate(tone, n_sc)
        if k < n_sc:
            assert abs(Xa[k] - n_fft) < 1e-8
            assert np.sum(np.abs(Xa) > 1e-6) == 1
        else:
            assert np.all(np.abs(Xa) < 1e-6)


# ----------------------------------------------------------------------------- beamforming

@pytest.mark.parametrize("nb,nr", [(16, 16), (32, 64), (5, 7)])
def test_dft_beamformer_rows_orthonormal(nb, nr):
    W = O.dft_beamformer(nb, nr)
    np.testing.assert_allclose(W @ W.conj().T, np.eye(nb), atol=1e-13)


def test_square_dft_beamforming_is_antenna_fft():
    nr, K = 16, 10
    X = crandn(3, nr, K)
    Y = O.beamform(O.dft_beamformer(nr, nr), X)
    np.testing.assert_allclose(Y, np.fft.fft(X, axis=1) / math.sqrt(nr), atol=1e-12)


def test_beamform_bruteforce():
    W = crandn(3, 5)
    X = crandn(2, 5, 4)
    Y = O.beamform(W, X)
    for s in range(2):
        for b in range(3):
            for k in range(4):
                acc = sum(W[b, r] * X[s, r, k] for r in range(5))
                assert abs(Y[s, b, k] - acc) < 1e-12


# ----------------------------------------------------------------------------- LS channel estimation

def test_ls_golden(golden):
    g = golden("ls_comb_small.txt")
    Yp = np.array(g["Y"], complex)[None, None, :]
    p = np.array(g["pilots"], complex)[None, :]
    H = O.ls_channel_estimate(Yp, p, g["n_ue"])
    np.testing.assert_allclose(H[:, 0, 0], g["H_ue0"], atol=1e-14)
    np.testing.assert_allclose(H[:, 0, 1], g["H_ue1"], atol=1e-14)


def _comb_pilot_grid(Hk, pilots, n_ue):
    """Beam-domain pilot symbols of a known channel Hk [K, NB, NL] (noiseless)."""
    n_pilot, K = pilots.shape
    Yp = np.zeros((n_pilot, Hk.shape[1], K), complex)
    for j in range(n_pilot):
        own = (np.arange(K) + j * (n_ue // n_pilot)) % n_ue
        Yp[j] = Hk[np.arange(K), :, own].T * pilots[j][None, :]
    return Yp


@pytest.mark.parametrize("n_ue,n_pilot,K", [(4, 1, 64), (16, 2, 200), (3, 2, 31)])
def test_ls_linear_channel_is_exact(n_ue, n_pilot, K):
    nb = 5
    A, B = crandn(nb, n_ue), crandn(nb, n_ue)
    k = np.arange(K, dtype=float)
    Hk = A[None] + B[None] * k[:, None, None]
    pil = synth.qam_modulate(RNG.integers(0, 2, (n_pilot, K, 2)), 2)
    H = O.ls_channel_estimate(_comb_pilot_grid(Hk, pil, n_ue), pil, n_ue)
    for l in range(n_ue):
        pos = [kk for kk in range(K) if any((kk + j * (n_ue // n_pilot)) % n_ue == l for j in range(n_pilot))]
        lo, hi = pos[0], pos[-1]
        np.testing.assert_allclose(H[lo:hi + 1, :, l], Hk[lo:hi + 1, :, l], atol=1e-11)
        # end-value hold beyond the outermost pilots
        np.testing.assert_allclose(H[:lo, :, l], np.broadcast_to(Hk[lo, :, l], (lo, nb)), atol=1e-11)
        np.testing.assert_allclose(H[hi + 1:, :, l], np.broadcast_to(Hk[hi, :, l], (K - hi - 1, nb)), atol=1e-11)


def test_ls_duplicate_positions_are_averaged():
    K, nb = 12, 3
    pil = synth.qam_modulate(RNG.integers(0, 2, (2, K, 2)), 2)
    Yp = crandn(2, nb, K)
    H = O.ls_channel_estimate(Yp, pil, 1)  # one UE: both pilot symbols hit every subcarrier
    ls = Yp * (np.conj(pil) / np.abs(pil) ** 2)[:, None, :]
    np.testing.assert_allclose(H[:, :, 0], ((ls[0] + ls[1]) / 2).T, atol=1e-13)


def test_ls_noise_variance_on_pilot_res():
    K, nb, sigma2 = 4000, 4, 0.05
    pil = synth.qam_modulate(RNG.integers(0, 2, (1, K, 2)), 2) * 1.7
    Hk = np.zeros((K, nb, 1), complex)
    Yp = _comb_pilot_grid(Hk, pil, 1) + crandn(1, nb, K) * math.sqrt(sigma2 / 2)
    H = O.ls_channel_estimate(Yp, pil, 1)
    est = np.mean(np.abs(H) ** 2)
    expect = sigma2 / 1.7 ** 2
    # 16000 samples of an exponential variable: relative std 1/sqrt(16000) ~ 0.8 %; 5 sigma bound
    assert abs(est / expect - 1) < 5 / math.sqrt(K * nb)


def test_ls_noiseless_flat_chain_recovers_beam_channel():
    cfg = synth.CFG1.replace(snr_db=None)
    s = synth.make_slot(cfg, 7)
    r = O.receive_slot(s["x_td"], s["pilots"], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, 0.0, n_beams=cfg.n_beams)
    H_beam = O.dft_beamformer(cfg.n_beams, cfg.n_ant) @ s["h_ant"]  # [K, NB, NL]
    assert M.nrmse(r["H"], H_beam) < 1e-6  # input is complex64: error is its rounding


# ----------------------------------------------------------------------------- Gram + Crout

def test_crout_golden_exact(golden):
    g = golden("crout_3x3.txt")
    L, ok = O.cholesky_crout(np.array(g["G"], complex))
    assert ok
    np.testing.assert_array_equal(L, np.array(g["L"], complex))


@pytest.mark.parametrize("n", [1, 2, 4, 16, 32])
def test_crout_reconstructs_and_matches_lapack(n):
    H = crandn(50, n + 3, n)
    G = O.gram(H, 0.1)
    L, ok = O.cholesky_crout(G)
    assert ok.all()
    np.testing.assert_allclose(L @ np.conj(np.swapaxes(L, -1, -2)), G, atol=1e-11 * n)
    assert np.all(np.triu(L, 1) == 0)
    d = np.diagonal(L, axis1=-2, axis2=-1)
    assert np.all(d.imag == 0) and np.all(d.real > 0)
    np.testing.assert_allclose(L, np.linalg.cholesky(G), atol=1e-11 * n)


def test_crout_2x2_closed_form():
    G = np.array([[5.0, 1 - 2j], [1 + 2j, 4.0]])
    L, ok = O.cholesky_crout(G)
    l11 = math.sqrt(5.0)
    l21 = (1 + 2j) / l11
    l22 = math.sqrt(4.0 - abs(l21) ** 2)
    np.testing.assert_allclose(L, [[l11, 0], [l21, l22]], atol=1e-15)


def test_gram_bruteforce():
    H = crandn(6, 3)
    G = O.gram(H, 0.25)
    for i in range(3):
        for j in range(3):
            acc = sum(np.conj(H[b, i]) * H[b, j] for b in range(6)) + (0.25 if i == j else 0)
            assert abs(G[i, j] - acc) < 1e-13


def test_crout_flags_non_pd():
    H = crandn(4, 8, 3)
    H[1, :, 2] = 0  # zero UE column, sigma^2 = 0: pivot exactly 0
    H[2, 0, 0] = np.nan
    G = O.gram(H, 0.0)
    G[3] = np.diag([1.0, -1.0, 1.0])
    _, ok = O.cholesky_crout(G)
    assert ok.tolist() == [True, False, False, False]


# ----------------------------------------------------------------------------- matched filter + substitution

def test_mmse_golden(golden):
    g = golden("mmse_2x2.txt")
    H = np.array(g["H"], complex)[None]
    y = np.array(g["y"], complex)[None, None]
    x, ok = O.mmse_detect(H, y, g["sigma2"])
    np.testing.assert_allclose(x[0, 0], g["x"], atol=1e-14)
    x0, _ = O.mmse_detect(H, y, 0.0)
    np.testing.assert_allclose(x0[0, 0], g["x_zf"], atol=1e-14)


@pytest.mark.parametrize("nb,nl", [(2, 2), (8, 4), (32, 16)])
def test_mmse_matches_explicit_inverse(nb, nl):
    K, D = 20, 3
    H = crandn(K, nb, nl)
    y = crandn(D, K, nb)
    s2 = 0.3
    x, ok = O.mmse_detect(H, y, s2)
    assert ok.all()
    for k in range(K):
        Gi = np.linalg.inv(H[k].conj().T @ H[k] + s2 * np.eye(nl))
        for d in range(D):
            np.testing.assert_allclose(x[d, k], Gi @ H[k].conj().T @ y[d, k], atol=1e-10)


def test_mmse_tends_to_zero_forcing():
    H = crandn(10, 8, 4)
    y = crandn(2, 10, 8)
    x, _ = O.mmse_detect(H, y, 1e-12)
    zf = np.einsum("klb,dkb->dkl", np.linalg.pinv(H), y)
    np.testing.assert_allclose(x, zf, atol=1e-9)


def test_mmse_single_ue_closed_form():
    h = crandn(30, 6, 1)
    y = crandn(4, 30, 6)
    s2 = 0.7
    x, _ = O.mmse_detect(h, y, s2)
    ref = np.einsum("kb,dkb->dk", np.conj(h[:, :, 0]), y) / (np.sum(np.abs(h[:, :, 0]) ** 2, -1) + s2)
    np.testing.assert_allclose(x[:, :, 0], ref, atol=1e-12)


def test_mmse_noiseless_exact_recovery():
    H = crandn(40, 16, 8)
    xs = crandn(5, 40, 8)
    y = np.einsum("kbl,dkl->dkb", H, xs)
    x, ok = O.mmse_detect(H, y, 0.0)
    np.testing.assert_allclose(x, xs, atol=1e-10)


def test_mmse_failed_subcarrier_is_zeroed():
    H = crandn(3, 4, 2)
    H[1, :, 1] = 0
    x, ok = O.mmse_detect(H, crandn(2, 3, 4), 0.0)
    assert ok.tolist() == [True, False, True]
    assert np.all(x[:, 1] == 0)


def test_single_ue_qpsk_ber_matches_rayleigh_mrc_closed_form():
    # N_L = 1: MMSE is a positive scaling of maximum-ratio combining, so QPSK
    # decisions follow the textbook L-branch MRC BER in i.i.d. Rayleigh fading:
    # P_b = ((1-mu)/2)^L sum_{k<L} C(L-1+k, k) ((1+mu)/2)^k, mu = sqrt(g/(1+g)),
    # with g the per-branch SNR per bit (Es/N0 / 2 for QPSK).
    rng = np.random.default_rng(99)
    n, nb, snr_db = 200_000, 2, 6.0
    s2 = 10 ** (-snr_db / 10)
    bits = rng.integers(0, 2, (n, 2))
    x = synth.qam_modulate(bits, 2)
    h = (rng.standard_normal((n, nb)) + 1j * rng.standard_normal((n, nb))) / math.sqrt(2)
    noise = (rng.standard_normal((n, nb)) + 1j * rng.standard_normal((n, nb))) * math.sqrt(s2 / 2)
    y = h * x[:, None] + noise
    xh, _ = O.mmse_detect(h[:, :, None], y[None], s2)
    pts, lab = synth.qam_table(2)
    _, bh = M.hard_decide(xh[0, :, 0], pts, lab)
    ber = np.mean(bh != bits)
    g = (1 / s2) / 2
    mu = math.sqrt(g / (1 + g))
    pb = ((1 - mu) / 2) ** nb * sum(math.comb(nb - 1 + k, k) * ((1 + mu) / 2) ** k for k in range(nb))
    sd = math.sqrt(pb * (1 - pb) / (2 * n))
    assert abs(ber - pb) < 5 * sd + 1e-4


# ----------------------------------------------------------------------------- noise estimation

def _ne_golden(mod, g, e):
    return mod.noise_variance_estimate(np.array(g[e + "_Y"], complex), np.array(g[e + "_pilots"], complex),
                                       g[e + "_n_ue"])


def test_noise_estimate_golden(golden):
    g = golden("ne_small.txt")
    for e in "ABC":
        assert abs(_ne_golden(O, g, e) - g[e + "_sigma2"]) <= 1e-14 * g[e + "_sigma2"], e


def _ne_inputs(rng, K, n_ue, n_pilot, n_beams, sigma2, slope=0.0):
    """Pilot symbols through a channel h_l(k) = a_l + slope * k b_l per beam, plus CN(0, sigma2) noise;
    pilots of random phase and magnitude 0.5..2."""
    a = crandn(n_ue, n_beams, rng=rng)
    b = crandn(n_ue, n_beams, rng=rng)
    p = rng.uniform(0.5, 2.0, (n_pilot, K)) * np.exp(2j * np.pi * rng.uniform(size=(n_pilot, K)))
    Y = np.zeros((n_pilot, n_beams, K), complex)
    for j in range(n_pilot):
        for k in range(K):
            l = (k + j * (n_ue // n_pilot)) % n_ue
            Y[j, :, k] = (a[l] + slope * k * b[l]) * p[j, k]
    Y += crandn(n_pilot, n_beams, K, rng=rng) * math.sqrt(sigma2 / 2)
    return Y, p


@pytest.mark.parametrize("n_ue,n_pilot", [(4, 2), (2, 4), (3, 2), (1, 1)])
def test_noise_estimate_noiseless_flat_channel_is_zero(n_ue, n_pilot):
    Y, p = _ne_inputs(np.random.default_rng(n_ue * 10 + n_pilot), 40, n_ue, n_pilot, 3, 0.0)
    assert O.noise_variance_estimate(Y, p, n_ue) <= 1e-28


@pytest.mark.parametrize("n_ue,n_pilot", [(4, 2), (2, 4), (3, 2)])
def test_noise_estimate_is_unbiased(n_ue, n_pilot):
    # stagger (4, 2), all pilot symbols on the same subcarriers (2, 4: four values averaged per
    # position) and unequal gaps (3, 2); pilots of unequal power
    rng = np.random.default_rng(77 + n_ue)
    sigma2 = 0.3
    ratios = []
    for _ in range(40):
        Y, p = _ne_inputs(rng, 200, n_ue, n_pilot, 4, sigma2)
        ratios.append(O.noise_variance_estimate(Y, p, n_ue) / sigma2)
    m, se = np.mean(ratios), np.std(ratios, ddof=1) / math.sqrt(len(ratios))
    assert abs(m - 1.0) < 5 * se, (m, se)
    assert se < 0.02


def _selective_inputs(rng, K, n_ue, n_pilot, n_beams, sigma2, aligned):
    """Pilot symbols through a channel drawn independently on every subcarrier (no frequency
    correlation at all), static over the slot, plus CN(0, sigma2) noise; unit pilots of random phase."""
    h = crandn(n_ue, n_beams, K, rng=rng)
    p = np.exp(2j * np.pi * rng.uniform(size=(n_pilot, K)))
    Y = np.zeros((n_pilot, n_beams, K), complex)
    for j in range(n_pilot):
        own = O.pilot_owner(K, j, n_ue, n_pilot, aligned)
        for k in range(K):
            Y[j, :, k] = h[own[k], :, k] * p[j, k]
    return Y + crandn(n_pilot, n_beams, K, rng=rng) * math.sqrt(sigma2 / 2), p


@pytest.mark.parametrize("n_pilot", [2, 3])
def test_noise_estimate_aligned_comb_is_unbiased_on_any_channel(n_pilot):
    # R21: with the aligned comb every pilot RE is compared at its own subcarrier, so even a channel
    # with no correlation between subcarriers leaves noise only; the staggered comb's leave-one-out
    # prediction cannot follow such a channel and counts the channel's own variation as noise
    rng = np.random.default_rng(300 + n_pilot)
    sigma2 = 0.01
    ratios = []
    for _ in range(30):
        Y, p = _selective_inputs(rng, 160, 4, n_pilot, 4, sigma2, aligned=True)
        ratios.append(O.noise_variance_estimate(Y, p, 4, aligned=True) / sigma2)
    m, se = np.mean(ratios), np.std(ratios, ddof=1) / math.sqrt(len(ratios))
    assert abs(m - 1.0) < 5 * se and se < 0.03, (m, se)
    Y, p = _selective_inputs(rng, 160, 4, n_pilot, 4, sigma2, aligned=False)
    assert O.noise_variance_estimate(Y, p, 4) > 20 * sigma2


def test_aligned_comb_places_every_ue_on_the_same_subcarriers():
    for j in range(3):
        assert np.array_equal(O.pilot_owner(12, j, 4, 3, aligned=True), np.arange(12) % 4)
    # a staggered comb of 16 UEs on two pilot symbols shifts by 8
    assert np.array_equal(O.pilot_owner(16, 1, 16, 2), (np.arange(16) + 8) % 16)
    assert np.array_equal(synth.pilot_owner(16, 1, 16, 2, aligned=True), O.pilot_owner(16, 1, 16, 2, aligned=True))


def test_noise_estimate_scales_with_power():
    Y, p = _ne_inputs(np.random.default_rng(5), 60, 4, 2, 3, 0.5, slope=0.1)
    s = O.noise_variance_estimate(Y, p, 4)
    assert abs(O.noise_variance_estimate(Y * (3 - 4j), p, 4) - 25 * s) <= 1e-12 * 25 * s
    # a common unit-modulus factor on the pilots and the received values changes nothing
    assert abs(O.noise_variance_estimate(Y * 1j, p * 1j, 4) - s) <= 1e-12 * s


def test_noise_estimate_needs_two_positions_per_ue():
    with pytest.raises(ValueError):
        O.noise_variance_estimate(np.ones((1, 2, 7)), np.ones((1, 7)), 4)


def test_noise_estimate_in_the_chain():
    cfg = synth.CFG1
    s = synth.make_slot(cfg, 1000)
    r = O.receive_slot(s["x_td"], s["pilots"], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, None, n_beams=cfg.n_beams)
    # 256 pilot REs x 16 beams: standard error about 3 %
    assert abs(r["sigma2"] / s["sigma2"] - 1.0) < 0.15
    pts, lab = synth.qam_table(cfg.qam_bits)
    _, bh = M.hard_decide(r["x_hat"], pts, lab)
    assert np.mean(bh != np.swapaxes(s["bits"], 1, 2)) == 0.0
    quiet = synth.make_slot(cfg.replace(snr_db=None), 1000)
    r0 = O.receive_slot(quiet["x_td"], quiet["pilots"], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, None,
                        n_beams=cfg.n_beams)
    assert r0["sigma2"] < 1e-10  # flat channel, no noise: only the input's FP32 rounding remains


# ----------------------------------------------------------------------------- time-varying channel estimate

def _linear_in_time(rng, K, n_ue, n_beams, pilot_symb):
    """Pilot symbols through a channel flat in frequency and linear in time, h_l(s) = a_l + s b_l."""
    n_pilot = len(pilot_symb)
    a = crandn(n_beams, n_ue, rng=rng)
    b = crandn(n_beams, n_ue, rng=rng)
    p = np.exp(2j * np.pi * rng.uniform(size=(n_pilot, K))) * rng.uniform(0.5, 2.0, (n_pilot, K))
    Y = np.zeros((n_pilot, n_beams, K), complex)
    for j, s in enumerate(pilot_symb):
        own = (np.arange(K) + j * (n_ue // n_pilot)) % n_ue
        Y[j] = (a + s * b)[:, own] * p[j][None, :]
    return Y, p, a, b


@pytest.mark.parametrize("pilot_symb,n_ue", [((2, 11), 4), ((0, 4, 7, 11), 8), ((3, 9), 3)])
def test_time_interpolation_is_exact_for_a_channel_linear_in_time(pilot_symb, n_ue):
    Y, p, a, b = _linear_in_time(np.random.default_rng(len(pilot_symb)), 40, n_ue, 3, pilot_symb)
    for s in range(14):
        t = min(max(s, pilot_symb[0]), pilot_symb[-1])  # held outside the pilot symbols
        H = O.time_interpolated_estimate(Y, p, n_ue, pilot_symb, s)
        assert np.allclose(H, (a + t * b)[None], atol=1e-12), s


def test_single_pilot_symbol_estimate_ignores_the_others():
    Y, p, _, _ = _linear_in_time(np.random.default_rng(3), 32, 4, 2, (2, 11))
    H0 = O.ls_channel_estimate(Y, p, 4, use=[0])
    Y2 = Y.copy()
    Y2[1] *= -7.0
    assert np.array_equal(O.ls_channel_estimate(Y2, p, 4, use=[0]), H0)
    assert not np.allclose(O.ls_channel_estimate(Y2, p, 4), O.ls_channel_estimate(Y, p, 4))


def test_time_varying_chain_equals_static_chain_with_one_pilot_symbol():
    cfg = synth.CFG1
    s = synth.make_slot(cfg, 1000)
    a = O.receive_slot(s["x_td"], s["pilots"], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, s["sigma2"], n_beams=cfg.n_beams)
    b = O.receive_slot(s["x_td"], s["pilots"], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, s["sigma2"], n_beams=cfg.n_beams,
                       time_varying=True)
    assert np.allclose(a["x_hat"], b["x_hat"], atol=1e-12)


def test_time_varying_receiver_tracks_doppler():
    # 300 Hz over a slot of 14 symbols at 30 kHz: the per-symbol estimate must
    # beat the static one that averages the two pilot symbols
    cfg = synth.CFG1.replace(n_ant=16, n_fft=256, n_sc=240, n_beams=16, n_ue=4, pilot_symb=(2, 11), channel="flat",
                             doppler_hz=300.0, snr_db=30.0)
    s = synth.make_slot(cfg, 21)
    data = np.swapaxes(s["data"], 1, 2)
    st = O.receive_slot(s["x_td"], s["pilots"], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, s["sigma2"], n_beams=cfg.n_beams)
    tv = O.receive_slot(s["x_td"], s["pilots"], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, s["sigma2"], n_beams=cfg.n_beams,
                        time_varying=True)
    assert M.evm_db(tv["x_hat"], data) < M.evm_db(st["x_hat"], data) - 3.0


# ----------------------------------------------------------------------------- end to end

def test_chain_noiseless_cfg1_recovers_bits_exactly():
    cfg = synth.CFG1.replace(snr_db=None)
    s = synth.make_slot(cfg, 1000)
    r = O.receive_slot(s["x_td"], s["pilots"], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, 0.0, n_beams=cfg.n_beams)
    x = np.swapaxes(s["data"], 1, 2)
    assert M.evm_db(r["x_hat"], x) < -100
    pts, lab = synth.qam_table(cfg.qam_bits)
    _, bh = M.hard_decide(r["x_hat"], pts, lab)
    np.testing.assert_array_equal(bh, np.swapaxes(s["bits"], 1, 2))


def test_chain_cfg1_20db_error_free():
    cfg = synth.CFG1
    s = synth.make_slot(cfg, 1000)
    r = O.receive_slot(s["x_td"], s["pilots"], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, s["sigma2"], n_beams=cfg.n_beams)
    pts, lab = synth.qam_table(cfg.qam_bits)
    _, bh = M.hard_decide(r["x_hat"], pts, lab)
    assert np.mean(bh != np.swapaxes(s["bits"], 1, 2)) == 0.0
    assert r["ok"].all()


# ----------------------------------------------------------------------------- planted mistakes

def _mutant(old: str, new: str) -> types.ModuleType:
    """A copy of the oracle with one textual change (a planted mistake)."""
    src = open(O.__file__).read()
    assert src.count(old) >= 1, old
    mod = types.ModuleType("oracle_mutant")
    exec(compile(src.replace(old, new, 1), "oracle_mutant", "exec"), mod.__dict__)
    return mod


def _pins_pass(mod, golden) -> bool:
    """Run a compact set of the pins above against a module; False if any fails."""
    try:
        x = crandn(16)
        assert np.allclose(mod.ofdm_demodulate(x), naive_dft(x), atol=1e-9)
        # DC lands on the centre active subcarrier, bin 1 on the next one
        tone = np.exp(2j * np.pi * np.arange(8) / 8)
        assert abs(mod.ofdm_demodulate(np.ones(8), 5)[2] - 8) < 1e-9
        assert abs(mod.ofdm_demodulate(tone, 5)[3] - 8) < 1e-9
        g = golden("crout_3x3.txt")
        L, ok = mod.cholesky_crout(np.array(g["G"], complex))
        assert ok and np.array_equal(L, np.array(g["L"], complex))
        g = golden("mmse_2x2.txt")
        xm, _ = mod.mmse_detect(np.array(g["H"], complex)[None], np.array(g["y"], complex)[None, None], g["sigma2"])
        assert np.allclose(xm[0, 0], g["x"], atol=1e-12)
        Yt, pt, at, bt = _linear_in_time(np.random.default_rng(9), 24, 3, 2, (2, 11))
        for s_ in (0, 5, 13):
            tt = min(max(s_, 2), 11)
            assert np.allclose(mod.time_interpolated_estimate(Yt, pt, 3, (2, 11), s_), (at + tt * bt)[None], atol=1e-12)
        g = golden("ne_small.txt")
        for e in "ABC":
            assert abs(_ne_golden(mod, g, e) - g[e + "_sigma2"]) <= 1e-12
        g = golden("ls_comb_small.txt")
        H = mod.ls_channel_estimate(np.array(g["Y"], complex)[None, None, :], np.array(g["pilots"], complex)[None], 2)
        assert np.allclose(H[:, 0, 0], g["H_ue0"]) and np.allclose(H[:, 0, 1], g["H_ue1"])
        W = mod.dft_beamformer(4, 4)
        X = crandn(1, 4, 3)
        assert np.allclose(mod.beamform(W, X), np.fft.fft(X, axis=1) / 2)
        Hs = crandn(5, 8, 3)
        ys = crandn(2, 5, 8)
        xs, _ = mod.mmse_detect(Hs, ys, 0.2)
        for k in range(5):
            Gi = np.linalg.inv(Hs[k].conj().T @ Hs[k] + 0.2 * np.eye(3))
            assert np.allclose(xs[:, k], (Gi @ Hs[k].conj().T @ ys[:, k].T).T, atol=1e-9)
        return True
    except AssertionError:
        return False


MUTATIONS = [
    ("X = np.fft.fft(x, axis=-1)", "X = np.fft.ifft(x, axis=-1) * x.shape[-1]"),  # wrong FFT sign
    ("return (np.arange(n_sc) - n_sc // 2) % n_fft", "return (np.arange(n_sc) + n_sc // 2) % n_fft"),
    ("np.exp(-2j * np.pi * ((b * r) % n_ant) / n_ant)", "np.exp(2j * np.pi * ((b * r) % n_ant) / n_ant)"),
    ("(np.conj(p) / (p.real ** 2 + p.imag ** 2))", "(p / (p.real ** 2 + p.imag ** 2))"),  # LS without conjugate
    ("(0 if aligned else j * (n_ue // n_pilot))) % n_ue", "(0 if aligned else j * (n_ue // n_pilot) + 1)) % n_ue"),
    ("G = np.matmul(np.conj(np.swapaxes(H, -1, -2)), H)", "G = np.matmul(np.swapaxes(H, -1, -2), H)"),
    ("L[..., i, :j] * np.conj(row_j)", "L[..., i, :j] * row_j"),  # Crout without conjugate
    ("np.sum(row_j.real ** 2 + row_j.imag ** 2, axis=-1)", "0.0"),  # dropped term in the pivot
    ("L[..., i, :i] * z[..., :i]", "L[..., :i, i] * z[..., :i]"),  # transposed operand
    ("np.conj(L[..., i + 1:, i]) * x[..., i + 1:]", "L[..., i + 1:, i] * x[..., i + 1:]"),
    ('np.einsum("kbl,dkb->dkl", np.conj(H), Yd)', 'np.einsum("kbl,dkb->dkl", H, Yd)'),
    ("return G + float(sigma2) * np.eye(n)", "return G + float(sigma2)"),
    # noise estimation: noise gain dropped, no leave-one-out, swapped weights, unsquared weights,
    # conjugated pilot in the prediction
    ("den += n_beams * (1.0 + abs(pilots[j, k]) ** 2 * gain)", "den += n_beams * 1.0"),
    ("h = sum(w * mean[m] for m, w in weights.items())", "h = mean[k]"),
    ("weights = {below: (above - k) / (above - below), above: (k - below) / (above - below)}",
     "weights = {below: (k - below) / (above - below), above: (above - k) / (above - below)}"),
    ("gain = sum((w / cnt[m]) ** 2 * inv_pow[m]", "gain = sum((w / cnt[m]) * inv_pow[m]"),
    ("r = Yp[j][:, k] - pilots[j, k] * h", "r = Yp[j][:, k] - np.conj(pilots[j, k]) * h"),
    # same-position residual (R21): its own share of the mean ignored, 1/c instead of 1/c^2, not used
    ("den += n_beams * (1.0 - 2.0 / c + abs(pilots[j, k]) ** 2 / c ** 2 * inv_pow[k])",
     "den += n_beams * (1.0 + abs(pilots[j, k]) ** 2 / c ** 2 * inv_pow[k])"),
    ("/ c ** 2 * inv_pow[k]", "/ c * inv_pow[k]"),
    ("if c >= 2:  # the same subcarrier", "if c >= 3:  # the same subcarrier"),
    # time-varying estimate: swapped time weights, the wrong end held after the last pilot symbol
    ("return ((ps[b] - symb) * Ha + (symb - ps[a]) * Hb) / (ps[b] - ps[a])",
     "return ((symb - ps[a]) * Ha + (ps[b] - symb) * Hb) / (ps[b] - ps[a])"),
    ("return ls_channel_estimate(Yp, pilots, n_ue, use=[len(ps) - 1], aligned=aligned)",
     "return ls_channel_estimate(Yp, pilots, n_ue, use=[0], aligned=aligned)"),
]


def test_pins_pass_on_the_oracle(golden):
    assert _pins_pass(O, golden)


@pytest.mark.parametrize("old,new", MUTATIONS)
def test_planted_mistake_is_caught(old, new, golden):
    assert not _pins_pass(_mutant(old, new), golden)


# ----------------------------------------------------------------------------- scoring metrics (O7)
#
# The metrics decide pass or fail for every GPU parity test, so they are pinned
# to values worked out by hand, not to their own formulas.

QPSK_PTS = np.array([1 + 1j, 1 - 1j, -1 + 1j, -1 - 1j]) / math.sqrt(2.0)
QPSK_LAB = np.array([[0, 0], [0, 1], [1, 0], [1, 1]], np.uint8)
QAM16_ROW = np.array([-3, -1, 1, 3]) / math.sqrt(10.0)  # one rail of unit-energy 16-QAM
QAM16_PTS = (QAM16_ROW[:, None] + 1j * QAM16_ROW[None, :]).ravel()


def _metric_pins_pass(mm) -> bool:
    """Hand-worked values of every metric; False if a module's metrics miss any."""
    try:
        # nrmse: ||a - ref|| / ||ref||
        assert abs(mm.nrmse([1 + 1j], [1]) - 1.0) < 1e-15  # |i| / |1|
        assert abs(mm.nrmse([1, 0], [0, 1]) - math.sqrt(2.0)) < 1e-15  # sqrt(1 + 1) / 1
        assert abs(mm.nrmse([2, 0], [1, 0]) - 1.0) < 1e-15  # normalised by ||ref|| = 1, not ||a|| = 2
        assert abs(mm.nrmse([3, 4j], [3, 4j]) - 0.0) < 1e-15
        assert abs(mm.nrmse([3.3, 4.4j], [3, 4j]) - 0.1) < 1e-14  # a 10 % scale error
        # max_rel_err: ref [3, 4i, 0, 0] has RMS sqrt(25 / 4) = 2.5; one error of 1 -> 0.4
        assert abs(mm.max_rel_err([3, 4j, 0, 1], [3, 4j, 0, 0]) - 0.4) < 1e-15
        assert abs(mm.max_rel_err([3, 4j, 0.5, 1j], [3, 4j, 0, 0]) - 0.4) < 1e-15  # the largest, not the sum
        # worst_slice_err: rows [[1, 1], [1, 1]] (RMS 1); errors (0, 0.3) in row 0, (0.4, 0) in row 1
        ref = np.ones((2, 2))
        got = ref + np.array([[0.0, 0.3], [0.4j, 0.0]])
        assert abs(mm.worst_slice_err(got, ref, 0) - math.sqrt(0.16 / 2)) < 1e-15  # row 1
        assert abs(mm.worst_slice_err(got, ref, 1) - math.sqrt(0.16 / 2)) < 1e-15  # column 0
        got = ref + np.array([[0.0, 0.3], [0.0, 0.0]])
        assert abs(mm.worst_slice_err(got, ref, 0) - math.sqrt(0.09 / 2)) < 1e-15
        assert abs(mm.worst_slice_err(got, 2 * ref, 0) - 0.5) < 1e-15  # row 1 misses by (1, 1): RMS 1 over RMS 2
        # evm_db: a 10 % amplitude error is -20 dB (power ratio 0.01); an error as large as x is 0 dB
        x = QPSK_PTS[[0, 1, 2, 3, 0, 2]]
        assert abs(mm.evm_db(1.1 * x, x) - (-20.0)) < 1e-12
        assert abs(mm.evm_db(0.9 * x, x) - (-20.0)) < 1e-12
        assert abs(mm.evm_db(x + x * 1j, x) - 0.0) < 1e-12
        assert abs(mm.evm_db(x[:2] + np.array([0.1, 0.0]), x[:2]) - 10 * math.log10(0.01 / 2)) < 1e-12
        # hard_decide: nearest point; a tie at the origin goes to the lowest index
        idx, bits = mm.hard_decide(np.array([0.6 + 0.8j, 0.6 - 0.1j, -0.2 + 0.05j, -1 - 3j, 0j]), QPSK_PTS, QPSK_LAB)
        assert idx.tolist() == [0, 1, 2, 3, 0]
        assert bits.tolist() == [[0, 0], [0, 1], [1, 0], [1, 1], [0, 0]]
        # decision_margin (squared distances): on a point of unit-energy QPSK the second-nearest
        # neighbour is sqrt(2) away -> 2; on a decision boundary -> 0
        m = mm.decision_margin(np.array([QPSK_PTS[0], 0j, 0.5 + 0j, 0.3j]), QPSK_PTS)
        assert np.allclose(m, [2.0, 0.0, 0.0, 0.0], atol=1e-15)
        # 16-QAM with sqrt(10) normalisation: at (1 + i)/sqrt(10) the neighbours are 2/sqrt(10) away -> 0.4;
        # moved 0.1/sqrt(10) towards (3 + i)/sqrt(10): 1.9^2 / 10 - 0.1^2 / 10 = 0.36
        s10 = math.sqrt(10.0)
        m = mm.decision_margin(np.array([(1 + 1j) / s10, (1.1 + 1j) / s10]), QAM16_PTS)
        assert np.allclose(m, [0.4, 0.36], atol=1e-14)
        # xhat_errors bundles the three parity figures over the subcarrier axis (-2)
        ref = np.ones((3, 4, 2), complex)
        got = ref.copy()
        got[1, 2, 0] += 0.5
        e = mm.xhat_errors(got, ref)
        assert abs(e["nrmse"] - 0.5 / math.sqrt(24)) < 1e-15
        assert abs(e["max_rel"] - 0.5) < 1e-15
        assert abs(e["worst_sc"] - math.sqrt(0.25 / 6)) < 1e-15
        return True
    except AssertionError:
        return False


def test_metric_pins_pass():
    assert _metric_pins_pass(M)


def _metric_mutant(old: str, new: str) -> types.ModuleType:
    src = open(M.__file__).read()
    assert src.count(old) >= 1, old
    mod = types.ModuleType("metrics_mutant")
    exec(compile(src.replace(old, new, 1), "metrics_mutant", "exec"), mod.__dict__)
    return mod


METRIC_MUTATIONS = [
    # nrmse: squared ratio; normalised by ||a||; mean instead of RMS over elements
    ("return float(np.linalg.norm((a - ref).ravel()) / (den if den > 0 else 1.0))",
     "return float((np.linalg.norm((a - ref).ravel()) / (den if den > 0 else 1.0)) ** 2)"),
    ("den = np.linalg.norm(ref.ravel())", "den = np.linalg.norm(a.ravel())"),
    ("return float(np.linalg.norm((a - ref).ravel()) / (den if den > 0 else 1.0))",
     "return float(np.sum(np.abs(a - ref)) / (den if den > 0 else 1.0))"),
    # max_rel_err: normalised by the largest reference magnitude, or by the norm
    ("rms = np.sqrt(np.mean(np.abs(ref) ** 2)) if ref.size else 1.0",
     "rms = np.max(np.abs(ref)) if ref.size else 1.0"),
    ("rms = np.sqrt(np.mean(np.abs(ref) ** 2)) if ref.size else 1.0",
     "rms = np.linalg.norm(ref.ravel()) if ref.size else 1.0"),
    # worst_slice_err: pooled over the wrong axis; mean over slices instead of the worst
    ("other = tuple(i for i in range(ref.ndim) if i != axis % ref.ndim)",
     "other = tuple(i for i in range(ref.ndim) if i == axis % ref.ndim)"),
    ("return float(np.max(per) / (rms if rms > 0 else 1.0))",
     "return float(np.mean(per) / (rms if rms > 0 else 1.0))"),
    # evm_db: 20 log10 of a power ratio; normalised by the estimate's power
    ("return float(10.0 * np.log10(np.sum(np.abs(x_hat - x) ** 2) / np.sum(np.abs(x) ** 2)))",
     "return float(20.0 * np.log10(np.sum(np.abs(x_hat - x) ** 2) / np.sum(np.abs(x) ** 2)))"),
    ("return float(10.0 * np.log10(np.sum(np.abs(x_hat - x) ** 2) / np.sum(np.abs(x) ** 2)))",
     "return float(10.0 * np.log10(np.sum(np.abs(x_hat - x) ** 2) / np.sum(np.abs(x_hat) ** 2)))"),
    # hard_decide: farthest point; highest index wins a tie
    ("idx = np.argmin(d, axis=-1)", "idx = np.argmax(d, axis=-1)"),
    ("idx = np.argmin(d, axis=-1)", "idx = d.shape[-1] - 1 - np.argmin(d[..., ::-1], axis=-1)"),
    # decision_margin: reversed order; plain distances; gap to the farthest point
    ("return d[..., 1] - d[..., 0]", "return d[..., 0] - d[..., 1]"),
    ("d = np.sort(np.abs(x_hat[..., None] - np.asarray(points)[None, :]) ** 2, axis=-1)",
     "d = np.sort(np.abs(x_hat[..., None] - np.asarray(points)[None, :]), axis=-1)"),
    ("return d[..., 1] - d[..., 0]", "return d[..., -1] - d[..., 0]"),
    # xhat_errors: the subcarrier figure taken over the UE axis
    ('"worst_sc": worst_slice_err(a, ref, sc_axis)}', '"worst_sc": worst_slice_err(a, ref, -1)}'),
]


@pytest.mark.parametrize("old,new", METRIC_MUTATIONS)
def test_planted_metric_mistake_is_caught(old, new):
    assert not _metric_pins_pass(_metric_mutant(old, new))
