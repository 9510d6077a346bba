"""Pins of the denoiser oracle (oracle/denoiser_oracle.py) against what the
mathematics fixes: a hand-worked convolution and post-MMSE residual
(tests/golden/conv3x3_small.txt), delta responses, an independent library
correlation (scipy.signal.correlate2d), finite differences of the loss for the
backward pass, bfloat16 rounding of known values, exact LS interpolation of a
channel linear in frequency.  Planted mistakes
in a copy of the oracle must fail these pins.
"""
import math
import types

import numpy as np
import pytest
from scipy import signal

from oracle import denoiser_oracle as DN
from oracle import pusch_oracle as O

RNG = np.random.default_rng(77)


def _params(rng, scale=1.0):
    layers = []
    for (ws, bs), (ci, co, _) in zip(DN.param_shapes(), DN.LAYERS):
        layers.append((rng.standard_normal(ws) * scale * math.sqrt(2.0 / (9 * ci)), rng.standard_normal(bs) * 0.1))
    return DN.pack(layers)


def _fd_check(mod, rng, idx, S=3, K=5, bf16=False):
    """Largest relative gap between backward() and central differences of the MSE loss."""
    p = _params(rng)
    grid = rng.standard_normal((S, K)) + 1j * rng.standard_normal((S, K))
    target = rng.standard_normal((S, K)) + 1j * rng.standard_normal((S, K))
    out, cache = mod.forward(grid, p)
    _, dout = mod.mse_loss(out, target)
    g = mod.backward(cache, dout)
    worst = 0.0
    for i in idx:
        e = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += e
        pm[i] -= e
        fp = mod.mse_loss(mod.forward(grid, pp)[0], target)[0]
        fm = mod.mse_loss(mod.forward(grid, pm)[0], target)[0]
        fd = (fp - fm) / (2 * e)
        worst = max(worst, abs(fd - g[i]) / max(abs(fd), 1e-3))
    return worst


def _sample_idx(rng):
    """Parameters to difference: samples of every layer's weights, every last-layer and first-layer bias."""
    idx, o = [], 0
    for ws, bs in DN.param_shapes():
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        idx += list(o + rng.choice(nw, 12, replace=False))
        idx += list(o + nw + np.arange(min(nb, 4)))
        o += nw + nb
    return idx


def _pins_pass(mod, golden) -> bool:
    try:
        g = golden("conv3x3_small.txt")
        x = np.array(g["x"], float)[..., None]
        W = np.array(g["W"], float)[None, :, :, None]
        assert np.array_equal(mod.conv3x3(x, W)[..., 0], np.array(g["out"], float))
        # delta responses: the forward correlation flips the kernel, its transpose does not
        d = np.zeros((3, 3, 1))
        d[1, 1, 0] = 1.0
        assert np.array_equal(mod.conv3x3(d, W)[..., 0], W[0, ::-1, ::-1, 0])
        assert np.array_equal(mod.conv3x3_transposed(d, W)[..., 0], W[0, :, :, 0])
        # multi-channel forward against scipy's 2-D correlation, channel pair by channel pair
        rng = np.random.default_rng(5)
        xs = rng.standard_normal((4, 7, 3))
        Ws = rng.standard_normal((2, 3, 3, 3))
        bs = rng.standard_normal(2)
        ref = np.stack([bs[o] + sum(signal.correlate2d(xs[..., i], Ws[o, :, :, i], mode="same") for i in range(3))
                        for o in range(2)], axis=-1)
        assert np.allclose(mod.conv3x3(xs, Ws, bs), ref, atol=1e-12)
        # transposed conv is the adjoint: <conv(x), y> = <x, conv_T(y)>
        ys = rng.standard_normal((4, 7, 2))
        assert abs(np.sum(mod.conv3x3(xs, Ws) * ys) - np.sum(xs * mod.conv3x3_transposed(ys, Ws))) < 1e-10
        # backward against finite differences of the MSE loss (FP64)
        assert _fd_check(mod, np.random.default_rng(11), _sample_idx(np.random.default_rng(12))) < 1e-5
        # in units of sigma: sigma * DN(grid / sigma)
        pr = _params(np.random.default_rng(21))
        gr = rng.standard_normal((3, 5)) + 1j * rng.standard_normal((3, 5))
        assert np.allclose(mod.forward(gr, pr, sigma=0.25)[0], 0.25 * mod.forward(gr / 0.25, pr)[0], atol=1e-12)
        assert not np.allclose(mod.forward(gr, pr, sigma=0.25)[0], mod.forward(gr, pr)[0])
        # zero network: the output is the LS grid, and the first three layers get no gradient
        z = np.zeros(mod.n_params())
        grid = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
        out, cache = mod.forward(grid, z)
        assert np.array_equal(out, grid)
        # post-MMSE residual worked by hand: pilot symbol 0, data symbol 1
        H = np.zeros((2, 2, 1, 1), complex)
        H[1, :, 0, 0] = g["res_h"]
        Y = np.zeros((2, 1, 2), complex)
        Y[1, 0] = g["res_y"]
        _, _, r = mod.detect_and_residual(Y, H, (0,), 1.0)
        assert abs(r - g["res_total"]) < 1e-12
        # each data symbol is equalised with its own estimate: a different channel on symbol 2
        H3 = np.concatenate([H, H[1:] * 0.5j], axis=0)
        Y3 = np.concatenate([Y, Y[1:] * 0.5j], axis=1 - 1)
        x3, _, r3 = mod.detect_and_residual(Y3, H3, (0,), 0.0)
        assert np.allclose(x3[1], x3[0]) and r3 < 1e-24
        # the weighted loss: weight 2 on the first grid, 0 on the second
        o = np.array([[[1 + 1j]], [[5.0]]])
        t = np.array([[[0.0]], [[0.0]]])
        lv, dv = mod.mse_loss(o, t, [2.0, 0.0])
        assert abs(lv - 2.0 * 2.0 / 2) < 1e-15 and np.allclose(dv, [[[2 * 2 * (1 + 1j) / 2]], [[0.0]]])
        return True
    except Exception:  # a wrong result, or a mutant that no longer runs
        return False


def test_pins_pass(golden):
    assert _pins_pass(DN, golden)


def test_param_count_and_layout():
    # 2->32, 32->32, 32->32, 32->2 with 3x3 kernels and biases
    assert DN.n_params() == (2 * 32 * 9 + 32) + 2 * (32 * 32 * 9 + 32) + (32 * 2 * 9 + 2) == 19682
    p = np.arange(DN.n_params(), dtype=float)
    layers = DN.unpack(p)
    assert layers[0][0][0, 0, 0, 1] == 1.0 and layers[0][1][0] == 576.0  # W1 c_in fastest, then b1
    assert np.array_equal(DN.pack(layers), p)


def test_bf16_rounding_known_values():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -9, -(1 + 2 ** -7), 3.0, 0.0, 2 ** -130])
    got = DN.to_bf16(v)
    # 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 is a tie -> even (1 + 2^-6); 1 + 2^-7 is representable
    assert got.tolist() == [1.0, 1.0, 1 + 2 ** -6, 1.0, -(1 + 2 ** -7), 3.0, 0.0, got[-1]]
    r = RNG.standard_normal(10000) * 10.0 ** RNG.uniform(-20, 20, 10000)
    assert np.max(np.abs(DN.to_bf16(r) - r) / np.abs(r)) <= 2 ** -8  # half an ulp of 8 significant bits


def test_bf16_forward_backward_are_close_to_fp64():
    rng = np.random.default_rng(3)
    p = _params(rng)
    grid = rng.standard_normal((14, 32)) + 1j * rng.standard_normal((14, 32))
    o64, c64 = DN.forward(grid, p)
    o16, c16 = DN.forward(grid, p, bf16=True)
    assert not np.array_equal(o64, o16)
    # the network's correction: about 2^-8 relative rounding per stored value, four layers
    assert np.linalg.norm(o16 - o64) / np.linalg.norm(o64 - grid) < 2e-2
    d = rng.standard_normal(grid.shape) + 1j * rng.standard_normal(grid.shape)
    g64, g16 = DN.backward(c64, d), DN.backward(c16, d)
    # the last layer's weight gradient sees only rounded activations: same order
    last = DN.n_params() - 578
    assert np.linalg.norm(g16[last:] - g64[last:]) / np.linalg.norm(g64[last:]) < 2e-2
    # earlier layers also see ReLU masks that differ where a pre-activation is within the rounding
    # of zero (about 0.3 % of them here), each an O(1) change of one gradient term: about
    # sqrt(0.003) ~ 6 % of the gradient
    assert np.linalg.norm(g16 - g64) / np.linalg.norm(g64) < 0.2


def test_ls_grid_is_exact_for_a_channel_linear_in_frequency():
    rng = np.random.default_rng(0)
    K, n_ue, n_beams = 40, 4, 3
    a = rng.standard_normal((n_beams, n_ue)) + 1j * rng.standard_normal((n_beams, n_ue))
    c = rng.standard_normal((n_beams, n_ue)) + 1j * rng.standard_normal((n_beams, n_ue))
    Hk = a[None] + np.arange(K)[:, None, None] * c[None] * 0.05  # [K, N_B, N_L]
    p = np.exp(0.5j * np.pi * rng.integers(0, 4, (1, K)))
    own = O.pilot_owner(K, 0, n_ue, 1)
    Yp = (Hk[np.arange(K), :, own] * p[0][:, None]).T[None]  # [1, N_B, K]
    H = DN.ls_grid(Yp, p, n_ue, (2,), 5)
    assert H.shape == (5, K, n_beams, n_ue)
    for l in range(n_ue):
        ks = np.nonzero(own == l)[0]
        inside = np.arange(ks[0], ks[-1] + 1)
        for s in range(5):  # one pilot symbol: the same estimate on every symbol
            assert np.allclose(H[s, inside, :, l], Hk[inside, :, l], atol=1e-12)
        assert np.allclose(H[0, :ks[0], :, l], Hk[ks[0], :, l], atol=1e-12)  # held below the first position


def test_ls_grid_matches_the_chain_estimator():
    rng = np.random.default_rng(8)
    K, n_ue, n_beams = 30, 3, 2
    Yp = rng.standard_normal((2, n_beams, K)) + 1j * rng.standard_normal((2, n_beams, K))
    p = np.exp(0.5j * np.pi * rng.integers(0, 4, (2, K)))
    H = DN.ls_grid(Yp, p, n_ue, (2, 11), 14)
    for s in (0, 5, 13):
        assert np.allclose(H[s], O.time_interpolated_estimate(Yp, p, n_ue, (2, 11), s), atol=1e-12)


def test_residual_is_the_noise_for_the_true_channel_and_grows_with_the_error():
    # with the true channel and noiseless data the residual is the regularisation's share only
    rng = np.random.default_rng(9)
    S, K, nb, nl = 4, 50, 8, 3
    H = rng.standard_normal((S, K, nb, nl)) + 1j * rng.standard_normal((S, K, nb, nl))
    x = np.exp(0.5j * np.pi * rng.integers(0, 4, (S, K, nl)))
    Y = np.einsum("skbl,skl->sbk", H, x)
    _, _, r0 = DN.detect_and_residual(Y, H, (0,), 0.0)
    assert r0 < 1e-18
    noisy = H + 0.1 * (rng.standard_normal(H.shape) + 1j * rng.standard_normal(H.shape))
    _, _, r1 = DN.detect_and_residual(Y, noisy, (0,), 0.0)
    worse = H + 0.3 * (rng.standard_normal(H.shape) + 1j * rng.standard_normal(H.shape))
    _, _, r2 = DN.detect_and_residual(Y, worse, (0,), 0.0)
    assert 0 < r1 < r2


def test_adam_first_steps_closed_form():
    # with m = v = 0 the first bias-corrected step is lr g / (|g| + eps); a constant gradient keeps
    # the bias-corrected moments at g and g^2, so every later step is the same
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = v = np.zeros(3)
    for step in (1, 2, 3):
        p2, m, v = DN.adam_step(p, g, m, v, step, 0.01)
        assert np.allclose(p2 - p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        p = p2
    # a sign flip after one step: m2 = 0.9 (0.1 g) - 0.1 g = -0.01 g over 1 - 0.81 = 0.19
    p0 = np.zeros(1)
    p1, m1, v1 = DN.adam_step(p0, np.array([1.0]), np.zeros(1), np.zeros(1), 1, 1.0, eps=0.0)
    p2, _, _ = DN.adam_step(p1, np.array([-1.0]), m1, v1, 2, 1.0, eps=0.0)
    assert np.allclose(p2 - p1, -(-0.01 / 0.19) / np.sqrt((0.999 * 0.001 + 0.001) / (1 - 0.999 ** 2)), rtol=1e-12)


def test_denoised_chain_with_a_zero_network_is_the_ls_chain():
    from paper_2210_09196_amd import synth
    cfg = synth.CFG1.replace(n_fft=64, n_sc=64, n_ant=8, n_beams=8)
    b = synth.make_batch(cfg, [3])
    r = DN.receive_slot_denoised(b["x_td"][0], b["pilots"][0], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                                 np.zeros(DN.n_params()), cfg.n_beams)
    ref = O.receive_slot(b["x_td"][0], b["pilots"][0], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                         n_beams=cfg.n_beams)
    assert r["used_dn"] and r["res_dn"] == r["res_ls"]
    assert np.allclose(r["x_hat"], ref["x_hat"], atol=1e-12)


def _mutant(old: str, new: str) -> types.ModuleType:
    src = open(DN.__file__).read()
    assert src.count(old) >= 1, old
    mod = types.ModuleType("denoiser_mutant")
    mod.__dict__["__file__"] = DN.__file__
    exec(compile(src.replace(old, new, 1), "denoiser_mutant", "exec"), mod.__dict__)
    return mod


MUTATIONS = [
    # convolution instead of correlation (flipped kernel)
    ('out += np.einsum("ski,oi->sko", xp[dy:dy + S, dx:dx + K], W[:, dy, dx, :])',
     'out += np.einsum("ski,oi->sko", xp[dy:dy + S, dx:dx + K], W[:, 2 - dy, 2 - dx, :])'),
    # wrap-around instead of zero padding
    ("    xp[1:-1, 1:-1] = x\n    out = np.zeros((S, K, W.shape[0]))",
     "    xp = np.pad(x, ((1, 1), (1, 1), (0, 0)), mode='wrap')\n    out = np.zeros((S, K, W.shape[0]))"),
    # transposed conv with the forward's offsets
    ('out += np.einsum("sko,oi->ski", gp[2 - dy:2 - dy + S, 2 - dx:2 - dx + K], W[:, dy, dx, :])',
     'out += np.einsum("sko,oi->ski", gp[dy:dy + S, dx:dx + K], W[:, dy, dx, :])'),
    # ReLU derivative dropped
    ("g = da * (acts[n] > 0)", "g = da"),
    # weight gradient against the wrong layer input
    ("grads[n] = conv3x3_weight_grad(g, acts[n])", "grads[n] = conv3x3_weight_grad(g, acts[max(n - 1, 0)])"),
    # bias gradient lost
    ("return dW, g.sum(axis=(0, 1))", "return dW, 0.0 * g.sum(axis=(0, 1))"),
    # loss gradient without the factor 2
    ("return float(np.sum(w * (e.real ** 2 + e.imag ** 2)) / n), 2.0 * w * e / n",
     "return float(np.sum(w * (e.real ** 2 + e.imag ** 2)) / n), w * e / n"),
    # no residual connection
    ("out = grid + sigma * (a[..., 0] + 1j * a[..., 1])", "out = sigma * (a[..., 0] + 1j * a[..., 1])"),
    # the correction not scaled back to the grid's units
    ("out = grid + sigma * (a[..., 0] + 1j * a[..., 1])", "out = grid + (a[..., 0] + 1j * a[..., 1])"),
    # weight-gradient offsets transposed
    ('dW[:, dy, dx, :] = np.einsum("sko,ski->oi", g, xp[dy:dy + S, dx:dx + K])',
     'dW[:, dx % 3, dy, :] = np.einsum("sko,ski->oi", g, xp[dy:dy + S, dx:dx + K])'),
    # residual: plus instead of minus; the estimate of the wrong symbol
    ('r = Y[s].T - np.einsum("kbl,kl->kb", H_grid[s], xs[0])', 'r = Y[s].T + np.einsum("kbl,kl->kb", H_grid[s], xs[0])'),
    ("xs, ok[d] = O.mmse_detect(H_grid[s], Y[s].T[None], sigma2)",
     "xs, ok[d] = O.mmse_detect(H_grid[data[0]], Y[s].T[None], sigma2)"),
    # loss weights ignored
    ("w = w.reshape((-1,) + (1,) * (e.ndim - 1))", "w = np.ones_like(w).reshape((-1,) + (1,) * (e.ndim - 1))"),
]


def test_pins_pass_on_the_oracle(golden):
    assert _pins_pass(DN, golden)


@pytest.mark.parametrize("old,new", MUTATIONS)
def test_planted_mistake_is_caught(old, new, golden):
    assert not _pins_pass(_mutant(old, new), golden)
