"""Pins of the denoiser oracle (oracle/denoiser_oracle.py) against what the
mathematics fixes: a hand-worked convolution and holdout residual
(tests/golden/conv3x3_small.txt), delta responses, an independent library
correlation (scipy.signal.correlate2d), finite differences of the loss for the
backward pass, bfloat16 rounding of known values, exact LS interpolation of a
channel linear in frequency from either half of the comb.  Planted mistakes
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
        # zero network: the output is the LS grid, and the first three layers get no gradient
        z = np.zeros(mod.n_params())
        grid = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
        out, cache = mod.forward(grid, z)
        assert np.array_equal(out, grid)
        # holdout residual worked by hand
        y = np.array(g["res_y"], complex)
        est = lambda fold: mod.ls_grid(y[None, None], np.ones((1, 4)), 1, (0,), 1, fold)
        r = mod.pilot_holdout_residual(y[None, None], np.ones((1, 4)), 1, (0,), 1, 0.0, est)
        assert abs(r - g["res_total"]) < 1e-12
        # two pilot symbols, a channel that is constant in frequency but different on each: the
        # held-out REs of pilot symbol j must be equalised with symbol pilot_symb[j]'s estimate
        K2, nb2 = 16, 2
        A = np.array([[1.0 + 0.5j, -0.3j], [0.2, 1.1 - 0.4j]])  # [N_B, N_L] on pilot symbol 2
        B = np.array([[0.4 - 1.0j, 0.9], [1.3j, -0.6 + 0.2j]])  # on pilot symbol 11
        p2 = np.exp(0.5j * np.pi * np.random.default_rng(4).integers(0, 4, (2, K2)))
        Y2 = np.zeros((2, nb2, K2), complex)
        for j, Hj in enumerate((A, B)):
            own = O.pilot_owner(K2, j, 2, 2)
            Y2[j] = Hj[:, own] * p2[j]
        est2 = lambda fold: mod.ls_grid(Y2, p2, 2, (2, 11), 14, fold)
        assert mod.pilot_holdout_residual(Y2, p2, 2, (2, 11), 14, 0.0, est2) < 1e-18
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


@pytest.mark.parametrize("fold", [0, 1, 2])
def test_fold_ls_is_exact_for_a_channel_linear_in_frequency(fold):
    rng = np.random.default_rng(fold)
    K, n_ue, n_beams = 40, 4, 3
    a = rng.standard_normal((n_beams, n_ue)) + 1j * rng.standard_normal((n_beams, n_ue))
    c = rng.standard_normal((n_beams, n_ue)) + 1j * rng.standard_normal((n_beams, n_ue))
    Hk = a[None] + np.arange(K)[:, None, None] * c[None] * 0.05  # [K, N_B, N_L]
    p = np.exp(0.5j * np.pi * rng.integers(0, 4, (1, K)))
    own = O.pilot_owner(K, 0, n_ue, 1)
    Yp = (Hk[np.arange(K), :, own] * p[0][:, None]).T[None]  # [1, N_B, K]
    H = DN.ls_grid(Yp, p, n_ue, (2,), 5, fold)
    assert H.shape == (5, K, n_beams, n_ue)
    for l in range(n_ue):
        ks = np.nonzero(own == l)[0]
        ks = ks if fold == 0 else ks[fold - 1::2]
        inside = np.arange(ks[0], ks[-1] + 1)
        for s in range(5):  # one pilot symbol: the same estimate on every symbol
            assert np.allclose(H[s, inside, :, l], Hk[inside, :, l], atol=1e-12)
        assert np.allclose(H[0, :ks[0], :, l], Hk[ks[0], :, l], atol=1e-12)  # held below the first position


def test_fold_zero_matches_the_chain_estimator():
    rng = np.random.default_rng(8)
    K, n_ue, n_beams = 30, 3, 2
    Yp = rng.standard_normal((2, n_beams, K)) + 1j * rng.standard_normal((2, n_beams, K))
    p = np.exp(0.5j * np.pi * rng.integers(0, 4, (2, K)))
    H = DN.ls_grid(Yp, p, n_ue, (2, 11), 14, 0)
    for s in (0, 5, 13):
        assert np.allclose(H[s], O.time_interpolated_estimate(Yp, p, n_ue, (2, 11), s), atol=1e-12)


def test_holdout_residual_noiseless_linear_channel_is_zero():
    rng = np.random.default_rng(9)
    K, n_ue, n_beams = 64, 4, 8
    a = rng.standard_normal((n_beams, n_ue)) + 1j * rng.standard_normal((n_beams, n_ue))
    c = rng.standard_normal((n_beams, n_ue)) + 1j * rng.standard_normal((n_beams, n_ue))
    Hk = a[None] + np.arange(K)[:, None, None] * c[None] * 0.02
    p = np.exp(0.5j * np.pi * rng.integers(0, 4, (1, K)))
    own = O.pilot_owner(K, 0, n_ue, 1)
    Yp = (Hk[np.arange(K), :, own] * p[0][:, None]).T[None]
    est = lambda fold: DN.ls_grid(Yp, p, n_ue, (2,), 14, fold)
    # held-out positions past a fold's last position see a held (not linear) value: keep the
    # comparison inside, by making the channel constant there
    r = DN.pilot_holdout_residual(Yp, p, n_ue, (2,), 14, 1e-12, est)
    assert r < 0.5  # only the end holds miss
    Hc = np.repeat(a[None], K, axis=0)
    Yc = (Hc[np.arange(K), :, own] * p[0][:, None]).T[None]
    estc = lambda fold: DN.ls_grid(Yc, p, n_ue, (2,), 14, fold)
    assert DN.pilot_holdout_residual(Yc, p, n_ue, (2,), 14, 0.0, estc) < 1e-18


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
    ("return float(np.sum(e.real ** 2 + e.imag ** 2) / n), 2.0 * e / n", "return float(np.sum(e.real ** 2 + e.imag ** 2) / n), e / n"),
    # no residual connection
    ("out = grid + (a[..., 0] + 1j * a[..., 1])", "out = a[..., 0] + 1j * a[..., 1]"),
    # weight-gradient offsets transposed
    ('dW[:, dy, dx, :] = np.einsum("sko,ski->oi", g, xp[dy:dy + S, dx:dx + K])',
     'dW[:, dx % 3, dy, :] = np.einsum("sko,ski->oi", g, xp[dy:dy + S, dx:dx + K])'),
    # folds: the same half twice
    ("return ks if fold == 0 else ks[fold - 1::2]", "return ks if fold == 0 else ks[0::2]"),
    # residual: held-out REs equalised with the estimate of the wrong symbol
    ("Hk = H[pilot_symb[j]][ks]", "Hk = H[0][ks]"),
]


def test_pins_pass_on_the_oracle(golden):
    assert _pins_pass(DN, golden)


@pytest.mark.parametrize("old,new", MUTATIONS)
def test_planted_mistake_is_caught(old, new, golden):
    assert not _pins_pass(_mutant(old, new), golden)
