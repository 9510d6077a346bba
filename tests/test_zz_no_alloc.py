"""pusch_noise_est_static -- the allocation-free variant of pusch_noise_est,
whose scratch is a device array inside the library -- against the workspace
entry point pusch_noise_est on the same inputs, through the C ABI.

Both run the same kernels with the same slices and a fixed-order reduction,
so the estimates must be bit-identical; both are also scored against the FP64
oracle (relative 2e-5: the stand-alone tolerance of the NE step on exact FP32
inputs).  Two calls in a row, the second with a smaller input (fewer items,
a smaller geometry), check that what the first call left in the shared
scratch does not leak into the second.
"""
import numpy as np
import pytest
import torch

from oracle import pusch_oracle as O
from paper_2210_09196_amd import pusch

pytestmark = pytest.mark.gpu

DEV = "cuda"
TOL_NE = 2e-5


def pilot_inputs(rng, batch, n_pilot, n_sc, n_beams, n_ue, sigma2):
    """Pilot symbols [batch, n_pilot, n_sc, n_beams] through a channel varying smoothly along k, plus noise."""
    k = np.arange(n_sc)
    Y = np.zeros((batch, n_pilot, n_sc, n_beams), complex)
    p = rng.uniform(0.5, 2.0, (batch, n_pilot, n_sc)) * np.exp(2j * np.pi * rng.uniform(size=(batch, n_pilot, n_sc)))
    for b in range(batch):
        a = rng.standard_normal((n_ue, n_beams)) + 1j * rng.standard_normal((n_ue, n_beams))
        c = rng.standard_normal((n_ue, n_beams)) + 1j * rng.standard_normal((n_ue, n_beams))
        for j in range(n_pilot):
            own = (k + j * (n_ue // n_pilot)) % n_ue
            Y[b, j] = (a[own] + np.exp(2j * np.pi * k / 97.0)[:, None] * c[own] * 0.3) * p[b, j][:, None]
    Y += (rng.standard_normal(Y.shape) + 1j * rng.standard_normal(Y.shape)) * np.sqrt(sigma2 / 2)
    return Y.astype(np.complex64), p.astype(np.complex64)


def test_static_noise_estimate_matches_the_workspace_entry_point():
    calls = [(24, 2, 3300, 32, 16, 0.02), (3, 1, 256, 16, 4, 0.1)]  # the second call is smaller
    for n, (batch, n_pilot, n_sc, n_beams, n_ue, s2) in enumerate(calls):
        print(f"[no-alloc] call {n}: batch {batch}, {n_pilot} pilot symbols, {n_sc} sc, {n_beams} beams, "
              f"{n_ue} UEs", flush=True)
        Y, p = pilot_inputs(np.random.default_rng(40 + n), batch, n_pilot, n_sc, n_beams, n_ue, s2)
        Yd, pd = torch.from_numpy(Y).to(DEV), torch.from_numpy(p).to(DEV)
        got = pusch.noise_est_static(Yd, pd, n_ue)
        ref = pusch.noise_est(Yd, pd, n_ue)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (got, ref)
        got = got.cpu().numpy()
        for b in range(batch):
            o = O.noise_variance_estimate(np.swapaxes(Y[b], 1, 2), p[b], n_ue)
            assert abs(got[b] - o) <= TOL_NE * o, (n, b, got[b], o)


def test_static_noise_estimate_limits():
    Y, p = pilot_inputs(np.random.default_rng(7), 2, 2, 64, 4, 2, 0.1)
    Yd, pd = torch.from_numpy(Y).to(DEV), torch.from_numpy(p).to(DEV)
    # the largest batch the scratch holds, then one more (rejected before any launch)
    big_Y = Yd[:1].expand(pusch.NOISE_EST_STATIC_MAX_BATCH, -1, -1, -1).contiguous()
    big_p = pd[:1].expand(pusch.NOISE_EST_STATIC_MAX_BATCH, -1, -1).contiguous()
    got = pusch.noise_est_static(big_Y, big_p, 2)
    torch.cuda.synchronize()
    assert torch.all(got == pusch.noise_est(Yd[:1], pd[:1], 2)[0]).item()
    over_Y = torch.cat([big_Y, Yd[:1]])
    over_p = torch.cat([big_p, pd[:1]])
    with pytest.raises(pusch.PuschError, match="at most"):
        pusch.noise_est_static(over_Y, over_p, 2)
    rc = pusch.lib().pusch_noise_est_static(over_Y.data_ptr(), over_p.data_ptr(), got.data_ptr(), 4, 2, 64, 2,
                                            pusch.NOISE_EST_STATIC_MAX_BATCH + 1, pusch._stream())
    assert rc == -2  # PUSCH_EUNSUPPORTED
    torch.cuda.synchronize()
