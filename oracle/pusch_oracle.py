"""FP64 CPU oracle of the PUSCH lower-PHY receive chain.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the package
entry file and the CPU-baseline leg of the benchmark may import this module.
The HIP product path never calls it, and this module shares no code, tables
or helpers with the HIP library (it does not import the package).

Everything is computed in complex128 from the plain definitions, in the order
the paper gives the chain (Sec. II, Fig. "PUSCH processing chain"): OFDM
demodulation (FFT per antenna and symbol), beamforming (matrix product with
known coefficients), least-squares channel estimation on the pilot symbols,
then the MIMO stage of Eq. 2 solved through a Cholesky decomposition of the
Gram matrix followed by two triangular solves.

Readings of points the paper leaves open (each also stated where used):
  R1  forward FFT e^{-2 pi i f n / N}, unscaled, natural output order;
  R3  active subcarrier k <-> FFT bin (k - N_act//2) mod N;
  R4  default beamformer = first N_B rows of the unitary N_R-point DFT;
  R5  pilots of the N_L UEs form a comb: pilot symbol j, subcarrier k belongs
      to UE (k + o_j) mod N_L with o_j = j * (N_L // N_pilot) (staggered), or
      o_j = 0 for every j when the call asks for an aligned comb (every pilot
      symbol then puts each UE's pilots on the same subcarriers);
  R6  the channel is static over the slot: all pilot symbols are merged into
      one estimate and the Cholesky factor is computed once per subcarrier and
      reused for every data symbol;
  R12 a non-positive or non-finite Cholesky pivot flags the subcarrier
      (status 1) and its detected symbols are set to 0;
  R17 noise estimation compares each pilot RE with the prediction from the
      UE's channel interpolated from its other pilot positions (leave one
      out), normalised by the exact noise gain of that prediction;
  R21 ... except at a position where c >= 2 pilot symbols carry the UE's
      pilot: there each of those REs is compared with its pilot times the
      mean of the c LS values at that same subcarrier, with noise gain
      1 - 2/c + |p_j|^2 / c^2 sum_s 1/|p_s|^2.  The channel is the same in
      every term, so this residual holds noise only, whatever the channel's
      frequency selectivity (for a channel static over the slot, R6);
  R18 for a channel that varies over the slot, each pilot symbol gives its own
      estimate (its own comb positions only), and data symbol s uses the
      linear interpolation in s between the two pilot symbols around it
      (held before the first and after the last); the MIMO stage then
      factors one Gram matrix per data symbol, as the paper counts it.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "active_bins",
    "ofdm_demodulate",
    "dft_beamformer",
    "beamform",
    "pilot_owner",
    "ls_channel_estimate",
    "time_interpolated_estimate",
    "noise_variance_estimate",
    "gram",
    "cholesky_crout",
    "forward_substitution",
    "back_substitution",
    "mmse_detect",
    "receive_slot",
]


def active_bins(n_fft: int, n_sc: int) -> np.ndarray:
    """FFT bin of each active subcarrier, centred band with DC used (reading R3)."""
    return (np.arange(n_sc) - n_sc // 2) % n_fft


def ofdm_demodulate(x_td, n_sc: int | None = None) -> np.ndarray:
    """OFDM demodulation (Sec. II; Table 1, row "OFDM dem."): one N-point FFT
    per antenna and OFDM symbol, X[f] = sum_n x[n] e^{-2 pi i f n / N}
    (reading R1).  With n_sc given, the n_sc active bins follow in subcarrier
    order (reading R3; for n_sc == N this is the centred reordering of all
    bins); with n_sc None the N bins are returned in natural order.

    x_td: [..., N] time-domain samples.  Returns [..., n_sc or N] complex128.
    """
    x = np.asarray(x_td, dtype=np.complex128)
    X = np.fft.fft(x, axis=-1)
    if n_sc is None:
        return X
    return X[..., active_bins(x.shape[-1], n_sc)]


def dft_beamformer(n_beams: int, n_ant: int) -> np.ndarray:
    """Beamforming coefficients (Sec. II: "known coefficients", reading R4):
    W[b, r] = e^{-2 pi i b r / N_R} / sqrt(N_R), b < N_B.  Rows are orthonormal."""
    b = np.arange(n_beams)[:, None]
    r = np.arange(n_ant)[None, :]
    return np.exp(-2j * np.pi * ((b * r) % n_ant) / n_ant) / np.sqrt(n_ant)


def beamform(W, Xa) -> np.ndarray:
    """Beamforming (Sec. II; Table 1, row "BF"): N_B beams as linear
    combinations of the N_R antennas on every subcarrier of every symbol,
    Y[..., b, k] = sum_r W[b, r] Xa[..., r, k].

    W: [N_B, N_R]; Xa: [..., N_R, K].  Returns [..., N_B, K]."""
    return np.matmul(np.asarray(W, np.complex128), np.asarray(Xa, np.complex128))


def pilot_owner(n_sc: int, j: int, n_ue: int, n_pilot: int, aligned: bool = False) -> np.ndarray:
    """UE owning each subcarrier of pilot symbol j (reading R5; aligned: o_j = 0)."""
    return (np.arange(n_sc) + (0 if aligned else j * (n_ue // n_pilot))) % n_ue


def ls_channel_estimate(Yp, pilots, n_ue: int, use=None, aligned: bool = False) -> np.ndarray:
    """Least-squares channel estimation on block-type pilot symbols (Sec. II,
    CHE; Table 1, row "CHE": an element-wise division per beam and UE).

    On pilot symbol j, subcarrier k (owned by UE l, reading R5) the LS estimate
    of UE l's beam-domain channel is Y_j[:, k] * conj(p_j[k]) / |p_j[k]|^2.
    Per UE, the estimates of all pilot symbols are merged by position
    (duplicates at one subcarrier are averaged, reading R6) and linearly
    interpolated along the subcarriers, holding the end values beyond the
    first and last pilot position.

    Yp: [N_p, N_B, K] beam-domain pilot symbols; pilots: [N_p, K]; use: the
    pilot symbols (indices j) to take, all by default; aligned: the comb of R5
    without stagger.
    Returns H_hat [K, N_B, N_L] (one N_B x N_L matrix per subcarrier, Eq. 1).
    """
    Yp = np.asarray(Yp, np.complex128)
    pilots = np.asarray(pilots, np.complex128)
    n_pilot, n_beams, K = Yp.shape
    use = range(n_pilot) if use is None else list(use)
    if K < n_ue:
        raise ValueError("every UE needs at least one pilot subcarrier")
    H = np.zeros((K, n_beams, n_ue), dtype=np.complex128)
    grid = np.arange(K, dtype=np.float64)
    for l in range(n_ue):
        pos_list, val_list = [], []
        for j in use:
            ks = np.nonzero(pilot_owner(K, j, n_ue, n_pilot, aligned) == l)[0]
            p = pilots[j, ks]
            pos_list.append(ks)
            val_list.append(Yp[j][:, ks] * (np.conj(p) / (p.real ** 2 + p.imag ** 2)))
        pos = np.concatenate(pos_list)
        val = np.concatenate(val_list, axis=1)  # [N_B, n_positions]
        upos, inv = np.unique(pos, return_inverse=True)
        acc = np.zeros((n_beams, len(upos)), dtype=np.complex128)
        cnt = np.zeros(len(upos))
        np.add.at(cnt, inv, 1.0)
        for b in range(n_beams):
            np.add.at(acc[b], inv, val[b])
        acc /= cnt[None, :]
        x = upos.astype(np.float64)
        for b in range(n_beams):
            H[:, b, l] = np.interp(grid, x, acc[b].real) + 1j * np.interp(grid, x, acc[b].imag)
    return H


def time_interpolated_estimate(Yp, pilots, n_ue: int, pilot_symb, symb, aligned: bool = False) -> np.ndarray:
    """Channel estimate of OFDM symbol `symb` for a channel that changes over
    the slot (reading R18): pilot symbol j alone gives H_j (ls_channel_estimate
    with use=[j]); between the pilot symbols p_a < symb < p_b next to it the
    estimate is ((p_b - symb) H_a + (symb - p_a) H_b) / (p_b - p_a), before the
    first pilot symbol it is H_0 and after the last it is H_{N_p - 1}.

    Yp: [N_p, N_B, K]; pilots: [N_p, K]; pilot_symb: the N_p ascending symbol
    indices.  Returns [K, N_B, N_L].
    """
    ps = list(pilot_symb)
    if symb <= ps[0]:
        return ls_channel_estimate(Yp, pilots, n_ue, use=[0], aligned=aligned)
    if symb >= ps[-1]:
        return ls_channel_estimate(Yp, pilots, n_ue, use=[len(ps) - 1], aligned=aligned)
    b = next(j for j, p in enumerate(ps) if p > symb)
    a = b - 1
    Ha = ls_channel_estimate(Yp, pilots, n_ue, use=[a], aligned=aligned)
    Hb = ls_channel_estimate(Yp, pilots, n_ue, use=[b], aligned=aligned)
    return ((ps[b] - symb) * Ha + (symb - ps[a]) * Hb) / (ps[b] - ps[a])


def noise_variance_estimate(Yp, pilots, n_ue: int, aligned: bool = False) -> float:
    """Noise estimation (Sec. II, NE; Table 1, row "NE"): the noise variance
    from the differences between the received pilot REs and the values that
    the estimated channel and the known pilots predict there (reading R17).

    Pilot RE (j, k) belongs to UE l (reading R5).  Its prediction is
    p_j[k] h(k), where h(k) is UE l's channel interpolated as in
    ls_channel_estimate (merged LS values, linear between the nearest
    positions, end-value hold) but from UE l's pilot positions other than k:
    the nearest one below and the nearest one above, or the nearest one on
    the only side there is.  The interpolation passes through every pilot
    position, so without leaving k out the difference would be zero.
    If h(k) = sum_i w_i m_i, with m_i the mean of c_i LS values at position i
    from pilots p_s, the difference r = Y_j[:, k] - p_j[k] h(k) has noise
    variance sigma^2 * kappa per beam, with
        kappa = 1 + |p_j[k]|^2 sum_i (w_i / c_i)^2 sum_{s at i} 1 / |p_s|^2,
    and the estimate is sum |r|^2 over all pilot REs and beams divided by
    N_B sum kappa: unbiased whenever the channel is linear in k between the
    positions used.  Requires K >= 2 N_L (every UE then has at least two
    pilot positions).

    Where c >= 2 pilot symbols put UE l's pilot at k (reading R21), those REs
    are compared at k itself instead: h(k) is the mean m of their c LS values,
    r = Y_j[:, k] - p_j[k] m, and since m holds 1/c of this RE's own noise,
        kappa = 1 - 2/c + |p_j[k]|^2 / c^2 sum_{s at k} 1 / |p_s|^2
    (the c REs of a position add up to c - 1 for equal pilot powers).  This
    is unbiased for any frequency selectivity.

    Yp: [N_p, N_B, K] beam-domain pilot symbols; pilots: [N_p, K]; aligned:
    the comb of R5 without stagger.
    Returns sigma2_hat (float).
    """
    Yp = np.asarray(Yp, np.complex128)
    pilots = np.asarray(pilots, np.complex128)
    n_pilot, n_beams, K = Yp.shape
    if K < 2 * n_ue:
        raise ValueError("noise estimation needs at least two pilot subcarriers per UE")
    num, den = 0.0, 0.0
    for l in range(n_ue):
        # the pilot REs of UE l, grouped by subcarrier
        at = {}
        for j in range(n_pilot):
            for k in np.nonzero(pilot_owner(K, j, n_ue, n_pilot, aligned) == l)[0]:
                at.setdefault(int(k), []).append(j)
        pos = sorted(at)
        mean, cnt, inv_pow = {}, {}, {}
        for k in pos:
            ls = [Yp[j][:, k] * np.conj(pilots[j, k]) / abs(pilots[j, k]) ** 2 for j in at[k]]
            mean[k] = sum(ls) / len(ls)
            cnt[k] = len(ls)
            inv_pow[k] = sum(1.0 / abs(pilots[j, k]) ** 2 for j in at[k])
        for i, k in enumerate(pos):
            c = cnt[k]
            if c >= 2:  # the same subcarrier on several pilot symbols (R21)
                for j in at[k]:
                    r = Yp[j][:, k] - pilots[j, k] * mean[k]
                    num += float(np.sum(r.real ** 2 + r.imag ** 2))
                    den += n_beams * (1.0 - 2.0 / c + abs(pilots[j, k]) ** 2 / c ** 2 * inv_pow[k])
                continue
            below = pos[i - 1] if i > 0 else None
            above = pos[i + 1] if i + 1 < len(pos) else None
            if below is not None and above is not None:
                weights = {below: (above - k) / (above - below), above: (k - below) / (above - below)}
            else:
                weights = {below if above is None else above: 1.0}
            h = sum(w * mean[m] for m, w in weights.items())
            gain = sum((w / cnt[m]) ** 2 * inv_pow[m] for m, w in weights.items())
            for j in at[k]:
                r = Yp[j][:, k] - pilots[j, k] * h
                num += float(np.sum(r.real ** 2 + r.imag ** 2))
                den += n_beams * (1.0 + abs(pilots[j, k]) ** 2 * gain)
    return num / den


def gram(H, sigma2: float) -> np.ndarray:
    """Regularised Gram matrix of Eq. 2: G = H^H H + sigma^2 I per subcarrier.

    H: [..., N_B, N_L].  Returns [..., N_L, N_L]."""
    H = np.asarray(H, np.complex128)
    G = np.matmul(np.conj(np.swapaxes(H, -1, -2)), H)
    n = H.shape[-1]
    return G + float(sigma2) * np.eye(n)


def cholesky_crout(G) -> tuple[np.ndarray, np.ndarray]:
    """Cholesky decomposition G = L L^H (Sec. II after Eq. 2; Sec. V-C: the
    Cholesky-Crout order, computing L column by column, each new column using
    the already-computed elements of the rows).

    For column j: d = G_jj - sum_{m<j} |L_jm|^2, L_jj = sqrt(d), and for i > j
    L_ij = (G_ij - sum_{m<j} L_im conj(L_jm)) / L_jj.  A pivot d that is not
    positive or not finite marks the matrix as failed (reading R12).

    G: [..., n, n] Hermitian.  Returns (L [..., n, n], ok [...] bool).
    """
    G = np.asarray(G, np.complex128)
    n = G.shape[-1]
    L = np.zeros_like(G)
    ok = np.ones(G.shape[:-2], dtype=bool)
    for j in range(n):
        row_j = L[..., j, :j]
        d = G[..., j, j].real - np.sum(row_j.real ** 2 + row_j.imag ** 2, axis=-1)
        good = (d > 0) & np.isfinite(d)
        ok &= good
        ljj = np.sqrt(np.where(good, d, np.nan))
        L[..., j, j] = ljj
        for i in range(j + 1, n):
            s = G[..., i, j] - np.sum(L[..., i, :j] * np.conj(row_j), axis=-1)
            L[..., i, j] = s / ljj
    return L, ok


def forward_substitution(L, b) -> np.ndarray:
    """Solve L z = b for lower-triangular L (first of the two triangular systems
    that replace the inverse in Eq. 2).  L: [..., n, n]; b: [..., n]."""
    L = np.asarray(L, np.complex128)
    b = np.asarray(b, np.complex128)
    n = L.shape[-1]
    z = np.zeros(np.broadcast_shapes(L.shape[:-1], b.shape), dtype=np.complex128)
    for i in range(n):
        s = b[..., i] - np.sum(L[..., i, :i] * z[..., :i], axis=-1)
        z[..., i] = s / L[..., i, i]
    return z


def back_substitution(L, z) -> np.ndarray:
    """Solve L^H x = z (second triangular system).  L: [..., n, n]; z: [..., n]."""
    L = np.asarray(L, np.complex128)
    z = np.asarray(z, np.complex128)
    n = L.shape[-1]
    x = np.zeros(np.broadcast_shapes(L.shape[:-1], z.shape), dtype=np.complex128)
    for i in range(n - 1, -1, -1):
        # row i of L^H holds conj(L_mi) for m >= i
        s = z[..., i] - np.sum(np.conj(L[..., i + 1:, i]) * x[..., i + 1:], axis=-1)
        x[..., i] = s / np.conj(L[..., i, i])
    return x


def mmse_detect(H, Yd, sigma2: float) -> tuple[np.ndarray, np.ndarray]:
    """MIMO stage, Eq. 2: x = (H^H H + sigma^2 I)^{-1} H^H y, evaluated as the
    paper prescribes: Gram matrix, Cholesky decomposition, matched filter
    b = H^H y, forward substitution L z = b, back substitution L^H x = z.
    One factorisation per subcarrier serves all data symbols (reading R6).

    H: [K, N_B, N_L]; Yd: [D, K, N_B].  Returns (x_hat [D, K, N_L], ok [K]).
    """
    H = np.asarray(H, np.complex128)
    Yd = np.asarray(Yd, np.complex128)
    G = gram(H, sigma2)
    L, ok = cholesky_crout(G)
    b = np.einsum("kbl,dkb->dkl", np.conj(H), Yd)
    z = forward_substitution(L[None], b)
    x = back_substitution(L[None], z)
    x[:, ~ok, :] = 0.0
    return x, ok


def receive_slot(x_td, pilots, pilot_symb, n_ue: int, n_sc: int, sigma2: float | None, W=None,
                 n_beams: int | None = None, time_varying: bool = False, aligned: bool = False) -> dict:
    """The whole receive chain of one slot (Sec. II), in the paper's order.

    x_td: [S, N_R, N] time-domain samples; pilots: [N_p, K]; pilot_symb: the
    0-based pilot symbol indices.  W defaults to the DFT beamformer with
    n_beams rows.  sigma2 None: the noise variance is estimated from the
    pilot symbols (noise_variance_estimate) and used in the MIMO stage.
    time_varying: every data symbol gets its own estimate
    (time_interpolated_estimate) and its own factorisation (reading R18).
    aligned: the pilot comb without stagger (reading R5).
    Returns a dict with the intermediates and the result: X [S, N_R, K],
    Y [S, N_B, K], H [K, N_B, N_L] (the merged static estimate), sigma2,
    x_hat [D, K, N_L], ok [K] (with time_varying: ok for every data symbol).
    """
    x_td = np.asarray(x_td)
    S, n_ant, _ = x_td.shape
    if W is None:
        W = dft_beamformer(n_beams, n_ant)
    X = ofdm_demodulate(x_td, n_sc)
    Y = beamform(W, X)
    pilot_symb = list(pilot_symb)
    data_symb = [s for s in range(S) if s not in pilot_symb]
    H = ls_channel_estimate(Y[pilot_symb], pilots, n_ue, aligned=aligned)
    if sigma2 is None:
        sigma2 = noise_variance_estimate(Y[pilot_symb], pilots, n_ue, aligned=aligned)
    Yd = np.swapaxes(Y[data_symb], -1, -2)  # [D, K, N_B]
    if not time_varying:
        x_hat, ok = mmse_detect(H, Yd, sigma2)
    else:
        x_hat = np.zeros((len(data_symb), n_sc, n_ue), dtype=np.complex128)
        ok = np.ones(n_sc, dtype=bool)
        for d, s in enumerate(data_symb):
            Hs = time_interpolated_estimate(Y[pilot_symb], pilots, n_ue, pilot_symb, s, aligned)
            xs, oks = mmse_detect(Hs, Yd[d:d + 1], sigma2)
            x_hat[d] = xs[0]
            ok &= oks
    return {"X": X, "Y": Y, "H": H, "sigma2": sigma2, "x_hat": x_hat, "ok": ok}
