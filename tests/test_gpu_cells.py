"""GPU parity of pusch_cells: independent cells of different geometries in one
call (grouped launches on the caller's stream, the other cells on side streams
forked from and joined to it).

Each cell must match the FP64 oracle (detected symbols NRMSE <= 1e-4, no
status flags) and be bit-identical to the same cell run alone by pusch_slot
(same kernels, same inputs).  A captured graph of the call, replayed several
times with eager work in between, must reproduce the eager result exactly.
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
TOL_X = 1e-4

# (geometry over the small workload's defaults, slots per cell)
CELLS = [
    (dict(), 1),
    (dict(n_ant=16, n_fft=1024, n_sc=825, n_beams=8, n_ue=4, pilot_symb=(2,), qam_bits=2, channel="tdl"), 2),
    (dict(n_ant=32, n_fft=2048, n_sc=1650, n_beams=16, n_ue=8, pilot_symb=(2, 11), qam_bits=8, channel="tdl"), 1),
    (dict(n_ant=8, n_fft=64, n_sc=60, n_beams=8, n_ue=3, pilot_symb=(3, 9), qam_bits=4), 1),
    # odd beam count: stand-alone estimation kernel and a stored estimate
    (dict(n_beams=15), 1),
    (dict(n_ant=64, n_fft=4096, n_sc=3300, n_beams=32, n_ue=16, pilot_symb=(2, 11), qam_bits=6, channel="tdl"), 1),
]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def make_cells(cells, seed0=700):
    cfgs, batches, geoms = [], [], []
    for c, (geom, n_slot) in enumerate(cells):
        cfg = synth.CFG1.replace(snr_db=25.0, **geom)
        b = synth.make_batch(cfg, [seed0 + 10 * c + k for k in range(n_slot)])
        cfgs.append(cfg)
        batches.append(b)
        geoms.append(dict(n_ant=cfg.n_ant, n_fft=cfg.n_fft, n_sc=cfg.n_sc, n_symb=cfg.n_symb, n_beams=cfg.n_beams,
                          n_ue=cfg.n_ue, pilot_symb=cfg.pilot_symb, sigma2=b["sigma2"], n_slot=n_slot))
    return cfgs, batches, geoms


def test_cells_match_oracle_and_single_slot_calls():
    cfgs, batches, geoms = make_cells(CELLS)
    print(f"[cells] {len(CELLS)} cells", flush=True)
    cells = pusch.Cells(geoms)
    xs = [dev(b["x_td"]) for b in batches]
    ps = [dev(b["pilots"]) for b in batches]
    xh, st = cells(xs, ps)
    for c, (cfg, b, g) in enumerate(zip(cfgs, batches, geoms)):
        got, flags = host(xh[c]), host(st[c])
        assert np.all(flags == 0), c
        slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb,
                          b["sigma2"], g["n_slot"])
        alone, alone_st = slot(xs[c], ps[c])
        assert torch.equal(alone, xh[c]) and torch.equal(alone_st, st[c]), c
        for k in range(g["n_slot"]):
            ref = O.receive_slot(b["x_td"][k], b["pilots"][k], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                                 n_beams=cfg.n_beams)
            assert_xhat(got[k], ref["x_hat"], TOL_X, (c, k))


def test_cells_graph_replay_matches_eager():
    cfgs, batches, geoms = make_cells(CELLS[:5], seed0=900)
    cells = pusch.Cells(geoms)
    xs = [dev(b["x_td"]) for b in batches]
    ps = [dev(b["pilots"]) for b in batches]
    ref, ref_st = cells(xs, ps)  # eager call: builds every device table before the capture
    torch.cuda.synchronize()
    out, out_st = cells.outputs()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        cells(xs, ps, out, out_st)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        cells(xs, ps, out, out_st)
    for r in range(3):
        for t in out:
            t.zero_()
        for t in out_st:
            t.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        for c in range(len(geoms)):
            assert torch.equal(out[c], ref[c]) and torch.equal(out_st[c], ref_st[c]), (r, c)
        # eager work between replays, on the same buffers the graph does not use
        e, e_st = cells(xs, ps)
        torch.cuda.synchronize()
        for c in range(len(geoms)):
            assert torch.equal(e[c], ref[c]), (r, c)


def test_cells_mixed_precision_match_single_mixed_calls():
    cfgs, batches, geoms = make_cells(CELLS[:4], seed0=1100)
    cells = pusch.Cells(geoms, precision="mixed")
    xs = [dev(b["x_td"]) for b in batches]
    ps = [dev(b["pilots"]) for b in batches]
    xh, st = cells(xs, ps)
    for c, (cfg, b, g) in enumerate(zip(cfgs, batches, geoms)):
        slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb,
                          b["sigma2"], g["n_slot"], precision="mixed")
        alone, alone_st = slot(xs[c], ps[c])
        assert torch.equal(alone, xh[c]) and torch.equal(alone_st, st[c]), c
        ref = O.receive_slot(b["x_td"][0], b["pilots"][0], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                             n_beams=cfg.n_beams)
        assert_xhat(host(xh[c])[0], ref["x_hat"], 2e-3, c)


def test_cells_graph_replay_with_noise_estimation_and_mixed_precision():
    # the noise-estimation kernels and the FP16 path inside a captured graph:
    # every replay must reproduce the eager call's symbols and estimates exactly
    cfgs, batches, geoms = make_cells(CELLS[:4], seed0=1300)
    for g in geoms:
        g["sigma2"] = None
    for precision in ("fp32", "mixed"):
        cells = pusch.Cells(geoms, precision=precision)
        xs = [dev(b["x_td"]) for b in batches]
        ps = [dev(b["pilots"]) for b in batches]
        ref, ref_st = cells(xs, ps)
        torch.cuda.synchronize()
        ref_est = [t.clone() for t in cells.sigma2_est]
        out, out_st = cells.outputs()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            cells(xs, ps, out, out_st)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            cells(xs, ps, out, out_st)
        for r in range(3):
            for t in out:
                t.zero_()
            for t in cells.sigma2_est:
                t.fill_(-1.0)
            g.replay()
            torch.cuda.synchronize()
            for c in range(len(geoms)):
                assert torch.equal(out[c], ref[c]) and torch.equal(out_st[c], ref_st[c]), (precision, r, c)
                assert torch.equal(cells.sigma2_est[c], ref_est[c]), (precision, r, c)
            cells(xs, ps)  # eager work between replays
            torch.cuda.synchronize()


def test_cells_graph_replay_with_refinement_and_time_varying_cells():
    # a plain cell, a refined cell (row kernel, stored estimate) and a
    # time-varying cell (one detection launch per data symbol, flags ORed)
    # with estimated noise, captured into one graph and replayed
    cfgs, batches, geoms = make_cells([CELLS[0], CELLS[2], CELLS[1]], seed0=1500)
    geoms[1]["refine"] = True
    geoms[2]["time_varying"] = True
    geoms[2]["sigma2"] = None
    cells = pusch.Cells(geoms)
    xs = [dev(b["x_td"]) for b in batches]
    ps = [dev(b["pilots"]) for b in batches]
    ref, ref_st = cells(xs, ps)
    torch.cuda.synchronize()
    for c, (cfg, b, g) in enumerate(zip(cfgs, batches, geoms)):
        s2 = b["sigma2"] if g["sigma2"] is not None else None
        for k in range(g["n_slot"]):
            o = O.receive_slot(b["x_td"][k], b["pilots"][k], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, s2,
                               n_beams=cfg.n_beams, time_varying=bool(g.get("time_varying")))
            assert_xhat(host(ref[c])[k], o["x_hat"], TOL_X, (c, k))
    out, out_st = cells.outputs()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        cells(xs, ps, out, out_st)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        cells(xs, ps, out, out_st)
    for r in range(3):
        for t in out:
            t.zero_()
        for t in out_st:
            t.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        for c in range(len(geoms)):
            assert torch.equal(out[c], ref[c]) and torch.equal(out_st[c], ref_st[c]), (r, c)
        cells(xs, ps)
        torch.cuda.synchronize()


@pytest.fixture(scope="module")
def uneven48():
    """The 48 uneven cells the batched benchmark times (same seeded geometry draw), each filled with
    a seeded TDL slot (QPSK..256-QAM by cell), run by one pusch_cells call."""
    geoms = synth.uneven_cells(48)
    cfgs, batches = [], []
    for c, g in enumerate(geoms):
        cfg = synth.CFG1.replace(n_ant=g["n_ant"], n_fft=g["n_fft"], n_sc=g["n_sc"], n_beams=g["n_beams"],
                                 n_ue=g["n_ue"], pilot_symb=g["pilot_symb"], qam_bits=(2, 4, 6, 8)[c % 4],
                                 channel="tdl", snr_db=20.0)
        b = synth.make_batch(cfg, [5000 + c])
        g["sigma2"] = b["sigma2"]
        cfgs.append(cfg)
        batches.append(b)
    print(f"[cells] 48 uneven cells generated", flush=True)
    xs, ps = [dev(b["x_td"]) for b in batches], [dev(b["pilots"]) for b in batches]
    xh, st = pusch.Cells(geoms)(xs, ps)
    torch.cuda.synchronize()
    return cfgs, batches, [host(t) for t in xh], [host(t) for t in st], geoms, xs, ps


@pytest.mark.parametrize("part", range(4))
def test_uneven_48_cell_mix_matches_oracle(uneven48, part):
    cfgs, batches, xh, st = uneven48[:4]
    for c in range(part * 12, part * 12 + 12):
        cfg, b = cfgs[c], batches[c]
        assert np.all(st[c] == 0), c
        ref = O.receive_slot(b["x_td"][0], b["pilots"][0], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                             n_beams=cfg.n_beams)
        assert_xhat(xh[c][0], ref["x_hat"], TOL_X, (c, cfg.n_fft, cfg.n_ant, cfg.n_ue))


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_uneven_48_grouped_launches_equal_side_streams(uneven48, precision):
    # the grouped launches (one per stage and kernel shape over all 48 cells) and the per-cell
    # launches on side streams run the same arithmetic per tile: identical bits
    geoms, xs, ps = uneven48[4:]
    g_out, g_st = pusch.Cells(geoms, precision=precision)(xs, ps)
    s_out, s_st = pusch.Cells(geoms, precision=precision, grouped=False)(xs, ps)
    torch.cuda.synchronize()
    for c in range(len(geoms)):
        assert torch.equal(g_out[c], s_out[c]) and torch.equal(g_st[c], s_st[c]), (precision, c)
    if precision == "fp32":
        for c in range(len(geoms)):
            assert np.array_equal(host(g_out[c]), uneven48[2][c]), c


def test_more_cells_of_one_shape_than_one_launch_holds():
    # 40 cells of one geometry: more than one grouped launch per stage (32 FFT, 24 beamforming and
    # 16 detection cells per launch), plus two cells the grouped kernels do not take (odd beam count,
    # refinement) on the side streams; each equals its cell run alone
    base = dict(n_ant=8, n_fft=64, n_sc=60, n_beams=8, n_ue=3, pilot_symb=(3, 9), qam_bits=4)
    spec = [(base, 1 + (c % 3 == 0)) for c in range(40)] + [(dict(base, n_beams=7), 1), (base, 1)]
    cfgs, batches, geoms = make_cells(spec, seed0=3000)
    geoms[-1]["refine"] = True
    cells = pusch.Cells(geoms)
    xs = [dev(b["x_td"]) for b in batches]
    ps = [dev(b["pilots"]) for b in batches]
    xh, st = cells(xs, ps)
    for c, (cfg, b, g) in enumerate(zip(cfgs, batches, geoms)):
        slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb,
                          b["sigma2"], g["n_slot"], refine=bool(g.get("refine")))
        alone, alone_st = slot(xs[c], ps[c])
        assert torch.equal(alone, xh[c]) and torch.equal(alone_st, st[c]), c
    for c in (0, 17, 39, 40, 41):
        cfg, b = cfgs[c], batches[c]
        for k in range(geoms[c]["n_slot"]):
            ref = O.receive_slot(b["x_td"][k], b["pilots"][k], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                                 n_beams=cfg.n_beams)
            assert_xhat(host(xh[c])[k], ref["x_hat"], TOL_X, (c, k))


def test_every_launch_plan_gives_the_same_bits(uneven48):
    # one launch per stage for every kernel shape, or one per shape: the same arithmetic per tile
    geoms, xs, ps = uneven48[4:]
    for precision in ("fp32", "mixed"):
        ref, ref_st = pusch.Cells(geoms, precision=precision, grouped=False)(xs, ps)
        for p in range(pusch.CELLS_PLANS):
            out, st = pusch.Cells(geoms, precision=precision, plan=p)(xs, ps)
            torch.cuda.synchronize()
            for c in range(len(geoms)):
                assert torch.equal(out[c], ref[c]) and torch.equal(st[c], ref_st[c]), (precision, p, c)


def test_tuner_records_the_fastest_plan_for_the_cell_set():
    cfgs, batches, geoms = make_cells(CELLS[:4], seed0=3300)
    cells = pusch.Cells(geoms)
    xs = [dev(b["x_td"]) for b in batches]
    ps = [dev(b["pilots"]) for b in batches]
    ref, ref_st = pusch.Cells(geoms, grouped=False)(xs, ps)
    plan0, tuned0 = cells.plan()
    assert not tuned0 and plan0 == {"fft_merged": True, "bf_merged": False, "mmse_merged": True}
    plan, us = cells.tune(xs, ps, reps=3)
    print(f"[cells] tuned plan {plan}; us per plan {[round(u, 1) for u in us]}", flush=True)
    assert all(u > 0 for u in us)
    best = min(range(len(us)), key=lambda p: us[p])
    assert plan == {"fft_merged": bool(best & 1), "bf_merged": bool(best & 2), "mmse_merged": bool(best & 4)}
    assert cells.plan() == (plan, True)
    out, st = cells(xs, ps)
    for c in range(len(geoms)):
        assert torch.equal(out[c], ref[c]) and torch.equal(st[c], ref_st[c]), c
    # another cell set keeps the default
    other = pusch.Cells(geoms[:3])
    assert other.plan() == (plan0, False)
