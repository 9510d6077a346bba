"""Throughput of the fused PUSCH receive chain on one MI355X.

One step = one pusch_slot call over a batch of 16 synthetic slots of the
paper-scale workload (64 receive antennas, 4096-point FFT with 3300 active
subcarriers, 14 OFDM symbols with pilots on symbols 2 and 11, 32 DFT beams,
16 UEs with 64-QAM, 8-tap 300 ns exponential-PDP channel, 20 dB SNR): FFT of
every antenna and symbol, beamforming, LS channel estimation and MMSE
detection.  Inputs sit in HBM before the timed region starts.

Prints ONE JSON line with slots/s and us/slot (p50/p99 over steps, one event
per step and nothing else recorded in the timed region), the per-stage device
time measured with HIP events that the library records on the launch stream
around every stage in a second pass over the same steps, the roofline of the
dominant kernel (the HBM or the FP32 roof, whichever binds at the kernel's
algorithmic intensity), the FP64 CPU oracle timed on a bounded sample of the
same slots (serial, and on every host core of the GPU's share), and the same
batch through the FP16 and the bfloat16 reduced-precision chains, through the
chain with the noise variance estimated from the pilots, and through the chain
with a channel estimate per data symbol.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
N_SLOT = 16
SEEDS = list(range(2000, 2000 + N_SLOT))

# Algorithmic bytes moved by each kernel per slot of the workload (its
# compulsory inputs + outputs; complex64 = 8 B, int32 status = 4 B).  With 16
# UEs the channel estimate is fused: the beamforming epilogue divides the
# pilot symbols by their pilots and the detection kernel interpolates the
# estimate from them, so no channel estimate is stored or re-read.
S, R, N, K, B, L, NP = 14, 64, 4096, 3300, 32, 16, 2
D = S - NP
STAGE_BYTES = {
    "fft": S * R * N * 8 + S * R * K * 8,
    "beamform": S * R * K * 8 + B * R * 8 + NP * K * 8 + S * K * B * 8,
    "mmse": NP * K * B * 8 + D * K * B * 8 + D * K * L * 8 + K * 4,
}
# Nominal arithmetic per slot (8 flops per complex MAC, 5 N log2 N per FFT).
# Detection counts the Hermitian half of the Gram matrix (B L (L + 1) / 2
# complex MACs), N_L^3 / 3 for the Cholesky factor, the matched filter and the
# two substitutions per data symbol; the fused stage also interpolates the
# channel estimate (about 27 MFLOP per slot at this geometry).
CHEST_FLOPS = 27_000_000
STAGE_FLOPS = {
    "fft": S * R * 5 * N * 12,
    "beamform": 8 * S * K * R * B,
    "mmse": 8 * K * (B * L * (L + 1) // 2 + L ** 3 // 3 + D * (B * L + L * L)) + CHEST_FLOPS,
}
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 (vector and MFMA, dense)
RIDGE = FP32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)  # flop/B where the two roofs meet
SLOT_FLOOR_BYTES = S * R * N * 8 + D * K * L * 8 + K * 4  # time-domain input + detected symbols
STAGE_KERNEL = {"fft": "k_fft<4096, 0>", "beamform": "k_beamform_k<2, 16>", "mmse": "k_mmse_mfma<8, true, 2, 12>"}
STAGE_SOURCE = {"fft": "fft.hip", "beamform": "beamform.hip", "mmse": "mmse.hip"}
TRAFFIC_FILE = "profiles/hbm_traffic_paper_scale.md"


def _source_sha(stage: str) -> str:
    path = os.path.join(ROOT, "paper_2210_09196_amd", "csrc", STAGE_SOURCE[stage])
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def _traffic(stage: str) -> float | None:
    """HBM bytes per launch of the stage's kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    rows = {}
    for line in open(path):
        cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
        if len(cells) >= 4 and cells[0] in STAGE_KERNEL:
            rows[cells[0]] = cells
    row = rows.get(stage)
    if not row or row[1] != _source_sha(stage):
        return None
    try:
        return float(row[-1])
    except ValueError:
        return None


_CPU_BATCH = None  # the slot batch, inherited by the forked oracle workers


def _oracle_worker(args) -> tuple[int, float]:
    """One host core: the FP64 oracle with one BLAS thread over slots first, first + stride, ...
    (cycling over the batch) until `seconds` have passed; returns (slots done, seconds)."""
    first, stride, seconds = args
    from threadpoolctl import threadpool_limits

    from oracle import pusch_oracle
    from paper_2210_09196_amd import synth

    cfg, batch = synth.CFG2, _CPU_BATCH
    done, t0 = 0, time.perf_counter()
    with threadpool_limits(limits=1):
        while time.perf_counter() - t0 < seconds:
            i = (first + stride * done) % N_SLOT
            pusch_oracle.receive_slot(batch["x_td"][i], batch["pilots"][i], cfg.pilot_symb, cfg.n_ue, cfg.n_sc,
                                      batch["sigma2"], n_beams=cfg.n_beams)
            done += 1
    return done, time.perf_counter() - t0


def _host_description() -> dict:
    import platform

    import numpy

    model = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = "unknown"
    try:
        from threadpoolctl import threadpool_info

        libs = [f"{i.get('internal_api')} {i.get('version')}" for i in threadpool_info() if i.get("user_api") == "blas"]
        blas = ", ".join(libs) or blas
    except Exception:
        pass
    return {"cpu_model": model, "numpy": numpy.__version__, "blas": blas}


def cpu_baseline(batch: dict, seconds: float, max_cores: int) -> dict:
    """The FP64 oracle on the host, as it stands, in two modes over the batch's slots (cycling):
    serial (one process, one BLAS thread; the paper's single-core baseline) and all cores (one
    forked process per core, one BLAS thread each, independent slots).  Must run before the
    process touches the GPU (the workers are forked)."""
    import multiprocessing as mp

    global _CPU_BATCH
    _CPU_BATCH = batch
    done, dt = _oracle_worker((0, 1, seconds))
    cores = max(1, min(max_cores, len(os.sched_getaffinity(0))))
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(c, cores, seconds) for c in range(cores)])
    all_done = sum(r[0] for r in res)
    all_dt = max(r[1] for r in res)
    host = _host_description()
    return {"value": all_done / all_dt, "unit": "slots/s", "cores": cores, "kind": "oracle",
            "sample": f"{all_done} slot evaluations of the same workload (the batch's {N_SLOT} slots in turn) by "
                      f"{cores} forked processes, one per core, one BLAS thread each, {all_dt:.1f} s",
            "serial": {"value": done / dt, "unit": "slots/s", "cores": 1,
                       "sample": f"{done} slot evaluations, one process, one BLAS thread, {dt:.1f} s"},
            **host}


def calibrate_copy() -> int:
    """A plain device-to-device copy of 1 GiB, five times (for scaling HBM counters)."""
    import torch

    n = 1 << 30
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    ev[0].record()
    for i in range(5):
        dst.copy_(src)
        ev[i + 1].record()
    torch.cuda.synchronize()
    ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(5)]
    gbs = [2 * n / (m / 1e3) / 1e9 for m in ms]  # read + write
    print(json.dumps({"calibrate_copy_bytes": n, "copies": 10, "timed_copies_ms": [round(m, 4) for m in ms],
                      "copy_GBs_read_plus_write": [round(g, 1) for g in gbs],
                      "copy_hbm_frac": round(max(gbs) / HBM_PEAK_GBS, 4)}), flush=True)
    return 0


def _evm_db(xh, xt) -> float:  # 10 log10(sum |x_hat - x|^2 / sum |x|^2)
    return float(10.0 * np.log10(np.sum(np.abs(xh - xt) ** 2) / np.sum(np.abs(xt) ** 2)))


def _run_variant(args, cfg, batch, x, p, x_hat32, precision: str, sigma2, time_varying: bool = False,
                 fft_mfma: bool = False):
    """Time the 16-slot launch of one chain variant with the same protocol as
    the headline run; returns (ms per step, stage us per launch, x_hat, status, slot)."""
    import torch

    from paper_2210_09196_amd import pusch

    dev = x.device
    slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb,
                      sigma2, N_SLOT, device=dev, precision=precision, time_varying=time_varying,
                      fft_mfma=fft_mfma)
    xh = torch.empty_like(x_hat32)
    st = torch.empty(N_SLOT, cfg.n_sc, dtype=torch.int32, device=dev)
    for _ in range(args.warmup):
        slot(x, p, xh, st)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        slot(x, p, xh, st)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    pusch.profile_begin(args.steps)  # stage times in a second pass, as for the headline
    for _ in range(args.steps):
        slot(x, p, xh, st)
    torch.cuda.synchronize()
    calls, stage_ms = pusch.profile_end()
    return ms, {k: round(v / calls * 1e3, 2) for k, v in stage_ms.items()}, xh, st, slot


def bench_mixed(args, cfg, batch, x, p, x_hat32, nd: int, ms32: float) -> dict:
    """The same batch through pusch_slot_mixed (FP16 active-bin grids between
    OFDM demodulation and beamforming, FP16-MFMA beamforming): time per step with the
    same protocol, and the EVM of both chains' detected symbols against the
    transmitted ones on the distinct slots."""
    ms, stage_us, xh, st, _ = _run_variant(args, cfg, batch, x, p, x_hat32, "mixed", batch["sigma2"])
    data = batch["data"][:nd].transpose(0, 1, 3, 2)  # x_hat layout [slot][D][K][L]
    e32 = _evm_db(x_hat32[:nd].cpu().numpy(), data)
    e16 = _evm_db(xh[:nd].cpu().numpy(), data)
    return {"precision": "FP16 active-bin grids between FFT and beamforming (power-of-two row scale), "
                         "beamforming on FP16 MFMA with FP32 accumulation, FP32 estimation and detection",
            "value": round(N_SLOT / (ms / 1e3), 1), "unit": "slots/s", "us_per_slot": round(1e3 * ms / N_SLOT, 3),
            "speedup_vs_fp32": round(ms32 / ms, 3), "stage_us_per_launch": stage_us,
            "evm_db_fp32": round(e32, 3), "evm_db_mixed": round(e16, 3), "evm_gap_db": round(e16 - e32, 4),
            "evm_slots": nd, "status_flags": int(st.sum().item())}


def bench_bf16(args, cfg, batch, x, p, x_hat32, nd: int, ms32: float) -> dict:
    """The same batch through pusch_slot_bf16 (bfloat16 active-bin grids, no
    row scales, BF16-MFMA beamforming): time per step and EVM, as bench_mixed."""
    ms, stage_us, xh, st, _ = _run_variant(args, cfg, batch, x, p, x_hat32, "bf16", batch["sigma2"])
    data = batch["data"][:nd].transpose(0, 1, 3, 2)
    e32 = _evm_db(x_hat32[:nd].cpu().numpy(), data)
    eb = _evm_db(xh[:nd].cpu().numpy(), data)
    return {"precision": "bfloat16 active-bin grids between FFT and beamforming (no scaling), beamforming on "
                         "BF16 MFMA with FP32 accumulation, FP32 estimation and detection",
            "value": round(N_SLOT / (ms / 1e3), 1), "unit": "slots/s", "us_per_slot": round(1e3 * ms / N_SLOT, 3),
            "speedup_vs_fp32": round(ms32 / ms, 3), "stage_us_per_launch": stage_us,
            "evm_db_fp32": round(e32, 3), "evm_db_bf16": round(eb, 3), "evm_gap_db": round(eb - e32, 4),
            "evm_slots": nd, "status_flags": int(st.sum().item())}


def bench_fft_mfma(args, cfg, batch, x, p, x_hat32, nd: int, ms32: float) -> dict:
    """The FP16 and bfloat16 chains with the FFT's radix-16 passes on the
    matrix cores (slot option fft_mfma): time per step, FFT stage time and EVM."""
    data = batch["data"][:nd].transpose(0, 1, 3, 2)
    e32 = _evm_db(x_hat32[:nd].cpu().numpy(), data)
    out = {"what": "radix-16 FFT passes as 16x16 DFT-matrix products on FP16 / BF16 MFMA, FP32 accumulation"}
    for prec in ("mixed", "bf16"):
        ms, stage_us, xh, st, _ = _run_variant(args, cfg, batch, x, p, x_hat32, prec, batch["sigma2"], fft_mfma=True)
        e = _evm_db(xh[:nd].cpu().numpy(), data)
        out[prec] = {"value": round(N_SLOT / (ms / 1e3), 1), "unit": "slots/s",
                     "us_per_slot": round(1e3 * ms / N_SLOT, 3), "speedup_vs_fp32": round(ms32 / ms, 3),
                     "stage_us_per_launch": stage_us, "evm_gap_db": round(e - e32, 4),
                     "status_flags": int(st.sum().item())}
    return out


def bench_noise_est(args, cfg, batch, x, p, x_hat32, nd: int, ms32: float) -> dict:
    """The FP32 chain with the noise variance estimated from the pilot symbols
    of every slot (the chain's NE step) instead of given: time per step, the
    estimation kernels' share (the chest stage, empty otherwise in the fused
    slot), the estimates and the EVM next to the chain given the true variance."""
    ms, stage_us, xh, st, slot = _run_variant(args, cfg, batch, x, p, x_hat32, "fp32", None)
    data = batch["data"][:nd].transpose(0, 1, 3, 2)
    est = slot.sigma2_est[:nd].cpu().numpy()
    return {"sigma2": batch["sigma2"], "sigma2_est": [round(float(v), 5) for v in est],
            "value": round(N_SLOT / (ms / 1e3), 1), "unit": "slots/s", "us_per_slot": round(1e3 * ms / N_SLOT, 3),
            "time_vs_given_sigma2": round(ms / ms32, 4), "ne_us_per_launch": stage_us["chest"],
            "stage_us_per_launch": stage_us,
            "evm_db_given": round(_evm_db(x_hat32[:nd].cpu().numpy(), data), 3),
            "evm_db_estimated": round(_evm_db(xh[:nd].cpu().numpy(), data), 3),
            "status_flags": int(st.sum().item())}


def bench_time_varying(args, cfg, batch, x, p, x_hat32, ms32: float) -> dict:
    """The FP32 chain with a channel estimate and a factorisation per data
    symbol (time_varying): time per step on the same batch, and the EVM of it
    and of the static chain on two slots whose channel turns at 300 Hz."""
    import torch

    from paper_2210_09196_amd import pusch, synth

    ms, stage_us, _, st, _ = _run_variant(args, cfg, batch, x, p, x_hat32, "fp32", batch["sigma2"], time_varying=True)
    dcfg = cfg.replace(doppler_hz=300.0)
    db = synth.make_batch(dcfg, [2100, 2101])
    dx, dp = torch.from_numpy(db["x_td"]).to(x.device), torch.from_numpy(db["pilots"]).to(x.device)
    data = db["data"].transpose(0, 1, 3, 2)
    evm = {}
    for tv in (False, True):
        slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb,
                          db["sigma2"], 2, device=x.device, time_varying=tv)
        xh, _ = slot(dx, dp)
        evm[tv] = _evm_db(xh.cpu().numpy(), data)
    return {"value": round(N_SLOT / (ms / 1e3), 1), "unit": "slots/s", "us_per_slot": round(1e3 * ms / N_SLOT, 3),
            "time_vs_static": round(ms / ms32, 3), "stage_us_per_launch": stage_us,
            "doppler_hz": 300.0, "evm_db_static": round(evm[False], 3), "evm_db_time_varying": round(evm[True], 3),
            "status_flags": int(st.sum().item())}


def _cell_chain_bytes(c: dict) -> int:
    """Algorithmic HBM bytes of one slot of a cell through the fused chain (as STAGE_BYTES)."""
    s_, r_, n_, k_, b_, l_, np_ = c["n_symb"], c["n_ant"], c["n_fft"], c["n_sc"], c["n_beams"], c["n_ue"], \
        len(c["pilot_symb"])
    d_ = s_ - np_
    return (s_ * r_ * n_ * 8 + s_ * r_ * k_ * 8                                        # FFT
            + s_ * r_ * k_ * 8 + b_ * r_ * 8 + np_ * k_ * 8 + s_ * k_ * b_ * 8           # beamforming
            + np_ * k_ * b_ * 8 + d_ * k_ * b_ * 8 + d_ * k_ * l_ * 8 + k_ * 4)          # detection


def cells_cpu_baseline(cfgs, batches, got) -> tuple[dict, dict]:
    """The oracle over every cell's slot, single-threaded, timed; and the GPU's detected symbols of
    each cell against it (NRMSE, worst over the cells)."""
    from oracle import metrics as M
    from oracle import pusch_oracle as O

    t0 = time.perf_counter()
    worst, flagged = 0.0, 0
    for c, (cfg, b) in enumerate(zip(cfgs, batches)):
        ref = O.receive_slot(b["x_td"][0], b["pilots"][0], cfg.pilot_symb, cfg.n_ue, cfg.n_sc, b["sigma2"],
                             n_beams=cfg.n_beams)
        e = M.xhat_errors(got[c][0], ref["x_hat"])
        worst = max(worst, e["nrmse"])
        flagged += int(e["nrmse"] > 1e-4 or e["max_rel"] > 1e-3 or e["worst_sc"] > 1e-3)
    dt = time.perf_counter() - t0
    base = {"value": round(len(cfgs) / dt, 3), "unit": "slots/s", "cores": 1, "kind": "oracle",
            "sample": f"all {len(cfgs)} cells, one slot each, FP64, one thread"}
    check = {"cells": len(cfgs), "max_nrmse": float(f"{worst:.3g}"), "cells_out_of_tolerance": flagged,
             "tolerance": "NRMSE 1e-4, max-rel and worst-subcarrier 1e-3", "pass": flagged == 0}
    return base, check


def bench_cells(n_cells: int, steps: int, warmup: int) -> int:
    """Batched uneven cells: one pusch_cells call over n_cells cells of
    different geometries, replayed from a captured HIP graph, grouped (one
    launch per stage and kernel shape) and on side streams, against the same
    cells as plain pusch_slot calls one after another on one stream; then the
    oracle over every cell (the CPU baseline) and the grouped result against it."""
    import torch

    from paper_2210_09196_amd import pusch, synth

    geoms = synth.uneven_cells(n_cells)
    cfgs, batches = [], []
    for c, g in enumerate(geoms):
        # a seeded TDL slot per cell at 20 dB, QPSK..256-QAM by cell
        cfg = synth.CFG1.replace(n_ant=g["n_ant"], n_fft=g["n_fft"], n_sc=g["n_sc"], n_beams=g["n_beams"],
                                 n_ue=g["n_ue"], pilot_symb=g["pilot_symb"], qam_bits=(2, 4, 6, 8)[c % 4],
                                 channel="tdl", snr_db=20.0)
        b = synth.make_batch(cfg, [5000 + c])
        g["sigma2"] = b["sigma2"]
        cfgs.append(cfg)
        batches.append(b)
    xs = [torch.from_numpy(b["x_td"]).cuda() for b in batches]
    ps = [torch.from_numpy(b["pilots"]).cuda() for b in batches]
    print(f"[bench] {n_cells} cells generated", file=sys.stderr, flush=True)

    def timed(fn, n):
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return np.array([a.elapsed_time(b) * 1e3 for a, b in ev])  # us per call

    tuned = {}

    def measure(precision, grouped):
        cells = pusch.Cells(geoms, precision=precision, grouped=grouped)
        out, out_st = cells.outputs()
        if grouped:
            # the autotuner times every launch plan on this cell set and records the fastest
            plan, us = cells.tune(xs, ps, reps=5, x_hats=out, statuses=out_st)
            tuned[precision] = {"plan": plan, "us_per_plan": [round(u, 1) for u in us]}
        run = lambda: cells(xs, ps, out, out_st)
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        eager = timed(run, steps)
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            run()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            run()
        for _ in range(warmup):
            graph.replay()
        torch.cuda.synchronize()
        replay = timed(graph.replay, steps)
        print(f"[bench] cells {precision} {'grouped' if grouped else 'streams'}: graph p50 "
              f"{np.percentile(replay, 50) / n_cells:.3f} us/slot", file=sys.stderr, flush=True)
        return eager, replay, [o.cpu().numpy() for o in out], [o.cpu().numpy() for o in out_st]

    eager, replay, out, out_st = measure("fp32", True)
    eager_s, replay_s, out_s, _ = measure("fp32", False)
    _, replay_mixed, _, _ = measure("mixed", True)
    _, replay_mixed_s, _, _ = measure("mixed", False)
    same = all(np.array_equal(a, b) for a, b in zip(out, out_s))
    slots = [pusch.Slot(c["n_ant"], c["n_fft"], c["n_sc"], 14, c["n_beams"], c["n_ue"], c["pilot_symb"], c["sigma2"], 1)
             for c in geoms]
    seq_out = [(torch.empty(1, 12, c["n_sc"], c["n_ue"], dtype=torch.complex64, device="cuda"),
                torch.empty(1, c["n_sc"], dtype=torch.int32, device="cuda")) for c in geoms]

    def sequential():
        for k, sl in enumerate(slots):
            sl(xs[k], ps[k], *seq_out[k])

    for _ in range(warmup):
        sequential()
    torch.cuda.synchronize()
    seq = timed(sequential, steps)
    base, check = cells_cpu_baseline(cfgs, batches, out)
    check["grouped_equals_streams"] = same
    check["status_flags"] = int(sum(int(np.count_nonzero(st)) for st in out_st))
    per = lambda a, q: round(float(np.percentile(a, q)) / n_cells, 3)
    chain_bytes = sum(_cell_chain_bytes(dict(g, n_symb=14)) for g in geoms)
    floor_us = chain_bytes / (HBM_PEAK_GBS * 1e9) * 1e6 / n_cells
    mix = {f"N{n}": sum(c["n_fft"] == n for c in geoms) for n in (1024, 2048, 4096)}
    mix.update({f"ant{a}": sum(c["n_ant"] == a for c in geoms) for a in (16, 32, 64)})
    print(json.dumps({
        "metric": "batched uneven cells: us/slot", "value": per(replay, 50), "unit": "us/slot",
        "higher_is_better": False, "cells": n_cells, "steps": steps, "warmup": warmup,
        "graph_p50_us_per_slot": per(replay, 50), "graph_p99_us_per_slot": per(replay, 99),
        "eager_p50_us_per_slot": per(eager, 50), "eager_p99_us_per_slot": per(eager, 99),
        "streams_graph_p50_us_per_slot": per(replay_s, 50), "streams_graph_p99_us_per_slot": per(replay_s, 99),
        "streams_eager_p50_us_per_slot": per(eager_s, 50),
        "sequential_slot_calls_p50_us_per_slot": per(seq, 50),
        "mixed_graph_p50_us_per_slot": per(replay_mixed, 50),
        "mixed_graph_p99_us_per_slot": per(replay_mixed, 99),
        "mixed_streams_graph_p50_us_per_slot": per(replay_mixed_s, 50),
        "chain_bytes_MB": round(chain_bytes / 1e6, 1), "byte_floor_us_per_slot": round(floor_us, 3),
        "floor_frac": round(floor_us / per(replay, 50), 4),
        "tuned_plans": tuned, "oracle_check": check, "cpu_baseline": base,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{n_cells} uneven cells, one slot each: N in 1024/2048/4096 (N*3300/4096 active), "
                               f"16/32/64 antennas, beams = antennas/2, 4-16 UEs, pilots 2+11, TDL at 20 dB, "
                               f"QPSK..256-QAM", "mix": mix},
    }), flush=True)
    return 0 if check["pass"] and same else 1


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--settle-s", type=float, default=2.0,
                    help="warm-up lasts at least this many seconds of back-to-back steps")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="per CPU-baseline mode")
    ap.add_argument("--cpu-cores", type=int, default=16,
                    help="most host cores the all-cores CPU baseline uses (the GPU's share of the host)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--distinct-slots", type=int, default=N_SLOT,
                    help="generate this many distinct slots and repeat them to fill the 16-slot launch "
                         "(for profiler passes; kernel time and traffic do not depend on the values)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    ap.add_argument("--cells", type=int, default=0,
                    help="instead: time one pusch_cells call over this many uneven cells (graph replay)")
    args = ap.parse_args()
    if args.calibrate_copy:
        return calibrate_copy()
    if args.cells > 0:
        if not os.path.exists(os.path.join(ROOT, "paper_2210_09196_amd", "libpusch.so")):
            from paper_2210_09196_amd.build import build
            build()
        return bench_cells(args.cells, min(args.steps, 100), min(args.warmup, 10))
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); slots are independent, so a "
              f"multi-GPU run would split the slot batch with no communication -- see the design notes.",
              file=sys.stderr)
        return 2

    import torch

    from paper_2210_09196_amd import pusch, synth

    if not os.path.exists(pusch.LIB_PATH):
        from paper_2210_09196_amd.build import build
        build()
    cfg = synth.CFG2
    nd = max(1, min(N_SLOT, args.distinct_slots))
    print(f"[bench] generating {nd} synthetic slots", file=sys.stderr, flush=True)
    batch = synth.make_batch(cfg, SEEDS[:nd])
    if nd < N_SLOT:
        for key in ("x_td", "pilots"):
            batch[key] = np.ascontiguousarray(np.resize(batch[key], (N_SLOT,) + batch[key].shape[1:]))
    cpu = None
    if not args.no_cpu_baseline:  # before the GPU is touched: the all-cores mode forks workers
        print(f"[bench] CPU oracle baseline (~{2 * args.cpu_seconds:.0f} s: serial, then all cores)",
              file=sys.stderr, flush=True)
        cpu = cpu_baseline(batch, args.cpu_seconds, args.cpu_cores)
        print(f"[bench] CPU oracle: {cpu['serial']['value']:.2f} slots/s serial, {cpu['value']:.2f} slots/s on "
              f"{cpu['cores']} cores", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(batch["x_td"]).to(dev)
    p = torch.from_numpy(batch["pilots"]).to(dev)
    slot = pusch.Slot(cfg.n_ant, cfg.n_fft, cfg.n_sc, cfg.n_symb, cfg.n_beams, cfg.n_ue, cfg.pilot_symb,
                      batch["sigma2"], N_SLOT, device=dev)
    x_hat = torch.empty(N_SLOT, cfg.n_data, cfg.n_sc, cfg.n_ue, dtype=torch.complex64, device=dev)
    status = torch.empty(N_SLOT, cfg.n_sc, dtype=torch.int32, device=dev)

    # warm-up: at least --warmup steps and at least --settle-s seconds of back-to-back steps, so
    # that clocks and caches have settled before the timed region
    print(f"[bench] warmup {args.warmup} steps / {args.settle_s} s", file=sys.stderr, flush=True)
    t_settle, warm_steps = time.perf_counter(), 0
    while warm_steps < args.warmup or time.perf_counter() - t_settle < args.settle_s:
        for _ in range(4):
            slot(x, p, x_hat, status)
        warm_steps += 4
        torch.cuda.synchronize()
    settle_s = time.perf_counter() - t_settle

    # headline: the chain alone, one event per step and nothing recorded in between
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        slot(x, p, x_hat, status)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    total_ms = ev[0].elapsed_time(ev[-1])
    ms_per_step = total_ms / args.steps
    bad = int(status.sum().item())
    print(f"[bench] {args.steps} steps in {total_ms:.2f} ms (wall {wall * 1e3:.1f} ms), status flags {bad}",
          file=sys.stderr, flush=True)
    # stage times: the same steps again with the library's events around every stage launch
    # (they add a few microseconds per stage boundary, so they stay out of the headline)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    pusch.profile_begin(args.steps)
    e0.record(stream)
    for _ in range(args.steps):
        slot(x, p, x_hat, status)
    e1.record(stream)
    torch.cuda.synchronize()
    calls, stage_ms = pusch.profile_end()
    ms_profiled = e0.elapsed_time(e1) / args.steps

    us_slot = 1e3 * step_ms / N_SLOT
    stages = {}
    for name in STAGE_KERNEL:
        per_launch_s = stage_ms[name] / 1e3 / calls
        gbs = STAGE_BYTES[name] * N_SLOT / per_launch_s / 1e9
        stages[name] = {"kernel": STAGE_KERNEL[name], "us_per_launch": round(per_launch_s * 1e6, 2),
                        "us_per_slot": round(per_launch_s * 1e6 / N_SLOT, 3),
                        "alg_bytes_per_launch": STAGE_BYTES[name] * N_SLOT, "achieved_GBs": round(gbs, 1),
                        "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                        "nominal_TFLOPs": round(STAGE_FLOPS[name] * N_SLOT / per_launch_s / 1e12, 2)}
    stages["chest"] = {"fused_into": "mmse", "us_per_launch": round(stage_ms["chest"] / calls * 1e3, 2)}
    for name in STAGE_KERNEL:  # which roof binds at the kernel's algorithmic intensity
        inten = STAGE_FLOPS[name] / STAGE_BYTES[name]
        stages[name]["flop_per_byte"] = round(inten, 2)
        stages[name]["bound"] = "mfma" if inten > RIDGE else "hbm"
        stages[name]["fp32_frac"] = round(stages[name]["nominal_TFLOPs"] / FP32_PEAK_TFLOPS, 4)
    dom = max(STAGE_KERNEL, key=lambda k: stages[k]["us_per_launch"])
    traffic = _traffic(dom)
    st_dom = stages[dom]
    if st_dom["bound"] == "mfma":
        roofline = {"bound": "mfma", "achieved": st_dom["nominal_TFLOPs"], "peak": FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": st_dom["fp32_frac"]}
    else:
        roofline = {"bound": "hbm", "achieved": st_dom["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": st_dom["hbm_frac"]}
    roofline.update({"traffic": traffic, "kernel": st_dom["kernel"], "flop_per_byte": st_dom["flop_per_byte"],
                     "ridge_flop_per_byte": round(RIDGE, 2),
                     "alg_bytes_per_launch": st_dom["alg_bytes_per_launch"],
                     "alg_flops_per_launch": STAGE_FLOPS[dom] * N_SLOT, "hbm_frac": st_dom["hbm_frac"],
                     "us_per_launch": st_dom["us_per_launch"]})
    chain_bytes = sum(STAGE_BYTES.values()) * N_SLOT
    mixed = bench_mixed(args, cfg, batch, x, p, x_hat, nd, ms_per_step)
    bf16 = bench_bf16(args, cfg, batch, x, p, x_hat, nd, ms_per_step)
    fft_mfma = bench_fft_mfma(args, cfg, batch, x, p, x_hat, nd, ms_per_step)
    noise = bench_noise_est(args, cfg, batch, x, p, x_hat, nd, ms_per_step)
    timevar = bench_time_varying(args, cfg, batch, x, p, x_hat, ms_per_step)
    out = {
        "metric": "PUSCH slots/s & \u00b5s/slot, 64ant\u00d74096-FFT; FP32 vs mixed+batched, EVM gap \u22640.1dB",
        "value": round(N_SLOT / (ms_per_step / 1e3), 1),
        "unit": "slots/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_steps_run": warm_steps,
        "settle_s": round(settle_s, 2),
        "ms_per_step": round(ms_per_step, 4),
        "us_per_slot": round(1e3 * ms_per_step / N_SLOT, 3),
        "us_per_slot_p50": round(float(np.percentile(us_slot, 50)), 3),
        "us_per_slot_p99": round(float(np.percentile(us_slot, 99)), 3),
        "ms_per_step_with_stage_events": round(ms_profiled, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper-scale PUSCH slot batch: 16 slots x (64 rx ant, 4096-FFT, 3300 active sc, "
                               "14 symb, pilots 2+11, 32 DFT beams, 16 UEs 64-QAM, TDL-8 300 ns, 20 dB)",
                   "n_slot": N_SLOT, "n_ant": 64, "n_fft": 4096, "n_sc": 3300, "n_symb": 14, "n_beams": 32,
                   "n_ue": 16},
        "chain_hbm_frac": round(chain_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "slot_floor_frac": round(SLOT_FLOOR_BYTES * N_SLOT / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "stages": stages,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "status_flags": bad,
        "mixed": mixed,
        "bf16": bf16,
        "fft_mfma": fft_mfma,
        "noise_est": noise,
        "time_varying": timevar,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
