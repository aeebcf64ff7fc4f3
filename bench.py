#!/usr/bin/env python3
"""Throughput of the Fourier-domain dedispersion hot path on one MI355X.

Workload (default): the paper-shaped problem of Sec. 4.1 at one GPU's size -- 1024 channels
over 1250-1550 MHz, 64 us sampling, 2^20 8-bit samples (Gaussian, mean 128, sigma 16) with
pulses injected at DM 100, 450 and 900, 2048 trial DMs from 0 to 1000, overlap-save chunks
of L = 2^16 with overlap ceil(max delay) = 14496 (21 chunks).  One step = one fdd_execute:
transpose/unpack, forward FFTs, phasor sum and inverse FFTs, input and output resident in HBM.

Prints one JSON line:  value = N_DM * N_t / (seconds per step)  (DM-trial samples/s) of the FP32
path; "forms" repeats the measurement with the FP16- and BF16-split phasor sums, the brute-force
time-domain kernel, down-sampled output, the batched workload (FP32 and FP16 split) and the
periodicity workload (FP16 split).  The roofline object refers to the phasor-sum kernel, whose
duration is the mean over the timed steps of HIP events recorded by the library on the execution
stream.

cpu_baseline: the FP64 oracle, in worker processes on the host's cores (at most --cpu-workers),
on a bounded sample of the same workload (--cpu-rows trial DMs over the first 4 chunks), both the
Fourier-domain and the brute-force time-domain method.  The sample's rows are kept and each
form's error against them ("err_vs_fp64_oracle": worst row relative to the row norm and to the
mean-removed row norm, and the largest absolute difference) is computed after the timed steps.

Other workloads (--workload):
  batched      32 uneven beams (256-1024 channels, 2^16-2^20 float32 samples, 512-4096 DMs,
               L = 2^16), one pulse each, dedispersed by one fdd_batch_execute (grouped launches
               replayed from one HIP graph, autotuned phasor-sum kernels); value = sum over
               beams of N_DM * N_t per second.
  periodicity  512 channels, one 2^22-sample float32 transform with a 33 ms pulsar at DM 57,
               4096 DMs 0-500, power spectra [4096][2^21] (fdd_power_spectrum, no inverse FFT).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from typing import Optional

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK = {  # MI355X published dense peaks
    "hbm_GBs": 8000.0,
    "fp32_mfma_TFLOPs": 157.3,
    "fp16_mfma_TFLOPs": 2500.0,
    "bf16_mfma_TFLOPs": 2500.0,
    "fp32_valu_TFLOPs": 157.3,
}
METRIC = "DM-trial samples/s (N_DM·N_t/s), FP32 FDD vs FP16-split MFMA at stated err"
KERNEL_SOURCES = {
    "mfma_f32": "paper_2110_03482_amd/csrc/phasor_mfma_f32.hip",
    "mfma_f16_split": "paper_2110_03482_amd/csrc/phasor_split.hip",
    "mfma_bf16_split": "paper_2110_03482_amd/csrc/phasor_split.hip",
    "valu": "paper_2110_03482_amd/csrc/phasor_valu.hip",
    "fac_f32": "paper_2110_03482_amd/csrc/phasor_fac.hip",
    "fac_f16_split": "paper_2110_03482_amd/csrc/phasor_fac.hip",
    "fac_bf16_split": "paper_2110_03482_amd/csrc/phasor_fac.hip",
    "facw_f32": "paper_2110_03482_amd/csrc/phasor_facw.hip",
    "facw_f16_split": "paper_2110_03482_amd/csrc/phasor_facw.hip",
    "facw_bf16_split": "paper_2110_03482_amd/csrc/phasor_facw.hip",
}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_digest(rel: str) -> str:
    with open(os.path.join(ROOT, rel), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it still matches."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    with open(path) as fh:
        table = json.load(fh)
    rec = table.get(f"{kernel}:{workload}")
    if rec is None or rec.get("source_sha") != source_digest(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("bytes_per_launch")


def make_paper_input(w, fdd):
    import workloads as W
    log(f"generating 8-bit input ({w.n_samp} x {w.n_chan}) ...")
    x = W.gaussian_u8(w.n_samp, w.n_chan, w.seed)
    for dm, t0 in ((100.0, 1 << 18), (450.0, 1 << 19), (900.0, 3 << 18)):
        tau = fdd.fdd_dispersion_delays(w.freqs, w.ref_freq_mhz, w.tsamp_s, dm)
        W.inject_pulse_u8(x, np.floor(tau + 0.5).astype(np.int64), t0, 80.0)
    return x


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# Oracle sample of the paper-shaped workload: these trial DMs (the three pulse trials among
# them) over the output of the first CPU_CHUNKS overlap-save chunks.  Worker processes are
# forked before the GPU is touched and share the input copy-on-write.
CPU_CHUNKS = 4
_CPU_JOB = {}


def _cpu_rows(task):
    import oracle as O
    kind, rows = task
    j = _CPU_JOB
    t0 = time.perf_counter()
    if kind == "o2":
        y = O.oracle_fdd_rows(j["x"], j["input_kind"], j["tau"], j["L"], j["S"], CPU_CHUNKS, False, j["mode"],
                              rows=rows)
    else:
        n_in = CPU_CHUNKS * j["S"] + j["D"]       # every input sample the kept outputs read
        y = O.tdd(j["x"][:n_in], j["input_kind"], j["d"], rows=rows)
    return np.ascontiguousarray(y[:, : CPU_CHUNKS * j["S"]]), time.perf_counter() - t0


def cpu_reference(w, x, mode: str, n_rows: int, workers: int) -> dict:
    """Time the FP64 oracle on all host cores (up to `workers` processes) on a bounded sample of
    the workload: Fourier-domain (Eqs. 3-7) and brute-force time-domain (Eq. 2) dedispersion of
    n_rows trial DMs over the first CPU_CHUNKS chunks.  The rows are kept to measure each GPU
    form's error on the same samples."""
    import multiprocessing as mp

    import oracle as O
    tau = O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s)
    S, n_chunks, D = O.chunk_geometry(w.n_samp, w.chunk_len, w.overlap, w.single_chunk, float(tau.max()))
    pulse_rows = {r for r in (0, 205, 921, 1842, w.n_dm - 1) if r < w.n_dm}
    rows = sorted(pulse_rows | {int(r) for r in np.linspace(0, w.n_dm - 1, max(0, n_rows - len(pulse_rows)))})
    _CPU_JOB.update(x=x, input_kind=w.input_kind, tau=tau, d=O.nearest_sample(tau), L=w.chunk_len, S=S, D=D,
                    mode=mode)
    n_out = CPU_CHUNKS * S
    workers = max(1, min(workers, len(rows)))
    parts = [rows[i::workers] for i in range(workers)]
    res = {}
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        for kind in ("o2", "o1"):
            log(f"cpu baseline: {kind} oracle on {len(rows)} DM rows x {n_out} output samples, {workers} processes")
            t0 = time.perf_counter()
            out = pool.map(_cpu_rows, [(kind, p) for p in parts])
            dt = time.perf_counter() - t0
            y = np.zeros((len(rows), n_out), dtype=np.float64)
            for i, (part, (yp, _)) in enumerate(zip(parts, out)):
                y[i::workers] = yp
            res[kind] = (y, dt)
            log(f"cpu baseline: {kind} {dt:.1f} s")
    _CPU_JOB.clear()
    o2_y, o2_dt = res["o2"]
    o1_y, o1_dt = res["o1"]
    sample = (f"{len(rows)} of {w.n_dm} trial DMs (incl. the pulse trials 205/921/1842) x the first {n_out} "
              f"output samples (the first {CPU_CHUNKS} of {n_chunks} overlap-save chunks) of the same workload")
    return {
        "rows": rows, "n_out": n_out, "o2": o2_y, "o1": o1_y,
        "baseline": {
            "value": len(rows) * n_out / o2_dt,
            "unit": "DM-trial samples/s",
            "cores": workers,
            "kind": "oracle",
            "sample": f"FP64 Fourier-domain oracle (numpy rfft, phasors, channel sum, irfft) on {sample}; "
                      f"{workers} worker processes, {o2_dt:.1f} s wall",
            "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(),
            "time_domain_o1": {
                "value": len(rows) * n_out / o1_dt, "unit": "DM-trial samples/s", "cores": workers,
                "sample": f"brute-force time-domain oracle (Eq. 2, nearest-sample delays) on the same {sample}; "
                          f"{o1_dt:.1f} s wall"},
        },
    }


def form_error(y: np.ndarray, ref: np.ndarray) -> dict:
    """Error of GPU rows y (float32) against oracle rows ref (float64), worst row: relative to the
    row norm, relative to the mean-removed row norm, and the largest absolute difference."""
    err = y.astype(np.float64) - ref
    rn = np.linalg.norm(ref, axis=1)
    cn = np.linalg.norm(ref - ref.mean(axis=1, keepdims=True), axis=1)
    en = np.linalg.norm(err, axis=1)
    return {"rel": float((en / rn).max()), "centred": float((en / cn).max()), "max_abs": float(np.abs(err).max()),
            "rows": int(ref.shape[0]), "samples_per_row": int(ref.shape[1])}


def timed_steps(fn, args, label: str) -> float:
    """Warm up, then time exactly args.steps calls of fn between two device synchronisations."""
    import torch
    for i in range(args.warmup):
        fn()
        torch.cuda.synchronize()
        log(f"{label}: warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()              # one GPU, one rank: this is the barrier
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fn()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    log(f"{label}: timed {args.steps} steps: {ms:.3f} ms/step")
    return ms


def base_result(args, value: float, ms: float, dtype: str, config: dict) -> dict:
    return {"metric": METRIC, "value": value, "unit": "DM-trial samples/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def batched_forms(args, dev, precisions) -> tuple:
    """Many uneven beams in one batched call per step; one form per precision."""
    import torch

    import paper_2110_03482_amd as fdd
    import workloads as W

    beams = W.batched_beams(args.beams, seed=0)
    xs, shapes = [], []
    for w, pulse_dm, t0 in beams:
        x = W.gaussian_f32(w.n_chan, w.n_samp, w.seed)
        tau = fdd.fdd_dispersion_delays(w.freqs, w.ref_freq_mhz, w.tsamp_s, pulse_dm)
        W.inject_pulse_f32(x, np.floor(tau + 0.5).astype(np.int64), t0, 5.0, circular=False)
        xs.append(torch.from_numpy(x).to(dev))
        shapes.append([w.n_chan, w.n_samp, w.n_dm])
        del x
    log(f"batched: {len(beams)} beams generated")
    samples = sum(w.n_dm * w.n_samp for w, _, _ in beams)
    outs = [torch.empty((w.n_dm, w.n_samp), dtype=torch.float32, device=dev) for w, _, _ in beams]
    forms = {}
    for prec in precisions:
        plans = [fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, input="f32",
                          precision=prec, mode=args.mode, device=dev, workspace=False) for w, _, _ in beams]
        flops = sum(8.0 * w.n_dm * w.n_chan * p.geometry.n_bins * p.geometry.n_chunks
                    for (w, _, _), p in zip(beams, plans))
        batch = fdd.Batch(plans, tune_cache=args.tune_cache)
        log(f"batched {prec}: {batch.n_waves} memory wave(s), scratch {batch.scratch_bytes / 2**30:.1f} GiB")
        t_first = time.perf_counter()
        batch.execute(xs, outs)           # autotune + graph capture
        torch.cuda.synchronize()
        log(f"batched {prec}: first call (tuning + capture) {time.perf_counter() - t_first:.1f} s")
        ms = timed_steps(lambda: batch.execute(xs, outs), args, f"batched {prec}")
        # detection check: every beam's pulse peaks within a few trials of its DM
        hits = 0
        for (w, pulse_dm, t0), y in zip(beams, outs):
            peak = int(torch.argmax(y[:, t0 - 2:t0 + 3].amax(dim=1)).item())
            hits += abs(w.dms[peak] - pulse_dm) <= 2.0 * (w.dms[1] - w.dms[0]) + 1.0
        d = batch.describe()
        forms[prec] = {"value": samples / (ms * 1e-3), "ms_per_step": ms, "pulses_found": f"{hits}/{len(beams)}",
                       "phasor_tflops_whole_step": flops / (ms * 1e-3) / 1e12, "waves": d["waves"],
                       "tuned": {c["key"]: c["choice"] for c in d["classes"]}}
        batch.close()
        for p in plans:
            p.close()
    config = {"workload": f"batched_{len(beams)}beams_seed0_{args.mode}", "beams": shapes, "chunk_len": 1 << 16,
              "input": "f32 channel-major", "band_mhz": [1250.0, 1550.0], "tsamp_s": 64e-6,
              "dm_range": [0.0, 1000.0], "precision": precisions[0]}
    del outs, xs
    torch.cuda.empty_cache()
    return forms, config


def run_batched(args, dev) -> int:
    precisions = ["fp32", "fp16_split"] if args.precision == "all" else [args.precision]
    forms, config = batched_forms(args, dev, precisions)
    main = forms[precisions[0]]
    result = base_result(args, main["value"], main["ms_per_step"],
                         "f32" if precisions[0] == "fp32" else "f16x2+f32acc", config)
    result["forms"] = forms
    print(json.dumps(result), flush=True)
    return 0


def periodicity_form(args, dev, prec: str, with_scaled: bool) -> dict:
    """Power spectra of a long single transform, without the inverse FFT."""
    import torch

    import paper_2110_03482_amd as fdd
    import workloads as W

    w = W.periodicity()
    x = W.gaussian_f32(w.n_chan, w.n_samp, 0)
    tau57 = fdd.fdd_dispersion_delays(w.freqs, w.ref_freq_mhz, w.tsamp_s, 57.0)
    W.inject_periodic_f32(x, tau57, 33.0e-3 / w.tsamp_s, 0.03, 0.3)
    xd = torch.from_numpy(x).to(dev)
    del x
    plan = fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, single_chunk=True,
                    input="f32", precision=prec, mode=args.mode, device=dev, power_only=True)
    out = torch.empty((w.n_dm, w.n_samp // 2), dtype=torch.float32, device=dev)
    plan.profile(args.steps)
    ms = timed_steps(lambda: plan.power_spectrum(xd, out), args, f"periodicity {prec}")
    stage_ms, _ = plan.stage_ms()
    g = plan.geometry
    flops = 8.0 * w.n_dm * w.n_chan * (w.n_samp // 2 + 1)
    achieved = flops / (stage_ms[2] * 1e-3) / 1e12
    peak = PEAK["fp32_mfma_TFLOPs"] if prec == "fp32" else PEAK["fp16_mfma_TFLOPs"]
    config = {"workload": w.name + f"_{args.mode}_power", "n_chan": w.n_chan, "n_samp": w.n_samp, "n_dm": w.n_dm,
              "chunk_len": int(g.chunk_len), "precision": prec, "phasor_kernel": plan.kernel}
    # detection check: the pulsar's harmonic sum (8 harmonics of 33 ms) peaks at trial 467 (DM 57.02)
    f1 = w.n_samp / (33.0e-3 / w.tsamp_s)
    idx = [c for h in range(1, 9) for c in range(int(round(h * f1)) - 2, int(round(h * f1)) + 3)]
    trial = int(out[:, idx].double().sum(dim=1).argmax().item())
    form = {"value": w.n_dm * w.n_samp / (ms * 1e-3), "ms_per_step": ms, "config": config,
            "stages_ms": {"forward_fft": stage_ms[1], "phasor_sum_power": stage_ms[2]},
            "roofline": {"kernel": f"phasor_sum_{plan.kernel}", "bound": "alu" if plan.kernel == "valu" else "mfma",
                         "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                         "traffic": measured_traffic(plan.kernel, f"{config['workload']}_{prec}"),
                         "algorithmic_flops_per_launch": flops},
            "pulsar_trial": trial}
    plan.close()
    if with_scaled:
        form["scaled"] = {f"scaled_dm_{p}": run_scaled(args, dev, w, xd, out, flops, p) for p in ("fp32", "fp16_split")}
    del out, xd
    torch.cuda.empty_cache()
    return form


def run_periodicity(args, dev) -> int:
    prec = "fp16_split" if args.precision == "all" else args.precision
    form = periodicity_form(args, dev, prec, args.precision == "all")
    result = base_result(args, form["value"], form["ms_per_step"], "f32" if prec == "fp32" else "f16x2+f32acc",
                         form.pop("config"))
    result["stages_ms"] = form["stages_ms"]
    result["roofline"] = form["roofline"]
    result["pulsar_trial"] = form["pulsar_trial"]
    if "scaled" in form:
        result["forms"] = form["scaled"]
    print(json.dumps(result), flush=True)
    return 0


def run_scaled(args, dev, w, xd, exact, exact_flops, precision: str) -> dict:
    """Spin-frequency-scaled DMs (Eq. 8) on the same input: time, matrix-core rate, and the
    approximation's error against the exact spectra in `exact`."""
    import torch

    import paper_2110_03482_amd as fdd

    plan = fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, single_chunk=True,
                    input="f32", precision=precision, mode="exact", device=dev, power_only=True, scaled_dm=True)
    g = plan.geometry
    f_min = int(g.scaled_min_bin)
    out = torch.empty_like(exact)
    plan.profile(args.steps)
    ms = timed_steps(lambda: plan.power_spectrum_scaled(xd, out), args, f"periodicity scaled DMs {precision}")
    stage_ms, _ = plan.stage_ms()
    n_blocks = -(-(w.n_samp // 2 - f_min) // 64)
    gemm_flops = 8.0 * (w.n_dm + 64) * w.n_chan * n_blocks * 64     # matrix work of the block products
    achieved = gemm_flops / (stage_ms[2] * 1e-3) / 1e12
    peak = PEAK["fp32_mfma_TFLOPs"] if precision == "fp32" else PEAK["fp16_mfma_TFLOPs"]
    err = []
    for r0 in range(0, w.n_dm, 256):
        a = out[r0: r0 + 256, f_min:].double()
        b = exact[r0: r0 + 256, f_min:].double()
        err.append(((a - b).norm(dim=1) / b.norm(dim=1)).cpu())
    err = torch.cat(err).numpy()
    f1 = w.n_samp / (33.0e-3 / w.tsamp_s)
    idx = [c for h in range(1, 9) for c in range(int(round(h * f1)) - 2, int(round(h * f1)) + 3)]
    hs = out[:, idx].double().sum(dim=1)
    he = exact[:, idx].double().sum(dim=1)
    plan.close()
    return {"value": w.n_dm * w.n_samp / (ms * 1e-3), "ms_per_step": ms,
            "stages_ms": {"forward_fft": stage_ms[1], "phasor_sum_power": stage_ms[2]},
            "f_min": f_min,
            "roofline": {"kernel": f"phasor_sum_scaled_{precision} (block products + low bins + resampling)",
                         "bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                         "frac": achieved / peak, "traffic": None,
                         "algorithmic_flops_per_launch": gemm_flops},
            "exact_equivalent_tflops": exact_flops / (stage_ms[2] * 1e-3) / 1e12,
            "approx_rel_l2_vs_exact": {"median": float(np.median(err)), "max": float(err.max())},
            "pulsar_trial": {"scaled_argmax": int(hs.argmax().item()), "exact_argmax": int(he.argmax().item()),
                             "harmonic_sum_ratio": float((hs[467] / he[467]).item())},
            "note": "approximation (Sec. 2.3, Eq. 8): DMs scaled by r/f within 64-bin blocks, power resampled "
                    "linearly in DM; bins below f_min exact"}


def run_crossover(args, dev) -> int:
    """Run time against the number of trial DMs (the paper's Sec. 4.1 comparison) on the
    paper-shaped 8-bit input: FDD FP32, FDD FP16 split and brute-force TDD."""
    import torch

    import paper_2110_03482_amd as fdd
    import workloads as W

    w0 = W.paper_shaped_u8(0)
    x = make_paper_input(w0, fdd)
    xd = torch.from_numpy(x).to(dev)
    del x
    rows = []
    for n_dm in (128, 256, 512, 1024, 2048, 4096):
        w = W.paper_shaped_u8(0, n_dm=n_dm)
        out = torch.empty((n_dm, w.n_samp), dtype=torch.float32, device=dev)
        row = {"n_dm": n_dm}
        for name, prec, tdd in (("fdd_fp32", "fp32", False), ("fdd_fp16_split", "fp16_split", False), ("tdd", "fp32", True)):
            plan = fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, input="u8",
                            precision=prec, mode="round" if tdd else args.mode, device=dev, power_only=tdd)
            fn = (lambda p=plan: p.tdd(xd, out)) if tdd else (lambda p=plan: p.execute(xd, out))
            ms = timed_steps(fn, args, f"{name} n_dm={n_dm}")
            row[name] = {"ms": ms, "value": n_dm * w.n_samp / (ms * 1e-3)}
            plan.close()
        rows.append(row)
        del out
        torch.cuda.empty_cache()
    main = [r for r in rows if r["n_dm"] == 2048][0]["fdd_fp32"]
    config = {"workload": f"crossover_paper_u8_1024ch_2p20s_{args.mode}", "n_chan": 1024, "n_samp": 1 << 20,
              "n_dm": [r["n_dm"] for r in rows], "chunk_len": 1 << 16}
    result = base_result(args, main["value"], main["ms"], "f32", config)
    result["crossover"] = rows
    print(json.dumps(result), flush=True)
    return 0


def run_multibeam(args, dev) -> int:
    """Beams of one set-up (Sec. 5 outlook): 16 beams of 512 channels x 2^17 float32 samples,
    2048 DMs 0..1000, L = 2^16 (3 chunks each), batched with and without phasor sharing."""
    import torch

    import paper_2110_03482_amd as fdd
    import workloads as W

    n_beams = 16
    w = W.Workload("multibeam_512ch_2p17s_2048dm", 512, 1250.0, 1550.0, 1550.0, 64e-6, 1 << 17,
                   np.linspace(0.0, 1000.0, 2048), 1 << 16, 0, False, "f32", 0)
    xs = [torch.from_numpy(W.gaussian_f32(w.n_chan, w.n_samp, 100 + i)).to(dev) for i in range(n_beams)]
    outs = [torch.empty((w.n_dm, w.n_samp), dtype=torch.float32, device=dev) for _ in range(n_beams)]
    samples = n_beams * w.n_dm * w.n_samp
    forms = {}
    precisions = ["fp32", "fp16_split"] if args.precision == "all" else [args.precision]
    for prec in precisions:
        for share in (False, True):
            plans = [fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, input="f32",
                              precision=prec, mode=args.mode, device=dev, workspace=False) for _ in range(n_beams)]
            batch = fdd.Batch(plans, share_phasors=share, tune_cache=args.tune_cache)
            label = f"multibeam {prec} share={share}"
            batch.execute(xs, outs)
            torch.cuda.synchronize()
            ms = timed_steps(lambda: batch.execute(xs, outs), args, label)
            d = batch.describe()
            forms[f"{prec}{'_shared' if share else ''}"] = {
                "value": samples / (ms * 1e-3), "ms_per_step": ms,
                "stacks": [sk["chunks"] for sk in d["stacks"]],
                "tuned": {c["key"]: c["choice"] for c in d["classes"]}}
            batch.close()
            for p in plans:
                p.close()
    main = forms[precisions[0]]
    config = {"workload": f"multibeam_{n_beams}x_512ch_2p17s_2048dm_{args.mode}", "beams": n_beams, "n_chan": 512,
              "n_samp": 1 << 17, "n_dm": 2048, "chunk_len": 1 << 16}
    result = base_result(args, main["value"], main["ms_per_step"], "f32" if precisions[0] == "fp32" else "f16x2+f32acc",
                         config)
    result["forms"] = forms
    print(json.dumps(result), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="all", choices=["all", "fp32", "fp16_split", "bf16_split"],
                    help="all: FP32 (reported as value) plus both split forms")
    ap.add_argument("--mode", default="exact", choices=["exact", "round"])
    ap.add_argument("--n-dm", type=int, default=2048)
    ap.add_argument("--log-samp", type=int, default=20,
                    help="paper workload: log2 of the samples per channel (21 doubles the band to 42 chunks)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=64, help="trial DMs in the oracle sample")
    ap.add_argument("--cpu-workers", type=int, default=16, help="oracle worker processes (at most the host's CPUs)")
    ap.add_argument("--no-extra-forms", action="store_true",
                    help="paper workload only: skip the batched and periodicity forms")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration) and exit")
    ap.add_argument("--workload", default="paper", choices=["paper", "batched", "periodicity", "crossover", "multibeam"])
    ap.add_argument("--beams", type=int, default=32, help="batched workload: number of beams")
    ap.add_argument("--tune-cache", default=None, help="batched workload: autotune cache file")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "single-GPU build: the path would shard across GPUs by DM trials, "
                                   "but only the one-GPU figure is measured; run with --gpus 1",
                          "n_gpus": args.gpus}), flush=True)
        return 2

    import torch

    import paper_2110_03482_amd as fdd
    import workloads as W

    paper = args.workload == "paper" and args.copy_probe_mib <= 0
    ref = None
    if paper:
        w = W.paper_shaped_u8(0, n_dm=args.n_dm)
        if args.log_samp != 20:
            w.n_samp = 1 << args.log_samp
            w.name = f"paper_u8_1024ch_2p{args.log_samp}s_{args.n_dm}dm"
        x = make_paper_input(w, fdd)
        if not args.no_cpu_baseline:
            # forked oracle workers start before anything touches the GPU
            ref = cpu_reference(w, x, args.mode, args.cpu_rows, min(args.cpu_workers, os.cpu_count() or 1))
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        return 1
    dev = torch.device("cuda:0")
    if args.copy_probe_mib > 0:
        # a plain copy of known size: calibrates rocprofv3's FETCH_SIZE / WRITE_SIZE counters
        n = args.copy_probe_mib << 20
        a = torch.ones(n, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n}), flush=True)
        return 0
    if args.workload == "batched":
        return run_batched(args, dev)
    if args.workload == "periodicity":
        return run_periodicity(args, dev)
    if args.workload == "crossover":
        return run_crossover(args, dev)
    if args.workload == "multibeam":
        return run_multibeam(args, dev)
    xd = torch.from_numpy(x).to(dev)
    samples = w.n_dm * w.n_samp
    sample_rows = None if ref is None else torch.tensor(ref["rows"], dtype=torch.int64, device=dev)

    def take_sample(out) -> Optional[np.ndarray]:
        """The oracle sample's rows and samples of a full-resolution output (after timing)."""
        if sample_rows is None:
            return None
        return out.index_select(0, sample_rows)[:, : ref["n_out"]].cpu().numpy()

    def run_form(precision: str, factors=None) -> dict:
        plan = fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, overlap=w.overlap,
                        single_chunk=w.single_chunk, input=w.input_kind, precision=precision, mode=args.mode,
                        device=dev, downsample=factors)
        g = plan.geometry
        shape = (int(g.out_samples),) if plan.downsampled else (w.n_dm, w.n_samp)
        out = torch.empty(shape, dtype=torch.float32, device=dev)
        log(f"{precision}: L={g.chunk_len} S={g.stride} D={g.overlap} chunks={g.n_chunks} kernel={plan.kernel} "
            f"segments={g.n_segments} workspace={g.workspace_bytes / 2**30:.2f} GiB")
        for i in range(args.warmup):
            plan.execute(xd, out)
            torch.cuda.synchronize()
            log(f"{precision}: warmup {i + 1}/{args.warmup} done")
        plan.profile(args.steps)
        torch.cuda.synchronize()          # one GPU, one rank: this is the barrier
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.execute(xd, out)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stage_ms, n_prof = plan.stage_ms()
        ms = (t1 - t0) * 1e3 / args.steps
        log(f"{precision}: timed {args.steps} steps: {ms:.3f} ms/step; stages {stage_ms} ({n_prof} calls)")
        res = {"precision": precision, "kernel": plan.kernel, "ms_per_step": ms, "value": samples / (ms * 1e-3),
               "stages_ms": {"transpose": stage_ms[0], "forward_fft": stage_ms[1], "phasor_sum": stage_ms[2],
                             "inverse_fft": stage_ms[3]},
               "geometry": g, "factors": factors,
               "sample": None if factors is not None else take_sample(out)}
        plan.close()
        del out
        torch.cuda.empty_cache()
        return res

    def run_tdd() -> dict:
        """The time-domain brute-force kernel (Eq. 2) on the same input and DM list."""
        plan = fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, overlap=w.overlap,
                        single_chunk=w.single_chunk, input=w.input_kind, mode="round", device=dev, power_only=True)
        out = torch.empty((w.n_dm, w.n_samp), dtype=torch.float32, device=dev)
        plan.profile(args.steps)
        ms = timed_steps(lambda: plan.tdd(xd, out), args, "tdd")
        stage_ms, _ = plan.stage_ms()
        sample = take_sample(out)
        plan.close()
        del out
        torch.cuda.empty_cache()
        res = {"value": samples / (ms * 1e-3), "ms_per_step": ms,
               "stages_ms": {"transpose": stage_ms[0], "shift_and_sum": stage_ms[2]},
               "note": "brute-force time-domain dedispersion, nearest-sample delays (the paper's comparison method)"}
        if sample is not None:
            res["err_vs_fp64_oracle_o1"] = form_error(sample, ref["o1"])
        return res

    forms = [run_form(p) for p in (["fp32", "fp16_split", "bf16_split"] if args.precision == "all" else [args.precision])]
    tdd_form = run_tdd() if args.precision == "all" else None
    # down-sampled output (Sec. 2.2): factors from the smearing across the lowest channel
    ds_factors = fdd.fdd_smearing_factors(w.freqs, w.tsamp_s, w.dms, 16)
    ds_forms = [run_form(p, ds_factors) for p in (["fp32", "fp16_split"] if args.precision == "all"
                                                    else [args.precision])]
    main_form = forms[0]
    g = main_form["geometry"]
    flops = 8.0 * w.n_dm * w.n_chan * g.n_bins * g.n_chunks      # complex MACs of Eq. 7, 8 flops each

    def form_flops(form: dict) -> float:
        fg = form["geometry"]
        if form["factors"] is None:
            return flops
        bins = (int(fg.chunk_len) // (2 * form["factors"].astype(np.int64)) + 1).sum()
        return 8.0 * w.n_chan * float(bins) * fg.n_chunks

    def roofline(form: dict) -> dict:
        flops = form_flops(form)
        achieved = flops / (form["stages_ms"]["phasor_sum"] * 1e-3) / 1e12
        peak = {"fp32": PEAK["fp32_mfma_TFLOPs"], "fp16_split": PEAK["fp16_mfma_TFLOPs"],
                "bf16_split": PEAK["bf16_mfma_TFLOPs"]}[form["precision"]]
        wl = w.name + f"_{args.mode}_{form['precision']}" + ("" if form["factors"] is None else "_downsampled")
        r = {"kernel": f"phasor_sum_{form['kernel']}", "bound": "alu" if form["kernel"] == "valu" else "mfma",
             "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
             "traffic": measured_traffic(form["kernel"], wl), "algorithmic_flops_per_launch": flops}
        if form["precision"] != "fp32":
            # each useful complex MAC costs three half-precision products (hi.hi, hi.lo, lo.hi)
            r["matrix_work_frac"] = 3.0 * achieved / peak
        return r

    def error(form: dict):
        """Measured against the oracle's rows (computed by the CPU baseline, outside the timed region)."""
        if ref is None or form["sample"] is None:
            return None
        e = form_error(form["sample"], ref["o2"] if args.mode == "exact" else ref["o1"])
        e["tol"] = {"fp32": 1e-5, "fp16_split": 1e-5, "bf16_split": 1e-4}[form["precision"]]
        return e
    result = {
        "metric": METRIC,
        "value": main_form["value"],
        "unit": "DM-trial samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_form["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16_split": "f16x2+f32acc", "bf16_split": "bf16x2+f32acc"}[main_form["precision"]],
        "data": "synthetic",
        "config": {
            "workload": w.name + f"_{args.mode}",
            "n_chan": w.n_chan, "n_samp": w.n_samp, "n_dm": w.n_dm, "input": "u8 time-major",
            "band_mhz": [w.f_lo_mhz, w.f_hi_mhz], "tsamp_s": w.tsamp_s, "dm_range": [0.0, float(w.dms[-1])],
            "chunk_len": int(g.chunk_len), "overlap": int(g.overlap), "n_chunks": int(g.n_chunks),
            "delay_mode": args.mode, "precision": main_form["precision"], "phasor_kernel": main_form["kernel"],
        },
        "stages_ms": main_form["stages_ms"],
        "roofline": roofline(main_form),
        "forms": {f["precision"]: {"value": f["value"], "ms_per_step": f["ms_per_step"], "stages_ms": f["stages_ms"],
                                   "roofline": roofline(f), "err_vs_fp64_oracle": error(f)}
                  for f in forms},
    }
    if tdd_form is not None:
        result["forms"]["tdd_u8"] = tdd_form
    counts = {int(d): int(n) for d, n in zip(*np.unique(ds_factors, return_counts=True))}
    for f in ds_forms:
        result["forms"][f["precision"] + "_downsampled"] = {
            "value": f["value"], "ms_per_step": f["ms_per_step"], "stages_ms": f["stages_ms"],
            "roofline": roofline(f), "segments": int(f["geometry"].n_segments), "factor_counts": counts,
            "output_samples": int(f["geometry"].out_samples),
            "note": "DMs whose smearing spans d >= 2 samples are inverted at L/d (Sec. 2.2); value counts input "
                    "samples per DM, as for the full-resolution forms"}
    del xd, x
    forms.clear()
    torch.cuda.empty_cache()
    if args.precision == "all" and not args.no_extra_forms:
        # the batched workload (32 uneven beams) and the periodicity workload (power spectra)
        bforms, bconfig = batched_forms(args, dev, ["fp32", "fp16_split"])
        for p, f in bforms.items():
            f["config"] = bconfig
            result["forms"][f"batched_{p}"] = f
        result["forms"]["periodicity_fp16_split"] = periodicity_form(args, dev, "fp16_split", False)
    if ref is not None:
        result["cpu_baseline"] = ref["baseline"]
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
