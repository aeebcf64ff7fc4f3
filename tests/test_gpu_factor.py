"""GPU parity of the DM-factorised phasor sums (uniform DM grid, exact delays).

For DM_j = DM_0 + j dDM the delay of trial a B + b is tau_A[a] + tau_B[b] exactly, so the
phasor factorises and the sum becomes a matrix product even for one chunk.  These tests run
the factorised kernels (forced with FDD_FACTOR=all where the default would not pick them)
against the FP64 oracle, which evaluates every phasor directly from its own delay, and against
the direct kernels (FDD_FACTOR=0).  DM counts that are not multiples of the fine block, 8-bit
input with its zero point, power spectra and every precision are covered.
"""
import dataclasses
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import check_power, check_rows, raw_start

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdd = pytest.importorskip("paper_2110_03482_amd")

TOL = {"fp32": 1e-5, "fp16_split": 1e-5, "bf16_split": 1e-4}


def make(seed, n_chan, n_samp, n_dm, L, single, kind, dm_lo, dm_hi):
    w = W.tiny_random(seed, n_chan, n_samp, n_dm, L, single_chunk=single, input_kind=kind)
    w = dataclasses.replace(w, dms=np.linspace(dm_lo, dm_hi, n_dm))
    x = W.gaussian_u8(n_samp, n_chan, seed) if kind == "u8" else W.gaussian_f32(n_chan, n_samp, seed)
    return w, x


def run(w, x, precision, factor, power=False, mode="exact"):
    old = os.environ.get("FDD_FACTOR")
    os.environ["FDD_FACTOR"] = factor
    try:
        p = fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, overlap=w.overlap,
                     single_chunk=w.single_chunk, input=w.input_kind, mode=mode, precision=precision,
                     power_only=power)
    finally:
        if old is None:
            del os.environ["FDD_FACTOR"]
        else:
            os.environ["FDD_FACTOR"] = old
    with p:
        xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        y = p.power_spectrum(xd) if power else p.execute(xd)
        torch.cuda.synchronize()
        g = p.geometry
        run.raw = raw_start(w.input_kind, w.n_samp, w.chunk_len, int(g.stride), int(g.n_chunks), w.single_chunk)
        return y.cpu().numpy(), p.kernel


CASES = [
    # seed, n_chan, n_samp, n_dm, L, single, kind, dm_lo, dm_hi     chunks -> fine DMs per row
    (1, 24, 4096, 64, 4096, True, "f32", 0.0, 63.0),          # 1 -> 32, 2 coarse rows
    (2, 40, 3000, 45, 4096, True, "f32", 2.5, 30.0),          # 1, 45 trials: partial coarse row
    (3, 33, 2048, 100, 2048, True, "u8", 0.0, 12.0),          # 1, 8-bit, full chunk (zero point)
    (4, 16, 3000, 20, 2048, False, "f32", 0.0, 3.0),          # 2 chunks -> 16
    (5, 20, 9000, 50, 2048, False, "u8", 0.0, 4.0),           # 5 chunks -> 6
    (6, 17, 30000, 70, 2048, False, "f32", 0.0, 6.0),         # 16 chunks -> 2
    (7, 8, 700, 3, 1024, True, "f32", 0.0, 1.0),              # 3 trials, 8 channels
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[1]}ch_{c[2]}s_{c[3]}dm_L{c[4]}_{c[6]}" for c in CASES])
@pytest.mark.parametrize("precision", ["fp32", "fp16_split", "bf16_split"])
def test_factorised_execute(case, precision):
    w, x = make(*case)
    print(f"factorised {case} {precision}", flush=True)
    y, kernel = run(w, x, precision, "all")
    assert kernel.startswith("fac_"), kernel
    ref = O.fdd(x, w.input_kind, w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len,
                single_chunk=w.single_chunk, mode="exact")
    raw = run.raw
    check_rows(y, ref, TOL[precision], raw_from=raw, label=f"{precision} {case} kernel={kernel}")
    yd, kd = run(w, x, precision, "0")
    assert not kd.startswith("fac_")
    check_rows(y, yd, 2 * TOL[precision], raw_from=raw, label=f"  vs direct kernel {kd}")


@pytest.mark.parametrize("precision", ["fp32", "fp16_split", "bf16_split"])
@pytest.mark.parametrize("kind", ["f32", "u8"])
def test_factorised_power(precision, kind):
    w, x = make(11, 37, 4096, 77, 4096, True, kind, 0.0, 40.0)
    P, kernel = run(w, x, precision, "1", power=True)
    assert kernel.startswith("fac_"), kernel
    tau = O.delays(w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s)
    ref = O.oracle_fdd_rows(x, kind, tau, w.chunk_len, w.chunk_len, 1, True, "exact", power=True)
    check_power(P, ref, TOL[precision], skip_dc=kind == "u8", label=f"{precision} {kind} power kernel={kernel}")
    if kind == "u8":
        np.testing.assert_allclose(P[:, 0], ref[:, 0], rtol=2e-6 if precision != "bf16_split" else 2e-5)


def test_selection_rules():
    w, x = make(1, 24, 4096, 64, 4096, True, "f32", 0.0, 63.0)
    _, k_exact = run(w, x, "fp32", "1")
    _, k_round = run(w, x, "fp32", "1", mode="round")
    wn = dataclasses.replace(w, dms=np.sort(np.random.default_rng(0).uniform(0, 63, 64)))
    _, k_nonuni = run(wn, x, "fp32", "1")
    assert k_exact == "fac_f32" and not k_round.startswith("fac_") and not k_nonuni.startswith("fac_")
