"""GPU tests of the batched form (fdd_batch_*): many uneven beams through grouped launches.

 - With the autotuner off the batch runs the kernels a single plan would run, so every beam's
   output must equal fdd_execute of its plan bit for bit, and the oracle to the FP32 bar.
 - Autotuned batches may pick other tile shapes (another summation order): oracle bar.
 - The captured graph is replayed several times with eager work in between, and re-captured
   when the tensors change; every replay is checked.
 - A small scratch limit splits the beams into memory waves that share one arena.
 - Beams shaped like the multi-beam workload (L = 2^16, 256-1024 channels, 512-4096 DMs)
   are checked on sampled rows, and each injected pulse is found at its DM.
"""
import json

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import check_rows, raw_start

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdd = pytest.importorskip("paper_2110_03482_amd")

TOL = 1e-5

# n_chan, n_samp, n_dm, L, single_chunk, input, dm_max, mode  -> chunks (phasor class)
BEAMS = [
    (24, 4000, 40, 4096, True, "f32", 5.0, "exact"),     # 1 chunk: VALU, one chunk per thread
    (16, 3000, 20, 2048, False, "f32", 3.0, "round"),    # 2 chunks: VALU (MFMA candidates when tuned)
    (20, 9000, 50, 2048, False, "u8", 4.0, "exact"),     # 5 chunks: MFMA, 1 column tile
    (33, 50000, 65, 4096, False, "f32", 10.0, "exact"),  # 13 chunks: 2 column tiles
    (40, 30000, 70, 2048, False, "f32", 6.0, "round"),   # 16 chunks: 2 column tiles
    (28, 40000, 45, 2048, False, "f32", 5.0, "exact"),   # 21 chunks: 3 column tiles
    (12, 60000, 30, 2048, False, "u8", 2.0, "round"),    # 30 chunks: MFMA over 2 chunk groups
    (8, 70000, 17, 1024, False, "f32", 1.0, "exact"),    # 70 chunks at L = 1024: 3 chunk groups
]


def raw_of(w):
    """First output sample of an 8-bit beam produced by a chunk past the end of its data."""
    g = fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, overlap=w.overlap,
                 single_chunk=w.single_chunk, input=w.input_kind, dry_run=True).geometry
    return raw_start(w.input_kind, w.n_samp, w.chunk_len, int(g.stride), int(g.n_chunks), w.single_chunk)


def make_beams(specs, precision="fp32", seed0=100):
    beams = []
    for i, (n_chan, n_samp, n_dm, L, single, kind, dm_max, mode) in enumerate(specs):
        w = W.tiny_random(seed0 + i, n_chan, n_samp, n_dm, L, single_chunk=single, input_kind=kind, dm_max=dm_max)
        x = W.gaussian_u8(n_samp, n_chan, seed0 + i) if kind == "u8" else W.gaussian_f32(n_chan, n_samp, seed0 + i)
        prec = precision if isinstance(precision, str) else precision[i % len(precision)]
        beams.append((w, x, mode, prec))
    return beams


def plan_of(w, mode, precision, workspace):
    return fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, overlap=w.overlap,
                    single_chunk=w.single_chunk, input=w.input_kind, mode=mode, precision=precision,
                    workspace=workspace)


def single_results(beams, xs):
    outs = []
    for (w, _, mode, prec), xd in zip(beams, xs):
        with plan_of(w, mode, prec, True) as p:
            outs.append(p.execute(xd).cpu().numpy())
    torch.cuda.synchronize()
    return outs


def check_oracle(beams, ys, bound):
    for (w, x, mode, prec), y in zip(beams, ys):
        ref = O.fdd(x, w.input_kind, w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len, overlap=w.overlap,
                    single_chunk=w.single_chunk, mode=mode)
        check_rows(y, ref, bound, raw_from=raw_of(w), label=f"{w.name} {w.input_kind} {mode} {prec}")


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_single_plans_and_oracle(graph):
    beams = make_beams(BEAMS)
    xs = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for _, x, _, _ in beams]
    print(f"batch of {len(beams)} beams, graph={graph}, no autotune", flush=True)
    plans = [plan_of(w, mode, prec, False) for w, _, mode, prec in beams]
    with fdd.Batch(plans, graph=graph, autotune=False) as b:
        ys = [y.cpu().numpy() for y in b.execute(xs)]
        desc = b.describe()
    print(json.dumps(desc["classes"]))
    keys = {c["key"] for c in desc["classes"]}
    assert len(keys) == len(desc["classes"]) >= 6
    singles = single_results(beams, xs)
    for (w, _, _, _), y, s in zip(beams, ys, singles):
        assert np.array_equal(y, s), f"{w.name}: batched output differs from fdd_execute"
    check_oracle(beams, ys, TOL)


@pytest.mark.parametrize("precision", [["fp16_split", "bf16_split"]])
def test_batch_split_precision(precision):
    beams = make_beams(BEAMS, precision)
    xs = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for _, x, _, _ in beams]
    print(f"split batch of {len(beams)} beams", flush=True)
    plans = [plan_of(w, mode, prec, False) for w, _, mode, prec in beams]
    with fdd.Batch(plans, autotune=False) as b:
        ys = [y.cpu().numpy() for y in b.execute(xs)]
    singles = single_results(beams, xs)
    for (w, _, _, prec), y, s in zip(beams, ys, singles):
        assert np.array_equal(y, s), f"{w.name} {prec}: batched output differs from fdd_execute"
    check_oracle(beams, ys, 1e-4)


def test_batch_autotuned_with_cache(tmp_path):
    beams = make_beams(BEAMS[1:6])
    xs = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for _, x, _, _ in beams]
    cache = str(tmp_path / "tune.json")
    plans = [plan_of(w, mode, prec, False) for w, _, mode, prec in beams]
    print("autotuned batch", flush=True)
    with fdd.Batch(plans, tune_cache=cache) as b:
        ys = [y.cpu().numpy() for y in b.execute(xs)]
        desc = b.describe()
    for c in desc["classes"]:
        print(c["key"], "->", c["choice"], c["candidates"])
        assert c["settled"]
        if len(c["candidates"]) > 1:
            assert c["candidates"][c["choice"]] is not None
            timed = [v for v in c["candidates"].values() if v is not None]
            assert len(timed) == len(c["candidates"]) and c["candidates"][c["choice"]] == min(timed)
    check_oracle(beams, ys, TOL)
    saved = json.load(open(cache))
    assert any(k.endswith(c["key"]) for k in saved for c in desc["classes"] if len(c["candidates"]) > 1)
    # a new batch finds every choice in the cache file and times nothing
    with fdd.Batch(plans, tune_cache=cache) as b2:
        d2 = b2.describe()
        assert all(c["settled"] for c in d2["classes"])
        assert [c["choice"] for c in d2["classes"]] == [c["choice"] for c in desc["classes"]]
        ys2 = [y.cpu().numpy() for y in b2.execute(xs)]
        d3 = b2.describe()
        assert all(v is None for c in d3["classes"] for v in c["candidates"].values())
    for y, y2 in zip(ys, ys2):
        assert np.array_equal(y, y2)


def test_graph_replays_and_recapture():
    specs = [s for s in BEAMS if s[5] == "f32"]
    beams = make_beams(specs, seed0=300)
    xs = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for _, x, _, _ in beams]
    plans = [plan_of(w, mode, prec, False) for w, _, mode, prec in beams]
    ref_plans = [plan_of(w, mode, prec, True) for w, _, mode, prec in beams]
    print("graph replays", flush=True)
    with fdd.Batch(plans, autotune=False) as b:
        outs = [torch.empty((p.n_dm, p.n_samp), dtype=torch.float32, device="cuda") for p in plans]
        for rep in range(4):
            # eager work on the same stream between replays: rescale and shift the inputs in place
            for x in xs:
                x.mul_(-0.5).add_(0.25)
            b.execute(xs, outs)
            eager = [p.execute(x) for p, x in zip(ref_plans, xs)]
            torch.cuda.synchronize()
            for y, e in zip(outs, eager):
                assert torch.equal(y, e), f"replay {rep} differs from the eager result"
        # new output tensors: descriptors rewritten and the graph captured again
        outs2 = b.execute(xs)
        torch.cuda.synchronize()
        for y, y2 in zip(outs, outs2):
            assert torch.equal(y, y2)
    for p in ref_plans:
        p.close()


def test_batch_calls_on_two_streams():
    """Calls of one batch on alternating streams: a call on another stream waits for the previous
    call (same descriptors and ticket counters), and a call with new tensors waits for all earlier
    ones before it rewrites the descriptors.  Each call's inputs are rescaled on its own stream
    just before it, so a call that ran early would read the previous values."""
    specs = [s for s in BEAMS if s[5] == "f32"][:4]
    beams = make_beams(specs, seed0=400)
    xs = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for _, x, _, _ in beams]
    plans = [plan_of(w, mode, prec, False) for w, _, mode, prec in beams]
    ref_plans = [plan_of(w, mode, prec, True) for w, _, mode, prec in beams]
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    print("batch calls on two streams", flush=True)
    with fdd.Batch(plans, autotune=False) as b:
        outs = [torch.empty((p.n_dm, p.n_samp), dtype=torch.float32, device="cuda") for p in plans]
        results = []
        # same tensors on the other stream, new tensors (descriptors rewritten), the first ones again
        for call, (st, fresh) in enumerate(((sa, False), (sb, False), (sa, True), (sb, False))):
            st.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(st):
                for x in xs:
                    x.mul_(-0.5).add_(0.25)
                ys = b.execute(xs, None if fresh else outs, stream=st)
                snap = [y.clone() for y in ys]
            torch.cuda.current_stream().wait_stream(st)
            eager = [p.execute(x) for p, x in zip(ref_plans, xs)]
            results.append((call, snap, eager))
        torch.cuda.synchronize()
        for call, snap, eager in results:
            for y, e in zip(snap, eager):
                assert torch.equal(y, e), f"call {call} differs from the eager result"
    for p in ref_plans:
        p.close()

def test_memory_waves():
    beams = make_beams(BEAMS, seed0=500)
    xs = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for _, x, _, _ in beams]
    plans = [plan_of(w, mode, prec, False) for w, _, mode, prec in beams]
    with fdd.Batch(plans, autotune=False) as whole:
        ys = [y.cpu().numpy() for y in whole.execute(xs)]
        assert whole.n_waves == 1
        per_beam = [sk["scratch_bytes"] for sk in whole.describe()["stacks"]]
    # a limit of the largest beam's scratch forces several waves
    limit = max(per_beam)
    print(f"memory waves: limit {limit} of {sum(per_beam)} bytes", flush=True)
    with fdd.Batch(plans, autotune=False, scratch_limit=limit) as waved:
        assert waved.n_waves > 1
        assert waved.scratch_bytes <= limit
        ys2 = [y.cpu().numpy() for y in waved.execute(xs)]
    for y, y2 in zip(ys, ys2):
        assert np.array_equal(y, y2)


def test_multibeam_shapes_sampled_rows():
    """Beams shaped like the multi-beam workload (L = 2^16), pulses found at their DMs."""
    beams = W.batched_beams(4, seed=1, max_log_samp=17)
    xs, plans, rows = [], [], []
    for w, pulse_dm, t0 in beams:
        x = W.gaussian_f32(w.n_chan, w.n_samp, w.seed)
        offs = O.nearest_sample(O.delays([pulse_dm], w.freqs, w.ref_freq_mhz, w.tsamp_s))[0]
        W.inject_pulse_f32(x, offs, t0, 5.0, circular=False)
        xs.append(x)
        plans.append(plan_of(w, "exact", "fp32", False))
        trial = int(np.argmin(np.abs(w.dms - pulse_dm)))
        rows.append(sorted({0, trial, w.n_dm - 1}))
        print(f"{w.name}: pulse DM {pulse_dm:.2f} (trial {trial}), t0 {t0}", flush=True)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    with fdd.Batch(plans) as b:
        ys = b.execute(xd)
        print(json.dumps(b.describe()["classes"]), flush=True)
        for (w, pulse_dm, t0), x, y, r in zip(beams, xs, ys, rows):
            yr = y[r].cpu().numpy()
            ref = O.fdd(x, "f32", w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len, mode="exact", rows=r)
            check_rows(yr, ref, TOL, label=f"{w.name} rows {r}")
            peak = int(torch.argmax(y[:, t0 - 2:t0 + 3].amax(dim=1)).item())
            assert abs(w.dms[peak] - pulse_dm) <= 2.0 * (w.dms[1] - w.dms[0]) + 1.0


def test_batch_rejections():
    w = W.small_fp32()
    lib = fdd.library()
    with pytest.raises(fdd.FddError) as e:
        fdd.Batch([])
    assert e.value.status == 1
    with plan_of(w, "exact", "fp32", False) as p:
        d = fdd.BatchDesc()
        d.flags = 1 << 7
        with pytest.raises(fdd.FddError):
            fdd.fdd_batch_create([p.handle], d)
    long = W.tiny_random(7, 4, 1 << 17, 3, 1 << 17, single_chunk=True)
    with plan_of(long, "exact", "fp32", False) as p:
        with pytest.raises(fdd.FddError) as e:
            fdd.Batch([p])
        assert e.value.status == 3
    dry = fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, single_chunk=True, dry_run=True)
    with pytest.raises(fdd.FddError) as e:
        fdd.Batch([dry])
    assert e.value.status == 1 and "dry-run" in str(e.value)
    power = fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, single_chunk=True,
                     power_only=True, workspace=False)
    with pytest.raises(fdd.FddError) as e:
        fdd.Batch([power])
    assert e.value.status == 3
    assert lib.fdd_batch_destroy(None) == 0


def test_batch_factorised_classes():
    """Uniform DM grids: the batch offers the DM-factorised kernels; defaults match fdd_execute."""
    import dataclasses
    specs = [(24, 4000, 40, 4096, True, "f32", 5.0, "exact"),      # 1 chunk: factorised by default
             (16, 3000, 20, 2048, False, "f32", 3.0, "exact"),     # 2 chunks: factorised by default
             (20, 9000, 50, 2048, False, "u8", 4.0, "exact"),      # 5 chunks: direct by default
             (33, 50000, 65, 4096, False, "f32", 10.0, "exact")]   # 13 chunks: direct by default
    for precision in ("fp32", "fp16_split"):
        beams = []
        for w, x, mode, prec in make_beams(specs, precision, seed0=700):
            beams.append((dataclasses.replace(w, dms=np.linspace(0.0, float(w.dms[-1]), w.n_dm)), x, mode, prec))
        xs = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for _, x, _, _ in beams]
        plans = [plan_of(w, mode, prec, False) for w, _, mode, prec in beams]
        print(f"factorised classes, {precision}: plan kernels {[p.kernel for p in plans]}", flush=True)
        with fdd.Batch(plans, autotune=False) as b:
            ys = [y.cpu().numpy() for y in b.execute(xs)]
            keys = [c["key"] for c in b.describe()["classes"]]
        assert any("+fac0" in k for k in keys) and any(k.endswith("+fac") for k in keys), keys
        singles = single_results(beams, xs)
        for (w, _, _, _), y, s in zip(beams, ys, singles):
            assert np.array_equal(y, s), f"{w.name}: batched output differs from fdd_execute"
        check_oracle(beams, ys, TOL)
        with fdd.Batch(plans) as b:
            ys = [y.cpu().numpy() for y in b.execute(xs)]
            for c in b.describe()["classes"]:
                print(c["key"], "->", c["choice"], c["candidates"])
        check_oracle(beams, ys, TOL)


@pytest.mark.parametrize("precision", ["fp32", "fp16_split"])
def test_batch_shared_phasors(precision):
    """Beams of one set-up stacked along the chunk axis share every phasor (FDD_BATCH_SHARE_PHASORS)."""
    import dataclasses
    base = W.tiny_random(900, 24, 3000, 40, 2048, single_chunk=False, input_kind="f32", dm_max=4.0)
    beams = []
    for i, (n_samp, kind) in enumerate([(3000, "f32"), (5000, "u8"), (2100, "f32"), (9000, "f32"), (4000, "u8")]):
        w = dataclasses.replace(base, n_samp=n_samp, input_kind=kind, name=f"shared{i}")
        x = W.gaussian_u8(n_samp, w.n_chan, 910 + i) if kind == "u8" else W.gaussian_f32(w.n_chan, n_samp, 910 + i)
        beams.append((w, x, "exact", precision))
    # one beam of another set-up, and single-chunk beams that stack into a matrix product
    other = W.tiny_random(901, 17, 3000, 40, 2048, single_chunk=False, input_kind="f32", dm_max=4.0)
    beams.append((other, W.gaussian_f32(17, 3000, 920), "round", precision))
    single = W.tiny_random(902, 20, 1500, 33, 2048, single_chunk=True, input_kind="f32", dm_max=6.0)
    for i in range(3):
        beams.append((dataclasses.replace(single, name=f"single{i}"), W.gaussian_f32(20, 1500, 930 + i), "exact", precision))
    xs = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for _, x, _, _ in beams]
    plans = [plan_of(w, mode, prec, False) for w, _, mode, prec in beams]
    print(f"shared-phasor batch, {precision}: chunks {[p.geometry.n_chunks for p in plans]}", flush=True)
    with fdd.Batch(plans, share_phasors=True) as b:
        ys = [y.cpu().numpy() for y in b.execute(xs)]
        d = b.describe()
    print(json.dumps(d["stacks"]), json.dumps(d["classes"]))
    sizes = sorted(sk["beams"] for sk in d["stacks"])
    assert sizes == [1, 3, 5], sizes
    assert len({bm["stack"] for bm in d["beams"][:5]}) == 1
    singles = single_results(beams, xs)
    bound = {"fp32": TOL, "fp16_split": TOL}[precision]
    for (w, _, _, _), y, s1 in zip(beams, ys, singles):
        check_rows(y, s1, bound, raw_from=raw_of(w), label=f"{w.name} shared vs own plan")
    check_oracle(beams, ys, bound)


@pytest.mark.slow
def test_batched_workload_full_size_sampled_rows():
    """The 32-beam batched workload at full size, as bench.py times it (seed 0, FP32,
    autotuned, graph): every pulse found at its DM, and sampled rows of one beam of each
    phasor shape class (chunk-column tiles, factorised or not) against the oracle."""
    beams = W.batched_beams(32, seed=0)
    xs = []
    for w, pulse_dm, t0 in beams:
        x = W.gaussian_f32(w.n_chan, w.n_samp, w.seed)
        offs = O.nearest_sample(O.delays([pulse_dm], w.freqs, w.ref_freq_mhz, w.tsamp_s))[0]
        W.inject_pulse_f32(x, offs, t0, 5.0, circular=False)
        xs.append(x)
    print("batched workload: inputs generated", flush=True)
    plans = [fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, input="f32",
                      precision="fp32", workspace=False) for w, _, _ in beams]
    # one beam per chunk count (which fixes its shape class), the largest first
    pick = {}
    for i, p in enumerate(plans):
        n = int(p.geometry.n_chunks)
        if n not in pick or beams[i][0].n_chan * beams[i][0].n_samp > beams[pick[n]][0].n_chan * beams[pick[n]][0].n_samp:
            pick[n] = i
    xd = [torch.from_numpy(x).cuda() for x in xs]
    outs = [torch.empty((w.n_dm, w.n_samp), dtype=torch.float32, device="cuda") for w, _, _ in beams]
    with fdd.Batch(plans) as b:
        b.execute(xd, outs)
        b.execute(xd, outs)                      # a graph replay
        torch.cuda.synchronize()
        print(f"batched workload: {b.n_waves} waves; classes "
              f"{[(c['key'], c['choice']) for c in b.describe()['classes']]}", flush=True)
    hits = 0
    for (w, pulse_dm, t0), y in zip(beams, outs):
        peak = int(torch.argmax(y[:, t0 - 2:t0 + 3].amax(dim=1)).item())
        hits += abs(w.dms[peak] - pulse_dm) <= 2.0 * (w.dms[1] - w.dms[0]) + 1.0
    assert hits == len(beams)
    for n, i in sorted(pick.items()):
        w, pulse_dm, t0 = beams[i]
        trial = int(np.argmin(np.abs(w.dms - pulse_dm)))
        rows = sorted({0, trial, w.n_dm - 1})
        yr = outs[i][rows].cpu().numpy()
        ref = O.fdd(xs[i], "f32", w.dms, w.freqs, w.ref_freq_mhz, w.tsamp_s, w.chunk_len, mode="exact", rows=rows)
        check_rows(yr, ref, TOL, label=f"{w.name} ({n} chunks) rows {rows}")
    for p in plans:
        p.close()
