"""GPU test of fdd_execute_noalloc, the variant of fdd_execute that allocates nothing: its
workspace lives in the library's static device scratch (64 MiB per device).

Two calls in a row, the second on a smaller problem (the scratch keeps the first call's
contents), each through the C ABI on a dry-run plan (no device memory of its own) and compared
with fdd_execute on a normal plan of the same descriptor: same kernels and tables, so the
outputs must be identical, and within the 1e-5 FP32 bar element by element.  A plan whose
workspace exceeds the scratch is rejected before any device work.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
import workloads as W
from parity import check_rows

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fdd = pytest.importorskip("paper_2110_03482_amd")


def _plans(w, mode, dry):
    kw = dict(overlap=w.overlap, single_chunk=w.single_chunk, input=w.input_kind, mode=mode)
    return fdd.Plan(w.freqs, w.ref_freq_mhz, w.tsamp_s, w.dms, w.n_samp, w.chunk_len, dry_run=dry, **kw)


def _compare(w, x, mode, label):
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    with _plans(w, mode, False) as ref_plan:
        y_ref = ref_plan.execute(xd)
        torch.cuda.synchronize()
        y_ref = y_ref.cpu().numpy()
    with _plans(w, mode, True) as p:
        assert p.geometry.workspace_bytes <= 64 << 20
        out = torch.full((w.n_dm, w.n_samp), float("nan"), dtype=torch.float32, device="cuda")
        print(f"{label}: fdd_execute_noalloc, workspace {p.geometry.workspace_bytes} bytes", flush=True)
        fdd.fdd_execute_noalloc(p.handle, xd.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        y = out.cpu().numpy()
    check_rows(y, y_ref, 1e-5, label=f"{label}: noalloc vs fdd_execute")
    np.testing.assert_array_equal(y, y_ref)
    return y


def test_noalloc_two_calls_second_smaller():
    # call 1: the small workload (64 ch x 4096 float32 samples x 64 DMs, one circular chunk)
    w1 = W.small_fp32(0)
    x1 = W.gaussian_f32(w1.n_chan, w1.n_samp, 0)
    offs = O.nearest_sample(O.delays([30.0], w1.freqs, w1.ref_freq_mhz, w1.tsamp_s))[0]
    W.inject_pulse_f32(x1, offs, 1000, 5.0, circular=True)
    y1 = _compare(w1, x1, "exact", "call 1 (64 ch, 4096 s, 64 DMs)")
    assert int(np.argmax(y1[:, 1000])) == 30
    # call 2, smaller: 24 channels of 8-bit time-major input, 3000 samples, overlap-save
    # chunks of 1024, 20 trial DMs, nearest-sample delays
    w2 = W.tiny_random(5, 24, 3000, 20, 1024, False, input_kind="u8", dm_max=4.0)
    x2 = W.gaussian_u8(w2.n_samp, w2.n_chan, 5)
    y2 = _compare(w2, x2, "round", "call 2 (24 ch, 3000 s, 20 DMs)")
    d = O.nearest_sample(O.delays(w2.dms, w2.freqs, w2.ref_freq_mhz, w2.tsamp_s))
    check_rows(y2, O.tdd(x2, "u8", d), 1e-5, raw_from=0, label="call 2 vs time-domain oracle")


def test_noalloc_rejects_a_workspace_beyond_the_scratch():
    w = W.paper_shaped_u8()
    with _plans(w, "exact", True) as p:
        x = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
        with pytest.raises(fdd.FddError) as e:
            fdd.fdd_execute_noalloc(p.handle, x.data_ptr(), x.data_ptr(), 0)
        assert e.value.status == 3
