"""Element-wise parity checks of the HIP path against the FP64 oracle (test infrastructure).

Every dedispersed row y (float32 from the GPU) is compared with the oracle's row ref (float64)
in three ways, so that a defect confined to a few samples (a chunk seam, a ragged tile, the
last chunk) cannot hide behind a row norm:

1. row norm:      ||y - ref|| / ||ref||                    <= tol
2. centred norm:  ||y - ref|| / ||ref - mean(ref)||        <= tol + floor
3. per sample:    max |y - ref|                            <= 10 (tol rms_c(ref) + floor_abs)

rms_c is the RMS of ref - mean(ref).  The centred norm matters for 8-bit input, whose rows
carry the 128 n_chan zero-point offset: against the plain norm an error of a few hundred
counts per sample would pass.  `floor` is the error that storing the exact result in float32
already makes (uniform rounding, RMS ulp/sqrt(12) per sample, relative to the centred norm):
at 1024 8-bit channels the values lie near 2^17, where it reaches ~7e-6 of the centred norm;
elsewhere it is negligible.

The raw region.  8-bit chunks that reach past the end of the data are transformed without
removing the zero point (the 128 -> 0 step at the end of the data is not a pure DC term), so
float32 rounding in their transforms scales with the 128 n_chan offset rather than with the
fluctuations.  Samples produced by such chunks (from output sample `raw_from` on) are checked
against the same tol relative to their own uncentred norm: ||y - ref||_raw <= tol ||ref||_raw,
and per sample max |y - ref| <= 10 tol rms(ref)_raw.  Every other sample meets the centred
bounds above.
"""
from __future__ import annotations

from typing import Optional, Sequence, Union

import numpy as np

PER_SAMPLE = 10.0


def f32_rounding_rms(ref: np.ndarray) -> float:
    """RMS of the error of rounding ref to float32 (ulp / sqrt(12) per sample)."""
    r = np.abs(np.asarray(ref, dtype=np.float64)).astype(np.float32)
    ulp = np.spacing(r).astype(np.float64)
    return float(np.sqrt(np.mean(ulp * ulp) / 12.0)) if r.size else 0.0


def raw_start(kind: str, n_samp: int, chunk_len: int, stride: int, n_chunks: int, single_chunk: bool,
              factor: int = 1) -> Optional[int]:
    """First output sample (at down-sampling factor `factor`) produced by an 8-bit chunk that
    runs past the end of the data, or None if there is no such chunk."""
    if kind != "u8":
        return None
    if single_chunk:
        return 0 if n_samp < chunk_len else None
    full = 0 if n_samp < chunk_len else min((n_samp - chunk_len) // stride + 1, n_chunks)
    if full >= n_chunks:
        return None
    return full * stride // factor


def raw_start_of(kind: str, geometry, n_samp: int, single_chunk: bool, factor: int = 1) -> Optional[int]:
    """raw_start from a plan's geometry."""
    return raw_start(kind, n_samp, int(geometry.chunk_len), int(geometry.stride), int(geometry.n_chunks),
                     single_chunk, factor)


class Stats:
    def __init__(self):
        self.rel = 0.0
        self.centred = 0.0
        self.sample = 0.0      # worst max|y - ref| / per-sample bound
        self.raw = 0.0         # worst raw-region ||err|| / ||ref||
        self.max_abs = 0.0
        self.rows = 0

    def line(self) -> str:
        s = (f"rows {self.rows}: rel {self.rel:.3e}, centred {self.centred:.3e}, "
             f"max abs {self.max_abs:.3e}, per-sample {self.sample:.3f} of bound")
        if self.raw > 0.0:
            s += f", raw region rel {self.raw:.3e}"
        return s


def check_rows(y, ref, tol: float, *, raw_from: Union[None, int, Sequence[Optional[int]]] = None,
               label: str = "", centred: bool = True) -> Stats:
    """Assert the three bounds on every row (y, ref: [rows, n] arrays or lists of 1-D rows)."""
    st = Stats()
    rows_y = [np.asarray(r, dtype=np.float64) for r in (y if isinstance(y, list) else np.atleast_2d(y))]
    rows_r = [np.asarray(r, dtype=np.float64) for r in (ref if isinstance(ref, list) else np.atleast_2d(ref))]
    assert len(rows_y) == len(rows_r), (label, len(rows_y), len(rows_r))
    for i, (yy, rr) in enumerate(zip(rows_y, rows_r)):
        assert yy.shape == rr.shape, (label, i, yy.shape, rr.shape)
        assert np.isfinite(yy).all(), f"{label}: row {i} not finite"
        rf = raw_from[i] if isinstance(raw_from, (list, tuple)) else raw_from
        n = rr.size
        cut = n if rf is None else max(0, min(int(rf), n))
        err = yy - rr
        nrm = np.linalg.norm(rr)
        e_rel = float(np.linalg.norm(err) / max(nrm, 1e-300))
        st.rel = max(st.rel, e_rel)
        st.max_abs = max(st.max_abs, float(np.abs(err).max()) if n else 0.0)
        assert e_rel <= tol, f"{label}: row {i} rel err {e_rel:.3e} > {tol:.1e}"
        if cut > 0:
            a, ra = err[:cut], rr[:cut]
            mean = ra.mean() if centred else 0.0
            rms_c = float(np.sqrt(np.mean((ra - mean) ** 2)))
            floor_abs = f32_rounding_rms(ra)
            e_c = float(np.sqrt(np.mean(a * a)) / max(rms_c, 1e-300))
            bound_c = tol + floor_abs / max(rms_c, 1e-300)
            st.centred = max(st.centred, e_c)
            assert e_c <= bound_c, f"{label}: row {i} centred err {e_c:.3e} > {bound_c:.3e} (samples < {cut})"
            lim = PER_SAMPLE * (tol * rms_c + floor_abs)
            worst = float(np.abs(a).max())
            st.sample = max(st.sample, worst / max(lim, 1e-300))
            assert worst <= lim, (f"{label}: row {i} sample {int(np.argmax(np.abs(a)))} off by {worst:.3e} "
                                  f"> {lim:.3e}")
        if cut < n:
            a, ra = err[cut:], rr[cut:]
            rms = float(np.sqrt(np.mean(ra * ra)))
            floor_abs = f32_rounding_rms(ra)
            e_raw = float(np.sqrt(np.mean(a * a)) / max(rms, 1e-300))
            st.raw = max(st.raw, e_raw)
            assert e_raw <= tol + floor_abs / max(rms, 1e-300), f"{label}: row {i} raw-region err {e_raw:.3e}"
            lim = PER_SAMPLE * (tol * rms + floor_abs)
            worst = float(np.abs(a).max())
            assert worst <= lim, (f"{label}: row {i} raw-region sample {cut + int(np.argmax(np.abs(a)))} off by "
                                  f"{worst:.3e} > {lim:.3e}")
        st.rows += 1
    if label:
        print(f"{label}: {st.line()}", flush=True)
    return st


def check_power(P, ref, tol: float, *, label: str = "", skip_dc: bool = False) -> Stats:
    """Power spectra P = |Y|^2, quadratic in the data: bounds derived from those on Y.

    Row norm: ||P - ref|| / ||ref|| <= 2 tol.  Per bin: an error of at most 10 tol rms|Y| in Y
    (the per-sample bound of check_rows, rms|Y| = sqrt(mean(ref))) moves |Y|^2 by at most
    2 |Y| (10 tol rms|Y|) + (10 tol rms|Y|)^2, with |Y| = sqrt(ref) of that bin, plus the float32
    rounding of ref.  A bin holding a large coherent power (DC offset, pulsar harmonic) is thus
    held to its own size rather than to the row's typical bin.  skip_dc leaves bin 0 to a
    separate check."""
    P = np.atleast_2d(np.asarray(P, dtype=np.float64))
    ref = np.atleast_2d(np.asarray(ref, dtype=np.float64))
    if skip_dc:
        P, ref = P[:, 1:], ref[:, 1:]
    st = Stats()
    for i, (pp, rr) in enumerate(zip(P, ref)):
        assert pp.shape == rr.shape, (label, i, pp.shape, rr.shape)
        assert np.isfinite(pp).all(), f"{label}: row {i} not finite"
        err = np.abs(pp - rr)
        e_rel = float(np.linalg.norm(err) / max(np.linalg.norm(rr), 1e-300))
        st.rel = max(st.rel, e_rel)
        st.max_abs = max(st.max_abs, float(err.max()) if err.size else 0.0)
        assert e_rel <= 2 * tol, f"{label}: row {i} rel err {e_rel:.3e} > {2 * tol:.1e}"
        dy = PER_SAMPLE * tol * np.sqrt(max(float(rr.mean()), 0.0))     # bound on |Y| error
        ulp = np.spacing(np.abs(rr).astype(np.float32)).astype(np.float64)
        lim = 2.0 * np.sqrt(np.maximum(rr, 0.0)) * dy + dy * dy + PER_SAMPLE * ulp
        ratio = err / np.maximum(lim, 1e-300)
        worst = int(np.argmax(ratio)) if ratio.size else 0
        st.sample = max(st.sample, float(ratio[worst]) if ratio.size else 0.0)
        assert not ratio.size or ratio[worst] <= 1.0, (f"{label}: row {i} bin {worst} off by {err[worst]:.3e} "
                                                       f"> {lim[worst]:.3e}")
        st.rows += 1
    if label:
        print(f"{label}: {st.line()}", flush=True)
    return st
