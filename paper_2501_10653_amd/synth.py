"""Seeded synthetic radio-image pairs for the tile-wise LISI / augLISI path.

The paper evaluates on two CLEAN-restored sky images of the same field: the
first holds 33 sources, the second the same field with 5 low-intensity sources
gone (Section 3, data simulation).  The simulated measurement sets are not
available, so this module draws stand-ins of the same shape and structure:
beam-convolved point sources with log-uniform amplitudes on Gaussian noise,
and a second image that drops the faintest sources and redraws the noise.

This module is input generation only.  It holds none of the similarity
arithmetic and is shared, unchanged, by the HIP path and by the CPU oracle.
All randomness comes from numpy's PCG64 seeded by ``(seed, stream)`` tuples, so
a given seed yields byte-identical images on every machine.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

FWHM_TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))

# Stream ids inside one seed: independent generators for each random draw.
_STREAM_SOURCES = 0
_STREAM_NOISE_A = 1
_STREAM_NOISE_B = 2
_STREAM_DROP = 3


@dataclasses.dataclass(frozen=True)
class PairSpec:
    """Recipe for one snapshot / reference image pair.

    ``n_drop`` faintest sources of image A are absent from image B; with
    ``n_drop == 0`` the pair differs only by its noise realisation.
    """

    N: int
    NT: int
    n_src: int
    amp_lo: float
    amp_hi: float
    fwhm: float
    noise_sigma: float
    n_drop: int
    seed: int

    def bytes_per_pair(self) -> int:
        return 8 * self.N * self.N


# Constants of the similarity indices: the paper only requires them to be much
# smaller than one; 1e-6 is used for every workload.
C_DEFAULT = 1e-6


def scaled_count(base: int, N: int, minimum: int = 0) -> int:
    """Source counts scale with image area relative to a 2048 x 2048 field."""
    return max(minimum, int(round(base * (N / 2048.0) ** 2)))


def spec_small(seed: int = 0) -> PairSpec:
    """256 x 256 pair with 32 x 32 tiles (8 x 8 IQA matrix): 10 sources of
    amplitude 1e-3..1, beam FWHM 3 px, noise sigma 1e-4, B drops the 2 faintest."""
    return PairSpec(N=256, NT=32, n_src=10, amp_lo=1e-3, amp_hi=1.0, fwhm=3.0,
                    noise_sigma=1e-4, n_drop=2, seed=seed)


def spec_paper_shape(seed: int = 1) -> PairSpec:
    """The paper's shape: 2048 x 2048 with 64 x 64 tiles (32 x 32 IQA matrix),
    33 sources (amplitude 1e-3..2, FWHM 4 px) on sigma=1e-4 noise, B drops the
    5 faintest -- mirroring the 33-source / 5-removed simulated pair."""
    return PairSpec(N=2048, NT=64, n_src=33, amp_lo=1e-3, amp_hi=2.0, fwhm=4.0,
                    noise_sigma=1e-4, n_drop=5, seed=seed)


def spec_sweep(N: int, NT: int) -> PairSpec:
    """One cell of the N x N_T size sweep: the paper-shape recipe with the
    source and dropped counts scaled by area."""
    return PairSpec(N=N, NT=NT, n_src=scaled_count(33, N, 1), amp_lo=1e-3,
                    amp_hi=2.0, fwhm=4.0, noise_sigma=1e-4,
                    n_drop=scaled_count(5, N, 1), seed=1000 * N + NT)


SWEEP_N = (1024, 2048, 4096, 8192)
SWEEP_NT = (16, 32, 64, 128, 256)


def _source_list(spec: PairSpec) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Sub-pixel positions (row, col) and log-uniform amplitudes, sorted from
    faintest to brightest.  Positions stay 3 beam sigmas inside the edges."""
    rng = np.random.default_rng((spec.seed, _STREAM_SOURCES))
    sig = spec.fwhm * FWHM_TO_SIGMA
    margin = min(3.0 * sig, (spec.N - 1) / 2.0)
    rows = rng.uniform(margin, spec.N - 1 - margin, spec.n_src)
    cols = rng.uniform(margin, spec.N - 1 - margin, spec.n_src)
    amps = np.exp(rng.uniform(math.log(spec.amp_lo), math.log(spec.amp_hi), spec.n_src))
    order = np.argsort(amps, kind="stable")
    return rows[order], cols[order], amps[order]


def render_sources(N: int, rows: Sequence[float], cols: Sequence[float],
                   amps: Sequence[float], fwhm: float) -> np.ndarray:
    """Peak-normalised Gaussian beams (Jy/beam convention) summed in float64.
    Each beam is evaluated on a window of +-6 sigma around its centre."""
    img = np.zeros((N, N), dtype=np.float64)
    sig = fwhm * FWHM_TO_SIGMA
    rad = int(math.ceil(6.0 * sig))
    inv2s2 = 1.0 / (2.0 * sig * sig)
    for r0, c0, a in zip(rows, cols, amps):
        ir, ic = int(round(r0)), int(round(c0))
        r_lo, r_hi = max(0, ir - rad), min(N, ir + rad + 1)
        c_lo, c_hi = max(0, ic - rad), min(N, ic + rad + 1)
        rr = (np.arange(r_lo, r_hi) - r0)[:, None]
        cc = (np.arange(c_lo, c_hi) - c0)[None, :]
        img[r_lo:r_hi, c_lo:c_hi] += a * np.exp(-(rr * rr + cc * cc) * inv2s2)
    return img


def _noise(N: int, sigma: float, seed: int, stream: int) -> np.ndarray:
    rng = np.random.default_rng((seed, stream))
    return rng.standard_normal((N, N), dtype=np.float64) * sigma


def make_pair(spec: PairSpec) -> Tuple[np.ndarray, np.ndarray, Dict]:
    """Return ``(x, y, meta)``: float32 C-contiguous N x N images.

    ``x`` is the earlier observation (all sources), ``y`` the later one with
    the ``n_drop`` faintest sources removed and independent noise.  ``meta``
    lists the sources and which ones were dropped.
    """
    rows, cols, amps = _source_list(spec)
    keep = np.arange(spec.n_src) >= spec.n_drop   # sorted faintest first
    x = render_sources(spec.N, rows, cols, amps, spec.fwhm)
    y = render_sources(spec.N, rows[keep], cols[keep], amps[keep], spec.fwhm)
    x += _noise(spec.N, spec.noise_sigma, spec.seed, _STREAM_NOISE_A)
    y += _noise(spec.N, spec.noise_sigma, spec.seed, _STREAM_NOISE_B)
    meta = {
        "spec": dataclasses.asdict(spec),
        "rows": rows, "cols": cols, "amps": amps,
        "dropped": np.nonzero(~keep)[0],
    }
    return (np.ascontiguousarray(x, dtype=np.float32),
            np.ascontiguousarray(y, dtype=np.float32), meta)


def ragged_specs(count: int = 256, seed: int = 7,
                 Ns: Sequence[int] = (512, 1024, 2048, 4096),
                 NTs: Sequence[int] = (32, 64, 128),
                 frac_transient: float = 0.2) -> List[PairSpec]:
    """Ragged batch recipe: N and N_T drawn uniformly per pair; a fraction of
    the pairs lose 1..5 of their faintest sources, the rest change only by noise."""
    rng = np.random.default_rng((seed, _STREAM_DROP))
    out = []
    for i in range(count):
        N = int(rng.choice(Ns))
        NT = int(rng.choice(NTs))
        transient = rng.uniform() < frac_transient
        n_src = scaled_count(33, N, 1)
        n_drop = int(min(n_src, rng.integers(1, 6))) if transient else 0
        out.append(PairSpec(N=N, NT=NT, n_src=n_src, amp_lo=1e-3, amp_hi=2.0,
                            fwhm=4.0, noise_sigma=1e-4, n_drop=n_drop,
                            seed=seed * 100003 + i))
    return out


def random_pair(N: int, rng: np.random.Generator, neg_frac: float = 0.3,
                nan_frac: float = 0.0, scale: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """Unstructured stress inputs: uniform values with a chosen fraction of
    negative pixels (and optionally NaN blanks), for edge-case tests."""
    x = rng.uniform(0.0, scale, (N, N))
    y = rng.uniform(0.0, scale, (N, N))
    x[rng.uniform(size=(N, N)) < neg_frac] *= -1.0
    y[rng.uniform(size=(N, N)) < neg_frac] *= -1.0
    if nan_frac > 0:
        x[rng.uniform(size=(N, N)) < nan_frac] = np.nan
        y[rng.uniform(size=(N, N)) < nan_frac] = np.nan
    return x.astype(np.float32), y.astype(np.float32)


_STREAM_TRANSIENT = 20


def bright_transient_pair(N: int = 2048, NT: int = 64, amp: float = 8.0,
                          seed: int = 21) -> Tuple[np.ndarray, np.ndarray, Dict]:
    """The paper-shape field in both images (independent noise, no source
    removed) plus one bright source of amplitude `amp` (FWHM 4 px, well above
    the field's brightest at 2) in the first image only.  In the tiles around
    it P/(Sx+Sy+C) exceeds 1/2, the regime in which augLISI = 1 - P/(Sx+Sy+C)
    loses relative accuracy."""
    base = PairSpec(N=N, NT=NT, n_src=scaled_count(33, N, 1), amp_lo=1e-3, amp_hi=2.0,
                    fwhm=4.0, noise_sigma=1e-4, n_drop=0, seed=seed)
    x, y, meta = make_pair(base)
    rng = np.random.default_rng((seed, _STREAM_TRANSIENT))
    sig = base.fwhm * FWHM_TO_SIGMA
    r0, c0 = rng.uniform(3 * sig, N - 1 - 3 * sig, 2)
    x = np.ascontiguousarray(
        x.astype(np.float64) + render_sources(N, [r0], [c0], [amp], base.fwhm), dtype=np.float32)
    meta = dict(meta, transient=(float(r0), float(c0), float(amp)))
    return x, y, meta


_STREAM_SNAPSHOT = 10


def serving_references(count: int = 16, Ns: Sequence[int] = (1024, 2048, 4096),
                       seed: int = 11) -> List[PairSpec]:
    """Resident references for the serving workload: N assigned round-robin
    over Ns; each reference is the all-sources image of a pair whose later
    snapshots lose the faintest sources (scaled by area, at least one)."""
    out = []
    for r in range(count):
        N = int(Ns[r % len(Ns)])
        out.append(PairSpec(N=N, NT=64, n_src=scaled_count(33, N, 1), amp_lo=1e-3, amp_hi=2.0,
                            fwhm=4.0, noise_sigma=1e-4, n_drop=scaled_count(5, N, 1),
                            seed=seed * 1000 + r))
    return out


def make_snapshot(spec: PairSpec, k: int) -> np.ndarray:
    """Snapshot k of a reference: the kept sources re-rendered with noise from
    an independent stream per k (the reference itself is make_pair(spec)[0])."""
    rows, cols, amps = _source_list(spec)
    keep = np.arange(spec.n_src) >= spec.n_drop
    img = render_sources(spec.N, rows[keep], cols[keep], amps[keep], spec.fwhm)
    img += _noise(spec.N, spec.noise_sigma, spec.seed, _STREAM_SNAPSHOT + k)
    return np.ascontiguousarray(img, dtype=np.float32)


def poisson_arrivals(rate: float, count: int, seed: int = 0) -> np.ndarray:
    """Open-loop arrival times (ns from the start) of a Poisson process."""
    rng = np.random.default_rng((seed, 77))
    gaps = rng.exponential(1.0 / rate, count)
    return np.cumsum(gaps * 1e9).astype(np.int64)
