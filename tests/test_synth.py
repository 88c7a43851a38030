"""The seeded input generators: deterministic, and the recipes have the
shapes and structure the workloads state."""

from __future__ import annotations

import numpy as np

from paper_2501_10653_amd import synth


def test_same_seed_same_bytes():
    a = synth.make_pair(synth.spec_small())
    b = synth.make_pair(synth.spec_small())
    assert a[0].tobytes() == b[0].tobytes() and a[1].tobytes() == b[1].tobytes()
    c = synth.make_pair(synth.spec_small(seed=3))
    assert a[0].tobytes() != c[0].tobytes()


def test_paper_shape_recipe():
    x, y, meta = synth.make_pair(synth.spec_paper_shape())
    assert x.shape == (2048, 2048) and x.dtype == np.float32 and x.flags.c_contiguous
    amps = meta["amps"]
    assert len(amps) == 33 and np.all(np.diff(amps) >= 0)
    assert 1e-3 <= amps.min() and amps.max() <= 2.0
    # the 5 faintest are the ones dropped
    assert list(meta["dropped"]) == [0, 1, 2, 3, 4]
    # negatives are present (noise), and the brightest peak is near its amplitude
    assert (x < 0).mean() > 0.3
    assert abs(x.max() - amps.max()) < 0.05 * amps.max()
    # y lacks the dropped sources: at the faintest source, x - y ~ its amplitude
    r, c = int(round(meta["rows"][4])), int(round(meta["cols"][4]))
    assert x[r, c] - y[r, c] > 0.3 * amps[4]


def test_sweep_counts_scale_with_area():
    assert [synth.spec_sweep(N, 64).n_src for N in synth.SWEEP_N] == [8, 33, 132, 528]
    assert [synth.spec_sweep(N, 64).n_drop for N in synth.SWEEP_N] == [1, 5, 20, 80]


def test_ragged_recipe():
    specs = synth.ragged_specs(count=256, seed=7)
    assert len(specs) == 256
    assert {s.N for s in specs} == {512, 1024, 2048, 4096}
    assert {s.NT for s in specs} == {32, 64, 128}
    frac = np.mean([s.n_drop > 0 for s in specs])
    assert 0.1 < frac < 0.3
    assert all(1 <= s.n_drop <= 5 for s in specs if s.n_drop)


def test_serving_recipe():
    refs = synth.serving_references()
    assert len(refs) == 16 and [r.N for r in refs].count(1024) == 6
    s0 = synth.make_snapshot(refs[0], 0)
    s1 = synth.make_snapshot(refs[0], 1)
    assert s0.shape == (1024, 1024) and s0.tobytes() != s1.tobytes()
    t = synth.poisson_arrivals(10000, 5000, seed=2)
    assert np.all(np.diff(t) >= 0)
    assert abs(5000 / (t[-1] / 1e9) - 10000) < 600


def test_bright_transient_pair_is_seeded_and_only_in_the_first_image():
    x1, y1, m1 = synth.bright_transient_pair(256, 32, amp=8.0, seed=4)
    x2, y2, m2 = synth.bright_transient_pair(256, 32, amp=8.0, seed=4)
    assert x1.dtype == np.float32 and x1.shape == (256, 256) and x1.flags.c_contiguous
    assert np.array_equal(x1, x2) and np.array_equal(y1, y2)
    r0, c0, amp = m1["transient"]
    i, j = int(round(r0)), int(round(c0))
    # the transient's peak stands in the first image only
    assert x1[i, j] - y1[i, j] > 0.5 * amp
    far = (abs(np.arange(256)[:, None] - r0) > 20) | (abs(np.arange(256)[None, :] - c0) > 20)
    assert np.abs(x1 - y1)[far].max() < 0.05
