"""Host-side logic of the autotuner and of the build step that compiles its
results in: candidate shapes are valid, and the generated table holds
exactly what the JSON cache says."""

from __future__ import annotations

import json

import pytest

from paper_2501_10653_amd import build, tune
from paper_2501_10653_amd.iqa import check_cfg


@pytest.mark.parametrize("N,NT", tune.SWEEP + tune.EXTRA)
def test_single_candidates_are_valid_and_varied(N, NT):
    cands = tune.candidates_single(N, NT)
    assert cands, (N, NT)
    for c in cands:
        assert check_cfg(N, NT, c) == 0, c
        assert c["vec"] == 4
    # the search covers more than one wave count and row-phase count
    assert len({c["waves"] for c in cands}) > 1
    assert len({(c["rp"], c["ksplit"]) for c in cands}) > 1


@pytest.mark.parametrize("NT", [32, 64, 128])
def test_batch_candidates_follow_the_batch_rules(NT):
    cands = tune.candidates_batch(NT)
    assert cands
    for c in cands:
        # batch geometry: vec 4, one wave per tile group or four splitting its
        # rows, no split across workgroups, unroll 8
        assert (c["vec"], c["ksplit"], c["unroll"]) == (4, 1, 8) and c["waves"] in (1, 4)
        assert check_cfg(4096, NT, c) == 0, c
    assert {c["waves"] for c in cands} == {1, 4}


def test_tuned_table_matches_the_json_cache(tmp_path):
    doc = {
        "single": {"2048x64": {"cfg": dict(vec=4, waves=4, unroll=8, seg=16, rp=2, ksplit=1)},
                   "1024x256": {"cfg": dict(vec=4, waves=4, unroll=8, seg=64, rp=1, ksplit=8)}},
        "batch": {"64": dict(vec=4, waves=1, unroll=8, seg=16, rp=2, ksplit=1)},
        "serve": {"1024x64": dict(vec=4, waves=4, unroll=8, seg=16, rp=2, ksplit=1)},
        "batch_waves": 4096,
    }
    src = tmp_path / "cache.json"
    src.write_text(json.dumps(doc))
    inc = tmp_path / "table.inc"
    assert build.write_tuned_table(str(src), str(inc)) == 4
    text = inc.read_text()
    assert "{1024, 256, 0, {4, 4, 8, 64, 1, 8}}," in text
    assert "{2048, 64, 0, {4, 4, 8, 16, 2, 1}}," in text
    assert "{0, 64, 1, {4, 1, 8, 16, 2, 1}}," in text
    assert "{1024, 64, 2, {4, 4, 8, 16, 2, 1}}," in text
    assert "kTunedCount = 4;" in text and "kTunedBatchWaves = 4096;" in text
    # no cache: an empty table that still compiles
    empty = tmp_path / "empty.inc"
    assert build.write_tuned_table(str(tmp_path / "missing.json"), str(empty)) == 0
    assert "kTunedCount = 0;" in empty.read_text()


def test_committed_cache_entries_are_valid():
    with open(build.TUNED_JSON) as fh:
        doc = json.load(fh)
    for key, rec in doc["single"].items():
        N, NT = (int(v) for v in key.split("x"))
        assert check_cfg(N, NT, rec["cfg"]) == 0, key
    for NT, cfg in doc["batch"].items():
        assert check_cfg(4096, int(NT), cfg) == 0, NT
    for key, cfg in doc.get("serve", {}).items():
        N, NT = (int(v) for v in key.split("x"))
        assert check_cfg(N, NT, cfg) == 0, key
        assert cfg["waves"] in (1, 4) and cfg["ksplit"] == 1 and cfg["unroll"] == 8, key
    assert doc["batch_waves"] >= 4 and doc["batch_waves"] % 4 == 0


def test_serving_geometry_covers_the_served_shapes():
    """The compiled-in serving table has an entry for every shape the server's
    tuner covers, and the Python helper reports what the library uses."""
    from paper_2501_10653_amd.serve import serve_cfg
    with open(build.TUNED_JSON) as fh:
        doc = json.load(fh)
    for N, NT in tune.SERVE_SHAPES:
        key = f"{N}x{NT}"
        assert key in doc.get("serve", {}), key
        assert serve_cfg(N, NT) == {k: int(v) for k, v in doc["serve"][key].items()}, key


def test_batch_entries_outside_the_batch_geometry_are_refused(tmp_path):
    """A hand-edited cache with a batch or server entry the batch kernel cannot
    run (two waves per tile group, a row split, unroll 4) does not build, and
    the library refuses the same entry at run time."""
    import ctypes
    import pytest
    from paper_2501_10653_amd import _lib
    from paper_2501_10653_amd._lib import LaunchCfg
    good = dict(vec=4, waves=1, unroll=8, seg=16, rp=2, ksplit=1)
    for bad in (dict(good, waves=2), dict(good, ksplit=2), dict(good, unroll=4),
                dict(good, vec=2)):
        for section, key in (("batch", "64"), ("serve", "1024x64")):
            src = tmp_path / "cache.json"
            src.write_text(json.dumps({section: {key: bad}}))
            with pytest.raises(ValueError):
                build.write_tuned_table(str(src), str(tmp_path / "t.inc"))
        assert _lib.load().iqa_tune_set(1024, 64, _lib.TUNE_BATCH,
                                        ctypes.byref(LaunchCfg.from_dict(bad))) == 6
