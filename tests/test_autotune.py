"""The launch-shape tuner's host logic, on the CPU: the candidate set for a
shape, the choice of the fastest, its application to the simulation, and the
cache (written once, reused without timing, re-timed on request).  Timing
itself needs a GPU; here a fake simulation and a table of timings stand in
for it."""
import json

import synth
from paper_2205_07125_amd import autotune

CANDIDATES = autotune.candidates    # before any test replaces it


class FakeSim:
    def __init__(self, wl, tile_neurons=8192):
        self.wl = wl
        self.tile_neurons = tile_neurons
        self.applied = []

    def set_tuning(self, **kw):
        self.applied.append(dict(kw))


def test_candidates_batched_shape():
    """64 uneven partitions on 8 nodes, 711 tiles, 256 CUs: one block per
    tile or persistent grids of 256 and 512 blocks (768 is not fewer than the
    tiles), one to 16 receive blocks per node (32 would need 256 blocks for 8
    nodes), both receive forms: 3 x 6 x 2 candidates."""
    sim = FakeSim(synth.get_workload("batched"))
    tiles = -(-sim.wl.n_neurons // sim.tile_neurons)
    assert tiles == 711 and sim.wl.n_nodes == 8
    c = autotune.candidates(sim, cu_count=256)
    assert len(c) == 36
    assert {x["update_blocks"] for x in c} == {0, 256, 512}
    assert {x["recv_split"] for x in c} == {0, 1, 2, 4, 8, 16}
    assert {x["recv_merged"] for x in c} == {0, 1}
    assert len({tuple(sorted(x.items())) for x in c}) == 36
    # the defaults are a candidate
    assert {"update_blocks": 0, "recv_split": 0, "recv_merged": 0} in c


def test_candidates_many_nodes():
    """250 nodes leave one receive block per node at most: no split
    candidates; 611 tiles allow persistent grids of 256 and 512."""
    sim = FakeSim(synth.get_workload("paper_share"))
    c = autotune.candidates(sim, cu_count=256)
    assert {x["recv_split"] for x in c} == {0}
    assert {x["update_blocks"] for x in c} == {0, 256, 512}
    assert len(c) == 6


def _timings(sim, cand, steps, warmup, mode):
    # a made-up cost per candidate, least at (0, 16, 1)
    return (1.0 + cand["update_blocks"] / 1000.0 + abs(cand["recv_split"] - 16) / 100.0
            + (0.0 if cand["recv_merged"] else 0.05))


def test_tune_picks_fastest_and_caches(tmp_path, monkeypatch):
    sim = FakeSim(synth.get_workload("batched"))
    calls = []
    monkeypatch.setattr(autotune, "shape_key", lambda s: "fake-gpu|batched")
    monkeypatch.setattr(autotune, "candidates", lambda s: CANDIDATES(s, cu_count=256))

    def fake_time(s, cand, steps, warmup, mode):
        calls.append(dict(cand))
        return _timings(s, cand, steps, warmup, mode)

    monkeypatch.setattr(autotune, "time_candidate", fake_time)
    cache = str(tmp_path / "tuning.json")
    best = {"update_blocks": 0, "recv_split": 16, "recv_merged": 1}

    r = autotune.tune(sim, cache=cache)
    assert not r["cached"] and r["tuning"] == best
    assert len(calls) == 36 and len(r["timings"]) == 36
    assert sim.applied[-1] == best
    assert r["ms_per_step"] == min(t["ms_per_step"] for t in r["timings"])
    with open(cache) as fh:
        db = json.load(fh)
    key = "fake-gpu|batched|mode=0"
    assert list(db) == [key] and db[key]["tuning"] == best

    # the same shape again: applied from the cache, nothing timed
    calls.clear()
    sim2 = FakeSim(sim.wl)
    r2 = autotune.tune(sim2, cache=cache)
    assert r2["cached"] and r2["tuning"] == best and calls == []
    assert sim2.applied == [best]

    # another route mode is another entry; force re-times
    autotune.tune(sim2, mode=1, cache=cache)
    assert len(calls) == 36
    calls.clear()
    r3 = autotune.tune(sim2, cache=cache, force=True)
    assert not r3["cached"] and len(calls) == 36
    with open(cache) as fh:
        assert sorted(json.load(fh)) == [key, "fake-gpu|batched|mode=1"]


def test_tune_without_cache(monkeypatch):
    sim = FakeSim(synth.get_workload("tiny"))
    monkeypatch.setattr(autotune, "shape_key", lambda s: "k")
    monkeypatch.setattr(autotune, "candidates",
                        lambda s: [{"update_blocks": 0, "recv_split": r, "recv_merged": 1}
                                   for r in (0, 1, 2)])
    monkeypatch.setattr(autotune, "time_candidate",
                        lambda s, c, *a: {0: 2.0, 1: 1.5, 2: 3.0}[c["recv_split"]])
    r = autotune.tune(sim, cache=None)
    assert r["tuning"]["recv_split"] == 1 and not r["cached"]
    assert sim.applied[-1]["recv_split"] == 1
