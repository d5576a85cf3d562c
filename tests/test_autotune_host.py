"""Host logic of the sweep autotuner: per-shape cache, one timing per shape."""
import json

from paper_2104_01284_amd import autotune
from paper_2104_01284_amd import instances as ins


def test_cache_times_each_shape_once(tmp_path, monkeypatch):
    import torch
    calls = []

    def fake_tune(inst, device=0, full=False, **kw):
        calls.append(inst["name"])
        return {"kernel": 2, "tile": 8, "ms": 1.0, "all": {"2/8": 1.0}}

    monkeypatch.setattr(autotune, "tune", fake_tune)
    monkeypatch.setattr(torch.cuda, "get_device_name", lambda d=0: "testdev")
    path = str(tmp_path / "tune.json")
    a, b = ins.plain(), ins.paper_shape()
    opts = autotune.tuned_options([a, b, a], cache_path=path)
    assert opts == [(2, 8, 0, 0)] * 3
    assert calls == [a["name"], b["name"]]
    with open(path) as f:
        cache = json.load(f)
    assert autotune.shape_key(a, "testdev") in cache and autotune.shape_key(b, "testdev") in cache
    autotune.tuned_options([b, a], cache_path=path)
    assert len(calls) == 2


def test_shape_key_distinguishes_grids():
    a = ins.plain()
    b = dict(a)
    b["t_grid"] = (0.0, 90.0, 32)
    assert autotune.shape_key(a, "d") != autotune.shape_key(b, "d")
    assert autotune.shape_key(a, "d") != autotune.shape_key(a, "e")


def test_batch_tuned_once_per_batch_of_shapes(tmp_path, monkeypatch):
    """A batch is timed once per (device, shapes of its members) and every
    member gets the winning tile."""
    import torch
    calls = []

    def fake_tune_batch(insts, device=0, **kw):
        calls.append(len(insts))
        return {"tile": 4, "ms": 1.0, "all": {"8": 2.0, "4": 1.0}}

    monkeypatch.setattr(autotune, "tune_batch", fake_tune_batch)
    monkeypatch.setattr(torch.cuda, "get_device_name", lambda d=0: "testdev")
    path = str(tmp_path / "tune.json")
    batch = [ins.plain(), ins.paper_shape()]
    assert autotune.tuned_batch_options(batch, cache_path=path) == [(0, 4, 0, 0)] * 2
    assert autotune.tuned_batch_options(batch, cache_path=path) == [(0, 4, 0, 0)] * 2
    assert calls == [2]
    other = [ins.paper_shape(), ins.plain()]
    assert autotune.batch_key(batch, "d") != autotune.batch_key(other, "d")
