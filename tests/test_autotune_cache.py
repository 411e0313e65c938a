"""Autotuner result cache (host logic only, no GPU)."""

import json

import numpy as np
import pytest
import torch

import paper_2408_02367_amd as sdn


def test_key_depends_on_trajectory_shape_and_minibatch():
    t = np.random.default_rng(0).uniform(-3, 3, (100, 3)).astype(np.float32)
    k0 = sdn.tune_key(t, (8, 8, 8), 4, 5)
    assert k0 == sdn.tune_key(t.copy(), (8, 8, 8), 4, 5)
    t2 = t.copy()
    t2[17, 1] += 1e-3
    assert sdn.tune_key(t2, (8, 8, 8), 4, 5) != k0
    assert sdn.tune_key(t, (8, 8, 9), 4, 5) != k0
    assert sdn.tune_key(t, (8, 8, 8), 2, 5) != k0
    assert sdn.tune_key(t, (8, 8, 8), 4, 5, frame_of_point=np.zeros(100, np.int32)) != k0


def test_cache_hit_returns_stored_options_without_tuning(tmp_path, monkeypatch):
    t = np.random.default_rng(1).uniform(-3, 3, (50, 3)).astype(np.float32)
    monkeypatch.setattr(torch.cuda, "current_device", lambda: 0)
    monkeypatch.setattr(torch.cuda, "get_device_name", lambda dev=None: "testdev")
    key = sdn.tune_key(torch.as_tensor(t), (8, 8, 8), 4, 5, device_name="testdev")
    stored = {"tile": 8, "max_points_per_item": 1024, "spread_engine": "gather", "ms": 1.5}
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({key: stored}))

    def boom(*a, **k):
        raise AssertionError("the tuner must not run on a cache hit")
    monkeypatch.setattr(sdn, "lib", boom)
    assert sdn.autotune(t, (8, 8, 8), 4, 5, cache=str(path)) == stored
