"""The autotuner picks one of its candidates by measurement and caches it;
the variants it chooses between are bit-identical (checked in the hydro and
batch tests), so here only the selection and the cache are tested."""
import json

import pytest
import torch

from gpu_common import say
from paper_2607_20704_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_tune_tree_and_cache(tmp_path, monkeypatch):
    from paper_2607_20704_amd import api, autotune
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("RG_TUNE_CACHE", str(cache))
    w = I.sedov_amr(base=4, lmax=6, radius=0.2)
    D = api.DeviceTree(w.ijkl, w.bc)
    u = D.to_key_order(w.u.reshape(-1, 5))
    best, times = autotune.tune_tree(D, u, w.gamma, api.RG_MIXED, reps=2)
    say("tree tuning", best, times)
    cands = autotune.tree_candidates(api.RG_MIXED)
    assert best in cands and set(times) == set(cands)
    entry = json.loads(cache.read_text())
    assert len(entry) == 1 and list(entry.values())[0]["best"] == list(best)
    again, t2 = autotune.tune_tree(D, u, w.gamma, api.RG_MIXED)
    assert again == best and t2 == {}


def test_tune_batch(tmp_path, monkeypatch):
    from paper_2607_20704_amd import api, autotune
    monkeypatch.setenv("RG_TUNE_CACHE", "off")
    boxes = I.batched_boxes(nbox=4, nsteps=2, base_range=(3, 4), extra_range=(0, 1))
    trees = [api.DeviceTree(b.ijkl, b.bc) for b in boxes]
    states = [D.to_key_order(b.u.reshape(-1, 5)) for D, b in zip(trees, boxes)]
    cands = autotune.BATCH_CANDIDATES[:4]
    best, times = autotune.tune_batch(trees, states, [b.gamma for b in boxes], [b.cfl for b in boxes],
                                      api.RG_FP64, reps=2, candidates=cands)
    torch.cuda.synchronize()
    say("batch tuning", best, times)
    assert best in cands and set(times) == set(cands)
