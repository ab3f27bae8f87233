"""Pack-size tuner: argument checks and the cache key (host logic, no GPU)."""
import numpy as np
import pytest

from paper_2606_28394_amd import autotune as A
from paper_2606_28394_amd import workloads as W


@pytest.fixture(scope="module")
def scene():
    return W.tilted_towers(3, 6, seed=5, n_steps=2)


def test_key_is_stable_and_tracks_the_batch(scene):
    k = A.batch_key(scene, 0, (0, 64), 40, 60, "dev")
    assert k == A.batch_key(scene, 0, (0, 64), 40, 60, "dev")
    assert k != A.batch_key(scene, 1, (0, 64), 40, 60, "dev")
    assert k != A.batch_key(scene, 0, (0, 80), 40, 60, "dev")
    assert k != A.batch_key(scene, 0, (0, 64), 41, 60, "dev")
    assert k != A.batch_key(scene, 0, (0, 64), 40, 60, "other")
    other = dict(scene, mu=np.asarray(scene["mu"]) * 1.5)
    assert k != A.batch_key(other, 0, (0, 64), 40, 60, "dev")
    fewer = W.tilted_towers(3, 5, seed=5, n_steps=2)
    assert k != A.batch_key(fewer, 0, (0, 64), 40, 60, "dev")


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    A._store(path, "a", {"pack_bodies": 64})
    A._store(path, "b", {"pack_bodies": 0})
    assert A._load(path) == {"a": {"pack_bodies": 64}, "b": {"pack_bodies": 0}}
    assert A._load(str(tmp_path / "missing.json")) == {}


@pytest.mark.parametrize("kw", [dict(candidates=()), dict(candidates=(0, 300)), dict(candidates=(-1,)),
                                dict(steps=0), dict(lead_in=-1)])
def test_bad_arguments_are_rejected(scene, kw):
    with pytest.raises(ValueError):
        A.tune_pack_bodies(scene, **kw)


def test_needs_a_gpu(scene):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        A.tune_pack_bodies(scene, candidates=(0,), steps=1, lead_in=0)
