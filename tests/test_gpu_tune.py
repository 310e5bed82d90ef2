"""The autotuner times every launch configuration and leaves a valid, loadable choice."""
import pytest

import paper_2212_05098_amd as utfx
from paper_2212_05098_amd import tune

pytestmark = pytest.mark.gpu


def test_tuner_small_run(tmp_path):
    with utfx.Context() as ctx:
        cache = tune.tune(ctx, size_mib=1, reps=1, log=lambda m: None)
        path = str(tmp_path / "tune.json")
        tune.save(cache, path)
    assert set(cache["ops"]) == {str(op) for op in range(6)}
    for op, (tile, seg, wgs) in cache["ops"].items():
        assert (tile, seg) in tune.CANDIDATES[int(op)]
    with utfx.Context() as ctx2:
        assert ctx2.load_tuning(path)
        for op, v in cache["ops"].items():
            assert list(ctx2.get_tuning(int(op))) == v
