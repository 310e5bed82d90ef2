"""The autotuner times every launch configuration (including the residency cap and the
batched call's tunables) and leaves a valid, loadable choice, keyed by the GPU."""
import pytest

import paper_2212_05098_amd as utfx
from paper_2212_05098_amd import tune

pytestmark = pytest.mark.gpu


def test_tuner_small_run(tmp_path):
    with utfx.Context() as ctx:
        entry = tune.tune(ctx, size_mib=1, reps=1, log=lambda m: None, batch_strings=2000)
        path = str(tmp_path / "tune.json")
        tune.save(entry, path)
    assert entry["key"] == tune.device_key()
    assert set(entry["ops"]) == {str(op) for op in range(6)}
    for op, (tile, seg, wgs) in entry["ops"].items():
        assert (tile, seg) in tune.CANDIDATES[int(op)] and wgs in tune.WGS
    assert tuple(entry["batch"]) in tune.BATCH_CANDIDATES
    with utfx.Context() as ctx2:
        assert ctx2.load_tuning(path)
        for op, v in entry["ops"].items():
            assert list(ctx2.get_tuning(int(op))) == v
        assert list(ctx2.get_batch_tuning()) == entry["batch"]
    assert tune.load(path, key="no such gpu") is None
