"""Host side of the tuning parameters: validation, round trip, and loading a
tuned file (no GPU needed)."""
import json

import pytest

lms = pytest.importorskip("paper_2111_04289_amd.lms")
from paper_2111_04289_amd import autotune  # noqa: E402


def test_set_get_roundtrip_and_reset():
    lms.set_tuning(chunk_rows=4096, part_rows=8192, piece_rows=2048, grid_per_cu=3, lds_groups=1024)
    assert lms.get_tuning() == {"chunk_rows": 4096, "part_rows": 8192, "piece_rows": 2048, "grid_per_cu": 3,
                                "lds_groups": 1024}
    assert lms.pane_limit(4) == 1024
    lms.set_tuning()
    assert lms.get_tuning() == {"chunk_rows": 0, "part_rows": 0, "piece_rows": 0, "grid_per_cu": 0, "lds_groups": 0}


@pytest.mark.parametrize("bad", [dict(chunk_rows=-1), dict(piece_rows=512), dict(grid_per_cu=-2),
                                 dict(lds_groups=768), dict(lds_groups=4096), dict(lds_groups=512)])
def test_invalid_tuning_rejected(bad):
    with pytest.raises(lms.LmsError) as e:
        lms.set_tuning(**bad)
    assert e.value.code == lms.LMS_EINVAL
    assert lms.get_tuning()["chunk_rows"] == 0


def test_workspace_follows_tuning():
    import torch
    cols = [torch.zeros(1 << 20, dtype=torch.int64), torch.zeros(1 << 20, dtype=torch.int64)]
    w = lms.Window(0, 1000, 0, 0)
    base = lms.lms_window_agg_workspace(cols, 1, w, [(lms.COUNT, 0)])
    lms.set_tuning(chunk_rows=1024)  # more chunks: a larger histogram
    try:
        assert lms.lms_window_agg_workspace(cols, 1, w, [(lms.COUNT, 0)]) > base
    finally:
        lms.set_tuning()


def test_apply_loads_file(tmp_path):
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"sliding": {"params": {"chunk_rows": 8192, "part_rows": 0, "piece_rows": 4096,
                                                    "grid_per_cu": 0, "lds_groups": 0}}}))
    try:
        got = autotune.apply("sliding", str(p))
        assert got["chunk_rows"] == 8192 and lms.get_tuning()["piece_rows"] == 4096
        assert autotune.apply("batched", str(p)) is None
        assert lms.get_tuning() == {k: 0 for k in autotune.SPACE}
    finally:
        lms.set_tuning()
