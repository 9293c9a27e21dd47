"""Run records (CPU): the JSON-lines log's header and progress records, and
checkpoint files (plain arrays only, atomic replacement, no pickling on load)."""
import json
import os

import numpy as np
import pytest

from paper_2308_08410_amd import runlog


def test_log_header_and_records(tmp_path):
    path = str(tmp_path / "run.jsonl")
    log = runlog.RunLog(path, "inverse", dict(nodes=1000, starts=4), device=False)
    log.write(event="iteration", iteration=0, loss=np.array([1.5, 2.5], np.float32))
    log.write(event="iteration", iteration=10, loss=[0.5, 0.25])
    log.close(iters_per_s=3.0)
    recs = runlog.read_log(path)
    assert [r["event"] for r in recs] == ["start", "iteration", "iteration", "end"]
    h = recs[0]
    assert h["kind"] == "inverse" and h["config"] == dict(nodes=1000, starts=4)
    assert h["host"]["nproc"] == os.cpu_count() and "cpu_model" in h["host"]
    assert recs[1]["loss"] == [1.5, 2.5] and recs[2]["iteration"] == 10
    assert all(r["elapsed_s"] >= 0 for r in recs)
    # appending: a resumed run adds its own header
    runlog.RunLog(path, "inverse", dict(resumed=True), device=False).close()
    assert len(runlog.read_log(path)) == 6
    for line in open(path):
        json.loads(line)


def test_checkpoint_round_trip(tmp_path):
    path = str(tmp_path / "ck.npz")
    a = np.arange(7, dtype=np.float32)
    runlog.save_checkpoint(path, vscale=a, iteration=np.int64(12), hist=np.zeros((0, 2)))
    c = runlog.load_checkpoint(path)
    assert np.array_equal(c["vscale"], a) and c["vscale"].dtype == np.float32
    assert int(c["iteration"]) == 12 and c["hist"].shape == (0, 2)
    assert not os.path.exists(path + ".tmp")
    # overwrite keeps one file
    runlog.save_checkpoint(path, vscale=a + 1, iteration=np.int64(13), hist=np.zeros((1, 2)))
    assert int(runlog.load_checkpoint(path)["iteration"]) == 13
    with pytest.raises(TypeError):
        runlog.save_checkpoint(path, bad=np.array([object()], dtype=object))
    assert int(runlog.load_checkpoint(path)["iteration"]) == 13   # the old file survives
