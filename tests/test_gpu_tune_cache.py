"""Persisted autotune choices (MDS_TUNE_CACHE): a plan tuned on its D
records its split-K choice; a new plan of the same key starts from it, runs
the same configuration (bit-identical result) and reports where its splits
came from; another key is not affected; a corrupt line is ignored."""
import os

import numpy as np
import pytest

import workloads as W
from gpu_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1803_02272_amd as mds  # noqa: E402


def test_autotune_choice_is_recorded_and_reused(tmp_path, monkeypatch):
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("MDS_TUNE_CACHE", str(path))
    reads, _ = W.amplicon_reads(6000, 20, seed=3)
    D = torch.from_numpy(W.hamming_distances(reads)).cuda()
    n, k, p, q = 6000, 30, 10, 2
    a = mds.Plan(n, k, p, q, 0, form="bf16")
    assert a.info()["tuned_from_cache"] == 0
    t = a.autotune(D)
    say(f"[tune cache] tuned {t}")
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split()[-4:] == [str(t["range_split"]), str(t["proj_split"]),
                                                         str(t["write_split"]), str(t["f32_split"])]
    ca, ea = a.run(D)
    b = mds.Plan(n, k, p, q, 0, form="bf16")
    ib = b.info()
    assert ib["tuned_from_cache"] == 1 and ib["gpass_split"] == a.info()["gpass_split"]
    cb, eb = b.run(D)
    assert torch.equal(ea, eb) and torch.equal(ca, cb)
    # another key (other q) starts from the defaults; a corrupt line is skipped
    with open(path, "a") as f:
        f.write("garbage line\n")
    c = mds.Plan(n, k, p, 1, 0, form="bf16")
    assert c.info()["tuned_from_cache"] == 0
    d = mds.Plan(n, k, p, q, 0, form="bf16")
    assert d.info()["tuned_from_cache"] == 1
    # re-tuning the same key replaces its line
    d.autotune(D)
    recs = [l for l in path.read_text().splitlines() if not l.startswith("garbage")]
    assert len(recs) == 1
    monkeypatch.delenv("MDS_TUNE_CACHE")
    e = mds.Plan(n, k, p, q, 0, form="bf16")
    assert e.info()["tuned_from_cache"] == 0
    for pl in (a, b, c, d, e):
        pl.close()
