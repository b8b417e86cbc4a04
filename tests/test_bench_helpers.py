"""Host logic of bench.py (no GPU): the HBM traffic figures it reports come
from committed rocprofv3 summaries only when they were taken with the
current kernel sources, matched by kernel name without template arguments."""
import hashlib
import os

import bench


def _sha():
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        with open(os.path.join(bench.ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def test_traffic_lookup_matches_template_instances_and_source_hash(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = _sha()
    (prof / "x.md").write_text(f"```\ntraffic k_raycast<true> {sha} 1234\ntraffic k_integrate 0123456789abcdef 99\n```\n")
    real_root = bench.ROOT
    for f in bench.KERNEL_SOURCES:   # the hashed sources, seen from the temporary root
        dst = tmp_path / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_bytes(open(os.path.join(real_root, f), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_raycast") == 1234
    assert bench.measured_traffic("k_integrate") is None      # taken with other sources
    assert bench.measured_traffic("k_alloc_rays") is None     # not in any summary



def test_traffic_lookup_needs_the_same_timed_frames(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = _sha()
    (prof / "x.md").write_text(f"traffic k_raycast {sha} 555 frames=280-299\n"
                               f"traffic k_integrate {sha} 777 frames=30-299\n")
    real_root = bench.ROOT
    for f in bench.KERNEL_SOURCES:
        dst = tmp_path / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_bytes(open(os.path.join(real_root, f), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_raycast", (280, 299)) == 555
    assert bench.measured_traffic("k_raycast", (30, 299)) is None
    assert bench.measured_traffic("k_integrate", (30, 299)) == 777
    assert bench.measured_traffic("k_raycast") is None        # a range-keyed figure needs a range


def test_schedule_fuses_the_whole_trajectory_and_times_its_end():
    pre, order = bench.c2_schedule(5, 20)
    assert pre == 275 and order == list(range(300))
    assert order[pre + 5] == 280 and order[-1] == 299
    pre, order = bench.c2_schedule(30, 270)
    assert pre == 0 and order[30] == 30 and order[-1] == 299
    pre, order = bench.c2_schedule(100, 300)       # more frames than the trajectory: wraps
    assert pre == 0 and len(order) == 400 and order[300] == 0 and order[-1] == 99
