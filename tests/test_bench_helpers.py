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

