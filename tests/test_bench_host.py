"""Host-side checks of the benchmark's contract (no GPU)."""
from __future__ import annotations

import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_measured_traffic_is_tied_to_the_device_sources(tmp_path, monkeypatch):
    b = _bench()
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(f))
    assert b.measured_traffic("heavy_items", "rmat20") is None  # no file
    rec = {"kernel": "heavy_items", "workload": "rmat20", "source_digest": b.source_digest(),
           "hbm_bytes_per_launch": 123456789}
    f.write_text(json.dumps(rec))
    assert b.measured_traffic("heavy_items", "rmat20") == 123456789
    assert b.measured_traffic("heavy_items", "rmat21") is None
    assert b.measured_traffic("merge_items", "rmat20") is None
    f.write_text(json.dumps(dict(rec, source_digest="0" * 64)))
    assert b.measured_traffic("heavy_items", "rmat20") is None  # sources changed since the counters


def test_source_digest_covers_the_product_kernels(tmp_path, monkeypatch):
    b = _bench()
    d0 = b.source_digest()
    assert len(d0) == 64 and d0 == b.source_digest()
    csrc = os.path.join(ROOT, "paper_2010_08526_amd", "csrc")
    names = sorted(n for n in os.listdir(csrc) if n.endswith((".hip", ".hpp")))
    assert "kernels.hip" in names and "device.hpp" in names
    # a copy of the sources: an edit to kernels.hip or a header changes the
    # digest, an edit to another translation unit does not
    pkg = tmp_path / "paper_2010_08526_amd" / "csrc"
    pkg.mkdir(parents=True)
    for n in names:
        (pkg / n).write_bytes(open(os.path.join(csrc, n), "rb").read())
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.source_digest() == d0
    (pkg / "prune.hip").write_text("// another translation unit\n")
    assert b.source_digest() == d0
    (pkg / "device.hpp").write_text("// a header\n")
    d1 = b.source_digest()
    assert d1 != d0
    (pkg / "kernels.hip").write_text("// the product kernels\n")
    assert b.source_digest() != d1



def test_default_run_covers_every_section():
    b = _bench()
    argv = sys.argv
    try:
        sys.argv = ["bench.py"]
        args = b._parse()
    finally:
        sys.argv = argv
    assert args.gpus == 1 and not args.no_extras
    assert set(args.extras.split(",")) == {"fwd_bwd", "batched", "layered", "bsweep", "prune", "aat", "sorted_output"}
    for name in args.extras.split(","):
        assert callable(getattr(b, name))
