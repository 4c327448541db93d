"""bench.py's HBM-traffic records (the `traffic-record:` lines of the profile
summaries): each parses, its byte count is its two counters scaled by the
copy calibration, and the lookup returns it only for the kernel it names and
only while that kernel's source still has the recorded hash."""
import glob
import hashlib
import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KEYS = ("kernel", "workload", "bytes_per_launch", "fetch_kib_per_dispatch", "write_kib_per_dispatch",
        "fetch_scale", "write_scale", "source", "source_sha256")


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _records():
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if line.startswith("traffic-record:"):
                yield path, json.loads(line.split(":", 1)[1])


def test_records_parse_and_add_up():
    recs = list(_records())
    assert recs, "no traffic records under profiles/"
    for path, r in recs:
        missing = [k for k in KEYS if k not in r]
        assert not missing, (path, missing)
        assert os.path.exists(os.path.join(ROOT, r["source"])), (path, r["source"])
        total = (r["fetch_kib_per_dispatch"] * 1024 * r["fetch_scale"] +
                 r["write_kib_per_dispatch"] * 1024 * r["write_scale"])
        # the KiB figures are stored to 0.1 KiB
        assert abs(total - r["bytes_per_launch"]) <= 1e-6 * total + 1024, (path, total, r["bytes_per_launch"])


def test_lookup_follows_kernel_name_and_source_hash(tmp_path, monkeypatch):
    b = _bench()
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel v1")
    (tmp_path / "profiles").mkdir()
    rec = {"kernel": "k<1>", "workload": "w", "bytes_per_launch": 123, "fetch_kib_per_dispatch": 0.0,
           "write_kib_per_dispatch": 0.0, "fetch_scale": 2.0, "write_scale": 1.0, "source": "k.hip",
           "source_sha256": hashlib.sha256(b"kernel v1").hexdigest()}
    (tmp_path / "profiles" / "k.md").write_text("# k\n\ntraffic-record: " + json.dumps(rec) + "\n")
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.traffic_record("k.hip", "k<1>") == 123
    assert b.traffic_record("k.hip", "k<2>") is None
    assert b.traffic_record("other.hip", "k<1>") is None
    src.write_bytes(b"kernel v2")
    assert b.traffic_record("k.hip", "k<1>") is None
