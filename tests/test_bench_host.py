"""Host logic of bench.py that needs no device: the roofline's HBM traffic
from the committed rocprofv3 counter record."""
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    import importlib.util

    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_committed_counter_record():
    """The SAP record under profiles/: while it was taken on the kernel source
    in the tree its bytes are FETCH_SIZE x 2 + WRITE_SIZE x 1 (KiB) per
    launch; after a change of that source the bench reports no traffic."""
    b = _bench()
    rec = json.load(open(os.path.join(ROOT, "profiles", "counters_48c96_fp32_batch4.json")))
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    k = rec["kernels"]["sap"]
    by, why = b.counter_traffic("counters_48c96_fp32_batch4.json", "sap")
    if b.kernel_source_digest(k["source"]) == k["source_sha256"]:
        assert by == pytest.approx((k["fetch_kib"] * 2.0 + k["write_kib"]) * 1024.0)
    else:
        assert by is None and "changed" in why


def test_counter_record_is_void_once_the_source_changes(tmp_path, monkeypatch):
    b = _bench()
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = dict(fetch_scale=2.0, write_scale=1.0,
               kernels=dict(sap=dict(fetch_kib=10.0, write_kib=3.0, dispatches=4, source="k.hip",
                                     source_sha256=b.kernel_source_digest(str(src)))))
    (prof / "r.json").write_text(json.dumps(rec))
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    by, _ = b.counter_traffic("r.json", "sap")
    assert by == (10.0 * 2.0 + 3.0) * 1024.0
    assert b.counter_traffic("r.json", "dirac64")[0] is None
    assert b.counter_traffic("missing.json", "sap")[0] is None
    src.write_text("kernel v2\n")
    by, why = b.counter_traffic("r.json", "sap")
    assert by is None and "changed" in why
