"""The HBM counter records committed under profiles/ (read by bench.py for the `traffic`
field of its roofline) are well formed and name kernels whose source section exists, so
that bench.py can match them against the current kernel source."""
import glob
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KEYS = {"kernel", "kernel_src_sha256_16", "fetch_kib", "write_kib", "fetch_factor",
        "write_factor"}   # "workload" and "schedule" are optional (absent: any)


def _records():
    out = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_pmc.md"))):
        for line in open(path):
            if line.startswith("pmc: "):
                out.append((os.path.basename(path), json.loads(line[5:])))
    return out


def test_counter_records_well_formed():
    recs = _records()
    assert recs
    for name, rec in recs:
        assert KEYS <= set(rec), name
        assert rec["fetch_kib"] > 0 and rec["write_kib"] >= 0, name
        assert rec["fetch_factor"] > 0 and rec["write_factor"] > 0, name
        assert len(rec["kernel_src_sha256_16"]) == 16, name
        assert bench.kernel_source_sha(rec["kernel"]) is not None, (name, rec["kernel"])


def test_traffic_lookup_matches_record():
    """measured_traffic returns 2.0 x FETCH + 1.0 x WRITE (scaled) of a record whose hash is
    current, and nothing for a kernel or schedule without one."""
    for _, rec in _records():
        if bench.kernel_source_sha(rec["kernel"]) != rec["kernel_src_sha256_16"]:
            continue
        workload = rec.get("workload", "coulomb_k10")
        got = bench.measured_traffic(rec["kernel"], workload, rec.get("schedule"))
        want = 1024.0 * (rec["fetch_kib"] * rec["fetch_factor"]
                         + rec["write_kib"] * rec["write_factor"])
        assert got == want
        other = {"sub_batches": 999, "split_div": 1}
        assert bench.measured_traffic(rec["kernel"], workload, other) is None
    assert bench.measured_traffic("no_such_kernel<1>", "coulomb_k10") is None
