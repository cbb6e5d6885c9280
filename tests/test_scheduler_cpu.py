"""Host-only tests of the serving scheduler (admission by footprint, slots,
FIFO with bounded skip-ahead, failure handling) with mock jobs."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run():
    exe = os.path.join(tempfile.mkdtemp(), "sched_test")
    subprocess.run(["g++", "-std=c++17", "-O1", "-pthread", "-I", os.path.join(ROOT, "paper_2507_19276_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpu", "sched_test.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=120).stdout
    res = {}
    for line in out.splitlines():
        name, *kv = line.split()
        res[name] = {k: int(v) for k, v in (x.split("=") for x in kv)}
    return res


def test_scheduler_invariants():
    r = _run()
    m = r["mix"]
    assert m["done"] == 200 and m["reserved_end"] == 0
    assert m["peak_reserved"] <= m["budget"] and m["over"] == 0
    assert m["peak_inflight"] <= 4 and m["max_running"] >= 2
    f = r["fail"]
    assert f["done"] == 20 and f["failed"] == 7 and f["reserved_end"] == 0 and f["inflight_end"] == 0
    assert r["oversize"]["rc"] == 1
    a = r["aging"]
    assert a["done"] == 12
    assert a["skips"] <= 3 and 1 <= a["big_started_at"] <= 4
    assert r["fifo"]["done"] == 30 and r["fifo"]["inorder"] == 1
