"""bench.py's host-side contract (no GPU): it refuses more than one GPU with
a message, a traffic figure is reported only while the kernel sources it was
taken on are unchanged (the sha1 gate), and every workload names a
generator."""
import importlib.util
import os
import subprocess
import sys

import datagen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_every_traffic_figure_names_its_sources_and_profile():
    b = _bench()
    for (kernel, workload), m in b.MEASURED_TRAFFIC.items():
        assert os.path.exists(os.path.join(ROOT, m["profile"])), m["profile"]
        for rel, sha in m["sources"].items():
            assert os.path.exists(os.path.join(ROOT, rel)) and len(sha) == 40, rel
        assert m["fetch_GB"] > 0 and m["write_GB"] >= 0
        got = b.measured_traffic(kernel, workload)
        assert got is None or abs(got - (m["fetch_GB"] + m["write_GB"])) < 1e-3


def test_traffic_gate_rejects_unknown_or_changed_sources(tmp_path):
    b = _bench()
    assert b.measured_traffic("dist_topk", "no-such-workload") is None
    key = next(iter(b.MEASURED_TRAFFIC))
    entry = dict(b.MEASURED_TRAFFIC[key])
    entry["sources"] = {k: "0" * 40 for k in entry["sources"]}
    b.MEASURED_TRAFFIC[key] = entry
    assert b.measured_traffic(*key) is None


def test_workloads_name_generators():
    b = _bench()
    for name, (gen, kw, k, lam) in b.WORKLOADS.items():
        assert callable(getattr(datagen, gen)), name
        assert k >= 1 and lam >= 1
