"""Host logic of the measurement and tuning code (no GPU): which committed counters a bench
line may carry, the run keys they are filed under, and the autotuner's cache."""
import argparse
import hashlib
import os

import bench
from paper_1711_00121_amd import tune


def _args(**kw):
    a = argparse.Namespace(n=None, m=None, steps=20, warmup=5)
    for k, v in kw.items():
        setattr(a, k, v)
    return a


def test_counters_are_keyed_by_workload_and_run_length():
    assert bench.counters_for(_args(), "batch_nodes_n50k") == "batch_nodes_n50k steps=20 warmup=5"
    assert bench.counters_for(_args(steps=3, warmup=1), "x") == "x steps=3 warmup=1"
    # a resized run matches no committed counters
    assert bench.counters_for(_args(n=1000), "batch_nodes_n50k") == "resized"


def _profile(root, name, workload_bytes, src_text):
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)
    src = os.path.join(root, "k.hip")
    with open(src, "w") as f:
        f.write(src_text)
    sha = hashlib.sha256(src_text.encode()).hexdigest()
    lines = [f"# {name}", "Source: `k.hip`", f"source_sha256: {sha}", ""]
    for w, b in workload_bytes:
        lines += [f"hbm_bytes_per_launch: {b:.6e}", f"workload: {w}", ""]
    wl = workload_bytes[0][0].split(" ")[0]
    with open(os.path.join(root, "profiles", f"{name}_{wl}_pmc.md"), "w") as f:
        f.write("\n".join(lines))


def test_traffic_takes_the_section_of_the_run(tmp_path, monkeypatch):
    root = str(tmp_path)
    _profile(root, "kern", [("wl steps=20 warmup=5", 1.5e11), ("wl steps=3 warmup=1", 4.0e10)],
             "kernel v1\n")
    monkeypatch.setattr(bench, "ROOT", root)
    assert bench.traffic("kern", "wl steps=20 warmup=5") == 1.5e11
    assert bench.traffic("kern (fused pass)", "wl steps=3 warmup=1") == 4.0e10
    # another run length, another workload or a resized run: no counters
    assert bench.traffic("kern", "wl steps=7 warmup=1") is None
    assert bench.traffic("kern", "other steps=3 warmup=1") is None
    assert bench.traffic("kern", "resized") is None
    assert bench.traffic("other_kernel", "wl steps=3 warmup=1") is None


def test_traffic_is_null_once_the_source_changed(tmp_path, monkeypatch):
    root = str(tmp_path)
    _profile(root, "kern", [("wl steps=3 warmup=1", 4.0e10)], "kernel v1\n")
    monkeypatch.setattr(bench, "ROOT", root)
    assert bench.traffic("kern", "wl steps=3 warmup=1") == 4.0e10
    with open(os.path.join(root, "k.hip"), "a") as f:
        f.write("// edited\n")
    assert bench.traffic("kern", "wl steps=3 warmup=1") is None


def test_committed_counters_match_their_sources():
    """Every committed counter summary names a source whose hash still matches, so the bench
    line of that run carries its traffic."""
    import re
    prof = os.path.join(bench.ROOT, "profiles")
    found = 0
    for f in sorted(os.listdir(prof)):
        if not f.endswith("_pmc.md"):
            continue
        text = open(os.path.join(prof, f)).read()
        src = re.search(r"Source: `([^`]+)`", text).group(1)
        sha = re.search(r"source_sha256:\s*([0-9a-f]{64})", text).group(1)
        data = open(os.path.join(bench.ROOT, src), "rb").read()
        assert hashlib.sha256(data).hexdigest() == sha, f
        kern = f[:-len("_pmc.md")]
        for w in re.findall(r"^workload:\s*(.+?)\s*$", text, flags=re.M):
            name = kern[:-len(w.split(" ")[0]) - 1]
            assert bench.traffic(name, w) is not None, (f, w)
            found += 1
    assert found >= 8


def test_tuning_keys_and_cache(tmp_path):
    assert tune.key_for(52362, 15, "hilo") == tune.key_for(50000, 15, "hilo")
    assert tune.key_for(52362, 15, "hilo") != tune.key_for(52362, 10, "hilo")
    assert tune.key_for(52362, 15, "hilo") != tune.key_for(52362, 15, "fp64")
    assert tune.key_for(10, 15, "fp64") == f"n{tune.BUCKET}_K15_fp64"
    path = str(tmp_path / "sub" / "cache.json")
    assert tune._load(path) == {}
    tune._store(path, {"k": {"batch_chunk": 64, "variant": 1}})
    assert tune._load(path) == {"k": {"batch_chunk": 64, "variant": 1}}
    with open(path, "w") as f:
        f.write("{not json")
    assert tune._load(path) == {}  # a damaged cache is ignored, not fatal


def test_host_description():
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and h["usable_cpus"] >= 1 and isinstance(h["cpu_model"], str)
