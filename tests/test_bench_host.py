"""Host-side logic of bench.py (CPU only): the code-only source digest that
keeps recorded HBM traffic tied to the kernel sources it was measured on,
the traffic lookup, and the refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_only_ignores_comments_and_layout():
    a = "int f(int x) {  // add one\n    return x + 1; /* done */\n}\n"
    b = "int f(int x) {\n/* a comment */ return x + 1;\n\n}"
    assert bench._code_only(a) == bench._code_only(b)
    # a change of code changes it, also inside a string literal
    assert bench._code_only(a) != bench._code_only(a.replace("x + 1", "x + 2"))
    s1 = 'const char *m = "// not a comment";'
    s2 = 'const char *m = "// not a comment!";'
    assert bench._code_only(s1) != bench._code_only(s2)
    assert "// not a comment" in bench._code_only(s1)


def test_kernel_digest_follows_code_only():
    srcs = {name: f"// header of {name}\nint v_{name.replace('.', '_')} = 1;\n"
            for name in bench.KERNEL_SOURCES["revise_kernel"]}
    base = bench.kernel_digest("revise_kernel", read=lambda n: srcs[n])
    commented = {k: v + "// a new comment\n" for k, v in srcs.items()}
    assert bench.kernel_digest("revise_kernel", read=lambda n: commented[n]) == base
    first = bench.KERNEL_SOURCES["revise_kernel"][0]
    changed = dict(srcs)
    changed[first] = srcs[first].replace("= 1", "= 2")
    assert bench.kernel_digest("revise_kernel", read=lambda n: changed[n]) != base


def test_recorded_traffic_requires_matching_digest(tmp_path, monkeypatch):
    table = {
        "current": dict(kernel="revise_kernel", fetch_bytes_per_launch=100.0,
                        write_bytes_per_launch=20.0, sha256=bench.kernel_digest("revise_kernel")),
        "stale": dict(kernel="revise_kernel", fetch_bytes_per_launch=100.0,
                      write_bytes_per_launch=20.0, sha256="0" * 64),
    }
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(table))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.recorded_traffic("current") == 120.0
    assert bench.recorded_traffic("stale") is None
    assert bench.recorded_traffic("absent") is None


def test_committed_traffic_entries_name_known_kernels():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        table = json.load(fh)
    for name, e in table.items():
        assert e["kernel"] in bench.KERNEL_SOURCES, name
        assert os.path.exists(os.path.join(ROOT, "profiles", name + ".txt")), name


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, CUDA_VISIBLE_DEVICES="", HIP_VISIBLE_DEVICES=""))
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""
