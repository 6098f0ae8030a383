"""CPU checks of the benchmark's measurement plumbing: the one-GPU refusal,
the source hash that ties counter summaries to the code they were taken on,
the copy calibration of the HBM byte counters, and the algorithmic bytes the
roofline entry divides by."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    line = json.loads(res.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def write_sources(root, text):
    csrc = root / "paper_1702_04250_amd" / "csrc"
    csrc.mkdir(parents=True, exist_ok=True)
    (csrc / "k.hip").write_text(text)


def test_source_hash_ignores_comments_and_whitespace(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    write_sources(tmp_path, '// header\nint f(int x) { return x + 1; }  /* note */\nconst char* s = "// kept";\n')
    h0 = bench.source_hash()
    write_sources(tmp_path, 'int f(int x)\n{\n    return x + 1;  // other words\n}\nconst char* s = "// kept";\n')
    assert bench.source_hash() == h0
    # code and string literals count
    write_sources(tmp_path, 'int f(int x) { return x + 2; }\nconst char* s = "// kept";\n')
    assert bench.source_hash() != h0
    write_sources(tmp_path, 'int f(int x) { return x + 1; }\nconst char* s = "// changed";\n')
    assert bench.source_hash() != h0


def write_counters(folder, rows):
    folder.mkdir(parents=True, exist_ok=True)
    with open(folder / "x_counter_collection.csv", "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for r in rows:
            f.write(",".join(f'"{v}"' if isinstance(v, str) else str(v) for v in r) + "\n")


def test_summarize_scales_the_counters_by_the_copy_calibration(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    write_sources(tmp_path, "int k;\n")
    (tmp_path / "trace").mkdir()
    with open(tmp_path / "trace" / "x_kernel_stats.csv", "w") as f:
        f.write('"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs","StdDev"\n')
        f.write('"void pppm::(anonymous namespace)::k_spread<5, false>(pppm::SpreadArgs)",4,148000,37000,50,'
                '36000,38000,0\n')
    # a 1 GiB copy: FETCH_SIZE reads half of it (factor 2), WRITE_SIZE all of it (factor 1)
    write_counters(tmp_path / "calib_fetch", [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288)])
    write_counters(tmp_path / "calib_write", [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576)])
    # two dispatches of k_spread, each counter summed over its two instances
    name = "void pppm::(anonymous namespace)::k_spread<5, false>(pppm::SpreadArgs)"
    write_counters(tmp_path / "fetch", [(7, name, "FETCH_SIZE", 60), (7, name, "FETCH_SIZE", 40),
                                        (9, name, "FETCH_SIZE", 50), (9, name, "FETCH_SIZE", 50)])
    write_counters(tmp_path / "write", [(7, name, "WRITE_SIZE", 30), (7, name, "WRITE_SIZE", 20),
                                        (9, name, "WRITE_SIZE", 25), (9, name, "WRITE_SIZE", 25)])
    text = bench.summarize(str(tmp_path))
    assert f"source hash: {bench.source_hash()}" in text
    assert "| k_spread | 4 | 37.00 | 36.00 | 38.00 | 50.0 |" in text
    expect = 100 * 1024 * 2.0 + 50 * 1024 * 1.0
    assert f"traffic[k_spread] = {expect:.0f}" in text
    # the committed-summary reader accepts it only for the same sources
    prof = tmp_path / "profile.md"
    prof.write_text(text)
    monkeypatch.setattr(bench, "PROFILE", str(prof))
    assert bench.recorded_traffic("k_spread") == pytest.approx(expect)
    assert bench.recorded_avg_us("k_spread") == pytest.approx(37.0)
    write_sources(tmp_path, "int k2;\n")
    assert bench.recorded_traffic("k_spread") is None and bench.recorded_avg_us("k_spread") is None


def test_algorithmic_bytes():
    n, cells = 524288, 128 ** 3
    # make_rho: the records once and the transform input once (FP32 in the
    # mixed form); the caller's FP64 mesh only when it is asked for
    assert bench.algorithmic_bytes("make_rho", n, cells, "mixed") == 16 * n + 4 * cells
    assert bench.algorithmic_bytes("make_rho", n, cells, "mixed", rho_out=True) == 16 * n + 12 * cells
    assert bench.algorithmic_bytes("make_rho", n, cells, "fp64") == 32 * n + 8 * cells
    # gathers: records, forces, and the field mesh(es) once
    assert bench.algorithmic_bytes("fieldforce_ad", n, cells, "mixed") == 28 * n + 4 * cells
    assert bench.algorithmic_bytes("fieldforce_ik", n, cells, "mixed") == 28 * n + 12 * cells
    with pytest.raises(ValueError):
        bench.algorithmic_bytes("poisson", n, cells, "mixed")
