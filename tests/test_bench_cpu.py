"""Host-side checks of the benchmark script: the committed counter summaries parse, their numbers
are consistent with themselves, and more than one GPU is refused."""
import glob
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _records():
    out = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "k_batch_*.md"))):
        text = open(path).read()
        start = text.index("```json")
        out.append((path, text, json.loads(text[start + 7:text.index("```", start + 7)])))
    return out


def test_profile_records_are_consistent():
    recs = _records()
    assert recs, "no k_batch counter summary under profiles/"
    for path, text, rec in recs:
        wl = os.path.basename(path)[len("k_batch_"):-3]
        assert rec["kernel"] == "k_batch" and rec["workload"] == wl
        assert rec["traffic_bytes"] == rec["read_bytes"] + rec["write_bytes"]
        assert abs(rec["read_bytes"] - rec["fetch_kib"] * 1024 * rec["fetch_scale"]) < 1e-3 * rec["read_bytes"]
        assert abs(rec["write_bytes"] - rec["write_kib"] * 1024 * rec["write_scale"]) < 1e-3 * rec["write_bytes"]
        # moved bytes cannot be below what the launch must read and write
        assert rec["traffic_bytes"] >= 0.99 * rec["algorithmic_bytes"]
        assert "rocprofv3 --kernel-trace --stats" in text and "--pmc FETCH_SIZE" in text


def test_profiled_traffic_follows_source_and_plan():
    import bench
    for path, _, rec in _records():
        plan = dict(zip(("waves_per_group", "column_groups", "groups_per_cu"), rec["plan"]),
                    window_rows=rec.get("window_rows", 0))
        got = bench.profiled_traffic(rec["workload"], plan)
        if rec["source"] == bench.kernel_source_id():
            assert got is not None and got["traffic_bytes"] == rec["traffic_bytes"]
        else:
            assert got is None
        other = dict(plan, groups_per_cu=plan["groups_per_cu"] + 1)
        assert bench.profiled_traffic(rec["workload"], other) is None
        other = dict(plan, window_rows=plan["window_rows"] + 32)      # another tile height
        assert bench.profiled_traffic(rec["workload"], other) is None
    assert bench.profiled_traffic("no-such-workload", {"waves_per_group": 8, "column_groups": 1,
                                                       "groups_per_cu": 1}) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("flag", ["--no-e2e", "--no-serve", "--no-plain", "--no-cpu-baseline",
                                  "--copy-reference-mb", "--no-tune", "--no-graph", "--plan"])
def test_bench_flags_are_offered(flag, capsys):
    import bench
    with pytest.raises(SystemExit) as e:
        bench.main(["--help"])
    assert e.value.code == 0
    assert flag in capsys.readouterr().out


def test_every_workload_has_a_peak_buffer_and_the_secondary_list_is_known():
    import bench
    from paper_2607_04067_amd import synth
    assert set(bench.MAX_PEAKS) == set(synth.WORKLOADS)
    assert bench.DEFAULT_WORKLOAD in synth.WORKLOADS
    assert set(bench.SECONDARY_WORKLOADS) <= set(synth.WORKLOADS)
    assert len(set(bench.SECONDARY_WORKLOADS)) == len(bench.SECONDARY_WORKLOADS)


def test_profile_commands_leave_out_the_secondary_section():
    """The other configurations launch the same kernels: a profiled command must skip them, or
    their launches would mix into the summary's kernel statistics."""
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if "rocprofv3" in line and "bench.py" in line and "--phases" not in line:
                assert "--no-secondary" in line, (path, line)
