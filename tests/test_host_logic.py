"""Host-side logic that needs no GPU: bench.py's contract checks, the
autotuner's candidate splits, the traffic-record lookup."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_autotune_candidates():
    from paper_2603_26232_amd.autotune import candidates, default_split
    assert candidates(12) == [] and candidates(13) == [] and candidates(20) == [[8]]
    assert candidates(21) == [[a, 9 - a] for a in range(1, 9)]
    assert [8, 8] in candidates(28) and len(candidates(28)) == 1
    c30 = candidates(30)
    assert all(len(x) == 3 and sum(x) == 18 and max(x) <= 8 for x in c30)
    for n in range(14, 31):
        d = default_split(n)
        assert sum(d) == n - 12 and max(d) - min(d) <= 1 and max(d) <= 8
        assert d in candidates(n) or len(candidates(n)) == 0


def test_traffic_record_lookup(tmp_path, monkeypatch):
    import hashlib
    import bench
    src = os.path.join(ROOT, "paper_2603_26232_amd", "csrc", "sim.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    recs = [{"kernel": "bwd_mid_g0", "source": "sim.hip", "source_sha256": sha, "hbm_bytes_per_launch": 123},
            {"kernel": "fwd_mid_g1", "source": "sim.hip", "source_sha256": "0" * 64, "hbm_bytes_per_launch": 7}]
    (prof / "pmc_passes_plain400.txt").write_text("\n".join("RECORD " + json.dumps(r) for r in recs) + "\n")
    # point the lookup at a temporary tree holding a copy of the real source
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "paper_2603_26232_amd").mkdir()
    (tmp_path / "paper_2603_26232_amd" / "csrc").mkdir()
    (tmp_path / "paper_2603_26232_amd" / "csrc" / "sim.hip").write_bytes(open(src, "rb").read())
    assert bench.traffic_record("bwd_mid_g0", "plain400")["hbm_bytes_per_launch"] == 123
    assert bench.traffic_record("fwd_mid_g1", "plain400") is None  # taken on another source
    assert bench.traffic_record("bwd_last_g0", "plain400") is None  # no record
    assert bench.traffic_record("bwd_mid_g0", "ragged2000") is None  # no file


def test_valu_record_lookup(tmp_path, monkeypatch):
    import hashlib
    import bench
    src = os.path.join(ROOT, "paper_2603_26232_amd", "csrc", "sim.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    recs = [{"kernel": "bwd_mid_g0", "source": "sim.hip", "source_sha256": sha, "valu_insts_per_launch": 99},
            {"kernel": "fwd_mid_g0", "source": "sim.hip", "source_sha256": "f" * 64, "valu_insts_per_launch": 5}]
    (prof / "pmc_valu_plain400.txt").write_text("header line\n" + "\n".join("RECORD " + json.dumps(r) for r in recs) + "\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "paper_2603_26232_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "paper_2603_26232_amd" / "csrc" / "sim.hip").write_bytes(open(src, "rb").read())
    assert bench.valu_record("bwd_mid_g0", "plain400")["valu_insts_per_launch"] == 99
    assert bench.valu_record("fwd_mid_g0", "plain400") is None
    assert bench.traffic_record("bwd_mid_g0", "plain400") is None  # the VALU file is not the traffic file
    # the issue peak follows from the unit counts and clock
    assert bench.VALU_PEAK == 614.4e9

