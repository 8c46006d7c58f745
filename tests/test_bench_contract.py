"""CPU checks of bench.py's contract: more than one GPU is refused with a message,
the roofline peaks are the stated ones, and counted traffic / instruction figures
are used only when they were taken on the kernel that runs and its sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    sys.path.insert(0, ROOT)
    import bench
    return bench


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""              # no JSON line


def test_roofline_peaks():
    b = _bench()
    assert b.HBM_PEAK_GBPS == 8000.0
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
    assert b.VALU_PEAK_TOPS == pytest.approx(39.3216)
    assert b.ALG_OPS_PER_LUP["f32"] == 29 + 14
    assert b.ALG_OPS_PER_LUP["f16s"] > b.ALG_OPS_PER_LUP["f32"]


def test_counted_figures_need_matching_kernel_and_sources(tmp_path, monkeypatch):
    b = _bench()
    h = b.kernel_source_hash()
    assert len(h) == 16
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"f32": {"source_hash": h, "kernel_bench": "k_step_fused<P_F32,4,22,3>", "traffic_bytes": 2.0e9,
                   "traffic_ratio": 1.25, "valu_per_dispatch": 1.0e8}}
    (prof / "traffic_periodic8192.json").write_text(json.dumps(rec))
    (prof / "valu_periodic8192.json").write_text(json.dumps(rec))
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    # kernel_source_hash reads the sources under ROOT: point it back at the repository
    monkeypatch.setattr(b, "kernel_source_hash", lambda: h)
    t = b.measured_traffic("f32", "k_step_fused<P_F32,4,22,3>", 0.5)
    assert t["GBps"] == pytest.approx(2.0e9 / 0.5e-3 / 1e9) and t["ratio"] == 1.25
    assert b.measured_valu("f32", "k_step_fused<P_F32,4,22,3>") == 64 * 1.0e8
    # another kernel, another storage format or other sources: no figure
    assert b.measured_traffic("f32", "k_step_fused<P_F32,4,14,3>", 0.5) is None
    assert b.measured_traffic("f16s", "k_step_fused<P_F32,4,22,3>", 0.5) is None
    # several strip shapes of one storage format: each finds its own record
    rec2 = dict(rec["f32"], kernel_bench="k_step_fused<P_F32,4,28,3>", traffic_ratio=1.12)
    (prof / "traffic_periodic8192.json").write_text(json.dumps({"f32": [rec2, rec["f32"]]}))
    assert b.measured_traffic("f32", "k_step_fused<P_F32,4,28,3>", 0.5)["ratio"] == 1.12
    assert b.measured_traffic("f32", "k_step_fused<P_F32,4,22,3>", 0.5)["ratio"] == 1.25
    assert b.measured_traffic("f32", "k_step_fused<P_F32,4,14,3>", 0.5) is None
    monkeypatch.setattr(b, "kernel_source_hash", lambda: "0" * 16)
    assert b.measured_traffic("f32", "k_step_fused<P_F32,4,22,3>", 0.5) is None
    assert b.measured_valu("f32", "k_step_fused<P_F32,4,22,3>") is None


def test_committed_profiles_match_the_sources():
    """The committed counter summaries were taken on the current kernel sources."""
    b = _bench()
    for name in ("traffic_periodic8192.json", "valu_periodic8192.json"):
        rec = json.load(open(os.path.join(ROOT, "profiles", name)))
        for st, rs in rec.items():
            for r in rs if isinstance(rs, list) else [rs]:
                assert r["source_hash"] == b.kernel_source_hash(), (name, st, r["kernel_bench"])
                assert b.profile_record(name, st, r["kernel_bench"]) == r


def test_reduction_cadence_does_not_follow_the_timed_length():
    """The FP64 reduction runs every 99 steps (three-step launches) or 100, counted from
    the start of the run with the warmup, whatever --steps is; segments split at each
    reduction and at the end of the warmup, whole launches apart from remainders."""
    b = _bench()
    assert b.reduction_block(3) == 99 and b.reduction_block(2) == 100 and b.reduction_block(1) == 100
    # the driver's short run: 5 warmup then 20 timed steps, no reduction falls inside
    sched = b.run_schedule(20, 5, 3)
    assert sched == [(False, 3, 2, False), (True, 18, 2, False)]
    assert sum(w + r for t, w, r, _ in sched if t) == 20
    assert not any(red for _, _, _, red in sched)
    # a long run: reductions at 99, 198, ... counted from step 0
    sched = b.run_schedule(1000, 100, 3)
    assert sum(w + r for t, w, r, _ in sched if t) == 1000
    ends, t = [], 0
    for _, w, r, red in sched:
        t += w + r
        if red:
            ends.append(t)
    assert ends == list(range(99, 1101, 99))
    assert all(w % 3 == 0 for _, w, _, _ in sched)
    # one step per launch: every 100 steps
    sched = b.run_schedule(250, 50, 1)
    assert [w for _, w, _, _ in sched] == [50, 50, 100, 100] and [x[3] for x in sched] == [False, True, True, True]
