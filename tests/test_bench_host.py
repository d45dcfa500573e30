"""Host logic of bench.py, without a GPU: the one-GPU guard, the roofline
arithmetic, the traffic record and its keying by kernel source, the summary
of the rocprofv3 counter passes, and the workload recipes."""

import json
import os
import subprocess
import sys

import pytest

import bench
from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr and res.stdout == ""


def test_kernel_short_name():
    assert bench.kernel_short_name("void srw::k_meet<4>(srw::StepDesc const*, long)") == "k_meet<4>"
    assert bench.kernel_short_name("srw::k_expand(srw::StepDesc const*)") == "k_expand"


def cls_stats(ms, launches, **extra):
    out = {"ms": dict.fromkeys(bench.CLASSES, 0.0), "launches": dict.fromkeys(bench.CLASSES, 0),
           "bytes_expand": 0, "bytes_insert": 0, "bytes_compact": 0}
    out["ms"].update(ms)
    out["launches"].update(launches)
    out.update(extra)
    return out


def test_roofline_of_the_meet_uses_the_widest_time_width(monkeypatch):
    monkeypatch.setattr(bench, "measured_traffic", lambda w, k: 123.0 if k == "k_meet<4, false, false>" else None)
    # timed region: launch times (the lean kernels count nothing); the extra
    # pass with the counting kernels: the set operations (here 5 launches)
    stats = {"meet_w": {1: {"ms": 2.0, "launches": 10, "ops": 0, "pair_words": 1e9},
                        4: {"ms": 50.0, "launches": 10, "ops": 0, "pair_words": 5e12}}}
    counted = {1: {"ms": 1.0, "launches": 5, "ops": 5e8, "pair_words": 5e8},
               4: {"ms": 26.0, "launches": 5, "ops": 1e12, "pair_words": 2.5e12}}
    r = bench.roofline(stats, cls_stats({"meet": 60.0, "expand": 5.0}, {"meet": 20, "expand": 40},
                                        meet_w=counted), "wl")
    assert r["kernel"] == "k_meet<4, false, false>" and r["bound"] == "alu" and r["unit"] == "TOP/s"
    # 2e11 lane-ops per launch in 5 ms: 40 T lane-ops/s
    assert r["achieved"] == pytest.approx(40.0)
    assert r["peak"] == pytest.approx(256 * 64 * 2.4e9 / 1e12)
    assert r["frac"] == pytest.approx(40.0 / r["peak"])
    assert r["traffic"] == 123.0
    assert r["per_launch_ms"] == pytest.approx(5.0)
    assert r["brute_force_lane_ops_per_launch"] == pytest.approx(1e12)


def test_roofline_of_the_bucketed_meet_uses_its_own_launches(monkeypatch):
    monkeypatch.setattr(bench, "measured_traffic", lambda w, k: None)
    # width 8: 32 meet launches of which 25 bucketed, 90% of the time
    stats = {"meet_w": {8: {"ms": 800.0, "launches": 32, "ops": 0, "pair_words": 3.2e13,
                            "b_launches": 25, "b_ms": 750.0, "b_ops": 0}}}
    counted = {8: {"ms": 900.0, "launches": 32, "ops": 1.3e12, "pair_words": 3.2e13,
                   "b_launches": 25, "b_ms": 850.0, "b_ops": 1.25e12}}
    r = bench.roofline(stats, cls_stats({"meet": 900.0}, {"meet": 32}, meet_w=counted), "wl")
    assert r["kernel"] == "k_meet_b<8, false>" and r["launches"] == 25
    assert r["per_launch_ms"] == pytest.approx(30.0)
    # 5e10 lane-ops per launch in 30 ms
    assert r["achieved"] == pytest.approx(5e10 / 0.03 / 1e12)


def test_roofline_of_an_hbm_class():
    c = cls_stats({"expand": 10.0, "meet": 1.0}, {"expand": 5, "meet": 3}, bytes_expand=4e10)
    r = bench.roofline({"meet_w": {}}, c, "wl")
    # 8e9 B per launch in 2 ms: 4000 GB/s
    assert r["kernel"] == "k_expand" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(4000.0)
    assert r["frac"] == pytest.approx(0.5)


def test_source_sha1_ignores_comments_only(tmp_path):
    a, b, c = tmp_path / "a.hip", tmp_path / "b.hip", tmp_path / "c.hip"
    a.write_text("int f(int x) {\n  return x + 1;\n}\n")
    b.write_text("// header\nint f(int x) { /* the\n next */\n  return x + 1; // one more\n}\n\n")
    c.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert bench.source_sha1(str(a)) == bench.source_sha1(str(b))
    assert bench.source_sha1(str(a)) != bench.source_sha1(str(c))


def write_counter_csv(path, rows):
    with open(path, "w") as f:
        f.write("Kernel_Name,Counter_Value\n")
        for name, v in rows:
            f.write(f'"{name}",{v}\n')


def test_pmc_summary_scales_by_the_copy_calibration(tmp_path, capsys):
    copy = "__amd_rocclr_copyBuffer"
    # the counters read twice the copy's bytes on fetch, exactly them on write
    fetch = [(copy, 2 * 256 * 1024)] * 3 + [("void srw::k_meet<4>(x)", 2 * 1024)] * 2
    write = [(copy, 256 * 1024)] * 3 + [("void srw::k_meet<4>(x)", 512)] * 2
    fp, wp, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    write_counter_csv(fp, fetch)
    write_counter_csv(wp, write)
    src = tmp_path / "k.hip"
    src.write_text("int g;\n")
    bench.pmc_summary(str(fp), str(wp), "wl", str(out), str(src))
    rec = json.loads(out.read_text())
    assert rec["_factors"] == {"fetch": pytest.approx(0.5), "write": pytest.approx(1.0)}
    # per dispatch: 1024 KiB fetched + 512 KiB written
    assert rec["wl"]["k_meet<4>"] == pytest.approx(1536 * 1024)
    assert rec["_kernel_source_sha1"] == bench.source_sha1(str(src))
    assert "factors fetch 0.500, write 1.000" in capsys.readouterr().out


def test_traffic_record_is_void_once_the_kernel_source_changed(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    rec = {"wl": {"k_meet<4>": 7.0}, "_kernel_source_sha1": "0" * 40}
    (tmp_path / "profiles" / "hbm_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("wl", "k_meet<4>") is None
    rec["_kernel_source_sha1"] = bench.source_sha1()
    (tmp_path / "profiles" / "hbm_traffic.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("wl", "k_meet<4>") == 7.0
    assert bench.measured_traffic("wl", "k_expand") is None
    assert bench.measured_traffic("other", "k_meet<4>") is None


class HostCheck:
    """Stands in for the library's synchronizability check in these tests."""
    check_sync = staticmethod(O.is_synchronizing)


def test_workload_recipes():
    w = bench.workload("n256k2x10+cerny16-32", HostCheck)
    assert [x[:2] for x in w[:10]] == [(256, 2)] * 10
    assert [x[0] for x in w[10:]] == list(range(16, 33))
    assert all(O.is_synchronizing(n, k, d) for n, k, d, _ in w[:10])
    assert len(bench.workload("n256k2x10", HostCheck)) == 10
    small = bench.workload("n64k2x100", HostCheck)
    assert len(small) == 100 and len({bytes(d.tobytes()) for _, _, d, _ in small}) == 100
    mix = bench.workload("mix4096-n32-320-k2-3", HostCheck, count=64, nmax=100)
    assert mix and all(32 <= n <= 100 and k in (2, 3) for n, k, _, _ in mix)
    (n, k, d, _), = bench.workload("sink26-k25", HostCheck)
    assert (n, k, len(d)) == (26, 25, 26 * 25)
    with pytest.raises(SystemExit):
        bench.workload("no-such-workload", HostCheck)


def test_cpu_baseline_times_the_oracle_on_a_bounded_sample():
    """The oracle leg runs each member in a child process, random members
    first, and reports the subsets it expanded per second of oracle time."""
    from paper_2207_05495_amd import inputs as I
    probs = [(n, 2, I.cerny(n), f"cerny{n}") for n in (6, 8)]
    d, _ = I.first_synchronizing(5, 2, I.member_seed(I.BASE_SEED, 0), O.is_synchronizing)
    probs.insert(0, (5, 2, d, "rand5"))
    out = bench.cpu_baseline(probs, 60.0)
    assert out["kind"] == "oracle" and out["cores"] == 1
    assert out["unit"] == "subsets expanded/s" and out["value"] > 0
    assert out["sample"].startswith("3 of 3 automata") and "rand5, cerny6, cerny8" in out["sample"]
    assert bench.cpu_baseline(probs, 0.1)["value"] is None
