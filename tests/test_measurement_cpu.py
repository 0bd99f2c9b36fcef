"""Host-side checks of the measurement tooling: the counter records the
benchmark reads (HBM bytes per launch from FETCH_SIZE / WRITE_SIZE scaled by
a plain copy of known size), the kernel-trace summaries, and the
benchmark's roofline arithmetic."""
import csv
import os

import pytest

from paper_1704_01144_amd import profile_summary as P


def _counter_csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Kernel_Name", "Counter_Name", "Counter_Value"], r)))


def test_counter_record_scaling(tmp_path, capsys):
    d = str(tmp_path)
    gib = 1 << 30
    # a copy of 1 GiB reads as 0.5 GiB fetched, 1 GiB written (KiB units)
    _counter_csv(f"{d}/cf", [("__amd_rocclr_copyBuffer", "FETCH_SIZE", gib / 2048)])
    _counter_csv(f"{d}/cw", [("__amd_rocclr_copyBuffer", "WRITE_SIZE", gib / 1024)])
    _counter_csv(f"{d}/f", [("void k_grad<double>(x)", "FETCH_SIZE", 1000.0),
                            ("void k_grad<double>(x)", "FETCH_SIZE", 3000.0),
                            ("void k_flux(x)", "FETCH_SIZE", 9.0)])
    _counter_csv(f"{d}/w", [("void k_grad<double>(x)", "WRITE_SIZE", 500.0)])
    P.main(["counters", "--kernel", "k_grad<double>", "--fetch", f"{d}/f", "--write", f"{d}/w",
            "--copy-fetch", f"{d}/cf", "--copy-write", f"{d}/cw", "--copy-bytes", str(gib),
            "--command", "c1", "--command", "c2"])
    out = capsys.readouterr().out
    path = tmp_path / "rec.txt"
    path.write_text(out)
    r = P.read_record(str(path))
    assert r["dispatches_fetch"] == "2" and r["command"] == ["c1", "c2"]
    assert float(r["fetch_scale"]) == pytest.approx(2.0) and float(r["write_scale"]) == pytest.approx(1.0)
    # mean fetch 2000 KiB x 2 + write 500 KiB x 1
    assert int(r["traffic_bytes_per_launch"]) == 2000 * 1024 * 2 + 500 * 1024
    assert r["sources_sha256"] == P.source_digest()


def test_stats_summary(tmp_path, capsys):
    d = tmp_path / "kt"
    d.mkdir()
    with open(d / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writerow(["void tafv::k_grad<double>(tafv::GradArgs<double>)", 10, 1000000, 100000, 75.0])
        w.writerow(["k_dt(int)", 5, 333333, 66666, 25.0])
    P.main(["stats", str(d), "--command", "cmd"])
    out = capsys.readouterr().out.splitlines()
    assert out[0] == "command: cmd"
    assert "k_grad<double>" in out[3] and "tafv::" not in out[3]
    assert out[3].split()[:3] == ["10", "1.000", "100.00"]
    assert "all kernels (2 names)" in out[-1]


def test_sq_per_wave_means(tmp_path, capsys):
    d = str(tmp_path)
    # two dispatches of one kernel: 100 + 300 waves, 1000 + 5000 VALU
    # instructions -> 15 per wave; a second run adds another counter
    _counter_csv(f"{d}/a", [("void k_grad<double>(x)", "SQ_WAVES", 100.0),
                            ("void k_grad<double>(x)", "SQ_INSTS_VALU", 1000.0),
                            ("void k_grad<double>(x)", "SQ_WAVES", 300.0),
                            ("void k_grad<double>(x)", "SQ_INSTS_VALU", 5000.0),
                            ("void k_flux(x)", "SQ_WAVES", 7.0),
                            ("void k_flux(x)", "SQ_INSTS_VALU", 70000.0)])
    _counter_csv(f"{d}/b", [("void k_grad<double>(x)", "SQ_WAVES", 100.0),
                            ("void k_grad<double>(x)", "SQ_WAIT_INST_ANY", 500.0),
                            ("void k_grad<double>(x)", "SQ_WAVES", 300.0),
                            ("void k_grad<double>(x)", "SQ_WAIT_INST_ANY", 1500.0)])
    P.main(["sq", "--kernel", "k_grad<double", "--dir", f"{d}/a", "--dir", f"{d}/b",
            "--command", "run a", "--command", "run b"])
    out = capsys.readouterr().out
    assert "  SQ_INSTS_VALU: 15.0" in out and "  SQ_WAIT_INST_ANY: 5.0" in out
    assert "kernel: k_grad<double (2 dispatches per run)" in out
    assert "command: run a" in out and "command: run b" in out
    with pytest.raises(SystemExit):
        P.main(["sq", "--kernel", "k_none", "--dir", f"{d}/a", "--command", "x"])


def test_roofline_arithmetic():
    import bench
    prof = {"grad": dict(ms=10.0, launches=100, items=1000000),
            "flux": dict(ms=5.0, launches=100, items=1000000),
            "gather": dict(ms=1.0, launches=100, items=100)}
    name, roof = bench.roofline(prof, {"grad": 400, "flux": 100, "gather": 200}, "fp64")
    assert name == "grad" and roof["kernel"] == "k_grad"
    assert roof["avg_launch_us"] == pytest.approx(100.0)
    assert roof["algorithmic_bytes_per_launch"] == 400 * 10000
    assert roof["achieved"] == pytest.approx(400 * 10000 / 100e-6 / 1e9, rel=1e-3)
    assert roof["frac"] == pytest.approx(roof["achieved"] / 8000.0, rel=1e-3)
