"""Host-side checks of bench.py (CPU): the one-GPU refusal, the code hash
that keeps the measured traffic attached to the code it was taken on, the
clock reading, and the launch-geometry bookkeeping of the profile summaries."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr and r.stdout == ""


def test_code_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    b = _bench()
    src = tmp_path / "k.hip"
    src.write_text("int f(int a) {  // add one\n  return a + 1; /* block\ncomment */\n}\n")
    monkeypatch.setattr(b, "KERNEL_SRCS", [str(src)])
    h0 = b.code_hash()
    src.write_text("// header\nint f(int a) {\n\n    return a + 1;   // other words\n}\n")
    assert b.code_hash() == h0
    src.write_text("int f(int a) {\n  return a + 2;\n}\n")
    assert b.code_hash() != h0


def test_traffic_is_null_for_other_code(tmp_path, monkeypatch):
    b = _bench()
    src = tmp_path / "k.hip"
    src.write_text("int g() { return 3; }\n")
    monkeypatch.setattr(b, "KERNEL_SRCS", [str(src)])
    assert b.traffic_entry("f32") is None


def test_gpu_clocks_from_dpm_tables(tmp_path, monkeypatch):
    b = _bench()
    dev = tmp_path / "card1" / "device"
    dev.mkdir(parents=True)
    (dev / "pp_dpm_sclk").write_text("0: 500Mhz\n1: 1400Mhz\n2: 2400Mhz *\n")
    (dev / "pp_dpm_mclk").write_text("0: 900Mhz\n1: 2000Mhz *\n")
    real = b.glob.glob
    monkeypatch.setattr(b.glob, "glob", lambda pat: real(pat.replace("/sys/class/drm", str(tmp_path))))
    assert b.gpu_clocks() == {"sclk": "2400Mhz", "mclk": "2000Mhz"}
    (dev / "pp_dpm_sclk").write_text("0: 500Mhz\n")
    (dev / "pp_dpm_mclk").unlink()
    assert b.gpu_clocks() is None


def test_launch_geometry_identifies_the_box():
    b = _bench()
    f32 = "void lbm::k_step<0, 1, true, false, 1>"
    f16 = "void lbm::k_step<1, 1, true, false, 4>"
    assert b.launch_threads(f32, 512) == 512 ** 3  # 64-cell runs, 4 per 256-thread block
    assert b.launch_threads(f16, 512) == 512 ** 3 // 4  # 4 cells per lane
    assert b.box_of(f32, 768 ** 3) == 768 and b.box_of(f16, 512 ** 3 // 4) == 512
    assert b.box_of("void lbm::k_adj<false, false, false>", 256 ** 3) == 256
    assert b.box_of(f32, 12345) is None


def test_trace_summary_against_the_bench_line(tmp_path, capsys):
    b = _bench()
    f32 = "void lbm::k_step<0, 1, true, false, 1>"
    cols = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X"]
    lines = [",".join(cols)]
    t = 0
    for k in range(6):  # 2 warm-up launches of 5 us, then 4 timed launches of 3 us
        dur = 5000 if k < 2 else 3000
        lines.append(f'"{f32}(args)",{t},{t + dur},{512 ** 3}')
        t += dur + 100
    (tmp_path / "x_kernel_trace.csv").write_text("\n".join(lines) + "\n")
    line = {"steps": 4, "warmup": 2, "ms_per_step": 0.003, "config": {"cells": 512 ** 3}}
    (tmp_path / "b.json").write_text(json.dumps(line) + "\n")
    assert b.trace_summary(str(tmp_path), str(tmp_path / "b.json")) == 0
    out = capsys.readouterr().out
    assert "| lbm::k_step<0, 1, true, false, 1> | 512^3 | 6 | 3.7 | 3.0 | 5.0 |" in out
    assert "4 launches after the 2 warm-up launches" in out and "average 3.0 us" in out


def test_repetition_sizes_keep_whole_launches():
    b = _bench()
    assert b.rep_sizes(980, 5) == [196] * 5
    assert b.rep_sizes(980, 5, unit=2) == [196] * 5
    assert b.rep_sizes(25, 5, unit=2) == [6, 6, 4, 4, 5]  # 12 pairs, the odd step last
    assert b.rep_sizes(3, 5, unit=2) == [3]
    assert b.rep_sizes(1, 5, unit=2) == [1]
    assert sum(b.rep_sizes(1001, 5, unit=2)) == 1001


def test_trace_summary_two_steps_per_launch(tmp_path, capsys):
    """A headline of two steps per launch is checked against the two-step
    kernel's launches: warm-up and timed steps count in pairs."""
    b = _bench()
    k2 = "void lbm::k_step2<0, 4, true, false, false>"
    g = b.launch_threads(k2, 512)
    assert b.box_of(k2, g) == 512
    kp = "void lbm::k_step2<0, 0, true, false, true>"  # periodic: the adjoint's 256^3 box
    assert b.launch_threads(kp, 256) == g and b.box_of(kp, g) == 256
    cols = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X"]
    lines, t = [",".join(cols)], 0
    for k in range(5):  # 1 warm-up launch of 9 us, then 4 timed launches of 6 us
        dur = 9000 if k < 1 else 6000
        lines.append(f'"{k2}(args)",{t},{t + dur},{g}')
        t += dur + 100
    (tmp_path / "x_kernel_trace.csv").write_text("\n".join(lines) + "\n")
    line = {"steps": 8, "warmup": 2, "ms_per_step": 0.003, "config": {"cells": 512 ** 3},
            "roofline": {"steps_per_launch": 2}}
    (tmp_path / "b.json").write_text(json.dumps(line) + "\n")
    assert b.trace_summary(str(tmp_path), str(tmp_path / "b.json")) == 0
    out = capsys.readouterr().out
    assert "6.0 us per launch (2 steps per launch" in out
    assert "4 launches after the 1 warm-up launches" in out and "average 6.0 us" in out


def test_roofline_of_two_step_leg(tmp_path, monkeypatch):
    """Algorithmic bytes per launch are those of the updates the launch
    performs; traffic comes from the counter record of the same kernel."""
    b = _bench()
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    json.dump({"code_sha256": b.code_hash(),
               "kernels": {"f32x2": {"fetch_bytes": 6e9, "write_bytes": 4e9}}},
              open(tmp_path / "traffic.json", "w"))
    leg = {"steps_per_launch": 2, "alg_gbs": 6800.0, "hbm_frac": 0.85,
           "alg_bytes_per_step": 1.0e10, "ms_per_step": 1.5}
    r = b.roofline_of("f32x2", leg)
    assert r["alg_bytes_per_launch"] == 2.0e10 and r["launch_ms"] == 3.0
    assert r["traffic"] == 1.0e10 and r["traffic_over_alg"] == 0.5
    assert r["frac"] == 0.85 and r["bound"] == "hbm" and "note" in r
    assert b.roofline_of("f16", dict(leg, steps_per_launch=1))["traffic"] is None


def test_profile_summary_calibrates_and_records(tmp_path, monkeypatch, capsys):
    """Synthetic trace and counter CSVs: the copy kernel's 4 GiB read and
    written calibrate FETCH_SIZE (x2 here) and WRITE_SIZE (x1); the FP32 step
    at 512^3 gets its traffic per launch, its ratio to the algorithmic bytes
    and a record in the traffic file, keyed to the code hash."""
    b = _bench()
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    f32 = "void lbm::k_step<0, 1, true, false, 1>"
    cp = "lbm::k_copy"
    tr = tmp_path / "tr"
    fe = tmp_path / "fe"
    wr = tmp_path / "wr"
    for d in (tr, fe, wr):
        d.mkdir()
    g = b.launch_threads(f32, 512)
    rows = ["Kernel_Name,Start_Timestamp,End_Timestamp,Grid_Size_X",
            f'"{f32}(x)",0,4000000,{g}', f'"{f32}(x)",5000000,9000000,{g}',
            f'"{cp}(x)",10000000,11400000,268435456']
    (tr / "t_kernel_trace.csv").write_text("\n".join(rows) + "\n")
    kib = 1024
    fetch_f32, write_f32 = 10.0e9, 10.2e9   # bytes the step moves per launch
    for d, cname, vals in ((fe, "FETCH_SIZE", {f32: fetch_f32 / 2, cp: (4 << 30) / 2}),
                           (wr, "WRITE_SIZE", {f32: write_f32, cp: 4 << 30})):
        lines = ["Kernel_Name,Grid_Size,Counter_Name,Counter_Value"]
        for name, v in vals.items():
            grid = g if name == f32 else 268435456
            lines.append(f'"{name}(x)",{grid},{cname},{v / kib}')
        (d / "c_counter_collection.csv").write_text("\n".join(lines) + "\n")
    assert b.profile_summary(str(tr), str(fe), str(wr), n=64) == 0
    out = capsys.readouterr().out
    assert "FETCH_SIZE x2.0000, WRITE_SIZE x1.0000" in out
    rec = json.load(open(tmp_path / "traffic.json"))
    assert rec["code_sha256"] == b.code_hash()
    k = rec["kernels"]["f32"]
    assert abs(k["fetch_bytes"] - fetch_f32) < 1 and abs(k["write_bytes"] - write_f32) < 1
    assert k["box"] == 512 and abs(k["avg_us"] - 4000.0) < 1e-9
    assert abs(rec["traffic_bytes_per_launch"] - (fetch_f32 + write_f32)) < 1
