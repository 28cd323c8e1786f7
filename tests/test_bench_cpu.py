"""Host-side checks of bench.py (CPU): the one-GPU refusal and the code hash
that keeps the measured traffic attached to the code it was taken on."""
import importlib.util
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
    assert b.traffic_entry(1, 1.0) is None


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
