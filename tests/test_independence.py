"""The oracle and the HIP path share no code (CPU): the product package never
imports, loads or names the oracle's library; the oracle never includes or
imports the package; and only the test-suite, the smoke check and the CPU
baseline leg of the benchmark reach the oracle.  Only the seeded input
generators (`paper_1112_0850_amd/inputs.py`, no arithmetic of the method)
serve both sides."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1112_0850_amd")
ORACLE = os.path.join(ROOT, "oracle")


def _files(top, exts):
    for d, _, names in os.walk(top):
        if "__pycache__" in d:
            continue
        for n in names:
            if n.endswith(exts):
                yield os.path.join(d, n)


def _code(path):
    """Source text, with C and C++ comments removed from native sources."""
    text = open(path).read()
    if path.endswith((".c", ".h", ".hip")):
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
    return text


def test_product_does_not_reach_the_oracle():
    for f in _files(PKG, (".py", ".hip", ".h", ".c", ".cpp")):
        code = _code(f)
        assert not re.search(r"^\s*(from|import)\s+oracle\b", code, re.M), f
        assert "liboracle" not in code and "lbm_oracle" not in code, f
        assert not re.search(r'#\s*include\s*["<][^">]*oracle', code), f


def test_oracle_does_not_reach_the_product():
    for f in _files(ORACLE, (".py", ".c", ".h")):
        code = _code(f)
        assert not re.search(r"^\s*(from|import)\s+paper_1112_0850_amd\b", code, re.M), f
        assert "liblbm" not in code and "csrc" not in code, f
        assert not re.search(r'#\s*include\s*["<][^">]*(lbm\.h|d3q19|kernels)', code), f


def test_only_allowed_callers_use_the_oracle():
    allowed = {os.path.join(ROOT, "bench.py"), os.path.join(ROOT, "__graft_entry__.py")}
    for f in _files(ROOT, (".py",)):
        rel = os.path.relpath(f, ROOT)
        if rel.startswith(("tests", "oracle", "_work")) or f in allowed:
            continue
        code = _code(f)
        assert not re.search(r"^\s*(from|import)\s+oracle\b", code, re.M), rel
