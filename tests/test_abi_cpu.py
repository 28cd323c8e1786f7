"""Host-side checks of the C ABI (no GPU): the library loads and exports
every symbol include/lbm.h declares, its tables match the interface order,
its byte model matches the paper's (Sec. 4), sizes are as documented, and
invalid arguments are rejected on the host with a message."""
import ctypes
import json
import math
import os
import re

import pytest

from paper_1112_0850_amd import _abi as A
from tests import lattice_ref as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_A-Z]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = A.lib()
    names = _declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(A._SIGNATURES), "binding and header disagree"


def test_lattice_tables_match_interface_order():
    e, w, opp = A.lbm_lattice()
    e_r, w_r, opp_r = R.e_w_opp()
    assert [tuple(map(int, c)) for c in e_r] == e
    assert list(w_r) == w
    assert list(opp_r) == opp


def test_byte_model_matches_paper():
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "byte_model.json")))
    assert A.lbm_bytes_per_update(A.LBM_F32) == gold["bytes_per_update_gpu"]["sp"]
    assert A.lbm_bytes_per_update(A.LBM_F64) == gold["bytes_per_update_gpu"]["dp"]
    assert A.lbm_bytes_per_update(A.LBM_F16) == 76
    assert A.lbm_bytes_per_update(A.LBM_BF16) == 76
    assert A.lbm_bytes_per_update(A.LBM_F32X) == 152
    assert A.lbm_bytes_per_update(7) == 0
    # the CPU variant adds the write-allocate transfer: 3 transfers per PDF
    assert 19 * 3 * 4 == gold["bytes_per_update_cpu_write_allocate"]["sp"]
    assert 19 * 3 * 8 == gold["bytes_per_update_cpu_write_allocate"]["dp"]
    # Table 4: the model is STREAM bandwidth / bytes per update
    node = gold["table4_mflups"]["Intel X5650 node"]
    assert round(node["stream_gbs"] * 1e3 / 228) == node["sp"]
    assert round(node["stream_gbs"] * 1e3 / 456) == node["dp"]
    for row in ("C2070", "C2070 ECC", "C1060"):
        r = gold["table4_mflups"][row]
        assert abs(r["sp"] * 152 - r["dp"] * 304) <= 304  # one bandwidth behind both columns


@pytest.mark.parametrize("shape,storage,align,xs", [
    ((4, 5, 1), A.LBM_F32, 0, 64), ((3, 2, 65), A.LBM_F32, 0, 128), ((3, 2, 65), A.LBM_F64, 1, 65),
    ((512, 512, 512), A.LBM_F16, 0, 512), ((2, 2, 100), A.LBM_BF16, 16, 112)])
def test_query_sizes(shape, storage, align, xs):
    p = A.params(shape, 0.6, storage=storage, x_align=align)
    x_stride, ds, gb, sb, ab = A.lbm_query(p)
    es = {A.LBM_F32: 4, A.LBM_F64: 8, A.LBM_F16: 2, A.LBM_BF16: 2}[storage]
    nz, ny, nx = shape
    assert x_stride == xs
    assert ds == nz * ny * xs + 256 // es  # 256 bytes between direction arrays
    assert gb >= 19 * ds * es and gb % 256 == 0 and gb - 19 * ds * es < 256
    assert sb == 1024 * 5 * 8
    nblocks = -(-(-(-nx // 64) * ny * nz) // 4)
    assert ab == nblocks * 3 * 8


def test_query_limits():
    A.lbm_query(A.params((768, 768, 768), 0.55, storage=A.LBM_F32))
    A.lbm_query(A.params((640, 640, 640), 0.55, storage=A.LBM_F64))
    with pytest.raises(A.LBMError) as e:
        A.lbm_query(A.params((1024, 1024, 1024), 0.55, storage=A.LBM_F32))
    assert e.value.status == A.LBM_E_UNSUPPORTED


@pytest.mark.parametrize("kw,msg", [
    (dict(shape=(0, 4, 4), tau=0.6), "dimensions"),
    (dict(shape=(4, 4, 4), tau=0.5), "tau"),
    (dict(shape=(4, 4, 4), tau=float("nan")), "tau"),
    (dict(shape=(4, 4, 4), tau=-math.inf), "tau"),
    (dict(shape=(4, 4, 4), tau=0.6, force=(math.inf, 0, 0)), "force"),
    (dict(shape=(4, 4, 4), tau=0.6, storage=9), "storage"),
    (dict(shape=(4, 4, 4), tau=0.6, storage=A.LBM_F16, f16_scale_log2=30), "scale"),
    (dict(shape=(4, 4, 4), tau=0.6, x_align=-2), "x_align"),
    (dict(shape=(4, 4, 4), tau=0.6, wall_u=(0, math.nan, 0)), "wall_u"),
    (dict(shape=(4, 4, 4), tau=0.6, equilibrium=2), "equilibrium"),
])
def test_invalid_params_rejected(kw, msg):
    with pytest.raises(A.LBMError) as e:
        A.lbm_query(A.params(**kw))
    assert e.value.status == A.LBM_E_ARG
    assert msg in str(e.value)


def test_params_layout_and_obstacle_field():
    # six int32, tau, force[3], wall_u[3], equilibrium, obstacle_kernel, steps_per_pass:
    # 92 bytes padded to 96 (the library checks the same layout at compile time)
    assert ctypes.sizeof(A.lbm_params) == 96
    assert A.lbm_params.wall_u.offset == 56 and A.lbm_params.equilibrium.offset == 80
    assert A.lbm_params.steps_per_pass.offset == 88
    p = A.params((4, 4, 4), 0.6, wall_u=(0.1, 0, 0), equilibrium=A.LBM_EQ_INCOMPRESSIBLE)
    A.lbm_query(p)
    p.obstacle_kernel = 1
    A.lbm_query(p)
    p.obstacle_kernel = 2
    with pytest.raises(A.LBMError) as e:
        A.lbm_query(p)
    assert e.value.status == A.LBM_E_ARG and "obstacle_kernel" in str(e.value)


def test_infinite_tau_accepted():
    A.lbm_query(A.params((4, 4, 4), math.inf))


def test_init_argument_errors_before_any_gpu_work():
    p = A.params((4, 4, 4), 0.6)
    fake = ctypes.c_void_p(0x10000)
    with pytest.raises(A.LBMError) as e:
        A.lbm_init(p, None, fake, None, fake, None, None, None)
    assert e.value.status == A.LBM_E_ARG and "grid" in str(e.value)
    with pytest.raises(A.LBMError) as e:
        A.lbm_init(p, fake, fake, None, fake, None, None, None)
    assert "differ" in str(e.value)
    with pytest.raises(A.LBMError) as e:
        A.lbm_init(p, ctypes.c_void_p(0x10010), fake, None, fake, None, None, None)
    assert "aligned" in str(e.value)
    with pytest.raises(A.LBMError) as e:
        A.lbm_init(p, fake, ctypes.c_void_p(0x20000), None, None, None, None, None)
    assert "scratch" in str(e.value)
    assert A.lbm_last_error() != ""


def test_null_context_rejected():
    with pytest.raises(A.LBMError) as e:
        A.lbm_step(None, 1)
    assert e.value.status == A.LBM_E_ARG
    with pytest.raises(A.LBMError):
        A.lbm_reduce(None, None)
    with pytest.raises(A.LBMError) as e:
        A.lbm_step2_from(None, ctypes.c_void_p(0x100), ctypes.c_void_p(0x200), ctypes.c_void_p(0x300))
    assert e.value.status == A.LBM_E_ARG
    assert A.lbm_current(None) == -1 and A.lbm_time(None) == -1
    with pytest.raises(A.LBMError):
        A.lbm_stream_copy(ctypes.c_void_p(0x100), ctypes.c_void_p(0x200), 17, None)


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """Without the built HIP library every call raises: there is no fallback."""
    monkeypatch.setattr(A, "_lib", None)
    monkeypatch.setattr(A, "LIB_PATH", str(tmp_path / "liblbm.so"))
    with pytest.raises(ImportError, match="no CPU fallback"):
        A.lib()
    with pytest.raises(ImportError):
        A.lbm_query(A.params((4, 4, 4), 0.7))


def _header_define(name):
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    m = re.search(rf"#define {name} (0x[0-9A-Fa-f]+)u?l?l?", src)
    return int(m.group(1), 16)


@pytest.mark.parametrize("storage,bits,expo,quiet", [
    (A.LBM_F32, 32, 8, 22), (A.LBM_F32X, 32, 8, 22), (A.LBM_F64, 64, 11, 51),
    (A.LBM_F16, 16, 5, 9), (A.LBM_BF16, 16, 8, 6)])
def test_solid_markers_are_reserved_quiet_nans(storage, bits, expo, quiet):
    """Each marker is a quiet NaN of its format with the sign bit set and a
    non-zero payload beyond the quiet bit -- neither the default NaN of
    arithmetic (positive, empty payload) nor an infinity -- the two differ in
    bit 0 only, and they are the values the header defines."""
    rest, mov = A.lbm_solid_markers(storage)
    assert mov == rest | 1 and rest & 1 == 0
    mant = bits - 1 - expo
    for v in (rest, mov):
        assert v >> (bits - 1) == 1                               # sign
        assert (v >> mant) & ((1 << expo) - 1) == (1 << expo) - 1  # all-ones exponent
        assert (v >> quiet) & 1 == 1                               # quiet NaN
        assert v & ((1 << quiet) - 1) != 0                         # payload
    name = {A.LBM_F32: "F32", A.LBM_F32X: "F32", A.LBM_F64: "F64", A.LBM_F16: "F16",
            A.LBM_BF16: "BF16"}[storage]
    assert rest == _header_define(f"LBM_MARK_{name}_REST")
    assert mov == _header_define(f"LBM_MARK_{name}_MOVING")
    with pytest.raises(A.LBMError):
        A.lbm_solid_markers(9)


def test_copy_probe_argument_errors():
    a, c = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000)
    for args in [(c, a, 17, 1, 0, 0), (c, a, 64, 3, 0, 0), (c, a, 64, 1, 2, 0),
                 (c, a, 64, 1, 0, -1), (ctypes.c_void_p(0x20010), a, 64, 1, 0, 0), (None, a, 64, 1, 0, 0)]:
        with pytest.raises(A.LBMError) as e:
            A.lbm_copy_probe(*args, None)
        assert e.value.status == A.LBM_E_ARG
    A.lbm_copy_probe(c, a, 0, 4, 1, 0, None)  # nothing to copy: no launch


def test_steps_per_pass_option():
    for v in (0, 1, 2, -1, "auto"):
        A.lbm_query(A.params((4, 4, 4), 0.6, steps_per_pass=v))
    A.lbm_query(A.params((4, 4, 4), 0.6, steps_per_pass="auto", obstacle_kernel=1))
    with pytest.raises(A.LBMError) as e:
        A.lbm_query(A.params((4, 4, 4), 0.6, steps_per_pass=-2))
    assert e.value.status == A.LBM_E_ARG
    with pytest.raises(A.LBMError) as e:
        A.lbm_query(A.params((4, 4, 4), 0.6, steps_per_pass=3))
    assert e.value.status == A.LBM_E_ARG and "steps_per_pass" in str(e.value)
    with pytest.raises(A.LBMError) as e:
        A.lbm_query(A.params((4, 4, 4), 0.6, steps_per_pass=2, obstacle_kernel=1))
    assert e.value.status == A.LBM_E_UNSUPPORTED


def test_scratch_holds_the_link_mask_where_pairs_may_run():
    """scratch_bytes: the reduction's partials, plus 4 bytes per cell (the
    two-step pass's link mask) when steps_per_pass is 2 or automatic -- not
    with single steps, the split design, or where a pair of direction arrays
    would span 4 GiB (the pass then keeps the marker test)."""
    shape = (10, 20, 30)
    sb = lambda **kw: A.lbm_query(A.params(shape, 0.6, **kw))[3]
    base = sb()
    assert base % 256 == 0 and sb(steps_per_pass=1) == base
    mask = (10 * 20 * 30 * 4 + 255) // 256 * 256
    assert sb(steps_per_pass=2) == base + mask
    assert sb(steps_per_pass="auto") == base + mask
    assert sb(steps_per_pass="auto", obstacle_kernel=1) == base
    # 1023^3 FP32 (x_stride 1024): one direction array fits 4 GiB, two do not
    big = A.lbm_query(A.params((1023, 1023, 1023), 0.6, steps_per_pass=2))[3]
    assert big == base
    # 768^3 FP32: two arrays of 1.8 GB, the mask is 1.8 GB
    large = A.lbm_query(A.params((768, 768, 768), 0.6, steps_per_pass=2))[3]
    assert large == base + 768 ** 3 * 4
    # FP64: 640^3 (two arrays of 2.1 GB: 4.19 GB < 4 GiB) has the mask, 650^3
    # (704-cell rows: two arrays of 2.4 GB) does not
    f64 = lambda n: A.lbm_query(A.params((n, n, n), 0.6, storage=A.LBM_F64, steps_per_pass=2))[3]
    assert f64(640) == base + 640 ** 3 * 4 and f64(650) == base
