"""The C ABI's behaviour on a live context: errors reported before any work
is enqueued (and the context left unchanged), storage types the adjoint does
not support, the stream a context runs on, independent contexts side by
side, optional outputs, and the padding the library must never touch."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1112_0850_amd import _abi as A
from paper_1112_0850_amd import inputs as I
from paper_1112_0850_amd.lbm import LBM
from tests.gpu_util import say

pytestmark = pytest.mark.gpu
P = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())


def _sim(storage="f32", shape=(6, 7, 70), **kw):
    flags = I.random_flags(shape, 5, solid_fraction=0.2, noforce_fraction=0.1)
    rng = np.random.default_rng(1)
    u0 = torch.from_numpy(0.03 * (rng.random((3,) + shape) - 0.5)).float()
    return LBM(shape, 0.7, (1e-4, 0, 0), storage, flags=flags, u0=u0, **kw)


def _bytes(sim):
    torch.cuda.synchronize()
    return sim.grids[sim.current].clone()


def test_argument_errors_leave_the_context_unchanged():
    say("argument errors on a live context")
    sim = _sim().step(3)
    before, t = _bytes(sim), sim.t
    with pytest.raises(A.LBMError) as e:
        A.lbm_step(sim.ctx, -1)
    assert e.value.status == A.LBM_E_ARG
    g = sim.grids[sim.current]
    with pytest.raises(A.LBMError) as e:
        A.lbm_step_from(sim.ctx, P(g), P(g))
    assert e.value.status == A.LBM_E_ARG and "differ" in str(e.value)
    other = sim.new_grid()
    with pytest.raises(A.LBMError) as e:
        A.lbm_step_from(sim.ctx, ctypes.c_void_p(g.data_ptr() + 16), P(other))
    assert "aligned" in str(e.value)
    with pytest.raises(A.LBMError) as e:
        A.lbm_set_current(sim.ctx, 2, 0)
    assert e.value.status == A.LBM_E_ARG
    with pytest.raises(A.LBMError):
        A.lbm_restore(sim.ctx, None, 0)
    for src, dst, what in ((P(g), P(g), "differ"), (None, P(other), "NULL"),
                           (ctypes.c_void_p(g.data_ptr() + 16), P(other), "aligned")):
        with pytest.raises(A.LBMError) as e:
            A.lbm_pull_copy(sim.ctx, src, dst)
        assert e.value.status == A.LBM_E_ARG and what in str(e.value)
    assert sim.t == t and torch.equal(_bytes(sim), before)
    sim.step(1)  # still usable
    assert sim.t == t + 1


@pytest.mark.parametrize("storage", ["f16", "bf16", "f64"])
def test_adjoint_rejects_unsupported_storage(storage):
    sim = _sim(storage)
    lam = torch.zeros(sim.grid_bytes // 4 + 64, dtype=torch.float32, device="cuda")
    part = torch.zeros(sim.adj_partials_bytes // 8, dtype=torch.float64, device="cuda")
    with pytest.raises(A.LBMError) as e:
        A.lbm_adjoint_seed(sim.ctx, P(sim.grids[sim.current]), None, None, P(lam), P(part))
    assert e.value.status == A.LBM_E_UNSUPPORTED


def test_steps_on_another_stream_match_the_default_stream():
    say("context on a second stream")
    ref = _sim().step(25)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        other = _sim()
    A.lbm_set_stream(other.ctx, ctypes.c_void_p(s.cuda_stream))
    other.stream = s
    other.step(25)
    s.synchronize()
    assert torch.equal(_bytes(ref), _bytes(other))


def test_graph_replays_across_a_stream_change():
    """Graphs replayed on one stream, the context moved to a second stream,
    replays there, then the graph length changed and the context destroyed:
    the results match plain launches and the graphs of the first stream are
    released only after their replays (waited through the replay event)."""
    say("graph replays across lbm_set_stream")
    ref = _sim().step(8 * 5 + 3)
    g = _sim().use_graphs(8)
    g.step(16)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    A.lbm_set_stream(g.ctx, ctypes.c_void_p(s.cuda_stream))
    g.stream = s
    g.step(8 * 3 + 3)
    g.use_graphs(4)  # waits for the latest replay (queued on s)
    s.synchronize()
    torch.cuda.synchronize()
    assert g.t == ref.t and torch.equal(_bytes(g), _bytes(ref))
    g.step(4)
    ref.step(4)
    s.synchronize()
    assert torch.equal(_bytes(g), _bytes(ref))
    del g


def test_graphs_released_after_their_replay_stream_is_destroyed():
    """Graphs replayed on a stream the caller then destroys: switching the
    graphs off afterwards waits for those replays through the event recorded
    after them (not on the dead stream) and succeeds; the results match
    plain launches."""
    say("graph replays on a destroyed stream")
    hip = ctypes.CDLL("libamdhip64.so.7")  # the runtime instance torch has loaded
    ref = _sim().step(8 * 4)
    g = _sim().use_graphs(8)
    torch.cuda.synchronize()
    s = ctypes.c_void_p()
    assert hip.hipStreamCreate(ctypes.byref(s)) == 0
    A.lbm_set_stream(g.ctx, s)
    g.step(8 * 4)
    A.lbm_set_stream(g.ctx, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert hip.hipStreamDestroy(s) == 0
    g.use_graphs(0)
    assert torch.equal(_bytes(g), _bytes(ref))


def test_interleaved_contexts_are_independent():
    say("interleaved contexts")
    a, b = _sim("f32"), _sim("f16", f16_scale_log2=10)
    ra, rb = _sim("f32").step(30), _sim("f16", f16_scale_log2=10).step(30)
    for _ in range(10):
        a.step(2)
        b.step(3)
        a.step(1)
    assert a.t == 30 and b.t == 30
    assert torch.equal(_bytes(a), _bytes(ra)) and torch.equal(_bytes(b), _bytes(rb))


def test_optional_outputs_and_padding():
    """Either macroscopic output may be NULL; after steps the padding of both
    grids is still zero (pads are never computed or written)."""
    sim = _sim("f32").step(5)
    rho, u = sim.macroscopics()
    rho2 = torch.empty_like(rho)
    u2 = torch.empty_like(u)
    A.lbm_macroscopics(sim.ctx, P(rho2), None)
    A.lbm_macroscopics(sim.ctx, None, P(u2))
    torch.cuda.synchronize()
    assert torch.equal(rho, rho2) and torch.equal(u, u2)
    nx = sim.shape[2]
    for g in sim.grids:
        assert not sim.grid_view(g)[..., nx:].any()


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_graph_replays_match_plain_launches(storage):
    """lbm_use_graphs: every replay (interleaved with eager steps of odd
    counts, so both starting grids get a graph, with macroscopics reads and
    synchronisations in between) leaves the same bytes as launching every
    step; changing and switching off the graph length keeps it so."""
    say("graph replays vs plain launches", storage)
    kw = dict(f16_scale_log2=10) if storage == "f16" else {}
    g, e = _sim(storage, **kw).use_graphs(8), _sim(storage, **kw)
    plan = [8, 3, 16, 5, 8, 24, 1, 8]
    for n in plan:
        g.step(n)
        e.step(n)
        rg, _ = g.macroscopics()
        re, _ = e.macroscopics()
        torch.cuda.synchronize()
        assert g.t == e.t and g.current == e.current
        assert torch.equal(_bytes(g), _bytes(e)), n
        assert torch.equal(rg, re)
    g.use_graphs(4)
    g.step(12)
    e.step(12)
    assert torch.equal(_bytes(g), _bytes(e))
    g.use_graphs(0)
    g.step(9)
    e.step(9)
    assert torch.equal(_bytes(g), _bytes(e))
    with pytest.raises(A.LBMError):
        g.use_graphs(3)
