#!/usr/bin/env python3
"""Benchmark of the D3Q19 BGK hot path on one MI355X.

Workload (the headline): porous periodic box 512^3, 10% solid from random
non-overlapping spheres of radius 4-12 (seed 12345), tau = 0.55, body force
g_x = 1e-6, fluid initially at rest; FP32 offset storage, pairs of steps
fused into one temporally blocked pass (bit-identical to single steps).  One
"step" is one stream-collide update of the whole box (a launch performs two).
Reported beside it, on the same geometry: the single-step kernel, FP16-offset
and BF16-offset storage (FP32 collide) and FP64 storage, one and two steps
per pass; the adjoint/forward time ratio of the
differentiable rollout (periodic 128^3, 400 steps, checkpoints every 20);
the STREAM-copy bandwidth of the GPU; and the FP64 CPU oracle timed on this
host's cores on a bounded sample (the 128^3 crop of the same geometry).

Output: one JSON line on stdout.  Inputs are synthetic and seeded, resident
in HBM before the timed region starts.
"""
import argparse
import glob
import hashlib
import re
import json
import math
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SRCS = [os.path.join(ROOT, "paper_1112_0850_amd", "csrc", f)
               for f in ("kernels.hip", "kernels.h", "d3q19.h", "abi.hip")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_porous512_f32.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=980,
                    help="timed steps of the headline legs (FP32, FP16, BF16); with the warm-up "
                         "they make the 1000 steps of the porous workload")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--aux-steps", type=int, default=200,
                    help="timed steps of the other legs (at most --steps)")
    ap.add_argument("--n", type=int, default=512, help="edge of the cubic porous box")
    ap.add_argument("--only", default="",
                    help="comma list of legs: f32,f16,bf16,f64,f32x (single steps), f32x2,f16x2,"
                         "bf16x2,f64x2 (two steps per pass),adjoint,copy,cpu,large,cavity,split,"
                         "incomp")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--sweep", action="store_true",
                    help="domain-size sweep instead of the headline run: periodic all-fluid cubes "
                         "N^3, padded (x_stride multiple of 64) vs unpadded, FP32/FP16/FP64; "
                         "prints one JSON line per point")
    ap.add_argument("--sweep-summary", metavar="SWEEP_JSONL",
                    help="print the markdown table of a --sweep output file and exit")
    ap.add_argument("--trace-summary", nargs=2, metavar=("TRACE_DIR", "BENCH_JSON"),
                    help="summarise a rocprofv3 kernel trace of the default run of this script "
                         "(split by kernel and box size, checked against the bench line it "
                         "printed) as markdown on stdout and exit")
    ap.add_argument("--profile-summary", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="summarise rocprofv3 CSV output (kernel trace, FETCH_SIZE and "
                         "WRITE_SIZE passes of this script) into profiles/ and exit")
    ap.add_argument("--valu-summary", nargs=2, metavar=("TRACE_DIR", "COUNTER_DIR"),
                    help="summarise a rocprofv3 --pmc SQ_INSTS_VALU SQ_ACTIVE_INST_VALU "
                         "SQ_BUSY_CYCLES GRBM_GUI_ACTIVE pass of this script (vector-instruction "
                         "issue of the step kernels at the porous 512^3 box) as markdown and exit")
    ap.add_argument("--stall-summary", nargs=1, metavar="COUNTER_DIR",
                    help="summarise a rocprofv3 --pmc SQ_WAVE_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY "
                         "SQ_ACTIVE_INST_ANY ... pass of this script (where the step kernels' "
                         "waves spend their time at the porous 512^3 box) as markdown and exit")
    return ap.parse_args()


REPS = 5


def rep_sizes(steps, reps, unit=1):
    """Steps of each timed repetition: `steps` split into at most `reps`
    near-equal parts that are multiples of `unit`, any remainder going to
    the last part."""
    units, rem = divmod(steps, unit)
    reps = max(1, min(reps, units))
    sizes = [unit * (units // reps + (1 if r < units % reps else 0)) for r in range(reps)]
    sizes[-1] += rem
    return sizes


def timed_steps(sim, torch, steps, warmup, clocks=None, detail=None, reps=REPS, unit=1):
    """Milliseconds per fused step: `warmup` untimed steps, then exactly
    `steps` timed steps bracketed by device synchronisation, split into
    `reps` consecutive repetitions whose HIP events (recorded on the solver's
    stream) give one per-step time each; returns their median.  Each
    repetition holds a multiple of `unit` steps (the steps one launch
    performs), any remainder going to the last.  With a dict `detail`, also
    the minimum, maximum, every repetition and the plain average over all
    `steps`.  With a dict `clocks`, a timer thread reads the GPU clocks
    (sysfs) 0.5 s into the timed steps."""
    import statistics
    sim.step(warmup)
    torch.cuda.synchronize()
    sizes = rep_sizes(steps, reps, unit)
    reps = len(sizes)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    timer = None
    if clocks is not None:
        timer = threading.Timer(0.5, lambda: clocks.update(gpu_clocks() or {}))
    ev[0].record(sim.stream)
    if timer:
        timer.start()
    for r, n in enumerate(sizes):
        sim.step(n)
        ev[r + 1].record(sim.stream)
    torch.cuda.synchronize()
    if timer:
        timer.join()
    per = [ev[r].elapsed_time(ev[r + 1]) / sizes[r] for r in range(reps)]
    med = statistics.median(per)
    if detail is not None:
        detail.update({"reps": reps, "steps_per_rep": sizes, "ms_median": med, "ms_min": min(per),
                       "ms_max": max(per), "ms_reps": per,
                       "ms_mean_all": ev[0].elapsed_time(ev[-1]) / steps})
    return med


def pull_copy_ms(sim, torch, reps=40):
    """Average time of the pull-copy probe on this grid layout (current grid
    into the other one, which the next step overwrites anyway)."""
    src, dst = sim.grids[sim.current], sim.grids[sim.current ^ 1]
    for _ in range(3):
        sim.pull_copy(src, dst)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    for _ in range(reps):
        sim.pull_copy(src, dst)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def forward_leg(torch, LBM, flags_t, n_cells, n_fluid, storage, steps, warmup, s=0,
                fields=None, clocks=None, pull=False, **kw):
    """Times `steps` steps after `warmup`; with a dict `fields`, stores the
    final (rho, u) there (FP64, on the GPU) for the cross-storage comparison;
    with `pull`, also times the pull-copy probe on the same grids."""
    from paper_1112_0850_amd import _abi as A
    n = round(n_cells ** (1 / 3))
    sim = LBM((n, n, n), 0.55, (1e-6, 0.0, 0.0), storage, flags=flags_t, f16_scale_log2=s, **kw)
    rep = {}
    spl = kw.get("steps_per_pass") or 1
    ms = timed_steps(sim, torch, steps, warmup, clocks, detail=rep, unit=spl)
    r = sim.reduce().cpu().numpy()
    if fields is not None:
        fields[storage] = sim.macroscopics(f64=True)
    pc = pull_copy_ms(sim, torch) if pull else None
    bpu = A.lbm_bytes_per_update(sim.storage)
    alg_bytes = bpu * n_fluid + n_cells  # populations of fluid cells + one flag byte per cell
    out = {
        "storage": storage, "timed_steps": steps, "ms_per_step": ms,
        "mlups": n_cells / ms / 1e3, "mflups": n_fluid / ms / 1e3,
        "bytes_per_update": bpu, "alg_bytes_per_step": alg_bytes,
        "alg_gbs": alg_bytes / ms / 1e6, "hbm_frac": alg_bytes / ms / 1e6 / HBM_PEAK_GBS,
        "mass": float(r[0]), "finite": bool(all(math.isfinite(float(v)) for v in r)),
        "timing": rep, "steps_per_launch": spl,
    }
    if storage == "f16":
        out["f16_scale_log2"] = s
    if pc:
        # the same loads and stores without geometry or collision, all cells
        out["pull_copy"] = {"ms": pc, "gbs": bpu * n_cells / pc / 1e6,
                            "step_time_over_probe": ms / pc}
    del sim
    torch.cuda.empty_cache()
    return out


def large_leg(torch, storage, n, steps=100, warmup=6, steps_per_pass=0):
    """Large box (5% solid random spheres r 4-12, seed 777, tau 0.55,
    g_x 1e-6, from rest): sustained MLUPS, bandwidth and FP64 mass drift;
    `steps_per_pass` = 2 runs fused pairs of steps."""
    from paper_1112_0850_amd import _abi as A
    from paper_1112_0850_amd import inputs as I
    from paper_1112_0850_amd.lbm import LBM
    flags = I.sphere_pack((n, n, n), 0.05, seed=777)
    n_cells, n_fluid = n ** 3, int((flags & 1 == 0).sum())
    sim = LBM((n, n, n), 0.55, (1e-6, 0.0, 0.0), storage, flags=torch.from_numpy(flags).cuda(),
              steps_per_pass=steps_per_pass)
    m0 = float(sim.reduce()[0].item())
    ms = timed_steps(sim, torch, steps, warmup, unit=max(1, steps_per_pass))
    m1 = float(sim.reduce()[0].item())
    bpu = A.lbm_bytes_per_update(sim.storage)
    alg = bpu * n_fluid + n_cells
    sched = ", two steps per pass" if steps_per_pass == 2 else ""
    out = {"workload": f"{n}^3 porous 5% spheres seed 777, {storage}{sched}",
           "grid_gb": 2 * sim.grid_bytes / 1e9,
           "ms_per_step": ms, "mlups": n_cells / ms / 1e3, "mflups": n_fluid / ms / 1e3,
           "alg_gbs": alg / ms / 1e6, "hbm_frac": alg / ms / 1e6 / HBM_PEAK_GBS,
           "mass_drift_rel": abs(m1 - m0) / m0, "steps": steps + warmup}
    del sim
    torch.cuda.empty_cache()
    return out


def cavity_leg(torch, storage, n, steps, warmup, s=0):
    """Lid-driven cavity (the paper's verification workload, Sec. 7): n^3 box
    with a one-cell solid layer on all faces, the top plane moving with
    (0.05, 0, 0), tau 0.55, from rest -- the moving-wall step kernel."""
    from paper_1112_0850_amd import _abi as A
    from paper_1112_0850_amd import inputs as I
    from paper_1112_0850_amd.lbm import LBM
    flags = I.cavity_flags((n, n, n))
    sim = LBM((n, n, n), 0.55, (0.0, 0.0, 0.0), storage, flags=torch.from_numpy(flags).cuda(),
              wall_u=(0.05, 0.0, 0.0), f16_scale_log2=s)
    m0 = float(sim.reduce()[0].item())
    ms = timed_steps(sim, torch, steps, warmup)
    m1 = float(sim.reduce()[0].item())
    n_fluid = (n - 2) ** 3
    alg = A.lbm_bytes_per_update(sim.storage) * n_fluid + n ** 3
    out = {"workload": f"{n}^3 lid-driven cavity, lid (0.05, 0, 0), tau 0.55, {storage}",
           "timed_steps": steps, "ms_per_step": ms, "mlups": n ** 3 / ms / 1e3,
           "mflups": n_fluid / ms / 1e3,
           "alg_gbs": alg / ms / 1e6, "hbm_frac": alg / ms / 1e6 / HBM_PEAK_GBS,
           "mass_drift_rel": abs(m1 - m0) / m0}
    if storage == "f16":
        out["f16_scale_log2"] = s
    del sim
    torch.cuda.empty_cache()
    return out


SWEEP_N = (32, 48, 64, 80, 96, 100, 128, 160, 192, 200, 250, 256, 300, 320, 384, 400, 448, 500,
           512, 576, 640, 700, 768)


def sweep(torch, storages=("f32", "f16", "f64"), sizes=SWEEP_N):
    """MLUPS against the edge N of a periodic all-fluid cube (tau 0.6, no
    force, at rest), with the x-stride padded to 64 cells or not padded
    (the paper's domain sweep with and without padding, Sec. 7).  Each
    point: the median of 5 timed repetitions (timed_steps); when N is a
    multiple of 64 both layouts are the same and the point is timed once.
    Up to N = 160 the padded layout is also timed with replayed graphs of
    32 steps, and every padded point once more with two steps per pass."""
    from paper_1112_0850_amd.lbm import LBM
    for st in storages:
        for n in sizes:
            for align in (0, 1):
                if align == 1 and n % 64 == 0:
                    continue
                sim = LBM((n, n, n), 0.6, (0.0, 0.0, 0.0), st, x_align=align)
                steps = max(10, min(400, int(2e9 / n ** 3)))
                rep = {}
                ms = timed_steps(sim, torch, steps, max(3, steps // 10), detail=rep)
                rec = {"sweep": st, "n": n, "padded": align == 0 or n % 64 == 0,
                       "x_stride": sim.x_stride, "same_layout": n % 64 == 0,
                       "ms_per_step": ms, "ms_min": rep["ms_min"], "ms_max": rep["ms_max"],
                       "mlups": n ** 3 / ms / 1e3, "grid_gb": 2 * sim.grid_bytes / 1e9}
                if align == 0 and n <= 160:  # launch-bound sizes: replayed step graphs
                    sim.use_graphs(32)
                    msg = timed_steps(sim, torch, 320, 64)
                    rec["graph_mlups"] = n ** 3 / msg / 1e3
                del sim
                if align == 0:  # the same box in fused pairs of steps
                    sim = LBM((n, n, n), 0.6, (0.0, 0.0, 0.0), st, steps_per_pass=2)
                    ms2 = timed_steps(sim, torch, steps + steps % 2, max(4, steps // 10 * 2),
                                      unit=2)
                    rec["two_step_mlups"] = n ** 3 / ms2 / 1e3
                    del sim
                print(json.dumps(rec), flush=True)
            torch.cuda.empty_cache()
    return 0


def sweep_summary(path):
    """Markdown table of the JSON lines `--sweep` printed (MLUPS, padded /
    unpadded, with graphs where timed, and the padded box in fused pairs of
    steps, per storage and edge N)."""
    rows = [json.loads(l) for l in open(path) if l.startswith("{")]
    sts = sorted({r["sweep"] for r in rows}, key=["f32", "f16", "bf16", "f64"].index)
    ns = sorted({r["n"] for r in rows})
    out = ["| N | " + " | ".join(f"{st.upper()} padded / unpadded MLUPS" for st in sts) + " |",
           "|---|" + "---|" * len(sts)]
    for n in ns:
        cells = []
        for st in sts:
            pad = [r for r in rows if r["sweep"] == st and r["n"] == n and r["padded"]]
            unp = [r for r in rows if r["sweep"] == st and r["n"] == n and not r["padded"]]
            c = f"{pad[0]['mlups'] / 1e3:.1f}k" if pad else "-"
            if unp:
                c += f" / {unp[0]['mlups'] / 1e3:.1f}k"
            if pad and "graph_mlups" in pad[0]:
                c += f" (graphs {pad[0]['graph_mlups'] / 1e3:.1f}k)"
            if pad and "two_step_mlups" in pad[0]:
                c += f"; two steps per pass {pad[0]['two_step_mlups'] / 1e3:.1f}k"
            cells.append(c)
        out.append(f"| {n} | " + " | ".join(cells) + " |")
    print("\n".join(out))
    return 0


def copy_leg(torch):
    """STREAM copy c = a of 4 GiB (the paper's Sec. 3 case study): the
    library's default copy kernel (one 16-byte element per thread), and a
    sweep over the copy's variants -- 1, 2 or 4 elements per thread per pass,
    plain or non-temporal accesses, one pass or a grid of 1024-16384 blocks
    striding through the array -- whose best is the attainable bandwidth
    (median of 10 timed repetitions each)."""
    import statistics
    from paper_1112_0850_amd.lbm import copy_probe, stream_copy
    nbytes = 4 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    c = torch.empty_like(a)
    a.fill_(1)

    def timed(fn, reps=10):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record()
        for r in range(reps):
            fn()
            ev[r + 1].record()
        torch.cuda.synchronize()
        return statistics.median(ev[r].elapsed_time(ev[r + 1]) for r in range(reps))

    ms = timed(lambda: stream_copy(c, a))
    sweep_rows = []
    for vec in (1, 2, 4):
        for nt in (False, True):
            for blocks in (0, 1024, 2048, 4096, 8192, 16384):
                m = timed(lambda: copy_probe(c, a, vec, nt, blocks))
                sweep_rows.append({"vec_per_thread": vec, "nontemporal": nt, "blocks": blocks,
                                   "gbs": 2 * nbytes / m / 1e6})
    best = max(sweep_rows, key=lambda r: r["gbs"])
    del a, c
    torch.cuda.empty_cache()
    return {"bytes": 2 * nbytes, "ms": ms, "gbs": 2 * nbytes / ms / 1e6,
            "best": best, "sweep": sweep_rows}


def adjoint_leg(torch, n=128, steps=400, k=20):
    """Forward vs backward time of the differentiable rollout (128^3 periodic,
    smooth random u0 amplitude 0.02, g = (1e-6, 0, 0), tau = 0.6)."""
    from paper_1112_0850_amd import inputs as I
    from paper_1112_0850_amd import _abi as A
    from paper_1112_0850_amd.lbm import LBM, rollout
    u0 = torch.from_numpy(I.smooth_field(n, 2024, amplitude=0.02)).float().cuda()
    target = torch.from_numpy(I.smooth_field(n, 7, amplitude=0.02)).float().cuda()
    g = torch.tensor([1e-6, 0.0, 0.0], dtype=torch.float64, requires_grad=True)
    u0.requires_grad_(True)

    def run():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho, u = rollout(u0, g, steps=steps, tau=0.6, checkpoint_every=k)
        loss = ((u - target) ** 2).mean()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    run()  # warm-up (allocations, first launches)
    u0.grad = None
    g.grad = None
    tf, tb = run()
    # the same forward sweep in fused pairs of steps (the same states, so the
    # same backward)
    with torch.no_grad():
        rollout(u0.detach(), g.detach(), steps=steps, tau=0.6, checkpoint_every=k, steps_per_pass=2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rollout(u0.detach(), g.detach(), steps=steps, tau=0.6, checkpoint_every=k, steps_per_pass=2)
        torch.cuda.synchronize()
        tf2 = time.perf_counter() - t0
    # pure kernel times at the same size: forward step vs adjoint step
    sim = LBM((n, n, n), 0.6, (1e-6, 0, 0), "f32", u0=u0.detach())
    ms_fwd = timed_steps(sim, torch, 200, 20)
    lam = [torch.zeros(sim.grid_bytes // 4, dtype=torch.float32, device="cuda") for _ in range(2)]
    part = torch.zeros(sim.adj_partials_bytes // 8, dtype=torch.float64, device="cuda")
    import ctypes
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    fst = sim.grids[sim.current]
    for _ in range(10):
        A.lbm_adjoint_step(sim.ctx, P(fst), P(lam[0]), P(lam[1]), P(part))
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    for i in range(200):
        A.lbm_adjoint_step(sim.ctx, P(fst), P(lam[i & 1]), P(lam[(i + 1) & 1]), P(part))
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms_adj = e0.elapsed_time(e1) / 200
    cells = n ** 3
    out = {
        "workload": f"periodic {n}^3 FP32, tau 0.6, {steps} steps, checkpoints every {k}",
        "forward_s": tf, "backward_s": tb, "bwd_over_fwd": tb / tf,
        "forward_s_two_steps_per_pass": tf2, "bwd_over_fwd_two_steps_per_pass": tb / tf2,
        "fwd_step_ms": ms_fwd, "adj_step_ms": ms_adj, "adj_kernel_over_fwd_kernel": ms_adj / ms_fwd,
        "adj_kernel_alg_gbs": 228 * cells / ms_adj / 1e6,
        "grad_finite": bool(torch.isfinite(u0.grad).all().item() and torch.isfinite(g.grad).all().item()),
    }
    del sim, lam, part
    torch.cuda.empty_cache()
    return out


def cpu_leg(flags_np, seconds):
    """The FP64 oracle (plain loops, OpenMP) on the 128^3 crop of the same
    geometry, timed on this host: a bounded sample of about `seconds` on all
    host threads, and a shorter one on one thread.  Also the host's STREAM
    copy bandwidth and the oracle's fraction of the paper's CPU model (copy
    bandwidth / 456 B per FP64 fluid update with write-allocate, Sec. 4)."""
    import numpy as np
    from oracle import oracle as O
    crop = np.ascontiguousarray(flags_np[:128, :128, :128])
    shape = crop.shape
    cells = int(np.prod(shape))
    fluid = int((crop & 1 == 0).sum())

    def timed(budget, chunk):
        f = O.init(shape, crop)
        f = O.step(f, 0.55, (1e-6, 0, 0), crop, n=1)  # warm-up (threads, pages)
        nsteps, dt = 0, 0.0
        while dt < budget:  # whole chunks of steps until the time budget is spent
            t0 = time.perf_counter()
            f = O.step(f, 0.55, (1e-6, 0, 0), crop, n=chunk)
            dt += time.perf_counter() - t0
            nsteps += chunk
        return nsteps, dt, f

    threads = O.threads()
    nsteps, dt, f_end = timed(seconds, 5)
    O.set_threads(1)
    n1, dt1, _ = timed(seconds / 4, 1)
    O.set_threads(threads)
    copy = O.host_copy_gbs()
    model_mflups = copy * 1e3 / 456
    mflups = fluid * nsteps / dt / 1e6
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            model = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": cells * nsteps / dt / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"FP64 oracle, {nsteps} steps of the 128^3 crop of the porous geometry "
                      f"({fluid} fluid cells), {dt:.1f} s",
            "mflups": mflups, "one_thread_mlups": cells * n1 / dt1 / 1e6,
            "one_thread_sample": f"{n1} steps, {dt1:.1f} s", "host_cpu": model,
            "host_copy_gbs": copy, "model_mflups_456B": model_mflups,
            "frac_of_model": mflups / model_mflups,
            "_state": (crop, nsteps + 1, f_end)}


def crop_error_leg(torch, crop, nsteps, f_ref):
    """The error against the FP64 oracle for every storage on the oracle's
    own sample: the 128^3 crop run as its own periodic box (tau 0.55,
    g_x 1e-6, from rest) for the same number of steps on the GPU; relative
    L-inf over fluid cells of rho, u and delta-rho (the stricter measure:
    normalised by max |rho - 1|), and the relative FP64 mass difference."""
    from oracle import oracle as O
    from paper_1112_0850_amd.lbm import LBM
    F = (1e-6, 0.0, 0.0)
    rho_r, u_r = O.macroscopics(f_ref, F, crop)
    fl = (crop & 1) == 0
    m_ref = O.reduce(f_ref, F, crop)[0]
    out = {"workload": f"128^3 crop of the porous geometry as a periodic box, tau 0.55, g_x 1e-6, "
                       f"from rest, {nsteps} steps (the oracle's CPU sample)"}
    for st, s in (("f32", 0), ("f16", 12), ("bf16", 0), ("f64", 0), ("f32x", 0)):
        sim = LBM(crop.shape, 0.55, F, st, flags=torch.from_numpy(crop).cuda(), f16_scale_log2=s)
        sim.step(nsteps)
        rho, u = sim.macroscopics(f64=True)
        m = float(sim.reduce()[0].item())
        rho, u = rho.cpu().numpy(), u.cpu().numpy()
        out[st] = {"rho_rel_linf": float(abs(rho - rho_r)[fl].max() / abs(rho_r)[fl].max()),
                   "u_rel_linf": float(abs(u - u_r)[:, fl].max() / abs(u_r)[:, fl].max()),
                   "drho_rel_linf": float(abs(rho - rho_r)[fl].max() / abs(rho_r - 1)[fl].max()),
                   "mass_rel_diff": abs(m - m_ref) / m_ref}
        if st == "f16":
            out[st]["f16_scale_log2"] = s
        del sim
    torch.cuda.empty_cache()
    return out


def gpu_clocks():
    """Current shader and memory clocks from the driver's DPM tables in sysfs
    (the level marked '*' of pp_dpm_sclk / pp_dpm_mclk of the first card that
    has them); a plain file read, no child process.  None where unavailable."""
    for dev in sorted(glob.glob("/sys/class/drm/card[0-9]*/device")):
        out = {}
        for name in ("pp_dpm_sclk", "pp_dpm_mclk", "pp_dpm_fclk"):
            try:
                with open(os.path.join(dev, name)) as fh:
                    cur = [ln.split(":", 1)[1].strip(" *\n") for ln in fh if ln.rstrip().endswith("*")]
            except (OSError, IndexError):
                continue
            if cur:
                out[name[7:]] = cur[0]
        if out:
            return out
    return None


def code_hash():
    """SHA-256 of the library's device and ABI code with comments and
    whitespace removed: the measured traffic stays attached to the code it
    was taken on, and a comment edit does not detach it."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        text = open(path).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def traffic_entry(key):
    """HBM bytes (FETCH_SIZE + WRITE_SIZE, calibrated) per launch of the
    kernel recorded under `key` in the committed rocprofv3 counter summary,
    or None when the kernel source changed since the counters were taken."""
    rec = traffic_record(key)
    return rec["fetch_bytes"] + rec["write_bytes"] if rec else None


def traffic_record(key):
    """The committed counter record of one kernel (see KERNELS), or None when
    the code changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = json.load(open(TRAFFIC_FILE))
    if t.get("code_sha256") != code_hash():
        return None
    return t.get("kernels", {}).get(key)


KERNELS = {  # record key -> (kernel name, box edge, bytes per fluid update, porous 512 geometry,
             #                steps per launch)
    "f32": ("void lbm::k_step<0, 1, true, false, 1>", 512, 152, True, 1),
    "f16": ("void lbm::k_step<1, 1, true, false, 4>", 512, 76, True, 1),
    "bf16": ("void lbm::k_step<2, 1, true, false, 4>", 512, 76, True, 1),
    "f64": ("void lbm::k_step<3, 1, true, false, 1>", 512, 304, True, 1),
    "f32x": ("void lbm::k_step<4, 1, true, false, 1>", 512, 152, True, 1),
    "f32x2": ("void lbm::k_step2<0, 4, true, false, false>", 512, 152, True, 2),
    "f16x2": ("void lbm::k_step2<1, 4, true, false, false>", 512, 76, True, 2),
    "f64x2": ("void lbm::k_step2<3, 4, true, false, false>", 512, 304, True, 2),
    "adjoint": ("void lbm::k_adj<false, false, false>", 256, 228, False, 1),  # periodic, no flags
}


def launch_threads(name, n):
    """Threads a launch of the named kernel has on an n^3 box (64 * M-cell
    segments per row, four per block, M = 4 for the 16-bit step kernels; the
    two-step kernel: 64 x TY tiles (TY = 13; 5 for FP64, 8 for F32X), z
    chunks of 128 planes halved down to 16 until there are 1280 blocks,
    64 (TY + 3) threads per block)."""
    if name.startswith("void lbm::k_step2<"):
        k = int(name.split("<")[1].split(",")[0])
        ty = {3: 5, 4: 8}.get(k, 13)
        tiles = -(-n // 64) * -(-n // ty)
        zc = min(n, 128)
        while zc > 16 and tiles * -(-n // zc) < 1280:
            zc = max(zc // 2, 16)
        return tiles * -(-n // zc) * 64 * (ty + 3)
    m = 4 if name.startswith("void lbm::k_step<1,") or name.startswith("void lbm::k_step<2,") else 1
    nseg = -(-n // (64 * m))
    return -(-nseg * n * n // 4) * 256


def box_of(name, grid):
    """The box edge of a launch from its grid size, trying the bench's own
    sizes first: the two-step kernel's launches at 256^3 and 512^3 have the
    same size (1280 blocks), and the bench runs it at 512^3 (and 768^3) on
    the porous box and at 256^3 (and 128^3) on the adjoint's periodic box,
    without solids (walls = 0)."""
    periodic2 = name.startswith("void lbm::k_step2<") and name.split("<")[1].split(",")[1].strip() == "0"
    order = (256, 128, 512, 768, 640) if periodic2 else (512, 768, 640, 256, 128)
    return next((n for n in order if launch_threads(name, n) == grid), None)


def profile_summary(trace_dir, fetch_dir, write_dir, n=512):
    """Summarise the rocprofv3 runs of this script per kernel and box size:
    average duration from the per-dispatch kernel trace, and HBM traffic per
    dispatch from FETCH_SIZE / WRITE_SIZE (KiB), each calibrated by the same
    counter on the copy kernel of known size."""
    import csv
    import glob
    import numpy as np
    from paper_1112_0850_amd import inputs as I

    def one(pattern):
        hits = glob.glob(os.path.join(pattern))
        if not hits:
            raise FileNotFoundError(pattern)
        return hits[0]

    times = {}
    for r in csv.DictReader(open(one(os.path.join(trace_dir, "*kernel_trace.csv")))):
        key = (r["Kernel_Name"].split("(")[0], int(r["Grid_Size_X"]))
        times.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    counters = {}
    for d, cname in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        for r in csv.DictReader(open(one(os.path.join(d, "*counter_collection.csv")))):
            if r["Counter_Name"] == cname:
                key = (r["Kernel_Name"].split("(")[0], int(r["Grid_Size"]), cname)
                counters.setdefault(key, []).append(float(r["Counter_Value"]))
    copy_keys = [k for k in counters if k[0].startswith("lbm::k_copy")]
    copy_bytes = 4 << 30  # the copy leg moves 4 GiB in, 4 GiB out
    scale = {c: copy_bytes / (1024 * np.mean([v for k in copy_keys if k[2] == c for v in counters[k]]))
             for c in ("FETCH_SIZE", "WRITE_SIZE")}
    flags = I.sphere_pack((n, n, n), 0.10, seed=12345)
    n_fluid = int((flags & 1 == 0).sum())
    total = sum(sum(v) for v in times.values())
    lines = ["| kernel | box | calls | avg us | fetch GB | write GB | alg GB | traffic/alg | actual TB/s |",
             "|---|---|---|---|---|---|---|---|---|"]
    record = {}
    for (name, grid), v in sorted(times.items(), key=lambda kv: -sum(kv[1])):
        if name.startswith("void lbm::k_copy_v"):
            continue  # the copy sweep's variants: reported on the bench line
        avg_us = float(np.mean(v))
        box = box_of(name, grid) if name.startswith("void lbm::k_") else None
        row = [name.replace("void ", "")[:44], f"{box}^3" if box else "", str(len(v)), f"{avg_us:.1f}"]
        rec_key = next((k for k, (kn, kb, _, _, _) in KERNELS.items() if kn == name and kb == box), None)
        fk, wk = (name, grid, "FETCH_SIZE"), (name, grid, "WRITE_SIZE")
        if fk in counters and wk in counters:
            fb = float(np.mean(counters[fk])) * 1024 * scale["FETCH_SIZE"]
            wb = float(np.mean(counters[wk])) * 1024 * scale["WRITE_SIZE"]
            row += [f"{fb / 1e9:.2f}", f"{wb / 1e9:.2f}"]
            if rec_key:
                _, kb, bpu, porous, nst = KERNELS[rec_key]
                alg = nst * (bpu * n_fluid + n ** 3 if porous else bpu * kb ** 3)
                row += [f"{alg / 1e9:.2f}", f"{(fb + wb) / alg:.3f}", f"{(fb + wb) / avg_us / 1e6:.2f}"]
                record[rec_key] = {"kernel": name, "box": box, "avg_us": avg_us, "fetch_bytes": fb,
                                   "write_bytes": wb, "alg_bytes": alg}
            else:
                row += ["", "", f"{(fb + wb) / avg_us / 1e6:.2f}"]
        else:
            row += ["", "", "", "", ""]
        if sum(v) / total > 0.002 or rec_key:
            lines.append("| " + " | ".join(row) + " |")
    out = {"code_sha256": code_hash(), "fetch_scale": scale["FETCH_SIZE"],
           "write_scale": scale["WRITE_SIZE"], "kernels": record}
    if "f32" in record:
        out["traffic_bytes_per_launch"] = record["f32"]["fetch_bytes"] + record["f32"]["write_bytes"]
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    json.dump(out, open(TRAFFIC_FILE, "w"), indent=1)
    text = "\n".join(lines)
    print(text)
    print(f"\ncounter calibration (copy kernel, 4 GiB): FETCH_SIZE x{scale['FETCH_SIZE']:.4f}, "
          f"WRITE_SIZE x{scale['WRITE_SIZE']:.4f}")
    return 0


def valu_summary(trace_dir, counter_dir, n=512, simds=1024, xcds=8):
    """Vector-instruction issue of the step kernels at the n^3 box from a
    VALU counter pass: wave-instructions per launch and per 64 cell updates,
    and VALU busy = SQ_ACTIVE_INST_VALU (quad-cycles) x 4 / simds against the
    kernel's own duration in cycles (GRBM_GUI_ACTIVE is summed over the
    xcds); the launch time is the kernel trace's average for the same kernel
    and box."""
    import csv
    import glob
    import statistics
    cnt = {}
    for r in csv.DictReader(open(glob.glob(os.path.join(counter_dir, "*counter_collection.csv"))[0])):
        name = r["Kernel_Name"].split("(")[0]
        if not name.startswith("void lbm::k_step"):
            continue
        key = (name, int(r["Grid_Size"]))
        cnt.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    times = {}
    for r in csv.DictReader(open(glob.glob(os.path.join(trace_dir, "*kernel_trace.csv"))[0])):
        key = (r["Kernel_Name"].split("(")[0], int(r["Grid_Size_X"]))
        times.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = ["| kernel | steps per launch | VALU wave-instr. per launch | per 64 cell updates | "
             "VALU busy | VALU issue per launch (ms) | launch (ms) |", "|---|---|---|---|---|---|---|"]
    for (name, grid), c in sorted(cnt.items()):
        if box_of(name, grid) != n or not all(k in c for k in ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU",
                                                                "GRBM_GUI_ACTIVE")):
            continue
        spl = 2 if name.startswith("void lbm::k_step2<") else 1
        insts = statistics.mean(c["SQ_INSTS_VALU"])
        quad = statistics.mean(c["SQ_ACTIVE_INST_VALU"])
        cycles = statistics.mean(c["GRBM_GUI_ACTIVE"]) / xcds
        busy = quad * 4 / simds / cycles
        launch = statistics.mean(times[(name, grid)]) / 1e3 if (name, grid) in times else None
        issue = busy * launch if launch else None
        lines.append(f"| {name.replace('void lbm::', '')} | {spl} | {insts:.4g} | "
                     f"{insts / (n ** 3 / 64 * spl):.0f} | {100 * busy:.0f}% | "
                     f"{issue:.2f} | {launch:.2f} |" if launch else
                     f"| {name.replace('void lbm::', '')} | {spl} | {insts:.4g} | "
                     f"{insts / (n ** 3 / 64 * spl):.0f} | {100 * busy:.0f}% | | |")
    print("\n".join(lines))
    return 0


def stall_summary(counter_dir, n=512):
    """Where the step kernels' waves spend their time at the n^3 box: the
    shares of SQ_WAVE_CYCLES (wave-cycles resident) spent waiting on a
    dependency (SQ_WAIT_ANY: loads, LDS, barriers), ready but not issued
    (SQ_WAIT_INST_ANY) and issuing (SQ_ACTIVE_INST_ANY), averaged over the
    dispatches of each kernel."""
    import csv
    import glob
    import statistics
    cnt = {}
    for r in csv.DictReader(open(glob.glob(os.path.join(counter_dir, "*counter_collection.csv"))[0])):
        name = r["Kernel_Name"].split("(")[0]
        if not name.startswith("void lbm::k_step"):
            continue
        cnt.setdefault((name, int(r["Grid_Size"])), {}).setdefault(
            r["Counter_Name"], []).append(float(r["Counter_Value"]))
    lines = ["| kernel | waiting on a dependency | ready, not issued | issuing | LDS bank conflicts "
             "per LDS instruction-cycle |", "|---|---|---|---|---|"]
    for (name, grid), c in sorted(cnt.items()):
        need = ("SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_ANY")
        if box_of(name, grid) != n or not all(k in c for k in need):
            continue
        m = {k: statistics.mean(v) for k, v in c.items()}
        w = m["SQ_WAVE_CYCLES"]
        lds = (f"{m['SQ_LDS_BANK_CONFLICT'] / m['SQ_ACTIVE_INST_LDS']:.3f}"
               if m.get("SQ_ACTIVE_INST_LDS") else "")
        lines.append(f"| {name.replace('void lbm::', '')} | {100 * m['SQ_WAIT_ANY'] / w:.0f}% | "
                     f"{100 * m['SQ_WAIT_INST_ANY'] / w:.0f}% | "
                     f"{100 * m['SQ_ACTIVE_INST_ANY'] / w:.0f}% | {lds} |")
    print("\n".join(lines))
    return 0


def trace_summary(trace_dir, bench_json):
    """Markdown table of a kernel trace of `python bench.py`, per kernel and
    box size, with the headline kernels' timed launches set against the
    bench line of the same run."""
    import csv
    import glob
    import statistics
    path = glob.glob(os.path.join(trace_dir, "*kernel_trace.csv"))[0]
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    d = json.loads(open(bench_json).read().strip().splitlines()[-1])
    groups, total = {}, 0
    for r in rows:
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        total += dur
        groups.setdefault((r["Kernel_Name"].split("(")[0], int(r["Grid_Size_X"])), []).append(dur)
    out = ["| kernel | box | calls | avg us | min us | max us | share of GPU time |",
           "|---|---|---|---|---|---|---|"]
    for (name, grid), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        if sum(v) / total < 0.002 or name.startswith("void lbm::k_copy_v"):
            continue
        box = box_of(name, grid) if name.startswith("void lbm::k_") else None
        out.append(f"| {name.replace('void ', '')} | {f'{box}^3' if box else ''} | {len(v)} | "
                   f"{statistics.mean(v):.1f} | {min(v):.1f} | {max(v):.1f} | {100 * sum(v) / total:.1f}% |")
    steps, warm = d["steps"], d["warmup"]
    out.append("")
    two = d.get("roofline", {}).get("steps_per_launch") == 2
    checks = [("f32x2" if two else "f32", "FP32 (headline)", d["ms_per_step"])]
    if two:
        checks.append(("f32", "FP32 single step", d.get("f32_single_step", {}).get("ms_per_step")))
    checks.append(("f16", "FP16 single step", d.get("f16_storage", {}).get("ms_per_step")))
    for key, label, ms in checks:
        name, spl = KERNELS[key][0], KERNELS[key][4]
        n = round(d["config"]["cells"] ** (1 / 3))
        v = groups.get((name, launch_threads(name, n)), [])
        wl, sl = warm // spl, steps // spl
        if ms and len(v) >= wl + sl:
            timed = v[wl:wl + sl]
            per = f"{spl} steps per launch, " if spl > 1 else ""
            out.append(f"{label}: the bench line reports {ms * spl * 1e3:.1f} us per launch "
                       f"({per}HIP events around {steps} timed steps); the trace's {sl} launches "
                       f"after the {wl} warm-up launches of {name.replace('void ', '')} at {n}^3 "
                       f"average {statistics.mean(timed):.1f} us.")
    print("\n".join(out))
    return 0


ROOFLINE_KERNELS = {  # leg -> kernel named in the roofline object
    "f32": "k_step<F32, static walls, force, Qian>",
    "f32x2": "k_step2<F32, static walls (link mask), force, Qian> (two steps per launch)",
    "f16": "k_step<F16, static walls, force, Qian>",
    "bf16": "k_step<BF16, static walls, force, Qian>",
    "f64": "k_step<F64, static walls, force, Qian>",
    "f32x": "k_step<F32X, static walls, force, Qian>",
    "f16x2": "k_step2<F16, static walls (link mask), force, Qian> (two steps per launch)",
    "bf16x2": "k_step2<BF16, static walls (link mask), force, Qian> (two steps per launch)",
    "f64x2": "k_step2<F64, static walls (link mask), force, Qian> (two steps per launch)",
}


def roofline_of(key, leg):
    """The roofline object of one forward leg: algorithmic bytes per launch
    (bytes per fluid-cell update x the updates one launch performs, plus the
    flag bytes it reads) over the launch time measured with HIP events, and
    the HBM bytes per launch from the committed counter summary."""
    spl = leg["steps_per_launch"]
    out = {"bound": "hbm", "achieved": leg["alg_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": leg["hbm_frac"], "traffic": traffic_entry(key),
           "kernel": ROOFLINE_KERNELS.get(key, key), "steps_per_launch": spl,
           "alg_bytes_per_launch": spl * leg["alg_bytes_per_step"],
           "launch_ms": spl * leg["ms_per_step"]}
    if out["traffic"]:
        out["traffic_over_alg"] = out["traffic"] / out["alg_bytes_per_launch"]
    if spl == 2:
        out["note"] = ("algorithmic bytes of two single-step updates (the intermediate level stays "
                       "in LDS, so the kernel's HBM traffic is below them); the pass is bound by "
                       "latency and instruction issue, not by HBM")
    return out


def main():
    args = parse()
    if args.sweep_summary:
        return sweep_summary(args.sweep_summary)
    if args.trace_summary:
        return trace_summary(*args.trace_summary)
    if args.valu_summary:
        return valu_summary(*args.valu_summary)
    if args.stall_summary:
        return stall_summary(*args.stall_summary)
    if args.profile_summary:
        return profile_summary(*args.profile_summary)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "domain decomposition is a design note, not part of this build", file=sys.stderr)
        return 2
    import numpy as np
    import torch
    from paper_1112_0850_amd import inputs as I
    from paper_1112_0850_amd.lbm import LBM
    if args.sweep:
        return sweep(torch)

    legs = set(args.only.split(",")) if args.only else {"f32", "f16", "bf16", "f64", "f32x",
                                                        "f32x2", "f16x2", "bf16x2", "f64x2",
                                                        "adjoint", "copy", "cpu", "large", "cavity",
                                                        "split", "incomp"}
    n = args.n
    log(f"geometry: {n}^3 sphere pack, 10% solid, seed 12345")
    flags = I.sphere_pack((n, n, n), 0.10, seed=12345)
    n_cells = n ** 3
    n_fluid = int((flags & 1 == 0).sum())
    flags_t = torch.from_numpy(flags).cuda()
    res = {}
    if "copy" in legs:
        log("copy probe")
        res["copy"] = copy_leg(torch)
    aux = min(args.aux_steps, args.steps)
    fields, clocks = {}, {}
    for st, s in (("f32", 0), ("f16", 12), ("bf16", 0), ("f64", 0), ("f32x", 0)):
        if st in legs:
            log(f"forward {st}")
            head = st in ("f32", "f16", "bf16")
            res[st] = forward_leg(torch, LBM, flags_t, n_cells, n_fluid, st,
                                  args.steps if head else aux, args.warmup, s,
                                  fields=fields if head else None,
                                  clocks=clocks if st == "f32" and "f32x2" not in legs else None,
                                  pull=st in ("f32", "f16", "f64"))
            log(f"  {res[st]['mlups']:.0f} MLUPS, {res[st]['alg_gbs']:.0f} GB/s algorithmic")
    if "f32" in fields:
        # 16-bit storage against FP32 storage on the full box at the same step
        fluid = (flags_t & 1) == 0
        rho32, u32 = fields["f32"]
        for st in ("f16", "bf16"):
            if st in fields:
                rho, u = fields[st]
                res[f"{st}_vs_f32"] = {
                    "steps": args.steps + args.warmup,
                    "u_rel_linf": float((u - u32)[:, fluid].abs().max() / u32[:, fluid].abs().max()),
                    "rho_rel_linf": float((rho - rho32)[fluid].abs().max() / rho32[fluid].abs().max()),
                    "drho_rel_linf": float((rho - rho32)[fluid].abs().max()
                                           / (rho32 - 1)[fluid].abs().max())}
        del fluid, rho32, u32
    fields.clear()
    torch.cuda.empty_cache()
    if legs & {"f32x2", "f16x2", "bf16x2", "f64x2"}:
        # the same workload with pairs of steps fused into one temporally blocked pass
        for st, s in (("f32", 0), ("f16", 12), ("bf16", 0), ("f64", 0)):
            if f"{st}x2" in legs:
                log(f"forward {st}, two steps per pass")
                res[f"{st}x2"] = forward_leg(torch, LBM, flags_t, n_cells, n_fluid, st,
                                             aux if st == "f64" else args.steps,
                                             args.warmup, s, steps_per_pass=2,
                                             clocks=clocks if st == "f32" else None)
                log(f"  {res[f'{st}x2']['mlups']:.0f} MLUPS, {res[f'{st}x2']['alg_gbs']:.0f} GB/s "
                    "algorithmic")
    if "split" in legs:
        # the paper's split design: a separate obstacle kernel before each step
        log("split design (separate obstacle kernel), f32 and f16")
        res["split"] = [forward_leg(torch, LBM, flags_t, n_cells, n_fluid, st, aux,
                                    args.warmup, s, obstacle_kernel=1)
                        for st, s in (("f32", 0), ("f16", 12))]
        log("  " + ", ".join(f"{c['mlups']:.0f}" for c in res["split"]) + " MLUPS")
    if "incomp" in legs:
        # the He-Luo incompressible equilibrium on the same porous workload
        log("incompressible equilibrium, f32 and f16")
        res["incomp"] = [forward_leg(torch, LBM, flags_t, n_cells, n_fluid, st, aux,
                                     args.warmup, s, equilibrium="incompressible")
                         for st, s in (("f32", 0), ("f16", 12))]
        log("  " + ", ".join(f"{c['mlups']:.0f}" for c in res["incomp"]) + " MLUPS")
    if "cavity" in legs:
        log(f"lid-driven cavity {n}^3, f32 and f16")
        res["cavity"] = [cavity_leg(torch, "f32", n, aux, args.warmup),
                         cavity_leg(torch, "f16", n, aux, args.warmup, 10)]
        log("  " + ", ".join(f"{c['mlups']:.0f}" for c in res["cavity"]) + " MLUPS")
    if "adjoint" in legs:
        log("adjoint 128^3 and 256^3")
        res["adjoint"] = adjoint_leg(torch)
        res["adjoint_256"] = adjoint_leg(torch, 256)
    if "large" in legs:
        del flags_t
        torch.cuda.empty_cache()
        log("large 768^3 f32 and 640^3 f64 (single steps, fused pairs)")
        res["large"] = [large_leg(torch, "f32", 768), large_leg(torch, "f32", 768, steps_per_pass=2),
                        large_leg(torch, "f64", 640), large_leg(torch, "f64", 640, steps_per_pass=2)]
    if "cpu" in legs:
        log("cpu oracle sample")
        res["cpu"] = cpu_leg(flags, args.cpu_seconds)
        log("error against the oracle on its sample, every storage")
        res["error_vs_oracle"] = crop_error_leg(torch, *res["cpu"].pop("_state"))

    # The headline is the fastest FP32 schedule: pairs of steps fused into one
    # temporally blocked pass (bit-identical to single steps), else the
    # single step, else the first other storage run.
    main_key = next((k for k in ("f32x2", "f32", "f16", "bf16", "f64", "f32x") if k in res), None)
    main_leg = res.get(main_key) if main_key else None
    two = bool(main_leg) and main_leg["steps_per_launch"] == 2
    line = {
        "metric": "MLUPS & %HBM roofline, D3Q19 512^3 FP32 vs FP16-offset; adjoint/fwd time",
        "value": main_leg["mlups"] if main_leg else None,
        "unit": "MLUPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"] if main_leg else None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32", "f16": "f32", "bf16": "f32", "f64": "f64",
                  "f32x": "f64"}[main_leg["storage"]]
        if main_leg else None,
        "data": "synthetic",
        "config": {"workload": f"D3Q19 BGK porous periodic box {n}^3, 10% solid random spheres "
                               f"r 4-12 (seed 12345), tau 0.55, g_x 1e-6, from rest, "
                               f"{args.warmup + args.steps} steps ({args.steps} timed), "
                               f"{main_leg['storage'] if main_leg else ''} offset storage"
                               + (", two steps per pass (temporal blocking)" if two else ""),
                   "cells": n_cells, "fluid_cells": n_fluid},
    }
    if main_leg:
        line["roofline"] = roofline_of(main_key, main_leg)
    if two and "f32" in res:
        # the single-step kernel on the same workload, with its own roofline
        line["f32_single_step"] = dict(res["f32"], roofline=roofline_of("f32", res["f32"]))
    if "cpu" in res:
        line["cpu_baseline"] = res["cpu"]
    line["mflups"] = main_leg["mflups"] if main_leg else None
    line["timing"] = main_leg["timing"] if main_leg else None
    for st in ("f16", "bf16", "f64", "f32x"):
        if st in res:
            line[f"{st}_storage"] = dict(res[st], roofline=roofline_of(st, res[st]))
            if f"{st}_vs_f32" in res:
                line[f"{st}_storage"]["vs_f32_same_step"] = res[f"{st}_vs_f32"]
    if "f16" in res and "f32" in res:
        # same schedule (single steps), the fused pairs, and best against best
        line["f16_over_f32"] = res["f16"]["mlups"] / res["f32"]["mlups"]
        if "f16x2" in res and "f32x2" in res:
            line["f16_over_f32_two_steps_per_pass"] = res["f16x2"]["mlups"] / res["f32x2"]["mlups"]
            line["f16_over_f32_best"] = (max(res["f16"]["mlups"], res["f16x2"]["mlups"])
                                         / max(res["f32"]["mlups"], res["f32x2"]["mlups"]))
    if "adjoint" in res:
        line["adjoint"] = res["adjoint"]
        line["adjoint_256"] = res["adjoint_256"]
        rec = traffic_record("adjoint")
        if rec:  # measured HBM traffic of the adjoint kernel at 256^3 (rocprofv3 counters)
            tb = rec["fetch_bytes"] + rec["write_bytes"]
            line["adjoint_256"]["kernel_traffic"] = {
                "bytes_per_launch": tb, "over_algorithmic": tb / rec["alg_bytes"],
                "actual_gbs": tb / res["adjoint_256"]["adj_step_ms"] / 1e6}
    if "large" in res:
        line["large"] = res["large"]
    if "cavity" in res:
        line["cavity"] = res["cavity"]
    if "split" in res:
        line["split_obstacle_kernel"] = res["split"]
    for st in ("f16", "bf16", "f64"):
        if f"{st}x2" in res:
            line[f"{st}_two_steps_per_pass"] = dict(res[f"{st}x2"],
                                                    roofline=roofline_of(f"{st}x2", res[f"{st}x2"]))
    if "incomp" in res:
        line["incompressible_equilibrium"] = res["incomp"]
    if "error_vs_oracle" in res:
        line["error_vs_oracle"] = res["error_vs_oracle"]
    if "copy" in res:
        line["copy_gbs"] = res["copy"]["gbs"]
        line["copy_best"] = res["copy"]["best"]
        line["copy_sweep"] = res["copy"]["sweep"]
        if main_leg:
            line["frac_of_copy_bw"] = main_leg["alg_gbs"] / res["copy"]["best"]["gbs"]
        if "f32_single_step" in line:
            line["f32_single_step"]["frac_of_copy_bw"] = (res["f32"]["alg_gbs"]
                                                          / res["copy"]["best"]["gbs"])
    single = res.get("f32")
    if single and "pull_copy" in single:
        # the single step's own access pattern without geometry or collision (lbm_pull_copy)
        line["pull_copy_probe"] = dict(single["pull_copy"])
    props = torch.cuda.get_device_properties(0)
    line["device"] = f"{props.name} ({getattr(props, 'gcnArchName', '?')}, "\
                     f"{props.multi_processor_count} CUs, {props.total_memory / 2**30:.0f} GiB)"
    line["hip_version"] = torch.version.hip
    line["clocks_during_headline_leg"] = clocks or None
    line["context"] = "paper: 650 MLUPS SP / 290 MLUPS DP on an NVIDIA Tesla C2070 (other hardware)"
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
