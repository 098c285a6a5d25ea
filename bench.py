"""Benchmark of the batched fast spectral collision operator on one MI355X.

Workload: 4096 independent space-homogeneous cells, hard spheres (gamma = 1),
velocity grid 32^3 on [-8, 8)^3, M = 32 directions (8 Gauss polar x 4
azimuthal), seeded two-Maxwellian cells.  One step = one call of
fks_collide_batch over the whole batch: forward FFT, 32 gain terms and the
loss term, FP64 conservation projection and the update f <- f + dt/tau Q_c
(FP32 transforms and products, FP64 fix), inputs resident in HBM.

Prints one JSON line: the throughput of the batch, the roofline of the dominant
kernel, the CPU oracle on a bounded sample of the same cells (which doubles as a
parity check of the timed configuration), the plain FP64 path, and the extra
workloads (BGK, two velocity dimensions, de-aliased variant).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cells·N³/s of Q(f,f) at N=32³, M=32 (FP32+fix vs FP64, rel err ≤1e-5)"
UNIT = "cells·N³/s"
PEAK_FP32_VECTOR_TFLOPS = 157.3     # MI355X dense FP32 vector (packed) peak
PEAK_FP64_VECTOR_TFLOPS = 78.6      # MI355X dense FP64 vector peak
N_V, T_BOX, NCELL = 32, 8.0, 4096
N_POLAR, N_AZIM = 8, 4
DT_OVER_TAU = 1e-3
EXTRAS = ("bgk", "moments", "halo", "collide2d", "dealias", "uneven")


def _oracle_worker(args):
    cells, = args
    import numpy as np
    import oracle as O
    import synth
    op = O.make_plan(N_V, T_BOX, n_polar=N_POLAR, n_azim=N_AZIM)
    out = []
    t0 = time.perf_counter()
    for c in cells:
        f = synth.two_maxwellian_cells(N_V, T_BOX, NCELL, first=c, count=1)[0]
        Q, _, loss = O.collide_fast64(f, op, parts=True)
        qc = O.conserve_Q(Q, N_V, T_BOX)
        out.append((c, qc, float(np.linalg.norm(loss) / np.linalg.norm(qc))))
    return out, time.perf_counter() - t0


def _oracle_extra_worker(args):
    """Times the oracle (as it stands) on a bounded sample of one extra workload, one core:
    cells in order until about 2.5 s of oracle time (inputs generated beforehand)."""
    kind, = args
    import oracle as O
    import synth
    budget = 2.5
    if kind == "collide2d":
        n, T, A = 32, 9.0, 8
        f = synth.two_maxwellian_cells_2d(n, T, 8192, seed_offset=123)
        p2 = O.fks_oracle2d.make_plan2(n, T, A)
        step = lambda g: g + 0.02 * O.fks_oracle2d.conserve2_Q(O.fks_oracle2d.collide2_fast64(g, p2), n, T)  # noqa: E731
        pts = n * n
    elif kind == "bgk":
        f = synth.two_maxwellian_cells(N_V, T_BOX, NCELL, first=0, count=512)
        nu = 2.0 * (2.0 * T_BOX / (3.0 + math.sqrt(2.0)))   # mu = 4 pi C (2R)^gamma, C = 1/(4 pi), gamma = 1
        step = lambda g: O.fks_oracle_bgk.bgk_step(g, N_V, T_BOX, 3, nu, DT_OVER_TAU)  # noqa: E731
        pts = N_V ** 3
    elif kind == "dealias":
        f = synth.two_maxwellian_cells(N_V, T_BOX, NCELL, first=0, count=8)
        op = O.make_plan(N_V, T_BOX, n_polar=N_POLAR, n_azim=N_AZIM)
        step = lambda g: g + DT_OVER_TAU * O.conserve_Q(O.fks_oracle_dealias.collide_dealias_fast64(g, op),  # noqa: E731
                                                        N_V, T_BOX)
        pts = N_V ** 3
    elif kind == "moments":
        # U = C f, then the projection of f onto U, per cell of the batch
        f = synth.two_maxwellian_cells(N_V, T_BOX, NCELL, first=0, count=1024)
        step = lambda g: O.project(g, O.moments(g, N_V, T_BOX), N_V, T_BOX)  # noqa: E731
        pts = N_V ** 3
    elif kind == "halo":
        # the whole-grid transport of the oracle (what the slabs reproduce) on a 2 x 2 x 4 grid of
        # 24^3 velocities, periodic, the bench's CFL; one step is one sample
        import numpy as np
        hn, hT = 24, 8.0
        dx = 0.5
        g0 = synth.rng(96).uniform(size=(4, 2, 2, hn, hn, hn))
        _, sh = O.transport_offsets_step(np.zeros((3, hn)), hn, hT, dx, 0.95 * dx / hT)
        f = [g0] * 64
        step = lambda g: O.transport_shift(g, sh, hn)  # noqa: E731
        pts = g0.size
    else:
        raise ValueError(kind)
    count, t0 = 0, time.perf_counter()
    while count < len(f) and (count == 0 or time.perf_counter() - t0 < budget):
        step(f[count])
        count += 1
    return kind, count, pts, time.perf_counter() - t0


def cpu_extras(kinds):
    """Oracle timings beside the extra GPU lines: {kind: cpu_baseline dict}, one process per kind."""
    ctx = mp.get_context("spawn")
    with ctx.Pool(len(kinds)) as pool:
        res = pool.map(_oracle_extra_worker, [(k,) for k in kinds])
    out = {}
    for kind, count, pts, t in res:
        unit = "cells·N²/s" if kind == "collide2d" else UNIT
        what = (f"{count} whole-grid transport steps of a 2x2x4 grid of 24^3 velocities (the oracle's "
                "element loop)" if kind == "halo" else
                f"{count} cells of the same workload (moments, then projection)" if kind == "moments" else
                f"{count} cells of the same workload")
        out[kind] = {"value": count * pts / t, "unit": unit, "cores": 1, "kind": "oracle",
                     "sample": f"{what}, numpy FP64, one single-threaded process ({t:.1f} s)"}
    return out


def cpu_baseline(sample_cells, workers):
    """Times the oracle (as it stands) on the sample; returns (result dict, {cell: (Q_c, ratio)})."""
    chunks = [sample_cells[i::workers] for i in range(workers)]
    chunks = [c for c in chunks if c]
    t0 = time.perf_counter()
    ctx = mp.get_context("spawn")
    with ctx.Pool(len(chunks)) as pool:
        res = pool.map(_oracle_worker, [(c,) for c in chunks])
    wall = time.perf_counter() - t0
    ref = {}
    busy = 0.0
    for out, t in res:
        busy = max(busy, t)
        for c, qc, r in out:
            ref[c] = (qc, r)
    n = len(sample_cells)
    return {
        "value": n * N_V ** 3 / busy,
        "unit": UNIT,
        "cores": len(chunks),
        "kind": "oracle",
        "sample": f"{n} of the {NCELL} cells (every {NCELL // n}th), numpy FP64 fast form + projection, "
                  f"one single-threaded process per core; timed inside the workers ({busy:.1f} s), "
                  f"pool start-up excluded (wall {wall:.1f} s)",
    }, ref


def _fused_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("fks_fused.hip", "fks_fft.hpp", "fks_common.hpp"):
        with open(os.path.join(ROOT, "paper_1608_08009_amd", "csrc", name), "rb") as fp:
            h.update(fp.read())
    return h.hexdigest()[:16]


def _traffic_per_launch():
    """HBM bytes per launch of the terms kernel from the committed counter summary,
    or None if the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_k_terms32_hs4096.json")
    try:
        with open(path) as fp:
            rec = json.load(fp)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != _fused_source_hash():
        return None
    return rec.get("bytes_per_launch")


def _valu_busy():
    """VALU-busy fraction of the terms kernel from the committed SQ counter summary, or None
    if the kernel sources changed since the counters were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", "sq_k_terms32_hs4096.json")) as fp:
            rec = json.load(fp)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != _fused_source_hash():
        return None
    return rec.get("valu_busy")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=512, help="cells timed on the CPU oracle (0 = skip)")
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--eager", dest="graph", action="store_false",
                    help="launch each step directly instead of replaying captured graphs")
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="skip the extra workloads (BGK, moments, halo, 2D, de-aliased, uneven batch)")
    ap.add_argument("--extras", dest="extra_set", default=",".join(EXTRAS),
                    help="comma-separated extra workloads to run (default: all of " + ",".join(EXTRAS) + ")")
    ap.add_argument("--uneven-quick", action="store_true",
                    help="uneven batch: time the FP32 + fix call only (no autotuning, no FP64 leg); for "
                         "profiler runs, where every dispatch is slow")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 512 MiB device copy (reference kernel for HBM counters)")
    args = ap.parse_args()
    extras = set(x for x in args.extra_set.split(",") if x) if args.extras else set()
    unknown = extras - set(EXTRAS)
    if unknown:
        ap.error(f"unknown extra workloads: {sorted(unknown)}")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(cells are independent: a batch shards across GPUs by contiguous cell ranges with no "
              "communication in the collision step). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1608_08009_amd as fks
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    print(f"[bench] device {torch.cuda.get_device_name(0)}; generating {NCELL} cells of {N_V}^3", file=sys.stderr,
          flush=True)
    f0 = synth.two_maxwellian_torch(N_V, T_BOX, NCELL, dev)
    fa = f0.clone()
    fb = torch.empty_like(f0)
    q = torch.empty_like(f0)

    desc = fks.Desc(n=N_V, T=T_BOX, gamma=1.0, n_polar=N_POLAR, n_azim=N_AZIM, precision=fks.PREC_F32_FIX64)
    plan = fks.Plan(desc)
    # a second plan of the same configuration, timed: the first one of the process also loads
    # the library's code objects
    torch.cuda.synchronize()
    t_plan = time.perf_counter()
    with fks.Plan(desc):
        torch.cuda.synchronize()
        plan_ms = (time.perf_counter() - t_plan) * 1e3   # directions, radial terms, device tables
    assert plan.info.fused == 1
    ws = fks.collide_batch([(plan, fa, q, None, NCELL, 0.0)])   # untimed parity run (Q_c)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]

    def step(src, dst):
        fks.collide_batch([(plan, src, None, dst, NCELL, DT_OVER_TAU)], workspace=ws)

    # one time step in each direction of the f ping-pong, captured as graphs and replayed
    graphs = []
    if args.graph:
        cap = torch.cuda.Stream()
        cap.wait_stream(stream)
        for src, dst in ((fa, fb), (fb, fa)):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=cap):
                step(src, dst)
            graphs.append(g)
        torch.cuda.synchronize()

    def run(i):
        if graphs:
            graphs[i % 2].replay()
        elif i % 2 == 0:
            step(fa, fb)
        else:
            step(fb, fa)

    for i in range(args.warmup):
        run(i)
    torch.cuda.synchronize()
    print(f"[bench] warmup done; timing {args.steps} steps ({'graph replay' if graphs else 'eager'})",
          file=sys.stderr, flush=True)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record(stream)
    for i in range(args.steps):
        ev[i][0].record(stream)
        run(args.warmup + i)
        ev[i][1].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    launch_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = total_ms / args.steps
    avg_call_ms = sum(launch_ms) / len(launch_ms)
    median_ms = sorted(launch_ms)[len(launch_ms) // 2]
    value = NCELL * N_V ** 3 / (ms_per_step * 1e-3)
    # per-kernel durations (HIP events recorded by the library on this stream)
    fks.profile_enable(True)
    kt = []
    for i in range(max(3, min(args.steps, 10))):
        step(fa, fb)
        fa, fb = fb, fa
        kt.append(fks.profile_last())
    fks.profile_enable(False)
    # one kernel when a workgroup takes whole cells (this batch), else terms + finish
    nk = len(kt[0])
    assert nk in (1, 2) and all(len(k) == nk for k in kt), kt
    terms_ms = sum(k[0] for k in kt) / len(kt)
    finish_ms = sum(k[1] for k in kt) / len(kt) if nk == 2 else 0.0
    kernel_name = "k_terms<32, one workgroup per cell>" if nk == 1 else "k_terms<32, pairs>"
    flops_launch = plan.info.flops_per_cell * NCELL
    achieved_tflops = flops_launch / (terms_ms * 1e-3) / 1e12
    print(f"[bench] fp32+fix: {ms_per_step:.3f} ms/step ({kernel_name} {terms_ms:.3f} ms, finish kernel "
          f"{finish_ms:.3f} ms), {achieved_tflops:.1f} TFLOP/s algorithmic in the terms kernel",
          file=sys.stderr, flush=True)

    if args.calibrate_copy:
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device=dev)    # 512 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # BGK relaxation (conservative discrete Maxwellian) on the same batch: HBM-bound
    bgk_line = None
    if "bgk" in extras:
        nu_mu = 4.0 * math.pi * plan.info.c_gamma * (2.0 * plan.info.R)   # mu for hard spheres
        fks.bgk(fa, N_V, T_BOX, nu_mu, dim=3, f_out=fb, dt_over_tau=DT_OVER_TAU)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fks.bgk(fa, N_V, T_BOX, nu_mu, dim=3, f_out=fb, dt_over_tau=DT_OVER_TAU)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_bgk = e0.elapsed_time(e1) / args.steps
        alg = NCELL * N_V ** 3 * 16.0            # read f, write f_out (FP64)
        bgk_line = {"workload": f"{NCELL} cells, 32^3, 3D, nu = mu, Euler step, f_out", "ms": round(ms_bgk, 4),
                    "value": NCELL * N_V ** 3 / (ms_bgk * 1e-3), "unit": UNIT,
                    "roofline": {"bound": "hbm", "achieved": round(alg / (ms_bgk * 1e-3) / 1e9, 1),
                                 "peak": 8000.0, "unit": "GB/s",
                                 "frac": round(alg / (ms_bgk * 1e-3) / 8e12, 4), "bytes_per_launch": alg}}
        print(f"[bench] bgk: {ms_bgk:.3f} ms per batch", file=sys.stderr, flush=True)

    # moments and the projection onto prescribed moments on the same batch (FP64, in place)
    moments_line = None
    if "moments" in extras:
        Um = torch.empty((NCELL, 5), dtype=torch.float64, device="cuda")
        fks.moments(fa, N_V, T_BOX, U=Um)
        fks.conserve(fa, Um, N_V, T_BOX)
        torch.cuda.synchronize()
        reps = 10
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        for _ in range(reps):                  # back to back: the launches stay ahead of the GPU
            fks.moments(fa, N_V, T_BOX, U=Um)
        ev[1].record(stream)
        for _ in range(reps):
            fks.conserve(fa, Um, N_V, T_BOX)
        ev[2].record(stream)
        torch.cuda.synchronize()
        ms_m = ev[0].elapsed_time(ev[1]) / reps
        ms_c = ev[1].elapsed_time(ev[2]) / reps
        pts = NCELL * N_V ** 3
        moments_line = {"workload": f"{NCELL} cells of 32^3, FP64: fks_moments, then fks_conserve onto those moments "
                                    "(in place)",
                        "ms_moments": round(ms_m, 4), "ms_conserve": round(ms_c, 4),
                        "value": pts / (ms_m * 1e-3), "unit": UNIT,
                        "roofline": {"bound": "hbm", "achieved": round(8.0 * pts / (ms_m * 1e-3) / 1e9, 1),
                                     "peak": 8000.0, "unit": "GB/s",
                                     "frac": round(8.0 * pts / (ms_m * 1e-3) / 8e12, 4),
                                     "bytes_per_launch": 8.0 * pts, "kernel": "k_moments (read f once)"},
                        "conserve_roofline": {"bound": "hbm",
                                              "achieved": round(24.0 * pts / (ms_c * 1e-3) / 1e9, 1),
                                              "peak": 8000.0, "unit": "GB/s",
                                              "frac": round(24.0 * pts / (ms_c * 1e-3) / 8e12, 4),
                                              "bytes_per_launch": 24.0 * pts,
                                              "bytes": "f read for the sums, read and written for the correction"}}
        del Um
        print(f"[bench] moments: {ms_m:.3f} ms, conserve {ms_c:.3f} ms", file=sys.stderr, flush=True)

    # z-slab transport with halo exchange: one GPU's share of the 32^3-cell, 24^3-velocity flow on
    # eight GPUs (4 planes of 32 x 32 cells).  Per step: pack the two outgoing messages, then the
    # slab transport, which reads what enters through the z faces from the incoming messages
    # (here the slab's own, a ring of one).  Moving the messages between GPUs is not part of this
    # one-GPU figure.
    halo_line = None
    if "halo" in extras:
        hn, hT, hx, hy, hz = 24, 8.0, 32, 32, 4
        hdx = 1.0 / hx
        hdt = 0.95 * hdx / hT
        g = torch.Generator(device="cuda").manual_seed(1608080096)
        sa = torch.rand((hz, hy, hx, hn ** 3), dtype=torch.float64, device="cuda", generator=g)
        sb = torch.empty_like(sa)
        msgs = {f: torch.empty(fks.halo_size(hx, hy, hz, hn, f) // 8, dtype=torch.float64, device="cuda")
                for f in (fks.FACE_ZLO, fks.FACE_ZHI)}
        off = np.zeros((3, hn))
        periodic = (fks.BC_PERIODIC, fks.BC_PERIODIC)

        def halo_exchange(ext):
            for f in (fks.FACE_ZLO, fks.FACE_ZHI):
                fks.halo_pack(ext, msgs[f], hx, hy, hz, hn, f)

        def slab_step(src, dst):
            fks.transport_shift_slab(src, dst, hx, hy, hz, hdx, periodic, hn, hT, hdt, off,
                                     msgs[fks.FACE_ZHI], msgs[fks.FACE_ZLO])

        for _ in range(2):
            halo_exchange(sa)
            slab_step(sa, sb)
            sa, sb = sb, sa
        torch.cuda.synchronize()
        reps = 10
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3 * reps)]
        for r in range(reps):
            ev[3 * r].record(stream)
            halo_exchange(sa)
            ev[3 * r + 1].record(stream)
            slab_step(sa, sb)
            ev[3 * r + 2].record(stream)
            sa, sb = sb, sa
        torch.cuda.synchronize()
        ms_x = sum(ev[3 * r].elapsed_time(ev[3 * r + 1]) for r in range(reps)) / reps
        ms_t = sum(ev[3 * r + 1].elapsed_time(ev[3 * r + 2]) for r in range(reps)) / reps
        msg_bytes = sum(m.numel() * 8 for m in msgs.values())
        x_bytes = 2.0 * msg_bytes                       # pack: read the face planes' velocities, write them
        t_bytes = hz * hy * hx * hn ** 3 * 16.0          # slab transport: read f (or a message), write f_out
        pts = hz * hy * hx * hn ** 3
        halo_line = {"workload": f"one GPU's share of a {hx}x{hy}x{8 * hz} grid on 8 GPUs: {hz} planes of "
                                 f"{hx}x{hy} cells, {hn}^3 velocities, periodic, CFL 0.95",
                     "ms": round(ms_x + ms_t, 4), "ms_halo_pack": round(ms_x, 4),
                     "ms_slab_transport": round(ms_t, 4), "message_bytes_per_face": msg_bytes // 2,
                     "value": pts / ((ms_x + ms_t) * 1e-3), "unit": UNIT,
                     "roofline": {"bound": "hbm", "achieved": round(x_bytes / (ms_x * 1e-3) / 1e9, 1),
                                  "peak": 8000.0, "unit": "GB/s",
                                  "frac": round(x_bytes / (ms_x * 1e-3) / 8e12, 4), "bytes_per_launch": x_bytes,
                                  "kernels": "halo pack, both faces"},
                     "transport_roofline": {"bound": "hbm", "achieved": round(t_bytes / (ms_t * 1e-3) / 1e9, 1),
                                            "peak": 8000.0, "unit": "GB/s",
                                            "frac": round(t_bytes / (ms_t * 1e-3) / 8e12, 4)}}
        del sa, sb, msgs
        print(f"[bench] halo: {ms_x:.3f} ms pack, {ms_t:.3f} ms slab transport", file=sys.stderr,
              flush=True)
        # the whole grid on one GPU: 32 x 32 x 32 cells of 24^3 velocities, periodic
        wa = torch.rand((8 * hz, hy, hx, hn ** 3), dtype=torch.float64, device="cuda", generator=g)
        wb = torch.empty_like(wa)
        offw = np.zeros((3, hn))
        per3 = (fks.BC_PERIODIC,) * 3
        for _ in range(2):
            fks.transport_shift(wa, wb, hx, hy, 8 * hz, hdx, per3, hn, hT, hdt, offw)
            wa, wb = wb, wa
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        reps = 5
        ev[0].record(stream)
        for _ in range(reps):
            fks.transport_shift(wa, wb, hx, hy, 8 * hz, hdx, per3, hn, hT, hdt, offw)
            wa, wb = wb, wa
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms_w = ev[0].elapsed_time(ev[1]) / reps
        w_bytes = 8 * hz * hy * hx * hn ** 3 * 16.0
        halo_line["whole_grid_transport"] = {
            "workload": f"{hx}x{hy}x{8 * hz} cells of {hn}^3 velocities on one GPU, periodic, CFL 0.95",
            "ms": round(ms_w, 4), "value": 8 * hz * hy * hx * hn ** 3 / (ms_w * 1e-3), "unit": UNIT,
            "roofline": {"bound": "hbm", "achieved": round(w_bytes / (ms_w * 1e-3) / 1e9, 1), "peak": 8000.0,
                         "unit": "GB/s", "frac": round(w_bytes / (ms_w * 1e-3) / 8e12, 4),
                         "bytes_per_launch": w_bytes}}
        del wa, wb
        print(f"[bench] whole-grid transport: {ms_w:.3f} ms", file=sys.stderr, flush=True)

    # two velocity dimensions: Maxwell molecules, 8192 cells of 32^2, A = 8 (Test 1.1 resolution)
    d2_line = None
    if "collide2d" in extras:
        n2, T2, c2 = 32, 9.0, 8192
        f2 = torch.as_tensor(synth.two_maxwellian_cells_2d(n2, T2, c2, seed_offset=123), device=dev)
        g2 = torch.empty_like(f2)
        d2_line = {}
        for prec, name in ((fks.PREC_F64, "f64"), (fks.PREC_F32_FIX64, "f32+f64fix")):
            with fks.Plan(fks.desc2d(n2, T2, 8, prec)) as p2:
                fks.collide(p2, f2, f_out=g2, dt_over_tau=0.02)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(args.steps):
                    fks.collide(p2, f2, f_out=g2, dt_over_tau=0.02)
                e1.record(stream)
                torch.cuda.synchronize()
                ms2 = e0.elapsed_time(e1) / args.steps
                fl = p2.info.flops_per_cell * c2 / (ms2 * 1e-3) / 1e12
                peak = PEAK_FP32_VECTOR_TFLOPS if prec == fks.PREC_F32_FIX64 else PEAK_FP64_VECTOR_TFLOPS
                roof = {"bound": "alu", "achieved": round(fl, 2), "peak": peak, "unit": "TFLOP/s",
                        "frac": round(fl / peak, 4)}
                d2_line[name] = {"ms": round(ms2, 4), "value": c2 * n2 * n2 / (ms2 * 1e-3),
                                 "unit": "cells·N²/s", "algorithmic_tflops": round(fl, 2), "roofline": roof}
        d2_line["workload"] = f"{c2} cells, 2D Maxwell molecules, 32^2 on [-9,9]^2, A = 8, f_out"
        del f2, g2
        print(f"[bench] 2d: {d2_line['f64']['ms']:.3f} ms (f64), {d2_line['f32+f64fix']['ms']:.3f} ms (f32)",
              file=sys.stderr, flush=True)

    # de-aliased (zero-padded 3n/2) variant, FP32 + FP64 fix, on the first 512 cells of the batch
    dealias_line = None
    if "dealias" in extras:
        cd = 512
        with fks.Plan(fks.Desc(n=N_V, T=T_BOX, gamma=1.0, n_polar=N_POLAR, n_azim=N_AZIM,
                               precision=fks.PREC_F32_FIX64, flags=fks.FLAG_DEALIAS)) as pd:
            fa_d, fb_d = fa[:cd], fb[:cd]
            wsd = fks.collide(pd, fa_d, f_out=fb_d, dt_over_tau=DT_OVER_TAU)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 2
            e0.record(stream)
            for _ in range(reps):
                fks.collide(pd, fa_d, f_out=fb_d, dt_over_tau=DT_OVER_TAU, workspace=wsd)
            e1.record(stream)
            torch.cuda.synchronize()
            msd = e0.elapsed_time(e1) / reps
            dealias_line = {"workload": f"{cd} cells of the batch, 32^3, M = 32, zero-padded 48^3 products, "
                                        "FP32 + FP64 fix, products and 48^3 transforms on the on-chip n = 48 "
                                        "kernel, multi-pass forward and truncating passes, f_out",
                            "ms": round(msd, 3), "value": cd * N_V ** 3 / (msd * 1e-3), "unit": UNIT,
                            "algorithmic_tflops": round(pd.info.flops_per_cell * cd / (msd * 1e-3) / 1e12, 2)}
            fl_d = pd.info.flops_per_cell * cd / (msd * 1e-3) / 1e12
            dealias_line["roofline"] = {"bound": "alu", "achieved": round(fl_d, 2), "peak": PEAK_FP32_VECTOR_TFLOPS,
                                        "unit": "TFLOP/s", "frac": round(fl_d / PEAK_FP32_VECTOR_TFLOPS, 4),
                                        "flops": "algorithmic: zero-padded transforms, products, truncation"}
            del wsd
        print(f"[bench] dealias: {msd:.2f} ms for {cd} cells", file=sys.stderr, flush=True)

    # uneven batch: 2048 cells with (n, M, gamma) drawn from {16, 24, 32, 48} x {16, 32, 64} x
    # {0, 0.5, 1}, one fks_collide_batch over 36 segments, FP32 + FP64 fix; timed with the built-in
    # schedules, then after fks_autotune
    uneven_line = None
    if "uneven" in extras:
        ns, Ms, gs = synth.uneven_batch_draws(2048)
        groups = {}
        for c in range(2048):
            groups.setdefault((int(ns[c]), int(Ms[c]), float(gs[c])), []).append(c)
        segs, segs64, plans_u, pts, flops = [], [], [], 0, 0.0
        for gi, (key, cells) in enumerate(sorted(groups.items())):
            nu_, mu_, gu_ = key
            npol, naz = synth.UNEVEN_SPLIT[mu_]
            pu = fks.Plan(fks.Desc(n=nu_, T=T_BOX, gamma=gu_, n_polar=npol, n_azim=naz,
                                   precision=fks.PREC_F32_FIX64))
            pu64 = fks.Plan(fks.Desc(n=nu_, T=T_BOX, gamma=gu_, n_polar=npol, n_azim=naz,
                                     precision=fks.PREC_F64))
            plans_u += [pu, pu64]
            fu = synth.two_maxwellian_torch(nu_, T_BOX, len(cells), dev, seed_offset=500 + gi)
            out = torch.empty_like(fu)
            segs.append((pu, fu, None, out, len(cells), DT_OVER_TAU))
            segs64.append((pu64, fu, None, out, len(cells), DT_OVER_TAU))
            pts += len(cells) * nu_ ** 3
            flops += len(cells) * pu.info.flops_per_cell

        def time_uneven(sg, reps=3):
            # the whole call captured once as a graph, then replayed
            wsu = torch.empty(max(fks.workspace_size(sg), 1), dtype=torch.uint8, device=dev)
            fks.collide_batch(sg, workspace=wsu)
            torch.cuda.synchronize()
            capu = torch.cuda.Stream()
            capu.wait_stream(stream)
            gu = torch.cuda.CUDAGraph()
            with torch.cuda.graph(gu, stream=capu):
                fks.collide_batch(sg, workspace=wsu)
            torch.cuda.synchronize()
            gu.replay()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                gu.replay()
            e1.record(stream)
            torch.cuda.synchronize()
            del gu, wsu
            return e0.elapsed_time(e1) / reps

        print(f"[bench] uneven: {len(plans_u)} plans built, timing", file=sys.stderr, flush=True)
        ms_cost = time_uneven(segs)
        if args.uneven_quick:
            choices, ms_tuned, ms_u64 = [], ms_cost, float("nan")
        else:
            choices = fks.autotune(segs)
            ms_tuned = time_uneven(segs)
            ms_u64 = time_uneven(segs64, reps=1)
        uneven_line = {"workload": "2048 cells, (n, M, gamma) from {16,24,32,48} x {16,32,64} x {0,0.5,1}, "
                                   "36 segments in one call, FP32 + FP64 fix, f_out",
                       "timing": "hipGraph replay of the whole call",
                       "ms_cost_model": round(ms_cost, 3), "ms_autotuned": round(ms_tuned, 3),
                       "ms_fp64_path": round(ms_u64, 3) if ms_u64 == ms_u64 else None,
                       "speedup_fp32fix_over_fp64": round(ms_u64 / ms_tuned, 2) if ms_u64 == ms_u64 else None,
                       "value": pts / (ms_tuned * 1e-3), "unit": UNIT,
                       "algorithmic_tflops": round(flops / (ms_tuned * 1e-3) / 1e12, 2),
                       "roofline": {"bound": "alu", "achieved": round(flops / (ms_tuned * 1e-3) / 1e12, 2),
                                    "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                                    "frac": round(flops / (ms_tuned * 1e-3) / 1e12 / PEAK_FP32_VECTOR_TFLOPS, 4)},
                       "launch_groups": "one work queue per n in {16, 24, 32} over its 9 segments (term "
                                        "ranges, partials, one FP64 finish); n = 48: one launch of the "
                                        "three-workgroup kernel over its 9 segments; the FP64 leg runs "
                                        "segment by segment on the multi-pass path",
                       "autotuned_alone": {"fused_one_per_cell": sum(1 for o, c, t in choices if o == 1),
                                           "fused_pairs": sum(1 for o, c, t in choices if o == 0)}}
        if not args.uneven_quick:
            # items per resident workgroup that fks_autotune kept for each work queue (the first
            # segment of each n leads its queue; 0 would be the cost model's 4)
            leads = {}
            for sg in segs:
                leads.setdefault(sg[0].info.n, sg[0].info.queue_items_per_wg)
            uneven_line["autotuned_queue_items_per_wg"] = {str(k): v for k, v in sorted(leads.items()) if k != 48}
        for pu in plans_u:
            pu.close()
        del segs, segs64
        print(f"[bench] uneven: {ms_cost:.2f} ms (cost model), {ms_tuned:.2f} ms (autotuned), "
              f"FP64 path {ms_u64:.2f} ms", file=sys.stderr, flush=True)

    # plain FP64 path (multi-pass), same workload
    fp64 = None
    if args.fp64_steps > 0:
        plan64 = fks.Plan(fks.Desc(n=N_V, T=T_BOX, gamma=1.0, n_polar=N_POLAR, n_azim=N_AZIM,
                                   precision=fks.PREC_F64))
        ws64 = fks.collide_batch([(plan64, f0, None, fb, NCELL, DT_OVER_TAU)])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.fp64_steps):
            fks.collide_batch([(plan64, f0, None, fb, NCELL, DT_OVER_TAU)], workspace=ws64)
        e1.record(stream)
        torch.cuda.synchronize()
        ms64 = e0.elapsed_time(e1) / args.fp64_steps
        fp64_roof_ms = plan64.info.flops_per_cell * NCELL / (PEAK_FP64_VECTOR_TFLOPS * 1e12) * 1e3
        fp64 = {"ms_per_step": round(ms64, 3), "value": NCELL * N_V ** 3 / (ms64 * 1e-3), "unit": UNIT,
                "speedup_fp32fix_over_fp64": round(ms64 / ms_per_step, 2),
                "fp64_roofline_ms": round(fp64_roof_ms, 3),
                "fp64_frac": round(fp64_roof_ms / ms64, 4),
                "fp32fix_ms_per_step": round(ms_per_step, 4),
                "note": "the FP64 path is multi-pass; fp64_roofline_ms is the same batch at the FP64 "
                        "vector peak, the time any FP64 kernel would need at least"}
        print(f"[bench] fp64 plain: {ms64:.2f} ms/step (FP64 roofline {fp64_roof_ms:.2f} ms; "
              f"FP32+fix {ms_per_step:.2f} ms)", file=sys.stderr, flush=True)
        del ws64
        plan64.close()

    # CPU oracle baseline on a bounded sample; also the parity check of the untimed Q_c run
    cpu = None
    parity = None
    if args.cpu_sample > 0:
        nsamp = args.cpu_sample
        sample = list(range(0, NCELL, NCELL // nsamp))[:nsamp]
        workers = args.cpu_workers or min(16, os.cpu_count() or 1, nsamp)
        print(f"[bench] oracle on {nsamp} cells with {workers} workers", file=sys.stderr, flush=True)
        cpu, ref = cpu_baseline(sample, workers)
        qs = q[sample].cpu().numpy()
        rs = np.stack([ref[c][0] for c in sample])
        ratios = np.array([ref[c][1] for c in sample])
        per = [float(np.sqrt(np.sum((qs[i] - rs[i]) ** 2) / np.sum(rs[i] ** 2))) for i in range(nsamp)]
        parity = {"cells": nsamp,
                  "aggregate_rel_l2": float(np.sqrt(np.sum((qs - rs) ** 2) / np.sum(rs ** 2))),
                  "per_cell_max": max(per), "per_cell_median": float(np.median(per)),
                  "max_cancellation_ratio": float(ratios.max())}

    # the oracle beside the extra lines (bounded samples, one core each)
    kinds = [k for k in ("collide2d", "bgk", "dealias", "halo", "moments") if k in extras]
    if kinds and args.cpu_sample > 0:
        extra_cpu = cpu_extras(kinds)
        for k, ln in (("collide2d", d2_line), ("bgk", bgk_line), ("dealias", dealias_line),
                      ("halo", halo_line), ("moments", moments_line)):
            if ln is not None and k in extra_cpu:
                ln["cpu_baseline"] = extra_cpu[k]

    line = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "ms_per_step_median": round(median_ms, 4),
        "timing": ("hipGraph replay of one captured step per ping-pong direction" if graphs else "eager launches")
                  + "; ms_per_step = total of the timed steps / steps",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64fix",
        "data": "synthetic",
        "config": {"workload": "4096 homogeneous hard-sphere cells, velocity 32^3 on [-8,8)^3, "
                               "M=32 (8 Gauss polar x 4 azimuthal), seeded two-Maxwellian data",
                   "cells": NCELL, "n": N_V, "M": plan.info.M, "gamma": 1.0, "T": T_BOX,
                   "R": plan.info.R, "dt_over_tau": DT_OVER_TAU, "terms_per_cell": plan.info.J},
        "roofline": {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved_tflops / PEAK_FP32_VECTOR_TFLOPS, 4),
                     "traffic": _traffic_per_launch(), "valu_busy_counters": _valu_busy(), "kernel": kernel_name,
                     "avg_launch_ms": round(terms_ms, 4), "finish_kernel_ms": round(finish_ms, 4),
                     "call_ms": round(avg_call_ms, 4), "flops_per_cell": plan.info.flops_per_cell,
                     "source_hash": _fused_source_hash()},
        "cpu_baseline": cpu,
        "plan": {"ms_create": round(plan_ms, 3), "table_bytes": plan.info.table_bytes,
                 "what": "fks_plan_create of the timed configuration (host rule and radial terms, FP64 "
                         "device tables, FP32 copies, loss table, Gram matrix), once per configuration, "
                         "outside the timed steps"},
        "fp64_path": fp64,
        "parity": parity,
        "bgk": bgk_line,
        "collide2d": d2_line,
        "dealias": dealias_line,
        "halo": halo_line,
        "moments": moments_line,
        "uneven": uneven_line,
    }
    del ws
    plan.close()
    torch.cuda.synchronize()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
