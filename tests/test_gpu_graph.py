"""The batched calls under graph capture: each captured call is replayed several
times, with eager work and synchronisations between the replays, and every
replay must reproduce the eager result bit for bit (the kernels are
deterministic and allocate nothing)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_1608_08009_amd as fks  # noqa: E402

pytestmark = pytest.mark.gpu


def _replays_match(call, outs, nrep=3):
    for o in outs:
        o.fill_(0.0)
    call()
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cap):
        call()
    torch.cuda.synchronize()
    for _ in range(nrep):
        for o in outs:
            o.fill_(-1.0)                      # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e)


@pytest.mark.parametrize("n,prec", [(32, fks.PREC_F32_FIX64), (16, fks.PREC_F64), (24, fks.PREC_F32_FIX64)])
def test_collide_batch_graph_replay(n, prec):
    f = torch.as_tensor(synth.two_maxwellian_cells(n, 8.0, 21, seed_offset=130 + n), device="cuda")
    q = torch.empty_like(f)
    g = torch.empty_like(f)
    with fks.Plan(fks.Desc(n=n, T=8.0, precision=prec)) as plan:
        seg = [(plan, f, q, g, 21, 0.01)]
        ws = torch.empty(max(fks.workspace_size(seg), 1), dtype=torch.uint8, device="cuda")
        _replays_match(lambda: fks.collide_batch(seg, workspace=ws), [q, g])


def test_one_workgroup_per_cell_graph_replay():
    # a batch large enough for the one-workgroup-per-cell kernel (ragged last round)
    with fks.Plan(fks.Desc(n=16, T=8.0, precision=fks.PREC_F32_FIX64)) as plan:
        ncell = 2 * plan.info.fused_grid - 7
        f = synth.two_maxwellian_torch(16, 8.0, ncell, "cuda", seed_offset=135)
        q, g = torch.empty_like(f), torch.empty_like(f)
        seg = [(plan, f, q, g, ncell, 0.01)]
        ws = torch.empty(max(fks.workspace_size(seg), 1), dtype=torch.uint8, device="cuda")
        _replays_match(lambda: fks.collide_batch(seg, workspace=ws), [q, g])


def test_collide2d_and_bgk_graph_replay():
    f2 = torch.as_tensor(synth.two_maxwellian_cells_2d(32, 9.0, 17, seed_offset=140), device="cuda")
    f3 = torch.as_tensor(synth.two_maxwellian_cells(32, 8.0, 5, seed_offset=141), device="cuda")
    q2, q3, g3 = torch.empty_like(f2), torch.empty_like(f3), torch.empty_like(f3)
    with fks.Plan(fks.desc2d(32, 9.0, 8, fks.PREC_F64)) as p2:
        def call():
            fks.collide(p2, f2, q_out=q2)
            fks.bgk(f3, 32, 8.0, 0.8, dim=3, q_out=q3, f_out=g3, dt_over_tau=0.1, nu_rho=True)
        _replays_match(call, [q2, q3, g3])


def test_uneven_batch_after_autotune_graph_replay():
    # one call over segments that form every launch group: a work queue (two n = 16 segments),
    # the n = 48 three-workgroup kernel over two segments, an n = 24 segment alone, an FP64
    # multi-pass segment; schedules and the queue's items per workgroup chosen by fks_autotune
    # first, then the captured call replayed against the eager one
    specs = [(16, fks.PREC_F32_FIX64, 1.0, 7), (48, fks.PREC_F32_FIX64, 1.0, 3), (16, fks.PREC_F32_FIX64, 0.5, 5),
             (24, fks.PREC_F32_FIX64, 1.0, 4), (48, fks.PREC_F32_FIX64, 0.0, 2), (16, fks.PREC_F64, 1.0, 6)]
    plans, segs, outs = [], [], []
    try:
        for i, (n, prec, gamma, c) in enumerate(specs):
            p = fks.Plan(fks.Desc(n=n, T=8.0, gamma=gamma, n_polar=4, n_azim=4, precision=prec))
            plans.append(p)
            f = synth.two_maxwellian_torch(n, 8.0, c, "cuda", seed_offset=150 + i)
            q, g = torch.empty_like(f), torch.empty_like(f)
            segs.append((p, f, q, g, c, 0.01))
            outs += [q, g]
        fks.autotune(segs)
        ws = torch.empty(max(fks.workspace_size(segs), 1), dtype=torch.uint8, device="cuda")
        _replays_match(lambda: fks.collide_batch(segs, workspace=ws), outs)
    finally:
        for p in plans:
            p.close()
