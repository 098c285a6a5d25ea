"""The autotuner (fks_autotune): it keeps, per (plan, ncell), the fastest of the schedules
fks_collide_batch can use; later calls follow the kept schedule; schedules never change the
operator (multi-pass chunking and terms per launch are bit-identical, the fused
decompositions agree to FP32 round-off); segments whose outputs feed their inputs are
rejected."""
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_1608_08009_amd as fks  # noqa: E402

pytestmark = pytest.mark.gpu

T_BOX = 8.0


def _kernels(call):
    fks.profile_enable(True)
    try:
        call()
        return len(fks.profile_last())
    finally:
        fks.profile_enable(False)


def test_fused_choice_is_kept_and_followed():
    n, ncell = 16, 300
    with fks.Plan(fks.Desc(n=n, T=T_BOX, precision=fks.PREC_F32_FIX64)) as plan, \
            fks.Plan(fks.Desc(n=n, T=T_BOX, precision=fks.PREC_F64)) as p64:
        f = synth.two_maxwellian_torch(n, T_BOX, ncell, "cuda", seed_offset=260)
        q, q64 = torch.empty_like(f), torch.empty_like(f)
        fks.collide(p64, f, q_out=q64)
        seg = [(plan, f, q, None, ncell, 0.0)]
        (one, chunk, terms), = fks.autotune(seg)
        assert one in (0, 1) and chunk == 0 and terms == 0
        ws = torch.empty(max(fks.workspace_size(seg), 1), dtype=torch.uint8, device="cuda")
        assert _kernels(lambda: fks.collide_batch(seg, workspace=ws)) == (1 if one else 2)
        torch.cuda.synchronize()
        rel = float(torch.sqrt(torch.sum((q - q64) ** 2) / torch.sum(q64 ** 2)))
        assert rel <= 1e-5, rel
        # another batch size keeps the cost model: 5 cells of this plan run as pairs
        g = f[:5].contiguous()
        assert _kernels(lambda: fks.collide(plan, g, q_out=torch.empty_like(g))) == 2


@pytest.mark.parametrize("n,prec,flags", [(48, fks.PREC_F32_FIX64, fks.FLAG_FORCE_GENERIC), (16, fks.PREC_F64, 0),
                                          (8, fks.PREC_F32_FIX64, fks.FLAG_DEALIAS)])
def test_multi_pass_chunking_is_bit_identical(n, prec, flags):
    ncell = 100
    f = synth.two_maxwellian_torch(n, T_BOX, ncell, "cuda", seed_offset=270 + n)
    with fks.Plan(fks.Desc(n=n, T=T_BOX, precision=prec, flags=flags)) as plan:
        assert plan.info.fused == 0
        q0, q1 = torch.empty_like(f), torch.empty_like(f)
        fks.collide(plan, f, q_out=q0)
        seg = [(plan, f, q1, None, ncell, 0.0)]
        (one, chunk, terms), = fks.autotune(seg)
        assert one == -1 and chunk in (32, 64, 100)
        assert terms == (0 if flags & fks.FLAG_DEALIAS else terms) and terms in (0, 1, 2, 4)
        q1.fill_(0.0)
        fks.collide_batch(seg)
        torch.cuda.synchronize()
        assert torch.equal(q0, q1)


def test_rejections_and_tight_workspace_and_2d():
    n, ncell = 16, 40
    f = synth.two_maxwellian_torch(n, T_BOX, ncell, "cuda", seed_offset=280)
    with fks.Plan(fks.Desc(n=n, T=T_BOX, precision=fks.PREC_F64)) as plan:
        with pytest.raises(fks.FksError) as e:
            fks.autotune([(plan, f, None, f, ncell, 0.1)])        # in place: outputs feed inputs
        assert e.value.status == fks.FKS_ERR_INVALID
        q = torch.empty_like(f)
        seg = [(plan, f, q, None, ncell, 0.0)]
        # a workspace for the default schedule only: the larger candidates are skipped
        ws = torch.empty(fks.workspace_size(seg), dtype=torch.uint8, device="cuda")
        (one, chunk, terms), = fks.autotune(seg, workspace=ws)
        assert one == -1 and chunk in (32, 40) and terms in (1, 2, 4)
    with fks.Plan(fks.desc2d(16, 6.0, 8, fks.PREC_F64)) as p2:
        g = torch.as_tensor(synth.two_maxwellian_cells_2d(16, 6.0, 4, seed_offset=281), device="cuda")
        assert fks.autotune([(p2, g, torch.empty_like(g), None, 4, 0.0)]) == [(-1, 0, 0)]


def test_work_queue_items_per_workgroup_is_tuned_and_followed():
    # fused segments of one n that fks_collide_batch runs as one work queue are timed as that
    # queue with 1, 2, 4 or 8 items per resident workgroup; the fastest is kept in every plan of
    # the group and changes only the term ranges of the items (the summation order of the FP32
    # partials), so the operator stays within FP32 round-off of the FP64 path
    n = 16
    specs = [(1.0, 8, 4, 0, 40), (0.5, 8, 4, 5, 17), (1.0, 4, 4, 0, 33)]
    plans, segs, refs = [], [], []
    try:
        for i, (gamma, npol, naz, K, c) in enumerate(specs):
            kw = dict(n=n, T=T_BOX, gamma=gamma, n_polar=npol, n_azim=naz, radial_terms=K)
            p32 = fks.Plan(fks.Desc(**kw, precision=fks.PREC_F32_FIX64))
            p64 = fks.Plan(fks.Desc(**kw, precision=fks.PREC_F64))
            plans += [p32, p64]
            f = synth.two_maxwellian_torch(n, T_BOX, c, "cuda", seed_offset=290 + i)
            q64 = torch.empty_like(f)
            fks.collide(p64, f, q_out=q64)
            segs.append((p32, f, torch.empty_like(f), None, c, 0.0))
            refs.append(q64)
        assert all(p.info.queue_items_per_wg == 0 for p in plans[::2])
        fks.collide_batch(segs)
        torch.cuda.synchronize()
        before = [s[2].clone() for s in segs]
        fks.autotune(segs)
        kept = {p.info.queue_items_per_wg for p in plans[::2]}
        assert len(kept) == 1 and kept.pop() in (1, 2, 4, 8)
        ws = torch.empty(max(fks.workspace_size(segs), 1), dtype=torch.uint8, device="cuda")
        for s in segs:
            s[2].fill_(float("nan"))
        assert _kernels(lambda: fks.collide_batch(segs, workspace=ws)) == 2   # still one queue
        torch.cuda.synchronize()
        for s, q64, q0 in zip(segs, refs, before):
            q = s[2]
            rel = float(torch.sqrt(torch.sum((q - q64) ** 2) / torch.sum(q64 ** 2)))
            assert rel <= 1e-5, rel
            rel0 = float(torch.sqrt(torch.sum((q - q0) ** 2) / torch.sum(q64 ** 2)))
            assert rel0 <= 1e-5, rel0
    finally:
        for p in plans:
            p.close()
