"""fks_collide_batch_static (the allocation-free variant of fks_collide_batch)
against fks_collide_batch with a caller workspace: same segments, same kernels
and schedules, so the outputs must agree bit for bit.  Two calls in a row, the
second on a smaller batch (the static workspace keeps the first call's contents),
then a request larger than the static workspace, which must be rejected before
anything is enqueued."""
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_1608_08009_amd as fks  # noqa: E402

pytestmark = pytest.mark.gpu


def _both(segs_static, segs_ws, outs_static, outs_ws):
    for o in outs_static + outs_ws:
        o.fill_(-7.0)
    ws = torch.empty(max(fks.workspace_size(segs_ws), 1), dtype=torch.uint8, device="cuda")
    fks.collide_batch(segs_ws, workspace=ws)
    fks.collide_batch_static(segs_static)
    torch.cuda.synchronize()
    for a, b in zip(outs_static, outs_ws):
        assert torch.equal(a, b)


@pytest.mark.parametrize("n,ncells", [(32, (4096, 37)), (16, (1100, 90)), (24, (64, 5))])
def test_static_matches_workspace_call_twice(n, ncells):
    T = 8.0
    with fks.Plan(fks.Desc(n=n, T=T, precision=fks.PREC_F32_FIX64)) as plan:
        for k, ncell in enumerate(ncells):   # second call: smaller batch, stale workspace
            print(f"static workspace: n={n} ncell={ncell} call {k}", flush=True)
            f = synth.two_maxwellian_torch(n, T, ncell, "cuda", seed_offset=600 + n + k)
            q1, g1, q2, g2 = (torch.empty_like(f) for _ in range(4))
            assert fks.workspace_size([(plan, f, q1, g1, ncell, 0.01)]) <= fks.STATIC_WORKSPACE_BYTES
            _both([(plan, f, q1, g1, ncell, 0.01)], [(plan, f, q2, g2, ncell, 0.01)], [q1, g1], [q2, g2])
            assert torch.isfinite(q1).all()


def test_static_uneven_batch_and_fp64():
    # several plans in one call: fused FP32 at two sizes, the multi-pass FP64 path and 2D
    T = 8.0
    with fks.Plan(fks.Desc(n=32, T=T)) as p32, fks.Plan(fks.Desc(n=16, T=T, gamma=0.5, radial_terms=3)) as p16, \
            fks.Plan(fks.Desc(n=16, T=T, precision=fks.PREC_F64)) as p64, fks.Plan(fks.desc2d(32, T)) as p2:
        fa = synth.two_maxwellian_torch(32, T, 20, "cuda", seed_offset=611)
        fb = synth.two_maxwellian_torch(16, T, 33, "cuda", seed_offset=612)
        fc = synth.two_maxwellian_torch(16, T, 9, "cuda", seed_offset=613)
        fd = torch.as_tensor(synth.two_maxwellian_cells_2d(32, T, 40, seed_offset=614), device="cuda")
        outs_s = [torch.empty_like(x) for x in (fa, fb, fc, fd)]
        outs_w = [torch.empty_like(x) for x in (fa, fb, fc, fd)]
        segs = lambda o: [(p32, fa, o[0], None, 20, 0.0), (p16, fb, o[1], None, 33, 0.0),
                          (p64, fc, o[2], None, 9, 0.0), (p2, fd, o[3], None, 40, 0.0)]
        assert fks.workspace_size(segs(outs_w)) <= fks.STATIC_WORKSPACE_BYTES
        print("static workspace: uneven batch", flush=True)
        _both(segs(outs_s), segs(outs_w), outs_s, outs_w)


def test_static_rejects_batches_beyond_its_size():
    T = 8.0
    with fks.Plan(fks.Desc(n=32, T=T, precision=fks.PREC_F64)) as plan:
        ncell = 1024
        f = torch.zeros((ncell, 32, 32, 32), dtype=torch.float64, device="cuda")
        q = torch.full_like(f, 3.0)
        seg = [(plan, f, q, None, ncell, 0.0)]
        assert fks.workspace_size(seg) > fks.STATIC_WORKSPACE_BYTES
        with pytest.raises(fks.FksError) as e:
            fks.collide_batch_static(seg)
        assert e.value.status == fks.FKS_ERR_INVALID
        torch.cuda.synchronize()
        assert bool((q == 3.0).all())   # nothing was enqueued
