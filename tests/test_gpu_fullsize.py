"""The multi-size workloads at their full sizes, checked on sampled cells that the
oracle evaluates one by one and through properties that hold at any size:

  * uneven batch: 2048 cells, (n, M, gamma) drawn from {16, 24, 32, 48} x
    {16, 32, 64} x {0, 0.5, 1}, two-Maxwellian data, one fks_collide_batch call
    over 36 segments, FP32 + FP64 fix (fused kernels; three workgroups per
    cell at n = 48) and the plain FP64 path;
  * 3D x 3D periodic blast: 32^3 cells x 24^3 velocities, VHS gamma = 0.5
    with K = 7 radial terms (225 terms per cell), tau = 0.3.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
import paper_1608_08009_amd as fks  # noqa: E402
from paper_1608_08009_amd.splitstep import Space, SplitStepper, stable_dt  # noqa: E402

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def _conservation(q, n, T):
    """max over cells and invariants of |C q|_a / (|C| |q|)_a (torch, FP64)."""
    v = torch.as_tensor(O.velocity_grid(n, T), device=q.device)
    vx, vy, vz = torch.meshgrid(v, v, v, indexing="ij")
    rows = [torch.ones_like(vx), vx, vy, vz, vx * vx + vy * vy + vz * vz]
    qq = q.reshape(q.shape[0], -1)
    worst = 0.0
    for r in rows:
        r = r.reshape(-1)
        num = (qq @ r).abs()
        den = qq.abs() @ r.abs()
        worst = max(worst, float((num / den).max()))
    return worst


def test_uneven_batch_full_size():
    T = 8.0
    ns, Ms, gs = synth.uneven_batch_draws(2048)
    groups = {}
    for c in range(2048):
        groups.setdefault((int(ns[c]), int(Ms[c]), float(gs[c])), []).append(c)
    assert len(groups) == 36
    segs, segs64, data, plans = [], [], {}, []
    for gi, (key, cells) in enumerate(sorted(groups.items())):
        n, M, gamma = key
        npol, naz = synth.UNEVEN_SPLIT[M]
        plan = fks.Plan(fks.Desc(n=n, T=T, gamma=gamma, n_polar=npol, n_azim=naz,
                                 precision=fks.PREC_F32_FIX64))
        plan64 = fks.Plan(fks.Desc(n=n, T=T, gamma=gamma, n_polar=npol, n_azim=naz,
                                   precision=fks.PREC_F64))
        plans += [plan, plan64]
        f = synth.two_maxwellian_cells(n, T, len(cells), seed_offset=500 + gi)
        fd = torch.as_tensor(f, device="cuda")
        q, q64 = torch.empty_like(fd), torch.empty_like(fd)
        segs.append((plan, fd, q, None, len(cells), 0.0))
        segs64.append((plan64, fd, q64, None, len(cells), 0.0))
        data[key] = (f, q, q64, plan, gi)
    for sg in (segs, segs64):   # FP32 + fix, then the plain FP64 path: one call each
        ws = torch.empty(max(fks.workspace_size(sg), 1), dtype=torch.uint8, device="cuda")
        print(f"uneven batch: precision {sg[0][0].info.precision}", flush=True)
        fks.collide_batch(sg, workspace=ws)
        torch.cuda.synchronize()
        del ws
    # every cell of every segment conserves mass, momentum and energy; FP32 + fix against FP64
    # per segment (aggregate over its cells, the metric's measure)
    for (n, M, gamma), (f, q, q64, plan, gi) in data.items():
        assert _conservation(q, n, T) <= 1e-12, (n, M, gamma)
        assert _conservation(q64, n, T) <= 1e-12, (n, M, gamma)
        assert plan.info.fused == 1
        agg = float(torch.sqrt(torch.sum((q - q64) ** 2) / torch.sum(q64 ** 2)))
        assert agg <= 1e-5, ((n, M, gamma), agg)
    # sampled cells against the oracle: one per (n, gamma), from the cheapest M (n = 48 with
    # K > 1 takes the oracle about 15 s per table set)
    errs = []
    for n in synth.UNEVEN_N:
        for gamma in synth.UNEVEN_GAMMA:
            key = min((k for k in data if k[0] == n and k[2] == gamma), key=lambda k: k[1])
            f, q, q64, plan, gi = data[key]
            npol, naz = synth.UNEVEN_SPLIT[key[1]]
            print(f"uneven batch: oracle cell of (n, M, gamma) = {key}", flush=True)
            op = O.make_plan(n, T, gamma=gamma, n_polar=npol, n_azim=naz)
            assert op.radial.K == plan.info.K
            Qf, _, loss = O.collide_fast64(f[0], op, parts=True)
            ref = O.conserve_Q(Qf, n, T)
            got = q[0].cpu().numpy()
            ratio = np.linalg.norm(loss) / np.linalg.norm(ref)
            e = _rel(got, ref)
            assert e <= 1.5e-6 * (1.0 + ratio), (key, e, ratio)
            # the FP64 path: round-off of the transforms; K-term plans 1e-11 (two eigen-solvers)
            e64 = _rel(q64[0].cpu().numpy(), ref)
            assert e64 <= (1e-12 if gamma == 1.0 else 1e-11) * (1.0 + ratio), (key, e64, ratio)
            errs.append((got, ref))
    agg = math.sqrt(sum(np.sum((a - b) ** 2) for a, b in errs) / sum(np.sum(b ** 2) for _, b in errs))
    assert agg <= 1e-5
    for p in plans:
        p.close()


def test_blast_full_size():
    nc, n, T, gamma, tau = 32, 24, 8.0, 0.5, 0.3
    rho = synth.blast_density(nc).ravel()                    # cell index (z nc + y) nc + x
    ncell = nc ** 3
    f_host = np.empty((ncell, n, n, n))
    for c in range(ncell):
        f_host[c] = synth.blast_cell(n, T, rho[c], c)
    U = np.zeros((ncell, 5))
    U[:, 0] = rho
    U[:, 4] = 3.0 * rho
    f0 = torch.as_tensor(f_host, device="cuda")
    fks.conserve(f0, torch.as_tensor(U, device="cuda"), n, T)   # t = 0 projection to the intended moments
    space = Space(nc, nc, nc, 1.0 / nc)
    sample = [0, 16 * 1024 + 16 * 32 + 16, ncell - 1, 12345]    # a corner, the blast centre, others
    with fks.Plan(fks.Desc(n=n, T=T, gamma=gamma, precision=fks.PREC_F32_FIX64)) as p32:
        assert p32.info.K == 7 and p32.info.J == 225 and p32.info.fused == 1
        # one collision evaluation of the whole batch, sampled against the oracle
        q = torch.empty_like(f0)
        fks.collide(p32, f0, q_out=q)
        torch.cuda.synchronize()
        op = O.make_plan(n, T, gamma=gamma)
        for c in sample:
            fo = O.project(f_host[c], U[c], n, T)
            assert np.max(np.abs(f0[c].cpu().numpy() - fo)) <= 1e-15 * np.max(fo)
            Qf, _, loss = O.collide_fast64(fo, op, parts=True)
            ref = O.conserve_Q(Qf, n, T)
            ratio = np.linalg.norm(loss) / np.linalg.norm(ref)
            e = _rel(q[c].cpu().numpy(), ref)
            assert e <= 1.5e-6 * (1.0 + ratio), (c, e, ratio)
        del q
        dt = stable_dt(space, T, tau, p32.info.R, gamma, p32.info.c_gamma, float(rho.max()))
        tot0 = fks.moments(f0, n, T).sum(dim=0).cpu().numpy()
        # FP32 + fix against FP64 over two split steps
        out = {}
        st32 = SplitStepper(p32, space, f0.clone())
        for _ in range(2):
            st32.step(dt, tau)
        out[32] = st32.f
        with fks.Plan(fks.Desc(n=n, T=T, gamma=gamma, precision=fks.PREC_F64)) as p64:
            st64 = SplitStepper(p64, space, f0.clone())
            for _ in range(2):
                st64.step(dt, tau)
            torch.cuda.synchronize()
            out[64] = st64.f
            del st64
        a, b = out[32], out[64]
        rel = float(torch.sqrt(torch.sum((a - b) ** 2) / torch.sum(b ** 2)))
        assert rel <= 1e-6, rel
        # ten more FP32 steps: the periodic totals are conserved to round-off
        for _ in range(10):
            st32.step(dt, tau)
        torch.cuda.synchronize()
        tot = fks.moments(st32.f, n, T).sum(dim=0).cpu().numpy()
        scale = np.array([tot0[0]] * 4 + [tot0[4]])
        assert np.all(np.abs(tot - tot0) <= 1e-12 * scale), (tot - tot0) / scale
