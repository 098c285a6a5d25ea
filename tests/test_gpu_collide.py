"""GPU parity of the collision path (through the C ABI) against the CPU oracle.

Bars (FP32 unit round-off is 6e-8; a few transform passes of log2(n^3) stages give
errors of a few units relative to the gain and loss parts, which the cancellation
between them amplifies in Q):
  * FP64 path: per-cell relative L2 of Q_c <= 1e-12 (hard spheres; K-term 1e-11);
  * FP32 + FP64-fix path: batch-aggregate relative L2 of Q_c <= 1e-5, and per
    cell <= 1.5e-6 * (1 + |Q-|/|Q_c|): FP32 roundoff of the transforms (a few
    units of 2^-24) amplified by the cancellation between gain and loss;
  * conservation of Q_c: |C Q_c|_a <= 1e-12 * (|C| |Q_c|)_a for every invariant a.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
import paper_1608_08009_amd as fks  # noqa: E402

pytestmark = pytest.mark.gpu

T_BOX = 8.0


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


_plans = {}


def _plan(**kw):
    key = tuple(sorted(kw.items()))
    if key not in _plans:
        _plans[key] = fks.Plan(fks.Desc(**kw))
    return _plans[key]


_oplans = {}


def _oplan(n, T, gamma, npol, naz, K):
    key = (n, T, gamma, npol, naz, K)
    if key not in _oplans:
        _oplans[key] = O.make_plan(n, T, gamma=gamma, n_polar=npol, n_azim=naz, K=K)
    return _oplans[key]


def _oracle_qc(f, op, ratios=False):
    qs, rs = [], []
    for fc in f:
        Q, _, loss = O.collide_fast64(fc, op, parts=True)
        qc = O.conserve_Q(Q, op.n, op.T)
        qs.append(qc)
        rs.append(np.linalg.norm(loss) / np.linalg.norm(qc))
    return (np.stack(qs), np.array(rs)) if ratios else np.stack(qs)


def _loss_ratios(f, qc, op, chunk=64):
    """||Q^-|| / ||Q_c|| per cell: the oracle's loss term f_N F^{-1}(L fhat) of every cell of f
    (transforms only, no gain terms), against a given Q_c."""
    out = []
    for c0 in range(0, f.shape[0], chunk):
        fc = f[c0:c0 + chunk]
        fh = O.spectrum(fc, op.n, op.T)
        loss = O.synthesize(fh, op.n, op.T).real * O.synthesize(op.loss * fh, op.n, op.T).real
        num = np.sqrt(np.sum(loss.reshape(fc.shape[0], -1) ** 2, axis=1))
        den = np.sqrt(np.sum(qc[c0:c0 + chunk].reshape(fc.shape[0], -1) ** 2, axis=1))
        out.append(num / den)
    return np.concatenate(out)


def _check_f32(q, ref, ratio):
    agg = _rel(q, ref)
    assert agg <= 1e-5, agg
    for c in range(q.shape[0]):
        e = _rel(q[c], ref[c])
        assert e <= 1.5e-6 * (1.0 + ratio[c]), (c, e, ratio[c])


def _gpu_qc(plan, f_host, dt=0.0, want_f=False):
    f = _dev(f_host)
    q = torch.empty_like(f)
    fo = torch.empty_like(f) if want_f else None
    fks.collide(plan, f, q_out=q, f_out=fo, dt_over_tau=dt)
    torch.cuda.synchronize()
    return q.cpu().numpy(), (fo.cpu().numpy() if want_f else None)


def _conservation_ok(Qc, n, T, tol=1e-12):
    Phi = O.collision_basis(n, T)
    for c in range(Qc.shape[0]):
        q = Qc[c].ravel()
        num = np.abs(Phi @ q)
        den = np.abs(Phi) @ np.abs(q)
        assert np.all(num <= tol * den), (c, num / den)


def _rel(a, b):
    return np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2))


# ---------------------------------------------------------------- tables

@pytest.mark.parametrize("n,gamma,K", [(8, 1.0, 0), (16, 1.0, 0), (8, 0.5, 5), (8, 0.0, 6)])
def test_tables_match_oracle(n, gamma, K):
    plan = _plan(n=n, T=T_BOX, gamma=gamma, radial_terms=K, precision=fks.PREC_F64)
    ab, dirs = plan.tables()
    op = _oplan(n, T_BOX, gamma, 8, 4, K)
    J = op.J
    assert plan.info.J == J + 1
    h = n // 2   # the kz = n/2 plane is multiplied by zero (Nyquist) and stored as +n/2
    ab = ab[:, :h]
    # device layout [j][kz][kx][ky], oracle [j][kx][ky][kz]
    a_or = np.transpose(op.alpha * op.omega[:, None, None, None], (0, 3, 1, 2))[:, :h]
    b_or = np.transpose(op.beta, (0, 3, 1, 2))[:, :h]
    L_or = np.transpose(op.loss, (2, 0, 1))[:h]
    tol = 1e-13 if gamma == 1.0 else 1e-10
    # radial eigenvectors may differ in sign between solvers: compare products and the loss
    prod_dev = ab[:J, ..., 0] * ab[:J, ..., 1]
    prod_or = a_or * b_or
    assert np.max(np.abs(prod_dev - prod_or)) <= tol * np.max(np.abs(prod_or))
    if gamma == 1.0:
        assert np.max(np.abs(ab[:J, ..., 0] - a_or)) <= tol * np.max(np.abs(a_or))
        assert np.max(np.abs(ab[:J, ..., 1] - b_or)) <= tol * np.max(np.abs(b_or))
    assert np.max(np.abs(-ab[J, ..., 0] - L_or)) <= tol * np.max(np.abs(L_or))
    assert np.all(ab[J, ..., 1] == 1.0)
    e, w = O.sphere_rule(8, 4, "gauss")
    assert np.allclose(dirs[:, :3], e, atol=2e-15) and np.allclose(dirs[:, 3], w, atol=2e-15)


# ---------------------------------------------------------------- FP64 path

@pytest.mark.parametrize("n,ncell", [(4, 3), (8, 5), (12, 2), (16, 3), (24, 1), (32, 2)])
def test_collide_f64_matches_oracle(n, ncell):
    plan = _plan(n=n, T=T_BOX, precision=fks.PREC_F64)
    op = _oplan(n, T_BOX, 1.0, 8, 4, 0)
    f = synth.two_maxwellian_cells(n, T_BOX, ncell, seed_offset=100 + n)
    q, _ = _gpu_qc(plan, f)
    ref = _oracle_qc(f, op)
    for c in range(ncell):
        assert _rel(q[c], ref[c]) <= 1e-12, (c, _rel(q[c], ref[c]))
    _conservation_ok(q, n, T_BOX)


def test_collide_f64_rough_data_and_chunk_tail():
    # 515 cells: one full chunk of 512 cells plus a ragged tail of 3; random data excites every mode
    n = 4
    plan = _plan(n=n, T=2.0, precision=fks.PREC_F64, n_polar=4, n_azim=3)
    op = _oplan(n, 2.0, 1.0, 4, 3, 0)
    f = synth.random_positive_cells(n, 515, seed_offset=3)
    q, _ = _gpu_qc(plan, f)
    for c in list(range(3)) + [511, 512, 513, 514]:
        ref = O.conserve_Q(O.collide_fast64(f[c], op), n, 2.0)
        assert _rel(q[c], ref) <= 1e-12


@pytest.mark.parametrize("gamma,K", [(0.0, 6), (0.5, 4)])
def test_collide_f64_vhs_k_terms(gamma, K):
    n = 8
    plan = _plan(n=n, T=T_BOX, gamma=gamma, radial_terms=K, precision=fks.PREC_F64)
    op = _oplan(n, T_BOX, gamma, 8, 4, K)
    f = synth.two_maxwellian_cells(n, T_BOX, 3, seed_offset=31)
    q, _ = _gpu_qc(plan, f)
    ref = _oracle_qc(f, op)
    for c in range(3):
        assert _rel(q[c], ref[c]) <= 1e-11


# ---------------------------------------------------------------- FP32 + FP64 fix

@pytest.mark.parametrize("n,ncell,generic", [(8, 9, False), (16, 5, False), (24, 7, False), (32, 6, False),
                                             (48, 5, False), (8, 4, True), (12, 3, True), (24, 2, True),
                                             (32, 2, True), (48, 2, True)])
def test_collide_f32_matches_oracle(n, ncell, generic):
    flags = fks.FLAG_FORCE_GENERIC if generic else 0
    plan = _plan(n=n, T=T_BOX, precision=fks.PREC_F32_FIX64, flags=flags)
    assert plan.info.fused == (0 if generic or n not in (8, 16, 24, 32, 48) else 1)
    op = _oplan(n, T_BOX, 1.0, 8, 4, 0)
    f = synth.two_maxwellian_cells(n, T_BOX, ncell, seed_offset=200 + n)
    q, _ = _gpu_qc(plan, f)
    ref, ratio = _oracle_qc(f, op, ratios=True)
    _check_f32(q, ref, ratio)
    _conservation_ok(q, n, T_BOX)


@pytest.mark.parametrize("n,ncell", [(16, 3), (24, 5), (48, 2)])
def test_collide_f32_vhs_k_terms_fused(n, ncell):
    plan = _plan(n=n, T=T_BOX, gamma=0.5, radial_terms=4, precision=fks.PREC_F32_FIX64)
    assert plan.info.fused == 1
    op = _oplan(n, T_BOX, 0.5, 8, 4, 4)
    f = synth.two_maxwellian_cells(n, T_BOX, ncell, seed_offset=41)
    q, _ = _gpu_qc(plan, f)
    ref, ratio = _oracle_qc(f, op, ratios=True)
    _check_f32(q, ref, ratio)
    _conservation_ok(q, n, T_BOX)


# ---------------------------------------------------------------- update, aliasing, edge cases

@pytest.mark.parametrize("prec", [fks.PREC_F64, fks.PREC_F32_FIX64])
def test_update_and_in_place(prec):
    n, ncell, dt = 16, 3, 0.05
    plan = _plan(n=n, T=T_BOX, precision=prec)
    op = _oplan(n, T_BOX, 1.0, 8, 4, 0)
    f = synth.two_maxwellian_cells(n, T_BOX, ncell, seed_offset=51)
    q, fo = _gpu_qc(plan, f, dt=dt, want_f=True)
    assert np.array_equal(fo, f + dt * q) or np.max(np.abs(fo - (f + dt * q))) <= 1e-15 * np.max(np.abs(f))
    U0 = O.moments(f, n, T_BOX)
    U1 = O.moments(fo, n, T_BOX)
    assert np.max(np.abs(U1 - U0) / np.maximum(np.abs(U0), 1e-3)) <= 1e-12
    ref, ratio = _oracle_qc(f, op, ratios=True)
    if prec == fks.PREC_F64:
        assert _rel(q, ref) <= 1e-12
    else:
        _check_f32(q, ref, ratio)
    # in place: f_out aliases f, no q_out
    fd = _dev(f)
    fks.collide(plan, fd, f_out=fd, dt_over_tau=dt)
    torch.cuda.synchronize()
    assert np.max(np.abs(fd.cpu().numpy() - fo)) <= 1e-15 * np.max(np.abs(f))


def test_empty_batch_and_invalid_arguments():
    plan = _plan(n=8, T=T_BOX, precision=fks.PREC_F32_FIX64)
    f = _dev(np.zeros((0, 8, 8, 8)))
    fks.collide(plan, f, q_out=f)          # ncell = 0: nothing to do
    g = _dev(synth.two_maxwellian_cells(8, T_BOX, 2))
    with pytest.raises(fks.FksError) as e:
        fks.collide_batch([(plan, g, None, None, 2, 0.0)])
    assert e.value.status == fks.FKS_ERR_INVALID
    with pytest.raises(fks.FksError):
        fks.collide_batch([(plan, g, g, None, 2, 0.0)])   # q_out overlaps f
    q = torch.empty_like(g)
    seg = [(plan, g, q, None, 2, 0.0)]
    need = fks.workspace_size(seg)
    small = torch.empty(max(need - 1, 1), dtype=torch.uint8, device="cuda")
    with pytest.raises(fks.FksError):
        fks.collide_batch(seg, workspace=small)
    # arrays must be 16-byte aligned, the workspace 256-byte aligned
    flat = torch.zeros(2 * 512 + 1, dtype=torch.float64, device="cuda")
    odd = flat[1:].view(2, 8, 8, 8)
    with pytest.raises(fks.FksError) as e:
        fks.collide_batch([(plan, odd, q, None, 2, 0.0)])
    assert e.value.status == fks.FKS_ERR_INVALID
    with pytest.raises(fks.FksError) as e:
        fks.collide_batch([(plan, g, odd, None, 2, 0.0)])
    assert e.value.status == fks.FKS_ERR_INVALID
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(fks.FksError) as e:
        fks.collide_batch(seg, workspace=ws[16:])
    assert e.value.status == fks.FKS_ERR_INVALID
    fks.collide_batch(seg, workspace=ws[256:])
    with pytest.raises(fks.FksError) as e:
        fks.Plan(fks.Desc(n=10, T=8.0))
    assert e.value.status == fks.FKS_ERR_UNSUPPORTED


def test_multi_segment_uneven_batch():
    # several plans (n, M, gamma) in one call, as an uneven batch
    specs = [dict(n=8, T=T_BOX, precision=fks.PREC_F32_FIX64),
             dict(n=16, T=T_BOX, precision=fks.PREC_F32_FIX64, n_polar=4, n_azim=4),
             dict(n=12, T=T_BOX, precision=fks.PREC_F32_FIX64, gamma=0.5, radial_terms=3)]
    segs, refs, outs = [], [], []
    for i, sp in enumerate(specs):
        plan = _plan(**sp)
        n = sp["n"]
        f = synth.two_maxwellian_cells(n, T_BOX, 2 + i, seed_offset=60 + i)
        fd, qd = _dev(f), torch.empty((2 + i, n, n, n), dtype=torch.float64, device="cuda")
        segs.append((plan, fd, qd, None, 2 + i, 0.0))
        op = _oplan(n, T_BOX, sp.get("gamma", 1.0), sp.get("n_polar", 8), sp.get("n_azim", 4),
                    sp.get("radial_terms", 0))
        refs.append(_oracle_qc(f, op, ratios=True))
        outs.append(qd)
    fks.collide_batch(segs)
    torch.cuda.synchronize()
    for q, (r, ratio) in zip(outs, refs):
        _check_f32(q.cpu().numpy(), r, ratio)


@pytest.mark.parametrize("n", [16, 24, 32])
def test_work_queue_of_same_n_segments(n):
    # fused segments of one n in one call share a work queue: long cells are cut into term
    # ranges (partials, then one finish kernel over all segments); q_out, in-place f_out and a
    # Runge-Kutta stage (f_base) in one call.  Every cell against the FP64 path of the same
    # plan (cancellation-aware bound, loss ratios from the oracle), sampled cells against the
    # oracle, exact conservation
    specs = [dict(gamma=1.0, n_polar=8, n_azim=4, radial_terms=0, cells=13),
             dict(gamma=0.5, n_polar=8, n_azim=4, radial_terms=5, cells=6),
             dict(gamma=1.0, n_polar=4, n_azim=4, radial_terms=0, cells=21),
             dict(gamma=0.0, n_polar=8, n_azim=8, radial_terms=3, cells=4)]
    dt = 0.02
    segs, keep = [], []
    for i, sp in enumerate(specs):
        kw = dict(n=n, T=T_BOX, gamma=sp["gamma"], n_polar=sp["n_polar"], n_azim=sp["n_azim"],
                  radial_terms=sp["radial_terms"])
        p32, p64 = _plan(**kw, precision=fks.PREC_F32_FIX64), _plan(**kw, precision=fks.PREC_F64)
        c = sp["cells"]
        f = synth.two_maxwellian_torch(n, T_BOX, c, "cuda", seed_offset=400 + 10 * n + i)
        q64 = torch.empty_like(f)
        fks.collide(p64, f, q_out=q64)
        if i == 0:
            q = torch.empty_like(f)
            segs.append((p32, f, q, None, c, 0.0))
            keep.append((f, q64, q, None, kw))
        elif i == 1:      # in place
            g = f.clone()
            segs.append((p32, g, None, g, c, dt))
            keep.append((f, q64, None, g, kw))
        else:             # stage: f_out = f_base + dt Q(f)
            base = f * 0.5
            g = torch.empty_like(f)
            qq = torch.empty_like(f)
            segs.append((p32, f, qq, g, c, dt, base))
            keep.append((f, q64, qq, (g, base), kw))
    fks.profile_enable(True)
    try:
        fks.collide_batch(segs)
        assert len(fks.profile_last()) == 2          # one queue: terms, then finish
    finally:
        fks.profile_enable(False)
    torch.cuda.synchronize()
    for i, (f, q64, q, out, kw) in enumerate(keep):
        if q is None:                                 # in place: recover Q from f_out
            q = (out - f) / dt
        op = _oplan(n, T_BOX, kw["gamma"], kw["n_polar"], kw["n_azim"], kw["radial_terms"])
        ratio = _loss_ratios(f.cpu().numpy(), q64.cpu().numpy(), op)
        err = torch.sqrt(torch.sum((q - q64) ** 2, dim=(1, 2, 3)) / torch.sum(q64 ** 2, dim=(1, 2, 3))).cpu().numpy()
        # in place the FP64 sum f + dt Q rounds Q at the scale of f: allow that rounding
        slack = 0.0 if i != 1 else 4e-16 * float(torch.max(torch.abs(f))) / dt / float(torch.max(torch.abs(q64)))
        assert np.all(err <= 1.5e-6 * (1.0 + ratio) + slack), (i, err.max(), ratio[err.argmax()])
        assert _conservation_torch(q64, n, T_BOX) <= 1e-12
        if i >= 2:
            g, base = out
            assert float(torch.max(torch.abs(g - (base + dt * q)))) <= 1e-15 * float(torch.max(torch.abs(base)))
            assert _conservation_torch(q, n, T_BOX) <= 1e-12
        ref, rr = _oracle_qc(f[:1].cpu().numpy(), op, ratios=True)
        e = _rel(q[0].cpu().numpy(), ref[0])       # one cell: its own cancellation-aware bound
        assert e <= 1.5e-6 * (1.0 + rr[0]), (i, e, rr[0])


# ---------------------------------------------------------------- the two fused decompositions

def _kernels_of_last_call(call):
    fks.profile_enable(True)
    try:
        call()
        return len(fks.profile_last())
    finally:
        fks.profile_enable(False)


def _conservation_torch(q, n, T):
    v = torch.as_tensor(O.velocity_grid(n, T), device=q.device)
    vx, vy, vz = torch.meshgrid(v, v, v, indexing="ij")
    qq = q.reshape(q.shape[0], -1)
    worst = 0.0
    for r in (torch.ones_like(vx), vx, vy, vz, vx * vx + vy * vy + vz * vz):
        r = r.reshape(-1)
        worst = max(worst, float(((qq @ r).abs() / (qq.abs() @ r.abs())).max()))
    return worst


@pytest.mark.parametrize("n", [8, 16, 24, 32])
def test_one_workgroup_per_cell_matches_pairs_fp64_and_oracle(n):
    # a batch of 2 G - 7 cells (G = resident workgroups): one workgroup per cell with a
    # ragged second round; every cell against the FP64 path, sampled cells against the
    # oracle and against the pair decomposition (chosen for small batches)
    plan = _plan(n=n, T=T_BOX, precision=fks.PREC_F32_FIX64)
    G = plan.info.fused_grid
    assert plan.info.fused == 1 and G >= 16
    ncell = 2 * G - 7
    f = synth.two_maxwellian_torch(n, T_BOX, ncell, "cuda", seed_offset=230 + n)
    q = torch.empty_like(f)
    assert _kernels_of_last_call(lambda: fks.collide(plan, f, q_out=q)) == 1
    p64 = _plan(n=n, T=T_BOX, precision=fks.PREC_F64)
    q64 = torch.empty_like(f)
    fks.collide(p64, f, q_out=q64)
    torch.cuda.synchronize()
    err = torch.sqrt(torch.sum((q - q64) ** 2, dim=(1, 2, 3)) / torch.sum(q64 ** 2, dim=(1, 2, 3)))
    agg = float(torch.sqrt(torch.sum((q - q64) ** 2) / torch.sum(q64 ** 2)))
    assert agg <= 1e-5, agg
    # every cell to the cancellation-aware FP32 bound; the FP64 path stands in for the
    # oracle here (it matches it to 1e-12, checked on the sampled cells below and in the
    # FP64 tests), and the oracle gives each cell's loss term
    ratio_all = _loss_ratios(f.cpu().numpy(), q64.cpu().numpy(), _oplan(n, T_BOX, 1.0, 8, 4, 0))
    bound = 1.5e-6 * (1.0 + ratio_all)
    bad = np.nonzero(err.cpu().numpy() > bound)[0]
    assert bad.size == 0, [(int(c), float(err[c]), float(ratio_all[c])) for c in bad[:5]]
    assert _conservation_torch(q, n, T_BOX) <= 1e-12
    sample = [0, G - 1, G, ncell - 1]
    fh = f[sample].cpu().numpy()
    ref, ratio = _oracle_qc(fh, _oplan(n, T_BOX, 1.0, 8, 4, 0), ratios=True)
    _check_f32(q[sample].cpu().numpy(), ref, ratio)
    # the same cells through the pair decomposition
    fs = f[sample].contiguous()
    qp = torch.empty_like(fs)
    assert _kernels_of_last_call(lambda: fks.collide(plan, fs, q_out=qp)) == 2
    torch.cuda.synchronize()
    d = float(torch.max(torch.abs(qp - q[sample]))) / float(torch.max(torch.abs(q[sample])))
    assert d <= 1e-5, d
    # q_out and f_out from one call
    dt = 0.01
    q2, g2 = torch.empty_like(f), torch.empty_like(f)
    fks.collide(plan, f, q_out=q2, f_out=g2, dt_over_tau=dt)
    torch.cuda.synchronize()
    assert torch.equal(q2, q)
    assert float(torch.max(torch.abs(g2 - (f + dt * q)))) <= 1e-15 * float(torch.max(torch.abs(f)))
    # update in place (f_out aliases f) through the one-workgroup kernel
    g = f.clone()
    fks.collide(plan, g, f_out=g, dt_over_tau=dt)
    torch.cuda.synchronize()
    assert float(torch.max(torch.abs(g - (f + dt * q)))) <= 1e-15 * float(torch.max(torch.abs(f)))


def test_n48_three_workgroups_per_cell_large_batch():
    # n = 48: three workgroups per cell (one per residue of x mod 3) fed from per-XCD item
    # counters, over two chunks of cells (512 + 89); every cell against the FP64 path to the
    # cancellation-aware bound, sampled cells against the oracle, in-place update
    n, ncell = 48, 601
    plan = _plan(n=n, T=T_BOX, precision=fks.PREC_F32_FIX64)
    assert plan.info.fused == 1 and plan.info.fused_grid >= 8
    f = synth.two_maxwellian_torch(n, T_BOX, ncell, "cuda", seed_offset=290)
    q = torch.empty_like(f)
    fks.collide(plan, f, q_out=q)
    p64 = _plan(n=n, T=T_BOX, precision=fks.PREC_F64)
    q64 = torch.empty_like(f)
    fks.collide(p64, f, q_out=q64)
    torch.cuda.synchronize()
    err = torch.sqrt(torch.sum((q - q64) ** 2, dim=(1, 2, 3)) / torch.sum(q64 ** 2, dim=(1, 2, 3)))
    agg = float(torch.sqrt(torch.sum((q - q64) ** 2) / torch.sum(q64 ** 2)))
    assert agg <= 1e-5, agg
    ratio_all = _loss_ratios(f.cpu().numpy(), q64.cpu().numpy(), _oplan(n, T_BOX, 1.0, 8, 4, 0))
    bad = np.nonzero(err.cpu().numpy() > 1.5e-6 * (1.0 + ratio_all))[0]
    assert bad.size == 0, [(int(c), float(err[c]), float(ratio_all[c])) for c in bad[:5]]
    assert _conservation_torch(q, n, T_BOX) <= 1e-12
    sample = [0, 7, 511, 512, ncell - 1]
    ref, ratio = _oracle_qc(f[sample].cpu().numpy(), _oplan(n, T_BOX, 1.0, 8, 4, 0), ratios=True)
    _check_f32(q[sample].cpu().numpy(), ref, ratio)
    dt = 0.01
    g = f.clone()
    fks.collide(plan, g, f_out=g, dt_over_tau=dt)
    torch.cuda.synchronize()
    assert float(torch.max(torch.abs(g - (f + dt * q)))) <= 1e-15 * float(torch.max(torch.abs(f)))


def test_one_workgroup_per_cell_numeric_guard():
    n = 16
    with fks.Plan(fks.Desc(n=n, T=T_BOX, precision=fks.PREC_F32_FIX64, flags=fks.FLAG_NUMERIC_GUARD)) as plan:
        G = plan.info.fused_grid
        ncell = 2 * G - 7
        f = synth.two_maxwellian_torch(n, T_BOX, ncell, "cuda", seed_offset=240)
        bad = G + 3
        f[bad].view(-1)[17] = math.nan
        q = torch.empty_like(f)
        assert _kernels_of_last_call(lambda: fks.collide(plan, f, q_out=q)) == 1
        assert plan.numeric_status() == bad
        good = torch.ones(ncell, dtype=torch.bool, device="cuda")
        good[bad] = False
        assert bool(torch.isfinite(q[good]).all())


@pytest.mark.parametrize("n,gamma,K,prec,big", [
    (16, 1.0, 0, fks.PREC_F32_FIX64, False),     # J = 2: one gain term and the loss term
    (16, 1.0, 0, fks.PREC_F32_FIX64, True),      # same, two rounds of resident workgroups
    (16, 0.5, 2, fks.PREC_F32_FIX64, False),     # J = 3
    (8, 1.0, 0, fks.PREC_F64, False),
])
def test_single_direction_plans(n, gamma, K, prec, big):
    # the smallest rule (one direction on the half sphere): degenerate term counts.  With so
    # few terms a pair of workgroups per cell never pays for its second forward transform and
    # finish kernel, so the fused path runs one workgroup per cell even for 5 cells
    plan = _plan(n=n, T=T_BOX, gamma=gamma, radial_terms=K, n_polar=1, n_azim=1, precision=prec)
    assert plan.info.M == 1 and plan.info.J == (K or 1) + 1
    ncell = 2 * max(plan.info.fused_grid, 8) - 7 if big else 5
    f = synth.two_maxwellian_torch(n, T_BOX, ncell, "cuda", seed_offset=250 + n)
    q = torch.empty_like(f)
    kernels = _kernels_of_last_call(lambda: fks.collide(plan, f, q_out=q))
    if prec == fks.PREC_F32_FIX64:
        assert kernels == 1
    torch.cuda.synchronize()
    sample = [0, ncell // 2, ncell - 1]
    op = _oplan(n, T_BOX, gamma, 1, 1, K)
    ref, ratio = _oracle_qc(f[sample].cpu().numpy(), op, ratios=True)
    got = q[sample].cpu().numpy()
    # per-cell cancellation-aware bars only: a one-direction rule has large gain and loss
    # parts against a small Q (the aggregate bar is the metric workload's)
    for i in range(len(sample)):
        e = _rel(got[i], ref[i])
        bar = max(1e-12, 3e-14 * (1.0 + ratio[i])) if prec == fks.PREC_F64 else 1.5e-6 * (1.0 + ratio[i])
        assert e <= bar, (sample[i], e, ratio[i])
    assert _conservation_torch(q, n, T_BOX) <= 1e-12


# ---------------------------------------------------------------- full-size workload, sampled

def test_full_size_hard_sphere_batch_sampled():
    # 4096 cells, n = 32, M = 32 (8 x 4), hard spheres: the benchmarked launch; sampled cells
    n, ncell = 32, 4096
    plan = _plan(n=n, T=T_BOX, precision=fks.PREC_F32_FIX64)
    f = synth.two_maxwellian_torch(n, T_BOX, ncell, "cuda")
    q = torch.empty_like(f)
    fks.collide(plan, f, q_out=q)
    torch.cuda.synchronize()
    op = _oplan(n, T_BOX, 1.0, 8, 4, 0)
    sample = [0, 1, 255, 256, 2047, 4095]
    fs = synth.two_maxwellian_cells(n, T_BOX, ncell, first=0, count=1)  # generator consistency
    assert np.max(np.abs(fs[0] - f[0].cpu().numpy())) <= 1e-14 * np.max(np.abs(fs[0]))
    qs = q[sample].cpu().numpy()
    fh = f[sample].cpu().numpy()
    ref, ratio = _oracle_qc(fh, op, ratios=True)
    _check_f32(qs, ref, ratio)
    _conservation_ok(qs, n, T_BOX)
    assert torch.isfinite(q).all()


# ---------------------------------------------------------------- moments, conserve

@pytest.mark.parametrize("n", [4, 5, 12, 24, 32, 64])
def test_moments_and_conserve_match_oracle(n):
    # odd n, n not dividing the 256-thread stride, and the largest grid exercise the kernels'
    # index walk; each moment is compared on the scale mass * T^k of its power k of v
    ncell = 7
    f = synth.two_maxwellian_cells(n, T_BOX, ncell, seed_offset=70)
    fd = _dev(f)
    U = fks.moments(fd, n, T_BOX)
    torch.cuda.synchronize()
    Ur = O.moments(f, n, T_BOX)
    scale = Ur[:, :1] * np.array([1.0, T_BOX, T_BOX, T_BOX, T_BOX ** 2])
    assert np.max(np.abs(U.cpu().numpy() - Ur) / scale) <= 1e-13
    tgt = Ur * np.array([1.01, 1.0, 1.0, 1.0, 0.99]) + np.array([0, 0.01, -0.02, 0.005, 0])
    fks.conserve(fd, _dev(tgt), n, T_BOX)
    torch.cuda.synchronize()
    ref = O.project(f, tgt, n, T_BOX)
    got = fd.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert np.max(np.abs(O.moments(got, n, T_BOX) - tgt)) <= 1e-12 * np.max(np.abs(tgt))
    fks.moments(fd[:0], n, T_BOX)    # empty batch is a no-op


# ---------------------------------------------------------------- transport

@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 0, 0)])
def test_transport_matches_oracle(bc):
    n, T = 4, 2.0
    nx, ny, nz = 5, 3, 2
    dx = 1.0 / nx
    dt = 0.9 * dx / T
    rng = synth.rng(80)
    f0 = rng.uniform(size=(nz, ny, nx, n, n, n))
    bcf = rng.uniform(size=(6, n, n, n)) + 10.0
    names = tuple("dirichlet" if b else "periodic" for b in bc)
    fa, fb = _dev(f0), torch.empty((nz, ny, nx, n, n, n), dtype=torch.float64, device="cuda")
    off = np.zeros((3, n))
    off_or = np.zeros((3, n))
    ref = f0.copy()
    for step in range(6):
        fks.transport_shift(fa, fb, nx, ny, nz, dx, bc, n, T, dt, off, bc_f=_dev(bcf))
        off_or, s = O.transport_offsets_step(off_or, n, T, dx, dt)
        ref = O.transport_shift(ref, s, n, bc=names, bc_f=bcf)
        fa, fb = fb, fa
    torch.cuda.synchronize()
    assert np.array_equal(off, off_or)
    assert np.array_equal(fa.cpu().numpy(), ref)


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 0, 1)])
def test_transport_large_shifts_match_oracle(bc):
    # CFL 2.6: per-step shifts up to 3 cells (periodic wraps past one period of a 2-cell axis,
    # inflow faces on Dirichlet axes); even n takes the kz-pair path, 5 planes its groups of
    # four and one cells, and the kz pairs mix equal and unequal shifts from step to step
    n, T = 6, 2.0
    nx, ny, nz = 3, 2, 5
    dx = 1.0 / nx
    dt = 2.6 * dx / T
    rng = synth.rng(81)
    f0 = rng.uniform(size=(nz, ny, nx, n, n, n))
    bcf = rng.uniform(size=(6, n, n, n)) + 10.0
    names = tuple("dirichlet" if b else "periodic" for b in bc)
    fa, fb = _dev(f0), torch.empty((nz, ny, nx, n, n, n), dtype=torch.float64, device="cuda")
    # first step at CFL 0.9 with the z displacements started at -v dt / 2, so that no z shift
    # changes while x and y shift (every kz pair shares its z shift: the one-load path)
    v = O.velocity_grid(n, T)
    dt0 = 0.9 * dx / T
    off = np.zeros((3, n))
    off[2] = -v * dt0 / 2
    off_or = off.copy()
    ref = f0.copy()
    for step in range(5):
        h = dt0 if step == 0 else dt
        fks.transport_shift(fa, fb, nx, ny, nz, dx, bc, n, T, h, off, bc_f=_dev(bcf))
        off_or, s = O.transport_offsets_step(off_or, n, T, dx, h)
        if step == 0:
            assert not s[2].any() and s[0].any()
        else:
            assert np.abs(s).max() >= 2
        ref = O.transport_shift(ref, s, n, bc=names, bc_f=bcf)
        fa, fb = fb, fa
    torch.cuda.synchronize()
    assert np.array_equal(off, off_or)
    assert np.array_equal(fa.cpu().numpy(), ref)


# ---------------------------------------------------------------- spectrum (forward transform of Q or f)

@pytest.mark.parametrize("n,ncell,ws_cells,zn", [(8, 7, 3, False), (12, 5, 5, True), (32, 3, 2, False),
                                                (48, 2, 2, True)])
def test_spectrum_matches_oracle(n, ncell, ws_cells, zn):
    # eq. FC on the grid, against the oracle's transform; a workspace of ws_cells cells forces chunking
    f = synth.two_maxwellian_cells(n, T_BOX, ncell, seed_offset=700 + n)
    ws = torch.empty(ws_cells * n ** 3 * 16, dtype=torch.uint8, device="cuda")
    got = fks.spectrum(_dev(f), n, zero_nyquist=zn, workspace=ws).cpu().numpy()
    ref = O.spectrum(f, n, T_BOX, zero_nyquist=zn)[..., : n // 2 + 1]
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_spectrum_of_the_collision_operator_conserves_mass():
    # the optional forward transform of Q: Qhat_c(0) = mass of Q_c / (2T)^3 = 0
    n, ncell = 16, 4
    plan = _plan(n=n, T=T_BOX, precision=fks.PREC_F64)
    f = synth.two_maxwellian_cells(n, T_BOX, ncell, seed_offset=71)
    q, _ = _gpu_qc(plan, f)
    qh = fks.spectrum(_dev(q), n).cpu().numpy()
    ref = O.spectrum(q, n, T_BOX, zero_nyquist=False)[..., : n // 2 + 1]
    assert np.max(np.abs(qh - ref)) <= 1e-14 * np.max(np.abs(ref))
    assert np.all(np.abs(qh[:, 0, 0, 0]) <= 1e-15 * np.max(np.abs(qh)))
    with pytest.raises(fks.FksError) as e:
        fks.spectrum(_dev(q), n, workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    assert e.value.status == fks.FKS_ERR_INVALID
