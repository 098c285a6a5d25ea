"""GPU runs of the configured workloads (reduced where the oracle must follow),
compared with oracle-driven CPU loops and with physical invariants.

  * single-cell 3D BKW relaxation, Maxwell molecules (K radial terms), 10 Euler steps;
  * 1D x 3D Sod tube: transport shift + collision, Dirichlet inflow;
  * the full-size Sod tube (256 cells, 32^3, 100 steps) in FP32+fix against FP64;
  * 3D x 3D periodic blast with VHS gamma = 0.5: exact conservation of the totals;
  * uneven batch: several (n, M, gamma) plans in one call.
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


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _rel(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


# ---------------------------------------------------------------- BKW single cell

def test_bkw_single_cell_trajectory():
    n, T, t0, dt, steps = 16, 8.0, 5.5, 0.01, 10
    op = O.make_plan(n, T, gamma=0.0, n_polar=8, n_azim=4, radial_tol=1e-4)
    K = op.radial.K
    U = np.array([1.0, 0.0, 0.0, 0.0, 3.0])
    f0 = O.project(synth.bkw3d(n, T, t0), U, n, T)
    ref = f0.copy()
    for _ in range(steps):
        ref = O.euler_update(ref, O.conserve_Q(O.collide_fast64(ref, op), n, T), dt)
    exact = synth.bkw3d(n, T, t0 + steps * dt)
    err_or = _rel(ref, exact)
    assert err_or < 0.05          # discretisation error of the 16^3 grid
    for prec, tol in ((fks.PREC_F64, 1e-11), (fks.PREC_F32_FIX64, 1e-6)):
        plan = fks.Plan(fks.Desc(n=n, T=T, gamma=0.0, radial_terms=K, precision=prec))
        f = _dev(f0[None])
        for _ in range(steps):
            fks.collide(plan, f, f_out=f, dt_over_tau=dt)
        torch.cuda.synchronize()
        got = f[0].cpu().numpy()
        assert _rel(got, ref) <= tol, (prec, _rel(got, ref))
        assert abs(_rel(got, exact) - err_or) <= 1e-3 * err_or + tol
        assert np.allclose(O.moments(got, n, T), U, atol=1e-12, rtol=0)
        plan.close()


# ---------------------------------------------------------------- Sod tube (reduced, vs oracle)

def _sod_initial(n, T, nx):
    xc, rho, theta = synth.sod_states(nx)
    f = np.stack([synth.maxwellian(n, T, r, (0, 0, 0), th) for r, th in zip(rho, theta)])
    U = np.stack([[r, 0, 0, 0, 3 * r * th] for r, th in zip(rho, theta)])
    f = O.project(f, U, n, T)
    bc = np.zeros((6, n, n, n))
    bc[0] = f[0]
    bc[1] = f[-1]
    return f, bc


@pytest.mark.parametrize("prec,tol", [(fks.PREC_F64, 1e-12), (fks.PREC_F32_FIX64, 1e-6)])
def test_sod_tube_reduced_matches_oracle(prec, tol):
    n, T, nx, tau, steps = 16, 8.0, 8, 1e-2, 3
    f0, bc = _sod_initial(n, T, nx)
    plan = fks.Plan(fks.Desc(n=n, T=T, precision=prec))
    space = Space(nx, 1, 1, 1.0 / nx, (fks.BC_DIRICHLET, fks.BC_PERIODIC, fks.BC_PERIODIC))
    dt = stable_dt(space, T, tau, plan.info.R, 1.0, plan.info.c_gamma, 1.0)
    st = SplitStepper(plan, space, _dev(f0.reshape(1, 1, nx, n, n, n)), bc_f=_dev(bc))
    for _ in range(steps):
        st.step(dt, tau)
    torch.cuda.synchronize()
    got = st.f.cpu().numpy().reshape(nx, n, n, n)
    # oracle loop
    op = O.make_plan(n, T)
    g = f0.reshape(1, 1, nx, n, n, n)
    off = np.zeros((3, n))
    for _ in range(steps):
        off, s = O.transport_offsets_step(off, n, T, space.dx, dt)
        g = O.transport_shift(g, s, n, bc=("dirichlet", "periodic", "periodic"), bc_f=bc)
        g = np.stack([O.euler_update(c, O.conserve_Q(O.collide_fast64(c, op), n, T), dt / tau)
                      for c in g.reshape(nx, n, n, n)]).reshape(g.shape)
    assert np.array_equal(st.offsets, off)
    assert _rel(got, g.reshape(nx, n, n, n)) <= tol
    plan.close()


def test_sod_tube_full_size_fp32_against_fp64():
    # 256 cells on [0, 1], 32^3 velocities, hard spheres, Kn = 1e-2, 100 split steps
    n, T, nx, tau, steps = 32, 8.0, 256, 1e-2, 100
    f0, bc = _sod_initial(n, T, nx)
    space = Space(nx, 1, 1, 1.0 / nx, (fks.BC_DIRICHLET, fks.BC_PERIODIC, fks.BC_PERIODIC))
    out = {}
    for prec in (fks.PREC_F32_FIX64, fks.PREC_F64):
        plan = fks.Plan(fks.Desc(n=n, T=T, precision=prec))
        dt = stable_dt(space, T, tau, plan.info.R, 1.0, plan.info.c_gamma, 1.0)
        st = SplitStepper(plan, space, _dev(f0.reshape(1, 1, nx, n, n, n)), bc_f=_dev(bc))
        for _ in range(steps):
            st.step(dt, tau)
        torch.cuda.synchronize()
        out[prec] = st.f.reshape(nx, n, n, n)
        plan.close()
    a, b = out[fks.PREC_F32_FIX64], out[fks.PREC_F64]
    rel = float(torch.sqrt(torch.sum((a - b) ** 2) / torch.sum(b ** 2)))
    assert rel <= 1e-4, rel
    U = fks.moments(b, n, T).cpu().numpy()
    rho, u, th = O.primitive(U)
    assert np.all(np.isfinite(U))
    assert 0.1 < rho.min() and rho.max() < 1.05
    assert np.all(th > 0.5) and np.all(th < 1.2)
    # the shock tube has moved mass to the right: monotone density profile is no longer a step
    assert 0.125 < rho[nx // 2 + 4] < 1.0


# ---------------------------------------------------------------- 3D x 3D periodic blast (reduced)

def test_blast_periodic_conservation_and_oracle():
    n, T, nc, gamma, K, tau = 16, 8.0, 4, 0.5, 4, 0.3
    rho = synth.blast_density(nc)
    rng = synth.rng(5)
    f0 = np.stack([synth.maxwellian(n, T, r, (0, 0, 0), 1.0) for r in rho.ravel()])
    f0 = f0 * (1.0 + 0.01 * rng.normal(size=f0.shape))
    U0 = np.stack([[r, 0, 0, 0, 3 * r] for r in rho.ravel()])
    f0 = O.project(f0, U0, n, T)
    space = Space(nc, nc, nc, 1.0 / nc)
    for prec, tol in ((fks.PREC_F64, 1e-12), (fks.PREC_F32_FIX64, 1e-6)):
        plan = fks.Plan(fks.Desc(n=n, T=T, gamma=gamma, radial_terms=K, precision=prec))
        dt = stable_dt(space, T, tau, plan.info.R, gamma, plan.info.c_gamma, float(rho.max()))
        st = SplitStepper(plan, space, _dev(f0.reshape(nc, nc, nc, n, n, n)))
        tot0 = O.moments(f0, n, T).sum(axis=0)
        st.step(dt, tau)
        torch.cuda.synchronize()
        f1 = st.f.cpu().numpy().reshape(nc ** 3, n, n, n)
        if prec == fks.PREC_F64:
            op = O.make_plan(n, T, gamma=gamma, K=K)
            off, s = O.transport_offsets_step(np.zeros((3, n)), n, T, space.dx, dt)
            g = O.transport_shift(f0.reshape(nc, nc, nc, n, n, n), s, n).reshape(nc ** 3, n, n, n)
            ref = np.stack([O.euler_update(c, O.conserve_Q(O.collide_fast64(c, op), n, T), dt / tau) for c in g])
            assert _rel(f1, ref) <= tol
        st.step(dt, tau)
        torch.cuda.synchronize()
        tot2 = fks.moments(st.f, n, T).cpu().numpy().sum(axis=0)
        scale = np.array([tot0[0], tot0[0], tot0[0], tot0[0], tot0[4]])
        assert np.all(np.abs(tot2 - tot0) <= 1e-12 * scale), (prec, (tot2 - tot0) / scale)
        plan.close()


# ---------------------------------------------------------------- uneven batch (reduced)

@pytest.mark.parametrize("prec", [fks.PREC_F64, fks.PREC_F32_FIX64])
def test_uneven_batch_reduced(prec):
    combos = [(16, 4, 4, 0.0, 3), (24, 8, 4, 0.5, 2), (32, 4, 4, 1.0, 0), (48, 4, 4, 1.0, 0), (12, 8, 8, 1.0, 0)]
    T = 8.0
    segs, checks = [], []
    plans = []
    for i, (n, npol, naz, gamma, K) in enumerate(combos):
        plan = fks.Plan(fks.Desc(n=n, T=T, gamma=gamma, n_polar=npol, n_azim=naz, radial_terms=K,
                                 precision=prec))
        plans.append(plan)
        f = synth.two_maxwellian_cells(n, T, 2, seed_offset=300 + i)
        fd = _dev(f)
        q = torch.empty_like(fd)
        segs.append((plan, fd, q, None, 2, 0.0))
        op = O.make_plan(n, T, gamma=gamma, n_polar=npol, n_azim=naz, K=K)
        refs, ratios = [], []
        for c in f:
            Q, _, loss = O.collide_fast64(c, op, parts=True)
            qc = O.conserve_Q(Q, n, T)
            refs.append(qc)
            ratios.append(np.linalg.norm(loss) / np.linalg.norm(qc))
        checks.append((q, np.stack(refs), np.array(ratios)))
    fks.collide_batch(segs)
    torch.cuda.synchronize()
    for q, ref, ratio in checks:
        got = q.cpu().numpy()
        for c in range(got.shape[0]):
            e = _rel(got[c], ref[c])
            if prec == fks.PREC_F64:
                assert e <= 1e-11
            else:
                assert e <= 1.5e-6 * (1 + ratio[c]), (e, ratio[c])
    for p in plans:
        p.close()


# ---------------------------------------------------------------- Runge-Kutta stages and Strang splitting

@pytest.mark.parametrize("prec,tol", [(fks.PREC_F64, 1e-13), (fks.PREC_F32_FIX64, 1e-6)])
def test_f_base_stage_and_aliasing(prec, tol):
    # f_out = f_base + dt Q_c(f): the midpoint rule as two calls, with f_out aliasing f_base
    n, T, ncell, dt = 16, 8.0, 5, 0.05
    f = synth.two_maxwellian_cells(n, T, ncell, seed_offset=610)
    op = O.make_plan(n, T)
    Qc = lambda g: np.stack([O.conserve_Q(O.collide_fast64(c, op), n, T) for c in g])   # noqa: E731
    ref = f + dt * Qc(f + 0.5 * dt * Qc(f))
    with fks.Plan(fks.Desc(n=n, T=T, precision=prec)) as plan:
        fd = _dev(f)
        mid = torch.empty_like(fd)
        fks.collide(plan, fd, f_out=mid, dt_over_tau=0.5 * dt)
        fks.collide(plan, mid, f_out=fd, dt_over_tau=dt, f_base=fd)        # f_out aliases f_base
        torch.cuda.synchronize()
        got = fd.cpu().numpy()
        q = torch.empty_like(fd)
        with pytest.raises(fks.FksError) as e:
            fks.collide(plan, mid, q_out=q, f_out=fd, dt_over_tau=dt, f_base=q)   # f_base overlaps q_out
        assert e.value.status == fks.FKS_ERR_INVALID
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.parametrize("scheme,collision", [("strang", "euler"), ("lie", "rk2"), ("strang", "rk2"),
                                              ("lie", "exp"), ("strang", "exp")])
def test_split_step_variants_match_oracle(scheme, collision):
    n, T, nx, tau, steps = 16, 8.0, 8, 1e-2, 3
    f0, bc = _sod_initial(n, T, nx)
    plan = fks.Plan(fks.Desc(n=n, T=T, precision=fks.PREC_F64))
    space = Space(nx, 1, 1, 1.0 / nx, (fks.BC_DIRICHLET, fks.BC_PERIODIC, fks.BC_PERIODIC))
    dt = stable_dt(space, T, tau, plan.info.R, 1.0, plan.info.c_gamma, 1.0)
    mu = 4.0 * math.pi * plan.info.c_gamma * 2.0 * plan.info.R     # loss-frequency bound at rho = 1
    if collision == "exp":
        dt *= 20.0                                                  # past the Euler limit tau / mu
    st = SplitStepper(plan, space, _dev(f0.reshape(1, 1, nx, n, n, n)), bc_f=_dev(bc),
                      scheme=scheme, collision=collision, mu=mu)
    for _ in range(steps):
        st.step(dt, tau)
    torch.cuda.synchronize()
    got = st.f.cpu().numpy().reshape(nx, n, n, n)
    op = O.make_plan(n, T)
    Qc = lambda c: O.conserve_Q(O.collide_fast64(c, op), n, T)   # noqa: E731
    g = f0.reshape(1, 1, nx, n, n, n)
    off = np.zeros((3, n))

    def transport(g, h):
        nonlocal off
        off, s = O.transport_offsets_step(off, n, T, space.dx, h)
        return O.transport_shift(g, s, n, bc=("dirichlet", "periodic", "periodic"), bc_f=bc)

    def collide(g):
        out = []
        for c in g.reshape(nx, n, n, n):
            if collision == "euler":
                out.append(c + dt / tau * Qc(c))
            elif collision == "exp":
                out.append(O.exp_euler_update(c, Qc(c), dt / tau, mu))
            else:
                out.append(c + dt / tau * Qc(c + 0.5 * dt / tau * Qc(c)))
        return np.stack(out).reshape(g.shape)

    for _ in range(steps):
        if scheme == "lie":
            g = collide(transport(g, dt))
        else:
            g = transport(collide(transport(g, 0.5 * dt)), 0.5 * dt)
    assert np.array_equal(st.offsets, off)
    assert _rel(got, g.reshape(nx, n, n, n)) <= 1e-12
    plan.close()
