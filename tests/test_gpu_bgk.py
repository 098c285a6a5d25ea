"""BGK relaxation with the conservative discrete Maxwellian (fks_bgk) on the GPU
against the oracle: both dimensions, both steps, nu = const and nu = rho,
in-place updates, a ragged batch, and Test 1.2's BGK/Boltzmann comparison."""
import numpy as np
import pytest

import oracle.fks_oracle2d as O2
import oracle.fks_oracle_bgk as B
import synth

torch = pytest.importorskip("torch")
import paper_1608_08009_amd as fks  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _cells(dim, n, T, ncell, seed):
    if dim == 2:
        return synth.two_maxwellian_cells_2d(n, T, ncell, seed_offset=seed)
    return synth.two_maxwellian_cells(n, T, ncell, seed_offset=seed)


@pytest.mark.parametrize("dim,n,T,ncell", [(3, 8, 6.0, 5), (3, 12, 6.0, 4), (3, 32, 8.0, 6), (3, 48, 10.0, 2),
                                           (2, 16, 6.0, 9), (2, 64, 10.0, 5), (2, 100, 12.0, 3)])
@pytest.mark.parametrize("nu_rho", [False, True])
def test_bgk_q_matches_oracle(dim, n, T, ncell, nu_rho):
    f = _cells(dim, n, T, ncell, 60 + n)
    nu = 0.7
    ref = np.stack([B.bgk_Q(c, n, T, dim, nu, nu_rho) for c in f])
    fd = _dev(f)
    q = torch.empty_like(fd)
    fks.bgk(fd, n, T, nu, dim=dim, q_out=q, nu_rho=nu_rho)
    torch.cuda.synchronize()
    got = q.cpu().numpy()
    for c in range(ncell):
        scale = nu * np.max(np.abs(f[c]))
        assert np.max(np.abs(got[c] - ref[c])) <= 1e-12 * scale
        U = B.bgk_moments(got[c], n, T, dim)
        assert np.all(np.abs(U) <= 1e-13 * nu * np.abs(B.bgk_moments(f[c], n, T, dim)).max())


@pytest.mark.parametrize("dim,n,T", [(2, 24, 8.0), (3, 16, 6.0)])
@pytest.mark.parametrize("step", [fks.BGK_EULER, fks.BGK_EXACT])
def test_bgk_update_in_place(dim, n, T, step):
    ncell, nu, dt = 7, 1.5, 0.4
    f = _cells(dim, n, T, ncell, 80)
    ref = np.stack([B.bgk_step(c, n, T, dim, nu, dt, nu_rho=True, exact=(step == fks.BGK_EXACT)) for c in f])
    fd = _dev(f)
    out = torch.empty_like(fd)
    fks.bgk(fd, n, T, nu, dim=dim, f_out=out, dt_over_tau=dt, nu_rho=True, step=step)
    fks.bgk(fd, n, T, nu, dim=dim, f_out=fd, dt_over_tau=dt, nu_rho=True, step=step)
    torch.cuda.synchronize()
    for g in (out, fd):
        assert np.max(np.abs(g.cpu().numpy() - ref)) <= 1e-13 * np.max(np.abs(f))


def test_bgk_leaves_a_cell_without_maxwellian_unchanged():
    n, T = 8, 6.0
    f = _cells(3, n, T, 2, 81)
    f[1] = -f[1]                       # negative density: no Maxwellian
    fd = _dev(f)
    q = torch.empty_like(fd)
    fks.bgk(fd, n, T, 1.0, dim=3, q_out=q)
    torch.cuda.synchronize()
    got = q.cpu().numpy()
    assert np.all(got[1] == 0.0)
    assert np.max(np.abs(got[0] - B.bgk_Q(f[0], n, T, 3, 1.0))) <= 1e-12 * np.max(f[0])


def test_bgk_invalid_arguments():
    fd = _dev(_cells(3, 8, 6.0, 2, 82))
    with pytest.raises(fks.FksError) as e:
        fks.bgk(fd, 8, 6.0, 1.0, dim=3)                     # no output
    assert e.value.status == fks.FKS_ERR_INVALID
    with pytest.raises(fks.FksError):
        fks.bgk(fd, 8, 6.0, 1.0, dim=3, q_out=fd)           # q_out overlaps f


def test_test12_bgk_boltzmann_comparison_on_gpu():
    # Test 1.2 (Section 5.1): BKW data, 2D Maxwell molecules on 32^2, [-9, 9]^2, nu = rho;
    # both models on the GPU against the oracle; the L1 difference peaks near t = 1.66
    n, T, A, dt, steps = 32, 9.0, 8, 0.02, 120
    f0 = O2.bkw2d_initial(n, T)
    p = O2.make_plan2(n, T, A)
    with fks.Plan(fks.desc2d(n, T, A, fks.PREC_F64)) as plan:
        fb, fB = _dev(f0[None]), _dev(f0[None])
        gb, gB = f0.copy(), f0.copy()
        diff = []
        for s in range(steps):
            fks.bgk(fb, n, T, 1.0, dim=2, f_out=fb, dt_over_tau=dt, nu_rho=True)
            fks.collide(plan, fB, f_out=fB, dt_over_tau=dt)
            gb = B.bgk_step(gb, n, T, 2, 1.0, dt, nu_rho=True)
            gB = gB + dt * O2.conserve2_Q(O2.collide2_fast64(gB, p), n, T)
            a, b = fb[0].cpu().numpy(), fB[0].cpu().numpy()
            diff.append(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))
        assert np.max(np.abs(a - gb)) <= 1e-11 * np.max(gb)
        assert np.max(np.abs(b - gB)) <= 1e-11 * np.max(gB)
    t_peak = (int(np.argmax(diff)) + 1) * dt
    assert abs(t_peak - 1.66) <= 0.15, t_peak
