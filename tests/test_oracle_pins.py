"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: adaptive
quadrature of an integral definition, a closed form, a physical invariant,
an exact solution, or a LAPACK routine.  The comment on each names the
passage of the paper it follows and the plausible mistake it catches.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle as O
import synth


# -- eqs. FU, FC: the normalisation and phase of the spectrum against a closed form --

def _gaussian_coefficients(n, T, theta, u):
    """Fourier coefficients of eq. FC on [-T, T)^3 for the drifting Maxwellian of
    temperature theta, sampled at the nodes: per axis (1/2T) sum_m exp(-theta xi^2/2 - i xi u)
    with xi = kappa (k + m n) (the continuous transform of the Gaussian plus its aliases, by
    the Poisson summation formula; the tails beyond the box are below 1e-25 here)."""
    kappa = math.pi / T
    k = np.fft.fftfreq(n, d=1.0 / n).round()
    out = []
    for a in range(3):
        s = np.zeros(n, dtype=np.complex128)
        for m in range(-4, 5):
            xi = kappa * (k + m * n)
            s += np.exp(-theta * xi * xi / 2 - 1j * xi * u[a])
        out.append(s / (2 * T))
    return out[0][:, None, None] * out[1][None, :, None] * out[2][None, None, :]


@pytest.mark.parametrize("n", [16, 32])
def test_spectrum_matches_closed_form(n):
    # eq. FC on the node grid: fhat_k = n^-3 sum_j f_j exp(-i kappa k.v_j).  For a centred
    # Maxwellian (theta = 1, T = 8) the coefficients are real and positive,
    # (2T)^-3 exp(-kappa^2 |k|^2 / 2) plus aliases; a drift u multiplies them by
    # exp(-i kappa k.u).  Catches a dropped (-1)^k phase of the nodes v_0 = -T, a missing n^-3,
    # a conjugated exponent (the sign of the drift phase) and a transposed axis (u differs
    # per axis)
    T = 8.0
    for u in ((0.0, 0.0, 0.0), (0.7, -0.4, 0.25)):
        # the periodic extension of the Maxwellian (images shifted by 2T): the closed form is then
        # exact up to rounding, without the 1e-12 tail that leaves the box
        f = sum(synth.maxwellian(n, T, 1.0, (u[0] + 2 * T * a, u[1] + 2 * T * b, u[2] + 2 * T * c), 1.0)
                for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1))
        got = O.spectrum(f, n, T, zero_nyquist=False)
        ref = _gaussian_coefficients(n, T, 1.0, u)
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
        if u == (0.0, 0.0, 0.0):
            assert np.all(ref.real > 0) and np.max(np.abs(got.imag)) <= 1e-16
    # Nyquist zeroing removes exactly the modes with a component -n/2
    got = O.spectrum(f, n, T)
    h = n // 2
    mask = np.ones((n, n, n), bool)
    mask[h], mask[:, h], mask[:, :, h] = False, False, False
    assert np.all(got[~mask] == 0) and np.max(np.abs(got[mask] - ref[mask])) <= 1e-13 * np.max(np.abs(ref))


def test_synthesize_matches_plane_waves():
    # eq. FU on the grid: a single coefficient at k0 synthesises exp(i kappa k0.v_j); catches a
    # sign of the exponent, a missing n^3 and an axis order different from [x][y][z]
    n, T = 8, 3.0
    v = O.velocity_grid(n, T)
    kappa = math.pi / T
    for k0 in ((1, 0, 0), (0, 2, -3), (-1, 3, 1)):
        gh = np.zeros((n, n, n), dtype=np.complex128)
        gh[k0[0] % n, k0[1] % n, k0[2] % n] = 1.0
        got = O.synthesize(gh, n, T)
        ref = np.exp(1j * kappa * (k0[0] * v[:, None, None] + k0[1] * v[None, :, None]
                                   + k0[2] * v[None, None, :]))
        assert np.max(np.abs(got - ref)) <= 1e-14


# -- P1: radial functions against their integral definitions (Section 3.3) --

@pytest.mark.parametrize("R", [1.3, 3.6247])
def test_hs_phi_matches_integral(R):
    # phi(s) = int_{-R}^{R} |rho| exp(i rho s) d rho; catches a signed rho or a lost factor 2
    for s in [0.0, 0.37, 1.0, 2.9, 7.5, 11.0]:
        ref, _ = integrate.quad(lambda r: 2 * r * math.cos(r * s), 0, R, limit=200, epsabs=1e-14)
        assert abs(O.hs_phi(s, R) - ref) <= 1e-12 * R * R


@pytest.mark.parametrize("R", [1.3, 3.6247])
def test_hs_psi_matches_great_circle_integral(R):
    # psi(s) = int_0^pi phi(s cos t) dt (great circle orthogonal to e, no sin t);
    # catches the sin t weighted variant, which gives 2 R^2 Sinc^2(Rs/2) instead
    for s in [0.0, 0.21, 1.0, 3.3, 9.0]:
        ref, _ = integrate.quad(lambda t: O.hs_phi(s * math.cos(t), R), 0, math.pi,
                                limit=200, epsabs=1e-13)
        assert abs(O.hs_psi(s, R) - ref) <= 1e-11 * R * R
    s = 1.7
    literal = 2 * R * R * np.sinc(R * s / 2 / math.pi) ** 2
    assert abs(O.hs_psi(s, R) - literal) > 1e-2 * R * R


def test_radial_expansion_reduces_to_closed_forms_for_hard_spheres():
    # the K-term machinery at gamma = 1 must be rank one and reproduce phi, psi
    R = 3.0
    rt = O.radial_terms(1.0, R, force_expansion=True)
    assert rt.K == 1
    s = np.linspace(0, 12, 61)
    sgn = np.sign(rt.coef[0, 0])
    assert np.max(np.abs(sgn * rt.phi(s)[:, 0] - O.hs_phi(s, R))) < 1e-12 * R * R
    assert np.max(np.abs(sgn * rt.psi(s)[:, 0] - O.hs_psi(s, R))) < 1e-12 * R * R


@pytest.mark.parametrize("gamma", [0.0, 0.5])
def test_radial_expansion_reproduces_kernel_double_integral(gamma):
    # sum_r phi_r(s) psi_r(s') against a direct double integral of the VHS radial kernel:
    # int_0^R int_0^R rho rho' k(rho,rho') 2cos(rho s) 2pi J0(rho' s') (eq. Btilde, decoupling)
    R = 2.5
    rt = O.radial_terms(gamma, R, K=24)
    for s, sp in [(0.0, 0.0), (0.8, 1.9), (2.5, 0.4)]:
        got = float(np.sum(rt.phi(s) * rt.psi(sp)))

        def integrand(rp, r):
            return (r * rp * (r * r + rp * rp) ** ((gamma - 1) / 2)
                    * 2 * math.cos(r * s) * 2 * math.pi * special.j0(rp * sp))
        ref, _ = integrate.dblquad(integrand, 0, R, 0, R, epsabs=1e-10, epsrel=1e-10)
        assert abs(got - ref) <= 1e-7 * abs(O.radial_terms(gamma, R, K=1).phi(0)[0] * 2 * math.pi * R * R)


def test_expansion_truncation_counts():
    # tolerance-driven K grows as gamma moves away from 1 (non-decoupled kernel)
    R = 3.0
    k0 = O.radial_terms(0.0, R, tol=1e-4).K
    k5 = O.radial_terms(0.5, R, tol=1e-4).K
    assert 1 < k5 < k0 < 20


# -- half-sphere rule (Section 3.3, spherical parametrisation) --

@pytest.mark.parametrize("rule,npol,naz,tol", [("gauss", 8, 4, 1e-14), ("midpoint", 64, 8, 2e-3)])
def test_sphere_rule_integrates_polynomials(rule, npol, naz, tol):
    e, w = O.sphere_rule(npol, naz, rule)
    assert abs(w.sum() - 2 * math.pi) < tol * 2 * math.pi
    assert np.allclose(np.linalg.norm(e, axis=1), 1.0, atol=1e-15)
    # exact half-sphere moments of even polynomials
    assert abs(np.sum(w * e[:, 2] ** 2) - 2 * math.pi / 3) < tol * 10
    assert abs(np.sum(w * e[:, 0] ** 2) - 2 * math.pi / 3) < tol * 10
    assert abs(np.sum(w * e[:, 0] ** 2 * e[:, 2] ** 2) - 2 * math.pi / 15) < tol * 10
    assert abs(np.sum(w * e[:, 2] ** 4) - 2 * math.pi / 5) < tol * 10


# -- P2: B_F(0,0) closed form of eq. FKM --

@pytest.mark.parametrize("gamma", [1.0, 0.5])
def test_BF00_closed_form(gamma):
    # B_F(0,0) = 4C * (int_{S2} int_{S2} delta(e.e') de de' = 8 pi^2) * int int rho rho' k;
    # hard spheres: 4C 2 pi^2 R^4.  Catches the weight pi^2/(A1 A2) without Jacobian,
    # a wrong 2^{d-1} or the sin t psi (0.637x).
    p = O.make_plan(4, 4.0, gamma=gamma, K=12 if gamma != 1 else 0)
    bf00 = float(np.sum(p.omega * p.alpha[:, 0, 0, 0] * p.beta[:, 0, 0, 0]))
    R, C = p.R, p.c_gamma
    if gamma == 1.0:
        ref = 4 * C * 2 * math.pi ** 2 * R ** 4
    else:
        I, _ = integrate.dblquad(lambda rp, r: r * rp * (r * r + rp * rp) ** ((gamma - 1) / 2),
                                 0, R, 0, R, epsabs=1e-12, epsrel=1e-12)
        ref = 4 * C * 8 * math.pi ** 2 * I
    assert abs(bf00 - ref) < 1e-9 * ref


# -- P3/P4: direct O(n^2) quadrature equals the fast form; mass is exact --

@pytest.mark.parametrize("n,gamma", [(4, 1.0), (6, 1.0), (8, 1.0), (6, 0.0), (8, 0.5)])
def test_direct_equals_fast(n, gamma):
    # eq. ode summed pair by pair vs the FFT convolution form; catches a transposed
    # (l, m), a wrong loss index, a lost Nyquist zeroing or a sign of the phase
    p = O.make_plan(n, 4.0, gamma=gamma, n_polar=4, n_azim=3, K=3 if gamma != 1 else 0)
    f = synth.random_positive_cells(n, 1, seed_offset=11 + n)[0]
    Qd = O.collide_direct(f, p)
    Qf, G, L = O.collide_fast64(f, p, parts=True)
    scale = np.max(np.abs(G))
    assert np.max(np.abs(Qd - Qf)) < 1e-14 * scale
    # mass (eq. i5 with phi = 1): exact for the discrete operator
    assert abs(Qf.sum()) < 1e-14 * np.abs(G).sum()


def test_nyquist_zeroing_matters():
    # without zeroing the -n/2 planes mass is lost on rough data (reading of eq. FU)
    n = 6
    p = O.make_plan(n, 4.0, n_polar=4, n_azim=3)
    f = synth.random_positive_cells(n, 1, seed_offset=3)[0]
    fh = O.spectrum(f, n, p.T, zero_nyquist=False)
    a = O.synthesize(p.alpha * fh, n, p.T).real
    b = O.synthesize(p.beta * fh, n, p.T).real
    gain = np.einsum("j,jxyz->xyz", p.omega, a * b)
    loss = O.synthesize(fh, n, p.T).real * O.synthesize(p.loss * fh, n, p.T).real
    assert abs((gain - loss).sum()) > 1e-6 * np.abs(gain).sum()


# -- P5: loss frequency against the exact truncated Carleman measure --

def _loss_frequency_exact(R, C, gamma):
    # Q-(v)/f(v) at v = 0 for a unit Maxwellian: 4 pi C int |z|^gamma clip(2R^2/|z|^2 - 1, 0, 1) M(z) dz
    # (the set {x + y = z, x.y = 0, |x|,|y| <= R} is a Thales sphere of area pi |z|^2 clip(...))
    def g(z):
        return (4 * math.pi * C * z ** gamma * min(max(2 * R * R / (z * z) - 1, 0.0), 1.0)
                * math.exp(-z * z / 2) / (2 * math.pi) ** 1.5 * 4 * math.pi * z * z)
    val, _ = integrate.quad(g, 0, math.sqrt(2) * R, points=[R], limit=400, epsabs=1e-14)
    return val


def test_hard_sphere_loss_frequency():
    n, T = 32, 8.0
    p = O.make_plan(n, T)
    f = synth.maxwellian(n, T, 1.0, (0, 0, 0), 1.0)
    Q, G, L = O.collide_fast64(f, p, parts=True)
    h = n // 2
    nu = L[h, h, h] / f[h, h, h]
    ref = _loss_frequency_exact(p.R, p.c_gamma, 1.0)
    assert abs(nu - ref) < 1e-8 * ref
    # and the sin t psi reading misses it by tens of percent
    assert 1.5 < ref < 1.7


def test_maxwell_loss_frequency_is_density():
    # gamma = 0: untruncated Q- = 4 pi C rho f = rho f (the paper's Maxwell stability bound);
    # truncation only removes the far tail of the Maxwellian
    n, T = 24, 8.0
    p = O.make_plan(n, T, gamma=0.0, K=12)
    f = synth.maxwellian(n, T, 1.0, (0, 0, 0), 1.0)
    _, _, L = O.collide_fast64(f, p, parts=True)
    h = n // 2
    nu = L[h, h, h] / f[h, h, h]
    ref = _loss_frequency_exact(p.R, p.c_gamma, 0.0)
    assert abs(nu - ref) < 1e-4 * ref
    assert abs(ref - 1.0) < 0.05


# -- P6: Q(M) = 0 for Maxwellians (eq. i6), spectrally in n --

def test_maxwellian_is_equilibrium():
    T = 8.0
    errs = []
    for n in (16, 32):
        p = O.make_plan(n, T)
        f = synth.maxwellian(n, T, 1.3, (0.4, -0.2, 0.1), 1.1)
        Q, G, L = O.collide_fast64(f, p, parts=True)
        errs.append(np.max(np.abs(Q)) / np.max(np.abs(G)))
    assert errs[1] < 1e-7
    assert errs[1] < 1e-2 * errs[0]


# -- P7: 3D BKW for Maxwell molecules: Q(f_BKW) = (1-K)/6 dK f_BKW --

@pytest.mark.slow
def test_bkw_rate_maxwell_molecules():
    n, T, t = 32, 8.0, 5.5
    p = O.make_plan(n, T, gamma=0.0, n_polar=8, n_azim=4, K=10)
    f = synth.bkw3d(n, T, t)
    Q = O.collide_fast64(f, p)
    K = 1 - math.exp(-t / 6)
    v = O.velocity_grid(n, T)
    v2 = v[:, None, None] ** 2 + v[None, :, None] ** 2 + v[None, None, :] ** 2
    h = 1e-6
    dK = (synth.bkw3d_K(v2, K + h) - synth.bkw3d_K(v2, K - h)) / (2 * h)
    g = (1 - K) * dK
    rate = float(np.sum(Q * g) / np.sum(g * g))
    assert abs(rate - 1 / 6) < 1e-3
    assert O.relative_l2(Q, g / 6) < 2e-2


# -- P8: the conservation projection (Section 3.2, eq. minim1) --

def test_projection_is_min_norm_correction():
    n, T = 6, 4.0
    rng = synth.rng(5)
    Q = rng.normal(size=(3, n, n, n))
    Qc = O.conserve_Q(Q, n, T)
    Phi = O.collision_basis(n, T)
    for c in range(3):
        # L2-minimal change subject to C Q_c = 0 (LAPACK min-norm least squares)
        delta, *_ = np.linalg.lstsq(Phi, Phi @ Q[c].ravel(), rcond=None)
        assert np.allclose(Qc[c].ravel(), Q[c].ravel() - delta, atol=1e-13, rtol=0)
        assert np.max(np.abs(Phi @ Qc[c].ravel())) < 1e-12 * np.abs(Phi).max() * np.abs(Q).max()
    assert np.allclose(O.conserve_Q(Qc, n, T), Qc, atol=1e-14)


def test_project_hits_target_moments():
    n, T = 8, 6.0
    f = synth.maxwellian(n, T, 1.0, (0.1, 0.2, -0.3), 0.9)
    U = np.array([1.0, 0.1, 0.2, -0.3, 0.14 + 3 * 0.9])
    g = O.project(f, U, n, T)
    assert np.allclose(O.moments(g, n, T), U, atol=1e-13, rtol=0)


def test_moments_of_maxwellian():
    n, T = 32, 8.0
    rho, u, th = 1.4, np.array([0.3, -0.5, 0.2]), 1.2
    f = synth.maxwellian(n, T, rho, u, th)
    U = O.moments(f, n, T)
    assert abs(U[0] - rho) < 1e-10
    assert np.allclose(U[1:4], rho * u, atol=1e-10)
    assert abs(U[4] - rho * (u @ u + 3 * th)) < 1e-9
    r, uu, tt = O.primitive(U)
    assert abs(tt - th) < 1e-9


# -- P10: FKS transport (Section 3.1 eq. f_bar; Section 4.1) --

def test_transport_periodic_round_trip_and_mass():
    n, T = 4, 2.0
    nx, ny, nz = 5, 3, 2
    dx = 1.0 / nx
    dt = 0.9 * dx / T
    rng = synth.rng(9)
    f0 = rng.uniform(size=(nz, ny, nx, n, n, n))
    f = f0.copy()
    off = np.zeros((3, n))
    shifts = []
    for _ in range(7):
        off, s = O.transport_offsets_step(off, n, T, dx, dt)
        assert np.all(np.abs(s) <= 1)            # CFL <= 1 moves at most one cell
        shifts.append(s)
        f = O.transport_shift(f, s, n)
    assert abs(f.sum() - f0.sum()) < 1e-12 * f0.sum()
    # exact solution: cumulative shift d(s) applied to the initial data
    d = np.floor(off / dx + 0.5).astype(int)
    assert np.array_equal(O.transport_shift(f0, d, n), f)
    for s in reversed(shifts):
        f = O.transport_shift(f, -s, n)
    assert np.array_equal(f, f0)


def test_transport_dirichlet_inflow():
    n = 2
    nx = 4
    f = np.arange(nx * n ** 3, dtype=float).reshape(1, 1, nx, n, n, n)
    bc = np.full((6, n, n, n), -1.0)
    bc[0] = 100.0
    bc[1] = 200.0
    shift = np.zeros((3, n), dtype=int)
    shift[0] = [-1, 1]                            # kx=0 moves left, kx=1 moves right
    g = O.transport_shift(f, shift, n, bc=("dirichlet", "periodic", "periodic"), bc_f=bc)
    assert np.all(g[0, 0, 0, 1] == 100.0)         # right-movers enter from x-low
    assert np.all(g[0, 0, nx - 1, 0] == 200.0)    # left-movers enter from x-high
    assert np.array_equal(g[0, 0, 1:, 1], f[0, 0, :-1, 1])
    assert np.array_equal(g[0, 0, :-1, 0], f[0, 0, 1:, 0])
