"""Pins of the BGK oracle (Section 2 eq. ibgk with the conservative discrete
Maxwellian of Section 3.2 eq. minimMax) against the properties the paper
states and against Test 1.2's printed observation."""
import math

import numpy as np
import pytest

import oracle.fks_oracle as O3
import oracle.fks_oracle2d as O2
import oracle.fks_oracle_bgk as B
import synth


@pytest.mark.parametrize("dim,n,T", [(2, 16, 6.0), (2, 24, 8.0), (3, 12, 6.0)])
def test_discrete_maxwellian_has_the_cell_moments(dim, n, T):
    # C E[U] = U exactly (eq. minimMax); catches a wrong temperature relation or projection
    if dim == 2:
        f = synth.two_maxwellian_cells_2d(n, T, 1, seed_offset=5)[0]
    else:
        f = synth.two_maxwellian_cells(n, T, 1, seed_offset=5)[0]
    U = B.bgk_moments(f, n, T, dim)
    E = B.bgk_equilibrium(f, n, T, dim)
    assert np.allclose(B.bgk_moments(E, n, T, dim), U, rtol=0, atol=1e-14 * np.abs(U).max())
    Q = B.bgk_Q(f, n, T, dim, nu=1.3)
    assert np.all(np.abs(B.bgk_moments(Q, n, T, dim)) <= 1e-14 * np.abs(U).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_resolved_maxwellian_is_a_fixed_point(dim):
    # for a well-resolved Maxwellian the pointwise Maxwellian of its moments is itself:
    # Q_BGK(M) = 0 to quadrature accuracy; catches a theta off by the factor d or 2
    n, T = (48, 10.0) if dim == 2 else (24, 8.0)
    if dim == 2:
        M = synth.maxwellian2(n, T, 1.2, (0.3, -0.2), 0.8)
    else:
        M = synth.maxwellian(n, T, 1.2, (0.3, -0.2, 0.1), 0.8)
    E = B.bgk_equilibrium(M, n, T, dim)
    assert np.max(np.abs(E - M)) <= 1e-12 * np.max(M)
    rho, u, theta = B.bgk_primitive(B.bgk_moments(M, n, T, dim), dim)
    assert abs(rho - 1.2) < 1e-12 and abs(theta - 0.8) < 1e-12


def test_exact_step_is_the_limit_of_small_euler_steps():
    # d f/dt = nu (E - f) with E fixed: many Euler steps converge to E + exp(-nu t)(f - E)
    n, T = 16, 6.0
    f = synth.two_maxwellian_cells_2d(n, T, 1, seed_offset=9)[0]
    ex = B.bgk_step(f, n, T, 2, nu=2.0, dt_over_tau=0.3, exact=True)
    g = f.copy()
    for _ in range(3000):
        g = B.bgk_step(g, n, T, 2, nu=2.0, dt_over_tau=0.3 / 3000)
    assert np.max(np.abs(g - ex)) <= 2e-4 * np.max(np.abs(f - ex))


def test_entropy_decreases_along_bgk_relaxation():
    # H = sum f log f decreases while f relaxes (positive data, small steps)
    n, T = 24, 8.0
    f = synth.two_maxwellian_cells_2d(n, T, 1, seed_offset=11)[0] + 1e-12
    H = [float(np.sum(f * np.log(f)))]
    for _ in range(20):
        f = B.bgk_step(f, n, T, 2, nu=1.0, dt_over_tau=0.05)
        f = np.maximum(f, 1e-300)
        H.append(float(np.sum(f * np.log(f))))
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(H, H[1:]))


def test_bgk_boltzmann_difference_peaks_where_test_1_2_says():
    # Test 1.2 (Section 5.1): BKW data, 2D Maxwell molecules, 32^2 on [-9, 9]^2; the L1
    # difference between the BGK (nu = rho) and Boltzmann solutions peaks near t = 1.66
    n, T, A, dt = 32, 9.0, 8, 0.02
    p = O2.make_plan2(n, T, A)
    fb = O2.bkw2d_initial(n, T)
    fB = fb.copy()
    best_t, best = 0.0, 0.0
    for s in range(1, 201):
        fb = B.bgk_step(fb, n, T, 2, nu=1.0, dt_over_tau=dt, nu_rho=True)
        fB = fB + dt * O2.conserve2_Q(O2.collide2_fast64(fB, p), n, T)
        d = np.sum(np.abs(fb - fB)) / np.sum(np.abs(fB))
        if d > best:
            best, best_t = d, s * dt
    assert abs(best_t - 1.66) <= 0.15, best_t
