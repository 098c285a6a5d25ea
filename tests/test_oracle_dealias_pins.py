"""Pins of the de-aliased (zero-padded) fast operator oracle against facts that do not
depend on it: its definition as a non-wrapped double sum, the coincidence with the
aliased operator for data whose products cannot wrap, independence of the padded grid
size once it is alias-free, exact mass, and a Maxwellian equilibrium."""
import math

import numpy as np
import pytest

import oracle as O
import oracle.fks_oracle_dealias as D


def _rough(n, seed):
    return np.random.default_rng(seed).uniform(0.1, 1.0, size=(n, n, n))


def _band_limited(n, T, kmax, seed):
    """Real f whose spectrum is supported in |k_i| <= kmax (random Hermitian coefficients)."""
    rng = np.random.default_rng(seed)
    k = O.wavenumbers(n)
    sel = np.abs(k) <= kmax
    gh = np.zeros((n, n, n), dtype=np.complex128)
    blk = rng.normal(size=(sel.sum(),) * 3) + 1j * rng.normal(size=(sel.sum(),) * 3)
    gh[np.ix_(sel, sel, sel)] = blk
    # Hermitian part: ghat(-k) = conj ghat(k)
    neg = (-np.arange(n)) % n
    gh = 0.5 * (gh + np.conj(gh[np.ix_(neg, neg, neg)]))
    gh[0, 0, 0] = 2.0 + 0j
    return O.synthesize(gh, n, T).real


@pytest.mark.parametrize("n,gamma,K", [(4, 1.0, 0), (6, 1.0, 0), (8, 1.0, 0), (8, 0.5, 3)])
def test_fast_equals_non_wrapped_double_sum(n, gamma, K):
    # the definition (l + m = k exactly, k in the band) against the zero-padded fast form;
    # catches a padding that still wraps, a wrong index map or a truncation off by one
    p = O.make_plan(n, 6.0, gamma=gamma, n_polar=4, n_azim=3, K=K)
    f = _rough(n, 300 + n)
    fast = D.collide_dealias_fast64(f, p)
    direct = D.collide_dealias_direct(f, p)
    assert np.max(np.abs(fast - direct)) <= 1e-13 * np.max(np.abs(direct))
    # and it is a different operator from the wrapped one on rough data
    wrapped = O.collide_direct(f, p)
    assert np.max(np.abs(direct - wrapped)) >= 1e-3 * np.max(np.abs(direct))


@pytest.mark.parametrize("n", [8, 12])
def test_equals_aliased_operator_when_no_product_can_wrap(n):
    # spectrum in |k_i| <= n/4 - 1: every l + m stays inside the band, so both operators
    # take exactly the same pairs
    T = 6.0
    p = O.make_plan(n, T, n_polar=4, n_azim=4)
    f = _band_limited(n, T, n // 4 - 1, seed=n)
    a = O.collide_fast64(f, p)
    d = D.collide_dealias_fast64(f, p)
    assert np.max(np.abs(a - d)) <= 1e-13 * np.max(np.abs(a))


@pytest.mark.parametrize("n", [6, 8])
def test_padded_grid_size_does_not_matter_once_alias_free(n):
    p = O.make_plan(n, 6.0, n_polar=4, n_azim=3)
    f = _rough(n, 40 + n)
    q1 = D.collide_dealias_fast64(f, p, npad=3 * n // 2)
    q2 = D.collide_dealias_fast64(f, p, npad=2 * n)
    q3 = D.collide_dealias_fast64(f, p, npad=3 * n // 2 - 2)    # the smallest alias-free size
    assert np.max(np.abs(q1 - q2)) <= 1e-13 * np.max(np.abs(q1))
    assert np.max(np.abs(q1 - q3)) <= 1e-13 * np.max(np.abs(q1))
    # one point fewer folds frequency n - 2 onto the band edge -(n/2 - 1)
    q4 = D.collide_dealias_fast64(f, p, npad=3 * n // 2 - 3)
    assert np.max(np.abs(q1 - q4)) >= 1e-8 * np.max(np.abs(q1))


def test_mass_exact_band_limited_and_maxwellian_equilibrium():
    n, T = 16, 8.0
    p = O.make_plan(n, T)
    f = _rough(n, 9)
    Q, gh, lh = D.collide_dealias_fast64(f, p, parts=True)
    assert abs(np.sum(Q)) <= 1e-14 * np.sum(np.abs(Q)) * n ** 3
    # nothing outside the band, Nyquist planes included
    full = O.spectrum(Q, n, T, zero_nyquist=False)
    assert np.max(np.abs(full[~D.band_mask(n)])) <= 1e-15 * np.max(np.abs(full))
    # Q(M) vanishes to spectral accuracy: the residual relative to the gain falls fast with n
    # (measured 2.0e-4 at n = 24 and 7.4e-7 at n = 32 on [-10, 10)^3)
    res = {}
    for n in (24, 32):
        T = 10.0
        p = O.make_plan(n, T)
        v = O.velocity_grid(n, T)
        vx, vy, vz = np.meshgrid(v, v, v, indexing="ij")
        M = np.exp(-((vx - 0.3) ** 2 + vy ** 2 + (vz + 0.2) ** 2) / 2.0) / (2 * math.pi) ** 1.5
        Q, gh, lh = D.collide_dealias_fast64(M, p, parts=True)
        res[n] = np.max(np.abs(Q)) / np.max(np.abs(O.synthesize(gh, n, T).real))
    assert res[32] <= 2e-6 and res[32] <= 1e-2 * res[24], res
