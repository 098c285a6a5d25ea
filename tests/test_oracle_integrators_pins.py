"""Pins of the collision-step integrators of the oracle: the exponential Euler step for stiff
collisions agrees with the Euler step to second order in h = dt/tau, and with mu at the
loss frequency it keeps f non-negative for steps far beyond the Euler stability limit, where
the Euler step does not (the property the stiff integrators are for)."""
import numpy as np

import oracle as O
import synth


def _cell_and_operator():
    n, T = 16, 8.0
    p = O.make_plan(n, T, n_polar=4, n_azim=4)
    f = synth.two_maxwellian_cells(n, T, 1, seed_offset=77)[0]
    Qc = O.conserve_Q(O.collide_fast64(f, p), n, T)
    nu = O.synthesize(p.loss * O.spectrum(f, n, T), n, T).real   # loss frequency F^{-1}(L fhat)
    return f, Qc, float(np.max(nu))


def test_exp_euler_is_second_order_close_to_euler():
    f, Qc, mu = _cell_and_operator()
    d = {}
    for h in (1e-2, 5e-3):
        d[h] = np.max(np.abs(O.exp_euler_update(f, Qc, h, mu) - O.euler_update(f, Qc, h)))
    assert 3.6 < d[1e-2] / d[5e-3] < 4.4          # the difference is O(h^2)
    assert d[1e-2] <= 0.5 * mu * 1e-4 * np.max(np.abs(Qc)) * 1.01


def test_exp_euler_stays_non_negative_where_euler_does_not():
    f, Qc, mu = _cell_and_operator()
    h = 50.0 / mu                                 # 50 times the Euler stability limit
    g = O.exp_euler_update(f, Qc, h, mu)
    e = O.euler_update(f, Qc, h)
    assert np.min(g) >= -1e-5 * np.max(f)         # spectral Q+ dips below zero at round-off level
    assert np.min(e) <= -0.1 * np.max(f)
    # mass, momentum and energy are those of f in both (Q_c is projected)
    n, T = 16, 8.0
    assert np.allclose(O.moments(g, n, T), O.moments(f, n, T), rtol=1e-12, atol=1e-14)
