"""FP64 CPU oracle of the two-dimensional fast spectral operator for Maxwell
molecules (test infrastructure; only tests, the smoke check and the bench's
CPU-baseline leg may use it, and it shares no code with the HIP library).

Conventions (readings of the paper):

* Velocity grid and Fourier representation as in three dimensions
  (Section 3.1, eqs. FU and FC on [-T, T)^2): nodes v_j = -T + j dv,
  dv = 2T/n, f(v) = sum_k fhat_k exp(i kappa k.v), kappa = pi/T; modes with a
  component equal to -n/2 are zeroed and the filtered f_N is used in the
  loss term.
* Carleman kernel (eq. Btilde with d_v = 2 and the Maxwell kernel of eq.
  defVHSKernel, alpha = 0): B~ = 2 C_0, constant.  C_0 = 1/(2 pi), so that the
  angular integral of B is 1 and the loss term is rho f, as Section 5.2 states
  for two-dimensional Maxwell molecules.
* Decoupled kernel for d_v = 2 (Section 3.3, two-dimensional formula and eq.
  dfor0): B_F(l, m) = B~ * integral over theta in [0, pi) of
  phi(kappa l.e_theta) phi(kappa m.e_{theta + pi/2}), with
  phi(s) = int_{-R}^{R} exp(i rho s) d rho = 2 R Sinc(R s); the integral is
  the A-point rectangle rule on theta_p = pi p / A, p = 1..A (weight pi/A), which
  is spectrally accurate because the integrand is pi-periodic.
* R = 2 T / (3 + sqrt 2) (Section 3.3, the same lambda in every dimension).
* Loss table L(m) = B_F(m, m), built with the same rule as the gain.
* Conservation: the invariants are (1, v_x, v_y, |v|^2) (Section 3.2 with
  d_v = 2); the projection is eq. minim1.

Test 1.1 of the paper (two-dimensional BKW solution) is reproduced by
``test11_errors``; its printed L1 and L2 errors are the pin of this module.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "velocity_grid2", "wavenumbers2", "default_R2", "maxwell2d_phi", "circle_rule",
    "Plan2", "make_plan2", "spectrum2", "synthesize2", "collide2_fast64",
    "collide2_direct", "collision_basis2", "conserve2_Q", "project2", "moments2",
    "bkw2d", "bkw2d_initial", "maxwellian2", "loss_frequency2_exact", "test11_errors",
]


def velocity_grid2(n: int, T: float) -> np.ndarray:
    """Nodes v_j = -T + j * 2T/n on each axis (Section 3.1)."""
    return -T + np.arange(n, dtype=np.float64) * (2.0 * T / n)


def wavenumbers2(n: int) -> np.ndarray:
    """Integer wavenumbers in FFT storage order: 0..n/2-1, -n/2..-1 (eq. FU)."""
    return np.fft.fftfreq(n, d=1.0 / n).round().astype(np.int64)


def default_R2(T: float) -> float:
    """R = lambda T with lambda = 2 / (3 + sqrt 2) (Section 3.3)."""
    return 2.0 * T / (3.0 + math.sqrt(2.0))


def maxwell2d_phi(s, R: float):
    """phi(s) = int_{-R}^{R} exp(i rho s) d rho = 2 R Sinc(R s) (Section 3.3, d_v = 2)."""
    s = np.asarray(s, dtype=np.float64)
    return 2.0 * R * np.sinc(R * s / math.pi)


def circle_rule(A: int):
    """Angles theta_p = pi p / A, p = 1..A, each of weight pi / A (eq. dfor0)."""
    theta = math.pi * np.arange(1, A + 1, dtype=np.float64) / A
    return theta, np.full(A, math.pi / A)


@dataclass
class Plan2:
    n: int
    T: float
    R: float
    A: int
    c0: float
    alpha: np.ndarray = None      # [A][n][n]: phi(kappa k.e_p)
    alphap: np.ndarray = None     # [A][n][n]: phi(kappa k.e_p^perp)
    omega: float = 0.0            # B~ * pi / A
    loss: np.ndarray = None       # [n][n]: L(k) = B_F(k, k)

    @property
    def kappa(self) -> float:
        return math.pi / self.T


def _kgrid2(n: int):
    k = wavenumbers2(n).astype(np.float64)
    return k[:, None] * np.ones((1, n)), k[None, :] * np.ones((n, 1))


def make_plan2(n: int, T: float, A: int = 8, R: float = 0.0, c0: float = 0.0) -> Plan2:
    """Tables of the decoupled two-dimensional kernel (eq. dfor0)."""
    R = R if R > 0 else default_R2(T)
    c0 = c0 if c0 > 0 else 1.0 / (2.0 * math.pi)
    p = Plan2(n=n, T=T, R=R, A=A, c0=c0)
    kx, ky = _kgrid2(n)
    theta, w = circle_rule(A)
    p.alpha = np.empty((A, n, n))
    p.alphap = np.empty((A, n, n))
    for i, t in enumerate(theta):
        c, s = math.cos(t), math.sin(t)
        p.alpha[i] = maxwell2d_phi(p.kappa * (kx * c + ky * s), R)
        p.alphap[i] = maxwell2d_phi(p.kappa * (-kx * s + ky * c), R)
    p.omega = 2.0 * c0 * w[0]
    p.loss = p.omega * np.sum(p.alpha * p.alphap, axis=0)
    return p


def _phase2(n: int, T: float):
    k = wavenumbers2(n).astype(np.float64)
    ph = np.exp(1j * (math.pi / T) * k * (-T))
    return ph[:, None] * ph[None, :]


def spectrum2(f: np.ndarray, n: int, T: float, zero_nyquist: bool = True) -> np.ndarray:
    """fhat_k = n^{-2} sum_j f_j exp(-i kappa k.v_j) (eq. FC), Nyquist modes zeroed."""
    fh = np.fft.fft2(f, axes=(-2, -1)) / float(n) ** 2 * np.conj(_phase2(n, T))
    if zero_nyquist:
        h = n // 2
        fh[..., h, :] = 0.0
        fh[..., :, h] = 0.0
    return fh


def synthesize2(gh: np.ndarray, n: int, T: float) -> np.ndarray:
    """g(v_j) = sum_k ghat_k exp(i kappa k.v_j) (eq. FU); complex result."""
    return np.fft.ifft2(gh * _phase2(n, T), axes=(-2, -1)) * float(n) ** 2


def collide2_fast64(f: np.ndarray, p: Plan2, parts: bool = False, zero_nyquist: bool = True):
    """Fast form Q = sum_p omega a_p b_p - f_N F^{-1}(L fhat), a_p = F^{-1}(alpha_p fhat),
    b_p = F^{-1}(alpha'_p fhat) (Section 3.3, eqs. ode and dfor0), FP64.
    ``zero_nyquist = False`` keeps the -n/2 modes (then Q is the real part)."""
    n, T = p.n, p.T
    fh = spectrum2(f, n, T, zero_nyquist=zero_nyquist)
    fN = synthesize2(fh, n, T).real
    a = synthesize2(p.alpha * fh, n, T).real
    b = synthesize2(p.alphap * fh, n, T).real
    gain = p.omega * np.sum(a * b, axis=0)
    loss = fN * synthesize2(p.loss * fh, n, T).real
    Q = gain - loss
    return (Q, gain, loss) if parts else Q


def collide2_direct(f: np.ndarray, p: Plan2) -> np.ndarray:
    """Direct double sum Qhat_k = sum_{l+m = k mod n} fhat_l fhat_m [B_F(l, m) - B_F(m, m)]
    (eq. ode) with B_F from the same angle rule; O(n^4), small n only."""
    n, T = p.n, p.T
    fh = spectrum2(f, n, T).reshape(-1)
    al = p.alpha.reshape(p.A, -1)
    ap = p.alphap.reshape(p.A, -1)
    BF = p.omega * al.T @ ap                      # [l, m]
    Lm = np.diag(BF).copy()
    k = wavenumbers2(n)
    idx = np.arange(n * n)
    lx, ly = k[idx // n], k[idx % n]
    Qh = np.zeros(n * n, dtype=np.complex128)
    for m in range(n * n):
        kx = (lx + k[m // n]) % n
        ky = (ly + k[m % n]) % n
        dst = kx * n + ky
        np.add.at(Qh, dst, fh * fh[m] * (BF[:, m] - Lm[m]))
    return synthesize2(Qh.reshape(n, n), n, T).real


def collision_basis2(n: int, T: float) -> np.ndarray:
    """Rows (1, v_x, v_y, |v|^2) over the grid (Section 3.2 with d_v = 2)."""
    v = velocity_grid2(n, T)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    return np.stack([np.ones_like(vx), vx, vy, vx * vx + vy * vy]).reshape(4, -1)


def conserve2_Q(Q: np.ndarray, n: int, T: float) -> np.ndarray:
    """Q_c = Q - C^T (C C^T)^{-1} C Q (eq. minim1 with U = C f); cell or batch."""
    Phi = collision_basis2(n, T)
    q = Q.reshape(-1, n * n)
    lam = np.linalg.solve(Phi @ Phi.T, Phi @ q.T)
    return (q - (Phi.T @ lam).T).reshape(Q.shape)


def project2(f: np.ndarray, U: np.ndarray, n: int, T: float) -> np.ndarray:
    """f + C^T (C C^T)^{-1} (U - C f) (eq. minim1); U[..., 4] in moment units."""
    C = (2.0 * T / n) ** 2 * collision_basis2(n, T)
    ff = f.reshape(-1, n * n)
    UU = np.asarray(U, dtype=np.float64).reshape(-1, 4)
    lam = np.linalg.solve(C @ C.T, (UU - ff @ C.T).T)
    return (ff + (C.T @ lam).T).reshape(f.shape)


def moments2(f: np.ndarray, n: int, T: float) -> np.ndarray:
    """U = C f = dv^2 sum_j f_j (1, v_j, |v_j|^2)."""
    Phi = collision_basis2(n, T)
    return (2.0 * T / n) ** 2 * (f.reshape(-1, n * n) @ Phi.T).reshape(f.shape[:-2] + (4,))


def maxwellian2(n: int, T: float, rho: float, u, theta: float) -> np.ndarray:
    """rho / (2 pi theta) exp(-|v - u|^2 / (2 theta)) on the grid (eq. i5 with d_v = 2)."""
    v = velocity_grid2(n, T)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    r2 = (vx - u[0]) ** 2 + (vy - u[1]) ** 2
    return rho / (2.0 * math.pi * theta) * np.exp(-r2 / (2.0 * theta))


def bkw2d(n: int, T: float, t: float, node_offset: float = 0.0) -> np.ndarray:
    """Exact BKW solution of Test 1.1 (eq. Jngb): S = 1 - exp(-t/8)/2,
    f = exp(-v^2/(2S)) [2S - 1 + (1 - S) v^2 / (2S)] / (2 pi S^2), sampled at
    v_j = -T + (j + node_offset) dv (node_offset = 1/2: cell-centred nodes)."""
    v = velocity_grid2(n, T) + node_offset * (2.0 * T / n)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    v2 = vx * vx + vy * vy
    S = 1.0 - 0.5 * math.exp(-t / 8.0)
    return np.exp(-v2 / (2.0 * S)) * (2.0 * S - 1.0 + (1.0 - S) * v2 / (2.0 * S)) / (2.0 * math.pi * S * S)


def bkw2d_initial(n: int, T: float, node_offset: float = 0.0) -> np.ndarray:
    """Initial condition of Test 1.1 (eq. BKW): f(v, 0) = v^2 / pi exp(-v^2), sampled at
    v_j = -T + (j + node_offset) dv."""
    v = velocity_grid2(n, T) + node_offset * (2.0 * T / n)
    vx, vy = np.meshgrid(v, v, indexing="ij")
    v2 = vx * vx + vy * vy
    return v2 / math.pi * np.exp(-v2)


def loss_frequency2_exact(R: float, c0: float = 1.0 / (2.0 * math.pi)) -> float:
    """Loss frequency Q^-(0) / f(0) of the truncated Carleman operator for the unit
    Maxwellian exp(-|z|^2/2)/(2 pi), by one-dimensional quadrature.

    For x + y = z, x orthogonal to y, the pairs lie on the circle of diameter
    |z|; the measure delta(x.y) dx dy over it is d psi / 2, and |x|, |y| <= R
    holds where |cos psi| <= 2R^2/|z|^2 - 1.  Hence the kernel weight is
    B~ * 2 arcsin(clip(2R^2/|z|^2 - 1, 0, 1)) and
    Q^-(0)/f(0) = int_0^inf r exp(-r^2/2) B~ 2 arcsin(c(r)) dr.
    """
    from scipy import integrate
    Bt = 2.0 * c0

    def g(r):
        c = min(1.0, max(0.0, 2.0 * R * R / (r * r) - 1.0)) if r > 0 else 1.0
        return r * math.exp(-0.5 * r * r) * Bt * 2.0 * math.asin(c)

    pts = [R, math.sqrt(2.0) * R]
    val, _ = integrate.quad(g, 0.0, math.sqrt(2.0) * R + 1e-12, points=pts, limit=400,
                            epsabs=1e-15, epsrel=1e-13)
    return val


def test11_errors(n: int, T: float, A: int = 8, dt: float = 0.02, t_final: float = 10.0,
                  conserve: bool = True, R: float = 0.0, node_offset: float = 0.0,
                  zero_nyquist: bool = True):
    """Test 1.1 of Section 5.1: explicit Euler steps of the space-homogeneous
    equation from f(v, 0) = v^2/pi exp(-v^2), with the conservation projection
    applied to each Q if ``conserve``; returns the discrete relative L1 and L2
    errors against the exact solution at t_final.

    R <= 0 takes the default radius.  ``node_offset`` places the samples of the
    datum and of the exact solution at v_j = -T + (j + node_offset) dv; the
    operator acts on the sample vector exactly as on the node grid (the same
    transforms and tables: the sample positions are a property of the data, which
    the paper does not state)."""
    p = make_plan2(n, T, A, R=R)
    f = bkw2d_initial(n, T, node_offset)
    steps = int(round(t_final / dt))
    for _ in range(steps):
        Q = collide2_fast64(f, p, zero_nyquist=zero_nyquist)
        if conserve:
            Q = conserve2_Q(Q, n, T)
        f = f + dt * Q
    ex = bkw2d(n, T, steps * dt, node_offset)
    l1 = float(np.sum(np.abs(f - ex)) / np.sum(np.abs(ex)))
    l2 = float(np.sqrt(np.sum((f - ex) ** 2) / np.sum(ex ** 2)))
    return l1, l2
