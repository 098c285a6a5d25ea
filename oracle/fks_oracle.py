"""FP64 CPU oracle of the fast spectral VHS collision operator (test infrastructure).

Only tests, the smoke check and the bench's CPU-baseline leg use this module.
Nothing here is called by the HIP library, and nothing here calls it.

Conventions (each is one reading of the paper):

* Velocity grid (Section 3.1, eq. DM1): n points per axis on [-T, T), nodes
  v_j = -T + j dv, dv = 2T/n.  Arrays are indexed f[x][y][z] (C order).
* Fourier representation (Section 3.3, eqs. FU and FC) with the box
  rescaled from [-pi, pi] to [-T, T]: f(v) = sum_k fhat_k exp(i kappa k.v),
  kappa = pi/T, k integer in [-n/2, n/2).  For even n the -n/2 planes are
  not Hermitian-consistent with the kernel tables; the oracle zeroes every
  fhat_k having a component equal to -n/2 and uses the filtered f_N in the
  loss term.
* Carleman kernel (eq. Btilde, VHS kernel of eq. defVHSKernel): in 3D,
  B~(x, y) = 4 C_gamma (|x|^2 + |y|^2)^((gamma-1)/2), constant for hard
  spheres (gamma = 1).  C_gamma defaults to 1/(4 pi).
* B_F(l, m) of eq. FKM is written, after the decoupling of Section 3.3, as
  4 C_gamma * integral over the half sphere of phi(kappa l.e) psi(kappa |Pi_e m|) de,
  with phi(s) = int_{-R}^{R} |rho| a(|rho|) exp(i rho s) d rho and
  psi(s) = int_0^pi phi_b(s cos t) dt (the integral over the great circle
  orthogonal to e; no sin t factor).  For hard spheres this gives
  phi(s) = R^2 [2 Sinc(Rs) - Sinc^2(Rs/2)] (as printed) and
  psi(s) = 2 pi R J_1(Rs)/s, psi(0) = pi R^2.
* Half-sphere rule: Gauss-Legendre in cos(theta) (n_polar nodes) times a
  uniform azimuth phi_q = q pi / n_azim; weights w_p * pi / n_azim (sum 2 pi).
  A midpoint-in-theta rule with the sin(theta) Jacobian is the option
  ``rule="midpoint"``.
* gamma != 1 (B~ not decoupled): the radial kernel is expanded in K
  separable terms from a symmetric eigen-decomposition on graded
  Gauss-Legendre radial nodes; each (direction, term) pair is one
  convolution of the fast form.
* Loss term: by linearity all directions share one table
  L(m) = B_F(m, m) = sum_e omega_e alpha_e(m) beta_e(m), built with the same
  rule as the gain so that B_F(-m, m) = L(m) and mass is exact.

Parity pins: see ``tests/test_oracle_pins.py``; every public function here is
pinned except where a docstring says "parity unpinned".
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import special

__all__ = [
    "velocity_grid", "wavenumbers", "default_R", "sphere_rule", "hs_phi", "hs_psi",
    "RadialTerms", "radial_terms", "Plan", "make_plan", "build_tables", "spectrum",
    "synthesize", "collide_fast64", "collide_direct", "collision_basis",
    "conserve_Q", "project", "moments", "primitive", "relative_l2",
    "transport_shift", "transport_offsets_step", "euler_update", "exp_euler_update",
]


# ---------------------------------------------------------------------------
# Grids (Section 3.1 and 3.3)
# ---------------------------------------------------------------------------

def velocity_grid(n: int, T: float) -> np.ndarray:
    """Velocity nodes v_j = -T + j * 2T/n (Section 3.1, eq. DM1)."""
    return -T + np.arange(n, dtype=np.float64) * (2.0 * T / n)


def wavenumbers(n: int) -> np.ndarray:
    """Integer wavenumbers in FFT storage order: 0..n/2-1, -n/2..-1 (eq. FU)."""
    return np.fft.fftfreq(n, d=1.0 / n).round().astype(np.int64)


def default_R(T: float) -> float:
    """Truncation radius R with T = (3 + sqrt 2) R / 2 (Section 3.3)."""
    return 2.0 * T / (3.0 + math.sqrt(2.0))


# ---------------------------------------------------------------------------
# Half-sphere quadrature (Section 3.3, 3D decoupling formula)
# ---------------------------------------------------------------------------

def sphere_rule(n_polar: int, n_azim: int, rule: str = "gauss"):
    """Directions e_pq on the half sphere and their weights.

    theta in [0, pi], phi in [0, pi): e = (sin t cos p, sin t sin p, cos t).
    ``gauss``: cos(theta_p) are Gauss-Legendre nodes, weight w_p * pi/n_azim.
    ``midpoint``: theta_p = (p + 1/2) pi / n_polar, weight
    sin(theta_p) * (pi/n_polar) * (pi/n_azim).
    Returns (e[M, 3], w[M]) with M = n_polar * n_azim, p-major order.
    """
    if rule == "gauss":
        x, wx = np.polynomial.legendre.leggauss(n_polar)
        theta = np.arccos(x)
        wt = wx
    elif rule == "midpoint":
        theta = (np.arange(n_polar) + 0.5) * math.pi / n_polar
        wt = np.sin(theta) * math.pi / n_polar
    else:
        raise ValueError(rule)
    phi = np.arange(n_azim) * math.pi / n_azim
    e = np.empty((n_polar * n_azim, 3))
    w = np.empty(n_polar * n_azim)
    for p in range(n_polar):
        for q in range(n_azim):
            i = p * n_azim + q
            e[i] = (math.sin(theta[p]) * math.cos(phi[q]),
                    math.sin(theta[p]) * math.sin(phi[q]),
                    math.cos(theta[p]))
            w[i] = wt[p] * math.pi / n_azim
    return e, w


# ---------------------------------------------------------------------------
# Radial functions (Section 3.3)
# ---------------------------------------------------------------------------

def _sinc(x):
    """sin(x)/x with the removable singularity filled (numpy's sinc is sin(pi x)/(pi x))."""
    return np.sinc(np.asarray(x) / math.pi)


def hs_phi(s, R: float):
    """phi(s) = int_{-R}^{R} |rho| e^{i rho s} d rho = R^2 [2 Sinc(Rs) - Sinc^2(Rs/2)]."""
    s = np.asarray(s, dtype=np.float64)
    return R * R * (2.0 * _sinc(R * s) - _sinc(0.5 * R * s) ** 2)


def hs_psi(s, R: float):
    """psi(s) = int_0^pi phi(s cos t) dt = 2 pi R J_1(Rs)/s, psi(0) = pi R^2."""
    s = np.asarray(s, dtype=np.float64)
    out = np.empty_like(s)
    small = np.abs(s) < 1e-12
    ss = np.where(small, 1.0, s)
    out[...] = 2.0 * math.pi * R * special.j1(R * ss) / ss
    out[small] = math.pi * R * R
    return out


@dataclass
class RadialTerms:
    """K separable radial terms phi_r, psi_r of the Carleman kernel.

    For gamma == 1 the kernel is constant and K = 1 with the closed forms.
    Otherwise ``nodes`` are radial quadrature nodes rho_i and ``coef`` [nq, K]
    the coefficients c_ir, with phi_r(s) = 2 sum_i c_ir cos(rho_i s) and
    psi_r(s) = 2 pi sum_i c_ir J_0(rho_i s).
    """
    gamma: float
    R: float
    K: int
    nodes: np.ndarray | None = None
    coef: np.ndarray | None = None
    eigenvalues: np.ndarray | None = None

    def phi(self, s):
        s = np.asarray(s, dtype=np.float64)
        if self.coef is None:
            return hs_phi(s, self.R)[..., None]
        arg = np.multiply.outer(s, self.nodes)
        return 2.0 * np.cos(arg) @ self.coef

    def psi(self, s):
        s = np.asarray(s, dtype=np.float64)
        if self.coef is None:
            return hs_psi(s, self.R)[..., None]
        arg = np.multiply.outer(s, self.nodes)
        return 2.0 * math.pi * special.j0(arg) @ self.coef


def radial_terms(gamma: float, R: float, K: int = 0, tol: float = 1e-4,
                 nq: int = 200, force_expansion: bool = False) -> RadialTerms:
    """Separable expansion of (rho^2 + rho'^2)^((gamma-1)/2) on [0, R]^2.

    The decoupling assumption (eq. decoup) holds exactly only for hard spheres
    in 3D.  For other gamma the radial double integral
    int int rho rho' k(rho, rho') g(rho) h(rho') with
    k = (rho^2 + rho'^2)^((gamma-1)/2) is discretised on nq graded
    Gauss-Legendre nodes rho_i = R u_i^2 (weights w_i); the symmetric matrix
    A_ij = sqrt(w_i rho_i) k_ij sqrt(w_j rho_j) = sum_r lambda_r U_ir U_jr is
    truncated to its K leading eigenpairs (K = 0: smallest K with
    lambda_K / lambda_0 < tol), giving c_ir = sqrt(w_i rho_i) U_ir sqrt(lambda_r).
    """
    if gamma == 1.0 and not force_expansion:
        return RadialTerms(gamma=1.0, R=R, K=1)
    u, wu = np.polynomial.legendre.leggauss(nq)
    u = 0.5 * (u + 1.0)
    wu = 0.5 * wu
    rho = R * u * u
    w = wu * 2.0 * R * u
    sq = np.sqrt(w * rho)
    kmat = (rho[:, None] ** 2 + rho[None, :] ** 2) ** ((gamma - 1.0) / 2.0)
    A = sq[:, None] * kmat * sq[None, :]
    lam, U = np.linalg.eigh(A)
    order = np.argsort(lam)[::-1]
    lam = lam[order]
    U = U[:, order]
    if K <= 0:
        ratio = lam / lam[0]
        K = int(np.argmax(ratio < tol)) if np.any(ratio < tol) else len(lam)
        K = max(K, 1)
    coef = sq[:, None] * U[:, :K] * np.sqrt(np.maximum(lam[:K], 0.0))[None, :]
    return RadialTerms(gamma=gamma, R=R, K=K, nodes=rho, coef=coef, eigenvalues=lam)


# ---------------------------------------------------------------------------
# Plan and kernel-mode tables (Section 3.3)
# ---------------------------------------------------------------------------

@dataclass
class Plan:
    n: int
    T: float
    R: float
    gamma: float
    c_gamma: float
    n_polar: int
    n_azim: int
    rule: str
    radial: RadialTerms
    alpha: np.ndarray = field(repr=False, default=None)   # [J, n, n, n]
    beta: np.ndarray = field(repr=False, default=None)    # [J, n, n, n]
    omega: np.ndarray = field(repr=False, default=None)   # [J]
    loss: np.ndarray = field(repr=False, default=None)    # [n, n, n]

    @property
    def kappa(self) -> float:
        return math.pi / self.T

    @property
    def J(self) -> int:
        return self.n_polar * self.n_azim * self.radial.K


def make_plan(n: int, T: float, gamma: float = 1.0, R: float = 0.0,
              c_gamma: float = 0.0, n_polar: int = 8, n_azim: int = 4,
              rule: str = "gauss", K: int = 0, radial_tol: float = 1e-4,
              force_expansion: bool = False) -> Plan:
    """Builds the oracle plan and its FP64 tables (R <= 0 -> default_R(T); C <= 0 -> 1/(4 pi))."""
    if n % 2:
        raise ValueError("n must be even")
    R = R if R > 0 else default_R(T)
    c_gamma = c_gamma if c_gamma > 0 else 1.0 / (4.0 * math.pi)
    rad = radial_terms(gamma, R, K=K, tol=radial_tol, force_expansion=force_expansion)
    p = Plan(n=n, T=T, R=R, gamma=gamma, c_gamma=c_gamma, n_polar=n_polar,
             n_azim=n_azim, rule=rule, radial=rad)
    build_tables(p)
    return p


def _kgrid(n: int):
    k = wavenumbers(n).astype(np.float64)
    kx = k[:, None, None] * np.ones((1, n, n))
    ky = k[None, :, None] * np.ones((n, 1, n))
    kz = k[None, None, :] * np.ones((n, n, 1))
    return kx, ky, kz


def build_tables(p: Plan) -> None:
    """alpha_{e,r}(k) = phi_r(kappa k.e), beta_{e,r}(k) = psi_r(kappa |Pi_e k|), omega, L.

    Index j = (direction e) * K + r.  omega_j = 4 C_gamma w_e (the 2^{d-1} of
    eq. Btilde times the kernel constant, times the sphere weight).
    L(k) = sum_j omega_j alpha_j(k) beta_j(k) = B_F(k, k) (eq. ode).
    """
    n = p.n
    kx, ky, kz = _kgrid(n)
    k2 = kx * kx + ky * ky + kz * kz
    e, w = sphere_rule(p.n_polar, p.n_azim, p.rule)
    K = p.radial.K
    J = len(w) * K
    alpha = np.empty((J, n, n, n))
    beta = np.empty((J, n, n, n))
    omega = np.empty(J)
    for d in range(len(w)):
        kd = kx * e[d, 0] + ky * e[d, 1] + kz * e[d, 2]
        kperp = np.sqrt(np.maximum(k2 - kd * kd, 0.0))
        ph = p.radial.phi(p.kappa * kd)
        ps = p.radial.psi(p.kappa * kperp)
        for r in range(K):
            j = d * K + r
            alpha[j] = ph[..., r]
            beta[j] = ps[..., r]
            omega[j] = 4.0 * p.c_gamma * w[d]
    p.alpha, p.beta, p.omega = alpha, beta, omega
    p.loss = np.einsum("j,jxyz,jxyz->xyz", omega, alpha, beta)


# ---------------------------------------------------------------------------
# Fourier transforms with the paper's normalisation (eqs. FU, FC)
# ---------------------------------------------------------------------------

def _phase(n: int, T: float):
    """exp(i kappa k . v_0) with v_0 = (-T, -T, -T): maps DFT index order to eq. FU."""
    k = wavenumbers(n).astype(np.float64)
    ph = np.exp(1j * (math.pi / T) * k * (-T))
    return ph[:, None, None] * ph[None, :, None] * ph[None, None, :]


def spectrum(f: np.ndarray, n: int, T: float, zero_nyquist: bool = True) -> np.ndarray:
    """fhat_k = n^{-3} sum_j f_j exp(-i kappa k . v_j) (eq. FC on the grid).

    With ``zero_nyquist`` every mode with a component equal to -n/2 is set to 0.
    """
    fh = np.fft.fftn(f, axes=(-3, -2, -1)) / float(n) ** 3 * np.conj(_phase(n, T))
    if zero_nyquist:
        h = n // 2
        fh[..., h, :, :] = 0.0
        fh[..., :, h, :] = 0.0
        fh[..., :, :, h] = 0.0
    return fh


def synthesize(gh: np.ndarray, n: int, T: float) -> np.ndarray:
    """g(v_j) = sum_k ghat_k exp(i kappa k . v_j) (eq. FU on the grid); complex result."""
    return np.fft.ifftn(gh * _phase(n, T), axes=(-3, -2, -1)) * float(n) ** 3


# ---------------------------------------------------------------------------
# Collision operator
# ---------------------------------------------------------------------------

def collide_fast64(f: np.ndarray, p: Plan, parts: bool = False, batch: int = 8):
    """Fast spectral Q(f) for one cell, FP64 (Section 3.3, eq. ode with the decoupled B_F).

    Steps in the paper's order (Section 4.2 describes the loop): one forward
    transform of f; for each direction (and radial term) the coefficients
    alpha_j, beta_j times fhat, two inverse transforms giving
    a_j = F^{-1}(alpha_j fhat) and b_j = F^{-1}(beta_j fhat); gain
    Q+ = sum_j omega_j a_j b_j; loss Q- = f_N F^{-1}(L fhat); Q = Q+ - Q-.
    Returns Q[n][n][n] (and (Q+, Q-) if ``parts``).
    """
    n, T = p.n, p.T
    fh = spectrum(f, n, T)
    fN = synthesize(fh, n, T).real
    gain = np.zeros((n, n, n))
    J = p.J
    for j0 in range(0, J, batch):
        j1 = min(J, j0 + batch)
        a = synthesize(p.alpha[j0:j1] * fh, n, T).real
        b = synthesize(p.beta[j0:j1] * fh, n, T).real
        gain += np.einsum("j,jxyz->xyz", p.omega[j0:j1], a * b)
    loss = fN * synthesize(p.loss * fh, n, T).real
    Q = gain - loss
    if parts:
        return Q, gain, loss
    return Q


def collide_direct(f: np.ndarray, p: Plan) -> np.ndarray:
    """Direct O(n^2) spectral quadrature (eq. ode), for small n only.

    Qhat_k = sum over (l, m) with l + m = k (mod n) of fhat_l fhat_m
    [B_F(l, m) - B_F(m, m)], with B_F(l, m) = sum_j omega_j alpha_j(l) beta_j(m)
    the direction-quadrature of eq. FKM; then Q = sum_k Qhat_k e^{i kappa k.v}.
    """
    n, T = p.n, p.T
    nn = n ** 3
    if nn > 1728:
        raise ValueError("direct form is limited to n <= 12")
    fh = spectrum(f, n, T).reshape(nn)
    A = p.alpha.reshape(p.J, nn)
    B = p.beta.reshape(p.J, nn)
    BF = (A * p.omega[:, None]).T @ B          # BF[l, m]
    Lm = np.diag(BF).copy()                    # B_F(m, m)
    kern = BF - Lm[None, :]
    k = wavenumbers(n)
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    kx, ky, kz = kx.ravel(), ky.ravel(), kz.ravel()
    # target index of l + m (mod n), in FFT storage order
    tx = np.mod(kx[:, None] + kx[None, :], n)
    ty = np.mod(ky[:, None] + ky[None, :], n)
    tz = np.mod(kz[:, None] + kz[None, :], n)
    tgt = ((tx * n + ty) * n + tz).ravel()
    wts = (fh[:, None] * fh[None, :] * kern).ravel()
    qh = (np.bincount(tgt, weights=wts.real, minlength=nn)
          + 1j * np.bincount(tgt, weights=wts.imag, minlength=nn))
    Q = synthesize(qh.reshape(n, n, n), n, T)
    return Q.real


# ---------------------------------------------------------------------------
# Conservation (Section 3.2, eqs. minim, legrange, minim1) and moments (eq. i5)
# ---------------------------------------------------------------------------

def collision_basis(n: int, T: float) -> np.ndarray:
    """Rows (1, v_x, v_y, v_z, |v|^2) over the grid: C = dv^3 * basis (Section 3.2)."""
    v = velocity_grid(n, T)
    vx, vy, vz = np.meshgrid(v, v, v, indexing="ij")
    return np.stack([np.ones_like(vx), vx, vy, vz, vx * vx + vy * vy + vz * vz]).reshape(5, -1)


def conserve_Q(Q: np.ndarray, n: int, T: float) -> np.ndarray:
    """Q_c = Q - C^T (C C^T)^{-1} C Q, i.e. eq. minim1 applied to f + h Q with U = C f.

    Works on a single cell [n,n,n] or a batch [c,n,n,n].  The dv^3 factors of C
    cancel in the projector.
    """
    Phi = collision_basis(n, T)
    G = Phi @ Phi.T
    q = Q.reshape(-1, n ** 3)
    lam = np.linalg.solve(G, Phi @ q.T)        # [5, c]
    return (q - (Phi.T @ lam).T).reshape(Q.shape)


def project(f: np.ndarray, U: np.ndarray, n: int, T: float) -> np.ndarray:
    """f + C^T (C C^T)^{-1} (U - C f) (eq. minim1), per cell; U[..., 5] in moment units."""
    Phi = collision_basis(n, T)
    dv3 = (2.0 * T / n) ** 3
    C = dv3 * Phi
    G = C @ C.T
    ff = f.reshape(-1, n ** 3)
    UU = np.asarray(U, dtype=np.float64).reshape(-1, 5)
    lam = np.linalg.solve(G, (UU - ff @ C.T).T)
    return (ff + (C.T @ lam).T).reshape(f.shape)


def moments(f: np.ndarray, n: int, T: float) -> np.ndarray:
    """U = C f = dv^3 sum_j f_j (1, v_j, |v_j|^2): (rho, rho u_x, rho u_y, rho u_z, sum |v|^2 f dv^3)."""
    Phi = collision_basis(n, T)
    dv3 = (2.0 * T / n) ** 3
    return dv3 * (f.reshape(-1, n ** 3) @ Phi.T).reshape(f.shape[:-3] + (5,))


def primitive(U: np.ndarray):
    """(rho, u, theta) from U with 3 rho theta = U_4 - rho |u|^2 (eq. i6 with d_v = 3)."""
    U = np.asarray(U)
    rho = U[..., 0]
    u = U[..., 1:4] / rho[..., None]
    theta = (U[..., 4] / rho - np.sum(u * u, axis=-1)) / 3.0
    return rho, u, theta


def euler_update(f: np.ndarray, Qc: np.ndarray, dt_over_tau: float) -> np.ndarray:
    """f^{n+1} = f* + (dt/tau) Q_c (eq. f_coll with the rescaling of Part 2)."""
    return f + dt_over_tau * Qc


def exp_euler_update(f: np.ndarray, Qc: np.ndarray, dt_over_tau: float, mu: float) -> np.ndarray:
    """Exponential Euler step of the collision ODE for stiff (small tau) collisions.

    Reading (Section 3.1 leaves the stiff case to the integrators of its references):
    split Q = [Q + mu (f - M)] - mu (f - M) with M the local Maxwellian, which the
    collision step does not change, and integrate the linear part exactly over
    h = dt/tau with the rest frozen.  Then f - M cancels and the step is
    f^{n+1} = f* + ((1 - exp(-mu h)) / mu) Q_c: Euler with its step capped at 1/mu.
    For BGK (Q = nu (M - f), mu = nu) this is the exact relaxation step."""
    return f + (-math.expm1(-mu * dt_over_tau) / mu) * Qc


def relative_l2(a: np.ndarray, b: np.ndarray) -> float:
    """(sum |a-b|^2 / sum |b|^2)^{1/2} over the whole array."""
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


# ---------------------------------------------------------------------------
# FKS transport (Section 3.1 eq. f_bar; particle form of Section 4.1)
# ---------------------------------------------------------------------------

def transport_offsets_step(offsets: np.ndarray, n: int, T: float, dx: float, dt: float):
    """Advance per-axis displacements s_a[k] += v_k dt; return (new offsets, shift[3][n]).

    The piece of f carried by velocity v_k covers the cell centre x_j when its
    displacement s satisfies |x_j - x_i - s| <= dx/2, so the mass seen at cell
    j is the one that started in cell j - d with d = floor(s/dx + 1/2).  The
    per-step index shift is d(s + v dt) - d(s).
    """
    v = velocity_grid(n, T)
    old = np.asarray(offsets, dtype=np.float64).reshape(3, n)
    new = old + v[None, :] * dt
    d_old = np.floor(old / dx + 0.5).astype(np.int64)
    d_new = np.floor(new / dx + 0.5).astype(np.int64)
    return new, d_new - d_old


def transport_shift(f: np.ndarray, shift: np.ndarray, n: int, bc=("periodic",) * 3,
                    bc_f: np.ndarray | None = None) -> np.ndarray:
    """Exact FKS transport of piecewise-constant data by an integer cell shift.

    f[nz][ny][nx][n][n][n]; shift[3][n] holds the per-axis shift (x, y, z) for
    each 1D velocity index.  new[iz,iy,ix,kx,ky,kz] = f[iz-sz, iy-sy, ix-sx, ...]
    with periodic wrap, or, for a ``dirichlet`` axis whose source index falls
    outside the domain, the inflow state bc_f[face][kx,ky,kz]
    (faces: 0 x-low, 1 x-high, 2 y-low, 3 y-high, 4 z-low, 5 z-high; the first
    out-of-range axis in x, y, z order decides the face).
    """
    nz, ny, nx = f.shape[:3]
    out = np.empty_like(f)
    dims = (nx, ny, nz)
    for kx in range(n):
        for ky in range(n):
            for kz in range(n):
                sx, sy, sz = shift[0][kx], shift[1][ky], shift[2][kz]
                for iz in range(nz):
                    for iy in range(ny):
                        for ix in range(nx):
                            src = [ix - sx, iy - sy, iz - sz]
                            face = -1
                            for a in range(3):
                                if bc[a] == "periodic":
                                    src[a] %= dims[a]
                                elif src[a] < 0 or src[a] >= dims[a]:
                                    if face < 0:
                                        face = 2 * a + (0 if src[a] < 0 else 1)
                            if face >= 0:
                                out[iz, iy, ix, kx, ky, kz] = bc_f[face, kx, ky, kz]
                            else:
                                out[iz, iy, ix, kx, ky, kz] = f[src[2], src[1], src[0], kx, ky, kz]
    return out
