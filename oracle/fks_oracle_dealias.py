"""FP64 CPU oracle of the de-aliased (zero-padded) fast spectral operator (test infrastructure).

Only tests, the smoke check and the bench's CPU-baseline leg use this module.
Nothing here is called by the HIP library, and nothing here calls it.

The operator of Section 3.3 evaluates the convolution Qhat_k = sum over
l + m = k of fhat_l fhat_m beta(l, m) with N-point transforms, so the sum wraps:
pairs with l + m = k +- n land on k (the periodisation discussed at eqs. FU, FC
and in the choice of T against R).  The de-aliased variant keeps only the
pairs with l + m = k exactly, for k in the band of the grid:

    Qhat_k = sum_{l, m in band, l + m = k} fhat_l fhat_m [B_F(l, m) - B_F(m, m)],
    band = {k : -n/2 < k_i < n/2}  (the Nyquist planes stay zero, as for fhat).

Readings:
* Both factors of every product (a_j, b_j, and f_N with F^{-1}(L fhat)) are band
  limited to |k_i| <= n/2 - 1, so their product holds |k_i| <= n - 2.  Sampled
  on a grid of n' points per axis over the same box [-T, T), frequency p shows
  up at p - n'; it stays out of the band when n' - (n - 2) >= n/2, i.e. for
  n' >= 3n/2 - 2 (the 3/2 rule of pseudo-spectral quadratic products), and
  the band coefficients of the sampled product are then exact.  The default
  n' is 3n/2.
* The result is the band projection of Q: the Nyquist planes of Qhat are
  zeroed, like those of fhat.  Q is then sampled on the original n grid.
* Mass stays exact (l + m = 0 pairs give B_F(-m, m) - L(m) = 0); momentum and
  energy are restored by the same FP64 projection as the aliased operator.
"""
import numpy as np

from .fks_oracle import Plan, spectrum, synthesize, wavenumbers

__all__ = ["padded_size", "band_mask", "pad_band", "synthesize_on", "band_spectrum_on",
           "collide_dealias_fast64", "collide_dealias_direct"]


def padded_size(n: int) -> int:
    """Default padded grid n' = 3n/2 (alias-free for quadratic products of band-limited data)."""
    return 3 * n // 2


def band_mask(n: int) -> np.ndarray:
    """Boolean [n][n][n] mask (FFT storage order) of the band -n/2 < k_i < n/2."""
    k = wavenumbers(n)
    b = np.abs(k) < n // 2
    return b[:, None, None] & b[None, :, None] & b[None, None, :]


def _positions(n: int, npad: int) -> np.ndarray:
    """Index of each band wavenumber of the n grid (FFT order) in the npad grid (FFT order);
    the Nyquist index n/2 maps to -1 (dropped)."""
    k = wavenumbers(n)
    pos = np.mod(k, npad)
    pos[np.abs(k) >= n // 2] = -1
    return pos


def pad_band(gh: np.ndarray, n: int, npad: int) -> np.ndarray:
    """Places the band coefficients of gh[..., n, n, n] into zeros[..., npad, npad, npad]."""
    pos = _positions(n, npad)
    keep = pos >= 0
    out = np.zeros(gh.shape[:-3] + (npad, npad, npad), dtype=np.complex128)
    ix = np.ix_(pos[keep], pos[keep], pos[keep])
    out[(Ellipsis,) + ix] = gh[(Ellipsis,) + np.ix_(keep, keep, keep)]
    return out


def synthesize_on(gh: np.ndarray, n: int, npad: int, T: float) -> np.ndarray:
    """g(v'_j) = sum over the band of ghat_k exp(i kappa k.v'_j) on the npad grid
    v'_j = -T + j 2T/npad (eq. FU evaluated on a finer grid of the same box); complex."""
    return synthesize(pad_band(gh * band_mask(n), n, npad), npad, T)


def band_spectrum_on(g: np.ndarray, n: int, npad: int, T: float) -> np.ndarray:
    """Band coefficients (n grid, FFT order, Nyquist planes zero) of samples g on the npad grid:
    ghat_k = npad^{-3} sum_j g(v'_j) exp(-i kappa k.v'_j) (eq. FC on the npad grid)."""
    full = spectrum(g, npad, T, zero_nyquist=False)
    pos = _positions(n, npad)
    keep = pos >= 0
    out = np.zeros(g.shape[:-3] + (n, n, n), dtype=np.complex128)
    out[(Ellipsis,) + np.ix_(keep, keep, keep)] = full[(Ellipsis,) + np.ix_(pos[keep], pos[keep], pos[keep])]
    return out


def collide_dealias_fast64(f: np.ndarray, p: Plan, npad: int = 0, parts: bool = False, batch: int = 8):
    """De-aliased fast Q(f) for one cell, FP64: the steps of the fast form (forward transform,
    a_j = F^{-1}(alpha_j fhat), b_j = F^{-1}(beta_j fhat), gain sum_j omega_j a_j b_j, loss
    f_N F^{-1}(L fhat)) with every inverse transform evaluated on the npad grid, then the band
    coefficients of gain - loss, sampled back on the n grid.  Returns Q[n][n][n] (and the band
    spectra (Qhat+, Qhat-) if ``parts``)."""
    n, T = p.n, p.T
    npad = npad or padded_size(n)
    fh = spectrum(f, n, T)
    fN = synthesize_on(fh, n, npad, T).real
    gain = np.zeros((npad, npad, npad))
    for j0 in range(0, p.J, batch):
        j1 = min(p.J, j0 + batch)
        a = synthesize_on(p.alpha[j0:j1] * fh, n, npad, T).real
        b = synthesize_on(p.beta[j0:j1] * fh, n, npad, T).real
        gain += np.einsum("j,jxyz->xyz", p.omega[j0:j1], a * b)
    loss = fN * synthesize_on(p.loss * fh, n, npad, T).real
    gh = band_spectrum_on(gain, n, npad, T)
    lh = band_spectrum_on(loss, n, npad, T)
    Q = synthesize(gh - lh, n, T).real
    if parts:
        return Q, gh, lh
    return Q


def collide_dealias_direct(f: np.ndarray, p: Plan) -> np.ndarray:
    """The definition written out, for small n only: the double sum over band pairs (l, m)
    with l + m = k exactly (no wrap), k in the band, weights B_F(l, m) - B_F(m, m) from the
    plan's tables; then Q = sum_k Qhat_k exp(i kappa k.v) on the n grid."""
    n, T = p.n, p.T
    nn = n ** 3
    if nn > 1728:
        raise ValueError("direct form is limited to n <= 12")
    fh = spectrum(f, n, T).reshape(nn)
    A = p.alpha.reshape(p.J, nn)
    B = p.beta.reshape(p.J, nn)
    BF = (A * p.omega[:, None]).T @ B          # BF[l, m]
    kern = BF - np.diag(BF)[None, :]
    k = wavenumbers(n)
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    kx, ky, kz = kx.ravel(), ky.ravel(), kz.ravel()
    sx = kx[:, None] + kx[None, :]
    sy = ky[:, None] + ky[None, :]
    sz = kz[:, None] + kz[None, :]
    h = n // 2
    inband = (np.abs(sx) < h) & (np.abs(sy) < h) & (np.abs(sz) < h)
    tgt = ((np.mod(sx, n) * n + np.mod(sy, n)) * n + np.mod(sz, n))
    wts = fh[:, None] * fh[None, :] * kern
    tgt, wts = tgt[inband], wts[inband]
    qh = (np.bincount(tgt, weights=wts.real, minlength=nn)
          + 1j * np.bincount(tgt, weights=wts.imag, minlength=nn))
    return synthesize(qh.reshape(n, n, n), n, T).real
