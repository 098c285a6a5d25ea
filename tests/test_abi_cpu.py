"""Host-side checks of libfks.so that need no GPU: loading, exported symbols,
descriptor validation, and the FP64 host precompute against the oracle."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_1608_08009_amd as fks

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "fks.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fks_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = fks.lib()
    declared = _declared_symbols()
    assert len(declared) >= 13
    for name in declared:
        assert hasattr(L, name), name
    assert set(fks.EXPORTED) == set(declared)


def test_status_strings():
    L = fks.lib()
    for s in (0, -1, -2, -3, -4, -5):
        assert L.fks_status_string(s).decode().startswith("FKS_")


@pytest.mark.parametrize("field,value,expect", [
    ("n", 7, fks.FKS_ERR_UNSUPPORTED), ("n", 10, fks.FKS_ERR_UNSUPPORTED), ("n", 64, fks.FKS_ERR_UNSUPPORTED),
    ("n", 0, fks.FKS_ERR_INVALID), ("T", -1.0, fks.FKS_ERR_INVALID), ("T", float("nan"), fks.FKS_ERR_INVALID),
    ("gamma", 1.5, fks.FKS_ERR_INVALID), ("n_polar", 0, fks.FKS_ERR_INVALID), ("rule", 5, fks.FKS_ERR_INVALID),
    ("precision", 9, fks.FKS_ERR_INVALID), ("flags", 0x80, fks.FKS_ERR_INVALID),
    ("radial_terms", -1, fks.FKS_ERR_INVALID),
])
def test_desc_validation_rejects(field, value, expect):
    d = fks.Desc(n=16, T=8.0)
    setattr(d, field, value)
    assert fks.desc_validate(d) == expect


def test_desc_validation_accepts_the_numeric_guard_flag():
    for flags in (fks.FLAG_NUMERIC_GUARD, fks.FLAG_NUMERIC_GUARD | fks.FLAG_FORCE_GENERIC):
        assert fks.desc_validate(fks.Desc(n=16, T=8.0, flags=flags)) == fks.FKS_OK
    d2 = fks.desc2d(16, 6.0)
    d2.flags = fks.FLAG_NUMERIC_GUARD
    assert fks.desc_validate(d2) == fks.FKS_OK
    assert fks.desc_validate(fks.Desc(n=16, T=8.0, flags=0x8)) == fks.FKS_ERR_INVALID


@pytest.mark.parametrize("kw,expect", [
    (dict(n=4), fks.FKS_OK), (dict(n=32), fks.FKS_OK), (dict(n=24, gamma=0.5), fks.FKS_OK),
    (dict(n=32, precision=fks.PREC_F64), fks.FKS_OK),
    (dict(n=6), fks.FKS_ERR_UNSUPPORTED), (dict(n=48), fks.FKS_ERR_UNSUPPORTED),
    (dict(n=16, gamma=0.0, n_azim=1, dim=2), fks.FKS_ERR_UNSUPPORTED),
])
def test_desc_validation_of_the_dealias_flag(kw, expect):
    base = dict(T=8.0, flags=fks.FLAG_DEALIAS)
    base.update(kw)
    assert fks.desc_validate(fks.Desc(**base)) == expect


def test_numeric_status_rejects_null_plan():
    cell = C.c_int64(7)
    assert fks.lib().fks_numeric_status(None, C.byref(cell), 0) == fks.FKS_ERR_INVALID
    assert cell.value == 7


@pytest.mark.parametrize("n", [4, 6, 8, 12, 16, 24, 32, 48])
def test_desc_validation_accepts_supported_sizes(n):
    assert fks.desc_validate(fks.Desc(n=n, T=8.0, gamma=0.5)) == fks.FKS_OK


@pytest.mark.parametrize("rule,name", [(fks.RULE_GAUSS, "gauss"), (fks.RULE_MIDPOINT, "midpoint")])
@pytest.mark.parametrize("npol,naz", [(1, 1), (4, 3), (8, 4), (8, 8), (16, 4)])
def test_host_sphere_rule_matches_oracle(rule, name, npol, naz):
    got = fks.host_sphere_rule(npol, naz, rule)
    e, w = O.sphere_rule(npol, naz, name)
    assert np.allclose(got[:, :3], e, atol=2e-15, rtol=0)
    assert np.allclose(got[:, 3], w, atol=2e-15, rtol=0)


@pytest.mark.parametrize("gamma,K", [(0.0, 11), (0.5, 7), (0.0, 4)])
def test_host_radial_terms_match_oracle(gamma, K):
    R = 3.6
    k, nodes, coef = fks.host_radial_terms(gamma, R, K=K)
    rt = O.radial_terms(gamma, R, K=K)
    assert k == rt.K == K
    assert np.allclose(nodes, rt.nodes, rtol=1e-14, atol=0)
    # eigenvector signs are arbitrary; compare the sign-invariant outer products
    for r in range(K):
        a, b = coef[:, r], rt.coef[:, r]
        sgn = np.sign(a @ b)
        assert np.max(np.abs(a - sgn * b)) < 1e-9 * np.max(np.abs(b)) * max(1.0, 10.0 ** r / 1e3)


def test_host_radial_terms_tolerance_selects_K():
    for gamma in (0.0, 0.5):
        k, _, _ = fks.host_radial_terms(gamma, 3.6, K=0, tol=1e-4)
        assert k == O.radial_terms(gamma, 3.6, tol=1e-4).K


# -- two velocity dimensions (dim = 2): validation and host tables ------------

@pytest.mark.parametrize("kw,expect", [
    (dict(dim=4), fks.FKS_ERR_INVALID),
    (dict(dim=2, gamma=1.0), fks.FKS_ERR_UNSUPPORTED),       # only Maxwell molecules decouple in 2D
    (dict(dim=2, n_azim=4), fks.FKS_ERR_INVALID),
    (dict(dim=2, n=10), fks.FKS_ERR_UNSUPPORTED),
    (dict(dim=2, n=64, precision=fks.PREC_F64), fks.FKS_ERR_UNSUPPORTED),
    (dict(dim=2, flags=fks.FLAG_FORCE_GENERIC), fks.FKS_ERR_UNSUPPORTED),
    (dict(dim=2, radial_terms=3), fks.FKS_ERR_INVALID),
])
def test_desc2d_validation_rejects(kw, expect):
    base = dict(n=16, T=6.0, gamma=0.0, n_polar=8, n_azim=1)
    base.update(kw)
    assert fks.desc_validate(fks.Desc(**base)) == expect


@pytest.mark.parametrize("n,prec", [(8, fks.PREC_F64), (12, fks.PREC_F64), (32, fks.PREC_F64),
                                    (48, fks.PREC_F32_FIX64), (64, fks.PREC_F32_FIX64)])
def test_desc2d_validation_accepts(n, prec):
    assert fks.desc_validate(fks.desc2d(n, 6.0, 8, prec)) == fks.FKS_OK


@pytest.mark.parametrize("n,T,A", [(8, 4.0, 8), (16, 6.0, 5), (24, 9.0, 16)])
def test_host_tables_2d_match_oracle(n, T, A):
    # the library's host tables against the oracle's alpha, alpha', omega and L (eq. dfor0)
    import oracle.fks_oracle2d as O2
    ab = fks.host_tables_2d(fks.desc2d(n, T, A))
    p = O2.make_plan2(n, T, A)
    assert ab.shape == (A + 1, n, n, 2)
    gain = ab[:A, ..., 0] * ab[:A, ..., 1]
    assert np.allclose(gain, p.omega * p.alpha * p.alphap, rtol=0, atol=1e-13 * p.R * p.R)
    assert np.allclose(ab[:A, ..., 0] ** 2, p.omega * p.alpha ** 2, rtol=0, atol=1e-13 * p.R * p.R)
    assert np.allclose(ab[A, ..., 0] * ab[A, ..., 1], -p.loss, rtol=0, atol=1e-13 * np.abs(p.loss).max())
    assert np.all(ab[A, ..., 1] == ab[A, 0, 0, 1]) and ab[A, 0, 0, 1] > 0


# -- BGK (fks_bgk): argument validation, no device work -----------------------

@pytest.mark.parametrize("kw,expect", [
    (dict(), fks.FKS_OK),
    (dict(dim=2, n=512), fks.FKS_OK),
    (dict(dim=4), fks.FKS_ERR_INVALID),
    (dict(n=1), fks.FKS_ERR_INVALID),
    (dict(n=65), fks.FKS_ERR_INVALID),
    (dict(dim=2, n=513), fks.FKS_ERR_INVALID),
    (dict(T=0.0), fks.FKS_ERR_INVALID),
    (dict(nu=-1.0), fks.FKS_ERR_INVALID),
    (dict(nu_rho=2), fks.FKS_ERR_INVALID),
    (dict(step=5), fks.FKS_ERR_INVALID),
    (dict(dt_over_tau=float("nan")), fks.FKS_ERR_INVALID),
])
def test_bgk_validation(kw, expect):
    args = dict(dim=3, n=32, T=8.0, nu=1.0)
    args.update(kw)
    assert fks.bgk_validate(**args) == expect


def test_spectrum_workspace_size_host():
    b = C.c_size_t()
    assert fks.lib().fks_spectrum_workspace_size(7, 32, C.byref(b)) == fks.FKS_OK
    assert b.value == 7 * 32 ** 3 * 16
    assert fks.lib().fks_spectrum_workspace_size(10_000, 16, C.byref(b)) == fks.FKS_OK
    assert b.value == 512 * 16 ** 3 * 16
    assert fks.lib().fks_spectrum_workspace_size(1, 10, C.byref(b)) == fks.FKS_ERR_UNSUPPORTED
    assert fks.lib().fks_spectrum(None, None, 0, 16, 0, None, 0, None) == fks.FKS_OK      # empty batch
    assert fks.lib().fks_spectrum(None, None, 1, 16, 2, None, 0, None) == fks.FKS_ERR_INVALID


def test_split_stepper_validates_its_options_before_touching_the_device():
    from paper_1608_08009_amd.splitstep import SplitStepper
    for kw in (dict(scheme="leapfrog"), dict(collision="rk4"), dict(collision="exp"),
               dict(collision="exp", mu=float("inf"))):
        with pytest.raises(ValueError):
            SplitStepper(None, None, None, **kw)


def test_halo_sizes_and_rejections_on_the_host():
    # message sizes of the z-slab exchange: ceil(n/2) values of kz leave through z-, n - 1 - floor(n/2) through z+
    for n, lo, hi in ((4, 2, 1), (5, 3, 2), (24, 12, 11)):
        assert fks.halo_size(3, 2, 5, n, fks.FACE_ZLO) == 3 * 2 * n * n * lo * 8
        assert fks.halo_size(3, 2, 5, n, fks.FACE_ZHI) == 3 * 2 * n * n * hi * 8
    for args in ((3, 2, 5, 4, 2), (3, 2, 5, 1, 0), (3, 2, 0, 4, 0), (0, 2, 5, 4, 1)):
        with pytest.raises(fks.FksError):
            fks.halo_size(*args)
    L = fks.lib()
    sp = fks.SpaceDesc(3, 2, 5, 0.25, (C.c_int32 * 3)(0, 0, 0))
    fake_a, fake_b = C.c_void_p(1 << 20), C.c_void_p(1 << 40)   # never dereferenced: rejected first
    assert L.fks_halo_pack(None, C.byref(sp), 4, 0, fake_b, None) == fks.FKS_ERR_INVALID
    assert L.fks_halo_pack(fake_a, C.byref(sp), 4, 3, fake_b, None) == fks.FKS_ERR_INVALID
    assert L.fks_halo_pack(fake_a, None, 4, 1, fake_b, None) == fks.FKS_ERR_INVALID
    assert L.fks_halo_pack(fake_a, C.byref(sp), 4, 1, None, None) == fks.FKS_ERR_INVALID
    # a slab step whose z shift exceeds what the messages hold is refused, offsets untouched;
    # so is a step without both messages
    n, T = 4, 2.0
    off = np.zeros((3, n))
    msg_a, msg_b = C.c_void_p(1 << 42), C.c_void_p(1 << 43)
    for dt in (2.2 * 0.25 / T, -0.5 * 0.25 / T):
        assert L.fks_transport_shift_slab(fake_a, fake_b, C.byref(sp), n, T, dt, C.c_void_p(off.ctypes.data),
                                          msg_a, msg_b, None, None) == fks.FKS_ERR_INVALID
        assert not off.any()
    for below, above in ((None, msg_b), (msg_a, None)):
        assert L.fks_transport_shift_slab(fake_a, fake_b, C.byref(sp), n, T, 0.1, C.c_void_p(off.ctypes.data),
                                          below, above, None, None) == fks.FKS_ERR_INVALID
        assert not off.any()


def test_static_workspace_size_and_host_validation():
    # the binding's constant is the header's; validation needs no device
    text = open(os.path.join(ROOT, "include", "fks.h")).read()
    m = re.search(r"#define FKS_STATIC_WORKSPACE_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == fks.STATIC_WORKSPACE_BYTES
    L = fks.lib()
    assert L.fks_collide_batch_static(None, -1, None) == fks.FKS_ERR_INVALID
    assert L.fks_collide_batch_static(None, 1, None) == fks.FKS_ERR_INVALID
    assert L.fks_collide_batch_static(None, 0, None) == fks.FKS_OK
    seg = (fks.Segment * 1)()
    seg[0] = fks.Segment(None, None, None, None, 4, 0.0, None)   # no plan
    assert L.fks_collide_batch_static(seg, 1, None) == fks.FKS_ERR_INVALID


def test_split_scheme_scalars():
    # fks_stable_dt: transport CFL or the collision bound, whichever is smaller
    R = 2 * 8.0 / (3 + math.sqrt(2))
    c = 1 / (4 * math.pi)
    mu = 4 * math.pi * c * (2 * R) ** 0.5 * 1.5
    assert fks.stable_dt(0.01, 8.0, 0.3, R, 0.5, c, 1.5) == pytest.approx(min(0.01 / 8.0, 0.3 / mu), rel=1e-15)
    assert fks.stable_dt(1.0, 8.0, 1e-3, R, 1.0, c, 1.0) == pytest.approx(1e-3 / (2 * R), rel=1e-15)
    # fks_exp_euler_step: Euler for small mu dt, capped at 1/mu, monotone in dt
    assert fks.exp_euler_step(2.0, 1e-9) == pytest.approx(1e-9, rel=1e-8)
    assert fks.exp_euler_step(2.0, 1e3) == pytest.approx(0.5, rel=1e-15)
    h = [fks.exp_euler_step(3.0, d) for d in (0.0, 0.1, 0.2, 0.4)]
    assert h[0] == 0.0 and all(a < b for a, b in zip(h, h[1:])) and h[-1] < 1 / 3.0
    assert fks.exp_euler_step(3.0, 0.1) == pytest.approx((1 - math.exp(-0.3)) / 3.0, rel=1e-14)
    L = fks.lib()
    out = C.c_double()
    assert L.fks_exp_euler_step(0.0, 0.1, C.byref(out)) == fks.FKS_ERR_INVALID
    assert L.fks_exp_euler_step(1.0, -0.1, C.byref(out)) == fks.FKS_ERR_INVALID
    assert L.fks_stable_dt(0.1, 8.0, 1.0, R, 1.5, c, 1.0, C.byref(out)) == fks.FKS_ERR_INVALID
    assert L.fks_stable_dt(0.1, 8.0, 1.0, R, 0.5, c, 0.0, C.byref(out)) == fks.FKS_ERR_INVALID
