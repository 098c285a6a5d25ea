"""Python binding of libfks.so, the MI355X fast spectral Boltzmann collision library.

Argument marshalling only: every step of the computation runs in the HIP
library (C ABI declared in ``include/fks.h``).  Device arrays are torch tensors
on the current HIP device; calls are enqueued on torch's current stream.

The library is loaded lazily on first use; if ``libfks.so`` has not been built
the call raises ``RuntimeError`` (there is no fallback implementation).
"""
from __future__ import annotations

import ctypes as C
import os
import sys
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfks.so")

FKS_OK = 0
FKS_ERR_INVALID = -1
FKS_ERR_UNSUPPORTED = -2
FKS_ERR_NOMEM = -3
FKS_ERR_DEVICE = -4
FKS_ERR_NUMERIC = -5

PREC_F64 = 0
PREC_F32_FIX64 = 1
RULE_GAUSS = 0
RULE_MIDPOINT = 1
FLAG_FORCE_GENERIC = 0x1
FLAG_NUMERIC_GUARD = 0x2
FLAG_DEALIAS = 0x4
BGK_EULER = 0
BGK_EXACT = 1
BC_PERIODIC = 0
BC_DIRICHLET = 1
FACE_ZLO = 0
FACE_ZHI = 1

EXPORTED = [
    "fks_plan_create", "fks_plan_destroy", "fks_plan_query", "fks_plan_copy_tables",
    "fks_workspace_size", "fks_collide_batch", "fks_moments", "fks_conserve",
    "fks_transport_shift", "fks_status_string", "fks_desc_validate",
    "fks_host_sphere_rule", "fks_host_radial_terms", "fks_profile_enable", "fks_profile_last",
    "fks_host_tables_2d", "fks_bgk", "fks_spectrum_workspace_size", "fks_spectrum",
    "fks_numeric_status", "fks_autotune_workspace_size", "fks_autotune",
    "fks_halo_size", "fks_halo_pack", "fks_transport_shift_slab", "fks_collide_batch_static",
    "fks_stable_dt", "fks_exp_euler_step",
]

STATIC_WORKSPACE_BYTES = 64 << 20   # FKS_STATIC_WORKSPACE_BYTES


class PlanDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("T", C.c_double), ("R", C.c_double), ("gamma", C.c_double),
        ("c_gamma", C.c_double), ("n_polar", C.c_int32), ("n_azim", C.c_int32),
        ("rule", C.c_int32), ("radial_terms", C.c_int32), ("radial_tol", C.c_double),
        ("precision", C.c_int32), ("flags", C.c_uint32), ("dim", C.c_int32),
    ]


class PlanInfo(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("M", C.c_int32), ("K", C.c_int32), ("J", C.c_int32),
        ("R", C.c_double), ("c_gamma", C.c_double), ("precision", C.c_int32),
        ("fused", C.c_int32), ("table_bytes", C.c_size_t), ("flops_per_cell", C.c_double),
        ("dim", C.c_int32), ("fused_grid", C.c_int32), ("queue_items_per_wg", C.c_int32),
    ]


class Segment(C.Structure):
    _fields_ = [
        ("plan", C.c_void_p), ("f", C.c_void_p), ("q_out", C.c_void_p), ("f_out", C.c_void_p),
        ("ncell", C.c_int64), ("dt_over_tau", C.c_double), ("f_base", C.c_void_p),
    ]


class BgkDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n", C.c_int32), ("T", C.c_double), ("nu", C.c_double),
        ("nu_rho", C.c_int32), ("step", C.c_int32),
    ]


class SpaceDesc(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("dx", C.c_double),
        ("bc", C.c_int32 * 3),
    ]


_lib = None


def lib() -> C.CDLL:
    """Loads libfks.so (once).  Raises RuntimeError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1608_08009_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    L.fks_plan_create.argtypes = [C.POINTER(PlanDesc), vp, C.POINTER(vp)]
    L.fks_plan_destroy.argtypes = [vp]
    L.fks_plan_query.argtypes = [vp, C.POINTER(PlanInfo)]
    L.fks_plan_copy_tables.argtypes = [vp, vp, vp]
    L.fks_workspace_size.argtypes = [C.POINTER(Segment), i32, C.POINTER(sz)]
    L.fks_collide_batch.argtypes = [C.POINTER(Segment), i32, vp, sz, vp]
    L.fks_collide_batch_static.argtypes = [C.POINTER(Segment), i32, vp]
    L.fks_stable_dt.argtypes = [dbl, dbl, dbl, dbl, dbl, dbl, dbl, C.POINTER(dbl)]
    L.fks_exp_euler_step.argtypes = [dbl, dbl, C.POINTER(dbl)]
    L.fks_moments.argtypes = [vp, i64, i32, dbl, vp, vp]
    L.fks_conserve.argtypes = [vp, vp, i64, i32, dbl, vp]
    L.fks_transport_shift.argtypes = [vp, vp, C.POINTER(SpaceDesc), i32, dbl, dbl, vp, vp, vp]
    L.fks_status_string.argtypes = [i32]
    L.fks_status_string.restype = C.c_char_p
    L.fks_desc_validate.argtypes = [C.POINTER(PlanDesc)]
    L.fks_host_sphere_rule.argtypes = [i32, i32, i32, vp]
    L.fks_host_radial_terms.argtypes = [dbl, dbl, i32, dbl, i32, C.POINTER(i32), vp, vp]
    L.fks_profile_enable.argtypes = [i32]
    L.fks_profile_last.argtypes = [vp, i32, C.POINTER(i32)]
    L.fks_host_tables_2d.argtypes = [C.POINTER(PlanDesc), C.POINTER(i32), vp]
    L.fks_bgk.argtypes = [C.POINTER(BgkDesc), vp, vp, vp, i64, dbl, vp]
    L.fks_spectrum_workspace_size.argtypes = [i64, i32, C.POINTER(sz)]
    L.fks_spectrum.argtypes = [vp, vp, i64, i32, i32, vp, sz, vp]
    L.fks_numeric_status.argtypes = [vp, C.POINTER(i64), i32]
    L.fks_autotune_workspace_size.argtypes = [C.POINTER(Segment), i32, C.POINTER(sz)]
    L.fks_autotune.argtypes = [C.POINTER(Segment), i32, vp, sz, vp, vp]
    L.fks_halo_size.argtypes = [C.POINTER(SpaceDesc), i32, i32, C.POINTER(sz)]
    L.fks_halo_pack.argtypes = [vp, C.POINTER(SpaceDesc), i32, i32, vp, vp]
    L.fks_transport_shift_slab.argtypes = [vp, vp, C.POINTER(SpaceDesc), i32, dbl, dbl, vp, vp, vp, vp, vp]
    for name in EXPORTED:
        if name != "fks_status_string":
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


class FksError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {lib().fks_status_string(status).decode()} ({status})")


def _check(status: int, what: str) -> None:
    if status != FKS_OK:
        raise FksError(status, what)


def _stream_ptr(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int | None:
    if t is None:
        return None
    return int(t.data_ptr())


def _require_device_f64(t, name: str, numel: int | None = None):
    import torch
    if t is None:
        return
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous float64")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


@dataclass
class Desc:
    """Operator description, mirrors fks_plan_desc (defaults resolved by the library)."""
    n: int
    T: float
    gamma: float = 1.0
    R: float = 0.0
    c_gamma: float = 0.0
    n_polar: int = 8
    n_azim: int = 4
    rule: int = RULE_GAUSS
    radial_terms: int = 0
    radial_tol: float = 0.0
    precision: int = PREC_F32_FIX64
    flags: int = 0
    dim: int = 3

    def c(self) -> PlanDesc:
        return PlanDesc(self.n, self.T, self.R, self.gamma, self.c_gamma, self.n_polar, self.n_azim,
                        self.rule, self.radial_terms, self.radial_tol, self.precision, self.flags,
                        self.dim)


def desc2d(n: int, T: float, A: int = 8, precision: int = PREC_F32_FIX64, R: float = 0.0,
           c0: float = 0.0) -> Desc:
    """Two-dimensional Maxwell molecules with A angles (fks_plan_desc with dim = 2)."""
    return Desc(n=n, T=T, gamma=0.0, R=R, c_gamma=c0, n_polar=A, n_azim=1, precision=precision, dim=2)


def desc_validate(d: Desc) -> int:
    cd = d.c()
    return lib().fks_desc_validate(C.byref(cd))


class Plan:
    """Owns an fks_plan (device tables).  Use as a context manager or call close()."""

    def __init__(self, desc: Desc, stream=None):
        self.desc = desc
        h = C.c_void_p()
        cd = desc.c()
        _check(lib().fks_plan_create(C.byref(cd), C.c_void_p(_stream_ptr(stream)), C.byref(h)),
               "fks_plan_create")
        self._h = h
        self._info = self._query()

    def _query(self) -> "PlanInfo":
        info = PlanInfo()
        _check(lib().fks_plan_query(self.handle, C.byref(info)), "fks_plan_query")
        return info

    @property
    def info(self) -> "PlanInfo":
        """fks_plan_query: the fields fixed at creation, and the work-queue knob that
        fks_autotune may change (queue_items_per_wg), queried again on each access."""
        if self._h is None:
            return self._info
        self._info = self._query()
        return self._info

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan is closed")
        return self._h

    @property
    def n(self) -> int:
        return self._info.n

    @property
    def dim(self) -> int:
        return self._info.dim

    @property
    def cell_size(self) -> int:
        """Velocity nodes per cell: n^dim."""
        return self._info.n ** self._info.dim

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().fks_plan_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        # at interpreter exit the HIP runtime (or a profiler wrapped around it) may already be
        # finalised: a plan still open then is left to the process teardown (module globals such
        # as sys may already be gone, hence the broad guard)
        try:
            if sys.is_finalizing():
                return
            self.close()
        except Exception:
            pass

    def numeric_status(self, reset: bool = True) -> int:
        """First cell (within its segment) whose Q_c was not finite since the last reset,
        or -1 (plans created with FLAG_NUMERIC_GUARD; synchronises the device)."""
        cell = C.c_int64(-1)
        st = lib().fks_numeric_status(self.handle, C.byref(cell), 1 if reset else 0)
        if st not in (FKS_OK, FKS_ERR_NUMERIC):
            _check(st, "fks_numeric_status")
        return int(cell.value)

    def tables(self):
        """(ab FP64 numpy, dirs [M, 4]) copied from the device; ab is [J, n/2+1, n, n, 2]
        for dim = 3 and [J, n, n, 2] for dim = 2."""
        import numpy as np
        n, J, M = self.info.n, self.info.J, self.info.M
        shape = (J, n, n, 2) if self.info.dim == 2 else (J, n // 2 + 1, n, n, 2)
        ab = np.empty(shape, dtype=np.float64)
        dirs = np.empty((M, 4), dtype=np.float64)
        _check(lib().fks_plan_copy_tables(self.handle, ab.ctypes.data, dirs.ctypes.data),
               "fks_plan_copy_tables")
        return ab, dirs


def _segment_fields(item):
    """(plan, f, q_out, f_out, ncell, dt_over_tau[, f_base]) -> the seven fields."""
    if len(item) == 6:
        return tuple(item) + (None,)
    return tuple(item)


def _segments(items):
    arr = (Segment * len(items))()
    for i, item in enumerate(items):
        plan, f, q_out, f_out, ncell, dt, f_base = _segment_fields(item)
        arr[i] = Segment(plan.handle.value if plan is not None else None, _ptr(f), _ptr(q_out),
                         _ptr(f_out), ncell, dt, _ptr(f_base))
    return arr


def workspace_size(segments) -> int:
    """segments: list of (plan, f, q_out, f_out, ncell, dt_over_tau[, f_base])."""
    arr = _segments(segments)
    out = C.c_size_t()
    _check(lib().fks_workspace_size(arr, len(segments), C.byref(out)), "fks_workspace_size")
    return out.value


def collide_batch(segments, workspace=None, stream=None):
    """fks_collide_batch over segments (plan, f, q_out, f_out, ncell, dt_over_tau).

    ``workspace`` is a uint8 device tensor of at least workspace_size() bytes
    (the library rejects a smaller one); allocated here if None.  Returns the
    workspace tensor (reuse it).
    """
    import torch
    for item in segments:
        plan, f, q_out, f_out, ncell, dt, f_base = _segment_fields(item)
        nn = ncell * plan.cell_size
        _require_device_f64(f, "f", nn)
        _require_device_f64(q_out, "q_out", nn)
        _require_device_f64(f_out, "f_out", nn)
        _require_device_f64(f_base, "f_base", nn)
    if workspace is None:
        need = workspace_size(segments)
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
    arr = _segments(segments)
    _check(lib().fks_collide_batch(arr, len(segments), C.c_void_p(_ptr(workspace)), workspace.numel(),
                                   C.c_void_p(_stream_ptr(stream))), "fks_collide_batch")
    return workspace


def collide_batch_static(segments, stream=None) -> None:
    """fks_collide_batch_static: fks_collide_batch with the library's static per-GPU
    workspace (no allocation anywhere in the call).  Raises FksError(FKS_ERR_INVALID) when
    the segments need more than STATIC_WORKSPACE_BYTES.  Calls that overlap on one GPU
    share that workspace and race."""
    for item in segments:
        plan, f, q_out, f_out, ncell, dt, f_base = _segment_fields(item)
        nn = ncell * plan.cell_size
        _require_device_f64(f, "f", nn)
        _require_device_f64(q_out, "q_out", nn)
        _require_device_f64(f_out, "f_out", nn)
        _require_device_f64(f_base, "f_base", nn)
    arr = _segments(segments)
    _check(lib().fks_collide_batch_static(arr, len(segments), C.c_void_p(_stream_ptr(stream))),
           "fks_collide_batch_static")


def stable_dt(dx: float, T: float, tau: float, R: float, gamma: float, c_gamma: float, rho_max: float) -> float:
    """fks_stable_dt: min(dx/T, tau/mu), mu = 4 pi C_gamma (2R)^gamma rho_max."""
    out = C.c_double()
    _check(lib().fks_stable_dt(dx, T, tau, R, gamma, c_gamma, rho_max, C.byref(out)), "fks_stable_dt")
    return out.value


def exp_euler_step(mu: float, dt_over_tau: float) -> float:
    """fks_exp_euler_step: (1 - exp(-mu dt_over_tau)) / mu."""
    out = C.c_double()
    _check(lib().fks_exp_euler_step(mu, dt_over_tau, C.byref(out)), "fks_exp_euler_step")
    return out.value


def autotune(segments, workspace=None, stream=None):
    """fks_autotune: times the schedules of every segment and keeps the fastest in its plan
    (for the same ncell).  The segments are evaluated several times, so their f_out must not
    overlap f or f_base.  Returns [(one, chunk, terms)] per segment: one = 1 (one workgroup
    per cell), 0 (pairs) or -1 (not a fused plan); chunk = cells per pass batch and terms =
    consecutive terms per launch of the multi-pass path, or 0."""
    import torch
    for item in segments:
        plan, f, q_out, f_out, ncell, dt, f_base = _segment_fields(item)
        nn = ncell * plan.cell_size
        _require_device_f64(f, "f", nn)
        _require_device_f64(q_out, "q_out", nn)
        _require_device_f64(f_out, "f_out", nn)
        _require_device_f64(f_base, "f_base", nn)
    arr = _segments(segments)
    if workspace is None:
        need = C.c_size_t()
        _check(lib().fks_autotune_workspace_size(arr, len(segments), C.byref(need)), "fks_autotune_workspace_size")
        workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device="cuda")
    choice = (C.c_int32 * (3 * max(len(segments), 1)))()
    _check(lib().fks_autotune(arr, len(segments), C.c_void_p(_ptr(workspace)), workspace.numel(),
                              C.c_void_p(_stream_ptr(stream)), choice), "fks_autotune")
    return [tuple(int(choice[3 * i + k]) for k in range(3)) for i in range(len(segments))]


def collide(plan: Plan, f, q_out=None, f_out=None, dt_over_tau: float = 0.0, workspace=None, stream=None,
            f_base=None):
    """Single-segment convenience wrapper; f is [ncell, n, n, n] (dim 3) or [ncell, n, n]
    (dim 2) float64 on the GPU.  f_out = f_base + dt_over_tau Q_c(f) (f_base defaults to f)."""
    ncell = f.numel() // plan.cell_size
    return collide_batch([(plan, f, q_out, f_out, ncell, dt_over_tau, f_base)], workspace, stream)


def moments(f, n: int, T: float, U=None, stream=None):
    """U[ncell, 5] = dv^3 sum f (1, v, |v|^2) (FP64, device)."""
    import torch
    ncell = f.numel() // n ** 3
    _require_device_f64(f, "f", ncell * n ** 3)
    if U is None:
        U = torch.empty((ncell, 5), dtype=torch.float64, device=f.device)
    _require_device_f64(U, "U", ncell * 5)
    _check(lib().fks_moments(C.c_void_p(_ptr(f)), ncell, n, T, C.c_void_p(_ptr(U)),
                             C.c_void_p(_stream_ptr(stream))), "fks_moments")
    return U


def conserve(f, U, n: int, T: float, stream=None):
    """In-place projection of every cell of f onto the moments U (eq. minim1)."""
    ncell = f.numel() // n ** 3
    _require_device_f64(f, "f", ncell * n ** 3)
    _require_device_f64(U, "U", ncell * 5)
    _check(lib().fks_conserve(C.c_void_p(_ptr(f)), C.c_void_p(_ptr(U)), ncell, n, T,
                              C.c_void_p(_stream_ptr(stream))), "fks_conserve")
    return f


def transport_shift(f_in, f_out, nx: int, ny: int, nz: int, dx: float, bc, n: int, T: float,
                    dt: float, offsets, bc_f=None, stream=None):
    """FKS transport step f_in -> f_out; offsets is a host float64 numpy array [3, n] (updated)."""
    import numpy as np
    total = nx * ny * nz * n ** 3
    _require_device_f64(f_in, "f_in", total)
    _require_device_f64(f_out, "f_out", total)
    if bc_f is not None:
        _require_device_f64(bc_f, "bc_f", 6 * n ** 3)
    if not (isinstance(offsets, np.ndarray) and offsets.dtype == np.float64 and offsets.size == 3 * n
            and offsets.flags.c_contiguous):
        raise ValueError("offsets must be a contiguous float64 numpy array of 3*n values")
    sp = SpaceDesc(nx, ny, nz, dx, (C.c_int32 * 3)(*bc))
    _check(lib().fks_transport_shift(C.c_void_p(_ptr(f_in)), C.c_void_p(_ptr(f_out)), C.byref(sp), n, T, dt,
                                     C.c_void_p(offsets.ctypes.data), C.c_void_p(_ptr(bc_f)),
                                     C.c_void_p(_stream_ptr(stream))), "fks_transport_shift")


def halo_size(nx: int, ny: int, nz: int, n: int, face: int) -> int:
    """Bytes of the message that leaves a z slab of nz owned planes through `face`."""
    sp = SpaceDesc(nx, ny, nz, 1.0, (C.c_int32 * 3)(BC_PERIODIC, BC_PERIODIC, BC_PERIODIC))
    out = C.c_size_t(0)
    _check(lib().fks_halo_size(C.byref(sp), n, face, C.byref(out)), "fks_halo_size")
    return out.value


def halo_pack(f, buf, nx: int, ny: int, nz: int, n: int, face: int, stream=None):
    """Packs the velocities leaving the slab f [nz, ny, nx, n^3] through `face` into buf."""
    _require_device_f64(f, "f", nz * nx * ny * n ** 3)
    _require_device_f64(buf, "buf", halo_size(nx, ny, nz, n, face) // 8)
    sp = SpaceDesc(nx, ny, nz, 1.0, (C.c_int32 * 3)(BC_PERIODIC, BC_PERIODIC, BC_PERIODIC))
    _check(lib().fks_halo_pack(C.c_void_p(_ptr(f)), C.byref(sp), n, face, C.c_void_p(_ptr(buf)),
                               C.c_void_p(_stream_ptr(stream))), "fks_halo_pack")


def transport_shift_slab(f_in, f_out, nx: int, ny: int, nz: int, dx: float, bc_xy, n: int, T: float,
                         dt: float, offsets, from_below, from_above, bc_f=None, stream=None):
    """Transport step of a z slab, f_in -> f_out (both [nz, ny, nx, n^3]); what enters through the
    z faces comes from the messages the neighbours packed (from_below: the slab below's z+ message,
    from_above: the slab above's z- message).  offsets as in transport_shift (updated)."""
    import numpy as np
    total = nz * nx * ny * n ** 3
    _require_device_f64(f_in, "f_in", total)
    _require_device_f64(f_out, "f_out", total)
    _require_device_f64(from_below, "from_below", halo_size(nx, ny, nz, n, FACE_ZHI) // 8)
    _require_device_f64(from_above, "from_above", halo_size(nx, ny, nz, n, FACE_ZLO) // 8)
    if bc_f is not None:
        _require_device_f64(bc_f, "bc_f", 6 * n ** 3)
    if not (isinstance(offsets, np.ndarray) and offsets.dtype == np.float64 and offsets.size == 3 * n
            and offsets.flags.c_contiguous):
        raise ValueError("offsets must be a contiguous float64 numpy array of 3*n values")
    sp = SpaceDesc(nx, ny, nz, dx, (C.c_int32 * 3)(bc_xy[0], bc_xy[1], BC_PERIODIC))
    _check(lib().fks_transport_shift_slab(C.c_void_p(_ptr(f_in)), C.c_void_p(_ptr(f_out)), C.byref(sp),
                                          n, T, dt, C.c_void_p(offsets.ctypes.data), C.c_void_p(_ptr(from_below)),
                                          C.c_void_p(_ptr(from_above)), C.c_void_p(_ptr(bc_f)),
                                          C.c_void_p(_stream_ptr(stream))), "fks_transport_shift_slab")


def bgk(f, n: int, T: float, nu: float, dim: int = 3, q_out=None, f_out=None, dt_over_tau: float = 0.0,
        nu_rho: bool = False, step: int = BGK_EULER, stream=None):
    """BGK relaxation with the conservative discrete Maxwellian (fks_bgk); f is
    [ncell, n^dim] float64 on the GPU (any shape with that many elements)."""
    cs = n ** dim
    ncell = f.numel() // cs
    _require_device_f64(f, "f", ncell * cs)
    _require_device_f64(q_out, "q_out", ncell * cs)
    _require_device_f64(f_out, "f_out", ncell * cs)
    d = BgkDesc(dim, n, T, nu, 1 if nu_rho else 0, step)
    _check(lib().fks_bgk(C.byref(d), C.c_void_p(_ptr(f)), C.c_void_p(_ptr(q_out)), C.c_void_p(_ptr(f_out)),
                         ncell, dt_over_tau, C.c_void_p(_stream_ptr(stream))), "fks_bgk")


def bgk_validate(dim: int, n: int, T: float, nu: float, nu_rho: int = 0, step: int = BGK_EULER,
                 dt_over_tau: float = 0.0) -> int:
    """Status of fks_bgk on an empty batch (argument validation only, no device work)."""
    d = BgkDesc(dim, n, T, nu, nu_rho, step)
    return lib().fks_bgk(C.byref(d), None, None, None, 0, dt_over_tau, None)


def spectrum(x, n: int, xhat=None, zero_nyquist: bool = False, workspace=None, stream=None):
    """xhat[ncell, n, n, n/2+1] complex128 = n^-3 sum_j x_j exp(-i kappa k.v_j) (fks_spectrum);
    x is [ncell, n, n, n] float64 on the GPU."""
    import torch
    ncell = x.numel() // n ** 3
    _require_device_f64(x, "x", ncell * n ** 3)
    if xhat is None:
        xhat = torch.empty((ncell, n, n, n // 2 + 1), dtype=torch.complex128, device=x.device)
    if not (isinstance(xhat, torch.Tensor) and xhat.is_cuda and xhat.dtype == torch.complex128
            and xhat.is_contiguous() and xhat.numel() == ncell * n * n * (n // 2 + 1)):
        raise ValueError("xhat must be a contiguous complex128 GPU tensor of ncell*n*n*(n/2+1) elements")
    if workspace is None:
        need = C.c_size_t()
        _check(lib().fks_spectrum_workspace_size(ncell, n, C.byref(need)), "fks_spectrum_workspace_size")
        workspace = torch.empty(max(need.value, 1), dtype=torch.uint8, device=x.device)
    _check(lib().fks_spectrum(C.c_void_p(_ptr(x)), C.c_void_p(_ptr(xhat)), ncell, n, 1 if zero_nyquist else 0,
                              C.c_void_p(_ptr(workspace)), workspace.numel(), C.c_void_p(_stream_ptr(stream))),
           "fks_spectrum")
    return xhat


def profile_enable(on: bool = True) -> None:
    _check(lib().fks_profile_enable(1 if on else 0), "fks_profile_enable")


def profile_last() -> list:
    """Durations (ms) of the kernels of the last fks_collide_batch call (fused path)."""
    import numpy as np
    out = np.zeros(8, dtype=np.float64)
    cnt = C.c_int32()
    _check(lib().fks_profile_last(out.ctypes.data, 8, C.byref(cnt)), "fks_profile_last")
    return [float(x) for x in out[:cnt.value]]


def host_sphere_rule(n_polar: int, n_azim: int, rule: int = RULE_GAUSS):
    import numpy as np
    out = np.empty((n_polar * n_azim, 4), dtype=np.float64)
    _check(lib().fks_host_sphere_rule(n_polar, n_azim, rule, out.ctypes.data), "fks_host_sphere_rule")
    return out


def host_tables_2d(d: Desc):
    """FP64 tables a dim = 2 plan uploads: [J, n, n, 2] (host computation, no GPU)."""
    import numpy as np
    cd = d.c()
    J = C.c_int32()
    _check(lib().fks_host_tables_2d(C.byref(cd), C.byref(J), None), "fks_host_tables_2d")
    ab = np.empty((J.value, d.n, d.n, 2), dtype=np.float64)
    _check(lib().fks_host_tables_2d(C.byref(cd), C.byref(J), ab.ctypes.data), "fks_host_tables_2d")
    return ab


def host_radial_terms(gamma: float, R: float, K: int = 0, tol: float = 1e-4, nq: int = 200):
    import numpy as np
    k = C.c_int32()
    _check(lib().fks_host_radial_terms(gamma, R, K, tol, nq, C.byref(k), None, None), "fks_host_radial_terms")
    nodes = np.empty(nq, dtype=np.float64)
    coef = np.empty((nq, k.value), dtype=np.float64)
    _check(lib().fks_host_radial_terms(gamma, R, k.value, tol, nq, C.byref(k), nodes.ctypes.data,
                                       coef.ctypes.data), "fks_host_radial_terms")
    return k.value, nodes, coef
