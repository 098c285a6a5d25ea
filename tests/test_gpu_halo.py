"""z-slab decomposition of the transport step (Section 4.2), emulated on one GPU.

The grid is cut into slabs of consecutive z planes.  Every step, each slab
packs the velocities leaving through its two z faces, and each slab runs the
slab transport, which takes what enters through its faces from the messages
of the neighbours below and above.  The slabs must equal the whole-grid
transport bit for bit (the step only moves values), against the oracle at
small sizes and against the library's whole-grid call at the shape of one
GPU's share of the 32^3 x 24^3 flow."""
import math

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_1608_08009_amd as fks  # noqa: E402
import oracle as O  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _message_range(n, face):
    # kz of the velocities that leave through a face: v_z < 0 through z-, v_z > 0 through z+
    return (0, (n + 1) // 2) if face == fks.FACE_ZLO else (n // 2 + 1, n - 1 - n // 2)


class Slabs:
    """The slabs of one grid on one GPU, wired as neighbours along a periodic z axis."""

    def __init__(self, f_global, sizes, nx, ny, n):
        self.nx, self.ny, self.n, self.sizes = nx, ny, n, sizes
        z0 = np.concatenate([[0], np.cumsum(sizes)[:-1]])
        self.a = [f_global[z:z + nz].reshape(nz, ny, nx, n ** 3).clone() for z, nz in zip(z0, sizes)]
        self.b = [torch.full_like(a, math.nan) for a in self.a]
        self.msg = [{f: torch.full((fks.halo_size(nx, ny, nz, n, f) // 8,), math.nan, dtype=torch.float64,
                                   device="cuda")
                     for f in (fks.FACE_ZLO, fks.FACE_ZHI)} for nz in sizes]

    def step(self, dx, bc_xy, T, dt, offsets, bc_f):
        S = len(self.sizes)
        for s, nz in enumerate(self.sizes):
            for face in (fks.FACE_ZLO, fks.FACE_ZHI):
                fks.halo_pack(self.a[s], self.msg[s][face], self.nx, self.ny, nz, self.n, face)
        for s, nz in enumerate(self.sizes):
            below, above = (s - 1) % S, (s + 1) % S
            # what the slab below sent up enters through z-; what the slab above sent down, through z+
            fks.transport_shift_slab(self.a[s], self.b[s], self.nx, self.ny, nz, dx, bc_xy, self.n, T, dt,
                                     offsets[s], self.msg[below][fks.FACE_ZHI], self.msg[above][fks.FACE_ZLO],
                                     bc_f=bc_f)
        self.a, self.b = self.b, self.a

    def owned(self):
        return torch.cat(self.a)


@pytest.mark.parametrize("n,sizes,bc_xy", [(4, (3, 1, 3), (fks.BC_DIRICHLET, fks.BC_PERIODIC)),
                                           (5, (2, 2, 1, 2), (fks.BC_PERIODIC, fks.BC_DIRICHLET)),
                                           (6, (7,), (fks.BC_PERIODIC, fks.BC_PERIODIC)),
                                           (16, (1, 2), (fks.BC_DIRICHLET, fks.BC_DIRICHLET))])
def test_slabs_reproduce_the_whole_grid_transport(n, sizes, bc_xy):
    T, nx, ny = 2.0, 3, 2
    nz = sum(sizes)
    dx = 1.0 / nx
    dt = 0.93 * dx / T
    rng = synth.rng(90 + n)
    f0 = rng.uniform(size=(nz, ny, nx, n, n, n))
    bcf = rng.uniform(size=(6, n, n, n)) + 10.0
    names = tuple("dirichlet" if b else "periodic" for b in bc_xy) + ("periodic",)
    slabs = Slabs(_dev(f0), sizes, nx, ny, n)
    offsets = [np.zeros((3, n)) for _ in sizes]
    whole_a = _dev(f0)
    whole_b = torch.empty_like(whole_a)
    off_whole = np.zeros((3, n))
    off_or = np.zeros((3, n))
    ref = f0.copy()
    for step in range(7):
        slabs.step(dx, bc_xy, T, dt, offsets, _dev(bcf))
        fks.transport_shift(whole_a, whole_b, nx, ny, nz, dx, bc_xy + (fks.BC_PERIODIC,), n, T, dt, off_whole,
                            bc_f=_dev(bcf))
        whole_a, whole_b = whole_b, whole_a
        off_or, s = O.transport_offsets_step(off_or, n, T, dx, dt)
        ref = O.transport_shift(ref, s, n, bc=names, bc_f=bcf)
        got = slabs.owned()
        assert torch.equal(got, whole_a.reshape(got.shape)), f"step {step}"
    torch.cuda.synchronize()
    for off in offsets:
        assert np.array_equal(off, off_or)
    assert np.array_equal(slabs.owned().cpu().numpy().reshape(ref.shape), ref)


@pytest.mark.parametrize("n", [4, 5, 24])
def test_pack_layout(n):
    nx, ny, nz = 3, 2, 3
    rng = synth.rng(95)
    f = _dev(rng.uniform(size=(nz, ny, nx, n, n, n)))
    host = f.cpu().numpy()
    for face, plane in ((fks.FACE_ZLO, 0), (fks.FACE_ZHI, nz - 1)):
        k0, h = _message_range(n, face)
        assert fks.halo_size(nx, ny, nz, n, face) == ny * nx * n * n * h * 8
        buf = torch.full((ny * nx * n * n * h,), math.nan, dtype=torch.float64, device="cuda")
        fks.halo_pack(f, buf, nx, ny, nz, n, face)
        assert np.array_equal(buf.cpu().numpy(), host[plane][..., k0:k0 + h].reshape(-1))


def test_slab_transport_rejects_shifts_the_messages_do_not_hold():
    n, T, nx, ny, nz = 4, 2.0, 3, 2, 2
    dx = 1.0 / nx
    a = torch.zeros((nz, ny, nx, n ** 3), dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)
    lo = torch.zeros(fks.halo_size(nx, ny, nz, n, fks.FACE_ZLO) // 8, dtype=torch.float64, device="cuda")
    hi = torch.zeros(fks.halo_size(nx, ny, nz, n, fks.FACE_ZHI) // 8, dtype=torch.float64, device="cuda")
    periodic = (fks.BC_PERIODIC, fks.BC_PERIODIC)
    for dt in (2.2 * dx / T, -0.5 * dx / T):   # a shift of two planes; v_z < 0 moving up
        off = np.zeros((3, n))
        with pytest.raises(fks.FksError):
            fks.transport_shift_slab(a, b, nx, ny, nz, dx, periodic, n, T, dt, off, hi, lo)
        assert not off.any()                   # offsets unchanged on error
    with pytest.raises(fks.FksError):          # overlapping buffers
        fks.transport_shift_slab(a, a, nx, ny, nz, dx, periodic, n, T, 0.5 * dx / T, np.zeros((3, n)), hi, lo)
    with pytest.raises(ValueError):            # message of the wrong face (size)
        fks.transport_shift_slab(a, b, nx, ny, nz, dx, periodic, n, T, 0.5 * dx / T, np.zeros((3, n)), lo, hi)
    assert torch.count_nonzero(b) == 0         # nothing was enqueued


def test_one_gpu_share_of_the_32cube_flow():
    # 32 x 32 cells per plane, 24^3 velocities, 8 slabs of 4 planes (one per GPU of 8):
    # the slab steps against the whole-grid call, and the periodic total mass
    n, T, nx, ny, sizes = 24, 8.0, 32, 32, (4,) * 8
    nz = sum(sizes)
    dx = 1.0 / nx
    dt = 0.6 * dx / T
    g = torch.Generator(device="cuda").manual_seed(1608080095)
    f0 = torch.rand((nz, ny, nx, n ** 3), dtype=torch.float64, device="cuda", generator=g)
    periodic = (fks.BC_PERIODIC, fks.BC_PERIODIC)
    slabs = Slabs(f0, sizes, nx, ny, n)
    offsets = [np.zeros((3, n)) for _ in sizes]
    whole_a, whole_b = f0.clone(), torch.empty_like(f0)
    off_whole = np.zeros((3, n))
    mass0 = f0.sum(dtype=torch.float64).item()
    del f0
    for _ in range(3):
        slabs.step(dx, periodic, T, dt, offsets, None)
        fks.transport_shift(whole_a, whole_b, nx, ny, nz, dx, periodic + (fks.BC_PERIODIC,), n, T, dt, off_whole)
        whole_a, whole_b = whole_b, whole_a
    got = slabs.owned()
    assert torch.equal(got, whole_a)
    assert abs(got.sum(dtype=torch.float64).item() - mass0) <= 1e-12 * mass0
    for off in offsets:
        assert np.array_equal(off, off_whole)


def test_transport_of_views_not_16_byte_aligned():
    # the shift kernel uses 16-byte accesses only for even n and 16-byte aligned arrays; views
    # offset by one double take the 8-byte path and must give the same result
    n, T, nx, ny, nz = 6, 2.0, 3, 2, 4
    dx = 1.0 / nx
    dt = 0.93 * dx / T
    total = nx * ny * nz * n ** 3
    rng = synth.rng(97)
    f0 = rng.uniform(size=total)
    bcf = rng.uniform(size=6 * n ** 3) + 10.0
    bc = (fks.BC_DIRICHLET, fks.BC_PERIODIC, fks.BC_DIRICHLET)
    a = _dev(f0)
    b = torch.empty_like(a)
    off = np.zeros((3, n))
    fks.transport_shift(a, b, nx, ny, nz, dx, bc, n, T, dt, off, bc_f=_dev(bcf))
    store_in = torch.empty(total + 1, dtype=torch.float64, device="cuda")
    store_out = torch.empty(total + 1, dtype=torch.float64, device="cuda")
    store_bc = torch.empty(6 * n ** 3 + 1, dtype=torch.float64, device="cuda")
    a1, b1, bc1 = store_in[1:], store_out[1:], store_bc[1:]
    assert a1.data_ptr() % 16 == 8
    a1.copy_(a)
    bc1.copy_(_dev(bcf))
    off1 = np.zeros((3, n))
    fks.transport_shift(a1, b1, nx, ny, nz, dx, bc, n, T, dt, off1, bc_f=bc1)
    assert torch.equal(b1, b)
    names = ("dirichlet", "periodic", "dirichlet")
    _, s = O.transport_offsets_step(np.zeros((3, n)), n, T, dx, dt)
    ref = O.transport_shift(f0.reshape(nz, ny, nx, n, n, n), s, n, bc=names, bc_f=bcf.reshape(6, n, n, n))
    assert np.array_equal(b.cpu().numpy(), ref.reshape(-1))
