"""The numeric guard (FKS_FLAG_NUMERIC_GUARD) on every collision path: a plan
created with the flag records the first cell whose Q_c is not finite, the
other cells are unaffected (each cell's result depends on that cell's data
only), and a reset clears the record."""
import math

import pytest

import synth

torch = pytest.importorskip("torch")
import paper_1608_08009_amd as fks  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [
    ("fused_f32", lambda fl: fks.Desc(n=16, T=8.0, precision=fks.PREC_F32_FIX64, flags=fl), 3),
    ("fused_f32_n24", lambda fl: fks.Desc(n=24, T=8.0, precision=fks.PREC_F32_FIX64, flags=fl), 3),
    ("generic_f32", lambda fl: fks.Desc(n=16, T=8.0, precision=fks.PREC_F32_FIX64,
                                        flags=fl | fks.FLAG_FORCE_GENERIC), 3),
    ("generic_f64", lambda fl: fks.Desc(n=8, T=8.0, precision=fks.PREC_F64, flags=fl), 3),
    ("twod_f64", lambda fl: fks.Desc(n=16, T=6.0, gamma=0.0, n_polar=8, n_azim=1,
                                     precision=fks.PREC_F64, flags=fl, dim=2), 2),
    ("twod_f32", lambda fl: fks.Desc(n=32, T=9.0, gamma=0.0, n_polar=8, n_azim=1,
                                     precision=fks.PREC_F32_FIX64, flags=fl, dim=2), 2),
]


def _cells(dim, n, T, ncell, seed):
    if dim == 2:
        return torch.as_tensor(synth.two_maxwellian_cells_2d(n, T, ncell, seed_offset=seed), device="cuda")
    return torch.as_tensor(synth.two_maxwellian_cells(n, T, ncell, seed_offset=seed), device="cuda")


@pytest.mark.parametrize("name,make,dim", CASES, ids=[c[0] for c in CASES])
def test_guard_records_first_bad_cell(name, make, dim):
    d = make(fks.FLAG_NUMERIC_GUARD)
    ncell = 11
    clean = _cells(dim, d.n, d.T, ncell, 170)
    bad = clean.clone()
    bad[7].view(-1)[5] = math.nan
    bad[4].view(-1)[0] = math.inf
    with fks.Plan(d) as plan, fks.Plan(make(0)) as plain:
        q_ref = torch.empty_like(clean)
        fks.collide(plain, clean, q_out=q_ref)
        q = torch.empty_like(clean)
        fks.collide(plan, clean, q_out=q)
        assert plan.numeric_status() == -1
        assert torch.equal(q, q_ref)                       # the guard changes no result
        fks.collide(plan, bad, q_out=q)
        assert plan.numeric_status(reset=False) == 4
        assert plan.numeric_status(reset=True) == 4
        assert plan.numeric_status() == -1                 # cleared by the reset
        assert not torch.isfinite(q[4]).all() and not torch.isfinite(q[7]).all()
        good = [c for c in range(ncell) if c not in (4, 7)]
        assert torch.equal(q[good], q_ref[good])           # other cells are unaffected
        # a batch of one bad cell at the end of a segment; f_out alone also triggers the record
        tail = bad[7:]
        g = torch.empty_like(tail)
        fks.collide(plan, tail, f_out=g, dt_over_tau=0.01)
        assert plan.numeric_status() == 0
        # a plan without the flag has no guard word
        with pytest.raises(fks.FksError):
            plain.numeric_status()
