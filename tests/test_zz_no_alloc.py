"""swfe_forces_static, the force evaluation that allocates nothing (its
scratch is the library's static device array), against the context path
(swfe_init_system + swfe_compute_forces, whose scratch is the caller's
workspace) through the C-ABI: forces, per-atom energies and the per-system
rows must agree bitwise, on two calls in a row where the second has a
smaller input (the array keeps the first call's contents), in both
precisions; inputs beyond the array are rejected before any work."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2103_10449_amd import inputs
from tests.gpu_helpers import betasn_spec, diamond_spec, force_err, liquid_spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swfe():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_10449_amd import swfe as m
    m.load_library()
    return m


def _force_only(specs):
    for s in specs:
        s.mode = inputs.MODE_FORCE
    return specs


def _context_path(swfe, specs, P, prec):
    eng = swfe.Engine(specs, P, precision=prec, want_e_atom=True)
    out = eng.compute_forces().cpu().numpy()
    res = (eng.f.cpu().numpy().copy(), eng.e_atom.cpu().numpy().copy(), out)
    eng.close()
    return res


def _static_path(swfe, specs, P, prec):
    import torch
    n = sum(s.n for s in specs)
    x = np.concatenate([s.x for s in specs]).T.copy()
    xd = torch.from_numpy(x).cuda()
    f = torch.full((3, n), np.nan, dtype=torch.float64, device="cuda")
    e = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    out = torch.full((len(specs), swfe.OUT_STRIDE), np.nan, dtype=torch.float64, device="cuda")
    swfe.forces_static(specs, P, xd, f, e, out, precision=prec)
    return f.cpu().numpy(), e.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_static_forces_equal_context_forces_twice(swfe, sw_params, prec):
    big = _force_only([diamond_spec(5, 130), liquid_spec(600, 131), betasn_spec(4, 132)])
    small = _force_only([diamond_spec(2, 133)])
    for k, specs in enumerate((big, small)):
        print(f"no-alloc {prec} call {k}: {len(specs)} systems, {sum(s.n for s in specs)} atoms", flush=True)
        fs, es, os_ = _static_path(swfe, specs, sw_params, prec)
        fc, ec, oc = _context_path(swfe, specs, sw_params, prec)
        assert np.array_equal(fs, fc)
        assert np.array_equal(es, ec)
        assert np.array_equal(os_, oc)
    # and the smaller call against the oracle (the array's previous contents
    # must not leak into it)
    ref = orc.sw_eval(small[0].x, small[0].box, sw_params)
    tol_f, tol_e = (1e-10, 1e-12) if prec == "fp64" else (1e-5, 1e-5)
    assert force_err(fs.T, ref["F"]) < tol_f
    assert abs(os_[0, 0] - ref["E"]) / small[0].n < tol_e


def test_static_forces_reject_inputs_beyond_the_scratch(swfe, sw_params):
    import torch
    xl, box = inputs.diamond((17, 17, 17), 5.431)      # 39304 atoms
    s = inputs.SystemSpec(x=xl, v=np.zeros_like(xl), box=box, mode=inputs.MODE_FORCE)
    x = torch.from_numpy(xl.T.copy()).cuda()
    f = torch.zeros_like(x)
    with pytest.raises(swfe.SwfeError) as ei:
        swfe.forces_static([s], sw_params, x, f)
    assert ei.value.code == swfe.E_NOMEM
    assert "static scratch" in str(ei.value)
    assert float(f.abs().max()) == 0.0
