"""Differentiation (step a10): the energy as a torch.autograd.Function whose
backward kernel returns forces, the 3x3 virial dE/dstrain and dE/dtheta,
checked against the FP64 oracle and central finite differences (h = 1e-5)
on the 32768-atom diamond at the 1700 K-like amplitude, FP64 and mixed."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2103_10449_amd import inputs
from tests.gpu_helpers import liquid_spec

pytestmark = pytest.mark.gpu

H = 1e-5


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def c5(sw_params):
    s = inputs.config5().systems[0]
    return s, orc.sw_eval(s.x, s.box, sw_params)


def _setup(torch_mod, specs, sw_params, precision):
    from paper_2103_10449_amd import swfe
    from paper_2103_10449_amd.autograd import theta_of
    eng = swfe.Engine(specs, sw_params, precision=precision)
    x = eng.x.clone().requires_grad_(True)
    strain = torch_mod.zeros((len(specs), 3, 3), dtype=torch_mod.float64, requires_grad=True)
    theta = theta_of(sw_params).requires_grad_(True)
    return eng, x, strain, theta


def test_backward_matches_oracle_fp64(torch_mod, sw_params, c5):
    from paper_2103_10449_amd.autograd import sw_energy
    s, ref = c5
    eng, x, strain, theta = _setup(torch_mod, [s], sw_params, "fp64")
    E = sw_energy(x, strain, theta, eng)
    assert E.item() == pytest.approx(ref["E"], rel=1e-12)
    E.sum().backward()
    F = -x.grad.cpu().numpy().T
    fs = max(np.abs(ref["F"]).max(), 1.0)
    assert np.abs(F - ref["F"]).max() / fs < 1e-10
    assert np.abs(strain.grad[0].cpu().numpy() - ref["virial"]).max() < 1e-9 * max(1, np.abs(ref["virial"]).max())
    assert np.allclose(theta.grad.numpy(), ref["dtheta"], rtol=1e-10, atol=1e-7)
    eng.close()


def test_finite_differences_fp64(torch_mod, sw_params, c5):
    """Central differences of the GPU energy: positions (sampled atoms),
    diagonal strains and every SW parameter."""
    from paper_2103_10449_amd.autograd import sw_energy
    torch = torch_mod
    s, _ = c5
    eng, x, strain, theta = _setup(torch, [s], sw_params, "fp64")
    E = sw_energy(x, strain, theta, eng)
    E.sum().backward()
    gx, gs, gt = x.grad.clone(), strain.grad.clone(), theta.grad.clone()

    def energy(xx=None, ss=None, tt=None):
        with torch.no_grad():
            return sw_energy(x.detach() if xx is None else xx, strain.detach() if ss is None else ss,
                             theta.detach() if tt is None else tt, eng).item()

    idx = inputs.rng(5, 0, 11).choice(s.n, 12, replace=False)
    gmax = max(gx.abs().max().item(), 1.0)
    for i in idx:
        for a in range(3):
            xp = x.detach().clone()
            xm = x.detach().clone()
            xp[a, i] += H
            xm[a, i] -= H
            fd = (energy(xx=xp) - energy(xx=xm)) / (2 * H)
            # total-energy differences carry eps * |E| / h ~ 2e-6 eV/A of rounding
            assert abs(fd - gx[a, i].item()) < 1e-5 * gmax
    for a in range(3):
        sp = torch.zeros_like(strain.detach())
        sm = torch.zeros_like(strain.detach())
        sp[0, a, a] = H
        sm[0, a, a] = -H
        fd = (energy(ss=sp) - energy(ss=sm)) / (2 * H)
        assert fd == pytest.approx(gs[0, a, a].item(), rel=1e-6, abs=2e-2)
    for k in range(9):
        h = H * max(1.0, abs(theta[k].item()))
        tp = theta.detach().clone()
        tm = theta.detach().clone()
        tp[k] += h
        tm[k] -= h
        fd = (energy(tt=tp) - energy(tt=tm)) / (2 * h)
        assert fd == pytest.approx(gt[k].item(), rel=1e-6, abs=5e-3), k
    eng.close()


def test_mixed_precision_gradients_vs_fp64(torch_mod, sw_params, c5):
    """FP32 terms with FP64 accumulation: forces within 1e-5 relative of the
    oracle, virial and dE/dtheta within 1e-5 of their scale."""
    from paper_2103_10449_amd.autograd import sw_energy
    s, ref = c5
    eng, x, strain, theta = _setup(torch_mod, [s], sw_params, "mixed")
    E = sw_energy(x, strain, theta, eng)
    E.sum().backward()
    F = -x.grad.cpu().numpy().T
    fs = max(np.abs(ref["F"]).max(), 1.0)
    ferr = np.abs(F - ref["F"]).max() / fs
    verr = np.abs(strain.grad[0].cpu().numpy() - ref["virial"]).max() / np.abs(ref["virial"]).max()
    terr = np.abs(theta.grad.numpy() - ref["dtheta"]) / np.maximum(np.abs(ref["dtheta"]), 1.0)
    print(f"mixed: energy err {(E.item() - ref['E']) / s.n:.2e} eV/atom, force {ferr:.2e}, "
          f"virial {verr:.2e}, dtheta {terr.max():.2e}", flush=True)
    assert ferr < 1e-5
    assert abs(E.item() - ref["E"]) / s.n < 1e-5
    assert verr < 1e-4
    assert terr.max() < 1e-4
    eng.close()


def test_upstream_gradient_scales_each_system(torch_mod, sw_params):
    """Two systems in one call: dL/dx of L = sum_s w_s E_s is w_s times the
    single-system gradient, and dL/dtheta sums over systems."""
    from paper_2103_10449_amd.autograd import sw_energy
    torch = torch_mod
    a, b = liquid_spec(300, 150), liquid_spec(200, 151)
    eng, x, strain, theta = _setup(torch, [a, b], sw_params, "fp64")
    w = torch.tensor([2.5, -0.5], dtype=torch.float64, device=eng.device)
    E = sw_energy(x, strain, theta, eng)
    (E * w).sum().backward()
    ra, rb = orc.sw_eval(a.x, a.box, sw_params), orc.sw_eval(b.x, b.box, sw_params)
    gx = x.grad.cpu().numpy().T
    assert np.allclose(gx[:300], -2.5 * ra["F"], atol=1e-10)
    assert np.allclose(gx[300:], 0.5 * rb["F"], atol=1e-10)
    assert np.allclose(strain.grad[0].cpu().numpy(), 2.5 * ra["virial"], atol=1e-9)
    assert np.allclose(theta.grad.numpy(), 2.5 * ra["dtheta"] - 0.5 * rb["dtheta"], rtol=1e-10, atol=1e-8)
    eng.close()
