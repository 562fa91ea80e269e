"""Uhlenbeck-Ford fluid reference (section 4.1, p = 25, sigma = 2 A) on the
GPU: the reference energy against the oracle, switching trajectories
against the oracle, and the free energy of switching a dilute ideal gas on
to the UF fluid against the second-virial closed form."""
import copy

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2103_10449_amd import inputs
from tests.gpu_helpers import liquid_spec, to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swfe():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_10449_amd import swfe as m
    m.load_library()
    return m


def _uf_liquid(n, seed, T=2200.0, **kw):
    return liquid_spec(n, seed, T=T, mode=inputs.MODE_UF, T0=T, tau_damp=0.1, uf_p=inputs.UF_P,
                       uf_sigma=inputs.UF_SIGMA, uf_T=T, uf_rcut=inputs.UF_RCUT, **kw)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-6)])
def test_uf_reference_energy_matches_oracle(swfe, sw_params, precision, tol):
    s = _uf_liquid(500, 80, stream=1)
    eng = swfe.Engine([s], sw_params, seed=1, precision=precision)
    out = eng.compute_forces().cpu().numpy()[0]
    ref = orc.uf_eval(s.x, s.box, s.uf_p, s.uf_sigma, s.uf_T, s.uf_rcut)
    print(f"{precision}: U_UF {out[1]:.10f} vs {ref['E']:.10f}", flush=True)
    assert abs(out[1] - ref["E"]) / s.n < tol * max(1.0, abs(ref["E"]) / s.n)
    eng.close()


def test_uf_switching_trajectory_matches_oracle(swfe, sw_params):
    """lambda 1 -> 0 (SW liquid to UF fluid) over 200 steps next to a plain
    NVT system in the same launch: positions within 1e-9 A, work and U_ref
    to 1e-9."""
    a = _uf_liquid(400, 81, stream=2, sched_start=1.0, sched_end=0.0, sched_steps=200)
    b = liquid_spec(300, 82, mode=inputs.MODE_NVT, T0=1700.0, tau_damp=0.1, stream=3)
    specs = [a, b]
    eng = swfe.Engine(copy.deepcopy(specs), sw_params, dt=0.001, seed=13, precision="fp64")
    o = orc.Oracle([to_oracle(s) for s in specs], sw_params, dt=0.001, seed=13)
    eng.step(200)
    o.run(200)
    st = eng.state()
    for k, s in enumerate(o.systems):
        dx = np.abs(eng.positions(k) - s.x).max()
        print(f"sys {k}: dx {dx:.2e} W {st[k]['W']:.10f} vs {s.W:.10f} U_ref {st[k]['U_ref']:.8f} vs "
              f"{s.U_ref:.8f}", flush=True)
        assert dx < 1e-9
        assert abs(st[k]["W"] - s.W) <= 1e-9 * max(1.0, abs(s.W))
        assert st[k]["U_ref"] == pytest.approx(s.U_ref, rel=1e-10, abs=1e-10)
    assert st[0]["lam"] == 0.0
    eng.close()


def test_ideal_gas_to_uf_free_energy_second_virial(swfe, sw_params):
    """SW off (an ideal gas) switched on to the UF fluid at low density:
    Delta F = N kB T rho B2 (1 + O(rho B2)), B2 = 129.86 A^3 from the closed
    form; 64 replicas of 64 atoms at rho B2 = 0.03, 4000 steps each way
    (dt = 2 fs), 1/2 (W_fwd - W_bwd) per replica."""
    P = dict(sw_params)
    P["epsilon"] = 0.0
    from math import comb, fsum, pi
    B2 = pi ** 1.5 * 8.0 / 2 * fsum((-1) ** (k + 1) * comb(25, k) * k ** -1.5 for k in range(1, 26))
    N, T, rb = 64, 2200.0, 0.03
    L = (N * B2 / rb) ** (1 / 3)
    specs = []
    for r in range(64):
        g = inputs.rng(980, r, 0)
        specs.append(inputs.SystemSpec(x=g.random((N, 3)) * L, v=inputs.maxwell(N, T, inputs.rng(980, r, 1)),
                                       box=np.array([L, L, L]), phase="gas", mode=inputs.MODE_UF, T0=T,
                                       tau_damp=0.1, stream=r, uf_p=25.0, uf_sigma=2.0, uf_T=T, uf_rcut=8.0,
                                       sched_start=1.0, sched_end=1.0, sched_steps=0))
    eng = swfe.Engine(specs, P, dt=0.002, seed=17, precision="fp64")
    eng.step(1000)
    n = 4000
    for s in specs:
        s.sched_start, s.sched_end, s.sched_steps = 1.0, 0.0, n
    eng.set_schedule(specs)
    eng.step(n)
    wf = eng.work_integral()["W"].copy()
    for s in specs:
        s.sched_start, s.sched_end = 0.0, 1.0
    eng.set_schedule(specs)
    eng.step(n)
    wb = eng.work_integral()["W"].copy()
    dF = 0.5 * (wf - wb)
    expect = N * orc.KB * T * rb
    err = dF.std() / np.sqrt(len(dF))
    print(f"Delta F {dF.mean():.4f} +- {err:.4f} eV, second virial {expect:.4f} eV", flush=True)
    assert dF.mean() == pytest.approx(expect, rel=0.1)
    eng.close()
