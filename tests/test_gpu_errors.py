"""Error paths of the library on the GPU, through the C-ABI, each forced by
its input from the host so that every kernel still runs to its normal end:

* a dCCI pair whose two phases are identical has Delta v = 0 exactly, where
  the coupling rule is singular (section 3, denominator of eq.
  l_coex_discreted; the Delta u / Delta v of eq. Ps_coex_discreted): the
  library holds lambda and P_S and reports SWFE_E_DCCI_SINGULAR;
* a NaN velocity put into the caller's array moves its atom to NaN: the
  kernels keep every index in range (non-finite positions bin to cell 0 and
  fail every distance test) and the library reports SWFE_E_NONFINITE for
  that system;
* after a strained force evaluation the dynamics start from the unstrained
  interaction again.
"""
import numpy as np
import pytest

from paper_2103_10449_amd import inputs
from tests.gpu_helpers import diamond_spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swfe():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_10449_amd import swfe as m
    m.load_library()
    return m


def test_dcci_identical_phases_are_singular(swfe, sw_params):
    kw = dict(mode=inputs.MODE_DCCI_T, T0=400.0, tau_damp=0.1, p_damp=0.2, pressure=13.0,
              sched_start=400.0, sched_end=600.0, sched_steps=100, stream=7)
    a = diamond_spec(2, 120, T=400.0, partner=1, **kw)
    b = diamond_spec(2, 120, T=400.0, partner=0, **kw)
    a.x0 = b.x0 = None
    print("dcci singular: two identical 64-atom phases", flush=True)
    eng = swfe.Engine([a, b], sw_params, seed=3)
    eng.step(5)
    with pytest.raises(swfe.SwfeError) as ei:
        eng.work_integral()
    assert ei.value.code == swfe.E_DCCI_SINGULAR
    # the error is cleared on read; lambda and P_S were held at their start
    w = eng.work_integral()
    assert np.all(w["lam"] == 1.0)
    assert w["Ps"] == pytest.approx([13.0, 13.0], rel=1e-14)
    assert np.all(w["W"] == 0.0)
    eng.close()


def test_nonfinite_velocity_is_reported(swfe, sw_params):
    bad = diamond_spec(2, 121, mode=inputs.MODE_NVT, T0=1000.0, tau_damp=0.1, stream=0)
    good = diamond_spec(2, 122, mode=inputs.MODE_NVT, T0=1000.0, tau_damp=0.1, stream=1)
    print("nonfinite: NaN velocity in system 1 of 2", flush=True)
    eng = swfe.Engine([good, bad], sw_params, seed=4)
    eng.step(2)
    eng.work_integral()
    eng.v[0, 64 + 5] = float("nan")
    eng.step(3)
    with pytest.raises(swfe.SwfeError) as ei:
        eng.work_integral()
    assert ei.value.code == swfe.E_NONFINITE
    assert "system 1" in str(ei.value)
    assert np.all(np.isfinite(eng.positions(0)))
    eng.close()


def test_step_after_strained_evaluation_uses_unstrained_forces(swfe, sw_params):
    mk = lambda: diamond_spec(3, 123, mode=inputs.MODE_FL, k_spring=5.0, T0=1000.0, tau_damp=0.1, stream=2,
                              sched_start=1.0, sched_end=0.0, sched_steps=50)
    ref = swfe.Engine([mk()], sw_params, seed=6)
    ref.step(20)
    eng = swfe.Engine([mk()], sw_params, seed=6)
    strain = np.diag([0.01, -0.02, 0.015]).reshape(1, 9)
    eng.compute_forces(strain=strain)
    eng.step(20)
    dx = np.abs(eng.positions(0) - ref.positions(0)).max()
    print(f"strained then stepped: dx {dx:.2e}", flush=True)
    assert dx < 1e-12
    assert eng.work_integral()["W"][0] == pytest.approx(ref.work_integral()["W"][0], rel=1e-12, abs=1e-12)
    eng.close()
    ref.close()
