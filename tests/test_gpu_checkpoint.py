"""Checkpoint / resume: a run saved mid-way and resumed in a fresh context
continues bitwise like the uninterrupted run (counter-based noise, fixed-order
sums, the whole workspace restored), including a schedule changed before
the save."""
import copy

import numpy as np
import pytest

from paper_2103_10449_amd import inputs
from tests.gpu_helpers import diamond_spec, liquid_spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swfe():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_10449_amd import swfe as m
    m.load_library()
    return m


def _specs():
    a = diamond_spec(3, 90, T=1000.0, mode=inputs.MODE_FL, T0=1000.0, tau_damp=0.1, k_spring=5.0, stream=1,
                     sched_start=1.0, sched_end=0.0, sched_steps=400)
    b = liquid_spec(400, 91, mode=inputs.MODE_RS, T0=1700.0, tau_damp=0.1, p_damp=0.2, pressure=1.0, stream=2,
                    sched_start=1.0, sched_end=0.6, sched_steps=400, baro=inputs.BARO_ANISO)
    return [a, b]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resume_is_bitwise(swfe, sw_params, precision):
    ref = swfe.Engine(copy.deepcopy(_specs()), sw_params, seed=5, precision=precision)
    ref.step(150)
    blob = ref.save_state()
    ref.step(120, use_graph=False)
    ref.step(80)
    want = [(ref.positions(k), ref.velocities(k), ref.state()[k]["W"]) for k in range(2)]
    ref.close()
    # a fresh context from the same descriptors, resumed from the blob
    eng = swfe.Engine(copy.deepcopy(_specs()), sw_params, seed=123, precision=precision)
    eng.step(7)  # state that the load must overwrite
    eng.load_state(blob)
    eng.step(120, use_graph=False)
    eng.step(80)
    for k in range(2):
        x, v, W = want[k]
        assert np.array_equal(eng.positions(k), x)
        assert np.array_equal(eng.velocities(k), v)
        assert eng.state()[k]["W"] == W
    eng.close()


def test_checkpoint_of_other_sizes_is_rejected(swfe, sw_params):
    a = swfe.Engine(copy.deepcopy(_specs()), sw_params)
    blob = a.save_state()
    a.close()
    b = swfe.Engine([liquid_spec(300, 92)], sw_params)
    with pytest.raises(swfe.SwfeError) as ei:
        b.load_state(blob)
    assert ei.value.code == swfe.E_INVALID_ARG
    with pytest.raises(swfe.SwfeError):
        b.load_state(blob[:100])
    b.close()


def test_autotune_leaves_the_dynamics_where_they_were(swfe, sw_params):
    """swfe_autotune runs trial steps at every block size and restores the
    state after each: the run then goes on bitwise like one that only
    switched to the chosen block size at the same point."""
    eng = swfe.Engine(copy.deepcopy(_specs()), sw_params, seed=5, precision="mixed")
    eng.step(60)
    before = [(eng.positions(k), eng.velocities(k), eng.state()[k]) for k in range(2)]
    block = eng.autotune()
    assert block in (64, 128, 256)
    for k in range(2):
        x, v, st = before[k]
        now = eng.state()[k]
        assert np.array_equal(eng.positions(k), x)
        assert np.array_equal(eng.velocities(k), v)
        assert (now["step"], now["sched_k"], now["lam"], now["W"]) == (st["step"], st["sched_k"], st["lam"], st["W"])
    eng.step(70)
    got = [(eng.positions(k), eng.state()[k]["W"]) for k in range(2)]
    eng.close()
    ref = swfe.Engine(copy.deepcopy(_specs()), sw_params, seed=5, precision="mixed")
    ref.step(60)
    ref.set_block(block)
    ref.step(70)
    for k in range(2):
        assert np.array_equal(ref.positions(k), got[k][0])
        assert ref.state()[k]["W"] == got[k][1]
    ref.close()


def test_skin_autotune_leaves_the_dynamics_where_they_were(swfe, sw_params):
    """swfe_autotune_skin times graph steps at each candidate skin from a
    snapshot of the state and restores it after each trial: the run then goes
    on bitwise like one that only switched to the chosen skin at that point."""
    eng = swfe.Engine(copy.deepcopy(_specs()), sw_params, seed=5, precision="mixed")
    eng.step(60)
    before = [(eng.positions(k), eng.velocities(k), eng.state()[k]) for k in range(2)]
    skin = eng.autotune_skin([0.5, 1.0, 1.5], steps=20)
    assert skin in (0.5, 1.0, 1.5)
    for k in range(2):
        x, v, st = before[k]
        now = eng.state()[k]
        assert np.array_equal(eng.positions(k), x)
        assert np.array_equal(eng.velocities(k), v)
        assert (now["step"], now["sched_k"], now["lam"], now["W"]) == (st["step"], st["sched_k"], st["lam"], st["W"])
    eng.step(70)
    got = [(eng.positions(k), eng.state()[k]["W"]) for k in range(2)]
    eng.close()
    ref = swfe.Engine(copy.deepcopy(_specs()), sw_params, seed=5, precision="mixed")
    ref.step(60)
    ref.set_skin(skin)
    ref.step(70)
    for k in range(2):
        assert np.array_equal(ref.positions(k), got[k][0])
        assert ref.state()[k]["W"] == got[k][1]
    ref.close()


def test_skin_autotune_rejects_bad_candidates(swfe, sw_params):
    eng = swfe.Engine(copy.deepcopy(_specs()), sw_params)
    # 2.5 A: beyond the 2 A the neighbour lists were sized for at set-up
    for bad in ([], [1.0, -0.2], [6.0], [float("nan")], [0.5] * 17, [1.0, 2.5]):
        with pytest.raises(swfe.SwfeError) as ei:
            eng.autotune_skin(bad)
        assert ei.value.code == swfe.E_INVALID_ARG
    with pytest.raises(swfe.SwfeError) as ei:
        eng.set_skin(2.5)
    assert ei.value.code == swfe.E_INVALID_ARG
    eng.set_skin(2.0)  # the largest the lists were sized for
    eng.step(5)
    eng.close()
