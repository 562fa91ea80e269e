"""GPU parity of the switched dynamics (steps a4-a9, a11): trajectories,
lambda / P_S schedules, work integral and dCCI coupling of the HIP path vs the
oracle on identical inputs and identical Philox noise streams.

FP64 bars: positions within 1e-9 A and work within 1e-9 relative after
short runs (the only differences are last-bit libm/FMA rounding, which the
dynamics amplify slowly); closed-form Einstein switching within statistics.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2103_10449_amd import inputs
from tests.gpu_helpers import betasn_spec, diamond_spec, liquid_spec, to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swfe():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_10449_amd import swfe as m
    m.load_library()
    return m


def _compare(swfe, sw_params, specs, steps, seed=11, use_graph=True, chunks=1, pos_tol=1e-9, w_tol=1e-9):
    eng = swfe.Engine(specs, sw_params, dt=0.001, seed=seed, precision="fp64")
    osys = [to_oracle(s) for s in specs]
    o = orc.Oracle(osys, sw_params, dt=0.001, seed=seed)
    for _ in range(chunks):
        eng.step(steps // chunks, use_graph=use_graph)
        o.run(steps // chunks)
    st = eng.state()
    for k, s in enumerate(osys):
        dx = np.abs(eng.positions(k) - s.x).max()
        dv = np.abs(eng.velocities(k) - s.v).max()
        print(f"sys {k} mode {s.mode}: dx {dx:.2e} dv {dv:.2e} W {st[k]['W']:.10f} vs {s.W:.10f} "
              f"lam {st[k]['lam']:.12f} vs {s.lam:.12f}", flush=True)
        assert dx < pos_tol
        assert dv < 100 * pos_tol
        assert abs(st[k]["W"] - s.W) <= w_tol * max(1.0, abs(s.W))
        assert st[k]["lam"] == pytest.approx(s.lam, rel=1e-12)
        assert st[k]["Ps"] == pytest.approx(s.Ps * orc.GPA_PER_EV_A3, rel=1e-9, abs=1e-9)
        assert np.allclose(st[k]["box"], s.box, rtol=1e-12)
        assert st[k]["U_int"] == pytest.approx(s.U_int, rel=1e-10)
    return eng, o


def test_frenkel_ladd_c1(swfe, sw_params):
    wl = inputs.config1()
    s = wl.systems[0]
    s.sched_steps = 200
    eng, o = _compare(swfe, sw_params, [s], 200)
    assert eng.state()[0]["lam"] == 0.0
    eng.close()


def test_frenkel_ladd_backward_and_eager_chunks(swfe, sw_params):
    wl = inputs.config1(lam_forward=False)
    s = wl.systems[0]
    s.sched_steps = 150
    eng, o = _compare(swfe, sw_params, [s], 150, use_graph=False, chunks=3)
    eng.close()


def test_nve_and_nvt(swfe, sw_params):
    a = diamond_spec(3, 40, T=1200.0, mode=inputs.MODE_NVE, stream=0)
    b = liquid_spec(300, 41, mode=inputs.MODE_NVT, T0=1700.0, tau_damp=0.1, stream=1)
    eng, o = _compare(swfe, sw_params, [a, b], 200)
    eng.close()


def test_reversible_scaling_npt(swfe, sw_params):
    """RS with the isotropic barostat: lambda 1 -> 0.5 with 1/lambda linear,
    P_S = lambda P, work increments d lambda U + d P_S V."""
    a = liquid_spec(400, 50, mode=inputs.MODE_RS, T0=1700.0, tau_damp=0.1, p_damp=0.2,
                    pressure=2.0, stream=3, sched_start=1.0, sched_end=0.5, sched_steps=200)
    b = diamond_spec(4, 51, T=1000.0, mode=inputs.MODE_RS, T0=1000.0, tau_damp=0.1, p_damp=0.2,
                     pressure=0.0, stream=4, sched_start=1.0, sched_end=0.5, sched_steps=200)
    b.x0 = None
    eng, o = _compare(swfe, sw_params, [a, b], 200)
    eng.close()


def test_pressure_switching(swfe, sw_params):
    a = liquid_spec(400, 55, mode=inputs.MODE_AS_P, T0=2200.0, tau_damp=0.1, p_damp=0.2,
                    pressure=0.0, stream=5, sched_start=0.0, sched_end=5.0, sched_steps=200)
    eng, o = _compare(swfe, sw_params, [a], 200)
    eng.close()


@pytest.mark.parametrize("mode", [inputs.MODE_DCCI_P, inputs.MODE_DCCI_T])
def test_dcci_pair_in_one_launch(swfe, sw_params, mode):
    """Coupled phases (diamond + beta-tin) share lambda and P_S updated from
    their instantaneous per-atom energy and volume differences."""
    if mode == inputs.MODE_DCCI_P:
        kw = dict(T0=400.0, tau_damp=0.1, p_damp=0.2, pressure=0.0, sched_start=0.0,
                  sched_end=2.0, sched_steps=200, mode=mode)
    else:
        kw = dict(T0=400.0, tau_damp=0.1, p_damp=0.2, pressure=13.17346, sched_start=400.0,
                  sched_end=600.0, sched_steps=200, mode=mode)
    a = diamond_spec(4, 60, T=400.0, partner=1, stream=0, **kw)
    b = betasn_spec(4, 61, T=400.0, partner=0, stream=1, **kw)
    a.x0 = b.x0 = None
    eng, o = _compare(swfe, sw_params, [a, b], 200)
    st = eng.state()
    assert st[0]["lam"] == st[1]["lam"] and st[0]["Ps"] == st[1]["Ps"]
    eng.close()


def test_graph_replay_equals_eager_bitwise(swfe, sw_params):
    mk = lambda: [diamond_spec(3, 70, mode=inputs.MODE_FL, k_spring=5.0, T0=1000.0, tau_damp=0.1,
                               stream=0, sched_start=1.0, sched_end=0.0, sched_steps=100),
                  liquid_spec(250, 71, mode=inputs.MODE_RS, T0=1700.0, tau_damp=0.1, p_damp=0.5,
                              stream=1, sched_start=1.0, sched_end=0.5, sched_steps=100)]
    e1 = swfe.Engine(mk(), sw_params, seed=3)
    e2 = swfe.Engine(mk(), sw_params, seed=3)
    e1.step(100, use_graph=True)
    for _ in range(4):
        e2.step(25, use_graph=False)
    for k in range(2):
        assert np.array_equal(e1.positions(k), e2.positions(k))
        assert np.array_equal(e1.velocities(k), e2.velocities(k))
    assert np.array_equal(e1.work_integral()["W"], e2.work_integral()["W"])
    e1.close()
    e2.close()


def test_replica_alone_equals_replica_in_batch_bitwise(swfe, sw_params):
    mk = lambda r: diamond_spec(2 + r % 2, 80 + r, mode=inputs.MODE_FL, k_spring=5.0, T0=1000.0,
                                tau_damp=0.1, stream=r, sched_start=1.0, sched_end=0.0, sched_steps=60)
    batch = swfe.Engine([mk(r) for r in range(5)], sw_params, seed=9)
    batch.step(60)
    alone = swfe.Engine([mk(3)], sw_params, seed=9)
    alone.step(60)
    assert np.array_equal(batch.positions(3), alone.positions(0))
    assert batch.work_integral()["W"][3] == alone.work_integral()["W"][0]
    batch.close()
    alone.close()


def test_einstein_switching_closed_form_batched(swfe, sw_params):
    """32 forward + 32 backward Einstein-Einstein switches (SW off) in one
    batch: Delta F = (3 (N-1)/2) kB T ln(1/2) (section 2.1 estimator, eq. dF)."""
    P = dict(sw_params)
    P["epsilon"] = 0.0
    T, k, lam_e, nst, nrep = 1000.0, 5.0, 0.5, 1000, 32
    x0, box = inputs.diamond((2, 2, 2), 5.431)
    specs = []
    for r in range(nrep):
        for d in (0, 1):
            lam0 = 0.0 if d == 0 else lam_e
            x = inputs.perturb(x0, np.sqrt(orc.KB * T / ((1 - lam0) * k)), inputs.rng(951, r, d))
            v = inputs.maxwell(64, T, inputs.rng(951, r, 10 + d))
            specs.append(inputs.SystemSpec(x=x, v=v, box=box, x0=x0, mode=inputs.MODE_FL, k_spring=k,
                                           T0=T, tau_damp=0.1, stream=2 * r + d, sched_start=lam0,
                                           sched_end=lam0, sched_steps=1))
    eng = swfe.Engine(specs, P, seed=123)
    eng.step(300)
    for i, s in enumerate(specs):
        s.sched_end = lam_e if i % 2 == 0 else 0.0
        s.sched_steps = nst
    eng.set_schedule(specs)
    eng.step(nst)
    W = eng.work_integral()["W"]
    wf, wb = W[0::2], W[1::2]
    dF = swfe.delta_f(wf, wb)
    exact = orc.einstein_free_energy_difference(k, (1 - lam_e) * k, T, 63)
    se = 0.5 * np.sqrt(wf.var(ddof=1) / nrep + wb.var(ddof=1) / nrep)
    print(f"dF {dF:.5f} exact {exact:.5f} se {se:.5f}", flush=True)
    assert abs(dF - exact) < max(4 * se, 0.01)
    assert abs(dF - exact) / 64 < 1e-3
    eng.close()


def test_mixed_precision_dynamics_track_fp64(swfe, sw_params):
    """FP32-term dynamics of a liquid (reversible scaling, NPT) and a
    Frenkel-Ladd crystal stay finite and their work stays within 1 meV/atom
    of the FP64 path with the same noise."""
    mk = lambda: [liquid_spec(600, 90, mode=inputs.MODE_RS, T0=1700.0, tau_damp=0.1, p_damp=1.0,
                              stream=0, sched_start=1.0, sched_end=0.5, sched_steps=400),
                  diamond_spec(4, 91, mode=inputs.MODE_FL, k_spring=5.0, T0=1000.0, tau_damp=0.1,
                               stream=1, sched_start=1.0, sched_end=0.0, sched_steps=400)]
    res = {}
    for prec in ("fp64", "mixed"):
        eng = swfe.Engine(mk(), sw_params, seed=5, precision=prec)
        eng.step(400)
        res[prec] = eng.work_integral()["W"]
        eng.close()
    n = np.array([600, 512])
    diff = np.abs(res["mixed"] - res["fp64"]) / n
    print(f"mixed-fp64 work difference per atom: {diff}", flush=True)
    assert np.all(diff < 1e-3)


@pytest.mark.parametrize("skin", [0.0, 1.0])
def test_verlet_skin_does_not_change_results(swfe, sw_params, skin):
    """Lists with any skin (0: rebuilt every step) give the oracle's
    trajectory; a hot liquid under the barostat rebuilds along the way."""
    a = liquid_spec(400, 95, mode=inputs.MODE_RS, T0=2500.0, tau_damp=0.1, p_damp=0.2, pressure=1.0,
                    stream=3, sched_start=1.0, sched_end=0.6, sched_steps=150)
    eng = swfe.Engine([a], sw_params, dt=0.001, seed=4, precision="fp64")
    eng.set_skin(skin)
    o = orc.Oracle([to_oracle(a)], sw_params, dt=0.001, seed=4)
    eng.step(150)
    o.run(150)
    st = eng.state()[0]
    s = o.systems[0]
    print(f"skin {skin}: rebuilds {st['n_rebuild']} dx {np.abs(eng.positions(0) - s.x).max():.2e}", flush=True)
    assert np.abs(eng.positions(0) - s.x).max() < 1e-9
    assert abs(st["W"] - s.W) < 1e-9 * max(1.0, abs(s.W))
    assert st["n_rebuild"] >= (150 if skin == 0.0 else 2)
    eng.close()


def _dilute_gas(seed):
    """1 728 atoms on a perturbed simple-cubic lattice of 12.5 A spacing in a
    150 A box: no pair within the cutoff, and a cell table (37^3 entries at a
    0.2 A skin) larger than the cell scan keeps in LDS."""
    g = np.arange(12) * 12.5 + 6.25
    xl = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    x = inputs.perturb(xl, 0.5, inputs.rng(708, seed, 0))
    v = inputs.maxwell(len(x), 1000.0, inputs.rng(708, seed, 1))
    return inputs.SystemSpec(x=x, v=v, box=np.array([150.0, 150.0, 150.0]), phase="gas", mode=inputs.MODE_NVT,
                             T0=1000.0, tau_damp=0.1, stream=50)


def test_rebuild_paths_agree_bitwise(swfe, sw_params):
    """The three ways a list rebuild re-sorts the atoms give the same atom
    order, hence the same trajectory bit for bit: the 216-atom crystal alone
    (every system small: one workgroup per system sorts in LDS), beside a
    3 000-atom liquid (the cell scan runs inside the scatter stage), and
    beside a dilute gas whose cell table is too large for LDS (a scan launch
    of its own).  A 0.2 A skin makes the crystal rebuild its list often."""
    crystal = lambda: diamond_spec(3, 91, mode=inputs.MODE_FL, k_spring=5.0, T0=1000.0, tau_damp=0.1, stream=7,
                                   sched_start=1.0, sched_end=0.0, sched_steps=80)
    others = {"sort in LDS": [],
              "scan in the scatter stage": [liquid_spec(3000, 92, mode=inputs.MODE_NVT, T0=1700.0, tau_damp=0.1,
                                                        stream=8)],
              "scan launch": [_dilute_gas(93)]}
    got = {}
    for name, rest in others.items():
        print(f"rebuild path: {name}", flush=True)
        eng = swfe.Engine([crystal()] + rest, sw_params, seed=11, block=128)
        eng.set_skin(0.2)
        eng.step(80)
        st = eng.state()
        assert st[0]["n_rebuild"] > 5
        got[name] = (eng.positions(0), eng.velocities(0), st[0]["W"])
        eng.close()
    ref = got["sort in LDS"]
    for name, (x, v, W) in got.items():
        assert np.array_equal(x, ref[0]), name
        assert np.array_equal(v, ref[1]), name
        assert W == ref[2], name
