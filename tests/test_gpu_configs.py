"""Parity at the workloads' own sizes, in the batched graph launch the
benchmark times.

* 64-atom diamond Frenkel-Ladd, 1000 steps forward and backward: per-
  trajectory work and Delta F vs the oracle with the same noise (FP64 within
  0.1 meV/atom, mixed within 1 meV/atom).
* 8000-atom diamond and liquid: forces/energy/virial at full size, then a
  short reversible-scaling NPT run vs the oracle.
* dCCI pair, 4096-atom diamond + 8000-atom beta-tin, pressure control: a
  short coupled run vs the oracle (shared lambda and P_S).
* the 64-replica batch in the launch configuration the benchmark times
  (HIP-graph steps, the block sizes its autotune picks: 128 threads for the
  mixed path, 256 for FP64; Verlet skin 1.8 A): the energy and 32 sampled
  forces of all 64 replicas; a 20-step switching trajectory of the whole
  batch, with positions, work and lambda of six replicas (diamond, beta-tin
  and liquid; the smallest and the largest) against the oracle run on those
  replicas alone (a replica alone equals itself in the batch, bitwise);
* Delta F of the benchmark's switching protocol (1000 steps each way): the
  FP64 path tracks the oracle trajectory by trajectory with the same noise,
  and the mixed path's ensemble mean over 32 realisations of the same
  replica agrees with the FP64 path's (eqs. dF, Qdiss).
"""
import copy
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2103_10449_amd import inputs
from tests.gpu_helpers import force_err, to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swfe():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_10449_amd import swfe as m
    m.load_library()
    return m


@pytest.mark.parametrize("precision,tol_mev", [("fp64", 0.1), ("mixed", 1.0)])
def test_c1_frenkel_ladd_delta_f(swfe, sw_params, precision, tol_mev):
    fwd = inputs.config1(lam_forward=True).systems[0]
    res = {}
    for name in ("gpu", "oracle"):
        s = copy.deepcopy(fwd)
        if name == "gpu":
            eng = swfe.Engine([s], sw_params, seed=17, precision=precision)
            eng.step(1000)
            wf = eng.work_integral()["W"][0]
            s.sched_start, s.sched_end = 0.0, 1.0
            eng.set_schedule([s])
            eng.step(1000)
            wb = eng.work_integral()["W"][0]
            eng.close()
        else:
            o = orc.Oracle([to_oracle(s)], sw_params, seed=17)
            o.run(1000)
            wf = o.systems[0].W
            o.systems[0].sched_start, o.systems[0].sched_end = 0.0, 1.0
            orc.initial_switch_state(o.systems[0])
            o.run(1000)
            wb = o.systems[0].W
        res[name] = (wf, wb, orc.delta_f([wf], [wb]))
    dF_g, dF_o = res["gpu"][2], res["oracle"][2]
    print(f"{precision}: dF gpu {dF_g:.6f} oracle {dF_o:.6f} eV; W fwd {res['gpu'][0]:.6f}/{res['oracle'][0]:.6f}",
          flush=True)
    assert abs(dF_g - dF_o) / 64 < tol_mev * 1e-3


@pytest.mark.parametrize("phase", ["diamond", "liquid"])
def test_c2_full_size_forces_and_rs_run(swfe, sw_params, phase):
    wl = inputs.config2(phase=phase, steps=20)
    s = wl.systems[0]
    ref = orc.sw_eval(s.x, s.box, sw_params)
    eng = swfe.Engine([copy.deepcopy(s)], sw_params, seed=23, precision="fp64")
    out = eng.compute_forces().cpu().numpy()[0]
    assert force_err(eng.forces(0), ref["F"]) < 1e-10
    assert out[0] == pytest.approx(ref["E"], rel=1e-12)
    assert np.abs(out[2:11].reshape(3, 3) - ref["virial"]).max() < 1e-9 * max(1.0, np.abs(ref["virial"]).max())
    o = orc.Oracle([to_oracle(s)], sw_params, seed=23)
    eng.step(20)
    o.run(20)
    st = eng.state()[0]
    dx = np.abs(eng.positions(0) - o.systems[0].x).max()
    print(f"c2 {phase}: dx {dx:.2e} W {st['W']:.8f} vs {o.systems[0].W:.8f}", flush=True)
    assert dx < 1e-9
    assert abs(st["W"] - o.systems[0].W) < 1e-9 * max(1.0, abs(o.systems[0].W))
    assert np.allclose(st["box"], o.systems[0].box, rtol=1e-12)
    eng.close()


def test_c3_dcci_pair_full_size(swfe, sw_params):
    wl = inputs.config3(steps=100000)
    specs = copy.deepcopy(wl.systems)
    eng = swfe.Engine(specs, sw_params, seed=31, precision="fp64")
    o = orc.Oracle([to_oracle(s) for s in wl.systems], sw_params, seed=31)
    eng.step(10)
    o.run(10)
    st = eng.state()
    for k in range(2):
        dx = np.abs(eng.positions(k) - o.systems[k].x).max()
        print(f"c3 sys {k}: dx {dx:.2e} lam {st[k]['lam']:.12f} vs {o.systems[k].lam:.12f} "
              f"Ps {st[k]['Ps']:.9f} vs {o.systems[k].Ps * orc.GPA_PER_EV_A3:.9f}", flush=True)
        assert dx < 1e-9
        assert st[k]["lam"] == pytest.approx(o.systems[k].lam, rel=1e-12)
        assert st[k]["Ps"] == pytest.approx(o.systems[k].Ps * orc.GPA_PER_EV_A3, rel=1e-9, abs=1e-9)
    assert st[0]["lam"] == st[1]["lam"]
    eng.close()


BENCH_BLOCK = {"mixed": 128, "fp64": 256}
BENCH_SKIN = 1.8
# replicas of the benchmark batch checked step by step: the smallest diamond,
# the largest diamond, the largest beta-tin, the smallest beta-tin, the
# smallest liquid and a large liquid
C4_TRACKED = (10, 16, 33, 44, 29, 12)


def _oracle_threads():
    return max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def c4_oracle_energies(sw_params):
    wl = inputs.config4(steps=1000)
    orc.set_threads(_oracle_threads())
    ref = [orc.sw_eval(s.x, s.box, sw_params, need_dtheta=False) for s in wl.systems]
    orc.set_threads(1)
    return wl, ref


@pytest.mark.parametrize("prec,ftol,etol", [("fp64", 1e-10, 1e-12), ("mixed", 1e-5, 1e-5)])
def test_c4_batch_every_replica(swfe, sw_params, c4_oracle_energies, prec, ftol, etol):
    """All 64 replicas of the batch in one launch: each replica's energy, and
    the forces of 32 sampled atoms of each, against the oracle (FP64 energy
    to 1e-12 relative, mixed to 1e-5 eV/atom)."""
    wl, ref = c4_oracle_energies
    eng = swfe.Engine(copy.deepcopy(wl.systems), sw_params, seed=3, precision=prec, block=BENCH_BLOCK[prec])
    eng.set_skin(BENCH_SKIN)
    out = eng.compute_forces().cpu().numpy()
    worst_f = worst_e = 0.0
    for k, s in enumerate(wl.systems):
        idx = inputs.rng(4, k, 99).choice(s.n, 32, replace=False)
        ef = force_err(eng.forces(k)[idx], ref[k]["F"][idx])
        ee = abs(out[k, 0] - ref[k]["E"]) / s.n
        worst_f, worst_e = max(worst_f, ef), max(worst_e, ee)
        assert ef < ftol, (prec, k)
        if prec == "fp64":
            assert abs(out[k, 0] - ref[k]["E"]) <= 1e-12 * abs(ref[k]["E"]), k
        else:
            assert ee < etol, k
    print(f"c4 {prec}: worst sampled force error {worst_f:.2e}, worst energy error {worst_e:.2e} eV/atom",
          flush=True)
    eng.close()


@pytest.fixture(scope="module")
def c4_oracle_trajectories(sw_params):
    """The tracked replicas alone in the oracle, 20 steps of their forward
    schedules (seed 3, as the batch)."""
    wl = inputs.config4(steps=1000)
    orc.set_threads(_oracle_threads())
    out = {}
    for k in C4_TRACKED:
        o = orc.Oracle([to_oracle(wl.systems[k])], sw_params, seed=3)
        o.run(C4_STEPS)
        s = o.systems[0]
        out[k] = (s.x.copy(), s.W, s.lam, s.U_int)
    orc.set_threads(1)
    return wl, out


C4_STEPS = 20


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_c4_batch_trajectory_in_bench_configuration(swfe, sw_params, c4_oracle_trajectories, prec):
    """The whole 64-replica batch takes 20 graph-replayed switching steps in
    the benchmark's launch configuration; six replicas' positions, work and
    lambda against the oracle.  FP64: 1e-9 A and 1e-9 relative.  Mixed: the
    force bar of 1e-5 (relative to max(|F|, 1 eV/A), about 5e-5 eV/A on
    these hot systems) displaces an atom by at most (dF/m) t^2 / 2 = 3.4e-6 A
    over 20 fs, so positions within 1e-5 A; each switching step's work has
    the energy error (1e-5 eV/atom) times its d lambda, so W within 1e-6
    eV/atom over the 0.02 (or less) of lambda these steps cover."""
    wl, ref = c4_oracle_trajectories
    eng = swfe.Engine(copy.deepcopy(wl.systems), sw_params, seed=3, precision=prec, block=BENCH_BLOCK[prec])
    eng.set_skin(BENCH_SKIN)
    eng.step(C4_STEPS, use_graph=True)
    w = eng.work_integral()
    st = eng.state()
    for k in C4_TRACKED:
        x, W, lam, U = ref[k]
        n = wl.systems[k].n
        dx = np.abs(eng.positions(k) - x).max()
        dw = abs(w["W"][k] - W)
        print(f"c4 {prec} replica {k} ({wl.systems[k].phase}, {n} atoms): dx {dx:.2e} A, "
              f"dW {dw:.2e} eV ({dw / n:.2e} eV/atom), lam {w['lam'][k]:.12f} vs {lam:.12f}", flush=True)
        assert w["lam"][k] == pytest.approx(lam, rel=1e-14)
        if prec == "fp64":
            assert dx < 1e-9
            assert dw <= 1e-9 * max(1.0, abs(W))
            assert st[k]["U_int"] == pytest.approx(U, rel=1e-10)
        else:
            assert dx < 1e-5
            assert dw / n < 1e-6
            assert abs(st[k]["U_int"] - U) / n < 1e-5
    eng.close()


# ---- Delta F at the benchmark's protocol ------------------------------------
DF_STEPS = 1000
DF_REPS = 32
DF_ORACLE_REPS = 1


def _df_specs(reps):
    """reps realisations (own noise streams) of a 512-atom diamond switched to
    its Einstein crystal (Frenkel-Ladd, 1000 K) and of a 550-atom liquid
    under reversible scaling (lambda 1 -> 0.5 at 1700 K), as in the
    benchmark batch."""
    wl = inputs.config4(steps=DF_STEPS)
    base = [wl.systems[10], wl.systems[53]]     # 512-atom diamond, 550-atom liquid
    specs = []
    for b in base:
        for r in range(reps):
            s = copy.deepcopy(b)
            s.stream = 1000 + 64 * r + len(specs)
            specs.append(s)
    return specs


def _oracle_delta_f(spec, P, seed):
    o = orc.Oracle([to_oracle(spec)], P, seed=seed)
    o.run(DF_STEPS)
    s = o.systems[0]
    wf = s.W
    s.sched_start, s.sched_end = s.sched_end, s.sched_start
    orc.initial_switch_state(s)
    o.run(DF_STEPS)
    return orc.delta_f([wf], [s.W])


def _gpu_delta_f(swfe, specs, P, prec, seed):
    eng = swfe.Engine(copy.deepcopy(specs), P, seed=seed, precision=prec, block=BENCH_BLOCK[prec])
    eng.set_skin(BENCH_SKIN)
    eng.step(DF_STEPS)
    wf = eng.work_integral()["W"].copy()
    back = copy.deepcopy(specs)
    for s in back:
        s.sched_start, s.sched_end = s.sched_end, s.sched_start
    eng.set_schedule(back)
    eng.step(DF_STEPS)
    wb = eng.work_integral()["W"].copy()
    eng.close()
    return 0.5 * (wf - wb)


@pytest.mark.slow
def test_delta_f_at_the_benchmark_protocol(swfe, sw_params):
    specs = _df_specs(DF_REPS)
    n = np.array([s.n for s in specs], float)
    seed = 29
    df = {prec: _gpu_delta_f(swfe, specs, sw_params, prec, seed) / n for prec in ("fp64", "mixed")}
    # the oracle on the first realisations of each replica, same noise
    picks = [r for b in range(2) for r in range(b * DF_REPS, b * DF_REPS + DF_ORACLE_REPS)]
    orc.set_threads(_oracle_threads())
    df_orc = np.array([_oracle_delta_f(specs[i], sw_params, seed) for i in picks]) / n[picks]
    orc.set_threads(1)
    for i, d in zip(picks, df_orc):
        print(f"realisation {i}: dF oracle {1e3 * d:.4f}, fp64 {1e3 * df['fp64'][i]:.4f}, "
              f"mixed {1e3 * df['mixed'][i]:.4f} meV/atom", flush=True)
        assert abs(df["fp64"][i] - d) < 1e-4           # 0.1 meV/atom, trajectory by trajectory
    for b, name in enumerate(("diamond 512 FL", "liquid 550 RS")):
        sl = slice(b * DF_REPS, (b + 1) * DF_REPS)
        diff = df["mixed"][sl] - df["fp64"][sl]
        mean, se = float(diff.mean()), float(diff.std(ddof=1) / np.sqrt(DF_REPS))
        print(f"{name}: mean dF mixed - fp64 = {1e3 * mean:.4f} +- {1e3 * se:.4f} meV/atom "
              f"(n = {DF_REPS}; single realisations up to {1e3 * np.abs(diff).max():.3f})", flush=True)
        assert abs(mean) < 1e-3 and 2.0 * se < 1e-3
