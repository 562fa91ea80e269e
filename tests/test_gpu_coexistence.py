"""Absolute free energies end to end: the cd / beta-tin coexistence pressure
at 400 K from Frenkel-Ladd switching of both crystals (section 2.1, section
4.1), the starting point the paper computes for its cd / beta-tin dCCI line
(P_coex(400 K) = 13.17346(5) GPa).

Protocol: 4096-atom diamond (isotropic piston) and 8000-atom beta-tin (one
piston per axis) equilibrated by NPT at 400 K and 13 GPa; each crystal is
then put in its mean box with its atoms on their lattice sites' Einstein
springs (k matched to the measured mean-square displacement, 3 kB T / k =
<u^2>) and switched crystal -> Einstein -> crystal at fixed volume; the
absolute Gibbs energy per atom g = F / N + P v, with F from the Einstein
reference, the centre-of-mass term and the switching free energy, gives
the pressure where the two g(P) cross.  Four realisations of each crystal,
all in one batch, mixed precision.

Measured: P_coex(400 K) = 13.07 +- 0.01 GPa (13.070 with 30 ps switching,
13.067 with 100 ps), the beta-tin spring matched to its fluctuations is
1.37 eV/A^2 (the paper's 1.362).  From this point the cd / beta-tin dCCI
line (temperature control 400 -> 1250 K) passes 1210 K at 9.86 GPa (two
realisations: 9.89, 9.82), against the paper's triple point (1210(2) K,
9.90(3) GPa)."""
import numpy as np
import pytest

from paper_2103_10449_amd import estimators as est
from paper_2103_10449_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

T, P = 400.0, 13.0
N_EQ, N_AVG, N_HOLD, N_SW, REAL = 20000, 20000, 10000, 100000, 4


def _lattice(kind):
    if kind == "cd":
        x, b = inputs.diamond((8, 8, 8), 5.431)
        return x, b, inputs.BARO_ISO
    x, b = inputs.beta_sn((10, 10, 20), 4.80, 2.65)
    return x, b, inputs.BARO_ANISO


@pytest.fixture(scope="module")
def phases(sw_params):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_10449_amd import swfe
    kinds = [kind for _ in range(REAL) for kind in ("cd", "bt")]
    npt = []
    for q, kind in enumerate(kinds):
        x, b, baro = _lattice(kind)
        npt.append(inputs.SystemSpec(x=x, v=inputs.maxwell(len(x), T, inputs.rng(996, q, 1)), box=b, phase=kind,
                                     mode=inputs.MODE_NVT, T0=T, tau_damp=0.1, p_damp=1.0, pressure=P,
                                     stream=q, baro=baro))
    eng = swfe.Engine(npt, sw_params, dt=0.001, seed=11, precision="mixed")
    eng.set_skin(1.0)
    eng.step(N_EQ)
    # mean box over the averaging window, and the mean-square displacement
    # from the lattice sites (scaled to the box, centre of mass aligned)
    boxes = [[] for _ in kinds]
    msd = [[] for _ in kinds]
    for _ in range(N_AVG // 1000):
        eng.step(1000)
        st = eng.state()
        for q, kind in enumerate(kinds):
            L = st[q]["box"]
            boxes[q].append(L)
            site = _lattice(kind)[0] / _lattice(kind)[1] * L
            d = eng.positions(q) - site
            d -= L * np.round(d / L)
            d -= d.mean(axis=0)
            msd[q].append(np.mean(np.sum(d * d, axis=1)))
    st = eng.state()
    fl = []
    info = []
    for q, kind in enumerate(kinds):
        lat, b0, _ = _lattice(kind)
        L = np.mean(boxes[q], axis=0)
        x = eng.positions(q) * (L / st[q]["box"])
        site = lat / b0 * L
        d = x - site
        d -= L * np.round(d / L)
        x0 = site + d.mean(axis=0)
        k = 3.0 * est.KB * T / np.mean(msd[q])
        fl.append(inputs.SystemSpec(x=x0 + (d - d.mean(axis=0)), v=eng.velocities(q), box=L, phase=kind, x0=x0,
                                    mode=inputs.MODE_FL, k_spring=k, T0=T, tau_damp=0.1, stream=100 + q,
                                    sched_start=1.0, sched_end=1.0, sched_steps=0))
        info.append(dict(kind=kind, n=len(lat), V=float(np.prod(L)), k=k))
    assert not any(s["err"] for s in st)
    eng.close()

    eng = swfe.Engine(fl, sw_params, dt=0.001, seed=12, precision="mixed")
    eng.set_skin(1.0)

    def run(a, b, n):
        for s in fl:
            s.sched_start, s.sched_end, s.sched_steps = a, b, n
        eng.set_schedule(fl)
        eng.step(n if n else N_HOLD)
        return eng.work_integral()["W"]

    run(1.0, 1.0, 0)
    wf = run(1.0, 0.0, N_SW)
    run(0.0, 0.0, 0)
    wb = run(0.0, 1.0, N_SW)
    assert not any(s["err"] for s in eng.state())
    eng.close()
    out = {"cd": [], "bt": []}
    for q, d in enumerate(info):
        F = est.solid_free_energy(d["n"], d["k"], T, inputs.SI_MASS_AMU, d["V"], [wf[q]], [wb[q]])
        v = d["V"] / d["n"]
        g = F / d["n"] + P * est.EV_A3_PER_GPA * v
        diss = est.dissipated_heat([wf[q]], [wb[q]]) / d["n"]
        out[d["kind"]].append((g, v, diss, d["k"]))
        print(f"{d['kind']}: k {d['k']:.3f} eV/A^2, v {v:.4f} A^3, g {g:.6f} eV, "
              f"dissipated {1e3 * diss:.3f} meV/atom", flush=True)
    return {kind: np.array(v) for kind, v in out.items()}


def test_switching_is_close_to_reversible(phases):
    for kind, a in phases.items():
        assert np.all(a[:, 2] < 2e-3), kind   # dissipated heat below 2 meV/atom


def test_coexistence_pressure_at_400_K(phases):
    cd, bt = phases["cd"], phases["bt"]
    Pc = est.coexistence_pressure(P, cd[:, 0].mean(), cd[:, 1].mean(), bt[:, 0].mean(), bt[:, 1].mean())
    sem = np.hypot(cd[:, 0].std(ddof=1), bt[:, 0].std(ddof=1)) / np.sqrt(REAL)
    dP = sem / ((cd[:, 1].mean() - bt[:, 1].mean()) * est.EV_A3_PER_GPA)
    print(f"g(cd) - g(beta-tin) at {P} GPa: {1e3 * (cd[:, 0].mean() - bt[:, 0].mean()):.3f} meV/atom; "
          f"P_coex(400 K) = {Pc:.3f} +- {dP:.3f} GPa (paper 13.17346(5))", flush=True)
    assert abs(Pc - 13.17346) < 0.5


@pytest.fixture(scope="module")
def coexistence_point(phases):
    cd, bt = phases["cd"], phases["bt"]
    return est.coexistence_pressure(P, cd[:, 0].mean(), cd[:, 1].mean(), bt[:, 0].mean(), bt[:, 1].mean())


def test_dcci_line_from_the_computed_point_reaches_the_triple_point(sw_params, coexistence_point):
    """dCCI with temperature control (eq. Ps_coex_discreted), T 400 -> 1250 K
    over 100 ps from (400 K, the computed P_coex), two realisations: the
    line passes 1210 K near the paper's triple point (1210(2) K, 9.90(3)
    GPa).  An error d in the starting P_S stays in P_S and appears as
    d / lambda = d T / 400 K in the pressure, so the line from the paper's
    13.17346 GPa lies about 0.3 GPa higher at 1210 K."""
    from paper_2103_10449_amd import swfe
    Pc = float(coexistence_point)
    eq = []
    for r in range(2):
        for j, kind in enumerate(("cd", "bt")):
            x, b, baro = _lattice(kind)
            eq.append(inputs.SystemSpec(x=x, v=inputs.maxwell(len(x), T, inputs.rng(997, r, j)), box=b, phase=kind,
                                        mode=inputs.MODE_NVT, T0=T, tau_damp=0.1, p_damp=1.0, pressure=Pc,
                                        stream=10 * r + j, baro=baro))
    eng = swfe.Engine(eq, sw_params, dt=0.001, seed=13, precision="mixed")
    eng.set_skin(1.0)
    eng.step(30000)
    st = eng.state()
    n_sw = 100000
    specs = []
    for k, s in enumerate(eq):
        specs.append(inputs.SystemSpec(
            x=eng.positions(k), v=eng.velocities(k), box=st[k]["box"].copy(), phase=s.phase,
            mode=inputs.MODE_DCCI_T, partner=k ^ 1, T0=T, tau_damp=0.1, p_damp=1.0, pressure=Pc,
            stream=100 + k, baro=s.baro, sched_start=400.0, sched_end=1250.0, sched_steps=n_sw))
    eng.close()
    eng = swfe.Engine(specs, sw_params, dt=0.001, seed=14, precision="mixed")
    eng.set_skin(1.0)
    tp = [[], []]
    for _ in range(n_sw // 1000):
        eng.step(1000)
        st = eng.state()
        for r in range(2):
            tp[r].append((T / st[2 * r]["lam"], st[2 * r]["Ps"] / st[2 * r]["lam"]))
    assert not any(s["err"] for s in eng.state())
    eng.close()
    ps = [np.interp(1210.0, np.array(v)[:, 0], np.array(v)[:, 1]) for v in tp]
    print(f"cd/beta-tin from P_coex(400 K) = {Pc:.3f} GPa: P(1210 K) = {np.round(ps, 3)} GPa, "
          f"mean {np.mean(ps):.3f} (paper 9.90(3))", flush=True)
    assert abs(np.mean(ps) - 9.90) < 0.3
