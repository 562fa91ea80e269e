"""Pins of the oracle's reversible-scaling branch, the one dCCI also takes:
forces lambda F_int, barostat virial lambda Xi, target P_S = lambda P and the
work increments Delta lambda U_int + Delta P_S V (eqs. H_RS, P_sc, dH_RS,
Wdyn_RS).  Each check is fixed by something outside the oracle's code:

* an exact time rescaling: at fixed lambda and without the thermostat, the
  dynamics of H = K + lambda U + lambda P V (plus the piston) with step dt is
  the dynamics of H = K + U + P V with step dt sqrt(lambda) and velocities
  (and piston rates) divided by sqrt(lambda).  Every operation of the
  discrete step maps onto its counterpart, so the two trajectories agree to
  rounding; a missing lambda in the force, in the barostat's virial or in
  P_S moves them apart by orders of magnitude more;
* the closed-form free energy of an ideal gas under reversible scaling at
  pressure P: G(lambda) - G(1) = N kB T0 ln lambda (the centre of mass is
  frozen in scaled coordinates, so the volume is Gamma-distributed with
  shape N);
* the closed-form free energy of a harmonic crystal at fixed volume:
  F(lambda) - F(1) = (lambda - 1) U0 + (3(N-1)/2) kB T0 ln lambda.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2103_10449_amd import inputs


def _diamond64(a=5.431, sigma=0.06, T=800.0, seed=0):
    xl, box = inputs.diamond((2, 2, 2), a)
    x = inputs.perturb(xl, sigma, inputs.rng(980, seed, 0))
    v = inputs.maxwell(len(x), T, inputs.rng(980, seed, 1))
    return x, v, box


@pytest.mark.parametrize("baro", [orc.BARO_ISO, orc.BARO_ANISO])
def test_rs_fixed_lambda_is_time_rescaled_nph(sw_params, baro):
    """Reversible scaling at fixed lambda = 0.64 with the barostat (target
    P_S = lambda P) and no thermostat, against plain NPH at P with step
    dt sqrt(lambda) from velocities v / sqrt(lambda): positions and boxes
    agree to rounding after 300 steps, velocities after rescaling."""
    lam, P_GPa, dt, n = 0.64, 3.0, 0.001, 300
    x, v, box = _diamond64(seed=1 + baro)
    rs = orc.OSystem(x=x.copy(), v=v.copy(), box=box.copy(), mode=orc.MODE_RS, T0=800.0, tau_damp=0.0,
                     p_damp=0.05, pressure=P_GPa, baro=baro, sched_start=lam, sched_end=lam, sched_steps=0)
    ref = orc.OSystem(x=x.copy(), v=v.copy() / np.sqrt(lam), box=box.copy(), mode=orc.MODE_NVE, T0=800.0,
                      p_damp=0.05, pressure=P_GPa, baro=baro)
    o_rs = orc.Oracle([rs], sw_params, dt=dt)
    o_ref = orc.Oracle([ref], sw_params, dt=dt * np.sqrt(lam))
    assert rs.Ps == pytest.approx(lam * P_GPa / orc.GPA_PER_EV_A3, rel=1e-15)
    o_rs.run(n)
    o_ref.run(n)
    assert np.abs(rs.box - box).max() > 1e-3            # the barostat did move the box
    assert np.abs(rs.x - ref.x).max() < 1e-9
    assert np.abs(rs.box - ref.box).max() < 1e-10
    assert np.abs(rs.v / np.sqrt(lam) - ref.v).max() < 1e-8
    assert rs.W == 0.0                                  # lambda and P_S never changed


def test_dcci_fixed_temperature_is_time_rescaled_nph(sw_params):
    """A dCCI pair under temperature control held at T = 1.5625 T0 keeps
    lambda = T0/T = 0.64 and P_S = lambda P (eq. Ps_coex_discreted with
    lambda_{k+1} = lambda_k), so each phase must follow the same time-rescaled
    NPH dynamics as reversible scaling."""
    lam, P_GPa, dt, n, T0 = 0.64, 2.0, 0.001, 200, 500.0
    T = T0 / lam
    xa, va, boxa = _diamond64(a=5.431, seed=3)
    xb, vb, boxb = _diamond64(a=5.50, seed=4)
    kw = dict(mode=orc.MODE_DCCI_T, T0=T0, tau_damp=0.0, p_damp=0.05, pressure=P_GPa,
              sched_start=T, sched_end=T, sched_steps=1000)
    pair = [orc.OSystem(x=xa.copy(), v=va.copy(), box=boxa.copy(), partner=1, **kw),
            orc.OSystem(x=xb.copy(), v=vb.copy(), box=boxb.copy(), partner=0, **kw)]
    refs = [orc.OSystem(x=x.copy(), v=v.copy() / np.sqrt(lam), box=b.copy(), mode=orc.MODE_NVE, T0=T0,
                        p_damp=0.05, pressure=P_GPa) for x, v, b in ((xa, va, boxa), (xb, vb, boxb))]
    o = orc.Oracle(pair, sw_params, dt=dt)
    o_ref = orc.Oracle(refs, sw_params, dt=dt * np.sqrt(lam))
    o.run(n)
    o_ref.run(n)
    for s, r in zip(pair, refs):
        assert s.lam == pytest.approx(lam, rel=1e-15) and s.err == 0
        assert np.abs(s.x - r.x).max() < 1e-9
        assert np.abs(s.box - r.box).max() < 1e-10


def test_rs_ideal_gas_gibbs_closed_form(sw_params):
    """Reversible scaling of an ideal gas (SW off) at P = 0.1 GPa and T0 =
    1000 K, lambda 1 -> 1/2 and back, with the Langevin thermostat and the
    isotropic barostat at P_S = lambda P: the work is all Delta P_S V, and
    1/2 (W_fwd - W_bwd) estimates G(1/2) - G(1) = N kB T0 ln(1/2) =
    -0.478 eV for N = 8 (the volume follows V^(N-1) exp(-lambda P V / kB T0),
    so G(lambda) = N kB T0 ln lambda + const)."""
    P = dict(sw_params)
    P["epsilon"] = 0.0
    N, T0, Pg, lam_f, n = 8, 1000.0, 0.1, 0.5, 10000
    L = (N * orc.KB * T0 / (Pg / orc.GPA_PER_EV_A3)) ** (1 / 3)
    g = inputs.rng(981, 0, 0)
    s = orc.OSystem(x=g.random((N, 3)) * L, v=inputs.maxwell(N, T0, inputs.rng(981, 0, 1)),
                    box=np.array([L, L, L]), mode=orc.MODE_RS, T0=T0, tau_damp=0.05, p_damp=0.1,
                    pressure=Pg, stream=2, sched_start=1.0, sched_end=1.0, sched_steps=0)
    o = orc.Oracle([s], P, seed=8)
    o.run(3000)
    dG = []
    for _ in range(2):
        s.sched_start, s.sched_end, s.sched_steps = 1.0, lam_f, n
        orc.initial_switch_state(s)
        o.run(n)
        wf = s.W
        s.sched_start, s.sched_end = lam_f, 1.0
        orc.initial_switch_state(s)
        o.run(n)
        dG.append(0.5 * (wf - s.W))
    expect = N * orc.KB * T0 * np.log(lam_f)
    assert np.mean(dG) == pytest.approx(expect, rel=0.06)


def test_rs_harmonic_crystal_closed_form(sw_params):
    """Reversible scaling of a nearly harmonic SW diamond (64 atoms, T0 = 30 K,
    fixed volume, Langevin) from lambda = 1 to 1/2 and back: 1/2 (W_fwd -
    W_bwd) = (lambda_f - 1) U0 + (3(N-1)/2) kB T0 ln lambda_f, with U0 the
    ideal lattice's energy.  The thermal part, -0.169 eV, is what the check
    resolves: with the forces left unscaled it would read (lambda_f - 1)
    (3(N-1)/2) kB T0 = -0.122 eV."""
    xl, box = inputs.diamond((2, 2, 2), 5.431)
    U0 = orc.sw_eval(xl, box, sw_params, need_dtheta=False)["E"]
    N, T0, lam_f, n, reps = 64, 30.0, 0.5, 3000, 3
    vals = []
    for r in range(reps):
        x = inputs.perturb(xl, 0.02, inputs.rng(982, r, 0))
        v = inputs.maxwell(N, T0, inputs.rng(982, r, 1))
        s = orc.OSystem(x=x, v=v, box=box.copy(), mode=orc.MODE_RS, T0=T0, tau_damp=0.1, stream=r,
                        sched_start=1.0, sched_end=1.0, sched_steps=0)
        o = orc.Oracle([s], sw_params, seed=12)
        o.run(1000)
        s.sched_start, s.sched_end, s.sched_steps = 1.0, lam_f, n
        orc.initial_switch_state(s)
        o.run(n)
        wf = s.W
        s.sched_start, s.sched_end = lam_f, 1.0
        orc.initial_switch_state(s)
        o.run(n)
        vals.append(0.5 * (wf - s.W) - (lam_f - 1.0) * U0)
    thermal = 1.5 * (N - 1) * orc.KB * T0 * np.log(lam_f)
    assert np.mean(vals) == pytest.approx(thermal, rel=0.05)
