"""The reversible-scaling pins must catch the mistakes they exist for.  Each
case plants one mistake in the oracle (on the CPU, through monkeypatch) and
runs the pin that should see it: lambda dropped from the force (eq. H_RS),
from the barostat's virial (trace or per-axis diagonal), P_S left at P
instead of lambda P (eq. P_sc), or the P_S V term dropped from the work
(eqs. dH_RS, Wdyn_RS)."""
import numpy as np
import pytest

from oracle import oracle as orc
from tests import test_oracle_rs as pins

_SCALED = (orc.MODE_RS, orc.MODE_DCCI_T, orc.MODE_DCCI_P)


def _unscaled_force(monkeypatch):
    orig = orc.Oracle.total_force

    def tf(self, s, lam):
        return s.F_int if s.mode in _SCALED else orig(self, s, lam)
    monkeypatch.setattr(orc.Oracle, "total_force", tf)


def _unscaled_trace(monkeypatch):
    monkeypatch.setattr(orc.Oracle, "_xi_trace", lambda self, s, lam: float(np.trace(s.Xi_int)))


def _unscaled_diag(monkeypatch):
    monkeypatch.setattr(orc.Oracle, "_xi_diag", lambda self, s, lam: np.diag(s.Xi_int).copy())


def _ps_is_p(monkeypatch):
    init, step = orc.initial_switch_state, orc.Oracle.step

    def fix(s):
        if s.mode == orc.MODE_RS:
            s.Ps = s.pressure / orc.GPA_PER_EV_A3

    def init2(s):
        init(s)
        fix(s)

    def step2(self):
        step(self)
        for s in self.systems:
            fix(s)
    monkeypatch.setattr(orc, "initial_switch_state", init2)
    monkeypatch.setattr(orc.Oracle, "step", step2)


def _no_psv_work(monkeypatch):
    orig = orc.hamiltonian_switch_part

    def hs(s, lam, Ps):
        return lam * s.U_int if s.mode in _SCALED else orig(s, lam, Ps)
    monkeypatch.setattr(orc, "hamiltonian_switch_part", hs)


@pytest.mark.parametrize("plant,pin", [
    (_unscaled_force, lambda P: pins.test_rs_fixed_lambda_is_time_rescaled_nph(P, orc.BARO_ISO)),
    (_unscaled_force, lambda P: pins.test_dcci_fixed_temperature_is_time_rescaled_nph(P)),
    (_unscaled_force, pins.test_rs_harmonic_crystal_closed_form),
    (_unscaled_trace, lambda P: pins.test_rs_fixed_lambda_is_time_rescaled_nph(P, orc.BARO_ISO)),
    (_unscaled_diag, lambda P: pins.test_rs_fixed_lambda_is_time_rescaled_nph(P, orc.BARO_ANISO)),
    (_ps_is_p, lambda P: pins.test_rs_fixed_lambda_is_time_rescaled_nph(P, orc.BARO_ISO)),
    (_no_psv_work, pins.test_rs_ideal_gas_gibbs_closed_form),
], ids=["force-rescale", "force-dcci", "force-harmonic", "virial-trace", "virial-diag", "ps-unscaled",
        "work-no-psv"])
def test_planted_mistake_fails_its_pin(monkeypatch, sw_params, plant, pin):
    plant(monkeypatch)
    with pytest.raises(AssertionError):
        pin(sw_params)
