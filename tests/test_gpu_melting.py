"""Melting temperatures of Stillinger-Weber silicon from absolute free
energies (section 2.1, section 4.1): the paper's T_m(0 GPa) = 1689.2(3) K
(diamond) and T_m(15 GPa) = 1365.3(3) K (beta-tin).

Both phases at the paper's (T_m, P) after NPT equilibration:
* the crystal (4096-atom diamond with one piston, or 8000-atom beta-tin
  with one piston per axis): Frenkel-Ladd switching to its Einstein crystal
  at its mean box, springs matched to the measured fluctuations;
* liquid (3000 atoms): the SW liquid switched to the Uhlenbeck-Ford fluid
  (p = 25, sigma = 2 A, cutoff 8 A) at its mean volume, and an ideal gas in
  the same box switched on to the same UF fluid, so that F_liquid = F_gas +
  (F_UF - F_gas) - (F_UF - F_liquid) with no tabulated UF free energy.
The per-atom Gibbs energies (g = F / N + P v) and enthalpies (u + P v, u
the mean potential energy per atom; the kinetic parts are equal) give the
crossing temperature.  Four realisations of each phase, 100 ps per
switching direction, mixed precision.

The bound is three standard deviations' coverage (Student t at the
Welch-Satterthwaite degrees of freedom of the two phases' realisations).
Measured at 0 GPa: T_m = 1684.8 +- 1.9 K (paper 1689.2(3)); g(liquid) -
g(cd) = -0.85 meV/atom at 1689.2 K, latent heat 0.323 eV/atom, liquid
18.87 A^3/atom against 20.35 for the crystal; dissipated heat 0.05-0.4
meV/atom (crystal) and about 3.5 meV/atom (liquid legs).  At 15 GPa: T_m =
1365.3 +- 1.1 K (paper 1365.3(3)); g(liquid) - g(beta-tin) = -0.001
meV/atom at 1365.3 K, latent heat 0.140 eV/atom, liquid 17.05 A^3/atom
against 16.60 for beta-tin.  A run whose trajectories differ only in
rounding gave 1684.0 +- 1.9 K and 1361.0 +- 1.4 K, another 1683.5 +- 2.2 K
and 1361.5 +- 1.7 K: both melting points sit a few kelvin below the
paper's."""
import numpy as np
import pytest

from tests import e2e

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.mark.parametrize("case", list(e2e.MELT_CASES))
def test_melting_temperature(sw_params, case):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    kind, T, P = e2e.MELT_CASES[case]
    ph = e2e.cached(("melting", case), e2e.melting_phases, sw_params, case)
    cr, liq = ph["crystal"], ph["liq"]
    Tm = e2e.melting_temperature(case, ph)
    dg = liq[:, 0].mean() - cr[:, 0].mean()
    # standard error of T_m: the realisations' spread of g of both phases
    # over the latent heat, T dg / dh
    k = T / (liq[:, 1].mean() - cr[:, 1].mean())
    parts = [(k * se, dof) for se, dof in (e2e.mean_se(cr[:, 0]), e2e.mean_se(liq[:, 0]))]
    dT, dof = e2e.combine(parts)
    print(f"{case}: g(liquid) - g({kind}) at {T} K: {1e3 * dg:.3f} meV/atom, latent heat "
          f"{liq[:, 1].mean() - cr[:, 1].mean():.4f} eV/atom; T_m({P} GPa) = {Tm:.1f} +- {dT:.1f} K "
          f"(paper {T}(3))", flush=True)
    # three standard deviations' coverage: this estimate's standard error
    # (Student t at its effective degrees of freedom) with the paper's +-0.3 K
    tol = e2e.bound3(parts + [(0.3, np.inf)])
    print(f"{case}: |T_m - paper| = {abs(Tm - T):.1f} K, bound {tol:.1f} K ({dof:.1f} degrees of freedom)",
          flush=True)
    assert abs(Tm - T) < tol
