"""Host-side estimators of the switching methods (section 2 and 3): free
energies from forward/backward dynamical work, the reversible-scaling
Gibbs curve G(T), the pressure-switching Gibbs curve G(P), and the dCCI
coexistence line.  Plain numpy on logged (lambda, work) or (P, work)
trajectories; they do no dynamics."""
from typing import Sequence, Tuple

import numpy as np

KB = 8.617333262e-5            # eV/K
HBAR = 6.582119569e-4          # eV ps
AMU_A2_PS2 = 1.0364269656e-4   # eV per amu A^2 / ps^2
EV_A3_PER_GPA = 1.0 / 160.21766208  # eV/A^3 per GPa


def delta_f(w_forward, w_backward) -> float:
    """F(b) - F(a) = (mean W(a->b) - mean W(b->a)) / 2 (eq. dF)."""
    return 0.5 * (float(np.mean(w_forward)) - float(np.mean(w_backward)))


def dissipated_heat(w_forward, w_backward) -> float:
    """Mean dissipated heat (mean W(a->b) + mean W(b->a)) / 2 (eq. Qdiss)."""
    return 0.5 * (float(np.mean(w_forward)) + float(np.mean(w_backward)))


def _with_start(x0: float, x_log: np.ndarray, w_log: np.ndarray):
    """The logged path (x, W) with its start (x0, W = 0) in front, unless the
    log already begins there."""
    if len(x_log) and x_log[0] == x0:
        return x_log, w_log
    return np.r_[x0, x_log], np.r_[0.0, w_log]


def _work_along(x_log: np.ndarray, w_log: np.ndarray, grid: np.ndarray) -> np.ndarray:
    """Accumulated work at the grid values of the switched variable, from a
    monotone logged path (x, W)."""
    x_log, w_log = np.asarray(x_log, float), np.asarray(w_log, float)
    order = np.argsort(x_log)
    return np.interp(grid, x_log[order], w_log[order])


def gibbs_rs(G0: float, n_atoms: int, T0: float, lam_fwd, w_fwd, lam_bwd, w_bwd, lam_grid,
             lam_f=None) -> Tuple[np.ndarray, np.ndarray]:
    """Gibbs free energy G(P, T0/lambda) on lam_grid from reversible scaling
    (eq. Gibbs_RS): G0/lambda + (3/2) N kB T0 ln(lambda)/lambda +
    [W(1->lambda) - W(lambda->1)] / (2 lambda).

    lam_fwd, w_fwd: the logged lambda and accumulated work of a run from 1
    to lambda_f; lam_bwd, w_bwd: those of the run back from lambda_f to 1.
    Each run starts with W = 0 at its schedule start (1, and lam_f for the
    way back), which is prepended to its log; a log read from the library
    holds its first row one logging interval after the start, so pass lam_f.
    lam_f = None takes the backward log's first point as its start (a log
    that already holds the start).  W(lambda->1) is the backward total
    minus the backward work done before reaching lambda.  Returns (T, G)."""
    lam = np.asarray(lam_grid, float)
    lf, wfl = np.asarray(lam_fwd, float), np.asarray(w_fwd, float)
    lam_b, w_b = np.asarray(lam_bwd, float), np.asarray(w_bwd, float)
    wf = _work_along(*_with_start(1.0, lf, wfl), lam)
    wb_total = float(w_b[-1])
    b_start = float(lam_f) if lam_f is not None else (float(lam_b[0]) if len(lam_b) else 1.0)
    wb_before = _work_along(*_with_start(b_start, lam_b, w_b), lam)
    wb = wb_total - wb_before
    G = G0 / lam + 1.5 * n_atoms * KB * T0 * np.log(lam) / lam + (wf - wb) / (2.0 * lam)
    return T0 / lam, G


def gibbs_as(G0: float, p_fwd, w_fwd, p_bwd, w_bwd, p_grid, p0=None, p1=None) -> Tuple[np.ndarray, np.ndarray]:
    """Gibbs free energy G(P, T) on p_grid from pressure switching (eq.
    Gibbs_AS): G0 + [W(P0->P) - W(P->P0)] / 2, with W = int dP/dt V dt (eq.
    Wmech_dyn) logged along the forward run P0 -> P1 and the backward run
    P1 -> P0 (pressures in the units of the work's P V, e.g. eV/A^3 with V
    in A^3).  Each run starts with W = 0 at its schedule start (p0 forward,
    p1 backward), prepended to its log; pass both with library logs, whose
    first row comes one logging interval after the start.  None takes the
    log's first point as the start (a log that already holds it).
    Returns (P, G)."""
    p = np.asarray(p_grid, float)
    pf, wfl = np.asarray(p_fwd, float), np.asarray(w_fwd, float)
    pb, wb = np.asarray(p_bwd, float), np.asarray(w_bwd, float)
    f_start = float(p0) if p0 is not None else float(pf[0])
    b_start = float(p1) if p1 is not None else float(pb[0])
    wf = _work_along(*_with_start(f_start, pf, wfl), p)
    wb_before = _work_along(*_with_start(b_start, pb, wb), p)
    return p, G0 + 0.5 * (wf - (float(wb[-1]) - wb_before))


def einstein_free_energy_difference(k1: float, k2: float, T: float, n_atoms: int) -> float:
    """F(k2) - F(k1) of a classical Einstein crystal of n_atoms 3D oscillators
    at temperature T: (3 n / 2) kB T ln(k2 / k1)."""
    return 1.5 * n_atoms * KB * T * np.log(k2 / k1)


def einstein_free_energy(n_atoms: int, k: float, T: float, mass: float) -> float:
    """Helmholtz free energy (eV) of n_atoms independent classical 3D
    oscillators of spring k (eV/A^2) and mass (amu) at T:
    3 N kB T ln(hbar omega / kB T), omega = sqrt(k / m)."""
    omega = np.sqrt(k / (mass * AMU_A2_PS2))  # 1/ps
    kT = KB * T
    return 3.0 * n_atoms * kT * np.log(HBAR * omega / kT)


def com_correction(n_atoms: int, k: float, T: float, volume: float) -> float:
    """Free energy (eV) that turns the Einstein reference of a run whose
    centre of mass is held fixed into the free crystal's:
    kB T ln[(N / V) (2 pi kB T / (N k))^(3/2)].

    Derivation (classical, atoms on their sites): holding the centre of mass
    R at the anchors' centre and the total momentum P at zero, the Einstein
    crystal's integrals over the N positions and momenta reduce to 3(N - 1)
    oscillators times N^(3/2) (positions, from delta(sum u / N)) and
    N^(-3/2) (momenta, from delta(sum p)); a translation-invariant crystal
    recovers its free integrals as (V / N) (2 pi N m kB T)^(3/2) times its
    constrained ones: R ranges over the volume per lattice translation (a
    translation by a lattice vector is a relabelling of the sites, which the
    crystal's basin already counts) and P is Gaussian with mass N m.  With
    the switching run's free-energy difference taken in the constrained
    ensemble, F_crystal = F_Einstein(N) + this term + F_SW,c - F_E,c.
    hbar and m cancel between the two pieces."""
    kT = KB * T
    return kT * np.log((n_atoms / volume) * (2.0 * np.pi * kT / (n_atoms * k)) ** 1.5)


def solid_free_energy(n_atoms: int, k: float, T: float, mass: float, volume: float,
                      w_to_einstein, w_from_einstein) -> float:
    """Absolute Helmholtz free energy (eV) of a crystal at (V, T) by
    Frenkel-Ladd switching (section 2.1): the Einstein reference (with the
    centre-of-mass term) minus F(Einstein) - F(crystal) = (mean W(crystal ->
    Einstein) - mean W(Einstein -> crystal)) / 2 (eq. dF), from runs whose
    centre of mass is fixed."""
    return (einstein_free_energy(n_atoms, k, T, mass) + com_correction(n_atoms, k, T, volume)
            - delta_f(w_to_einstein, w_from_einstein))


def ideal_gas_free_energy(n_atoms: int, volume: float, T: float, mass: float) -> float:
    """Helmholtz free energy (eV) of n_atoms classical ideal-gas atoms of mass
    (amu) in volume (A^3) at T: -kB T ln(V^N / (N! Lambda^(3N))), Lambda =
    h / sqrt(2 pi m kB T), with ln N! exact (lgamma)."""
    from math import lgamma
    kT = KB * T
    lam = 2.0 * np.pi * HBAR / np.sqrt(2.0 * np.pi * mass * AMU_A2_PS2 * kT)  # A
    return -kT * (n_atoms * np.log(volume) - lgamma(n_atoms + 1.0) - 3.0 * n_atoms * np.log(lam))


def liquid_free_energy(n_atoms: int, volume: float, T: float, mass: float, w_gas_to_uf, w_uf_to_gas,
                       w_liquid_to_uf, w_uf_to_liquid) -> float:
    """Absolute Helmholtz free energy (eV) of a liquid at (V, T) through the
    Uhlenbeck-Ford fluid (section 4.1): the ideal gas, plus F_UF - F_gas from
    switching the UF pair potential on in the ideal gas, minus F_UF -
    F_liquid from switching the liquid to the UF fluid, both at this volume
    and temperature (eq. dF for each).  Both Hamiltonians along the way are
    translation invariant, so holding the centre of mass fixed in the runs
    changes neither difference."""
    return (ideal_gas_free_energy(n_atoms, volume, T, mass) + delta_f(w_gas_to_uf, w_uf_to_gas)
            - delta_f(w_liquid_to_uf, w_uf_to_liquid))


def transition_temperature(T: float, g1: float, h1: float, g2: float, h2: float) -> float:
    """Temperature where two phases with per-atom Gibbs energies g1, g2 and
    enthalpies h1, h2 (eV) at T have equal g, taking the enthalpies constant
    near T (Gibbs-Helmholtz: g / T changes by h d(1/T)): T / (1 - (g2 - g1) /
    (h2 - h1))."""
    return T / (1.0 - (g2 - g1) / (h2 - h1))


def coexistence_pressure(P: float, g1: float, v1: float, g2: float, v2: float) -> float:
    """Pressure (GPa) where two phases with per-atom Gibbs energies g1, g2 (eV)
    and volumes v1, v2 (A^3) at pressure P (GPa) have equal g, to first order
    in the pressure: g_i(P') = g_i + v_i (P' - P)."""
    return P + (g2 - g1) / ((v1 - v2) * EV_A3_PER_GPA)


def dcci_coexistence(T0: float, lam: Sequence[float], Ps: Sequence[float]) -> Tuple[np.ndarray, np.ndarray]:
    """Points (T, P) of a dCCI coexistence line from the logged coupling
    (section 3): T = T0 / lambda, P = P_S / lambda."""
    lam = np.asarray(lam, float)
    return T0 / lam, np.asarray(Ps, float) / lam
