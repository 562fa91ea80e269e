"""Seeded synthetic inputs for the switched-Hamiltonian silicon MD path.

This module only *generates inputs*: lattice positions, random liquids,
perturbations, initial velocities, replica mixes and run settings.  It holds
none of the method's arithmetic (no potential, no integrator, no schedule), so
that the CPU oracle and the GPU path can both consume its arrays while sharing
no computational code.

Workloads follow the paper's applications section (silicon described by the
Stillinger-Weber potential; diamond, beta-tin and liquid cells of a few
thousand atoms, periodic boundaries, 1 fs time step).  The paper uses no
public dataset: every array here is synthetic and seeded.

Units are LAMMPS "metal": eV, Angstrom, ps, amu, K.  Velocities are in A/ps.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED0 = 210310449  # base seed of every generator (arXiv id of the paper)

# Physical constants used only to draw Maxwell velocities.
_KB_EV_PER_K = 8.617333262e-5          # Boltzmann constant, eV/K (CODATA 2018)
# 1 amu*A^2/ps^2 in eV, from the CODATA 2018 atomic mass unit and electronvolt
_EV_PER_AMU_A2_PS2 = 1.66053906660e-27 * 1e-20 / 1e-24 / 1.602176634e-19
SI_MASS_AMU = 28.0855

# Stillinger-Weber silicon parameters of the original 1985 paper, which the
# paper cites for its potential (applications section).  They are inputs to
# both sides; the paper itself does not print them.
SW_SILICON = dict(A=7.049556277, B=0.6022245584, p=4.0, q=0.0, a=1.80,
                  lambda_sw=21.0, gamma=1.20, sigma=2.0951, epsilon=2.1683,
                  cos0=-1.0 / 3.0)

LIQUID_DENSITY_G_CM3 = 2.57


def rng(config: int, replica: int = 0, purpose: int = 0) -> np.random.Generator:
    """PCG64 stream keyed by (SEED0, config, replica, purpose)."""
    ss = np.random.SeedSequence([SEED0, int(config), int(replica), int(purpose)])
    return np.random.Generator(np.random.PCG64(ss))


# ----------------------------------------------------------------------------
# Lattices
# ----------------------------------------------------------------------------
_DIAMOND_BASIS = np.array([
    [0.00, 0.00, 0.00], [0.00, 0.50, 0.50], [0.50, 0.00, 0.50], [0.50, 0.50, 0.00],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25],
])

# beta-tin as a body-centred tetragonal cell of 4 atoms (fractions of a, a, c)
_BETA_SN_BASIS = np.array([
    [0.0, 0.0, 0.00], [0.5, 0.5, 0.50], [0.0, 0.5, 0.25], [0.5, 0.0, 0.75],
])

_FCC_BASIS = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], dtype=float)
_SC_BASIS = np.array([[0.0, 0.0, 0.0]])


def _replicate(basis_frac: np.ndarray, cell: np.ndarray, reps) -> np.ndarray:
    nx, ny, nz = (int(r) for r in reps)
    grid = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                                indexing="ij"), axis=-1).reshape(-1, 3)
    frac = (grid[:, None, :] + basis_frac[None, :, :]).reshape(-1, 3)
    return frac * cell[None, :]


def diamond(reps=(2, 2, 2), a: float = 5.431):
    """Cubic diamond, 8 atoms per conventional cell.  Returns (x[N,3], box[3])."""
    cell = np.array([a, a, a], dtype=float)
    x = _replicate(_DIAMOND_BASIS, cell, reps)
    return x, cell * np.asarray(reps, dtype=float)


def beta_sn(reps=(10, 10, 20), a: float = 4.80, c: float = 2.65):
    """beta-tin (body-centred tetragonal, 4-atom cell).  Returns (x, box)."""
    cell = np.array([a, a, c], dtype=float)
    x = _replicate(_BETA_SN_BASIS, cell, reps)
    return x, cell * np.asarray(reps, dtype=float)


def fcc(reps=(3, 3, 3), a: float = 4.5):
    cell = np.array([a, a, a], dtype=float)
    return _replicate(_FCC_BASIS, cell, reps), cell * np.asarray(reps, dtype=float)


def simple_cubic(reps=(3, 3, 3), a: float = 3.0):
    cell = np.array([a, a, a], dtype=float)
    return _replicate(_SC_BASIS, cell, reps), cell * np.asarray(reps, dtype=float)


def liquid_number_density(rho_g_cm3: float = LIQUID_DENSITY_G_CM3,
                          mass_amu: float = SI_MASS_AMU) -> float:
    """Atoms per A^3 at a mass density in g/cm^3."""
    avogadro = 6.02214076e23
    return rho_g_cm3 * avogadro / mass_amu * 1e-24


def liquid_rsa(n_atoms: int, g: np.random.Generator, density: Optional[float] = None,
               d_min: float = 2.0, max_tries: int = 200):
    """Random sequential addition of hard spheres of diameter d_min in a cubic box.

    A disordered (liquid-like) start at the given number density; with
    d_min = 2.0 A the packing fraction at 2.57 g/cm^3 is about 0.23, far below
    the RSA jamming limit, so placement always succeeds.  Candidates are
    tested against the atoms already placed in the 27 surrounding bins (bin
    width >= d_min).  max_tries bounds the attempts per atom.
    """
    if density is None:
        density = liquid_number_density()
    L = (n_atoms / density) ** (1.0 / 3.0)
    nb = max(1, int(L // d_min))
    bw = L / nb
    cap = 64
    bins = -np.ones((nb, nb, nb, cap), dtype=np.int64)
    fill = np.zeros((nb, nb, nb), dtype=np.int64)
    rng_off = np.array([-1, 0, 1]) if nb >= 3 else np.arange(nb)
    offs = np.array([(a, b, c) for a in rng_off for b in rng_off for c in rng_off])
    x = np.empty((n_atoms, 3))
    d2 = d_min * d_min
    placed = 0
    tries = 0
    while placed < n_atoms:
        tries += 1
        if tries > max_tries * n_atoms:
            raise RuntimeError("RSA failed to place all atoms")
        p = g.random(3) * L
        b = (p // bw).astype(np.int64) % nb
        nbr = (b[None, :] + offs) % nb if nb >= 3 else offs
        cand = bins[nbr[:, 0], nbr[:, 1], nbr[:, 2]].ravel()
        cand = cand[cand >= 0]
        if cand.size:
            d = x[cand] - p
            d -= L * np.round(d / L)
            if np.einsum("ij,ij->i", d, d).min() < d2:
                continue
        if fill[b[0], b[1], b[2]] >= cap:
            raise RuntimeError("RSA bin capacity exceeded")
        x[placed] = p
        bins[b[0], b[1], b[2], fill[b[0], b[1], b[2]]] = placed
        fill[b[0], b[1], b[2]] += 1
        placed += 1
    return x, np.array([L, L, L])


# ----------------------------------------------------------------------------
# Perturbations and velocities
# ----------------------------------------------------------------------------
def perturb(x: np.ndarray, sigma: float, g: np.random.Generator) -> np.ndarray:
    """Gaussian displacement per Cartesian component, with zero mean displacement."""
    d = g.normal(0.0, sigma, size=x.shape)
    d -= d.mean(axis=0, keepdims=True)
    return x + d


def maxwell(n_atoms: int, T: float, g: np.random.Generator,
            mass: float = SI_MASS_AMU) -> np.ndarray:
    """Maxwell velocities (A/ps) with zero total momentum, rescaled so that the
    kinetic temperature over 3N-3 degrees of freedom is exactly T."""
    if T <= 0.0 or n_atoms < 2:
        return np.zeros((n_atoms, 3))
    sig = np.sqrt(_KB_EV_PER_K * T / (mass * _EV_PER_AMU_A2_PS2))
    v = g.normal(0.0, sig, size=(n_atoms, 3))
    v -= v.mean(axis=0, keepdims=True)
    ke2 = mass * _EV_PER_AMU_A2_PS2 * float((v * v).sum())       # 2K in eV
    t_now = ke2 / ((3 * n_atoms - 3) * _KB_EV_PER_K)
    return v * np.sqrt(T / t_now)


# ----------------------------------------------------------------------------
# Workload descriptions (shapes, sizes, settings).  Mode names match the
# library's: 0 force-only, 1 NVE, 2 NVT, 3 Frenkel-Ladd, 4 reversible scaling,
# 5 pressure switching, 6 dCCI (temperature control), 7 dCCI (pressure control)
# ----------------------------------------------------------------------------
MODE_FORCE, MODE_NVE, MODE_NVT, MODE_FL, MODE_RS, MODE_AS_P, MODE_DCCI_T, MODE_DCCI_P, MODE_UF = range(9)
BARO_ISO, BARO_ANISO = 0, 1
# Uhlenbeck-Ford fluid reference of the liquid (section 4.1): p, sigma (A);
# the temperature is the run's, the cutoff 4 sigma
UF_P, UF_SIGMA, UF_RCUT = 25.0, 2.0, 8.0


@dataclass
class SystemSpec:
    x: np.ndarray                 # (N,3) positions, A
    v: np.ndarray                 # (N,3) velocities, A/ps
    box: np.ndarray               # (3,) orthorhombic box, A
    phase: str = "diamond"
    x0: Optional[np.ndarray] = None   # Einstein anchors (Frenkel-Ladd)
    mode: int = MODE_NVT
    partner: int = -1
    k_spring: float = 0.0          # eV/A^2
    T0: float = 1000.0             # thermostat temperature, K
    tau_damp: float = 0.1          # Langevin damping time, ps
    p_damp: float = 0.0            # barostat period, ps (0: fixed box)
    pressure: float = 0.0          # physical pressure P, GPa
    stream: int = 0                # noise stream id (Philox key word 1)
    baro: int = 0                  # 0: one piston (volume), 1: one piston per box length
    uf_p: float = 0.0              # Uhlenbeck-Ford reference (MODE_UF): p, sigma (A), T (K), cutoff (A)
    uf_sigma: float = 0.0
    uf_T: float = 0.0
    uf_rcut: float = 0.0
    # schedule: lam_start/lam_end (FL, RS), or the controlled variable's
    # start/end (P in GPa for pressure switching and dCCI-P, T in K for dCCI-T)
    sched_start: float = 1.0
    sched_end: float = 1.0
    sched_steps: int = 0

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclass
class Workload:
    name: str
    systems: List[SystemSpec] = field(default_factory=list)
    dt: float = 0.001              # ps
    steps: int = 1000
    seed: int = SEED0

    @property
    def n_atoms(self) -> int:
        return sum(s.n for s in self.systems)


def config1(lam_forward: bool = True) -> Workload:
    """64-atom diamond (2x2x2, a = 5.431), sigma = 0.05 A perturbation,
    Maxwell 1000 K, Frenkel-Ladd with k = 5 eV/A^2, 1000 steps, 0.1 ps damping.
    lam_forward: interacting -> Einstein (lambda 1 -> 0, the paper's direction);
    otherwise the reverse."""
    g = rng(1, 0, 0)
    x0, box = diamond((2, 2, 2), 5.431)
    x = perturb(x0, 0.05, g)
    v = maxwell(len(x), 1000.0, rng(1, 0, 1))
    s0, s1 = (1.0, 0.0) if lam_forward else (0.0, 1.0)
    sys = SystemSpec(x=x, v=v, box=box, phase="diamond", x0=x0.copy(), mode=MODE_FL,
                     k_spring=5.0, T0=1000.0, tau_damp=0.1, stream=0,
                     sched_start=s0, sched_end=s1, sched_steps=1000)
    return Workload("c1-diamond64-fl", [sys], steps=1000)


def config2(phase: str = "diamond", steps: int = 20000) -> Workload:
    """8000-atom diamond (10^3 cells) or 8000-atom liquid (RSA at 2.57 g/cm^3),
    reversible scaling T 1000 -> 2000 K (lambda 1 -> 0.5) at P = 0, NPT."""
    if phase == "diamond":
        x0, box = diamond((10, 10, 10), 5.431)
        x = perturb(x0, 0.05, rng(2, 0, 0))
    else:
        x, box = liquid_rsa(8000, rng(2, 1, 0))
    v = maxwell(len(x), 1000.0 if phase == "diamond" else 3000.0, rng(2, 0 if phase == "diamond" else 1, 1))
    sys = SystemSpec(x=x, v=v, box=box, phase=phase, mode=MODE_RS, T0=1000.0, tau_damp=0.1,
                     p_damp=1.0, pressure=0.0, stream=0 if phase == "diamond" else 1,
                     sched_start=1.0, sched_end=0.5, sched_steps=steps)
    return Workload(f"c2-{phase}8000-rs", [sys], steps=steps)


def config3(steps: int = 100000) -> Workload:
    """dCCI coupled pair: 4096-atom diamond + 8000-atom beta-tin, NPT at
    T0 = 400 K, pressure-controlled, P 0 -> 15 GPa over `steps`."""
    xd, bd = diamond((8, 8, 8), 5.431)
    xd = perturb(xd, 0.05, rng(3, 0, 0))
    xb, bb = beta_sn((10, 10, 20), 4.80, 2.65)
    xb = perturb(xb, 0.05, rng(3, 1, 0))
    T0 = 400.0
    s0 = SystemSpec(x=xd, v=maxwell(len(xd), T0, rng(3, 0, 1)), box=bd, phase="diamond",
                    mode=MODE_DCCI_P, partner=1, T0=T0, tau_damp=0.1, p_damp=1.0,
                    pressure=0.0, stream=0, sched_start=0.0, sched_end=15.0, sched_steps=steps)
    s1 = SystemSpec(x=xb, v=maxwell(len(xb), T0, rng(3, 1, 1)), box=bb, phase="beta-sn",
                    mode=MODE_DCCI_P, partner=0, T0=T0, tau_damp=0.1, p_damp=1.0,
                    pressure=0.0, stream=1, sched_start=0.0, sched_end=15.0, sched_steps=steps)
    return Workload("c3-dcci-diamond4096-betasn8000", [s0, s1], steps=steps)


def config4_sizes(n_rep: int = 64):
    """Seeded replica mix: phases and sizes log-uniform in [512, 13824].
    Solids are snapped to 8 n^3 atoms (n = 4..12); liquids keep a free size."""
    g = rng(4, 0, 0)
    phases = g.choice(["diamond", "beta-sn", "liquid"], size=n_rep)
    raw = np.exp(g.uniform(np.log(512.0), np.log(13824.0), size=n_rep))
    out = []
    for ph, n in zip(phases, raw):
        if ph == "liquid":
            out.append((str(ph), int(round(n))))
        else:
            m = int(np.clip(round((n / 8.0) ** (1.0 / 3.0)), 4, 12))
            out.append((str(ph), 8 * m ** 3))
    return out


def config4(n_rep: int = 64, steps: int = 1000, sizes=None) -> Workload:
    """64 independent switching replicas of uneven size.  Solids (diamond,
    beta-tin) run Frenkel-Ladd (k = 5 eV/A^2, lambda 1 -> 0, NVT at 1000 K);
    liquids run reversible scaling (lambda 1 -> 0.5, NPT at P = 0, T0 = 1700 K)."""
    sizes = sizes if sizes is not None else config4_sizes(n_rep)
    systems = []
    for r, (ph, n) in enumerate(sizes):
        if ph == "diamond":
            m = round((n / 8) ** (1 / 3))
            xl, box = diamond((m, m, m), 5.431)
            x = perturb(xl, 0.05, rng(4, r, 1))
            T0 = 1000.0
            spec = SystemSpec(x=x, v=maxwell(n, T0, rng(4, r, 2)), box=box, phase=ph, x0=xl,
                              mode=MODE_FL, k_spring=5.0, T0=T0, tau_damp=0.1, stream=r,
                              sched_start=1.0, sched_end=0.0, sched_steps=steps)
        elif ph == "beta-sn":
            m = round((n / 8) ** (1 / 3))
            xl, box = beta_sn((m, m, 2 * m), 4.80, 2.65)
            x = perturb(xl, 0.05, rng(4, r, 1))
            T0 = 1000.0
            spec = SystemSpec(x=x, v=maxwell(n, T0, rng(4, r, 2)), box=box, phase=ph, x0=xl,
                              mode=MODE_FL, k_spring=5.0, T0=T0, tau_damp=0.1, stream=r,
                              sched_start=1.0, sched_end=0.0, sched_steps=steps)
        else:
            x, box = liquid_rsa(n, rng(4, r, 1))
            T0 = 1700.0
            spec = SystemSpec(x=x, v=maxwell(n, T0, rng(4, r, 2)), box=box, phase=ph,
                              mode=MODE_RS, T0=T0, tau_damp=0.1, p_damp=1.0, pressure=0.0,
                              stream=r, sched_start=1.0, sched_end=0.5, sched_steps=steps)
        systems.append(spec)
    return Workload(f"c4-batched{n_rep}", systems, steps=steps)


def config5(T: float = 1700.0) -> Workload:
    """32768-atom diamond (16^3 cells), Gaussian sigma = 0.15 A (about the
    harmonic amplitude at 1700 K), for energy/force/virial/parameter gradients."""
    xl, box = diamond((16, 16, 16), 5.431)
    x = perturb(xl, 0.15, rng(5, 0, 0))
    sys = SystemSpec(x=x, v=np.zeros_like(x), box=box, phase="diamond", mode=MODE_FORCE, T0=T)
    return Workload("c5-diamond32768-grad", [sys], steps=0)


def random_box(n_atoms: int, L: float, g: np.random.Generator, d_min: float = 1.9):
    """Small random configurations for brute-force checks."""
    x, _ = liquid_rsa(n_atoms, g, density=n_atoms / L ** 3, d_min=d_min)
    return x, np.array([L, L, L])
