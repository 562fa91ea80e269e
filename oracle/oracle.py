"""Plain FP64 CPU oracle for switched-Hamiltonian silicon MD.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code,
constant or helper with the GPU library (``paper_2103_10449_amd``): the two
meet only through arrays drawn by the seeded input generators.

Contents, each citing the passage of the paper it follows:

* ``sw_eval``      Stillinger-Weber energy / forces / virial / dE/dtheta by
                   direct pair and triplet sums (``sw_oracle.c``); the paper's
                   silicon model (applications section).
* ``einstein``     Einstein-crystal reference (section 2.1, the reference
                   system for solids).
* ``uf_eval``      Uhlenbeck-Ford fluid reference (section 4.1, p = 25,
                   sigma = 2.0; model of Leite et al.), switched to like the
                   Einstein crystal: H = lam U + (1 - lam) U_UF.
* ``philox4x64``   Philox4x64-10 (Salmon et al., SC'11), from its published
                   definition; drives the thermostat noise.
* ``Oracle.step``  one step of the switched dynamics: the lambda switch with
                   its work increment (eq. Wdyn, section 2), velocity Verlet
                   with a Langevin O-step and an isotropic or per-axis
                   (anisotropic) barostat.
* schedules        Frenkel-Ladd lambda(t) (section 2.1), reversible scaling
                   lambda(t) = 1/(1 + t/t_s (1/lambda_f - 1)) with P_S =
                   lambda P (eqs. T_sc, P_sc, section 4.1), pressure switching
                   (eq. Wmech_dyn), dCCI with lambda control (eq.
                   Ps_coex_discreted) and pressure control (eq.
                   l_coex_discreted), section 3.
* estimators       Delta F and Q_diss (eqs. dF, Qdiss), the reversible-scaling
                   Gibbs free energy (eq. Gibbs_RS), Einstein free energies.

Readings where the paper is silent (integrator splitting, barostat, noise
scheme, work discretisation) are the same ones the GPU library implements,
each stated at the function that takes it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# ---------------------------------------------------------------------------
# Physical constants (CODATA 2018), defined here independently of the GPU side
# ---------------------------------------------------------------------------
KB = 8.617333262e-5                                   # eV/K
MVV2E = 1.66053906660e-27 * 1e-20 / 1e-24 / 1.602176634e-19  # eV per amu*A^2/ps^2
GPA_PER_EV_A3 = 1.602176634e-19 / 1e-30 / 1e9         # GPa per eV/A^3
MASS_SI = 28.0855                                     # amu

PARAM_NAMES = ("A", "B", "p", "q", "a", "lambda_sw", "gamma", "sigma", "epsilon")

MODE_FORCE, MODE_NVE, MODE_NVT, MODE_FL, MODE_RS, MODE_AS_P, MODE_DCCI_T, MODE_DCCI_P = range(8)
# switching between the interaction and the Uhlenbeck-Ford fluid (section 4.1)
MODE_UF = 8
# barostat: one piston for the volume (isotropic) or one per box length (the
# paper's `aniso` runs of beta-tin, section 4.1)
BARO_ISO, BARO_ANISO = 0, 1
ERR_DCCI_SINGULAR = 1


def build(force: bool = True) -> str:
    """Compile the C part with gcc.  Returns the library path."""
    src = os.path.join(_HERE, "sw_oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _SW(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("A", "B", "p", "q", "a", "lam", "gam", "sig", "eps", "cos0")]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_sw_eval.argtypes = [ctypes.c_int, dp, dp, ctypes.POINTER(_SW), ctypes.c_int,
                                    dp, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_int)]
        lib.orc_sw_eval.restype = ctypes.c_int
        lib.orc_einstein.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, dp]
        lib.orc_uf_eval.argtypes = [ctypes.c_int, dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, dp, dp, dp, dp]
        lib.orc_uf_eval.restype = ctypes.c_int
        lib.orc_einstein.restype = ctypes.c_double
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = None
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    """Threads of the neighbour search (default 1).  Each atom's neighbours
    are found independently and listed in the same order for any count, so
    no result depends on it; it only shortens large evaluations."""
    _load().orc_set_threads(int(n))


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _sw_struct(params: dict) -> _SW:
    return _SW(params["A"], params["B"], params["p"], params["q"], params["a"],
               params["lambda_sw"], params["gamma"], params["sigma"], params["epsilon"],
               params.get("cos0", -1.0 / 3.0))


def cell_matrix(box) -> np.ndarray:
    """3x3 cell matrix, columns are box vectors; accepts (3,) lengths or (3,3)."""
    b = np.asarray(box, dtype=np.float64)
    return np.diag(b) if b.shape == (3,) else np.ascontiguousarray(b)


def sw_eval(x: np.ndarray, box, params: dict, force_images: bool = False,
            need_forces: bool = True, need_dtheta: bool = True) -> dict:
    """Stillinger-Weber energy, forces, virial and parameter gradient.

    x: (N,3) Cartesian positions; box: (3,) orthorhombic lengths or a (3,3)
    cell matrix (columns are box vectors).  Returns a dict with E2, E3, E,
    F (N,3), virial (3,3) = dE/dstrain, dtheta (9,) in PARAM_NAMES order,
    e_atom (N,), nnb (N,).
    """
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    h = cell_matrix(box)
    sw = _sw_struct(params)
    e = np.zeros(2)
    F = np.zeros((n, 3)) if need_forces else None
    vir = np.zeros(9)
    dth = np.zeros(9) if need_dtheta else None
    ea = np.zeros(n)
    nnb = np.zeros(n, dtype=np.int32)
    rc = lib.orc_sw_eval(n, _ptr(x), _ptr(h), ctypes.byref(sw), int(force_images), _ptr(e),
                         _ptr(F), _ptr(vir), _ptr(dth), _ptr(ea),
                         nnb.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if rc != 0:
        raise MemoryError("oracle neighbour list allocation failed")
    return dict(E2=e[0], E3=e[1], E=e[0] + e[1], F=F, virial=vir.reshape(3, 3),
                dtheta=dth, e_atom=ea, nnb=nnb)


def uf_eval(x: np.ndarray, box, p: float, sigma: float, T: float, rcut: float,
            force_images: bool = False) -> dict:
    """Uhlenbeck-Ford reference (section 4.1; Leite et al.): energy, forces,
    virial and per-atom energy of phi(r) = -p kB T ln(1 - exp(-(r/sigma)^2)),
    truncated at rcut."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = x.shape[0]
    h = cell_matrix(box)
    e = np.zeros(1)
    F = np.zeros((n, 3))
    vir = np.zeros(9)
    ea = np.zeros(n)
    rc = lib.orc_uf_eval(n, _ptr(x), _ptr(h), p * KB * T, sigma, rcut, int(force_images), _ptr(e), _ptr(F),
                         _ptr(vir), _ptr(ea))
    if rc != 0:
        raise MemoryError("oracle neighbour list allocation failed")
    return dict(E=e[0], F=F, virial=vir.reshape(3, 3), e_atom=ea)


def einstein(x: np.ndarray, x0: np.ndarray, k: float):
    """Einstein crystal U_ref = sum k/2 |x - x0|^2 and F_ref = -k (x - x0)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    F = np.zeros_like(x)
    U = lib.orc_einstein(x.shape[0], _ptr(x), _ptr(x0), float(k), _ptr(F))
    return U, F


# ---------------------------------------------------------------------------
# Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
# as 1, 2, 3", SC'11), vectorised over counters.
# ---------------------------------------------------------------------------
_M32 = np.uint64(0xFFFFFFFF)
_PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
_PHILOX_M1 = np.uint64(0xCA5A826395121157)
_PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
_PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)


def _mulhilo(a: np.uint64, b: np.ndarray):
    """64x64 -> 128-bit product of a constant and an array: (hi, lo)."""
    a_lo, a_hi = a & _M32, a >> np.uint64(32)
    b_lo, b_hi = b & _M32, b >> np.uint64(32)
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> np.uint64(32)) + (lh & _M32) + (hl & _M32)
    hi = hh + (lh >> np.uint64(32)) + (hl >> np.uint64(32)) + (mid >> np.uint64(32))
    lo = a * b
    return hi, lo


def philox4x64(counter: Sequence[np.ndarray], key: Sequence[int]) -> List[np.ndarray]:
    """Ten rounds of Philox4x64 on counters (c0..c3, arrays or scalars) with a
    two-word key.  Returns the four output words as uint64 arrays."""
    with np.errstate(over="ignore"):
        c = [np.asarray(ci, dtype=np.uint64) for ci in np.broadcast_arrays(*counter)]
        k0, k1 = np.uint64(key[0]), np.uint64(key[1])
        for r in range(10):
            if r > 0:
                k0 = k0 + _PHILOX_W0
                k1 = k1 + _PHILOX_W1
            hi0, lo0 = _mulhilo(_PHILOX_M0, c[0])
            hi1, lo1 = _mulhilo(_PHILOX_M1, c[2])
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def uniform_open0(w: np.ndarray) -> np.ndarray:
    """53-bit uniform in (0, 1] from a 64-bit word."""
    return ((w >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)


def normals(seed: int, stream: int, step: int, n_atoms: int) -> np.ndarray:
    """Three standard normals per atom for one step: Philox4x64-10 with key
    (seed, stream) and counter (step, atom, 0, 0); Box-Muller on the words."""
    atoms = np.arange(n_atoms, dtype=np.uint64)
    w = philox4x64([np.uint64(step), atoms, np.uint64(0), np.uint64(0)], (seed, stream))
    u0, u1, u2, u3 = (uniform_open0(wi) for wi in w)
    r01 = np.sqrt(-2.0 * np.log(u0))
    r23 = np.sqrt(-2.0 * np.log(u2))
    out = np.empty((n_atoms, 3))
    out[:, 0] = r01 * np.cos(2.0 * np.pi * u1)
    out[:, 1] = r01 * np.sin(2.0 * np.pi * u1)
    out[:, 2] = r23 * np.cos(2.0 * np.pi * u3)
    return out


# ---------------------------------------------------------------------------
# Switched dynamics
# ---------------------------------------------------------------------------
@dataclass
class OSystem:
    """One periodic system and its switching state (all FP64)."""
    x: np.ndarray
    v: np.ndarray
    box: np.ndarray
    mode: int = MODE_NVT
    x0: Optional[np.ndarray] = None
    partner: int = -1
    k_spring: float = 0.0
    T0: float = 0.0
    tau_damp: float = 0.0
    p_damp: float = 0.0
    pressure: float = 0.0          # GPa
    stream: int = 0
    baro: int = BARO_ISO
    # Uhlenbeck-Ford reference (MODE_UF): p, sigma (A), temperature (K), cutoff (A)
    uf_p: float = 25.0
    uf_sigma: float = 2.0
    uf_T: float = 0.0
    uf_rcut: float = 8.0
    sched_start: float = 1.0
    sched_end: float = 1.0
    sched_steps: int = 0
    # dynamic state
    lam: float = 1.0
    Ps: float = 0.0                # scaled barostat target, eV/A^3
    veps: float = 0.0              # barostat rate p_eps / W, 1/ps (isotropic)
    veps3: Optional[np.ndarray] = None  # per-axis rates d ln L_a / dt, 1/ps (anisotropic)
    W: float = 0.0                 # accumulated work, eV
    step: int = 0                  # global step counter (noise counter)
    k: int = 0                     # steps since the schedule started
    err: int = 0
    # cached interaction at the current positions
    F_int: Optional[np.ndarray] = None
    U_int: float = 0.0
    Xi_int: Optional[np.ndarray] = None
    U_ref: float = 0.0
    log: list = field(default_factory=list)

    @property
    def n(self) -> int:
        return self.x.shape[0]

    @property
    def volume(self) -> float:
        return float(np.prod(self.box))

    def kinetic(self) -> float:
        return 0.5 * MASS_SI * MVV2E * float((self.v * self.v).sum())

    def kinetic_axes(self) -> np.ndarray:
        """K_a = m/2 sum_i v_ia^2 for a = x, y, z."""
        return 0.5 * MASS_SI * MVV2E * (self.v * self.v).sum(axis=0)

    def temperature(self) -> float:
        return 2.0 * self.kinetic() / ((3 * self.n - 3) * KB)


def _progress(s: OSystem, k: int) -> float:
    if s.sched_steps <= 0:
        return 1.0
    return min(k, s.sched_steps) / s.sched_steps


def _controlled(s: OSystem, k: int) -> float:
    """Linear ramp of the controlled variable (lambda for FL, 1/lambda for RS,
    P in GPa for pressure switching and dCCI-P, T in K for dCCI-T)."""
    f = _progress(s, k)
    return s.sched_start + (s.sched_end - s.sched_start) * f


def initial_switch_state(s: OSystem):
    """lambda and P_S at the start of a schedule."""
    if s.mode in (MODE_FL, MODE_UF):
        s.lam, s.Ps = s.sched_start, 0.0
    elif s.mode == MODE_RS:
        # reversible scaling: T = T0/lambda (eq. T_sc), P_S = lambda P (eq. P_sc)
        s.lam = s.sched_start
        s.Ps = s.lam * s.pressure / GPA_PER_EV_A3
    elif s.mode == MODE_AS_P:
        s.lam, s.Ps = 1.0, s.sched_start / GPA_PER_EV_A3
    elif s.mode == MODE_DCCI_T:
        s.lam = s.T0 / s.sched_start
        s.Ps = s.lam * s.pressure / GPA_PER_EV_A3
    elif s.mode == MODE_DCCI_P:
        s.lam = 1.0
        s.Ps = s.sched_start / GPA_PER_EV_A3
    else:
        s.lam, s.Ps = 1.0, s.pressure / GPA_PER_EV_A3
    s.W = 0.0
    s.k = 0


def _lam_rs(s: OSystem, k: int) -> float:
    # 1/lambda linear in time, i.e. lambda(t) = 1/(1 + t/t_s (1/lambda_f - 1))
    f = _progress(s, k)
    inv = 1.0 / s.sched_start + (1.0 / s.sched_end - 1.0 / s.sched_start) * f
    return 1.0 / inv


def hamiltonian_switch_part(s: OSystem, lam: float, Ps: float) -> float:
    """The lambda- and P_S-dependent part of H at the current microstate."""
    if s.mode in (MODE_FL, MODE_UF):
        return lam * s.U_int + (1.0 - lam) * s.U_ref
    if s.mode in (MODE_RS, MODE_DCCI_T, MODE_DCCI_P):
        return lam * s.U_int + Ps * s.volume
    if s.mode == MODE_AS_P:
        return Ps * s.volume
    return 0.0


def dcci_update(sI: OSystem, sII: OSystem, k: int):
    """Next (lambda, P_S) of a coupled pair from the instantaneous per-atom
    energy and volume differences of the two phases (section 3).  Returns
    (lam, Ps, singular)."""
    du = sI.U_int / sI.n - sII.U_int / sII.n
    dv = sI.volume / sI.n - sII.volume / sII.n
    lam, Ps = sI.lam, sI.Ps
    if abs(dv) < 1e-6:
        return lam, Ps, True
    if sI.mode == MODE_DCCI_T:
        # temperature control: T linear, lambda = T0/T, eq. Ps_coex_discreted
        lam_new = sI.T0 / _controlled(sI, k + 1)
        Ps_new = Ps - (lam_new - lam) * du / dv
    else:
        # pressure control: P linear, eq. l_coex_discreted, then P_S = lambda P
        Pk = _controlled(sI, k) / GPA_PER_EV_A3
        Pk1 = _controlled(sI, k + 1) / GPA_PER_EV_A3
        if du == 0.0:
            return lam, Ps, True
        den = 1.0 + Pk1 * dv / du
        if abs(den) < 1e-3:
            return lam, Ps, True
        lam_new = lam * (1.0 + Pk * dv / du) / den
        Ps_new = lam_new * Pk1
    if not (0.05 < lam_new < 20.0):
        return lam, Ps, True
    return lam_new, Ps_new, False


class Oracle:
    """Lock-step switched dynamics of a list of systems (dCCI pairs coupled).

    Step order (identical on the GPU side):
      1. switch lambda_k -> lambda_{k+1} (and P_S) at the current microstate,
         W += H(lambda_{k+1}, z_k) - H(lambda_k, z_k)
      2. barostat half step of the piston rate
      3. B: half kick with F(lambda_{k+1})
      4. A: half drift (with box scaling, isotropic or per axis)
      5. O: Langevin step with zero-sum noise
      6. A: half drift
      7. interaction at the new positions
      8. B: half kick
      9. barostat half step
    """

    def __init__(self, systems: List[OSystem], params: dict, dt: float = 0.001, seed: int = 0):
        self.systems = systems
        self.params = params
        self.dt = dt
        self.seed = seed
        for s in systems:
            s.x = np.array(s.x, dtype=np.float64)
            s.v = np.array(s.v, dtype=np.float64)
            s.box = np.array(s.box, dtype=np.float64)
            initial_switch_state(s)
            self.forces(s)

    # ---- interaction --------------------------------------------------------
    def forces(self, s: OSystem):
        r = sw_eval(s.x, s.box, self.params, need_dtheta=False)
        s.F_int, s.U_int, s.Xi_int = r["F"], r["E"], r["virial"]
        if s.mode == MODE_FL and s.x0 is not None:
            s.U_ref, s.F_ref = einstein(s.x, s.x0, s.k_spring)
        elif s.mode == MODE_UF:
            u = uf_eval(s.x, s.box, s.uf_p, s.uf_sigma, s.uf_T, s.uf_rcut)
            s.U_ref, s.F_ref = u["E"], u["F"]
        else:
            s.U_ref, s.F_ref = 0.0, np.zeros_like(s.x)

    def total_force(self, s: OSystem, lam: float) -> np.ndarray:
        if s.mode in (MODE_FL, MODE_UF):
            return lam * s.F_int + (1.0 - lam) * s.F_ref
        if s.mode in (MODE_RS, MODE_DCCI_T, MODE_DCCI_P):
            return lam * s.F_int
        return s.F_int

    def _xi_trace(self, s: OSystem, lam: float) -> float:
        tr = float(np.trace(s.Xi_int))
        return lam * tr if s.mode in (MODE_RS, MODE_DCCI_T, MODE_DCCI_P) else tr

    def _xi_diag(self, s: OSystem, lam: float) -> np.ndarray:
        d = np.diag(s.Xi_int).copy()
        return lam * d if s.mode in (MODE_RS, MODE_DCCI_T, MODE_DCCI_P) else d

    # ---- barostat -----------------------------------------------------------
    def _baro_half(self, s: OSystem, lam: float, Ps: float):
        """Half step of the piston rate(s).  Isotropic (MTK, one piston of mass
        W = (N_f + 3) kB T0 tau_p^2 for eps = ln L):
            dv_eps/dt = [alpha 2K - tr Xi - 3 V P_S] / W,  alpha = 1 + 3/N_f.
        Per axis (eps_a = ln L_a, pistons of mass W/3 so that equal stresses
        move the three axes as the isotropic piston):
            dv_a/dt = [2K_a + 2K/N_f - Xi_aa - V P_S] / (W/3)."""
        if s.p_damp <= 0.0:
            return
        nf = 3 * s.n - 3
        wp = (nf + 3) * KB * s.T0 * s.p_damp ** 2
        if s.baro == BARO_ANISO:
            if s.veps3 is None:
                s.veps3 = np.zeros(3)
            g = 2.0 * s.kinetic_axes() + 2.0 * s.kinetic() / nf - self._xi_diag(s, lam) - s.volume * Ps
            s.veps3 = s.veps3 + 0.5 * self.dt * g / (wp / 3.0)
            return
        alpha = 1.0 + 3.0 / nf
        g = alpha * 2.0 * s.kinetic() - self._xi_trace(s, lam) - 3.0 * s.volume * Ps
        s.veps += 0.5 * self.dt * g / wp

    def _factors(self, s: OSystem):
        """Per-axis factors of the kick (velocity damping by the piston:
        dv_a/dt = F_a/m - (v_eps,a + tr v_eps / N_f) v_a) and of the drift
        (dx_a/dt = v_a + v_eps,a x_a), exact over a half step."""
        dt = self.dt
        nf = 3 * s.n - 3
        if s.baro == BARO_ANISO and s.p_damp > 0.0:
            v3 = s.veps3 if s.veps3 is not None else np.zeros(3)
            zk = (v3 + v3.sum() / nf) * 0.5 * dt
            za = v3 * 0.5 * dt
        else:
            alpha = 1.0 + 3.0 / nf
            zk = np.full(3, alpha * s.veps * 0.5 * dt)
            za = np.full(3, s.veps * 0.5 * dt)
        decay = np.exp(-zk)
        phi = np.where(zk == 0.0, 1.0, -np.expm1(-zk) / np.where(zk == 0.0, 1.0, zk))
        grow = np.exp(za)
        psi = np.where(za == 0.0, 1.0, np.expm1(za) / np.where(za == 0.0, 1.0, za))
        return decay, phi, grow, psi

    # ---- the step -----------------------------------------------------------
    def step(self):
        dt = self.dt
        new = []
        for i, s in enumerate(self.systems):
            if s.mode in (MODE_DCCI_T, MODE_DCCI_P):
                if s.partner > i:
                    lam, Ps, bad = dcci_update(s, self.systems[s.partner], s.k)
                    new.append((lam, Ps, bad))
                else:
                    new.append(None)
            elif s.mode in (MODE_FL, MODE_UF):
                new.append((_controlled(s, s.k + 1), 0.0, False))
            elif s.mode == MODE_RS:
                lam = _lam_rs(s, s.k + 1)
                new.append((lam, lam * s.pressure / GPA_PER_EV_A3, False))
            elif s.mode == MODE_AS_P:
                new.append((1.0, _controlled(s, s.k + 1) / GPA_PER_EV_A3, False))
            else:
                new.append((s.lam, s.Ps, False))
        for i, s in enumerate(self.systems):
            if new[i] is None:
                new[i] = new[s.partner]
        # 1. switch and work
        for s, (lam, Ps, bad) in zip(self.systems, new):
            if bad:
                s.err |= ERR_DCCI_SINGULAR
            s.W += hamiltonian_switch_part(s, lam, Ps) - hamiltonian_switch_part(s, s.lam, s.Ps)
            s.lam, s.Ps = lam, Ps
        for s in self.systems:
            if s.mode == MODE_FORCE:
                continue
            # 2. barostat half step
            self._baro_half(s, s.lam, s.Ps)
            decay, phi, grow, psi = self._factors(s)
            acc = 1.0 / MVV2E / MASS_SI
            # 3. B
            s.v = s.v * decay + 0.5 * dt * acc * self.total_force(s, s.lam) * phi
            # 4. A
            s.x = s.x * grow + s.v * (0.5 * dt) * psi
            s.box = s.box * grow
            # 5. O
            if s.mode != MODE_NVE and s.tau_damp > 0.0 and s.T0 > 0.0:
                c1 = np.exp(-dt / s.tau_damp)
                c2 = np.sqrt(1.0 - c1 * c1)
                sv = np.sqrt(KB * s.T0 / (MASS_SI * MVV2E))
                xi = normals(self.seed, s.stream, s.step, s.n)
                xi -= xi.mean(axis=0, keepdims=True)
                s.v = c1 * s.v + c2 * sv * xi
            # 6. A
            s.x = s.x * grow + s.v * (0.5 * dt) * psi
            s.box = s.box * grow
            # 7. interaction
            self.forces(s)
            # 8. B
            s.v = s.v * decay + 0.5 * dt * acc * self.total_force(s, s.lam) * phi
            # 9. barostat half step
            self._baro_half(s, s.lam, s.Ps)
            s.step += 1
            s.k += 1

    def run(self, n_steps: int, log_every: int = 0):
        for _ in range(n_steps):
            self.step()
            if log_every and self.systems[0].k % log_every == 0:
                for s in self.systems:
                    s.log.append((s.k, s.lam, s.Ps * GPA_PER_EV_A3, s.temperature(),
                                  s.U_int / s.n, s.volume / s.n, s.W))


# ---------------------------------------------------------------------------
# Estimators (host side)
# ---------------------------------------------------------------------------
def delta_f(w_forward, w_backward) -> float:
    """F(lambda_f) - F(lambda_i) = (mean W(i->f) - mean W(f->i)) / 2 (eq. dF)."""
    return 0.5 * (float(np.mean(w_forward)) - float(np.mean(w_backward)))


def q_diss(w_forward, w_backward) -> float:
    """Mean dissipated heat (mean W(i->f) + mean W(f->i)) / 2 (eq. Qdiss)."""
    return 0.5 * (float(np.mean(w_forward)) + float(np.mean(w_backward)))


def einstein_free_energy_difference(k1: float, k2: float, T: float, n_modes_atoms: int) -> float:
    """F(k2) - F(k1) of classical Einstein crystals with n_modes_atoms
    independent 3D oscillators: (3 n / 2) kB T ln(k2 / k1)."""
    return 1.5 * n_modes_atoms * KB * T * np.log(k2 / k1)


def gibbs_rs(G0: float, lam: float, n_atoms: int, T0: float, w_fwd: float, w_bwd: float) -> float:
    """G(P, T0/lambda) from reversible scaling (eq. Gibbs_RS)."""
    return (G0 / lam + 1.5 * n_atoms * KB * T0 * np.log(lam) / lam
            + (w_fwd - w_bwd) / (2.0 * lam))


def dcci_curve_const_ratio(T, T0, P0, du_dv):
    """Coexistence pressure from the scaled Clausius-Clapeyron equation
    (eq. RS_CCE) when the per-atom energy/volume ratio is constant: with
    lambda = T0/T, P_S(lambda) = P0 - (lambda - 1) du/dv and P = P_S/lambda."""
    lam = T0 / np.asarray(T, dtype=float)
    Ps = P0 - (lam - 1.0) * du_dv
    return Ps / lam
