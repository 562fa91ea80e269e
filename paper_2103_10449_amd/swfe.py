"""ctypes binding of libswfe (include/swfe.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory (tensors whose data pointers are
passed through) and the current HIP stream.  The library must be built
(``paper_2103_10449_amd.build.build()``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswfe.so")

OK = 0
E_INVALID_ARG, E_BOX_TOO_SMALL, E_OVERFLOW, E_NONFINITE, E_DCCI_SINGULAR, E_HIP, E_STATE, E_NOMEM = \
    -1, -2, -3, -4, -5, -6, -7, -8
MODE_FORCE, MODE_NVE, MODE_NVT, MODE_FL, MODE_RS, MODE_AS_P, MODE_DCCI_T, MODE_DCCI_P, MODE_UF = range(9)
BARO_ISO, BARO_ANISO = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
PARAM_GRAD, STRAIN = 1, 2
OUT_STRIDE = 20
LOG_STRIDE = 8
PARAM_NAMES = ("A", "B", "p", "q", "a", "lambda_sw", "gamma", "sigma", "epsilon")


class SwfeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"swfe error {code}: {msg}")
        self.code = code


class SwParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("A", "B", "p", "q", "a", "lambda_sw", "gamma", "sigma", "epsilon", "cos0", "mass")]


class SystemDesc(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int64), ("offset", ctypes.c_int64),
                ("box", ctypes.c_double * 3), ("mode", ctypes.c_int32), ("partner", ctypes.c_int32),
                ("k_spring", ctypes.c_double), ("T0", ctypes.c_double), ("tau_damp", ctypes.c_double),
                ("p_damp", ctypes.c_double), ("pressure", ctypes.c_double), ("stream", ctypes.c_uint64),
                ("sched_start", ctypes.c_double), ("sched_end", ctypes.c_double),
                ("sched_steps", ctypes.c_int64), ("baro", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("uf_p", ctypes.c_double), ("uf_sigma", ctypes.c_double), ("uf_T", ctypes.c_double),
                ("uf_rcut", ctypes.c_double)]


class Buffers(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("v", ctypes.c_void_p), ("f", ctypes.c_void_p),
                ("x0", ctypes.c_void_p), ("e_atom", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


class SystemState(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("Ps", ctypes.c_double), ("W", ctypes.c_double),
                ("U_int", ctypes.c_double), ("U_ref", ctypes.c_double), ("K", ctypes.c_double),
                ("V", ctypes.c_double), ("virial", ctypes.c_double * 9), ("box", ctypes.c_double * 3),
                ("veps", ctypes.c_double), ("T_inst", ctypes.c_double), ("step", ctypes.c_int64),
                ("sched_k", ctypes.c_int64), ("err", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("n_rebuild", ctypes.c_int64), ("veps_axes", ctypes.c_double * 3)]


EXPORTS = ("swfe_create", "swfe_destroy", "swfe_last_error", "swfe_workspace_bytes", "swfe_init_system",
           "swfe_build_neighbors", "swfe_compute_forces", "swfe_set_schedule", "swfe_step_switched",
           "swfe_work_integral", "swfe_get_state", "swfe_set_log", "swfe_read_log", "swfe_set_block",
           "swfe_autotune", "swfe_sizes", "swfe_profile_steps", "swfe_neighbor_stats", "swfe_set_skin",
           "swfe_set_params", "swfe_checkpoint_bytes", "swfe_save_state", "swfe_load_state", "swfe_forces_static",
           "swfe_autotune_skin")
KERNEL_NAMES = ("integrate", "rebuild_count", "rebuild_scan", "rebuild_scatter", "rebuild_order",
                "rebuild_list", "pass1", "pass2", "finalize")

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Open libswfe.so and declare its signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libswfe.so not found at {path}: build it with "
                           "paper_2103_10449_amd.build.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, \
        ctypes.POINTER(ctypes.c_double)
    sig = {
        "swfe_create": ([ctypes.POINTER(vp)], ctypes.c_int),
        "swfe_destroy": ([vp], None),
        "swfe_last_error": ([vp], ctypes.c_char_p),
        "swfe_workspace_bytes": ([ctypes.POINTER(SystemDesc), i32, ctypes.POINTER(SwParams),
                                  ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "swfe_init_system": ([vp, ctypes.POINTER(SystemDesc), i32, ctypes.POINTER(SwParams),
                              ctypes.POINTER(Buffers), ctypes.c_uint64, ctypes.c_double, i32, vp], ctypes.c_int),
        "swfe_build_neighbors": ([vp, vp], ctypes.c_int),
        "swfe_compute_forces": ([vp, u32, dp, vp, vp, vp, vp], ctypes.c_int),
        "swfe_set_schedule": ([vp, ctypes.POINTER(SystemDesc), vp], ctypes.c_int),
        "swfe_step_switched": ([vp, i64, i32, vp], ctypes.c_int),
        "swfe_work_integral": ([vp, dp, dp, dp, ctypes.POINTER(i64), vp], ctypes.c_int),
        "swfe_get_state": ([vp, ctypes.POINTER(SystemState), vp], ctypes.c_int),
        "swfe_set_log": ([vp, i32, i32], ctypes.c_int),
        "swfe_read_log": ([vp, dp, i32, ctypes.POINTER(i32), vp], ctypes.c_int),
        "swfe_set_block": ([vp, i32, vp], ctypes.c_int),
        "swfe_autotune": ([vp, ctypes.POINTER(i32), vp], ctypes.c_int),
        "swfe_sizes": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i32)], ctypes.c_int),
        "swfe_profile_steps": ([vp, i64, dp, vp], ctypes.c_int),
        "swfe_checkpoint_bytes": ([vp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "swfe_save_state": ([vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "swfe_load_state": ([vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "swfe_neighbor_stats": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i64), vp],
                                ctypes.c_int),
        "swfe_set_skin": ([vp, ctypes.c_double, vp], ctypes.c_int),
        "swfe_set_params": ([vp, ctypes.POINTER(SwParams)], ctypes.c_int),
        "swfe_autotune_skin": ([vp, dp, i32, i32, dp, vp], ctypes.c_int),
        "swfe_forces_static": ([ctypes.POINTER(SystemDesc), i32, ctypes.POINTER(SwParams), vp, vp, vp, vp, i32, vp],
                               ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    if path == LIB_PATH:
        _lib = lib
    return lib


def sw_params_struct(params: dict, mass: float = 28.0855) -> SwParams:
    return SwParams(params["A"], params["B"], params["p"], params["q"], params["a"], params["lambda_sw"],
                    params["gamma"], params["sigma"], params["epsilon"], params.get("cos0", -1.0 / 3.0),
                    params.get("mass", mass))


def system_descs(systems: Sequence) -> "ctypes.Array":
    """Descriptor array from objects with the fields of inputs.SystemSpec."""
    arr = (SystemDesc * len(systems))()
    off = 0
    for i, s in enumerate(systems):
        d = arr[i]
        d.n_atoms = int(s.x.shape[0])
        d.offset = off
        for k in range(3):
            d.box[k] = float(s.box[k])
        d.mode = int(s.mode)
        d.partner = int(getattr(s, "partner", -1))
        d.k_spring = float(getattr(s, "k_spring", 0.0))
        d.T0 = float(getattr(s, "T0", 0.0))
        d.tau_damp = float(getattr(s, "tau_damp", 0.0))
        d.p_damp = float(getattr(s, "p_damp", 0.0))
        d.pressure = float(getattr(s, "pressure", 0.0))
        d.stream = int(getattr(s, "stream", i))
        d.sched_start = float(getattr(s, "sched_start", 1.0))
        d.sched_end = float(getattr(s, "sched_end", 1.0))
        d.sched_steps = int(getattr(s, "sched_steps", 0))
        d.baro = int(getattr(s, "baro", 0))
        d.reserved = 0
        d.uf_p = float(getattr(s, "uf_p", 0.0))
        d.uf_sigma = float(getattr(s, "uf_sigma", 0.0))
        d.uf_T = float(getattr(s, "uf_T", 0.0))
        d.uf_rcut = float(getattr(s, "uf_rcut", 0.0))
        off += d.n_atoms
    return arr


def _dp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Engine:
    """A set of systems resident on one GPU behind one library context.

    Arrays are packed structure-of-arrays, [3][n_total] FP64, in torch tensors
    on `device`; work goes to torch's current stream on that device."""

    def __init__(self, systems: Sequence, params: dict, dt: float = 0.001, seed: int = 0,
                 precision: str = "fp64", device: str = "cuda:0", block: int = 0,
                 want_e_atom: bool = False):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device)
        self.systems = list(systems)
        self.n_sys = len(self.systems)
        self.counts = [int(s.x.shape[0]) for s in self.systems]
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)]).astype(np.int64)
        self.n_total = int(self.offsets[-1])
        self.params = dict(params)
        self._desc = system_descs(self.systems)
        self._sw = sw_params_struct(self.params)
        prec = PREC_MIXED if precision == "mixed" else PREC_FP64

        def pack(get):
            out = np.zeros((3, self.n_total))
            for s, o, n in zip(self.systems, self.offsets[:-1], self.counts):
                a = get(s)
                if a is not None:
                    out[:, o:o + n] = np.asarray(a, dtype=np.float64).T
            return torch.from_numpy(out).to(self.device)

        self.x = pack(lambda s: s.x)
        self.v = pack(lambda s: s.v)
        self.f = torch.zeros((3, self.n_total), dtype=torch.float64, device=self.device)
        has_x0 = any(getattr(s, "x0", None) is not None for s in self.systems)
        self.x0 = pack(lambda s: getattr(s, "x0", None)) if has_x0 else None
        self.e_atom = torch.zeros(self.n_total, dtype=torch.float64, device=self.device) if want_e_atom else None
        nbytes = ctypes.c_size_t(0)
        self._check(self.lib.swfe_workspace_bytes(self._desc, self.n_sys, ctypes.byref(self._sw),
                                                  ctypes.byref(nbytes)), ctx=False)
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self._buf = Buffers(self.x.data_ptr(), self.v.data_ptr(), self.f.data_ptr(),
                            self.x0.data_ptr() if self.x0 is not None else None,
                            self.e_atom.data_ptr() if self.e_atom is not None else None,
                            self.workspace.data_ptr(), int(nbytes.value))
        self.ctx = ctypes.c_void_p()
        self._check(self.lib.swfe_create(ctypes.byref(self.ctx)), ctx=False)
        self._check(self.lib.swfe_init_system(self.ctx, self._desc, self.n_sys, ctypes.byref(self._sw),
                                              ctypes.byref(self._buf), int(seed), float(dt), prec,
                                              self._stream()))
        if block:
            self._check(self.lib.swfe_set_block(self.ctx, int(block), self._stream()))

    # ------------------------------------------------------------------ misc --
    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _check(self, rc: int, ctx: bool = True):
        if rc != OK:
            msg = self.lib.swfe_last_error(self.ctx).decode() if ctx else "invalid descriptors"
            raise SwfeError(rc, msg)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.swfe_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ the path --
    def build_neighbors(self):
        self._check(self.lib.swfe_build_neighbors(self.ctx, self._stream()))

    def compute_forces(self, param_grad: bool = False, strain: Optional[np.ndarray] = None,
                       grad_scale=None, grad_x=None, out=None):
        """Interaction at the current positions; returns the per-system output
        rows (n_sys, 20) as a device tensor: E, U_ref, dE/dstrain (9), dE/dtheta (9)."""
        torch = self.torch
        if out is None:
            out = torch.zeros((self.n_sys, OUT_STRIDE), dtype=torch.float64, device=self.device)
        flags = (PARAM_GRAD if param_grad else 0) | (STRAIN if strain is not None else 0)
        st = None
        if strain is not None:
            st = np.ascontiguousarray(np.asarray(strain, dtype=np.float64).reshape(self.n_sys, 9))
        self._check(self.lib.swfe_compute_forces(
            self.ctx, flags, _dp(st),
            ctypes.c_void_p(grad_scale.data_ptr()) if grad_scale is not None else None,
            ctypes.c_void_p(grad_x.data_ptr()) if grad_x is not None else None,
            ctypes.c_void_p(out.data_ptr()), self._stream()))
        return out

    def set_params(self, params: dict):
        """New Stillinger-Weber parameters (dict with the keys of PARAM_NAMES, cos0, mass)."""
        self.params = dict(params)
        self._sw = sw_params_struct(self.params)
        self._check(self.lib.swfe_set_params(self.ctx, ctypes.byref(self._sw)))

    def set_schedule(self, specs: Optional[Sequence] = None):
        desc = system_descs(specs) if specs is not None else None
        self._check(self.lib.swfe_set_schedule(self.ctx, desc, self._stream()))

    def step(self, n_steps: int, use_graph: bool = True, persistent: bool = False):
        """n_steps switched steps: eager launches, a replayed step graph, or
        (persistent=True) the persistent step kernel."""
        mode = 2 if persistent else int(bool(use_graph))
        self._check(self.lib.swfe_step_switched(self.ctx, int(n_steps), mode, self._stream()))

    def work_integral(self):
        W, lam, Ps = (np.zeros(self.n_sys) for _ in range(3))
        k = np.zeros(self.n_sys, dtype=np.int64)
        self._check(self.lib.swfe_work_integral(self.ctx, _dp(W), _dp(lam), _dp(Ps),
                                                k.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                                self._stream()))
        return dict(W=W, lam=lam, Ps=Ps, steps=k)

    def state(self) -> List[dict]:
        arr = (SystemState * self.n_sys)()
        self._check(self.lib.swfe_get_state(self.ctx, arr, self._stream()))
        out = []
        for s in arr:
            out.append(dict(lam=s.lam, Ps=s.Ps, W=s.W, U_int=s.U_int, U_ref=s.U_ref, K=s.K, V=s.V,
                            virial=np.array(s.virial[:]).reshape(3, 3), box=np.array(s.box[:]),
                            veps=s.veps, veps_axes=np.array(s.veps_axes[:]), T=s.T_inst, step=s.step,
                            sched_k=s.sched_k, err=s.err, n_rebuild=s.n_rebuild))
        return out

    def set_log(self, every: int, capacity: int = 4096):
        self._check(self.lib.swfe_set_log(self.ctx, int(every), int(capacity)))

    def read_log(self, max_rows: int = 16384) -> np.ndarray:
        rows = np.zeros((max_rows, LOG_STRIDE))
        n = ctypes.c_int32(0)
        self._check(self.lib.swfe_read_log(self.ctx, _dp(rows), max_rows, ctypes.byref(n), self._stream()))
        return rows[:n.value]

    def read_log_by_system(self, max_rows: int = 16384) -> List[np.ndarray]:
        """The log split per system: rows (step, lambda, P_S, P, T, U/N, V/N, W)."""
        rows = self.read_log(max_rows)
        return [rows[k::self.n_sys] for k in range(self.n_sys)]

    def set_block(self, block: int):
        self._check(self.lib.swfe_set_block(self.ctx, int(block), self._stream()))

    def autotune(self) -> int:
        b = ctypes.c_int32(0)
        self._check(self.lib.swfe_autotune(self.ctx, ctypes.byref(b), self._stream()))
        return int(b.value)

    def autotune_skin(self, candidates=None, steps: int = 40) -> float:
        """Pick the Verlet skin by timing graph steps at each candidate (the
        library's autotuner); returns the chosen skin in A."""
        c = None if candidates is None else np.ascontiguousarray(candidates, dtype=np.float64)
        out = ctypes.c_double(0.0)
        self._check(self.lib.swfe_autotune_skin(self.ctx, _dp(c), 0 if c is None else len(c), int(steps),
                                                ctypes.byref(out), self._stream()))
        return float(out.value)

    def profile_steps(self, n_steps: int) -> dict:
        """Per-kernel HIP-event durations (ms, summed over n_steps eager steps)."""
        ms = np.zeros(16)
        self._check(self.lib.swfe_profile_steps(self.ctx, int(n_steps), _dp(ms), self._stream()))
        return dict(zip(KERNEL_NAMES, ms[:len(KERNEL_NAMES)]))

    def neighbor_stats(self):
        """(ordered pairs within the cutoff, max per atom, Verlet-list entries)."""
        tot, mx, ll = ctypes.c_int64(0), ctypes.c_int32(0), ctypes.c_int64(0)
        self._check(self.lib.swfe_neighbor_stats(self.ctx, ctypes.byref(tot), ctypes.byref(mx),
                                                 ctypes.byref(ll), self._stream()))
        return int(tot.value), int(mx.value), int(ll.value)

    def save_state(self) -> np.ndarray:
        """Checkpoint of the whole run state as a host byte array (the library
        blob: settings, workspace, x, v, f)."""
        n = ctypes.c_size_t(0)
        self._check(self.lib.swfe_checkpoint_bytes(self.ctx, ctypes.byref(n)))
        blob = np.empty(n.value, dtype=np.uint8)
        self._check(self.lib.swfe_save_state(self.ctx, blob.ctypes.data_as(ctypes.c_void_p), n.value,
                                             self._stream()))
        return blob

    def load_state(self, blob: np.ndarray):
        """Resume from a checkpoint of a context with the same system sizes."""
        blob = np.ascontiguousarray(blob, dtype=np.uint8)
        self._check(self.lib.swfe_load_state(self.ctx, blob.ctypes.data_as(ctypes.c_void_p), blob.size,
                                             self._stream()))

    def set_skin(self, skin: float):
        self._check(self.lib.swfe_set_skin(self.ctx, float(skin), self._stream()))

    # --------------------------------------------------------------- views --
    def _unpack(self, t, s: int) -> np.ndarray:
        o, n = int(self.offsets[s]), self.counts[s]
        return t[:, o:o + n].detach().cpu().numpy().T.copy()

    def positions(self, s: int = 0) -> np.ndarray:
        return self._unpack(self.x, s)

    def velocities(self, s: int = 0) -> np.ndarray:
        return self._unpack(self.v, s)

    def forces(self, s: int = 0) -> np.ndarray:
        return self._unpack(self.f, s)

    def atom_energies(self, s: int = 0) -> np.ndarray:
        o, n = int(self.offsets[s]), self.counts[s]
        return self.e_atom[o:o + n].detach().cpu().numpy().copy()


def forces_static(systems: Sequence, params: dict, x, f, e_atom=None, out=None, precision: str = "fp64"):
    """swfe_forces_static: forces (and optionally per-atom energies and the
    per-system rows E, -, dE/dstrain) of force-only systems into the caller's
    device tensors x [3][n_total] (read), f [3][n_total], e_atom [n_total],
    out [n_sys][20], with the library's static scratch (no allocation in the
    call).  Synchronises torch's current stream."""
    import torch
    lib = load_library()
    desc = system_descs(systems)
    sw = sw_params_struct(params)
    stream = ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    rc = lib.swfe_forces_static(desc, len(systems), ctypes.byref(sw), ptr(x), ptr(f), ptr(e_atom), ptr(out),
                                PREC_MIXED if precision == "mixed" else PREC_FP64, stream)
    if rc != OK:
        raise SwfeError(rc, lib.swfe_last_error(None).decode())


# ---------------------------------------------------------------------------
# Host estimators (section 2): the same formulas the oracle uses, written
# here independently for library users.
# ---------------------------------------------------------------------------
from .estimators import delta_f, dissipated_heat  # noqa: E402,F401  (eqs. dF, Qdiss)
