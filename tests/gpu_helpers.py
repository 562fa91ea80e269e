"""Shared helpers of the GPU parity tests (run the HIP path and the oracle on
the same seeded inputs)."""
import numpy as np

from oracle import oracle as orc
from paper_2103_10449_amd import inputs


def to_oracle(spec):
    return orc.OSystem(x=spec.x, v=spec.v, box=spec.box, mode=spec.mode, x0=spec.x0,
                       partner=spec.partner, k_spring=spec.k_spring, T0=spec.T0,
                       tau_damp=spec.tau_damp, p_damp=spec.p_damp, pressure=spec.pressure,
                       stream=spec.stream, sched_start=spec.sched_start, sched_end=spec.sched_end,
                       sched_steps=spec.sched_steps, baro=getattr(spec, "baro", 0), uf_p=spec.uf_p,
                       uf_sigma=spec.uf_sigma, uf_T=spec.uf_T, uf_rcut=spec.uf_rcut)


def force_err(f, fref):
    """max_i |F - F_ref|_inf / max(|F_ref|_inf, 1 eV/A)."""
    return float(np.abs(f - fref).max() / max(np.abs(fref).max(), 1.0))


def spec(x, box, **kw):
    n = len(x)
    d = dict(v=np.zeros((n, 3)), mode=inputs.MODE_FORCE)
    d.update(kw)
    return inputs.SystemSpec(x=np.asarray(x, float), box=np.asarray(box, float), **d)


def liquid_spec(n, seed, T=1700.0, **kw):
    x, box = inputs.liquid_rsa(n, inputs.rng(700, seed, 0))
    v = inputs.maxwell(n, T, inputs.rng(700, seed, 1))
    return inputs.SystemSpec(x=x, v=v, box=box, phase="liquid", **kw)


def diamond_spec(m, seed, T=1000.0, sigma=0.05, **kw):
    xl, box = inputs.diamond((m, m, m), 5.431)
    x = inputs.perturb(xl, sigma, inputs.rng(701, seed, 0))
    v = inputs.maxwell(len(x), T, inputs.rng(701, seed, 1))
    return inputs.SystemSpec(x=x, v=v, box=box, phase="diamond", x0=xl, **kw)


def betasn_spec(m, seed, T=400.0, sigma=0.05, **kw):
    xl, box = inputs.beta_sn((m, m, 2 * m), 4.80, 2.65)
    x = inputs.perturb(xl, sigma, inputs.rng(702, seed, 0))
    v = inputs.maxwell(len(x), T, inputs.rng(702, seed, 1))
    return inputs.SystemSpec(x=x, v=v, box=box, phase="beta-sn", x0=xl, **kw)
