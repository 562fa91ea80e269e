"""The persistent step kernel (systems dealt to the XCDs, one cooperative
launch for many steps) against the captured step graph: the same per-tile
arithmetic and the same fixed-order reductions, so positions, velocities,
boxes, lambda, P_S and work must agree bitwise, for every mode and with list
rebuilds in every step (skin 0) or now and then."""
import copy

import numpy as np
import pytest

from paper_2103_10449_amd import inputs
from tests.gpu_helpers import betasn_spec, diamond_spec, liquid_spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swfe():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_10449_amd import swfe as m
    m.load_library()
    return m


def _mixed_batch():
    """Every mode in one batch: Frenkel-Ladd, reversible scaling with the
    isotropic barostat, pressure switching, a dCCI pair under pressure
    control with one piston per axis on the beta-tin phase, switching to the
    Uhlenbeck-Ford fluid, NVE and NVT."""
    dcci = dict(T0=400.0, tau_damp=0.1, p_damp=0.2, pressure=0.0, sched_start=0.0, sched_end=2.0,
                sched_steps=150, mode=inputs.MODE_DCCI_P)
    a = diamond_spec(3, 140, mode=inputs.MODE_FL, k_spring=5.0, T0=1000.0, tau_damp=0.1, stream=0,
                     sched_start=1.0, sched_end=0.0, sched_steps=150)
    b = liquid_spec(400, 141, mode=inputs.MODE_RS, T0=2000.0, tau_damp=0.1, p_damp=0.2, pressure=1.0, stream=1,
                    sched_start=1.0, sched_end=0.6, sched_steps=150)
    c = liquid_spec(300, 142, mode=inputs.MODE_AS_P, T0=2200.0, tau_damp=0.1, p_damp=0.2, stream=2,
                    sched_start=0.0, sched_end=3.0, sched_steps=150)
    d = diamond_spec(4, 143, T=400.0, partner=4, stream=3, **dcci)
    e = betasn_spec(4, 144, T=400.0, partner=3, stream=4, baro=inputs.BARO_ANISO, **dcci)
    f = liquid_spec(500, 145, mode=inputs.MODE_UF, T0=1700.0, tau_damp=0.1, stream=5, sched_start=1.0,
                    sched_end=0.5, sched_steps=150, uf_p=25.0, uf_sigma=2.0, uf_T=1700.0, uf_rcut=8.0)
    g = diamond_spec(2, 146, mode=inputs.MODE_NVE, stream=6)
    h = liquid_spec(250, 147, mode=inputs.MODE_NVT, T0=1700.0, tau_damp=0.1, stream=7)
    for s in (b, c, d, e, f, h):
        s.x0 = None
    return [a, b, c, d, e, f, g, h]


def _run(swfe, specs, P, prec, steps, persistent, skin, chunks=1, block=0):
    eng = swfe.Engine(copy.deepcopy(specs), P, seed=21, precision=prec, block=block)
    eng.set_skin(skin)
    for _ in range(chunks):
        eng.step(steps // chunks, use_graph=True, persistent=persistent)
    w = eng.work_integral()
    st = eng.state()
    out = dict(x=eng.x.cpu().numpy().copy(), v=eng.v.cpu().numpy().copy(), W=w["W"], lam=w["lam"], Ps=w["Ps"],
               box=np.array([s["box"] for s in st]), rebuilds=sum(s["n_rebuild"] for s in st))
    eng.close()
    return out


def _same(a, b):
    for k in ("x", "v", "W", "lam", "Ps", "box"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("prec,skin,block", [("fp64", 0.0, 256), ("fp64", 1.0, 256), ("mixed", 0.0, 128),
                                             ("fp64", 1.0, 64)])
def test_persistent_equals_graph_every_mode(swfe, sw_params, prec, skin, block):
    specs = _mixed_batch()
    print(f"persistent vs graph: {len(specs)} systems, {prec}, skin {skin}, block {block}", flush=True)
    g = _run(swfe, specs, sw_params, prec, 150, False, skin, block=block)
    p = _run(swfe, specs, sw_params, prec, 150, True, skin, chunks=3, block=block)
    print(f"rebuilds graph {g['rebuilds']} persistent {p['rebuilds']}", flush=True)
    assert p["rebuilds"] == g["rebuilds"]
    _same(g, p)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_persistent_equals_graph_single_small_system(swfe, sw_params, prec):
    wl = inputs.config1()
    print(f"persistent vs graph: 64-atom crystal, {prec}", flush=True)
    g = _run(swfe, wl.systems, sw_params, prec, 200, False, 0.5)
    p = _run(swfe, wl.systems, sw_params, prec, 200, True, 0.5)
    _same(g, p)


@pytest.mark.parametrize("prec,block", [("fp64", 256), ("mixed", 128)])
def test_persistent_equals_graph_batched_replicas(swfe, sw_params, prec, block):
    wl = inputs.config4(steps=1000)
    print(f"persistent vs graph: 64 replicas, {prec}, block {block}", flush=True)
    g = _run(swfe, wl.systems, sw_params, prec, 30, False, 1.4, block=block)
    p = _run(swfe, wl.systems, sw_params, prec, 30, True, 1.4, block=block)
    assert g["rebuilds"] == p["rebuilds"]
    _same(g, p)
