"""CPU checks of the C-ABI library: it loads, exports every function that
include/swfe.h declares, and validates descriptors without a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2103_10449_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def swfe():
    from paper_2103_10449_amd import swfe as m
    if not os.path.exists(m.LIB_PATH):
        from paper_2103_10449_amd import build
        build.build()
    m.load_library()
    return m


def test_exports_match_header(swfe):
    hdr = open(os.path.join(ROOT, "include", "swfe.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char \*)\s*(swfe_\w+)\(", hdr, re.M))
    assert declared == set(swfe.EXPORTS)
    lib = swfe.load_library()
    for name in declared:
        assert hasattr(lib, name), name


def _bytes(swfe, specs, params):
    desc = swfe.system_descs(specs)
    sw = swfe.sw_params_struct(params)
    n = ctypes.c_size_t(0)
    rc = swfe.load_library().swfe_workspace_bytes(desc, len(specs), ctypes.byref(sw), ctypes.byref(n))
    return rc, n.value


def test_workspace_sizing(swfe, sw_params):
    specs = inputs.config4(n_rep=8, steps=10).systems
    rc, n = _bytes(swfe, specs, sw_params)
    assert rc == 0
    n_atoms = sum(s.n for s in specs)
    assert n > n_atoms * (32 * 4 + 11 * 8)


def test_box_too_small_rejected(swfe, sw_params):
    x, box = inputs.diamond((1, 1, 1), 5.431)
    s = inputs.SystemSpec(x=x, v=np.zeros_like(x), box=box, mode=inputs.MODE_FORCE)
    rc, _ = _bytes(swfe, [s], sw_params)
    assert rc == swfe.E_BOX_TOO_SMALL


def test_invalid_descriptors_rejected(swfe, sw_params):
    x, box = inputs.diamond((2, 2, 2), 5.431)
    base = dict(x=x, v=np.zeros_like(x), box=box)
    # dCCI partner must point back
    a = inputs.SystemSpec(mode=inputs.MODE_DCCI_P, partner=1, T0=400, **base)
    b = inputs.SystemSpec(mode=inputs.MODE_DCCI_P, partner=1, T0=400, **base)
    assert _bytes(swfe, [a, b], sw_params)[0] == swfe.E_INVALID_ARG
    # Frenkel-Ladd runs at fixed volume
    c = inputs.SystemSpec(mode=inputs.MODE_FL, p_damp=1.0, T0=400, **base)
    assert _bytes(swfe, [c], sw_params)[0] == swfe.E_INVALID_ARG
    # barostat needs a temperature
    d = inputs.SystemSpec(mode=inputs.MODE_NVT, p_damp=1.0, T0=0.0, **base)
    assert _bytes(swfe, [d], sw_params)[0] == swfe.E_INVALID_ARG
    # reversible scaling needs positive lambda
    e = inputs.SystemSpec(mode=inputs.MODE_RS, sched_start=1.0, sched_end=0.0, T0=400, **base)
    assert _bytes(swfe, [e], sw_params)[0] == swfe.E_INVALID_ARG
    # unknown mode and barostat kind
    f = inputs.SystemSpec(mode=9, **base)
    assert _bytes(swfe, [f], sw_params)[0] == swfe.E_INVALID_ARG
    g = inputs.SystemSpec(mode=inputs.MODE_NVT, T0=400, baro=2, **base)
    assert _bytes(swfe, [g], sw_params)[0] == swfe.E_INVALID_ARG
    # the UF reference switches at fixed volume, with positive parameters
    h = inputs.SystemSpec(mode=inputs.MODE_UF, T0=1000, p_damp=1.0, uf_p=25.0, uf_sigma=2.0, uf_T=1000.0,
                          uf_rcut=5.0, **base)
    assert _bytes(swfe, [h], sw_params)[0] == swfe.E_INVALID_ARG
    u = inputs.SystemSpec(mode=inputs.MODE_UF, T0=1000, uf_p=0.0, **base)
    assert _bytes(swfe, [u], sw_params)[0] == swfe.E_INVALID_ARG


def test_degenerate_sizes_rejected(swfe, sw_params):
    """No systems, a one-atom system, and systems that are not contiguous."""
    x, box = inputs.diamond((2, 2, 2), 5.431)
    sw = swfe.sw_params_struct(sw_params)
    n = ctypes.c_size_t(0)
    lib = swfe.load_library()
    one = inputs.SystemSpec(x=x, v=np.zeros_like(x), box=box, mode=inputs.MODE_FORCE)
    assert lib.swfe_workspace_bytes(swfe.system_descs([one]), 0, ctypes.byref(sw), ctypes.byref(n)) \
        == swfe.E_INVALID_ARG
    single = inputs.SystemSpec(x=x[:1], v=np.zeros_like(x[:1]), box=box, mode=inputs.MODE_FORCE)
    assert _bytes(swfe, [single], sw_params)[0] == swfe.E_INVALID_ARG
    desc = swfe.system_descs([one, one])
    desc[1].offset = 3
    assert lib.swfe_workspace_bytes(desc, 2, ctypes.byref(sw), ctypes.byref(n)) == swfe.E_INVALID_ARG


def test_calls_before_init_fail_cleanly(swfe):
    lib = swfe.load_library()
    ctx = ctypes.c_void_p()
    assert lib.swfe_create(ctypes.byref(ctx)) == 0
    assert lib.swfe_step_switched(ctx, 10, 1, None) == swfe.E_STATE
    assert b"not initialised" in lib.swfe_last_error(ctx)
    lib.swfe_destroy(ctx)


def test_header_structs_match_binding(tmp_path):
    """Sizes and field offsets of the C structs in include/swfe.h, compiled
    with the host compiler, equal those of the ctypes mirrors."""
    import ctypes
    import subprocess
    from paper_2103_10449_amd import swfe as m
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    structs = {"swfe_system_desc": m.SystemDesc, "swfe_system_state": m.SystemState,
               "swfe_buffers": m.Buffers, "swfe_sw_params": m.SwParams}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "swfe.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_static_forces_reject_oversized_input_before_any_gpu_work(swfe, sw_params):
    """swfe_forces_static checks its input against the static scratch before
    it touches the GPU: a 39304-atom system is refused with SWFE_E_NOMEM and
    a message (the device pointers are not dereferenced)."""
    xl, box = inputs.diamond((17, 17, 17), 5.431)
    s = inputs.SystemSpec(x=xl, v=np.zeros_like(xl), box=box, mode=inputs.MODE_FORCE)
    lib = swfe.load_library()
    dummy = ctypes.c_void_p(16)
    rc = lib.swfe_forces_static(swfe.system_descs([s]), 1, ctypes.byref(swfe.sw_params_struct(sw_params)),
                                dummy, dummy, None, None, swfe.PREC_FP64, None)
    assert rc == swfe.E_NOMEM
    assert b"static scratch" in lib.swfe_last_error(None)
    x, box = inputs.diamond((1, 1, 1), 5.431)
    s = inputs.SystemSpec(x=x, v=np.zeros_like(x), box=box, mode=inputs.MODE_FORCE)
    rc = lib.swfe_forces_static(swfe.system_descs([s]), 1, ctypes.byref(swfe.sw_params_struct(sw_params)),
                                dummy, dummy, None, None, swfe.PREC_FP64, None)
    assert rc == swfe.E_BOX_TOO_SMALL
