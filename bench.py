"""Throughput of the batched switched-Hamiltonian step on one MI355X.

Workload (default): 64 independent switching replicas of seeded uneven sizes
(512-13824 atoms; diamond and beta-tin run Frenkel-Ladd lambda 1 -> 0 at
1000 K, liquids run reversible scaling lambda 1 -> 0.5 at P = 0), all in one
batch, one captured HIP-graph step replayed per MD step.  A "step" is one
pass of the whole hot path over every replica: kick/drift/Langevin, cell
binning, pair + three-body moments, force gather, reductions, lambda switch
and work.  The timed K steps are K/2 forward + K/2 backward switching steps.

Reported: atom-steps/s of the mixed path (FP32 terms, FP64 accumulation) as
`value`, the plain FP64 path for the speedup, the |Delta F| gate between the
two, the dominant kernel's roofline fraction (HIP events on the launch
stream), and the CPU oracle's rate on a bounded sample of the same batch.
"""
import argparse
import copy
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-steps/s per GPU, batched mixed vs plain FP64 at |ΔF|<1 meV/atom"

# Algorithmic flops of the moment form, each unique term counted once (add,
# sub and mul one flop, fused multiply-add two; exp, reciprocal, square root
# and reciprocal square root one each; rounding, compares and conversions
# none).  The operation count behind each constant is tabulated in the
# design notes (kernels and rooflines):
C_PAIR = 74     # per unordered pair: minimum-image distance, phi2 and its derivative,
                # force on both atoms, energy, virial, g(r) and g'(r) shared by both ends
C_MOM = 21      # per (centre, neighbour): the centre's moments s, q, v, M
C_D3 = 76       # per (centre, neighbour): dE3_centre/dr (55), force on both atoms (6),
                # three-body virial (15)
C_ATOM2 = 50    # per atom in pass 2: own three-body energy, Einstein spring, final kick,
                # kinetic energy
# Algorithmic HBM bytes of one integrate launch per atom: position and
# velocity read and written (4 x 24), force, stored normals and build position
# read (3 x 24), FP32 position written (12); Frenkel-Ladd atoms also read
# their anchor (24).
INTEGRATE_BYTES = 180
INTEGRATE_BYTES_FL = 24
# Bytes per atom-step of a step done in one pass over the atoms: position,
# velocity and force each read and written once (3 x 48) and the cell
# binning (12); Frenkel-Ladd atoms also read their anchor (24).
ONE_PASS_BYTES = 156
PEAK = {"mixed": 157.3e12, "fp64": 78.6e12}  # vector FLOP/s: FP32, FP64
PEAK_HBM = 8.0e12                             # B/s
SKINS = (0.7, 1.0, 1.4, 1.8, 2.0)  # Verlet skins the autotuner tries with --skin 0, A
REPEATS = 5                   # timed windows of K steps; the value is their median
PEAK_FP32_NONPACKED = 78.6e12 # FP32 vector roof without packed FP32 instructions (the library's build)
# Delta F gate: the switching protocol of the workload (1000 steps each way),
# whatever the timed window; ensembles of realisations (own noise streams) of
# one small replica per phase
DF_STEPS = 1000
DF_REALISATIONS = 32
DF_ENSEMBLE_REPLICAS = {"diamond": 10, "beta-sn": 44, "liquid": 53}

# HBM bytes per launch of the step kernels on this workload (64 replicas,
# skin 1.8 A), from rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per dispatch,
# averaged over the dispatches of a short run of both precisions; a rebuild
# stage's mean holds its steps with and without rebuilds), each
# scaled by what the counter reads for a plain 512 MiB device copy:
# FETCH_SIZE reads half the copied bytes (factor 2.000), WRITE_SIZE all of
# them (1.000).  The figures hold only for the block sizes, the kernel
# sources and the host code that places blocks on the XCDs they were taken
# on (digest).
MEASURED_TRAFFIC = {
    "sources_sha256": "572204af4744aabbd126feefc30a4a16a7ce9ea36dbd16bcf3cb9e57468cdc38",
    "skin": 1.8, "replicas": 64, "block": {"mixed": 128, "fp64": 256},
    "fetch_factor": 2.0, "write_factor": 1.0,
    "kib": {  # (FETCH_SIZE, WRITE_SIZE)
        ("mixed", "pass1"): (20990.7, 23250.6), ("mixed", "pass2"): (27899.3, 18730.2),
        ("fp64", "pass1"): (18936.9, 31871.0), ("fp64", "pass2"): (28289.3, 18293.2),
        ("mixed", "integrate"): (18130.4, 18222.6), ("fp64", "integrate"): (18120.3, 18181.2),
        ("mixed", "rebuild_count"): (189.7, 210.6), ("mixed", "rebuild_scatter"): (463.1, 839.0),
        ("mixed", "rebuild_order"): (435.7, 1028.4),
        # the scan runs inside the scatter stage on this workload: no launch
        ("mixed", "rebuild_scan"): (0.0, 0.0),
        # kernels of one workgroup size in both precisions: mean over both runs
        ("mixed", "rebuild_list"): (1083.1, 1238.3), ("mixed", "finalize"): (478.5, 32.0),
    },
}


def kernel_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("swfe_kernels.hip", "swfe_internal.h", "swfe_api.hip"):
        with open(os.path.join(ROOT, "paper_2103_10449_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(name, skin, replicas, precision, block):
    """HBM bytes per launch of kernel `name`, or None when the counters were
    not taken on this configuration and these kernel sources."""
    m = MEASURED_TRAFFIC
    key = (precision, name)
    if (key not in m["kib"] or skin != m["skin"] or replicas != m["replicas"]
            or block != m["block"][precision] or kernel_sources_digest() != m["sources_sha256"]):
        return None
    fetch, write = m["kib"][key]
    return 1024.0 * (fetch * m["fetch_factor"] + write * m["write_factor"])


def kernel_flops(name, n_atoms, ordered_pairs):
    """Algorithmic flops of one launch of a force pass: pass 1 holds the pair
    part and the moments, pass 2 the three-body gather."""
    if name == "pass1":
        return ordered_pairs / 2 * C_PAIR + ordered_pairs * C_MOM
    if name == "pass2":
        return ordered_pairs * C_D3 + n_atoms * C_ATOM2
    return None


STEP_KERNELS = ("integrate", "rebuild_count", "rebuild_scan", "rebuild_scatter", "rebuild_order",
                "rebuild_list", "pass1", "pass2", "finalize")


def step_algorithmic_bytes(n_atoms, n_fl, pairs, list_entries, rebuilt_atoms, n_tiles, mom_bytes):
    """Algorithmic HBM bytes of one dynamics step, per kernel: every per-atom
    operand read or written once, neighbour data gathered from cache not
    counted.  integrate as INTEGRATE_BYTES; pass 1: position (24), list count
    (4), 16-bit list entries, moments written, short-list entries (2 per
    pair) and count (4), pair force written (24); pass 2: position,
    moments, short list and count, caller index (4), force and velocity
    read and written (96), next normals written (24), Frenkel-Ladd anchors
    (24); the rebuild stages per rebuilt atom: position, velocity, force and
    anchor staged and placed (384) and 16-bit list entries (2 each, at the
    batch's mean list length); finalize: both passes' tile partials."""
    list_per_atom = list_entries / n_atoms
    return {
        "integrate": INTEGRATE_BYTES * n_atoms + INTEGRATE_BYTES_FL * n_fl,
        "rebuild": rebuilt_atoms * (384 + 2 * list_per_atom),
        "pass1": n_atoms * (24 + 4 + mom_bytes + 4 + 24) + 2 * list_entries + 2 * pairs,
        "pass2": n_atoms * (24 + mom_bytes + 4 + 4 + 96 + 24) + 24 * n_fl + 2 * pairs,
        "finalize": n_tiles * 2 * 26 * 8,
    }


def step_traffic(run, skin, replicas, precision, n_fl, mom_bytes):
    """Whole-step HBM bytes from the counters (sum over the step's kernels of
    the bytes per launch) against the algorithmic bytes of one step; None
    when the counters were not taken on this configuration and sources."""
    meas = {k: measured_traffic(k, skin, replicas, precision, run["block"]) for k in STEP_KERNELS}
    if any(v is None for v in meas.values()):
        return None
    alg = step_algorithmic_bytes(run["n_atoms"], n_fl, run["pairs"], run["list_entries"],
                                 run["rebuilt_atoms_per_step"], run["n_tiles"], mom_bytes)
    counter = sum(meas.values())
    total = sum(alg.values())
    one_pass = ONE_PASS_BYTES * run["n_atoms"] + INTEGRATE_BYTES_FL * n_fl
    return {"counter_bytes": counter, "algorithmic_bytes": total, "ratio": counter / total,
            "one_pass_bytes": one_pass, "ratio_one_pass": counter / one_pass,
            "counter_bytes_per_kernel": meas, "algorithmic_bytes_per_kernel": alg}


def run_precision(precision, wl_builder, steps, warmup, P, seed, profile_steps, skins=None, block=0):
    import torch
    from paper_2103_10449_amd import swfe

    half = steps // 2
    wl = wl_builder(half)
    specs = copy.deepcopy(wl.systems)
    n_atoms = sum(s.n for s in specs)
    eng = swfe.Engine(specs, P, dt=wl.dt, seed=seed, precision=precision)
    starts = [(s.sched_start, s.sched_end) for s in specs]
    # warm-up at the start of the path (lambda held); with no skin given the
    # library's autotuner picks it (rebuild frequency vs list length) by
    # timing.  The block size is tuned at the skin of the run: the rebuild
    # frequency changes which size is fastest.
    for s, (a, b) in zip(specs, starts):
        s.sched_start, s.sched_end, s.sched_steps = a, a, 0
    eng.set_schedule(specs)
    if skins and len(skins) == 1:
        skin = skins[0]
        eng.set_skin(skin)
    else:
        skin = eng.autotune_skin(skins or SKINS, steps=40)
    if block:
        eng.set_block(block)
    else:
        block = eng.autotune()
    print(f"# {precision}: engine ready, skin {skin} A, block {block}", file=sys.stderr, flush=True)
    eng.step(warmup, use_graph=True)
    torch.cuda.synchronize()
    eng.state()  # raises on a device error (non-finite, overflow, box)
    print(f"# {precision}: {warmup} warm-up steps done", file=sys.stderr, flush=True)
    rb0 = [x["n_rebuild"] for x in eng.state()]
    walls, gpus = [], []
    for rep in range(REPEATS):
        t_total = 0.0
        ev_total = 0.0
        for direction in ("fwd", "bwd"):
            for s, (a, b) in zip(specs, starts):
                s.sched_start, s.sched_end, s.sched_steps = (a, b, half) if direction == "fwd" else (b, a, half)
            eng.set_schedule(specs)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record()
            eng.step(half, use_graph=True)
            e1.record()
            torch.cuda.synchronize()
            t_total += time.perf_counter() - t0
            ev_total += e0.elapsed_time(e1) / 1e3
        walls.append(t_total)
        gpus.append(ev_total)
        print(f"# {precision}: window {rep}: {2 * half} steps in {t_total:.4f} s", file=sys.stderr, flush=True)
    rb1 = [x["n_rebuild"] for x in eng.state()]
    n_rebuild = sum(rb1) - sum(rb0)
    rebuilt_atoms = sum((b - a) * sp.n for a, b, sp in zip(rb0, rb1, specs))
    eng.state()  # raises on a device error (non-finite, overflow, box)
    pairs, max_nb, list_entries = eng.neighbor_stats()
    prof = eng.profile_steps(profile_steps) if profile_steps else None
    eng.close()
    return dict(n_atoms=n_atoms, wall=float(np.median(walls)), walls=walls, gpu=float(np.median(gpus)),
                steps=2 * half, block=block, skin=skin, pairs=pairs, max_nb=max_nb, list_entries=list_entries,
                rebuilds_per_step=n_rebuild / (REPEATS * 2 * half),
                rebuilt_atoms_per_step=rebuilt_atoms / (REPEATS * 2 * half), prof=prof, n_rep=len(specs),
                n_tiles=sum(-(-sp.n // block) for sp in specs))


def _switch_both_ways(eng, specs, n_steps):
    """Forward then backward switching from the current state; returns the
    per-system Delta F = (W_fwd - W_bwd)/2 in eV (eq. dF)."""
    fwd = copy.deepcopy(specs)
    for s in fwd:
        s.sched_steps = n_steps
    eng.set_schedule(fwd)
    eng.step(n_steps, use_graph=True)
    wf = eng.work_integral()["W"].copy()
    for s in fwd:
        s.sched_start, s.sched_end = s.sched_end, s.sched_start
    eng.set_schedule(fwd)
    eng.step(n_steps, use_graph=True)
    wb = eng.work_integral()["W"].copy()
    return 0.5 * (wf - wb)


def _mean_se(d):
    d = np.asarray(d, float)
    return float(d.mean()), float(d.std(ddof=1) / np.sqrt(len(d))) if len(d) > 1 else float("nan")


def delta_f_gate(base, P, seed, blocks, skin):
    """|Delta F_mixed - Delta F_FP64| at the workload's own switching protocol
    (1000 steps each way, eqs. dF and Qdiss), whatever the timed window.

    Per replica of the batch: the two precisions run with the same noise, but
    their trajectories decorrelate over 2 ps, so a single replica's difference
    carries its Delta F's statistical spread (a few meV/atom); the figures are
    reported (n, mean, standard error, largest).  The gate itself follows the
    ensemble reading: for one small replica of each phase, DF_REALISATIONS
    realisations with their own noise streams, mixed and FP64; the mean
    difference over the realisations and twice its standard error must both
    stay below 1 meV/atom for every phase."""
    import torch
    from paper_2103_10449_amd import swfe
    res = {}
    counts = np.array([s.n for s in base.systems], float)
    for prec in ("mixed", "fp64"):
        eng = swfe.Engine(copy.deepcopy(base.systems), P, dt=base.dt, seed=seed, precision=prec, block=blocks[prec])
        eng.set_skin(skin)
        res[prec] = _switch_both_ways(eng, base.systems, DF_STEPS) / counts
        eng.close()
    d = 1e3 * (res["mixed"] - res["fp64"])            # meV/atom
    mean, se = _mean_se(d)
    phases = [s.phase for s in base.systems]
    out = {"protocol_steps_each_way": DF_STEPS,
           "per_replica": {"n": len(d), "mean_meV_per_atom": mean, "se_meV_per_atom": se,
                           "max_abs_meV_per_atom": float(np.abs(d).max()),
                           "by_phase": {ph: dict(zip(("mean_meV_per_atom", "se_meV_per_atom"),
                                                     _mean_se(d[[p == ph for p in phases]])))
                                        for ph in sorted(set(phases))}}}
    ens_specs, labels = [], []
    for ph, k in DF_ENSEMBLE_REPLICAS.items():
        for r in range(DF_REALISATIONS):
            s = copy.deepcopy(base.systems[k])
            s.stream = 5000 + len(ens_specs)
            ens_specs.append(s)
            labels.append(ph)
    counts = np.array([s.n for s in ens_specs], float)
    ens = {}
    for prec in ("mixed", "fp64"):
        eng = swfe.Engine(copy.deepcopy(ens_specs), P, dt=base.dt, seed=seed + 1, precision=prec,
                          block=blocks[prec])
        eng.set_skin(skin)
        ens[prec] = _switch_both_ways(eng, ens_specs, DF_STEPS) / counts
        eng.close()
    torch.cuda.synchronize()
    de = 1e3 * (ens["mixed"] - ens["fp64"])
    gate = {}
    ok = True
    for ph, k in DF_ENSEMBLE_REPLICAS.items():
        sel = [l == ph for l in labels]
        m, e = _mean_se(de[sel])
        gate[ph] = {"replica": k, "atoms": int(base.systems[k].n), "realisations": int(sum(sel)),
                    "mean_meV_per_atom": m, "se_meV_per_atom": e,
                    "dF_fp64_meV_per_atom": float(1e3 * ens["fp64"][sel].mean())}
        ok = ok and abs(m) < 1.0 and 2.0 * e < 1.0
    out["ensembles"] = gate
    out["pass"] = bool(ok)
    return out


def per_config_rates(P, seed, steps=200):
    """Atom-steps/s of the smaller single-workload configurations (mixed and
    FP64), each alone on the GPU: the 64-atom Frenkel-Ladd crystal, the
    8000-atom diamond and liquid reversible-scaling runs (and their force
    evaluations per second), the dCCI pair of
    4096-atom diamond and 8000-atom beta-tin; and force evaluations per
    second (with the forced list build) of the 32768-atom crystal.  Small
    systems are bound by the launch sequence, not by the atoms."""
    import torch
    from paper_2103_10449_amd import inputs, swfe
    out = {}
    cases = [("c1_diamond64_fl", lambda: inputs.config1()),
             ("c2_diamond8000_rs", lambda: inputs.config2("diamond", steps=steps)),
             ("c2_liquid8000_rs", lambda: inputs.config2("liquid", steps=steps)),
             ("c3_dcci_diamond4096_betasn8000", lambda: inputs.config3(steps=steps))]
    for name, mk in cases:
        wl = mk()
        row = {"atoms": wl.n_atoms}
        for prec in ("mixed", "fp64"):
            eng = swfe.Engine(copy.deepcopy(wl.systems), P, dt=wl.dt, seed=seed, precision=prec)
            eng.set_skin(1.0)
            eng.step(20, use_graph=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            eng.step(steps, use_graph=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            eng.state()
            row[prec] = wl.n_atoms * steps / dt
            if name.startswith("c2"):
                # force-only throughput (with the forced list build) of the same system
                eng.compute_forces()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(20):
                    eng.compute_forces()
                torch.cuda.synchronize()
                row[prec + "_forces_atoms_per_s"] = wl.n_atoms * 20 / (time.perf_counter() - t0)
            eng.close()
        out[name] = row
        print(f"# per-config {name}: {row}", file=sys.stderr, flush=True)
    wl = inputs.config5()
    row = {"atoms": wl.n_atoms, "unit": "atom force evaluations/s (forced list build)"}
    for prec in ("mixed", "fp64"):
        eng = swfe.Engine(copy.deepcopy(wl.systems), P, dt=wl.dt, seed=seed, precision=prec)
        for grad in (False, True):
            eng.compute_forces(param_grad=grad)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(20):
                eng.compute_forces(param_grad=grad)
            torch.cuda.synchronize()
            row[prec + ("_param_grad" if grad else "")] = wl.n_atoms * 20 / (time.perf_counter() - t0)
        eng.close()
    out["c5_diamond32768_forces"] = row
    print(f"# per-config c5: {row}", file=sys.stderr, flush=True)
    return out


def _oracle_systems(specs):
    from oracle import oracle as orc
    return [orc.OSystem(x=s.x, v=s.v, box=s.box, mode=s.mode, x0=s.x0, partner=s.partner,
                        k_spring=s.k_spring, T0=s.T0, tau_damp=s.tau_damp, p_damp=s.p_damp,
                        pressure=s.pressure, stream=s.stream, sched_start=s.sched_start,
                        sched_end=s.sched_end, sched_steps=s.sched_steps, baro=s.baro, uf_p=s.uf_p, uf_sigma=s.uf_sigma,
                        uf_T=s.uf_T, uf_rcut=s.uf_rcut) for s in specs]


def _oracle_steps(job):
    """Worker: the FP64 oracle on a share of the (independent) replicas for a
    fixed number of steps; returns (atom-steps, seconds)."""
    specs, P, dt, seed, n_steps = job
    from oracle import oracle as orc
    o = orc.Oracle(_oracle_systems(specs), P, dt=dt, seed=seed)
    t0 = time.perf_counter()
    for _ in range(n_steps):
        o.step()
    return sum(s.n for s in specs) * n_steps, time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


CPU_WINDOW_STEPS = 3   # steps every process takes in the all-core baseline


def cpu_baseline(wl, P, seed, budget_s=12.0):
    """The FP64 oracle on the same batch.  Single thread: every replica, as
    many whole steps as fit in about budget_s (at least one).  All cores: the
    replicas (independent systems) dealt to one process per core, each
    stepping its share CPU_WINDOW_STEPS steps (a bounded window of the
    workload's 2000; the oracle is not tuned for this)."""
    import multiprocessing as mp
    specs = copy.deepcopy(wl.systems)
    n = sum(s.n for s in specs)
    o_specs = _oracle_systems(specs)
    from oracle import oracle as orc
    o = orc.Oracle(o_specs, P, dt=wl.dt, seed=seed)
    t0 = time.perf_counter()
    k = 0
    while True:
        o.step()
        k += 1
        if time.perf_counter() - t0 > budget_s or k >= 10:
            break
    dt1 = time.perf_counter() - t0
    single = n * k / dt1
    cores = max(1, min(16, os.cpu_count() or 1, len(specs)))
    # deal replicas largest first to the least loaded share
    shares = [[] for _ in range(cores)]
    load = [0] * cores
    for s in sorted(specs, key=lambda s: -s.n):
        q = load.index(min(load))
        shares[q].append(s)
        load[q] += s.n
    jobs = [(sh, P, wl.dt, seed, CPU_WINDOW_STEPS) for sh in shares if sh]
    with mp.get_context("spawn").Pool(len(jobs)) as pool:
        res = pool.map(_oracle_steps, jobs)
    dtn = max(r[1] for r in res)  # the slowest share's stepping time
    model = cpu_model()
    return dict(value=n * CPU_WINDOW_STEPS / dtn, unit="atom-steps/s", cores=len(jobs), kind="oracle",
                single_thread_value=single, cpu_model=model, nproc=os.cpu_count(),
                window_steps=CPU_WINDOW_STEPS,
                sample=f"all {len(specs)} replicas ({n} atoms) of the batched workload, {CPU_WINDOW_STEPS} steps "
                       f"after set-up, on {len(jobs)} processes (replicas dealt by size; slowest share "
                       f"{dtn:.1f} s) of {model}; single thread: {k} step(s) in {dt1:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-df-gate", action="store_true",
                    help="skip the Delta F gate at the full switching protocol (1000 steps each way)")
    ap.add_argument("--no-per-config", action="store_true",
                    help="skip the per-configuration rates of the smaller workloads")
    ap.add_argument("--replicas", type=int, default=64)
    ap.add_argument("--block", type=int, default=0, choices=(0, 64, 128, 256),
                    help="block size of the mixed-precision run (0: swfe_autotune)")
    ap.add_argument("--block-fp64", type=int, default=0, choices=(0, 64, 128, 256),
                    help="block size of the FP64 run (0: swfe_autotune)")
    ap.add_argument("--skin", type=float, default=1.8,
                    help="Verlet skin in A (default 1.8: 1.4, 1.6, 1.8 and 2.0 A give 134.8, 130.4, 128.6 and "
                         "127.8 us per step on this workload, 2.0 A being the largest the lists are sized for; "
                         "0: the library autotuner chooses among 0.7, 1.0, 1.4, 1.8, 2.0 A)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="only run a plain device copy of this many MB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the batched replicas of this workload do not "
              f"communicate and are not split across GPUs (asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)
    from paper_2103_10449_amd import inputs
    if args.calib_copy_mb:
        import torch
        n = args.calib_copy_mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": 8 * n, "bytes_written": 8 * n, "launches": 5}))
        return
    P = dict(inputs.SW_SILICON)
    seed = inputs.SEED0
    steps = max(2, args.steps - args.steps % 2)
    base = inputs.config4(n_rep=args.replicas, steps=steps // 2)
    base_df = inputs.config4(n_rep=args.replicas, steps=DF_STEPS)
    print(f"# workload: {base.n_atoms} atoms in {len(base.systems)} replicas", file=sys.stderr, flush=True)
    builder = lambda half: base
    # the oracle runs first, before this process touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        print("# oracle baseline on the host cores ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(base, P, seed)
        print(f"# oracle: {cpu['value']:.3g} atom-steps/s on {cpu['cores']} cores", file=sys.stderr, flush=True)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    skins = (args.skin,) if args.skin > 0 else None
    mixed = run_precision("mixed", builder, steps, args.warmup, P, seed, args.profile_steps, skins, args.block)
    print(f"# mixed: {mixed['n_atoms']} atoms, {mixed['steps']} steps in {mixed['wall']:.3f} s "
          f"(block {mixed['block']}, {mixed['pairs'] / mixed['n_atoms']:.2f} neighbours/atom)", file=sys.stderr, flush=True)
    fp64 = None
    if not args.no_fp64:
        fp64 = run_precision("fp64", builder, steps, args.warmup, P, seed, args.profile_steps, skins, args.block_fp64)
        print(f"# fp64: {fp64['steps']} steps in {fp64['wall']:.3f} s", file=sys.stderr, flush=True)

    value = mixed["n_atoms"] * mixed["steps"] / mixed["wall"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": mixed["steps"],
        "warmup": args.warmup,
        "ms_per_step": 1e3 * mixed["wall"] / mixed["steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.replicas} switching replicas, 512-13824 atoms each "
                               "(diamond/beta-tin Frenkel-Ladd, liquid reversible scaling), one batch, "
                               "HIP-graph step",
                   "replicas": mixed["n_rep"], "atoms": mixed["n_atoms"], "precision": "mixed",
                   "dt_ps": 0.001, "forward_steps": steps // 2, "backward_steps": steps // 2,
                   "block": mixed["block"], "skin_A": mixed["skin"],
                   "list_rebuilds_per_step": mixed["rebuilds_per_step"],
                   "rebuilt_atoms_per_step": mixed["rebuilt_atoms_per_step"],
                   "ordered_pairs_within_rc": mixed["pairs"], "verlet_list_entries": mixed["list_entries"]},
        "timing": {"value_from": f"median of {REPEATS} timed windows of {mixed['steps']} steps",
                   "windows_s": mixed["walls"], "median_window_gpu_events_s": mixed["gpu"]},
    }
    if fp64 is not None:
        v64 = fp64["n_atoms"] * fp64["steps"] / fp64["wall"]
        out["fp64_value"] = v64
        out["speedup_vs_fp64"] = value / v64
        if not args.no_df_gate:
            print("# Delta F gate at the full switching protocol ...", file=sys.stderr, flush=True)
            out["dF_gate"] = delta_f_gate(base_df, P, seed, {"mixed": mixed["block"], "fp64": fp64["block"]},
                                          mixed["skin"])
            print(f"# Delta F gate: {json.dumps(out['dF_gate'])}", file=sys.stderr, flush=True)
    prof = mixed["prof"]
    if prof:
        # the longer force pass (the kernels with a flop model); the longest
        # kernel of the step is reported beside it
        name = max(("pass1", "pass2"), key=prof.get)
        n_prof = args.profile_steps
        avg = prof[name] / n_prof / 1e3              # s per launch
        fl = kernel_flops(name, mixed["n_atoms"], mixed["pairs"])
        ach = fl / avg / 1e12 if fl else None
        traffic = measured_traffic(name, mixed["skin"], args.replicas, "mixed", mixed["block"])
        out["roofline"] = {"bound": "alu", "kernel": name, "achieved": ach, "peak": PEAK["mixed"] / 1e12,
                           "unit": "TFLOP/s", "frac": (ach / (PEAK["mixed"] / 1e12)) if ach else None,
                           "peak_nonpacked": PEAK_FP32_NONPACKED / 1e12,
                           "frac_nonpacked": (ach / (PEAK_FP32_NONPACKED / 1e12)) if ach else None,
                           "traffic": traffic, "avg_launch_us": 1e6 * avg,
                           "hbm_GBps": traffic / avg / 1e9 if traffic else None,
                           "hbm_frac": traffic / avg / PEAK_HBM if traffic else None,
                           "per_kernel_us": {k: 1e3 * v / n_prof for k, v in prof.items()},
                           "longest_kernel": max(prof, key=prof.get)}
        # the other force pass against the same roofs
        other = "pass2" if name == "pass1" else "pass1"
        avg_o = prof[other] / n_prof / 1e3
        fl_o = kernel_flops(other, mixed["n_atoms"], mixed["pairs"])
        tr_o = measured_traffic(other, mixed["skin"], args.replicas, "mixed", mixed["block"])
        out["roofline_" + other] = {"bound": "alu", "kernel": other, "achieved": fl_o / avg_o / 1e12,
                                    "peak": PEAK["mixed"] / 1e12, "unit": "TFLOP/s",
                                    "frac": fl_o / avg_o / PEAK["mixed"],
                                    "frac_nonpacked": fl_o / avg_o / PEAK_FP32_NONPACKED,
                                    "traffic": tr_o, "avg_launch_us": 1e6 * avg_o,
                                    "hbm_frac": tr_o / avg_o / PEAK_HBM if tr_o else None}
        if fp64 is not None and fp64["prof"]:
            p64 = fp64["prof"]
            avg64 = p64[name] / n_prof / 1e3
            fl64 = kernel_flops(name, fp64["n_atoms"], fp64["pairs"])
            tr64 = measured_traffic(name, fp64["skin"], args.replicas, "fp64", fp64["block"])
            out["roofline_fp64"] = {"kernel": name, "achieved": fl64 / avg64 / 1e12, "peak": PEAK["fp64"] / 1e12,
                                    "frac": fl64 / avg64 / PEAK["fp64"], "traffic": tr64,
                                    "avg_launch_us": 1e6 * avg64,
                                    "hbm_GBps": tr64 / avg64 / 1e9 if tr64 else None,
                                    "hbm_frac": tr64 / avg64 / PEAK_HBM if tr64 else None,
                                    "per_kernel_us": {k: 1e3 * v / n_prof for k, v in p64.items()}}
        if "integrate" in prof:
            # the step's streaming kernel, against the HBM roof
            avg_i = prof["integrate"] / n_prof / 1e3
            n_fl = sum(s.n for s in base.systems if s.mode == inputs.MODE_FL)
            alg = INTEGRATE_BYTES * mixed["n_atoms"] + INTEGRATE_BYTES_FL * n_fl
            tr_i = measured_traffic("integrate", mixed["skin"], args.replicas, "mixed", mixed["block"])
            out["roofline_integrate"] = {"bound": "hbm", "kernel": "integrate", "achieved": alg / avg_i / 1e9,
                                         "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": alg / avg_i / PEAK_HBM,
                                         "algorithmic_bytes": alg, "traffic": tr_i, "avg_launch_us": 1e6 * avg_i}
        n_fl = sum(s.n for s in base.systems if s.mode == inputs.MODE_FL)
        out["step_traffic"] = step_traffic(mixed, mixed["skin"], args.replicas, "mixed", n_fl, 36)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if not args.no_per_config:
        out["per_config"] = per_config_rates(P, seed)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
