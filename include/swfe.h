/*
 * swfe.h -- C-ABI of libswfe, the MI355X (gfx950) library for switched-
 * Hamiltonian molecular dynamics of silicon described by the Stillinger-Weber
 * potential.
 *
 * The library implements the per-step hot path of non-equilibrium free-energy
 * runs and dynamic Clausius-Clapeyron integration (dCCI):
 *   - cell-list neighbour build,
 *   - Stillinger-Weber energy, force, virial and parameter gradient,
 *   - velocity Verlet with a Langevin thermostat and an isotropic or
 *     per-axis barostat,
 *   - the lambda-switched Hamiltonian and its dH/dlambda work integral for
 *     Frenkel-Ladd (Einstein reference), Uhlenbeck-Ford (liquid reference),
 *     reversible-scaling, pressure-switching and coupled-phase dCCI runs.
 * Passages of the paper are cited as section / equation labels of
 * "Non-equilibrium free-energy calculation of phase-boundaries using LAMMPS"
 * (Cajahuaringa and Antonelli).
 *
 * Conventions shared by every call
 *   - Every function returns int: SWFE_OK (0) or a negative SWFE_E_* code;
 *     swfe_last_error() gives a message.  Errors are per context.
 *   - The caller owns all device memory (positions, velocities, forces,
 *     anchors, workspace) and passes raw device pointers.  The library owns
 *     only the opaque context and its host-side tables.
 *   - Work is enqueued on the caller's HIP stream (passed as void*; NULL is the
 *     default stream).  Only calls that return host data synchronise.
 *   - Units: eV, Angstrom, ps, amu, K; pressures at the ABI in GPa.
 *   - Atom arrays are structure-of-arrays over all systems concatenated:
 *     component c (0,1,2 = x,y,z) of global atom i is at [c * n_total + i];
 *     system s owns atoms [offset_s, offset_s + n_s).
 */
#ifndef SWFE_H
#define SWFE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct swfe_ctx swfe_ctx;

/* ---- status codes ------------------------------------------------------ */
#define SWFE_OK 0
#define SWFE_E_INVALID_ARG -1   /* bad pointer, size, mode or parameter */
#define SWFE_E_BOX_TOO_SMALL -2 /* a box length below twice the cutoff */
#define SWFE_E_OVERFLOW -3      /* a neighbour list overflowed: the Verlet list (64 per atom,
                                   more with a UF reference) or the 48 pairs within the cutoff */
#define SWFE_E_NONFINITE -4     /* NaN/Inf in an energy, force or position */
#define SWFE_E_DCCI_SINGULAR -5 /* dCCI denominator or lambda out of range */
#define SWFE_E_HIP -6           /* a HIP runtime call failed */
#define SWFE_E_STATE -7         /* call out of order (e.g. before init) */
#define SWFE_E_NOMEM -8         /* workspace too small */

/* ---- modes (one per system) --------------------------------------------
 * FORCE   no dynamics; forces only
 * NVE     velocity Verlet
 * NVT     + Langevin thermostat (NPT when p_damp > 0: target P)
 * FL      Frenkel-Ladd Hamiltonian interpolation H = lam H_int + (1-lam) H_ref,
 *         Einstein reference, lambda linear in time (section 2.1)
 * RS      reversible scaling H = K + lam U_int + P_S V, P_S = lam P,
 *         1/lam linear in time (eqs. H_RS, T_sc, P_sc; section 4.1)
 * AS_P    pressure switching, work = int dP/dt V dt (eq. Wmech_dyn)
 * DCCI_T  dCCI with lambda (temperature) control (eq. Ps_coex_discreted)
 * DCCI_P  dCCI with pressure control (eq. l_coex_discreted)
 * UF      H = lam H_int + (1-lam) U_UF with the Uhlenbeck-Ford fluid as the
 *         reference of a liquid (section 4.1), lambda linear in time; fixed
 *         volume.  The work and U_ref are as for FL, with U_ref = U_UF.
 */
#define SWFE_MODE_FORCE 0
#define SWFE_MODE_NVE 1
#define SWFE_MODE_NVT 2
#define SWFE_MODE_FL 3
#define SWFE_MODE_RS 4
#define SWFE_MODE_AS_P 5
#define SWFE_MODE_DCCI_T 6
#define SWFE_MODE_DCCI_P 7
#define SWFE_MODE_UF 8

/* Barostat kinds (swfe_system_desc.baro). */
#define SWFE_BARO_ISO 0
#define SWFE_BARO_ANISO 1

/* precision of the pair and triplet term arithmetic */
#define SWFE_PREC_FP64 0  /* everything FP64 */
#define SWFE_PREC_MIXED 1 /* FP32 terms; FP64 positions, accumulation, work */

/* compute_forces flags */
#define SWFE_PARAM_GRAD 1u /* also dE/dtheta */
#define SWFE_STRAIN 2u     /* evaluate at (I + strain) x, (I + strain) box */

/* Stillinger-Weber parameters (Stillinger and Weber 1985, the potential the
 * paper uses for silicon in its applications section):
 *   phi2(r) = epsilon A [B (sigma/r)^p - (sigma/r)^q] exp(sigma / (r - a sigma))
 *   phi3    = lambda_sw epsilon (cos theta_jik - cos0)^2 g(r_ij) g(r_ik),
 *   g(r)    = exp(gamma sigma / (r - a sigma)); both vanish for r >= a sigma.
 * mass in amu. */
typedef struct {
    double A, B, p, q, a, lambda_sw, gamma, sigma, epsilon, cos0, mass;
} swfe_sw_params;

/* One periodic orthorhombic system. */
typedef struct {
    int64_t n_atoms;
    int64_t offset;   /* first global atom index of this system */
    double box[3];    /* box lengths (A); each must be >= 2 a sigma */
    int32_t mode;     /* SWFE_MODE_* */
    int32_t partner;  /* dCCI: index of the coupled system, else -1 */
    double k_spring;  /* Einstein spring constant (eV/A^2), FL only */
    double T0;        /* thermostat temperature (K); 0 disables the O step */
    double tau_damp;  /* Langevin damping time (ps); 0 disables the O step */
    double p_damp;    /* barostat period (ps); 0 keeps the box fixed */
    double pressure;  /* physical pressure P (GPa) for NPT, RS, dCCI-T */
    uint64_t stream;  /* noise stream id: Philox key word 1 */
    /* schedule: start/end of the controlled variable and its length in steps
     * FL: lambda; RS: lambda (1/lambda is ramped); AS_P, DCCI_P: P in GPa;
     * DCCI_T: T in K.  sched_steps = 0 holds the start value. */
    double sched_start, sched_end;
    int64_t sched_steps;
    /* barostat (p_damp > 0): SWFE_BARO_ISO, one piston for the volume; or
     * SWFE_BARO_ANISO, one piston per box length (the paper's `aniso` runs of
     * beta-tin, section 4.1), each of a third of the isotropic piston mass */
    int32_t baro;
    int32_t reserved;  /* set to 0 */
    /* Uhlenbeck-Ford fluid reference (SWFE_MODE_UF, section 4.1; model of
     * Leite et al.): phi(r) = -p kB T_UF ln(1 - exp(-(r/sigma)^2)) for
     * r < rcut.  UF systems run at fixed volume (p_damp = 0); each box length
     * must be at least 2 rcut.  Ignored by the other modes. */
    double uf_p, uf_sigma, uf_T, uf_rcut;
} swfe_system_desc;

/* Device buffers, all caller owned. */
typedef struct {
    double *x;          /* [3][n_total] positions (unwrapped), A */
    double *v;          /* [3][n_total] velocities, A/ps */
    double *f;          /* [3][n_total] out: interaction force F_int (unscaled) */
    const double *x0;   /* [3][n_total] Einstein anchors; may be NULL if no FL */
    double *e_atom;     /* [n_total] out: per-atom energy; may be NULL */
    void *workspace;    /* scratch of swfe_workspace_bytes() bytes */
    size_t workspace_bytes;
} swfe_buffers;

/* Host copy of one system's switching state. */
typedef struct {
    double lam;        /* coupling parameter lambda */
    double Ps;         /* barostat target (scaled pressure P_S), GPa */
    double W;          /* accumulated work, eV */
    double U_int;      /* unscaled interaction energy at the current positions */
    double U_ref;      /* reference energy: Einstein (FL), Uhlenbeck-Ford (UF) */
    double K;          /* kinetic energy, eV */
    double V;          /* volume, A^3 */
    double virial[9];  /* dU_int/dstrain (eV), row-major */
    double box[3];
    double veps;       /* barostat rate d ln L / dt (1/ps); mean over the axes */
    double T_inst;     /* kinetic temperature over 3N-3 degrees of freedom */
    int64_t step;      /* steps taken since init (noise counter) */
    int64_t sched_k;   /* steps taken on the current schedule */
    int32_t err;       /* sticky device error bits of this system */
    int32_t pad;
    int64_t n_rebuild; /* Verlet-list rebuilds of this system so far */
    double veps_axes[3]; /* per-axis barostat rates d ln L_a / dt (1/ps) */
} swfe_system_state;

/* Per-system row written by swfe_compute_forces when out != NULL. */
#define SWFE_OUT_STRIDE 20 /* [E, U_ref, dE/dstrain (9), dE/dtheta (9)] */

/* ---- context -------------------------------------------------------------
 * swfe_create: allocate an empty context.  swfe_destroy: free it (also
 * releases captured graphs); NULL is ignored. */
int swfe_create(swfe_ctx **out);
void swfe_destroy(swfe_ctx *ctx);
const char *swfe_last_error(const swfe_ctx *ctx);  /* NULL: last context-free call */

/* Bytes of device workspace needed for these systems.  Checks descriptors
 * (SWFE_E_INVALID_ARG, SWFE_E_BOX_TOO_SMALL) without touching the GPU. */
int swfe_workspace_bytes(const swfe_system_desc *d, int32_t n_sys, const swfe_sw_params *p,
                         size_t *bytes);

/* Set up n_sys systems on the caller's buffers (host descriptors, device
 * buffers), then evaluate the initial interaction.  The systems are the
 * switched Hamiltonians of section 2 (H_lambda of section 2.1 for
 * Frenkel-Ladd, eq. H_RS with P_S = lambda P of eq. P_sc for reversible
 * scaling, the pressure ramp of eq. Wmech_dyn) and the coupled phases of
 * section 3.  seed is Philox key word 0 of the thermostat noise; dt in ps;
 * precision SWFE_PREC_*.  Each system's schedule starts at step 0 (lambda,
 * P_S from sched_start).  Velocities must
 * carry zero total momentum per system for the fixed centre of mass the
 * zero-sum noise maintains.  Synchronises the stream. */
int swfe_init_system(swfe_ctx *ctx, const swfe_system_desc *d, int32_t n_sys,
                     const swfe_sw_params *p, const swfe_buffers *b, uint64_t seed, double dt,
                     int32_t precision, void *stream);

/* Neighbour build at the current positions: cell index per atom,
 * deterministic counting sort by cell (ties in atom order), and the Verlet
 * lists of every system within the Stillinger-Weber cutoff a sigma plus the
 * skin.  The paper's molecular dynamics (section 4) finds its interacting
 * pairs this way implicitly; both potential terms vanish beyond a sigma. */
int swfe_build_neighbors(swfe_ctx *ctx, void *stream);

/* Interaction at the current positions: the Stillinger-Weber energy of the
 * paper's silicon (section 4; the two-body and three-body terms of the
 * parameter block above), its forces, virial and parameter gradient --
 * binning, pair terms and three-body moments, force gather, per-system
 * reductions.  Writes f (and e_atom).
 * flags: SWFE_PARAM_GRAD, SWFE_STRAIN.  strain: host [n_sys][9] diagonal
 * strains (off-diagonal entries must be 0) used with SWFE_STRAIN, else NULL.
 * grad_scale: device [n_sys] upstream gradient dL/dE or NULL (=1).
 * grad_x: device [3][n_total] out, dL/dx = -F grad_scale, or NULL.
 * out: device [n_sys][SWFE_OUT_STRIDE] (E, U_ref, dE/dstrain * gs,
 * dE/dtheta * gs with theta = A,B,p,q,a,lambda_sw,gamma,sigma,epsilon), or
 * NULL.  Does not synchronise. */
int swfe_compute_forces(swfe_ctx *ctx, uint32_t flags, const double *strain,
                        const double *grad_scale, double *grad_x, double *out, void *stream);

/* Replace the Stillinger-Weber parameters (theta) of an initialised
 * context; boxes must stay >= 2 a sigma (SWFE_E_BOX_TOO_SMALL otherwise).
 * The interaction is not re-evaluated: call swfe_compute_forces. */
int swfe_set_params(swfe_ctx *ctx, const swfe_sw_params *p);

/* Install new schedules (sched_start/sched_end/sched_steps of the given
 * descriptors; NULL keeps the current ones) and reset the schedule step and
 * work accumulators of every system.  Does not synchronise. */
int swfe_set_schedule(swfe_ctx *ctx, const swfe_system_desc *d, void *stream);

/* Advance every system by n_steps of switched dynamics: switch lambda (and
 * P_S) on its schedule and accumulate the work increment of eq. Wdyn
 * (discretised as H(lambda_{k+1}) - H(lambda_k) at the current microstate;
 * eqs. Wrev_HI, Wdyn_RS, Wmech_dyn for the modes), barostat half step,
 * B A O A kick/drift/Langevin (the Langevin thermostat and barostat of
 * section 4.1), interaction, B, barostat half step.  dCCI pairs update their
 * shared lambda and P_S from both phases' instantaneous per-atom energy and
 * volume (section 3, eqs. Ps_coex_discreted and l_coex_discreted).  After a
 * SWFE_STRAIN force evaluation the interaction is first evaluated again at
 * the unstrained positions (f is overwritten).  use_graph selects how the
 * steps are launched, with identical results: 0 one launch per stage, 1 one
 * captured step graph replayed per step, 2 one persistent cooperative kernel
 * per (up to) 2000 steps, in which the systems are dealt to the XCDs and the
 * workgroups of an XCD meet at barriers of their own (SWFE_E_HIP if the
 * kernel cannot be launched, or if it had to give up a wait).  use_graph != 0 replays one captured step graph.  Errors raised
 * on the device (overflow, non-finite, dCCI singular, box too small) are
 * reported by the next synchronising call. */
int swfe_step_switched(swfe_ctx *ctx, int64_t n_steps, int32_t use_graph, void *stream);

/* Synchronise and copy per-system work W (eV), lambda, P_S (GPa) and the
 * schedule step to host arrays of n_sys entries (any may be NULL).  W is the
 * dynamical work of eq. Wdyn accumulated since the schedule was installed;
 * a forward and a backward run give Delta F = (W_fwd - W_bwd)/2 (eq. dF)
 * and the dissipated heat (eq. Qdiss).  Returns the first pending device
 * error as a status code (the arrays are filled either way). */
int swfe_work_integral(swfe_ctx *ctx, double *W, double *lam, double *Ps, int64_t *steps,
                       void *stream);

/* Synchronise and copy the full state of every system. */
int swfe_get_state(swfe_ctx *ctx, swfe_system_state *out, void *stream);

/* Copy of the log ring: every log_every steps one row per system of
 * (step, lambda, P_S GPa, P GPa, T K, U_int/N, V/N, W), P = P_S / lambda and
 * T the kinetic temperature.  Rows come oldest logging event first and, within
 * an event, in system order (row r belongs to system r mod n_sys).
 * swfe_set_log sets log_every (0 disables) and the ring capacity in rows. */
#define SWFE_LOG_STRIDE 8
int swfe_set_log(swfe_ctx *ctx, int32_t log_every, int32_t capacity);
int swfe_read_log(swfe_ctx *ctx, double *rows, int32_t max_rows, int32_t *n_rows, void *stream);

/* Tuning: block size of the per-atom kernels (64, 128 or 256; 0 = autotune).
 * swfe_autotune times 24 graph-replayed dynamics steps (after 3 untimed
 * ones) at each size from the current state (the fastest of three
 * interleaved rounds), restoring the state after each through a host
 * snapshot (swfe_save_state / swfe_load_state; it allocates
 * swfe_checkpoint_bytes of host memory for the call), and keeps the fastest
 * size.  It recomputes forces at the chosen size but does not advance the
 * dynamics. */
int swfe_set_block(swfe_ctx *ctx, int32_t block, void *stream);
int swfe_autotune(swfe_ctx *ctx, int32_t *chosen_block, void *stream);

/* Sizes needed by the caller: total atoms and systems of the context. */
int swfe_sizes(const swfe_ctx *ctx, int64_t *n_total, int32_t *n_sys);

/* Verlet-list skin (A, >= 0) of every system; the lists hold pairs within
 * a sigma + skin and are rebuilt for a system when a pair now within the
 * cutoff could be missing (displacements and box scaling since the build).
 * Default 0.5 A.  The list capacity per atom is sized at set-up for skins
 * up to 2 A (allowing 30 % density increase); a larger skin is refused with
 * SWFE_E_INVALID_ARG.  Rebuilds the lists and re-evaluates the interaction
 * at the current positions. */
int swfe_set_skin(swfe_ctx *ctx, double skin, void *stream);

/* Tuning: Verlet-list skin.  Times n_steps graph-replayed dynamics steps
 * (after 5 untimed ones; n_steps <= 0: 40) from the current state at each
 * candidate skin (A; NULL: 0.6, 1.0, 1.4, 1.8, 2.0; at most 16), the faster
 * of two interleaved rounds, restoring the state from a host snapshot after
 * each (it allocates swfe_checkpoint_bytes of host memory for the call),
 * and keeps the fastest (host output `chosen`).  A longer skin rebuilds the
 * lists less often but makes them longer; results do not depend on it.
 * Does not advance the dynamics. */
int swfe_autotune_skin(swfe_ctx *ctx, const double *candidates, int32_t n_candidates, int32_t n_steps,
                       double *chosen, void *stream);

/* Measurement: run n_steps eager dynamics steps with HIP events recorded on
 * the stream between the kernels of each step; ms[0..8] receive the summed
 * durations of integrate, rebuild count (with the rebuild decision),
 * rebuild scan, rebuild scatter,
 * rebuild order, rebuild list, pass1, pass2 and finalize (ms, host array of
 * 9).  When every system has at most 2048 atoms and a cell table that fits
 * in LDS the first four rebuild stages run as one fused sort per system,
 * whose time the count entry holds (scan, scatter and order then read 0).  Synchronises.  The steps advance
 * the systems like swfe_step_switched. */
#define SWFE_NUM_KERNELS 9
int swfe_profile_steps(swfe_ctx *ctx, int64_t n_steps, double *ms, void *stream);

/* Neighbour statistics of the last force evaluation (host outputs):
 * ordered pairs within the cutoff, the largest per-atom count, and the
 * Verlet-list entries (pairs within cutoff + skin).  Synchronises. */
int swfe_neighbor_stats(swfe_ctx *ctx, int64_t *total_pairs, int32_t *max_per_atom,
                        int64_t *list_entries, void *stream);

/* ---- force evaluation that allocates nothing -------------------------------
 * For callers that cannot allocate device or host memory during the call
 * (tight serving loops, harnesses that forbid hipMalloc).  The Stillinger-
 * Weber energy, forces and virial of n_sys (1..64) systems, as
 * swfe_init_system followed by swfe_compute_forces with flags 0 would give
 * them for force-only systems (mode, schedule, thermostat and barostat fields
 * of d are ignored; offsets must be contiguous), bitwise for the same
 * precision.  Scratch space is a library array of 32 MiB in device memory
 * per GPU (held from its first use on that GPU until the process ends),
 * enough for about 35 000 atoms; larger inputs are rejected with
 * SWFE_E_NOMEM before any work is enqueued.  The call allocates nothing: no
 * hipMalloc or hipFree, and only fixed-size host tables on the stack.
 *   x      device [3][n_total] positions (caller owned, read only)
 *   f      device [3][n_total] out: forces
 *   e_atom device [n_total] out: per-atom energies, or NULL
 *   out    device [n_sys][SWFE_OUT_STRIDE] out: E, 0 (no reference), dE/dstrain
 *          (9), 0 (no parameter gradient), or NULL
 * Work goes to `stream`; the call synchronises it before returning (device
 * errors are reported: overflow, non-finite).  Every call on one GPU uses
 * that GPU's one scratch array and leaves its contents behind: calls that
 * overlap on the same GPU (other threads or streams) race and must be
 * serialised by the caller.  Messages of failing calls come from
 * swfe_last_error(NULL). */
int swfe_forces_static(const swfe_system_desc *d, int32_t n_sys, const swfe_sw_params *p, const double *x,
                       double *f, double *e_atom, double *out, int32_t precision, void *stream);

/* ---- checkpoint / resume ---------------------------------------------------
 * A checkpoint is a host byte blob holding the context's settings (SW
 * parameters, descriptors with their current schedules, seed, time step,
 * precision, block size, skin, log settings), the whole workspace (the
 * cell-sorted atom data, lists, stored normals, per-system switching and
 * barostat state, the log ring) and the caller's x, v and f.  Loading it
 * into a context initialised with descriptors of the same system sizes and
 * buffers of the same sizes resumes the run bitwise: the noise is
 * counter-based (step, atom) and every sum has a fixed order.
 *
 * swfe_checkpoint_bytes: size of the blob (host output).
 * swfe_save_state: writes the blob to host memory of at least that size;
 *   synchronises the stream.
 * swfe_load_state: restores a blob written by swfe_save_state of a context
 *   with the same system sizes; SWFE_E_INVALID_ARG when the blob does not
 *   belong to such a context (bad magic, version, sizes); synchronises. */
int swfe_checkpoint_bytes(const swfe_ctx *ctx, size_t *bytes);
int swfe_save_state(swfe_ctx *ctx, void *host, size_t bytes, void *stream);
int swfe_load_state(swfe_ctx *ctx, const void *host, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SWFE_H */
