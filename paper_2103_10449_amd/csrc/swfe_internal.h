// swfe_internal.h -- layouts shared by the host runtime and the HIP kernels of
// libswfe (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace swfe {

constexpr int kMaxNb = 32;        // neighbour-list capacity per atom
constexpr int kBinThreads = 1024; // threads of the per-system binning workgroup
constexpr int kFinThreads = 256;  // threads of the finalize workgroup

// Per-tile partial sums written by the two force passes (fixed slots).
enum : int {
    P_E = 0,        // energy (pass 1: two-body, pass 2: three-body)
    P_VIR = 1,      // 9 virial components dE/dstrain
    P_DTH = 10,     // 9 parameter derivatives
    P_UREF = 19,    // Einstein energy (pass 2)
    P_K = 20,       // kinetic energy (pass 2)
    P_NOISE = 21,   // 3 sums of the next O step's normals (pass 2)
    kNumPart = 24
};

// Device error bits (per system, sticky until read by the host).
enum : int {
    ERR_OVERFLOW = 1,
    ERR_NONFINITE = 2,
    ERR_DCCI = 4,
    ERR_BOX = 8,
};

enum : int {
    MODE_FORCE = 0, MODE_NVE = 1, MODE_NVT = 2, MODE_FL = 3,
    MODE_RS = 4, MODE_AS_P = 5, MODE_DCCI_T = 6, MODE_DCCI_P = 7
};

struct SwParams {
    double A, B, p, q, a, lam, gam, sig, eps, cos0;
    double rc, rc2, eA, le;   // a*sig, rc^2, eps*A, lambda_sw*eps
    int32_t ip, iq;           // integer exponents, or -1 when not integral
};

// Constant per-system description (uploaded once).
struct SysDesc {
    int64_t off, n;
    int32_t mode, partner;
    int32_t cell_base;        // first slot of this system in the cell arrays
    int32_t cell_cap;         // capacity (cells) of this system
    int32_t nc_max[3];
    int32_t tile_begin, tile_end;
    int32_t pad0;
    double k_spring, T0, tau_damp, p_damp;
    double pressure;          // eV/A^3
    double nf;                // 3N - 3
    double alpha;             // 1 + 3/nf
    double wpiston;           // piston mass, eV ps^2
    double c1, c2, sigv;      // O-step constants; sigv in A/ps
    double acc;               // (A/ps^2) per (eV/A): 1 / (m * mvv2e)
    double mvv2e_m;           // 0.5 m mvv2e: kinetic energy eV per (A/ps)^2
    uint64_t stream;
    double s_start, s_end;
    int64_t s_steps;
};

// Dynamic per-system state (device resident).
struct SysState {
    double lam, Ps, W, veps;
    double box[3];
    double U_int, U_ref, K, V, E2, E3;
    double vir[9];
    double dth[9];
    double noise_mean[3];
    double decay, phi, grow, psi;   // integrator factors of the current step
    double pscale[3];               // diagonal strain applied by compute_forces
    int64_t step;                   // steps since init (noise counter)
    int64_t k;                      // steps on the current schedule
    int32_t nc[3];                  // cell grid of the current box
    int32_t err;
};

struct Tile {
    int32_t sys, start, count, pad;
};

// Workspace carve-up (offsets in bytes from the workspace base).
struct Layout {
    size_t cell_of, sorted, cell_count, cell_start, cursor, nbr, nnb, mom, f2, part1, part2,
        desc, state, tiles, log, misc, total;
};

// Global launch parameters of one force / step pass.
struct Ctl {
    int64_t n_total;
    int32_t n_sys, n_tiles;
    double dt;
    uint64_t seed;
    int32_t flags;       // PARAM_GRAD / STRAIN
    int32_t in_step;     // 1: the pass belongs to a dynamics step
};

struct DevPtrs {
    double *x, *v, *f;
    const double *x0;
    double *e_atom;
    int32_t *cell_of, *sorted, *cell_count, *cell_start, *cursor;
    int32_t *nbr, *nnb;
    double *mom;     // [11][n_total]
    double *f2;      // [3][n_total]
    double *part1, *part2;  // [n_tiles][kNumPart]
    const SysDesc *desc;
    SysState *state;
    const Tile *tiles;
    double *log;     // ring of rows
    int32_t *misc;   // [0] call_end low, ... see kernels
    int64_t *ctr;    // [0] steps remaining in the current call, [1] log head
    const double *grad_scale;
    double *grad_x;
    double *out;
};

// Launchers (defined in swfe_kernels.hip).  `block` is the tile size.
hipError_t launch_assign_cells(const Ctl &c, const DevPtrs &p, const SwParams &sw, int block,
                               hipStream_t s);
hipError_t launch_bin(const Ctl &c, const DevPtrs &p, const SwParams &sw, hipStream_t s);
hipError_t launch_pass1(const Ctl &c, const DevPtrs &p, const SwParams &sw, int mixed, int block,
                        hipStream_t s);
hipError_t launch_pass2(const Ctl &c, const DevPtrs &p, const SwParams &sw, int mixed, int block,
                        hipStream_t s);
// mode: 0 = reductions only, 1 = end of a step (+ next step's start), 2 = start of a step
hipError_t launch_finalize(const Ctl &c, const DevPtrs &p, const SwParams &sw, int mode,
                           int log_every, int log_cap, hipStream_t s);
hipError_t launch_integrate(const Ctl &c, const DevPtrs &p, const SwParams &sw, int block,
                            hipStream_t s);
hipError_t launch_reset_schedule(const Ctl &c, const DevPtrs &p, hipStream_t s);
hipError_t launch_set_pscale(const Ctl &c, const DevPtrs &p, const double *diag, hipStream_t s);

}  // namespace swfe
