// swfe_internal.h -- layouts shared by the host runtime and the HIP kernels of
// libswfe (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace swfe {

constexpr int kMaxList = 64;       // smallest Verlet-list capacity per atom
constexpr int kMaxListUF = 1024;   // largest capacity the planning may ask for
// Verlet lists are sized for skins up to this (A), or up to the context's
// skin when it is larger; set_skin refuses a larger skin afterwards.
constexpr double kPlanSkin = 2.0;
constexpr int kMaxShort = 48;      // neighbours within rc per atom (pass 1 -> pass 2)
// short-list entries pass 1 keeps in LDS per atom (the rest, rarely any, in
// the global short list): its term loop reads them without a round trip to
// memory
constexpr int kLdsShort = 24;
constexpr int kFxChunks = 4;      // runs of tiles per XCD (block placement)
constexpr int kSortThreads = 1024; // threads of the per-system sort workgroup
constexpr int kSortLdsCells = 12288; // cell table entries the fused sort keeps in LDS (48 KB)
// The fused sort puts a whole system on one workgroup: it pays off only when
// every system of the batch is small (the separate stages spread a large
// system's sort over the chip; measured on the 64-replica batch with systems
// of up to 13 824 atoms, the fused sort became the longest kernel of a step).
constexpr int kSortFuseMaxAtoms = 2048;
constexpr int kNumKernels = 9;     // launches of one dynamics step (for profiling)
constexpr int kRebuildStages = 5;  // rebuild stages
constexpr int kWorkGrid = 512;     // blocks of the work-list rebuild kernels

// Per-tile partial sums of the two force passes (fixed slots).
enum : int {
    P_E = 0,        // pass 1: two-body energy
    P_VIR = 1,      // 9 virial components dE/dstrain
    P_DTH = 10,     // 9 parameter derivatives
    P_UREF = 19,    // pass 2: Einstein energy
    P_K = 20,       // pass 2: kinetic energy per axis (3)
    P_NOISE = 23,   // pass 2: 3 sums of the next O step's normals
    P_E3 = 19,      // pass 1: three-body energy (slot 19 of the pass-1 row)
    P_UUF = 20,     // pass-1 row: Uhlenbeck-Ford reference energy (UF kernel)
    kNumPart = 26
};

// Device error bits (per system, sticky until read by the host).
enum : int { ERR_OVERFLOW = 1, ERR_NONFINITE = 2, ERR_DCCI = 4, ERR_BOX = 8, ERR_PERSIST = 16 };

// Persistent step kernel: the systems of the batch are dealt to the 8 XCDs
// (whole reduction groups), and the workgroups running on an XCD step that
// XCD's systems, meeting at barriers of their own XCD.
constexpr int kXcds = 8;
constexpr int kPersistMaxSysPerXcd = 256;  // systems one XCD may own
constexpr int kSyncWords = 16 * 16;        // 64-bit words of the barrier area
// barrier-area word offsets (each counter on its own 128-byte line)
constexpr int SYNC_START = 0;              // arrivals at the start-up barrier
constexpr int SYNC_XCD = 16;               // 16 * (1 + x): barrier counter of XCD x
constexpr int SYNC_REG = 16 * 9;           // + x: workgroups that registered on XCD x
constexpr int SYNC_ABORT = 16 * 10;        // non-zero: a wait gave up; every block leaves

struct XcdPlan {
    int32_t tile_off[kXcds + 1];   // XCD x steps tiles xtiles[tile_off[x] .. tile_off[x + 1])
    int32_t group_off[kXcds + 1];  // and groups xgroups[group_off[x] .. group_off[x + 1])
    int32_t sys_off[kXcds + 1];    // whose systems are xsys[sys_off[x] .. sys_off[x + 1])
};

enum : int {
    MODE_FORCE = 0, MODE_NVE = 1, MODE_NVT = 2, MODE_FL = 3,
    MODE_RS = 4, MODE_AS_P = 5, MODE_DCCI_T = 6, MODE_DCCI_P = 7, MODE_UF = 8
};

struct SwParams {
    double A, B, p, q, a, lam, gam, sig, eps, cos0;
    double rc, rc2, eA, le;   // a*sig, rc^2, eps*A, lambda_sw*eps
    int32_t ip, iq;           // integer exponents, or -1 when not integral
};

// Constant per-system description (uploaded at set-up).
struct SysDesc {
    int64_t off, n;
    int32_t mode, partner;
    int32_t cell_base, cell_cap;  // cell-array slots of this system
    int32_t nc_max[3];
    int32_t tile_begin, tile_end; // tiles of this system (contiguous)
    int32_t group;                // reduction group (a system or a dCCI pair)
    int32_t baro;                 // 0: one piston (volume), 1: one piston per axis
    double uf_pkT, uf_is2, uf_rc; // UF reference: p kB T_UF (eV), 1/sigma^2, cutoff (0: none)
    double k_spring, T0, tau_damp, p_damp;
    double pressure;          // eV/A^3
    double nf;                // 3N - 3
    double alpha;             // 1 + 3/nf
    double wpiston;           // piston mass, eV ps^2
    double c1, c2, sigv;      // O-step constants; sigv in A/ps
    double acc;               // (A/ps^2) per (eV/A): 1 / (m * mvv2e)
    double mvv2e_m;           // 0.5 m mvv2e: kinetic energy eV per (A/ps)^2
    double skin;              // Verlet-list skin, A
    uint64_t stream;
    double s_start, s_end;
    int64_t s_steps;
};

// Reduction group: one system, or the two phases of a dCCI pair.
struct Group {
    int32_t s0, s1;                // s1 = -1 for a single system
    int32_t tile_begin, tile_end;  // tiles of both systems (contiguous)
};

// Dynamic per-system state (device resident).
struct SysState {
    double lam, Ps, W;
    double veps[3];                 // piston rates d ln L_a / dt (equal when isotropic)
    double box[3];
    double box_build[3];            // box in which the Verlet list was built
    double U_int, U_ref, K, V, E2, E3;
    double K3[3];                   // kinetic energy per axis
    double vir[9];
    double dth[9];
    double noise_mean[3];
    double decay[3], phi[3], grow[3], psi[3];  // per-axis integrator factors of the current step
    double pscale[3];               // diagonal strain applied by compute_forces
    int64_t step;                   // steps since set-up (noise counter)
    int64_t k;                      // steps on the current schedule
    int64_t remaining;              // steps left in the current call
    int64_t n_rebuild;              // Verlet-list rebuilds so far
    int32_t err;
    int32_t pad;
};

// Three doubles (24 bytes) for the per-atom vectors that are streamed and
// never gathered by neighbours; the gathered positions stay double4, one
// aligned 32-byte record per atom.
struct dvec3 {
    double x, y, z;
};

__host__ __device__ __forceinline__ dvec3 make_dvec3(double x, double y, double z) { return dvec3{x, y, z}; }

struct Tile {
    int32_t sys, start, count, pad;
};

// Global launch parameters.
struct Ctl {
    int64_t n_total;
    int32_t n_sys, n_tiles, n_groups, fx_len;  // fx_len: tiles per run (tile placement)
    double dt;
    uint64_t seed;
    int32_t flags;          // PARAM_GRAD / STRAIN
    int32_t list_cap;       // Verlet-list capacity per atom (entries)
    int32_t list16;         // 1: 16-bit list entries (every system below 65537 atoms)
    int32_t has_uf;         // 1: some system switches to the UF reference
    int32_t in_step;        // 1: the pass belongs to a dynamics step
    int32_t force_rebuild;  // 1: rebuild every system's list now
    int32_t log_every, log_cap;
    int32_t sort_cells;     // LDS cell-table entries of the fused sort (0: separate stages)
    int32_t scan_cells;     // > 0: the scatter stage scans each system's cell counts in LDS (this many
                            // entries) and the scan launch is skipped; 0: separate scan launch
    // The tiles are cut into 8 * kFxChunks runs of fx_len tiles; XCD x runs
    // the runs fx_chunk[x * kFxChunks + j], j < kFxChunks.
    int32_t fx_chunk[8 * kFxChunks];
};

struct DevPtrs {
    // caller arrays, original atom order, [3][n_total]
    double *x, *v, *f;
    const double *x0;
    double *e_atom;
    // internal arrays, cell-sorted order
    double4 *xs;                          // positions
    dvec3 *vs, *fs, *x0s, *xb;            // velocities, F_int, anchors, build positions
    double4 *txs;                         // permutation staging
    dvec3 *tvs, *tfs, *tx0s;
    dvec3 *zs;                            // normals of the next O step, sorted order
    float4 *xf;                           // FP32 positions wrapped into the box (list filter)
    int32_t *perm, *tperm, *norder, *rank, *cellid;  // norder: staged cell index
    int32_t *cell_count, *cell_start;
    int32_t *nl, *nl_cnt;                 // Verlet list of sorted positions (layouts at list_put)
    int32_t *nnb;                         // neighbours within rc per atom (last pass 1)
    int32_t *sl;                          // those neighbours, in the Verlet list's entry format (list_put)
    void *mom;                            // [n_total][9] moments (v, M) in term precision
    double *e_s;                          // per-atom energy, sorted order
    double *part1, *part2;                // [n_tiles][kNumPart]
    dvec3 *fref;                          // UF reference force per atom (UF systems), sorted order
    int32_t *work, *n_work;               // tiles to rebuild in this step, and their count
    double *disp_max;                     // [n_sys][2] max squared displacement since build
                                          // (two slots alternate between steps)
    const SysDesc *desc;
    SysState *state;
    const Tile *tiles;
    const Group *groups;
    double *log;
    // persistent step kernel: per-XCD tile, group and system lists, each
    // system's index in its XCD's list, and the barrier area
    int32_t *xtiles, *xtloc, *xgroups, *xsys;  // xtloc: XCD-list index of each listed tile's system
    unsigned long long *sync;
    // per-call outputs of compute_forces
    const double *grad_scale;
    double *grad_x;
    double *out;
};

// Launchers (defined in swfe_kernels.hip).  `block` is the tile size.
hipError_t launch_iota(const Ctl &c, const DevPtrs &p, int block, hipStream_t s);
hipError_t launch_gather(const Ctl &c, const DevPtrs &p, int block, int with_f, hipStream_t s);
hipError_t launch_scatter(const Ctl &c, const DevPtrs &p, int block, int what, hipStream_t s);
hipError_t launch_integrate(const Ctl &c, const DevPtrs &p, const SwParams &sw, int block,
                            hipStream_t s);
hipError_t launch_rebuild(const Ctl &c, const DevPtrs &p, const SwParams &sw, int block, int stage,
                          hipStream_t s);
hipError_t launch_fill_noise(const Ctl &c, const DevPtrs &p, int block, hipStream_t s);
hipError_t launch_pass1(const Ctl &c, const DevPtrs &p, const SwParams &sw, int mixed, int block,
                        hipStream_t s);
hipError_t launch_pass2(const Ctl &c, const DevPtrs &p, const SwParams &sw, int mixed, int block,
                        hipStream_t s);
hipError_t launch_finalize(const Ctl &c, const DevPtrs &p, const SwParams &sw, hipStream_t s);
hipError_t launch_begin_step(const Ctl &c, const DevPtrs &p, const SwParams &sw, int64_t n_steps,
                             hipStream_t s);
hipError_t launch_reset_schedule(const Ctl &c, const DevPtrs &p, hipStream_t s);
hipError_t launch_set_pscale(const Ctl &c, const DevPtrs &p, const double *diag, hipStream_t s);
hipError_t launch_clear_err(const Ctl &c, const DevPtrs &p, hipStream_t s);
hipError_t launch_zero_words(void *w, size_t bytes, hipStream_t s);
// Persistent step kernel (cooperative launch of `grid` blocks of `block`
// threads) running n_steps steps, then the check that turns a failed wait
// into ERR_PERSIST on every system.
int persist_blocks_per_cu(int mixed, int block);
hipError_t launch_persist(const Ctl &c, const DevPtrs &p, const SwParams &sw, const XcdPlan &xp, int mixed,
                          int block, int grid, int64_t n_steps, hipStream_t s);

}  // namespace swfe
