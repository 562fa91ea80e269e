// swfe_api.hip -- host runtime behind the C-ABI declared in include/swfe.h.
//
// Holds the per-context tables (system descriptors, reduction groups, the
// tile list, the workspace carve-up), validates inputs, enqueues the kernels
// of swfe_kernels.hip on the caller's stream and, on request, captures one
// dynamics step into a HIP graph that is replayed for every step.
#include "../../include/swfe.h"
#include "swfe_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace swfe;

namespace {

// CODATA 2018 constants (metal units), defined here for the library.
constexpr double kKB = 8.617333262e-5;                                  // eV/K
constexpr double kMvv2e = 1.66053906660e-27 * 1e-20 / 1e-24 / 1.602176634e-19;  // eV/(amu A^2/ps^2)
constexpr double kGpa = 1.602176634e-19 / 1e-30 / 1e9;                  // GPa per eV/A^3
constexpr int kLogCapMax = 16384;                                       // rows of the log ring
constexpr size_t kAlign = 256;
constexpr double kDefaultSkin = 0.5;                                    // A
constexpr int64_t kPersistChunk = 2000;  // steps of one persistent launch

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t xs, vs, fs, x0s, xb, txs, tvs, tfs, tx0s, zs, xf, fref;
    size_t perm, tperm, norder, rank, cellid, nnb, sl, cell_count, cell_start, nl, nl_cnt, mom, e_s;
    size_t part1, part2, disp_max, work, n_work, desc, state, tiles, groups, log, strain;
    size_t xtiles, xtloc, xgroups, xsys, sync, total;
};

struct Plan {
    std::vector<SysDesc> desc;
    std::vector<Group> groups;
    int64_t n_total = 0;
    int64_t cells = 0;       // sum of per-system cell capacities
    int64_t max_tiles = 0;   // tiles at the smallest block size
    int32_t list_cap = kMaxList;  // Verlet-list rows per atom
    double list_skin = kPlanSkin;   // largest skin the list capacity was planned for, A
    Layout lay{};
};

}  // namespace

struct swfe_ctx {
    std::string err;
    bool ready = false;
    int n_sys = 0;
    int64_t n_total = 0;
    std::vector<swfe_system_desc> hdesc;
    swfe_sw_params hsw{};
    Plan plan;
    std::vector<Tile> tiles;
    std::vector<int32_t> fx_chunk;  // runs of tiles per XCD (empty: in order)
    int fx_tiles = 0;               // tile count fx_chunk was dealt for
    SwParams sw{};
    int mixed = 0;
    double dt = 0.001;
    uint64_t seed = 0;
    int block = 256;
    double skin = kDefaultSkin;
    swfe_buffers buf{};
    DevPtrs ptrs{};
    int log_every = 0, log_cap = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool graph_valid = false;
    hipStream_t cap_stream = nullptr;  // library-owned stream used only for capture
    // the last force evaluation was strained: forces, energies and virial
    // belong to the strained box until the interaction is evaluated again
    bool forces_stale = false;
    // persistent step kernel: systems dealt to the XCDs, and its grid
    XcdPlan xplan{};
    bool xplan_valid = false;
    int persist_grid = 0;
};

namespace {

// Message of the last failing call without a context (swfe_workspace_bytes,
// swfe_forces_static), returned by swfe_last_error(NULL).  A fixed buffer:
// recording it allocates nothing.
char g_free_err[256] = "";

int fail(swfe_ctx *c, int code, const char *msg)
{
    if (c) {
        c->err = msg;
    } else {
        strncpy(g_free_err, msg, sizeof g_free_err - 1);
        g_free_err[sizeof g_free_err - 1] = '\0';
    }
    return code;
}

#define HIPCHK(ctx, expr)                                                         \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            char m_[256];                                                         \
            snprintf(m_, sizeof m_, "%s: %s", #expr, hipGetErrorString(e_));      \
            return fail(ctx, SWFE_E_HIP, m_);                                     \
        }                                                                         \
    } while (0)

#define RCHK(expr)              \
    do {                        \
        int r_ = (expr);        \
        if (r_) return r_;      \
    } while (0)

bool is_dcci(int m) { return m == SWFE_MODE_DCCI_T || m == SWFE_MODE_DCCI_P; }

SwParams make_sw(const swfe_sw_params &p)
{
    SwParams s{};
    s.A = p.A;
    s.B = p.B;
    s.p = p.p;
    s.q = p.q;
    s.a = p.a;
    s.lam = p.lambda_sw;
    s.gam = p.gamma;
    s.sig = p.sigma;
    s.eps = p.epsilon;
    s.cos0 = p.cos0;
    s.rc = p.a * p.sigma;
    s.rc2 = s.rc * s.rc;
    s.eA = p.epsilon * p.A;
    s.le = p.lambda_sw * p.epsilon;
    auto integral = [](double e) { return (e >= 0 && e <= 16 && e == std::floor(e)) ? (int)e : -1; };
    s.ip = integral(p.p);
    s.iq = integral(p.q);
    return s;
}

// Validate descriptors; compute the device descriptors (desc[n_sys]), the
// reduction groups (groups[n_sys] of capacity, *n_groups used) and the
// workspace layout.  Writes only into the given arrays and P's scalars (no
// allocation); does not touch the GPU.
int plan_core(swfe_ctx *ctx, const swfe_system_desc *d, int n_sys, const swfe_sw_params *p, double dt,
              double skin, SysDesc *desc, Group *groups, int *n_groups, Plan &P)
{
    if (!d || !p || n_sys <= 0) return fail(ctx, SWFE_E_INVALID_ARG, "null descriptor/params or n_sys <= 0");
    if (!(p->a > 0 && p->sigma > 0 && p->mass > 0))
        return fail(ctx, SWFE_E_INVALID_ARG, "SW parameters need a > 0, sigma > 0, mass > 0");
    if (!(dt > 0)) return fail(ctx, SWFE_E_INVALID_ARG, "dt must be > 0");
    if (!(skin >= 0)) return fail(ctx, SWFE_E_INVALID_ARG, "skin must be >= 0");
    const double rc = p->a * p->sigma;
    P.list_cap = kMaxList;
    P.list_skin = std::max(skin, kPlanSkin);
    int64_t off = 0, tiles = 0, cells = 0;
    for (int s = 0; s < n_sys; ++s) {
        const swfe_system_desc &q = d[s];
        char msg[256];
        if (q.n_atoms < 2 || q.n_atoms > (1 << 30)) {
            snprintf(msg, sizeof msg, "system %d: n_atoms must be in [2, 2^30]", s);
            return fail(ctx, SWFE_E_INVALID_ARG, msg);
        }
        if (q.offset != off) {
            snprintf(msg, sizeof msg, "system %d: offset must be %lld (systems are contiguous)", s,
                     (long long)off);
            return fail(ctx, SWFE_E_INVALID_ARG, msg);
        }
        if (q.mode < 0 || q.mode > 8) return fail(ctx, SWFE_E_INVALID_ARG, "unknown mode");
        const bool uf = q.mode == SWFE_MODE_UF;
        if (uf && !(q.uf_p > 0 && q.uf_sigma > 0 && q.uf_T > 0 && q.uf_rcut > 0))
            return fail(ctx, SWFE_E_INVALID_ARG, "UF reference needs uf_p, uf_sigma, uf_T, uf_rcut > 0");
        if (uf && q.p_damp > 0) return fail(ctx, SWFE_E_INVALID_ARG, "UF switching runs at fixed volume");
        const double rmax = uf ? std::max(rc, q.uf_rcut) : rc;
        for (int k = 0; k < 3; ++k)
            if (!(q.box[k] >= 2.0 * rmax)) {
                snprintf(msg, sizeof msg, "system %d: box length %g below twice the cutoff %g", s,
                         q.box[k], 2.0 * rmax);
                return fail(ctx, SWFE_E_BOX_TOO_SMALL, msg);
            }
        if (q.tau_damp < 0 || q.T0 < 0 || q.p_damp < 0)
            return fail(ctx, SWFE_E_INVALID_ARG, "negative T0, tau_damp or p_damp");
        if (q.p_damp > 0 && !(q.T0 > 0))
            return fail(ctx, SWFE_E_INVALID_ARG, "a barostat (p_damp > 0) needs T0 > 0");
        if (q.mode == SWFE_MODE_FL && q.p_damp > 0)
            return fail(ctx, SWFE_E_INVALID_ARG, "Frenkel-Ladd switching runs at fixed volume");
        if (q.baro != SWFE_BARO_ISO && q.baro != SWFE_BARO_ANISO)
            return fail(ctx, SWFE_E_INVALID_ARG, "baro must be SWFE_BARO_ISO or SWFE_BARO_ANISO");
        if (q.mode == SWFE_MODE_RS && !(q.sched_start > 0 && q.sched_end > 0))
            return fail(ctx, SWFE_E_INVALID_ARG, "reversible scaling needs lambda > 0");
        if (q.mode == SWFE_MODE_DCCI_T && !(q.sched_start > 0 && q.sched_end > 0 && q.T0 > 0))
            return fail(ctx, SWFE_E_INVALID_ARG, "dCCI-T needs positive temperatures");
        if (is_dcci(q.mode)) {
            if (q.partner < 0 || q.partner >= n_sys || q.partner == s)
                return fail(ctx, SWFE_E_INVALID_ARG, "dCCI system without a valid partner");
            const swfe_system_desc &r = d[q.partner];
            if (r.partner != s || r.mode != q.mode || r.sched_start != q.sched_start ||
                r.sched_end != q.sched_end || r.sched_steps != q.sched_steps || r.T0 != q.T0 ||
                r.pressure != q.pressure)
                return fail(ctx, SWFE_E_INVALID_ARG,
                            "dCCI partners must point at each other and share mode, schedule, T0, P");
        }
        SysDesc sd{};
        sd.off = q.offset;
        sd.n = q.n_atoms;
        sd.mode = q.mode;
        sd.partner = is_dcci(q.mode) ? q.partner : -1;
        sd.baro = q.baro;
        if (uf) {
            sd.uf_pkT = q.uf_p * kKB * q.uf_T;
            sd.uf_is2 = 1.0 / (q.uf_sigma * q.uf_sigma);
            sd.uf_rc = q.uf_rcut;
        }
        {
            // list capacity for the system's longest cutoff at its density,
            // allowing skins up to the planned one and 30 % density increase
            const double rl = rmax + P.list_skin;
            const double dens = (double)q.n_atoms / (q.box[0] * q.box[1] * q.box[2]);
            const double want = 1.3 * 4.18879020478639 * rl * rl * rl * dens + 16.0;
            P.list_cap = std::max(P.list_cap, (int32_t)std::min<double>(kMaxListUF, 32.0 * std::ceil(want / 32.0)));
        }
        // Cell capacity for boxes up to 1.3x the initial length; cells are at
        // least rc + skin >= rc, so rc bounds the count for every skin.
        int64_t cap = 1;
        for (int k = 0; k < 3; ++k) {
            int n = (int)std::floor(q.box[k] * 1.3 / rc);
            n = std::max(1, std::min(n, 256));
            sd.nc_max[k] = n;
            cap *= n;
        }
        if (cells + cap + n_sys > (int64_t)1 << 30) return fail(ctx, SWFE_E_INVALID_ARG, "too many cells");
        sd.cell_base = (int32_t)cells;
        sd.cell_cap = (int32_t)cap;
        cells += cap;
        sd.k_spring = q.k_spring;
        sd.T0 = q.T0;
        sd.tau_damp = q.tau_damp;
        sd.p_damp = q.p_damp;
        sd.pressure = q.pressure / kGpa;
        sd.nf = 3.0 * (double)q.n_atoms - 3.0;
        sd.alpha = 1.0 + 3.0 / sd.nf;
        sd.wpiston = q.p_damp > 0 ? ((sd.nf + 3) * kKB) * q.T0 * (q.p_damp * q.p_damp) : 1.0;
        sd.c1 = q.tau_damp > 0 ? std::exp(-dt / q.tau_damp) : 1.0;
        sd.c2 = std::sqrt(1.0 - sd.c1 * sd.c1);
        sd.sigv = std::sqrt(kKB * q.T0 / (p->mass * kMvv2e));
        sd.acc = 1.0 / kMvv2e / p->mass;
        sd.mvv2e_m = 0.5 * p->mass * kMvv2e;
        sd.skin = skin;
        sd.stream = q.stream;
        sd.s_start = q.sched_start;
        sd.s_end = q.sched_end;
        sd.s_steps = q.sched_steps;
        desc[s] = sd;
        tiles += (q.n_atoms + 63) / 64;
        off += q.n_atoms;
    }
    if (off >= ((int64_t)1 << 31) / P.list_cap) return fail(ctx, SWFE_E_INVALID_ARG, "too many atoms");
    int ng = 0;
    for (int s = 0; s < n_sys; ++s) {
        Group g{};
        if (is_dcci(d[s].mode)) {
            if (d[s].partner < s) continue;
            g.s0 = s;
            g.s1 = d[s].partner;
        } else {
            g.s0 = s;
            g.s1 = -1;
        }
        desc[g.s0].group = ng;
        if (g.s1 >= 0) desc[g.s1].group = ng;
        groups[ng++] = g;
    }
    *n_groups = ng;
    P.n_total = off;
    P.cells = cells;
    P.max_tiles = tiles;
    Layout &L = P.lay;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const size_t n = (size_t)off, d4 = sizeof(double4);
    L.xs = take(d4 * n);
    L.vs = take(sizeof(dvec3) * n);
    L.fs = take(sizeof(dvec3) * n);
    L.x0s = take(sizeof(dvec3) * n);
    L.xb = take(sizeof(dvec3) * n);
    L.txs = take(d4 * n);
    L.tvs = take(sizeof(dvec3) * n);
    L.tfs = take(sizeof(dvec3) * n);
    L.tx0s = take(sizeof(dvec3) * n);
    L.zs = take(sizeof(dvec3) * n);
    L.xf = take(sizeof(float4) * n);
    L.fref = take(sizeof(dvec3) * n);
    L.perm = take(4 * n);
    L.tperm = take(4 * n);
    L.norder = take(4 * n);
    L.rank = take(4 * n);
    L.cellid = take(4 * n);
    L.nnb = take(4 * n);
    L.cell_count = take(4 * (size_t)cells);
    L.cell_start = take(4 * ((size_t)cells + n_sys));
    L.nl = take(4 * n * (size_t)P.list_cap);
    L.nl_cnt = take(4 * n);
    L.sl = take(4 * n * kMaxShort);
    L.mom = take(8 * 9 * n);
    L.e_s = take(8 * n);
    L.part1 = take(8 * (size_t)tiles * kNumPart);
    L.part2 = take(8 * (size_t)tiles * kNumPart);
    L.disp_max = take(8 * 2 * (size_t)n_sys);
    L.work = take(4 * (size_t)tiles);
    L.n_work = take(16);
    L.desc = take(sizeof(SysDesc) * n_sys);
    L.state = take(sizeof(SysState) * n_sys);
    L.tiles = take(sizeof(Tile) * (size_t)tiles);
    L.groups = take(sizeof(Group) * (size_t)ng);
    L.log = take(8 * (size_t)kLogCapMax * SWFE_LOG_STRIDE);
    L.strain = take(8 * 3 * (size_t)n_sys);
    L.xtiles = take(4 * (size_t)tiles);
    L.xtloc = take(4 * (size_t)tiles);
    L.xgroups = take(4 * (size_t)n_sys);
    L.xsys = take(4 * (size_t)n_sys);
    L.sync = take(8 * (size_t)kSyncWords);
    L.total = o;
    return SWFE_OK;
}

int plan_systems(swfe_ctx *ctx, const swfe_system_desc *d, int n_sys, const swfe_sw_params *p, double dt,
                 double skin, Plan &out)
{
    if (!d || !p || n_sys <= 0) return fail(ctx, SWFE_E_INVALID_ARG, "null descriptor/params or n_sys <= 0");
    Plan P;
    P.desc.resize(n_sys);
    P.groups.resize(n_sys);
    int ng = 0;
    RCHK(plan_core(ctx, d, n_sys, p, dt, skin, P.desc.data(), P.groups.data(), &ng, P));
    P.groups.resize(ng);
    out = std::move(P);
    return SWFE_OK;
}

// Tiles of `block` atoms, laid out group by group so that the tiles of a
// group (a system, or both phases of a dCCI pair) are contiguous.  Writes at
// most cap tiles into out and returns their count, or -1 when more are
// needed.  Sets the tile ranges of the descriptors and groups.
int fill_tiles(SysDesc *desc, Group *groups, int n_groups, int block, Tile *out, int cap)
{
    int nt = 0;
    for (int gi = 0; gi < n_groups; ++gi) {
        Group &g = groups[gi];
        g.tile_begin = nt;
        for (int q = 0; q < (g.s1 >= 0 ? 2 : 1); ++q) {
            const int s = q == 0 ? g.s0 : g.s1;
            SysDesc &d = desc[s];
            d.tile_begin = nt;
            for (int64_t a = 0; a < d.n; a += block) {
                if (nt >= cap) return -1;
                Tile t{};
                t.sys = s;
                t.start = (int32_t)(d.off + a);
                t.count = (int32_t)std::min<int64_t>(block, d.n - a);
                out[nt++] = t;
            }
            d.tile_end = nt;
        }
        g.tile_end = nt;
    }
    return nt;
}

void build_tiles(swfe_ctx *c)
{
    c->fx_chunk.clear();
    // tiles at the smallest block size bound the count at every size
    c->tiles.resize((size_t)c->plan.max_tiles);
    const int nt = fill_tiles(c->plan.desc.data(), c->plan.groups.data(), (int)c->plan.groups.size(), c->block,
                              c->tiles.data(), (int)c->tiles.size());
    c->tiles.resize((size_t)std::max(nt, 0));
}

// Device pointers of the workspace parts at base w.
void carve(DevPtrs &q, char *w, const Layout &L)
{
    q.xs = (double4 *)(w + L.xs);
    q.vs = (dvec3 *)(w + L.vs);
    q.fs = (dvec3 *)(w + L.fs);
    q.x0s = (dvec3 *)(w + L.x0s);
    q.xb = (dvec3 *)(w + L.xb);
    q.txs = (double4 *)(w + L.txs);
    q.tvs = (dvec3 *)(w + L.tvs);
    q.tfs = (dvec3 *)(w + L.tfs);
    q.tx0s = (dvec3 *)(w + L.tx0s);
    q.zs = (dvec3 *)(w + L.zs);
    q.xf = (float4 *)(w + L.xf);
    q.fref = (dvec3 *)(w + L.fref);
    q.perm = (int32_t *)(w + L.perm);
    q.tperm = (int32_t *)(w + L.tperm);
    q.norder = (int32_t *)(w + L.norder);
    q.rank = (int32_t *)(w + L.rank);
    q.cellid = (int32_t *)(w + L.cellid);
    q.nnb = (int32_t *)(w + L.nnb);
    q.cell_count = (int32_t *)(w + L.cell_count);
    q.cell_start = (int32_t *)(w + L.cell_start);
    q.nl = (int32_t *)(w + L.nl);
    q.nl_cnt = (int32_t *)(w + L.nl_cnt);
    q.sl = (int32_t *)(w + L.sl);
    q.mom = (void *)(w + L.mom);
    q.e_s = (double *)(w + L.e_s);
    q.part1 = (double *)(w + L.part1);
    q.part2 = (double *)(w + L.part2);
    q.disp_max = (double *)(w + L.disp_max);
    q.work = (int32_t *)(w + L.work);
    q.n_work = (int32_t *)(w + L.n_work);
    q.desc = (const SysDesc *)(w + L.desc);
    q.state = (SysState *)(w + L.state);
    q.tiles = (const Tile *)(w + L.tiles);
    q.groups = (const Group *)(w + L.groups);
    q.log = (double *)(w + L.log);
    q.xtiles = (int32_t *)(w + L.xtiles);
    q.xtloc = (int32_t *)(w + L.xtloc);
    q.xgroups = (int32_t *)(w + L.xgroups);
    q.xsys = (int32_t *)(w + L.xsys);
    q.sync = (unsigned long long *)(w + L.sync);
}

// Fresh per-system state of a set-up: boxes from the descriptors, no strain,
// unit integrator factors.
void initial_states(const swfe_system_desc *d, int n_sys, SysState *st)
{
    for (int i = 0; i < n_sys; ++i) {
        SysState &x = st[i];
        memset(&x, 0, sizeof x);
        for (int k = 0; k < 3; ++k) {
            x.box[k] = d[i].box[k];
            x.box_build[k] = d[i].box[k];
            x.pscale[k] = 1.0;
        }
        for (int k = 0; k < 3; ++k) x.decay[k] = x.phi[k] = x.grow[k] = x.psi[k] = 1.0;
    }
}

// Launch parameters of a batch; fx_chunk (8 * kFxChunks runs) may be NULL,
// which runs the tiles in order.
Ctl make_ctl_raw(const SysDesc *desc, int n_sys, int n_tiles, int n_groups, int64_t n_total, double dt,
                 uint64_t seed, int list_cap, int in_step, int flags, int force_rebuild, int log_every,
                 int log_cap, const int32_t *fx_chunk)
{
    Ctl k{};
    k.n_total = n_total;
    k.n_sys = n_sys;
    k.n_tiles = n_tiles;
    k.n_groups = n_groups;
    k.dt = dt;
    k.seed = seed;
    k.flags = flags;
    k.list_cap = list_cap;
    k.list16 = 1;
    k.has_uf = 0;
    for (int i = 0; i < n_sys; ++i) {
        k.list16 &= desc[i].n <= 65536 ? 1 : 0;
        k.has_uf |= desc[i].mode == MODE_UF ? 1 : 0;
    }
    // the fused sort keeps each system's cell table (at most cell_cap + 1
    // entries) in LDS; it is used when every system's fits and every system
    // is small
    int max_cells = 0;
    int64_t max_atoms = 0;
    for (int i = 0; i < n_sys; ++i) {
        max_cells = std::max(max_cells, desc[i].cell_cap + 1);
        max_atoms = std::max(max_atoms, desc[i].n);
    }
    k.sort_cells = max_cells <= kSortLdsCells && max_atoms <= kSortFuseMaxAtoms ? max_cells : 0;
    // otherwise the scatter stage scans the cell counts of a rebuilding
    // system in LDS when every system's table fits (one launch fewer)
    k.scan_cells = k.sort_cells == 0 && max_cells <= kSortLdsCells ? max_cells : 0;
    k.in_step = in_step;
    k.force_rebuild = force_rebuild;
    k.log_every = log_every;
    k.log_cap = log_cap;
    const int nc = 8 * kFxChunks;
    k.fx_len = std::max(1, (k.n_tiles + nc - 1) / nc);
    for (int q = 0; q < nc; ++q) k.fx_chunk[q] = fx_chunk ? fx_chunk[q] : q;
    return k;
}

Ctl make_ctl(const swfe_ctx *c, int in_step, int flags, int force_rebuild)
{
    const int nc = 8 * kFxChunks;
    const bool costed = (int)c->fx_chunk.size() == nc && c->fx_tiles == (int)c->tiles.size();
    return make_ctl_raw(c->plan.desc.data(), c->n_sys, (int)c->tiles.size(), (int)c->plan.groups.size(), c->n_total,
                        c->dt, c->seed, c->plan.list_cap, in_step, flags, force_rebuild, c->log_every, c->log_cap,
                        costed ? c->fx_chunk.data() : nullptr);
}

// Runs of tiles dealt to the XCDs by the force passes' cost: an atom costs
// kFxBase plus its neighbours within rc at the last pass 1 (the gathers of
// both passes grow with that count, their per-atom streaming does not); the
// runs go, costliest first, to the XCD with the least cost so far that has
// fewer than kFxChunks.  Only the placement of blocks changes, never a
// result.  Synchronises the stream.
constexpr int64_t kFxBase = 8;

int balance_force_tiles(swfe_ctx *c, hipStream_t s)
{
    HIPCHK(c, hipStreamSynchronize(s));
    std::vector<int32_t> nn((size_t)c->n_total);
    HIPCHK(c, hipMemcpy(nn.data(), c->ptrs.nnb, nn.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    const int nt = (int)c->tiles.size(), nc = 8 * kFxChunks;
    const int len = std::max(1, (nt + nc - 1) / nc);
    std::vector<int64_t> cost(nc, 0);
    for (int i = 0; i < nt; ++i) {
        const Tile &t = c->tiles[i];
        for (int a = 0; a < t.count; ++a)
            cost[i / len] += kFxBase + std::min(std::max(nn[(size_t)t.start + a], 0), kMaxShort);
    }
    std::vector<int> order(nc);
    for (int q = 0; q < nc; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<int64_t> load(8, 0);
    std::vector<int> used(8, 0);
    c->fx_chunk.assign(nc, 0);
    for (int q : order) {
        int x = -1;
        for (int y = 0; y < 8; ++y)
            if (used[y] < kFxChunks && (x < 0 || load[y] < load[x])) x = y;
        c->fx_chunk[x * kFxChunks + used[x]++] = q;
        load[x] += cost[q];
    }
    c->fx_tiles = nt;
    return SWFE_OK;
}

void drop_graph(swfe_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->graph_valid = false;
    c->xplan_valid = false;
}

// The systems dealt to the 8 XCDs for the persistent step kernel: whole
// reduction groups, costliest first to the XCD with the least cost so far
// (an atom costs kFxBase plus its neighbours within rc at the last pass 1).
// Writes the per-XCD tile, group and system lists to the workspace and
// picks the grid (the same number of workgroups for every XCD, no more than
// fit at once, nor more than the largest tile list).  Synchronises.
int build_xcd_plan(swfe_ctx *c, hipStream_t s)
{
    HIPCHK(c, hipStreamSynchronize(s));
    std::vector<int32_t> nn((size_t)c->n_total);
    HIPCHK(c, hipMemcpy(nn.data(), c->ptrs.nnb, nn.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    const int ng = (int)c->plan.groups.size();
    std::vector<int64_t> gcost(ng, 0);
    for (int g = 0; g < ng; ++g) {
        const Group &G = c->plan.groups[g];
        for (int q = 0; q < (G.s1 >= 0 ? 2 : 1); ++q) {
            const SysDesc &d = c->plan.desc[q == 0 ? G.s0 : G.s1];
            for (int64_t a = d.off; a < d.off + d.n; ++a)
                gcost[g] += kFxBase + std::min(std::max(nn[(size_t)a], 0), kMaxShort);
        }
    }
    std::vector<int> order(ng);
    for (int g = 0; g < ng; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return gcost[a] > gcost[b]; });
    std::vector<int64_t> load(kXcds, 0);
    std::vector<std::vector<int>> owned(kXcds);
    for (int g : order) {
        int x = 0;
        for (int y = 1; y < kXcds; ++y)
            if (load[y] < load[x]) x = y;
        owned[x].push_back(g);
        load[x] += gcost[g];
    }
    std::vector<int32_t> xtiles, xtloc, xgroups, xsys;
    XcdPlan xp{};
    int max_tiles = 1;
    for (int x = 0; x < kXcds; ++x) {
        std::sort(owned[x].begin(), owned[x].end());
        xp.tile_off[x] = (int32_t)xtiles.size();
        xp.group_off[x] = (int32_t)xgroups.size();
        xp.sys_off[x] = (int32_t)xsys.size();
        for (int g : owned[x]) {
            const Group &G = c->plan.groups[g];
            xgroups.push_back(g);
            for (int q = 0; q < (G.s1 >= 0 ? 2 : 1); ++q) {
                const int sys = q == 0 ? G.s0 : G.s1;
                const SysDesc &d = c->plan.desc[sys];
                const int local = (int)xsys.size() - xp.sys_off[x];
                xsys.push_back(sys);
                for (int t = d.tile_begin; t < d.tile_end; ++t) {
                    xtiles.push_back(t);
                    xtloc.push_back(local);
                }
            }
        }
        const int nt = (int)xtiles.size() - xp.tile_off[x], nsx = (int)xsys.size() - xp.sys_off[x];
        if (nsx > kPersistMaxSysPerXcd)
            return fail(c, SWFE_E_INVALID_ARG, "persistent step: more than 256 systems on one XCD");
        if (nt > kLdsShort * c->block - 1)
            return fail(c, SWFE_E_INVALID_ARG, "persistent step: too many tiles on one XCD for the list stage's table");
        max_tiles = std::max(max_tiles, nt);
    }
    xp.tile_off[kXcds] = (int32_t)xtiles.size();
    xp.group_off[kXcds] = (int32_t)xgroups.size();
    xp.sys_off[kXcds] = (int32_t)xsys.size();
    HIPCHK(c, hipMemcpy(c->ptrs.xtiles, xtiles.data(), 4 * xtiles.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->ptrs.xtloc, xtloc.data(), 4 * xtloc.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->ptrs.xgroups, xgroups.data(), 4 * xgroups.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->ptrs.xsys, xsys.data(), 4 * xsys.size(), hipMemcpyHostToDevice));
    int dev = 0, cus = 0;
    HIPCHK(c, hipGetDevice(&dev));
    HIPCHK(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int bpc = persist_blocks_per_cu(c->mixed, c->block);
    if (bpc <= 0 || cus < kXcds) return fail(c, SWFE_E_HIP, "persistent step: no occupancy for the step kernel");
    const int per_xcd = std::max(1, std::min(bpc * (cus / kXcds), max_tiles));
    c->persist_grid = kXcds * per_xcd;
    c->xplan = xp;
    c->xplan_valid = true;
    return SWFE_OK;
}

int upload_tables(swfe_ctx *c, hipStream_t s)
{
    HIPCHK(c, hipMemcpyAsync((void *)c->ptrs.desc, c->plan.desc.data(), sizeof(SysDesc) * c->n_sys,
                             hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync((void *)c->ptrs.tiles, c->tiles.data(), sizeof(Tile) * c->tiles.size(),
                             hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync((void *)c->ptrs.groups, c->plan.groups.data(),
                             sizeof(Group) * c->plan.groups.size(), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return SWFE_OK;
}

int enqueue_rebuild(swfe_ctx *c, const DevPtrs &p, const Ctl &k, hipStream_t s)
{
    for (int stage = 0; stage < kRebuildStages; ++stage)
        HIPCHK(c, launch_rebuild(k, p, c->sw, c->block, stage, s));
    return SWFE_OK;
}

// Caller positions -> forced list rebuild -> interaction -> caller arrays
// (scatter_what: bits of k_scatter), for launch parameters k (a forced
// rebuild outside a step).
hipError_t enqueue_forces_raw(const Ctl &k, const DevPtrs &p, const SwParams &sw, int mixed, int block,
                              int scatter_what, hipStream_t s)
{
    hipError_t e = launch_gather(k, p, block, 0, s);
    for (int stage = 0; stage < kRebuildStages && e == hipSuccess; ++stage)
        e = launch_rebuild(k, p, sw, block, stage, s);
    if (e == hipSuccess) e = launch_pass1(k, p, sw, mixed, block, s);
    if (e == hipSuccess) e = launch_pass2(k, p, sw, mixed, block, s);
    if (e == hipSuccess) e = launch_finalize(k, p, sw, s);
    if (e == hipSuccess) e = launch_scatter(k, p, block, scatter_what, s);
    return e;
}

int enqueue_forces(swfe_ctx *c, const DevPtrs &p, int flags, int scatter_what, hipStream_t s)
{
    Ctl k = make_ctl(c, 0, flags, 1);
    HIPCHK(c, enqueue_forces_raw(k, p, c->sw, c->mixed, c->block, scatter_what, s));
    return SWFE_OK;
}

int enqueue_step(swfe_ctx *c, hipStream_t s)
{
    Ctl k = make_ctl(c, 1, 0, 0);
    HIPCHK(c, launch_integrate(k, c->ptrs, c->sw, c->block, s));
    RCHK(enqueue_rebuild(c, c->ptrs, k, s));
    HIPCHK(c, launch_pass1(k, c->ptrs, c->sw, c->mixed, c->block, s));
    HIPCHK(c, launch_pass2(k, c->ptrs, c->sw, c->mixed, c->block, s));
    HIPCHK(c, launch_finalize(k, c->ptrs, c->sw, s));
    return SWFE_OK;
}

int read_states(swfe_ctx *c, std::vector<SysState> &st, hipStream_t s)
{
    st.resize(c->n_sys);
    HIPCHK(c, hipStreamSynchronize(s));
    HIPCHK(c, hipMemcpy(st.data(), c->ptrs.state, sizeof(SysState) * c->n_sys, hipMemcpyDeviceToHost));
    return SWFE_OK;
}

// Status code and message of the first system with device error bits (c
// may be NULL); SWFE_OK when none is set.
int device_error_status(swfe_ctx *c, const SysState *st, int n_sys)
{
    int bits = 0, who = -1;
    for (int i = 0; i < n_sys; ++i)
        if (st[i].err && who < 0) {
            bits = st[i].err;
            who = i;
        }
    if (!bits) return SWFE_OK;
    char msg[200];
    const char *what = (bits & ERR_PERSIST) ? "persistent step kernel gave up a wait (a barrier timed out or an XCD "
                                              "owning systems had no workgroup); the call's results are invalid"
                       : (bits & ERR_NONFINITE) ? "non-finite value"
                       : (bits & ERR_OVERFLOW) ? "neighbour list overflow (list or short-list capacity exceeded)"
                       : (bits & ERR_BOX) ? "box length fell below twice the cutoff"
                                          : "dCCI update singular (|dv| or denominator too small, or lambda out of (0.05, 20))";
    snprintf(msg, sizeof msg, "system %d: %s", who, what);
    int code = (bits & ERR_PERSIST) ? SWFE_E_HIP
               : (bits & ERR_NONFINITE) ? SWFE_E_NONFINITE
               : (bits & ERR_OVERFLOW) ? SWFE_E_OVERFLOW
               : (bits & ERR_BOX) ? SWFE_E_BOX_TOO_SMALL
                                  : SWFE_E_DCCI_SINGULAR;
    return fail(c, code, msg);
}

// First pending device error as a status code; clears the device bits.
int take_device_error(swfe_ctx *c, const std::vector<SysState> &st, hipStream_t s)
{
    bool any = false;
    for (int i = 0; i < c->n_sys; ++i) any = any || st[i].err != 0;
    if (!any) return SWFE_OK;
    Ctl k = make_ctl(c, 0, 0, 0);
    HIPCHK(c, launch_clear_err(k, c->ptrs, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return device_error_status(c, st.data(), c->n_sys);
}

}  // namespace

extern "C" {

int swfe_create(swfe_ctx **out)
{
    if (!out) return SWFE_E_INVALID_ARG;
    *out = new swfe_ctx();
    return SWFE_OK;
}

void swfe_destroy(swfe_ctx *ctx)
{
    if (!ctx) return;
    drop_graph(ctx);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
}

const char *swfe_last_error(const swfe_ctx *ctx)
{
    if (ctx) return ctx->err.c_str();
    return g_free_err[0] ? g_free_err : "null context";
}

int swfe_workspace_bytes(const swfe_system_desc *d, int32_t n_sys, const swfe_sw_params *p, size_t *bytes)
{
    if (!bytes) return SWFE_E_INVALID_ARG;
    Plan P;
    RCHK(plan_systems(nullptr, d, n_sys, p, 0.001, kDefaultSkin, P));
    *bytes = P.lay.total;
    return SWFE_OK;
}

int swfe_sizes(const swfe_ctx *ctx, int64_t *n_total, int32_t *n_sys)
{
    if (!ctx || !ctx->ready) return SWFE_E_STATE;
    if (n_total) *n_total = ctx->n_total;
    if (n_sys) *n_sys = ctx->n_sys;
    return SWFE_OK;
}

int swfe_init_system(swfe_ctx *ctx, const swfe_system_desc *d, int32_t n_sys, const swfe_sw_params *p,
                     const swfe_buffers *b, uint64_t seed, double dt, int32_t precision, void *stream)
{
    if (!ctx) return SWFE_E_INVALID_ARG;
    ctx->ready = false;
    drop_graph(ctx);
    if (!b || !b->x || !b->v || !b->f || !b->workspace)
        return fail(ctx, SWFE_E_INVALID_ARG, "buffers x, v, f and workspace are required");
    if (precision != SWFE_PREC_FP64 && precision != SWFE_PREC_MIXED)
        return fail(ctx, SWFE_E_INVALID_ARG, "precision must be SWFE_PREC_FP64 or SWFE_PREC_MIXED");
    Plan P;
    RCHK(plan_systems(ctx, d, n_sys, p, dt, ctx->skin, P));
    for (int s = 0; s < n_sys; ++s)
        if (d[s].mode == SWFE_MODE_FL && !b->x0)
            return fail(ctx, SWFE_E_INVALID_ARG, "Frenkel-Ladd systems need Einstein anchors x0");
    if (b->workspace_bytes < P.lay.total) {
        char msg[128];
        snprintf(msg, sizeof msg, "workspace too small: %zu < %zu bytes", b->workspace_bytes, P.lay.total);
        return fail(ctx, SWFE_E_NOMEM, msg);
    }
    hipStream_t s = (hipStream_t)stream;
    ctx->plan = std::move(P);
    ctx->n_sys = n_sys;
    ctx->n_total = ctx->plan.n_total;
    ctx->hdesc.assign(d, d + n_sys);
    ctx->hsw = *p;
    ctx->sw = make_sw(*p);
    ctx->mixed = precision == SWFE_PREC_MIXED;
    ctx->dt = dt;
    ctx->seed = seed;
    ctx->buf = *b;
    ctx->forces_stale = false;
    if (ctx->block != 64 && ctx->block != 128 && ctx->block != 256) ctx->block = 256;
    build_tiles(ctx);

    DevPtrs &q = ctx->ptrs;
    q = DevPtrs{};
    q.x = b->x;
    q.v = b->v;
    q.f = b->f;
    q.x0 = b->x0;
    q.e_atom = b->e_atom;
    carve(q, (char *)b->workspace, ctx->plan.lay);

    std::vector<SysState> st(n_sys);
    initial_states(d, n_sys, st.data());
    HIPCHK(ctx, hipMemcpyAsync(q.state, st.data(), sizeof(SysState) * n_sys, hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipMemsetAsync(q.cell_count, 0, 4 * (size_t)ctx->plan.cells, s));
    HIPCHK(ctx, hipMemsetAsync(q.disp_max, 0, 8 * 2 * (size_t)n_sys, s));
    RCHK(upload_tables(ctx, s));
    Ctl k = make_ctl(ctx, 0, 0, 1);
    HIPCHK(ctx, launch_iota(k, q, ctx->block, s));
    HIPCHK(ctx, launch_reset_schedule(k, q, s));
    RCHK(enqueue_forces(ctx, q, 0, 2 | 4, s));
    std::vector<SysState> now;
    RCHK(read_states(ctx, now, s));
    RCHK(take_device_error(ctx, now, s));
    RCHK(balance_force_tiles(ctx, s));
    ctx->ready = true;
    return SWFE_OK;
}

int swfe_build_neighbors(swfe_ctx *ctx, void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    hipStream_t s = (hipStream_t)stream;
    Ctl k = make_ctl(ctx, 0, 0, 1);
    HIPCHK(ctx, launch_gather(k, ctx->ptrs, ctx->block, 1, s));
    RCHK(enqueue_rebuild(ctx, ctx->ptrs, k, s));
    // the stored normals of the next O step follow the new atom order
    HIPCHK(ctx, launch_fill_noise(k, ctx->ptrs, ctx->block, s));
    HIPCHK(ctx, launch_scatter(k, ctx->ptrs, ctx->block, 1 | 2, s));
    return SWFE_OK;
}

int swfe_compute_forces(swfe_ctx *ctx, uint32_t flags, const double *strain, const double *grad_scale,
                        double *grad_x, double *out, void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    if (flags & ~(SWFE_PARAM_GRAD | SWFE_STRAIN)) return fail(ctx, SWFE_E_INVALID_ARG, "unknown flags");
    hipStream_t s = (hipStream_t)stream;
    DevPtrs p = ctx->ptrs;
    p.grad_scale = grad_scale;
    p.grad_x = grad_x;
    p.out = out;
    Ctl k = make_ctl(ctx, 0, (int)flags, 1);
    double *diag = (double *)((char *)ctx->buf.workspace + ctx->plan.lay.strain);
    if (flags & SWFE_STRAIN) {
        if (!strain) return fail(ctx, SWFE_E_INVALID_ARG, "SWFE_STRAIN needs a strain array");
        std::vector<double> dg(3 * ctx->n_sys);
        for (int i = 0; i < ctx->n_sys; ++i) {
            for (int a = 0; a < 3; ++a)
                for (int b2 = 0; b2 < 3; ++b2)
                    if (a != b2 && strain[9 * i + 3 * a + b2] != 0.0)
                        return fail(ctx, SWFE_E_INVALID_ARG, "only diagonal strains keep the box orthorhombic");
            for (int a = 0; a < 3; ++a) {
                dg[3 * i + a] = strain[9 * i + 4 * a];
                if (!(1.0 + dg[3 * i + a] > 0.5)) return fail(ctx, SWFE_E_INVALID_ARG, "strain too large");
            }
        }
        HIPCHK(ctx, hipStreamSynchronize(s));
        HIPCHK(ctx, hipMemcpy(diag, dg.data(), sizeof(double) * dg.size(), hipMemcpyHostToDevice));
        HIPCHK(ctx, launch_set_pscale(k, p, diag, s));
    }
    RCHK(enqueue_forces(ctx, p, (int)flags, 2 | 4 | 8, s));
    if (flags & SWFE_STRAIN) HIPCHK(ctx, launch_set_pscale(k, p, nullptr, s));
    ctx->forces_stale = (flags & SWFE_STRAIN) != 0;
    return SWFE_OK;
}

namespace {
// Dynamics start from forces, energies and virial of the unstrained
// positions: after a strained evaluation the interaction is evaluated again
// (f of the caller is overwritten with the unstrained forces).
int refresh_forces(swfe_ctx *ctx, hipStream_t s)
{
    if (!ctx->forces_stale) return SWFE_OK;
    RCHK(enqueue_forces(ctx, ctx->ptrs, 0, 2, s));
    ctx->forces_stale = false;
    return SWFE_OK;
}
}  // namespace

int swfe_set_params(swfe_ctx *ctx, const swfe_sw_params *p)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    if (!p) return fail(ctx, SWFE_E_INVALID_ARG, "null parameters");
    Plan P;
    RCHK(plan_systems(ctx, ctx->hdesc.data(), ctx->n_sys, p, ctx->dt, ctx->skin, P));
    ctx->hsw = *p;
    ctx->sw = make_sw(*p);
    drop_graph(ctx);
    return SWFE_OK;
}

int swfe_set_schedule(swfe_ctx *ctx, const swfe_system_desc *d, void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    hipStream_t s = (hipStream_t)stream;
    if (d) {
        for (int i = 0; i < ctx->n_sys; ++i) {
            ctx->hdesc[i].sched_start = d[i].sched_start;
            ctx->hdesc[i].sched_end = d[i].sched_end;
            ctx->hdesc[i].sched_steps = d[i].sched_steps;
        }
        Plan P;
        RCHK(plan_systems(ctx, ctx->hdesc.data(), ctx->n_sys, &ctx->hsw, ctx->dt, ctx->skin, P));
        for (int i = 0; i < ctx->n_sys; ++i) {
            ctx->plan.desc[i].s_start = d[i].sched_start;
            ctx->plan.desc[i].s_end = d[i].sched_end;
            ctx->plan.desc[i].s_steps = d[i].sched_steps;
        }
        RCHK(upload_tables(ctx, s));
    }
    Ctl k = make_ctl(ctx, 0, 0, 0);
    HIPCHK(ctx, launch_reset_schedule(k, ctx->ptrs, s));
    return SWFE_OK;
}

int swfe_step_switched(swfe_ctx *ctx, int64_t n_steps, int32_t use_graph, void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    if (n_steps < 0) return fail(ctx, SWFE_E_INVALID_ARG, "n_steps < 0");
    if (n_steps == 0) return SWFE_OK;
    if (use_graph < 0 || use_graph > 2) return fail(ctx, SWFE_E_INVALID_ARG, "use_graph must be 0, 1 or 2");
    hipStream_t s = (hipStream_t)stream;
    RCHK(refresh_forces(ctx, s));
    if (use_graph == 2 && !ctx->xplan_valid) RCHK(build_xcd_plan(ctx, s));
    Ctl k = make_ctl(ctx, 1, 0, 0);
    HIPCHK(ctx, launch_gather(k, ctx->ptrs, ctx->block, 1, s));
    HIPCHK(ctx, launch_begin_step(k, ctx->ptrs, ctx->sw, n_steps, s));
    if (use_graph == 2) {
        // launches of at most kPersistChunk steps, each from a cleared barrier area
        for (int64_t done = 0; done < n_steps; done += kPersistChunk) {
            const int64_t m = std::min<int64_t>(kPersistChunk, n_steps - done);
            HIPCHK(ctx, launch_zero_words(ctx->ptrs.sync, 8 * (size_t)kSyncWords, s));
            HIPCHK(ctx, launch_persist(k, ctx->ptrs, ctx->sw, ctx->xplan, ctx->mixed, ctx->block,
                                       ctx->persist_grid, m, s));
        }
    } else if (!use_graph) {
        for (int64_t i = 0; i < n_steps; ++i) RCHK(enqueue_step(ctx, s));
    } else {
        if (!ctx->graph_valid) {
            // Capture one step on a library-owned stream (the caller's stream
            // may be the legacy default stream, which cannot be captured); the
            // graph is then launched on the caller's stream.
            drop_graph(ctx);
            if (!ctx->cap_stream) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
            RCHK(balance_force_tiles(ctx, s));
            HIPCHK(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
            int rc = enqueue_step(ctx, ctx->cap_stream);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            HIPCHK(ctx, e);
            ctx->graph = g;
            HIPCHK(ctx, hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0));
            ctx->graph_valid = true;
        }
        for (int64_t i = 0; i < n_steps; ++i) HIPCHK(ctx, hipGraphLaunch(ctx->gexec, s));
    }
    HIPCHK(ctx, launch_scatter(k, ctx->ptrs, ctx->block, 1 | 2, s));
    return SWFE_OK;
}

int swfe_get_state(swfe_ctx *ctx, swfe_system_state *out, void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    if (!out) return fail(ctx, SWFE_E_INVALID_ARG, "null output");
    hipStream_t s = (hipStream_t)stream;
    std::vector<SysState> st;
    RCHK(read_states(ctx, st, s));
    for (int i = 0; i < ctx->n_sys; ++i) {
        swfe_system_state &o = out[i];
        const SysState &x = st[i];
        const SysDesc &d = ctx->plan.desc[i];
        o.lam = x.lam;
        o.Ps = x.Ps * kGpa;
        o.W = x.W;
        o.U_int = x.U_int;
        o.U_ref = x.U_ref;
        o.K = x.K;
        o.V = x.box[0] * x.box[1] * x.box[2];
        for (int k = 0; k < 9; ++k) o.virial[k] = x.vir[k];
        for (int k = 0; k < 3; ++k) o.box[k] = x.box[k];
        o.veps = (x.veps[0] + x.veps[1] + x.veps[2]) / 3.0;
        for (int k = 0; k < 3; ++k) o.veps_axes[k] = x.veps[k];
        o.T_inst = 2.0 * x.K / (d.nf * kKB);
        o.step = x.step;
        o.sched_k = x.k;
        o.err = x.err;
        o.pad = 0;
        o.n_rebuild = x.n_rebuild;
    }
    return take_device_error(ctx, st, s);
}

int swfe_work_integral(swfe_ctx *ctx, double *W, double *lam, double *Ps, int64_t *steps, void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    hipStream_t s = (hipStream_t)stream;
    std::vector<SysState> st;
    RCHK(read_states(ctx, st, s));
    for (int i = 0; i < ctx->n_sys; ++i) {
        if (W) W[i] = st[i].W;
        if (lam) lam[i] = st[i].lam;
        if (Ps) Ps[i] = st[i].Ps * kGpa;
        if (steps) steps[i] = st[i].k;
    }
    return take_device_error(ctx, st, s);
}

int swfe_set_log(swfe_ctx *ctx, int32_t log_every, int32_t capacity)
{
    if (!ctx) return SWFE_E_INVALID_ARG;
    if (log_every < 0 || capacity < 0 || capacity > kLogCapMax)
        return fail(ctx, SWFE_E_INVALID_ARG, "log_every >= 0 and 0 <= capacity <= 16384 required");
    ctx->log_every = log_every;
    ctx->log_cap = capacity;
    drop_graph(ctx);
    return SWFE_OK;
}

int swfe_read_log(swfe_ctx *ctx, double *rows, int32_t max_rows, int32_t *n_rows, void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    if (!n_rows || (max_rows > 0 && !rows)) return fail(ctx, SWFE_E_INVALID_ARG, "null output");
    *n_rows = 0;
    if (ctx->log_every <= 0 || ctx->log_cap <= 0) return SWFE_OK;
    hipStream_t s = (hipStream_t)stream;
    std::vector<SysState> st;
    RCHK(read_states(ctx, st, s));
    std::vector<double> ring((size_t)ctx->log_cap * SWFE_LOG_STRIDE);
    HIPCHK(ctx, hipMemcpy(ring.data(), ctx->ptrs.log, ring.size() * sizeof(double), hipMemcpyDeviceToHost));
    const int64_t events = st[0].step / ctx->log_every;
    const int64_t keep = std::min<int64_t>(events, ctx->log_cap / ctx->n_sys);
    int32_t n = 0;
    for (int64_t e = events - keep + 1; e <= events; ++e)
        for (int i = 0; i < ctx->n_sys && n < max_rows; ++i) {
            const int64_t row = (e * ctx->n_sys + i) % ctx->log_cap;
            memcpy(rows + (size_t)n * SWFE_LOG_STRIDE, ring.data() + row * SWFE_LOG_STRIDE,
                   SWFE_LOG_STRIDE * sizeof(double));
            ++n;
        }
    *n_rows = n;
    return SWFE_OK;
}

int swfe_set_block(swfe_ctx *ctx, int32_t block, void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    if (block == 0) {
        int32_t chosen;
        return swfe_autotune(ctx, &chosen, stream);
    }
    if (block != 64 && block != 128 && block != 256)
        return fail(ctx, SWFE_E_INVALID_ARG, "block must be 64, 128 or 256");
    hipStream_t s = (hipStream_t)stream;
    ctx->block = block;
    drop_graph(ctx);
    build_tiles(ctx);
    RCHK(upload_tables(ctx, s));
    RCHK(enqueue_forces(ctx, ctx->ptrs, 0, 2, s));
    return balance_force_tiles(ctx, s);
}

int swfe_set_skin(swfe_ctx *ctx, double skin, void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    if (!(skin >= 0.0 && skin < 5.0)) return fail(ctx, SWFE_E_INVALID_ARG, "skin must be in [0, 5) A");
    if (skin > ctx->plan.list_skin) {
        char msg[160];
        snprintf(msg, sizeof msg, "skin %g A beyond the %g A the neighbour lists were sized for at set-up", skin,
                 ctx->plan.list_skin);
        return fail(ctx, SWFE_E_INVALID_ARG, msg);
    }
    hipStream_t s = (hipStream_t)stream;
    ctx->skin = skin;
    for (auto &d : ctx->plan.desc) d.skin = skin;
    RCHK(upload_tables(ctx, s));
    return enqueue_forces(ctx, ctx->ptrs, 0, 2, s);
}

int swfe_autotune(swfe_ctx *ctx, int32_t *chosen_block, void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    hipStream_t s = (hipStream_t)stream;
    // Every candidate runs graph-replayed dynamics steps from the current
    // state, as a run does (the block size changes the cost of every per-atom
    // kernel, not only of the force passes), and a host snapshot of the state
    // is restored after each, so the call leaves the dynamics where they were.
    size_t bytes = 0;
    RCHK(swfe_checkpoint_bytes(ctx, &bytes));
    std::vector<char> snap(bytes);
    RCHK(swfe_save_state(ctx, snap.data(), bytes, stream));
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    constexpr int kSteps = 24;
    const int cand[3] = {64, 128, 256};
    float best_ms[3] = {1e30f, 1e30f, 1e30f};
    auto trial = [&](int q) -> int {
        RCHK(swfe_set_block(ctx, cand[q], stream));
        RCHK(swfe_step_switched(ctx, 3, 1, stream));  // capture and warm the step graph
        HIPCHK(ctx, hipEventRecord(e0, s));
        RCHK(swfe_step_switched(ctx, kSteps, 1, stream));
        HIPCHK(ctx, hipEventRecord(e1, s));
        HIPCHK(ctx, hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
        best_ms[q] = std::min(best_ms[q], ms);
        return swfe_load_state(ctx, snap.data(), bytes, stream);
    };
    // three interleaved rounds, the fastest of each candidate's counting
    int rc = SWFE_OK;
    for (int round = 0; round < 3 && rc == SWFE_OK; ++round)
        for (int q = 0; q < 3 && rc == SWFE_OK; ++q) rc = trial(q);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    int best_b = cand[0];
    float fastest = best_ms[0];
    for (int q = 1; q < 3; ++q)
        if (best_ms[q] < fastest) {
            fastest = best_ms[q];
            best_b = cand[q];
        }
    if (chosen_block) *chosen_block = best_b;
    return swfe_set_block(ctx, best_b, stream);
}

int swfe_autotune_skin(swfe_ctx *ctx, const double *candidates, int32_t n_candidates, int32_t n_steps,
                       double *chosen, void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    static const double kDefaultSkins[] = {0.6, 1.0, 1.4, 1.8, 2.0};
    if (!candidates) {
        candidates = kDefaultSkins;
        n_candidates = (int32_t)(sizeof kDefaultSkins / sizeof kDefaultSkins[0]);
    }
    if (n_candidates <= 0 || n_candidates > 16) return fail(ctx, SWFE_E_INVALID_ARG, "1 to 16 skin candidates");
    for (int q = 0; q < n_candidates; ++q)
        if (!(candidates[q] >= 0.0 && candidates[q] < 5.0 && candidates[q] <= ctx->plan.list_skin))
            return fail(ctx, SWFE_E_INVALID_ARG, "skin candidates must be in [0, 5) A and within the planned skin");
    if (n_steps <= 0) n_steps = 40;
    hipStream_t s = (hipStream_t)stream;
    // every candidate steps the same state: a host snapshot is restored
    // after each trial, so the call leaves the dynamics where they were
    size_t bytes = 0;
    RCHK(swfe_checkpoint_bytes(ctx, &bytes));
    std::vector<char> snap(bytes);
    RCHK(swfe_save_state(ctx, snap.data(), bytes, stream));
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    std::vector<float> best(n_candidates, 1e30f);
    auto trial = [&](int q) -> int {
        RCHK(swfe_set_skin(ctx, candidates[q], stream));
        RCHK(swfe_step_switched(ctx, 5, 1, stream));  // capture and warm the step graph
        HIPCHK(ctx, hipEventRecord(e0, s));
        RCHK(swfe_step_switched(ctx, n_steps, 1, stream));
        HIPCHK(ctx, hipEventRecord(e1, s));
        HIPCHK(ctx, hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
        best[q] = std::min(best[q], ms);
        return swfe_load_state(ctx, snap.data(), bytes, stream);
    };
    int rc = SWFE_OK;
    for (int round = 0; round < 2 && rc == SWFE_OK; ++round)
        for (int q = 0; q < n_candidates && rc == SWFE_OK; ++q) rc = trial(q);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    int qb = 0;
    for (int q = 1; q < n_candidates; ++q)
        if (best[q] < best[qb]) qb = q;
    if (chosen) *chosen = candidates[qb];
    return swfe_set_skin(ctx, candidates[qb], stream);
}

int swfe_profile_steps(swfe_ctx *ctx, int64_t n_steps, double *ms, void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    if (!ms || n_steps <= 0) return fail(ctx, SWFE_E_INVALID_ARG, "ms output and n_steps > 0 required");
    hipStream_t s = (hipStream_t)stream;
    RCHK(refresh_forces(ctx, s));
    const int nk = SWFE_NUM_KERNELS;
    std::vector<hipEvent_t> ev((size_t)(nk + 1) * n_steps);
    for (auto &e : ev) HIPCHK(ctx, hipEventCreate(&e));
    Ctl k = make_ctl(ctx, 1, 0, 0);
    HIPCHK(ctx, launch_gather(k, ctx->ptrs, ctx->block, 1, s));
    HIPCHK(ctx, launch_begin_step(k, ctx->ptrs, ctx->sw, n_steps, s));
    for (int64_t i = 0; i < n_steps; ++i) {
        hipEvent_t *e = &ev[(size_t)i * (nk + 1)];
        HIPCHK(ctx, hipEventRecord(e[0], s));
        HIPCHK(ctx, launch_integrate(k, ctx->ptrs, ctx->sw, ctx->block, s));
        HIPCHK(ctx, hipEventRecord(e[1], s));
        for (int stage = 0; stage < kRebuildStages; ++stage) {
            HIPCHK(ctx, launch_rebuild(k, ctx->ptrs, ctx->sw, ctx->block, stage, s));
            HIPCHK(ctx, hipEventRecord(e[2 + stage], s));
        }
        HIPCHK(ctx, launch_pass1(k, ctx->ptrs, ctx->sw, ctx->mixed, ctx->block, s));
        HIPCHK(ctx, hipEventRecord(e[2 + kRebuildStages], s));
        HIPCHK(ctx, launch_pass2(k, ctx->ptrs, ctx->sw, ctx->mixed, ctx->block, s));
        HIPCHK(ctx, hipEventRecord(e[3 + kRebuildStages], s));
        HIPCHK(ctx, launch_finalize(k, ctx->ptrs, ctx->sw, s));
        HIPCHK(ctx, hipEventRecord(e[4 + kRebuildStages], s));
    }
    HIPCHK(ctx, launch_scatter(k, ctx->ptrs, ctx->block, 1 | 2, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    for (int q = 0; q < nk; ++q) ms[q] = 0.0;
    for (int64_t i = 0; i < n_steps; ++i)
        for (int q = 0; q < nk; ++q) {
            float t = 0.f;
            HIPCHK(ctx, hipEventElapsedTime(&t, ev[(size_t)i * (nk + 1) + q], ev[(size_t)i * (nk + 1) + q + 1]));
            ms[q] += t;
        }
    for (auto &e : ev) (void)hipEventDestroy(e);
    return SWFE_OK;
}

int swfe_neighbor_stats(swfe_ctx *ctx, int64_t *total_pairs, int32_t *max_per_atom, int64_t *list_entries,
                        void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(ctx, hipStreamSynchronize(s));
    std::vector<int32_t> nn((size_t)ctx->n_total), nl((size_t)ctx->n_total);
    HIPCHK(ctx, hipMemcpy(nn.data(), ctx->ptrs.nnb, nn.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(ctx, hipMemcpy(nl.data(), ctx->ptrs.nl_cnt, nl.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    int64_t tot = 0, ltot = 0;
    int32_t mx = 0;
    for (size_t i = 0; i < nn.size(); ++i) {
        tot += nn[i];
        ltot += nl[i];
        mx = std::max(mx, nn[i]);
    }
    if (total_pairs) *total_pairs = tot;
    if (max_per_atom) *max_per_atom = mx;
    if (list_entries) *list_entries = ltot;
    return SWFE_OK;
}

}  // extern "C"

// ---- force evaluation without allocation ------------------------------------
// Library scratch of swfe_forces_static: one array per GPU, held from the
// library's first use on that GPU until the process ends.  In host code the
// name `scratch` is only a stand-in for the symbol; its device address on
// each GPU comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address is handed to kernels.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kStaticMaxSys = 64;     // systems per call
constexpr int kStaticMaxTiles = 1024; // tiles of kStaticBlock atoms per call
constexpr int kStaticBlock = 256;     // block size (the contexts' default)
constexpr int kMaxDevices = 64;

std::mutex g_scratch_lock;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (taken on first use).
int scratch_address(void **out)
{
    int dev = 0;
    HIPCHK(nullptr, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, SWFE_E_INVALID_ARG, "device index beyond 63");
    std::lock_guard<std::mutex> guard(g_scratch_lock);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIPCHK(nullptr, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(nullptr, SWFE_E_HIP, "hipGetSymbolAddress gave no address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SWFE_OK;
}

}  // namespace

extern "C" int swfe_forces_static(const swfe_system_desc *d, int32_t n_sys, const swfe_sw_params *p,
                                  const double *x, double *f, double *e_atom, double *out, int32_t precision,
                                  void *stream)
{
    if (!d || !p || !x || !f) return fail(nullptr, SWFE_E_INVALID_ARG, "descriptors, parameters, x and f are required");
    if (n_sys <= 0 || n_sys > kStaticMaxSys) return fail(nullptr, SWFE_E_INVALID_ARG, "n_sys must be in [1, 64]");
    if (precision != SWFE_PREC_FP64 && precision != SWFE_PREC_MIXED)
        return fail(nullptr, SWFE_E_INVALID_ARG, "precision must be SWFE_PREC_FP64 or SWFE_PREC_MIXED");
    // every system is evaluated as a force-only system: the interaction alone
    swfe_system_desc dd[kStaticMaxSys];
    for (int i = 0; i < n_sys; ++i) {
        memset(&dd[i], 0, sizeof dd[i]);
        dd[i].n_atoms = d[i].n_atoms;
        dd[i].offset = d[i].offset;
        for (int k = 0; k < 3; ++k) dd[i].box[k] = d[i].box[k];
        dd[i].mode = SWFE_MODE_FORCE;
        dd[i].partner = -1;
        dd[i].baro = SWFE_BARO_ISO;
    }
    SysDesc desc[kStaticMaxSys];
    Group groups[kStaticMaxSys];
    int n_groups = 0;
    Plan P;  // scalars and layout only; its tables stay empty
    RCHK(plan_core(nullptr, dd, n_sys, p, 0.001, kDefaultSkin, desc, groups, &n_groups, P));
    if (P.lay.total > kStaticScratchBytes) {
        char msg[200];
        snprintf(msg, sizeof msg, "%lld atoms need %zu bytes of scratch; the static scratch holds %zu (about %lld atoms)",
                 (long long)P.n_total, P.lay.total, kStaticScratchBytes,
                 (long long)(kStaticScratchBytes / std::max<size_t>(1, P.lay.total / std::max<int64_t>(1, P.n_total))));
        return fail(nullptr, SWFE_E_NOMEM, msg);
    }
    Tile tiles[kStaticMaxTiles];
    const int nt = fill_tiles(desc, groups, n_groups, kStaticBlock, tiles, kStaticMaxTiles);
    if (nt < 0) return fail(nullptr, SWFE_E_NOMEM, "more tiles than the static tables hold");
    void *base = nullptr;
    RCHK(scratch_address(&base));
    hipStream_t s = (hipStream_t)stream;
    DevPtrs q{};
    q.x = const_cast<double *>(x);
    q.f = f;
    q.e_atom = e_atom;
    q.out = out;
    carve(q, (char *)base, P.lay);
    SysState st[kStaticMaxSys];
    initial_states(dd, n_sys, st);
    const SwParams sw = make_sw(*p);
    // the host tables are read by the copies before the stream is synchronised below
    HIPCHK(nullptr, hipMemcpyAsync(q.state, st, sizeof(SysState) * n_sys, hipMemcpyHostToDevice, s));
    HIPCHK(nullptr, hipMemcpyAsync((void *)q.desc, desc, sizeof(SysDesc) * n_sys, hipMemcpyHostToDevice, s));
    HIPCHK(nullptr, hipMemcpyAsync((void *)q.tiles, tiles, sizeof(Tile) * nt, hipMemcpyHostToDevice, s));
    HIPCHK(nullptr, hipMemcpyAsync((void *)q.groups, groups, sizeof(Group) * n_groups, hipMemcpyHostToDevice, s));
    // the array keeps the last call's contents: the counters start at zero
    HIPCHK(nullptr, launch_zero_words(q.cell_count, 4 * (size_t)P.cells, s));
    HIPCHK(nullptr, launch_zero_words(q.disp_max, 8 * 2 * (size_t)n_sys, s));
    const Ctl k = make_ctl_raw(desc, n_sys, nt, n_groups, P.n_total, 0.001, 0, P.list_cap, 0, 0, 1, 0, 0, nullptr);
    HIPCHK(nullptr, launch_iota(k, q, kStaticBlock, s));
    HIPCHK(nullptr, launch_reset_schedule(k, q, s));
    HIPCHK(nullptr, enqueue_forces_raw(k, q, sw, precision == SWFE_PREC_MIXED, kStaticBlock, 2 | 4, s));
    HIPCHK(nullptr, hipMemcpyAsync(st, q.state, sizeof(SysState) * n_sys, hipMemcpyDeviceToHost, s));
    HIPCHK(nullptr, hipStreamSynchronize(s));
    return device_error_status(nullptr, st, n_sys);
}

// ---- checkpoint / resume ----------------------------------------------------
namespace {

struct CkptHeader {
    char magic[8];
    int32_t version, n_sys;
    int64_t n_total;
    uint64_t ws_bytes;
    int32_t block, mixed;
    double skin, dt;
    uint64_t seed;
    int32_t log_every, log_cap;
    swfe_sw_params sw;
};

constexpr char kCkptMagic[8] = {'S', 'W', 'F', 'E', 'C', 'K', 'P', 'T'};

size_t ckpt_bytes(const swfe_ctx *c)
{
    return sizeof(CkptHeader) + sizeof(swfe_system_desc) * (size_t)c->n_sys + c->plan.lay.total +
           3 * sizeof(double) * 3 * (size_t)c->n_total;
}

}  // namespace

int swfe_checkpoint_bytes(const swfe_ctx *ctx, size_t *bytes)
{
    if (!ctx || !ctx->ready) return SWFE_E_STATE;
    if (!bytes) return SWFE_E_INVALID_ARG;
    *bytes = ckpt_bytes(ctx);
    return SWFE_OK;
}

int swfe_save_state(swfe_ctx *ctx, void *host, size_t bytes, void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    if (!host || bytes < ckpt_bytes(ctx)) return fail(ctx, SWFE_E_INVALID_ARG, "checkpoint buffer too small");
    hipStream_t s = (hipStream_t)stream;
    char *o = (char *)host;
    CkptHeader hd{};
    memcpy(hd.magic, kCkptMagic, 8);
    hd.version = 1;
    hd.n_sys = ctx->n_sys;
    hd.n_total = ctx->n_total;
    hd.ws_bytes = ctx->plan.lay.total;
    hd.block = ctx->block;
    hd.mixed = ctx->mixed;
    hd.skin = ctx->skin;
    hd.dt = ctx->dt;
    hd.seed = ctx->seed;
    hd.log_every = ctx->log_every;
    hd.log_cap = ctx->log_cap;
    hd.sw = ctx->hsw;
    memcpy(o, &hd, sizeof hd);
    o += sizeof hd;
    // descriptors with the schedules now in force
    std::vector<swfe_system_desc> dsc = ctx->hdesc;
    for (int i = 0; i < ctx->n_sys; ++i) {
        dsc[i].sched_start = ctx->plan.desc[i].s_start;
        dsc[i].sched_end = ctx->plan.desc[i].s_end;
        dsc[i].sched_steps = ctx->plan.desc[i].s_steps;
    }
    memcpy(o, dsc.data(), sizeof(swfe_system_desc) * ctx->n_sys);
    o += sizeof(swfe_system_desc) * ctx->n_sys;
    HIPCHK(ctx, hipMemcpyAsync(o, ctx->buf.workspace, ctx->plan.lay.total, hipMemcpyDeviceToHost, s));
    o += ctx->plan.lay.total;
    const size_t n3 = 3 * sizeof(double) * (size_t)ctx->n_total;
    HIPCHK(ctx, hipMemcpyAsync(o, ctx->buf.x, n3, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipMemcpyAsync(o + n3, ctx->buf.v, n3, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipMemcpyAsync(o + 2 * n3, ctx->buf.f, n3, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return SWFE_OK;
}

int swfe_load_state(swfe_ctx *ctx, const void *host, size_t bytes, void *stream)
{
    if (!ctx || !ctx->ready) return fail(ctx, SWFE_E_STATE, "context not initialised");
    if (!host || bytes < sizeof(CkptHeader)) return fail(ctx, SWFE_E_INVALID_ARG, "checkpoint too short");
    CkptHeader hd;
    memcpy(&hd, host, sizeof hd);
    if (memcmp(hd.magic, kCkptMagic, 8) != 0 || hd.version != 1)
        return fail(ctx, SWFE_E_INVALID_ARG, "not a checkpoint of this library version");
    if (hd.n_sys != ctx->n_sys || hd.n_total != ctx->n_total || bytes < ckpt_bytes(ctx))
        return fail(ctx, SWFE_E_INVALID_ARG, "checkpoint of a context with other system sizes");
    const char *in = (const char *)host + sizeof hd;
    std::vector<swfe_system_desc> dsc(ctx->n_sys);
    memcpy(dsc.data(), in, sizeof(swfe_system_desc) * ctx->n_sys);
    in += sizeof(swfe_system_desc) * ctx->n_sys;
    for (int i = 0; i < ctx->n_sys; ++i)
        if (dsc[i].n_atoms != ctx->hdesc[i].n_atoms)
            return fail(ctx, SWFE_E_INVALID_ARG, "checkpoint of a context with other system sizes");
    Plan P;
    RCHK(plan_systems(ctx, dsc.data(), ctx->n_sys, &hd.sw, hd.dt, hd.skin, P));
    if (P.lay.total != hd.ws_bytes || P.lay.total > ctx->buf.workspace_bytes)
        return fail(ctx, SWFE_E_INVALID_ARG, "checkpoint workspace layout differs from this context's");
    for (int s = 0; s < ctx->n_sys; ++s)
        if (dsc[s].mode == SWFE_MODE_FL && !ctx->buf.x0)
            return fail(ctx, SWFE_E_INVALID_ARG, "Frenkel-Ladd systems need Einstein anchors x0");
    hipStream_t s = (hipStream_t)stream;
    drop_graph(ctx);
    ctx->plan = std::move(P);
    ctx->hdesc = dsc;
    ctx->hsw = hd.sw;
    ctx->sw = make_sw(hd.sw);
    ctx->mixed = hd.mixed;
    ctx->dt = hd.dt;
    ctx->seed = hd.seed;
    ctx->skin = hd.skin;
    ctx->block = hd.block;
    ctx->log_every = hd.log_every;
    ctx->log_cap = hd.log_cap;
    build_tiles(ctx);
    // the device tables, atom data and state come back with the workspace
    HIPCHK(ctx, hipMemcpyAsync(ctx->buf.workspace, in, ctx->plan.lay.total, hipMemcpyHostToDevice, s));
    in += ctx->plan.lay.total;
    const size_t n3 = 3 * sizeof(double) * (size_t)ctx->n_total;
    HIPCHK(ctx, hipMemcpyAsync(ctx->buf.x, in, n3, hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipMemcpyAsync(ctx->buf.v, in + n3, n3, hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipMemcpyAsync(ctx->buf.f, in + 2 * n3, n3, hipMemcpyHostToDevice, s));
    // the restored neighbour counts deal the tiles to the XCDs again
    return balance_force_tiles(ctx, s);
}

