// swfe_kernels.hip -- HIP kernels for gfx950 of the switched-Hamiltonian
// Stillinger-Weber silicon step.
//
// Data layout.  Internally every atom array lives in cell-sorted order as
// double4 (x, y, z, -), one contiguous range per system; perm[t] is the
// caller's atom index at sorted position t.  Neighbour lists hold sorted
// positions, so neighbours of a tile are nearby in memory.
//
// One dynamics step is nine launches over all systems at once:
//   integrate    B kick, A drift, O Langevin, A drift; per-tile maximum
//                displacement since the last list build
//   rebuild 0-4  (only systems whose list may miss a pair do any work; the
//                decision is taken per block from the displacement bound)
//                0 count:   cell index and rank within the cell
//                1 scan:    per-system cell starts, and the tiles of the
//                           later stages' work list
//                2 scatter: atom data into its cell's segment (staging)
//                3 order:   in-cell order by the caller's atom index
//                4 list:    Verlet list within rc + skin from the 27 cells
//   pass1        filter of the Verlet list (16-bit entries relative to the
//                system when every system has at most 65536 atoms) to the
//                short list (within rc), then pair terms and the 11
//                three-body moments per atom
//   pass2        three-body force gather from own and neighbour moments,
//                Einstein springs, final B kick, per-tile partial sums, the
//                normals of the next O step (stored, and summed for its
//                zero-sum correction)
//   finalize     one block per group (a system or a dCCI pair): fixed-order
//                reduction of its tiles, the barostat, the lambda switch and
//                work increment, the dCCI coupling and the integrator
//                factors of the next step.
//
// Three-body term in moment form.  With g_j = g(r_ij), u_j = r_ij/|r_ij| and
// the moments of centre i
//     s = sum g_j, q = sum g_j^2, v = sum g_j u_j, M = sum g_j u_j u_j^T,
// the triplet sum sum_{j<k} (u_j.u_k - c0)^2 g_j g_k equals
//     Phi/2,  Phi = |M|_F^2 - 2 c0 |v|^2 + c0^2 s^2 - (1 - c0)^2 q,
// so E3_i = (lambda_sw eps / 2) Phi_i, and dE3_i/dr_ij depends only on r_ij
// and centre i's moments: the three-body force becomes an O(n) gather.
// No floating-point atomics are used: every sum has a fixed order, so runs
// are bitwise reproducible.
#include "swfe_internal.h"

#include <math.h>

#include <algorithm>

namespace swfe {

// ------------------------------------------------------------------ utils --
// Blocks are dispatched round robin over the 8 XCDs, block b to XCD b % 8.
// The tiles are cut into 8 * kFxChunks runs of fx_len consecutive tiles
// (neighbouring cells of a system) and XCD x works on the runs
// fx_chunk[x * kFxChunks + j], so each XCD keeps its runs' data in its own
// L2 and holds the same number of blocks.  The host deals the runs to the
// XCDs by cost, because the force passes' work per atom grows with its
// neighbour count.  -1: no tile.
__device__ __forceinline__ int tile_of_block(const Ctl &c)
{
    const int b = blockIdx.x, x = b & 7, i = b >> 3;
    const int j = i / c.fx_len;
    if (j >= kFxChunks) return -1;
    const int t = c.fx_chunk[x * kFxChunks + j] * c.fx_len + (i - j * c.fx_len);
    return t < c.n_tiles ? t : -1;
}

// General power, kept out of line: it is only reached for non-integer
// exponents (parameter derivatives by finite differences).
template <typename R>
__device__ __noinline__ R pow_general(R s, R p)
{
    return pow(s, p);
}

// s^p with ip = p when p is a non-negative integer (ip < 0 otherwise).
template <typename R>
__device__ __forceinline__ R powi_or_pow(R s, int ip, R p)
{
    if (ip >= 0) {
        R r = R(1);
        for (int k = 0; k < ip; ++k) r *= s;
        return r;
    }
    return pow_general(s, p);
}

__device__ __forceinline__ void eff_box(const SysState &st, double box[3], double ibox[3])
{
    for (int k = 0; k < 3; ++k) {
        box[k] = st.box[k] * st.pscale[k];
        ibox[k] = 1.0 / box[k];
    }
}

// Radius of a system's Verlet list: the longest interaction cutoff (the SW
// cutoff, or the UF reference's when longer) plus the skin.
__device__ __forceinline__ double list_radius(const SwParams &sw, const SysDesc &d)
{
    return fmax(sw.rc, d.uf_rc) + d.skin;
}

// Cell grid for the list build: cells of at least the list radius, capped.
// The range tests run in FP64 before any conversion to int, so a
// non-finite box or position (which the step flags as an error) still
// yields an index inside the grid: converting NaN or an out-of-range double
// to int would be undefined.
__device__ __forceinline__ void cell_grid(const SysDesc &d, const double box[3], double rl, int nc[3])
{
    for (int k = 0; k < 3; ++k) {
        const double n = floor(box[k] / rl);
        nc[k] = n >= 1.0 ? (n < (double)d.nc_max[k] ? (int)n : d.nc_max[k]) : 1;
    }
}

__device__ __forceinline__ int cell_coord(double x, double ibox, int nc)
{
    double s = x * ibox;
    s -= floor(s);
    const double f = s * nc;
    return f >= 0.0 ? (f < (double)nc ? (int)f : nc - 1) : 0;
}

__device__ __forceinline__ int cell_of_pos(const double4 &x, const double ibox[3], const int nc[3])
{
    const int cx = cell_coord(x.x, ibox[0], nc[0]);
    const int cy = cell_coord(x.y, ibox[1], nc[1]);
    const int cz = cell_coord(x.z, ibox[2], nc[2]);
    return (cz * nc[1] + cy) * nc[0] + cx;
}

__device__ __forceinline__ double min_image(double d, double box, double ibox)
{
    return d - box * rint(d * ibox);
}

// FP32 copy of a position, wrapped into [0, box) with the box the force
// passes use for the minimum image (the wrap shifts by whole boxes, which
// the minimum image removes again).  The list filter reads it.
__device__ __forceinline__ float4 pos_f32(const double4 &x, const double box[3], const double ibox[3])
{
    return make_float4((float)(x.x - box[0] * floor(x.x * ibox[0])), (float)(x.y - box[1] * floor(x.y * ibox[1])),
                       (float)(x.z - box[2] * floor(x.z * ibox[2])), 0.0f);
}

// Philox4x64-10 (Salmon et al., SC'11) and Box-Muller: three normals per
// (step, atom) with key (seed, stream).
__device__ __forceinline__ void normals3(uint64_t seed, uint64_t stream, uint64_t step,
                                         uint64_t atom, double out[3])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = step, c1 = atom, c2 = 0, c3 = 0, k0 = seed, k1 = stream;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    const double two53 = 1.1102230246251565e-16;  // 2^-53
    double u0 = ((double)(c0 >> 11) + 1.0) * two53;
    double u1 = ((double)(c1 >> 11) + 1.0) * two53;
    double u2 = ((double)(c2 >> 11) + 1.0) * two53;
    double u3 = ((double)(c3 >> 11) + 1.0) * two53;
    // cos(2 pi u) and sin(2 pi u) through sincospi(2 u): 2 u is exact and
    // lies in (0, 2], so no general argument reduction is needed
    const double r01 = sqrt(-2.0 * log(u0));
    const double r23 = sqrt(-2.0 * log(u2));
    double sn1, cs1, sn3, cs3;
    sincospi(2.0 * u1, &sn1, &cs1);
    sincospi(2.0 * u3, &sn3, &cs3);
    out[0] = r01 * cs1;
    out[1] = r01 * sn1;
    out[2] = r23 * cs3;
}

__device__ __forceinline__ bool o_step_on(const SysDesc &d)
{
    return d.mode != MODE_FORCE && d.mode != MODE_NVE && d.tau_damp > 0.0 && d.T0 > 0.0;
}

__device__ __forceinline__ bool scales_interaction(int mode)
{
    return mode == MODE_RS || mode == MODE_DCCI_T || mode == MODE_DCCI_P;
}

// Total force component at coupling lam: FL interpolates with the Einstein
// reference (section 2.1), UF with the Uhlenbeck-Ford fluid (fref), RS and
// dCCI scale the interaction (eq. H_RS).
__device__ __forceinline__ double total_force(int mode, double lam, double fint, double x, double x0,
                                              double k, double fref)
{
    if (mode == MODE_FL) return lam * fint + (1.0 - lam) * (-k * (x - x0));
    if (mode == MODE_UF) return lam * fint + (1.0 - lam) * fref;
    if (scales_interaction(mode)) return lam * fint;
    return fint;
}

// Deterministic block reduction of NV doubles per thread into out[0..NV).
// Only the slots in MASK are summed (the others are zero in every thread of
// the caller, and are written as zeros).
template <int NV, uint32_t MASK = (NV >= 32 ? ~0u : (1u << NV) - 1u)>
__device__ __forceinline__ void block_reduce(double (&v)[NV], double *out)
{
    __shared__ double red[4][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        if (!((MASK >> k) & 1u)) continue;
        double a = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
        if (lane == 0) red[wave][k] = a;
    }
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        double s = 0.0;
        if ((MASK >> threadIdx.x) & 1u)
            for (int w = 0; w < nw; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();  // red may be written again by the block's next call
}

// Slots of the tile partials each force pass fills (block_reduce masks):
// pass 1 the two-body energy, the virial's upper triangle and the
// three-body energy, with parameter gradients also the derivatives; pass 2
// the virial's upper triangle, Einstein energy, kinetic energy and noise
// sums, with gradients also its three parameter derivatives.
constexpr uint32_t kVirUpper = (1u << 1) | (1u << 2) | (1u << 3) | (1u << 5) | (1u << 6) | (1u << 9);
constexpr uint32_t kPass1Slots = 1u | kVirUpper | (1u << P_E3);
constexpr uint32_t kPass1GradSlots = kPass1Slots | (0x1FFu << P_DTH);
constexpr uint32_t kPass2Slots = kVirUpper | (0x7Fu << P_UREF);
constexpr uint32_t kPass2GradSlots = kPass2Slots | (1u << 14) | (1u << 16) | (1u << 17);

__device__ __forceinline__ double block_max(double v)
{
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double m = 0.0;
    for (int w = 0; w < nw; ++w) m = fmax(m, red[w]);
    __syncthreads();  // red may be written again by the block's next call
    return m;
}

// -------------------------------------------------------- gather/scatter ---
__global__ void __launch_bounds__(256) k_iota(Ctl c, DevPtrs p)
{
    const int ti = tile_of_block(c);
    if (ti < 0) return;
    const Tile tile = p.tiles[ti];
    if ((int)threadIdx.x < tile.count) {
        const int t = tile.start + threadIdx.x;
        p.perm[t] = t;
    }
}

// Caller arrays (original order, [3][N]) -> sorted internal arrays.
__global__ void __launch_bounds__(256) k_gather(Ctl c, DevPtrs p, int with_f)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) p.n_work[0] = 0;
    const int ti = tile_of_block(c);
    if (ti < 0) return;
    const Tile tile = p.tiles[ti];
    if ((int)threadIdx.x >= tile.count) return;
    const SysState &st = p.state[tile.sys];
    const int64_t N = c.n_total;
    const int t = tile.start + threadIdx.x;
    const int i = p.perm[t];
    const double4 x = make_double4(p.x[i] * st.pscale[0], p.x[N + i] * st.pscale[1], p.x[2 * N + i] * st.pscale[2], 0.0);
    double box[3], ibox[3];
    eff_box(st, box, ibox);
    p.xs[t] = x;
    p.xf[t] = pos_f32(x, box, ibox);
    // force evaluations without dynamics may pass no velocities
    p.vs[t] = p.v ? make_dvec3(p.v[i], p.v[N + i], p.v[2 * N + i]) : make_dvec3(0.0, 0.0, 0.0);
    if (with_f) p.fs[t] = make_dvec3(p.f[i], p.f[N + i], p.f[2 * N + i]);
    if (p.x0) p.x0s[t] = make_dvec3(p.x0[i], p.x0[N + i], p.x0[2 * N + i]);
}

// Sorted internal arrays -> caller arrays.  what: 1 x and v, 2 f, 4 e_atom,
// 8 grad_x = -F grad_scale.
__global__ void __launch_bounds__(256) k_scatter(Ctl c, DevPtrs p, int what)
{
    const int ti = tile_of_block(c);
    if (ti < 0) return;
    const Tile tile = p.tiles[ti];
    if ((int)threadIdx.x >= tile.count) return;
    const int64_t N = c.n_total;
    const int t = tile.start + threadIdx.x;
    const int i = p.perm[t];
    if (what & 1) {
        const double4 x = p.xs[t];
        const dvec3 v = p.vs[t];
        p.x[i] = x.x;
        p.x[N + i] = x.y;
        p.x[2 * N + i] = x.z;
        p.v[i] = v.x;
        p.v[N + i] = v.y;
        p.v[2 * N + i] = v.z;
    }
    const dvec3 f = p.fs[t];
    if (what & 2) {
        p.f[i] = f.x;
        p.f[N + i] = f.y;
        p.f[2 * N + i] = f.z;
    }
    if ((what & 4) && p.e_atom) p.e_atom[i] = p.e_s[t];
    if ((what & 8) && p.grad_x) {
        const double g = p.grad_scale ? p.grad_scale[tile.sys] : 1.0;
        p.grad_x[i] = -f.x * g;
        p.grad_x[N + i] = -f.y * g;
        p.grad_x[2 * N + i] = -f.z * g;
    }
}

// Cell of an atom at its current position and its rank among the atoms
// counted into that cell (the order of the ranks is fixed later).
__device__ __forceinline__ void bin_atom(const DevPtrs &p, const SwParams &sw, const SysDesc &d,
                                         const SysState &st, int t, const double4 &x)
{
    double box[3], ibox[3];
    int nc[3];
    eff_box(st, box, ibox);
    cell_grid(d, box, list_radius(sw, d), nc);
    const int cell = cell_of_pos(x, ibox, nc);
    p.cellid[t] = cell;
    p.rank[t] = atomicAdd(&p.cell_count[d.cell_base + cell], 1);
}

// Normals of the next O step for every atom in the current order (after a
// list build outside a step reorders the atoms).
__global__ void __launch_bounds__(256) k_fill_noise(Ctl c, DevPtrs p)
{
    const int ti = tile_of_block(c);
    if (ti < 0) return;
    const Tile tile = p.tiles[ti];
    if ((int)threadIdx.x >= tile.count) return;
    const SysDesc &d = p.desc[tile.sys];
    if (!o_step_on(d)) return;
    const int t = tile.start + threadIdx.x;
    double z[3];
    normals3(c.seed, d.stream, (uint64_t)p.state[tile.sys].step, (uint64_t)(p.perm[t] - d.off), z);
    p.zs[t] = make_dvec3(z[0], z[1], z[2]);
}

// ------------------------------------------------------------- integrate ---
// Steps 3-6 of the switched step for one atom: B kick with F(lambda_{k+1}),
// A half drift with isotropic box scaling, O Langevin step with zero-sum
// noise, A half drift.  Then the displacement from the list-build position
// (scaled with the box) for the rebuild test.
__device__ __forceinline__ void integrate_tile(const Ctl &c, const DevPtrs &p, const SwParams &sw, int ti)
{
    const Tile tile = p.tiles[ti];
    const int sys = tile.sys;
    const SysDesc &d = p.desc[sys];
    const SysState &st = p.state[sys];
    double dmax = 0.0;
    if ((int)threadIdx.x < tile.count) {
        const int t = tile.start + threadIdx.x;
        double4 x = p.xs[t];
        if (d.mode != MODE_FORCE) {
            dvec3 v = p.vs[t];
            const dvec3 f = p.fs[t];
            const dvec3 x0 = d.mode == MODE_FL ? p.x0s[t] : make_dvec3(0, 0, 0);
            const dvec3 fr = d.mode == MODE_UF ? p.fref[t] : make_dvec3(0, 0, 0);
            const double hdt = 0.5 * c.dt, ka = hdt * d.acc;
            v.x = v.x * st.decay[0] + ka * total_force(d.mode, st.lam, f.x, x.x, x0.x, d.k_spring, fr.x) * st.phi[0];
            v.y = v.y * st.decay[1] + ka * total_force(d.mode, st.lam, f.y, x.y, x0.y, d.k_spring, fr.y) * st.phi[1];
            v.z = v.z * st.decay[2] + ka * total_force(d.mode, st.lam, f.z, x.z, x0.z, d.k_spring, fr.z) * st.phi[2];
            x.x = x.x * st.grow[0] + (v.x * hdt) * st.psi[0];
            x.y = x.y * st.grow[1] + (v.y * hdt) * st.psi[1];
            x.z = x.z * st.grow[2] + (v.z * hdt) * st.psi[2];
            if (o_step_on(d)) {
                // this step's normals, drawn by the force pass that ended
                // the previous step (it also formed their mean)
                const dvec3 z = p.zs[t];
                const double c2s = d.c2 * d.sigv;
                v.x = d.c1 * v.x + c2s * (z.x - st.noise_mean[0]);
                v.y = d.c1 * v.y + c2s * (z.y - st.noise_mean[1]);
                v.z = d.c1 * v.z + c2s * (z.z - st.noise_mean[2]);
            }
            x.x = x.x * st.grow[0] + (v.x * hdt) * st.psi[0];
            x.y = x.y * st.grow[1] + (v.y * hdt) * st.psi[1];
            x.z = x.z * st.grow[2] + (v.z * hdt) * st.psi[2];
            p.xs[t] = x;
            p.vs[t] = v;
            double box[3], ibox[3];
            eff_box(st, box, ibox);
            p.xf[t] = pos_f32(x, box, ibox);
        }
        if (!(isfinite(x.x) && isfinite(x.y) && isfinite(x.z))) atomicOr(&p.state[sys].err, ERR_NONFINITE);
        const dvec3 b = p.xb[t];
        const double dx = x.x - b.x * (st.box[0] / st.box_build[0]);
        const double dy = x.y - b.y * (st.box[1] / st.box_build[1]);
        const double dz = x.z - b.z * (st.box[2] / st.box_build[2]);
        dmax = dx * dx + dy * dy + dz * dz;
        if (!(dmax == dmax)) dmax = 1e300;  // NaN forces a rebuild (and is flagged above)
    }
    dmax = block_max(dmax);
    // non-negative doubles order like their bit patterns: one atomic max per
    // block into this step's slot of the system
    if (threadIdx.x == 0)
        atomicMax(reinterpret_cast<unsigned long long *>(&p.disp_max[2 * sys + (st.step & 1)]),
                  (unsigned long long)__double_as_longlong(dmax));
}

// Every launch sequence that may rebuild lists starts with integrate or
// gather, which empty the rebuild work list for it.
__global__ void __launch_bounds__(256) k_integrate(Ctl c, DevPtrs p, SwParams sw)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) p.n_work[0] = 0;
    const int ti = tile_of_block(c);
    if (ti >= 0) integrate_tile(c, p, sw, ti);
}

// --------------------------------------------------------------- rebuild ---
// Does this system's Verlet list need a rebuild?  A pair now within rc that
// is missing from the list was at least rc + skin apart at the build; after
// box scaling by s and displacements of at most delta per atom it is at
// least s (rc + skin) - 2 delta apart, so the list is still complete while
// 2 delta + (1 - s)(rc + skin) <= skin.
__device__ bool list_stale(const Ctl &c, const DevPtrs &p, const SwParams &sw, int sys)
{
    if (c.force_rebuild) return true;
    const SysDesc &d = p.desc[sys];
    const SysState &st = p.state[sys];
    // both displacement slots load with the state (no wait for the step
    // count before the slot's load)
    const double m0 = p.disp_max[2 * sys], m1 = p.disp_max[2 * sys + 1];
    const double m = (st.step & 1) ? m1 : m0;
    double smin = 1e300;
    for (int k = 0; k < 3; ++k) smin = fmin(smin, (st.box[k] * st.pscale[k]) / st.box_build[k]);
    const double shrink = smin < 1.0 ? 1.0 - smin : 0.0;
    return 2.0 * sqrt(m) + list_radius(sw, d) * shrink > d.skin;
}

// Binning of the atoms of every system whose list is stale (each block
// takes the decision for its tile's system; the scan stage takes the same
// decision from the same inputs).  The rebuild work list starts empty
// (integrate or gather empties it).
__device__ __forceinline__ void rb_count_tile(const DevPtrs &p, const SwParams &sw, int ti)
{
    const Tile tile = p.tiles[ti];
    for (int a = threadIdx.x; a < tile.count; a += blockDim.x) {
        const int t = tile.start + a;
        bin_atom(p, sw, p.desc[tile.sys], p.state[tile.sys], t, p.xs[t]);
    }
}

// The displacement slots of one system at a rebuild decision: the slot the
// next step's integrate fills is cleared (both on a forced build, which
// reads neither).
__device__ __forceinline__ void clear_disp_slots(const Ctl &c, const DevPtrs &p, int sys)
{
    const int64_t step = p.state[sys].step;
    p.disp_max[2 * sys + ((step + 1) & 1)] = 0.0;
    if (c.force_rebuild) p.disp_max[2 * sys + (step & 1)] = 0.0;
}

__global__ void __launch_bounds__(256) k_rb_count(Ctl c, DevPtrs p, SwParams sw)
{
    const int ti = tile_of_block(c);
    if (ti < 0) return;
    const int sys = p.tiles[ti].sys;
    // without a scan launch, the block of a system's first tile clears its
    // displacement slot (a slot the decision below does not read)
    if (c.scan_cells > 0 && threadIdx.x == 0 && ti == p.desc[sys].tile_begin) clear_disp_slots(c, p, sys);
    if (!list_stale(c, p, sw, sys)) return;
    rb_count_tile(p, sw, ti);
    // and each stale tile goes to the work list of the later stages itself
    // (their tiles are independent: the order of the list does not matter)
    if (c.scan_cells > 0 && threadIdx.x == 0) p.work[atomicAdd(&p.n_work[0], 1)] = ti;
}

// For one system, by all threads of a block: clear the next step's
// displacement slot, and for a stale list (rb) the exclusive scan of the cell
// counts into cell starts (sorted positions), the counts cleared for the
// next binning, the build box and the rebuild count; with `append` the
// system's tiles go to the work list of the later stages.
// NT bounds the block's thread count (the LDS of the scan).
template <int NT>
__device__ void rb_scan_sys(const Ctl &c, const DevPtrs &p, const SwParams &sw, int sys, bool rb, bool append)
{
    SysState &st = p.state[sys];
    const SysDesc &d = p.desc[sys];
    double box[3], ibox[3];
    int nc3[3];
    eff_box(st, box, ibox);
    cell_grid(d, box, list_radius(sw, d), nc3);
    const int nc = nc3[0] * nc3[1] * nc3[2];
    int32_t *cnt = p.cell_count + d.cell_base;
    const int tid = threadIdx.x, nth = blockDim.x;
    __shared__ int at_s;
    if (tid == 0) {
        clear_disp_slots(c, p, sys);
        at_s = rb && append ? atomicAdd(&p.n_work[0], d.tile_end - d.tile_begin) : 0;
    }
    __syncthreads();
    if (rb) {
        if (append)
            for (int q = tid; q < d.tile_end - d.tile_begin; q += nth) p.work[at_s + q] = d.tile_begin + q;
        int32_t *start = p.cell_start + d.cell_base + sys;  // nc + 1 entries
        const int off = (int)d.off, n = (int)d.n;
        __shared__ int32_t part[NT];
        const int per = (nc + nth - 1) / nth;
        const int lo = min(tid * per, nc), hi = min(lo + per, nc);
        int sum = 0;
        for (int q = lo; q < hi; ++q) sum += cnt[q];
        part[tid] = sum;
        __syncthreads();
        for (int o = 1; o < nth; o <<= 1) {
            const int add = tid >= o ? part[tid - o] : 0;
            __syncthreads();
            part[tid] += add;
            __syncthreads();
        }
        int run = off + part[tid] - sum;
        for (int q = lo; q < hi; ++q) {
            start[q] = run;
            run += cnt[q];
            cnt[q] = 0;
        }
        if (tid == 0) {
            start[nc] = off + n;
            for (int k = 0; k < 3; ++k) st.box_build[k] = box[k];
            st.n_rebuild += 1;
        }
    }
    __syncthreads();  // at_s and part may be written again by the block's next call
}

// One workgroup per system: the rebuild decision, then the scan above with
// the stale systems' tiles appended to the work list of the later stages.
__global__ void __launch_bounds__(kSortThreads) k_rb_scan(Ctl c, DevPtrs p, SwParams sw)
{
    const int sys = blockIdx.x;
    __shared__ int rb_s;
    if (threadIdx.x == 0) rb_s = list_stale(c, p, sw, sys) ? 1 : 0;
    __syncthreads();
    rb_scan_sys<kSortThreads>(c, p, sw, sys, rb_s != 0, true);
}

// Atom data into its cell's segment of the staging arrays (slot by rank, so
// the order inside a cell is not yet fixed).
// lstart: the system's cell starts in LDS, or null to read them from memory
__device__ __forceinline__ void rb_scatter_tile(const DevPtrs &p, int ti, const int32_t *lstart)
{
    const Tile tile = p.tiles[ti];
    for (int a = threadIdx.x; a < tile.count; a += blockDim.x) {
        const int sys = tile.sys;
        const SysDesc &d = p.desc[sys];
        const int t = tile.start + a;
        const int cell = p.cellid[t];
        const int s = (lstart ? lstart[cell] : p.cell_start[d.cell_base + sys + cell]) + p.rank[t];
        p.txs[s] = p.xs[t];
        p.tvs[s] = p.vs[t];
        p.tfs[s] = p.fs[t];
        if (p.x0) p.tx0s[s] = p.x0s[t];
        p.tperm[s] = p.perm[t];
        p.norder[s] = cell;
    }
}

// Exclusive scan of a rebuilding system's cell counts into LDS (nc + 1
// entries: cell starts in sorted positions, then the system's end), by all
// threads of the block (at most 256).  The block of the system's first tile
// also writes them out for the later stages, with the build box and the
// rebuild count.  Same arithmetic as the scan stage.
__device__ void scan_cells_lds(const Ctl &c, const DevPtrs &p, const SwParams &sw, int sys, bool first,
                               int32_t *lstart)
{
    SysState &st = p.state[sys];
    const SysDesc &d = p.desc[sys];
    double box[3], ibox[3];
    int nc3[3];
    eff_box(st, box, ibox);
    cell_grid(d, box, list_radius(sw, d), nc3);
    const int nc = nc3[0] * nc3[1] * nc3[2];
    const int32_t *cnt = p.cell_count + d.cell_base;
    const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wave = tid >> 6;
    __shared__ int32_t wsum[4];
    for (int q = tid; q < nc; q += nth) lstart[q] = cnt[q];
    __syncthreads();
    const int per = (nc + nth - 1) / nth;
    const int lo = min(tid * per, nc), hi = min(lo + per, nc);
    int sum = 0;
    for (int q = lo; q < hi; ++q) sum += lstart[q];
    // inclusive scan of the segment sums: within each wave by lane
    // exchanges, then over the waves' totals
    int incl = sum;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    for (int w = 0; w < wave; ++w) incl += wsum[w];
    int run = (int)d.off + incl - sum;
    for (int q = lo; q < hi; ++q) {
        const int k = lstart[q];
        lstart[q] = run;
        run += k;
    }
    if (tid == 0) lstart[nc] = (int)(d.off + d.n);
    __syncthreads();
    if (first) {
        int32_t *start = p.cell_start + d.cell_base + sys;
        for (int q = tid; q <= nc; q += nth) start[q] = lstart[q];
        if (tid == 0) {
            for (int k = 0; k < 3; ++k) st.box_build[k] = box[k];
            st.n_rebuild += 1;
        }
    }
}

__global__ void __launch_bounds__(256) k_rb_scatter(Ctl c, DevPtrs p, SwParams sw)
{
    extern __shared__ int32_t lstart[];  // c.scan_cells entries when the scan is folded in
    const int n_work = p.n_work[0];
    for (int w = blockIdx.x; w < n_work; w += gridDim.x) {
        const int ti = p.work[w];
        if (c.scan_cells > 0) {
            const int sys = p.tiles[ti].sys;
            scan_cells_lds(c, p, sw, sys, ti == p.desc[sys].tile_begin, lstart);
            rb_scatter_tile(p, ti, lstart);
            __syncthreads();  // lstart is written again for the block's next tile
        } else {
            rb_scatter_tile(p, ti, nullptr);
        }
    }
}

// Final order: inside a cell atoms follow the caller's atom index.  Each
// staged atom counts the smaller indices of its cell and moves there.
__device__ __forceinline__ void rb_order_tile(const DevPtrs &p, int ti)
{
    const Tile tile = p.tiles[ti];
    for (int a = threadIdx.x; a < tile.count; a += blockDim.x) {
        const int sys = tile.sys;
        const SysDesc &d = p.desc[sys];
        const int i = tile.start + a;
        const int cell = p.norder[i];
        const int32_t *start = p.cell_start + d.cell_base + sys;
        const int b = start[cell], e = start[cell + 1];
        const int key = p.tperm[i];
        int rank = 0;
        for (int j = b; j < e; ++j) rank += p.tperm[j] < key ? 1 : 0;
        const int s = b + rank;
        const double4 x = p.txs[i];
        double box[3], ibox[3];
        eff_box(p.state[sys], box, ibox);
        p.xs[s] = x;
        p.xf[s] = pos_f32(x, box, ibox);
        p.xb[s] = make_dvec3(x.x, x.y, x.z);
        p.vs[s] = p.tvs[i];
        p.fs[s] = p.tfs[i];
        if (p.x0) p.x0s[s] = p.tx0s[i];
        p.perm[s] = key;
    }
}

__global__ void __launch_bounds__(256) k_rb_order(Ctl c, DevPtrs p, SwParams sw)
{
    const int n_work = p.n_work[0];
    for (int w = blockIdx.x; w < n_work; w += gridDim.x) {
        const int ti = p.work[w];
        rb_order_tile(p, ti);
        if (c.scan_cells > 0) {
            // the counts were last read by the scatter stage: clear them for
            // the next binning (the block of the system's first tile)
            const int sys = p.tiles[ti].sys;
            const SysDesc &d = p.desc[sys];
            if (ti == d.tile_begin) {
                double box[3], ibox[3];
                int nc3[3];
                eff_box(p.state[sys], box, ibox);
                cell_grid(d, box, list_radius(sw, d), nc3);
                const int nc = nc3[0] * nc3[1] * nc3[2];
                for (int q = threadIdx.x; q < nc; q += blockDim.x) p.cell_count[d.cell_base + q] = 0;
            }
        }
    }
}

// Rebuild stages 0-3 fused, one workgroup of kSortThreads per system (used
// when every system's cell table fits in LDS, c.sort_cells entries): the
// rebuild decision; for a stale list the cell of each atom and its rank among
// the atoms counted into that cell (LDS counters), the exclusive scan of the
// counts into cell starts (kept in LDS, written out for the list stage), the
// atoms staged into their cells' segments, and their final order inside a
// cell by caller index.  The system's tiles go to the list stage's work list.
// The atoms come out in the same order as through the separate stages.
__global__ void __launch_bounds__(kSortThreads) k_rb_sort(Ctl c, DevPtrs p, SwParams sw)
{
    extern __shared__ int32_t lcell[];  // counts, then starts: nc + 1 entries
    __shared__ int rb_s, at_s;
    __shared__ int32_t part[kSortThreads];
    const int sys = blockIdx.x, tid = threadIdx.x, nth = blockDim.x;
    SysState &st = p.state[sys];
    const SysDesc &d = p.desc[sys];
    double box[3], ibox[3];
    int nc3[3];
    eff_box(st, box, ibox);
    cell_grid(d, box, list_radius(sw, d), nc3);
    const int nc = nc3[0] * nc3[1] * nc3[2];
    const int off = (int)d.off, n = (int)d.n;
    if (tid == 0) {
        const bool rb = list_stale(c, p, sw, sys);
        // clear the slot the next step's integrate fills (both on a forced build)
        p.disp_max[2 * sys + ((st.step + 1) & 1)] = 0.0;
        if (c.force_rebuild) p.disp_max[2 * sys + (st.step & 1)] = 0.0;
        rb_s = rb ? 1 : 0;
        at_s = rb ? atomicAdd(&p.n_work[0], d.tile_end - d.tile_begin) : 0;
    }
    __syncthreads();
    if (!rb_s) return;
    for (int q = tid; q < d.tile_end - d.tile_begin; q += nth) p.work[at_s + q] = d.tile_begin + q;
    for (int q = tid; q <= nc; q += nth) lcell[q] = 0;
    __syncthreads();
    // cell of every atom and its rank among the atoms counted into the cell
#pragma unroll 4
    for (int a = tid; a < n; a += nth) {
        const int t = off + a;
        const int cell = cell_of_pos(p.xs[t], ibox, nc3);
        p.cellid[t] = cell;
        p.rank[t] = atomicAdd(&lcell[cell], 1);
    }
    __syncthreads();
    // exclusive scan of the counts into starts (sorted positions)
    const int per = (nc + nth - 1) / nth;
    const int lo = min(tid * per, nc), hi = min(lo + per, nc);
    int sum = 0;
    for (int q = lo; q < hi; ++q) sum += lcell[q];
    part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < nth; o <<= 1) {
        const int add = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
    }
    int32_t *start = p.cell_start + d.cell_base + sys;  // nc + 1 entries
    int run = off + part[tid] - sum;
    for (int q = lo; q < hi; ++q) {
        const int v = lcell[q];
        lcell[q] = run;
        start[q] = run;
        run += v;
    }
    if (tid == 0) {
        lcell[nc] = off + n;
        start[nc] = off + n;
    }
    __syncthreads();
    // atom data into its cell's segment of the staging arrays (by rank)
#pragma unroll 4
    for (int a = tid; a < n; a += nth) {
        const int t = off + a;
        const int cell = p.cellid[t];
        const int s = lcell[cell] + p.rank[t];
        p.txs[s] = p.xs[t];
        p.tvs[s] = p.vs[t];
        p.tfs[s] = p.fs[t];
        if (p.x0) p.tx0s[s] = p.x0s[t];
        p.tperm[s] = p.perm[t];
        p.norder[s] = cell;
    }
    __syncthreads();
    // final order: inside a cell atoms follow the caller's atom index
    for (int a = tid; a < n; a += nth) {
        const int i = off + a;
        const int cell = p.norder[i];
        const int b = lcell[cell], e = lcell[cell + 1];
        const int key = p.tperm[i];
        int rank = 0;
#pragma unroll 4
        for (int j = b; j < e; ++j) rank += p.tperm[j] < key ? 1 : 0;
        const int s = b + rank;
        const double4 x = p.txs[i];
        p.xs[s] = x;
        p.xf[s] = pos_f32(x, box, ibox);
        p.xb[s] = make_dvec3(x.x, x.y, x.z);
        p.vs[s] = p.tvs[i];
        p.fs[s] = p.tfs[i];
        if (p.x0) p.x0s[s] = p.tx0s[i];
        p.perm[s] = key;
    }
    if (tid == 0) {
        for (int k = 0; k < 3; ++k) st.box_build[k] = box[k];
        st.n_rebuild += 1;
    }
}

// Verlet-list storage.  With 32-bit entries, entry k of sorted atom s is the
// sorted position of the neighbour at nl[k * N + s].  With 16-bit entries
// (every system below 65537 atoms) it is the position relative to the
// system's first atom, two entries per 32-bit word: halfword k & 1 of word
// (k / 2) * N + s.  In both forms a row is contiguous over the atoms, so a
// wavefront's list loads are coalesced; the 16-bit form halves their
// number and their bytes.
__device__ __forceinline__ void list_put(const Ctl &c, int32_t *nl, int k, int64_t N, int s, int j, int off)
{
    if (c.list16)
        reinterpret_cast<uint16_t *>(nl)[((int64_t)(k >> 1) * N + s) * 2 + (k & 1)] = (uint16_t)(j - off);
    else
        nl[(int64_t)k * N + s] = j;
}

// Raw words holding entries k0 .. k0 + B - 1 (k0 and B even) of atom t's
// Verlet list: B / 2 words in the 16-bit form, B in the 32-bit form.  Rows
// at or past `rows` re-read row rows - 1 (no branch around the load); with
// rows = list_cap the addresses do not depend on the atom's entry count, so
// the first batch can load together with that count.
template <int B>
__device__ __forceinline__ void list_load(const Ctl &c, const int32_t *nl, int k0, int rows, int64_t N, int t,
                                          uint32_t (&w)[B])
{
    static_assert(B % 2 == 0, "pairs of entries");
    const uint32_t *w32 = reinterpret_cast<const uint32_t *>(nl);
    if (c.list16) {
        const int last = (rows - 1) >> 1;
#pragma unroll
        for (int u = 0; u < B / 2; ++u) {
            const int pr = (k0 >> 1) + u;
            w[u] = w32[(int64_t)(pr < last ? pr : last) * N + t];
        }
#pragma unroll
        for (int u = B / 2; u < B; ++u) w[u] = 0u;
    } else {
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int k = k0 + u < rows ? k0 + u : rows - 1;
            w[u] = w32[(int64_t)k * N + t];
        }
    }
}

// Sorted positions of entries k0 .. k0 + B - 1 from their raw words; entries
// at or past cnt yield t itself, whose position is always valid to load.
template <int B>
__device__ __forceinline__ void list_decode(const Ctl &c, const uint32_t (&w)[B], int k0, int cnt, int t, int off,
                                            int (&jb)[B])
{
    if (c.list16) {
#pragma unroll
        for (int u = 0; u < B / 2; ++u) {
            jb[2 * u] = k0 + 2 * u < cnt ? off + (int)(w[u] & 0xffffu) : t;
            jb[2 * u + 1] = k0 + 2 * u + 1 < cnt ? off + (int)(w[u] >> 16) : t;
        }
    } else {
#pragma unroll
        for (int u = 0; u < B; ++u) jb[u] = k0 + u < cnt ? (int)w[u] : t;
    }
}

// Entries k0 .. k0 + B - 1 of atom t's Verlet list of cnt >= 1 entries.
template <int B>
__device__ __forceinline__ void list_batch(const Ctl &c, const int32_t *nl, int k0, int cnt, int64_t N, int t,
                                           int off, int (&jb)[B])
{
    uint32_t w[B];
    list_load<B>(c, nl, k0, cnt, N, t, w);
    list_decode<B>(c, w, k0, cnt, t, off, jb);
}

// Verlet list of sorted positions within rc + skin from the (up to) 27 cells
// around the atom's cell (fewer when a dimension has fewer than 3 cells, so
// that no cell is visited twice).  32 lanes per atom, one per stencil cell:
// each lane marks the candidates of its cell, a prefix sum over the lanes
// gives every cell its slot range, so the list is in stencil-cell order and,
// inside a cell, in sorted order.  A block holds blockDim / 32 atoms; sub
// numbers the blocks' shares of one tile.
__device__ __forceinline__ void list_block(const Ctl &c, const DevPtrs &p, const SwParams &sw, int ti, int sub)
{
    const Tile tile = p.tiles[ti];
    const int sys = tile.sys;
    const int a_loc = sub * (int)(blockDim.x >> 5) + (threadIdx.x >> 5);
    const int lane = threadIdx.x & 31;
    const bool valid = a_loc < tile.count;
    const SysDesc &d = p.desc[sys];
    const SysState &st = p.state[sys];
    double box[3], ibox[3];
    int nc[3];
    eff_box(st, box, ibox);
    const double rl = list_radius(sw, d), rl2 = rl * rl;
    cell_grid(d, box, rl, nc);
    const int64_t N = c.n_total;
    const int s = tile.start + (valid ? a_loc : 0);
    const double4 xi = p.xs[s];
    const float4 xif = p.xf[s];
    const int ci = cell_of_pos(xi, ibox, nc);
    const int cx = ci % nc[0], cy = (ci / nc[0]) % nc[1], cz = ci / (nc[0] * nc[1]);
    const int nxo = nc[0] >= 3 ? 3 : nc[0], nyo = nc[1] >= 3 ? 3 : nc[1], nzo = nc[2] >= 3 ? 3 : nc[2];
    const int x0c = nc[0] >= 3 ? cx - 1 : 0, y0c = nc[1] >= 3 ? cy - 1 : 0, z0c = nc[2] >= 3 ? cz - 1 : 0;
    const int32_t *start = p.cell_start + d.cell_base + sys;
    const int ncell = nxo * nyo * nzo;
    // Candidates of one chunk of up to 64 atoms of this lane's cell, as a
    // mask, from the FP32 positions wrapped into the box, eight loads in
    // flight: the test is conservative (the rounding of the wrapped FP32
    // coordinates moves d^2 by far less than the margin), so the list holds
    // every pair within rl and a few just beyond it, which the force passes'
    // exact test drops.
    const float bx = (float)box[0], by = (float)box[1], bz = (float)box[2];
    const float ibx = (float)ibox[0], iby = (float)ibox[1], ibz = (float)ibox[2];
    const double bmax = fmax(box[0], fmax(box[1], box[2]));
    const float cut2 = (float)(rl2 * (1.0 + 1e-3) + 32.0 * rl * bmax * 1.1920928955078125e-7);
    auto chunk_mask = [&](int j0, int j1) {
        unsigned long long m = 0;
        for (int jb = j0; jb < j1; jb += 8) {
            float4 xj[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) xj[u] = p.xf[jb + u < j1 ? jb + u : j1 - 1];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                float dx = xj[u].x - xif.x, dy = xj[u].y - xif.y, dz = xj[u].z - xif.z;
                dx -= bx * rintf(dx * ibx);
                dy -= by * rintf(dy * iby);
                dz -= bz * rintf(dz * ibz);
                const int j = jb + u;
                if (j < j1 && j != s && dx * dx + dy * dy + dz * dz < cut2) m |= 1ull << (j - j0);
            }
        }
        return m;
    };
    unsigned long long mask = 0;
    int b = 0, e = 0, cnt = 0;
    if (valid && lane < ncell) {
        const int ox = lane % nxo, oy = (lane / nxo) % nyo, oz = lane / (nxo * nyo);
        int xx = x0c + ox, yy = y0c + oy, zz = z0c + oz;
        xx = xx < 0 ? xx + nc[0] : (xx >= nc[0] ? xx - nc[0] : xx);
        yy = yy < 0 ? yy + nc[1] : (yy >= nc[1] ? yy - nc[1] : yy);
        zz = zz < 0 ? zz + nc[2] : (zz >= nc[2] ? zz - nc[2] : zz);
        const int cell = (zz * nc[1] + yy) * nc[0] + xx;
        b = start[cell];
        e = start[cell + 1];
        // cells of more than 64 atoms (long UF cutoffs) are counted chunk by
        // chunk here and re-scanned when the entries are written
        for (int j0 = b; j0 < e; j0 += 64) {
            const unsigned long long m = chunk_mask(j0, min(j0 + 64, e));
            if (j0 == b) mask = m;
            cnt += __popcll(m);
        }
    }
    // exclusive prefix of the per-cell counts over the 32 lanes of this atom
    int incl = cnt;
    for (int o = 1; o < 32; o <<= 1) {
        const int u = __shfl_up(incl, o, 32);
        if (lane >= o) incl += u;
    }
    const int total = __shfl(incl, 31, 32);
    int slot = incl - cnt;
    for (int j0 = b; j0 < e; j0 += 64) {
        unsigned long long m = j0 == b ? mask : chunk_mask(j0, min(j0 + 64, e));
        while (m) {
            const int k = __ffsll((long long)m) - 1;
            m &= m - 1;
            if (slot < c.list_cap) list_put(c, p.nl, slot, N, s, j0 + k, (int)d.off);
            ++slot;
        }
    }
    if (valid) {
        if (total > c.list_cap) atomicOr(&p.state[sys].err, ERR_OVERFLOW);
        if (lane == 0) p.nl_cnt[s] = total < c.list_cap ? total : c.list_cap;
    }
}

__global__ void __launch_bounds__(256) k_rb_list(Ctl c, DevPtrs p, SwParams sw, int S)
{
    const int nv = p.n_work[0] * S;
    for (int v = blockIdx.x; v < nv; v += gridDim.x) list_block(c, p, sw, p.work[v / S], v % S);
}


// ---------------------------------------------------------------- pass 1 ---
// Pair terms (energy, force, virial, parameter derivative: half per ordered
// pair), the three-body moments and the atom's own three-body energy.  R is
// the arithmetic type of the terms; sums are FP64.
// Moments a neighbour's gather needs, in term precision: v (3), then M
// (xx, yy, zz, xy, xz, yz).  s = tr M is not stored (|u| = 1), and q is not
// needed by the gather.
template <typename R>
struct Mom {
    R v[9];
};

// Term arithmetic.  FP32 terms use the hardware reciprocal, reciprocal
// square root, exponential and logarithm (about 1 ulp each, no IEEE
// correction steps); FP64 terms use the correctly rounded operations.
template <typename R>
struct Fm;

template <>
struct Fm<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    // distance and its inverse from the squared distance
    static __device__ __forceinline__ void dist(float r2, float &r, float &ri)
    {
        ri = __builtin_amdgcn_rsqf(r2);
        r = r2 * ri;
    }
    static __device__ __forceinline__ float exp(float x) { return __expf(x); }
    static __device__ __forceinline__ float log(float x) { return __logf(x); }
    static __device__ __forceinline__ float expm1(float x) { return ::expm1f(x); }
};

template <>
struct Fm<double> {
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ void dist(double r2, double &r, double &ri)
    {
        r = ::sqrt(r2);
        ri = 1.0 / r;
    }
    static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
    static __device__ __forceinline__ double log(double x) { return ::log(x); }
    static __device__ __forceinline__ double expm1(double x) { return ::expm1(x); }
};

// Gather batch sizes: list candidates (filter), short-list neighbours in
// pass 1 and in pass 2 (smaller where the registers are needed elsewhere).
constexpr int kBatchA = 8;
template <typename R, bool GRAD>
struct Batch {
    static constexpr int B = GRAD ? 2 : 4;
    static constexpr int P2 = sizeof(R) == 4 ? 4 : 2;
};

// lsl: [kLdsShort][blockDim.x] short-list entries in LDS
template <typename R, bool GRAD>
__device__ __forceinline__ void pass1_tile(const Ctl &c, const DevPtrs &p, const SwParams &sw, int ti, int32_t *lsl)
{
    const int lb = blockDim.x, lt = threadIdx.x;
    constexpr int NV = 20;  // E2, virial 9, dtheta 9, E3
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    const Tile tile = p.tiles[ti];
    const int sys = tile.sys;
    const SysState &st = p.state[sys];
    const int64_t N = c.n_total;

    if ((int)threadIdx.x < tile.count) {
        double box[3], ibox[3];
        eff_box(st, box, ibox);
        const int t = tile.start + threadIdx.x;
        const double4 xi = p.xs[t];
        // the first batch of list words loads together with the count
        uint32_t w0[kBatchA];
        list_load<kBatchA>(c, p.nl, 0, c.list_cap, N, t, w0);
        const int cnt = p.nl_cnt[t];
        const int off = (int)p.desc[sys].off;
        // Filter: the list candidates now within rc go to the short list.
        // It is cheap per candidate, so lanes whose candidates are mostly
        // outside rc do not hold the wave in the term evaluation below.
        int nin = 0;
        {
            // Conservative FP32 test: the rounding of the wrapped FP32
            // coordinates moves d^2 by far less than the margin, so every
            // pair within rc passes; the exact FP64 test follows in the
            // term loop, which also drops the few extra pairs.
            const float4 xif = p.xf[t];
            const float bx = (float)box[0], by = (float)box[1], bz = (float)box[2];
            const float ibx = (float)ibox[0], iby = (float)ibox[1], ibz = (float)ibox[2];
            const double bmax = fmax(box[0], fmax(box[1], box[2]));
            const float cut2 = (float)(sw.rc2 * (1.0 + 1e-3) + 32.0 * sw.rc * bmax * 1.1920928955078125e-7);
            // batches of kBatchA candidates: all their indices, then all
            // their positions, are in flight together
            for (int k0 = 0; k0 < cnt; k0 += kBatchA) {
                uint32_t w[kBatchA];
                if (k0 == 0) {
#pragma unroll
                    for (int u = 0; u < kBatchA; ++u) w[u] = w0[u];
                } else {
                    list_load<kBatchA>(c, p.nl, k0, cnt, N, t, w);
                }
                int jb[kBatchA];
                list_decode<kBatchA>(c, w, k0, cnt, t, off, jb);
                float4 xj[kBatchA];
#pragma unroll
                for (int u = 0; u < kBatchA; ++u) xj[u] = p.xf[jb[u]];
#pragma unroll
                for (int u = 0; u < kBatchA; ++u) {
                    float dx = xj[u].x - xif.x, dy = xj[u].y - xif.y, dz = xj[u].z - xif.z;
                    dx -= bx * rintf(dx * ibx);
                    dy -= by * rintf(dy * iby);
                    dz -= bz * rintf(dz * ibz);
                    if (k0 + u < cnt && dx * dx + dy * dy + dz * dz < cut2) {
                        if (nin < kLdsShort) lsl[nin * lb + lt] = jb[u];
                        else if (nin < kMaxShort) p.sl[(int64_t)nin * N + t] = jb[u];
                        ++nin;
                    }
                }
            }
        }
        const int ns = nin < kMaxShort ? nin : kMaxShort;
        const R rc = (R)sw.rc, sig = (R)sw.sig, eA = (R)sw.eA, B = (R)sw.B, pp = (R)sw.p,
                qq = (R)sw.q, gsig = (R)(sw.gam * sw.sig);
        double m[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        double F2x = 0, F2y = 0, F2z = 0;
        double vxx = 0, vyy = 0, vzz = 0, vxy = 0, vxz = 0, vyz = 0;
        // Terms over the short list, in batches whose indices and positions
        // are loaded together.
        int nkeep = 0;
        constexpr int kBatchB = Batch<R, GRAD>::B;
        for (int k0 = 0; k0 < ns; k0 += kBatchB) {
            int jb[kBatchB];
#pragma unroll
            for (int u = 0; u < kBatchB; ++u) {
                const int k = k0 + u < ns ? k0 + u : ns - 1;
                const int j = k < kLdsShort ? lsl[k * lb + lt] : p.sl[(int64_t)k * N + t];
                jb[u] = k0 + u < ns ? j : t;
            }
            double4 xjb[kBatchB];
#pragma unroll
            for (int u = 0; u < kBatchB; ++u) xjb[u] = p.xs[jb[u]];
#pragma unroll
            for (int u = 0; u < kBatchB; ++u) {
                if (k0 + u >= ns) break;
                const double4 xj = xjb[u];
                const double dx = min_image(xj.x - xi.x, box[0], ibox[0]);
                const double dy = min_image(xj.y - xi.y, box[1], ibox[1]);
                const double dz = min_image(xj.z - xi.z, box[2], ibox[2]);
                // exact membership; the kept entries form the global short
                // list of pass 2, in the Verlet list's entry format (16-bit
                // entries fill words 0 .. kMaxShort/2 - 1, below the rows
                // from kLdsShort on that this loop still reads; 32-bit
                // entries rewrite a row only after it has been read)
                if (!(dx * dx + dy * dy + dz * dz < sw.rc2)) continue;
                list_put(c, p.sl, nkeep, N, t, jb[u], off);
                ++nkeep;
                const R ddx = (R)dx, ddy = (R)dy, ddz = (R)dz;
                R r, ri;
                Fm<R>::dist(ddx * ddx + ddy * ddy + ddz * ddz, r, ri);
                const R ux = ddx * ri, uy = ddy * ri, uz = ddz * ri;
                // inside the cutoff in FP64 may round to r >= rc in the term
                // precision; the terms vanish there, so they are zeroed
                const R den = r - rc;
                const bool in = den < R(0);
                const R di = in ? Fm<R>::rcp(den) : R(0);
                const R sr = sig * ri;
                const R sp = powi_or_pow(sr, sw.ip, pp);
                const R sq = powi_or_pow(sr, sw.iq, qq);
                const R ex = in ? Fm<R>::exp(sig * di) : R(0);
                const R br = B * sp - sq;
                const R phi = eA * br * ex;
                const R dphi = eA * ex * ((qq * sq - pp * B * sp) * ri - br * sig * di * di);
                const R g = in ? Fm<R>::exp(gsig * di) : R(0);
                const R gx = g * ux, gy = g * uy, gz = g * uz;
                m[0] += (double)g;
                m[1] += (double)(g * g);
                m[2] += (double)gx;
                m[3] += (double)gy;
                m[4] += (double)gz;
                m[5] += (double)(gx * ux);
                m[6] += (double)(gy * uy);
                m[7] += (double)(gz * uz);
                m[8] += (double)(gx * uy);
                m[9] += (double)(gx * uz);
                m[10] += (double)(gy * uz);
                // F_i += phi2'(r) u_ij ; E_i += phi2/2 ; virial, half per ordered pair
                const R fx = dphi * ux, fy = dphi * uy, fz = dphi * uz;
                F2x += (double)fx;
                F2y += (double)fy;
                F2z += (double)fz;
                acc[0] += 0.5 * (double)phi;
                const R hr = R(0.5) * r;
                vxx += (double)(hr * fx * ux);
                vyy += (double)(hr * fy * uy);
                vzz += (double)(hr * fz * uz);
                vxy += (double)(hr * fx * uy);
                vxz += (double)(hr * fx * uz);
                vyz += (double)(hr * fy * uz);
                if (GRAD) {
                    const R lns = Fm<R>::log(sr);
                    acc[10] += 0.5 * (double)((R)sw.eps * br * ex);                   // A
                    acc[11] += 0.5 * (double)(eA * sp * ex);                          // B
                    acc[12] += 0.5 * (double)(eA * B * sp * lns * ex);                // p
                    acc[13] += 0.5 * (double)(-eA * sq * lns * ex);                   // q
                    acc[14] += 0.5 * (double)(phi * sig * sig * di * di);             // a
                    acc[17] += 0.5 * (double)(eA * ex * ((pp * B * sp - qq * sq) / sig + br * r * di * di));  // sigma
                    acc[18] += 0.5 * (double)((R)sw.A * br * ex);                     // epsilon
                }
            }
        }
        // the virial is symmetric: the tile partials hold its upper triangle
        // (slots yx, zx, zy stay zero; finalize mirrors them)
        acc[1] = vxx;
        acc[2] = vxy;
        acc[3] = vxz;
        acc[5] = vyy;
        acc[6] = vyz;
        acc[9] = vzz;
        // own three-body energy from the FP64 moments
        const double c0 = sw.cos0, omc = 1.0 - c0;
        const double MF = m[5] * m[5] + m[6] * m[6] + m[7] * m[7] + 2.0 * (m[8] * m[8] + m[9] * m[9] + m[10] * m[10]);
        const double vv = m[2] * m[2] + m[3] * m[3] + m[4] * m[4];
        const double Phi = MF - 2.0 * c0 * vv + c0 * c0 * m[0] * m[0] - omc * omc * m[1];
        acc[19] = 0.5 * sw.le * Phi;
        if (GRAD) {
            acc[15] = 0.5 * sw.eps * Phi;  // lambda_sw
            acc[18] += 0.5 * sw.lam * Phi; // epsilon (three-body part)
        }
        Mom<R> mo;
#pragma unroll
        for (int k = 0; k < 9; ++k) mo.v[k] = (R)m[k + 2];
        reinterpret_cast<Mom<R> *>(p.mom)[t] = mo;
        if (nin > kMaxShort) atomicOr(&p.state[sys].err, ERR_OVERFLOW);
        p.nnb[t] = nkeep;
        p.fs[t] = make_dvec3(F2x, F2y, F2z);
        if (!c.in_step) p.e_s[t] = acc[0] + acc[19];  // per-atom energies: force calls only
    }
    block_reduce<NV, GRAD ? kPass1GradSlots : kPass1Slots>(acc, p.part1 + (int64_t)ti * kNumPart);
}

template <typename R, bool GRAD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 2))) k_pass1(Ctl c, DevPtrs p, SwParams sw)
{
    extern __shared__ int32_t lsl[];
    const int ti = tile_of_block(c);
    if (ti >= 0) pass1_tile<R, GRAD>(c, p, sw, ti, lsl);
}

// ------------------------------------------------------ UF reference ---
// Uhlenbeck-Ford reference of the UF systems (section 4.1; model of Leite et
// al.): phi(r) = -p kB T ln(1 - exp(-(r/sigma)^2)) over each atom's whole
// list, half per ordered pair.  Writes the reference force of every atom and
// the tile's energy into its pass-1 row.  Launched only when a UF system is
// present; other tiles leave at once.
template <typename R>
__device__ __forceinline__ void uf_tile(const Ctl &c, const DevPtrs &p, int ti)
{
    const Tile tile = p.tiles[ti];
    const SysDesc &d = p.desc[tile.sys];
    if (d.mode != MODE_UF) return;
    const SysState &st = p.state[tile.sys];
    const int64_t N = c.n_total;
    double e = 0.0;
    if ((int)threadIdx.x < tile.count) {
        double box[3], ibox[3];
        eff_box(st, box, ibox);
        const int t = tile.start + threadIdx.x;
        const double4 xi = p.xs[t];
        const int cnt = p.nl_cnt[t];
        const double rc2 = d.uf_rc * d.uf_rc;
        const R pkT = (R)d.uf_pkT, is2 = (R)d.uf_is2;
        double fx = 0, fy = 0, fz = 0;
        for (int k0 = 0; k0 < cnt; k0 += kBatchA) {
            int jb[kBatchA];
            list_batch<kBatchA>(c, p.nl, k0, cnt, N, t, (int)d.off, jb);
            double4 xj[kBatchA];
#pragma unroll
            for (int u = 0; u < kBatchA; ++u) xj[u] = p.xs[jb[u]];
#pragma unroll
            for (int u = 0; u < kBatchA; ++u) {
                const double dx = min_image(xj[u].x - xi.x, box[0], ibox[0]);
                const double dy = min_image(xj[u].y - xi.y, box[1], ibox[1]);
                const double dz = min_image(xj[u].z - xi.z, box[2], ibox[2]);
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (k0 + u >= cnt || !(r2 < rc2)) continue;
                const R x = (R)r2 * is2;
                const R em = Fm<R>::exp(-x);
                const R om = -Fm<R>::expm1(-x);  // 1 - exp(-x)
                const R phi = -pkT * Fm<R>::log(om);
                const R g = -pkT * R(2) * is2 * em / om;  // phi'(r) / r
                fx += (double)(g * (R)dx);
                fy += (double)(g * (R)dy);
                fz += (double)(g * (R)dz);
                e += 0.5 * (double)phi;
            }
        }
        p.fref[t] = make_dvec3(fx, fy, fz);
    }
    double acc[1] = {e};
    block_reduce<1>(acc, p.part1 + (int64_t)ti * kNumPart + P_UUF);
}

template <typename R>
__global__ void __launch_bounds__(256) k_uf(Ctl c, DevPtrs p)
{
    const int ti = tile_of_block(c);
    if (ti >= 0) uf_tile<R>(c, p, ti);
}

// ---------------------------------------------------------------- pass 2 ---
// d E3_c / d r_cj for a centre with moments (s, q, v, M) and a neighbour at
// unit vector u, distance r, g = g(r), dg = g'(r):
//   (le/2) [ dg H u + (4 g / r) ((M u - (u.M.u) u) - c0 (v - (v.u) u)) ],
//   H = 2 u.M.u - 4 c0 v.u + 2 c0^2 s - 2 (1 - c0)^2 g,
// evaluated as alpha u + beta (M u - c0 v) with
//   alpha = (le/2) (dg H - (4 g / r) (u.M.u - c0 v.u)),  beta = (le/2) 4 g / r.
// hdg = (le/2) dg and hb = beta are shared by both ends of a pair.
template <typename R>
__device__ __forceinline__ void d_e3(const R *mom, R ux, R uy, R uz, R g, R hdg, R hb, R c0, R out[3], R &H)
{
    const R vx = mom[0], vy = mom[1], vz = mom[2];
    const R Mxx = mom[3], Myy = mom[4], Mzz = mom[5], Mxy = mom[6], Mxz = mom[7], Myz = mom[8];
    const R s = Mxx + Myy + Mzz;  // sum g (u.u = 1)
    const R mux = Mxx * ux + Mxy * uy + Mxz * uz;
    const R muy = Mxy * ux + Myy * uy + Myz * uz;
    const R muz = Mxz * ux + Myz * uy + Mzz * uz;
    const R umu = ux * mux + uy * muy + uz * muz;
    const R vu = vx * ux + vy * uy + vz * uz;
    const R omc = R(1) - c0;
    H = R(2) * umu - R(4) * c0 * vu + R(2) * c0 * c0 * s - R(2) * omc * omc * g;
    const R alpha = hdg * H - hb * (umu - c0 * vu);
    out[0] = alpha * ux + hb * (mux - c0 * vx);
    out[1] = alpha * uy + hb * (muy - c0 * vy);
    out[2] = alpha * uz + hb * (muz - c0 * vz);
}

// ---- per-group reduction and scalar update (last tile of a group) --------
constexpr double kGpaPerEvA3 = 1.602176634e-19 / 1e-30 / 1e9;

__device__ double progress(const SysDesc &d, int64_t k)
{
    if (d.s_steps <= 0) return 1.0;
    const int64_t kk = k < d.s_steps ? k : d.s_steps;
    return (double)kk / (double)d.s_steps;
}

__device__ double controlled(const SysDesc &d, int64_t k)
{
    return d.s_start + (d.s_end - d.s_start) * progress(d, k);
}

// lambda- and P_S-dependent part of H at the current microstate
__device__ double h_switch(const SysDesc &d, const SysState &st, double lam, double Ps)
{
    switch (d.mode) {
        case MODE_FL:
        case MODE_UF: return lam * st.U_int + (1.0 - lam) * st.U_ref;
        case MODE_RS:
        case MODE_DCCI_T:
        case MODE_DCCI_P: return lam * st.U_int + Ps * st.V;
        case MODE_AS_P: return Ps * st.V;
        default: return 0.0;
    }
}

// Barostat half step (MTK).  One piston of mass W for eps = ln L:
//   dv/dt = [alpha 2K - tr Xi - 3 V P_S] / W,  alpha = 1 + 3/N_f;
// or one piston per axis (eps_a = ln L_a), of mass W/3 so that equal axis
// stresses move the three axes as the single piston:
//   dv_a/dt = [2K_a + 2K/N_f - Xi_aa - V P_S] / (W/3).
__device__ void baro_half(const SysDesc &d, SysState &st, double dt)
{
    if (d.p_damp <= 0.0 || d.mode == MODE_FORCE) return;
    const double ls = scales_interaction(d.mode) ? st.lam : 1.0;
    if (d.baro) {
        for (int a = 0; a < 3; ++a) {
            const double xi = ls * st.vir[4 * a];
            const double g = 2.0 * st.K3[a] + 2.0 * st.K / d.nf - xi - st.V * st.Ps;
            st.veps[a] += 0.5 * dt * g / (d.wpiston / 3.0);
        }
        return;
    }
    double tr = st.vir[0] + st.vir[4] + st.vir[8];
    if (scales_interaction(d.mode)) tr = st.lam * tr;
    const double g = d.alpha * 2.0 * st.K - tr - 3.0 * st.V * st.Ps;
    const double v = st.veps[0] + 0.5 * dt * g / d.wpiston;
    st.veps[0] = st.veps[1] = st.veps[2] = v;
}

// dCCI coupling (section 3): next (lambda, P_S) of a pair from instantaneous
// per-atom energy and volume differences; returns false when singular.
__device__ bool dcci_next(const SysDesc &dI, const SysState &I, const SysDesc &dII, const SysState &II,
                          double &lam_new, double &Ps_new)
{
    const double du = I.U_int / (double)dI.n - II.U_int / (double)dII.n;
    const double dv = I.V / (double)dI.n - II.V / (double)dII.n;
    lam_new = I.lam;
    Ps_new = I.Ps;
    if (fabs(dv) < 1e-6) return false;
    double l, P;
    if (dI.mode == MODE_DCCI_T) {
        // eq. Ps_coex_discreted with T linear and lambda = T0/T
        l = dI.T0 / controlled(dI, I.k + 1);
        P = I.Ps - (l - I.lam) * du / dv;
    } else {
        // eq. l_coex_discreted with P linear, then P_S = lambda P (eq. P_sc)
        const double Pk = controlled(dI, I.k) / kGpaPerEvA3;
        const double Pk1 = controlled(dI, I.k + 1) / kGpaPerEvA3;
        if (du == 0.0) return false;
        const double den = 1.0 + Pk1 * dv / du;
        if (fabs(den) < 1e-3) return false;
        l = I.lam * (1.0 + Pk * dv / du) / den;
        P = l * Pk1;
    }
    if (!(l > 0.05 && l < 20.0)) return false;
    lam_new = l;
    Ps_new = P;
    return true;
}

__device__ void next_lambda(const SysDesc &d, const SysState &st, double &lam, double &Ps)
{
    lam = st.lam;
    Ps = st.Ps;
    if (d.mode == MODE_FL || d.mode == MODE_UF) {
        lam = controlled(d, st.k + 1);
        Ps = 0.0;
    } else if (d.mode == MODE_RS) {
        const double f = progress(d, st.k + 1);
        const double inv = 1.0 / d.s_start + (1.0 / d.s_end - 1.0 / d.s_start) * f;
        lam = 1.0 / inv;
        Ps = lam * d.pressure;
    } else if (d.mode == MODE_AS_P) {
        lam = 1.0;
        Ps = controlled(d, st.k + 1) / kGpaPerEvA3;
    }
}

__device__ void apply_switch(const SysDesc &d, SysState &st, double lam, double Ps)
{
    st.W += h_switch(d, st, lam, Ps) - h_switch(d, st, st.lam, st.Ps);
    st.lam = lam;
    st.Ps = Ps;
}

// integrator factors for the coming step; moves the box to its post-drift size
__device__ void step_factors(const SysDesc &d, SysState &st, double dt, double rc)
{
    // velocities: dv_a/dt = F_a/m - (v_eps,a + tr v_eps / N_f) v_a; positions:
    // dx_a/dt = v_a + v_eps,a x_a; both exact over a half step
    // (a zero rate gives factors of exactly 1, and equal rates equal
    // factors: the exponentials are evaluated once per distinct axis rate)
    const double tr = st.veps[0] + st.veps[1] + st.veps[2];
    for (int a = 0; a < 3; ++a) {
        const double zk = d.baro ? (st.veps[a] + tr / d.nf) * 0.5 * dt : d.alpha * st.veps[a] * 0.5 * dt;
        const double za = st.veps[a] * 0.5 * dt;
        if (a > 0 && zk == (d.baro ? (st.veps[a - 1] + tr / d.nf) * 0.5 * dt : d.alpha * st.veps[a - 1] * 0.5 * dt) &&
            za == st.veps[a - 1] * 0.5 * dt) {
            st.decay[a] = st.decay[a - 1];
            st.phi[a] = st.phi[a - 1];
            st.grow[a] = st.grow[a - 1];
            st.psi[a] = st.psi[a - 1];
            continue;
        }
        st.decay[a] = zk == 0.0 ? 1.0 : exp(-zk);
        st.phi[a] = zk == 0.0 ? 1.0 : -expm1(-zk) / zk;
        st.grow[a] = za == 0.0 ? 1.0 : exp(za);
        st.psi[a] = za == 0.0 ? 1.0 : expm1(za) / za;
    }
    if (d.mode != MODE_FORCE)
        for (int k = 0; k < 3; ++k) st.box[k] = (st.box[k] * st.grow[k]) * st.grow[k];
    for (int k = 0; k < 3; ++k)
        if (!(st.box[k] >= 2.0 * rc)) st.err |= ERR_BOX;
}

// Start of a step for a group (one system, or a dCCI pair when d1 and s1
// are given): switch (1), barostat half step (2), factors.
__device__ void group_start_step(const Ctl &c, const SwParams &sw, const SysDesc &d0, SysState &s0,
                                 const SysDesc *d1, SysState *s1)
{
    double lam, Ps;
    if (s1) {
        if (!dcci_next(d0, s0, *d1, *s1, lam, Ps)) {
            s0.err |= ERR_DCCI;
            s1->err |= ERR_DCCI;
        }
    } else {
        next_lambda(d0, s0, lam, Ps);
    }
    apply_switch(d0, s0, lam, Ps);
    baro_half(d0, s0, c.dt);
    step_factors(d0, s0, c.dt, sw.rc);
    if (s1) {
        apply_switch(*d1, *s1, lam, Ps);
        baro_half(*d1, *s1, c.dt);
        step_factors(*d1, *s1, c.dt, sw.rc);
    }
}

// Cooperative copy of n bytes (a multiple of 4) by the threads of a block.
__device__ __forceinline__ void block_copy(void *dst, const void *src, int n)
{
    for (int w = threadIdx.x; w < n / 4; w += blockDim.x)
        static_cast<int32_t *>(dst)[w] = static_cast<const int32_t *>(src)[w];
}

// The sums of one system into its state, the outputs of a force call, and
// at the end of a dynamics step the closing barostat half step (step 9),
// the counters and the log row.  Returns the steps left in the call (0
// outside a step).
__device__ __forceinline__ int64_t finish_system(const Ctl &c, const DevPtrs &p, const SysDesc &d, SysState &st,
                                                 const double *a, const double *b, int s, bool step_end)
{
    int64_t remaining = 0;
    st.E2 = a[P_E];
    st.E3 = a[P_E3];
    st.U_int = st.E2 + st.E3;
    for (int m = 0; m < 9; ++m) st.vir[m] = a[P_VIR + m] + b[P_VIR + m];
    st.vir[3] = st.vir[1];  // lower triangle from the upper one
    st.vir[6] = st.vir[2];
    st.vir[7] = st.vir[5];
    for (int m = 0; m < 9; ++m) st.dth[m] = a[P_DTH + m] + b[P_DTH + m];
    st.U_ref = b[P_UREF] + (d.mode == MODE_UF ? a[P_UUF] : 0.0);
    for (int m = 0; m < 3; ++m) st.K3[m] = b[P_K + m];
    st.K = (st.K3[0] + st.K3[1]) + st.K3[2];
    for (int m = 0; m < 3; ++m) st.noise_mean[m] = b[P_NOISE + m] / (double)d.n;
    st.V = st.box[0] * st.box[1] * st.box[2];
    if (!isfinite(st.U_int) || !isfinite(st.K) || !isfinite(st.vir[0] + st.vir[4] + st.vir[8]))
        st.err |= ERR_NONFINITE;
    if (p.out) {
        // dE/dstrain at diagonal strain e: Xi' (I + e)^-T
        const double gsc = p.grad_scale ? p.grad_scale[s] : 1.0;
        double *o = p.out + (int64_t)s * 20;
        o[0] = st.U_int;
        o[1] = st.U_ref;
        for (int u = 0; u < 3; ++u)
            for (int w = 0; w < 3; ++w) o[2 + 3 * u + w] = st.vir[3 * u + w] / st.pscale[w] * gsc;
        for (int m = 0; m < 9; ++m) o[11 + m] = st.dth[m] * gsc;
    }
    if (step_end) {
        baro_half(d, st, c.dt);  // step 9
        st.step += 1;
        st.k += 1;
        st.remaining -= 1;
        remaining = st.remaining;
        if (c.log_every > 0 && c.log_cap > 0 && (st.step % c.log_every) == 0) {
            const int64_t row = ((st.step / c.log_every) * c.n_sys + s) % c.log_cap;
            double *L = p.log + row * 8;
            L[0] = (double)st.step;
            L[1] = st.lam;
            L[2] = st.Ps * kGpaPerEvA3;
            L[3] = st.lam != 0.0 ? st.Ps / st.lam * kGpaPerEvA3 : 0.0;
            L[4] = 2.0 * st.K / (d.nf * 8.617333262e-5);
            L[5] = st.U_int / (double)d.n;
            L[6] = st.V / (double)d.n;
            L[7] = st.W;
        }
    }
    return remaining;
}

// Reductions of one group over its tiles in a fixed order (all threads of
// the block), then the scalar update by thread 0 on copies of the group's
// descriptors and states held in LDS (one load and one store of each field
// instead of a chain of dependent global accesses), written back at the end.
__device__ void group_finalize(const Ctl &c, const DevPtrs &p, const SwParams &sw, const Group &G)
{
    static_assert(sizeof(SysState) % 4 == 0 && sizeof(SysDesc) % 4 == 0, "word copies");
    __shared__ double red[4][64];
    __shared__ double sums[2][2 * kNumPart];
    __shared__ SysState sst[2];
    __shared__ SysDesc sdesc[2];
    const int nq = G.s1 >= 0 ? 2 : 1;
    const int sid[2] = {G.s0, G.s1};
    for (int q = 0; q < nq; ++q) {
        block_copy(&sst[q], &p.state[sid[q]], sizeof(SysState));
        block_copy(&sdesc[q], &p.desc[sid[q]], sizeof(SysDesc));
    }
    // Four partial sums per slot, over the tiles of each residue mod 4, in
    // rounds of sixteen independent loads in flight (the last one padded with
    // zeros), then added in order: the same summation order whatever the
    // block's wave count (a wave takes several residues when fewer than four).
    constexpr int NJ = 4;
    const int k = threadIdx.x & 63, j = threadIdx.x >> 6, nj = blockDim.x >> 6;
    for (int q = 0; q < nq; ++q) {
        const SysDesc &d = p.desc[sid[q]];
        for (int jj = j; jj < NJ; jj += nj) {
            double a = 0.0;
            if (k < 2 * kNumPart) {
                const double *src = k < kNumPart ? p.part1 + k : p.part2 + (k - kNumPart);
                for (int t = d.tile_begin + jj; t < d.tile_end; t += 16 * NJ) {
                    double v[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u)
                        v[u] = t + u * NJ < d.tile_end ? src[(int64_t)(t + u * NJ) * kNumPart] : 0.0;
#pragma unroll
                    for (int u = 0; u < 16; ++u) a += v[u];
                }
            }
            red[jj][k] = a;
        }
        __syncthreads();
        if (j == 0 && k < 2 * kNumPart) {
            double s = 0.0;
            for (int w = 0; w < NJ; ++w) s += red[w][k];
            sums[q][k] = s;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const bool step_end = c.in_step != 0;
        if (nq == 1) {
            // one system: the scalar chain runs on a register copy of its
            // state (no LDS round trip per field)
            SysState st = sst[0];
            const int64_t remaining = finish_system(c, p, sdesc[0], st, sums[0], sums[0] + kNumPart, sid[0], step_end);
            if (step_end && remaining > 0) group_start_step(c, sw, sdesc[0], st, nullptr, nullptr);
            sst[0] = st;
        } else {
            int64_t remaining = 0;
            for (int q = 0; q < 2; ++q)
                remaining = finish_system(c, p, sdesc[q], sst[q], sums[q], sums[q] + kNumPart, sid[q], step_end);
            if (step_end && remaining > 0) group_start_step(c, sw, sdesc[0], sst[0], &sdesc[1], &sst[1]);
        }
    }
    __syncthreads();
    for (int q = 0; q < nq; ++q) block_copy(&p.state[sid[q]], &sst[q], sizeof(SysState));
    __syncthreads();  // the LDS copies may be written again by the block's next group
}

// Normals of atom t's next O step: stored in zs and added to the tile's
// noise sums.
template <int NV>
__device__ __forceinline__ void next_normals(const Ctl &c, const SysDesc &d, const SysState &st, int t, int atom,
                                             dvec3 *zs, double (&acc)[NV])
{
    double z[3];
    normals3(c.seed, d.stream, (uint64_t)(st.step + c.in_step), (uint64_t)atom, z);
    zs[t] = make_dvec3(z[0], z[1], z[2]);
    acc[P_NOISE] = z[0];
    acc[P_NOISE + 1] = z[1];
    acc[P_NOISE + 2] = z[2];
}

template <typename R, bool GRAD>
__device__ __forceinline__ void pass2_tile(const Ctl &c, const DevPtrs &p, const SwParams &sw, int ti)
{
    constexpr int NV = kNumPart;  // -, virial 9, dtheta 9, U_ref, K per axis 3, noise 3
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    const Tile tile = p.tiles[ti];
    const int sys = tile.sys;
    const SysDesc &d = p.desc[sys];
    const SysState &st = p.state[sys];
    const int64_t N = c.n_total;

    if ((int)threadIdx.x < tile.count) {
        double box[3], ibox[3];
        eff_box(st, box, ibox);
        const int t = tile.start + threadIdx.x;
        const double4 xa = p.xs[t];
        const Mom<R> *mom = reinterpret_cast<const Mom<R> *>(p.mom);
        const Mom<R> mA = mom[t];
        // per-atom operands of the tail, in flight during the gather
        const dvec3 F2 = p.fs[t];
        const dvec3 v0 = p.vs[t];
        const dvec3 x0 = d.mode == MODE_FL ? p.x0s[t] : make_dvec3(0, 0, 0);
        // the first batch of short-list entries loads together with its count
        constexpr int kBatch2 = Batch<R, GRAD>::P2;
        uint32_t s0[kBatch2];
        list_load<kBatch2>(c, p.sl, 0, kMaxShort, N, t, s0);
        const int cnt = p.nnb[t];
        const int atom = p.perm[t] - d.off;
        // normals of the next O step (stored for it, and summed for its
        // zero-sum correction), drawn while the operands above load; the
        // gradient variant draws them at the end, where registers are free
        if (!GRAD && o_step_on(d)) next_normals(c, d, st, t, atom, p.zs, acc);
        const R rc = (R)sw.rc, gsig = (R)(sw.gam * sw.sig), c0 = (R)sw.cos0, hle = (R)(0.5 * sw.le);
        double F3x = 0, F3y = 0, F3z = 0;
        double vxx = 0, vyy = 0, vzz = 0, vxy = 0, vxz = 0, vyz = 0;
        double gg = 0, ga = 0, gs = 0;  // sum H g dln g/d(gamma, a, sigma)
        // the neighbours within rc that pass 1 found at these positions, in
        // batches whose indices, positions and moments are loaded together
        for (int k0 = 0; k0 < cnt; k0 += kBatch2) {
            int jb[kBatch2];
            if (k0 == 0) list_decode<kBatch2>(c, s0, 0, cnt, t, (int)d.off, jb);
            else list_batch<kBatch2>(c, p.sl, k0, cnt, N, t, (int)d.off, jb);
            double4 xjb[kBatch2];
            Mom<R> mjb[kBatch2];
#pragma unroll
            for (int u = 0; u < kBatch2; ++u) {
                xjb[u] = p.xs[jb[u]];
                mjb[u] = mom[jb[u]];
            }
#pragma unroll
            for (int u = 0; u < kBatch2; ++u) {
                if (k0 + u >= cnt) break;
                const double4 xj = xjb[u];
                const Mom<R> &mJ = mjb[u];
                const double dx = min_image(xj.x - xa.x, box[0], ibox[0]);
                const double dy = min_image(xj.y - xa.y, box[1], ibox[1]);
                const double dz = min_image(xj.z - xa.z, box[2], ibox[2]);
                const R ddx = (R)dx, ddy = (R)dy, ddz = (R)dz;
                R r, ri;
                Fm<R>::dist(ddx * ddx + ddy * ddy + ddz * ddz, r, ri);
                const R ux = ddx * ri, uy = ddy * ri, uz = ddz * ri;
                const R den = r - rc;
                const bool in = den < R(0);
                const R di = in ? Fm<R>::rcp(den) : R(0);
                const R g = in ? Fm<R>::exp(gsig * di) : R(0);
                const R hdg = -hle * g * gsig * di * di;  // (le/2) g'(r)
                const R hb = R(4) * hle * g * ri;
                R tA[3], tJ[3], HA, HJ;
                d_e3<R>(mA.v, ux, uy, uz, g, hdg, hb, c0, tA, HA);
                d_e3<R>(mJ.v, -ux, -uy, -uz, g, hdg, hb, c0, tJ, HJ);
                F3x += (double)(tA[0] - tJ[0]);
                F3y += (double)(tA[1] - tJ[1]);
                F3z += (double)(tA[2] - tJ[2]);
                vxx += (double)(tA[0] * ddx);
                vyy += (double)(tA[1] * ddy);
                vzz += (double)(tA[2] * ddz);
                vxy += (double)(R(0.5) * (tA[0] * ddy + tA[1] * ddx));
                vxz += (double)(R(0.5) * (tA[0] * ddz + tA[2] * ddx));
                vyz += (double)(R(0.5) * (tA[1] * ddz + tA[2] * ddy));
                if (GRAD) {
                    const R hg = HA * g;
                    gg += (double)(hg * (R)sw.sig * di);
                    ga += (double)(hg * gsig * (R)sw.sig * di * di);
                    gs += (double)(hg * (R)sw.gam * r * di * di);
                }
            }
        }
        // the virial is symmetric: the tile partials hold its upper triangle
        // (slots yx, zx, zy stay zero; finalize mirrors them)
        acc[1] = vxx;
        acc[2] = vxy;
        acc[3] = vxz;
        acc[5] = vyy;
        acc[6] = vyz;
        acc[9] = vzz;
        if (GRAD) {
            const double hl = 0.5 * sw.le;
            acc[14] = hl * ga;  // a
            acc[16] = hl * gg;  // gamma
            acc[17] = hl * gs;  // sigma
        }
        dvec3 F = F2;
        F.x += F3x;
        F.y += F3y;
        F.z += F3z;
        p.fs[t] = F;
        // Einstein reference (Frenkel-Ladd systems)
        if (d.mode == MODE_FL) {
            const double ex = xa.x - x0.x, ey = xa.y - x0.y, ez = xa.z - x0.z;
            acc[19] = 0.5 * d.k_spring * (ex * ex + ey * ey + ez * ez);
        }
        // final half kick of a dynamics step, then the kinetic energy
        dvec3 v = v0;
        if (c.in_step && d.mode != MODE_FORCE) {
            const double ka = (0.5 * c.dt) * d.acc;
            const dvec3 fr = d.mode == MODE_UF ? p.fref[t] : make_dvec3(0, 0, 0);
            v.x = v.x * st.decay[0] + ka * total_force(d.mode, st.lam, F.x, xa.x, x0.x, d.k_spring, fr.x) * st.phi[0];
            v.y = v.y * st.decay[1] + ka * total_force(d.mode, st.lam, F.y, xa.y, x0.y, d.k_spring, fr.y) * st.phi[1];
            v.z = v.z * st.decay[2] + ka * total_force(d.mode, st.lam, F.z, xa.z, x0.z, d.k_spring, fr.z) * st.phi[2];
            p.vs[t] = v;
        }
        acc[P_K] = d.mvv2e_m * (v.x * v.x);
        acc[P_K + 1] = d.mvv2e_m * (v.y * v.y);
        acc[P_K + 2] = d.mvv2e_m * (v.z * v.z);
        if (GRAD && o_step_on(d)) next_normals(c, d, st, t, atom, p.zs, acc);
    }
    block_reduce<NV, GRAD ? kPass2GradSlots : kPass2Slots>(acc, p.part2 + (int64_t)ti * kNumPart);
}

template <typename R, bool GRAD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 2))) k_pass2(Ctl c, DevPtrs p, SwParams sw)
{
    const int ti = tile_of_block(c);
    if (ti >= 0) pass2_tile<R, GRAD>(c, p, sw, ti);
}

// One block per group: fixed-order reductions of the group's tiles and the
// scalar update (barostat, switch and work, dCCI coupling, next factors).
__global__ void __launch_bounds__(256) k_finalize(Ctl c, DevPtrs p, SwParams sw)
{
    const Group G = p.groups[blockIdx.x];
    group_finalize(c, p, sw, G);
}

// Start-of-call prologue: steps left, then the start of the first step.
__global__ void k_begin_step(Ctl c, DevPtrs p, SwParams sw, int64_t n_steps)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= c.n_groups) return;
    const Group G = p.groups[g];
    p.state[G.s0].remaining = n_steps;
    if (G.s1 >= 0) p.state[G.s1].remaining = n_steps;
    const bool pair = G.s1 >= 0;
    group_start_step(c, sw, p.desc[G.s0], p.state[G.s0], pair ? &p.desc[G.s1] : nullptr,
                     pair ? &p.state[G.s1] : nullptr);
}

// Reset of every system's schedule state (lambda, P_S, work, schedule step)
// from its descriptor; used at set-up and when a new schedule is installed.
__global__ void k_reset_schedule(Ctl c, DevPtrs p)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= c.n_sys) return;
    const SysDesc &d = p.desc[s];
    SysState &st = p.state[s];
    switch (d.mode) {
        case MODE_FL:
        case MODE_UF: st.lam = d.s_start; st.Ps = 0.0; break;
        case MODE_RS: st.lam = d.s_start; st.Ps = st.lam * d.pressure; break;
        case MODE_AS_P: st.lam = 1.0; st.Ps = d.s_start / kGpaPerEvA3; break;
        case MODE_DCCI_T: st.lam = d.T0 / d.s_start; st.Ps = st.lam * d.pressure; break;
        case MODE_DCCI_P: st.lam = 1.0; st.Ps = d.s_start / kGpaPerEvA3; break;
        default: st.lam = 1.0; st.Ps = d.pressure; break;
    }
    st.W = 0.0;
    st.k = 0;
}

// Diagonal strain for the next force evaluation (NULL: none).
__global__ void k_set_pscale(Ctl c, DevPtrs p, const double *diag)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= c.n_sys) return;
    for (int k = 0; k < 3; ++k) p.state[s].pscale[k] = diag ? 1.0 + diag[3 * s + k] : 1.0;
}

// Zero n 32-bit words (a kernel rather than a memset, so that a caller may
// capture the call).
__global__ void k_zero_words(uint32_t *w, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        w[i] = 0u;
}

__global__ void k_clear_err(Ctl c, DevPtrs p)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < c.n_sys) p.state[s].err = 0;
}

// ------------------------------------------------------- persistent step ---
// One cooperative launch runs n_steps whole steps.  The systems are dealt to
// the XCDs beforehand (whole reduction groups, by cost); each workgroup reads
// the XCD it runs on from the hardware and steps only that XCD's systems,
// meeting the XCD's other workgroups at barriers between the stages of a
// step.  During the kernel a system's data is written and read only by
// workgroups of its own XCD, whose L2 they share: a barrier needs the
// arrivals' stores complete in that L2 (the L1 writes through) and each
// arriving CU's L1 invalidated, but no L2 write-back.  Every wait is bounded:
// a wait that gives up raises the abort word, every workgroup then leaves,
// and the check kernel that follows marks every system with ERR_PERSIST.
constexpr long kSpinLimit = 1L << 22;  // polls of one wait (seconds) before giving up

__device__ __forceinline__ unsigned long long ld_agent(unsigned long long *w)
{
    return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void add_agent(unsigned long long *w, unsigned long long v)
{
    __hip_atomic_fetch_add(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0: wait until *w >= target; false when the kernel is abandoned.
__device__ bool wait_at_least(unsigned long long *w, unsigned long long target, unsigned long long *abort_w)
{
    long spins = 0;
    while (ld_agent(w) < target) {
        if (ld_agent(abort_w)) return false;
        if (++spins > kSpinLimit) {
            __hip_atomic_store(abort_w, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

// Barrier of the nb workgroups of one XCD (counter ctr, reaching target).
__device__ bool xcd_barrier(unsigned long long *ctr, unsigned long long target, unsigned long long *abort_w,
                            int nb, int *flag_s)
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        bool ok = true;
        if (nb > 1) {
            add_agent(ctr, 1ull);
            ok = wait_at_least(ctr, target, abort_w);
            // device-scope invalidate: the CU's L1 (a group-scope invalidate
            // leaves it when a workgroup is not split across CUs).  A lone
            // workgroup reads only what its own CU wrote and needs none.
            asm volatile("buffer_inv sc1\n\ts_waitcnt vmcnt(0)" ::: "memory");
        }
        *flag_s = ok ? 1 : 0;
    }
    __syncthreads();
    return *flag_s != 0;
}

// In-place exclusive prefix of a[0 .. n) in LDS by all threads of a block
// (at most 256); a[n] receives the total.
__device__ void block_exclusive_scan(int32_t *a, int n)
{
    __shared__ int32_t part[256];
    const int tid = threadIdx.x, nth = blockDim.x;
    const int per = (n + nth - 1) / nth;
    const int lo = min(tid * per, n), hi = min(lo + per, n);
    int sum = 0;
    for (int q = lo; q < hi; ++q) sum += a[q];
    part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < nth; o <<= 1) {
        const int add = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
    }
    int run = part[tid] - sum;
    for (int q = lo; q < hi; ++q) {
        const int v = a[q];
        a[q] = run;
        run += v;
    }
    if (tid == nth - 1) a[n] = part[nth - 1];
    __syncthreads();
}

// Two waves per SIMD in both precisions: the whole step in one function
// needs the registers (at four waves the FP32 variant spilled 496 bytes per
// lane to scratch and ran the 64-replica batch at 366 us per step against
// 231 us here).
template <typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_persist(Ctl c, DevPtrs p, SwParams sw, XcdPlan xp, int64_t n_steps)
{
    extern __shared__ int32_t lsl[];  // pass 1's short list; the list stage's tile tables
    __shared__ int s_flag, s_x, s_j, s_nb, s_any;
    __shared__ unsigned char s_stale[kPersistMaxSysPerXcd];
    unsigned long long *sync = p.sync;
    unsigned long long *abort_w = sync + SYNC_ABORT;
    // start-up: each workgroup joins the XCD it runs on
    if (threadIdx.x == 0) {
        unsigned v;
        asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(v));
        const int x = (int)(v & 0xFu);
        int ok = x < kXcds ? 1 : 0;
        int j = 0;
        if (ok) j = (int)__hip_atomic_fetch_add(sync + SYNC_REG + x, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else __hip_atomic_store(abort_w, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        add_agent(sync + SYNC_START, 1ull);
        if (!wait_at_least(sync + SYNC_START, gridDim.x, abort_w) || ld_agent(abort_w)) ok = 0;
        // every XCD that owns systems needs workgroups
        for (int y = 0; y < kXcds && ok; ++y)
            if (xp.tile_off[y + 1] > xp.tile_off[y] && ld_agent(sync + SYNC_REG + y) == 0) ok = 0;
        if (!ok) __hip_atomic_store(abort_w, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_x = ok ? x : 0;
        s_j = j;
        s_nb = ok ? (int)ld_agent(sync + SYNC_REG + x) : 0;
        s_flag = ok;
    }
    __syncthreads();
    if (!s_flag) return;
    const int x = s_x, j = s_j, nb = s_nb;
    const int tb = xp.tile_off[x], te = xp.tile_off[x + 1];
    if (tb == te) return;  // this XCD owns no systems
    const int gb = xp.group_off[x], ge = xp.group_off[x + 1];
    const int sb = xp.sys_off[x], se = xp.sys_off[x + 1];
    unsigned long long *ctr = sync + SYNC_XCD + 16 * x;
    unsigned long long epoch = 0;
    const int apb = (int)(blockDim.x >> 5);  // atoms per list-build share
    int32_t *lpref = lsl;  // the list stage's share table (at most kLdsShort * blockDim - 1 tiles)
#define SWFE_XCD_SYNC()                                                          \
    if (!xcd_barrier(ctr, ++epoch * (unsigned long long)nb, abort_w, nb, &s_flag)) \
        break
    for (int64_t step = 0; step < n_steps; ++step) {
        for (int i = tb + j; i < te; i += nb) integrate_tile(c, p, sw, p.xtiles[i]);
        SWFE_XCD_SYNC();
        // rebuild decisions of the XCD's systems, taken by every block from
        // the same state (nothing they read changes before the count stage)
        if (threadIdx.x == 0) s_any = 0;
        __syncthreads();
        for (int q = sb + (int)threadIdx.x; q < se; q += blockDim.x) {
            const bool rb = list_stale(c, p, sw, p.xsys[q]);
            s_stale[q - sb] = rb ? 1 : 0;
            if (rb) s_any = 1;
        }
        // the displacement slot the next step's integrate fills starts at zero
        if (threadIdx.x == 0)
            for (int q = sb + j; q < se; q += nb) {
                const int sys = p.xsys[q];
                p.disp_max[2 * sys + ((p.state[sys].step + 1) & 1)] = 0.0;
            }
        __syncthreads();
        if (s_any) {
            for (int i = tb + j; i < te; i += nb)
                if (s_stale[p.xtloc[i]]) rb_count_tile(p, sw, p.xtiles[i]);
            SWFE_XCD_SYNC();
            for (int q = sb + j; q < se; q += nb)
                if (s_stale[q - sb]) rb_scan_sys<256>(c, p, sw, p.xsys[q], true, false);
            SWFE_XCD_SYNC();
            for (int i = tb + j; i < te; i += nb)
                if (s_stale[p.xtloc[i]]) rb_scatter_tile(p, p.xtiles[i], nullptr);
            SWFE_XCD_SYNC();
            for (int i = tb + j; i < te; i += nb)
                if (s_stale[p.xtloc[i]]) rb_order_tile(p, p.xtiles[i]);
            SWFE_XCD_SYNC();
            // list-build shares of the XCD's tiles (none for a tile whose
            // list stays), and their exclusive prefix, in LDS
            const int nt = te - tb;
            for (int i = threadIdx.x; i < nt; i += blockDim.x)
                lpref[i] = s_stale[p.xtloc[tb + i]] ? (p.tiles[p.xtiles[tb + i]].count + apb - 1) / apb : 0;
            __syncthreads();
            block_exclusive_scan(lpref, nt);
            const int nv = lpref[nt];
            for (int v = j; v < nv; v += nb) {
                int lo = 0, hi = nt - 1;  // the last tile whose shares start at or before v
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (lpref[mid] <= v) lo = mid;
                    else hi = mid - 1;
                }
                list_block(c, p, sw, p.xtiles[tb + lo], v - lpref[lo]);
            }
            SWFE_XCD_SYNC();
        }
        for (int i = tb + j; i < te; i += nb) {
            const int ti = p.xtiles[i];
            pass1_tile<R, false>(c, p, sw, ti, lsl);
            if (c.has_uf) uf_tile<R>(c, p, ti);
        }
        SWFE_XCD_SYNC();
        for (int i = tb + j; i < te; i += nb) pass2_tile<R, false>(c, p, sw, p.xtiles[i]);
        SWFE_XCD_SYNC();
        for (int g = gb + j; g < ge; g += nb) group_finalize(c, p, sw, p.groups[p.xgroups[g]]);
        SWFE_XCD_SYNC();
    }
#undef SWFE_XCD_SYNC
}

// After a persistent launch: a wait that gave up marks every system.
__global__ void k_persist_check(Ctl c, DevPtrs p)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < c.n_sys && p.sync[SYNC_ABORT]) p.state[s].err |= ERR_PERSIST;
}

// ----------------------------------------------------------- launchers -----
static inline dim3 tile_grid(const Ctl &c) { return dim3(8 * kFxChunks * c.fx_len); }

hipError_t launch_iota(const Ctl &c, const DevPtrs &p, int block, hipStream_t s)
{
    hipLaunchKernelGGL(k_iota, tile_grid(c), dim3(block), 0, s, c, p);
    return hipGetLastError();
}

hipError_t launch_gather(const Ctl &c, const DevPtrs &p, int block, int with_f, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather, tile_grid(c), dim3(block), 0, s, c, p, with_f);
    return hipGetLastError();
}

hipError_t launch_scatter(const Ctl &c, const DevPtrs &p, int block, int what, hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter, tile_grid(c), dim3(block), 0, s, c, p, what);
    return hipGetLastError();
}

hipError_t launch_integrate(const Ctl &c, const DevPtrs &p, const SwParams &sw, int block, hipStream_t s)
{
    (void)sw;
    hipLaunchKernelGGL(k_integrate, tile_grid(c), dim3(block), 0, s, c, p, sw);
    return hipGetLastError();
}

hipError_t launch_rebuild(const Ctl &c, const DevPtrs &p, const SwParams &sw, int block, int stage,
                          hipStream_t s)
{
    if (c.sort_cells > 0 && stage < 4) {
        // the fused sort does stages 0-3 in one launch
        if (stage == 0)
            hipLaunchKernelGGL(k_rb_sort, dim3(c.n_sys), dim3(kSortThreads), sizeof(int32_t) * (size_t)c.sort_cells,
                               s, c, p, sw);
        return hipGetLastError();
    }
    switch (stage) {
        case 0: hipLaunchKernelGGL(k_rb_count, tile_grid(c), dim3(block), 0, s, c, p, sw); break;
        case 1:
            // folded into the scatter stage when the cell tables fit in LDS
            if (c.scan_cells == 0)
                hipLaunchKernelGGL(k_rb_scan, dim3(c.n_sys), dim3(kSortThreads), 0, s, c, p, sw);
            break;
        case 2:
            hipLaunchKernelGGL(k_rb_scatter, dim3(kWorkGrid), dim3(block), sizeof(int32_t) * (size_t)c.scan_cells,
                               s, c, p, sw);
            break;
        case 3: hipLaunchKernelGGL(k_rb_order, dim3(kWorkGrid), dim3(block), 0, s, c, p, sw); break;
        default:
            hipLaunchKernelGGL(k_rb_list, dim3(4 * kWorkGrid), dim3(256), 0, s, c, p, sw, (block + 7) / 8);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_fill_noise(const Ctl &c, const DevPtrs &p, int block, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_noise, tile_grid(c), dim3(block), 0, s, c, p);
    return hipGetLastError();
}

hipError_t launch_pass1(const Ctl &c, const DevPtrs &p, const SwParams &sw, int mixed, int block,
                        hipStream_t s)
{
    const bool g = (c.flags & 1) != 0;
    const size_t lds = sizeof(int32_t) * kLdsShort * (size_t)block;
    if (mixed) {
        if (g) hipLaunchKernelGGL((k_pass1<float, true>), tile_grid(c), dim3(block), lds, s, c, p, sw);
        else hipLaunchKernelGGL((k_pass1<float, false>), tile_grid(c), dim3(block), lds, s, c, p, sw);
    } else {
        if (g) hipLaunchKernelGGL((k_pass1<double, true>), tile_grid(c), dim3(block), lds, s, c, p, sw);
        else hipLaunchKernelGGL((k_pass1<double, false>), tile_grid(c), dim3(block), lds, s, c, p, sw);
    }
    if (c.has_uf) {
        if (mixed) hipLaunchKernelGGL((k_uf<float>), tile_grid(c), dim3(block), 0, s, c, p);
        else hipLaunchKernelGGL((k_uf<double>), tile_grid(c), dim3(block), 0, s, c, p);
    }
    return hipGetLastError();
}

hipError_t launch_pass2(const Ctl &c, const DevPtrs &p, const SwParams &sw, int mixed, int block,
                        hipStream_t s)
{
    const bool g = (c.flags & 1) != 0;
    if (mixed) {
        if (g) hipLaunchKernelGGL((k_pass2<float, true>), tile_grid(c), dim3(block), 0, s, c, p, sw);
        else hipLaunchKernelGGL((k_pass2<float, false>), tile_grid(c), dim3(block), 0, s, c, p, sw);
    } else {
        if (g) hipLaunchKernelGGL((k_pass2<double, true>), tile_grid(c), dim3(block), 0, s, c, p, sw);
        else hipLaunchKernelGGL((k_pass2<double, false>), tile_grid(c), dim3(block), 0, s, c, p, sw);
    }
    return hipGetLastError();
}

hipError_t launch_finalize(const Ctl &c, const DevPtrs &p, const SwParams &sw, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(c.n_groups), dim3(256), 0, s, c, p, sw);
    return hipGetLastError();
}

hipError_t launch_begin_step(const Ctl &c, const DevPtrs &p, const SwParams &sw, int64_t n_steps,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_begin_step, dim3((c.n_groups + 63) / 64), dim3(64), 0, s, c, p, sw, n_steps);
    return hipGetLastError();
}

hipError_t launch_reset_schedule(const Ctl &c, const DevPtrs &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_schedule, dim3((c.n_sys + 63) / 64), dim3(64), 0, s, c, p);
    return hipGetLastError();
}

hipError_t launch_set_pscale(const Ctl &c, const DevPtrs &p, const double *diag, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_pscale, dim3((c.n_sys + 63) / 64), dim3(64), 0, s, c, p, diag);
    return hipGetLastError();
}

hipError_t launch_zero_words(void *w, size_t bytes, hipStream_t s)
{
    const int64_t n = (int64_t)(bytes / 4);
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)w, n);
    return hipGetLastError();
}

hipError_t launch_clear_err(const Ctl &c, const DevPtrs &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_err, dim3((c.n_sys + 63) / 64), dim3(64), 0, s, c, p);
    return hipGetLastError();
}
}  // namespace swfe

namespace swfe {
int persist_blocks_per_cu(int mixed, int block)
{
    int n = 0;
    const size_t lds = sizeof(int32_t) * kLdsShort * (size_t)block;
    hipError_t e = mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persist<float>, block, lds)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persist<double>, block, lds);
    return e == hipSuccess ? n : 0;
}

hipError_t launch_persist(const Ctl &c, const DevPtrs &p, const SwParams &sw, const XcdPlan &xp, int mixed,
                          int block, int grid, int64_t n_steps, hipStream_t s)
{
    const size_t lds = sizeof(int32_t) * kLdsShort * (size_t)block;
    Ctl cc = c;
    DevPtrs pp = p;
    SwParams ss = sw;
    XcdPlan xx = xp;
    int64_t ns = n_steps;
    void *args[] = {&cc, &pp, &ss, &xx, &ns};
    hipError_t e = mixed ? hipLaunchCooperativeKernel((const void *)k_persist<float>, dim3(grid), dim3(block), args,
                                                      lds, s)
                         : hipLaunchCooperativeKernel((const void *)k_persist<double>, dim3(grid), dim3(block), args,
                                                      lds, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_persist_check, dim3((c.n_sys + 63) / 64), dim3(64), 0, s, c, p);
    return hipGetLastError();
}
}  // namespace swfe
