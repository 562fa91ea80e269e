// swfe_kernels.hip -- HIP kernels for gfx950 of the switched-Hamiltonian
// Stillinger-Weber silicon step.
//
// One MD step is five launches over all systems at once:
//   integrate  per atom:  B kick, A drift, O Langevin, A drift, cell index
//   bin        per system (one 1024-thread workgroup): deterministic counting
//              sort of atoms by cell (ties in atom order)
//   pass1      per tile of cell-sorted atoms: 27-cell search, neighbour
//              list, pair terms, and the 11 three-body moments per atom
//   pass2      per tile: three-body force gather from own and neighbour
//              moments (no atomics), Einstein springs, final B kick,
//              per-tile partial sums
//   finalize   one workgroup: per-system reductions in a fixed order, the
//              barostat, the lambda switch and its work increment, dCCI
//              coupling, integrator factors for the next step.
//
// Three-body term in moment form.  With g_j = g(r_ij), u_j = r_ij/|r_ij| and
// the moments of centre i
//     s = sum g_j, q = sum g_j^2, v = sum g_j u_j, M = sum g_j u_j u_j^T,
// the triplet sum sum_{j<k} (u_j.u_k - c0)^2 g_j g_k equals
//     Phi/2,  Phi = |M|_F^2 - 2 c0 |v|^2 + c0^2 s^2 - (1 - c0)^2 q,
// so E3_i = (lambda_sw eps / 2) Phi_i.  dE3_i/dr_ij depends only on r_ij and
// centre i's moments, which turns the three-body force into an O(n) gather.
// No floating-point atomics are used anywhere: every sum has a fixed order,
// so runs are bitwise reproducible.
#include "swfe_internal.h"

#include <math.h>

namespace swfe {

// ------------------------------------------------------------------ utils --
__device__ __forceinline__ int ld_coherent(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_coherent(int32_t *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename R>
__device__ __forceinline__ R powi_or_pow(R s, int ip, R p)
{
    if (ip >= 0) {
        R r = R(1);
        for (int k = 0; k < ip; ++k) r *= s;
        return r;
    }
    return pow(s, p);
}

// Cell grid of a system for its current (strained) box: floor(L / rc) cells
// per dimension, at least 1 and at most the capacity fixed at set-up.
__device__ __forceinline__ void grid_of(const SysDesc &d, const SysState &st, double rc,
                                        int nc[3], double box[3], double ibox[3])
{
    for (int k = 0; k < 3; ++k) {
        box[k] = st.box[k] * st.pscale[k];
        ibox[k] = 1.0 / box[k];
        int n = (int)floor(box[k] / rc);
        n = n < 1 ? 1 : n;
        n = n > d.nc_max[k] ? d.nc_max[k] : n;
        nc[k] = n;
    }
}

__device__ __forceinline__ int cell_coord(double x, double ibox, int nc)
{
    double s = x * ibox;
    s -= floor(s);
    int c = (int)(s * nc);
    c = c < 0 ? 0 : c;
    c = c >= nc ? nc - 1 : c;
    return c;
}

__device__ __forceinline__ double min_image(double d, double box, double ibox)
{
    return d - box * rint(d * ibox);
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
    const double twopi = 2.0 * 3.141592653589793;
    double r01 = sqrt(-2.0 * log(u0));
    double r23 = sqrt(-2.0 * log(u2));
    out[0] = r01 * cos(twopi * u1);
    out[1] = r01 * sin(twopi * u1);
    out[2] = r23 * cos(twopi * u3);
}

__device__ __forceinline__ bool o_step_on(const SysDesc &d)
{
    return d.mode != MODE_FORCE && d.mode != MODE_NVE && d.tau_damp > 0.0 && d.T0 > 0.0;
}

// Total force on an atom at coupling lam: FL interpolates with the Einstein
// reference (section 2.1), RS and dCCI scale the interaction (eq. H_RS).
__device__ __forceinline__ double total_force(int mode, double lam, double fint, double x,
                                              const double *x0, int64_t idx, double k)
{
    if (mode == MODE_FL) {
        double fref = x0 ? -k * (x - x0[idx]) : 0.0;
        return lam * fint + (1.0 - lam) * fref;
    }
    if (mode == MODE_RS || mode == MODE_DCCI_T || mode == MODE_DCCI_P) return lam * fint;
    return fint;
}

// Deterministic block reduction of NV doubles per thread into out[0..NV).
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], double *out)
{
    __shared__ double red[4][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double a = v[k];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
        if (lane == 0) red[wave][k] = a;
    }
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// ------------------------------------------------------------ cell index ---
__global__ void __launch_bounds__(256) k_assign_cells(Ctl c, DevPtrs p, double rc)
{
    const Tile tile = p.tiles[blockIdx.x];
    if ((int)threadIdx.x >= tile.count) return;
    const SysDesc &d = p.desc[tile.sys];
    const SysState &st = p.state[tile.sys];
    int nc[3];
    double box[3], ibox[3];
    grid_of(d, st, rc, nc, box, ibox);
    const int64_t i = tile.start + threadIdx.x, N = c.n_total;
    int cc[3];
    bool fin = true;
    for (int k = 0; k < 3; ++k) {
        double xk = p.x[k * N + i] * st.pscale[k];
        fin = fin && isfinite(xk);
        cc[k] = cell_coord(xk, ibox[k], nc[k]);
    }
    if (!fin) atomicOr(&p.state[tile.sys].err, ERR_NONFINITE);
    p.cell_of[i] = (cc[2] * nc[1] + cc[1]) * nc[0] + cc[0];
}

// ------------------------------------------------------------------ bin ----
// One workgroup per system: zero counts, count, exclusive scan (cell starts
// in global sorted positions), placement, then an insertion sort of every
// cell's segment so that the order inside a cell is by atom index.
__global__ void __launch_bounds__(kBinThreads) k_bin(Ctl c, DevPtrs p, double rc)
{
    const int sys = blockIdx.x;
    const SysDesc &d = p.desc[sys];
    const SysState &st = p.state[sys];
    int nc3[3];
    double box[3], ibox[3];
    grid_of(d, st, rc, nc3, box, ibox);
    const int nc = nc3[0] * nc3[1] * nc3[2];
    int32_t *cnt = p.cell_count + d.cell_base;
    int32_t *cur = p.cursor + d.cell_base;
    int32_t *start = p.cell_start + d.cell_base + sys;  // nc + 1 entries per system
    const int64_t off = d.off;
    const int n = (int)d.n;
    const int tid = threadIdx.x;

    for (int q = tid; q < nc; q += kBinThreads) cnt[q] = 0;
    __threadfence();
    __syncthreads();
    for (int i = tid; i < n; i += kBinThreads) atomicAdd(&cnt[p.cell_of[off + i]], 1);
    __threadfence();
    __syncthreads();

    __shared__ int32_t part[kBinThreads];
    const int per = (nc + kBinThreads - 1) / kBinThreads;
    const int lo = tid * per, hi = min(lo + per, nc);
    int sum = 0;
    for (int q = lo; q < hi; ++q) sum += ld_coherent(&cnt[q]);
    part[tid] = sum;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 1024 partial sums
    for (int o = 1; o < kBinThreads; o <<= 1) {
        int add = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
    }
    int run = (int)off + part[tid] - sum;
    for (int q = lo; q < hi; ++q) {
        start[q] = run;
        cur[q] = run;
        run += ld_coherent(&cnt[q]);
    }
    if (tid == 0) start[nc] = (int)off + n;
    __threadfence();
    __syncthreads();
    for (int i = tid; i < n; i += kBinThreads) {
        int slot = atomicAdd(&cur[p.cell_of[off + i]], 1);
        p.sorted[slot] = (int32_t)(off + i);
    }
    __threadfence();
    __syncthreads();
    for (int q = tid; q < nc; q += kBinThreads) {
        const int b = ld_coherent(&start[q]), e = ld_coherent(&start[q + 1]);
        for (int a = b + 1; a < e; ++a) {
            int key = ld_coherent(&p.sorted[a]);
            int m = a - 1;
            while (m >= b) {
                int w = ld_coherent(&p.sorted[m]);
                if (w <= key) break;
                st_coherent(&p.sorted[m + 1], w);
                --m;
            }
            st_coherent(&p.sorted[m + 1], key);
        }
    }
}

// ---------------------------------------------------------------- pass 1 ---
// Neighbour search over the (up to) 27 cells around the atom's cell, pair
// terms (energy, force, virial, parameter derivative: half per ordered pair)
// and three-body moments.  R is the arithmetic type of the terms.
template <typename R>
__global__ void __launch_bounds__(256) k_pass1(Ctl c, DevPtrs p, SwParams sw)
{
    constexpr int NV = 19;  // E, virial 9, dtheta 9
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;

    const Tile tile = p.tiles[blockIdx.x];
    const int sys = tile.sys;
    const SysDesc &d = p.desc[sys];
    const SysState &st = p.state[sys];
    const int64_t N = c.n_total;
    const bool grad = (c.flags & 1) != 0;

    if ((int)threadIdx.x < tile.count) {
        int nc[3];
        double box[3], ibox[3];
        grid_of(d, st, sw.rc, nc, box, ibox);
        const int64_t t = tile.start + threadIdx.x;
        const int i = p.sorted[t];
        const double ps0 = st.pscale[0], ps1 = st.pscale[1], ps2 = st.pscale[2];
        const double xi = p.x[i] * ps0, yi = p.x[N + i] * ps1, zi = p.x[2 * N + i] * ps2;
        const int ci = p.cell_of[i];
        const int cx = ci % nc[0], cy = (ci / nc[0]) % nc[1], cz = ci / (nc[0] * nc[1]);
        const int nxo = nc[0] >= 3 ? 3 : nc[0], nyo = nc[1] >= 3 ? 3 : nc[1],
                  nzo = nc[2] >= 3 ? 3 : nc[2];
        const int x0c = nc[0] >= 3 ? cx - 1 : 0, y0c = nc[1] >= 3 ? cy - 1 : 0,
                  z0c = nc[2] >= 3 ? cz - 1 : 0;
        const int32_t *start = p.cell_start + d.cell_base + sys;

        const R rc = (R)sw.rc, sig = (R)sw.sig, eA = (R)sw.eA, B = (R)sw.B, pp = (R)sw.p,
                qq = (R)sw.q, gam = (R)sw.gam;
        double m_s = 0, m_q = 0, m_v[3] = {0, 0, 0}, m_M[6] = {0, 0, 0, 0, 0, 0};
        double F2[3] = {0, 0, 0};
        int nn = 0;

        for (int oz = 0; oz < nzo; ++oz) {
            int zz = z0c + oz;
            zz = zz < 0 ? zz + nc[2] : (zz >= nc[2] ? zz - nc[2] : zz);
            for (int oy = 0; oy < nyo; ++oy) {
                int yy = y0c + oy;
                yy = yy < 0 ? yy + nc[1] : (yy >= nc[1] ? yy - nc[1] : yy);
                for (int ox = 0; ox < nxo; ++ox) {
                    int xx = x0c + ox;
                    xx = xx < 0 ? xx + nc[0] : (xx >= nc[0] ? xx - nc[0] : xx);
                    const int cell = (zz * nc[1] + yy) * nc[0] + xx;
                    const int b = start[cell], e = start[cell + 1];
                    for (int s = b; s < e; ++s) {
                        const int j = p.sorted[s];
                        if (j == i) continue;
                        double dx = min_image(p.x[j] * ps0 - xi, box[0], ibox[0]);
                        double dy = min_image(p.x[N + j] * ps1 - yi, box[1], ibox[1]);
                        double dz = min_image(p.x[2 * N + j] * ps2 - zi, box[2], ibox[2]);
                        double r2d = dx * dx + dy * dy + dz * dz;
                        if (r2d >= sw.rc2) continue;
                        if (nn < kMaxNb) p.nbr[(int64_t)nn * N + t] = j;
                        ++nn;
                        const R ddx = (R)dx, ddy = (R)dy, ddz = (R)dz;
                        const R r = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
                        const R ri = R(1) / r;
                        const R ux = ddx * ri, uy = ddy * ri, uz = ddz * ri;
                        // Inside the cutoff in FP64 may round to r >= rc in the
                        // term precision; the terms vanish there, so zero them.
                        const R den = r - rc;
                        const bool in = den < R(0);
                        const R di = in ? R(1) / den : R(0);
                        const R sr = sig * ri;
                        const R sp = powi_or_pow(sr, sw.ip, pp);
                        const R sq = powi_or_pow(sr, sw.iq, qq);
                        const R ex = in ? exp(sig * di) : R(0);
                        const R br = B * sp - sq;
                        const R phi = eA * br * ex;
                        const R dphi = eA * ex * ((qq * sq - pp * B * sp) * ri - br * sig * di * di);
                        const R g = in ? exp(gam * sig * di) : R(0);
                        // moments
                        m_s += (double)g;
                        m_q += (double)(g * g);
                        m_v[0] += (double)(g * ux);
                        m_v[1] += (double)(g * uy);
                        m_v[2] += (double)(g * uz);
                        m_M[0] += (double)(g * ux * ux);
                        m_M[1] += (double)(g * uy * uy);
                        m_M[2] += (double)(g * uz * uz);
                        m_M[3] += (double)(g * ux * uy);
                        m_M[4] += (double)(g * ux * uz);
                        m_M[5] += (double)(g * uy * uz);
                        // pair: F_i += phi2'(r) u_ij ; E_i += phi2/2 ; virial half
                        F2[0] += (double)(dphi * ux);
                        F2[1] += (double)(dphi * uy);
                        F2[2] += (double)(dphi * uz);
                        acc[0] += 0.5 * (double)phi;
                        const R hv = R(0.5) * dphi * r;
                        const R uu[3] = {ux, uy, uz};
#pragma unroll
                        for (int a = 0; a < 3; ++a)
#pragma unroll
                            for (int bb = 0; bb < 3; ++bb) acc[1 + 3 * a + bb] += (double)(hv * uu[a] * uu[bb]);
                        if (grad) {
                            const R lns = log(sr);
                            acc[10] += 0.5 * (double)((R)sw.eps * br * ex);                  // A
                            acc[11] += 0.5 * (double)(eA * sp * ex);                         // B
                            acc[12] += 0.5 * (double)(eA * B * sp * lns * ex);               // p
                            acc[13] += 0.5 * (double)(-eA * sq * lns * ex);                  // q
                            acc[14] += 0.5 * (double)(phi * sig * sig * di * di);            // a
                            acc[17] += 0.5 * (double)(eA * ex * ((pp * B * sp - qq * sq) / sig + br * r * di * di));  // sigma
                            acc[18] += 0.5 * (double)((R)sw.A * br * ex);                    // epsilon
                        }
                    }
                }
            }
        }
        if (nn > kMaxNb) {
            atomicOr(&p.state[sys].err, ERR_OVERFLOW);
            nn = kMaxNb;
        }
        p.nnb[t] = nn;
        p.mom[0 * N + i] = m_s;
        p.mom[1 * N + i] = m_q;
        p.mom[2 * N + i] = m_v[0];
        p.mom[3 * N + i] = m_v[1];
        p.mom[4 * N + i] = m_v[2];
#pragma unroll
        for (int k = 0; k < 6; ++k) p.mom[(5 + k) * N + i] = m_M[k];
        p.f[i] = F2[0];
        p.f[N + i] = F2[1];
        p.f[2 * N + i] = F2[2];
        if (p.e_atom) p.e_atom[i] = acc[0];
    }
    block_reduce<NV>(acc, p.part1 + (int64_t)blockIdx.x * kNumPart);
}

// ---------------------------------------------------------------- pass 2 ---
// d E3_c / d r_cj for a centre with moments (s, q, v, M) and a neighbour at
// unit vector u, distance r, g = g(r), dg = g'(r):
//   (le/2) [ dg H u + (4 g / r) ((M u - (u.M.u) u) - c0 (v - (v.u) u)) ],
//   H = 2 u.M.u - 4 c0 v.u + 2 c0^2 s - 2 (1 - c0)^2 g.
template <typename R>
__device__ __forceinline__ void d_e3(const R mom[11], R ux, R uy, R uz, R g, R dg, R ri, R c0,
                                     R hle, R out[3], R &H)
{
    const R s = mom[0], vx = mom[2], vy = mom[3], vz = mom[4];
    const R Mxx = mom[5], Myy = mom[6], Mzz = mom[7], Mxy = mom[8], Mxz = mom[9], Myz = mom[10];
    const R mux = Mxx * ux + Mxy * uy + Mxz * uz;
    const R muy = Mxy * ux + Myy * uy + Myz * uz;
    const R muz = Mxz * ux + Myz * uy + Mzz * uz;
    const R umu = ux * mux + uy * muy + uz * muz;
    const R vu = vx * ux + vy * uy + vz * uz;
    const R omc = R(1) - c0;
    H = R(2) * umu - R(4) * c0 * vu + R(2) * c0 * c0 * s - R(2) * omc * omc * g;
    const R a = dg * H;
    const R b = R(4) * g * ri;
    out[0] = hle * (a * ux + b * ((mux - umu * ux) - c0 * (vx - vu * ux)));
    out[1] = hle * (a * uy + b * ((muy - umu * uy) - c0 * (vy - vu * uy)));
    out[2] = hle * (a * uz + b * ((muz - umu * uz) - c0 * (vz - vu * uz)));
}

template <typename R>
__global__ void __launch_bounds__(256) k_pass2(Ctl c, DevPtrs p, SwParams sw)
{
    constexpr int NV = 24;  // E3, virial 9, dtheta 9, U_ref, K, noise 3
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;

    const Tile tile = p.tiles[blockIdx.x];
    const int sys = tile.sys;
    const SysDesc &d = p.desc[sys];
    const SysState &st = p.state[sys];
    const int64_t N = c.n_total;
    const bool grad = (c.flags & 1) != 0;

    if ((int)threadIdx.x < tile.count) {
        int nc[3];
        double box[3], ibox[3];
        grid_of(d, st, sw.rc, nc, box, ibox);
        const int64_t t = tile.start + threadIdx.x;
        const int a = p.sorted[t];
        const double ps0 = st.pscale[0], ps1 = st.pscale[1], ps2 = st.pscale[2];
        const double xa = p.x[a] * ps0, ya = p.x[N + a] * ps1, za = p.x[2 * N + a] * ps2;
        double momA_d[11];
#pragma unroll
        for (int k = 0; k < 11; ++k) momA_d[k] = p.mom[k * N + a];
        R momA[11];
#pragma unroll
        for (int k = 0; k < 11; ++k) momA[k] = (R)momA_d[k];
        const R rc = (R)sw.rc, sig = (R)sw.sig, gam = (R)sw.gam, c0 = (R)sw.cos0;
        const R hle = (R)(0.5 * sw.le);
        double F3[3] = {0, 0, 0};
        double gg = 0, ga = 0, gs = 0;  // sum H g dln g/d(gamma, a, sigma)
        const int nn = p.nnb[t];
        for (int k = 0; k < nn; ++k) {
            const int j = p.nbr[(int64_t)k * N + t];
            const double dx = min_image(p.x[j] * ps0 - xa, box[0], ibox[0]);
            const double dy = min_image(p.x[N + j] * ps1 - ya, box[1], ibox[1]);
            const double dz = min_image(p.x[2 * N + j] * ps2 - za, box[2], ibox[2]);
            const R ddx = (R)dx, ddy = (R)dy, ddz = (R)dz;
            const R r = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
            const R ri = R(1) / r;
            const R ux = ddx * ri, uy = ddy * ri, uz = ddz * ri;
            const R den = r - rc;
            const bool in = den < R(0);
            const R di = in ? R(1) / den : R(0);
            const R g = in ? exp(gam * sig * di) : R(0);
            const R dg = -g * gam * sig * di * di;
            R momJ[11];
#pragma unroll
            for (int m = 0; m < 11; ++m) momJ[m] = (R)p.mom[m * N + j];
            R tA[3], tJ[3], HA, HJ;
            d_e3<R>(momA, ux, uy, uz, g, dg, ri, c0, hle, tA, HA);
            d_e3<R>(momJ, -ux, -uy, -uz, g, dg, ri, c0, hle, tJ, HJ);
            F3[0] += (double)tA[0] - (double)tJ[0];
            F3[1] += (double)tA[1] - (double)tJ[1];
            F3[2] += (double)tA[2] - (double)tJ[2];
            const R dd[3] = {ddx, ddy, ddz};
#pragma unroll
            for (int aa = 0; aa < 3; ++aa)
#pragma unroll
                for (int bb = 0; bb < 3; ++bb) acc[1 + 3 * aa + bb] += (double)(tA[aa] * dd[bb]);
            if (grad) {
                const R hg = HA * g;
                gg += (double)(hg * sig * di);
                ga += (double)(hg * gam * sig * sig * di * di);
                gs += (double)(hg * gam * r * di * di);
            }
        }
        // own three-body energy from the FP64 moments
        {
            const double *m = momA_d;
            const double c0d = sw.cos0, omc = 1.0 - c0d;
            const double MF = m[5] * m[5] + m[6] * m[6] + m[7] * m[7] +
                              2.0 * (m[8] * m[8] + m[9] * m[9] + m[10] * m[10]);
            const double vv = m[2] * m[2] + m[3] * m[3] + m[4] * m[4];
            const double Phi = MF - 2.0 * c0d * vv + c0d * c0d * m[0] * m[0] - omc * omc * m[1];
            acc[0] = 0.5 * sw.le * Phi;
            if (grad) {
                const double hle_d = 0.5 * sw.le;
                acc[10 + 4] = hle_d * ga;                 // a
                acc[10 + 5] = 0.5 * sw.eps * Phi;         // lambda_sw
                acc[10 + 6] = hle_d * gg;                 // gamma
                acc[10 + 7] = hle_d * gs;                 // sigma
                acc[10 + 8] = 0.5 * sw.lam * Phi;         // epsilon
            }
        }
        if (p.e_atom) p.e_atom[a] += acc[0];
        double F[3];
        F[0] = p.f[a] + F3[0];
        F[1] = p.f[N + a] + F3[1];
        F[2] = p.f[2 * N + a] + F3[2];
        p.f[a] = F[0];
        p.f[N + a] = F[1];
        p.f[2 * N + a] = F[2];
        if (p.grad_x) {
            const double gsc = p.grad_scale ? p.grad_scale[sys] : 1.0;
            p.grad_x[a] = -F[0] * gsc;
            p.grad_x[N + a] = -F[1] * gsc;
            p.grad_x[2 * N + a] = -F[2] * gsc;
        }
        // Einstein reference (Frenkel-Ladd systems)
        const bool fl = d.mode == MODE_FL && p.x0 != nullptr;
        if (fl) {
            double u = 0.0;
            for (int k = 0; k < 3; ++k) {
                double dd = p.x[k * N + a] - p.x0[k * N + a];
                u += dd * dd;
            }
            acc[19] = 0.5 * d.k_spring * u;
        }
        // final half kick of a dynamics step, then the kinetic energy
        double vsq = 0.0;
        for (int k = 0; k < 3; ++k) {
            double vk = p.v[k * N + a];
            if (c.in_step && d.mode != MODE_FORCE) {
                double ft = total_force(d.mode, st.lam, F[k], p.x[k * N + a], p.x0, k * N + a,
                                        d.k_spring);
                vk = vk * st.decay + ((0.5 * c.dt) * d.acc) * ft * st.phi;
                p.v[k * N + a] = vk;
            }
            vsq += vk * vk;
        }
        acc[20] = d.mvv2e_m * vsq;
        // normals of the next O step, for its zero-sum correction
        if (o_step_on(d)) {
            double z[3];
            normals3(c.seed, d.stream, (uint64_t)(st.step + c.in_step), (uint64_t)(a - d.off), z);
            acc[21] = z[0];
            acc[22] = z[1];
            acc[23] = z[2];
        }
    }
    block_reduce<NV>(acc, p.part2 + (int64_t)blockIdx.x * kNumPart);
}

// ------------------------------------------------------------- integrate ---
// Steps 3-6 of the switched step for one atom: B kick with F(lambda_{k+1}),
// A half drift with isotropic box scaling, O Langevin step with zero-sum
// noise, A half drift; then the cell index in the new box.
__global__ void __launch_bounds__(256) k_integrate(Ctl c, DevPtrs p, double rc)
{
    const Tile tile = p.tiles[blockIdx.x];
    if ((int)threadIdx.x >= tile.count) return;
    const int sys = tile.sys;
    const SysDesc &d = p.desc[sys];
    const SysState &st = p.state[sys];
    const int64_t i = tile.start + threadIdx.x, N = c.n_total;
    int nc[3];
    double box[3], ibox[3];
    grid_of(d, st, rc, nc, box, ibox);
    double x[3], v[3];
    for (int k = 0; k < 3; ++k) {
        x[k] = p.x[k * N + i];
        v[k] = p.v[k * N + i];
    }
    if (d.mode != MODE_FORCE) {
        const double hdt = 0.5 * c.dt;
        for (int k = 0; k < 3; ++k) {
            double ft = total_force(d.mode, st.lam, p.f[k * N + i], x[k], p.x0, k * N + i, d.k_spring);
            v[k] = v[k] * st.decay + (hdt * d.acc) * ft * st.phi;
        }
        for (int k = 0; k < 3; ++k) x[k] = x[k] * st.grow + (v[k] * hdt) * st.psi;
        if (o_step_on(d)) {
            double z[3];
            normals3(c.seed, d.stream, (uint64_t)st.step, (uint64_t)(i - d.off), z);
            const double c2s = d.c2 * d.sigv;
            for (int k = 0; k < 3; ++k) v[k] = d.c1 * v[k] + c2s * (z[k] - st.noise_mean[k]);
        }
        for (int k = 0; k < 3; ++k) x[k] = x[k] * st.grow + (v[k] * hdt) * st.psi;
        for (int k = 0; k < 3; ++k) {
            p.x[k * N + i] = x[k];
            p.v[k * N + i] = v[k];
        }
    }
    int cc[3];
    bool fin = true;
    for (int k = 0; k < 3; ++k) {
        fin = fin && isfinite(x[k]);
        cc[k] = cell_coord(x[k], ibox[k], nc[k]);
    }
    if (!fin) atomicOr(&p.state[sys].err, ERR_NONFINITE);
    p.cell_of[i] = (cc[2] * nc[1] + cc[1]) * nc[0] + cc[0];
}

// -------------------------------------------------------------- finalize ---
constexpr double kGpaPerEvA3 = 1.602176634e-19 / 1e-30 / 1e9;

__device__ double progress(const SysDesc &d, int64_t k)
{
    if (d.s_steps <= 0) return 1.0;
    int64_t kk = k < d.s_steps ? k : d.s_steps;
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
        case MODE_FL: return lam * st.U_int + (1.0 - lam) * st.U_ref;
        case MODE_RS:
        case MODE_DCCI_T:
        case MODE_DCCI_P: return lam * st.U_int + Ps * st.V;
        case MODE_AS_P: return Ps * st.V;
        default: return 0.0;
    }
}

__device__ void baro_half(const SysDesc &d, SysState &st, double dt)
{
    if (d.p_damp <= 0.0 || d.mode == MODE_FORCE) return;
    double tr = st.vir[0] + st.vir[4] + st.vir[8];
    if (d.mode == MODE_RS || d.mode == MODE_DCCI_T || d.mode == MODE_DCCI_P) tr = st.lam * tr;
    double g = d.alpha * 2.0 * st.K - tr - 3.0 * st.V * st.Ps;
    st.veps += 0.5 * dt * g / d.wpiston;
}

// dCCI coupling (section 3): next (lambda, P_S) of a pair from instantaneous
// per-atom energy and volume differences; returns false when singular.
__device__ bool dcci_next(const SysDesc &dI, const SysState &I, const SysDesc &dII,
                          const SysState &II, double &lam_new, double &Ps_new)
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
    if (d.mode == MODE_FL) {
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
    const double zk = d.alpha * st.veps * 0.5 * dt;
    st.decay = exp(-zk);
    st.phi = zk == 0.0 ? 1.0 : -expm1(-zk) / zk;
    const double za = st.veps * 0.5 * dt;
    st.grow = exp(za);
    st.psi = za == 0.0 ? 1.0 : expm1(za) / za;
    if (d.mode != MODE_FORCE)
        for (int k = 0; k < 3; ++k) st.box[k] = (st.box[k] * st.grow) * st.grow;
    for (int k = 0; k < 3; ++k)
        if (!(st.box[k] >= 2.0 * rc)) st.err |= ERR_BOX;
}

__global__ void __launch_bounds__(kFinThreads) k_finalize(Ctl c, DevPtrs p, SwParams sw, int mode,
                                                            int log_every, int log_cap)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = kFinThreads / 64;
    // ---- phase A: per-system sums over tiles, fixed order ----------------
    for (int s = wave; s < c.n_sys; s += nw) {
        const SysDesc &d = p.desc[s];
        SysState &st = p.state[s];
        double sum1[kNumPart], sum2[kNumPart];
        for (int k = 0; k < kNumPart; ++k) sum1[k] = sum2[k] = 0.0;
        for (int t = d.tile_begin + lane; t < d.tile_end; t += 64) {
            const double *a = p.part1 + (int64_t)t * kNumPart;
            const double *b = p.part2 + (int64_t)t * kNumPart;
            for (int k = 0; k < 19; ++k) sum1[k] += a[k];
            for (int k = 0; k < kNumPart; ++k) sum2[k] += b[k];
        }
        for (int k = 0; k < kNumPart; ++k) {
            for (int off = 32; off > 0; off >>= 1) {
                sum1[k] += __shfl_down(sum1[k], off, 64);
                sum2[k] += __shfl_down(sum2[k], off, 64);
            }
        }
        if (lane == 0) {
            st.E2 = sum1[P_E];
            st.E3 = sum2[P_E];
            st.U_int = st.E2 + st.E3;
            for (int k = 0; k < 9; ++k) st.vir[k] = sum1[P_VIR + k] + sum2[P_VIR + k];
            for (int k = 0; k < 9; ++k) st.dth[k] = sum1[P_DTH + k] + sum2[P_DTH + k];
            st.U_ref = sum2[P_UREF];
            st.K = sum2[P_K];
            for (int k = 0; k < 3; ++k) st.noise_mean[k] = sum2[P_NOISE + k] / (double)d.n;
            st.V = st.box[0] * st.box[1] * st.box[2];
            if (!isfinite(st.U_int) || !isfinite(st.K) || !isfinite(st.vir[0] + st.vir[4] + st.vir[8]))
                st.err |= ERR_NONFINITE;
            if (p.out) {
                // dE/dstrain at diagonal strain e: Xi' (I + e)^-T
                const double gsc = p.grad_scale ? p.grad_scale[s] : 1.0;
                double *o = p.out + (int64_t)s * 20;
                o[0] = st.U_int;
                o[1] = st.U_ref;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) o[2 + 3 * a + b] = st.vir[3 * a + b] / st.pscale[b] * gsc;
                for (int k = 0; k < 9; ++k) o[11 + k] = st.dth[k] * gsc;
            }
        }
    }
    __syncthreads();
    // ---- phase B: per-system scalar updates ---------------------------------
    const int64_t remaining = p.ctr[0];
    for (int s = threadIdx.x; s < c.n_sys; s += kFinThreads) {
        const SysDesc &d = p.desc[s];
        SysState &st = p.state[s];
        const bool pair_lead = (d.mode == MODE_DCCI_T || d.mode == MODE_DCCI_P) && d.partner > s;
        const bool pair_follow = (d.mode == MODE_DCCI_T || d.mode == MODE_DCCI_P) && d.partner < s;
        if (pair_follow) continue;  // handled together with its partner
        SysState *ss[2] = {&st, pair_lead ? &p.state[d.partner] : nullptr};
        const SysDesc *dd[2] = {&d, pair_lead ? &p.desc[d.partner] : nullptr};
        const int m = pair_lead ? 2 : 1;
        bool start_next = (mode == 2);
        if (mode == 1) {
            for (int q = 0; q < m; ++q) {
                baro_half(*dd[q], *ss[q], c.dt);  // step 9
                ss[q]->step += 1;
                ss[q]->k += 1;
                if (log_every > 0 && log_cap > 0 && (ss[q]->step % log_every) == 0) {
                    const int sidx = q == 0 ? s : d.partner;
                    const int64_t row = ((ss[q]->step / log_every) * c.n_sys + sidx) % log_cap;
                    double *L = p.log + row * 8;
                    const double nfk = dd[q]->nf * 8.617333262e-5;
                    L[0] = (double)ss[q]->step;
                    L[1] = ss[q]->lam;
                    L[2] = ss[q]->Ps * kGpaPerEvA3;
                    L[3] = ss[q]->lam != 0.0 ? ss[q]->Ps / ss[q]->lam * kGpaPerEvA3 : 0.0;
                    L[4] = 2.0 * ss[q]->K / nfk;
                    L[5] = ss[q]->U_int / (double)dd[q]->n;
                    L[6] = ss[q]->V / (double)dd[q]->n;
                    L[7] = ss[q]->W;
                }
            }
            start_next = remaining > 1;
        }
        if (!start_next) continue;
        // ---- start of the next step: switch (1), barostat half (2), factors
        double lam[2], Ps[2];
        if (pair_lead) {
            double l, P;
            if (!dcci_next(d, st, *dd[1], *ss[1], l, P)) {
                st.err |= ERR_DCCI;
                ss[1]->err |= ERR_DCCI;
            }
            lam[0] = lam[1] = l;
            Ps[0] = Ps[1] = P;
        } else {
            next_lambda(d, st, lam[0], Ps[0]);
        }
        for (int q = 0; q < m; ++q) {
            apply_switch(*dd[q], *ss[q], lam[q], Ps[q]);
            baro_half(*dd[q], *ss[q], c.dt);
            step_factors(*dd[q], *ss[q], c.dt, sw.rc);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && mode == 1) p.ctr[0] = remaining - 1;
}

// ----------------------------------------------------------- launchers -----
// Reset of every system's schedule state (lambda, P_S, work, schedule step)
// from its descriptor; used at set-up and when a new schedule is installed.
__global__ void k_reset_schedule(Ctl c, DevPtrs p)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= c.n_sys) return;
    const SysDesc &d = p.desc[s];
    SysState &st = p.state[s];
    switch (d.mode) {
        case MODE_FL: st.lam = d.s_start; st.Ps = 0.0; break;
        case MODE_RS: st.lam = d.s_start; st.Ps = st.lam * d.pressure; break;
        case MODE_AS_P: st.lam = 1.0; st.Ps = d.s_start / kGpaPerEvA3; break;
        case MODE_DCCI_T: st.lam = d.T0 / d.s_start; st.Ps = st.lam * d.pressure; break;
        case MODE_DCCI_P: st.lam = 1.0; st.Ps = d.s_start / kGpaPerEvA3; break;
        default: st.lam = 1.0; st.Ps = d.pressure; break;
    }
    st.W = 0.0;
    st.k = 0;
}

// Diagonal strain for the next force evaluation (1 = none).
__global__ void k_set_pscale(Ctl c, DevPtrs p, const double *diag)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= c.n_sys) return;
    for (int k = 0; k < 3; ++k) p.state[s].pscale[k] = diag ? 1.0 + diag[3 * s + k] : 1.0;
}

hipError_t launch_assign_cells(const Ctl &c, const DevPtrs &p, const SwParams &sw, int block,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_assign_cells, dim3(c.n_tiles), dim3(block), 0, s, c, p, sw.rc);
    return hipGetLastError();
}

hipError_t launch_bin(const Ctl &c, const DevPtrs &p, const SwParams &sw, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin, dim3(c.n_sys), dim3(kBinThreads), 0, s, c, p, sw.rc);
    return hipGetLastError();
}

hipError_t launch_pass1(const Ctl &c, const DevPtrs &p, const SwParams &sw, int mixed, int block,
                        hipStream_t s)
{
    if (mixed)
        hipLaunchKernelGGL(k_pass1<float>, dim3(c.n_tiles), dim3(block), 0, s, c, p, sw);
    else
        hipLaunchKernelGGL(k_pass1<double>, dim3(c.n_tiles), dim3(block), 0, s, c, p, sw);
    return hipGetLastError();
}

hipError_t launch_pass2(const Ctl &c, const DevPtrs &p, const SwParams &sw, int mixed, int block,
                        hipStream_t s)
{
    if (mixed)
        hipLaunchKernelGGL(k_pass2<float>, dim3(c.n_tiles), dim3(block), 0, s, c, p, sw);
    else
        hipLaunchKernelGGL(k_pass2<double>, dim3(c.n_tiles), dim3(block), 0, s, c, p, sw);
    return hipGetLastError();
}

hipError_t launch_finalize(const Ctl &c, const DevPtrs &p, const SwParams &sw, int mode,
                           int log_every, int log_cap, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, c, p, sw, mode, log_every,
                       log_cap);
    return hipGetLastError();
}

hipError_t launch_integrate(const Ctl &c, const DevPtrs &p, const SwParams &sw, int block,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_integrate, dim3(c.n_tiles), dim3(block), 0, s, c, p, sw.rc);
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
}  // namespace swfe
