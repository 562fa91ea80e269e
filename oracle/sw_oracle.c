/*
 * sw_oracle.c -- plain FP64 reference for the Stillinger-Weber silicon model.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the GPU library is
 * checked against.  Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product path never does.  It shares no
 * code, header or constant with the GPU library.
 *
 * What it computes (the plain definition, no reformulation):
 *   E = sum_{i<j} phi2(r_ij) + sum_i sum_{j<k; j,k != i} phi3(r_ij, r_ik, theta_jik)
 *   phi2(r) = eps*A*[B*(sig/r)^p - (sig/r)^q] * exp(sig/(r - a*sig))       r < a*sig
 *   phi3    = lam*eps*(cos theta_jik - cos0)^2 * g(r_ij) * g(r_ik)
 *   g(r)    = exp(gam*sig/(r - a*sig))                                     r < a*sig
 * This is the potential the paper uses for silicon (applications section,
 * Stillinger and Weber 1985).  Pairs are enumerated by brute force over all
 * atoms: with the minimum-image convention when every perpendicular box width
 * is at least twice the cutoff, otherwise with an explicit sum over periodic
 * images (small cells).  Forces are -dE/dr, the virial is
 * Xi_ab = dE/d(strain_ab) under r -> (I+strain) r (box included), and the
 * parameter gradient is dE/d(A, B, p, q, a, lam, gam, sig, eps).
 *
 * Per-atom energy convention: half of each pair term to each of its two
 * atoms, each triplet term to its centre atom i.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double A, B, p, q, a, lam, gam, sig, eps, cos0;
} orc_sw_t;

typedef struct {
    int j;
    double d[3];  /* r_j + image - r_i */
    double r;
} orc_nb_t;

static void inv3(const double h[9], double out[9])
{
    double det = h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) +
                 h[2] * (h[3] * h[7] - h[4] * h[6]);
    out[0] = (h[4] * h[8] - h[5] * h[7]) / det;
    out[1] = (h[2] * h[7] - h[1] * h[8]) / det;
    out[2] = (h[1] * h[5] - h[2] * h[4]) / det;
    out[3] = (h[5] * h[6] - h[3] * h[8]) / det;
    out[4] = (h[0] * h[8] - h[2] * h[6]) / det;
    out[5] = (h[2] * h[3] - h[0] * h[5]) / det;
    out[6] = (h[3] * h[7] - h[4] * h[6]) / det;
    out[7] = (h[1] * h[6] - h[0] * h[7]) / det;
    out[8] = (h[0] * h[4] - h[1] * h[3]) / det;
}

/* perpendicular width of the cell along box vector k (h columns are box vectors) */
static double perp_width(const double h[9], int k)
{
    int l = (k + 1) % 3, m = (k + 2) % 3;
    double bl[3] = {h[0 * 3 + l], h[1 * 3 + l], h[2 * 3 + l]};
    double bm[3] = {h[0 * 3 + m], h[1 * 3 + m], h[2 * 3 + m]};
    double c[3] = {bl[1] * bm[2] - bl[2] * bm[1], bl[2] * bm[0] - bl[0] * bm[2],
                   bl[0] * bm[1] - bl[1] * bm[0]};
    double vol = fabs(h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) +
                      h[2] * (h[3] * h[7] - h[4] * h[6]));
    return vol / sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
}

/* Threads of the neighbour search (1 unless a caller asks for more).  Every
 * atom's list is built independently and in the same order whatever the
 * count, so results do not depend on it. */
static int orc_threads = 1;

void orc_set_threads(int n) { orc_threads = n > 0 ? n : 1; }

/*
 * The neighbours (j, image) of atom i with |r_j + image - r_i| < rc, in the
 * order j, then image.  Writes them to out (when not NULL) and returns their
 * count.
 */
static int atom_neighbours(int i, int n, const double* x, const double h[9], const double hinv[9],
                           const int m[3], double rc2, orc_nb_t* out)
{
    int cnt = 0;
    for (int j = 0; j < n; ++j) {
        double d0[3], s[3];
        for (int a = 0; a < 3; ++a) d0[a] = x[3 * j + a] - x[3 * i + a];
        for (int a = 0; a < 3; ++a)
            s[a] = hinv[a * 3 + 0] * d0[0] + hinv[a * 3 + 1] * d0[1] + hinv[a * 3 + 2] * d0[2];
        for (int a = 0; a < 3; ++a) s[a] -= round(s[a]);
        for (int i0 = -m[0]; i0 <= m[0]; ++i0)
            for (int i1 = -m[1]; i1 <= m[1]; ++i1)
                for (int i2 = -m[2]; i2 <= m[2]; ++i2) {
                    double t[3] = {s[0] + i0, s[1] + i1, s[2] + i2};
                    double d[3];
                    for (int a = 0; a < 3; ++a)
                        d[a] = h[a * 3 + 0] * t[0] + h[a * 3 + 1] * t[1] + h[a * 3 + 2] * t[2];
                    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    if (r2 >= rc2) continue;
                    if (j == i && i0 == 0 && i1 == 0 && i2 == 0) continue;
                    if (r2 == 0.0) continue;
                    if (out) {
                        out[cnt].j = j;
                        for (int a = 0; a < 3; ++a) out[cnt].d[a] = d[a];
                        out[cnt].r = sqrt(r2);
                    }
                    ++cnt;
                }
    }
    return cnt;
}

/*
 * Build, for every atom i, the list of (j, image) with |r_j + image - r_i| < rc.
 * x is [n][3]; h is the 3x3 cell matrix (row a, column b = component a of box
 * vector b).  force_images != 0 selects the explicit-image sum even for large
 * cells.  The lists are counted first, then written at their offsets.
 * Returns 0, or -1 on allocation failure.
 */
static int neighbours(int n, const double* x, const double h[9], double rc, int force_images,
                      int** start_out, orc_nb_t** list_out)
{
    double hinv[9];
    inv3(h, hinv);
    int m[3];
    int use_images = force_images;
    for (int k = 0; k < 3; ++k) {
        double w = perp_width(h, k);
        if (w < 2.0 * rc) use_images = 1;
        m[k] = (int)ceil(rc / w) + 1;
    }
    if (!use_images) m[0] = m[1] = m[2] = 0;

    int* start = (int*)malloc(sizeof(int) * (n + 1));
    if (!start) return -1;
    const double rc2 = rc * rc;
#pragma omp parallel for num_threads(orc_threads) schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) start[i + 1] = atom_neighbours(i, n, x, h, hinv, m, rc2, NULL);
    start[0] = 0;
    for (int i = 0; i < n; ++i) start[i + 1] += start[i];
    orc_nb_t* list = (orc_nb_t*)malloc(sizeof(orc_nb_t) * (start[n] > 0 ? start[n] : 1));
    if (!list) { free(start); return -1; }
#pragma omp parallel for num_threads(orc_threads) schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) atom_neighbours(i, n, x, h, hinv, m, rc2, list + start[i]);
    *start_out = start;
    *list_out = list;
    return 0;
}

/*
 * Energy, forces, virial and parameter gradient of one periodic system.
 *   out_e[0] = E (two-body), out_e[1] = E (three-body)
 *   f       [n][3]   forces (may be NULL)
 *   vir     [9]      Xi_ab, row-major (may be NULL)
 *   dtheta  [9]      dE/d(A,B,p,q,a,lam,gam,sig,eps) (may be NULL)
 *   e_atom  [n]      per-atom energy (may be NULL)
 *   nnb     [n]      neighbour count per atom (may be NULL)
 * Returns 0, or -1 on allocation failure.
 */
int orc_sw_eval(int n, const double* x, const double* h, const orc_sw_t* P, int force_images,
                double* out_e, double* f, double* vir, double* dtheta, double* e_atom, int* nnb)
{
    const double rc = P->a * P->sig;
    int* start;
    orc_nb_t* nb;
    if (neighbours(n, x, h, rc, force_images, &start, &nb)) return -1;

    double E2 = 0.0, E3 = 0.0, X[9] = {0}, G[9] = {0};
    if (f) memset(f, 0, sizeof(double) * 3 * n);
    if (e_atom) memset(e_atom, 0, sizeof(double) * n);

    const double eA = P->eps * P->A;
    for (int i = 0; i < n; ++i) {
        if (nnb) nnb[i] = start[i + 1] - start[i];
        /* ---- two-body: every ordered pair (i -> j) carries half of phi2 ---- */
        for (int e = start[i]; e < start[i + 1]; ++e) {
            const orc_nb_t* b = &nb[e];
            double r = b->r, s = P->sig / r, den = r - rc;
            double sp = pow(s, P->p), sq = pow(s, P->q);
            double ex = exp(P->sig / den);
            double br = P->B * sp - sq;
            double phi = eA * br * ex;
            double dbr = (-P->p * P->B * sp + P->q * sq) / r;     /* d(br)/dr */
            double dex = ex * (-P->sig / (den * den));             /* d(ex)/dr */
            double dphi = eA * (dbr * ex + br * dex);
            E2 += 0.5 * phi;
            if (e_atom) e_atom[i] += 0.5 * phi;
            double gvec[3];
            for (int a = 0; a < 3; ++a) gvec[a] = 0.5 * dphi * b->d[a] / r;  /* dE/dd */
            if (f)
                for (int a = 0; a < 3; ++a) { f[3 * b->j + a] -= gvec[a]; f[3 * i + a] += gvec[a]; }
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) X[a * 3 + c] += gvec[a] * b->d[c];
            if (dtheta) {
                double lns = log(s);
                G[0] += 0.5 * phi / P->A;                                   /* A */
                G[1] += 0.5 * eA * sp * ex;                                 /* B */
                G[2] += 0.5 * eA * P->B * sp * lns * ex;                    /* p */
                G[3] += 0.5 * (-eA * sq * lns * ex);                        /* q */
                G[4] += 0.5 * phi * P->sig * P->sig / (den * den);          /* a */
                G[7] += 0.5 * eA * ex *
                        ((P->p * P->B * sp - P->q * sq) / P->sig + br * r / (den * den)); /* sig */
                G[8] += 0.5 * phi / P->eps;                                 /* eps */
            }
        }
        /* ---- three-body: each unordered neighbour pair (j,k) of centre i ---- */
        for (int e1 = start[i]; e1 < start[i + 1]; ++e1) {
            const orc_nb_t* b1 = &nb[e1];
            double r1 = b1->r, den1 = b1->r - rc;
            double g1 = exp(P->gam * P->sig / den1);
            double dg1 = g1 * (-P->gam * P->sig / (den1 * den1));
            for (int e2 = e1 + 1; e2 < start[i + 1]; ++e2) {
                const orc_nb_t* b2 = &nb[e2];
                double r2 = b2->r, den2 = b2->r - rc;
                double g2 = exp(P->gam * P->sig / den2);
                double dg2 = g2 * (-P->gam * P->sig / (den2 * den2));
                double dot = b1->d[0] * b2->d[0] + b1->d[1] * b2->d[1] + b1->d[2] * b2->d[2];
                double cs = dot / (r1 * r2);
                double dc = cs - P->cos0;
                double le = P->lam * P->eps;
                double phi = le * dc * dc * g1 * g2;
                E3 += phi;
                if (e_atom) e_atom[i] += phi;
                double t1[3], t2[3];
                for (int a = 0; a < 3; ++a) {
                    double dcos1 = b2->d[a] / (r1 * r2) - cs * b1->d[a] / (r1 * r1);
                    double dcos2 = b1->d[a] / (r1 * r2) - cs * b2->d[a] / (r2 * r2);
                    t1[a] = le * (2.0 * dc * dcos1 * g1 * g2 + dc * dc * dg1 * g2 * b1->d[a] / r1);
                    t2[a] = le * (2.0 * dc * dcos2 * g1 * g2 + dc * dc * g1 * dg2 * b2->d[a] / r2);
                }
                if (f)
                    for (int a = 0; a < 3; ++a) {
                        f[3 * b1->j + a] -= t1[a];
                        f[3 * b2->j + a] -= t2[a];
                        f[3 * i + a] += t1[a] + t2[a];
                    }
                for (int a = 0; a < 3; ++a)
                    for (int c = 0; c < 3; ++c) X[a * 3 + c] += t1[a] * b1->d[c] + t2[a] * b2->d[c];
                if (dtheta) {
                    G[4] += phi * P->gam * P->sig * P->sig * (1.0 / (den1 * den1) + 1.0 / (den2 * den2));
                    G[5] += phi / P->lam;
                    G[6] += phi * P->sig * (1.0 / den1 + 1.0 / den2);
                    G[7] += phi * P->gam * (r1 / (den1 * den1) + r2 / (den2 * den2));
                    G[8] += phi / P->eps;
                }
            }
        }
    }
    out_e[0] = E2;
    out_e[1] = E3;
    if (vir) memcpy(vir, X, sizeof X);
    if (dtheta) memcpy(dtheta, G, sizeof G);
    free(start);
    free(nb);
    return 0;
}

/* Einstein crystal: U = sum_i k/2 |x_i - x0_i|^2, F_i = -k (x_i - x0_i). */
double orc_einstein(int n, const double* x, const double* x0, double k, double* f)
{
    double U = 0.0;
    for (int i = 0; i < 3 * n; ++i) {
        double d = x[i] - x0[i];
        U += 0.5 * k * d * d;
        if (f) f[i] = -k * d;
    }
    return U;
}

/*
 * Uhlenbeck-Ford pair potential, the fluid reference the paper switches its
 * liquids to (section 4.1, model of Leite et al., p = 25, sigma = 2.0 A):
 *   phi_UF(r) = -p kB T_UF ln(1 - exp(-(r/sigma)^2))   r < rcut, 0 beyond
 * pkT = p kB T_UF in eV.  Every ordered pair carries half of phi, as in
 * orc_sw_eval; forces are -dE/dr, the virial dE/d(strain).
 */
int orc_uf_eval(int n, const double* x, const double* h, double pkT, double sigma, double rcut,
                int force_images, double* out_e, double* f, double* vir, double* e_atom)
{
    int* start;
    orc_nb_t* nb;
    if (neighbours(n, x, h, rcut, force_images, &start, &nb)) return -1;
    double E = 0.0, X[9] = {0};
    if (f) memset(f, 0, sizeof(double) * 3 * n);
    if (e_atom) memset(e_atom, 0, sizeof(double) * n);
    const double is2 = 1.0 / (sigma * sigma);
    for (int i = 0; i < n; ++i) {
        for (int e = start[i]; e < start[i + 1]; ++e) {
            const orc_nb_t* b = &nb[e];
            double r = b->r, u = r * r * is2;
            double om = -expm1(-u);                        /* 1 - exp(-u) */
            double phi = -pkT * log(om);
            double dphi = -pkT * (2.0 * r * is2) * exp(-u) / om;   /* dphi/dr */
            E += 0.5 * phi;
            if (e_atom) e_atom[i] += 0.5 * phi;
            double gvec[3];
            for (int a = 0; a < 3; ++a) gvec[a] = 0.5 * dphi * b->d[a] / r;
            if (f)
                for (int a = 0; a < 3; ++a) { f[3 * b->j + a] -= gvec[a]; f[3 * i + a] += gvec[a]; }
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) X[a * 3 + c] += gvec[a] * b->d[c];
        }
    }
    *out_e = E;
    if (vir) memcpy(vir, X, sizeof X);
    free(start);
    free(nb);
    return 0;
}

/* Total neighbour-pair count (ordered) for a system, for workload statistics. */
int orc_count_neighbours(int n, const double* x, const double* h, double rc, int64_t* total)
{
    int* start;
    orc_nb_t* nb;
    if (neighbours(n, x, h, rc, 0, &start, &nb)) return -1;
    *total = start[n];
    free(start);
    free(nb);
    return 0;
}
