/*
 * mdref.c -- plain, slow CPU oracle for the Lennard-Jones MD hot path of
 * Watanabe, Suzuki and Ito, "Efficient Implementations of Molecular Dynamics
 * Simulations for Lennard-Jones Systems".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU path shares
 * no code, header, table or constant with it.
 *
 * Conventions (reduced units, unit mass):
 *   - positions, velocities, forces are arrays of N rows of 3 doubles (q[N]);
 *   - every floating-point quantity is IEEE double; per-particle and global
 *     sums accumulate in long double (x87 80-bit) so that the oracle's own
 *     rounding error sits far below the tolerances it is used to judge;
 *   - compiled with -ffp-contract=off: no silent fused multiply-adds, so the
 *     pair predicate below is exactly the written sequence of roundings.
 *
 * Parity status of each function is stated at the function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long double acc_t;

/* ------------------------------------------------------------------------- */
/* Potential (Sec. 2.1, eq. lj_cutoff)                                        */
/* ------------------------------------------------------------------------- */

/* Coefficients c2, c0 of the truncated potential
 *   V(r) = 4 eps [ (sigma/r)^12 - (sigma/r)^6 + c2 (r/sigma)^2 + c0 ]
 * fixed by V(rc) = V'(rc) = 0 (Sec. 2.1).  With x = sigma/rc:
 *   V'(rc) = 0  ->  c2 = 6 x^14 - 3 x^8
 *   V(rc)  = 0  ->  c0 = -7 x^12 + 4 x^6
 * Pinned by exact rational arithmetic in the tests (V(rc) = V'(rc) = 0). */
void mdref_lj_coeffs(double sigma, double rc, double* c2, double* c0)
{
    double x = sigma / rc;
    double x2 = x * x;
    double x6 = x2 * x2 * x2;
    double x8 = x6 * x2;
    double x12 = x6 * x6;
    double x14 = x12 * x2;
    *c2 = 6.0 * x14 - 3.0 * x8;
    *c0 = -7.0 * x12 + 4.0 * x6;
}

/* Pair energy V(r) and g(r) = -V'(r)/r at squared distance r2 (Sec. 2.1).
 * The force on particle i from j is F_i = -g d with d = q_j - q_i; this is the
 * update of the explicit force algorithm in Sec. 3.2, whose bracket
 * [(24 r^6 - 48)/r^14 + 8 c2] equals -g for eps = sigma = 1.
 * Valid for any r2 > 0; the cutoff test (r < rc) is applied by the caller. */
void mdref_pair(double r2, double eps, double sigma, double rc, double* V, double* g)
{
    double c2, c0;
    mdref_lj_coeffs(sigma, rc, &c2, &c0);
    double s2 = (sigma * sigma) / r2;       /* (sigma/r)^2 */
    double s6 = s2 * s2 * s2;               /* (sigma/r)^6 */
    double s12 = s6 * s6;                   /* (sigma/r)^12 */
    double q2 = r2 / (sigma * sigma);       /* (r/sigma)^2 */
    *V = 4.0 * eps * (s12 - s6 + c2 * q2 + c0);
    /* dV/dr = 4 eps [ -12 s12/r + 6 s6/r + 2 c2 r / sigma^2 ] */
    *g = 4.0 * eps * (12.0 * s12 - 6.0 * s6) / r2 - 8.0 * eps * c2 / (sigma * sigma);
}

/* d^2 V / dr^2 and the parameter derivatives used by the adjoint:
 *   dV/deps = V/eps,   dV/dsigma,   dg/deps = g/eps,   dg/dsigma.
 * c2 and c0 depend on sigma through x = sigma/rc, so they are differentiated
 * too (the truncation keeps V(rc) = V'(rc) = 0 for every sigma). */
void mdref_pair_derivs(double r2, double eps, double sigma, double rc,
                       double* d2V, double* dV_dsig, double* dg_dsig)
{
    double r = sqrt(r2);
    /* V = 4 eps [ sigma^12 r^-12 - sigma^6 r^-6 + c2 r^2 sigma^-2 + c0 ],
     * with c2 sigma^-2 = 6 sigma^12 rc^-14 - 3 sigma^6 rc^-8 and
     * c0 = -7 sigma^12 rc^-12 + 4 sigma^6 rc^-6.  Collect powers of sigma:
     * V = 4 eps [ sigma^12 A(r) - sigma^6 B(r) ],
     * A = r^-12 + 6 r^2 rc^-14 - 7 rc^-12,  B = r^-6 + 3 r^2 rc^-8 - 4 rc^-6. */
    double rc2 = rc * rc;
    double rc6 = rc2 * rc2 * rc2;
    double rc8 = rc6 * rc2;
    double rc12 = rc6 * rc6;
    double rc14 = rc12 * rc2;
    double ri2 = 1.0 / r2;
    double ri6 = ri2 * ri2 * ri2;
    double ri12 = ri6 * ri6;
    double sig6 = sigma * sigma * sigma * sigma * sigma * sigma;
    double sig12 = sig6 * sig6;
    double A = ri12 + 6.0 * r2 / rc14 - 7.0 / rc12;
    double B = ri6 + 3.0 * r2 / rc8 - 4.0 / rc6;
    /* dA/dr = -12 r^-13 + 12 r rc^-14 ;  d2A/dr2 = 156 r^-14 + 12 rc^-14 */
    /* dB/dr = -6 r^-7 + 6 r rc^-8 ;      d2B/dr2 = 42 r^-8 + 6 rc^-8 */
    double d2A = 156.0 * ri12 * ri2 + 12.0 / rc14;
    double d2B = 42.0 * ri6 * ri2 + 6.0 / rc8;
    *d2V = 4.0 * eps * (sig12 * d2A - sig6 * d2B);
    *dV_dsig = 4.0 * eps * (12.0 * (sig12 / sigma) * A - 6.0 * (sig6 / sigma) * B);
    /* g = -(1/r) dV/dr = -(4 eps / r) [ sigma^12 A' - sigma^6 B' ] */
    double dA = -12.0 * ri12 / r + 12.0 * r / rc14;
    double dB = -6.0 * ri6 / r + 6.0 * r / rc8;
    *dg_dsig = -(4.0 * eps / r) * (12.0 * (sig12 / sigma) * dA - 6.0 * (sig6 / sigma) * dB);
}

/* ------------------------------------------------------------------------- */
/* Periodic geometry                                                          */
/* ------------------------------------------------------------------------- */

/* Minimum image of one displacement component (periodic on all axes, Sec. 4.5).
 * For positions in [0, L) the rounded quotient is -1, 0 or 1, so L * k is exact. */
static double min_image(double d, double L, double invL)
{
    return d - L * rint(d * invL);
}

/* The pair predicate, fixed bit for bit so that two implementations can agree
 * exactly on the set of listed pairs:
 *   d = q_j - q_i per axis, minimum image, r2 = fma(dz,dz, fma(dy,dy, dx*dx)),
 *   listed iff r2 < rs^2 (strict, as the cutoff tests of Sec. 2.3 / 3.1). */
static double pair_r2(const double* qi, const double* qj, const double* L, const double* invL,
                      double* d)
{
    double dx = min_image(qj[0] - qi[0], L[0], invL[0]);
    double dy = min_image(qj[1] - qi[1], L[1], invL[1]);
    double dz = min_image(qj[2] - qi[2], L[2], invL[2]);
    if (d) { d[0] = dx; d[1] = dy; d[2] = dz; }
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

double mdref_pair_r2(const double* qi, const double* qj, const double* L)
{
    double invL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
    return pair_r2(qi, qj, L, invL, NULL);
}

/* Put a coordinate back into [0, L) after a drift: x - L floor(x/L), then the
 * two corner fixes for rounding at exactly L or just below 0. */
static double wrap_coord(double x, double L, double invL)
{
    double y = x - L * floor(x * invL);
    if (y >= L) y -= L;
    if (y < 0.0) y += L;
    return y;
}

/* ------------------------------------------------------------------------- */
/* Grid (Sec. 2.2): inexclusive cells of side >= rs, GridList counting sort   */
/* ------------------------------------------------------------------------- */

/* Number of cells per axis: the largest count whose side L/n is still >= rs.
 * Returns 0 when an axis has fewer than 3 cells (the 27-cell neighbourhood
 * would then contain repeated cells). */
int mdref_cell_dims(const double* L, double rs, int* nc)
{
    int ok = 1;
    for (int a = 0; a < 3; ++a) {
        nc[a] = (int)floor(L[a] / rs);
        if (nc[a] < 3) ok = 0;
    }
    return ok;
}

static int cell_coord(double x, double inv, int n)
{
    int c = (int)(x * inv);
    if (c > n - 1) c = n - 1;
    if (c < 0) c = 0;
    return c;
}

/* GridList construction (Sec. 2.2 and the GridList figure):
 *   1. label each particle with the serial number of its cell,
 *   2. count the particles per cell (GridParticleNumber),
 *   3. set a pointer to where each cell's first particle goes (GridPointer,
 *      the exclusive prefix sum of the counts),
 *   4. visiting particles in index order, place each index at its cell's
 *      pointer and advance that pointer.
 * Cells are numbered (cx * ny + cy) * nz + cz with cx = floor(x * nx / L)
 * (clamped to the grid).  Step 4 makes the sort stable.
 * Outputs: cell_of[n], count[nc], start[nc + 1] (start[nc] = n), order[n]. */
void mdref_bin(int64_t n, const double* q, const double* L, const int* nc,
               int32_t* cell_of, int32_t* count, int32_t* start, int32_t* order)
{
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    double inv[3];
    for (int a = 0; a < 3; ++a) inv[a] = (double)nc[a] / L[a];
    double invL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
    for (int64_t c = 0; c < ncell; ++c) count[c] = 0;
    for (int64_t i = 0; i < n; ++i) {
        /* the wrap is the identity for coordinates already in [0, L) */
        int cx = cell_coord(wrap_coord(q[3 * i + 0], L[0], invL[0]), inv[0], nc[0]);
        int cy = cell_coord(wrap_coord(q[3 * i + 1], L[1], invL[1]), inv[1], nc[1]);
        int cz = cell_coord(wrap_coord(q[3 * i + 2], L[2], invL[2]), inv[2], nc[2]);
        int32_t c = (int32_t)(((int64_t)cx * nc[1] + cy) * nc[2] + cz);
        cell_of[i] = c;
        count[c] += 1;
    }
    int64_t run = 0;
    for (int64_t c = 0; c < ncell; ++c) { start[c] = (int32_t)run; run += count[c]; }
    start[ncell] = (int32_t)run;
    int32_t* ptr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ncell > 0 ? ncell : 1));
    for (int64_t c = 0; c < ncell; ++c) ptr[c] = start[c];
    for (int64_t i = 0; i < n; ++i) order[ptr[cell_of[i]]++] = (int32_t)i;
    free(ptr);
}

/* ------------------------------------------------------------------------- */
/* Pair finding (Sec. 2.2-2.3)                                                 */
/* ------------------------------------------------------------------------- */

/* Brute force O(N^2): all i < j with minimum-image r2 < rs^2.  Writes up to
 * cap pairs, returns the number found (which may exceed cap). */
int64_t mdref_pairs_brute(int64_t n, const double* q, const double* L, double rs,
                          int64_t cap, int32_t* pi, int32_t* pj)
{
    double invL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
    double rs2 = rs * rs;
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j)
            if (pair_r2(q + 3 * i, q + 3 * j, L, invL, NULL) < rs2) {
                if (m < cap) { pi[m] = (int32_t)i; pj[m] = (int32_t)j; }
                ++m;
            }
    return m;
}

static int64_t cell_id_wrapped(int cx, int cy, int cz, const int* nc)
{
    cx = (cx % nc[0] + nc[0]) % nc[0];
    cy = (cy % nc[1] + nc[1]) % nc[1];
    cz = (cz % nc[2] + nc[2]) % nc[2];
    return ((int64_t)cx * nc[1] + cy) * nc[2] + cz;
}

/* The 13 "forward" neighbour offsets: half of the 26 surrounding cells, so that
 * each pair of distinct cells is visited once (Newton's third law, Sec. 2.3). */
static void half_stencil(int off[13][3])
{
    int m = 0;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                int key = (dx * 3 + dy) * 3 + dz;   /* in -13..13 */
                if (key > 0) { off[m][0] = dx; off[m][1] = dy; off[m][2] = dz; ++m; }
            }
}

/* Pair finding over the grid (the pair-finding algorithm of Sec. 2.3): for
 * every cell, the candidate list is the cell's own particles followed by those
 * of its 13 forward neighbours; pairs (k, l) with k over the own particles and
 * l > k over the candidate list are tested.  Needs >= 3 cells per axis.
 * Output pairs are (min id, max id).  Returns the number found. */
int64_t mdref_pairs_cells(int64_t n, const double* q, const double* L, double rs,
                          int64_t cap, int32_t* pi, int32_t* pj)
{
    int nc[3];
    if (!mdref_cell_dims(L, rs, nc)) return -1;
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int32_t* cell_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* count = (int32_t*)malloc(sizeof(int32_t) * (size_t)ncell);
    int32_t* start = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ncell + 1));
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    mdref_bin(n, q, L, nc, cell_of, count, start, order);
    double invL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
    double rs2 = rs * rs;
    int off[13][3];
    half_stencil(off);
    int64_t cand_cap = 1024;
    int32_t* cand = (int32_t*)malloc(sizeof(int32_t) * (size_t)cand_cap);
    int64_t m = 0;
    for (int cx = 0; cx < nc[0]; ++cx)
        for (int cy = 0; cy < nc[1]; ++cy)
            for (int cz = 0; cz < nc[2]; ++cz) {
                int64_t c = ((int64_t)cx * nc[1] + cy) * nc[2] + cz;
                int64_t nown = count[c];
                int64_t tot = nown;
                for (int s = 0; s < 13; ++s)
                    tot += count[cell_id_wrapped(cx + off[s][0], cy + off[s][1], cz + off[s][2], nc)];
                if (tot > cand_cap) {
                    cand_cap = 2 * tot;
                    cand = (int32_t*)realloc(cand, sizeof(int32_t) * (size_t)cand_cap);
                }
                int64_t t = 0;
                for (int64_t k = 0; k < nown; ++k) cand[t++] = order[start[c] + k];
                for (int s = 0; s < 13; ++s) {
                    int64_t nb = cell_id_wrapped(cx + off[s][0], cy + off[s][1], cz + off[s][2], nc);
                    for (int64_t k = 0; k < count[nb]; ++k) cand[t++] = order[start[nb] + k];
                }
                for (int64_t k = 0; k < nown; ++k)
                    for (int64_t l = k + 1; l < tot; ++l) {
                        int32_t a = cand[k], b = cand[l];
                        if (pair_r2(q + 3 * (int64_t)a, q + 3 * (int64_t)b, L, invL, NULL) < rs2) {
                            if (m < cap) {
                                pi[m] = a < b ? a : b;
                                pj[m] = a < b ? b : a;
                            }
                            ++m;
                        }
                    }
            }
    free(cand); free(order); free(start); free(count); free(cell_of);
    return m;
}

/* ------------------------------------------------------------------------- */
/* Forces, potential energy, virial (Sec. 3.1-3.2)                             */
/* ------------------------------------------------------------------------- */

/* Forces from a pair list: for every listed pair with r < rc (strict; pairs
 * beyond the cutoff add nothing, the if-elimination of Sec. 3.1), add
 *   F_i -= g d,  F_j += g d   with d = q_j - q_i,
 *   PE += V(r),  W += g r^2   (virial sum of r_ij . f_ij).
 * Sums are carried in long double and rounded once at the end. */
void mdref_forces_pairs(int64_t n, const double* q, const double* L,
                        double eps, double sigma, double rc,
                        int64_t npairs, const int32_t* pi, const int32_t* pj,
                        double* F, double* pe, double* w)
{
    double invL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
    double rc2 = rc * rc;
    acc_t* acc = (acc_t*)calloc((size_t)(3 * n), sizeof(acc_t));
    acc_t PE = 0.0L, W = 0.0L;
    for (int64_t p = 0; p < npairs; ++p) {
        int64_t i = pi[p], j = pj[p];
        double d[3];
        double r2 = pair_r2(q + 3 * i, q + 3 * j, L, invL, d);
        if (!(r2 < rc2)) continue;
        double V, g;
        mdref_pair(r2, eps, sigma, rc, &V, &g);
        for (int a = 0; a < 3; ++a) {
            acc[3 * i + a] -= (acc_t)g * d[a];
            acc[3 * j + a] += (acc_t)g * d[a];
        }
        PE += V;
        W += (acc_t)g * r2;
    }
    for (int64_t k = 0; k < 3 * n; ++k) F[k] = (double)acc[k];
    *pe = (double)PE;
    *w = (double)W;
    free(acc);
}

/* Forces over all pairs found by the grid search at search length rs
 * (any rs >= rc gives the same result up to summation order). */
int mdref_forces(int64_t n, const double* q, const double* L, double eps, double sigma,
                 double rc, double rs, double* F, double* pe, double* w)
{
    int nc[3];
    int64_t cap, m;
    int32_t *pi, *pj;
    int use_cells = mdref_cell_dims(L, rs, nc);
    if (!use_cells && !(rs < 0.5 * L[0] && rs < 0.5 * L[1] && rs < 0.5 * L[2])) return -2;
    cap = n * 64 + 1024;
    for (;;) {
        pi = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
        pj = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
        m = use_cells ? mdref_pairs_cells(n, q, L, rs, cap, pi, pj)
                      : mdref_pairs_brute(n, q, L, rs, cap, pi, pj);
        if (m <= cap) break;
        free(pi); free(pj);
        cap = m;
    }
    mdref_forces_pairs(n, q, L, eps, sigma, rc, m, pi, pj, F, pe, w);
    free(pi); free(pj);
    return 0;
}

/* Forces on a sample of particles only, by a direct scan of the 27 cells
 * around each sampled particle (no stored list); for checking very large
 * systems one particle at a time.  Also returns, per sampled particle,
 *   S_i  = sum_j |g_ij| r_ij  (the scale of the pair forces acting on i),
 *   pe_i = (1/2) sum_j V(r_ij),  w_i = (1/2) sum_j g_ij r_ij^2,
 *   nb_i = the number of partners with r < rs (list row length).
 * cell_of/count/start/order are a GridList of q (from mdref_bin). */
void mdref_forces_sample(int64_t n, const double* q, const double* L, double eps, double sigma,
                         double rc, double rs, const int* nc,
                         const int32_t* count, const int32_t* start, const int32_t* order,
                         int64_t nsample, const int64_t* idx,
                         double* F, double* S, double* pe_i, double* w_i, int32_t* nb_i)
{
    (void)n;
    double invL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
    double inv[3];
    for (int a = 0; a < 3; ++a) inv[a] = (double)nc[a] / L[a];
    double rc2 = rc * rc, rs2 = rs * rs;
    for (int64_t s = 0; s < nsample; ++s) {
        int64_t i = idx[s];
        const double* qi = q + 3 * i;
        int cx = cell_coord(wrap_coord(qi[0], L[0], invL[0]), inv[0], nc[0]);
        int cy = cell_coord(wrap_coord(qi[1], L[1], invL[1]), inv[1], nc[1]);
        int cz = cell_coord(wrap_coord(qi[2], L[2], invL[2]), inv[2], nc[2]);
        acc_t f[3] = {0, 0, 0}, sc = 0, pe = 0, w = 0;
        int32_t nb = 0;
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    int64_t c = cell_id_wrapped(cx + dx, cy + dy, cz + dz, nc);
                    for (int32_t k = 0; k < count[c]; ++k) {
                        int64_t j = order[start[c] + k];
                        if (j == i) continue;
                        double d[3];
                        double r2 = pair_r2(qi, q + 3 * j, L, invL, d);
                        if (r2 < rs2) ++nb;
                        if (!(r2 < rc2)) continue;
                        double V, g;
                        mdref_pair(r2, eps, sigma, rc, &V, &g);
                        for (int a = 0; a < 3; ++a) f[a] -= (acc_t)g * d[a];
                        sc += fabsl((acc_t)g) * sqrtl((acc_t)r2);
                        pe += 0.5L * V;
                        w += 0.5L * (acc_t)g * r2;
                    }
                }
        for (int a = 0; a < 3; ++a) F[3 * s + a] = (double)f[a];
        S[s] = (double)sc;
        pe_i[s] = (double)pe;
        w_i[s] = (double)w;
        nb_i[s] = nb;
    }
}

/* Neighbour sets of sampled particles: all j != i with r2 < rs^2 (the row of
 * i in a full list), written as ids in increasing order.  Returns the total
 * number written (rows are delimited by rowlen). */
int64_t mdref_neighbors_sample(const double* q, const double* L, double rs, const int* nc,
                               const int32_t* count, const int32_t* start, const int32_t* order,
                               int64_t nsample, const int64_t* idx, int64_t cap,
                               int32_t* rowlen, int32_t* out)
{
    double invL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
    double inv[3];
    for (int a = 0; a < 3; ++a) inv[a] = (double)nc[a] / L[a];
    double rs2 = rs * rs;
    int64_t m = 0;
    for (int64_t s = 0; s < nsample; ++s) {
        int64_t i = idx[s];
        const double* qi = q + 3 * i;
        int cx = cell_coord(wrap_coord(qi[0], L[0], invL[0]), inv[0], nc[0]);
        int cy = cell_coord(wrap_coord(qi[1], L[1], invL[1]), inv[1], nc[1]);
        int cz = cell_coord(wrap_coord(qi[2], L[2], invL[2]), inv[2], nc[2]);
        int64_t m0 = m;
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    int64_t c = cell_id_wrapped(cx + dx, cy + dy, cz + dz, nc);
                    for (int32_t k = 0; k < count[c]; ++k) {
                        int32_t j = order[start[c] + k];
                        if (j == i) continue;
                        if (pair_r2(qi, q + 3 * (int64_t)j, L, invL, NULL) < rs2) {
                            /* insertion into the sorted tail of this row */
                            int64_t p = m;
                            if (p < cap) {
                                while (p > m0 && out[p - 1] > j) { out[p] = out[p - 1]; --p; }
                                out[p] = j;
                            }
                            ++m;
                        }
                    }
                }
        rowlen[s] = (int32_t)(m - m0);
    }
    return m;
}

/* ------------------------------------------------------------------------- */
/* Velocity Verlet with the bookkeeping (skin) rebuild rule                    */
/* ------------------------------------------------------------------------- */

typedef struct {
    int64_t n;
    double L[3];
    double eps, sigma, rc, rs;
    int32_t* pi;
    int32_t* pj;
    int64_t npairs, cap;
    double* qref;
} list_t;

static int list_build(list_t* ls, const double* q)
{
    int nc[3];
    int use_cells = mdref_cell_dims(ls->L, ls->rs, nc);
    for (;;) {
        int64_t m = use_cells ? mdref_pairs_cells(ls->n, q, ls->L, ls->rs, ls->cap, ls->pi, ls->pj)
                              : mdref_pairs_brute(ls->n, q, ls->L, ls->rs, ls->cap, ls->pi, ls->pj);
        if (m < 0) return -1;
        if (m <= ls->cap) { ls->npairs = m; break; }
        ls->cap = m + m / 4;
        ls->pi = (int32_t*)realloc(ls->pi, sizeof(int32_t) * (size_t)ls->cap);
        ls->pj = (int32_t*)realloc(ls->pj, sizeof(int32_t) * (size_t)ls->cap);
    }
    memcpy(ls->qref, q, sizeof(double) * (size_t)(3 * ls->n));
    return 0;
}

static double max_disp2(const list_t* ls, const double* q)
{
    double invL[3] = {1.0 / ls->L[0], 1.0 / ls->L[1], 1.0 / ls->L[2]};
    double m = 0.0;
    for (int64_t i = 0; i < ls->n; ++i) {
        double d2 = pair_r2(ls->qref + 3 * i, q + 3 * i, ls->L, invL, NULL);
        if (d2 > m) m = d2;
    }
    return m;
}

/* ------------------------------------------------------------------------- */
/* Validity check of a pair list: DUTC and LDC (Sec. 2.3, Alg. alg_validity_check) */
/* ------------------------------------------------------------------------- */

/* Large-displacement check.  The list built at positions qold lists every pair
 * whose (pinned) squared distance was below rs^2.  It becomes invalid only if
 * some pair not listed (old squared distance >= rs^2; the paper writes "> rs",
 * read here as the complement of the strict list predicate) now interacts
 * (squared distance < rc^2).  Such a pair needs dr_i + dr_j > rs - rc, where
 * dr_i = |q_i - qold_i|, so only particles with dr_i > t = (rs - rc) - dr_max
 * can take part (dr_max the largest displacement).  The test is made on
 * squares: member iff t < 0 or dr_i^2 > t^2, with t lowered by 1e-12 so that
 * rounding can only add members.  More than n_l members invalidates the list
 * outright; otherwise every pair of members is checked.
 * Returns 1 if the list is still valid, 0 if not; *n_ld = member count,
 * *dmax2 = dr_max^2. */
int mdref_ldc_check(int64_t n, const double* q, const double* qold, const double* L, double rc, double rs,
                    int64_t n_l, int64_t* n_ld, double* dmax2)
{
    double invL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d2 = pair_r2(qold + 3 * i, q + 3 * i, L, invL, NULL);
        if (d2 > m) m = d2;
    }
    *dmax2 = m;
    double t = (rs - rc) - sqrt(m) - 1e-12;
    double t2 = t * t;
    int64_t cnt = 0;
    int64_t* ld = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_l > 0 ? n_l : 1));
    for (int64_t i = 0; i < n; ++i) {
        double d2 = pair_r2(qold + 3 * i, q + 3 * i, L, invL, NULL);
        if (t < 0.0 || d2 > t2) {
            if (cnt < n_l) ld[cnt] = i;
            ++cnt;
        }
    }
    *n_ld = cnt;
    int valid = cnt <= n_l;
    double rs2 = rs * rs, rc2 = rc * rc;
    for (int64_t a = 0; valid && a < cnt; ++a)
        for (int64_t b = a + 1; b < cnt; ++b) {
            const int64_t i = ld[a], j = ld[b];
            if (pair_r2(qold + 3 * i, qold + 3 * j, L, invL, NULL) >= rs2 &&
                pair_r2(q + 3 * i, q + 3 * j, L, invL, NULL) < rc2) {
                valid = 0;
                break;
            }
        }
    free(ld);
    return valid;
}

/* Largest squared speed, |v|^2 = fma(vz,vz, fma(vy,vy, vx*vx)) (the DUTC's
 * v_max, Sec. 2.3), over the velocities v[n][3]. */
static double max_speed2(int64_t n, const double* v)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = fma(v[3 * i + 2], v[3 * i + 2], fma(v[3 * i + 1], v[3 * i + 1], v[3 * i] * v[3 * i]));
        if (s > m) m = s;
    }
    return m;
}

static acc_t kinetic(int64_t n, const double* v)
{
    acc_t k = 0.0L;
    for (int64_t i = 0; i < 3 * n; ++i) k += (acc_t)v[i] * v[i];
    return 0.5L * k;
}

/* NVE run with velocity Verlet (kick-drift-kick, unit mass):
 *   v += (dt/2) F;  q = wrap(q + dt v);  [rebuild?];  F = F(q);  v += (dt/2) F.
 * The paper specifies a second-order symplectic integrator (Sec. 4.5); velocity
 * Verlet is that scheme.  Rebuild rules:
 *   rule 0, half skin (Sec. 2.3 and the search-length figure): the list of
 *     pairs within rs stays valid until some particle has moved more than half
 *     the margin rs - rc since the last build, so the list is rebuilt when
 *     max_i |q_i - q_i^ref|^2 > ((rs - rc)/2)^2;
 *   rule 1, DUTC then LDC (Alg. alg_validity_check): at each build the buffer
 *     length is rs - rc; each step it shrinks by 2 v_max dt, with v_max the
 *     largest speed of the drift just made; while it is positive the list is
 *     valid, afterwards the large-displacement check decides (n_l members at
 *     most).
 * Every sample_every steps, log[k] = (KE, PE, W, KE + PE) after the step.
 * stats = (rebuild count, pairs at last build, LDC checks made, LDC checks that
 * kept the list).  Returns 0, or -1 on a geometry error. */
int mdref_run(int64_t n, double* q, double* v, const double* L, double eps, double sigma,
              double rc, double rs, double dt, int64_t nsteps, int64_t sample_every,
              double* log, int64_t* stats, int32_t rule, int64_t n_l)
{
    list_t ls;
    memset(&ls, 0, sizeof(ls));
    ls.n = n;
    for (int a = 0; a < 3; ++a) ls.L[a] = L[a];
    ls.eps = eps; ls.sigma = sigma; ls.rc = rc; ls.rs = rs;
    ls.cap = n * 32 + 1024;
    ls.pi = (int32_t*)malloc(sizeof(int32_t) * (size_t)ls.cap);
    ls.pj = (int32_t*)malloc(sizeof(int32_t) * (size_t)ls.cap);
    ls.qref = (double*)malloc(sizeof(double) * (size_t)(3 * n));
    double* F = (double*)malloc(sizeof(double) * (size_t)(3 * n));
    double invL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
    double half_skin = 0.5 * (rs - rc);
    double thr2 = half_skin * half_skin;
    double h = 0.5 * dt;
    double pe, w;
    int64_t rebuilds = 0, k = 0, checks = 0, kept = 0;
    double buffer = rs - rc;
    if (list_build(&ls, q) != 0) { stats[0] = -1; return -1; }
    mdref_forces_pairs(n, q, L, eps, sigma, rc, ls.npairs, ls.pi, ls.pj, F, &pe, &w);
    for (int64_t s = 1; s <= nsteps; ++s) {
        for (int64_t i = 0; i < 3 * n; ++i) v[i] = v[i] + h * F[i];
        for (int64_t i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a)
                q[3 * i + a] = wrap_coord(q[3 * i + a] + dt * v[3 * i + a], L[a], invL[a]);
        int rebuild;
        if (rule == 0) {
            rebuild = max_disp2(&ls, q) > thr2;
        } else {
            buffer -= 2.0 * sqrt(max_speed2(n, v)) * dt;
            rebuild = 0;
            if (!(buffer > 0.0)) {
                int64_t nld;
                double dm2;
                ++checks;
                rebuild = !mdref_ldc_check(n, q, ls.qref, L, rc, rs, n_l, &nld, &dm2);
                kept += !rebuild;
            }
        }
        if (rebuild) {
            list_build(&ls, q);
            ++rebuilds;
            buffer = rs - rc;
        }
        mdref_forces_pairs(n, q, L, eps, sigma, rc, ls.npairs, ls.pi, ls.pj, F, &pe, &w);
        for (int64_t i = 0; i < 3 * n; ++i) v[i] = v[i] + h * F[i];
        if (sample_every > 0 && s % sample_every == 0) {
            acc_t ke = kinetic(n, v);
            log[4 * k + 0] = (double)ke;
            log[4 * k + 1] = pe;
            log[4 * k + 2] = w;
            log[4 * k + 3] = (double)(ke + (acc_t)pe);
            ++k;
        }
    }
    stats[0] = rebuilds;
    stats[1] = ls.npairs;
    stats[2] = checks;
    stats[3] = kept;
    free(F); free(ls.qref); free(ls.pi); free(ls.pj);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Adjoint: Hessian-vector product and parameter derivatives                   */
/* ------------------------------------------------------------------------- */

/* Plain pair list of all pairs within rc (via the grid search at rs) */
static int64_t pairs_for(int64_t n, const double* q, const double* L, double rs,
                         int32_t** pi, int32_t** pj)
{
    int nc[3];
    int use_cells = mdref_cell_dims(L, rs, nc);
    int64_t cap = n * 32 + 1024, m;
    for (;;) {
        *pi = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
        *pj = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
        m = use_cells ? mdref_pairs_cells(n, q, L, rs, cap, *pi, *pj)
                      : mdref_pairs_brute(n, q, L, rs, cap, *pi, *pj);
        if (m <= cap) return m;
        free(*pi); free(*pj);
        cap = m;
    }
}

/* Hessian-vector product of U(q) = sum_pairs V(|q_j - q_i|):
 *   (H u)_i = sum_j d^2 V/dq_i dq_j u_j.
 * For one pair with unit vector e = d/r and du = u_j - u_i, the pair adds
 *   -[ (V'' - V'/r) (e . du) e + (V'/r) du ]  to (H u)_i  and the negative
 * to (H u)_j.  Pairs with r >= rc add nothing.
 * Also returns dparam[0..1] = u . dF/d(eps, sigma), the derivative of the force
 * field contracted with u (F_i = -sum_j g d_ij), i.e. per pair
 *   (dg/dtheta) d . (u_j - u_i). */
void mdref_hvp(int64_t n, const double* q, const double* L, double eps, double sigma,
               double rc, double rs, const double* u, double* Hu, double* dparam)
{
    int32_t *pi, *pj;
    int64_t m = pairs_for(n, q, L, rs, &pi, &pj);
    double invL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
    double rc2 = rc * rc;
    acc_t* acc = (acc_t*)calloc((size_t)(3 * n), sizeof(acc_t));
    acc_t de = 0.0L, ds = 0.0L;
    for (int64_t p = 0; p < m; ++p) {
        int64_t i = pi[p], j = pj[p];
        double d[3];
        double r2 = pair_r2(q + 3 * i, q + 3 * j, L, invL, d);
        if (!(r2 < rc2)) continue;
        double r = sqrt(r2);
        double V, g, d2V, dVs, dgs;
        mdref_pair(r2, eps, sigma, rc, &V, &g);
        mdref_pair_derivs(r2, eps, sigma, rc, &d2V, &dVs, &dgs);
        double dVr = -g;                 /* V'(r)/r */
        double du[3], edu = 0.0, e[3];
        for (int a = 0; a < 3; ++a) {
            e[a] = d[a] / r;
            du[a] = u[3 * j + a] - u[3 * i + a];
            edu += e[a] * du[a];
        }
        for (int a = 0; a < 3; ++a) {
            acc_t t = (acc_t)(d2V - dVr) * edu * e[a] + (acc_t)dVr * du[a];
            acc[3 * i + a] -= t;
            acc[3 * j + a] += t;
        }
        double ddu = d[0] * du[0] + d[1] * du[1] + d[2] * du[2];
        de += (acc_t)(g / eps) * ddu;
        ds += (acc_t)dgs * ddu;
    }
    for (int64_t k = 0; k < 3 * n; ++k) Hu[k] = (double)acc[k];
    dparam[0] = (double)de;
    dparam[1] = (double)ds;
    free(acc); free(pi); free(pj);
}

/* dU/deps and dU/dsigma of the total potential energy (sum over pairs within
 * rc of dV/deps = V/eps and dV/dsigma). */
void mdref_param_grad(int64_t n, const double* q, const double* L, double eps, double sigma,
                      double rc, double rs, double* dU)
{
    int32_t *pi, *pj;
    int64_t m = pairs_for(n, q, L, rs, &pi, &pj);
    double invL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
    double rc2 = rc * rc;
    acc_t de = 0.0L, ds = 0.0L;
    for (int64_t p = 0; p < m; ++p) {
        double r2 = pair_r2(q + 3 * (int64_t)pi[p], q + 3 * (int64_t)pj[p], L, invL, NULL);
        if (!(r2 < rc2)) continue;
        double V, g, d2V, dVs, dgs;
        mdref_pair(r2, eps, sigma, rc, &V, &g);
        mdref_pair_derivs(r2, eps, sigma, rc, &d2V, &dVs, &dgs);
        de += (acc_t)V / eps;
        ds += dVs;
    }
    dU[0] = (double)de;
    dU[1] = (double)ds;
    free(pi); free(pj);
}

/* Gradient of the trajectory observable
 *   O = (1/K) sum_{k=1..K} U(q_k)
 * over K velocity-Verlet steps from (q0, v0), with respect to q0 (v0 held
 * fixed), eps and sigma.  Forward states are stored every `ckpt` steps and each
 * segment is recomputed before it is swept backwards (checkpointing).
 * The reverse sweep of one step
 *   v' = v + h F(q);  q' = q + dt v';  v'' = v' + h F(q')      (h = dt/2)
 * with adjoints (a_q, a_v) and F = -grad U, dF/dq = -H:
 *   a_q' += -h H(q') a_v''            (second kick)
 *   a_v'  = a_v'' + dt a_q'           (drift)
 *   a_q   = a_q' - h H(q) a_v'        (first kick)
 * and the parameter adjoint collects h * a_v . dF/dtheta at both kicks.
 * Positions are not wrapped during the run (the wrap is a relabelling of the
 * same periodic point and has zero derivative).  Outputs: O, gq[3n], gparam[2]. */
int mdref_traj_mean_pe_grad(int64_t n, const double* q0, const double* v0, const double* L,
                            double eps, double sigma, double rc, double rs, double dt,
                            int64_t K, int64_t ckpt, double* O, double* gq, double* gparam)
{
    int64_t nseg = (K + ckpt - 1) / ckpt;
    size_t sz = (size_t)(3 * n);
    double* cq = (double*)malloc(sizeof(double) * sz * (size_t)nseg);
    double* cv = (double*)malloc(sizeof(double) * sz * (size_t)nseg);
    double* q = (double*)malloc(sizeof(double) * sz);
    double* v = (double*)malloc(sizeof(double) * sz);
    double* F = (double*)malloc(sizeof(double) * sz);
    double* segq = (double*)malloc(sizeof(double) * sz * (size_t)(ckpt + 1));
    double* aq = (double*)calloc(sz, sizeof(double));
    double* av = (double*)calloc(sz, sizeof(double));
    double* Hu = (double*)malloc(sizeof(double) * sz);
    double h = 0.5 * dt;
    double pe, w, dp[2], dU[2];
    acc_t Osum = 0.0L, gth[2] = {0.0L, 0.0L};
    memcpy(q, q0, sizeof(double) * sz);
    memcpy(v, v0, sizeof(double) * sz);
    if (mdref_forces(n, q, L, eps, sigma, rc, rs, F, &pe, &w) != 0) return -2;
    /* forward pass: checkpoints and the observable */
    for (int64_t k = 0; k < K; ++k) {
        if (k % ckpt == 0) {
            memcpy(cq + sz * (size_t)(k / ckpt), q, sizeof(double) * sz);
            memcpy(cv + sz * (size_t)(k / ckpt), v, sizeof(double) * sz);
        }
        for (size_t i = 0; i < sz; ++i) v[i] += h * F[i];
        for (size_t i = 0; i < sz; ++i) q[i] += dt * v[i];
        mdref_forces(n, q, L, eps, sigma, rc, rs, F, &pe, &w);
        for (size_t i = 0; i < sz; ++i) v[i] += h * F[i];
        Osum += pe;
    }
    *O = (double)(Osum / (acc_t)K);
    /* backward pass, one segment at a time */
    double invK = 1.0 / (double)K;
    for (int64_t sgi = nseg - 1; sgi >= 0; --sgi) {
        int64_t k0 = sgi * ckpt;
        int64_t k1 = k0 + ckpt < K ? k0 + ckpt : K;
        memcpy(q, cq + sz * (size_t)sgi, sizeof(double) * sz);
        memcpy(v, cv + sz * (size_t)sgi, sizeof(double) * sz);
        memcpy(segq, q, sizeof(double) * sz);
        mdref_forces(n, q, L, eps, sigma, rc, rs, F, &pe, &w);
        for (int64_t k = k0; k < k1; ++k) {
            for (size_t i = 0; i < sz; ++i) v[i] += h * F[i];
            for (size_t i = 0; i < sz; ++i) q[i] += dt * v[i];
            mdref_forces(n, q, L, eps, sigma, rc, rs, F, &pe, &w);
            for (size_t i = 0; i < sz; ++i) v[i] += h * F[i];
            memcpy(segq + sz * (size_t)(k - k0 + 1), q, sizeof(double) * sz);
        }
        for (int64_t k = k1 - 1; k >= k0; --k) {
            const double* qa = segq + sz * (size_t)(k - k0);      /* q_k */
            const double* qb = segq + sz * (size_t)(k - k0 + 1);  /* q_{k+1} */
            /* observable term at q_{k+1}: dO/dq = (1/K) grad U = -(1/K) F */
            mdref_forces(n, qb, L, eps, sigma, rc, rs, F, &pe, &w);
            for (size_t i = 0; i < sz; ++i) aq[i] -= invK * F[i];
            mdref_param_grad(n, qb, L, eps, sigma, rc, rs, dU);
            gth[0] += (acc_t)invK * dU[0];
            gth[1] += (acc_t)invK * dU[1];
            /* second kick at q_{k+1} */
            mdref_hvp(n, qb, L, eps, sigma, rc, rs, av, Hu, dp);
            for (size_t i = 0; i < sz; ++i) aq[i] -= h * Hu[i];
            gth[0] += (acc_t)h * dp[0];
            gth[1] += (acc_t)h * dp[1];
            /* drift */
            for (size_t i = 0; i < sz; ++i) av[i] += dt * aq[i];
            /* first kick at q_k */
            mdref_hvp(n, qa, L, eps, sigma, rc, rs, av, Hu, dp);
            for (size_t i = 0; i < sz; ++i) aq[i] -= h * Hu[i];
            gth[0] += (acc_t)h * dp[0];
            gth[1] += (acc_t)h * dp[1];
        }
    }
    memcpy(gq, aq, sizeof(double) * sz);
    gparam[0] = (double)gth[0];
    gparam[1] = (double)gth[1];
    free(cq); free(cv); free(q); free(v); free(F); free(segq); free(aq); free(av); free(Hu);
    return 0;
}
