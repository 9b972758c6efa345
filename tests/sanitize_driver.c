/*
 * Drives every entry point of the CPU oracle once on a small jittered fcc
 * lattice, so that the oracle can be built and run under AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure, host code only).  It also
 * checks a few facts that tie the calls together: the grid search and the
 * all-pairs search find the same number of pairs, the grid force equals the
 * force summed over the all-pairs list, a list is valid at the positions it
 * was built at, and both rebuild rules run.  Prints "OK" and exits 0 when all
 * hold.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void mdref_lj_coeffs(double sigma, double rc, double* c2, double* c0);
void mdref_pair(double r2, double eps, double sigma, double rc, double* V, double* g);
void mdref_pair_derivs(double r2, double eps, double sigma, double rc, double* d2V, double* dV_dsig,
                       double* dg_dsig);
double mdref_pair_r2(const double* qi, const double* qj, const double* L);
int mdref_cell_dims(const double* L, double rs, int* nc);
void mdref_bin(int64_t n, const double* q, const double* L, const int* nc, int32_t* cell_of, int32_t* count,
               int32_t* start, int32_t* order);
int64_t mdref_pairs_brute(int64_t n, const double* q, const double* L, double rs, int64_t cap, int32_t* pi,
                          int32_t* pj);
int64_t mdref_pairs_cells(int64_t n, const double* q, const double* L, double rs, int64_t cap, int32_t* pi,
                          int32_t* pj);
void mdref_forces_pairs(int64_t n, const double* q, const double* L, double eps, double sigma, double rc,
                        int64_t npairs, const int32_t* pi, const int32_t* pj, double* F, double* pe, double* w);
int mdref_forces(int64_t n, const double* q, const double* L, double eps, double sigma, double rc, double rs,
                 double* F, double* pe, double* w);
void mdref_forces_sample(int64_t n, const double* q, const double* L, double eps, double sigma, double rc,
                         double rs, const int* nc, const int32_t* count, const int32_t* start,
                         const int32_t* order, int64_t nsample, const int64_t* idx, double* F, double* S,
                         double* pe_i, double* w_i, int32_t* nb_i);
int64_t mdref_neighbors_sample(const double* q, const double* L, double rs, const int* nc, const int32_t* count,
                               const int32_t* start, const int32_t* order, int64_t nsample, const int64_t* idx,
                               int64_t cap, int32_t* rowlen, int32_t* out);
int mdref_ldc_check(int64_t n, const double* q, const double* qold, const double* L, double rc, double rs,
                    int64_t n_l, int64_t* n_ld, double* dmax2);
int mdref_run(int64_t n, double* q, double* v, const double* L, double eps, double sigma, double rc, double rs,
              double dt, int64_t nsteps, int64_t sample_every, double* log, int64_t* stats, int32_t rule,
              int64_t n_l);
void mdref_hvp(int64_t n, const double* q, const double* L, double eps, double sigma, double rc, double rs,
               const double* u, double* Hu, double* dparam);
void mdref_param_grad(int64_t n, const double* q, const double* L, double eps, double sigma, double rc,
                      double rs, double* dU);
int mdref_traj_mean_pe_grad(int64_t n, const double* q0, const double* v0, const double* L, double eps,
                            double sigma, double rc, double rs, double dt, int64_t K, int64_t ckpt, double* O,
                            double* gq, double* gparam);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static double uniform(void) /* splitmix64, top 53 bits */
{
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

#define FAIL(msg)                                   \
    do {                                            \
        fprintf(stderr, "sanitize driver: %s\n", msg); \
        return 1;                                   \
    } while (0)

int main(void)
{
    const int m = 6;
    const int64_t n = 4 * m * m * m;
    const double a = cbrt(4.0 / 0.8442);
    const double L[3] = {m * a, m * a, m * a};
    const double eps = 1.0, sigma = 1.0, rc = 2.5, rs = 2.8, dt = 0.005;
    const double basis[4][3] = {{0, 0, 0}, {0.5, 0.5, 0}, {0.5, 0, 0.5}, {0, 0.5, 0.5}};
    double* q = malloc(sizeof(double) * 3 * n);
    double* v = malloc(sizeof(double) * 3 * n);
    int64_t k = 0;
    for (int x = 0; x < m; ++x)
        for (int y = 0; y < m; ++y)
            for (int z = 0; z < m; ++z)
                for (int b = 0; b < 4; ++b, ++k) {
                    const int c[3] = {x, y, z};
                    for (int d = 0; d < 3; ++d) {
                        double t = (c[d] + basis[b][d]) * a + 0.1 * (uniform() - 0.5);
                        q[3 * k + d] = t - L[d] * floor(t / L[d]);
                        v[3 * k + d] = uniform() - 0.5;
                    }
                }

    double c2, c0, V, g, d2V, dVs, dgs;
    mdref_lj_coeffs(sigma, rc, &c2, &c0);
    mdref_pair(1.2, eps, sigma, rc, &V, &g);
    mdref_pair_derivs(1.2, eps, sigma, rc, &d2V, &dVs, &dgs);
    (void)mdref_pair_r2(q, q + 3, L);

    int nc[3];
    if (!mdref_cell_dims(L, rs, nc)) FAIL("box too small");
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int32_t* cell_of = malloc(sizeof(int32_t) * n);
    int32_t* count = malloc(sizeof(int32_t) * ncell);
    int32_t* start = malloc(sizeof(int32_t) * (ncell + 1));
    int32_t* order = malloc(sizeof(int32_t) * n);
    mdref_bin(n, q, L, nc, cell_of, count, start, order);

    const int64_t cap = 64 * n;
    int32_t* pi = malloc(sizeof(int32_t) * cap);
    int32_t* pj = malloc(sizeof(int32_t) * cap);
    const int64_t mb = mdref_pairs_brute(n, q, L, rs, cap, pi, pj);
    const int64_t mc = mdref_pairs_cells(n, q, L, rs, cap, pi + 0, pj + 0);
    if (mb <= 0 || mb > cap || mc != mb) FAIL("grid and all-pairs counts differ");
    (void)mdref_pairs_brute(n, q, L, rs, cap, pi, pj);

    double* F1 = malloc(sizeof(double) * 3 * n);
    double* F2 = malloc(sizeof(double) * 3 * n);
    double pe1, w1, pe2, w2;
    mdref_forces_pairs(n, q, L, eps, sigma, rc, mb, pi, pj, F1, &pe1, &w1);
    if (mdref_forces(n, q, L, eps, sigma, rc, rs, F2, &pe2, &w2) != 0) FAIL("forces failed");
    for (int64_t i = 0; i < 3 * n; ++i)
        if (fabs(F1[i] - F2[i]) > 1e-12 * (1.0 + fabs(F1[i]))) FAIL("grid force differs from pair-list force");
    if (fabs(pe1 - pe2) > 1e-12 * fabs(pe1)) FAIL("potential energies differ");

    const int64_t ns = 5;
    const int64_t idx[5] = {0, 1, n / 2, n - 2, n - 1};
    double Fs[15], S[5], pes[5], ws[5];
    int32_t nb[5], rowlen[5];
    mdref_forces_sample(n, q, L, eps, sigma, rc, rs, nc, count, start, order, ns, idx, Fs, S, pes, ws, nb);
    int32_t* rows = malloc(sizeof(int32_t) * 1024);
    if (mdref_neighbors_sample(q, L, rs, nc, count, start, order, ns, idx, 1024, rowlen, rows) > 1024)
        FAIL("neighbour rows overflow");
    (void)mdref_neighbors_sample(q, L, rs, nc, count, start, order, ns, idx, 4, rowlen, rows);

    int64_t nld;
    double dmax2;
    if (!mdref_ldc_check(n, q, q, L, rc, rs, 16, &nld, &dmax2)) FAIL("list invalid where it was built");

    double* u = malloc(sizeof(double) * 3 * n);
    double* Hu = malloc(sizeof(double) * 3 * n);
    double dp[2], dU[2];
    for (int64_t i = 0; i < 3 * n; ++i) u[i] = uniform() - 0.5;
    mdref_hvp(n, q, L, eps, sigma, rc, rs, u, Hu, dp);
    mdref_param_grad(n, q, L, eps, sigma, rc, rs, dU);

    double O, gp[2];
    double* gq = malloc(sizeof(double) * 3 * n);
    if (mdref_traj_mean_pe_grad(n, q, v, L, eps, sigma, rc, rs, dt, 12, 5, &O, gq, gp) != 0)
        FAIL("trajectory gradient failed");

    double log[4 * 4];
    int64_t stats[4];
    for (int rule = 0; rule < 2; ++rule) {
        double* qr = malloc(sizeof(double) * 3 * n);
        double* vr = malloc(sizeof(double) * 3 * n);
        for (int64_t i = 0; i < 3 * n; ++i) {
            qr[i] = q[i];
            vr[i] = 4.0 * v[i];
        }
        if (mdref_run(n, qr, vr, L, eps, sigma, rc, rs, dt, 40, 10, log, stats, rule, 64) != 0)
            FAIL("run failed");
        if (stats[0] < 1) FAIL("fast run never rebuilt");
        free(qr);
        free(vr);
    }

    free(q), free(v), free(cell_of), free(count), free(start), free(order), free(pi), free(pj);
    free(F1), free(F2), free(rows), free(u), free(Hu), free(gq);
    printf("OK\n");
    return 0;
}
