/* Exercises the CPU oracle under AddressSanitizer / UndefinedBehaviorSanitizer: dense and
 * banded QR (complex and real), products with T and T^H, gradients and lag sums on small
 * random problems (every shape class: m > n, m < n, m = n, single entries), with
 * consistency checks between the dense and the banded solvers.  Exit status 0 = clean. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int tikh_oracle_qr_solve(int64_t m, int64_t n, const double* col, const double* row, const double* top,
                         const double* bot, double lambda, double* x, int nthreads);
int tikh_oracle_band_solve(int64_t m, int64_t n, const double* col, const double* row, int64_t nrhs,
                           const double* top, const double* bot, double lambda, double* x);
int tikh_oracle_band_solve_real(int64_t m, int64_t n, const double* col, const double* row, int64_t nrhs,
                                const double* top, const double* bot, double lambda, double* x);
void tikh_oracle_T_apply(int64_t m, int64_t n, const double* col, const double* row, const double* v, double* y);
void tikh_oracle_TH_apply(int64_t m, int64_t n, const double* col, const double* row, const double* v, double* y);
int tikh_oracle_gradients(int64_t m, int64_t n, const double* col, const double* row, const double* b,
                          double lambda, const double* gx, double* x, double* gb, double* gcol, double* grow,
                          double* glam, int nthreads);
void tikh_oracle_lag_sums(int64_t m, int64_t n, const double* r, const double* w, const double* Tw,
                          const double* x, double* gcol, double* grow);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static double urand(void) {   /* splitmix64 -> [-1, 1) */
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}
static double* cvec(int64_t k) {   /* complex interleaved */
    double* v = malloc(sizeof(double) * 2 * (size_t)(k > 0 ? k : 1));
    for (int64_t i = 0; i < 2 * k; ++i) v[i] = urand();
    return v;
}

int main(void) {
    const int64_t shapes[][2] = {{1, 1}, {1, 4}, {4, 1}, {7, 3}, {3, 7}, {20, 20}, {33, 17}, {17, 33}};
    int bad = 0;
    for (size_t t = 0; t < sizeof shapes / sizeof shapes[0]; ++t) {
        const int64_t m = shapes[t][0], n = shapes[t][1];
        const double lam = 0.3;
        double *col = cvec(m), *row = cvec(n), *b = cvec(m), *gx = cvec(n);
        row[0] = col[0]; row[1] = col[1];
        double *xd = cvec(n), *xb = cvec(n), *y = cvec(m), *z = cvec(n);
        double *x = cvec(n), *gb = cvec(m), *gcol = cvec(m), *grow = cvec(n), glam = 0.0;
        bad |= tikh_oracle_qr_solve(m, n, col, row, b, NULL, lam, xd, 1) != 0;
        bad |= tikh_oracle_band_solve(m, n, col, row, 1, b, NULL, lam, xb) != 0;
        double e = 0.0, s = 0.0;
        for (int64_t i = 0; i < 2 * n; ++i) { e += (xd[i] - xb[i]) * (xd[i] - xb[i]); s += xd[i] * xd[i]; }
        if (!(e <= 1e-24 * (s + 1e-300))) { bad = 1; fprintf(stderr, "dense/band mismatch at %lld x %lld\n", (long long)m, (long long)n); }
        tikh_oracle_T_apply(m, n, col, row, xd, y);
        tikh_oracle_TH_apply(m, n, col, row, y, z);
        bad |= tikh_oracle_gradients(m, n, col, row, b, lam, gx, x, gb, gcol, grow, &glam, 1) != 0;
        tikh_oracle_lag_sums(m, n, b, gx, y, xd, gcol, grow);
        /* real variant on the real parts */
        double *rc = malloc(sizeof(double) * m), *rr = malloc(sizeof(double) * n), *rb = malloc(sizeof(double) * m);
        double *rx = malloc(sizeof(double) * n);
        for (int64_t i = 0; i < m; ++i) { rc[i] = col[2 * i]; rb[i] = b[2 * i]; }
        for (int64_t i = 0; i < n; ++i) rr[i] = row[2 * i];
        rr[0] = rc[0];
        bad |= tikh_oracle_band_solve_real(m, n, rc, rr, 1, rb, NULL, lam, rx) != 0;
        bad |= tikh_oracle_band_solve_real(m, n, rc, rr, 1, NULL, rx, lam, rx) != 0;   /* normal form */
        free(col); free(row); free(b); free(gx); free(xd); free(xb); free(y); free(z);
        free(x); free(gb); free(gcol); free(grow); free(rc); free(rr); free(rb); free(rx);
    }
    printf(bad ? "oracle sanitizer run: FAILED\n" : "oracle sanitizer run: clean\n");
    return bad;
}
