/*
 * Plain, slow, FP64 CPU oracle for the Tikhonov-regularized Toeplitz
 * least-squares problem (Turnes, Balcan, Romberg, "Superfast Tikhonov
 * Regularization of Toeplitz Systems", Sec. 2, eq. (tik) and (tiksol), with
 * the l2-norm penalization case L = lambda*I).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) may link, load or call this file.  It shares no code with
 * the GPU path.  Only tests/, __graft_entry__.smoke() and the cpu_baseline leg
 * of bench.py use it.
 *
 * What it computes is the plain definition of the result:
 *
 *     x = argmin_x ||T x - b||^2 + lambda^2 ||x||^2 = (T^H T + lambda^2 I)^{-1} T^H b,
 *
 * obtained as the least-squares solution of the stacked system
 *     [ T        ]     [ b ]
 *     [ lambda I ] x ~ [ d ]
 * by dense Householder QR followed by back-substitution (and, for generators of
 * finite support at sizes where the dense matrix is out of reach, by a banded
 * QR of the same stacked system, tikh_oracle_band_solve).  With d = 0 this is
 * eq. (tiksol).  With b = 0 and d = y / lambda the normal equations of the
 * stacked system read (T^H T + lambda^2 I) x = y, the "normal-form" problem
 * the paper's experiments solve (Sec. 7.1, systems (G_T + G_L) x = y).
 *
 * Toeplitz convention (Sec. 1: T = [a_{i-j}], m x n, generator a_s for
 * s = -(n-1) .. m-1):  col[i] = a_i for i = 0..m-1,  row[j] = a_{-j} for
 * j = 1..n-1 (row[0] is ignored; a_0 is col[0]).
 *
 * Complex numbers are interleaved (re, im) doubles.  Real problems are passed
 * as complex with zero imaginary parts.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double re, im; } cplx;

static inline cplx cadd(cplx a, cplx b) { cplx r = {a.re + b.re, a.im + b.im}; return r; }
static inline cplx csub(cplx a, cplx b) { cplx r = {a.re - b.re, a.im - b.im}; return r; }
static inline cplx cmul(cplx a, cplx b) { cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static inline cplx cconjmul(cplx a, cplx b) /* conj(a) * b */ { cplx r = {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; return r; }
static inline cplx cscale(cplx a, double s) { cplx r = {a.re * s, a.im * s}; return r; }
static inline double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }
static inline cplx cdiv(cplx a, cplx b) {
    /* Smith's algorithm */
    cplx r;
    if (fabs(b.re) >= fabs(b.im)) {
        double t = b.im / b.re, d = b.re + b.im * t;
        r.re = (a.re + a.im * t) / d; r.im = (a.im - a.re * t) / d;
    } else {
        double t = b.re / b.im, d = b.re * t + b.im;
        r.re = (a.re * t + a.im) / d; r.im = (a.im * t - a.re) / d;
    }
    return r;
}

/* Generator entry a_s, s = i - j (Sec. 1: T = [a_{i-j}]). */
static inline cplx gen(const cplx* col, const cplx* row, int64_t s) {
    return s >= 0 ? col[s] : row[-s];
}

/*
 * Dense Householder QR least squares of A = [T; lambda I] ((m+n) x n) with
 * right-hand side c = [top; bot].  top has m entries (may be NULL = 0), bot
 * has n entries (may be NULL = 0).  Writes x (n entries).  Returns 0, or -1
 * on allocation failure, or -2 if R is exactly singular.
 * nthreads > 1 splits the trailing update over columns with OpenMP.
 */
int tikh_oracle_qr_solve(int64_t m, int64_t n, const double* col_, const double* row_,
                         const double* top_, const double* bot_, double lambda,
                         double* x_, int nthreads)
{
    const cplx* col = (const cplx*)col_;
    const cplx* row = (const cplx*)row_;
    const cplx* top = (const cplx*)top_;
    const cplx* bot = (const cplx*)bot_;
    cplx* x = (cplx*)x_;
    const int64_t R = m + n;             /* rows of the stacked matrix */
    cplx* A = (cplx*)malloc(sizeof(cplx) * (size_t)R * (size_t)n);   /* column major */
    cplx* c = (cplx*)malloc(sizeof(cplx) * (size_t)R);
    cplx* u = (cplx*)malloc(sizeof(cplx) * (size_t)R);
    if (!A || !c || !u) { free(A); free(c); free(u); return -1; }

    /* Form A = [T; lambda I] and c = [top; bot]. */
    for (int64_t j = 0; j < n; ++j) {
        cplx* Aj = A + (size_t)j * R;
        for (int64_t i = 0; i < m; ++i) Aj[i] = gen(col, row, i - j);
        for (int64_t i = 0; i < n; ++i) { Aj[m + i].re = (i == j) ? lambda : 0.0; Aj[m + i].im = 0.0; }
    }
    for (int64_t i = 0; i < m; ++i) { if (top) c[i] = top[i]; else { c[i].re = 0; c[i].im = 0; } }
    for (int64_t i = 0; i < n; ++i) { if (bot) c[m + i] = bot[i]; else { c[m + i].re = 0; c[m + i].im = 0; } }

    for (int64_t j = 0; j < n; ++j) {
        cplx* Aj = A + (size_t)j * R;
        /* v = A[j:, j];  alpha = -e^{i arg v0} ||v||  (sign chosen against cancellation) */
        double nrm2 = 0.0;
        for (int64_t i = j; i < R; ++i) nrm2 += cabs2(Aj[i]);
        double nrm = sqrt(nrm2);
        if (nrm == 0.0) continue;                      /* nothing to annihilate */
        double a0 = sqrt(cabs2(Aj[j]));
        cplx ph; if (a0 > 0) { ph.re = Aj[j].re / a0; ph.im = Aj[j].im / a0; } else { ph.re = 1; ph.im = 0; }
        cplx alpha = cscale(ph, -nrm);
        /* u = v - alpha e_0, normalized to unit 2-norm: H = I - 2 u u^H */
        for (int64_t i = j; i < R; ++i) u[i] = Aj[i];
        u[j] = csub(u[j], alpha);
        double un2 = 0.0;
        for (int64_t i = j; i < R; ++i) un2 += cabs2(u[i]);
        double un = sqrt(un2);
        if (un == 0.0) continue;
        for (int64_t i = j; i < R; ++i) u[i] = cscale(u[i], 1.0 / un);
        /* Column j becomes alpha e_0. */
        Aj[j] = alpha;
        for (int64_t i = j + 1; i < R; ++i) { Aj[i].re = 0; Aj[i].im = 0; }
        /* Trailing columns: A_k -= 2 u (u^H A_k). */
#ifdef _OPENMP
#pragma omp parallel for num_threads(nthreads) schedule(static) if (nthreads > 1 && (n - j) > 16)
#endif
        for (int64_t k = j + 1; k < n; ++k) {
            cplx* Ak = A + (size_t)k * R;
            cplx s = {0, 0};
            for (int64_t i = j; i < R; ++i) s = cadd(s, cconjmul(u[i], Ak[i]));
            s = cscale(s, 2.0);
            for (int64_t i = j; i < R; ++i) Ak[i] = csub(Ak[i], cmul(u[i], s));
        }
        {
            cplx s = {0, 0};
            for (int64_t i = j; i < R; ++i) s = cadd(s, cconjmul(u[i], c[i]));
            s = cscale(s, 2.0);
            for (int64_t i = j; i < R; ++i) c[i] = csub(c[i], cmul(u[i], s));
        }
    }
    /* Back-substitution R x = c[0:n], R = triu(A[0:n, 0:n]). */
    int status = 0;
    for (int64_t i = n - 1; i >= 0; --i) {
        cplx s = c[i];
        for (int64_t k = i + 1; k < n; ++k) s = csub(s, cmul(A[(size_t)k * R + i], x[k]));
        cplx d = A[(size_t)i * R + i];
        if (d.re == 0.0 && d.im == 0.0) { status = -2; x[i].re = 0; x[i].im = 0; continue; }
        x[i] = cdiv(s, d);
    }
    free(A); free(c); free(u);
    return status;
}

/* Band limits of the generator: a_s = 0 for s > wl and for s < -wu. */
static void gen_band(int64_t m, int64_t n, const cplx* col, const cplx* row, int64_t* wl, int64_t* wu) {
    *wl = 0; *wu = 0;
    for (int64_t s = 0; s < m; ++s) if (col[s].re != 0.0 || col[s].im != 0.0) *wl = s;
    for (int64_t s = 1; s < n; ++s) if (row[s].re != 0.0 || row[s].im != 0.0) *wu = s;
}

/* y = T v (m entries), the sum of the definition T = [a_{i-j}] over the
 * generator's support (the terms left out are exact zeros). */
void tikh_oracle_T_apply(int64_t m, int64_t n, const double* col_, const double* row_,
                         const double* v_, double* y_)
{
    const cplx* col = (const cplx*)col_; const cplx* row = (const cplx*)row_;
    const cplx* v = (const cplx*)v_; cplx* y = (cplx*)y_;
    int64_t wl, wu;
    gen_band(m, n, col, row, &wl, &wu);
    for (int64_t i = 0; i < m; ++i) {
        cplx s = {0, 0};
        int64_t j0 = i - wl > 0 ? i - wl : 0, j1 = i + wu < n - 1 ? i + wu : n - 1;
        for (int64_t j = j0; j <= j1; ++j) s = cadd(s, cmul(gen(col, row, i - j), v[j]));
        y[i] = s;
    }
}

/* y = T^H v (n entries), likewise over the support. */
void tikh_oracle_TH_apply(int64_t m, int64_t n, const double* col_, const double* row_,
                          const double* v_, double* y_)
{
    const cplx* col = (const cplx*)col_; const cplx* row = (const cplx*)row_;
    const cplx* v = (const cplx*)v_; cplx* y = (cplx*)y_;
    int64_t wl, wu;
    gen_band(m, n, col, row, &wl, &wu);
    for (int64_t j = 0; j < n; ++j) {
        cplx s = {0, 0};
        int64_t i0 = j - wu > 0 ? j - wu : 0, i1 = j + wl < m - 1 ? j + wl : m - 1;
        for (int64_t i = i0; i <= i1; ++i) s = cadd(s, cconjmul(gen(col, row, i - j), v[i]));
        y[j] = s;
    }
}

/*
 * Gradients of a scalar loss L(x) through x = (T^H T + lambda^2 I)^{-1} T^H b,
 * given gx = dL/dRe(x) + i dL/dIm(x).  Derived from eq. (tiksol) by
 * differentiating A x = T^H b with A = T^H T + lambda^2 I:
 *     w      = A^{-1} gx                          (adjoint solve, normal form)
 *     g_b    = T w
 *     g_lam  = -2 lambda Re<w, x>
 *     G_T    = (b - T x) w^H - (T w) x^H,  g_{a_s} = sum_{i-j=s} (G_T)_{ij}
 * Outputs: x (n), g_b (m), g_col (m), g_row (n, entry 0 is zero: a_0 lives
 * in col), *g_lam.  All complex interleaved.  Returns the solver status.
 */
int tikh_oracle_gradients(int64_t m, int64_t n, const double* col_, const double* row_,
                          const double* b_, double lambda, const double* gx_,
                          double* x_, double* gb_, double* gcol_, double* grow_,
                          double* glam, int nthreads)
{
    const cplx* col = (const cplx*)col_; const cplx* row = (const cplx*)row_;
    const cplx* b = (const cplx*)b_; const cplx* gx = (const cplx*)gx_;
    cplx* x = (cplx*)x_; cplx* gb = (cplx*)gb_; cplx* gcol = (cplx*)gcol_; cplx* grow = (cplx*)grow_;
    int st = tikh_oracle_qr_solve(m, n, col_, row_, b_, NULL, lambda, x_, nthreads);
    if (st) return st;
    cplx* d = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    cplx* w = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    cplx* Tx = (cplx*)malloc(sizeof(cplx) * (size_t)m);
    cplx* r = (cplx*)malloc(sizeof(cplx) * (size_t)m);
    if (!d || !w || !Tx || !r) { free(d); free(w); free(Tx); free(r); return -1; }
    for (int64_t j = 0; j < n; ++j) d[j] = cscale(gx[j], 1.0 / lambda);
    st = tikh_oracle_qr_solve(m, n, col_, row_, NULL, (const double*)d, lambda, (double*)w, nthreads);
    tikh_oracle_T_apply(m, n, col_, row_, x_, (double*)Tx);
    tikh_oracle_T_apply(m, n, col_, row_, (const double*)w, gb_);        /* g_b = T w */
    for (int64_t i = 0; i < m; ++i) r[i] = csub(b[i], Tx[i]);
    /* g_lam = -2 lambda Re(w^H x) */
    double re = 0.0;
    for (int64_t j = 0; j < n; ++j) re += w[j].re * x[j].re + w[j].im * x[j].im;
    *glam = -2.0 * lambda * re;
    /* Diagonal sums of G_T = r w^H - (T w) x^H over i - j = s. */
    for (int64_t i = 0; i < m; ++i) { gcol[i].re = 0; gcol[i].im = 0; }
    for (int64_t j = 0; j < n; ++j) { grow[j].re = 0; grow[j].im = 0; }
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            /* (r w^H)_{ij} = r_i conj(w_j); ((Tw) x^H)_{ij} = (Tw)_i conj(x_j) */
            cplx g1 = { r[i].re * w[j].re + r[i].im * w[j].im, r[i].im * w[j].re - r[i].re * w[j].im };
            cplx g2 = { gb[i].re * x[j].re + gb[i].im * x[j].im, gb[i].im * x[j].re - gb[i].re * x[j].im };
            cplx g = csub(g1, g2);
            int64_t s = i - j;
            if (s >= 0) gcol[s] = cadd(gcol[s], g); else grow[-s] = cadd(grow[-s], g);
        }
    }
    free(d); free(w); free(Tx); free(r);
    return st;
}

/*
 * Banded QR least squares (exact for generators of finite support, at any n).
 *
 * When a_s = 0 for s > wl and for s < -wu, the stacked matrix [T; lambda I]
 * has at most wl + wu + 1 nonzeros per row, and its QR factor R is upper
 * triangular with bandwidth bw = wl + wu.  The least-squares solution of
 * [T; lambda I] x ~ [top; bot] (the same problem as tikh_oracle_qr_solve) is
 * formed by absorbing the rows one at a time into R with Givens rotations
 * (the row-by-row orthogonal factorization of sparse least-squares problems):
 * a row meeting an empty row k of R becomes that row; otherwise a rotation
 * between R row k and the incoming row zeroes the incoming entry k.  The
 * rotations are applied to the right-hand sides as well, so R x = Q^H c is
 * left to back-substitution.  Rows are taken in the order of their leading
 * column (the rows of T, then the row lambda e_j of column j), which keeps
 * every incoming row inside the window [k, k + bw] of the row of R it meets.
 * Row order does not change the least-squares solution.
 *
 * top: nrhs right-hand sides of m entries ([nrhs][m], or NULL = 0);
 * bot: nrhs of n entries ([nrhs][n], or NULL = 0); x: [nrhs][n].
 * All complex interleaved.  Returns 0, -1 on allocation failure, -2 if R is
 * singular (not possible for lambda > 0).
 */
int tikh_oracle_band_solve(int64_t m, int64_t n, const double* col_, const double* row_, int64_t nrhs,
                           const double* top_, const double* bot_, double lambda, double* x_)
{
    const cplx* col = (const cplx*)col_;
    const cplx* row = (const cplx*)row_;
    const cplx* top = (const cplx*)top_;
    const cplx* bot = (const cplx*)bot_;
    cplx* x = (cplx*)x_;
    int64_t wl, wu;
    gen_band(m, n, col, row, &wl, &wu);
    const int64_t bw = wl + wu, W = bw + 1;
    cplx* R = (cplx*)calloc((size_t)n * (size_t)W, sizeof(cplx));   /* R[k][t] = entry (k, k+t) */
    cplx* d = (cplx*)calloc((size_t)n * (size_t)nrhs, sizeof(cplx)); /* d[k][r] = (Q^H c)_k */
    char* have = (char*)calloc((size_t)n, 1);
    cplx* v = (cplx*)calloc((size_t)(n + W + 1), sizeof(cplx));      /* incoming row, by column */
    cplx* cv = (cplx*)calloc((size_t)nrhs, sizeof(cplx));
    if (!R || !d || !have || !v || !cv) { free(R); free(d); free(have); free(v); free(cv); return -1; }

    /* rows in order of leading column: T rows i with max(0, i - wl) = j, then lambda e_j */
    for (int64_t j = 0; j < n; ++j) {
        int64_t i0 = (j == 0) ? 0 : j + wl, i1 = j + wl;
        for (int64_t ii = i0; ii <= i1 + 1; ++ii) {
            int64_t lo, hi;
            if (ii <= i1) {                              /* row ii of T */
                if (ii >= m) continue;
                lo = ii - wl < 0 ? 0 : ii - wl;
                hi = ii + wu < n - 1 ? ii + wu : n - 1;
                for (int64_t c = lo; c <= hi; ++c) v[c] = gen(col, row, ii - c);
                for (int64_t r = 0; r < nrhs; ++r) {
                    if (top) cv[r] = top[r * m + ii]; else { cv[r].re = 0; cv[r].im = 0; }
                }
            } else {                                     /* row lambda e_j */
                lo = hi = j;
                v[j].re = lambda; v[j].im = 0.0;
                for (int64_t r = 0; r < nrhs; ++r) {
                    if (bot) cv[r] = bot[r * n + j]; else { cv[r].re = 0; cv[r].im = 0; }
                }
            }
            for (int64_t k = lo; k <= hi; ++k) {
                cplx b = v[k];
                if (b.re == 0.0 && b.im == 0.0) continue;
                cplx* Rk = R + (size_t)k * W;
                cplx* dk = d + (size_t)k * nrhs;
                if (!have[k]) {                          /* the row becomes row k of R */
                    for (int64_t t = 0; t < W && k + t < n; ++t) { Rk[t] = v[k + t]; v[k + t].re = 0; v[k + t].im = 0; }
                    for (int64_t r = 0; r < nrhs; ++r) dk[r] = cv[r];
                    have[k] = 1;
                    break;
                }
                /* rotation [c s; -conj(s) c] with c real: [R_kk; b] -> [rho; 0] */
                cplx a = Rk[0];
                double aa = sqrt(cabs2(a)), bb = sqrt(cabs2(b));
                double nrm = hypot(aa, bb);
                double c;
                cplx s;
                if (aa == 0.0) { c = 0.0; s.re = b.re / bb; s.im = -b.im / bb; }
                else {
                    c = aa / nrm;
                    cplx ph = {a.re / aa, a.im / aa};
                    cplx cb = {b.re / nrm, -b.im / nrm};
                    s = cmul(ph, cb);
                }
                cplx sc = {s.re, -s.im};                 /* conj(s) */
                for (int64_t t = 0; t < W && k + t < n; ++t) {
                    cplx rt = Rk[t], vt = v[k + t];
                    Rk[t] = cadd(cscale(rt, c), cmul(s, vt));
                    v[k + t] = csub(cscale(vt, c), cmul(sc, rt));
                }
                v[k].re = 0.0; v[k].im = 0.0;
                for (int64_t r = 0; r < nrhs; ++r) {
                    cplx rt = dk[r], vt = cv[r];
                    dk[r] = cadd(cscale(rt, c), cmul(s, vt));
                    cv[r] = csub(cscale(vt, c), cmul(sc, rt));
                }
                if (k + bw > hi) hi = k + bw < n - 1 ? k + bw : n - 1;
            }
        }
    }
    /* back-substitution R x = d */
    int status = 0;
    for (int64_t r = 0; r < nrhs; ++r) {
        cplx* xr = x + (size_t)r * n;
        for (int64_t k = n - 1; k >= 0; --k) {
            const cplx* Rk = R + (size_t)k * W;
            cplx s = d[(size_t)k * nrhs + r];
            for (int64_t t = 1; t < W && k + t < n; ++t) s = csub(s, cmul(Rk[t], xr[k + t]));
            if (!have[k] || (Rk[0].re == 0.0 && Rk[0].im == 0.0)) { status = -2; xr[k].re = 0; xr[k].im = 0; continue; }
            xr[k] = cdiv(s, Rk[0]);
        }
    }
    free(R); free(d); free(have); free(v); free(cv);
    return status;
}

/*
 * The same banded QR for real data (all generator entries and right-hand sides
 * real): real rotations [c s; -s c], real R.  Arrays are plain doubles:
 * col[m], row[n], top[nrhs][m] (or NULL), bot[nrhs][n] (or NULL), x[nrhs][n].
 */
int tikh_oracle_band_solve_real(int64_t m, int64_t n, const double* col, const double* row, int64_t nrhs,
                                const double* top, const double* bot, double lambda, double* x)
{
    int64_t wl = 0, wu = 0;
    for (int64_t s = 0; s < m; ++s) if (col[s] != 0.0) wl = s;
    for (int64_t s = 1; s < n; ++s) if (row[s] != 0.0) wu = s;
    const int64_t bw = wl + wu, W = bw + 1;
    double* R = (double*)calloc((size_t)n * (size_t)W, sizeof(double));
    double* d = (double*)calloc((size_t)n * (size_t)nrhs, sizeof(double));
    char* have = (char*)calloc((size_t)n, 1);
    double* v = (double*)calloc((size_t)(n + W + 1), sizeof(double));
    double* cv = (double*)calloc((size_t)nrhs, sizeof(double));
    if (!R || !d || !have || !v || !cv) { free(R); free(d); free(have); free(v); free(cv); return -1; }
    for (int64_t j = 0; j < n; ++j) {
        int64_t i0 = (j == 0) ? 0 : j + wl, i1 = j + wl;
        for (int64_t ii = i0; ii <= i1 + 1; ++ii) {
            int64_t lo, hi;
            if (ii <= i1) {
                if (ii >= m) continue;
                lo = ii - wl < 0 ? 0 : ii - wl;
                hi = ii + wu < n - 1 ? ii + wu : n - 1;
                for (int64_t c = lo; c <= hi; ++c) v[c] = (ii - c >= 0) ? col[ii - c] : row[c - ii];
                for (int64_t r = 0; r < nrhs; ++r) cv[r] = top ? top[r * m + ii] : 0.0;
            } else {
                lo = hi = j;
                v[j] = lambda;
                for (int64_t r = 0; r < nrhs; ++r) cv[r] = bot ? bot[r * n + j] : 0.0;
            }
            for (int64_t k = lo; k <= hi; ++k) {
                double b = v[k];
                if (b == 0.0) continue;
                double* Rk = R + (size_t)k * W;
                double* dk = d + (size_t)k * nrhs;
                if (!have[k]) {
                    for (int64_t t = 0; t < W && k + t < n; ++t) { Rk[t] = v[k + t]; v[k + t] = 0.0; }
                    for (int64_t r = 0; r < nrhs; ++r) dk[r] = cv[r];
                    have[k] = 1;
                    break;
                }
                double a = Rk[0], nrm = hypot(a, b);
                double c = a / nrm, s = b / nrm;
                const int64_t tmax = (k + W <= n) ? W : n - k;
                for (int64_t t = 0; t < tmax; ++t) {
                    double rt = Rk[t], vt = v[k + t];
                    Rk[t] = c * rt + s * vt;
                    v[k + t] = c * vt - s * rt;
                }
                v[k] = 0.0;
                for (int64_t r = 0; r < nrhs; ++r) {
                    double rt = dk[r], vt = cv[r];
                    dk[r] = c * rt + s * vt;
                    cv[r] = c * vt - s * rt;
                }
                if (k + bw > hi) hi = k + bw < n - 1 ? k + bw : n - 1;
            }
        }
    }
    int status = 0;
    for (int64_t r = 0; r < nrhs; ++r) {
        double* xr = x + (size_t)r * n;
        for (int64_t k = n - 1; k >= 0; --k) {
            const double* Rk = R + (size_t)k * W;
            double s = d[(size_t)k * nrhs + r];
            for (int64_t t = 1; t < W && k + t < n; ++t) s -= Rk[t] * xr[k + t];
            if (!have[k] || Rk[0] == 0.0) { status = -2; xr[k] = 0.0; continue; }
            xr[k] = s / Rk[0];
        }
    }
    free(R); free(d); free(have); free(v); free(cv);
    return status;
}

/*
 * Generator gradient of the adjoint (derived from eq. (tiksol)): the lag sums
 *     g_col[s] = sum_{i-j=s} G_ij (s = 0..m-1),  g_row[s] = sum_{j-i=s} G_ij (s = 1..n-1),
 * of G = r w^H - (T w) x^H, written out term by term (O(mn)).  Inputs r, Tw
 * (m entries) and w, x (n entries); g_row[0] = 0.  Complex interleaved.
 */
void tikh_oracle_lag_sums(int64_t m, int64_t n, const double* r_, const double* w_, const double* Tw_,
                          const double* x_, double* gcol_, double* grow_)
{
    const cplx* r = (const cplx*)r_; const cplx* w = (const cplx*)w_;
    const cplx* Tw = (const cplx*)Tw_; const cplx* x = (const cplx*)x_;
    cplx* gcol = (cplx*)gcol_; cplx* grow = (cplx*)grow_;
    for (int64_t i = 0; i < m; ++i) { gcol[i].re = 0; gcol[i].im = 0; }
    for (int64_t j = 0; j < n; ++j) { grow[j].re = 0; grow[j].im = 0; }
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            cplx g = csub(cconjmul(w[j], r[i]), cconjmul(x[j], Tw[i]));   /* r_i conj(w_j) - (Tw)_i conj(x_j) */
            int64_t s = i - j;
            if (s >= 0) gcol[s] = cadd(gcol[s], g); else grow[-s] = cadd(grow[-s], g);
        }
    }
}
