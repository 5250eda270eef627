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
 * by dense Householder QR followed by back-substitution.  With d = 0 this is
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

/* y = T v (m entries), direct O(mn) sum from the definition T = [a_{i-j}]. */
void tikh_oracle_T_apply(int64_t m, int64_t n, const double* col_, const double* row_,
                         const double* v_, double* y_)
{
    const cplx* col = (const cplx*)col_; const cplx* row = (const cplx*)row_;
    const cplx* v = (const cplx*)v_; cplx* y = (cplx*)y_;
    for (int64_t i = 0; i < m; ++i) {
        cplx s = {0, 0};
        for (int64_t j = 0; j < n; ++j) s = cadd(s, cmul(gen(col, row, i - j), v[j]));
        y[i] = s;
    }
}

/* y = T^H v (n entries), direct O(mn). */
void tikh_oracle_TH_apply(int64_t m, int64_t n, const double* col_, const double* row_,
                          const double* v_, double* y_)
{
    const cplx* col = (const cplx*)col_; const cplx* row = (const cplx*)row_;
    const cplx* v = (const cplx*)v_; cplx* y = (cplx*)y_;
    for (int64_t j = 0; j < n; ++j) {
        cplx s = {0, 0};
        for (int64_t i = 0; i < m; ++i) s = cadd(s, cconjmul(gen(col, row, i - j), v[i]));
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
