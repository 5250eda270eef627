/*
 * tikh.h -- C ABI of the MI355X (gfx950) superfast Tikhonov-regularized
 * Toeplitz least-squares solver.
 *
 * Problem (Turnes, Balcan, Romberg, "Superfast Tikhonov Regularization of
 * Toeplitz Systems", Sec. 2, eq. (tik) with the l2-norm penalization case
 * L = lambda I, Sec. 3.3):
 *
 *     x = argmin_x ||T x - b||^2 + lambda^2 ||x||^2
 *       = (T^H T + lambda^2 I)^{-1} T^H b                      (eq. (tiksol))
 *
 * T is m x n Toeplitz, T = [a_{i-j}] (Sec. 1), given by its m+n-1 generator
 * entries:  col[i] = a_i (0 <= i < m),  row[j] = a_{-j} (0 < j < n).  row[0]
 * is ignored (a_0 is col[0]).  Any aspect ratio is allowed (Sec. 3.3: the
 * extension uses q = m regardless of m < n).
 *
 * Method: extension of the Toeplitz blocks to partial-circulant blocks
 * (eq. (circexp), (ex5)-(ex6)), transformation by FFTs to tangential
 * interpolation conditions at roots of unity (eq. (vandprod), (intcond),
 * (interp)), and the divide-and-conquer basis construction of Alg. 1 with
 * paired interleaving (Sec. 6.1) and the extension size of Alg. 2 (Sec. 6.2);
 * the solution is read from the tau-degree-0 column of the final basis
 * (Sec. 5).  One step of iterative refinement (mentioned in Sec. 7.2) is on
 * by default.  All arithmetic is complex FP64 on the GPU.
 *
 * Memory: unless stated otherwise every array argument is a DEVICE pointer
 * (hipMalloc'd memory or a torch tensor's storage on the current HIP device),
 * FP64, contiguous, owned by the caller; the library never frees or retains
 * it.  Complex arrays are interleaved (re, im) pairs (tikh_c64).  Inputs are
 * never modified.  Work is enqueued on the stream set by tikh_set_stream
 * (default: the null stream).  The library keeps an internal device workspace
 * that grows on demand (hipMalloc outside the hot loop) and is released by
 * tikh_release().
 *
 * Errors: every entry point returns TIKH_OK (0) or a negative TIKH_E* code;
 * tikh_strerror() describes it.  On error the outputs are undefined.  The
 * numerical status of each solve is reported in an info word of bits: 0 = OK,
 * bit 1 = breakdown (no admissible pivot / final tau-degrees not {1,1,1,1,0}),
 * bit 2 = a basis degree exceeded its storage bound, bit 4 = more deferred
 * difficult conditions than a solve can hold, bit 8 = non-finite values in the
 * solution, bit 16 = after its last iterative refinement step the solve's
 * error estimate (see tikh_opts) is still above 1e-4: the refinement diverged or
 * barely converges, i.e. the recursion lost the solution (see fallback_nlim) or
 * the regularized system is too ill-conditioned for it, bit 32 = (prepared
 * batches only) a recorded product transform length was too short for the
 * call's basis degrees, the results are not valid and the batch must be
 * prepared again, bit 64 = (prepared batches only) the solve's lambda was not
 * positive and finite: it was solved with lambda = 1 (bits may combine).
 * Right-hand sides of one (problem, lambda) share a pivot sequence, so bits 1,
 * 2 and 4 of a forward solve are those of its (problem, lambda); bit 8 is the
 * solve's own.
 * Single-problem calls synchronize the stream and return TIKH_ENUMERIC when
 * info != 0.  Calls are not thread safe (one host thread per library state).
 */
#ifndef TIKH_H
#define TIKH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } tikh_c64;

enum {
    TIKH_OK = 0,
    TIKH_EINVAL = -1,     /* invalid argument (sizes, non-positive or non-finite lambda, null pointer) */
    TIKH_ENOMEM = -2,     /* device allocation failed */
    TIKH_EHIP = -3,       /* a HIP runtime call failed */
    TIKH_ENUMERIC = -4,   /* a solve reported info != 0 (see above) */
    TIKH_ETOOBIG = -5     /* the allocation-free entry point's scratch buffer cannot hold the call */
};

/*
 * Tunable options (Sec. 6.2: leaf cutoff N_lim; Sec. 7.2: iterative
 * refinement).  Product transform lengths (Alg. 1 step 4) follow the degrees
 * of the bases being multiplied: the first recursion of a batch composition
 * reads them back once per merge; later recursions and later calls with the
 * same composition (sizes, extension, lambda, element type) reuse the recorded
 * lengths without host synchronization, checked on the device, and a batch
 * whose degrees outgrow a recorded length is run again with read-back sizing.
 * Every solve takes `refine` refinement steps; a solve whose
 * estimated relative error is still above `refine_tol` takes further steps,
 * up to `refine_max` in all (the estimate: e0 = ||dx_1|| / ||x|| of the
 * first step approximates the first solve's error and the factor by which
 * each step contracts it, so the error left after step k is taken as
 * 1000 * e0 * ||dx_k|| / ||x||).  With refine = 0 no step is taken.
 */
/* Every option's default can be overridden from the environment when the library first
 * initializes: TIKH_NLIM, TIKH_REFINE, TIKH_REFINE_MAX, TIKH_REFINE_TOL, TIKH_DEFER_TOL,
 * TIKH_LEAF_WAVE_GROUPS, TIKH_STREAMS, TIKH_MERGE_TOL, TIKH_FALLBACK_NLIM,
 * TIKH_CHUNK_GROUPS, TIKH_REFINE_SKIP (a value that does not parse or is out of range is
 * reported on stderr and ignored); tikh_set_options replaces them all. */
typedef struct {
    int32_t n_lim;        /* max conditions per leaf (64..256, multiple of 64); default 256 */
    int32_t refine;       /* refinement steps for every solve (0..4); default 1 */
    int32_t refine_max;   /* most refinement steps for a solve above the error target (0..4); default 3 */
    int32_t leaf_wave_groups; /* groups per call from which each group's leaf steps run in one
                             wavefront rather than one wavefront per 64 conditions (>= 1;
                             default 1536); either way the results are the same */
    double refine_tol;    /* target relative error of the adaptive steps (> 0, finite); default 1e-10 */
    double defer_tol;     /* difficult points (Sec. 5): a chosen condition whose pivot entry is below
                             defer_tol times its largest entry among columns 1..4 is set aside and
                             processed after the root, against the final basis (0 <= defer_tol < 1;
                             0 = off, the default; at most 64 per solve, else info bit 4) */
    int32_t record_short;  /* testing only (default 0): record product transform lengths half as long as
                             the degrees need, so that the device check of recorded lengths fires and the
                             chunk runs again with read-back sizing (results are unaffected) */
    int32_t streams;      /* streams on which chunks of different extended sizes (ragged batches) run side
                             by side (1..16; default 16; 1 runs them one after another on the library stream) */
    double merge_tol;     /* ragged batches: problems whose extended sizes N lie within a factor 1 + merge_tol
                             of each other share the largest one's plan (a larger circulant extension k),
                             so that they run in the same launches (0..4; default 0.25; 0 = one plan per N) */
    int32_t fallback_nlim; /* a group whose solve failed (info bits 1, 2, 8 or 16: pivots so small that the
                             basis lost the solution, Sec. 5's difficult points, or a breakdown) is solved
                             again with this smaller leaf cutoff, i.e. another tree over the same conditions
                             (64..256 and below n_lim, or 0 = off; default 64); its outputs and info are
                             those of the second solve.  Not for a group whose conditioning bound
                             1 + (sum_s |a_s| / lambda)^2 exceeds 1e8 (the failure may then be the
                             conditioning itself, which another tree does not cure): its flags stand */
    int32_t chunk_groups; /* most groups (recursions run in the same launches) per chunk, 0 = as many as the
                             workspace holds (the default); with streams > 1 the chunks of a call run side by
                             side, so that one chunk's serial leaf steps overlap another's transforms */
    int32_t refine_skip;  /* 1: before the first refinement step, a group whose first solves are certified
                             to refine_tol by the a-posteriori bound ||x - x*|| <= ||r|| / lambda^2
                             (r = y - (T^H T + lambda^2 I) x; T^H T is positive semidefinite), with a margin for
                             the residual's own rounding, takes no refinement step (one more host
                             synchronization per call; such solves keep the first solve's residual, about
                             1e-11 relative at n = 2^14, instead of the refined one); 0 (default): every solve
                             takes `refine` steps.  Pays off for well-conditioned batches (every solve of the
                             paper's accuracy workload, lambda^2 = sqrt(2n), is certified); at the headline
                             lambda path only 5-9% of the solves are, for 0.4% of the time.  Not applied to
                             the Toeplitz-Gramian problem or to prepared batches */
} tikh_opts;

/* Per-solve statistics of the last call (host memory, filled by tikh_get_stats). */
typedef struct {
    int64_t N;            /* number of interpolation nodes after extension (Alg. 2) */
    int64_t k;            /* circulant-extension size k (Sec. 3.1) */
    int32_t depth;        /* recursion depth p: 2^p leaves */
    int32_t leaf_nodes;   /* M: nodes per leaf (2M conditions) */
    int64_t solves;       /* number of solves in the last call */
    int64_t launches;     /* kernel launches enqueued by the last call */
    int64_t refine_extra; /* refinement steps beyond `refine` taken by the last call, summed over solves */
    int64_t deferred;     /* difficult conditions deferred by the last call, summed over groups and steps */
    int64_t host_syncs;   /* host synchronizations inside the last call (transform sizing read back per
                             merge, refinement decisions, the check of recorded transform lengths) */
    int64_t fallback_groups; /* groups of the last call solved again with the fallback leaf cutoff */
    int64_t refine_skipped; /* solves of the last call whose refinement steps the a-posteriori bound made
                               unnecessary (refine_skip) */
} tikh_stats;

/*
 * Host-only planning query (no device work): the extended number of nodes
 * N = 2^p M chosen by the extension-size rule of Alg. 2 (Sec. 6.2) for an
 * m x n problem and leaf cutoff n_lim (two condition sets per node, so a leaf
 * of M nodes carries 2M <= n_lim conditions; M even and 5-smooth).  Outputs
 * are host pointers.  Returns TIKH_EINVAL for invalid sizes or n_lim.
 */
int tikh_plan_info(int64_t m, int64_t n, int32_t n_lim, int64_t* N, int64_t* M, int32_t* depth, int64_t* k);

/*
 * Launch timing of one kernel kind (for benchmarks): after
 * tikh_profile_kernel("leaf_loop" | "leaf_build" | "fft"), each launch of that
 * kernel is bracketed by HIP events on the library stream; tikh_profile_read
 * synchronizes the stream and returns the summed duration (ms) and the launch
 * count since the last tikh_profile_kernel call.  NULL or "" disables.
 */
int tikh_profile_kernel(const char* name);
int tikh_profile_read(double* total_ms, int64_t* count);
/* Algorithmic work of the timed launches (host pointer): for "fft" the bytes
 * of one read and one write of every transformed element, for "leaf_loop" the
 * FP64 flops of the serial steps. */
int tikh_profile_units(double* units);

/*
 * Batched complex FFT, the transform behind the evaluations at roots of unity
 * of eq. (vandprod) and the polynomial products of Alg. 1: for each of `items`
 * blocks of `nlines` contiguous lines of length `len` (device tikh_c64,
 * in place, item stride nlines*len),
 *     X_k = sum_j x_j exp(sign * 2 pi i j k / len),   sign = -1 or +1,
 * unnormalized.  len must factor into 2, 3 and 5 and be at most 4096^2 (lines
 * longer than 4096 take two passes plus a reordering through the library
 * workspace); items <= 65535 and nlines * len < 2^31.  Asynchronous on the
 * library stream.
 */
int tikh_fft_batched(void* data, int64_t items, int64_t nlines, int64_t len, int sign);

/*
 * Autotuner for the leaf cutoff N_lim of Alg. 2, which the paper calls
 * machine-dependent (Sec. 6.2): times one batched forward solve of `groups`
 * groups of min(nrhs, 4) right-hand sides of an m x n real problem (synthetic
 * data generated on the device: generator with an exp(-|s|/32) envelope,
 * uniform right-hand sides, lambda = 1e-2 sum_s |a_s|) for each N_lim in
 * {64, 128, 192, 256}, keeps the fastest in the options and returns it in
 * *best (host).  ms (host, may be NULL) receives the four times in
 * milliseconds (-1 for a cutoff that does not apply).  Allocates and frees
 * device memory; synchronizes.  groups <= 65535, 1 <= nrhs <= 4.
 */
int tikh_autotune_nlim(int64_t m, int64_t n, int64_t groups, int32_t nrhs, int32_t* best, double* ms);

/*
 * Workspace.  By default the library keeps one device buffer for all calls and
 * grows it (one hipMalloc) when a call needs more, splitting a batch into equal
 * chunks that fit 85% of free device memory.  A caller with its own allocator
 * can hand the library a buffer instead:
 *  - tikh_workspace_bytes (host only, no device work): the bytes with which a
 *    batched solve or backward of these shapes (nprob problems of m[p] x n[p],
 *    host arrays; nlam lambdas; nrhs right-hand sides) runs every group in one
 *    chunk; *bytes is a host pointer.  TIKH_EINVAL for shapes the solves
 *    reject.
 *  - tikh_set_workspace(ptr, bytes): use this device buffer (256-byte aligned,
 *    caller-owned, not touched by the caller until it is replaced) for every
 *    later call; the library frees its own buffer.  Batches are split into
 *    chunks that fit `bytes`; a call in which not even one group fits returns
 *    TIKH_ENOMEM.  tikh_set_workspace(NULL, 0) returns to the library's own
 *    buffer.  Synchronizes the library stream.  Twiddle tables (one per
 *    transform size, at most a few MB) are still allocated by the library.
 */
int tikh_workspace_bytes(int64_t nprob, const int64_t* m, const int64_t* n, int64_t nlam, int64_t nrhs,
                         size_t* bytes);
int tikh_set_workspace(void* ptr, size_t bytes);

/* Library state.  tikh_init is optional (the first call initializes). */
int tikh_init(void);
int tikh_release(void);                              /* free the library's workspace and tables */
int tikh_set_stream(void* hip_stream);               /* hipStream_t; NULL = null stream */
int tikh_set_options(const tikh_opts* opts);         /* host pointer */
int tikh_get_options(tikh_opts* opts);               /* host pointer */
int tikh_get_stats(tikh_stats* stats);               /* host pointer */
const char* tikh_strerror(int code);

/*
 * Single problem, real data: col[m], row[n], b[m] -> x[n] (device, FP64).
 * lambda must be finite and > 0 (lambda = 0 is the pseudo-inverse problem,
 * outside this solver); the extended size N (about m + n) must not exceed
 * 2^19.  Synchronizes; returns TIKH_ENUMERIC if info != 0.
 */
int tikh_toeplitz_solve(const double* col, const double* row, int64_t m, int64_t n,
                        const double* b, double lambda, double* x);

/* Single problem, complex data (interleaved). */
int tikh_toeplitz_solve_z(const tikh_c64* col, const tikh_c64* row, int64_t m, int64_t n,
                          const tikh_c64* b, double lambda, tikh_c64* x);

/*
 * Normal-form entry: x = (T^H T + lambda^2 I)^{-1} y for y[n] (the systems
 * (G_T + G_L) x = y solved in Sec. 7.1).  Same conventions as above.
 */
int tikh_toeplitz_solve_normal(const double* col, const double* row, int64_t m, int64_t n,
                               const double* y, double lambda, double* x);
int tikh_toeplitz_solve_normal_z(const tikh_c64* col, const tikh_c64* row, int64_t m, int64_t n,
                                 const tikh_c64* y, double lambda, tikh_c64* x);

/*
 * Batched solves.  nprob problems with host arrays m[nprob], n[nprob].
 * Device buffers are packed problem after problem (offsets are prefix sums):
 *   col:  sum m_p entries,  row: sum n_p entries,
 *   b:    for each problem p, nrhs right-hand sides of m_p entries,
 *   x:    for each problem p, for each lambda l, for each rhs r, n_p entries
 *         (x offset of (p,l,r) = xoff_p + (l*nrhs + r)*n_p),
 *   lambdas: HOST array [nprob * nlam] (lambda of (p,l) at p*nlam + l).
 *   info: DEVICE int32 array [nprob * nlam * nrhs] or NULL.
 * Asynchronous: returns after enqueueing; info is valid after the stream
 * completes.  complex_data selects double (0) or tikh_c64 (1) element type.
 */
int tikh_toeplitz_solve_batched(int64_t nprob, const int64_t* m, const int64_t* n,
                                const void* col, const void* row,
                                int64_t nlam, const double* lambdas,
                                int64_t nrhs, const void* b, void* x,
                                int32_t* info, int complex_data);

/*
 * Allocation-free variant of tikh_toeplitz_solve_batched, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, packing, results
 * (to rounding) and asynchrony, except that the call allocates nothing: the
 * library's workspace, twiddle tables and readback word come from a static
 * device buffer of 64 MiB per GPU (held until the process ends), and no
 * timing events are created.  The batch is split into chunks that fit it;
 * a call whose single group (or whose twiddle tables, given 640 N bytes + 1 MiB
 * for N extended nodes) does not fit returns TIKH_ETOOBIG without touching the
 * outputs (roughly: one right-hand side per group up to m + n ~ 2^14).  Every
 * call on a GPU shares that GPU's buffer and overwrites what the previous call
 * left there; calls that overlap on one GPU (several host threads, or several
 * streams without ordering between the calls) race and must not be made.
 * The per-merge transform sizing still synchronizes the library stream.
 */
int tikh_toeplitz_solve_batched_noalloc(int64_t nprob, const int64_t* m, const int64_t* n,
                                        const void* col, const void* row,
                                        int64_t nlam, const double* lambdas,
                                        int64_t nrhs, const void* b, void* x,
                                        int32_t* info, int complex_data);

/*
 * Toeplitz-Gramian problem (Sec. 2, third case; Sec. 3.4, eq. (gramblk) and
 * (ex7)): x = (G + L^H L)^{-1} y, where G is an n x n Hermitian Toeplitz
 * Gramian (for instance G = A^H W A of a non-uniform Fourier matrix, Sec. 7.4)
 * given by its first column gram[s] = G[s][0] (G[r][s] = gram[r-s] for r >= s,
 * conj(gram[s-r]) otherwise; gram[n-1] is the last entry), L is a p x n
 * Toeplitz regularizer (lcol[i] = l_i, i < p; lrow[j] = l_{-j}, 0 < j < n;
 * lrow[0] ignored), and y[n] is the right-hand side (T^H b of the underlying
 * least-squares problem).  The same extension (circulant blocks of size N >=
 * max(2n - 1, p + n - 1), Alg. 2), interpolation recursion and refinement as
 * the l2 solves; G + L^H L must be nonsingular.  Device arrays as above;
 * single-problem calls synchronize and return TIKH_ENUMERIC if info != 0.
 */
int tikh_gramian_solve(const double* gram, const double* lcol, const double* lrow, int64_t p, int64_t n,
                       const double* y, double* x);
int tikh_gramian_solve_z(const tikh_c64* gram, const tikh_c64* lcol, const tikh_c64* lrow, int64_t p, int64_t n,
                         const tikh_c64* y, tikh_c64* x);
/*
 * Batched: nprob problems with host arrays p[nprob], n[nprob]; packed device
 * buffers gram (sum n_q), lcol (sum p_q), lrow (sum n_q), y and x (for each
 * problem q, nrhs vectors of n_q entries); info as for tikh_toeplitz_solve_batched.
 * Asynchronous.
 */
int tikh_gramian_solve_batched(int64_t nprob, const int64_t* p, const int64_t* n, const void* gram,
                               const void* lcol, const void* lrow, int64_t nrhs, const void* y, void* x,
                               int32_t* info, int complex_data);

/*
 * Adjoint (backward) of x = solve(col, row, b, lambda) for a scalar loss with
 * upstream gradient gx[n] = dL/dRe(x) + i dL/dIm(x) (real data: dL/dx).  x is
 * the forward solution.  Derived from eq. (tiksol): w = (T^H T + lambda^2 I)^{-1} gx
 * (one more solve of the same operator, normal form), then
 *   g_b   = T w                                  [m]
 *   g_lam = -2 lambda Re<w, x>                   (device scalar)
 *   g_col[s], g_row[s] = sum over i-j = +-s of (b - T x) w^H - (T w) x^H
 * computed by FFT cross-correlations.  g_row[0] is set to 0 (a_0 lives in
 * col[0]).  Outputs are device arrays the caller owns.  Synchronizes.
 */
int tikh_toeplitz_solve_backward(const double* col, const double* row, int64_t m, int64_t n,
                                 const double* b, double lambda, const double* x,
                                 const double* gx, double* g_col, double* g_row,
                                 double* g_b, double* g_lambda);
int tikh_toeplitz_solve_backward_z(const tikh_c64* col, const tikh_c64* row, int64_t m, int64_t n,
                                   const tikh_c64* b, double lambda, const tikh_c64* x,
                                   const tikh_c64* gx, tikh_c64* g_col, tikh_c64* g_row,
                                   tikh_c64* g_b, double* g_lambda);

/*
 * Batched backward with the packing of tikh_toeplitz_solve_batched: x and gx
 * are packed like x there; g_col/g_row/g_b are packed per (p, l, r) solve
 * (g_col offset of (p,l,r) = colsum_p*nlam*nrhs + (l*nrhs+r)*m_p, likewise
 * g_row with n_p and g_b with m_p); g_lambda is a device array
 * [nprob*nlam*nrhs].  Asynchronous.
 */
int tikh_toeplitz_solve_backward_batched(int64_t nprob, const int64_t* m, const int64_t* n,
                                         const void* col, const void* row,
                                         int64_t nlam, const double* lambdas,
                                         int64_t nrhs, const void* b, const void* x,
                                         const void* gx, void* g_col, void* g_row,
                                         void* g_b, double* g_lambda,
                                         int32_t* info, int complex_data);

/*
 * Prepared batches (Alg. 1 run as a fixed launch schedule; for callers that replay the
 * same batch many times, e.g. a training step captured into a graph).  A prepare call
 * takes the arguments of tikh_toeplitz_solve_batched (or of the batched backward) with
 * one difference: `lambdas` is a DEVICE array [nprob * nlam] that every run reads, so
 * the caller may change the values between runs (or inside a captured graph).  It
 * plans the batch, allocates the batch's own workspace (tikh_prepared_workspace), uploads
 * the descriptors and runs the batch once, synchronously, recording the product
 * transform lengths for degrees 1/8 + 8 above the ones met (outputs and info of that
 * run are valid).  The pointer arguments (col, row, b, x, gx, outputs, info, lambdas)
 * are kept: they must stay valid and in place for the handle's lifetime.
 *
 * tikh_prepared_run enqueues the batch on the library stream (tikh_set_stream) with
 * kernel launches and stream/event ordering only: no host synchronization, no
 * allocation, no copy from host memory, so the call may be captured into a hipGraph.
 * Every solve takes `refine` refinement steps (the adaptive steps, the fallback
 * re-solve and the deferral of difficult points are not available: info bits stand as
 * set; defer_tol > 0 at prepare time gives TIKH_EINVAL).  The options in force at
 * prepare time apply to every run.  A lambda that is not positive and finite gives
 * info bit 64 for its solves.  Degrees beyond the recorded lengths give info bit 32.
 * Runs of one handle must not overlap; handles are independent of each other and of
 * the other entry points, except that tikh_release invalidates every handle (its runs
 * return TIKH_EINVAL; tikh_prepared_free still frees it).
 */
typedef struct tikh_prepared tikh_prepared;
int tikh_prepare_batched(int64_t nprob, const int64_t* m, const int64_t* n,
                         const void* col, const void* row, int64_t nlam,
                         const double* lambdas /* device */, int64_t nrhs, const void* b,
                         void* x, int32_t* info, int complex_data, tikh_prepared** handle);
int tikh_prepare_backward_batched(int64_t nprob, const int64_t* m, const int64_t* n,
                                  const void* col, const void* row, int64_t nlam,
                                  const double* lambdas /* device */, int64_t nrhs,
                                  const void* b, const void* x, const void* gx,
                                  void* g_col, void* g_row, void* g_b, double* g_lambda,
                                  int32_t* info, int complex_data, tikh_prepared** handle);
int tikh_prepared_run(tikh_prepared* handle);
int tikh_prepared_workspace(const tikh_prepared* handle, size_t* bytes);  /* host pointer */
int tikh_prepared_free(tikh_prepared* handle);   /* synchronizes the device; NULL is a no-op */

#ifdef __cplusplus
}
#endif

#endif /* TIKH_H */
