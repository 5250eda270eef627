// Internal declarations shared by the device kernels and the host driver of
// the superfast Tikhonov-Toeplitz solver.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tikh {

// The l2 basis for one right-hand side is 5 x 5 (x, sigma1, gamma1, gamma2, 1).
// Right-hand sides of the same operator (same T and lambda) share the pivot
// sequence, because the constant column is never a pivot: a group of NR
// right-hand sides carries the basis [[B0, v_1 .. v_NR], [0, I]] with
// C = 4 + NR columns, of which rows 0..3 are stored (4 C polynomials).
constexpr int MAXNR = 4;           // right-hand sides per group
constexpr int MAXC = 4 + MAXNR;    // basis columns
constexpr int LEAF_MAX = 256;      // max conditions per leaf (one wavefront, 4 per lane)
constexpr int FFT_LDS_MAX = 4096;  // max complex elements held by one LDS FFT workgroup
constexpr int FFT_THREADS = 256;

// One solve (one right-hand side) of a bucket (device array element).  The
// solves of a group are consecutive; col/row/m/n/k/lam/cplx are equal within a
// group.  A padding solve (group not full) has rhs == nullptr: zero data, no output.
struct SolveDesc {
    const void* col;   // generator a_0..a_{m-1}    (double or double2)
    const void* row;   // a_0, a_{-1}..a_{-(n-1)}   (double or double2)
    const void* rhs;   // b[m] (mode 0) or y[n] (mode 1)
    void* x;           // output x[n]
    int64_t m, n;
    int64_t k;         // circulant extension size: N - (m + n - 1)
    double lam;
    int32_t cplx;      // element type of col/row/rhs/x: 0 real double, 1 complex
    int32_t mode;      // 0: least squares with b, 1: normal form with y
    // backward (adjoint) solves only: rhs = upstream gradient gx (mode 1)
    const void* bin;   // forward right-hand side b[m]
    const void* xin;   // forward solution x[n]
    void* gcol;        // dL/d col [m]
    void* grow;        // dL/d row [n]
    void* gb;          // dL/d b [m]
    double* glam;      // dL/d lambda (scalar)
    int32_t backward;
    int32_t orig;      // index of this solve in the caller's info array (-1: padding solve)
    // Toeplitz-Gramian problem (G + L^H L) x = y: col/row/m hold the regularizer L
    // (p x n), gram the first column of the Hermitian Toeplitz Gramian G (n entries)
    const void* gram;
    int32_t gramian;
    int32_t lamx;      // index of this solve's lambda in the caller's array (problem * nlam + lambda)
};

// Per-group running state of the recursion.
struct SolveState {
    int32_t delta[4];  // tau-degrees of basis columns 1..4 (column 5 stays 0)
    int32_t info;      // 0 ok; or of bits 1 breakdown, 2 degree bound, 4 too many deferred conditions, 8 non-finite,
                       // 16 refinement estimate above its target after the last step, 32 recorded
                       // transform length too short, 64 invalid lambda (prepared batches)
    int32_t ndef;      // deferred (difficult) conditions of the current solve
    int32_t wide;      // set by the narrow pass of a two-pass kernel: this group is left to the wide pass
    double e0;         // relative size of the first refinement correction (error estimate of the first solve)
};

// Per-group metadata of a stored basis (one per slot).
struct SlotMeta {
    int32_t deg[MAXC]; // max polynomial degree of each column over rows 0..3 (-1 = zero column)
    unsigned long long colmax_bits[4];  // max |coefficient| of B0 columns (bit pattern of a non-negative double)
};

// One step of the serial single-condition construction (eq. (spbasis)).
struct LeafRec {
    double2 mu[MAXC];  // multipliers mu_i = -r_i / r_piv (mu[piv] = 0)
    double2 sig;       // node of the processed condition
    int32_t piv;       // pivot column (0..3), -1 if the step was skipped
    int32_t q;         // condition index (tree order)
    int32_t pad[2];
};

struct Plan {
    int64_t N;         // nodes, N = 2^p * M
    int64_t M;         // nodes per leaf (even, 5-smooth)
    int32_t p;         // depth
    int32_t K;         // conditions per leaf = 2M
    int64_t Q;         // twiddle-table size (multiple of every FFT length used)
    int64_t cap[40];   // degree capacity of bases stored for a subtree at depth d
    int64_t P[40];     // product FFT length at parent depth d
};

}  // namespace tikh
