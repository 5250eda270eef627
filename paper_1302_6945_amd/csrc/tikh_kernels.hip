// Device kernels of the superfast Tikhonov-Toeplitz solver for gfx950.
//
// Paper: Turnes, Balcan, Romberg, "Superfast Tikhonov Regularization of
// Toeplitz Systems".  Section/equation references are to that paper.
//
// All arithmetic is complex FP64 (double2 = (re, im)).  Evaluations follow the
// convention of eq. (vandprod): a vector rho is the polynomial
// rho(z) = sum_i rho_i z^i and F rho = [rho(w_nu)], w_nu = exp(+2 pi i nu / N).
#include "tikh_internal.h"
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <limits.h>

namespace tikh {

// ---------------------------------------------------------------- complex
__device__ __forceinline__ double2 c2(double a, double b) { return make_double2(a, b); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return c2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return c2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return c2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// a * b + c
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {
    return c2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ double2 cconj(double2 a) { return c2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return c2(a.x * s, a.y * s); }
__device__ __forceinline__ double cabs2(double2 a) { return fma(a.x, a.x, a.y * a.y); }
__device__ __forceinline__ double2 cneg(double2 a) { return c2(-a.x, -a.y); }
__device__ __forceinline__ bool cnonzero(double2 a) { return a.x != 0.0 || a.y != 0.0; }
// a / b by Smith's method
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    if (fabs(b.x) >= fabs(b.y)) {
        double t = b.y / b.x, d = fma(b.y, t, b.x);
        return c2((a.x + a.y * t) / d, (a.y - a.x * t) / d);
    } else {
        double t = b.x / b.y, d = fma(b.x, t, b.y);
        return c2((a.x * t + a.y) / d, (a.y * t - a.x) / d);
    }
}

// a / d for 0 <= a < 2^24, d >= 1, with a single-precision reciprocal estimate
// (error < 1) corrected by one step
__device__ __forceinline__ int fdiv(int a, float inv, int d) {
    int q = (int)((float)a * inv);
    int r = a - q * d;
    if (r < 0) --q;
    else if (r >= d) ++q;
    return q;
}

// x mod n for 0 <= x < 2^53 via a double-precision quotient (exact after one correction)
__device__ __forceinline__ int64_t mod_fast(int64_t x, int64_t n, double invn) {
    int64_t q = (int64_t)((double)x * invn);
    int64_t r = x - q * n;
    if (r < 0) r += n;
    else if (r >= n) r -= n;
    return r;
}

// e^{sign * 2 pi i idx / Q} for 0 <= idx < Q
__device__ __forceinline__ double2 twd(const double2* __restrict__ tw, int idx, int sign) {
    double2 t = tw[idx];
    return sign > 0 ? t : cconj(t);
}

// e^{sign * 2 pi i idx / Q} from the table tw[q] = e^{2 pi i q / Q}
__device__ __forceinline__ double2 twq(const double2* __restrict__ tw, int64_t Q, int64_t idx, int sign) {
    int64_t r = idx % Q;
    if (r < 0) r += Q;
    double2 t = tw[r];
    return sign > 0 ? t : cconj(t);
}

// e^{2 pi i x / M} (0 <= x < M) from a two-level table
// t = [e^{2 pi i j / M}, j < 2^bits | e^{2 pi i j 2^bits / M}, j <= (M - 1) >> bits]:
// both parts are small, so scattered indices stay in cache
__device__ __forceinline__ double2 tw2(const double2* __restrict__ t, int bits, int x) {
    return cmul(t[(1 << bits) + (x >> bits)], t[x & ((1 << bits) - 1)]);
}

__device__ __forceinline__ double2 load_elem(const void* p, int64_t i, int cplx) {
    if (cplx) return ((const double2*)p)[i];
    return c2(((const double*)p)[i], 0.0);
}
__device__ __forceinline__ double2 gen_coef(const SolveDesc& d, int64_t s) {
    // a_s of T = [a_{i-j}] (Sec. 1)
    return s >= 0 ? load_elem(d.col, s, d.cplx) : load_elem(d.row, -s, d.cplx);
}

__device__ __forceinline__ int bitrev(int v, int bits) {
    return bits == 0 ? 0 : (int)(__brev((unsigned)v) >> (32 - bits));
}

// Power-of-two scale 2^-e bringing a positive maximum to [0.5, 1).
__device__ __forceinline__ double pow2_inv_scale(unsigned long long bits) {
    double m = __longlong_as_double((long long)bits);
    if (!(m > 0.0) || !isfinite(m)) return 1.0;
    int e;
    frexp(m, &e);
    return ldexp(1.0, -e);
}

// ---------------------------------------------------------------- wave reductions
__device__ __forceinline__ int wave_min_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// ---------------------------------------------------------------- FFT (LDS, Stockham)
// DFT of size R with root w = e^{sign 2 pi i / R}, in registers.
template <int R> __device__ __forceinline__ void bfly(double2* v, int sign);

template <> __device__ __forceinline__ void bfly<2>(double2* v, int) {
    double2 a = v[0], b = v[1];
    v[0] = cadd(a, b); v[1] = csub(a, b);
}
template <> __device__ __forceinline__ void bfly<4>(double2* v, int sign) {
    double2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    double2 b0 = cadd(v[1], v[3]), b1 = csub(v[1], v[3]);
    // b1 * (sign * i)
    double2 jb1 = sign > 0 ? c2(-b1.y, b1.x) : c2(b1.y, -b1.x);
    v[0] = cadd(a0, b0); v[2] = csub(a0, b0);
    v[1] = cadd(a1, jb1); v[3] = csub(a1, jb1);
}
template <> __device__ __forceinline__ void bfly<3>(double2* v, int sign) {
    const double c = -0.5, s = sign * 0.86602540378443864676;   // e^{sign 2 pi i/3}
    double2 t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
    double2 a = v[0];
    v[0] = cadd(a, t1);
    double2 m1 = c2(a.x + c * t1.x, a.y + c * t1.y);
    double2 m2 = c2(-s * t2.y, s * t2.x);                          // i s t2
    v[1] = cadd(m1, m2); v[2] = csub(m1, m2);
}
template <> __device__ __forceinline__ void bfly<5>(double2* v, int sign) {
    const double c1 = 0.30901699437494742410, c2_ = -0.80901699437494742410;
    const double s1 = sign * 0.95105651629515357212, s2 = sign * 0.58778525229247312917;
    double2 a = v[0];
    double2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    double2 u1 = csub(v[1], v[4]), u2 = csub(v[2], v[3]);
    v[0] = cadd(a, cadd(t1, t2));
    double2 m1 = c2(a.x + c1 * t1.x + c2_ * t2.x, a.y + c1 * t1.y + c2_ * t2.y);
    double2 m2 = c2(a.x + c2_ * t1.x + c1 * t2.x, a.y + c2_ * t1.y + c1 * t2.y);
    // i*(s1 u1 + s2 u2), i*(s2 u1 - s1 u2)
    double2 n1 = c2(-(s1 * u1.y + s2 * u2.y), s1 * u1.x + s2 * u2.x);
    double2 n2 = c2(-(s2 * u1.y - s1 * u2.y), s2 * u1.x - s1 * u2.x);
    v[1] = cadd(m1, n1); v[4] = csub(m1, n1);
    v[2] = cadd(m2, n2); v[3] = csub(m2, n2);
}

// Split-radix butterfly of size R = R1 * R2 (R a divisor of 16): R2 DFTs of
// size R1 over the inputs n = R2 n1 + n2, twiddles e^{sign 2 pi i n2 k1 / R},
// then R1 DFTs of size R2, giving output k = k1 + R1 k2.
__device__ __forceinline__ double2 rot16(double2 a, int e, int sign) {
    // a * e^{sign 2 pi i e / 16}
    e &= 15;
    if (e == 0) return a;
    if (e == 4) return sign > 0 ? c2(-a.y, a.x) : c2(a.y, -a.x);
    if (e == 8) return cneg(a);
    if (e == 12) return sign > 0 ? c2(a.y, -a.x) : c2(-a.y, a.x);
    const double C1 = 0.92387953251128675613, S1 = 0.38268343236508977173, RH = 0.70710678118654752440;
    double c, s;
    switch (e) {
        case 1: c = C1; s = S1; break;
        case 2: c = RH; s = RH; break;
        case 3: c = S1; s = C1; break;
        case 5: c = -S1; s = C1; break;
        case 6: c = -RH; s = RH; break;
        case 7: c = -C1; s = S1; break;
        case 9: c = -C1; s = -S1; break;
        case 10: c = -RH; s = -RH; break;
        case 11: c = -S1; s = -C1; break;
        case 13: c = S1; s = -C1; break;
        case 14: c = RH; s = -RH; break;
        default: c = C1; s = -S1; break;   // 15
    }
    return cmul(a, c2(c, sign > 0 ? s : -s));
}

// a * e^{sign 2 pi i e / R} for R = 6, 8, 9, 12, 16 (quarter turns exactly)
template <int R>
__device__ __forceinline__ double2 rotR(double2 a, int e, int sign) {
    e %= R;
    if (e == 0) return a;
    if (R == 16) return rot16(a, e, sign);
    if (R == 8) return rot16(a, 2 * e, sign);
    if ((4 * e) % R == 0) {
        const int q = 4 * e / R;
        if (q == 2) return cneg(a);
        const bool pos = (q == 1) == (sign > 0);
        return pos ? c2(-a.y, a.x) : c2(a.y, -a.x);
    }
    const double H = 0.5, T = 0.866025403784438646764;
    double c = 1.0, s = 0.0;
    if (R == 6 || R == 12) {
        const int e12 = R == 6 ? 2 * e : e;
        switch (e12) {
            case 1: c = T; s = H; break;
            case 2: c = H; s = T; break;
            case 4: c = -H; s = T; break;
            case 5: c = -T; s = H; break;
            case 7: c = -T; s = -H; break;
            case 8: c = -H; s = -T; break;
            case 10: c = H; s = -T; break;
            default: c = T; s = -H; break;   // 11
        }
    } else {   // R == 9
        const double C1 = 0.766044443118978035202, S1 = 0.642787609686539326323;
        const double C2 = 0.173648177666930348852, S2 = 0.984807753012208059367;
        const double C4 = -0.939692620785908384054, S4 = 0.342020143325668733044;
        switch (e) {
            case 1: c = C1; s = S1; break;
            case 2: c = C2; s = S2; break;
            case 3: c = -H; s = T; break;
            case 4: c = C4; s = S4; break;
            case 5: c = C4; s = -S4; break;
            case 6: c = -H; s = -T; break;
            case 7: c = C2; s = -S2; break;
            default: c = C1; s = -S1; break;  // 8
        }
    }
    return cmul(a, c2(c, sign > 0 ? s : -s));
}

template <int R1, int R2>
__device__ __forceinline__ void bfly_split(double2* v, int sign) {
    constexpr int R = R1 * R2;
    double2 y[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
        double2 t[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[R2 * n1 + n2];
        bfly<R1>(t, sign);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) y[n2 * R1 + k1] = rotR<R>(t[k1], n2 * k1, sign);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        double2 t[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) t[n2] = y[n2 * R1 + k1];
        bfly<R2>(t, sign);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
    }
}
template <> __device__ __forceinline__ void bfly<6>(double2* v, int sign) { bfly_split<2, 3>(v, sign); }
template <> __device__ __forceinline__ void bfly<8>(double2* v, int sign) { bfly_split<2, 4>(v, sign); }
template <> __device__ __forceinline__ void bfly<9>(double2* v, int sign) { bfly_split<3, 3>(v, sign); }
template <> __device__ __forceinline__ void bfly<12>(double2* v, int sign) { bfly_split<4, 3>(v, sign); }
template <> __device__ __forceinline__ void bfly<16>(double2* v, int sign) { bfly_split<4, 4>(v, sign); }

// v[r] *= e^{sign 2 pi i r idx / L} for r = 1..R-1 (ltw[j] = e^{2 pi i j / L},
// r idx < L).  For R > 5 only the powers of two below R are read from the
// table; the others are products of at most three of them.
template <int R>
__device__ __forceinline__ void stage_twiddle(double2* v, const double2* __restrict__ ltw, int idx, int sign) {
    if (R <= 5) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twd(ltw, r * idx, sign));
    } else {
        double2 w[R];
#pragma unroll
        for (int h = 1; h < R; h *= 2) w[h] = twd(ltw, h * idx, sign);
#pragma unroll
        for (int r = 3; r < R; ++r) {
            const int h = r >= 8 ? 8 : (r >= 4 ? 4 : 2);
            if (r != h) w[r] = cmul(w[h], w[r - h]);
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r]);
    }
}

// LDS index with one padding element per 16: strided butterfly accesses of
// 16-byte elements then fall on distinct banks.
__device__ __forceinline__ int lds_ix(int i) { return i + (i >> 4); }

struct FftPlanDev {
    int L;
    int nst;
    int radix[24];
};

// One Stockham stage of radix R over `nl` lines of length L (Ns = product of
// the previous radices): butterfly j of a line reads elements j + r L/R and
// writes (j / Ns) Ns R + (j % Ns) + r Ns.  The first stage reads its inputs
// through `ld` (global memory) and the last writes through `st`; the stages
// between go through LDS.  `linefast` maps consecutive threads to
// consecutive lines (strided lines in global memory).
template <int R, int CAP, typename LD, typename ST>
__device__ __forceinline__ void fft_stage(double2* sm, int L, int nl, int Ns, int sign, const double2* __restrict__ ltw, bool gin,
                          bool gout, bool linefast, LD& ld, ST& st) {
    constexpr int MB = (CAP / R + FFT_THREADS - 1) / FFT_THREADS;
    const int per = L / R;
    const int nb = nl * per;
    const int tstep = L / (Ns * R);
    const float invper = 1.0f / (float)per, invNs = 1.0f / (float)Ns, invnl = 1.0f / (float)nl;
    const bool lf = linefast && (gin || gout);
    double2 v[MB][R];
#pragma unroll
    for (int it = 0; it < MB; ++it) {
        const int b = threadIdx.x + it * FFT_THREADS;
        if (b < nb) {
            int line, j;
            if (lf) { j = fdiv(b, invnl, nl); line = b - j * nl; }
            else { line = fdiv(b, invper, per); j = b - line * per; }
            if (gin) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[it][r] = ld(line, j + r * per);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) v[it][r] = sm[lds_ix(line * L + j + r * per)];
            }
        }
    }
    if (!gin && !gout) __syncthreads();
#pragma unroll
    for (int it = 0; it < MB; ++it) {
        const int b = threadIdx.x + it * FFT_THREADS;
        if (b < nb) {
            int line, j;
            if (lf) { j = fdiv(b, invnl, nl); line = b - j * nl; }
            else { line = fdiv(b, invper, per); j = b - line * per; }
            const int blk = fdiv(j, invNs, Ns);
            const int k = j - blk * Ns;
            if (Ns > 1) stage_twiddle<R>(v[it], ltw, k * tstep, sign);
            bfly<R>(v[it], sign);
            const int ob = blk * Ns * R + k;
            if (gout) {
#pragma unroll
                for (int r = 0; r < R; ++r) st(line, ob + r * Ns, v[it][r]);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) sm[lds_ix(line * L + ob + r * Ns)] = v[it][r];
            }
        }
    }
    if (!gout) __syncthreads();
}

// Batched in-place FFT of lines held in global memory.
// Line l of solve s starts at data + s*solve_stride + (l / lines_inner)*outer_stride
// + (l % lines_inner)*line_stride; element k at + k*elem_stride.  lpw lines
// per workgroup (lpw*L <= the kernel's capacity).  Optional four-step twiddle: output
// element j of line l multiplied by e^{sign 2 pi i j (l % lines_inner) / post_L}.
//
// The first pass of a transform can read its input directly from a stored
// basis instead of `data` (load_mode), and the last pass of an inverse
// product transform can write into a basis slot (store_mode); "original line"
// o = l / lines_inner and "offset" = (l % lines_inner)*line_stride + k*elem_stride
// index the transform of one basis entry.
struct FftArgs {
    double2* data;
    int64_t solve_stride, line_stride, elem_stride, outer_stride;
    int64_t nlines, lines_inner;
    int sign;
    int lpw;
    int64_t post_L;
    double scale;
    const double2* tw;               // e^{2 pi i q / Q}, q < Q (fused twist of evaluation lines)
    int64_t Q;
    const double2* ltw;              // e^{2 pi i j / L}, j < L (stages)
    const double2* ptw;              // two-level table of e^{2 pi i j / post_L} (four-step twiddle)
    int pbits;
    const double2* ftw;              // two-level table of e^{2 pi i j / fold_N} (evaluation twist)
    int fbits;
    FftPlanDev pl;
    // fused load: 0 = data, 1 = zero-padded basis entry elist[o], 2 = twisted and folded
    // basis entry o/2 at coset offset fold_o + (o & 1) (evaluation)
    int load_mode;
    const double2* src;
    int64_t src_stride, src_cp1;
    const SlotMeta* src_meta;
    const int* elist;
    int C;
    int64_t fold_L, fold_o, fold_N;
    // fused store: 0 = data, 1 = basis slot entry dst_elist[o], scaled by 1/L_total,
    // offsets <= degree only, with column maxima
    int store_mode;
    double2* dst;
    int64_t dst_stride, dst_cp1;
    SlotMeta* dst_meta;
    const int* dst_elist;
    double dst_scale;
    // fused store, columns 4..C-1: add the same entry of this basis (the left factor's
    // V block, which enters the product unchanged), offsets up to its degree
    const double2* add_src;
    int64_t add_stride, add_cp1;
    const SlotMeta* add_meta;
};

// Per-line descriptors of the fused loads and stores, computed once per
// workgroup.  Fused load 1: element k of the line is
// src[lsrc + k*es] * lsc if k*es <= llim, else 0.  Fused load 2: entry
// src[lsrc + i] folded over i = off + t*fold_L (off = in*line_stride + k*es,
// i <= llim) and twisted by w^{loc*i}.  Fused store: element k goes to
// dst[dbase + k*es] (scaled by dst_scale) if k*es <= dlim.
// Offsets are 32-bit, relative to the line's group (every per-group region
// holds fewer than 2^31 elements).
struct FftLineInfo {
    int lsrc, llim;
    int64_t loc;
    double lsc;
    double2 lstep;                   // fused load 2: w^{loc fold_L}
    int dbase, dlim;
    int dcol;
    int abase, alim;
};

__device__ __forceinline__ void fft_line_info(const FftArgs& a, int64_t s, int64_t o, int64_t in, FftLineInfo& li) {
    const int64_t inoff = in * a.line_stride;
    if (a.load_mode) {
        const SlotMeta& mt = a.src_meta[s];
        const int e = a.load_mode == 1 ? a.elist[o] : (int)(o >> 1);
        const int col = e % a.C;
        li.lsc = col < 4 ? pow2_inv_scale(mt.colmax_bits[col]) : 1.0;
        li.lsrc = (int)((int64_t)e * a.src_cp1 + (a.load_mode == 1 ? inoff : 0));
        li.llim = (int)(a.load_mode == 1 ? (int64_t)mt.deg[col] - inoff : (int64_t)mt.deg[col]);
        li.loc = a.load_mode == 2 ? a.fold_o + (o & 1) : 0;
        if (a.load_mode == 2)
            li.lstep = tw2(a.ftw, a.fbits, mod_fast(li.loc * a.fold_L, a.fold_N, 1.0 / (double)a.fold_N));
    }
    if (a.store_mode) {
        const int e = a.dst_elist[o];
        const int col = e % a.C;
        li.dcol = col;
        li.dbase = (int)((int64_t)e * a.dst_cp1 + inoff);
        li.dlim = (int)(min((int64_t)a.dst_meta[s].deg[col], a.dst_cp1 - 1) - inoff);
        li.alim = -1;
        li.abase = 0;
        if (a.add_src && col >= 4) {
            li.abase = (int)((int64_t)e * a.add_cp1 + inoff);
            li.alim = (int)((int64_t)a.add_meta[s].deg[col] - inoff);
        }
    }
}

// twisted and folded evaluation input: sum over i = off + t L <= deg of B[i] w^{oc i},
// with w^{oc (off + t L)} = w^{oc off} (w^{oc L})^t.  Split into the first
// term (its loads are independent of other elements, so several elements
// issue them together) and the remaining terms.
struct FoldTerm {
    double2 acc, w;
    int off;
};
__device__ __forceinline__ FoldTerm fft_fold_first(const FftArgs& a, const double2* __restrict__ srcg,
                                                   const FftLineInfo& li, int off) {
    FoldTerm f;
    f.off = off;
    f.acc = c2(0.0, 0.0);
    f.w = c2(1.0, 0.0);
    if (off <= li.llim) {
        const double invN = 1.0 / (double)a.fold_N;
        f.w = tw2(a.ftw, a.fbits, mod_fast(li.loc * off, a.fold_N, invN));
        f.acc = cmul(srcg[li.lsrc + off], f.w);
    }
    return f;
}
__device__ __forceinline__ double2 fft_fold_rest(const FftArgs& a, const double2* __restrict__ srcg,
                                                 const FftLineInfo& li, FoldTerm f) {
    const int fl = (int)a.fold_L;
    if (f.off + fl <= li.llim) {
        const double2 wstep = li.lstep;
        for (int i = f.off + fl; i <= li.llim; i += fl) {
            f.w = cmul(f.w, wstep);
            f.acc = cfma(srcg[li.lsrc + i], f.w, f.acc);
        }
    }
    return cscale(f.acc, li.lsc);
}

// Batched FFT of lines (see FftArgs).  The first stage reads its inputs and
// the last stage writes its outputs directly between registers and global
// memory (plain lines, zero-padded slot entries, slot stores); the folded
// evaluation input goes through one LDS prologue loop.
// CAP = points held by one workgroup: 4096 (radices up to 16) or 2048 (radices up
// to 9: half the LDS and registers, so twice the workgroups per CU).
template <int CAP>
__global__ __launch_bounds__(FFT_THREADS, CAP <= 2048 ? 4 : 1) void k_fft(const FftArgs a) {
    __shared__ double2 sm[CAP + CAP / 16];
    __shared__ int sh_base[64];
    __shared__ int sh_in[64];
    __shared__ FftLineInfo sh_li[64];
    const int L = a.pl.L;
    const int64_t l0 = (int64_t)blockIdx.x * a.lpw;
    const int nl = (int)min((int64_t)a.lpw, a.nlines - l0);
    const int64_t s = blockIdx.y;
    // per-group base pointers; offsets below are 32-bit
    double2* base = a.data + s * a.solve_stride;
    const double2* srcg = a.load_mode ? a.src + s * a.src_stride : nullptr;
    double2* dstg = a.store_mode ? a.dst + s * a.dst_stride : nullptr;
    const double2* addg = a.add_src ? a.add_src + s * a.add_stride : nullptr;
    if ((int)threadIdx.x < nl) {
        const int64_t l = l0 + threadIdx.x, o = l / a.lines_inner, in = l - o * a.lines_inner;
        sh_base[threadIdx.x] = (int)(o * a.outer_stride + in * a.line_stride);
        sh_in[threadIdx.x] = (int)in;
        if (a.load_mode || a.store_mode) fft_line_info(a, s, o, in, sh_li[threadIdx.x]);
    }
    __syncthreads();
    const int nst = a.pl.nst;
    const bool linefast = (a.elem_stride != 1);
    const bool dload = (a.load_mode != 2) && nst > 0, dstore = nst > 0;
    const int tot = nl * L;
    const float invL = 1.0f / (float)L, invnl = 1.0f / (float)nl;
    const int es = (int)a.elem_stride;
    const int lstr = (int)a.line_stride;
    double cmx[4] = {0.0, 0.0, 0.0, 0.0};
    auto ld = [&](int g, int k) -> double2 {
        if (a.load_mode == 1) {
            const FftLineInfo& li = sh_li[g];
            const int off = k * es;
            return off <= li.llim ? cscale(srcg[li.lsrc + off], li.lsc) : c2(0.0, 0.0);
        }
        return base[sh_base[g] + k * es];
    };
    auto st = [&](int g, int k, double2 v) {
        // k * in < post_L: k < L and in < post_L / L for both four-step passes
        if (a.post_L) {
            const double2 t = tw2(a.ptw, a.pbits, k * sh_in[g]);
            v = cmul(v, a.sign > 0 ? t : cconj(t));
        }
        if (a.scale != 1.0) v = cscale(v, a.scale);
        if (a.store_mode) {
            const FftLineInfo& li = sh_li[g];
            const int off = k * es;
            if (off <= li.dlim) {
                v = cscale(v, a.dst_scale);
                if (off <= li.alim) v = cadd(v, addg[li.abase + off]);
                dstg[li.dbase + off] = v;
                const int col = li.dcol;
                if (col < 4) {
                    const double m2 = cabs2(v);
#pragma unroll
                    for (int c = 0; c < 4; ++c) if (c == col) cmx[c] = fmax(cmx[c], m2);
                }
            }
        } else {
            base[sh_base[g] + k * es] = v;
        }
    };
    if (!dload) {
        // four elements per thread at a time: their first loads are issued together
        constexpr int U = 4;
        for (int i0 = threadIdx.x; i0 < tot; i0 += U * FFT_THREADS) {
            FoldTerm f[U];
            int gg[U], kk[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = min(i0 + u * FFT_THREADS, tot - 1);
                int g, k;
                if (!linefast) { g = fdiv(i, invL, L); k = i - g * L; } else { k = fdiv(i, invnl, nl); g = i - k * nl; }
                gg[u] = g; kk[u] = k;
                if (a.load_mode == 2)
                    f[u] = fft_fold_first(a, srcg, sh_li[g], sh_in[g] * lstr + k * es);
                else
                    f[u].acc = ld(g, k);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (i0 + u * FFT_THREADS < tot) {
                    const double2 v = a.load_mode == 2 ? fft_fold_rest(a, srcg, sh_li[gg[u]], f[u]) : f[u].acc;
                    if (nst == 0) st(gg[u], kk[u], v);
                    else sm[lds_ix(gg[u] * L + kk[u])] = v;
                }
            }
        }
        __syncthreads();
    } else if (nst == 0) {
        for (int g = threadIdx.x; g < nl; g += FFT_THREADS) st(g, 0, ld(g, 0));
    }
    int Ns = 1;
    for (int q = 0; q < nst; ++q) {
        const int R = a.pl.radix[q];
        const bool gin = (q == 0) && dload, gout = (q == nst - 1) && dstore;
        if (CAP > 2048 && R == 16) fft_stage<16, CAP>(sm, L, nl, Ns, a.sign, a.ltw, gin, gout, linefast, ld, st);
        else if (CAP > 2048 && R == 12) fft_stage<12, CAP>(sm, L, nl, Ns, a.sign, a.ltw, gin, gout, linefast, ld, st);
        else if (R == 9) fft_stage<9, CAP>(sm, L, nl, Ns, a.sign, a.ltw, gin, gout, linefast, ld, st);
        else if (R == 8) fft_stage<8, CAP>(sm, L, nl, Ns, a.sign, a.ltw, gin, gout, linefast, ld, st);
        else if (R == 6) fft_stage<6, CAP>(sm, L, nl, Ns, a.sign, a.ltw, gin, gout, linefast, ld, st);
        else if (R == 4) fft_stage<4, CAP>(sm, L, nl, Ns, a.sign, a.ltw, gin, gout, linefast, ld, st);
        else if (R == 2) fft_stage<2, CAP>(sm, L, nl, Ns, a.sign, a.ltw, gin, gout, linefast, ld, st);
        else if (R == 3) fft_stage<3, CAP>(sm, L, nl, Ns, a.sign, a.ltw, gin, gout, linefast, ld, st);
        else fft_stage<5, CAP>(sm, L, nl, Ns, a.sign, a.ltw, gin, gout, linefast, ld, st);
        Ns *= R;
    }
    if (a.store_mode) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double mx = wave_max_d(cmx[c]);
            if ((threadIdx.x & 63) == 0 && mx > 0.0)
                atomicMax(&a.dst_meta[s].colmax_bits[c], (unsigned long long)__double_as_longlong(sqrt(mx)));
        }
    }
}

// Four-step order to natural order, out of place: src holds, for each line of length
// L1*L2, the four-step order X[j1 + L1 j2] at j1*L2 + j2; dst receives natural order.
// A transpose of each line's L1 x L2 matrix, dst[j2 L1 + j1] = src[j1 L2 + j2], through
// 32 x 32 LDS tiles so that both sides are read and written in order.  Block x: (line,
// tile row, tile column); block y: item; 256 threads (32 x 8).
__global__ __launch_bounds__(256) void k_fourstep_transpose(const double2* __restrict__ src, double2* __restrict__ dst,
                                                            int64_t src_solve_stride, int64_t dst_solve_stride,
                                                            int64_t line_stride, int64_t L1, int64_t L2) {
    __shared__ double2 tile[32][33];
    const int64_t t1n = (L1 + 31) / 32, t2n = (L2 + 31) / 32;
    const int64_t b = blockIdx.x;
    const int64_t line = b / (t1n * t2n), rem = b - line * (t1n * t2n);
    const int64_t t1 = rem / t2n, t2 = rem - t1 * t2n;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const double2* sl = src + blockIdx.y * src_solve_stride + line * line_stride;
    double2* dl = dst + blockIdx.y * dst_solve_stride + line * line_stride;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t j1 = t1 * 32 + ty + 8 * r, j2 = t2 * 32 + tx;
        if (j1 < L1 && j2 < L2) tile[ty + 8 * r][tx] = sl[j1 * L2 + j2];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t j2 = t2 * 32 + ty + 8 * r, j1 = t1 * 32 + tx;
        if (j1 < L1 && j2 < L2) dl[j2 * L1 + j1] = tile[tx][ty + 8 * r];
    }
}

__global__ void k_copy(const double2* __restrict__ src, double2* __restrict__ dst, int64_t src_solve_stride,
                       int64_t dst_solve_stride, int64_t count) {
    const int64_t s = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[s * dst_solve_stride + i] = src[s * src_solve_stride + i];
}

// ---------------------------------------------------------------- setup (Sec. 3.1, 3.3, 4.1)
// Indexing: a bucket holds G groups of nr solves; solve s = g * nr + r.
// Group-level kernels use sd[g * nr] for the operator (col, row, m, n, k, lambda).

// Root-mean-square of the generator (scale of the arbitrary extension
// entries, Sec. 6.2: chosen "similar in value" to the known coefficients).
// Also the sum of the generator's magnitudes, sum_s |a_s| >= ||T||_2 (asum, may be null).
__global__ __launch_bounds__(256) void k_gen_rms(const SolveDesc* __restrict__ sd, int nr, double* __restrict__ rms,
                                                 double* __restrict__ asum) {
    const SolveDesc d = sd[(int64_t)blockIdx.x * nr];
    double acc = 0.0, acc1 = 0.0;
    const int64_t cnt = d.m + d.n - 1;
    for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
        const double a2 = cabs2(gen_coef(d, i - (d.n - 1)));
        acc += a2;
        acc1 += sqrt(a2);
    }
    __shared__ double red[256], red1[256];
    red[threadIdx.x] = acc;
    red1[threadIdx.x] = acc1;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) { red[threadIdx.x] += red[threadIdx.x + o]; red1[threadIdx.x] += red1[threadIdx.x + o]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        rms[blockIdx.x] = sqrt(red[0] / (double)cnt);
        if (asum) asum[blockIdx.x] = red1[0];
    }
}

__device__ __forceinline__ double hash_unit(uint64_t x) {
    // splitmix64 finalizer -> uniform in [-1, 1)
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Synthetic real data for timing runs: out[i] = u_i e^{-|i - center| / decay}
// (decay <= 0: no envelope), u_i uniform in [-1, 1) from a hash of (seed, i).
__global__ void k_synth(double* __restrict__ out, int64_t count, uint64_t seed, int64_t center, double decay) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        double v = hash_unit(seed * 0x9E3779B97F4A7C15ull + (uint64_t)i);
        if (decay > 0.0) v *= exp(-fabs((double)(i - center)) / decay);
        out[i] = v;
    }
}

// First column of the k-circulant extension (eq. (circexp)) per group:
// c_T[r] = a_{r-(n+k-1)} for r >= k; r < k are the arbitrary entries a_{-n-k+1..-n}.
__global__ void k_build_ct(const SolveDesc* __restrict__ sd, int nr, const double* __restrict__ rms,
                           double2* __restrict__ out, int64_t N, int64_t stride) {
    const int64_t g = blockIdx.y;
    const SolveDesc d = sd[g * nr];
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x) {
        double2 v;
        if (r >= d.k) {
            v = gen_coef(d, r - (N - d.m));
        } else {
            double sc = rms[g] * 1.7320508075688772;   // uniform in [-sqrt3, sqrt3) has unit rms
            uint64_t key = ((uint64_t)d.m << 20) ^ (uint64_t)d.n ^ ((uint64_t)r << 44);
            v = c2(sc * hash_unit(key), d.cplx ? sc * hash_unit(key ^ 0x5851F42D4C957F2Dull) : 0.0);
        }
        out[g * stride + r] = v;
    }
}

// Toeplitz-Gramian problem (Sec. 3.4): entry g_s of the Hermitian Toeplitz
// Gramian, s = -(n-1) .. n-1 (g_{-s} = conj(g_s)).
__device__ __forceinline__ double2 gram_coef(const SolveDesc& d, int64_t s) {
    const double2 v = load_elem(d.gram, s >= 0 ? s : -s, d.cplx);
    return s >= 0 ? v : cconj(v);
}

// Root-mean-square of the Gramian's 2n - 1 generator entries (scale of its
// arbitrary extension entries).
__global__ __launch_bounds__(256) void k_gram_rms(const SolveDesc* __restrict__ sd, int nr, double* __restrict__ rms) {
    const SolveDesc d = sd[(int64_t)blockIdx.x * nr];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < d.n; i += blockDim.x) acc += (i == 0 ? 1.0 : 2.0) * cabs2(gram_coef(d, i));
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) rms[blockIdx.x] = sqrt(red[0] / (double)(2 * d.n - 1));
}

// First column of the circulant extension of the Gramian G (n x n), eq. (gramblk):
// c_G[N - n + s] = g_s for |s| < n, so that rows N-n.. N-1 and columns 0..n-1 of the
// circulant hold G; the N - 2n + 1 entries r <= N - 2n are arbitrary.
__global__ void k_build_cg(const SolveDesc* __restrict__ sd, int nr, const double* __restrict__ rms,
                           double2* __restrict__ out, int64_t N, int64_t stride) {
    const int64_t g = blockIdx.y;
    const SolveDesc d = sd[g * nr];
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x) {
        double2 v;
        if (r > N - 2 * d.n) {
            v = gram_coef(d, r - (N - d.n));
        } else {
            double sc = rms[g] * 1.7320508075688772;
            uint64_t key = ((uint64_t)d.n << 21) ^ ((uint64_t)r << 43) ^ 0x2545F4914F6CDD1Dull;
            v = c2(sc * hash_unit(key), d.cplx ? sc * hash_unit(key ^ 0x5851F42D4C957F2Dull) : 0.0);
        }
        out[g * stride + r] = v;
    }
}

// dst[i] = scale * src[off + i] for i < len, 0 for len <= i < N, per solve.
// src is either a user array (per-solve pointer in SolveDesc: which = 0 rhs,
// 1 x, 2 the forward solution xin of an adjoint solve; padding solves read 0)
// or an internal complex buffer (isrc != nullptr).
__global__ void k_load_pad(const SolveDesc* __restrict__ sd, int which, const double2* __restrict__ isrc,
                           int64_t isrc_stride, int len_kind, int64_t off, double scale,
                           double2* __restrict__ dst, int64_t N, int64_t stride) {
    const int64_t s = blockIdx.y;
    const SolveDesc d = sd[s];
    const int64_t len = len_kind == 0 ? d.m : d.n;
    const void* src = which == 0 ? d.rhs : (which == 1 ? (const void*)d.x : d.xin);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        double2 v = c2(0.0, 0.0);
        if (i < len) {
            if (isrc) v = isrc[s * isrc_stride + off + i];
            else if (d.rhs) v = load_elem(src, off + i, d.cplx);
            v = cscale(v, scale);
        }
        dst[s * stride + i] = v;
    }
}

// buf[nu] *= symbol: mode 0: c^(nu) (C_k(T), Sec. 3.1 eq. (circdiag));
// mode 1: w^{(k-1) nu} conj(c^(nu)) (C_k(T^H), whose symbol follows from T's in O(N), Sec. 7.3).
// chat is per group (solve s uses group s / nr).
__global__ void k_mul_symbol(const SolveDesc* __restrict__ sd, int nr, const double2* __restrict__ chat,
                             double2* __restrict__ buf, int64_t N, int64_t stride, int mode,
                             const double2* __restrict__ tw, int64_t Q) {
    const int64_t s = blockIdx.y;
    const int64_t g = s / nr;
    const int64_t k = sd[s].k;
    for (int64_t nu = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; nu < N; nu += (int64_t)gridDim.x * blockDim.x) {
        double2 c = chat[g * stride + nu];
        double2 sym;
        if (mode == 0) sym = c;
        else sym = cmul(twq(tw, Q, (((k - 1) % N + N) % N) * nu % N * (Q / N), +1), cconj(c));
        buf[s * stride + nu] = cmul(buf[s * stride + nu], sym);
    }
}

// dst[i] = scale * buf[N - len + i] for i < len (len = m or n): the bottom block
// of a circulant product (rows of T inside C_k(T), or of T^H inside C_k(T^H)).
__global__ void k_take_tail(const SolveDesc* __restrict__ sd, const double2* __restrict__ buf, int64_t N,
                            int64_t stride, int len_kind, double scale, double2* __restrict__ dst,
                            int64_t dst_stride) {
    const int64_t s = blockIdx.y;
    const SolveDesc d = sd[s];
    const int64_t len = len_kind == 0 ? d.m : d.n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
        dst[s * dst_stride + i] = cscale(buf[s * stride + N - len + i], scale);
}

// Residual of the normal equations: r = y - (T^H T x) - lam^2 x  (all length n);
// for the Toeplitz-Gramian problem (gx != nullptr, T = L): r = y - L^H L x - G x.
__global__ void k_normal_residual(const SolveDesc* __restrict__ sd, const double2* __restrict__ y,
                                  const double2* __restrict__ thtx, const double2* __restrict__ x,
                                  double2* __restrict__ r, int64_t stride, const double2* __restrict__ gx,
                                  int64_t gx_stride) {
    const int64_t s = blockIdx.y;
    const SolveDesc d = sd[s];
    const double l2 = d.lam * d.lam;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.n; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 reg = gx ? gx[s * gx_stride + i] : cscale(x[s * stride + i], l2);
        r[s * stride + i] = csub(csub(y[s * stride + i], thtx[s * stride + i]), reg);
    }
}

// Interpolation data of the l2 problem (eq. (ex6) transformed as in eq. (ex4),
// conditions (intcond)), two conditions per node nu, written in tree order.
// Unknown p* = [x; sigma1; gamma1; gamma2; 1] with degree bounds n, m, m+k-1, n+k-1, 1.
//   F_nu = [lam^2 w^{(m+k-1)nu},  w^{(k-1)nu} conj(c^),  1,  0,  -w^{(m+k-1)nu} y^]
//   G_nu = [-c^,  w^{(n+k-1)nu},  0,  1,  0]
// The nr right-hand sides of a group give columns 4 .. 3+nr (one y^ each).
// Tree order: leaf t (in-order) holds nodes nu = o_t + c + j*2^{p+1}, o_t = 2*bitrev_p(t),
// c in {0,1}, j < M/2 (paired interleaving, Sec. 6.1); slot h = c*M + 2j + type.
// Toeplitz-Gramian problem (eq. (ex7), sizes n, p, N-n, N-p, 1; T = L): the first
// entry of F_nu is the symbol of the extended Gramian, cg(nu), in place of lam^2 w^{(N-n) nu}.
__global__ void k_assemble(const SolveDesc* __restrict__ sd, int nr, const double2* __restrict__ chat,
                           const double2* __restrict__ yhat, int64_t vstride, double2* __restrict__ phi,
                           int64_t phi_stride, int64_t N, int64_t M, int p, int K,
                           const double2* __restrict__ tw, int64_t Q, const double2* __restrict__ cg) {
    const int64_t g = blockIdx.y;
    const SolveDesc d = sd[g * nr];
    const int64_t twN = Q / N;
    const double l2 = d.lam * d.lam;
    const int64_t nq = 2 * N;
    double2* ph = phi + g * phi_stride;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += (int64_t)gridDim.x * blockDim.x) {
        int64_t t = q / K, h = q - t * K;
        int64_t c = h / M, rem = h - c * M;
        int64_t j = rem >> 1;
        int type = (int)(rem & 1);
        int64_t nu = 2 * (int64_t)bitrev((int)t, p) + c + (j << (p + 1));
        double2 ch = chat[g * vstride + nu];
        if (type == 0) {
            double2 wmk = twq(tw, Q, ((N - d.n) * nu % N) * twN, +1);        // w^{(m+k-1) nu}
            double2 wk1 = twq(tw, Q, ((((d.k - 1) % N + N) % N) * nu % N) * twN, +1);
            ph[0 * nq + q] = d.gramian ? cg[g * vstride + nu] : cscale(wmk, l2);
            ph[1 * nq + q] = cmul(wk1, cconj(ch));
            ph[2 * nq + q] = c2(1.0, 0.0);
            ph[3 * nq + q] = c2(0.0, 0.0);
            for (int r = 0; r < nr; ++r)
                ph[(4 + r) * nq + q] = cneg(cmul(wmk, yhat[(g * nr + r) * vstride + nu]));
        } else {
            double2 wnk = twq(tw, Q, ((N - d.m) * nu % N) * twN, +1);        // w^{(n+k-1) nu}
            ph[0 * nq + q] = cneg(ch);
            ph[1 * nq + q] = wnk;
            ph[2 * nq + q] = c2(0.0, 0.0);
            ph[3 * nq + q] = c2(1.0, 0.0);
            for (int r = 0; r < nr; ++r) ph[(4 + r) * nq + q] = c2(0.0, 0.0);
        }
    }
}

// Node of condition q (tree order).
__device__ __forceinline__ double2 cond_node(int64_t q, int64_t N, int64_t M, int p, int K,
                                             const double2* __restrict__ tw, int64_t Q) {
    int64_t t = q / K, h = q - t * K;
    int64_t c = h / M, j = (h - c * M) >> 1;
    int64_t nu = 2 * (int64_t)bitrev((int)t, p) + c + (j << (p + 1));
    return tw[nu * (Q / N)];
}

// ---------------------------------------------------------------- leaf: serial TanInt
// The fast-only construction of Sec. 4.3 on one leaf's K conditions: one
// workgroup per group with one wavefront per 64 conditions, residuals in
// registers (one condition per lane).  Each wave finds its best candidate
// with DPP reductions and leaves the key, residual row and node in LDS; after
// one barrier every wave takes the overall best and updates its own
// conditions (the LDS records alternate with the step parity, so a wave may
// write step s+1 while another still reads step s).  Each step
// processes one condition with the single-condition basis of eq. (spbasis):
//   pivot column pi = the lowest tau-degree among columns 1..4 whose residual
//   entry is not negligible (|r_i| > ZTOL max_j |r_j|), ties to the largest
//   |r_i|; the condition is the remaining one with the lowest such degree and,
//   among those, the largest |r_pi| (partial pivoting of the conditions,
//   Sec. 5).  The constant columns are never pivots, so the basis keeps the
//   block form [[B0, V], [0, I]] and every right-hand side of the group shares
//   the pivot sequence.
//   mu_i = -r_i / r_pi;  B_:i += mu_i B_:pi (i != pi);  B_:pi *= (z - sigma);
//   remaining residuals r_i += mu_i r_pi,  r_pi *= (sigma_q - sigma);  delta_pi += 1.
// The basis itself is formed afterwards from the step records (k_leaf_build).
// Deferred (difficult) conditions of each group, Sec. 5: condition index,
// node and residual row (C entries) with respect to the part of the basis
// built so far; count in SolveState.ndef.
struct DeferList {
    int32_t* q;            // [G][cap]
    double2* node;         // [G][cap]
    double2* res;          // [G][cap][C]
    int32_t cap;
    int32_t C;
};

struct LeafArgs {
    const SolveDesc* sd;
    SolveState* st;
    double2* phi;
    int64_t phi_stride;
    LeafRec* rec;
    int64_t rec_stride;
    int64_t N, M;
    int p, K, leaf;
    const double2* tw;
    int64_t Q;
    // difficult points: a chosen condition whose pivot entry satisfies
    // |r_pi|^2 < defer_tol2 max_{j<4} |r_j|^2 is deferred (0 disables)
    double defer_tol2;
    DeferList dl;
};

#define TIKH_ZTOL2 1e-18   // (1e-9)^2: relative size below which a residual entry counts as zero

// ---- cross-lane helpers (DPP, wave64)
template <int CTRL, int RM = 0xF>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long old, unsigned long long v) {
    int lo = __builtin_amdgcn_update_dpp((int)(unsigned)old, (int)(unsigned)v, CTRL, RM, 0xF, false);
    int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(old >> 32), (int)(unsigned)(v >> 32), CTRL, RM, 0xF, false);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
// maximum over the 64 lanes, returned uniformly
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
    unsigned long long t;
    t = dpp_u64<0xB1>(v, v); v = v > t ? v : t;          // quad_perm [1,0,3,2]
    t = dpp_u64<0x4E>(v, v); v = v > t ? v : t;          // quad_perm [2,3,0,1]
    t = dpp_u64<0x141>(v, v); v = v > t ? v : t;         // row_half_mirror
    t = dpp_u64<0x140>(v, v); v = v > t ? v : t;         // row_mirror: every lane holds its row maximum
    t = dpp_u64<0x142, 0xA>(v, v); v = v > t ? v : t;    // row_bcast:15 into rows 1, 3
    t = dpp_u64<0x143, 0xC>(v, v); v = v > t ? v : t;    // row_bcast:31 into rows 2, 3: lane 63 holds the maximum
    unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
    unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}
// lane i receives lane i-1 (lane 0 receives 0)
__device__ __forceinline__ double wave_shr1_d(double v) {
    int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Candidate key, compared as an unsigned integer: lowest tau-degree first
// (20 bits, delta offset by 2^19), then the largest |r_pi|^2 (top 34 bits of the
// non-negative double), then the pivot column (2 bits) and the lowest
// slot/lane index (8 bits).  0 = no candidate.
__device__ __forceinline__ unsigned long long cand_key(int delta, double a2, int piv, int idx) {
    unsigned long long kd = (unsigned long long)((1 << 19) - delta) & 0xFFFFFull;
    unsigned long long km = ((unsigned long long)__double_as_longlong(a2) >> 29) & 0x3FFFFFFFFull;
    return (kd << 44) | (km << 10) | ((unsigned long long)piv << 8) | (unsigned long long)(255 - idx);
}

template <int NR>
__global__ __launch_bounds__(256) void k_leaf_loop(const LeafArgs a) {
    constexpr int C = 4 + NR;
    // per step parity and wave: the wave's best candidate key and its residual row and node
    __shared__ unsigned long long skey[2][4];
    __shared__ double2 srow[2][4][C + 1];
    const int64_t g = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int W = blockDim.x >> 6;
    const int K = a.K;
    const int h = wv * 64 + lane;                    // condition of this lane within the leaf
    const int64_t nq = 2 * a.N;
    const int64_t q0 = (int64_t)a.leaf * K;
    double2* ph = a.phi + g * a.phi_stride;
    LeafRec* rec = a.rec + g * a.rec_stride;
    double2 r[C];
    double2 sg = c2(0.0, 0.0);
    bool alive = h < K;
    bool passive = false;                            // deferred: updated, never chosen
#pragma unroll
    for (int c = 0; c < C; ++c) r[c] = alive ? ph[c * nq + q0 + h] : c2(0.0, 0.0);
    if (alive) sg = cond_node(q0 + h, a.N, a.M, a.p, K, a.tw, a.Q);
    int dl[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) dl[c] = a.st[g].delta[c];
    // keys of absent waves stay 0
    if (threadIdx.x < 8 && (int)(threadIdx.x & 3) >= W) skey[threadIdx.x >> 2][threadIdx.x & 3] = 0ull;
    __syncthreads();
    int info = 0;
    for (int step = 0; step < K; ++step) {
        const int par = step & 1;
        unsigned long long key = 0ull;
        {
            // every lane scores its row (absent and chosen rows are zero or finite); only
            // active conditions enter the reduction
            double a2[4];
            double amax = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) { a2[c] = cabs2(r[c]); amax = fmax(amax, a2[c]); }
            const double thr = TIKH_ZTOL2 * amax;
            int kd = INT_MAX, piv = -1;
            double pm = -1.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (a2[c] > thr && a2[c] > 0.0 && (dl[c] < kd || (dl[c] == kd && a2[c] > pm))) {
                    kd = dl[c]; piv = c; pm = a2[c];
                }
            }
            key = (alive && piv >= 0) ? cand_key(kd, pm, piv, h) : 0ull;
        }
        const unsigned long long wk = wave_max_u64(key);
        if (wk != 0ull && h == 255 - (int)(wk & 255ull)) {
#pragma unroll
            for (int c = 0; c < C; ++c) srow[par][wv][c] = r[c];
            srow[par][wv][C] = sg;
        }
        if (lane == 0) skey[par][wv] = wk;
        __syncthreads();
        unsigned long long best = 0ull;
#pragma unroll
        for (int w = 0; w < 4; ++w) { const unsigned long long t = skey[par][w]; best = t > best ? t : best; }
        if (best == 0ull) { info = 1; break; }      // no admissible pivot: breakdown
        const int idx = 255 - (int)(best & 255ull);
        const int piv = (int)((best >> 8) & 3ull);
        const int ww = idx >> 6;
        double2 rc[C];
#pragma unroll
        for (int c = 0; c < C; ++c) rc[c] = srow[par][ww][c];
        const double2 sc = srow[par][ww][C];
        double2 rp = rc[0];
#pragma unroll
        for (int c = 1; c < 4; ++c) if (c == piv) rp = rc[c];
        if (a.defer_tol2 > 0.0) {
            double amax = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) amax = fmax(amax, cabs2(rc[c]));
            if (cabs2(rp) < a.defer_tol2 * amax) {
                // difficult point: set aside for the end of the solve; no step is taken
                if (h == idx) { alive = false; passive = true; }
                if (threadIdx.x == 0) rec[step].piv = -1;
                continue;
            }
        }
        if (h == idx) alive = false;
        // -1 / r_pi
        const double den = 1.0 / cabs2(rp);
        const double2 inv = c2(-rp.x * den, rp.y * den);
        double2 mu[C];
#pragma unroll
        for (int c = 0; c < C; ++c) mu[c] = (c == piv) ? c2(0.0, 0.0) : cmul(rc[c], inv);
        if (threadIdx.x == 0) {
            LeafRec& o = rec[step];
#pragma unroll
            for (int c = 0; c < C; ++c) o.mu[c] = mu[c];
            o.sig = sc;
            o.piv = piv;
            o.q = (int)(q0 + idx);
        }
        {
            // every lane is updated: rows of absent and chosen conditions are never read
            double2 rpv;
            switch (piv) {
                case 0: rpv = r[0]; break;
                case 1: rpv = r[1]; break;
                case 2: rpv = r[2]; break;
                default: rpv = r[3]; break;
            }
            // mu[piv] = 0 leaves the pivot column unchanged here
#pragma unroll
            for (int c = 0; c < C; ++c) r[c] = cfma(mu[c], rpv, r[c]);
            const double2 np = cmul(rpv, csub(sg, sc));
            switch (piv) {
                case 0: r[0] = np; break;
                case 1: r[1] = np; break;
                case 2: r[2] = np; break;
                default: r[3] = np; break;
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) if (c == piv) dl[c] += 1;
    }
    if (a.defer_tol2 > 0.0) {
        // append the deferred conditions of this leaf with their current residual rows
        __shared__ int sh_nd;
        if (threadIdx.x == 0) sh_nd = 0;
        __syncthreads();
        const int nd0 = a.st[g].ndef;
        if (passive) {
            const int pos = nd0 + atomicAdd(&sh_nd, 1);
            if (pos < a.dl.cap) {
                const int64_t e = g * a.dl.cap + pos;
                a.dl.q[e] = (int32_t)(q0 + h);
                a.dl.node[e] = sg;
#pragma unroll
                for (int c = 0; c < C; ++c) a.dl.res[e * C + c] = r[c];
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const int nd = nd0 + sh_nd;
            a.st[g].ndef = min(nd, a.dl.cap);
            if (nd > a.dl.cap) info |= 4;
        }
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) a.st[g].delta[c] = dl[c];
        if (info) a.st[g].info |= info;
    }
}

// Position of the k-th set bit (k = 0, 1, ...) of m; k < popcount(m).
__device__ __forceinline__ int nth_set_bit(unsigned long long m, int k) {
    unsigned w = (unsigned)m;
    int pos = 0;
    int c = __popc(w);
    if (k >= c) { k -= c; pos = 32; w = (unsigned)(m >> 32); }
    c = __popc(w & 0xFFFFu); if (k >= c) { k -= c; pos += 16; w >>= 16; }
    c = __popc(w & 0xFFu);   if (k >= c) { k -= c; pos += 8;  w >>= 8; }
    c = __popc(w & 0xFu);    if (k >= c) { k -= c; pos += 4;  w >>= 4; }
    c = __popc(w & 0x3u);    if (k >= c) { k -= c; pos += 2;  w >>= 2; }
    if (k >= (int)(w & 1u)) pos += 1;
    return pos;
}
__device__ __forceinline__ double bperm_d(int addr, double v) {
    const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Single-wavefront variant for large batches: one wave per group holds up to R
// conditions per lane (slots), so the per-step work that is the same for every
// condition (candidate reduction, division, multipliers) is done once per group
// rather than once per wave.  A chosen condition leaves a hole; whenever the
// conditions still held fit in fewer slots they are packed to the front in
// (slot, lane) order by lane permutes, so that the per-condition work of a step
// covers ceil(held / 64) slots rather than R.  Each condition keeps its index
// within the leaf, which breaks ties between candidates as above.
template <int R, int NR>
__global__ __launch_bounds__(64) void k_leaf_loop_sw(const LeafArgs a) {
    constexpr int C = 4 + NR;
    constexpr int PASSIVE = 0x100;           // deferred: updated, never chosen
    const int64_t g = blockIdx.x;
    const int lane = threadIdx.x;
    const int K = a.K;
    const int64_t nq = 2 * a.N;
    const int64_t q0 = (int64_t)a.leaf * K;
    double2* ph = a.phi + g * a.phi_stride;
    LeafRec* rec = a.rec + g * a.rec_stride;
    double2 r[R][C];
    double2 sg[R];
    int hid[R];                              // condition index within the leaf (| PASSIVE); -1 = empty
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int h = lane + 64 * i;
        const bool in = h < K;
        hid[i] = in ? h : -1;
#pragma unroll
        for (int c = 0; c < C; ++c) r[i][c] = in ? ph[c * nq + q0 + h] : c2(0.0, 0.0);
        sg[i] = in ? cond_node(q0 + h, a.N, a.M, a.p, K, a.tw, a.Q) : c2(0.0, 0.0);
    }
    int held = K;                            // conditions held (chosen ones leave)
    int ns = (K + 63) / 64;                  // slots in use
    int dl[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) dl[c] = a.st[g].delta[c];
    int info = 0;
    for (int step = 0; step < K; ++step) {
        unsigned long long best = 0ull;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            if (i >= ns) break;
            // every lane scores its slot (empty and chosen rows are zero or finite); only
            // held, active conditions enter the reduction
            const bool act = hid[i] >= 0 && !(hid[i] & PASSIVE);
            double a2[4];
            double amax = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) { a2[c] = cabs2(r[i][c]); amax = fmax(amax, a2[c]); }
            const double thr = TIKH_ZTOL2 * amax;
            int kd = INT_MAX, piv = -1;
            double pm = -1.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (a2[c] > thr && a2[c] > 0.0 && (dl[c] < kd || (dl[c] == kd && a2[c] > pm))) {
                    kd = dl[c]; piv = c; pm = a2[c];
                }
            }
            const unsigned long long k = (act && piv >= 0) ? cand_key(kd, pm, piv, hid[i] & 0xFF) : 0ull;
            best = k > best ? k : best;
        }
        const unsigned long long wk = wave_max_u64(best);
        if (wk == 0ull) { info = 1; break; }      // no admissible pivot: breakdown
        const int idx = 255 - (int)(wk & 255ull);
        const int piv = (int)((wk >> 8) & 3ull);
        // slot and lane holding the chosen condition
        int si = 0, wl = 0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            if (i >= ns) break;
            const unsigned long long m = __ballot(hid[i] == idx);
            if (m) { si = i; wl = (int)__builtin_ctzll(m); }
        }
        double2 rc[C];
        double2 sc = c2(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < R; ++i) {
            if (i == si) {
#pragma unroll
                for (int c = 0; c < C; ++c) rc[c] = c2(readlane_d(r[i][c].x, wl), readlane_d(r[i][c].y, wl));
                sc = c2(readlane_d(sg[i].x, wl), readlane_d(sg[i].y, wl));
            }
        }
        double2 rp = rc[0];
#pragma unroll
        for (int c = 1; c < 4; ++c) if (c == piv) rp = rc[c];
        if (a.defer_tol2 > 0.0) {
            double amax = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) amax = fmax(amax, cabs2(rc[c]));
            if (cabs2(rp) < a.defer_tol2 * amax) {
                // difficult point: set aside for the end of the solve; no step is taken
#pragma unroll
                for (int i = 0; i < R; ++i)
                    if (i == si && lane == wl) hid[i] |= PASSIVE;
                if (lane == 0) rec[step].piv = -1;
                continue;
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i) if (i == si && lane == wl) hid[i] = -1;
        held -= 1;
        // -1 / r_pi
        const double den = 1.0 / cabs2(rp);
        const double2 inv = c2(-rp.x * den, rp.y * den);
        double2 mu[C];
#pragma unroll
        for (int c = 0; c < C; ++c) mu[c] = (c == piv) ? c2(0.0, 0.0) : cmul(rc[c], inv);
        if (lane == 0) {
            LeafRec& o = rec[step];
#pragma unroll
            for (int c = 0; c < C; ++c) o.mu[c] = mu[c];
            o.sig = sc;
            o.piv = piv;
            o.q = (int)(q0 + idx);
        }
#pragma unroll
        for (int i = 0; i < R; ++i) {
            if (i >= ns) break;
            // empty lanes are updated too: their rows stay finite and are never read
            double2 rpv;
            switch (piv) {
                case 0: rpv = r[i][0]; break;
                case 1: rpv = r[i][1]; break;
                case 2: rpv = r[i][2]; break;
                default: rpv = r[i][3]; break;
            }
            // mu[piv] = 0 leaves the pivot column unchanged here
#pragma unroll
            for (int c = 0; c < C; ++c) r[i][c] = cfma(mu[c], rpv, r[i][c]);
            const double2 np = cmul(rpv, csub(sg[i], sc));
            switch (piv) {
                case 0: r[i][0] = np; break;
                case 1: r[i][1] = np; break;
                case 2: r[i][2] = np; break;
                default: r[i][3] = np; break;
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) if (c == piv) dl[c] += 1;
        const int nsn = (held + 63) / 64;
        if (nsn < ns) {
            // pack: destination position p = 64 j + lane takes the p-th held condition in
            // (slot, lane) order, which sits at a position >= p, so slot j is rewritten only
            // after every read of it
            unsigned long long m[R];
            int pre[R + 1];
            pre[0] = 0;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                m[i] = i < ns ? __ballot(hid[i] >= 0) : 0ull;
                pre[i + 1] = pre[i] + __popcll(m[i]);
            }
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if (j >= nsn) break;
                const int p = 64 * j + lane;
                int ssl = j;
#pragma unroll
                for (int i = j + 1; i < R; ++i) if (i < ns && p >= pre[i]) ssl = i;
                unsigned long long ms = m[j];
#pragma unroll
                for (int i = j + 1; i < R; ++i) if (ssl == i) ms = m[i];
                const bool valid = p < held;
                const int addr = valid ? 4 * nth_set_bit(ms, p - pre[ssl]) : 4 * lane;
                double2 tr[C];
                double2 ts = c2(0.0, 0.0);
                int th = -1;
#pragma unroll
                for (int c = 0; c < C; ++c) tr[c] = c2(0.0, 0.0);
#pragma unroll
                for (int i = j; i < R; ++i) {
                    if (i >= ns) break;
                    const bool take = valid && ssl == i;
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        const double x = bperm_d(addr, r[i][c].x), y = bperm_d(addr, r[i][c].y);
                        if (take) tr[c] = c2(x, y);
                    }
                    const double x = bperm_d(addr, sg[i].x), y = bperm_d(addr, sg[i].y);
                    const int hh = __builtin_amdgcn_ds_bpermute(addr, hid[i]);
                    if (take) { ts = c2(x, y); th = hh; }
                }
#pragma unroll
                for (int c = 0; c < C; ++c) r[j][c] = tr[c];
                sg[j] = ts;
                hid[j] = th;
            }
#pragma unroll
            for (int j = 0; j < R; ++j) if (j >= nsn) hid[j] = -1;
            ns = nsn;
        }
    }
    if (a.defer_tol2 > 0.0) {
        // append the deferred conditions of this leaf with their current residual rows
        __shared__ int sh_nd;
        if (lane == 0) sh_nd = 0;
        __syncthreads();
        const int nd0 = a.st[g].ndef;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            if (hid[i] >= 0 && (hid[i] & PASSIVE)) {
                const int pos = nd0 + atomicAdd(&sh_nd, 1);
                if (pos < a.dl.cap) {
                    const int64_t e = g * a.dl.cap + pos;
                    a.dl.q[e] = (int32_t)(q0 + (hid[i] & 0xFF));
                    a.dl.node[e] = sg[i];
#pragma unroll
                    for (int c = 0; c < C; ++c) a.dl.res[e * C + c] = r[i][c];
                }
            }
        }
        __syncthreads();
        if (lane == 0) {
            const int nd = nd0 + sh_nd;
            a.st[g].ndef = min(nd, a.dl.cap);
            if (nd > a.dl.cap) info |= 4;
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) a.st[g].delta[c] = dl[c];
        if (info) a.st[g].info |= info;
    }
}

// Basis of one leaf from its step records: B = E_1 E_2 ... E_K with the
// elementary factors of eq. (spbasis).  One wavefront per row of [B0 | V]
// (4 waves), coefficient k of each polynomial on lane k%64, slot k/64; the
// records are staged in LDS, the shift by z is a DPP lane shift.
struct BuildArgs {
    const SolveState* st;
    const LeafRec* rec;
    int64_t rec_stride;
    double2* out;          // slot data [g][4C][cap+1]
    int64_t out_stride;
    int64_t cap;
    SlotMeta* meta;        // [g]
    int K;
    // narrow pass (one slot of 64 coefficients): a group whose basis needs more is only
    // flagged; the wide pass then builds the flagged groups alone
    int narrow, wide_pass;
};

template <int S>
__device__ __forceinline__ void pick_slots(double2 (&dst)[S], const double2 (&src)[S]) {
#pragma unroll
    for (int sl = 0; sl < S; ++sl) dst[sl] = src[sl];
}

template <int S, int NR>
__global__ __launch_bounds__(256) void k_leaf_build(const BuildArgs a) {
    constexpr int C = 4 + NR;
    const int64_t g = blockIdx.x;
    const int row = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    if (a.wide_pass && a.st[g].wide == 0) return;    // built by the narrow pass
    extern __shared__ double2 lds_dyn[];             // K records
    LeafRec* lrec = (LeafRec*)lds_dyn;
    {
        const double2* src = (const double2*)(a.rec + g * a.rec_stride);
        double2* dstp = lds_dyn;
        const int nv = a.K * (int)(sizeof(LeafRec) / sizeof(double2));
        for (int i = threadIdx.x; i < nv; i += 256) dstp[i] = src[i];
    }
    __syncthreads();
    if (a.narrow) {
        // every column degree is at most the largest number of steps pivoting on one column
        __shared__ int npiv[4];
        if (threadIdx.x < 4) npiv[threadIdx.x] = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < a.K; i += 256) {
            const int pv = lrec[i].piv;
            if (pv >= 0) atomicAdd(&npiv[pv], 1);
        }
        __syncthreads();
        const bool wide = max(max(npiv[0], npiv[1]), max(npiv[2], npiv[3])) > 64 * S - 1;
        __syncthreads();
        if (threadIdx.x == 0) ((SolveState*)a.st)[g].wide = wide ? 1 : 0;
        if (wide) return;
    }
    double2 P[C][S];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int sl = 0; sl < S; ++sl) P[c][sl] = c2((c == row && sl == 0 && lane == 0) ? 1.0 : 0.0, 0.0);
    int deg[C];
#pragma unroll
    for (int c = 0; c < C; ++c) deg[c] = c < 4 ? 0 : -1;
    const bool broken = a.st[g].info != 0;
    for (int step = 0; step < a.K && !broken; ++step) {
        const LeafRec& rr = lrec[step];
        const int piv = rr.piv;
        if (piv < 0) continue;
        double2 mu[C];                               // mu[piv] = 0
#pragma unroll
        for (int c = 0; c < C; ++c) mu[c] = rr.mu[c];
        const double2 sg = rr.sig;
        int dp = deg[0];
#pragma unroll
        for (int c = 1; c < 4; ++c) if (c == piv) dp = deg[c];
        // the pivot column (its coefficients beyond slot dp >> 6 are zero)
        double2 pv[S];
        switch (piv) {
            case 0: pick_slots<S>(pv, P[0]); break;
            case 1: pick_slots<S>(pv, P[1]); break;
            case 2: pick_slots<S>(pv, P[2]); break;
            default: pick_slots<S>(pv, P[3]); break;
        }
        const int act = dp >> 6, act2 = (dp + 1) >> 6;
        // B_:c += mu_c B_:pi for every column (unchanged for c = pi)
#pragma unroll
        for (int sl = 0; sl < S; ++sl) {
            if (sl <= act) {
#pragma unroll
                for (int c = 0; c < C; ++c) P[c][sl] = cfma(mu[c], pv[sl], P[c][sl]);
            }
        }
        // B_:pi *= (z - sigma): coefficient k becomes B[k-1] - sigma B[k]; the shift by
        // one coefficient is a lane shift, with lane 63 of the previous slot entering lane 0
        double2 nv[S];
#pragma unroll
        for (int sl = 0; sl < S; ++sl) {
            if (sl <= act2) {
                double ux = wave_shr1_d(pv[sl].x), uy = wave_shr1_d(pv[sl].y);
                if (sl > 0 && lane == 0) {
                    ux = readlane_d(pv[sl - 1].x, 63);
                    uy = readlane_d(pv[sl - 1].y, 63);
                }
                nv[sl] = csub(c2(ux, uy), cmul(sg, pv[sl]));
            } else {
                nv[sl] = c2(0.0, 0.0);
            }
        }
        switch (piv) {
            case 0: pick_slots<S>(P[0], nv); break;
            case 1: pick_slots<S>(P[1], nv); break;
            case 2: pick_slots<S>(P[2], nv); break;
            default: pick_slots<S>(P[3], nv); break;
        }
#pragma unroll
        for (int c = 0; c < C; ++c)
            if (cnonzero(mu[c])) deg[c] = max(deg[c], dp);
#pragma unroll
        for (int c = 0; c < 4; ++c) if (c == piv) deg[c] = dp + 1;
    }
    // column maxima of B0 over the 4 rows
    __shared__ double cm[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double mx = 0.0;
#pragma unroll
        for (int sl = 0; sl < S; ++sl) mx = fmax(mx, cabs2(P[c][sl]));
        mx = wave_max_d(mx);
        if (lane == 0) cm[row][c] = mx;
    }
    __syncthreads();
    double2* out = a.out + g * a.out_stride;
    const int64_t cp1 = a.cap + 1;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        double2* dst = out + (int64_t)(row * C + c) * cp1;
#pragma unroll
        for (int sl = 0; sl < S; ++sl) {
            int64_t k = lane + 64 * sl;
            if (k <= deg[c] && k < cp1) dst[k] = P[c][sl];
        }
    }
    if (threadIdx.x == 0) {
        SlotMeta m;
        int bad = 0;
        for (int c = 0; c < MAXC; ++c) m.deg[c] = -1;
        for (int c = 0; c < C; ++c) {
            if (deg[c] > a.cap) bad = 1;
            m.deg[c] = (int)min((int64_t)deg[c], a.cap);   // never read past the slot
        }
        for (int c = 0; c < 4; ++c) {
            double mx = fmax(fmax(cm[0][c], cm[1][c]), fmax(cm[2][c], cm[3][c]));
            m.colmax_bits[c] = (unsigned long long)__double_as_longlong(sqrt(mx));
        }
        a.meta[g] = m;
        if (bad) atomicOr(&((SolveState*)a.st)[g].info, 2);
    }
}

// ---------------------------------------------------------------- evaluation, Alg. 1 step 2
// The completed left child is evaluated at the nodes of its right sibling by
// the batched FFT: its first pass reads each basis entry twisted by the coset
// offset and folded modulo the coset length (FftArgs load mode 2).

// phi <- phi B_L(sigma) for every condition of the right subtree
// (Alg. 1 step 2, with Thm. 1 giving the data phi_k B_kappa(sigma_k)).
// The right subtree (depth d, coset offset oR) spans leaves [t0, t0 + 2^{p-d}); each coset
// holds L = 2^{p-d} M/2 of its nodes, node jn = jlo + 2^{p-d} jhi being node jhi of the
// leaf whose offset is oR + 2^{d+1} jlo.  V holds each line in four-step order: value jn
// at position (jn % L1) * L2 + jn / L1 (L2 = L / L1; natural order when L1 = L).
// Threads run over the positions of V, so that the 4C evaluation lines (four fifths of
// the data read) are read in order; the residual rows they update are then scattered
// (two adjacent conditions, F and G, per node).
template <int NR>
__global__ __launch_bounds__(256) void k_eval_apply(double2* __restrict__ phi, int64_t phi_stride,
                                                    const double2* __restrict__ V, int64_t v_stride, int64_t L,
                                                    int64_t L1, int64_t oR, int d, int64_t t0, int64_t nleaves,
                                                    int64_t N, int64_t M, int p, int K) {
    constexpr int C = 4 + NR;
    const int64_t g = blockIdx.y;
    const int64_t nq = 2 * N;
    // one thread per node: its F and G conditions (adjacent in tree order) share B_L(sigma)
    const int iL = (int)L, nodes = 2 * iL, hm = (int)(M / 2);
    const int L2 = (int)(L / L1), iL1 = (int)L1, sh = p - d;
    const float inv_L2 = 1.0f / (float)L2;
    double2* ph = phi + g * phi_stride;
    const double2* Vs = V + g * v_stride;
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < nodes; u += gridDim.x * blockDim.x) {
        const int c = u >= iL ? 1 : 0;                                  // coset
        const int64_t j = u - c * iL;                                   // position in the line
        const int j1 = fdiv((int)j, inv_L2, L2), j2 = (int)j - j1 * L2;
        const int jn = j1 + iL1 * j2;                                   // node index within the coset
        const int jlo = jn & (int)(nleaves - 1), jhi = jn >> sh;
        const int64_t t = bitrev((int)((oR + ((int64_t)jlo << (d + 1))) >> 1), p);
        if (t < t0 || t >= t0 + nleaves || jhi >= hm) continue;        // (not reached: jn < L)
        const int hn = c * hm + jhi;                                    // node within the leaf
        const int64_t q = t * K + 2 * (int64_t)hn;                     // its F condition; q + 1 is G
        double2 f0[C], f1[C];
#pragma unroll
        for (int col = 0; col < C; ++col) { f0[col] = ph[col * nq + q]; f1[col] = ph[col * nq + q + 1]; }
        double2 o0[C], o1[C];
#pragma unroll
        for (int col = 0; col < C; ++col) {
            o0[col] = col < 4 ? c2(0.0, 0.0) : f0[col];
            o1[col] = col < 4 ? c2(0.0, 0.0) : f1[col];
        }
#pragma unroll
        for (int row = 0; row < 4; ++row) {
#pragma unroll
            for (int col = 0; col < C; ++col) {
                const double2 E = Vs[(int64_t)((row * C + col) * 2 + c) * L + j];
                o0[col] = cfma(f0[row], E, o0[col]);
                o1[col] = cfma(f1[row], E, o1[col]);
            }
        }
#pragma unroll
        for (int col = 0; col < C; ++col) { ph[col * nq + q] = o0[col]; ph[col * nq + q + 1] = o1[col]; }
    }
}

// Direct evaluation of a completed left child at the nodes of its right
// sibling subtree (small subtrees), updating the residual rows in place:
// phi_c <- sum_row phi_row B[row][c](z) (+ phi_c for the constant columns).
// One workgroup per group.  The column-scaled coefficients and the subtree's
// residual rows are staged in LDS; each thread evaluates one (node, column)
// item as four independent Horner chains (rows 0..3).  Groups whose degrees
// exceed the LDS budget evaluate from global memory, one node per thread.
// Two passes: the narrow pass (MODE 1, a smaller LDS budget, so more workgroups
// per CU) handles the groups that fit it and flags the others (SolveState::wide);
// the wide pass (MODE 2) handles only the flagged groups, with the larger budget
// and the global-memory path.  MODE 0 handles every group in one pass.
constexpr int ED_LDS = 4608;       // complex elements of LDS staging (wide pass)
constexpr int ED_LDS_NARROW = 2496;

template <int NR, int LDSN, int MODE>
__global__ __launch_bounds__(256) void k_eval_direct(double2* __restrict__ phi, int64_t phi_stride,
                                                     const double2* __restrict__ B, int64_t b_stride, int64_t cp1,
                                                     const SlotMeta* __restrict__ meta, int64_t t0, int64_t nleaves,
                                                     int64_t N, int64_t M, int p, int K,
                                                     const double2* __restrict__ tw, int64_t Q,
                                                     SolveState* __restrict__ st) {
    constexpr int C = 4 + NR;
    __shared__ double2 sh[LDSN];
    __shared__ int sdeg[C];
    __shared__ double ssc[C];
    const int64_t g = blockIdx.x;
    if (MODE == 2 && st[g].wide == 0) return;
    if (threadIdx.x < C) {
        const SlotMeta& mt = meta[g];
        sdeg[threadIdx.x] = mt.deg[threadIdx.x];
        ssc[threadIdx.x] = threadIdx.x < 4 ? pow2_inv_scale(mt.colmax_bits[threadIdx.x]) : 1.0;
    }
    __syncthreads();
    const double2* Bs = B + g * b_stride;
    double2* ph = phi + g * phi_stride;
    const int64_t nq = 2 * N;
    const int nodes = (int)(nleaves * K / 2);
    const int64_t qb = t0 * K;                       // first condition of the subtree
    int dmax = -1;
#pragma unroll
    for (int c = 0; c < C; ++c) dmax = max(dmax, sdeg[c]);
    const int bs = dmax + 1;                         // coefficient stride of an entry in LDS
    const bool staged = 4 * C * max(bs, 0) + 2 * C * nodes <= LDSN;
    if (MODE == 1) {
        if (threadIdx.x == 0) st[g].wide = staged ? 0 : 1;
        if (!staged) return;
    }
    if (staged) {
        double2* shB = sh;                           // [4C][bs], entry row*C + col
        double2* shF = sh + 4 * C * bs;              // [C][2*nodes] residual rows of the subtree
        for (int w = threadIdx.x; w < 4 * C * bs; w += blockDim.x) {
            const int e = w / bs, t = w - e * bs;
            const int col = e % C;
            shB[w] = t <= sdeg[col] ? cscale(Bs[(int64_t)e * cp1 + t], ssc[col]) : c2(0.0, 0.0);
        }
        for (int w = threadIdx.x; w < 2 * C * nodes; w += blockDim.x) {
            const int c = w / (2 * nodes), h = w - c * 2 * nodes;
            shF[w] = ph[c * nq + qb + h];
        }
        __syncthreads();
        for (int w = threadIdx.x; w < C * nodes; w += blockDim.x) {
            const int u = w / C, col = w - u * C;
            const int64_t q = qb + 2 * u;            // the F condition; q + 1 is the G condition of the same node
            const double2 z = cond_node(q, N, M, p, K, tw, Q);
            const int dg = sdeg[col];
            double2 acc[4] = {c2(0.0, 0.0), c2(0.0, 0.0), c2(0.0, 0.0), c2(0.0, 0.0)};
            for (int k = dg; k >= 0; --k) {
#pragma unroll
                for (int row = 0; row < 4; ++row) acc[row] = cfma(acc[row], z, shB[(row * C + col) * bs + k]);
            }
            double2 o0 = col < 4 ? c2(0.0, 0.0) : shF[col * 2 * nodes + 2 * u];
            double2 o1 = col < 4 ? c2(0.0, 0.0) : shF[col * 2 * nodes + 2 * u + 1];
#pragma unroll
            for (int row = 0; row < 4; ++row) {
                o0 = cfma(shF[row * 2 * nodes + 2 * u], acc[row], o0);
                o1 = cfma(shF[row * 2 * nodes + 2 * u + 1], acc[row], o1);
            }
            ph[col * nq + q] = o0;
            ph[col * nq + q + 1] = o1;
        }
        return;
    }
    if constexpr (MODE != 1) {
    for (int u = threadIdx.x; u < nodes; u += blockDim.x) {
        const int64_t q = qb + 2 * u;
        const double2 z = cond_node(q, N, M, p, K, tw, Q);
        double2 f0[C], f1[C], o0[C], o1[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            f0[c] = ph[c * nq + q]; f1[c] = ph[c * nq + q + 1];
            o0[c] = c < 4 ? c2(0.0, 0.0) : f0[c];
            o1[c] = c < 4 ? c2(0.0, 0.0) : f1[c];
        }
#pragma unroll
        for (int col = 0; col < C; ++col) {
            const int dg = sdeg[col];
#pragma unroll
            for (int row = 0; row < 4; ++row) {
                const double2* src = Bs + (int64_t)(row * C + col) * cp1;
                double2 acc = c2(0.0, 0.0);
                for (int k = dg; k >= 0; --k) acc = cfma(acc, z, src[k]);
                acc = cscale(acc, ssc[col]);
                o0[col] = cfma(f0[row], acc, o0[col]);
                o1[col] = cfma(f1[row], acc, o1[col]);
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) { ph[c * nq + q] = o0[c]; ph[c * nq + q + 1] = o1[c]; }
    }
    }
}

// Small subtrees: direct block product [[B0L, VL],[0,I]] [[B0R, VR],[0,I]]
// = [[B0L B0R, B0L VR + VL],[0,I]] by convolution of the coefficient
// sequences, one workgroup per group; writes the parent basis, its degrees
// and its column maxima.  The column-scaled B0L block and, one output column
// at a time, the zero-padded rows 0..3 of that column of the right factor are
// staged in LDS; each thread forms four consecutive output coefficients of
// one entry from a sliding window of right-factor coefficients.  Groups whose
// degrees exceed the LDS budget read the factors from global memory instead.
// Two passes as for the direct evaluation: the narrow pass takes the groups whose
// factors fit its budget with every column staged at once.
constexpr int PD_LDS = 4096;       // complex elements of LDS staging (wide pass)
constexpr int PD_LDS_NARROW = 2496;
constexpr int PD_PAD = 3;          // zero padding on each side of a right-factor entry

template <int LDSN, int MODE>
__global__ __launch_bounds__(256) void k_prod_direct(const double2* __restrict__ BL, int64_t l_stride, int64_t lcp1,
                                                     const SlotMeta* __restrict__ mL,
                                                     const double2* __restrict__ BR, int64_t r_stride, int64_t rcp1,
                                                     const SlotMeta* __restrict__ mR,
                                                     double2* __restrict__ out, int64_t o_stride, int64_t ocp1,
                                                     SlotMeta* __restrict__ mO, SolveState* __restrict__ st, int C) {
    __shared__ double2 sh[LDSN];
    __shared__ double red[4][4];
    __shared__ int sdl[MAXC], sdr[MAXC], sdout[MAXC];
    __shared__ double ssl[MAXC], ssr[MAXC];
    __shared__ int sbad;
    const int64_t g = blockIdx.x;
    if (MODE == 2 && st[g].wide == 0) return;
    if (threadIdx.x == 0) {
        const SlotMeta a = mL[g], b = mR[g];
        int dl = -1;
        for (int l = 0; l < 4; ++l) dl = max(dl, a.deg[l]);
        int bad = 0;
        for (int j = 0; j < MAXC; ++j) {
            ssl[j] = j < 4 ? pow2_inv_scale(a.colmax_bits[j]) : 1.0;
            ssr[j] = j < 4 ? pow2_inv_scale(b.colmax_bits[j]) : 1.0;
            sdl[j] = a.deg[j];
            sdr[j] = b.deg[j];
            int dj = -1;
            if (j < C) {
                dj = (b.deg[j] < 0 || dl < 0) ? -1 : dl + b.deg[j];
                if (j >= 4) dj = max(dj, a.deg[j]);
                if (dj >= ocp1) { bad = 1; dj = (int)ocp1 - 1; }
            }
            sdout[j] = dj;
        }
        sbad = bad;
    }
    __syncthreads();
    int dl = -1, drm = -1;
    for (int l = 0; l < 4; ++l) dl = max(dl, sdl[l]);
    for (int j = 0; j < C; ++j) drm = max(drm, sdr[j]);
    const double2* L = BL + g * l_stride;
    const double2* R = BR + g * r_stride;
    double2* O = out + g * o_stride;
    // LDS staging: the B0 block of the left factor [16][ls] (entry i*4 + l), then the
    // rows 0..3 of the right factor, zero-padded by PD_PAD on both sides: all columns
    // at once when they fit (every (column, row, block) item in one pass over the
    // threads), else one column at a time
    const int ls = dl + 1, rs = drm + 1 + 2 * PD_PAD;
    const bool staged = dl >= 0 && drm >= 0 && 16 * ls + 4 * rs <= LDSN;
    const bool all_cols = staged && 16 * ls + 4 * C * rs <= LDSN;
    if (MODE == 1) {
        if (threadIdx.x == 0) st[g].wide = all_cols ? 0 : 1;
        if (!all_cols) return;
    }
    double2* shL = sh;
    double2* shR = sh + 16 * max(ls, 0);
    if (staged) {
        for (int w = threadIdx.x; w < 16 * ls; w += blockDim.x) {
            const int e = w / ls, t = w - e * ls;
            const int i = e >> 2, l = e & 3;
            shL[w] = t <= sdl[l] ? cscale(L[(int64_t)(i * C + l) * lcp1 + t], ssl[l]) : c2(0.0, 0.0);
        }
    }
    double cmx[4] = {0.0, 0.0, 0.0, 0.0};
    // one item: four consecutive output coefficients k0..k0+3 of entry (i, j); rj = the
    // staged column j of the right factor (rows 0..3, stride rs)
    auto item = [&](int j, int i, int k0, const double2* rj) {
        const int doj = sdout[j];
        const int dr = sdr[j];
        double2 acc[4] = {c2(0.0, 0.0), c2(0.0, 0.0), c2(0.0, 0.0), c2(0.0, 0.0)};
        if (MODE == 1 || staged) {
            if (dr >= 0) {
                for (int l = 0; l < 4; ++l) {
                    const int dla = sdl[l];
                    if (dla < 0) continue;
                    const int t0 = max(0, k0 - dr), t1 = min(dla, k0 + 3);
                    if (t0 > t1) continue;
                    const double2* lp = shL + (i * 4 + l) * ls;
                    const double2* rp = rj + l * rs + PD_PAD + k0;   // rp[u - t] = R[k0 + u - t]
                    // window win[u] = R[k0 + u - t], starting at t = t1, t decreasing
                    double2 win[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) win[u] = rp[u - t1];
                    for (int t = t1; t >= t0; --t) {
                        const double2 lv = lp[t];
#pragma unroll
                        for (int u = 0; u < 4; ++u) acc[u] = cfma(lv, win[u], acc[u]);
                        if (t > t0) {
#pragma unroll
                            for (int u = 0; u < 3; ++u) win[u] = win[u + 1];
                            win[3] = rp[4 - t];
                        }
                    }
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = k0 + u;
                for (int l = 0; l < 4; ++l) {
                    const int dla = sdl[l];
                    if (dla < 0 || dr < 0) continue;
                    const int t0 = max(0, k - dr), t1 = min(k, dla);
                    const double2* lp = L + (int64_t)(i * C + l) * lcp1;
                    const double2* rp = R + (int64_t)(l * C + j) * rcp1;
                    double2 part = c2(0.0, 0.0);
                    for (int t = t0; t <= t1; ++t) part = cfma(lp[t], rp[k - t], part);
                    acc[u] = cfma(part, c2(ssl[l] * ssr[j], 0.0), acc[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u;
            if (k > doj) break;
            double2 v = acc[u];
            if (j >= 4 && k <= sdl[j]) v = cadd(v, L[(int64_t)(i * C + j) * lcp1 + k]);
            O[(int64_t)(i * C + j) * ocp1 + k] = v;
#pragma unroll
            for (int c = 0; c < 4; ++c) if (c == j) cmx[c] = fmax(cmx[c], cabs2(v));
        }
    };
    auto stage_col = [&](int j, double2* dst) {
        const int dr = sdr[j];
        for (int w = threadIdx.x; w < 4 * rs; w += blockDim.x) {
            const int l = w / rs, t = w - l * rs - PD_PAD;
            dst[w] = (t >= 0 && t <= dr) ? cscale(R[(int64_t)(l * C + j) * rcp1 + t], ssr[j]) : c2(0.0, 0.0);
        }
    };
    if (MODE == 1 || all_cols) {
        for (int j = 0; j < C; ++j) stage_col(j, shR + j * 4 * rs);
        __syncthreads();
        // items of all columns: column j has 4 * nblk_j items (nblk_j = blocks of 4 coefficients)
        int nit = 0;
        for (int j = 0; j < C; ++j) nit += sdout[j] < 0 ? 0 : 4 * ((sdout[j] + 4) / 4);
        for (int w = threadIdx.x; w < nit; w += blockDim.x) {
            int j = 0, rem = w;
            for (; j < C; ++j) {
                const int nj = sdout[j] < 0 ? 0 : 4 * ((sdout[j] + 4) / 4);
                if (rem < nj) break;
                rem -= nj;
            }
            item(j, rem & 3, (rem >> 2) * 4, shR + j * 4 * rs);
        }
    } else {
        for (int j = 0; j < C; ++j) {
            const int doj = sdout[j];
            if (doj < 0) continue;
            if (staged) {
                __syncthreads();                     // previous column's readers are done
                stage_col(j, shR);
                __syncthreads();
            }
            const int nblk = (doj + 4) / 4;
            for (int w = threadIdx.x; w < 4 * nblk; w += blockDim.x) item(j, w & 3, (w >> 2) * 4, shR);
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double mx = wave_max_d(cmx[c]);
        if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        SlotMeta m;
        for (int j = 0; j < MAXC; ++j) m.deg[j] = sdout[j];
        for (int c = 0; c < 4; ++c)
            m.colmax_bits[c] = (unsigned long long)__double_as_longlong(
                sqrt(fmax(fmax(red[c][0], red[c][1]), fmax(red[c][2], red[c][3]))));
        mO[g] = m;
        if (sbad) atomicOr(&st[g].info, 2);
    }
}

// ---------------------------------------------------------------- product, Alg. 1 step 4
// B = B_L B_R: the forward transforms read the zero-padded, column-scaled
// basis entries (FftArgs load mode 1), the pointwise block product runs per
// frequency, and the inverse transform writes the truncated, 1/P-scaled
// entries into the destination slot (store mode 1).

// Pointwise block product per frequency, B0_L times the rows 0..3 of B_R (the
// left factor's V block is added to the coefficients by the inverse
// transform's store).  Full mode: FL holds the 16 entries of B0_L (i*4 + t),
// FR all 4C entries of B_R (row-major, C columns); output all 4C entries
// (i*C + j) in place over FL.  Root mode 1: FL holds row 0 of B0_L (4 entries),
// FR the columns 4..C-1 of rows 0..3 (4 NR entries, row-major); output the NR
// solution polynomials.  Root mode 2: FL row 0 of B0_L, FR all 4C entries,
// output row 0 of every column.  Each thread reads all its inputs before it
// writes, so the outputs may overlay FL.
template <int NR>
__global__ __launch_bounds__(64) void k_prod_mul(const double2* FL, const double2* __restrict__ FR,
                           double2* FO, int64_t f_stride, int64_t P, int root) {
    constexpr int C = 4 + NR;
    const int64_t g = blockIdx.y;
    const double2* L = FL + g * f_stride;
    const double2* R = FR + g * f_stride;
    double2* O = FO + g * f_stride;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P; k += (int64_t)gridDim.x * blockDim.x) {
        if (root == 2) {
            double2 l[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) l[t] = L[t * P + k];
            double2 o[C];
#pragma unroll
            for (int j = 0; j < C; ++j) {
                double2 acc = c2(0.0, 0.0);
#pragma unroll
                for (int t = 0; t < 4; ++t) acc = cfma(l[t], R[(t * C + j) * P + k], acc);
                o[j] = acc;
            }
#pragma unroll
            for (int j = 0; j < C; ++j) O[j * P + k] = o[j];
        } else if (root) {
            double2 l[4], r[4][NR];
#pragma unroll
            for (int t = 0; t < 4; ++t) l[t] = L[t * P + k];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < NR; ++j) r[i][j] = R[(i * NR + j) * P + k];
#pragma unroll
            for (int j = 0; j < NR; ++j) {
                double2 acc = c2(0.0, 0.0);
#pragma unroll
                for (int t = 0; t < 4; ++t) acc = cfma(l[t], r[t][j], acc);
                O[j * P + k] = acc;
            }
        } else {
            double2 l[4][4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int t = 0; t < 4; ++t) l[i][t] = L[(i * 4 + t) * P + k];
            double2 r[4][C];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int j = 0; j < C; ++j) r[t][j] = R[(t * C + j) * P + k];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
#pragma unroll
                for (int j = 0; j < C; ++j) {
                    double2 acc = c2(0.0, 0.0);
#pragma unroll
                    for (int t = 0; t < 4; ++t) acc = cfma(l[i][t], r[t][j], acc);
                    O[(i * C + j) * P + k] = acc;
                }
            }
        }
    }
}

// Largest product degree + 1 over a chunk of groups (sizes the product
// transforms).  One workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_deg_need(const SlotMeta* __restrict__ mL, const SlotMeta* __restrict__ mR,
                                                  int ngroup, int C, int* __restrict__ need) {
    int v = 0;
    for (int s = threadIdx.x; s < ngroup; s += 256) {
        SlotMeta a = mL[s], b = mR[s];
        int dl = -1, dr = -1, dv = -1;
        for (int l = 0; l < 4; ++l) dl = max(dl, a.deg[l]);
        for (int j = 0; j < C; ++j) dr = max(dr, b.deg[j]);
        for (int j = 4; j < C; ++j) dv = max(dv, a.deg[j]);
        v = max(v, max(dl + dr, dv) + 1);
    }
    __shared__ int red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *need = red[0];
}

// Check of a recorded product length P against this chunk's degrees: raises *overflow
// if a product needs more than P coefficients (the length would wrap it around).
__global__ __launch_bounds__(256) void k_deg_check(const SlotMeta* __restrict__ mL, const SlotMeta* __restrict__ mR,
                                                   int ngroup, int C, int P, int* __restrict__ overflow) {
    bool bad = false;
    for (int s = threadIdx.x; s < ngroup; s += 256) {
        SlotMeta a = mL[s], b = mR[s];
        int dl = -1, dr = -1, dv = -1;
        for (int l = 0; l < 4; ++l) dl = max(dl, a.deg[l]);
        for (int j = 0; j < C; ++j) dr = max(dr, b.deg[j]);
        for (int j = 4; j < C; ++j) dv = max(dv, a.deg[j]);
        bad |= max(dl + dr, dv) + 1 > P;
    }
    if (bad) atomicOr(overflow, 1);
}

__global__ void k_zero_i32(int* __restrict__ p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Degrees of the product: column j of B0L B0R has degree <= max_l degL(l) + degR(j);
// V columns: max(max_l degL(l) + degR(j), degL(j)).  Resets the column maxima.
__global__ void k_prod_meta(const SlotMeta* __restrict__ mL, const SlotMeta* __restrict__ mR,
                            SlotMeta* __restrict__ mO, SolveState* __restrict__ st, int64_t cap, int ngroup, int C) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ngroup) return;
    SlotMeta a = mL[s], b = mR[s], o;
    int dl = -1;
    for (int l = 0; l < 4; ++l) dl = max(dl, a.deg[l]);
    int bad = 0;
    for (int j = 0; j < MAXC; ++j) o.deg[j] = -1;
    for (int j = 0; j < C; ++j) {
        int dj = (b.deg[j] < 0 || dl < 0) ? -1 : dl + b.deg[j];
        if (j >= 4) dj = max(dj, a.deg[j]);
        if (dj > cap) { bad = 1; dj = (int)cap; }
        o.deg[j] = dj;
    }
    for (int c = 0; c < 4; ++c) o.colmax_bits[c] = 0ull;
    mO[s] = o;
    if (bad) atomicOr(&st[s].info, 2);
}

// ---------------------------------------------------------------- difficult points (Sec. 5)
// Before the product B = (B_L S_L)(B_R S_R) of the children of a subtree
// (S = the power-of-two column scales its consumers apply), bring the
// residual of every deferred condition of that subtree up to date: a
// condition of the left child has seen B_L only, r <- (r S_L) B_R(z) S_R; one
// of the right child has seen B_L S_L (through the evaluation) and B_R,
// r <- r S_R.  Leaves [lo, mid) form the left child, [mid, hi) the right one.
// One workgroup per group; one thread per (deferred condition, column).
template <int NR>
__global__ __launch_bounds__(256) void k_defer_update(DeferList dl, const SolveState* __restrict__ st,
                                                      const SlotMeta* __restrict__ mL, const double2* __restrict__ BR,
                                                      int64_t r_stride, int64_t rcp1, const SlotMeta* __restrict__ mR,
                                                      int K, int64_t lo, int64_t mid, int64_t hi) {
    constexpr int C = 4 + NR;
    const int64_t g = blockIdx.x;
    const int nd = st[g].ndef;
    if (nd == 0) return;
    __shared__ double2 sres[64][C];
    __shared__ double sl[C], sr[C];
    __shared__ int sdeg[C];
    if (threadIdx.x < C) {
        const int c = threadIdx.x;
        sl[c] = c < 4 ? pow2_inv_scale(mL[g].colmax_bits[c]) : 1.0;
        sr[c] = c < 4 ? pow2_inv_scale(mR[g].colmax_bits[c]) : 1.0;
        sdeg[c] = mR[g].deg[c];
    }
    const int64_t e0 = g * dl.cap;
    for (int w = threadIdx.x; w < nd * C; w += blockDim.x) sres[w / C][w % C] = dl.res[(e0 + w / C) * C + w % C];
    __syncthreads();
    const double2* Bs = BR + g * r_stride;
    for (int w = threadIdx.x; w < nd * C; w += blockDim.x) {
        const int j = w / C, c = w - j * C;
        const int64_t t = dl.q[e0 + j] / K;
        if (t < lo || t >= hi) continue;
        double2 v;
        if (t < mid) {
            const double2 z = dl.node[e0 + j];
            const int dg = sdeg[c];
            double2 acc[4] = {c2(0.0, 0.0), c2(0.0, 0.0), c2(0.0, 0.0), c2(0.0, 0.0)};
            for (int k = dg; k >= 0; --k) {
#pragma unroll
                for (int row = 0; row < 4; ++row) acc[row] = cfma(acc[row], z, Bs[(int64_t)(row * C + c) * rcp1 + k]);
            }
            v = c >= 4 ? cscale(sres[j][c], sl[c]) : c2(0.0, 0.0);
#pragma unroll
            for (int row = 0; row < 4; ++row) v = cfma(cscale(sres[j][row], sl[row]), acc[row], v);
        } else {
            v = sres[j][c];
        }
        dl.res[(e0 + j) * C + c] = cscale(v, sr[c]);
    }
}

// After the root: each deferred condition, in order, takes one step of
// eq. (spbasis) on the final basis (pivot rule as in the leaves), applied to
// row 0 of every column (all that the solution needs), to the residuals of
// the deferred conditions still waiting, and to the tau-degrees.  Row 0 of
// the root basis is R[c][0..cap] with degrees in meta.  One workgroup per group.
template <int NR>
__global__ __launch_bounds__(256) void k_defer_complete(DeferList dl, SolveState* __restrict__ st,
                                                        double2* __restrict__ R, int64_t r_stride, int64_t rcp1,
                                                        SlotMeta* __restrict__ meta) {
    constexpr int C = 4 + NR;
    const int64_t g = blockIdx.x;
    const int nd = st[g].ndef;
    if (nd == 0 || st[g].info != 0) return;
    __shared__ double2 sres[64][C];
    __shared__ double2 snode[64];
    __shared__ double2 smu[C];
    __shared__ int sdeg[C], sdl[4], spiv;
    const int64_t e0 = g * dl.cap;
    for (int w = threadIdx.x; w < nd * C; w += blockDim.x) sres[w / C][w % C] = dl.res[(e0 + w / C) * C + w % C];
    for (int w = threadIdx.x; w < nd; w += blockDim.x) snode[w] = dl.node[e0 + w];
    if (threadIdx.x < C) sdeg[threadIdx.x] = meta[g].deg[threadIdx.x];
    if (threadIdx.x < 4) sdl[threadIdx.x] = st[g].delta[threadIdx.x];
    __syncthreads();
    double2* Rg = R + g * r_stride;
    int info = 0;
    for (int j = 0; j < nd; ++j) {
        if (threadIdx.x == 0) {
            double a2[4], amax = 0.0;
            for (int c = 0; c < 4; ++c) { a2[c] = cabs2(sres[j][c]); amax = fmax(amax, a2[c]); }
            const double thr = TIKH_ZTOL2 * amax;
            int kd = INT_MAX, piv = -1;
            double pm = -1.0;
            for (int c = 0; c < 4; ++c)
                if (a2[c] > thr && a2[c] > 0.0 && (sdl[c] < kd || (sdl[c] == kd && a2[c] > pm))) { kd = sdl[c]; piv = c; pm = a2[c]; }
            spiv = piv;
            if (piv >= 0) {
                const double2 rp = sres[j][piv];
                const double den = 1.0 / cabs2(rp);
                const double2 inv = c2(-rp.x * den, rp.y * den);
                for (int c = 0; c < C; ++c) smu[c] = c == piv ? c2(0.0, 0.0) : cmul(sres[j][c], inv);
            }
        }
        __syncthreads();
        const int piv = spiv;
        if (piv < 0) { info = 1; break; }
        const double2 sg = snode[j];
        const int dp = sdeg[piv];
        if (dp + 1 >= rcp1) { info = 2; break; }
        // row 0: B_c += mu_c B_pi (c != pi), then B_pi <- (z - sigma) B_pi, in chunks of
        // blockDim coefficients from the top down (each chunk reads before it writes)
        double2 mu[C];
#pragma unroll
        for (int c = 0; c < C; ++c) mu[c] = smu[c];
        double2* Bp = Rg + (int64_t)piv * rcp1;
        for (int k0 = ((dp + 1) / (int)blockDim.x) * (int)blockDim.x; k0 >= 0; k0 -= (int)blockDim.x) {
            const int k = k0 + (int)threadIdx.x;
            double2 cur = c2(0.0, 0.0), prv = c2(0.0, 0.0);
            if (k <= dp + 1) {
                cur = k <= dp ? Bp[k] : c2(0.0, 0.0);
                prv = k >= 1 ? Bp[k - 1] : c2(0.0, 0.0);
            }
            __syncthreads();
            if (k <= dp + 1) {
                if (k <= dp) {
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        if (c != piv && cnonzero(mu[c])) Rg[(int64_t)c * rcp1 + k] = cfma(mu[c], cur, Rg[(int64_t)c * rcp1 + k]);
                }
                Bp[k] = csub(prv, cmul(sg, cur));
            }
            __syncthreads();
        }
        // the deferred conditions still waiting
        for (int w = j + 1 + (int)threadIdx.x; w < nd; w += blockDim.x) {
            const double2 rpv = sres[w][piv];
#pragma unroll
            for (int c = 0; c < C; ++c) if (c != piv) sres[w][c] = cfma(mu[c], rpv, sres[w][c]);
            sres[w][piv] = cmul(rpv, csub(snode[w], sg));
        }
        if (threadIdx.x == 0) {
            for (int c = 0; c < C; ++c) if (c != piv && cnonzero(mu[c])) sdeg[c] = max(sdeg[c], dp);
            sdeg[piv] = dp + 1;
            sdl[piv] += 1;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int c = 0; c < C; ++c) meta[g].deg[c] = sdeg[c];
        for (int c = 0; c < 4; ++c) st[g].delta[c] = sdl[c];
        if (info) atomicOr(&st[g].info, info);
    }
}

// ---------------------------------------------------------------- extraction (Sec. 5)
// x = B*_{1j} / B*_{5j} with j the tau-degree-0 column: the constant columns
// are never pivoted, so for right-hand side r the solution column is 4 + r
// with unit constant entry, and x_i = [z^i] V_{1r}.  Accumulates into xacc
// (refinement adds the correction) and checks the final degrees {1,1,1,1,0..}.
// x (or, when accumulating, the refinement correction added to x) from
// the final basis, Sec. 5.  When accumulating, the squared norms of the
// correction and of the updated x are added to nrm[2s], nrm[2s+1].
__global__ __launch_bounds__(256) void k_extract(const SolveDesc* __restrict__ sd, int nr, SolveState* __restrict__ st,
                          const double2* __restrict__ B, int64_t b_stride, int64_t cp1,
                          const SlotMeta* __restrict__ meta, double2* __restrict__ xacc, int64_t x_stride,
                          int accumulate, double* __restrict__ nrm) {
    const int64_t s = blockIdx.y;
    const int64_t g = s / nr;
    const int r = (int)(s - g * nr);
    const SolveDesc d = sd[s];
    const int dg = meta[g].deg[4 + r];
    const double2* v1 = B + g * b_stride + (int64_t)(4 + r) * cp1;     // entry (row 0, column 4 + r)
    double ndx = 0.0, nx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.n; i += (int64_t)gridDim.x * blockDim.x) {
        double2 v = (i <= dg && i < cp1) ? v1[i] : c2(0.0, 0.0);
        if (!isfinite(v.x) || !isfinite(v.y)) atomicOr(&st[g].info, 8);
        if (accumulate) {
            const double2 xn = cadd(xacc[s * x_stride + i], v);
            ndx += cabs2(v);
            nx += cabs2(xn);
            xacc[s * x_stride + i] = xn;
        } else {
            xacc[s * x_stride + i] = v;
        }
    }
    if (accumulate) {
        for (int o = 32; o > 0; o >>= 1) { ndx += __shfl_xor(ndx, o, 64); nx += __shfl_xor(nx, o, 64); }
        if ((threadIdx.x & 63) == 0) { atomicAdd(&nrm[2 * s], ndx); atomicAdd(&nrm[2 * s + 1], nx); }
    }
    if (r == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        for (int c = 0; c < 4; ++c)
            if (st[g].delta[c] != 1) atomicOr(&st[g].info, 1);
    }
}

// info words of the chunk's solves are cleared before k_store_x ORs bits into them
__global__ void k_clear_info(const SolveDesc* __restrict__ sd, int64_t S, int32_t* __restrict__ info) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S && sd[s].rhs) info[sd[s].orig] = 0;
}

// Prepared batches: every solve takes its lambda from the caller's device array; a value
// that is not positive and finite is replaced by 1 (finite arithmetic throughout; the
// solve is flagged by k_prepared_info).
__global__ void k_set_lam(SolveDesc* __restrict__ sd, int64_t S, const double* __restrict__ lam) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const double v = lam[sd[s].lamx];
    sd[s].lam = (v > 0.0 && isfinite(v)) ? v : 1.0;
}

// Prepared batches, after the results are stored: bit 32 when a recorded transform length
// was too short for this call's degrees, bit 64 when the solve's lambda was not positive
// and finite.
__global__ void k_prepared_info(const SolveDesc* __restrict__ sd, int64_t S, const int* __restrict__ ovf,
                                const double* __restrict__ lam, int32_t* __restrict__ info) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S || sd[s].orig < 0) return;
    const double v = lam[sd[s].lamx];
    const int32_t bits = (*ovf ? 32 : 0) | ((v > 0.0 && isfinite(v)) ? 0 : 64);
    if (bits) info[sd[s].orig] |= bits;
}

// Stores x and the solve's info word: the group's bits other than the non-finite
// bit (the right-hand sides of a group share the pivot sequence), and the
// non-finite bit (8) from this solve's own entries.
__global__ void k_store_x(const SolveDesc* __restrict__ sd, int nr, const double2* __restrict__ xacc, int64_t x_stride,
                          const SolveState* __restrict__ st, int32_t* __restrict__ info) {
    const int64_t s = blockIdx.y;
    const SolveDesc d = sd[s];
    if (!d.rhs) return;                        // padding solve
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.n; i += (int64_t)gridDim.x * blockDim.x) {
        double2 v = xacc[s * x_stride + i];
        bad |= !isfinite(v.x) || !isfinite(v.y);
        if (d.cplx) ((double2*)d.x)[i] = v;
        else ((double*)d.x)[i] = v.x;
    }
    if (!info) return;
    if (bad) atomicOr(&info[d.orig], 8);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int32_t gi = st[s / nr].info & ~8;
        if (gi) atomicOr(&info[d.orig], gi);
    }
}

// ---------------------------------------------------------------- adjoint (backward)
// Gradients of a loss through x = (T^H T + lam^2 I)^{-1} T^H b (eq. (tiksol)), given
// w = (T^H T + lam^2 I)^{-1} gx:  g_b = T w,  g_lam = -2 lam Re<w, x>,
// g_{a_s} = sum_{i-j=s} [(b - T x) w^H - (T w) x^H]_{ij}, a lag-s cross-correlation.

// out[i] = user_b[i] - v[i] for i < m  (r = b - T x)
__global__ void k_sub_from_b(const SolveDesc* __restrict__ sd, const double2* __restrict__ v, double2* __restrict__ out,
                             int64_t stride) {
    const int64_t s = blockIdx.y;
    const SolveDesc d = sd[s];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d.m; i += (int64_t)gridDim.x * blockDim.x)
        out[s * stride + i] = csub(d.rhs ? load_elem(d.bin, i, d.cplx) : c2(0.0, 0.0), v[s * stride + i]);
}

// dst = A * conj(B) (accumulate = 0) or dst -= A * conj(B) (accumulate = 1), length N
__global__ void k_xcorr_spec(const double2* __restrict__ A, const double2* __restrict__ B, double2* dst,
                             int64_t N, int64_t stride, int accumulate) {
    const int64_t s = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        double2 v = cmul(A[s * stride + i], cconj(B[s * stride + i]));
        dst[s * stride + i] = accumulate ? csub(dst[s * stride + i], v) : v;
    }
}

// Lag sums (already inverse transformed, scale 1/N): g_col[s] = G[s] (s < m),
// g_row[s] = G[N - s] (0 < s < n), g_row[0] = 0; g_b = T w.
__global__ void k_store_grads(const SolveDesc* __restrict__ sd, const double2* __restrict__ G, int64_t N,
                              int64_t gstride, double invN, const double2* __restrict__ Tw, int64_t vstride) {
    const int64_t s = blockIdx.y;
    const SolveDesc d = sd[s];
    if (!d.rhs) return;
    const int64_t tot = d.m + d.n + d.m;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < tot; u += (int64_t)gridDim.x * blockDim.x) {
        double2 v;
        void* out;
        int64_t i;
        if (u < d.m) { i = u; v = cscale(G[s * gstride + i], invN); out = d.gcol; }
        else if (u < d.m + d.n) { i = u - d.m; v = i == 0 ? c2(0.0, 0.0) : cscale(G[s * gstride + N - i], invN); out = d.grow; }
        else { i = u - d.m - d.n; v = Tw[s * vstride + i]; out = d.gb; }
        if (d.cplx) ((double2*)out)[i] = v;
        else ((double*)out)[i] = v.x;
    }
}

// g_lam = -2 lam Re sum_j conj(w_j) x_j
__global__ __launch_bounds__(256) void k_grad_lambda(const SolveDesc* __restrict__ sd, int nr,
                                                     const double2* __restrict__ w, int64_t stride,
                                                     SolveState* __restrict__ st, int32_t* __restrict__ info) {
    const int64_t s = blockIdx.x;
    const SolveDesc d = sd[s];
    if (!d.rhs) return;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < d.n; i += blockDim.x) {
        double2 wv = w[s * stride + i];
        double2 xv = load_elem(d.xin, i, d.cplx);
        acc += wv.x * xv.x + wv.y * xv.y;
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *d.glam = -2.0 * d.lam * red[0];
        if (info) info[d.orig] = st[s / nr].info;
    }
}

// Adaptive refinement (Sec. 7.2 mentions iterative refinement; the stopping
// rule is ours).  After refinement step `it`, with rel = max over the group's
// right-hand sides of ||dx|| / ||x||: the first step's rel is e0, an
// estimate of the first solve's error; the error left after step it is
// estimated as cfac * e0 * rel (refinement contracts the error by a factor
// of about the first solve's relative error).  flags[g] = 1 asks for one
// more step.
// flags == nullptr: after the last step, a group whose estimate is still above tol
// (here the caller passes a failure threshold, far above the refinement target) gets
// info bit 16: its refinement diverged or converges too slowly to be trusted.
__global__ void k_refine_decide(const double* __restrict__ nrm, int nr, SolveState* __restrict__ st, int ngroup,
                                int first, double cfac, double tol, int32_t* __restrict__ flags) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroup) return;
    double rel = 0.0;
    for (int r = 0; r < nr; ++r) {
        const double dx2 = nrm[2 * ((int64_t)g * nr + r)], x2 = nrm[2 * ((int64_t)g * nr + r) + 1];
        if (!isfinite(dx2) || !isfinite(x2)) continue;   // a non-finite solve reports itself (bit 8)
        if (x2 > 0.0) rel = fmax(rel, sqrt(dx2 / x2));
        else if (dx2 > 0.0) rel = INFINITY;
    }
    if (first) st[g].e0 = rel;
    const double est = cfac * st[g].e0 * rel;
    const bool above = est > tol || !(est == est);
    if (flags) flags[g] = above && st[g].info == 0 ? 1 : 0;
    else if (above) st[g].info |= 16;
}

// A-posteriori bound on a solve's error before a refinement step (Sec. 7.2): with
// A = T^H T + lam^2 I >= lam^2 I the error of x against A^{-1} y is at most ||r|| / lam^2
// for the exact residual r = y - A x.  The residual computed with transforms of length N
// differs from it by a small multiple of eps ||C||^2 ||x||, where ||C||_2 = max_nu |c^_nu|
// bounds ||T||_2 (T is a block of the circulant C); REFINE_BOUND_EPS (1e-13) covers that
// about 20 times at N = 2^19.  flags[g] = 1 unless every solve of the group is certified:
// (||r|| + REFINE_BOUND_EPS (||C||^2 + lam^2) ||x||) / (lam^2 ||x||) <= tol.
#define REFINE_BOUND_EPS 1e-13
__device__ __forceinline__ double block_sum256(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}
__global__ __launch_bounds__(256) void k_refine_bound(const SolveDesc* __restrict__ sd, int nr,
                                                      const double2* __restrict__ chat, int64_t sN, int64_t N,
                                                      const double2* __restrict__ res, const double2* __restrict__ x,
                                                      int64_t sn, double tol, int32_t* __restrict__ flags) {
    __shared__ double red[4];
    const int64_t g = blockIdx.x;
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += 256) m = fmax(m, cabs2(chat[g * sN + i]));
    m = wave_max_d(m);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    const double c2max = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    int need = 0;
    for (int q = 0; q < nr; ++q) {
        const int64_t s = g * nr + q;
        if (sd[s].orig < 0) continue;                  // padding solve
        const int64_t n = sd[s].n;
        const double lam = sd[s].lam;
        double rr = 0.0, xx = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += 256) {
            rr += cabs2(res[s * sn + i]);
            xx += cabs2(x[s * sn + i]);
        }
        rr = block_sum256(rr, red);
        xx = block_sum256(xx, red);
        const double lam2 = lam * lam, nx = sqrt(xx);
        const double bound = (sqrt(rr) + REFINE_BOUND_EPS * (c2max + lam2) * nx) / (lam2 * nx);
        if (!(bound <= tol)) need = 1;                 // also a zero or non-finite solution
    }
    if (threadIdx.x == 0) flags[g] = need;
}

__global__ void k_zero_d(double* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// Exchange the refinement state of the group pairs (a, b) = pairs[y]: solve
// descriptors, state, symbol, right-hand side and current solution.
__global__ void k_swap_groups(SolveDesc* __restrict__ sd, SolveState* __restrict__ st, double2* __restrict__ chat,
                              int64_t sN, double2* __restrict__ yv, double2* __restrict__ xacc, int64_t sn, int nr,
                              const int2* __restrict__ pairs, double2* __restrict__ cg, double* __restrict__ asum) {
    const int2 pr = pairs[blockIdx.y];
    const int64_t a = pr.x, b = pr.y;
    const int64_t nsym = cg ? 2 * sN : sN;         // the Gramian's symbol too, when there is one
    const int64_t tot = nsym + 2 * nr * sn;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        double2 *pa, *pb;
        if (i < sN) { pa = chat + a * sN + i; pb = chat + b * sN + i; }
        else if (i < nsym) { pa = cg + a * sN + (i - sN); pb = cg + b * sN + (i - sN); }
        else {
            const int64_t j = i - nsym, which = j / (nr * sn), rem = j - which * nr * sn;
            double2* base = which == 0 ? yv : xacc;
            pa = base + a * nr * sn + rem;
            pb = base + b * nr * sn + rem;
        }
        const double2 t = *pa;
        *pa = *pb;
        *pb = t;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int r = 0; r < nr; ++r) {
            const SolveDesc t = sd[a * nr + r];
            sd[a * nr + r] = sd[b * nr + r];
            sd[b * nr + r] = t;
        }
        const SolveState t = st[a];
        st[a] = st[b];
        st[b] = t;
        const double u = asum[a];
        asum[a] = asum[b];
        asum[b] = u;
    }
}

__global__ void k_init_state(const SolveDesc* __restrict__ sd, int nr, SolveState* __restrict__ st, int ngroup,
                             int keep_info) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ngroup) return;
    const SolveDesc d = sd[(int64_t)g * nr];
    // delta = -tau, tau = [n-1, m-1, m+k-2, n+k-2, 0] (eq. (taudef) adapted to eq. (ex6))
    st[g].delta[0] = -(int)(d.n - 1);
    st[g].delta[1] = -(int)(d.m - 1);
    st[g].delta[2] = -(int)(d.m + d.k - 2);
    st[g].delta[3] = -(int)(d.n + d.k - 2);
    st[g].ndef = 0;
    if (!keep_info) st[g].info = 0;
}

}  // namespace tikh
