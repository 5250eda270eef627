// Host driver and C ABI of the superfast Tikhonov-Toeplitz solver (gfx950).
//
// Paper: Turnes, Balcan, Romberg, "Superfast Tikhonov Regularization of
// Toeplitz Systems".  The driver plans the extension (Alg. 2), builds the
// interpolation data (Sec. 3-4) and walks the recursion tree of Alg. 1 in
// order, launching one kernel per task for all solves of a bucket at once
// (solves that share the extended size N share the tree).
#include "../../include/tikh.h"
#include "tikh_kernels.hip"

#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

namespace tikh {

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) {                     \
            last_hip_error = e_;                    \
            return TIKH_EHIP;                       \
        }                                           \
    } while (0)

static hipError_t last_hip_error = hipSuccess;

struct Ctx {
    bool init = false;
    hipStream_t stream = nullptr;
    tikh_opts opts{};
    tikh_stats stats{};
    char* ws = nullptr;
    size_t ws_size = 0;
    bool ws_ext = false;                 // ws is the caller's buffer (tikh_set_workspace)
    std::map<int64_t, double2*> tw;      // twiddle tables by size Q
    std::map<int64_t, double2*> tw2;     // two-level twiddle tables by size
    int64_t launches = 0;
    int* dneed = nullptr;                // device / pinned host word for degree readback
    int* hneed = nullptr;
    // allocation-free calls: twiddle tables and the readback word live in an arena at
    // the front of the device's static scratch buffer (re-filled by every such call)
    bool noalloc = false;
    char* arena = nullptr;
    size_t arena_size = 0, arena_used = 0;
    std::map<int64_t, double2*> ntw, ntw2;
    int* ndneed = nullptr;
    std::map<int64_t, std::vector<double2>> htw, htw2;   // host copies of the tables, by size
    // Product transform lengths by merge (depth, index) for a batch composition: recorded
    // from the degrees read back while a chunk's first recursion runs, then reused without
    // host synchronization by its later recursions and by later calls with the same
    // composition, and checked on the device (a product that would need a longer transform
    // raises the chunk's overflow flag, and the chunk is run again with read-back sizing).
    struct Sizes {
        std::map<int64_t, int64_t> P;
        bool complete = false;
    };
    std::map<uint64_t, Sizes> sizes;
    Sizes* cur_sizes = nullptr;          // entry of the running chunk (nullptr: read back every merge)
    bool replay = false;                 // the running recursion takes its lengths from cur_sizes
    int* overflow = nullptr;             // device flag of the running chunk
    bool headroom = false;               // record lengths for degrees 1/8 + 8 above the ones read back
    int64_t generation = 0;              // counts tikh_release calls (prepared batches hold tables of one)
    int64_t syncs = 0;                   // host synchronizations of the last call
    std::vector<hipStream_t> pool;       // streams of chunks run side by side
    std::vector<hipEvent_t> events;      // their fork and join events
};
static Ctx g;

// Optional timing of one kernel kind: HIP event pairs recorded on the library
// stream around each launch whose name matches (used by the benchmark to
// measure the dominant kernel's average launch duration live).
struct KProf {
    std::string name;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    double total_ms = 0.0;
    int64_t count = 0;
    double units = 0.0;          // algorithmic work of the timed launches (bytes or flops, per kernel kind)
    // per-shape breakdown, printed to stderr when TIKH_PROF_DETAIL is set
    std::string label;           // shape label of the next launch
    std::vector<std::string> labels;
    std::map<std::string, std::pair<double, int64_t>> detail;
};
static KProf kprof;

static bool prof_on(const char* name) { return !kprof.name.empty() && kprof.name == name; }
static void prof_begin(const char* name) {
    if (!prof_on(name) || g.noalloc) return;     // allocation-free calls create no events
    if (kprof.used + 2 > kprof.pool.size()) {
        for (int i = 0; i < 256; ++i) { hipEvent_t e; if (hipEventCreate(&e) == hipSuccess) kprof.pool.push_back(e); }
    }
    if (kprof.used + 2 <= kprof.pool.size()) (void)hipEventRecord(kprof.pool[kprof.used], g.stream);
}
static void prof_end(const char* name) {
    if (!prof_on(name) || g.noalloc) return;
    if (kprof.used + 2 <= kprof.pool.size()) {
        (void)hipEventRecord(kprof.pool[kprof.used + 1], g.stream);
        kprof.used += 2;
        kprof.labels.push_back(kprof.label);
    }
}
static void prof_units(const char* name, double u) {
    if (prof_on(name)) kprof.units += u;
}
static void prof_collect() {
    if (kprof.used == 0) return;
    (void)hipStreamSynchronize(g.stream);
    for (size_t i = 0; i + 1 < kprof.used; i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, kprof.pool[i], kprof.pool[i + 1]) == hipSuccess) {
            kprof.total_ms += ms;
            kprof.count++;
            auto& d = kprof.detail[kprof.labels[i / 2]];
            d.first += ms;
            d.second++;
        }
    }
    kprof.used = 0;
    kprof.labels.clear();
}
static void prof_print_detail() {
    if (!getenv("TIKH_PROF_DETAIL") || kprof.detail.empty()) return;
    std::vector<std::pair<double, std::string>> v;
    for (auto& kv : kprof.detail) v.push_back({kv.second.first, kv.first});
    std::sort(v.rbegin(), v.rend());
    for (auto& e : v)
        fprintf(stderr, "[tikh prof] %-70s %10.3f ms %8lld launches\n", e.second.c_str(), e.first,
                (long long)kprof.detail[e.second].second);
}
#define LAUNCH_SH(kname, kern, grid, block, shmem, ...)                                     \
    do {                                                                                 \
        prof_begin(kname);                                                               \
        hipLaunchKernelGGL(kern, grid, block, shmem, g.stream, __VA_ARGS__);             \
        prof_end(kname);                                                                 \
        g.launches++;                                                                    \
    } while (0)
#define LAUNCH(kname, kern, grid, block, ...) LAUNCH_SH(kname, kern, grid, block, 0, __VA_ARGS__)

static bool opts_valid(const tikh_opts* o);

// Environment overrides of the defaults, read once: TIKH_<NAME> for every option (for
// example TIKH_NLIM=128, TIKH_REFINE=2, TIKH_DEFER_TOL=1e-3).  A value that does not parse,
// or that would make the options invalid, is reported on stderr and ignored.
static void env_overrides(tikh_opts& o) {
    struct Ent { const char* name; int32_t* i; double* d; };
    const Ent ents[] = {{"TIKH_NLIM", &o.n_lim, nullptr}, {"TIKH_REFINE", &o.refine, nullptr},
                        {"TIKH_REFINE_MAX", &o.refine_max, nullptr}, {"TIKH_REFINE_TOL", nullptr, &o.refine_tol},
                        {"TIKH_DEFER_TOL", nullptr, &o.defer_tol},
                        {"TIKH_LEAF_WAVE_GROUPS", &o.leaf_wave_groups, nullptr},
                        {"TIKH_STREAMS", &o.streams, nullptr}, {"TIKH_MERGE_TOL", nullptr, &o.merge_tol},
                        {"TIKH_FALLBACK_NLIM", &o.fallback_nlim, nullptr},
                        {"TIKH_CHUNK_GROUPS", &o.chunk_groups, nullptr},
                        {"TIKH_REFINE_SKIP", &o.refine_skip, nullptr}};
    for (const Ent& e : ents) {
        const char* v = getenv(e.name);
        if (!v || !*v) continue;
        char* end = nullptr;
        tikh_opts t = o;
        bool ok;
        if (e.i) {
            const long x = strtol(v, &end, 10);
            ok = end && *end == 0 && x >= INT32_MIN && x <= INT32_MAX;
            if (ok) *(int32_t*)((char*)&t + ((char*)e.i - (char*)&o)) = (int32_t)x;
        } else {
            const double x = strtod(v, &end);
            ok = end && *end == 0;
            if (ok) *(double*)((char*)&t + ((char*)e.d - (char*)&o)) = x;
        }
        if (ok && opts_valid(&t)) o = t;
        else fprintf(stderr, "tikh: ignoring %s=%s (not a valid value)\n", e.name, v);
    }
}

// Options take their defaults once; the degree readback words are (re)allocated
// until both exist, and a merge that finds either missing reports TIKH_ENOMEM.
static void init_opts() {
    if (g.init) return;
    g.opts.n_lim = 256;
    g.opts.refine = 1;
    g.opts.refine_max = 3;
    g.opts.leaf_wave_groups = 1536;
    g.opts.streams = 16;
    g.opts.merge_tol = 0.25;
    g.opts.fallback_nlim = 64;
    g.opts.refine_skip = 0;
    g.opts.refine_tol = 1e-10;
    g.opts.defer_tol = 0.0;
    env_overrides(g.opts);
    g.init = true;
}
static void ensure_init() {
    init_opts();
    if (!g.dneed && hipMalloc((void**)&g.dneed, sizeof(int)) != hipSuccess) g.dneed = nullptr;
    if (!g.hneed && hipHostMalloc((void**)&g.hneed, sizeof(int), hipHostMallocDefault) != hipSuccess) g.hneed = nullptr;
}

// ---------------------------------------------------------------- planning (Alg. 2)
static bool smooth5(int64_t v) {
    if (v <= 0) return false;
    for (int f : {2, 3, 5}) while (v % f == 0) v /= f;
    return v == 1;
}

// OptExtend adapted to the paired split of the l2 problem: two condition sets
// per node, so a leaf of M nodes holds 2M conditions and must satisfy
// 2M <= n_lim; M is forced even (the leaf is two cosets of M/2 nodes) and
// rounded up to a 5-smooth value so that every FFT length is a product of
// radices 2, 3, 4, 5.  Returns false if n_lim is unusable.
static bool opt_extend(int64_t Nt, int nlim, int64_t* N, int64_t* M, int* p) {
    int64_t m = Nt;
    int pp = 0;
    while (2 * m > nlim) { ++pp; m = (m + 1) / 2; }
    if (m % 2) ++m;
    while (!smooth5(m)) m += 2;
    if (2 * m > nlim) return false;
    *M = m; *p = pp; *N = ((int64_t)1 << pp) * m;
    return true;
}

static int64_t smallest_divisor_geq(int64_t Q, int64_t need) {
    int64_t best = Q;
    for (int64_t a = 1; a * a <= Q; ++a) {
        if (Q % a) continue;
        int64_t b = Q / a;
        if (a >= need && a < best) best = a;
        if (b >= need && b < best) best = b;
    }
    return best;
}

static bool make_plan(int64_t N, int64_t M, int p, Plan* pl) {
    memset(pl, 0, sizeof(*pl));
    pl->N = N; pl->M = M; pl->p = p; pl->K = (int)(2 * M);
    pl->Q = 8 * N;
    // Degree capacity of a basis built from the cnt conditions of a depth-d
    // subtree: every condition raises the largest degree by at most one, so
    // deg <= cnt; cnt itself is reached only if one column takes every pivot,
    // which the degree bookkeeping reports as info = 2.  cap = cnt - 1 makes the
    // product length of the parent exactly cnt_parent (a divisor of Q).
    for (int d = 0; d <= p; ++d) {
        int64_t cnt = (2 * N) >> d;
        pl->cap[d] = (p == 0) ? cnt : cnt - 1;
    }
    for (int d = 0; d < p; ++d) {
        int64_t need = 2 * pl->cap[d + 1] + 1;
        pl->P[d] = smallest_divisor_geq(pl->Q, need);
        if (!smooth5(pl->P[d])) return false;
    }
    return true;
}

// Stages of an LDS transform of length L = 2^a 3^b 5^c <= 4096: radix 16
// while possible (radix 8 when the line fits the 2048-point kernel, which
// holds at most 9 values per butterfly), radix 9 per pair of threes, a single
// three merged with a leftover 2 or 4 (radix 6, or 12 in the large kernel),
// the remaining power of two as one stage, then the fives.
static const int FFT_SMALL_CAP = 2048;
static bool fft_plan(int64_t L, FftPlanDev* f, bool small) {
    if (L < 1 || L > (small ? FFT_SMALL_CAP : FFT_LDS_MAX)) return false;
    f->L = (int)L; f->nst = 0;
    int64_t v = L;
    int a = 0, b = 0, c = 0;
    while (v % 2 == 0) { v /= 2; ++a; }
    while (v % 3 == 0) { v /= 3; ++b; }
    while (v % 5 == 0) { v /= 5; ++c; }
    if (v != 1) return false;
    if (small) {
        while (a >= 3) { f->radix[f->nst++] = 8; a -= 3; }
    } else {
        while (a >= 4) { f->radix[f->nst++] = 16; a -= 4; }
    }
    while (b >= 2) { f->radix[f->nst++] = 9; b -= 2; }
    if (b == 1) {
        if (a == 1) { f->radix[f->nst++] = 6; a = 0; }
        else if (a == 2 && !small) { f->radix[f->nst++] = 12; a = 0; }
        else f->radix[f->nst++] = 3;
    }
    if (a == 3) f->radix[f->nst++] = 8;
    else if (a == 2) f->radix[f->nst++] = 4;
    else if (a == 1) f->radix[f->nst++] = 2;
    while (c-- > 0) f->radix[f->nst++] = 5;
    return true;
}
static bool fft_plan(int64_t L, FftPlanDev* f) { return fft_plan(L, f, false); }

// Two-level table of e^{2 pi i x / M}: [x < 2^bits | (x >> bits) <= (M - 1) >> bits].
static int tw2_bits(int64_t M) {
    int lg = 0;
    while (((int64_t)1 << lg) < M) ++lg;
    return std::max(1, (lg + 1) / 2);
}

// Host tables (long double angles, rounded once), kept for the life of the library.
static const std::vector<double2>& host_twiddles2(int64_t M) {
    auto it = g.htw2.find(M);
    if (it != g.htw2.end()) return it->second;
    const int bits = tw2_bits(M);
    const int64_t nlo = (int64_t)1 << bits, nhi = ((M - 1) >> bits) + 1;
    std::vector<double2> h(nlo + nhi);
    const long double pi2 = 6.283185307179586476925286766559005768L;
    for (int64_t j = 0; j < nlo; ++j) {
        long double a = pi2 * (long double)j / (long double)M;
        h[j] = make_double2((double)cosl(a), (double)sinl(a));
    }
    for (int64_t j = 0; j < nhi; ++j) {
        long double a = pi2 * (long double)(j * nlo) / (long double)M;
        h[nlo + j] = make_double2((double)cosl(a), (double)sinl(a));
    }
    return g.htw2[M] = std::move(h);
}
static const std::vector<double2>& host_twiddles(int64_t Q) {
    auto it = g.htw.find(Q);
    if (it != g.htw.end()) return it->second;
    std::vector<double2> h(Q);
    const long double pi2 = 6.283185307179586476925286766559005768L;
    for (int64_t q = 0; q < Q; ++q) {
        long double a = pi2 * (long double)q / (long double)Q;
        h[q] = make_double2((double)cosl(a), (double)sinl(a));
    }
    return g.htw[Q] = std::move(h);
}

// A device copy of a host table: in an allocation-free call carved from the arena
// (and copied on the library stream), otherwise allocated once and kept.
static double2* device_table(std::map<int64_t, double2*>& keep, std::map<int64_t, double2*>& per_call, int64_t key,
                             const std::vector<double2>& h) {
    const size_t bytes = sizeof(double2) * h.size();
    if (g.noalloc) {
        auto it = per_call.find(key);
        if (it != per_call.end()) return it->second;
        const size_t off = (g.arena_used + 255) & ~(size_t)255;
        if (off + bytes > g.arena_size) return nullptr;
        double2* d = (double2*)(g.arena + off);
        if (hipMemcpyAsync(d, h.data(), bytes, hipMemcpyHostToDevice, g.stream) != hipSuccess) return nullptr;
        g.arena_used = off + bytes;
        return per_call[key] = d;
    }
    auto it = keep.find(key);
    if (it != keep.end()) return it->second;
    double2* d = nullptr;
    if (hipMalloc(&d, bytes) != hipSuccess) return nullptr;
    if (hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) { (void)hipFree(d); return nullptr; }
    return keep[key] = d;
}
static double2* twiddles2(int64_t M, int* bits) {
    *bits = tw2_bits(M);
    return device_table(g.tw2, g.ntw2, M, host_twiddles2(M));
}
static double2* twiddles(int64_t Q) { return device_table(g.tw, g.ntw, Q, host_twiddles(Q)); }

// Adaptive refinement: the factor of the estimate cfac * e0 * ||dx|| / ||x||
// of the error left after a step.
static const double REFINE_CFAC = 1000.0;
// Estimate above which a solve's refinement counts as failed after its last step (info bit 16):
// far above the refinement target, so that slow but converging refinement is not flagged
// (measured: an adjoint solve whose refinement contracted by 1e-2 per step ended with an
// estimate of 1e-6 and an error of 1e-9), while a basis that lost the solution is.
static const double REFINE_FAIL = 1e-4;

// Deferred (difficult) conditions held per group and solve; more set info bit 4.
static const int DEFER_CAP = 64;
static bool defer_on() { return g.opts.defer_tol > 0.0; }

// subtrees with at most this many conditions are merged by the direct kernels
static const int64_t DIRECT_MAX_COND = 256;

// ---------------------------------------------------------------- workspace layout
// A bucket holds G groups of nr solves (nr right-hand sides of one operator).
// Group data: symbol, interpolation data, step records, basis slots.
// Solve data: per right-hand side FFT lines and vectors.
struct Layout {
    int nr, C;
    int64_t nmax, mmax;
    // strides in double2 units
    int64_t sN, sn, sphi, srec, sV, sF, sscr;
    int64_t sslot[40];
    int64_t sT;                      // stride of the shared right-child slot
    int64_t tOff;                    // offset of odd-depth results inside it
    int64_t Lmax;
    size_t group_bytes;              // per group, held for the whole solve
    size_t solve_bytes;              // per right-hand side
    size_t temp_bytes;               // per group of a merge chunk (evaluation and product scratch)
};

static void make_layout(const Plan& pl, int nr, int64_t mmax, int64_t nmax, Layout* L) {
    L->nr = nr; L->C = 4 + nr;
    const int64_t E = 4 * L->C;      // stored basis entries
    L->nmax = nmax; L->mmax = mmax;
    L->sN = pl.N;
    L->sn = std::max(mmax, nmax);
    L->sphi = (int64_t)L->C * 2 * pl.N;
    L->srec = (int64_t)pl.K * (int64_t)(sizeof(LeafRec) / sizeof(double2));
    L->Lmax = pl.p >= 1 ? pl.N / 4 : 1;
    L->sV = 2 * E * L->Lmax;
    int64_t fmax = 1;
    for (int d = 0; d < pl.p; ++d)
        fmax = std::max(fmax, (d == 0 && !defer_on() ? std::max<int64_t>(L->C, 4 * nr) : E) * pl.P[d]);
    L->sF = fmax;
    L->sscr = std::max(L->sV, L->sF);
    size_t tot = 0;
    tot += 2 * L->sN + L->sphi + L->srec;     // symbols of T (or L) and of the Gramian, residuals, step records
    // pending left children: one slot per depth; right-child results: one
    // shared slot (a right child's basis is consumed by the next product,
    // which reads it completely before it writes its own result).  Results
    // at odd depths sit at offset tOff, so a fused direct product (which reads
    // its right factor while it writes the parent) never overwrites its input.
    L->sT = 0;
    L->tOff = 0;
    for (int d = 0; d <= pl.p; ++d) {
        L->sslot[d] = E * (pl.cap[d] + 1);
        if (d >= 1) tot += L->sslot[d];
        if (((2 * pl.N) >> d) <= 2 * DIRECT_MAX_COND || d >= pl.p - 1) L->tOff = std::max(L->tOff, L->sslot[d]);
    }
    for (int d = 0; d <= pl.p; ++d) {
        int64_t sz = (d == 0 && pl.p > 0) ? (int64_t)(4 + nr) * (pl.cap[0] + 1) : L->sslot[d];
        L->sT = std::max(L->sT, ((d & 1) ? L->tOff : 0) + sz);
    }
    tot += L->sT;
    L->group_bytes = tot * sizeof(double2) + 2 * (pl.p + 1) * sizeof(SlotMeta) + sizeof(SolveState) + 3 * sizeof(double) +
                     sizeof(int32_t) + sizeof(int2) + DEFER_CAP * (sizeof(int32_t) + (1 + L->C) * sizeof(double2)) + 256;
    L->solve_bytes = (size_t)(4 * L->sN + 4 * L->sn) * sizeof(double2) + sizeof(SolveDesc) + 2 * sizeof(double) + 64;
    L->temp_bytes = (size_t)(L->sV + 2 * L->sF + L->sscr) * sizeof(double2);
}

struct Bufs {
    int nr;
    SolveDesc* sd;                   // [G*nr]
    SolveState* st;                  // [G]
    double* rms;                     // [G]
    double* asum;                    // [G] sum of the generator's magnitudes (a bound on ||T||_2)
    double* rmsg;                    // [G] Gramian generator rms (Toeplitz-Gramian problem)
    double2* chat;                   // [G][N]
    double2* cg;                     // [G][N] symbol of the extended Gramian
    double2 *bA, *bB, *bC, *bS;      // [G*nr][N]
    double2 *yv, *xacc, *t1, *t2;    // [G*nr][sn]
    double2* phi;                    // [G][C][2N]
    LeafRec* rec;                    // [G][K]
    double2* slotS[40];
    double2* slotT[40];
    SlotMeta* metaS[40];
    SlotMeta* metaT[40];
    // merge scratch shared by the groups of one merge chunk
    double2* V;
    double2 *FL, *FR, *scr;
    DeferList dl;                    // deferred (difficult) conditions, [G][DEFER_CAP]
    double* nrm;                     // [2S] refinement norms (correction, solution)
    int32_t* flags;                  // [G] one more refinement step
    int2* pairs;                     // [G] group exchanges of the compaction
    int64_t chunk;                   // groups per merge chunk at the largest level
    double2* pool;                   // V, FL, FR and scr as one region (re-split per level)
    int64_t pool_elems;
    int* elist;                      // device entry lists
    int* ovf;                        // product-length overflow flag of the chunk
};

// Group pointers advanced by c0 groups, solve pointers by c0*nr solves
// (merge scratch and entry lists stay).
static Bufs shift_bufs(const Bufs& b, const Layout& L, const Plan& pl, int64_t c0) {
    Bufs o = b;
    const int64_t s0 = c0 * b.nr;
    o.sd += s0; o.st += c0; o.rms += c0; o.rmsg += c0; o.asum += c0;
    o.chat += c0 * L.sN;
    o.cg += c0 * L.sN;
    o.bA += s0 * L.sN; o.bB += s0 * L.sN; o.bC += s0 * L.sN; o.bS += s0 * L.sN;
    o.yv += s0 * L.sn; o.xacc += s0 * L.sn; o.t1 += s0 * L.sn; o.t2 += s0 * L.sn;
    o.phi += c0 * L.sphi;
    o.rec += c0 * pl.K;
    for (int d = 0; d <= pl.p; ++d) {
        if (b.slotS[d]) o.slotS[d] = b.slotS[d] + c0 * L.sslot[d];
        o.slotT[d] = b.slotT[d] + c0 * L.sT;
        o.metaS[d] = b.metaS[d] + c0;
        o.metaT[d] = b.metaT[d] + c0;
    }
    return o;
}

static int ensure_ws(size_t bytes) {
    if (bytes <= g.ws_size) return TIKH_OK;
    if (g.ws_ext) return TIKH_ENOMEM;                // the caller's buffer is too small
    if (g.ws) { (void)hipStreamSynchronize(g.stream); (void)hipFree(g.ws); g.ws = nullptr; g.ws_size = 0; }
    if (hipMalloc(&g.ws, bytes) != hipSuccess) { g.ws = nullptr; return TIKH_ENOMEM; }
    g.ws_size = bytes;
    return TIKH_OK;
}

static char* carve(char*& p, size_t bytes) {
    char* r = p;
    p += (bytes + 255) & ~(size_t)255;
    return r;
}

// Entry lists of the product (entry e = row * C + column):
//   all 4C entries; root: left row 0 (C entries), right columns 4..C-1 of rows 0..3, output row 0 columns 4..C-1.
struct EList {
    int all[4 * MAXC];
    int row0[MAXC];
    int vcols[4 * MAXNR];
    int xout[MAXNR];
    int b0[16];            // the B0 block, i * C + t
    int row0b0[4];         // row 0 of the B0 block
};
static EList make_elist(int nr) {
    EList e{};
    const int C = 4 + nr;
    for (int i = 0; i < 4 * C; ++i) e.all[i] = i;
    for (int j = 0; j < C; ++j) e.row0[j] = j;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < nr; ++j) e.vcols[i * nr + j] = i * C + 4 + j;
    for (int j = 0; j < nr; ++j) e.xout[j] = 4 + j;
    for (int i = 0; i < 4; ++i)
        for (int t = 0; t < 4; ++t) e.b0[i * 4 + t] = i * C + t;
    for (int t = 0; t < 4; ++t) e.row0b0[t] = t;
    return e;
}

// fixed part of a chunk's workspace beyond its per-group, per-solve and merge-scratch
// terms (small buffers and the 256-byte alignment of every carved buffer)
static const size_t WS_FIXED = 64 * 1024 + 256 * 128;

static size_t chunk_bytes(const Layout& L, int64_t G, int64_t CH) {
    return (size_t)G * L.group_bytes + (size_t)(G * L.nr) * L.solve_bytes + (size_t)CH * L.temp_bytes + WS_FIXED;
}

// Carves a chunk's buffers from the workspace region at base (chunk_bytes(L, G, CH) long).
static int carve_bufs(const Plan& pl, const Layout& L, int64_t G, int64_t CH, char* base, Bufs* b) {
    const int nr = L.nr;
    const int64_t S = G * nr;
    char* p = base;
    b->nr = nr;
    b->chunk = CH;
    b->sd = (SolveDesc*)carve(p, sizeof(SolveDesc) * S);
    b->st = (SolveState*)carve(p, sizeof(SolveState) * G);
    b->rms = (double*)carve(p, sizeof(double) * G);
    b->asum = (double*)carve(p, sizeof(double) * G);
    b->rmsg = (double*)carve(p, sizeof(double) * G);
    b->elist = (int*)carve(p, sizeof(EList));
    b->ovf = (int*)carve(p, sizeof(int));
    b->dl.cap = DEFER_CAP;
    b->dl.C = L.C;
    b->dl.q = (int32_t*)carve(p, sizeof(int32_t) * G * DEFER_CAP);
    b->dl.node = (double2*)carve(p, sizeof(double2) * G * DEFER_CAP);
    b->dl.res = (double2*)carve(p, sizeof(double2) * G * DEFER_CAP * L.C);
    b->nrm = (double*)carve(p, sizeof(double) * 2 * S);
    b->flags = (int32_t*)carve(p, sizeof(int32_t) * G);
    b->pairs = (int2*)carve(p, sizeof(int2) * G);
    auto cv = [&](int64_t per, int64_t cnt) { return (double2*)carve(p, sizeof(double2) * per * cnt); };
    b->chat = cv(L.sN, G);
    b->cg = cv(L.sN, G);
    b->bA = cv(L.sN, S); b->bB = cv(L.sN, S); b->bC = cv(L.sN, S); b->bS = cv(L.sN, S);
    b->yv = cv(L.sn, S); b->xacc = cv(L.sn, S); b->t1 = cv(L.sn, S); b->t2 = cv(L.sn, S);
    b->phi = cv(L.sphi, G);
    b->rec = (LeafRec*)cv(L.srec, G);
    double2* tslot = cv(L.sT, G);
    for (int d = 0; d <= pl.p; ++d) {
        b->slotS[d] = d >= 1 ? cv(L.sslot[d], G) : nullptr;
        b->slotT[d] = tslot + ((d & 1) ? L.tOff : 0);
        b->metaS[d] = (SlotMeta*)carve(p, sizeof(SlotMeta) * G);
        b->metaT[d] = (SlotMeta*)carve(p, sizeof(SlotMeta) * G);
    }
    b->V = cv(L.sV, CH);
    b->FL = cv(L.sF, CH); b->FR = cv(L.sF, CH); b->scr = cv(L.sscr, CH);
    b->pool = b->V;
    b->pool_elems = (int64_t)((p - (char*)b->V) / sizeof(double2));
    if ((size_t)(p - base) > chunk_bytes(L, G, CH)) return TIKH_ENOMEM;
    return TIKH_OK;
}

// ---------------------------------------------------------------- launch helpers
static inline dim3 grid1(int64_t work, int64_t S, int bs = 256) {
    int64_t gx = (work + bs - 1) / bs;
    gx = std::max<int64_t>(1, std::min<int64_t>(gx, 4096));
    return dim3((unsigned)gx, (unsigned)S, 1);
}

// Split of a long FFT into L1 x L2 (both <= FFT_LDS_MAX, balanced); the
// same split is used for every transform of a given length, so a spectrum
// left in four-step order by a forward transform is read back correctly by
// the inverse.  Returns L1 (L1 = Lf for a single-pass length).
static int64_t fft_split(int64_t Lf) {
    if (Lf <= FFT_LDS_MAX) return Lf;
    int64_t L1 = 0;
    for (int64_t c = 1; c <= FFT_LDS_MAX; ++c)
        if (Lf % c == 0 && Lf / c <= FFT_LDS_MAX && smooth5(c)) {
            if (L1 == 0 || std::llabs((long long)(c * c - Lf)) < std::llabs((long long)(L1 * L1 - Lf))) L1 = c;
        }
    return L1;
}

enum FftOrder {
    FFT_NATURAL = 0,   // natural order in and out (four-step followed by a reordering pass)
    FFT_FWD_T = 1,     // natural in, four-step order out: X[j1 + L1 j2] at j1*L2 + j2
    FFT_INV_T = 2      // four-step order in, natural out
};

static void fft_pass(double2* data, int64_t S, int64_t sstride, int64_t nlines, int64_t lines_inner,
                     int64_t line_stride, int64_t outer_stride, int64_t elem_stride, int64_t L, int sign,
                     int64_t post_L, const double2* tw, int64_t Q, int lpw_cap, const FftArgs* fuse = nullptr,
                     bool first = true, bool last = true) {
    FftArgs a{};
    if (fuse) {
        a = *fuse;
        if (!first) a.load_mode = 0;
        if (!last) a.store_mode = 0;
    }
    a.data = data; a.solve_stride = sstride; a.sign = sign; a.scale = 1.0; a.tw = tw; a.Q = Q;
    a.ltw = twiddles(L);              // per-length tables: contiguous twiddle reads
    a.ptw = post_L ? twiddles2(post_L, &a.pbits) : nullptr;
    if (a.load_mode == 2) a.ftw = twiddles2(a.fold_N, &a.fbits);
    // lines of at most 2048 points use the smaller kernel: twice the workgroups per CU
    // outweigh its extra stage for some lengths (measured in the solver's fused passes)
    const bool small = L <= FFT_SMALL_CAP;
    fft_plan(L, &a.pl, small);
    a.nlines = nlines; a.lines_inner = lines_inner; a.line_stride = line_stride; a.outer_stride = outer_stride;
    a.elem_stride = elem_stride; a.post_L = post_L;
    a.lpw = (int)std::max<int64_t>(1, std::min<int64_t>((small ? FFT_SMALL_CAP : FFT_LDS_MAX) / L, lpw_cap));
    dim3 gr((unsigned)((nlines + a.lpw - 1) / a.lpw), (unsigned)S);
    // algorithmic traffic: every element of every line read once and written once
    prof_units("fft", 32.0 * (double)S * (double)nlines * (double)L);
    if (prof_on("fft") && getenv("TIKH_PROF_DETAIL")) {
        char lab[160];
        snprintf(lab, sizeof lab, "L=%lld es=%lld lines=%lld S=%lld load=%d store=%d post=%d", (long long)L,
                 (long long)elem_stride, (long long)nlines, (long long)S, a.load_mode, a.store_mode, post_L ? 1 : 0);
        kprof.label = lab;
    }
    if (small) LAUNCH("fft", k_fft<FFT_SMALL_CAP>, gr, dim3(FFT_THREADS), a);
    else LAUNCH("fft", k_fft<FFT_LDS_MAX>, gr, dim3(FFT_THREADS), a);
}

// In-place FFT of `nlines` contiguous lines of length Lf per item (line
// stride Lf, item stride sstride), direction `sign`.  `fuse` (optional)
// carries a fused first-pass load and/or last-pass store.
static int fft_lines(double2* data, int64_t S, int64_t sstride, int64_t nlines, int64_t Lf, int sign,
                     const double2* tw, int64_t Q, double2* scratch, int64_t scr_stride, int order = FFT_NATURAL,
                     const FftArgs* fuse = nullptr) {
    FftPlanDev chk;
    if (Lf <= FFT_LDS_MAX) {
        if (!fft_plan(Lf, &chk)) return TIKH_EINVAL;
        // one original line per transformed line: o = line, offset = element index
        fft_pass(data, S, sstride, nlines, 1, 0, Lf, 1, Lf, sign, 0, tw, Q, 64, fuse, true, true);
        return TIKH_OK;
    }
    const int64_t L1 = fft_split(Lf);
    if (L1 == 0) return TIKH_EINVAL;
    const int64_t L2 = Lf / L1;
    if (!fft_plan(L1, &chk) || !fft_plan(L2, &chk)) return TIKH_EINVAL;
    if (order == FFT_INV_T) {
        // rows j1 (contiguous, length L2) with twiddle w^{j1 k2}, then columns k2 (stride L2, length L1)
        fft_pass(data, S, sstride, nlines * L1, L1, L2, Lf, 1, L2, sign, Lf, tw, Q, 64, fuse, true, false);
        fft_pass(data, S, sstride, nlines * L2, L2, 1, Lf, L2, L1, sign, 0, tw, Q, 64, fuse, false, true);
        return TIKH_OK;
    }
    // columns k2 (stride L2, length L1) with twiddle w^{j1 k2}, then rows j1 (contiguous, length L2)
    fft_pass(data, S, sstride, nlines * L2, L2, 1, Lf, L2, L1, sign, Lf, tw, Q, 64, fuse, true, false);
    fft_pass(data, S, sstride, nlines * L1, L1, L2, Lf, 1, L2, sign, 0, tw, Q, 64, fuse, false, true);
    if (order == FFT_NATURAL) {
        const int64_t tiles = ((L1 + 31) / 32) * ((L2 + 31) / 32);
        hipLaunchKernelGGL(k_fourstep_transpose, dim3((unsigned)(nlines * tiles), (unsigned)S), dim3(256), 0,
                           g.stream, data, scratch, sstride, scr_stride, Lf, L1, L2);
        hipLaunchKernelGGL(k_copy, grid1(nlines * Lf, S), dim3(256), 0, g.stream, scratch, data, scr_stride, sstride,
                           nlines * Lf);
        g.launches += 2;
    }
    return TIKH_OK;
}

// ---------------------------------------------------------------- recursion (Alg. 1)
template <int NR>
static void launch_leaf(const Plan& pl, const LeafArgs& la, const BuildArgs& ba, int64_t G, int slots) {
    const int waves = (pl.K + 63) / 64;           // one wavefront per 64 conditions (K <= 256)
    if (G >= g.opts.leaf_wave_groups && waves > 1) {
        // large batches: one wavefront per group does the per-step common work once
        if (waves == 2) LAUNCH("leaf_loop", (k_leaf_loop_sw<2, NR>), dim3((unsigned)G), dim3(64), la);
        else if (waves == 3) LAUNCH("leaf_loop", (k_leaf_loop_sw<3, NR>), dim3((unsigned)G), dim3(64), la);
        else LAUNCH("leaf_loop", (k_leaf_loop_sw<4, NR>), dim3((unsigned)G), dim3(64), la);
    } else {
        LAUNCH("leaf_loop", k_leaf_loop<NR>, dim3((unsigned)G), dim3(64 * waves), la);
    }
    // the basis is built with one slot of 64 coefficients per polynomial (the pivot rule keeps
    // the column degrees near K/4); a group with a column degree of 64 or more is flagged and
    // built by a second launch with `slots` slots that skips every other group
    const size_t shm = sizeof(LeafRec) * (size_t)pl.K;
    BuildArgs b1 = ba;
    b1.narrow = slots > 1;
    b1.wide_pass = 0;
    LAUNCH_SH("leaf_build", (k_leaf_build<1, NR>), dim3((unsigned)G), dim3(256), shm, b1);
    if (slots <= 1) return;
    BuildArgs b2 = ba;
    b2.narrow = 0;
    b2.wide_pass = 1;
    if (slots <= 2) LAUNCH_SH("leaf_build", (k_leaf_build<2, NR>), dim3((unsigned)G), dim3(256), shm, b2);
    else if (slots <= 3) LAUNCH_SH("leaf_build", (k_leaf_build<3, NR>), dim3((unsigned)G), dim3(256), shm, b2);
    else if (slots <= 4) LAUNCH_SH("leaf_build", (k_leaf_build<4, NR>), dim3((unsigned)G), dim3(256), shm, b2);
    else LAUNCH_SH("leaf_build", (k_leaf_build<5, NR>), dim3((unsigned)G), dim3(256), shm, b2);
}

static int run_leaf(const Plan& pl, const Layout& L, const Bufs& b, int64_t G, int t, double2* dst, int64_t dstride,
                    SlotMeta* dmeta, int64_t dcap, const double2* tw) {
    LeafArgs la{};
    la.sd = b.sd; la.st = b.st; la.phi = b.phi; la.phi_stride = L.sphi; la.rec = b.rec;
    la.rec_stride = pl.K; la.N = pl.N; la.M = pl.M; la.p = pl.p; la.K = pl.K; la.leaf = t; la.tw = tw; la.Q = pl.Q;
    la.defer_tol2 = defer_on() ? g.opts.defer_tol * g.opts.defer_tol : 0.0;
    la.dl = b.dl;
    BuildArgs ba{};
    ba.st = b.st; ba.rec = b.rec; ba.rec_stride = pl.K; ba.out = dst; ba.out_stride = dstride;
    ba.cap = dcap; ba.meta = dmeta; ba.K = pl.K;
    const int slots = (int)((std::min<int64_t>(dcap, pl.K) + 1 + 63) / 64);
    {
        // leaf-loop flops: at step c the K-c remaining rows are scored (4 |r|^2, 12 flops) and
        // K-c-1 are updated (C-1 complex multiply-adds, one complex multiply and subtract: 8C flops)
        const double K = (double)pl.K, C = (double)L.C;
        prof_units("leaf_loop", (double)G * (12.0 * K * (K + 1) / 2 + 8.0 * C * K * (K - 1) / 2));
    }
    if (L.nr == 1) launch_leaf<1>(pl, la, ba, G, slots);
    else if (L.nr == 2) launch_leaf<2>(pl, la, ba, G, slots);
    else launch_leaf<4>(pl, la, ba, G, slots);
    return TIKH_OK;
}

// Evaluate the completed left child (depth d, index idx) at the nodes of its
// right sibling and update the sibling subtree's residual data.
static int run_eval_chunk(const Plan& pl, const Layout& L, const Bufs& b, int64_t G, int d, int64_t idx,
                          const double2* tw) {
    const int64_t ridx = idx + 1;
    const int64_t oR = 2 * (int64_t)(d == 0 ? 0 : (int)(__builtin_bitreverse32((uint32_t)ridx) >> (32 - d)));
    const int64_t Lc = pl.N >> (d + 1);
    const int64_t cp1 = pl.cap[d] + 1;
    const int E = 4 * L.C;
    // the transform reads the twisted, folded basis entries directly from the slot
    FftArgs fu{};
    fu.load_mode = 2; fu.src = b.slotS[d]; fu.src_stride = L.sslot[d]; fu.src_cp1 = cp1; fu.src_meta = b.metaS[d];
    fu.C = L.C; fu.fold_L = Lc; fu.fold_o = oR; fu.fold_N = pl.N;
    int rc = fft_lines(b.V, G, L.sV, 2 * E, Lc, +1, tw, pl.Q, b.scr, L.sscr, FFT_FWD_T, &fu);
    if (rc) return rc;
    const int64_t L1 = fft_split(Lc);
    const int64_t nleaves = (int64_t)1 << (pl.p - d);
    const int64_t t0 = ridx << (pl.p - d);
    if (L.nr == 1)
        LAUNCH("eval_apply", k_eval_apply<1>, grid1(nleaves * pl.K / 2, G), dim3(256), b.phi, L.sphi, b.V, L.sV, Lc, L1, oR,
               d, t0, nleaves, pl.N, pl.M, pl.p, pl.K);
    else if (L.nr == 2)
        LAUNCH("eval_apply", k_eval_apply<2>, grid1(nleaves * pl.K / 2, G), dim3(256), b.phi, L.sphi, b.V, L.sV, Lc, L1, oR,
               d, t0, nleaves, pl.N, pl.M, pl.p, pl.K);
    else
        LAUNCH("eval_apply", k_eval_apply<4>, grid1(nleaves * pl.K / 2, G), dim3(256), b.phi, L.sphi, b.V, L.sV, Lc, L1, oR,
               d, t0, nleaves, pl.N, pl.M, pl.p, pl.K);
    return TIKH_OK;
}

// B_parent = B_L B_R for the parent at depth dp (children at depth dp+1), one merge chunk.
static int run_product_chunk(const Plan& pl, const Layout& L, const Bufs& b, int64_t G, int dp, int64_t pidx,
                             double2* dst, int64_t dstride, SlotMeta* dmeta, int64_t dcap, const double2* tw) {
    const int dc = dp + 1;
    const int C = L.C, nr = L.nr;
    int64_t P = pl.P[dp];
    const int64_t site = ((int64_t)dp << 40) | pidx;
    auto known = g.cur_sizes ? g.cur_sizes->P.find(site) : std::map<int64_t, int64_t>::iterator();
    if (g.replay && g.cur_sizes && known != g.cur_sizes->P.end()) {
        // recorded length: checked on the device against this chunk's degrees
        P = known->second;
        hipLaunchKernelGGL(k_deg_check, dim3(1), dim3(256), 0, g.stream, b.metaS[dc], b.metaT[dc], (int)G, C, (int)P,
                           g.overflow);
        g.launches += 1;
    } else {
        // size the transforms by the actual degrees of this chunk (host readback)
        int hword = 0;
        int* dneed = g.noalloc ? g.ndneed : g.dneed;
        int* hneed = g.noalloc ? &hword : g.hneed;
        if (!dneed || !hneed) return TIKH_ENOMEM;
        hipLaunchKernelGGL(k_deg_need, dim3(1), dim3(256), 0, g.stream, b.metaS[dc], b.metaT[dc], (int)G, C, dneed);
        HIPCHK(hipMemcpyAsync(hneed, dneed, sizeof(int), hipMemcpyDeviceToHost, g.stream));
        HIPCHK(hipStreamSynchronize(g.stream));
        g.launches += 1;
        g.syncs += 1;
        const int64_t need = std::max<int64_t>(1, (int64_t)*hneed);
        if (need <= P) P = smallest_divisor_geq(pl.Q, need);
        if (P > pl.P[dp]) P = pl.P[dp];
        if (g.cur_sizes) {
            int64_t& rec = g.cur_sizes->P[site];
            int64_t keep = g.opts.record_short ? smallest_divisor_geq(pl.Q, std::max<int64_t>(1, need / 2)) : P;
            if (g.headroom && !g.opts.record_short)
                keep = std::min(pl.P[dp], smallest_divisor_geq(pl.Q, need + need / 8 + 8));
            rec = std::max(rec, g.headroom ? keep : std::min(keep, P));
        }
    }
    const int64_t cp1 = pl.cap[dc] + 1;
    const bool root = (dp == 0);
    // the root forms row 0 only: the solution columns, or every column when deferred
    // conditions are still to be processed against it
    const bool full_root = root && defer_on();
    // only the left factor's B0 block is transformed: its V block is added to the
    // coefficients of the product by the inverse transform's store
    const int nL = root ? 4 : 16, nR = root && !full_root ? 4 * nr : 4 * C, nO = root ? (full_root ? C : nr) : 4 * C;
    const int* eL = b.elist + (root ? offsetof(EList, row0b0) : offsetof(EList, b0)) / sizeof(int);
    const int* eR = b.elist + (root && !full_root ? offsetof(EList, vcols) : offsetof(EList, all)) / sizeof(int);
    const int* eO = b.elist + (root ? (full_root ? offsetof(EList, row0) : offsetof(EList, xout)) : offsetof(EList, all)) /
                    sizeof(int);
    const int pmode = full_root ? 2 : (root ? 1 : 0);
    hipLaunchKernelGGL(k_prod_meta, dim3((unsigned)((G + 63) / 64)), dim3(64), 0, g.stream, b.metaS[dc], b.metaT[dc],
                       dmeta, b.st, dcap, (int)G, C);
    g.launches += 1;
    // forward transforms read the zero-padded, column-scaled entries directly from the slots
    FftArgs fl{};
    fl.load_mode = 1; fl.src = b.slotS[dc]; fl.src_stride = L.sslot[dc]; fl.src_cp1 = cp1; fl.src_meta = b.metaS[dc];
    fl.elist = eL; fl.C = C;
    int rc = fft_lines(b.FL, G, L.sF, nL, P, -1, tw, pl.Q, b.scr, L.sscr, FFT_FWD_T, &fl);
    if (rc) return rc;
    FftArgs fr{};
    fr.load_mode = 1; fr.src = b.slotT[dc]; fr.src_stride = L.sT; fr.src_cp1 = cp1; fr.src_meta = b.metaT[dc];
    fr.elist = eR; fr.C = C;
    rc = fft_lines(b.FR, G, L.sF, nR, P, -1, tw, pl.Q, b.scr, L.sscr, FFT_FWD_T, &fr);
    if (rc) return rc;
    // the pointwise product reads every input of a frequency before writing, so it runs in place over FL
    if (nr == 1) LAUNCH("prod_mul", k_prod_mul<1>, grid1(P, G, 64), dim3(64), b.FL, b.FR, b.FL, L.sF, P, pmode);
    else if (nr == 2) LAUNCH("prod_mul", k_prod_mul<2>, grid1(P, G, 64), dim3(64), b.FL, b.FR, b.FL, L.sF, P, pmode);
    else LAUNCH("prod_mul", k_prod_mul<4>, grid1(P, G, 64), dim3(64), b.FL, b.FR, b.FL, L.sF, P, pmode);
    // the inverse transform writes the truncated, 1/P-scaled coefficients into the destination slot
    FftArgs fo{};
    fo.store_mode = 1; fo.dst = dst; fo.dst_stride = dstride; fo.dst_cp1 = dcap + 1; fo.dst_meta = dmeta;
    fo.dst_elist = eO; fo.C = C; fo.dst_scale = 1.0 / (double)P;
    fo.add_src = b.slotS[dc]; fo.add_stride = L.sslot[dc]; fo.add_cp1 = cp1; fo.add_meta = b.metaS[dc];
    rc = fft_lines(b.FL, G, L.sF, nO, P, +1, tw, pl.Q, b.scr, L.sscr, FFT_INV_T, &fo);
    if (rc) return rc;
    return TIKH_OK;
}

// direct evaluation in two passes: groups that fit the narrow LDS budget, then the flagged rest
template <int NR>
static void launch_eval_direct(const Plan& pl, const Layout& L, const Bufs& b, int64_t G, int d, int64_t t0,
                               int64_t nleaves, const double2* tw) {
    LAUNCH("eval_direct", (k_eval_direct<NR, ED_LDS_NARROW, 1>), dim3((unsigned)G), dim3(256), b.phi, L.sphi,
           b.slotS[d], L.sslot[d], pl.cap[d] + 1, b.metaS[d], t0, nleaves, pl.N, pl.M, pl.p, pl.K, tw, pl.Q, b.st);
    LAUNCH("eval_direct", (k_eval_direct<NR, ED_LDS, 2>), dim3((unsigned)G), dim3(256), b.phi, L.sphi,
           b.slotS[d], L.sslot[d], pl.cap[d] + 1, b.metaS[d], t0, nleaves, pl.N, pl.M, pl.p, pl.K, tw, pl.Q, b.st);
}

static int run_eval(const Plan& pl, const Layout& L, const Bufs& b, int64_t G, int d, int64_t idx, const double2* tw) {
    if (d == pl.p || ((2 * pl.N) >> d) <= DIRECT_MAX_COND) {
        const int64_t ridx = idx + 1;
        const int64_t nleaves = (int64_t)1 << (pl.p - d);
        const int64_t t0 = ridx << (pl.p - d);
        if (L.nr == 1) launch_eval_direct<1>(pl, L, b, G, d, t0, nleaves, tw);
        else if (L.nr == 2) launch_eval_direct<2>(pl, L, b, G, d, t0, nleaves, tw);
        else launch_eval_direct<4>(pl, L, b, G, d, t0, nleaves, tw);
        return TIKH_OK;
    }
    // the scratch pool is split for this level: as many groups per launch as fit
    Layout Ld = L;
    Ld.sV = 2 * (int64_t)(4 * L.C) * (pl.N >> (d + 1));
    const int64_t ch = std::max<int64_t>(1, std::min<int64_t>(G, b.pool_elems / Ld.sV));
    for (int64_t c0 = 0; c0 < G; c0 += ch) {
        Bufs bc = shift_bufs(b, L, pl, c0);
        bc.V = b.pool;
        int rc = run_eval_chunk(pl, Ld, bc, std::min(ch, G - c0), d, idx, tw);
        if (rc) return rc;
    }
    return TIKH_OK;
}

// dst / dmeta are given for group 0 with per-group stride dstride
static int run_product(const Plan& pl, const Layout& L, const Bufs& b, int64_t G, int dp, int64_t pidx, double2* dst,
                       int64_t dstride, SlotMeta* dmeta, int64_t dcap, const double2* tw) {
    const int dc = dp + 1;
    if (defer_on()) {
        // deferred conditions of this subtree: residuals with respect to the product (Sec. 5)
        const int64_t nl = (int64_t)1 << (pl.p - dp), lo = pidx * nl, mid = lo + nl / 2, hi = lo + nl;
        if (L.nr == 1)
            LAUNCH("defer_update", k_defer_update<1>, dim3((unsigned)G), dim3(256), b.dl, b.st, b.metaS[dc],
                   b.slotT[dc], L.sT, pl.cap[dc] + 1, b.metaT[dc], pl.K, lo, mid, hi);
        else if (L.nr == 2)
            LAUNCH("defer_update", k_defer_update<2>, dim3((unsigned)G), dim3(256), b.dl, b.st, b.metaS[dc],
                   b.slotT[dc], L.sT, pl.cap[dc] + 1, b.metaT[dc], pl.K, lo, mid, hi);
        else
            LAUNCH("defer_update", k_defer_update<4>, dim3((unsigned)G), dim3(256), b.dl, b.st, b.metaS[dc],
                   b.slotT[dc], L.sT, pl.cap[dc] + 1, b.metaT[dc], pl.K, lo, mid, hi);
    }
    if (dp > 0 && dc == pl.p) {
        // two passes: groups whose factors fit the narrow LDS budget, then the flagged rest
        LAUNCH("prod_direct", (k_prod_direct<PD_LDS_NARROW, 1>), dim3((unsigned)G), dim3(256), b.slotS[dc], L.sslot[dc],
               pl.cap[dc] + 1, b.metaS[dc], b.slotT[dc], L.sT, pl.cap[dc] + 1, b.metaT[dc], dst, dstride, dcap + 1,
               dmeta, b.st, L.C);
        LAUNCH("prod_direct", (k_prod_direct<PD_LDS, 2>), dim3((unsigned)G), dim3(256), b.slotS[dc], L.sslot[dc],
               pl.cap[dc] + 1, b.metaS[dc], b.slotT[dc], L.sT, pl.cap[dc] + 1, b.metaT[dc], dst, dstride, dcap + 1,
               dmeta, b.st, L.C);
        return TIKH_OK;
    }
    // the scratch pool is split for this level: FL and FR hold the largest
    // operand set at the level's bound on the product length
    Layout Ld = L;
    const int64_t lines = dp == 0 && !defer_on() ? std::max<int64_t>(L.C, 4 * L.nr) : 4 * L.C;
    Ld.sF = lines * pl.P[dp];
    const int64_t ch = std::max<int64_t>(1, std::min<int64_t>(G, b.pool_elems / (2 * Ld.sF)));
    for (int64_t c0 = 0; c0 < G; c0 += ch) {
        Bufs bc = shift_bufs(b, L, pl, c0);
        bc.FL = b.pool;
        bc.FR = b.pool + ch * Ld.sF;
        int rc = run_product_chunk(pl, Ld, bc, std::min(ch, G - c0), dp, pidx, dst + c0 * dstride, dstride,
                                   dmeta + c0, dcap, tw);
        if (rc) return rc;
    }
    return TIKH_OK;
}

static int run_recursion(const Plan& pl, const Layout& L, const Bufs& b, int64_t G, const double2* tw) {
    const int p = pl.p;
    const int64_t nleaf = (int64_t)1 << p;
    for (int64_t t = 0; t < nleaf; ++t) {
        double2* dst;
        int64_t dstr;
        SlotMeta* dm;
        if (p == 0) { dst = b.slotT[0]; dm = b.metaT[0]; dstr = L.sT; }
        else if (t & 1) { dst = b.slotT[p]; dm = b.metaT[p]; dstr = L.sT; }
        else { dst = b.slotS[p]; dm = b.metaS[p]; dstr = L.sslot[p]; }
        int rc = run_leaf(pl, L, b, G, (int)t, dst, dstr, dm, pl.cap[p], tw);
        if (rc) return rc;
        int d = p;
        int64_t idx = t;
        while (d > 0) {
            if ((idx & 1) == 0) {
                rc = run_eval(pl, L, b, G, d, idx, tw);
                if (rc) return rc;
                break;
            }
            const int dp = d - 1;
            const int64_t pidx = idx >> 1;
            double2* pdst;
            int64_t pstr;
            SlotMeta* pm;
            if (dp == 0 || (pidx & 1)) { pdst = b.slotT[dp]; pm = b.metaT[dp]; pstr = L.sT; }
            else { pdst = b.slotS[dp]; pm = b.metaS[dp]; pstr = L.sslot[dp]; }
            rc = run_product(pl, L, b, G, dp, pidx, pdst, pstr, pm, pl.cap[dp], tw);
            if (rc) return rc;
            d = dp;
            idx = pidx;
        }
    }
    return TIKH_OK;
}

// circulant products on length-N per-solve buffers (symbol from the group)
static void circ_apply(const Plan& pl, const Layout& L, const Bufs& b, int64_t S, double2* buf, int mode,
                       const double2* tw, const double2* symbol = nullptr) {
    fft_lines(buf, S, L.sN, 1, pl.N, +1, tw, pl.Q, b.bS, L.sN);
    hipLaunchKernelGGL(k_mul_symbol, grid1(pl.N, S), dim3(256), 0, g.stream, b.sd, L.nr, symbol ? symbol : b.chat, buf,
                       pl.N, L.sN, mode, tw, pl.Q);
    fft_lines(buf, S, L.sN, 1, pl.N, -1, tw, pl.Q, b.bS, L.sN);
    g.launches++;
}

// Key of a chunk's composition for the recorded product lengths: the plan, the
// right-hand sides per group, the deferral threshold and every group's operator
// (sizes, extension, element type, entry, variant, lambda).
static uint64_t sizes_key(const Plan& pl, int nr, const std::vector<SolveDesc>& sds) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](uint64_t v) {
        for (int i = 0; i < 8; ++i) { h ^= (v >> (8 * i)) & 0xffu; h *= 1099511628211ull; }
    };
    auto bits = [](double v) { uint64_t u; memcpy(&u, &v, 8); return u; };
    mix((uint64_t)pl.N); mix((uint64_t)pl.M); mix((uint64_t)pl.p); mix((uint64_t)nr); mix(sds.size());
    mix(bits(g.opts.defer_tol));
    for (size_t i = 0; i < sds.size(); i += (size_t)nr) {
        const SolveDesc& d = sds[i];
        mix((uint64_t)d.m); mix((uint64_t)d.n); mix((uint64_t)d.k); mix(bits(d.lam));
        mix((uint64_t)(d.cplx | (d.mode << 1) | (d.gramian << 2) | (d.backward << 3)));
    }
    return h;
}

static const int TIKH_RESIZE = 100;   // internal: a recorded product length was too short

// One chunk of groups sharing the plan (sds holds G*nr solves, group-major), run in
// phases so that chunks of different plans can proceed side by side on their own
// streams: chunk_begin, chunk_adapt until done, chunk_finish, chunk_check.  With
// use_sizes, product lengths recorded for this composition are reused (the first
// recursion records them if there are none yet); chunk_check returns TIKH_RESIZE if the
// device found a recorded length too short, after which the chunk must run again.
struct ChunkRun {
    Plan pl;
    int nr = 1;
    std::vector<SolveDesc> sds;
    int32_t* info = nullptr;
    int64_t mchunk = 1;
    bool use_sizes = true;
    hipStream_t stream = nullptr;
    char* base = nullptr;                // workspace region (chunk_bytes long)
    Layout L;
    Bufs b;
    const double2* tw = nullptr;
    int64_t S = 0, G = 0, Ga = 0, Sa = 0, mmax = 1, nmax = 1;
    bool gramian = false, replayed = false, done = false;
    int steps_min = 1, steps_max = 1, it = 0;
    bool fixed_steps = false;            // prepared batches: no adaptive steps (no host decisions)
    Ctx::Sizes* sizes = nullptr;
    std::vector<SolveDesc> failed;       // descriptors of the groups whose solve failed
};

static void chunk_layout(ChunkRun& r) {
    r.mmax = 1; r.nmax = 1;
    for (auto& d : r.sds) { r.mmax = std::max(r.mmax, d.m); r.nmax = std::max(r.nmax, d.n); }
    make_layout(r.pl, r.nr, r.mmax, r.nmax, &r.L);
}
static size_t chunk_run_bytes(const ChunkRun& r) {
    const int64_t G = (int64_t)r.sds.size() / r.nr;
    return chunk_bytes(r.L, G, std::min<int64_t>(G, r.mchunk));
}
// the chunk's stream and recorded lengths become the library's current ones
static void chunk_enter(ChunkRun& r) {
    g.stream = r.stream;
    g.cur_sizes = r.sizes;
    g.overflow = r.b.ovf;
}

// Residual of the normal equations of the first Sa solves into b.t1: r = y - (T^H T + lam^2) x
// (Sec. 7.2: iterative refinement); Toeplitz-Gramian problem: r = y - (L^H L + G) x, with G x
// (bC) from the Gramian's circulant.
static void chunk_residual(ChunkRun& r) {
    const Plan& pl = r.pl;
    const Layout& L = r.L;
    const Bufs& b = r.b;
    const double2* tw = r.tw;
    const int64_t Sa = r.Sa, mmax = r.mmax, nmax = r.nmax, N = pl.N;
    const double invN = 1.0 / (double)N;
    const bool gramian = r.gramian;
    if (gramian) {
        hipLaunchKernelGGL(k_load_pad, grid1(N, Sa), dim3(256), 0, g.stream, b.sd, 0, b.xacc, L.sn, 1, 0, 1.0,
                           b.bB, N, L.sN);
        circ_apply(pl, L, b, Sa, b.bB, 0, tw, b.cg);
        hipLaunchKernelGGL(k_take_tail, grid1(nmax, Sa), dim3(256), 0, g.stream, b.sd, b.bB, N, L.sN, 1, invN,
                           b.bC, L.sN);
        g.launches += 2;
    }
    hipLaunchKernelGGL(k_load_pad, grid1(N, Sa), dim3(256), 0, g.stream, b.sd, 0, b.xacc, L.sn, 1, 0, 1.0,
                       b.bB, N, L.sN);
    circ_apply(pl, L, b, Sa, b.bB, 0, tw);
    hipLaunchKernelGGL(k_take_tail, grid1(mmax, Sa), dim3(256), 0, g.stream, b.sd, b.bB, N, L.sN, 0, invN,
                       b.t1, L.sn);
    hipLaunchKernelGGL(k_load_pad, grid1(N, Sa), dim3(256), 0, g.stream, b.sd, 0, b.t1, L.sn, 0, 0, 1.0, b.bB,
                       N, L.sN);
    circ_apply(pl, L, b, Sa, b.bB, 1, tw);
    hipLaunchKernelGGL(k_take_tail, grid1(nmax, Sa), dim3(256), 0, g.stream, b.sd, b.bB, N, L.sN, 1, invN,
                       b.t2, L.sn);
    hipLaunchKernelGGL(k_normal_residual, grid1(nmax, Sa), dim3(256), 0, g.stream, b.sd, b.yv, b.t2, b.xacc,
                       b.t1, L.sn, gramian ? (const double2*)b.bC : (const double2*)nullptr, L.sN);
    g.launches += 5;
}

// Moves the groups flagged in hflags[0, Ga) to the front of the chunk (exchanging each with an
// unflagged group of that prefix: descriptors, state, symbols, right-hand side, solution)
// and makes them the active prefix.
static int compact_groups(ChunkRun& r, const std::vector<int32_t>& hflags) {
    Bufs& b = r.b;
    const Layout& L = r.L;
    const int64_t Ga = r.Ga;
    std::vector<int64_t> want, holes;
    int64_t G2 = 0;
    for (int64_t gi = 0; gi < Ga; ++gi) G2 += hflags[gi] ? 1 : 0;
    for (int64_t gi = 0; gi < G2; ++gi) if (!hflags[gi]) holes.push_back(gi);
    for (int64_t gi = G2; gi < Ga; ++gi) if (hflags[gi]) want.push_back(gi);
    if (!holes.empty()) {
        std::vector<int2> hp(holes.size());
        for (size_t i = 0; i < holes.size(); ++i) hp[i] = make_int2((int)holes[i], (int)want[i]);
        HIPCHK(hipMemcpyAsync(b.pairs, hp.data(), sizeof(int2) * hp.size(), hipMemcpyHostToDevice, g.stream));
        HIPCHK(hipStreamSynchronize(g.stream));
        g.syncs += 1;
        hipLaunchKernelGGL(k_swap_groups, dim3(64, (unsigned)hp.size()), dim3(256), 0, g.stream, b.sd, b.st, b.chat,
                           L.sN, b.yv, b.xacc, L.sn, r.nr, b.pairs, r.gramian ? b.cg : nullptr, b.asum);
        g.launches++;
    }
    r.Ga = G2;
    r.Sa = G2 * r.nr;
    return TIKH_OK;
}

// Before the first refinement step: the groups whose first solve the a-posteriori bound
// already certifies to refine_tol (k_refine_bound) take no refinement step (one host
// synchronization for the decisions).  Not for the Toeplitz-Gramian problem (A >= lam^2 I
// does not hold there) nor for prepared batches (no host decisions).
static bool filter_on(const ChunkRun& r) { return g.opts.refine_skip && !r.gramian && !r.fixed_steps; }
static int chunk_filter(ChunkRun& r) {
    if (r.Ga == 0) return TIKH_OK;
    chunk_residual(r);
    hipLaunchKernelGGL(k_refine_bound, dim3((unsigned)r.Ga), dim3(256), 0, g.stream, r.b.sd, r.nr, r.b.chat, r.L.sN,
                       r.pl.N, r.b.t1, r.b.xacc, r.L.sn, g.opts.refine_tol, r.b.flags);
    g.launches++;
    std::vector<int32_t> hflags((size_t)r.Ga);
    HIPCHK(hipMemcpyAsync(hflags.data(), r.b.flags, sizeof(int32_t) * r.Ga, hipMemcpyDeviceToHost, g.stream));
    HIPCHK(hipStreamSynchronize(g.stream));
    g.syncs += 1;
    const int64_t before = r.Sa;
    int rc = compact_groups(r, hflags);
    g.stats.refine_skipped += before - r.Sa;
    return rc;
}

// One solve of the chunk's current right-hand sides (it = 0: y; it > 0: the
// refinement residual of the solutions so far) over its first Ga groups.
static int chunk_step(ChunkRun& r, int it) {
    const Plan& pl = r.pl;
    const Layout& L = r.L;
    const Bufs& b = r.b;
    const double2* tw = r.tw;
    const int nr = r.nr;
    const int64_t Ga = r.Ga, Sa = r.Sa, mmax = r.mmax, nmax = r.nmax, N = pl.N;
    const double invN = 1.0 / (double)N;
    const bool gramian = r.gramian;
    const int steps_max = r.steps_max;
    int rc = TIKH_OK;
    const double2* rhs = b.yv;
    if (it > 0) {
        chunk_residual(r);
        hipLaunchKernelGGL(k_init_state, dim3((unsigned)((Ga + 63) / 64)), dim3(64), 0, g.stream, b.sd, nr, b.st,
                           (int)Ga, 1);
        hipLaunchKernelGGL(k_zero_d, grid1(2 * Sa, 1), dim3(256), 0, g.stream, b.nrm, 2 * Sa);
        g.launches += 2;
        rhs = b.t1;
    }
    hipLaunchKernelGGL(k_load_pad, grid1(N, Sa), dim3(256), 0, g.stream, b.sd, 0, rhs, L.sn, 1, 0, 1.0, b.bA, N,
                       L.sN);
    g.launches++;
    rc = fft_lines(b.bA, Sa, L.sN, 1, N, +1, tw, pl.Q, b.bS, L.sN);
    if (rc) return rc;
    hipLaunchKernelGGL(k_assemble, grid1(2 * N, Ga), dim3(256), 0, g.stream, b.sd, nr, b.chat, b.bA, L.sN, b.phi,
                       L.sphi, N, pl.M, pl.p, pl.K, tw, pl.Q, (const double2*)b.cg);
    g.launches++;
    g.replay = g.cur_sizes && g.cur_sizes->complete;
    r.replayed |= g.replay;
    rc = run_recursion(pl, L, b, Ga, tw);
    g.replay = false;
    if (rc) return rc;
    if (g.cur_sizes) g.cur_sizes->complete = true;   // every merge of the tree has been sized
    const int64_t xcp1 = pl.cap[0] + 1;
    if (defer_on()) {
        // deferred conditions, one step each on the final basis (Sec. 5)
        if (nr == 1)
            LAUNCH("defer_complete", k_defer_complete<1>, dim3((unsigned)Ga), dim3(256), b.dl, b.st, b.slotT[0],
                   L.sT, xcp1, b.metaT[0]);
        else if (nr == 2)
            LAUNCH("defer_complete", k_defer_complete<2>, dim3((unsigned)Ga), dim3(256), b.dl, b.st, b.slotT[0],
                   L.sT, xcp1, b.metaT[0]);
        else
            LAUNCH("defer_complete", k_defer_complete<4>, dim3((unsigned)Ga), dim3(256), b.dl, b.st, b.slotT[0],
                   L.sT, xcp1, b.metaT[0]);
        // count them for the statistics
        std::vector<SolveState> hst((size_t)Ga);
        HIPCHK(hipMemcpyAsync(hst.data(), b.st, sizeof(SolveState) * Ga, hipMemcpyDeviceToHost, g.stream));
        HIPCHK(hipStreamSynchronize(g.stream));
        for (const SolveState& x : hst) g.stats.deferred += x.ndef;
    }
    hipLaunchKernelGGL(k_extract, grid1(nmax, Sa), dim3(256), 0, g.stream, b.sd, nr, b.st, b.slotT[0], L.sT,
                       xcp1, b.metaT[0], b.xacc, L.sn, it > 0 ? 1 : 0, b.nrm);
    g.launches++;
    if (it > 0 && it + 1 < steps_max) {
        hipLaunchKernelGGL(k_refine_decide, dim3((unsigned)((Ga + 63) / 64)), dim3(64), 0, g.stream, b.nrm, nr,
                           b.st, (int)Ga, it == 1 ? 1 : 0, REFINE_CFAC, g.opts.refine_tol, b.flags);
        g.launches++;
    }
    return TIKH_OK;
}

// Uploads the chunk, builds its symbols and right-hand sides and runs the steps every
// group takes (the solve and `refine` refinement steps).  Device work goes to r.stream.
// Carves the chunk's buffers from its workspace region and uploads its descriptors.
static int chunk_upload(ChunkRun& r) {
    const Plan& pl = r.pl;
    const int nr = r.nr;
    r.S = (int64_t)r.sds.size();
    r.G = r.S / nr;
    int rc = carve_bufs(pl, r.L, r.G, std::min<int64_t>(r.G, r.mchunk), r.base, &r.b);
    if (rc) return rc;
    r.tw = twiddles(pl.Q);
    if (!r.tw) return TIKH_ENOMEM;
    const EList el = make_elist(nr);
    HIPCHK(hipMemcpyAsync(r.b.sd, r.sds.data(), sizeof(SolveDesc) * r.S, hipMemcpyHostToDevice, g.stream));
    HIPCHK(hipMemcpyAsync(r.b.elist, &el, sizeof(EList), hipMemcpyHostToDevice, g.stream));
    return TIKH_OK;
}

static int chunk_setup(ChunkRun& r);

static int chunk_begin(ChunkRun& r) {
    int rc = chunk_upload(r);
    if (rc) return rc;
    if (g.sizes.size() > 4096) g.sizes.clear();   // bound the record over many compositions
    r.sizes = r.use_sizes ? &g.sizes[sizes_key(r.pl, r.nr, r.sds)] : nullptr;
    return chunk_setup(r);
}

// Builds the uploaded chunk's symbols and right-hand sides and runs the steps every
// group takes; only kernel launches unless transform lengths are read back (a first
// call of a composition).
static int chunk_setup(ChunkRun& r) {
    const Plan& pl = r.pl;
    const int nr = r.nr;
    const std::vector<SolveDesc>& sds = r.sds;
    const int64_t S = r.S, G = r.G;
    int rc = TIKH_OK;
    const Layout& L = r.L;
    Bufs& b = r.b;
    const double2* tw = r.tw;
    const int64_t mmax = r.mmax, nmax = r.nmax;
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, g.stream, b.ovf, (int64_t)1);
    g.launches++;
    g.cur_sizes = r.sizes;
    g.overflow = b.ovf;
    const int64_t N = pl.N;
    const double invN = 1.0 / (double)N;
    hipLaunchKernelGGL(k_init_state, dim3((unsigned)((G + 63) / 64)), dim3(64), 0, g.stream, b.sd, nr, b.st, (int)G, 0);
    // extension (eq. (circexp)) and its symbol c^ = F c_T (eq. (circdiag)), per group
    hipLaunchKernelGGL(k_gen_rms, dim3((unsigned)G), dim3(256), 0, g.stream, b.sd, nr, b.rms, b.asum);
    hipLaunchKernelGGL(k_build_ct, grid1(N, G), dim3(256), 0, g.stream, b.sd, nr, b.rms, b.chat, N, L.sN);
    g.launches += 3;
    rc = fft_lines(b.chat, G, L.sN, 1, N, +1, tw, pl.Q, b.bS, L.sN);
    if (rc) return rc;
    const bool gramian = sds[0].gramian != 0;
    if (gramian) {
        // Toeplitz-Gramian problem: the extended Gramian's symbol (Sec. 3.4)
        hipLaunchKernelGGL(k_gram_rms, dim3((unsigned)G), dim3(256), 0, g.stream, b.sd, nr, b.rmsg);
        hipLaunchKernelGGL(k_build_cg, grid1(N, G), dim3(256), 0, g.stream, b.sd, nr, b.rmsg, b.cg, N, L.sN);
        g.launches += 2;
        rc = fft_lines(b.cg, G, L.sN, 1, N, +1, tw, pl.Q, b.bS, L.sN);
        if (rc) return rc;
    }
    // right-hand side y = T^H b as the bottom n entries of C_k(T^H) [b; 0], per solve
    const bool normal = sds[0].mode == 1;
    if (!normal) {
        hipLaunchKernelGGL(k_load_pad, grid1(N, S), dim3(256), 0, g.stream, b.sd, 0, (const double2*)nullptr, 0, 0,
                           0, 1.0, b.bB, N, L.sN);
        circ_apply(pl, L, b, S, b.bB, 1, tw);
        hipLaunchKernelGGL(k_take_tail, grid1(nmax, S), dim3(256), 0, g.stream, b.sd, b.bB, N, L.sN, 1, invN, b.yv,
                           L.sn);
    } else {
        hipLaunchKernelGGL(k_load_pad, grid1(nmax, S), dim3(256), 0, g.stream, b.sd, 0, (const double2*)nullptr, 0, 1,
                           0, 1.0, b.yv, nmax, L.sn);
    }
    g.launches += 2;
    r.gramian = gramian;
    // Refinement: `refine` steps for every group, then up to `refine_max` steps in
    // all for the groups whose estimated error is still above refine_tol (chunk_adapt).
    r.steps_min = 1 + std::max(0, std::min(4, (int)g.opts.refine));
    r.steps_max = g.opts.refine > 0 ? std::max(r.steps_min, 1 + std::min(4, (int)g.opts.refine_max)) : r.steps_min;
    if (r.fixed_steps) r.steps_max = r.steps_min;
    r.done = false;
    r.Ga = G;
    r.Sa = S;
    // with the a-posteriori filter the refinement steps are taken in chunk_adapt
    const int upfront = filter_on(r) ? 1 : r.steps_min;
    for (r.it = 0; r.it < upfront; ++r.it) {
        rc = chunk_step(r, r.it);
        if (rc) return rc;
    }
    return TIKH_OK;
}

// One adaptive refinement step: the groups whose estimated error is still above
// refine_tol are exchanged into a prefix [0, Ga) and take another step (one host
// synchronization for the decisions).  Sets r.done when no group needs one.
static int chunk_adapt(ChunkRun& r) {
    if (r.done) return TIKH_OK;
    if (r.it < r.steps_min) {
        // a refinement step every group takes, unless the bound certified it before the first
        if (r.it == 1) {
            int rc = chunk_filter(r);
            if (rc) return rc;
            if (r.Ga == 0) { r.done = true; return TIKH_OK; }
        }
        int rc = chunk_step(r, r.it);
        r.it++;
        return rc;
    }
    if (r.it >= r.steps_max) {
        if (r.it > 1) {
            // the groups that took the last step: did their refinement fail (estimate above 1e-4)?
            hipLaunchKernelGGL(k_refine_decide, dim3((unsigned)((r.Ga + 63) / 64)), dim3(64), 0, g.stream, r.b.nrm,
                               r.nr, r.b.st, (int)r.Ga, r.it == 2 ? 1 : 0, REFINE_CFAC, REFINE_FAIL,
                               (int32_t*)nullptr);
            g.launches++;
        }
        r.done = true;
        return TIKH_OK;
    }
    Bufs& b = r.b;
    const int64_t Ga = r.Ga;
    std::vector<int32_t> hflags;
    {
        // groups still above the tolerance after the last step
        hflags.resize((size_t)Ga);
        HIPCHK(hipMemcpyAsync(hflags.data(), b.flags, sizeof(int32_t) * Ga, hipMemcpyDeviceToHost, g.stream));
        HIPCHK(hipStreamSynchronize(g.stream));
        g.syncs += 1;
        int64_t G2 = 0;
        for (int64_t gi = 0; gi < Ga; ++gi) G2 += hflags[gi] ? 1 : 0;
        if (G2 == 0) { r.done = true; return TIKH_OK; }
        int rc = compact_groups(r, hflags);
        if (rc) return rc;
        g.stats.refine_extra += r.Sa;
    }
    int rc = chunk_step(r, r.it);
    r.it++;
    return rc;
}

// Results: x and info (forward), or the gradients of the adjoint.
static int chunk_finish(ChunkRun& r) {
    const Plan& pl = r.pl;
    const Layout& L = r.L;
    const Bufs& b = r.b;
    const double2* tw = r.tw;
    const int nr = r.nr;
    const int64_t S = r.S, mmax = r.mmax, nmax = r.nmax, N = pl.N;
    const double invN = 1.0 / (double)N;
    const std::vector<SolveDesc>& sds = r.sds;
    int32_t* info = r.info;
    int rc = TIKH_OK;
    if (!sds[0].backward) {
        if (info) {
            hipLaunchKernelGGL(k_clear_info, dim3((unsigned)((S + 255) / 256)), dim3(256), 0, g.stream, b.sd, S, info);
            g.launches++;
        }
        hipLaunchKernelGGL(k_store_x, grid1(nmax, S), dim3(256), 0, g.stream, b.sd, nr, b.xacc, L.sn, b.st, info);
        g.launches++;
    } else {
        // adjoint: xacc holds w = (T^H T + lam^2 I)^{-1} gx
        const int64_t lmax = std::max(mmax, nmax);
        // X = F[x; 0]; T x = tail_m(F^-1(c^ X)) / N; r = b - T x  (t1)
        hipLaunchKernelGGL(k_load_pad, grid1(N, S), dim3(256), 0, g.stream, b.sd, 2, (const double2*)nullptr, 0, 1, 0,
                           1.0, b.bA, N, L.sN);
        rc = fft_lines(b.bA, S, L.sN, 1, N, +1, tw, pl.Q, b.bS, L.sN);
        if (rc) return rc;
        hipLaunchKernelGGL(k_copy, grid1(N, S), dim3(256), 0, g.stream, b.bA, b.bB, L.sN, L.sN, N);
        hipLaunchKernelGGL(k_mul_symbol, grid1(N, S), dim3(256), 0, g.stream, b.sd, nr, b.chat, b.bB, N, L.sN, 0, tw,
                           pl.Q);
        rc = fft_lines(b.bB, S, L.sN, 1, N, -1, tw, pl.Q, b.bS, L.sN);
        if (rc) return rc;
        hipLaunchKernelGGL(k_take_tail, grid1(mmax, S), dim3(256), 0, g.stream, b.sd, b.bB, N, L.sN, 0, invN, b.t2, L.sn);
        hipLaunchKernelGGL(k_sub_from_b, grid1(mmax, S), dim3(256), 0, g.stream, b.sd, b.t2, b.t1, L.sn);
        // W = F[w; 0]; T w = tail_m(F^-1(c^ W)) / N  (t2)
        hipLaunchKernelGGL(k_load_pad, grid1(N, S), dim3(256), 0, g.stream, b.sd, 0, b.xacc, L.sn, 1, 0, 1.0, b.bC, N,
                           L.sN);
        rc = fft_lines(b.bC, S, L.sN, 1, N, +1, tw, pl.Q, b.bS, L.sN);
        if (rc) return rc;
        hipLaunchKernelGGL(k_copy, grid1(N, S), dim3(256), 0, g.stream, b.bC, b.bB, L.sN, L.sN, N);
        hipLaunchKernelGGL(k_mul_symbol, grid1(N, S), dim3(256), 0, g.stream, b.sd, nr, b.chat, b.bB, N, L.sN, 0, tw,
                           pl.Q);
        rc = fft_lines(b.bB, S, L.sN, 1, N, -1, tw, pl.Q, b.bS, L.sN);
        if (rc) return rc;
        hipLaunchKernelGGL(k_take_tail, grid1(mmax, S), dim3(256), 0, g.stream, b.sd, b.bB, N, L.sN, 0, invN, b.t2, L.sn);
        // G^ = F[r;0] conj(W) - F[Tw;0] conj(X); lag sums = F^-1(G^) / N
        hipLaunchKernelGGL(k_load_pad, grid1(N, S), dim3(256), 0, g.stream, b.sd, 0, b.t1, L.sn, 0, 0, 1.0, b.bB, N,
                           L.sN);
        rc = fft_lines(b.bB, S, L.sN, 1, N, +1, tw, pl.Q, b.bS, L.sN);
        if (rc) return rc;
        hipLaunchKernelGGL(k_xcorr_spec, grid1(N, S), dim3(256), 0, g.stream, b.bB, b.bC, b.bB, N, L.sN, 0);
        hipLaunchKernelGGL(k_load_pad, grid1(N, S), dim3(256), 0, g.stream, b.sd, 0, b.t2, L.sn, 0, 0, 1.0, b.bC, N,
                           L.sN);
        rc = fft_lines(b.bC, S, L.sN, 1, N, +1, tw, pl.Q, b.bS, L.sN);
        if (rc) return rc;
        hipLaunchKernelGGL(k_xcorr_spec, grid1(N, S), dim3(256), 0, g.stream, b.bC, b.bA, b.bB, N, L.sN, 1);
        rc = fft_lines(b.bB, S, L.sN, 1, N, -1, tw, pl.Q, b.bS, L.sN);
        if (rc) return rc;
        hipLaunchKernelGGL(k_store_grads, grid1(2 * lmax + nmax, S), dim3(256), 0, g.stream, b.sd, b.bB, N, L.sN, invN,
                           b.t2, L.sn);
        hipLaunchKernelGGL(k_grad_lambda, dim3((unsigned)S), dim3(256), 0, g.stream, b.sd, nr, b.xacc, L.sn, b.st, info);
        g.launches += 14;
    }
    HIPCHK(hipGetLastError());
    return rc;
}

// After the chunk's stream has drained: were the recorded lengths long enough?
static int chunk_check(ChunkRun& r) {
    if (!r.replayed) return TIKH_OK;
    int hovf = 0;
    HIPCHK(hipMemcpyAsync(&hovf, r.b.ovf, sizeof(int), hipMemcpyDeviceToHost, r.stream));
    HIPCHK(hipStreamSynchronize(r.stream));
    g.syncs += 1;
    return hovf ? TIKH_RESIZE : TIKH_OK;
}

// Info bits of a failed solve (breakdown, degree bound, non-finite, refinement failure):
// such groups are solved again with the fallback leaf cutoff.
static const int32_t FAIL_BITS = 1 | 2 | 8 | 16;

// Condition number below which (by the bound 1 + (sum_s |a_s| / lambda)^2 >= kappa) a failed
// solve is solved again with the fallback leaf cutoff; above it the failure may be the
// conditioning itself, which another tree does not cure, and the flag stands.
static const double FALLBACK_KAPPA = 1e8;

// After the chunk's stream has drained: the descriptors (in their final order after the
// refinement's exchanges) of the groups whose solve failed and whose conditioning bound
// is below FALLBACK_KAPPA.
static int chunk_failed(ChunkRun& r) {
    r.failed.clear();
    std::vector<SolveState> st((size_t)r.G);
    std::vector<SolveDesc> sd((size_t)r.S);
    std::vector<double> asum((size_t)r.G);
    HIPCHK(hipMemcpyAsync(st.data(), r.b.st, sizeof(SolveState) * r.G, hipMemcpyDeviceToHost, r.stream));
    HIPCHK(hipMemcpyAsync(sd.data(), r.b.sd, sizeof(SolveDesc) * r.S, hipMemcpyDeviceToHost, r.stream));
    HIPCHK(hipMemcpyAsync(asum.data(), r.b.asum, sizeof(double) * r.G, hipMemcpyDeviceToHost, r.stream));
    HIPCHK(hipStreamSynchronize(r.stream));
    g.syncs += 1;
    for (int64_t gi = 0; gi < r.G; ++gi) {
        if (!(st[gi].info & FAIL_BITS)) continue;
        const SolveDesc& d = sd[gi * r.nr];
        // (the Gramian problem has no such bound at hand: always solved again)
        const double kb = 1.0 + (asum[gi] / d.lam) * (asum[gi] / d.lam);
        if (!d.gramian && !(kb <= FALLBACK_KAPPA)) continue;
        for (int q = 0; q < r.nr; ++q) r.failed.push_back(sd[gi * r.nr + q]);
    }
    return TIKH_OK;
}

// A chunk on its own: phases in order on the library stream; a chunk whose recorded
// lengths were too short runs again with read-back sizing.
static int run_chunk(ChunkRun& spec) {
    for (int attempt = 0; attempt < 2; ++attempt) {
        ChunkRun r;
        r.pl = spec.pl; r.nr = spec.nr; r.sds = spec.sds; r.info = spec.info; r.mchunk = spec.mchunk;
        r.use_sizes = attempt == 0;
        r.stream = g.stream;
        chunk_layout(r);
        int rc = ensure_ws(chunk_run_bytes(r));
        if (rc) return rc;
        r.base = g.ws;
        rc = chunk_begin(r);
        while (rc == TIKH_OK && !r.done) rc = chunk_adapt(r);
        if (rc == TIKH_OK) rc = chunk_finish(r);
        if (rc == TIKH_OK) rc = chunk_check(r);
        if (rc == TIKH_OK && g.opts.fallback_nlim > 0) rc = chunk_failed(r);
        g.cur_sizes = nullptr;
        spec.failed.swap(r.failed);
        if (rc != TIKH_RESIZE) return rc;
        g.sizes.erase(sizes_key(spec.pl, spec.nr, spec.sds));
    }
    return TIKH_EHIP;
}

// Chunks of different plans (ragged batches) side by side: each wave of chunks that fits
// the workspace gets disjoint workspace regions and its own streams (default priority,
// ordered after the library stream's earlier work by an event and joined back by events),
// and the phases are interleaved over the wave, so one chunk's host synchronizations
// (transform sizing read back on a first call, adaptive refinement decisions) leave the
// other chunks' queued work running.  Chunks whose recorded lengths were too short run
// again afterwards, one at a time.
static int run_concurrent(std::vector<std::unique_ptr<ChunkRun>>& runs, size_t budget) {
    const int nstreams = std::max(1, std::min((int)g.opts.streams, 16));
    while ((int)g.pool.size() < nstreams) {
        hipStream_t st;
        HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        g.pool.push_back(st);
    }
    while (g.events.size() < (size_t)nstreams + 1) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        g.events.push_back(e);
    }
    const hipStream_t user = g.stream;
    std::vector<ChunkRun*> rerun;
    size_t i0 = 0;
    int rc = TIKH_OK;
    while (i0 < runs.size() && rc == TIKH_OK) {
        // the next wave: consecutive chunks while they fit the budget and the stream pool
        size_t i1 = i0, total = 0;
        while (i1 < runs.size() && (int)(i1 - i0) < nstreams) {
            const size_t bytes = (chunk_run_bytes(*runs[i1]) + 255) & ~(size_t)255;
            if (i1 > i0 && total + bytes > budget) break;
            total += bytes;
            ++i1;
        }
        rc = ensure_ws(total);
        if (rc) break;
        HIPCHK(hipEventRecord(g.events[nstreams], user));
        size_t off = 0;
        for (size_t i = i0; i < i1; ++i) {
            ChunkRun& r = *runs[i];
            r.stream = g.pool[i - i0];
            r.base = g.ws + off;
            off += (chunk_run_bytes(r) + 255) & ~(size_t)255;
            HIPCHK(hipStreamWaitEvent(r.stream, g.events[nstreams], 0));
        }
        for (size_t i = i0; i < i1 && rc == TIKH_OK; ++i) { chunk_enter(*runs[i]); rc = chunk_begin(*runs[i]); }
        for (bool more = true; more && rc == TIKH_OK;) {
            more = false;
            for (size_t i = i0; i < i1 && rc == TIKH_OK; ++i) {
                ChunkRun& r = *runs[i];
                if (r.done) continue;
                chunk_enter(r);
                rc = chunk_adapt(r);
                more |= !r.done;
            }
        }
        for (size_t i = i0; i < i1 && rc == TIKH_OK; ++i) { chunk_enter(*runs[i]); rc = chunk_finish(*runs[i]); }
        for (size_t i = i0; i < i1 && rc == TIKH_OK; ++i) {
            chunk_enter(*runs[i]);
            int c = chunk_check(*runs[i]);
            if (c == TIKH_OK && g.opts.fallback_nlim > 0) c = chunk_failed(*runs[i]);
            if (c == TIKH_RESIZE) rerun.push_back(runs[i].get());
            else rc = c;
        }
        // join the wave back into the library stream
        for (size_t i = i0; i < i1; ++i) {
            (void)hipEventRecord(g.events[i - i0], runs[i]->stream);
            (void)hipStreamWaitEvent(user, g.events[i - i0], 0);
        }
        g.stream = user;
        g.cur_sizes = nullptr;
        i0 = i1;
    }
    g.stream = user;
    g.cur_sizes = nullptr;
    if (rc) return rc;
    for (ChunkRun* r : rerun) {
        g.sizes.erase(sizes_key(r->pl, r->nr, r->sds));
        rc = run_chunk(*r);
        if (rc) return rc;
    }
    return TIKH_OK;
}

// Ragged batches: extended sizes within a factor 1 + merge_tol of the smallest of a run
// share the largest one's plan (a larger extension k, Sec. 3.1), so fewer, fuller
// launches walk fewer trees.  Maps every N (ascending keys) to the N it runs at.
static std::map<int64_t, int64_t> merged_sizes(const std::vector<int64_t>& Ns) {
    std::map<int64_t, int64_t> to;
    size_t i = 0;
    while (i < Ns.size()) {
        size_t j = i;
        while (j + 1 < Ns.size() && g.opts.merge_tol > 0.0 &&
               (double)Ns[j + 1] <= (1.0 + g.opts.merge_tol) * (double)Ns[i])
            ++j;
        for (size_t u = i; u <= j; ++u) to[Ns[u]] = Ns[j];
        i = j + 1;
    }
    return to;
}

// Group solves by plan and run them in chunks that fit the workspace budget.
// sds is group-major: solves g*nr .. g*nr + nr - 1 share the operator.
static int run_solves_core(std::vector<SolveDesc>& sds, int nr, int32_t* info,
                           std::vector<SolveDesc>* failed);

// Groups whose solve failed (FAIL_BITS: the recursion met pivots so small that its
// basis lost the solution, Sec. 5 "difficult points", or broke down) are solved again
// with the smaller leaf cutoff fallback_nlim: a different tree over the same
// conditions, whose leaves hold fewer of them.  Their outputs and info are overwritten.
static int run_solves(std::vector<SolveDesc>& sds, int nr, int32_t* info) {
    init_opts();                 // (allocation-free calls pass through here too)
    g.launches = 0;
    g.syncs = 0;
    g.stats.refine_extra = 0;
    g.stats.refine_skipped = 0;
    g.stats.deferred = 0;
    g.stats.fallback_groups = 0;
    std::vector<SolveDesc> failed;
    const bool fb = g.opts.fallback_nlim > 0 && g.opts.fallback_nlim < g.opts.n_lim;
    int rc = run_solves_core(sds, nr, info, fb ? &failed : nullptr);
    if (rc || failed.empty()) return rc;
    g.stats.fallback_groups = (int64_t)failed.size() / nr;
    const int32_t keep = g.opts.n_lim;
    g.opts.n_lim = g.opts.fallback_nlim;
    const tikh_stats st = g.stats;
    rc = run_solves_core(failed, nr, info, nullptr);
    g.opts.n_lim = keep;
    // the statistics describe the main solve (plan, shapes), with the fallback's counts added
    const int64_t launches = g.stats.launches, syncs = g.stats.host_syncs, extra = g.stats.refine_extra;
    const int64_t skipped = g.stats.refine_skipped;
    g.stats = st;
    g.stats.launches = launches;
    g.stats.host_syncs = syncs;
    g.stats.refine_extra += extra;
    g.stats.refine_skipped += skipped;
    return rc;
}

// The chunks of a call: solves grouped by plan (extended sizes merged within merge_tol),
// each plan's groups in equal chunks that fit the budget (and chunk_groups).
static int make_runs(std::vector<SolveDesc>& sds, int nr, int32_t* info, size_t budget,
                     std::vector<std::unique_ptr<ChunkRun>>& runs) {
    if (nr != 1 && nr != 2 && nr != 4) return TIKH_EINVAL;
    const int64_t G = (int64_t)sds.size() / nr;
    std::map<int64_t, std::vector<int64_t>> buckets;     // N -> group indices
    std::map<int64_t, std::pair<int64_t, int>> shapes;   // N -> (M, p)
    for (int64_t gi = 0; gi < G; ++gi) {
        SolveDesc& d0 = sds[gi * nr];
        int64_t N, M;
        int p;
        // the circulant must hold T (m + n - 1 generator entries), or for the Toeplitz-Gramian
        // problem both L (p + n - 1) and the Gramian (2n - 1)
        const int64_t Nt = d0.gramian ? std::max(d0.m + d0.n - 1, 2 * d0.n - 1) : d0.m + d0.n - 1;
        if (!opt_extend(Nt, g.opts.n_lim, &N, &M, &p)) return TIKH_EINVAL;
        if (N > ((int64_t)1 << 19)) return TIKH_EINVAL;   // tau-degrees must fit the 20-bit pivot key
        for (int r = 0; r < nr; ++r) sds[gi * nr + r].k = N - (d0.m + d0.n - 1);
        buckets[N].push_back(gi);
        shapes[N] = {M, p};
    }
    {
        std::vector<int64_t> Ns;
        for (auto& kv : buckets) Ns.push_back(kv.first);
        const std::map<int64_t, int64_t> to = merged_sizes(Ns);
        std::map<int64_t, std::vector<int64_t>> merged;
        for (auto& kv : buckets) {
            const int64_t Nt = to.at(kv.first);
            for (int64_t gi : kv.second) {
                SolveDesc& d0 = sds[gi * nr];
                for (int r = 0; r < nr; ++r) sds[gi * nr + r].k = Nt - (d0.m + d0.n - 1);
                merged[Nt].push_back(gi);
            }
        }
        buckets.swap(merged);
    }
    for (auto& kv : buckets) {
        Plan pl;
        if (!make_plan(kv.first, shapes[kv.first].first, shapes[kv.first].second, &pl)) return TIKH_EINVAL;
        std::vector<int64_t>& idx = kv.second;
        int64_t mmax = 1, nmax = 1;
        for (int64_t gi : idx) { mmax = std::max(mmax, sds[gi * nr].m); nmax = std::max(nmax, sds[gi * nr].n); }
        Layout L;
        make_layout(pl, nr, mmax, nmax, &L);
        // merge scratch for up to 128 groups at the largest level (at most a quarter of the
        // budget; smaller levels fit more), the rest held per group
        int64_t mchunk = std::max<int64_t>(1, std::min<int64_t>(128, (int64_t)(budget / 4 / L.temp_bytes)));
        const size_t per_group = L.group_bytes + (size_t)nr * L.solve_bytes;
        const size_t fixed = (size_t)mchunk * L.temp_bytes;
        // at least one group per chunk: if even that does not fit, the workspace reports it
        int64_t chunk = std::max<int64_t>(1, budget > fixed ? (int64_t)((budget - fixed) / per_group) : 0);
        chunk = std::min<int64_t>(chunk, 65535);
        if (g.opts.chunk_groups > 0) chunk = std::min<int64_t>(chunk, g.opts.chunk_groups);
        // equal chunks: a small remainder chunk would repeat the whole serial recursion
        // for a handful of groups
        {
            const int64_t nch = ((int64_t)idx.size() + chunk - 1) / chunk;
            chunk = ((int64_t)idx.size() + nch - 1) / nch;
        }
        for (size_t c0 = 0; c0 < idx.size(); c0 += (size_t)chunk) {
            size_t c1 = std::min(idx.size(), c0 + (size_t)chunk);
            auto r = std::make_unique<ChunkRun>();
            r->pl = pl; r->nr = nr; r->info = info; r->mchunk = mchunk;
            r->sds.reserve((c1 - c0) * nr);
            for (size_t u = c0; u < c1; ++u)
                for (int q = 0; q < nr; ++q) r->sds.push_back(sds[idx[u] * nr + q]);
            chunk_layout(*r);
            runs.push_back(std::move(r));
            g.stats.N = pl.N;
            g.stats.k = runs.back()->sds[0].k;
            g.stats.depth = pl.p;
            g.stats.leaf_nodes = (int32_t)pl.M;
        }
    }
    return TIKH_OK;
}

static int run_solves_core(std::vector<SolveDesc>& sds, int nr, int32_t* info,
                           std::vector<SolveDesc>* failed) {
    if (sds.empty()) return TIKH_OK;
    size_t budget;
    if (g.ws_ext) {
        budget = g.ws_size > WS_FIXED ? g.ws_size - WS_FIXED : 0;
    } else {
        size_t freeb = 0, totb = 0;
        (void)hipMemGetInfo(&freeb, &totb);
        budget = std::max<size_t>((size_t)1 << 30, (size_t)((double)(freeb + g.ws_size) * 0.85)) - WS_FIXED;
    }
    std::vector<std::unique_ptr<ChunkRun>> runs;
    {
        int rc0 = make_runs(sds, nr, info, budget, runs);
        if (rc0) return rc0;
    }
    int rc = (runs.size() > 1 && !g.noalloc && g.opts.streams > 1) ? run_concurrent(runs, budget + WS_FIXED)
                                                                    : TIKH_OK;
    if (runs.size() <= 1 || g.noalloc || g.opts.streams <= 1) {
        for (auto& r : runs) {
            rc = run_chunk(*r);
            if (rc) break;
        }
    }
    if (rc) return rc;
    if (failed)
        for (auto& r : runs) failed->insert(failed->end(), r->failed.begin(), r->failed.end());
    g.stats.solves = (int64_t)sds.size();
    g.stats.launches = g.launches;
    g.stats.host_syncs = g.syncs;
    return TIKH_OK;
}

static bool bad_lambda(double lam) { return !(lam > 0.0) || !std::isfinite(lam); }

static int sync_info(int rc, int32_t* dinfo) {
    int32_t hinfo = 0;
    if (rc == TIKH_OK) HIPCHK(hipMemcpyAsync(&hinfo, dinfo, sizeof(int32_t), hipMemcpyDeviceToHost, g.stream));
    HIPCHK(hipStreamSynchronize(g.stream));
    (void)hipFreeAsync(dinfo, g.stream);
    HIPCHK(hipStreamSynchronize(g.stream));
    if (rc) return rc;
    return hinfo ? TIKH_ENUMERIC : TIKH_OK;
}

static int solve_single(const void* col, const void* row, int64_t m, int64_t n, const void* rhs, double lambda,
                        void* x, int cplx, int mode) {
    ensure_init();
    if (!col || !row || !rhs || !x || m < 1 || n < 1 || bad_lambda(lambda)) return TIKH_EINVAL;
    if (m + n > ((int64_t)1 << 30)) return TIKH_EINVAL;
    std::vector<SolveDesc> sds(1);
    SolveDesc& d = sds[0];
    d.col = col; d.row = row; d.rhs = rhs; d.x = x; d.m = m; d.n = n; d.lam = lambda; d.cplx = cplx; d.mode = mode;
    d.orig = 0;
    int32_t* dinfo = nullptr;
    HIPCHK(hipMallocAsync((void**)&dinfo, sizeof(int32_t), g.stream));
    HIPCHK(hipMemsetAsync(dinfo, 0, sizeof(int32_t), g.stream));
    return sync_info(run_solves(sds, 1, dinfo), dinfo);
}

// right-hand sides per group for a batched call
static int group_size(int64_t nrhs) { return nrhs >= 4 ? 4 : (nrhs >= 2 ? 2 : 1); }

}  // namespace tikh

using namespace tikh;

extern "C" {

int tikh_init(void) { ensure_init(); return TIKH_OK; }

int tikh_profile_kernel(const char* name) {
    ensure_init();
    prof_collect();
    prof_print_detail();
    kprof.detail.clear();
    kprof.label.clear();
    kprof.name = name ? std::string(name) : std::string();
    kprof.total_ms = 0.0;
    kprof.count = 0;
    kprof.units = 0.0;
    return TIKH_OK;
}

int tikh_profile_read(double* total_ms, int64_t* count) {
    if (!total_ms || !count) return TIKH_EINVAL;
    prof_collect();
    *total_ms = kprof.total_ms;
    *count = kprof.count;
    return TIKH_OK;
}

int tikh_profile_units(double* units) {
    if (!units) return TIKH_EINVAL;
    *units = kprof.units;
    return TIKH_OK;
}

int tikh_plan_info(int64_t m, int64_t n, int32_t n_lim, int64_t* N, int64_t* M, int32_t* depth, int64_t* k) {
    if (m < 1 || n < 1 || n_lim < 4 || !N || !M || !depth || !k) return TIKH_EINVAL;
    int64_t NN, MM;
    int pp;
    if (!opt_extend(m + n - 1, n_lim, &NN, &MM, &pp)) return TIKH_EINVAL;
    *N = NN; *M = MM; *depth = pp; *k = NN - (m + n - 1);
    return TIKH_OK;
}

int tikh_fft_batched(void* data, int64_t items, int64_t nlines, int64_t len, int sign) {
    ensure_init();
    if (!data || items < 1 || items > 65535 || nlines < 1 || len < 1 || (sign != 1 && sign != -1)) return TIKH_EINVAL;
    // one item's lines are addressed with 32-bit offsets
    if (!smooth5(len) || len > (int64_t)FFT_LDS_MAX * FFT_LDS_MAX || nlines > (((int64_t)1 << 31) - 1) / len)
        return TIKH_EINVAL;
    if (len > FFT_LDS_MAX && fft_split(len) == 0) return TIKH_EINVAL;
    const double2* tw = twiddles(len);
    if (!tw) return TIKH_ENOMEM;
    double2* scr = nullptr;
    if (len > FFT_LDS_MAX) {
        // the four-step reordering goes through a scratch copy
        int rc = ensure_ws((size_t)items * nlines * len * sizeof(double2));
        if (rc) return rc;
        scr = (double2*)g.ws;
    }
    g.launches = 0;
    int rc = fft_lines((double2*)data, items, nlines * len, nlines, len, sign, tw, len, scr, nlines * len);
    if (rc) return rc;
    return hipGetLastError() == hipSuccess ? TIKH_OK : TIKH_EHIP;
}

int tikh_autotune_nlim(int64_t m, int64_t n, int64_t groups, int32_t nrhs, int32_t* best, double* ms) {
    ensure_init();
    if (m < 1 || n < 1 || groups < 1 || groups > 65535 || nrhs < 1 || nrhs > MAXNR || !best) return TIKH_EINVAL;
    const int nr = group_size(nrhs);
    // synthetic real problem: generator with an exp(-|s|/32) envelope about the main
    // diagonal, uniform right-hand sides, lambda = 1e-2 sum |a_s| (so kappa <= 1e4)
    double *col = nullptr, *row = nullptr, *bb = nullptr, *xx = nullptr;
    const int64_t nx = groups * nr * n;
    if (hipMalloc(&col, sizeof(double) * (m + n)) != hipSuccess) return TIKH_ENOMEM;
    row = col + m;
    if (hipMalloc(&bb, sizeof(double) * nr * m) != hipSuccess) { (void)hipFree(col); return TIKH_ENOMEM; }
    if (hipMalloc(&xx, sizeof(double) * nx) != hipSuccess) { (void)hipFree(col); (void)hipFree(bb); return TIKH_ENOMEM; }
    hipLaunchKernelGGL(k_synth, grid1(m, 1), dim3(256), 0, g.stream, col, m, 1ull, (int64_t)0, 32.0);
    hipLaunchKernelGGL(k_synth, grid1(n, 1), dim3(256), 0, g.stream, row, n, 2ull, (int64_t)0, 32.0);
    hipLaunchKernelGGL(k_synth, grid1(nr * m, 1), dim3(256), 0, g.stream, bb, nr * m, 3ull, (int64_t)0, 0.0);
    std::vector<double> hc(m + n);
    int rc = TIKH_OK;
    if (hipMemcpyAsync(hc.data(), col, sizeof(double) * (m + n), hipMemcpyDeviceToHost, g.stream) != hipSuccess ||
        hipStreamSynchronize(g.stream) != hipSuccess)
        rc = TIKH_EHIP;
    double asum = 0.0;
    for (int64_t i = 0; i < m + n; ++i) asum += std::fabs(hc[i]) * (i == m ? 0.0 : 1.0);   // row[0] unused
    std::vector<SolveDesc> sds;
    for (int64_t gi = 0; gi < groups; ++gi)
        for (int r = 0; r < nr; ++r) {
            SolveDesc d{};
            d.col = col; d.row = row; d.m = m; d.n = n; d.lam = 1e-2 * asum; d.cplx = 0; d.mode = 0;
            d.rhs = bb + (int64_t)r * m;
            d.x = xx + (gi * nr + r) * n;
            d.orig = -1;
            sds.push_back(d);
        }
    const tikh_opts saved = g.opts;
    const int32_t cand[4] = {64, 128, 192, 256};
    double best_ms = 0.0;
    int32_t best_n = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == TIKH_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = TIKH_EHIP;
    for (int c = 0; c < 4 && rc == TIKH_OK; ++c) {
        double t = -1.0;
        int64_t NN, MM;
        int pp;
        if (opt_extend(m + n - 1, cand[c], &NN, &MM, &pp) && NN <= ((int64_t)1 << 19)) {
            g.opts.n_lim = cand[c];
            std::vector<SolveDesc> w = sds;
            rc = run_solves(w, nr, nullptr);                      // warm-up (workspace, tables)
            if (rc) break;
            w = sds;
            (void)hipEventRecord(e0, g.stream);
            rc = run_solves(w, nr, nullptr);
            if (rc) break;
            (void)hipEventRecord(e1, g.stream);
            if (hipEventSynchronize(e1) != hipSuccess) { rc = TIKH_EHIP; break; }
            float f = 0.f;
            (void)hipEventElapsedTime(&f, e0, e1);
            t = f;
            if (best_n == 0 || t < best_ms) { best_ms = t; best_n = cand[c]; }
        }
        if (ms) ms[c] = t;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(g.stream);
    (void)hipFree(col);
    (void)hipFree(bb);
    (void)hipFree(xx);
    g.opts = saved;
    if (rc) return rc;
    if (best_n == 0) return TIKH_EINVAL;
    g.opts.n_lim = best_n;
    *best = best_n;
    return TIKH_OK;
}

int tikh_workspace_bytes(int64_t nprob, const int64_t* m, const int64_t* n, int64_t nlam, int64_t nrhs,
                         size_t* bytes) {
    if (nprob < 0 || nlam < 1 || nrhs < 1 || !bytes || (nprob > 0 && (!m || !n))) return TIKH_EINVAL;
    const int nr = group_size(nrhs);
    const int64_t gpp = nlam * ((nrhs + nr - 1) / nr);  // groups per problem
    init_opts();
    const int32_t nlim = g.opts.n_lim;
    struct Bucket { int64_t M; int p; int64_t G = 0, mmax = 1, nmax = 1; };
    std::map<int64_t, Bucket> buckets;
    for (int64_t q = 0; q < nprob; ++q) {
        if (m[q] < 1 || n[q] < 1 || m[q] + n[q] > ((int64_t)1 << 30)) return TIKH_EINVAL;
        int64_t N, M;
        int p;
        if (!opt_extend(m[q] + n[q] - 1, nlim, &N, &M, &p)) return TIKH_EINVAL;
        if (N > ((int64_t)1 << 19)) return TIKH_EINVAL;
        Bucket& bk = buckets[N];
        bk.M = M; bk.p = p;
        bk.G += gpp;
        bk.mmax = std::max(bk.mmax, m[q]);
        bk.nmax = std::max(bk.nmax, n[q]);
    }
    init_opts();
    std::vector<int64_t> Ns;
    for (auto& kv : buckets) Ns.push_back(kv.first);
    const std::map<int64_t, int64_t> to = merged_sizes(Ns);
    std::map<int64_t, Bucket> merged;
    for (auto& kv : buckets) {
        Bucket& bk = merged[to.at(kv.first)];
        const Bucket& src = buckets[to.at(kv.first)];
        bk.M = src.M; bk.p = src.p;
        bk.G += kv.second.G;
        bk.mmax = std::max(bk.mmax, kv.second.mmax);
        bk.nmax = std::max(bk.nmax, kv.second.nmax);
    }
    // every bucket in one chunk, or in equal chunks of at most chunk_groups groups; with
    // several streams up to `streams` chunks side by side (the largest ones bound the sum)
    std::vector<size_t> sizes;
    for (auto& kv : merged) {
        Plan pl;
        if (!make_plan(kv.first, kv.second.M, kv.second.p, &pl)) return TIKH_EINVAL;
        Layout L;
        make_layout(pl, nr, kv.second.mmax, kv.second.nmax, &L);
        const int64_t G = kv.second.G;
        const int64_t cg = g.opts.chunk_groups > 0 ? std::min<int64_t>(G, g.opts.chunk_groups) : G;
        const int64_t nch = (G + cg - 1) / cg, cs = (G + nch - 1) / nch;
        for (int64_t c0 = 0; c0 < G; c0 += cs) {
            const int64_t gc = std::min(cs, G - c0);
            sizes.push_back((chunk_bytes(L, gc, std::min<int64_t>(gc, 128)) + 255) & ~(size_t)255);
        }
    }
    std::sort(sizes.begin(), sizes.end(), std::greater<size_t>());
    size_t total = 0;
    const size_t side = g.opts.streams > 1 ? std::min(sizes.size(), (size_t)g.opts.streams) : 1;
    for (size_t i = 0; i < side && i < sizes.size(); ++i) total += sizes[i];
    *bytes = total;
    return TIKH_OK;
}

int tikh_set_workspace(void* ptr, size_t bytes) {
    ensure_init();
    if ((ptr && bytes == 0) || ((uintptr_t)ptr & 255)) return TIKH_EINVAL;
    HIPCHK(hipStreamSynchronize(g.stream));
    if (g.ws && !g.ws_ext) (void)hipFree(g.ws);
    g.ws = (char*)ptr;
    g.ws_size = ptr ? bytes : 0;
    g.ws_ext = ptr != nullptr;
    return TIKH_OK;
}

int tikh_release(void) {
    if (g.ws) {
        (void)hipStreamSynchronize(g.stream);
        if (!g.ws_ext) (void)hipFree(g.ws);
        g.ws = nullptr; g.ws_size = 0; g.ws_ext = false;
    }
    for (auto& kv : g.tw) (void)hipFree(kv.second);
    g.tw.clear();
    for (auto& kv : g.tw2) (void)hipFree(kv.second);
    g.tw2.clear();
    g.sizes.clear();
    g.generation++;
    for (hipStream_t st : g.pool) (void)hipStreamDestroy(st);
    g.pool.clear();
    for (hipEvent_t e : g.events) (void)hipEventDestroy(e);
    g.events.clear();
    return TIKH_OK;
}

int tikh_set_stream(void* s) { ensure_init(); g.stream = (hipStream_t)s; return TIKH_OK; }

int tikh_set_options(const tikh_opts* o) {
    ensure_init();
    if (!o || !opts_valid(o)) return TIKH_EINVAL;
    g.opts = *o;
    return TIKH_OK;
}

}  // extern "C"

static bool tikh::opts_valid(const tikh_opts* o) {
    if (o->n_lim < 64 || o->n_lim > LEAF_MAX || o->refine < 0 || o->refine > 4 || o->refine_max < 0 ||
        o->refine_max > 4 || !(o->refine_tol > 0.0) || !std::isfinite(o->refine_tol) || !(o->defer_tol >= 0.0) ||
        !(o->defer_tol < 1.0) || o->leaf_wave_groups < 1 || o->streams < 1 || o->streams > 16 ||
        !(o->merge_tol >= 0.0) || !(o->merge_tol <= 4.0) ||
        (o->fallback_nlim != 0 && (o->fallback_nlim < 64 || o->fallback_nlim > LEAF_MAX)) || o->chunk_groups < 0 ||
        (o->refine_skip != 0 && o->refine_skip != 1))
        return false;
    return true;
}

extern "C" {

int tikh_get_options(tikh_opts* o) { ensure_init(); if (!o) return TIKH_EINVAL; *o = g.opts; return TIKH_OK; }

int tikh_get_stats(tikh_stats* s) { ensure_init(); if (!s) return TIKH_EINVAL; *s = g.stats; return TIKH_OK; }

const char* tikh_strerror(int code) {
    switch (code) {
        case TIKH_OK: return "ok";
        case TIKH_EINVAL: return "invalid argument";
        case TIKH_ENOMEM: return "device allocation failed";
        case TIKH_EHIP: return hipGetErrorString(last_hip_error);
        case TIKH_ENUMERIC: return "numerical breakdown reported by a solve (info != 0)";
        case TIKH_ETOOBIG: return "the batch does not fit the allocation-free scratch buffer (64 MiB per device)";
        default: return "unknown error";
    }
}

int tikh_toeplitz_solve(const double* col, const double* row, int64_t m, int64_t n, const double* b, double lambda,
                        double* x) {
    return solve_single(col, row, m, n, b, lambda, x, 0, 0);
}

int tikh_toeplitz_solve_z(const tikh_c64* col, const tikh_c64* row, int64_t m, int64_t n, const tikh_c64* b,
                          double lambda, tikh_c64* x) {
    return solve_single(col, row, m, n, b, lambda, x, 1, 0);
}

int tikh_toeplitz_solve_normal(const double* col, const double* row, int64_t m, int64_t n, const double* y,
                               double lambda, double* x) {
    return solve_single(col, row, m, n, y, lambda, x, 0, 1);
}

int tikh_toeplitz_solve_normal_z(const tikh_c64* col, const tikh_c64* row, int64_t m, int64_t n, const tikh_c64* y,
                                 double lambda, tikh_c64* x) {
    return solve_single(col, row, m, n, y, lambda, x, 1, 1);
}

// Solve descriptors of a batched call (group-major, the last group of each
// (problem, lambda) padded with empty solves).
static int batched_sds(int64_t nprob, const int64_t* m, const int64_t* n, const void* col, const void* row,
                       int64_t nlam, const double* lambdas, int64_t nrhs, const void* b, void* x, int complex_data,
                       std::vector<SolveDesc>& sds) {
    if (!col || !row || !b || !x) return TIKH_EINVAL;
    const size_t es = complex_data ? sizeof(double2) : sizeof(double);
    const int nr = group_size(nrhs);
    int64_t co = 0, ro = 0, bo = 0, xo = 0, si = 0;
    for (int64_t p = 0; p < nprob; ++p) {
        if (m[p] < 1 || n[p] < 1) return TIKH_EINVAL;
        for (int64_t l = 0; l < nlam; ++l) {
            double lam = lambdas[p * nlam + l];
            if (bad_lambda(lam)) return TIKH_EINVAL;
            for (int64_t r0 = 0; r0 < nrhs; r0 += nr) {
                for (int64_t r = r0; r < r0 + nr; ++r) {
                    SolveDesc d{};
                    d.col = (const char*)col + es * co;
                    d.row = (const char*)row + es * ro;
                    d.m = m[p]; d.n = n[p]; d.lam = lam; d.cplx = complex_data ? 1 : 0; d.mode = 0;
                    d.lamx = (int32_t)(p * nlam + l);
                    if (r < nrhs) {
                        d.rhs = (const char*)b + es * (bo + r * m[p]);
                        d.x = (char*)x + es * (xo + (l * nrhs + r) * n[p]);
                        d.orig = (int32_t)(si + l * nrhs + r);
                    } else {
                        d.orig = -1;
                    }
                    sds.push_back(d);
                }
            }
        }
        co += m[p]; ro += n[p]; bo += nrhs * m[p]; xo += nlam * nrhs * n[p]; si += nlam * nrhs;
    }
    return TIKH_OK;
}

int tikh_toeplitz_solve_batched(int64_t nprob, const int64_t* m, const int64_t* n, const void* col, const void* row,
                                int64_t nlam, const double* lambdas, int64_t nrhs, const void* b, void* x,
                                int32_t* info, int complex_data) {
    ensure_init();
    if (nprob < 0 || nlam < 1 || nrhs < 1 || !m || !n || !lambdas) return TIKH_EINVAL;
    if (nprob == 0) return TIKH_OK;
    std::vector<SolveDesc> sds;
    int rc = batched_sds(nprob, m, n, col, row, nlam, lambdas, nrhs, b, x, complex_data, sds);
    if (rc) return rc;
    return run_solves(sds, group_size(nrhs), info);
}

}  // extern "C"

namespace tikh {

// Allocation-free batched solves: every device buffer the library needs beyond
// the caller's inputs and outputs comes from this file-scope array.  Each GPU
// holds its own copy; its address on a device is looked up once with
// hipGetSymbolAddress (the array's name is not a device address in host code).
static const size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
static const int NOALLOC_MAX_DEVICES = 64;
static void* scratch_ptr[NOALLOC_MAX_DEVICES];

}  // namespace tikh

extern "C" {

int tikh_toeplitz_solve_batched_noalloc(int64_t nprob, const int64_t* m, const int64_t* n, const void* col,
                                        const void* row, int64_t nlam, const double* lambdas, int64_t nrhs,
                                        const void* b, void* x, int32_t* info, int complex_data) {
    init_opts();
    if (nprob < 0 || nlam < 1 || nrhs < 1 || !m || !n || !lambdas) return TIKH_EINVAL;
    if (nprob == 0) return TIKH_OK;
    std::vector<SolveDesc> sds;
    int rc = batched_sds(nprob, m, n, col, row, nlam, lambdas, nrhs, b, x, complex_data, sds);
    if (rc) return rc;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return TIKH_EINVAL;
    if (!scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            last_hip_error = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return TIKH_EHIP;
        }
        scratch_ptr[dev] = ptr;
    }
    // arena for the twiddle tables: the Q = 8N table, the per-length tables of the transforms
    // (lengths dividing 8N that the chunks' degrees select; 32N entries leave room for several
    // product lengths per level) and the two-level tables, plus the readback word
    int64_t Nmax = 1;
    for (int64_t p = 0; p < nprob; ++p) {
        int64_t N, M;
        int pp;
        if (!opt_extend(m[p] + n[p] - 1, g.opts.n_lim, &N, &M, &pp)) return TIKH_EINVAL;
        Nmax = std::max(Nmax, N);
    }
    const size_t arena = ((sizeof(double2) * (size_t)(40 * Nmax + 65536) + 4096) + 255) & ~(size_t)255;
    if (arena + WS_FIXED >= NOALLOC_SCRATCH_BYTES) return TIKH_ETOOBIG;
    char* base = (char*)scratch_ptr[dev];
    char* save_ws = g.ws;
    const size_t save_size = g.ws_size;
    const bool save_ext = g.ws_ext;
    g.noalloc = true;
    g.arena = base;
    g.arena_size = arena;
    g.arena_used = 256;
    g.ndneed = (int*)base;
    g.ntw.clear();
    g.ntw2.clear();
    g.ws = base + arena;
    g.ws_size = NOALLOC_SCRATCH_BYTES - arena;
    g.ws_ext = true;
    rc = run_solves(sds, group_size(nrhs), info);
    g.ws = save_ws;
    g.ws_size = save_size;
    g.ws_ext = save_ext;
    g.noalloc = false;
    g.arena = nullptr;
    g.ndneed = nullptr;
    g.ntw.clear();
    g.ntw2.clear();
    return rc == TIKH_ENOMEM ? TIKH_ETOOBIG : rc;
}

// Toeplitz-Gramian problem (Sec. 2 third case, Sec. 3.4): solve descriptors with the
// regularizer L in col/row/m, the Gramian's first column in gram, normal-form y.
static int gramian_sds(int64_t nprob, const int64_t* p, const int64_t* n, const void* gram, const void* lcol,
                       const void* lrow, int64_t nrhs, const void* y, void* x, int complex_data,
                       std::vector<SolveDesc>& sds) {
    if (!gram || !lcol || !lrow || !y || !x) return TIKH_EINVAL;
    const size_t es = complex_data ? sizeof(double2) : sizeof(double);
    const int nr = group_size(nrhs);
    int64_t go = 0, lo = 0, ro = 0, yo = 0, si = 0;
    for (int64_t q = 0; q < nprob; ++q) {
        if (p[q] < 1 || n[q] < 1) return TIKH_EINVAL;
        for (int64_t r0 = 0; r0 < nrhs; r0 += nr) {
            for (int64_t r = r0; r < r0 + nr; ++r) {
                SolveDesc d{};
                d.col = (const char*)lcol + es * lo;
                d.row = (const char*)lrow + es * ro;
                d.gram = (const char*)gram + es * go;
                d.gramian = 1;
                d.m = p[q]; d.n = n[q]; d.lam = 1.0; d.cplx = complex_data ? 1 : 0; d.mode = 1;
                if (r < nrhs) {
                    d.rhs = (const char*)y + es * (yo + r * n[q]);
                    d.x = (char*)x + es * (yo + r * n[q]);
                    d.orig = (int32_t)(si + r);
                } else {
                    d.orig = -1;
                }
                sds.push_back(d);
            }
        }
        go += n[q]; lo += p[q]; ro += n[q]; yo += nrhs * n[q]; si += nrhs;
    }
    return TIKH_OK;
}

int tikh_gramian_solve_batched(int64_t nprob, const int64_t* p, const int64_t* n, const void* gram, const void* lcol,
                               const void* lrow, int64_t nrhs, const void* y, void* x, int32_t* info,
                               int complex_data) {
    ensure_init();
    if (nprob < 0 || nrhs < 1 || !p || !n) return TIKH_EINVAL;
    if (nprob == 0) return TIKH_OK;
    std::vector<SolveDesc> sds;
    int rc = gramian_sds(nprob, p, n, gram, lcol, lrow, nrhs, y, x, complex_data, sds);
    if (rc) return rc;
    return run_solves(sds, group_size(nrhs), info);
}

static int gramian_single(const void* gram, const void* lcol, const void* lrow, int64_t p, int64_t n, const void* y,
                          void* x, int cplx) {
    ensure_init();
    if (p < 1 || n < 1 || p + 2 * n > ((int64_t)1 << 30)) return TIKH_EINVAL;
    std::vector<SolveDesc> sds;
    int rc = gramian_sds(1, &p, &n, gram, lcol, lrow, 1, y, x, cplx, sds);
    if (rc) return rc;
    int32_t* dinfo = nullptr;
    HIPCHK(hipMallocAsync((void**)&dinfo, sizeof(int32_t), g.stream));
    HIPCHK(hipMemsetAsync(dinfo, 0, sizeof(int32_t), g.stream));
    return sync_info(run_solves(sds, 1, dinfo), dinfo);
}

int tikh_gramian_solve(const double* gram, const double* lcol, const double* lrow, int64_t p, int64_t n,
                       const double* y, double* x) {
    return gramian_single(gram, lcol, lrow, p, n, y, x, 0);
}

int tikh_gramian_solve_z(const tikh_c64* gram, const tikh_c64* lcol, const tikh_c64* lrow, int64_t p, int64_t n,
                         const tikh_c64* y, tikh_c64* x) {
    return gramian_single(gram, lcol, lrow, p, n, y, x, 1);
}

static int backward_single(const void* col, const void* row, int64_t m, int64_t n, const void* b, double lambda,
                           const void* x, const void* gx, void* gcol, void* grow, void* gb, double* glam, int cplx) {
    ensure_init();
    if (!col || !row || !b || !x || !gx || !gcol || !grow || !gb || !glam || m < 1 || n < 1 || bad_lambda(lambda))
        return TIKH_EINVAL;
    std::vector<SolveDesc> sds(1);
    SolveDesc& d = sds[0];
    d.col = col; d.row = row; d.rhs = gx; d.x = nullptr; d.m = m; d.n = n; d.lam = lambda; d.cplx = cplx; d.mode = 1;
    d.bin = b; d.xin = x; d.gcol = gcol; d.grow = grow; d.gb = gb; d.glam = glam; d.backward = 1; d.orig = 0;
    int32_t* dinfo = nullptr;
    HIPCHK(hipMallocAsync((void**)&dinfo, sizeof(int32_t), g.stream));
    HIPCHK(hipMemsetAsync(dinfo, 0, sizeof(int32_t), g.stream));
    return sync_info(run_solves(sds, 1, dinfo), dinfo);
}

int tikh_toeplitz_solve_backward(const double* col, const double* row, int64_t m, int64_t n, const double* b,
                                 double lambda, const double* x, const double* gx, double* g_col, double* g_row,
                                 double* g_b, double* g_lambda) {
    return backward_single(col, row, m, n, b, lambda, x, gx, g_col, g_row, g_b, g_lambda, 0);
}

int tikh_toeplitz_solve_backward_z(const tikh_c64* col, const tikh_c64* row, int64_t m, int64_t n, const tikh_c64* b,
                                   double lambda, const tikh_c64* x, const tikh_c64* gx, tikh_c64* g_col,
                                   tikh_c64* g_row, tikh_c64* g_b, double* g_lambda) {
    return backward_single(col, row, m, n, b, lambda, x, gx, g_col, g_row, g_b, g_lambda, 1);
}

static int backward_sds(int64_t nprob, const int64_t* m, const int64_t* n, const void* col, const void* row,
                        int64_t nlam, const double* lambdas, int64_t nrhs, const void* b, const void* x,
                        const void* gx, void* g_col, void* g_row, void* g_b, double* g_lambda, int complex_data,
                        std::vector<SolveDesc>& sds) {
    if (!col || !row || !b || !x || !gx || !g_col || !g_row || !g_b || !g_lambda) return TIKH_EINVAL;
    const size_t es = complex_data ? sizeof(double2) : sizeof(double);
    const int nr = group_size(nrhs);
    int64_t co = 0, ro = 0, bo = 0, xo = 0, gco = 0, gro = 0, gbo = 0, si = 0;
    for (int64_t p = 0; p < nprob; ++p) {
        if (m[p] < 1 || n[p] < 1) return TIKH_EINVAL;
        for (int64_t l = 0; l < nlam; ++l) {
            double lam = lambdas[p * nlam + l];
            if (bad_lambda(lam)) return TIKH_EINVAL;
            for (int64_t r0 = 0; r0 < nrhs; r0 += nr) {
                for (int64_t r = r0; r < r0 + nr; ++r) {
                    SolveDesc d{};
                    d.col = (const char*)col + es * co;
                    d.row = (const char*)row + es * ro;
                    d.m = m[p]; d.n = n[p]; d.lam = lam; d.cplx = complex_data ? 1 : 0; d.mode = 1; d.backward = 1;
                    d.lamx = (int32_t)(p * nlam + l);
                    if (r < nrhs) {
                        const int64_t u = l * nrhs + r;
                        d.bin = (const char*)b + es * (bo + r * m[p]);
                        d.xin = (const char*)x + es * (xo + u * n[p]);
                        d.rhs = (const char*)gx + es * (xo + u * n[p]);
                        d.gcol = (char*)g_col + es * (gco + u * m[p]);
                        d.grow = (char*)g_row + es * (gro + u * n[p]);
                        d.gb = (char*)g_b + es * (gbo + u * m[p]);
                        d.glam = g_lambda + si + u;
                        d.orig = (int32_t)(si + u);
                    } else {
                        d.orig = -1;
                    }
                    sds.push_back(d);
                }
            }
        }
        co += m[p]; ro += n[p]; bo += nrhs * m[p]; xo += nlam * nrhs * n[p];
        gco += nlam * nrhs * m[p]; gro += nlam * nrhs * n[p]; gbo += nlam * nrhs * m[p]; si += nlam * nrhs;
    }
    return TIKH_OK;
}

int tikh_toeplitz_solve_backward_batched(int64_t nprob, const int64_t* m, const int64_t* n, const void* col,
                                         const void* row, int64_t nlam, const double* lambdas, int64_t nrhs,
                                         const void* b, const void* x, const void* gx, void* g_col, void* g_row,
                                         void* g_b, double* g_lambda, int32_t* info, int complex_data) {
    ensure_init();
    if (nprob < 0 || nlam < 1 || nrhs < 1 || !m || !n || !lambdas) return TIKH_EINVAL;
    if (nprob == 0) return TIKH_OK;
    std::vector<SolveDesc> sds;
    int rc = backward_sds(nprob, m, n, col, row, nlam, lambdas, nrhs, b, x, gx, g_col, g_row, g_b, g_lambda,
                          complex_data, sds);
    if (rc) return rc;
    return run_solves(sds, group_size(nrhs), info);
}

}  // extern "C"

// ---------------------------------------------------------------- prepared batches
// A prepared batch fixes a call's composition once: its chunks, their workspace regions
// and uploaded descriptors, and the product transform lengths recorded (with headroom)
// by a first run.  Every later run takes the lambdas from the caller's device array and
// enqueues kernel launches and stream/event ordering only (no host synchronization,
// allocation or copy from host memory), so that a caller can capture a run into a graph
// and replay it.
struct tikh_prepared {
    std::vector<std::unique_ptr<tikh::ChunkRun>> runs;
    std::vector<std::unique_ptr<tikh::Ctx::Sizes>> sizes;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    const double* dlam = nullptr;
    int32_t* info = nullptr;
    tikh_opts opts{};
    int64_t generation = 0;
};

namespace tikh {

// restores the library's options, stream and recording mode however a prepared run ends
struct PreparedScope {
    tikh_opts opts;
    hipStream_t stream;
    explicit PreparedScope(const tikh_opts& o) : opts(g.opts), stream(g.stream) { g.opts = o; }
    ~PreparedScope() {
        g.opts = opts;
        g.stream = stream;
        g.cur_sizes = nullptr;
        g.headroom = false;
        g.replay = false;
    }
};

// Enqueues one run of every chunk, side by side on the stream pool (forked from and joined
// back into the library stream by events).  The first run records the transform lengths.
static int prepared_enqueue(tikh_prepared* h, bool first) {
    PreparedScope scope(h->opts);
    g.launches = 0;
    g.syncs = 0;
    const hipStream_t user = g.stream;
    const int nuse = (int)std::min<size_t>(h->runs.size(), (size_t)std::max(1, std::min((int)g.opts.streams, 16)));
    if ((int)g.pool.size() < nuse || g.events.size() < (size_t)nuse + 1) return TIKH_EINVAL;
    HIPCHK(hipEventRecord(g.events[nuse], user));
    for (int i = 0; i < nuse; ++i) HIPCHK(hipStreamWaitEvent(g.pool[i], g.events[nuse], 0));
    g.headroom = first;
    for (size_t i = 0; i < h->runs.size(); ++i) {
        ChunkRun& r = *h->runs[i];
        r.stream = g.pool[i % (size_t)nuse];
        chunk_enter(r);
        hipLaunchKernelGGL(k_set_lam, dim3((unsigned)((r.S + 255) / 256)), dim3(256), 0, g.stream, r.b.sd, r.S,
                           h->dlam);
        g.launches++;
        int rc = chunk_setup(r);
        while (rc == TIKH_OK && !r.done) rc = chunk_adapt(r);
        if (rc == TIKH_OK) rc = chunk_finish(r);
        if (rc) return rc;
        if (h->info) {
            hipLaunchKernelGGL(k_prepared_info, dim3((unsigned)((r.S + 255) / 256)), dim3(256), 0, g.stream, r.b.sd,
                               r.S, r.b.ovf, h->dlam, h->info);
            g.launches++;
        }
    }
    for (int i = 0; i < nuse; ++i) {
        HIPCHK(hipEventRecord(g.events[i], g.pool[i]));
        HIPCHK(hipStreamWaitEvent(user, g.events[i], 0));
    }
    HIPCHK(hipGetLastError());
    g.stats.launches = g.launches;
    g.stats.host_syncs = g.syncs;
    return TIKH_OK;
}

static int prepare(std::vector<SolveDesc>& sds, int nr, const double* dlam, int64_t nlamtot, int32_t* info,
                   tikh_prepared** out) {
    if (!out || !dlam) return TIKH_EINVAL;
    *out = nullptr;
    if (g.opts.defer_tol > 0.0) return TIKH_EINVAL;     // deferral reads its counts back
    if (sds.empty()) return TIKH_EINVAL;
    // the lambdas the batch is planned and first run with
    std::vector<double> hl((size_t)nlamtot);
    HIPCHK(hipMemcpyAsync(hl.data(), dlam, sizeof(double) * nlamtot, hipMemcpyDeviceToHost, g.stream));
    HIPCHK(hipStreamSynchronize(g.stream));
    for (SolveDesc& d : sds) {
        if (d.lamx < 0 || d.lamx >= nlamtot || bad_lambda(hl[(size_t)d.lamx])) return TIKH_EINVAL;
        d.lam = hl[(size_t)d.lamx];
    }
    std::unique_ptr<tikh_prepared> h(new tikh_prepared());
    h->opts = g.opts;
    h->dlam = dlam;
    h->info = info;
    h->generation = g.generation;
    size_t freeb = 0, totb = 0;
    (void)hipMemGetInfo(&freeb, &totb);
    const size_t budget = std::max<size_t>((size_t)1 << 30, (size_t)((double)freeb * 0.85)) - WS_FIXED;
    int rc = make_runs(sds, nr, info, budget, h->runs);
    if (rc) return rc;
    size_t total = 0;
    for (auto& r : h->runs) total += (chunk_run_bytes(*r) + 255) & ~(size_t)255;
    if (total > budget + WS_FIXED) return TIKH_ENOMEM;   // every chunk keeps its own region
    if (hipMalloc(&h->ws, total) != hipSuccess) return TIKH_ENOMEM;
    h->ws_bytes = total;
    const int nstreams = std::max(1, std::min((int)g.opts.streams, 16));
    while ((int)g.pool.size() < nstreams) {
        hipStream_t st;
        HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        g.pool.push_back(st);
    }
    while (g.events.size() < (size_t)nstreams + 1) {
        hipEvent_t e;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        g.events.push_back(e);
    }
    size_t off = 0;
    for (auto& rp : h->runs) {
        ChunkRun& r = *rp;
        r.base = h->ws + off;
        off += (chunk_run_bytes(r) + 255) & ~(size_t)255;
        r.fixed_steps = true;
        r.stream = g.stream;
        h->sizes.emplace_back(new Ctx::Sizes());
        r.sizes = h->sizes.back().get();
        rc = chunk_upload(r);
        if (rc) break;
    }
    g.cur_sizes = nullptr;
    if (rc == TIKH_OK) rc = prepared_enqueue(h.get(), true);
    if (rc == TIKH_OK) HIPCHK(hipStreamSynchronize(g.stream));
    if (rc) {
        (void)hipStreamSynchronize(g.stream);
        (void)hipFree(h->ws);
        return rc;
    }
    *out = h.release();
    return TIKH_OK;
}

}  // namespace tikh

extern "C" {

int tikh_prepare_batched(int64_t nprob, const int64_t* m, const int64_t* n, const void* col, const void* row,
                         int64_t nlam, const double* lambdas, int64_t nrhs, const void* b, void* x, int32_t* info,
                         int complex_data, tikh_prepared** handle) {
    ensure_init();
    if (!handle) return TIKH_EINVAL;
    *handle = nullptr;
    if (nprob < 1 || nlam < 1 || nrhs < 1 || !m || !n || !lambdas) return TIKH_EINVAL;
    // the descriptors are built with a placeholder lambda; the device array supplies them
    std::vector<double> one((size_t)(nprob * nlam), 1.0);
    std::vector<SolveDesc> sds;
    int rc = batched_sds(nprob, m, n, col, row, nlam, one.data(), nrhs, b, x, complex_data, sds);
    if (rc) return rc;
    return prepare(sds, group_size(nrhs), lambdas, nprob * nlam, info, handle);
}

int tikh_prepare_backward_batched(int64_t nprob, const int64_t* m, const int64_t* n, const void* col,
                                  const void* row, int64_t nlam, const double* lambdas, int64_t nrhs, const void* b,
                                  const void* x, const void* gx, void* g_col, void* g_row, void* g_b,
                                  double* g_lambda, int32_t* info, int complex_data, tikh_prepared** handle) {
    ensure_init();
    if (!handle) return TIKH_EINVAL;
    *handle = nullptr;
    if (nprob < 1 || nlam < 1 || nrhs < 1 || !m || !n || !lambdas) return TIKH_EINVAL;
    std::vector<double> one((size_t)(nprob * nlam), 1.0);
    std::vector<SolveDesc> sds;
    int rc = backward_sds(nprob, m, n, col, row, nlam, one.data(), nrhs, b, x, gx, g_col, g_row, g_b, g_lambda,
                          complex_data, sds);
    if (rc) return rc;
    return prepare(sds, group_size(nrhs), lambdas, nprob * nlam, info, handle);
}

int tikh_prepared_run(tikh_prepared* handle) {
    ensure_init();
    if (!handle || handle->generation != g.generation) return TIKH_EINVAL;
    return prepared_enqueue(handle, false);
}

int tikh_prepared_workspace(const tikh_prepared* handle, size_t* bytes) {
    if (!handle || !bytes) return TIKH_EINVAL;
    *bytes = handle->ws_bytes;
    return TIKH_OK;
}

int tikh_prepared_free(tikh_prepared* handle) {
    if (!handle) return TIKH_OK;
    (void)hipDeviceSynchronize();
    (void)hipFree(handle->ws);
    delete handle;
    return TIKH_OK;
}

}  // extern "C"
