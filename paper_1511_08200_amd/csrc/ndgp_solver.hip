// ndgp_solver.hip -- host side of the library: argument checks, workspace
// carve-up, the FAS multigrid driver and the C ABI declared in ndgp.h.
//
// Order of work (arXiv:1511.08200, Sec. III.A): the periodic domain level is
// solved first; each refinement then takes its boundary values (a ghost shell)
// and its initial guess by interpolation from the level above and is relaxed
// with its own multigrid hierarchy, or, in the truncated mode of Sec. III.B,
// keeps the interpolated field.  Relaxation is red-black with the per-cell
// root of the cell's own quadratic; multigrid is a full-approximation-storage
// V(nu1, nu2) cycle (the coarse levels see the nonlinear operator itself).

#include "ndgp.h"
#include "ndgp_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace ndgp;

// Device scratch of ndgp_residual_noalloc, one copy per GPU, held until the
// process ends: the level's source (at most NDGP_NOALLOC_MAX_CELLS doubles),
// then kReduceBlocks reduction partials, then a few sums.
static __device__ __align__(256) double scratch[NDGP_NOALLOC_MAX_CELLS + kReduceBlocks + 32];
static_assert(sizeof(scratch) == NDGP_NOALLOC_SCRATCH_BYTES, "scratch size as documented");

namespace {

thread_local std::string g_err;

// A named range on the host timeline (rocprofv3 --marker-trace): a solve, its
// domain V-cycles, each refinement or box, each plan step.  Without a tool
// attached a push or pop is one call that returns at once.
struct Range {
    explicit Range(const char *what) { roctxRangePushA(what); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

ndgp_status fail(ndgp_status st, std::string msg) {
    g_err = std::move(msg);
    return st;
}

struct HipFailure {
    hipError_t err;
    const char *what;
};

#define HIP_TRY(x)                                                                           \
    do {                                                                                     \
        hipError_t e_ = (x);                                                                 \
        if (e_ != hipSuccess) throw HipFailure{e_, #x};                                      \
    } while (0)

// ------------------------------------------------------------------------
// pinned 8-byte mailboxes for the per-cycle residual norm (allocated once,
// reused across calls; each call holds its own while it runs)

class PinnedSlots {
  public:
    double *acquire() {
        std::lock_guard<std::mutex> g(mu_);
        if (!free_.empty()) {
            double *p = free_.back();
            free_.pop_back();
            return p;
        }
        void *p = nullptr;
        HIP_TRY(hipHostMalloc(&p, 64 * sizeof(double), hipHostMallocDefault));
        return static_cast<double *>(p);
    }
    void release(double *p) {
        std::lock_guard<std::mutex> g(mu_);
        free_.push_back(p);
    }

  private:
    std::mutex mu_;
    std::vector<double *> free_;
};

PinnedSlots &pinned_slots() {
    static PinnedSlots s;
    return s;
}

struct SlotGuard {
    double *p;
    SlotGuard() : p(pinned_slots().acquire()) {}
    ~SlotGuard() { pinned_slots().release(p); }
    SlotGuard(const SlotGuard &) = delete;
    SlotGuard &operator=(const SlotGuard &) = delete;
};

// ------------------------------------------------------------------------
// configuration

int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

struct Cfg {
    int n = 0, lgn = 0, nl = 0;
    double h = 0.0;
    int np = 0;
    int nrelax = 0; // patches 0 .. nrelax-1 are relaxed, the rest interpolated
    int pn[NDGP_MAX_PATCHES] = {};
    int po[NDGP_MAX_PATCHES][3] = {};
    int pnl[NDGP_MAX_PATCHES] = {};
    double alpha = 0.0; // r_c^2 / (3 beta a^2), physical
    double fsrc = 0.0;  // Omega_m / (a beta)
    double tol = 0.0;
    int maxc = 50, nu1 = 2, nu2 = 2;
    int mode = NDGP_MODE_FULL, prec = NDGP_PREC_FP64;
    unsigned flags = 0;

    double hl(int level) const { return h / (double)(1 << level); } // patch p is level p+1
    int nlev(int level) const { return level == 0 ? n : pn[level - 1]; }
};

bool child_fits(int np, const int origin[3], int nc, int nlev) {
    for (int a = 0; a < 3; ++a)
        if (!child_fits_axis(np, origin[a], nc, nlev)) return false;
    return true;
}

bool resolve(const ndgp_grid *g, const ndgp_params *p, Cfg &c, std::string &why) {
    if (!g || !p) {
        why = "grid and params must not be NULL";
        return false;
    }
    if (!pow2(g->n) || g->n < 8 || g->n > 1024) {
        why = "n must be a power of two in [8, 1024]";
        return false;
    }
    if (!finite_pos(g->h)) {
        why = "h must be finite and > 0";
        return false;
    }
    if (!(std::isfinite(p->rc) && p->rc >= 0.0) || !finite_pos(p->beta) || !finite_pos(p->a) ||
        !finite_pos(p->omega_m)) {
        why = "need rc >= 0 and beta, a, omega_m > 0, all finite";
        return false;
    }
    if (!(std::isfinite(p->tol) && p->tol >= 0.0)) {
        why = "tol must be finite and >= 0";
        return false;
    }
    c.n = g->n;
    c.lgn = ilog2(g->n);
    c.h = g->h;
    c.maxc = p->max_cycles ? p->max_cycles : 50;
    c.nu1 = p->nu1 ? p->nu1 : 2;
    c.nu2 = p->nu2 ? p->nu2 : 2;
    if (c.maxc < 1 || c.maxc > 1000 || c.nu1 < 1 || c.nu1 > 16 || c.nu2 < 1 || c.nu2 > 16) {
        why = "max_cycles must be in [1, 1000] and nu1, nu2 in [1, 16] (0 = default)";
        return false;
    }
    c.nl = p->n_levels ? p->n_levels : default_levels(c.n);
    if (c.nl < 1 || c.nl > c.lgn || (c.n >> (c.nl - 1)) > kCoarsestMax) {
        why = "n_levels must coarsen the domain grid to at most 8 and at least 2 cells per side";
        return false;
    }
    if (p->mode != NDGP_MODE_FULL && p->mode != NDGP_MODE_INTERPOLATED &&
        p->mode != NDGP_MODE_TRUNCATED) {
        why = "unknown mode";
        return false;
    }
    if (p->precision != NDGP_PREC_FP64 && p->precision != NDGP_PREC_MIXED) {
        why = "unknown precision";
        return false;
    }
    if (p->flags & ~(NDGP_WARM_START | NDGP_PROFILE | NDGP_TWO_PASS | NDGP_DAMPED)) {
        why = "unknown flag bits";
        return false;
    }
    c.mode = p->mode;
    c.prec = p->precision;
    c.flags = p->flags;
    c.tol = p->tol;
    c.alpha = p->rc * p->rc / (3.0 * p->beta * p->a * p->a);
    c.fsrc = p->omega_m / (p->a * p->beta);
    if (g->n_patch < 0 || g->n_patch > NDGP_MAX_PATCHES) {
        why = "n_patch must be in [0, " + std::to_string(NDGP_MAX_PATCHES) + "]";
        return false;
    }
    c.np = g->n_patch;
    // Sec. IV.A: levels from l_trunc = l_d + trunc_level on are interpolated
    if (c.mode == NDGP_MODE_TRUNCATED) {
        if (p->trunc_level < 1 || p->trunc_level > c.np + 1) {
            why = "trunc_level must be in [1, n_patch + 1]";
            return false;
        }
        c.nrelax = p->trunc_level - 1;
    } else {
        c.nrelax = c.mode == NDGP_MODE_FULL ? c.np : 0;
    }
    for (int q = 0; q < c.np; ++q) {
        const int m = g->patch_n[q];
        const int parent_n = q == 0 ? c.n : c.pn[q - 1];
        if (!pow2(m) || m < 8 || m > 512 || m > 2 * parent_n) {
            why = "patch_n must be a power of two in [8, 512] covering at most its parent";
            return false;
        }
        c.pn[q] = m;
        c.pnl[q] = default_levels(m);
        for (int a = 0; a < 3; ++a) {
            const int o = g->patch_origin[q][a];
            if (o < -4 * c.n || o > 4 * c.n) {
                why = "patch origin out of range";
                return false;
            }
            c.po[q][a] = o;
        }
        if (q >= 1) {
            const int need = q < c.nrelax ? c.pnl[q] : 1;
            if (!child_fits(c.pn[q - 1], c.po[q], m, need)) {
                why = "patch " + std::to_string(q + 1) + " must lie inside patch " +
                      std::to_string(q) + " with room for the interpolation stencils of its " +
                      (q < c.nrelax ? "multigrid levels" : "cells");
                return false;
            }
        }
    }
    return true;
}

// ------------------------------------------------------------------------
// workspace

// Debugging aid: with the environment variable NDGP_GUARD_BANDS=1 (read once
// per process) every sub-buffer of the solve's workspace is followed by a
// guard band of kGuardWords words holding kGuardWord, written after the
// carve and checked when the solve ends; an overwritten band fails the call
// with NDGP_EDEVICE.  The workspace sizes grow to match.
constexpr size_t kGuardWords = 32;
constexpr uint64_t kGuardWord = 0x7ff4dead5eedbeefull; // a signalling-NaN payload

bool guard_bands_on() {
    static const bool on = [] {
        const char *v = std::getenv("NDGP_GUARD_BANDS");
        return v && v[0] && v[0] != '0';
    }();
    return on;
}

struct Carver {
    char *base;
    size_t off = 0;
    std::vector<size_t> *guards = nullptr; // offsets of the guard bands laid out
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        if (guard_bands_on()) {
            off = (off + 255) & ~(size_t)255;
            if (guards) guards->push_back(off);
            off += kGuardWords * sizeof(uint64_t);
        }
        return p;
    }
};

// FP32 V-cycles on the correction per FP64 defect-correction iteration
constexpr int kMixedInner = 2;

struct Plan {
    Cfg c;
    Level base[kMaxLevels];
    Level32 base32[kMaxLevels]; // mixed precision only
    Level patch[NDGP_MAX_PATCHES][kMaxLevels];
    unsigned char *mask[NDGP_MAX_PATCHES][kMaxLevels] = {}; // cell-wise truncation
    unsigned char *active[NDGP_MAX_PATCHES] = {}; // block activity of each patch's finest mask
    double *partials = nullptr;
    double *scal = nullptr; // [0] sum delta, [1] sum s^2, [2] sum r^2, [3] sum phi
    unsigned *fallbacks = nullptr;
    bool phi32_fresh = false; // base32[0].phi holds (float) base[0].phi
    char *ws = nullptr;               // the carved workspace (guard bands on)
    std::vector<size_t> guards;       // their offsets in it
};

// Lays out every array in `base` (or only counts bytes when base == nullptr).
size_t carve(Plan &P, char *base) {
    Carver cv{base};
    P.guards.clear();
    P.ws = base;
    if (base) cv.guards = &P.guards;
    const Cfg &c = P.c;
    for (int l = 0; l < c.nl; ++l) {
        Level &L = P.base[l];
        L.n = c.n >> l;
        L.lg = c.lgn - l;
        L.periodic = true;
        const double hl = c.h * (double)(1 << l);
        L.alpha = c.alpha / (hl * hl);
        L.phi = l ? cv.take<double>(L.slots()) : nullptr;
        L.alt = cv.take<double>(L.slots());
        L.s = cv.take<double>(L.cells());
        L.hat = l ? cv.take<double>(L.slots()) : nullptr;
    }
    if (c.prec == NDGP_PREC_MIXED) {
        for (int l = 0; l < c.nl; ++l) {
            Level32 &L = P.base32[l];
            L.n = c.n >> l;
            L.lg = c.lgn - l;
            L.alpha = P.base[l].alpha;
            L.phi = cv.take<float>(L.cells());
            L.e = cv.take<float>(L.cells());
            L.ealt = cv.take<float>(L.cells());
            L.r = cv.take<float>(L.cells());
            L.ehat = l ? cv.take<float>(L.cells()) : nullptr;
        }
    }
    {
        for (int q = 0; q < c.nrelax; ++q) {
            const double hp = c.hl(q + 1);
            for (int m = 0; m < c.pnl[q]; ++m) {
                Level &L = P.patch[q][m];
                L.n = c.pn[q] >> m;
                L.lg = ilog2(L.n);
                L.periodic = false;
                const double hm = hp * (double)(1 << m);
                L.alpha = c.alpha / (hm * hm);
                L.phi = m ? cv.take<double>(L.slots()) : nullptr;
                L.alt = cv.take<double>(L.slots());
                L.s = cv.take<double>(L.cells());
                L.hat = m ? cv.take<double>(L.slots()) : nullptr;
                L.dyn_bc = m > 0;
                P.mask[q][m] = cv.take<unsigned char>(L.cells());
            }
            P.active[q] = cv.take<unsigned char>(block_activity_bytes(c.pn[q]));
        }
    }
    P.partials = cv.take<double>(kReduceBlocks);
    P.scal = cv.take<double>(16);
    P.fallbacks = cv.take<unsigned>(16);
    return cv.off;
}

void arm_guards(const Plan &P, hipStream_t st) {
    for (size_t off : P.guards)
        launch_guard_fill(P.ws + off, (int)kGuardWords, kGuardWord, st);
}

// counts overwritten guard words into P.fallbacks[2]
void check_guards(const Plan &P, hipStream_t st) {
    for (size_t off : P.guards)
        launch_guard_check(P.ws + off, (int)kGuardWords, kGuardWord, P.fallbacks + 2, st);
}

// workspace of ndgp_residual on the largest level
size_t residual_bytes(const Cfg &c) {
    size_t cells = (size_t)c.n * c.n * c.n;
    for (int q = 0; q < c.np; ++q) cells = std::max(cells, (size_t)c.pn[q] * c.pn[q] * c.pn[q]);
    Carver cv{nullptr};
    cv.take<double>(cells);
    cv.take<double>(kReduceBlocks);
    cv.take<double>(16);
    return cv.off;
}

size_t total_bytes(const Cfg &c) {
    Plan P;
    P.c = c;
    return std::max(carve(P, nullptr), residual_bytes(c)) + 256;
}

char *aligned_base(void *ws) {
    const uintptr_t u = reinterpret_cast<uintptr_t>(ws);
    return reinterpret_cast<char *>((u + 255) & ~(uintptr_t)255);
}

// ------------------------------------------------------------------------
// the multigrid driver

// HIP events around the domain level's relaxation phases (NDGP_PROFILE)
struct SmoothTimer {
    bool on = false;
    std::vector<hipEvent_t> ev; // start/stop pairs
    int launches = 0;
    size_t cells_per_launch = 0;
    ~SmoothTimer() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    void mark(hipStream_t st) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        ev.push_back(e);
        HIP_TRY(hipEventRecord(e, st));
    }
    double total_ms() {
        double t = 0.0;
        for (size_t q = 0; q + 1 < ev.size(); q += 2) {
            HIP_TRY(hipEventSynchronize(ev[q + 1]));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev[q], ev[q + 1]));
            t += ms;
        }
        return t;
    }
};

// The monitor of a level's cycles (CycleMonitor, ndgp_internal.h), with the
// status of its end as an error message.
ndgp_status verdict(const CycleMonitor &m) {
    switch (m.verdict_code()) {
    case kTolNotReached: return fail(NDGP_ENOCONV, "tolerance not reached within max_cycles");
    case kStagnated: return fail(NDGP_ENOCONV, "stagnated above rounding level");
    default: return NDGP_OK;
    }
}

inline void set_step(Level *H, Level32 *H32, int nl, double w) {
    for (int l = 0; l < nl; ++l) {
        H[l].omega = w;
        if (H32) H32[l].omega = w;
    }
}

struct Runner {
    Plan &P;
    hipStream_t st;
    double *host;
    SmoothTimer *timer = nullptr; // times smooth() calls on this level's arrays
    const double *timed_s = nullptr;

    double read_scalar(const double *dev) {
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(host, dev, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        return host[0];
    }

    // host[0..count) = dev[0..count) with one copy and one wait
    void read_scalars(const double *dev, int count) {
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(host, dev, count * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }

    // enqueue a reduction into P.scal[slot] without waiting for it
    void enqueue_sum(const double *a, size_t count, bool squares, int slot) {
        launch_partial_sums(a, count, squares, P.partials, st);
        launch_reduce_final(P.partials, P.scal + slot, st);
    }

    void enqueue_residual(Level *H, Level32 *H32) {
        if (P.c.prec == NDGP_PREC_MIXED)
            launch_residual_to32(H[0], H32[0].r, P.partials, st);
        else
            launch_residual_sumsq(H[0], P.partials, nullptr, 0.0, st);
        launch_reduce_final(P.partials, P.scal + 2, st);
    }

    // one outer iteration of the mixed-precision loop (without its residual)
    // (phi += e also leaves the FP32 copy of phi for the next iteration)
    void mixed_outer(Level *H, Level32 *H32, int nl) {
        const size_t cells = H[0].cells();
        if (!P.phi32_fresh) launch_to32(H[0].phi, H32[0].phi, cells, st);
        for (int l = 1; l < nl; ++l) launch_avg32(H32[l - 1], H32[l], st);
        // the correction starts from zero: the first fused sweep takes it as
        // such without reading it, else it is filled
        const bool from_zero = corr_first_sweep_from_zero(H32[0]);
        if (!from_zero) launch_fill32(H32[0].e, cells, 0.f, st);
        for (int q = 0; q < kMixedInner; ++q) corr_vcycle(H32, nl, 0, from_zero && q == 0);
        launch_add_to32(H[0].phi, H32[0].e, H32[0].phi, cells, st);
        P.phi32_fresh = true;
    }

    double sum(const double *a, size_t count, bool squares, int slot) {
        launch_partial_sums(a, count, squares, P.partials, st);
        launch_reduce_final(P.partials, P.scal + slot, st);
        return read_scalar(P.scal + slot);
    }

    double residual_sumsq(const Level &L) {
        launch_residual_sumsq(L, P.partials, nullptr, 0.0, st);
        launch_reduce_final(P.partials, P.scal + 2, st);
        return read_scalar(P.scal + 2);
    }

    // `sweeps` red-black sweeps; the iterate ends in the buffer it started in
    // (the fused kernel swaps once per sweep, so an odd last sweep takes the
    // two-launch path, which swaps twice).  With C the coarse-grid correction
    // from C is added first: on load in the first fused sweep, else by its
    // own launch.
    void smooth(Level &L, int sweeps, const Level *C = nullptr) {
        const bool fused = !(P.c.flags & NDGP_TWO_PASS) && fused_sweep_ok(L);
        const int nf = fused ? (sweeps & ~1) : 0;
        const bool pro = nf > 0 && fused_prolong_ok(L); // the correction added on load
        int s = 0;
        if (C && !pro) launch_prolong_correct(L, *C, st);
        if (C && pro) {
            launch_sweep_fused_prolong(L, *C, L.phi, L.alt, P.fallbacks, st);
            std::swap(L.phi, L.alt);
            s = 1;
        }
        // the timed launches: plain fused sweeps (or half sweeps) only
        const bool timed = timer && timer->on && L.s == timed_s;
        if (timed) timer->mark(st);
        for (; s < nf; ++s) {
            launch_sweep_fused(L, L.phi, L.alt, P.fallbacks, st);
            std::swap(L.phi, L.alt);
        }
        for (s = nf; s < sweeps; ++s)
            for (int col = 0; col < 2; ++col) {
                launch_smooth_half(L, L.phi, L.alt, col, P.fallbacks, st);
                std::swap(L.phi, L.alt);
            }
        if (timed) {
            timer->mark(st);
            timer->launches += (C && nf > 0 ? nf - 1 : nf) + 2 * (sweeps - nf);
            timer->cells_per_launch = nf ? L.cells() : L.cells() / 2;
        }
    }

    void vcycle(Level *H, int nl, int l) {
        Level &L = H[l];
        if (l == nl - 1) {
            launch_coarsest(L, kCoarsestSweeps, P.fallbacks, st);
            return;
        }
        if (!(P.c.flags & NDGP_TWO_PASS) && bottom_ok(H, l, nl)) {
            launch_bottom(H, l, nl, P.c.nu1, P.c.nu2, kCoarsestSweeps, P.fallbacks, st);
            return;
        }
        if (!(P.c.flags & NDGP_TWO_PASS) && bottom_dir_ok(H, l, nl)) {
            launch_bottom_dir(H, l, nl, P.c.nu1, P.c.nu2, kCoarsestSweeps, P.fallbacks, st);
            return;
        }
        smooth(L, P.c.nu1);
        Level &C = H[l + 1];
        launch_restrict_residual(L, C, !(P.c.flags & NDGP_TWO_PASS), st);
        launch_coarse_source(C, !(P.c.flags & NDGP_TWO_PASS), st);
        vcycle(H, nl, l + 1);
        smooth(L, P.c.nu2, &C);
    }

    // Initial guess by nested iteration: average the source down, solve the
    // coarsest level, then interpolate each solution up and improve it by one
    // V-cycle (the way the paper starts a refinement from its coarser level,
    // applied to the multigrid levels; a zero guess can diverge for strongly
    // screened sources).
    void nested_start(Level *H, int nl) {
        P.phi32_fresh = false;
        for (int l = 1; l < nl; ++l) launch_restrict_source(H[l - 1], H[l], st);
        launch_fill(H[nl - 1].phi, H[nl - 1].slots(), 0.0, st);
        launch_coarsest(H[nl - 1], kCoarsestSweeps, P.fallbacks, st);
        for (int l = nl - 2; l >= 0; --l) {
            launch_prolong_full(H[l], H[l + 1], st);
            if (l > 0) vcycle(H, nl, l);
        }
    }

    // ---- mixed precision: FP32 FAS on the correction e of
    //      L[phi + e] - L[phi] = r, inside an FP64 defect-correction loop
    // as smooth(): fused sweeps on large levels, an odd last sweep in two
    // launches.  (Adding the coarse-grid correction on load, as the FP64
    // sweep does, spills registers here and is slower than its own launch.)
    bool corr_first_sweep_from_zero(const Level32 &L) const {
        return !(P.c.flags & NDGP_TWO_PASS) && corr_fused_ok(L) && P.c.nu1 >= 2;
    }

    // with C the coarse-grid correction from C is added first: on load in
    // the first fused sweep, else by its own launch (same bits); with
    // from_zero the correction is zero and the first fused sweep does not
    // read it (corr_first_sweep_from_zero(L) holds)
    void corr_smooth(Level32 &L, int sweeps, const Level32 *C = nullptr, bool from_zero = false) {
        const bool fused = !(P.c.flags & NDGP_TWO_PASS) && corr_fused_ok(L);
        const int nf = fused ? (sweeps & ~1) : 0;
        int s = 0;
        if (from_zero) {
            launch_corr_sweep_fused_from_zero(L, L.ealt, P.fallbacks, st);
            std::swap(L.e, L.ealt);
            s = 1;
        }
        if (C && nf == 0) launch_corr_prolong(L, *C, st);
        if (C && nf > 0) {
            launch_corr_sweep_fused_prolong(L, *C, L.e, L.ealt, P.fallbacks, st);
            std::swap(L.e, L.ealt);
            s = 1;
        }
        for (; s < nf; ++s) {
            launch_corr_sweep_fused(L, L.e, L.ealt, P.fallbacks, st);
            std::swap(L.e, L.ealt);
        }
        for (int s = nf; s < sweeps; ++s)
            for (int col = 0; col < 2; ++col) {
                launch_corr_half(L, L.e, L.ealt, col, P.fallbacks, st);
                std::swap(L.e, L.ealt);
            }
    }

    void corr_vcycle(Level32 *H, int nl, int l, bool from_zero = false) {
        Level32 &L = H[l];
        if (l == nl - 1) {
            launch_corr_coarsest(L, kCoarsestSweeps, P.fallbacks, st);
            return;
        }
        corr_smooth(L, P.c.nu1, nullptr, from_zero);
        Level32 &C = H[l + 1];
        launch_corr_restrict(L, C, !(P.c.flags & NDGP_TWO_PASS), st);
        launch_corr_coarse_source(C, st);
        corr_vcycle(H, nl, l + 1);
        corr_smooth(L, P.c.nu2, &C);
    }

    double residual_to32(const Level &L, float *r32) {
        launch_residual_to32(L, r32, P.partials, st);
        launch_reduce_final(P.partials, P.scal + 2, st);
        return read_scalar(P.scal + 2);
    }

    // Outer iterations: r = s - L[phi] in FP64 (also the stopping test), the
    // FP32 copy of phi on every level, kMixedInner FP32 V-cycles on the
    // correction from e = 0, phi += e in FP64.
    // cycles accumulates over a restart; *restart is set (and the call
    // returns) when the safeguard asks for a damped solve from the start.
    // rr0 >= 0: the squared residual norm of the start, already enqueued
    // (enqueue_residual) and read; else it is computed here
    ndgp_status drive_mixed(Level *H, Level32 *H32, int nl, double snorm2, int &outer,
                            double &rel, double *hist, int *hist_len, bool *restart,
                            double rr0 = -1.0) {
        CycleMonitor m{P.c.tol, P.c.maxc};
        m.damped = H[0].omega != 1.0;
        m.start(std::sqrt((rr0 >= 0.0 ? rr0 : residual_to32(H[0], H32[0].r)) / snorm2));
        rel = m.rel;
        while (outer < m.maxc && !m.converged()) {
            mixed_outer(H, H32, nl);
            ++outer;
            const double r = std::sqrt(residual_to32(H[0], H32[0].r) / snorm2);
            if (hist && outer - 1 < NDGP_HIST_LEN) {
                hist[outer - 1] = r;
                *hist_len = outer;
            }
            const bool again = m.record(r);
            rel = m.rel;
            if (again && restart) {
                *restart = true;
                return NDGP_OK;
            }
            if (m.diverged()) return fail(NDGP_ENOCONV, "mixed-precision iteration diverged");
            if (m.stalled()) break;
        }
        return verdict(m);
    }

    // V-cycles on H[0] until ||r|| <= tol ||s|| (tol > 0) or until the
    // residual stops falling (tol == 0); cycles and restart as drive_mixed.
    ndgp_status drive(Level *H, int nl, double snorm2, int &cycles, double &rel, double *hist,
                      int *hist_len, bool *restart, double rr0 = -1.0) {
        CycleMonitor m{P.c.tol, P.c.maxc};
        m.damped = H[0].omega != 1.0;
        m.start(std::sqrt((rr0 >= 0.0 ? rr0 : residual_sumsq(H[0])) / snorm2));
        rel = m.rel;
        while (cycles < m.maxc && !m.converged()) {
            vcycle(H, nl, 0);
            ++cycles;
            const double r = std::sqrt(residual_sumsq(H[0]) / snorm2);
            if (hist && cycles - 1 < NDGP_HIST_LEN) {
                hist[cycles - 1] = r;
                *hist_len = cycles;
            }
            const bool again = m.record(r);
            rel = m.rel;
            if (again && restart) {
                *restart = true;
                return NDGP_OK;
            }
            if (m.diverged()) return fail(NDGP_ENOCONV, "multigrid diverged");
            if (m.stalled()) break;
        }
        return verdict(m);
    }
};

// One refinement relaxed from its solved parent (Sec. III.A).  The caller has
// interpolated the parent into the patch's field (H[0].phi, interior and ghost
// shell) and set any cell masks; here the ghost shells of the other arrays of
// every level of the patch's own hierarchy are interpolated too, the source
// S = Omega_m (delta - mean)/(a beta) is formed against the domain's mean
// (whose sum sits in P.scal[0]), and FAS V-cycles run to the tolerance, with
// the divergence safeguard.
struct PatchOutcome {
    int cycles = 0;
    double rel = 0.0;
    int damped_from = 0;
    ndgp_status status = NDGP_OK;
};

PatchOutcome relax_patch(Runner &run, Level *H, int nlev, const double *parent, int npar,
                         bool parent_periodic, const int origin[3], int m, double hq,
                         const double *delta, double inv_cells0) {
    const Cfg &c = run.P.c;
    hipStream_t st = run.st;
    PatchOutcome out;
    ChildBox b0{{origin[0], origin[1], origin[2]}, 0, m};
    // with held cells the partner array holds their values too (blocks of held
    // cells are never written again)
    launch_interpolate(parent, npar, parent_periodic, b0, H[0].alt, H[0].active == nullptr, st);
    for (int l = 1; l < nlev; ++l) {
        ChildBox bm{{origin[0], origin[1], origin[2]}, l, m >> l};
        launch_interpolate(parent, npar, parent_periodic, bm, H[l].phi, true, st);
        launch_interpolate(parent, npar, parent_periodic, bm, H[l].alt, true, st);
        launch_interpolate(parent, npar, parent_periodic, bm, H[l].hat, true, st);
    }
    const size_t cq = (size_t)m * m * m;
    launch_source(delta, cq, run.P.scal + 0, inv_cells0, c.fsrc * hq * hq, H[0].s, st);
    double sn2 = run.sum(H[0].s, cq, true, 1);
    if (!std::isfinite(sn2)) {
        out.status = fail(NDGP_EINVAL, "a patch density has non-finite values");
        return out;
    }
    if (sn2 == 0.0) sn2 = std::max(run.residual_sumsq(H[0]), 1e-300);
    bool restart = false;
    if (c.flags & NDGP_DAMPED) {
        set_step(H, nullptr, nlev, kDampedStep);
        out.damped_from = 1;
    }
    out.status = run.drive(H, nlev, sn2, out.cycles, out.rel, nullptr, nullptr, &restart);
    if (restart) { // the safeguard: from the interpolated guess again, damped
        set_step(H, nullptr, nlev, kDampedStep);
        out.damped_from = out.cycles + 1;
        launch_interpolate(parent, npar, parent_periodic, b0, H[0].phi, false, st);
        out.status = run.drive(H, nlev, sn2, out.cycles, out.rel, nullptr, nullptr, nullptr);
    }
    return out;
}

ndgp_status check_arrays(const Cfg &c, const double *const *delta, double *const *phi) {
    if (!delta || !phi || !delta[0] || !phi[0])
        return fail(NDGP_EINVAL, "delta[0] and phi[0] must not be NULL");
    if (reinterpret_cast<uintptr_t>(phi[0]) % 16 != 0)
        return fail(NDGP_EINVAL, "phi[0] must be 16-byte aligned");
    for (int q = 0; q < c.np; ++q) {
        if (!phi[q + 1]) return fail(NDGP_EINVAL, "phi of every patch must not be NULL");
        if (q < c.nrelax && !delta[q + 1])
            return fail(NDGP_EINVAL, "delta of every relaxed patch must not be NULL");
    }
    return NDGP_OK;
}

// Cell-wise truncation (Sec. III.C) when psi != nullptr: psi[l] is the
// Newtonian potential of level l (layout of phi[l]) for every parent of a
// relaxed patch, and threshold the fifth-to-Newtonian force ratio below
// which a parent's children are held.
ndgp_status solve_impl(const ndgp_grid *grid, const ndgp_params *params,
                       const double *const delta[], double *const phi[], void *ws,
                       size_t ws_bytes, hipStream_t st, ndgp_report *rep,
                       const double *const *psi = nullptr, double threshold = 0.0) {
    const auto t0 = std::chrono::steady_clock::now();
    Plan P;
    std::string why;
    if (!resolve(grid, params, P.c, why)) return fail(NDGP_EINVAL, why);
    const Cfg &c = P.c;
    ndgp_status s = check_arrays(c, delta, phi);
    if (s != NDGP_OK) return s;
    if (psi) {
        if (!(threshold >= 0.0)) return fail(NDGP_EINVAL, "threshold must be >= 0 (not NaN)");
        for (int q = 0; q < c.nrelax; ++q)
            if (!psi[q])
                return fail(NDGP_EINVAL, "psi of the domain and of every parent of a relaxed "
                                         "patch must not be NULL");
    }
    const size_t need = total_bytes(c);
    if (!ws || ws_bytes < need)
        return fail(NDGP_ENOMEM, "workspace smaller than ndgp_workspace_bytes() = " +
                                     std::to_string(need));
    carve(P, aligned_base(ws));
    P.base[0].phi = phi[0];
    arm_guards(P, st);

    ndgp_report R;
    std::memset(&R, 0, sizeof(R));
    for (int l = 0; l <= NDGP_MAX_PATCHES; ++l) R.rel_res[l] = -1.0;
    R.iterated_fraction[0] = 1.0;
    for (int q = 0; q < c.nrelax; ++q) R.iterated_fraction[q + 1] = 1.0;
    SlotGuard slot;
    SmoothTimer timer;
    Runner run{P, st, slot.p};
    run.timer = &timer;
    run.timed_s = P.base[0].s;
    HIP_TRY(hipMemsetAsync(P.fallbacks, 0, 3 * sizeof(unsigned), st));

    // domain source: S = Omega_m (delta - mean) / (a beta), in cell units (x
    // h^2); its norm, the initial guess and the first residual norm are
    // enqueued together and read with one wait
    const size_t cells0 = (size_t)c.n * c.n * c.n;
    run.enqueue_sum(delta[0], cells0, false, 0);
    launch_source(delta[0], cells0, P.scal + 0, 1.0 / (double)cells0, c.fsrc * c.h * c.h,
                  P.base[0].s, st);
    run.enqueue_sum(P.base[0].s, cells0, true, 1);
    if (c.flags & NDGP_DAMPED) { // the damped step from the start
        set_step(P.base, c.prec == NDGP_PREC_MIXED ? P.base32 : nullptr, c.nl, kDampedStep);
        R.damped_from[0] = 1;
    }
    if (!(c.flags & NDGP_WARM_START)) run.nested_start(P.base, c.nl);
    run.enqueue_residual(P.base, P.base32);
    run.read_scalars(P.scal, 3);
    const double dsum = slot.p[0], snorm2 = slot.p[1], rr0 = slot.p[2];
    if (!std::isfinite(dsum)) return fail(NDGP_EINVAL, "delta[0] has non-finite values");
    R.removed_mean = dsum / (double)cells0;

    ndgp_status status = NDGP_OK;
    if (snorm2 == 0.0) {
        launch_fill(phi[0], cells0, 0.0, st); // no source: phi = 0
        R.rel_res[0] = 0.0;
    } else {
        double rel = 0.0;
        Range domain("ndgp domain V-cycles");
        for (bool first = true;; first = false) {
            if (!first) run.nested_start(P.base, c.nl); // the first start is enqueued above
            timer.on = (c.flags & NDGP_PROFILE) != 0; // the V-cycles only, not the start
            bool restart = false;
            if (c.prec == NDGP_PREC_MIXED)
                status = run.drive_mixed(P.base, P.base32, c.nl, snorm2, R.cycles[0], rel,
                                         R.res_hist, &R.hist_len, first ? &restart : nullptr,
                                         first ? rr0 : -1.0);
            else
                status = run.drive(P.base, c.nl, snorm2, R.cycles[0], rel, R.res_hist,
                                   &R.hist_len, first ? &restart : nullptr, first ? rr0 : -1.0);
            timer.on = false;
            if (!restart) break;
            // the safeguard: solve again from the nested start with the damped step
            set_step(P.base, c.prec == NDGP_PREC_MIXED ? P.base32 : nullptr, c.nl, kDampedStep);
            R.damped_from[0] = R.cycles[0] + 1;
        }
        R.rel_res[0] = rel;
        if (timer.launches) {
            R.t_smooth_ms = timer.total_ms();
            R.smooth_launches = timer.launches;
            R.smooth_cells_per_launch = (int32_t)timer.cells_per_launch;
        }
        if (status != NDGP_OK && !std::isfinite(rel)) {
            if (rep) *rep = R;
            return status;
        }
    }
    // gauge: only derivatives of phi enter, report the zero-mean field
    const double psum = run.sum(phi[0], cells0, false, 3);
    R.phi_mean = psum / (double)cells0;
    launch_shift_by_mean(phi[0], cells0, P.scal + 3, st);

    if (psi) // the Newtonian potentials of the parents must be finite everywhere
        for (int q = 0; q < c.nrelax; ++q) {
            const size_t np3 = q == 0 ? cells0 : (size_t)(c.pn[q - 1] + 2) * (c.pn[q - 1] + 2) *
                                                     (c.pn[q - 1] + 2);
            if (!std::isfinite(run.sum(psi[q], np3, false, 5)))
                return fail(NDGP_EINVAL, "psi[" + std::to_string(q) + "] has non-finite values");
        }
    for (int q = 0; q < c.np; ++q) {
        const bool parent_periodic = q == 0;
        const double *parent = phi[q];
        const int npar = q == 0 ? c.n : c.pn[q - 1];
        ChildBox b0{{c.po[q][0], c.po[q][1], c.po[q][2]}, 0, c.pn[q]};
        launch_interpolate(parent, npar, parent_periodic, b0, phi[q + 1], false, st);
        if (q >= c.nrelax) continue; // Sec. III.B: a truncated level keeps the guess
        Level *H = P.patch[q];
        H[0].phi = phi[q + 1];
        if (psi) { // Sec. III.C: iterate only where the parent's fifth force is large
            launch_cell_mask(parent, psi[q], npar, parent_periodic, b0, threshold, P.mask[q][0],
                             P.partials, st);
            launch_reduce_final(P.partials, P.scal + 8 + q, st); // read after the last patch
            H[0].mask = P.mask[q][0];
            launch_block_activity(P.mask[q][0], c.pn[q], P.active[q], st);
            H[0].active = P.active[q];
            H[0].tile_on = tile_activity(P.active[q], c.pn[q]);
            for (int m = 1; m < c.pnl[q]; ++m) {
                launch_mask_restrict(P.mask[q][m - 1], H[m].n, P.mask[q][m], st);
                H[m].mask = P.mask[q][m];
            }
        }
        Range patch_range("ndgp refinement");
        const PatchOutcome po = relax_patch(run, H, c.pnl[q], parent, npar, parent_periodic,
                                            c.po[q], c.pn[q], c.hl(q + 1), delta[q + 1],
                                            1.0 / (double)cells0);
        if (po.status == NDGP_EINVAL) return po.status;
        const double rel = po.rel;
        const ndgp_status sq = po.status;
        R.cycles[q + 1] = po.cycles;
        R.damped_from[q + 1] = po.damped_from;
        R.rel_res[q + 1] = rel;
        if (sq != NDGP_OK && status == NDGP_OK) status = sq;
    }
    unsigned fb[3] = {0, 0, 0};
    check_guards(P, st);
    HIP_TRY(hipGetLastError());
    if (psi && c.nrelax > 0) // iterated cells per masked patch, counted on the device
        HIP_TRY(hipMemcpyAsync(slot.p + 8, P.scal + 8, c.nrelax * sizeof(double),
                               hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(slot.p, P.fallbacks, 3 * sizeof(unsigned), hipMemcpyDeviceToHost,
                           st));
    HIP_TRY(hipStreamSynchronize(st));
    std::memcpy(fb, slot.p, 3 * sizeof(unsigned));
    if (fb[2]) return fail(NDGP_EDEVICE, std::to_string(fb[2]) + " workspace guard-band words "
                                         "were overwritten");
    R.fallbacks = (int32_t)fb[0];
    R.holds = (int32_t)fb[1];
    if (psi)
        for (int q = 0; q < c.nrelax; ++q)
            R.iterated_fraction[q + 1] = slot.p[8 + q] / ((double)c.pn[q] * c.pn[q] * c.pn[q]);
    R.t_total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = R;
    return status;
}

// ------------------------------------------------------------------------
// adaptive refinement: a tree of cubic boxes, several per level (Sec. IV.A)

struct AmrTree {
    int nb = 0;
    int parent[NDGP_AMR_MAX_BOXES] = {};
    int n[NDGP_AMR_MAX_BOXES] = {};
    int depth[NDGP_AMR_MAX_BOXES] = {};
    int nlev[NDGP_AMR_MAX_BOXES] = {};
    int origin[NDGP_AMR_MAX_BOXES][3] = {};
    bool relaxed[NDGP_AMR_MAX_BOXES] = {};
    int max_relaxed_n = 0; // largest relaxed box (0: none)
};

// [o1, o1 + w1) and [o2, o2 + w2) intersect, on a ring of `period` cells if
// period > 0
bool spans_overlap(int o1, int w1, int o2, int w2, int period) {
    if (period <= 0) return o1 < o2 + w2 && o2 < o1 + w1;
    const int d12 = ((o2 - o1) % period + period) % period;
    const int d21 = ((o1 - o2) % period + period) % period;
    return d12 < w1 || d21 < w2;
}

bool resolve_tree(const ndgp_grid *grid, const ndgp_params *params, const ndgp_box *boxes,
                  int nb, Cfg &c, AmrTree &T, std::string &why) {
    if (!grid || !params) {
        why = "grid and params must not be NULL";
        return false;
    }
    if (grid->n_patch != 0) {
        why = "the tree's boxes replace ndgp_grid's nested patches: n_patch must be 0";
        return false;
    }
    ndgp_params p0 = *params; // the domain level's own checks
    p0.mode = NDGP_MODE_FULL;
    p0.trunc_level = 0;
    if (!resolve(grid, &p0, c, why)) return false;
    c.mode = params->mode;
    if (c.mode == NDGP_MODE_TRUNCATED && params->trunc_level < 1) {
        why = "trunc_level must be >= 1";
        return false;
    }
    if (nb < 0 || nb > NDGP_AMR_MAX_BOXES || (nb > 0 && !boxes)) {
        why = "n_boxes must be in [0, NDGP_AMR_MAX_BOXES] with a box list";
        return false;
    }
    T.nb = nb;
    for (int b = 0; b < nb; ++b) {
        const ndgp_box &x = boxes[b];
        if (x.parent < -1 || x.parent >= b) {
            why = "box " + std::to_string(b) + ": parent must be -1 or an earlier box";
            return false;
        }
        const int pn = x.parent < 0 ? c.n : T.n[x.parent];
        if (!pow2(x.n) || x.n < 8 || x.n > 512 || x.n > 2 * pn) {
            why = "box " + std::to_string(b) +
                  ": n must be a power of two in [8, 512] covering at most its parent";
            return false;
        }
        T.parent[b] = x.parent;
        T.n[b] = x.n;
        T.depth[b] = x.parent < 0 ? 1 : T.depth[x.parent] + 1;
        T.nlev[b] = default_levels(x.n);
        T.relaxed[b] = c.mode == NDGP_MODE_FULL ||
                       (c.mode == NDGP_MODE_TRUNCATED && T.depth[b] < params->trunc_level);
        if (T.depth[b] > 20) {
            why = "tree deeper than 20 levels";
            return false;
        }
        for (int a = 0; a < 3; ++a) {
            T.origin[b][a] = x.origin[a];
            if (x.origin[a] < -4 * pn || x.origin[a] > 4 * pn) {
                why = "box " + std::to_string(b) + ": origin out of range";
                return false;
            }
        }
        if (x.parent >= 0 && !child_fits(pn, x.origin, x.n, T.relaxed[b] ? T.nlev[b] : 1)) {
            why = "box " + std::to_string(b) + " must lie inside its parent box with room for "
                  "the interpolation stencils of its " +
                  (T.relaxed[b] ? "multigrid levels" : "cells");
            return false;
        }
        for (int q = 0; q < b; ++q) {
            if (T.parent[q] != x.parent) continue;
            const int period = x.parent < 0 ? c.n : 0;
            bool all = true;
            for (int a = 0; a < 3; ++a)
                all = all && spans_overlap(T.origin[q][a], T.n[q] / 2, x.origin[a], x.n / 2, period);
            if (all) {
                why = "boxes " + std::to_string(q) + " and " + std::to_string(b) +
                      " (same parent) overlap";
                return false;
            }
        }
        if (T.relaxed[b]) T.max_relaxed_n = std::max(T.max_relaxed_n, x.n);
    }
    return true;
}

// the arrays the boxes' relaxation shares (one box at a time): reduction
// scratch, event counters and a hierarchy sized for the largest relaxed box
struct AmrScratch {
    double *phi[kMaxLevels] = {}, *alt[kMaxLevels] = {}, *s[kMaxLevels] = {},
           *hat[kMaxLevels] = {};
    double *partials = nullptr, *scal = nullptr;
    unsigned *fallbacks = nullptr;
    // the boxes solved one workgroup each: descriptors, results, and the
    // global levels of each 32^3 one
    BoxJob *jobs = nullptr;
    BoxResult *results = nullptr;
    double *box32 = nullptr;
};

// scratch doubles of one 32^3 box solved by one workgroup: the finest level's
// partner (padded) and source, its 16^3 level's phi, partner and hat (padded)
// and source
constexpr size_t kBox32Doubles = 34 * 34 * 34 + 32 * 32 * 32 + 3 * 18 * 18 * 18 + 16 * 16 * 16;

size_t carve_amr(AmrScratch &A, char *base, int maxn, int nb = 0, int n32 = 0,
                 std::vector<size_t> *guards = nullptr) {
    Carver cv{base};
    cv.guards = guards;
    A.jobs = cv.take<BoxJob>((size_t)nb);
    A.results = cv.take<BoxResult>((size_t)nb);
    A.box32 = cv.take<double>((size_t)n32 * kBox32Doubles);
    if (maxn > 0) {
        const int nl = default_levels(maxn);
        for (int l = 0; l < nl; ++l) {
            const size_t m = (size_t)(maxn >> l);
            const size_t slots = (m + 2) * (m + 2) * (m + 2);
            A.phi[l] = l ? cv.take<double>(slots) : nullptr;
            A.alt[l] = cv.take<double>(slots);
            A.s[l] = cv.take<double>(m * m * m);
            A.hat[l] = l ? cv.take<double>(slots) : nullptr;
        }
    }
    A.partials = cv.take<double>(kReduceBlocks);
    A.scal = cv.take<double>(16);
    A.fallbacks = cv.take<unsigned>(16);
    return cv.off;
}

// A relaxed box is solved by the one-workgroup kernel if it has at most 16^3
// cells, or 32^3 when at least kBatch32Min boxes of that size share its tree
// level: one workgroup relaxes a 32^3 box's two finer levels from L2, about
// four times as slowly as the per-level launches do one box, so a few such
// boxes go faster one after the other (measured: even at four).
constexpr int kBatch32Min = 4;

struct BatchPlan {
    int n32_at_depth[22] = {}; // relaxed 32^3 boxes per tree level
    bool batched(const Cfg &c, const AmrTree &T, int b) const {
        if (!T.relaxed[b] || T.n[b] > kBoxBatchMaxN || (c.flags & NDGP_TWO_PASS)) return false;
        return T.n[b] < 32 || n32_at_depth[T.depth[b]] >= kBatch32Min;
    }
};

// relaxed boxes that one workgroup each solves, and how many of them are 32^3
int batched_boxes(const Cfg &c, const AmrTree &T, int *n32, BatchPlan *plan = nullptr) {
    BatchPlan bp;
    for (int b = 0; b < T.nb; ++b)
        if (T.relaxed[b] && T.n[b] == 32) ++bp.n32_at_depth[T.depth[b]];
    int k = 0, k32 = 0;
    for (int b = 0; b < T.nb; ++b)
        if (bp.batched(c, T, b)) {
            ++k;
            k32 += T.n[b] == 32;
        }
    if (n32) *n32 = k32;
    if (plan) *plan = bp;
    return k;
}

size_t amr_bytes(const Cfg &c, const AmrTree &T) {
    AmrScratch A;
    int n32 = 0;
    const int k = batched_boxes(c, T, &n32);
    return total_bytes(c) + carve_amr(A, nullptr, T.max_relaxed_n, k, n32) + 256;
}

ndgp_status solve_amr_impl(const ndgp_grid *grid, const ndgp_params *params,
                           const ndgp_box *boxes, int32_t nb, const double *const *delta,
                           double *const *phi, void *ws, size_t ws_bytes, hipStream_t st,
                           ndgp_report *rep, ndgp_box_report *brep) {
    const auto t0 = std::chrono::steady_clock::now();
    Cfg c;
    AmrTree T;
    std::string why;
    if (!resolve_tree(grid, params, boxes, nb, c, T, why)) return fail(NDGP_EINVAL, why);
    if (!delta || !phi || !delta[0] || !phi[0])
        return fail(NDGP_EINVAL, "delta[0] and phi[0] must not be NULL");
    for (int b = 0; b < nb; ++b) {
        if (!phi[1 + b]) return fail(NDGP_EINVAL, "phi of every box must not be NULL");
        if (T.relaxed[b] && !delta[1 + b])
            return fail(NDGP_EINVAL, "delta of every relaxed box must not be NULL");
    }
    const size_t need = amr_bytes(c, T);
    if (!ws || ws_bytes < need)
        return fail(NDGP_ENOMEM, "workspace smaller than ndgp_amr_workspace_bytes() = " +
                                     std::to_string(need));
    // the domain level: ndgp_solve's path with no patches, in the front of the workspace
    const size_t dom = total_bytes(c);
    ndgp_grid g0 = *grid;
    ndgp_params p0 = *params;
    p0.mode = NDGP_MODE_FULL;
    p0.trunc_level = 0;
    const double *d0[1 + NDGP_MAX_PATCHES] = {delta[0]};
    double *f0[1 + NDGP_MAX_PATCHES] = {phi[0]};
    ndgp_report R;
    std::memset(&R, 0, sizeof(R));
    ndgp_status status = solve_impl(&g0, &p0, d0, f0, ws, dom, st, &R);
    if (status != NDGP_OK && status != NDGP_ENOCONV) return status;

    AmrScratch A;
    int n32 = 0;
    BatchPlan bplan;
    const int nbatch = batched_boxes(c, T, &n32, &bplan);
    char *abase = aligned_base(static_cast<char *>(ws) + dom);
    std::vector<size_t> guards;
    carve_amr(A, abase, T.max_relaxed_n, nbatch, n32, &guards);
    for (size_t off : guards) launch_guard_fill(abase + off, (int)kGuardWords, kGuardWord, st);
    Plan P;
    P.c = c;
    P.partials = A.partials;
    P.scal = A.scal;
    P.fallbacks = A.fallbacks;
    SlotGuard slot;
    Runner run{P, st, slot.p};
    const size_t cells0 = (size_t)c.n * c.n * c.n;
    HIP_TRY(hipMemsetAsync(P.fallbacks, 0, 3 * sizeof(unsigned), st));
    run.enqueue_sum(delta[0], cells0, false, 0); // the domain's mean for the box sources
    // Level by level of the tree (a box after its parent): relaxed boxes of at
    // most kBoxBatchMaxN cells per side all in one launch, one workgroup each
    // (the same bits as relax_patch); the others one after the other.
    const BoxRun brun{P.scal + 0, 1.0 / (double)cells0, c.nu1, c.nu2, kCoarsestSweeps, c.maxc,
                      c.tol, (c.flags & NDGP_DAMPED) ? 1 : 0, P.fallbacks};
    std::vector<BoxJob> jobs;
    std::vector<int> job_box;
    jobs.reserve((size_t)nbatch); // no reallocation: copies read from these elements
    int max_depth = 0, k32 = 0;
    for (int b = 0; b < nb; ++b) max_depth = std::max(max_depth, T.depth[b]);
    // within a level the larger boxes first: their workgroups take longest, the
    // small ones fill the compute units behind them
    std::vector<int> order(nb);
    for (int b = 0; b < nb; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return T.n[x] > T.n[y]; });
    for (int d = 1; d <= max_depth; ++d) {
        const size_t first = jobs.size();
        for (int b : order) {
            if (T.depth[b] != d) continue;
            const int pb = T.parent[b];
            const bool parent_periodic = pb < 0;
            const double *parent = pb < 0 ? phi[0] : phi[1 + pb];
            const int npar = pb < 0 ? c.n : T.n[pb];
            const double hb = c.h / (double)(1 << T.depth[b]);
            if (bplan.batched(c, T, b)) {
                BoxJob J{};
                J.parent = parent;
                J.np = npar;
                J.parent_periodic = parent_periodic ? 1 : 0;
                for (int a = 0; a < 3; ++a) J.origin[a] = T.origin[b][a];
                J.n = T.n[b];
                J.nl = T.nlev[b];
                J.phi = phi[1 + b];
                J.delta = delta[1 + b];
                J.f = c.fsrc * hb * hb;
                for (int l = 0; l < 3; ++l) {
                    const double hm = hb * (double)(1 << l);
                    J.alpha[l] = c.alpha / (hm * hm);
                }
                if (J.n == 32) {
                    J.alt = A.box32 + (size_t)(k32++) * kBox32Doubles;
                    J.s0 = J.alt + 34 * 34 * 34;
                    J.phi1 = J.s0 + 32 * 32 * 32;
                    J.alt1 = J.phi1 + 18 * 18 * 18;
                    J.hat1 = J.alt1 + 18 * 18 * 18;
                    J.s1 = J.hat1 + 18 * 18 * 18;
                }
                jobs.push_back(J);
                job_box.push_back(b);
                continue;
            }
            ChildBox b0{{T.origin[b][0], T.origin[b][1], T.origin[b][2]}, 0, T.n[b]};
            launch_interpolate(parent, npar, parent_periodic, b0, phi[1 + b], false, st);
            ndgp_box_report br{T.depth[b], 0, 0, -1.0};
            if (T.relaxed[b]) {
                Level H[kMaxLevels];
                for (int l = 0; l < T.nlev[b]; ++l) {
                    Level &L = H[l];
                    L.n = T.n[b] >> l;
                    L.lg = ilog2(L.n);
                    L.periodic = false;
                    const double hm = hb * (double)(1 << l);
                    L.alpha = c.alpha / (hm * hm);
                    L.phi = l ? A.phi[l] : phi[1 + b];
                    L.alt = A.alt[l];
                    L.s = A.s[l];
                    L.hat = l ? A.hat[l] : nullptr;
                    L.dyn_bc = l > 0;
                }
                Range box_range("ndgp box");
                const PatchOutcome po = relax_patch(run, H, T.nlev[b], parent, npar,
                                                    parent_periodic, T.origin[b], T.n[b], hb,
                                                    delta[1 + b], 1.0 / (double)cells0);
                if (po.status == NDGP_EINVAL) return po.status;
                if (po.status != NDGP_OK && status == NDGP_OK) status = po.status;
                br.cycles = po.cycles;
                br.damped_from = po.damped_from;
                br.rel_res = po.rel;
            }
            if (brep) brep[b] = br;
        }
        const int count = (int)(jobs.size() - first);
        if (count > 0) {
            Range boxes_range("ndgp small boxes, one workgroup each");
            HIP_TRY(hipMemcpyAsync(A.jobs + first, jobs.data() + first, count * sizeof(BoxJob),
                                   hipMemcpyHostToDevice, st));
            launch_solve_boxes(A.jobs + first, A.results + first, count, brun, st);
        }
    }
    if (!jobs.empty()) {
        std::vector<BoxResult> res(jobs.size());
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(res.data(), A.results, res.size() * sizeof(BoxResult),
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (size_t q = 0; q < jobs.size(); ++q) {
            const BoxResult &r = res[q];
            const int b = job_box[q];
            if (r.status == kBoxBadSource)
                return fail(NDGP_EINVAL, "a patch density has non-finite values");
            CycleMonitor m{c.tol, c.maxc};
            m.rel = r.rel;
            ndgp_status sq = NDGP_OK;
            if (r.status == kBoxDiverged)
                sq = fail(NDGP_ENOCONV, "multigrid diverged");
            else if (r.status)
                sq = verdict(m);
            if (sq != NDGP_OK && status == NDGP_OK) status = sq;
            if (brep) brep[b] = ndgp_box_report{T.depth[b], r.cycles, r.damped_from, r.rel};
        }
    }
    unsigned fb[3] = {0, 0, 0};
    for (size_t off : guards)
        launch_guard_check(abase + off, (int)kGuardWords, kGuardWord, P.fallbacks + 2, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(slot.p, P.fallbacks, 3 * sizeof(unsigned), hipMemcpyDeviceToHost,
                           st));
    HIP_TRY(hipStreamSynchronize(st));
    std::memcpy(fb, slot.p, 3 * sizeof(unsigned));
    if (fb[2]) return fail(NDGP_EDEVICE, std::to_string(fb[2]) + " workspace guard-band words "
                                         "were overwritten");
    R.fallbacks += (int32_t)fb[0];
    R.holds += (int32_t)fb[1];
    R.t_total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = R;
    if (status != NDGP_OK && status != NDGP_ENOCONV) return status;
    if (status == NDGP_ENOCONV) return fail(NDGP_ENOCONV, "a level did not reach the tolerance");
    return NDGP_OK;
}

ndgp_status residual_impl(const ndgp_grid *grid, const ndgp_params *params, int32_t level,
                          const double *const delta[], const double *phi, double *r_out,
                          double *rel_out, void *ws, size_t ws_bytes, hipStream_t st) {
    Cfg c;
    std::string why;
    if (!resolve(grid, params, c, why)) return fail(NDGP_EINVAL, why);
    if (level < 0 || level > c.np) return fail(NDGP_EINVAL, "level out of range");
    if (!delta || !delta[0] || !delta[level] || !phi)
        return fail(NDGP_EINVAL, "delta[0], delta[level] and phi must not be NULL");
    const size_t need = total_bytes(c);
    if (!ws || ws_bytes < need)
        return fail(NDGP_ENOMEM, "workspace smaller than ndgp_workspace_bytes() = " +
                                     std::to_string(need));
    Plan P;
    P.c = c;
    Carver cv{aligned_base(ws)};
    const int nlv = c.nlev(level);
    Level L;
    L.n = nlv;
    L.lg = ilog2(nlv);
    L.periodic = level == 0;
    const double hl = c.hl(level);
    L.alpha = c.alpha / (hl * hl);
    L.phi = const_cast<double *>(phi);
    L.s = cv.take<double>(L.cells());
    P.partials = cv.take<double>(kReduceBlocks);
    P.scal = cv.take<double>(16);
    SlotGuard slot;
    Runner run{P, st, slot.p};
    const size_t cells0 = (size_t)c.n * c.n * c.n;
    const double dsum = run.sum(delta[0], cells0, false, 0);
    if (!std::isfinite(dsum)) return fail(NDGP_EINVAL, "delta[0] has non-finite values");
    launch_source(delta[level], L.cells(), P.scal + 0, 1.0 / (double)cells0, c.fsrc * hl * hl,
                  L.s, st);
    const double sn2 = run.sum(L.s, L.cells(), true, 1);
    launch_residual_sumsq(L, P.partials, r_out, 1.0 / (hl * hl), st);
    launch_reduce_final(P.partials, P.scal + 2, st);
    const double rr = run.read_scalar(P.scal + 2);
    if (rel_out) *rel_out = sn2 > 0.0 ? std::sqrt(rr / sn2) : std::sqrt(rr);
    return NDGP_OK;
}

// ------------------------------------------------------------------------
// ndgp_residual_noalloc: the residual with the library's own scratch array
// instead of a caller workspace.  `scratch` is a host-side stand-in for the
// device array in host code: host code only ever uses the address that
// hipGetSymbolAddress returns for the current device (each GPU holds its own
// copy of the array, at its own address).

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxScratchDevices] = {};

double *scratch_for_current_device() {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices)
        throw HipFailure{hipErrorInvalidDevice, "device id above the scratch table"};
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    return g_scratch_ptr[dev];
}

ndgp_status residual_noalloc_impl(const ndgp_grid *grid, const ndgp_params *params, int32_t level,
                                  const double *const delta[], const double *phi, double *r_out,
                                  double *norms_out, hipStream_t st) {
    Cfg c;
    std::string why;
    if (!resolve(grid, params, c, why)) return fail(NDGP_EINVAL, why);
    if (level < 0 || level > c.np) return fail(NDGP_EINVAL, "level out of range");
    if (!delta || !delta[0] || !delta[level] || !phi || !norms_out)
        return fail(NDGP_EINVAL, "delta[0], delta[level], phi and norms_out must not be NULL");
    const int nlv = c.nlev(level);
    Level L;
    L.n = nlv;
    L.lg = ilog2(nlv);
    L.periodic = level == 0;
    if (L.cells() > (size_t)NDGP_NOALLOC_MAX_CELLS)
        return fail(NDGP_EINVAL, "level " + std::to_string(level) + " has " +
                                     std::to_string(L.cells()) +
                                     " cells, more than NDGP_NOALLOC_MAX_CELLS = " +
                                     std::to_string(NDGP_NOALLOC_MAX_CELLS) +
                                     " (use ndgp_residual with a workspace)");
    double *base = scratch_for_current_device();
    const double hl = c.hl(level);
    L.alpha = c.alpha / (hl * hl);
    L.phi = const_cast<double *>(phi);
    L.s = base;                                      // the level's source, cell units
    double *partials = base + NDGP_NOALLOC_MAX_CELLS; // one per reduction block
    double *sums = partials + kReduceBlocks;          // [0] sum delta, [1] sum s^2, [2] sum r^2
    const size_t cells0 = (size_t)c.n * c.n * c.n;
    // every scratch value is written before it is read: nothing to clear
    launch_partial_sums(delta[0], cells0, false, partials, st);
    launch_reduce_final(partials, sums + 0, st);
    launch_source(delta[level], L.cells(), sums + 0, 1.0 / (double)cells0, c.fsrc * hl * hl, L.s,
                  st);
    launch_partial_sums(L.s, L.cells(), true, partials, st);
    launch_reduce_final(partials, sums + 1, st);
    launch_residual_sumsq(L, partials, r_out, 1.0 / (hl * hl), st);
    launch_reduce_final(partials, sums + 2, st);
    launch_residual_norms(sums, norms_out, st);
    HIP_TRY(hipGetLastError());
    return NDGP_OK;
}

ndgp_status force_impl(const ndgp_grid *grid, const double *const phi[], double *const force[],
                       hipStream_t st) {
    if (!grid) return fail(NDGP_EINVAL, "grid must not be NULL");
    ndgp_params p;
    std::memset(&p, 0, sizeof(p));
    p.beta = 1.0;
    p.a = 1.0;
    p.omega_m = 1.0;
    p.mode = NDGP_MODE_INTERPOLATED; // geometry checks only need the finest patch levels
    Cfg c;
    std::string why;
    if (!resolve(grid, &p, c, why)) return fail(NDGP_EINVAL, why);
    if (!phi || !force) return fail(NDGP_EINVAL, "phi and force must not be NULL");
    for (int l = 0; l <= c.np; ++l)
        if (!phi[l] || !force[l]) return fail(NDGP_EINVAL, "phi/force of every level must not be NULL");
    for (int l = 0; l <= c.np; ++l) launch_force(phi[l], c.nlev(l), l == 0, c.hl(l), force[l], st);
    HIP_TRY(hipGetLastError());
    return NDGP_OK;
}

// geometry-only view of a grid (the patch checks of the interpolated mode)
bool resolve_grid(const ndgp_grid *grid, Cfg &c, std::string &why) {
    if (!grid) {
        why = "grid must not be NULL";
        return false;
    }
    ndgp_params p;
    std::memset(&p, 0, sizeof(p));
    p.beta = 1.0;
    p.a = 1.0;
    p.omega_m = 1.0;
    p.mode = NDGP_MODE_INTERPOLATED;
    return resolve(grid, &p, c, why);
}

ndgp_status total_force_impl(const ndgp_grid *grid, const double *const phi[],
                             const double *const psi[], double *const force[], hipStream_t st) {
    Cfg c;
    std::string why;
    if (!resolve_grid(grid, c, why)) return fail(NDGP_EINVAL, why);
    if (!phi || !psi || !force) return fail(NDGP_EINVAL, "phi, psi and force must not be NULL");
    for (int l = 0; l <= c.np; ++l)
        if (!phi[l] || !psi[l] || !force[l])
            return fail(NDGP_EINVAL, "phi/psi/force of every level must not be NULL");
    for (int l = 0; l <= c.np; ++l)
        launch_total_force(phi[l], psi[l], c.nlev(l), l == 0, c.hl(l), force[l], st);
    HIP_TRY(hipGetLastError());
    return NDGP_OK;
}

ndgp_status geff_stats_impl(const ndgp_grid *grid, const double *const phi[],
                            const double *const psi[], const double *edges, int32_t n_edges,
                            ndgp_geff_level *out, int64_t *hist, void *ws, size_t ws_bytes,
                            hipStream_t st) {
    Cfg c;
    std::string why;
    if (!resolve_grid(grid, c, why)) return fail(NDGP_EINVAL, why);
    if (!phi || !psi || !edges || !out || !hist)
        return fail(NDGP_EINVAL, "phi, psi, edges, out and hist must not be NULL");
    for (int l = 0; l <= c.np; ++l)
        if (!phi[l] || !psi[l]) return fail(NDGP_EINVAL, "phi/psi of every level must not be NULL");
    if (n_edges < 1 || n_edges > NDGP_GEFF_MAX_EDGES)
        return fail(NDGP_EINVAL, "n_edges must be in [1, NDGP_GEFF_MAX_EDGES]");
    for (int b = 0; b < n_edges; ++b)
        if (std::isnan(edges[b]) || (b && !(edges[b - 1] < edges[b])))
            return fail(NDGP_EINVAL, "edges must be strictly ascending numbers");
    static_assert(kGeffMaxEdges == NDGP_GEFF_MAX_EDGES, "edge limit");
    Carver cv{aligned_base(ws)};
    double *partials = cv.take<double>(5 * (size_t)kReduceBlocks);
    double *d_edges = cv.take<double>(NDGP_GEFF_MAX_EDGES);
    unsigned long long *d_hist = cv.take<unsigned long long>(NDGP_GEFF_MAX_EDGES + 1);
    double *d_out = cv.take<double>(8);
    if (!ws || cv.off + 256 > ws_bytes)
        return fail(NDGP_ENOMEM, "workspace smaller than NDGP_GEFF_WORKSPACE");
    SlotGuard slot; // pinned doubles for the five results of a level
    std::vector<unsigned long long> h((size_t)n_edges + 1);
    HIP_TRY(hipMemcpyAsync(d_edges, edges, sizeof(double) * n_edges, hipMemcpyHostToDevice, st));
    for (int l = 0; l <= c.np; ++l) {
        const int zero[3] = {0, 0, 0};
        const bool child = l < c.np;
        launch_geff_level(phi[l], psi[l], c.nlev(l), l == 0, child ? c.po[l] : zero,
                          child ? c.pn[l] / 2 : 0, d_edges, n_edges, partials, d_hist, d_out, st);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(slot.p, d_out, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(h.data(), d_hist, sizeof(unsigned long long) * (n_edges + 1),
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        out[l].cells = (int64_t)slot.p[0];
        out[l].sum = slot.p[1];
        out[l].sum_sq = slot.p[2];
        out[l].min = slot.p[3];
        out[l].max = slot.p[4];
        for (int b = 0; b <= n_edges; ++b) hist[(size_t)l * (n_edges + 1) + b] = (int64_t)h[b];
    }
    return NDGP_OK;
}

// lower corner of every level in domain cells (level q + 1 at corner(q) +
// origin(q) 2^-q)
void level_corners(const Cfg &c, double corner[][3]) {
    corner[0][0] = corner[0][1] = corner[0][2] = 0.0;
    for (int q = 0; q < c.np; ++q)
        for (int a = 0; a < 3; ++a)
            corner[q + 1][a] = corner[q][a] + std::ldexp((double)c.po[q][a], -q);
}

size_t cic_bytes(const Cfg &c) {
    Carver cv{nullptr};
    for (int l = 0; l <= c.np; ++l) {
        const size_t m = (size_t)c.nlev(l);
        cv.take<unsigned long long>(m * m * m);
    }
    return cv.off + 256;
}

ndgp_status cic_density_impl(const ndgp_grid *grid, const double *pos, int64_t np,
                             double *const delta[], void *ws, size_t ws_bytes, hipStream_t st) {
    Cfg c;
    std::string why;
    if (!resolve_grid(grid, c, why)) return fail(NDGP_EINVAL, why);
    if (!pos || !delta) return fail(NDGP_EINVAL, "pos and delta must not be NULL");
    if (np < 1 || np > NDGP_CIC_MAX_PARTICLES)
        return fail(NDGP_EINVAL, "n_particles must be in [1, NDGP_CIC_MAX_PARTICLES]");
    for (int l = 0; l <= c.np; ++l)
        if (!delta[l]) return fail(NDGP_EINVAL, "delta of every level must not be NULL");
    if (!ws || ws_bytes < cic_bytes(c))
        return fail(NDGP_ENOMEM, "workspace smaller than ndgp_cic_workspace_bytes() = " +
                                     std::to_string(cic_bytes(c)));
    double corner[1 + NDGP_MAX_PATCHES][3];
    level_corners(c, corner);
    Carver cv{aligned_base(ws)};
    for (int l = 0; l <= c.np; ++l) {
        const int m = c.nlev(l);
        unsigned long long *acc = cv.take<unsigned long long>((size_t)m * m * m);
        launch_cic_deposit(pos, (long long)np, c.n, corner[l], l, m, acc, delta[l], st);
    }
    HIP_TRY(hipGetLastError());
    return NDGP_OK;
}

ndgp_status refine_flags_impl(const ndgp_grid *grid, const double *const delta[], int64_t np,
                              double n_ref, unsigned char *const flags[], int64_t *n_flagged,
                              void *ws, size_t ws_bytes, hipStream_t st) {
    Cfg c;
    std::string why;
    if (!resolve_grid(grid, c, why)) return fail(NDGP_EINVAL, why);
    if (!delta || !flags || !n_flagged)
        return fail(NDGP_EINVAL, "delta, flags and n_flagged must not be NULL");
    if (np < 1 || !std::isfinite(n_ref))
        return fail(NDGP_EINVAL, "need n_particles >= 1 and a finite n_ref");
    Carver cv{aligned_base(ws)};
    double *partials = cv.take<double>(kReduceBlocks);
    double *total = cv.take<double>(1 + NDGP_MAX_PATCHES);
    if (!ws || cv.off + 256 > ws_bytes)
        return fail(NDGP_ENOMEM, "workspace smaller than NDGP_DIFF_NORMS_WORKSPACE");
    for (int l = 0; l <= c.np; ++l) {
        if (!delta[l] || !flags[l]) return fail(NDGP_EINVAL, "delta/flags of every level must not be NULL");
        const size_t m = (size_t)c.nlev(l);
        const double mean = (double)np / std::ldexp((double)c.n * c.n * c.n, 3 * l);
        launch_refine_flags(delta[l], m * m * m, mean, n_ref, flags[l], partials, st);
        launch_reduce_final(partials, total + l, st);
    }
    SlotGuard slot;
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(slot.p, total, (c.np + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int l = 0; l <= c.np; ++l) n_flagged[l] = (int64_t)slot.p[l];
    return NDGP_OK;
}

ndgp_status cic_force_impl(const ndgp_grid *grid, const double *const force[], const double *pos,
                           int64_t np, double *out, hipStream_t st) {
    Cfg c;
    std::string why;
    if (!resolve_grid(grid, c, why)) return fail(NDGP_EINVAL, why);
    if (!pos || !force || !out) return fail(NDGP_EINVAL, "pos, force and out must not be NULL");
    if (np < 1 || np > NDGP_CIC_MAX_PARTICLES)
        return fail(NDGP_EINVAL, "n_particles must be in [1, NDGP_CIC_MAX_PARTICLES]");
    static_assert(kCicMaxLevels == 1 + NDGP_MAX_PATCHES, "one gather slot per level");
    CicLevels lv{};
    lv.levels = c.np + 1;
    lv.n = c.n;
    double corner[1 + NDGP_MAX_PATCHES][3];
    level_corners(c, corner);
    for (int l = 0; l <= c.np; ++l) {
        if (!force[l]) return fail(NDGP_EINVAL, "force of every level must not be NULL");
        lv.m[l] = c.nlev(l);
        lv.cells_per_domain[l] = std::ldexp(1.0, l);
        for (int a = 0; a < 3; ++a) lv.corner[l][a] = corner[l][a];
        lv.force[l] = force[l];
    }
    launch_cic_gather(pos, (long long)np, lv, out, st);
    HIP_TRY(hipGetLastError());
    return NDGP_OK;
}

} // namespace

// ------------------------------------------------------------------------
// serving plans: the steps of solve_impl, each enqueued without blocking

struct ndgp_plan {
    Plan P;
    hipStream_t st = nullptr;
    double *slot = nullptr; // pinned: [0] sum delta, [1] sum s^2, [2] sum r^2,
                            //         [3] sum phi, [4..5] the two relaxation
                            //         event counters and the guard-band count
                            //         (bits)
    hipEvent_t ev = nullptr;
    const double *delta[1 + NDGP_MAX_PATCHES] = {};
    double *phi[1 + NDGP_MAX_PATCHES] = {};
    enum State { RUNNING, READY, FINISHING, DONE } state = RUNNING;
    bool started = false, restarting = false;
    double snorm2 = 0.0;
    CycleMonitor mon;
    ndgp_status status = NDGP_OK;
    std::string message;
    ndgp_report R;
    std::chrono::steady_clock::time_point t0;
};

namespace {

Runner plan_runner(ndgp_plan *pl) { return Runner{pl->P, pl->st, pl->slot}; }

void plan_record(ndgp_plan *pl) { HIP_TRY(hipEventRecord(pl->ev, pl->st)); }

// gauge, patch interpolation, and the numbers the report needs
void plan_enqueue_tail(ndgp_plan *pl, bool zero_field) {
    const Cfg &c = pl->P.c;
    Runner run = plan_runner(pl);
    const size_t cells0 = (size_t)c.n * c.n * c.n;
    if (zero_field) launch_fill(pl->phi[0], cells0, 0.0, pl->st);
    run.enqueue_sum(pl->phi[0], cells0, false, 3);
    launch_shift_by_mean(pl->phi[0], cells0, pl->P.scal + 3, pl->st);
    for (int q = 0; q < c.np; ++q) {
        ChildBox b0{{c.po[q][0], c.po[q][1], c.po[q][2]}, 0, c.pn[q]};
        launch_interpolate(pl->phi[q], q == 0 ? c.n : c.pn[q - 1], q == 0, b0, pl->phi[q + 1],
                           false, pl->st);
    }
    HIP_TRY(hipMemcpyAsync(pl->slot + 3, pl->P.scal + 3, sizeof(double), hipMemcpyDeviceToHost,
                           pl->st));
    check_guards(pl->P, pl->st);
    HIP_TRY(hipMemcpyAsync(pl->slot + 4, pl->P.fallbacks, 3 * sizeof(unsigned),
                           hipMemcpyDeviceToHost, pl->st));
    plan_record(pl);
    pl->state = ndgp_plan::FINISHING;
}

ndgp_status plan_create_impl(const ndgp_grid *grid, const ndgp_params *params,
                             const double *const delta[], double *const phi[], void *ws,
                             size_t ws_bytes, hipStream_t st, ndgp_plan **out) {
    if (!out) return fail(NDGP_EINVAL, "plan must not be NULL");
    *out = nullptr;
    Cfg c;
    std::string why;
    if (!resolve(grid, params, c, why)) return fail(NDGP_EINVAL, why);
    if (c.nrelax > 0)
        return fail(NDGP_EINVAL, "plans relax the domain level only: patches must all be "
                                 "interpolated");
    ndgp_status s = check_arrays(c, delta, phi);
    if (s != NDGP_OK) return s;
    const size_t need = total_bytes(c);
    if (!ws || ws_bytes < need)
        return fail(NDGP_ENOMEM, "workspace smaller than ndgp_workspace_bytes() = " +
                                     std::to_string(need));
    ndgp_plan *pl = new ndgp_plan();
    pl->t0 = std::chrono::steady_clock::now();
    pl->P.c = c;
    carve(pl->P, aligned_base(ws));
    pl->P.base[0].phi = phi[0];
    pl->st = st;
    for (int l = 0; l <= c.np; ++l) {
        pl->delta[l] = delta[l];
        pl->phi[l] = phi[l];
    }
    std::memset(&pl->R, 0, sizeof(pl->R));
    for (int l = 0; l <= NDGP_MAX_PATCHES; ++l) pl->R.rel_res[l] = -1.0;
    try {
        pl->slot = pinned_slots().acquire();
        HIP_TRY(hipEventCreateWithFlags(&pl->ev, hipEventDisableTiming));
        Runner run = plan_runner(pl);
        const size_t cells0 = (size_t)c.n * c.n * c.n;
        arm_guards(pl->P, st);
        HIP_TRY(hipMemsetAsync(pl->P.fallbacks, 0, 3 * sizeof(unsigned), st));
        run.enqueue_sum(delta[0], cells0, false, 0);
        launch_source(delta[0], cells0, pl->P.scal + 0, 1.0 / (double)cells0, c.fsrc * c.h * c.h,
                      pl->P.base[0].s, st);
        run.enqueue_sum(pl->P.base[0].s, cells0, true, 1);
        if (c.flags & NDGP_DAMPED) {
            set_step(pl->P.base, c.prec == NDGP_PREC_MIXED ? pl->P.base32 : nullptr, c.nl,
                     kDampedStep);
            pl->R.damped_from[0] = 1;
        }
        if (!(c.flags & NDGP_WARM_START)) run.nested_start(pl->P.base, c.nl);
        run.enqueue_residual(pl->P.base, pl->P.base32);
        HIP_TRY(hipMemcpyAsync(pl->slot, pl->P.scal, 3 * sizeof(double), hipMemcpyDeviceToHost,
                               st));
        plan_record(pl);
    } catch (...) {
        // a copy into the slot may be in flight: the slot returns to the pool
        // only once the stream is idle (else it is leaked, never reused)
        if (pl->ev) (void)hipEventDestroy(pl->ev);
        if (pl->slot && hipStreamSynchronize(st) == hipSuccess) pinned_slots().release(pl->slot);
        delete pl;
        throw;
    }
    *out = pl;
    return NDGP_OK;
}

ndgp_status plan_finish(ndgp_plan *pl, int32_t *done, ndgp_report *rep) {
    if (done) *done = 1;
    if (rep) *rep = pl->R;
    if (pl->status != NDGP_OK) g_err = pl->message;
    return pl->status;
}

void plan_fail(ndgp_plan *pl, ndgp_status st, const char *msg) {
    if (pl->status == NDGP_OK) {
        pl->status = st;
        pl->message = msg;
    }
}

ndgp_status plan_poll_impl(ndgp_plan *pl, int32_t *done, ndgp_report *rep) {
    if (!pl) return fail(NDGP_EINVAL, "plan must not be NULL");
    if (done) *done = 0;
    if (pl->state == ndgp_plan::DONE) return plan_finish(pl, done, rep);
    if (pl->state == ndgp_plan::READY) return NDGP_OK;
    const hipError_t q = hipEventQuery(pl->ev);
    if (q == hipErrorNotReady) return NDGP_OK;
    HIP_TRY(q);
    const Cfg &c = pl->P.c;
    const size_t cells0 = (size_t)c.n * c.n * c.n;
    if (pl->state == ndgp_plan::FINISHING) {
        unsigned fb[3] = {0, 0, 0};
        std::memcpy(fb, pl->slot + 4, 3 * sizeof(unsigned));
        pl->R.fallbacks = (int32_t)fb[0];
        pl->R.holds = (int32_t)fb[1];
        if (fb[2])
            plan_fail(pl, NDGP_EDEVICE, "workspace guard-band words were overwritten");
        pl->R.phi_mean = pl->slot[3] / (double)cells0;
        pl->R.t_total_ms = std::chrono::duration<double, std::milli>(
                               std::chrono::steady_clock::now() - pl->t0)
                               .count();
        pl->state = ndgp_plan::DONE;
        return plan_finish(pl, done, rep);
    }
    // RUNNING and its work has completed: a residual norm is in slot[2]
    if (!pl->started) {
        pl->started = true;
        const double dsum = pl->slot[0];
        if (!std::isfinite(dsum)) {
            plan_fail(pl, NDGP_EINVAL, "delta[0] has non-finite values");
            pl->state = ndgp_plan::DONE;
            return plan_finish(pl, done, rep);
        }
        pl->R.removed_mean = dsum / (double)cells0;
        pl->snorm2 = pl->slot[1];
        if (pl->snorm2 == 0.0) { // no source: phi = 0
            pl->R.rel_res[0] = 0.0;
            plan_enqueue_tail(pl, true);
            return NDGP_OK;
        }
        pl->mon = CycleMonitor{c.tol, c.maxc};
        pl->mon.damped = (c.flags & NDGP_DAMPED) != 0;
        pl->mon.start(std::sqrt(pl->slot[2] / pl->snorm2));
    } else if (pl->restarting) { // the damped nested start has completed
        pl->restarting = false;
        pl->mon = CycleMonitor{c.tol, c.maxc};
        pl->mon.damped = true;
        pl->mon.start(std::sqrt(pl->slot[2] / pl->snorm2));
    } else {
        const double r = std::sqrt(pl->slot[2] / pl->snorm2);
        const int cyc = pl->R.cycles[0];
        if (cyc - 1 < NDGP_HIST_LEN) {
            pl->R.res_hist[cyc - 1] = r;
            pl->R.hist_len = cyc;
        }
        if (pl->mon.record(r)) { // the safeguard: from the nested start again, damped
            set_step(pl->P.base, c.prec == NDGP_PREC_MIXED ? pl->P.base32 : nullptr, c.nl,
                     kDampedStep);
            pl->R.damped_from[0] = cyc + 1;
            pl->restarting = true;
            Runner run = plan_runner(pl);
            run.nested_start(pl->P.base, c.nl);
            run.enqueue_residual(pl->P.base, pl->P.base32);
            HIP_TRY(hipMemcpyAsync(pl->slot + 2, pl->P.scal + 2, sizeof(double),
                                   hipMemcpyDeviceToHost, pl->st));
            plan_record(pl);
            return NDGP_OK; // still RUNNING
        }
        if (pl->mon.diverged()) {
            pl->R.rel_res[0] = pl->mon.rel;
            plan_fail(pl, NDGP_ENOCONV, "multigrid diverged");
            plan_enqueue_tail(pl, false);
            return NDGP_OK;
        }
    }
    pl->R.rel_res[0] = pl->mon.rel;
    if (pl->mon.converged() || pl->mon.stalled() || pl->R.cycles[0] >= c.maxc) {
        const ndgp_status v = verdict(pl->mon);
        if (v != NDGP_OK) plan_fail(pl, v, g_err.c_str());
        plan_enqueue_tail(pl, false);
        return NDGP_OK;
    }
    pl->state = ndgp_plan::READY;
    return NDGP_OK;
}

ndgp_status plan_step_impl(ndgp_plan *pl) {
    if (!pl) return fail(NDGP_EINVAL, "plan must not be NULL");
    if (pl->state != ndgp_plan::READY) return NDGP_OK;
    Runner run = plan_runner(pl);
    if (pl->P.c.prec == NDGP_PREC_MIXED)
        run.mixed_outer(pl->P.base, pl->P.base32, pl->P.c.nl);
    else
        run.vcycle(pl->P.base, pl->P.c.nl, 0);
    run.enqueue_residual(pl->P.base, pl->P.base32);
    HIP_TRY(hipMemcpyAsync(pl->slot + 2, pl->P.scal + 2, sizeof(double), hipMemcpyDeviceToHost,
                           pl->st));
    plan_record(pl);
    pl->R.cycles[0] += 1;
    pl->state = ndgp_plan::RUNNING;
    return NDGP_OK;
}

ndgp_status diff_norms_impl(const double *a, const double *b, size_t count, double out[3],
                            void *ws, size_t ws_bytes, hipStream_t st) {
    if (!a || !out) return fail(NDGP_EINVAL, "a and out must not be NULL");
    if (!ws || ws_bytes < NDGP_DIFF_NORMS_WORKSPACE)
        return fail(NDGP_ENOMEM, "workspace smaller than NDGP_DIFF_NORMS_WORKSPACE");
    Carver cv{aligned_base(ws)};
    double *partials = cv.take<double>(3 * kReduceBlocks);
    double *sums = cv.take<double>(3);
    SlotGuard slot;
    launch_diff_partials(a, b, count, partials, st);
    for (int q = 0; q < 3; ++q) launch_reduce_final(partials + q * kReduceBlocks, sums + q, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(slot.p, sums, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int q = 0; q < 3; ++q) out[q] = slot.p[q];
    return NDGP_OK;
}

template <class F>
ndgp_status guarded(F &&f) {
    try {
        return f();
    } catch (const HipFailure &e) {
        return fail(NDGP_EDEVICE, std::string(e.what) + ": " + hipGetErrorString(e.err));
    } catch (const std::exception &e) {
        return fail(NDGP_EDEVICE, e.what());
    } catch (...) {
        return fail(NDGP_EDEVICE, "unknown failure");
    }
}

} // namespace

// ------------------------------------------------------------------------
// C ABI

void ndgp::set_last_error(const char *msg) { g_err = msg; }

extern "C" {

int32_t ndgp_version(void) { return NDGP_ABI_VERSION; }

const char *ndgp_last_error(void) { return g_err.c_str(); }

double ndgp_beta_lcdm(double a, double omega_m, double rc) {
    // E^2 = Om a^-3 + 1 - Om; Hdot / (3 H^2) = -Om(a) / 2 with Om(a) = Om a^-3 / E^2
    const double E2 = omega_m / (a * a * a) + 1.0 - omega_m;
    const double om_a = omega_m / (a * a * a) / E2;
    return 1.0 + 2.0 * std::sqrt(E2) * rc * (1.0 - 0.5 * om_a);
}

size_t ndgp_workspace_bytes(const ndgp_grid *grid, const ndgp_params *params) {
    Cfg c;
    std::string why;
    if (!resolve(grid, params, c, why)) {
        g_err = why;
        return 0;
    }
    return total_bytes(c);
}

ndgp_status ndgp_solve(const ndgp_grid *grid, const ndgp_params *params,
                       const double *const delta[1 + NDGP_MAX_PATCHES],
                       double *const phi[1 + NDGP_MAX_PATCHES], void *workspace,
                       size_t workspace_bytes, hipStream_t stream, ndgp_report *report) {
    return guarded([&] {
        Range r("ndgp_solve");
        return solve_impl(grid, params, delta, phi, workspace, workspace_bytes, stream, report);
    });
}

size_t ndgp_cic_workspace_bytes(const ndgp_grid *grid) {
    Cfg c;
    std::string why;
    if (!resolve_grid(grid, c, why)) {
        g_err = why;
        return 0;
    }
    return cic_bytes(c);
}

ndgp_status ndgp_cic_density(const ndgp_grid *grid, const double *pos, int64_t n_particles,
                             double *const delta[1 + NDGP_MAX_PATCHES], void *workspace,
                             size_t workspace_bytes, hipStream_t stream) {
    return guarded([&] {
        return cic_density_impl(grid, pos, n_particles, delta, workspace, workspace_bytes, stream);
    });
}

ndgp_status ndgp_cic_force(const ndgp_grid *grid, const double *const force[1 + NDGP_MAX_PATCHES],
                           const double *pos, int64_t n_particles, double *out,
                           hipStream_t stream) {
    return guarded([&] { return cic_force_impl(grid, force, pos, n_particles, out, stream); });
}

ndgp_status ndgp_refine_flags(const ndgp_grid *grid, const double *const delta[1 + NDGP_MAX_PATCHES],
                              int64_t n_particles, double n_ref,
                              unsigned char *const flags[1 + NDGP_MAX_PATCHES],
                              int64_t n_flagged[1 + NDGP_MAX_PATCHES], void *workspace,
                              size_t workspace_bytes, hipStream_t stream) {
    return guarded([&] {
        return refine_flags_impl(grid, delta, n_particles, n_ref, flags, n_flagged, workspace,
                                 workspace_bytes, stream);
    });
}

ndgp_status ndgp_total_force(const ndgp_grid *grid, const double *const phi[1 + NDGP_MAX_PATCHES],
                             const double *const psi[1 + NDGP_MAX_PATCHES],
                             double *const force[1 + NDGP_MAX_PATCHES], hipStream_t stream) {
    return guarded([&] { return total_force_impl(grid, phi, psi, force, stream); });
}

ndgp_status ndgp_geff_stats(const ndgp_grid *grid, const double *const phi[1 + NDGP_MAX_PATCHES],
                            const double *const psi[1 + NDGP_MAX_PATCHES], const double *edges,
                            int32_t n_edges, ndgp_geff_level out[1 + NDGP_MAX_PATCHES],
                            int64_t *hist, void *workspace, size_t workspace_bytes,
                            hipStream_t stream) {
    return guarded([&] {
        return geff_stats_impl(grid, phi, psi, edges, n_edges, out, hist, workspace,
                               workspace_bytes, stream);
    });
}

ndgp_status ndgp_solve_cellwise(const ndgp_grid *grid, const ndgp_params *params,
                                const double *const delta[1 + NDGP_MAX_PATCHES],
                                const double *const psi[1 + NDGP_MAX_PATCHES], double threshold,
                                double *const phi[1 + NDGP_MAX_PATCHES], void *workspace,
                                size_t workspace_bytes, hipStream_t stream,
                                ndgp_report *report) {
    return guarded([&] {
        if (!psi) return fail(NDGP_EINVAL, "psi must not be NULL");
        Range r("ndgp_solve_cellwise");
        return solve_impl(grid, params, delta, phi, workspace, workspace_bytes, stream, report,
                          psi, threshold);
    });
}

ndgp_status ndgp_residual(const ndgp_grid *grid, const ndgp_params *params, int32_t level,
                          const double *const delta[1 + NDGP_MAX_PATCHES], const double *phi,
                          double *r_out, double *rel_norm_out, void *workspace,
                          size_t workspace_bytes, hipStream_t stream) {
    return guarded([&] {
        return residual_impl(grid, params, level, delta, phi, r_out, rel_norm_out, workspace,
                             workspace_bytes, stream);
    });
}

size_t ndgp_amr_workspace_bytes(const ndgp_grid *grid, const ndgp_params *params,
                                const ndgp_box *boxes, int32_t n_boxes) {
    Cfg c;
    AmrTree T;
    std::string why;
    if (!resolve_tree(grid, params, boxes, n_boxes, c, T, why)) {
        g_err = why;
        return 0;
    }
    return amr_bytes(c, T);
}

ndgp_status ndgp_solve_amr(const ndgp_grid *grid, const ndgp_params *params,
                           const ndgp_box *boxes, int32_t n_boxes, const double *const *delta,
                           double *const *phi, void *workspace, size_t workspace_bytes,
                           hipStream_t stream, ndgp_report *report,
                           ndgp_box_report *box_report) {
    return guarded([&] {
        Range r("ndgp_solve_amr");
        return solve_amr_impl(grid, params, boxes, n_boxes, delta, phi, workspace,
                              workspace_bytes, stream, report, box_report);
    });
}

ndgp_status ndgp_residual_noalloc(const ndgp_grid *grid, const ndgp_params *params,
                                  int32_t level, const double *const delta[1 + NDGP_MAX_PATCHES],
                                  const double *phi, double *r_out, double *norms_out,
                                  hipStream_t stream) {
    return guarded([&] {
        return residual_noalloc_impl(grid, params, level, delta, phi, r_out, norms_out, stream);
    });
}

ndgp_status ndgp_force(const ndgp_grid *grid, const double *const phi[1 + NDGP_MAX_PATCHES],
                       double *const force[1 + NDGP_MAX_PATCHES], hipStream_t stream) {
    return guarded([&] { return force_impl(grid, phi, force, stream); });
}

ndgp_status ndgp_plan_create(const ndgp_grid *grid, const ndgp_params *params,
                             const double *const delta[1 + NDGP_MAX_PATCHES],
                             double *const phi[1 + NDGP_MAX_PATCHES], void *workspace,
                             size_t workspace_bytes, hipStream_t stream, ndgp_plan **plan) {
    return guarded([&] {
        return plan_create_impl(grid, params, delta, phi, workspace, workspace_bytes, stream,
                                plan);
    });
}

ndgp_status ndgp_plan_poll(ndgp_plan *plan, int32_t *done, ndgp_report *report) {
    return guarded([&] { return plan_poll_impl(plan, done, report); });
}

ndgp_status ndgp_plan_step(ndgp_plan *plan) {
    return guarded([&] {
        Range r("ndgp_plan_step");
        return plan_step_impl(plan);
    });
}

void ndgp_plan_destroy(ndgp_plan *plan) {
    if (!plan) return;
    // Every enqueue of a plan ends with a copy into its pinned slot and a
    // record of its event.  A plan destroyed before its work has finished
    // waits for that event first: the slot goes back to the pool, and a
    // later plan must not receive this one's late copy.  If the wait fails
    // the slot is leaked rather than reused.
    bool idle = true;
    if (plan->ev) {
        idle = hipEventSynchronize(plan->ev) == hipSuccess;
        (void)hipEventDestroy(plan->ev);
    }
    if (plan->slot && idle) pinned_slots().release(plan->slot);
    delete plan;
}

ndgp_status ndgp_diff_norms(const double *a, const double *b, size_t count, double out[3],
                            void *workspace, size_t workspace_bytes, hipStream_t stream) {
    return guarded(
        [&] { return diff_norms_impl(a, b, count, out, workspace, workspace_bytes, stream); });
}

} // extern "C"
