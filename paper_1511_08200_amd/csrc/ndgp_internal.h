// ndgp_internal.h -- types and kernel launchers shared by the library's two
// translation units (kernels, host driver).  Not part of the public ABI.
#pragma once

#include <cmath>

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ndgp {

constexpr int kMaxLevels = 12;
constexpr int kBlock = 256;        // threads per block of the streaming kernels
constexpr int kReduceBlocks = 4096; // fixed partial count of the deterministic reductions
constexpr int kCoarsestMax = 8;    // the single-workgroup coarsest solve holds <= 8^3 cells
constexpr int kCoarsestSweeps = 16;

// One grid of a multigrid hierarchy.
//  periodic: phi/alt/hat are natural n^3 with periodic wrap-around;
//  else    : phi/alt/hat are padded (n+2)^3 with a fixed ghost shell.
// s (the source) is always natural n^3.  Everything is in cell units: the
// level's spacing is 1, alpha is alpha_phys / h_l^2 and s is h_l^2 S_phys.
struct Level {
    int n = 0;
    int lg = 0;            // log2(n)
    bool periodic = true;
    double alpha = 0.0;    // cell-unit coefficient of the nonlinear term
    double omega = 1.0;    // step factor of the per-cell update (1: the root itself)
    double *phi = nullptr; // current iterate
    double *alt = nullptr; // ping-pong partner of phi (same layout, same ghosts)
    double *s = nullptr;   // source, natural n^3
    double *hat = nullptr; // restriction of the finer iterate (levels >= 1)
    // Coarse level of a refinement's hierarchy: the ghost shell follows the
    // interior (ghost = hat + (-1/3)^d (phi - hat) of the adjacent interior
    // cell, d = number of axes along which the ghost lies outside), so that
    // the coarse correction vanishes where the fine boundary values sit.
    bool dyn_bc = false;
    // Cell-wise truncation: natural n^3, 0 = the cell is held at its value
    // (no relaxation, no residual, no coarse-grid correction); null = none held.
    const unsigned char *mask = nullptr;
    // With a mask on a level with fixed ghosts: per colour and block of the
    // half-sweep launch, 1 if the block relaxes any cell; blocks of held cells
    // are skipped (both ping-pong arrays must then hold the held values).
    const unsigned char *active = nullptr;
    // The same per workgroup of the fused sweep (1 if it writes any relaxed cell).
    const unsigned char *tile_on = nullptr;

    size_t cells() const { return (size_t)n * n * n; }
    size_t slots() const {
        return periodic ? cells() : (size_t)(n + 2) * (n + 2) * (n + 2);
    }
};

// The bookkeeping of the cycle loop on one level, shared by the blocking
// drivers, the plans and the one-workgroup box solves (host and device):
// stopping test, divergence, and the safeguard.  The red-black sweep updates
// same-colour edge neighbours simultaneously (Jacobi within a colour); where
// the nonlinear coupling through those edges is strong (extreme densities
// with large r_c) that iteration can amplify an error mode, and the cycles
// diverge after first converging.  Damping the step from the middle of such
// a run does not recover it (the iterate has left the basin), but a run
// damped from its start converges.  So once the residual has grown to
// kRiseFactor times the smallest one seen (well above rounding level) with
// the plain step, the level is solved again from its initial guess with the
// damped step u + kDampedStep du everywhere.  Plateaus with small ups and
// downs, common before the screened regions settle, do not trigger it; runs
// that never grow keep the plain root, bit for bit.
constexpr double kDampedStep = 0.8;
constexpr double kRiseFactor = 2.0;
constexpr double kDampAbove = 1e-9; // rel. residual; below it a rise is rounding noise
constexpr int kTolNotReached = 1, kStagnated = 2; // verdict codes (0: reached)

struct CycleMonitor {
    double tol = 0.0;
    int maxc = 0;
    double rel0 = 0.0, prev = 0.0, rel = 0.0, best = 0.0;
    int slow = 0;
    bool damped = false;

    __host__ __device__ void start(double r) { rel = rel0 = prev = best = r; }
    // a zero residual is exact (e.g. a patch whose every cell is held)
    __host__ __device__ bool converged() const { return rel == 0.0 || (tol > 0.0 && rel <= tol); }
    __host__ __device__ bool diverged() const {
        return !__builtin_isfinite(rel) || rel > 1e6 * (rel0 < 1.0 ? 1.0 : rel0);
    }
    // after a cycle: true when the level is to be solved again with the damped step
    __host__ __device__ bool record(double r) {
        rel = r;
        bool damp = false;
        if (!damped && rel > kRiseFactor * best && rel > kDampAbove) {
            damped = damp = true;
            slow = 0;
        } else if (tol == 0.0) {
            slow = rel > 0.7 * prev ? slow + 1 : 0;
        }
        best = rel < best ? rel : best;
        prev = rel;
        return damp;
    }
    __host__ __device__ bool stalled() const { return tol == 0.0 && slow >= 2; }
    // once the loop has stopped (not diverged): 0, kTolNotReached or kStagnated
    __host__ __device__ int verdict_code() const {
        if (tol > 0.0 && rel > tol) return kTolNotReached;
        if (tol == 0.0 && rel > 1e-11) return kStagnated;
        return 0;
    }
};

// ---- the small boxes of an adaptive tree, one workgroup each (ndgp_boxes.hip)
// Relaxed boxes of at most kBoxBatchMaxN cells per side (32^3 ones when
// several share a tree level) are solved by one launch per tree level.  A
// box's status: 0, kTolNotReached, kStagnated, kBoxDiverged, or kBoxBadSource
// (non-finite density).
constexpr int kBoxBatchMaxN = 32;
constexpr int kBoxDiverged = 8, kBoxBadSource = 9;
struct BoxJob {
    const double *parent;  // the parent's solution: natural n^3 (domain) or padded
    int np, parent_periodic;
    int origin[3];         // lower corner in parent cells
    int n, nl;             // cells per side (8, 16 or 32) and levels (n = 8 -> 1)
    double *phi;           // out: padded (n+2)^3
    double *alt, *s0;      // n = 32: partner and source of the finest level (scratch)
    double *phi1, *alt1, *hat1, *s1; // n = 32: its 16^3 level (scratch; padded, natural s)
    const double *delta;   // natural n^3
    double f;              // source factor Omega_m / (a beta) h^2 of the box
    double alpha[3];       // per level, cell units
};
struct BoxResult {
    int cycles, damped_from, status;
    double rel;
};
struct BoxRun {
    const double *dsum;    // device: the domain's delta sum
    double inv_cells0;     // 1 / cells of the domain
    int nu1, nu2, csweeps, maxc;
    double tol;
    int damped_start;
    unsigned *fallbacks;   // event counters (no real root, past the vertex)
};
void launch_solve_boxes(const BoxJob *jobs, BoxResult *results, int count, const BoxRun &run,
                        hipStream_t st);

// levels of a hierarchy that coarsens by 2 down to <= 8 cells per side
inline int default_levels(int n) {
    int l = 1;
    while ((n >> (l - 1)) > kCoarsestMax) ++l;
    return l;
}

// Can every multigrid level (nlev of them) of a Dirichlet child of nc cells
// with its lower corner at `origin` parent cells (along one axis) interpolate
// its ghost shell (and, on the finest level, its interior) from a padded
// parent of np cells?  Level m's cells are 2^m / 2 parent cells wide.
inline bool child_fits_axis(int np, int origin, int nc, int nlev) {
    for (int m = 0; m < nlev; ++m) {
        const int nm = nc >> m;
        const double q = std::ldexp(1.0, m - 1);
        const double xmin = origin + (-1 + 0.5) * q - 0.5;
        const double xmax = origin + (nm + 0.5) * q - 0.5;
        if (std::floor(xmin) < -1.0 || std::floor(xmax) + 1.0 > (double)np) return false;
    }
    return true;
}

// Where a child box sits in its parent: lower corner in parent cells and a
// cell size of 2^m / 2 parent cells.
struct ChildBox {
    int origin[3];
    int m;
    int nc;
};

// ---- kernel launchers (ndgp_kernels.hip); all enqueue on `st` ------------

// Red-black half sweep: cells of colour `colour` ((i+j+k) & 1) get the root
// of their own discrete quadratic from pin; the other colour is copied.
void launch_smooth_half(const Level &L, const double *pin, double *pout, int colour,
                        unsigned *fallbacks, hipStream_t st);
// One full red-black sweep (both colours) in one launch through LDS tiles;
// identical results to two launch_smooth_half calls.  Periodic levels with
// n >= 128 only (fused_sweep_ok).
bool fused_prolong_ok(const Level &L);
bool fused_sweep_ok(const Level &L);
void launch_sweep_fused(const Level &L, const double *pin, double *pout, unsigned *fallbacks,
                        hipStream_t st);
// The same sweep starting from pin + P(C.phi - C.hat) (the coarse-grid
// correction, added on load): bit for bit launch_prolong_correct followed by
// launch_sweep_fused.
void launch_sweep_fused_prolong(const Level &L, const Level &C, const double *pin, double *pout,
                                unsigned *fallbacks, hipStream_t st);
// Per-block partial sums of r^2, r = s - L[phi]; optionally r_out = r * scale.
void launch_residual_sumsq(const Level &L, double *partials, double *r_out, double r_scale,
                           hipStream_t st);
// The LDS-tiled residual (periodic, n >= 128: residual_tiled_ok) with r rounded
// to FP32 into r32 and the partial sums of r^2 (FP64).
bool residual_tiled_ok(const Level &L);
void launch_residual_tiled_to32(const Level &L, float *r32, double *partials, hipStream_t st);
// Per-block partial sums of a[i]^2 (squares != 0) or a[i] over count values.
void launch_partial_sums(const double *a, size_t count, bool squares, double *partials,
                         hipStream_t st);
// out[0] = sum of the kReduceBlocks partials, in a fixed order.
void launch_reduce_final(const double *partials, double *out, hipStream_t st);
// out[0..3) = sum r^2, sum s^2 and the relative norm, from sums[1] = sum s^2
// and sums[2] = sum r^2 (one thread).
void launch_residual_norms(const double *sums, double *out, hipStream_t st);
// FAS restriction: C.hat = mean of children of F.phi; C.s = 4 * mean of children residuals.
// tiled: through LDS on periodic levels of n >= 128 (same bits).
void launch_restrict_residual(const Level &F, const Level &C, bool tiled, hipStream_t st);
// FAS coarse source C.s = L_C[C.hat] + C.s; C.phi = C.hat (interior).
// tiled: through LDS on periodic levels of n >= 128 (same bits).
void launch_coarse_source(const Level &C, bool tiled, hipStream_t st);
// F.phi += trilinear(C.phi - C.hat)
void launch_prolong_correct(const Level &F, const Level &C, hipStream_t st);
// F.phi = trilinear(C.phi)    (periodic levels; nested-iteration start)
void launch_prolong_full(const Level &F, const Level &C, hipStream_t st);
// C.s = 4 * mean of children of F.s
void launch_restrict_source(const Level &F, const Level &C, hipStream_t st);
// Many red-black sweeps of a <= 8^3 level in one workgroup (LDS resident).
void launch_coarsest(const Level &L, int sweeps, unsigned *fallbacks, hipStream_t st);
// The V-cycle of level l (n <= 16, periodic) and every coarser level in one
// workgroup with its arrays in LDS; bit for bit the per-level launches.
constexpr int kBottomMaxLevels = 4;
struct BottomLevels {
    int levels;                       // l .. nl-1
    double alpha[kBottomMaxLevels];   // per level, cell units
    double omega;                     // step factor of the per-cell update
};
bool bottom_ok(const Level *H, int l, int nl);
void launch_bottom(const Level *H, int l, int nl, int nu1, int nu2, int csweeps,
                   unsigned *fallbacks, hipStream_t st);
// The same for the coarse levels of a refinement (padded, ghost shells that
// follow the interior, held cells): level l (n <= 16) and every coarser level.
struct BottomDirLevels {
    int levels;                                 // l .. nl-1
    int lg0;                                    // log2(n) of level l
    double alpha[kBottomMaxLevels];
    double omega;
    double *phi0;                               // level l: in/out, padded
    const double *s0;                           // level l: natural
    const double *hat[kBottomMaxLevels];        // padded (ghost shells; interiors of
                                                // the coarser levels are recomputed)
    const unsigned char *mask[kBottomMaxLevels]; // natural, or null (none held)
};
bool bottom_dir_ok(const Level *H, int l, int nl);
void launch_bottom_dir(const Level *H, int l, int nl, int nu1, int nu2, int csweeps,
                       unsigned *fallbacks, hipStream_t st);
// s = f * (delta - sum[0] * inv_count_mean)     (sum: device scalar)
void launch_source(const double *delta, size_t count, const double *sum, double inv_count_mean,
                   double f, double *s, hipStream_t st);
// a[i] -= sum[0] / count        (sum: device scalar; removes the mean)
void launch_shift_by_mean(double *a, size_t count, const double *sum, hipStream_t st);
// a[i] = v
void launch_fill(double *a, size_t count, double v, hipStream_t st);
// Cell-centred trilinear interpolation of a parent level into a padded child
// (interior and ghost shell, or ghost shell only).
void launch_interpolate(const double *parent, int np, bool parent_periodic, const ChildBox &b,
                        double *child_pad, bool ghosts_only, hipStream_t st);
// F = -grad(phi)/2 by central differences; f has 3 * n^3 values (x, y, z).
void launch_force(const double *phi, int n, bool periodic, double h, double *f, hipStream_t st);
// partials[0..B) = per-block sum (a-b)^2, [B..2B) sum a^2, [2B..3B) sum b^2
// (B = kReduceBlocks; b may be null)
void launch_diff_partials(const double *a, const double *b, size_t count, double *partials,
                          hipStream_t st);
// dst[i] = src[i]
void launch_copy(const double *src, double *dst, size_t count, hipStream_t st);

// Cell-wise truncation mask of a ratio-2 child box (m = 0) from its parent's
// phi and Newtonian potential psi (same layout as phi: periodic natural or
// padded): 1 where |grad phi| / 2 >= threshold |grad psi| on the parent cell.
// partials[0..kReduceBlocks) receive per-block counts of the 1s.
void launch_cell_mask(const double *phi_parent, const double *psi_parent, int np,
                      bool parent_periodic, const ChildBox &b, double threshold,
                      unsigned char *mask, double *partials, hipStream_t st);
// mask_c (nc^3) = 1 where all eight children in mask_f ((2 nc)^3) are 1
// Guard bands of the workspace (words <= 64): fill with `word`; count the
// words that differ into *bad.
void launch_guard_fill(void *band, int words, uint64_t word, hipStream_t st);
void launch_guard_check(const void *band, int words, uint64_t word, unsigned *bad,
                        hipStream_t st);
// Block activity of a masked level: per block of the half sweeps of both
// colours, then per workgroup of the fused sweep (tile_activity points there).
size_t block_activity_bytes(int n);
const unsigned char *tile_activity(const unsigned char *active, int n);
void launch_block_activity(const unsigned char *mask, int n, unsigned char *active,
                           hipStream_t st);
void launch_mask_restrict(const unsigned char *mask_f, int nc, unsigned char *mask_c,
                          hipStream_t st);

// Total force F = -grad(psi) - grad(phi)/2 (Eq. modpoisson) on one level,
// 3 * n^3 values (x, y, z); phi and psi in the level's layout.
void launch_total_force(const double *phi, const double *psi, int n, bool periodic, double h,
                        double *f, hipStream_t st);
// G_eff - 1 = |F_5th| / |F_GR| over the cells of one level outside the child box
// [child_origin, child_origin + child_half) (child_half = 0: none):
// out[0..4] = count, sum, sum of squares, min, max (device); hist[0..n_edges]
// = bin counts (device, zeroed here); partials: 5 * kReduceBlocks doubles.
constexpr int kGeffMaxEdges = 255;
void launch_geff_level(const double *phi, const double *psi, int n, bool periodic,
                       const int child_origin[3], int child_half, const double *edges,
                       int n_edges, double *partials, unsigned long long *hist, double *out,
                       hipStream_t st);

// Cloud-in-cell deposit of np particles (pos: x, y, z arrays of np doubles
// each, box units) onto one level: m^3 cells of 2^-q domain cells with lower
// corner `corner` (domain cells); q = 0 is the periodic domain (m = n).
// acc: m^3 fixed-point accumulators; delta = count / mean - 1.
void launch_cic_deposit(const double *pos, long long np, int n, const double corner[3], int q,
                        int m, unsigned long long *acc, double *delta, hipStream_t st);
// flags = (delta + 1) mean > n_ref; partials[0..kReduceBlocks) = per-block
// counts of flagged cells.
void launch_refine_flags(const double *delta, size_t cells, double mean, double n_ref,
                         unsigned char *flags, double *partials, hipStream_t st);
// Geometry and per-level fields (3 * m^3, x then y then z) for the gather.
constexpr int kCicMaxLevels = 5;
struct CicLevels {
    int levels;
    int n;
    int m[kCicMaxLevels];
    double cells_per_domain[kCicMaxLevels];
    double corner[kCicMaxLevels][3];
    const double *force[kCicMaxLevels];
};
// out (3 * np, x then y then z) = cloud-in-cell interpolation of the finest
// level whose eight cells around the particle lie inside it.
void launch_cic_gather(const double *pos, long long np, const CicLevels &lv, double *out,
                       hipStream_t st);

// message for ndgp_last_error() in the calling thread
void set_last_error(const char *msg);

} // namespace ndgp

namespace ndgp {

// FP32 side of the mixed-precision solve: per periodic level the FP32 copy
// of the current FP64 field (`phi`, the base of the correction), the
// correction e and its ping-pong partner, the correction equation's source
// r and, on coarse levels, the restriction of the finer correction.  Cell
// units as in Level.
struct Level32 {
    int n = 0, lg = 0;
    double alpha = 0.0;
    double omega = 1.0; // step factor of the per-cell update (1: the root itself)
    float *phi = nullptr;
    float *e = nullptr;
    float *ealt = nullptr;
    float *r = nullptr;
    float *ehat = nullptr;
    size_t cells() const { return (size_t)n * n * n; }
};

// ---- mixed-precision launchers (ndgp_mixed.hip) ---------------------------

// r32 = float(s - L[phi]) with FP64 arithmetic, and per-block partials of
// (s - L[phi])^2.
void launch_residual_to32(const Level &L, float *r32, double *partials, hipStream_t st);
// phi32 = float(phi64)
void launch_to32(const double *a, float *b, size_t count, hipStream_t st);
// coarse = mean of the 8 children (FP32 field)
void launch_avg32(const Level32 &F, const Level32 &C, hipStream_t st);
// phi64 += double(e32)
void launch_add32(double *phi, const float *e, size_t count, hipStream_t st);
// phi += e and phi32 = (float)phi in one pass (same bits as launch_add32 + launch_to32)
void launch_add_to32(double *phi, const float *e, float *phi32, size_t count, hipStream_t st);
void launch_fill32(float *a, size_t count, float v, hipStream_t st);
// one colour of a red-black sweep of the correction equation
// L[phi + e] - L[phi] = r on a periodic level
void launch_corr_half(const Level32 &L, const float *ein, float *eout, int colour,
                      unsigned *fallbacks, hipStream_t st);
// Both colours of the correction in one launch through LDS tiles, n >= 128
// (corr_fused_ok); bit for bit two launch_corr_half calls.
bool corr_fused_ok(const Level32 &L);
void launch_corr_sweep_fused(const Level32 &L, const float *ein, float *eout,
                             unsigned *fallbacks, hipStream_t st);
// the same sweep starting from e = 0 (nothing read): bit for bit a zero fill
// of the input followed by launch_corr_sweep_fused
void launch_corr_sweep_fused_from_zero(const Level32 &L, float *eout, unsigned *fallbacks,
                                       hipStream_t st);
// the same sweep starting from ein + trilinear(C.e - C.ehat): bit for bit
// launch_corr_prolong followed by launch_corr_sweep_fused
void launch_corr_sweep_fused_prolong(const Level32 &L, const Level32 &C, const float *ein,
                                     float *eout, unsigned *fallbacks, hipStream_t st);
// C.ehat = mean children of F.e; C.r = 4 mean children of (r - A(e));
// tiled: through LDS for n >= 128 (same bits)
void launch_corr_restrict(const Level32 &F, const Level32 &C, bool tiled, hipStream_t st);
// C.r = A_C(C.ehat) + C.r; C.e = C.ehat
void launch_corr_coarse_source(const Level32 &C, hipStream_t st);
// F.e += trilinear(C.e - C.ehat)
void launch_corr_prolong(const Level32 &F, const Level32 &C, hipStream_t st);
// many sweeps of the correction equation on a <= 8^3 level in one workgroup
void launch_corr_coarsest(const Level32 &L, int sweeps, unsigned *fallbacks, hipStream_t st);

} // namespace ndgp
