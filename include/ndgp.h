/*
 * ndgp.h -- C ABI of the MI355X (gfx950) solver for the nDGP scalar field.
 *
 * The equation is the quasi-static scalar-field equation of the normal-branch
 * DGP model, Sec. II Eq. (eomvarphi) of Barreira, Bose & Li, arXiv:1511.08200:
 *
 *     lap(phi) + r_c^2 / (3 beta a^2) [ (lap phi)^2 - (d_i d_j phi)^2 ]
 *         = 8 pi G a^2 delta rho_m / (3 beta),
 *
 * written with H0 = c = 1 (lengths in units of c/H0, phi in units of c^2) as
 *
 *     lap(phi) + alpha [ ... ] = S,   alpha = r_c^2/(3 beta a^2),
 *                                     S = Omega_m (delta - mean delta)/(a beta).
 *
 * It is solved on a periodic domain grid and on up to four static nested
 * refinement patches (Sec. III.A: domain level first, then refinements with
 * boundary values and initial guess interpolated from the coarser level).
 * In NDGP_MODE_INTERPOLATED the refinements keep the interpolated guess as
 * their answer: the paper's speed-up, Sec. III.B.  NDGP_MODE_TRUNCATED
 * relaxes the refinements below a given level and interpolates from there on
 * (the truncation criteria l >= l_trunc of Sec. IV.A).  The fifth force is
 * -grad(phi)/2 (Eq. modpoisson) by central differences (Sec. III.B).
 *
 * Discretisation (the paper defers it to another work): cell-centred fields;
 * second differences D_aa on the diagonal; each mixed derivative squared is
 * the mean over the four corners of its plane of the one-sided mixed
 * difference squared.  This 19-point form is conservative: the nonlinear term
 * sums to zero over a periodic grid, as it must for a zero-mean source.
 *
 * Conventions for every entry point
 *  - Grid arrays are float64 in natural layout [z][y][x], x fastest.  Domain
 *    arrays have n^3 cells.  Patch SOLUTION arrays are "padded":
 *    (m+2)^3 cells, the m^3 interior plus a one-cell ghost shell, cell (i,j,k)
 *    with i,j,k in [-1, m] at ((k+1)(m+2) + (j+1))(m+2) + (i+1).  Patch
 *    DENSITY arrays have m^3 cells (no shell).
 *  - Array and workspace pointers are DEVICE pointers; the caller owns them
 *    and keeps them alive until the work enqueued on `stream` has finished.
 *    ndgp_grid, ndgp_params and ndgp_report are HOST structs.
 *  - The library never allocates device memory: all scratch space is carved
 *    from the caller's workspace (size from ndgp_workspace_bytes, 256-byte
 *    aligned start).
 *  - Work is enqueued on `stream` (0 = the null stream).  Nothing throws
 *    across the ABI; every call returns an ndgp_status and, on failure,
 *    leaves a message for ndgp_last_error() in the calling thread.
 *  - Results are deterministic: the same inputs give the same bits, whatever
 *    else runs on the GPU (all reductions have a fixed order, no atomics
 *    touch results).
 */
#ifndef NDGP_H
#define NDGP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NDGP_ABI_VERSION 3
#define NDGP_MAX_PATCHES 4
#define NDGP_HIST_LEN 64

typedef enum {
    NDGP_OK = 0,
    NDGP_EINVAL = -1,  /* bad argument: sizes, parameters, pointers, non-finite delta */
    NDGP_ENOMEM = -2,  /* workspace smaller than ndgp_workspace_bytes()             */
    NDGP_ENOCONV = -3, /* tolerance not reached in max_cycles, or divergence:
                          phi holds the last iterate                                 */
    NDGP_EDEVICE = -4  /* a HIP call failed                                          */
} ndgp_status;

typedef enum {
    NDGP_MODE_FULL = 0,         /* refinements relaxed to convergence (Sec. III.A)    */
    NDGP_MODE_INTERPOLATED = 1, /* refinements = interpolated coarse field (Sec. III.B) */
    NDGP_MODE_TRUNCATED = 2     /* refinements 1 .. trunc_level-1 relaxed, trunc_level ..
                                   n_patch interpolated from their relaxed or
                                   interpolated parent (Sec. III.B, Sec. IV.A: the
                                   paper's l_trunc is l_d + trunc_level, so its
                                   criteria l_d+1, l_d+2, l_d+4 are trunc_level 1, 2,
                                   4; 1 is NDGP_MODE_INTERPOLATED, n_patch+1 is
                                   NDGP_MODE_FULL)                                     */
} ndgp_mode;

typedef enum {
    NDGP_PREC_FP64 = 0, /* every kernel in FP64                                       */
    NDGP_PREC_MIXED = 1 /* domain level: FP32 multigrid on the correction e of
                           L[phi + e] - L[phi] = s - L[phi] inside an FP64
                           defect-correction loop (FP64 residual, update and
                           quadratic discriminant); ndgp_report.cycles[0] counts
                           the outer iterations (2 FP32 V-cycles each).  Patches
                           relax in FP64. */
} ndgp_precision;

/* flags */
#define NDGP_WARM_START 1u /* phi[0] holds the initial guess of the domain level
                              (the paper allows the previous time step's field);
                              otherwise the guess comes from nested iteration */
#define NDGP_PROFILE 2u    /* time the domain level's relaxation sweeps with HIP
                              events on `stream` (ndgp_report.t_smooth_ms) */
#define NDGP_TWO_PASS 4u   /* one launch per colour, per transfer and per level,
                              one thread per cell: no fused one-launch sweep or
                              LDS-tiled restriction on large levels, no
                              one-workgroup bottom of the V-cycle on levels of
                              at most 16^3 cells, and the boxes of a tree solved
                              one after the other; same results, bit for bit */
#define NDGP_DAMPED 8u     /* relax every level with the damped step u + 0.8 du from
                              the start (the mode the divergence safeguard restarts
                              in; ndgp_report.damped_from = 1 on relaxed levels) */

typedef struct {
    int32_t n;             /* domain cells per side: power of two, 8..1024              */
    double h;              /* domain cell size in c/H0 (> 0)                            */
    int32_t n_patch;       /* number of nested refinement levels, 0..NDGP_MAX_PATCHES  */
    int32_t patch_n[NDGP_MAX_PATCHES];       /* cells per side, power of two, 8..512   */
    int32_t patch_origin[NDGP_MAX_PATCHES][3]; /* lower corner (x,y,z) in PARENT cells;
                                                  patch 1 may wrap around the periodic
                                                  domain; patch q > 1 must lie inside
                                                  patch q-1 with room for the
                                                  interpolation stencils of all its
                                                  multigrid levels (of its finest level
                                                  only if it is interpolated)           */
} ndgp_grid;

typedef struct {
    double rc;         /* r_c H0 (>= 0; 0 gives the linear Poisson equation)          */
    double beta;       /* beta(a) of Eq. (beta) (> 0); see ndgp_beta_lcdm              */
    double a;          /* scale factor (> 0)                                           */
    double omega_m;    /* Omega_m0 (> 0)                                               */
    double tol;        /* stop when ||S - L phi||_2 / ||S||_2 <= tol on every relaxed
                          level (>= 0; 0 = run max_cycles)                              */
    int32_t max_cycles; /* V-cycles per level (1..1000; 0 = 50)                         */
    int32_t nu1, nu2;  /* pre/post red-black sweeps per level (0 = 2; at most 16)       */
    int32_t n_levels;  /* multigrid levels of the domain grid (0 = down to 8^3)         */
    int32_t mode;      /* ndgp_mode                                                    */
    int32_t precision; /* ndgp_precision                                               */
    uint32_t flags;    /* NDGP_WARM_START | NDGP_PROFILE | NDGP_TWO_PASS | NDGP_DAMPED */
    int32_t trunc_level; /* NDGP_MODE_TRUNCATED: first interpolated refinement level,
                            1..n_patch+1; ignored by the other modes                    */
} ndgp_params;

typedef struct {
    int32_t cycles[1 + NDGP_MAX_PATCHES];  /* V-cycles (or outer iterations) per level  */
    double rel_res[1 + NDGP_MAX_PATCHES];  /* final relative residual per level
                                              (-1 for a level filled by interpolation) */
    double removed_mean;   /* mean of delta projected out of the domain source         */
    double phi_mean;       /* mean of the domain phi removed at the end (gauge)        */
    int32_t fallbacks;     /* relaxation visits where the cell quadratic had no real
                              root (moved to its vertex instead, Eq. newton's
                              linearisation is then stationary)                         */
    int32_t hist_len;      /* entries of res_hist used                                 */
    double res_hist[NDGP_HIST_LEN]; /* relative residual of the domain level per cycle */
    double t_total_ms;     /* wall time of the call                                    */
    double t_smooth_ms;    /* NDGP_PROFILE: GPU time of the domain level's relaxation
                              kernels (V-cycles after the start; events on `stream`)    */
    int32_t smooth_launches; /* relaxation kernel launches inside t_smooth_ms           */
    int32_t smooth_cells_per_launch; /* cells one such launch updates                   */
    int32_t damped_from[1 + NDGP_MAX_PATCHES]; /* per level: the first cycle (outer
                              iteration) of the solve restarted with the damped step
                              u + 0.8 du after the residual grew to twice its smallest
                              value; 0 = never damped                                   */
    double iterated_fraction[1 + NDGP_MAX_PATCHES]; /* per level: share of the cells
                              that were relaxed (1 for relaxed levels, 0 for levels
                              filled by interpolation, in between with
                              ndgp_solve_cellwise)                                     */
    int32_t holds;         /* relaxation visits of cells past the vertex of their own
                              quadratic (dL/dphi of Eq. newton had the non-elliptic
                              sign there): moved to the root on the elliptic side      */
} ndgp_report;

/* Library ABI version (NDGP_ABI_VERSION of the build). */
int32_t ndgp_version(void);

/* Message of the last failure in the calling thread ("" if none).  The string
   stays valid until the next failing call in that thread. */
const char *ndgp_last_error(void);

/* beta(a) of Eq. (beta), 1 + 2 H r_c (1 + Hdot/(3 H^2)), for the normal branch
   whose expansion is tuned to LCDM (Sec. II): H^2 = Omega_m a^-3 + 1 - Omega_m,
   H0 = 1.  Host function. */
double ndgp_beta_lcdm(double a, double omega_m, double rc);

/*
 * Screening in NFW haloes, to choose the truncation level (Sec. II.B, Sec. V).
 * Host functions; no GPU work.  Masses in M_sun/h, lengths in Mpc/h, both
 * physical (at z = 0 the same as comoving); e_z = H(z)/H0 (1 at z = 0); rc is
 * r_c H0 and beta is beta(a) of Eq. (beta).  Invalid arguments give NaN (or -1)
 * and a message for ndgp_last_error().
 *
 * ndgp_nfw_r200           R_200 of Eq. (r200), read with exponent 1/3: the
 *                         radius inside which the mean density is 200 times
 *                         the critical density 3 H(z)^2 / (8 pi G).
 * ndgp_nfw_force_ratio    G_eff - 1 = F_5th / F_GR at radius r of an NFW halo
 *                         (Eqs. nfw, nfwparams) from the spherical solution,
 *                         Eqs. (eomvarphi_sph2) and (rv).  Depends on r / R_200
 *                         and c200 only; tends to 1/(3 beta) far outside
 *                         (Eq. forcelarge) and to 0 deep inside.
 * ndgp_nfw_screening_radius  r_t: the radius where G_eff - 1 has fallen to
 *                         `fraction` (Sec. V); +inf if the unscreened value
 *                         1/(3 beta) is not above it (or rc = 0), 0 for
 *                         fraction <= 0.
 * ndgp_nfw_trunc_level    the first truncated refinement level k >= 1
 *                         (NDGP_MODE_TRUNCATED's trunc_level, the paper's
 *                         l_trunc - l_d): the coarsest refinement whose cell
 *                         size h_domain / 2^k is at most r_t (Sec. V: the
 *                         truncated levels are those with cells smaller than
 *                         r_t).  h_domain is the domain cell size in the same
 *                         physical Mpc/h.  A result above n_patch means no
 *                         patch is truncated.
 */
double ndgp_nfw_r200(double m200, double e_z);
double ndgp_nfw_force_ratio(double r, double m200, double c200, double rc, double beta,
                            double e_z);
double ndgp_nfw_screening_radius(double fraction, double m200, double c200, double rc,
                                 double beta, double e_z);
int32_t ndgp_nfw_trunc_level(double h_domain, double fraction, double m200, double c200,
                             double rc, double beta, double e_z);

/* Bytes of device workspace that ndgp_solve / ndgp_residual need for this
   grid and these parameters (0 if the arguments are invalid). */
size_t ndgp_workspace_bytes(const ndgp_grid *grid, const ndgp_params *params);

/*
 * Solve Eq. (eomvarphi) on the domain grid and every patch (Sec. III.A), or
 * fill the patches by interpolation (Sec. III.B, NDGP_MODE_INTERPOLATED), or
 * relax the patches below trunc_level and interpolate the rest
 * (NDGP_MODE_TRUNCATED).
 *   delta[0]      domain density contrast, n^3 (its mean is projected out)
 *   delta[q]      patch density contrasts, patch_n^3, measured against the
 *                 same mean density as the domain (needed only for relaxed
 *                 patches; may be NULL for interpolated ones)
 *   phi[0]        out: domain phi, n^3, zero mean (in: initial guess with
 *                 NDGP_WARM_START); 16-byte aligned
 *   phi[q]        out: patch phi, padded (patch_n+2)^3 with its ghost shell
 *                 (the fixed boundary values interpolated from the parent)
 *   report        optional (NULL allowed)
 * Blocks until the domain level converged (one 8-byte device-to-host read of
 * the residual norm per V-cycle), then until the whole call completed.
 * Returns NDGP_ENOCONV if a relaxed level did not reach tol; phi then holds
 * the last iterate.
 */
ndgp_status ndgp_solve(const ndgp_grid *grid, const ndgp_params *params,
                       const double *const delta[1 + NDGP_MAX_PATCHES],
                       double *const phi[1 + NDGP_MAX_PATCHES], void *workspace,
                       size_t workspace_bytes, hipStream_t stream, ndgp_report *report);

/*
 * Cell-wise truncation, the generalisation Sec. III.C proposes: as ndgp_solve,
 * but on every relaxed patch a cell is iterated only if the fifth force on its
 * parent cell is still large, |F_5th| >= threshold |F_GR| (F_5th = -grad(phi)/2
 * of the parent's final field, F_GR = -grad(psi), central differences on the
 * parent level); the other cells keep the value interpolated from the parent
 * and enter their neighbours' stencils as fixed values.  On the coarse levels
 * of the patch's multigrid a cell is held when any of its eight children is,
 * so that the held regions act as fixed boundaries on every level.
 * The relative residual of a patch counts the iterated cells only, against
 * ||S|| over the whole patch.  Patches above trunc_level (NDGP_MODE_TRUNCATED)
 * are interpolated as in ndgp_solve.
 *   psi[l]        Newtonian potential of level l, same layout as phi[l] (domain
 *                 natural n^3, patches padded with ghosts), for every level
 *                 that is the parent of a relaxed patch; others may be NULL.
 *                 Psi_N solves lap Psi_N = 4 pi G a^2 delta rho (Eq. modpoisson's
 *                 GR part); in the units of this ABI that is (3 beta / 2) times
 *                 the field ndgp_solve returns with rc = 0.
 *   threshold     >= 0; 0 iterates every cell (ndgp_solve's result, bit for
 *                 bit), +inf holds every cell (the interpolated patches).
 * report->iterated_fraction gives the share of iterated cells per level.
 */
ndgp_status ndgp_solve_cellwise(const ndgp_grid *grid, const ndgp_params *params,
                                const double *const delta[1 + NDGP_MAX_PATCHES],
                                const double *const psi[1 + NDGP_MAX_PATCHES], double threshold,
                                double *const phi[1 + NDGP_MAX_PATCHES], void *workspace,
                                size_t workspace_bytes, hipStream_t stream,
                                ndgp_report *report);

/*
 * Discrete residual of Eq. (eomgen-disc) on one level, r = S - L_h[phi], and its
 * relative 2-norm ||r|| / ||S||.
 *   level         0 = domain (phi n^3 natural); 1..n_patch = patch (phi padded,
 *                 its ghost shell used as boundary values)
 *   delta         delta[0] is always needed (its mean defines S on every level);
 *                 delta[level] is the level's density
 *   r_out         optional device array, n^3 / patch_n^3 natural, physical units
 *   rel_norm_out  optional host double
 * Blocks until rel_norm_out is written.
 */
ndgp_status ndgp_residual(const ndgp_grid *grid, const ndgp_params *params, int32_t level,
                          const double *const delta[1 + NDGP_MAX_PATCHES], const double *phi,
                          double *r_out, double *rel_norm_out, void *workspace,
                          size_t workspace_bytes, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the residual
 * of ndgp_residual without a workspace and without blocking.  Same arguments
 * and the same kernels, with two differences:
 *   norms_out     DEVICE, 3 doubles: sum r^2 and sum S^2 (both in the level's
 *                 cell units, h^2 S) and the relative norm ||r|| / ||S||, the
 *                 bits ndgp_residual returns in *rel_norm_out
 *   (no checks)   the call only enqueues: a non-finite delta gives NaN norms
 *                 instead of NDGP_EINVAL
 * The scratch space is a static device array of the library, one per GPU
 * (NDGP_NOALLOC_SCRATCH_BYTES, held until the process ends): a level of more
 * than NDGP_NOALLOC_MAX_CELLS cells is rejected with NDGP_EINVAL.  Every call
 * on a GPU uses that GPU's one array, whatever the stream: calls that overlap
 * on one GPU race (serialise them, e.g. on one stream).  `stream` must belong
 * to the current device.  The call never allocates device or pinned memory,
 * never synchronises, and enqueues no memset.
 */
#define NDGP_NOALLOC_MAX_CELLS 2097152 /* 128^3 */
#define NDGP_NOALLOC_SCRATCH_BYTES ((NDGP_NOALLOC_MAX_CELLS + 4096 + 32) * 8)
ndgp_status ndgp_residual_noalloc(const ndgp_grid *grid, const ndgp_params *params,
                                  int32_t level, const double *const delta[1 + NDGP_MAX_PATCHES],
                                  const double *phi, double *r_out, double *norms_out,
                                  hipStream_t stream);

/*
 * Fifth force F = -grad(phi)/2 by central differences on every level
 * (Sec. III.B), patches using their ghost shells.
 *   phi[l]        as produced by ndgp_solve
 *   force[l]      out: 3 * cells(l) doubles, x then y then z components, each
 *                 natural (n^3 or patch_n^3)
 * Enqueues only; does not block.
 */
ndgp_status ndgp_force(const ndgp_grid *grid, const double *const phi[1 + NDGP_MAX_PATCHES],
                       double *const force[1 + NDGP_MAX_PATCHES], hipStream_t stream);

/*
 * Total force on every level (Eq. modpoisson: the dynamical potential is
 * Psi_N + phi/2): F = -grad(Psi_N) - grad(phi)/2 by central differences,
 * patches using their ghost shells.
 *   phi[l]        as produced by ndgp_solve
 *   psi[l]        Newtonian potential, same layout as phi[l] (see
 *                 ndgp_solve_cellwise for its normalisation)
 *   force[l]      out: 3 * cells(l) doubles, x then y then z, each natural
 * Enqueues only; does not block.
 */
ndgp_status ndgp_total_force(const ndgp_grid *grid, const double *const phi[1 + NDGP_MAX_PATCHES],
                             const double *const psi[1 + NDGP_MAX_PATCHES],
                             double *const force[1 + NDGP_MAX_PATCHES], hipStream_t stream);

/*
 * Effective gravity per refinement level, the cell analogue of the paper's
 * G_eff against the AMR level (Sec. III.B, Sec. IV.B Fig. 3): for every cell,
 * G_eff - 1 = |F_5th| / |F_GR| with F_5th = -grad(phi)/2 and F_GR =
 * -grad(Psi_N), central differences (the spacing cancels; computed as
 * sqrt(sum dphi^2 / sum dpsi^2) / 2, a cell with no Newtonian force counts as
 * 0 without a fifth force, else +inf).  A cell of level l covered by patch
 * l+1 is left out: every cell counts on the finest level that holds it.
 *   edges         HOST, n_edges ascending values (1 <= n_edges <=
 *                 NDGP_GEFF_MAX_EDGES): bin 0 holds x < edges[0], bin b holds
 *                 edges[b-1] <= x < edges[b], bin n_edges holds x >= the last
 *   out[l]        HOST: cells counted, sum, sum of squares, min and max of
 *                 G_eff - 1 on level l (l = 0..n_patch)
 *   hist          HOST, (n_patch + 1) * (n_edges + 1) counts, level-major
 *   workspace     NDGP_GEFF_WORKSPACE bytes of device memory
 * Deterministic (fixed-order sums; exact integer counts).  Blocks until out
 * and hist are written.
 */
#define NDGP_GEFF_MAX_EDGES 255
#define NDGP_GEFF_WORKSPACE 262144
typedef struct {
    int64_t cells;
    double sum, sum_sq, min, max;
} ndgp_geff_level;
ndgp_status ndgp_geff_stats(const ndgp_grid *grid, const double *const phi[1 + NDGP_MAX_PATCHES],
                            const double *const psi[1 + NDGP_MAX_PATCHES], const double *edges,
                            int32_t n_edges, ndgp_geff_level out[1 + NDGP_MAX_PATCHES],
                            int64_t *hist, void *workspace, size_t workspace_bytes,
                            hipStream_t stream);

/*
 * Cloud-in-cell transfers between equal-mass particles and the grid levels
 * (Sec. IV.A: density and forces are interpolated back and forth between the
 * particles and the cells by cloud-in-cell).  Particle positions are DEVICE
 * arrays in structure-of-arrays order: pos[0..N) = x, pos[N..2N) = y,
 * pos[2N..3N) = z, in units of the box, each in [0, 1).  A patch compares
 * positions with its cells modulo the box, so patch 1 may wrap the domain.
 *
 * ndgp_cic_density    delta[l] (natural n^3 / patch_n^3, the layout ndgp_solve
 *                     takes) = count / mean - 1, mean = N / (n 2^l)^3 particles
 *                     per level-l cell: every level is measured against the
 *                     domain's mean density.  The weights are summed as
 *                     64-bit fixed-point numbers (2^-36 of a particle), so the
 *                     result is the same bits on every run.  1 <= N <=
 *                     NDGP_CIC_MAX_PARTICLES.  Workspace:
 *                     ndgp_cic_workspace_bytes(grid).  Enqueues only.
 * ndgp_cic_force      out (3 * N, x then y then z) = cloud-in-cell interpolation
 *                     of force[l] (3 * cells(l), as ndgp_force or
 *                     ndgp_total_force write it) from the finest level whose
 *                     eight cells around the particle all lie inside it.
 *                     Enqueues only.
 */
#define NDGP_CIC_MAX_PARTICLES (1LL << 28)
/* Refinement criterion (Sec. IV.A): a cell is refined when the particles in
   its volume number more than n_ref (the paper uses 4).  From the density
   contrast ndgp_cic_density wrote for N particles: flags[l][c] = 1 where
   (delta + 1) N / (n 2^l)^3 > n_ref, else 0 (device, cells(l) bytes each);
   n_flagged[l] (HOST) = number of flagged cells.  Blocks until n_flagged is
   written.  Workspace: NDGP_DIFF_NORMS_WORKSPACE bytes. */
ndgp_status ndgp_refine_flags(const ndgp_grid *grid, const double *const delta[1 + NDGP_MAX_PATCHES],
                              int64_t n_particles, double n_ref,
                              unsigned char *const flags[1 + NDGP_MAX_PATCHES],
                              int64_t n_flagged[1 + NDGP_MAX_PATCHES], void *workspace,
                              size_t workspace_bytes, hipStream_t stream);
size_t ndgp_cic_workspace_bytes(const ndgp_grid *grid);
ndgp_status ndgp_cic_density(const ndgp_grid *grid, const double *pos, int64_t n_particles,
                             double *const delta[1 + NDGP_MAX_PATCHES], void *workspace,
                             size_t workspace_bytes, hipStream_t stream);
ndgp_status ndgp_cic_force(const ndgp_grid *grid, const double *const force[1 + NDGP_MAX_PATCHES],
                           const double *pos, int64_t n_particles, double *out,
                           hipStream_t stream);

/*
 * Serving: the same solve as ndgp_solve, split into non-blocking steps so that
 * one host thread can keep many solves in flight on different streams
 * (continuous batching).  A plan owns nothing on the device: delta, phi and
 * the workspace stay the caller's and must stay alive until the plan is done
 * or destroyed.  Patches must all be interpolated: NDGP_MODE_INTERPOLATED, or
 * NDGP_MODE_TRUNCATED with trunc_level 1.  The
 * number of V-cycles a plan runs depends only on its own residual history,
 * so its result is bit for bit the one ndgp_solve gives, whatever else runs.
 *
 * ndgp_plan_create  checks the arguments, enqueues the source, the initial
 *                   guess and the first residual norm on `stream`; does not
 *                   block.
 * ndgp_plan_poll    never blocks: *done = 0 while work is in flight or the
 *                   plan waits for ndgp_plan_step; *done = 1 once phi is final
 *                   (report filled if non-NULL; the returned status is then
 *                   the solve's: NDGP_OK, NDGP_ENOCONV or NDGP_EINVAL for a
 *                   non-finite delta).  When a V-cycle has finished it decides
 *                   whether to stop (then it enqueues the gauge and the patch
 *                   interpolation).
 * ndgp_plan_step    enqueues the next V-cycle (mixed precision: the next outer
 *                   iteration) and its residual norm if the last poll found
 *                   the plan waiting; otherwise does nothing.  Never blocks.
 * ndgp_plan_destroy releases the plan's host resources.  Called before poll
 *                   has reported done, it blocks until the work the plan
 *                   has enqueued is finished (the only call that blocks);
 *                   the caller must not free the device buffers before.
 */
typedef struct ndgp_plan ndgp_plan;
ndgp_status ndgp_plan_create(const ndgp_grid *grid, const ndgp_params *params,
                             const double *const delta[1 + NDGP_MAX_PATCHES],
                             double *const phi[1 + NDGP_MAX_PATCHES], void *workspace,
                             size_t workspace_bytes, hipStream_t stream, ndgp_plan **plan);
ndgp_status ndgp_plan_poll(ndgp_plan *plan, int32_t *done, ndgp_report *report);
ndgp_status ndgp_plan_step(ndgp_plan *plan);
void ndgp_plan_destroy(ndgp_plan *plan);

/*
 * Adaptive refinement (Sec. IV.A: a cell is refined when it holds more than
 * N_ref particles; the refinements form a tree of patches, several per level).
 *
 * ndgp_box            one cubic refinement patch of a tree: its parent (-1 =
 *                     the domain, else the index of an earlier box), cells per
 *                     side (power of two, 8..512, at most twice its parent's)
 *                     and lower corner in parent cells.  Children of the
 *                     domain may wrap around it; a child of a box must lie
 *                     inside it with room for the interpolation stencils of
 *                     every multigrid level of the child (the rule of
 *                     ndgp_grid's nested patches).  Children of one parent
 *                     must not overlap (they may touch).
 * ndgp_refine_boxes   clusters the refinement flags of one level into cubic
 *                     patches by the point-clustering algorithm of Berger &
 *                     Rigoutsos (IEEE Trans. Syst. Man Cybern. 21, 1991):
 *                     bounding box of the flagged cells, accepted when at least
 *                     `efficiency` of its cells are flagged, otherwise split at
 *                     a hole of the flag signatures, else at the strongest sign
 *                     change of their second difference, else in the middle of
 *                     its longest side; a periodic level is cut open along the
 *                     widest empty slab of each axis first.  Each cluster then
 *                     becomes the smallest power-of-two cube of child cells
 *                     (refinement ratio 2, at least 8 cells) centred on it;
 *                     cubes that overlap are merged into one around both
 *                     clusters until none do.  On a patch parent the cubes are
 *                     kept inside it with the stencil room above: flagged cells
 *                     closer to its boundary than that stay unrefined.
 *   flags             the level's flags (natural n^3 bytes, nonzero = refine),
 *                     DEVICE memory if flags_on_device, else HOST memory (the
 *                     clustering itself runs on the host)
 *   n, periodic       the level: the domain (periodic) or a patch
 *   parent_index      written into every box's parent field
 *   efficiency        in (0, 1]; min_width >= 1: clusters no wider than this
 *                     (parent cells) are not split further
 *   boxes, max_boxes  HOST output; NDGP_ENOMEM if more boxes are needed
 *   n_boxes           HOST output: boxes written (0 if nothing is flagged)
 * ndgp_solve_amr      the domain level as ndgp_solve with n_patch = 0, then
 *                     every box from its solved (or interpolated) parent, tree
 *                     depth by tree depth: ghost shell and initial guess
 *                     interpolated, then relaxed with its own FAS multigrid
 *                     (NDGP_MODE_FULL; boxes of at most 16^3 cells, and 32^3
 *                     ones when four or more share a depth, all in one launch
 *                     of one workgroup each; the result is bit for bit that of
 *                     relaxing them one after the other, which NDGP_TWO_PASS
 *                     forces), or
 *                     kept at the interpolated field (NDGP_MODE_INTERPOLATED;
 *                     NDGP_MODE_TRUNCATED interpolates the boxes of tree depth
 *                     trunc_level and deeper).  Mixed precision applies to the
 *                     domain level.  delta[1 + b] is box b's density contrast
 *                     (n^3, measured against the domain's mean density as for
 *                     ndgp_solve; may be NULL for interpolated boxes) and
 *                     phi[1 + b] its padded solution ((n+2)^3).  box_report
 *                     (HOST, n_boxes entries, optional) receives each box's
 *                     tree depth, V-cycles, restart cycle and relative residual
 *                     (-1 if interpolated).  Workspace: ndgp_amr_workspace_bytes.
 */
#define NDGP_AMR_MAX_BOXES 4096
typedef struct {
    int32_t parent;
    int32_t n;
    int32_t origin[3];
} ndgp_box;
typedef struct {
    int32_t depth;
    int32_t cycles;
    int32_t damped_from;
    double rel_res;
} ndgp_box_report;
ndgp_status ndgp_refine_boxes(const unsigned char *flags, int32_t flags_on_device, int32_t n,
                              int32_t periodic, int32_t parent_index, double efficiency,
                              int32_t min_width, ndgp_box *boxes, int32_t max_boxes,
                              int32_t *n_boxes, hipStream_t stream);
size_t ndgp_amr_workspace_bytes(const ndgp_grid *grid, const ndgp_params *params,
                                const ndgp_box *boxes, int32_t n_boxes);
ndgp_status ndgp_solve_amr(const ndgp_grid *grid, const ndgp_params *params,
                           const ndgp_box *boxes, int32_t n_boxes, const double *const *delta,
                           double *const *phi, void *workspace, size_t workspace_bytes,
                           hipStream_t stream, ndgp_report *report,
                           ndgp_box_report *box_report);

/*
 * Norms for comparing two fields, e.g. the force of the interpolated mode with
 * the fully relaxed one (the error of Sec. III.B, Eqs. errors-errors2):
 *   out[0] = sum (a - b)^2,  out[1] = sum a^2,  out[2] = sum b^2
 * over `count` doubles (b may be NULL: then it counts as zero).  out is a HOST
 * array; the workspace needs NDGP_DIFF_NORMS_WORKSPACE bytes.  Deterministic;
 * blocks until out is written.
 */
#define NDGP_DIFF_NORMS_WORKSPACE 131072
ndgp_status ndgp_diff_norms(const double *a, const double *b, size_t count, double out[3],
                            void *workspace, size_t workspace_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* NDGP_H */
