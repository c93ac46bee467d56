/*
 * ndgp_oracle.c -- CPU reference for the nDGP scalar-field solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke check
 * and the benchmark's CPU-baseline leg may load this library.  It shares no
 * code with the GPU library: the two are written separately from the paper
 * (Barreira, Bose & Li, arXiv:1511.08200) and meet only through the seeded
 * input arrays.
 *
 * Plain FP64, cell-by-cell, with the operator written out exactly as defined.
 * Everything is in physical units: lengths in c/H0, phi in units of c^2.
 *
 * What is computed (section / equation of the paper):
 *   - the nDGP scalar equation, Sec. II Eq. (eomvarphi), in the form
 *       lap(phi) + alpha [ (lap phi)^2 - (d_i d_j phi)^2 ] = S,
 *       alpha = r_c^2 / (3 beta a^2),   S = Omega_m delta / (a beta)   (H0 = c = 1);
 *   - beta(a) of Eq. (beta) with the LCDM expansion history of Sec. II;
 *   - the discrete residual T = L[phi] - S of Eq. (eomgen-disc) on a cell-
 *     centred grid, with the cross-derivative term in conservative corner-
 *     averaged form (the paper defers its discretisation to another work;
 *     this is the reading adopted here);
 *   - Newton-Raphson relaxation cell by cell, Eq. (newton), in a Gauss-Seidel
 *     sweep, accelerated by multigrid V-cycles (Sec. III.A) in full
 *     approximation storage form;
 *   - periodic domain level first, then refined patches with boundary values
 *     and initial guess interpolated from the coarser level (Sec. III.A), or,
 *     in the truncated mode of Sec. III.B, the interpolated guess kept as the
 *     answer;
 *   - the fifth force F = -grad(phi)/2 by central differences (Sec. III.B;
 *     Eq. (modpoisson) puts phi/2 in the dynamical potential).
 *
 * Array layout: every grid array handed to this library is either "natural"
 * (n^3 doubles, index (k*n + j)*n + i, x fastest) or "padded" ((n+2)^3
 * doubles: the n^3 interior plus a one-cell ghost shell, cell (i,j,k) for
 * i,j,k in [-1, n] at ((k+1)*(n+2) + (j+1))*(n+2) + (i+1)).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_LEVELS 12
#define ORACLE_NCOARSE 8
/* a run to stagnation counts as converged only below this relative residual */
#define ORACLE_STAGNATION_OK 1e-11
#ifndef NEWTON_ITERS
#define NEWTON_ITERS 30
#endif

/* ------------------------------------------------------------------------ */
/* indexing                                                                  */

static inline int64_t pidx(int n, int i, int j, int k)
{
    const int64_t p = (int64_t)n + 2;
    return ((int64_t)(k + 1) * p + (int64_t)(j + 1)) * p + (int64_t)(i + 1);
}

static inline int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

static double *alloc_padded(int n)
{
    const int64_t p = (int64_t)n + 2;
    double *a = (double *)calloc((size_t)(p * p * p), sizeof(double));
    return a;
}

/* Visit every ghost-shell cell of a padded n^3 box: whole rows where j or k
   is outside [0, n), else only i = -1 and i = n. */
#define FOR_SHELL(n, BODY)                                                     \
    for (int k = -1; k <= (n); ++k)                                            \
        for (int j = -1; j <= (n); ++j) {                                      \
            const int edge_row = (k < 0 || k >= (n) || j < 0 || j >= (n));     \
            for (int i = -1; i <= (n); i += (edge_row || i == (n)) ? 1 : (n) + 1) { \
                BODY;                                                          \
            }                                                                  \
        }

/* Copy interior values into the ghost shell so that the padded array
   represents a periodic field. */
static void fill_periodic(int n, double *a)
{
    FOR_SHELL(n, a[pidx(n, i, j, k)] = a[pidx(n, wrap(i, n), wrap(j, n), wrap(k, n))])
}

static void natural_to_padded(int n, const double *src, double *dst)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                dst[pidx(n, i, j, k)] = src[((int64_t)k * n + j) * n + i];
}

static void padded_to_natural(int n, const double *src, double *dst)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                dst[((int64_t)k * n + j) * n + i] = src[pidx(n, i, j, k)];
}

/* ------------------------------------------------------------------------ */
/* background and source: Sec. II, Eqs. (dgpH) ff. and (beta)                */

/* beta(a) = 1 + 2 H r_c (1 + Hdot / (3 H^2)), Eq. (beta).  The normal branch
   is tuned so that H(a) is the LCDM one (Sec. II): H^2 = Om a^-3 + 1 - Om and
   Hdot = dH/dt = -(3/2) Om a^-3 in units H0 = 1. */
double oracle_beta_lcdm(double a, double omega_m, double rc)
{
    const double H = sqrt(omega_m / (a * a * a) + 1.0 - omega_m);
    const double Hdot = -1.5 * omega_m / (a * a * a);
    return 1.0 + 2.0 * H * rc * (1.0 + Hdot / (3.0 * H * H));
}

/* Coefficient of the nonlinear term of Eq. (eomvarphi): r_c^2 / (3 beta a^2). */
double oracle_alpha(double rc, double beta, double a)
{
    return rc * rc / (3.0 * beta * a * a);
}

/* Right-hand side of Eq. (eomvarphi): 8 pi G a^2 delta rho_m / (3 beta).  With
   8 pi G rho_m0 = 3 Om H0^2 and comoving a^2 delta rho_m = rho_m0 delta / a this
   is Om delta / (a beta).  The mean of delta is removed first: the density
   perturbation delta rho = rho - mean(rho) averages to zero on the periodic
   domain, and only then can the periodic problem have a solution. */
void oracle_source(int64_t count, const double *delta, double omega_m, double a,
                   double beta, double *S, double *removed_mean)
{
    double sum = 0.0;
    for (int64_t c = 0; c < count; ++c) sum += delta[c];
    const double mean = count ? sum / (double)count : 0.0;
    const double f = omega_m / (a * beta);
    for (int64_t c = 0; c < count; ++c) S[c] = f * (delta[c] - mean);
    if (removed_mean) *removed_mean = mean;
}

/* Same scaling for a refined patch: the patch density contrast is measured
   against the same background as the domain, so the same mean is removed. */
void oracle_source_shift(int64_t count, const double *delta, double mean, double omega_m,
                         double a, double beta, double *S)
{
    const double f = omega_m / (a * beta);
    for (int64_t c = 0; c < count; ++c) S[c] = f * (delta[c] - mean);
}

/* ------------------------------------------------------------------------ */
/* discrete operator L_h[phi] at one cell (the residual of Eq. eomgen-disc    */
/* is L_h[phi] - S)                                                         */
/*
 *   D_aa = (phi[c+e_a] + phi[c-e_a] - 2 phi[c]) / h^2       second differences
 *   lap  = D_xx + D_yy + D_zz
 *   C_ab(s,t) = (phi[c+s e_a+t e_b] - phi[c+s e_a] - phi[c+t e_b] + phi[c]) / h^2
 *               mixed difference at the corner (s,t) of the a-b plane
 *   (lap phi)^2 - (d_i d_j phi)^2 = 2 sum_{a<b} (phi_aa phi_bb - phi_ab^2)
 *     is discretised as  2 sum_{a<b} ( D_aa D_bb - (1/4) sum_{s,t} C_ab(s,t)^2 )
 *   L_h[phi] = lap + alpha * that.
 *
 * Also returns dL/dphi[c], the derivative needed by the Newton step of
 * Eq. (newton): d D_aa/d phi[c] = -2/h^2 and d C/d phi[c] = +1/h^2.
 */
static double op_cell(const double *a, int n, int i, int j, int k, double h, double alpha,
                      double *dLdphi)
{
    const double ih2 = 1.0 / (h * h);
    const int64_t c = pidx(n, i, j, k);
    const int64_t e[3] = {1, (int64_t)n + 2, ((int64_t)n + 2) * ((int64_t)n + 2)};
    const double u = a[c];
    double D[3];
    for (int ax = 0; ax < 3; ++ax)
        D[ax] = (a[c + e[ax]] + a[c - e[ax]] - 2.0 * u) * ih2;
    const double lap = D[0] + D[1] + D[2];

    double cross_sq = 0.0; /* sum over pairs and corners of C^2 */
    double cross_sum = 0.0; /* sum over pairs and corners of C   */
    double prod = 0.0;     /* sum over pairs of D_aa D_bb       */
    for (int ax = 0; ax < 3; ++ax) {
        for (int bx = ax + 1; bx < 3; ++bx) {
            prod += D[ax] * D[bx];
            for (int s = -1; s <= 1; s += 2) {
                for (int t = -1; t <= 1; t += 2) {
                    const double C = (a[c + s * e[ax] + t * e[bx]] - a[c + s * e[ax]]
                                      - a[c + t * e[bx]] + u) * ih2;
                    cross_sq += C * C;
                    cross_sum += C;
                }
            }
        }
    }
    const double nonlin = 2.0 * (prod - 0.25 * cross_sq);
    if (dLdphi) {
        /* d/dphi[c]: lap -> -6/h^2; prod -> -(2/h^2) sum_{a<b}(D_aa + D_bb) = -(4/h^2) lap;
           cross_sq -> (2/h^2) sum C */
        const double dprod = -4.0 * lap * ih2;
        const double dcross = 2.0 * cross_sum * ih2;
        *dLdphi = -6.0 * ih2 + alpha * 2.0 * (dprod - 0.25 * dcross);
    }
    return lap + alpha * nonlin;
}

/* ------------------------------------------------------------------------ */
/* grids                                                                    */

typedef struct {
    int n;
    double h;
    double *phi;    /* padded */
    double *S;      /* padded (ghosts unused) */
    double *phihat; /* padded: restriction of the finer phi (FAS); NULL on the top level */
    double *work;   /* padded scratch */
    double *ghost;  /* padded: fixed boundary values (Dirichlet levels); NULL if periodic */
    const unsigned char *mask; /* natural n^3: 0 = cell held at its initial value
                                  (cell-wise truncation); NULL = every cell relaxed */
    unsigned char *mask_own;   /* coarse levels: the mask this level owns */
} level_t;

typedef struct {
    int nl;
    int periodic;
    double alpha;
    level_t lv[ORACLE_MAX_LEVELS];
} hier_t;

static void hier_free(hier_t *H)
{
    for (int l = 0; l < H->nl; ++l) {
        free(H->lv[l].phi);
        free(H->lv[l].S);
        free(H->lv[l].phihat);
        free(H->lv[l].work);
        free(H->lv[l].ghost);
        free(H->lv[l].mask_own);
    }
    H->nl = 0;
}

static int hier_alloc(hier_t *H, int n, double h, int periodic, double alpha)
{
    memset(H, 0, sizeof(*H));
    H->periodic = periodic;
    H->alpha = alpha;
    int nl = 0;
    int m = n;
    double hm = h;
    for (;;) {
        level_t *L = &H->lv[nl];
        L->n = m;
        L->h = hm;
        L->phi = alloc_padded(m);
        L->S = alloc_padded(m);
        L->work = alloc_padded(m);
        L->phihat = nl ? alloc_padded(m) : NULL;
        L->ghost = periodic ? NULL : alloc_padded(m);
        if (!L->phi || !L->S || !L->work || (nl && !L->phihat) || (!periodic && !L->ghost)) {
            H->nl = nl + 1;
            hier_free(H);
            return -1;
        }
        ++nl;
        if (m <= ORACLE_NCOARSE || (m & 1) || nl == ORACLE_MAX_LEVELS) break;
        m /= 2;
        hm *= 2.0;
    }
    H->nl = nl;
    return 0;
}

/* Put the level's boundary into a padded array: periodic copy, or the
   Dirichlet values held in L->ghost.
   On the coarse levels of a refinement's hierarchy the iterate differs from
   the restricted fine field R phi by a correction that must vanish where the
   fine boundary values sit, half a fine cell outside the patch, while the
   coarse ghost centres lie a fine cell and a half outside.  Extrapolating the
   correction linearly through zero at the fine ghost position gives the
   coarse ghost -1/3 of the correction of the interior cell next to it (a
   factor -1/3 per axis along which the ghost lies outside).  This only
   changes how fast the cycles converge, not the solution on the patch. */
static void apply_bc(const hier_t *H, const level_t *L, double *a)
{
    const int n = L->n;
    if (H->periodic) {
        fill_periodic(n, a);
        return;
    }
    if (L->phihat && a == L->phi) {
        FOR_SHELL(n, {
            const int ci = i < 0 ? 0 : (i >= n ? n - 1 : i);
            const int cj = j < 0 ? 0 : (j >= n ? n - 1 : j);
            const int ck = k < 0 ? 0 : (k >= n ? n - 1 : k);
            const int d = (ci != i) + (cj != j) + (ck != k);
            const double f = d == 1 ? -1.0 / 3.0 : (d == 2 ? 1.0 / 9.0 : -1.0 / 27.0);
            const int64_t q = pidx(n, ci, cj, ck);
            a[pidx(n, i, j, k)] = L->ghost[pidx(n, i, j, k)] + f * (a[q] - L->phihat[q]);
        })
        return;
    }
    FOR_SHELL(n, a[pidx(n, i, j, k)] = L->ghost[pidx(n, i, j, k)])
}

/* ------------------------------------------------------------------------ */
/* relaxation: Newton-Raphson per cell, Eq. (newton), Gauss-Seidel order     */
/* over 8 colours (parities of i, j, k).  No two cells of one colour touch    */
/* each other's 19-point stencil, so each colour may be updated in parallel  */
/* and the sweep is a true Gauss-Seidel sweep.                                */

static void newton_gs_sweep(const hier_t *H, level_t *L)
{
    const int n = L->n;
    for (int colour = 0; colour < 8; ++colour) {
        const int pi = colour & 1, pj = (colour >> 1) & 1, pk = (colour >> 2) & 1;
        apply_bc(H, L, L->phi);
#pragma omp parallel for schedule(static)
        for (int k = pk; k < n; k += 2)
            for (int j = pj; j < n; j += 2)
                for (int i = pi; i < n; i += 2) {
                    if (L->mask && !L->mask[((int64_t)k * n + j) * n + i]) continue;
                    /* Newton-Raphson on the cell's own equation, Eq. (newton),
                       repeated until the cell residual stops changing. */
                    const int64_t c = pidx(n, i, j, k);
                    for (int it = 0; it < NEWTON_ITERS; ++it) {
                        double dL;
                        const double Lc = op_cell(L->phi, n, i, j, k, L->h, H->alpha, &dL);
                        const double T = Lc - L->S[c];
                        /* The cell equation is a parabola in phi[c] (leading
                           coefficient 18 alpha / h^4).  dT/dphi >= 0 means the
                           value is past its vertex, on the branch where the
                           linearised operator is not elliptic: reflect it across
                           the vertex (same T, slope of the elliptic sign), from
                           where the Newton steps reach the elliptic root. */
                        if (!(dL < 0.0)) {
                            const double a2 = 18.0 * H->alpha / (L->h * L->h * L->h * L->h);
                            if (!(dL > 0.0) || !(a2 > 0.0)) break;
                            L->phi[c] -= dL / a2;
                            continue;
                        }
                        const double step = T / dL;
                        L->phi[c] -= step;
                        if (fabs(step) <= 1e-15 * fabs(L->phi[c])) break;
                    }
                }
    }
    apply_bc(H, L, L->phi);
}

/* r = S - L[phi] into L->work; returns sum r^2 (fixed order) */
static double residual(const hier_t *H, level_t *L)
{
    const int n = L->n;
    apply_bc(H, L, L->phi);
    double *part = (double *)calloc((size_t)n, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                /* a held cell is not part of the equations being solved */
                const int held = L->mask && !L->mask[((int64_t)k * n + j) * n + i];
                const double r = held ? 0.0
                                      : L->S[pidx(n, i, j, k)]
                                            - op_cell(L->phi, n, i, j, k, L->h, H->alpha, NULL);
                L->work[pidx(n, i, j, k)] = r;
                s += r * r;
            }
        part[k] = s;
    }
    double tot = 0.0;
    for (int k = 0; k < n; ++k) tot += part[k];
    free(part);
    return tot;
}

static double sum_sq_interior(int n, const double *a)
{
    double tot = 0.0;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const double v = a[pidx(n, i, j, k)];
                tot += v * v;
            }
    return tot;
}

/* ------------------------------------------------------------------------ */
/* multigrid transfers (Sec. III.A: coarsify, iterate, interpolate back)     */

/* coarse cell = mean of its 8 children */
static void restrict_avg(int nf, const double *fine, double *coarse)
{
    const int nc = nf / 2;
#pragma omp parallel for schedule(static)
    for (int K = 0; K < nc; ++K)
        for (int J = 0; J < nc; ++J)
            for (int I = 0; I < nc; ++I) {
                double s = 0.0;
                for (int dk = 0; dk < 2; ++dk)
                    for (int dj = 0; dj < 2; ++dj)
                        for (int di = 0; di < 2; ++di)
                            s += fine[pidx(nf, 2 * I + di, 2 * J + dj, 2 * K + dk)];
                coarse[pidx(nc, I, J, K)] = s / 8.0;
            }
}

/* fine += trilinear interpolation of the coarse correction.  A fine cell
   centre lies a quarter of a coarse cell from its parent's centre along each
   axis: weight 3/4 on the parent and 1/4 on the neighbour on its side. */
static void prolong_add(int nc, const double *corr, int nf, double *fine,
                        const unsigned char *mask)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nf; ++k)
        for (int j = 0; j < nf; ++j)
            for (int i = 0; i < nf; ++i) {
                if (mask && !mask[((int64_t)k * nf + j) * nf + i]) continue; /* held */
                const int I = i >> 1, J = j >> 1, K = k >> 1;
                const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
                double v = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int c = 0; c < 2; ++c) {
                            const double w = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (c ? 0.25 : 0.75);
                            v += w * corr[pidx(nc, I + a * si, J + b * sj, K + c * sk)];
                        }
                fine[pidx(nf, i, j, k)] += v;
            }
}

typedef struct {
    int nu1, nu2, coarse_sweeps_max;
    double coarse_reduction;
} mgopt_t;

static void vcycle(hier_t *H, int l, const mgopt_t *o)
{
    level_t *L = &H->lv[l];
    if (l == H->nl - 1) {
        /* coarsest level: relax until the residual has dropped enough */
        const double r0 = sqrt(residual(H, L));
        for (int s = 0; s < o->coarse_sweeps_max; ++s) {
            newton_gs_sweep(H, L);
            if ((s & 7) == 7 && sqrt(residual(H, L)) <= o->coarse_reduction * r0) break;
        }
        return;
    }
    for (int s = 0; s < o->nu1; ++s) newton_gs_sweep(H, L);

    level_t *C = &H->lv[l + 1];
    residual(H, L);                 /* r in L->work */
    restrict_avg(L->n, L->phi, C->phihat);
    restrict_avg(L->n, L->work, C->work);
    /* coarse source of the full-approximation scheme: S_c = L_c[R phi] + R r */
    apply_bc(H, C, C->phihat);
    const int nc = C->n;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nc; ++k)
        for (int j = 0; j < nc; ++j)
            for (int i = 0; i < nc; ++i)
                C->S[pidx(nc, i, j, k)] = op_cell(C->phihat, nc, i, j, k, C->h, H->alpha, NULL)
                                          + C->work[pidx(nc, i, j, k)];
    memcpy(C->phi, C->phihat, sizeof(double) * (size_t)((nc + 2) * (nc + 2)) * (size_t)(nc + 2));

    vcycle(H, l + 1, o);

    /* correction e = phi_c - R phi (zero on Dirichlet ghosts), interpolated back */
    apply_bc(H, C, C->phi);
    const int64_t pc = (int64_t)(nc + 2) * (nc + 2) * (nc + 2);
    for (int64_t q = 0; q < pc; ++q) C->work[q] = C->phi[q] - C->phihat[q];
    if (H->periodic) fill_periodic(nc, C->work);
    prolong_add(nc, C->work, L->n, L->phi, L->mask);
    apply_bc(H, L, L->phi);

    for (int s = 0; s < o->nu2; ++s) newton_gs_sweep(H, L);
}

/* fine = trilinear interpolation of the whole coarse field (same weights as
   prolong_add) */
static void prolong_full(const hier_t *H, level_t *C, level_t *F)
{
    apply_bc(H, C, C->phi);
    const int64_t pf = (int64_t)(F->n + 2) * (F->n + 2) * (F->n + 2);
    for (int64_t q = 0; q < pf; ++q) F->phi[q] = 0.0;
    prolong_add(C->n, C->phi, F->n, F->phi, NULL);
    apply_bc(H, F, F->phi);
}

/* Initial guess by nested iteration: the source is averaged down to the
   coarsest level, solved there, and each solution interpolated to the next
   finer level and improved by `cycles` V-cycles there.  This is the paper's
   way of starting a refinement (initial guess interpolated from the coarser
   solution, Sec. III.A) applied to the levels of the multigrid hierarchy; a
   zero initial guess on the domain level diverges for strongly screened
   sources. */
static void nested_start(hier_t *H, const mgopt_t *o, int cycles)
{
    for (int l = 1; l < H->nl; ++l) restrict_avg(H->lv[l - 1].n, H->lv[l - 1].S, H->lv[l].S);
    level_t *Cst = &H->lv[H->nl - 1];
    memset(Cst->phi, 0, sizeof(double) * (size_t)((Cst->n + 2) * (Cst->n + 2)) * (size_t)(Cst->n + 2));
    vcycle(H, H->nl - 1, o);
    for (int l = H->nl - 2; l >= 0; --l) {
        prolong_full(H, &H->lv[l + 1], &H->lv[l]);
        if (l > 0)
            for (int c = 0; c < cycles; ++c) vcycle(H, l, o);
    }
}

/* Drive V-cycles on the top level until ||S - L phi|| / ||S|| <= tol.  With
   tol <= 0 the cycles continue until the residual stops falling (ratio above
   0.7 twice in a row), i.e. to rounding-level stagnation. */
static int drive(hier_t *H, const mgopt_t *o, int max_cycles, double tol, double *hist,
                 int hist_len, int *cycles_out, double *relres_out)
{
    level_t *L = &H->lv[0];
    const double snorm = sqrt(sum_sq_interior(L->n, L->S));
    double prev = sqrt(residual(H, L)) / snorm;
    int slow = 0, cyc = 0;
    double rel = prev;
    while (cyc < max_cycles) {
        if (tol > 0 && rel <= tol) break;
        if (rel == 0.0) break; /* exact, e.g. every cell held */
        vcycle(H, 0, o);
        ++cyc;
        rel = sqrt(residual(H, L)) / snorm;
        if (hist && cyc - 1 < hist_len) hist[cyc - 1] = rel;
        if (!isfinite(rel)) break;
        if (tol <= 0) {
            slow = (rel > 0.7 * prev) ? slow + 1 : 0;
            if (slow >= 2) break;
        }
        prev = rel;
    }
    if (cycles_out) *cycles_out = cyc;
    if (relres_out) *relres_out = rel;
    if (!isfinite(rel)) return -3;
    if (tol > 0 && rel > tol) return -3;
    if (tol <= 0 && rel > ORACLE_STAGNATION_OK) return -3;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* public: operator and residual                                            */

/* L_h[phi] over the interior of a padded field whose ghost shell the caller
   filled (or, with periodic != 0, that is filled here by periodic copy). */
void oracle_operator(int n, int periodic, double h, double alpha, double *phi_pad, double *out)
{
    if (periodic) fill_periodic(n, phi_pad);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i)
                out[((int64_t)k * n + j) * n + i] = op_cell(phi_pad, n, i, j, k, h, alpha, NULL);
}

/* L_h[phi] at listed cells of a periodic natural-layout field. */
void oracle_operator_at(int n, double h, double alpha, const double *phi, int64_t count,
                        const int32_t *cells /* count x (i,j,k) */, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < count; ++q) {
        /* the 3x3x3 neighbourhood is a padded box of one interior cell */
        double loc[27];
        const int ci = cells[3 * q], cj = cells[3 * q + 1], ck = cells[3 * q + 2];
        for (int dk = -1; dk <= 1; ++dk)
            for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di)
                    loc[((dk + 1) * 3 + (dj + 1)) * 3 + (di + 1)] =
                        phi[((int64_t)wrap(ck + dk, n) * n + wrap(cj + dj, n)) * n + wrap(ci + di, n)];
        out[q] = op_cell(loc, 1, 0, 0, 0, h, alpha, NULL);
    }
}

/* Newton step of Eq. (newton) at one cell of a padded field: returns the
   updated value phi[c] - T / (dT/dphi[c]). */
double oracle_newton_update(int n, double h, double alpha, const double *phi_pad, double S,
                            int i, int j, int k)
{
    double dL;
    const double Lc = op_cell(phi_pad, n, i, j, k, h, alpha, &dL);
    return phi_pad[pidx(n, i, j, k)] - (Lc - S) / dL;
}

/* ------------------------------------------------------------------------ */
/* public: interpolation from a coarser level (Sec. III.A / III.B)           */

/* Value of a parent field at the continuous coordinate x (per axis, in parent
   cell units with parent cell c's centre at c) by trilinear interpolation
   between the eight surrounding parent cell centres.  A periodic parent wraps;
   a non-periodic one is read from its padded array (indices -1..n). */
static int parent_value(const double *parent, int np, int periodic, const double x[3],
                        double *out)
{
    int i0[3];
    double w[3];
    for (int a = 0; a < 3; ++a) {
        const double f = floor(x[a]);
        i0[a] = (int)f;
        w[a] = x[a] - f;
        if (!periodic && (i0[a] < -1 || i0[a] + 1 > np)) return -1;
    }
    double v = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const double wt = (a ? w[0] : 1.0 - w[0]) * (b ? w[1] : 1.0 - w[1])
                                  * (c ? w[2] : 1.0 - w[2]);
                int ii = i0[0] + a, jj = i0[1] + b, kk = i0[2] + c;
                double pv;
                if (periodic)
                    pv = parent[((int64_t)wrap(kk, np) * np + wrap(jj, np)) * np + wrap(ii, np)];
                else
                    pv = parent[pidx(np, ii, jj, kk)];
                v += wt * pv;
            }
    *out = v;
    return 0;
}

/*
 * Fill a child box from its parent.  The child box has nc^3 cells, its lower
 * corner at integer parent cell `origin`, and cells of size 2^m / 2 parent
 * cells (m = 0: the refined patch itself, twice as fine as the parent).  The
 * parent is periodic natural (np^3) or padded non-periodic ((np+2)^3).
 * Fills the padded child: interior and ghost shell (ghosts_only = 0) or the
 * ghost shell only.  Returns -1 if a needed parent cell lies outside the parent.
 */
int oracle_interpolate(const double *parent, int np, int parent_periodic, const int origin[3],
                       int m, int nc, double *child_pad, int ghosts_only)
{
    const double q = ldexp(1.0, m - 1); /* child cell size in parent cells */
    int bad = 0;
    for (int k = -1; k <= nc; ++k)
        for (int j = -1; j <= nc; ++j)
            for (int i = -1; i <= nc; ++i) {
                const int interior = (i >= 0 && i < nc && j >= 0 && j < nc && k >= 0 && k < nc);
                if (ghosts_only && interior) continue;
                const int ijk[3] = {i, j, k};
                double x[3];
                for (int a = 0; a < 3; ++a) x[a] = origin[a] + (ijk[a] + 0.5) * q - 0.5;
                double v;
                if (parent_value(parent, np, parent_periodic, x, &v)) {
                    bad = 1;
                    continue;
                }
                child_pad[pidx(nc, i, j, k)] = v;
            }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* public: solves                                                           */

/* Periodic domain level (Sec. III.A).  S natural n^3 (zero mean), phi natural
   n^3: solution out, shifted to zero mean; with warm_start != 0 phi also
   holds the initial guess (the paper allows the previous time step's field),
   otherwise the guess comes from nested iteration (only derivatives
   of phi enter the equation, so the constant is free).  Returns 0, or -3 if
   tol > 0 was not reached, -2 on allocation failure. */
int oracle_solve_periodic(int n, double h, double alpha, const double *S, double *phi,
                          int warm_start, int max_cycles, double tol, int nu1, int nu2,
                          double *hist, int hist_len, int *cycles_out, double *relres_out)
{
    const int64_t cells = (int64_t)n * n * n;
    double snorm = 0.0;
    for (int64_t c = 0; c < cells; ++c) snorm += S[c] * S[c];
    if (snorm == 0.0) { /* no source: phi = 0 */
        memset(phi, 0, sizeof(double) * (size_t)cells);
        if (cycles_out) *cycles_out = 0;
        if (relres_out) *relres_out = 0.0;
        return 0;
    }
    hier_t H;
    if (hier_alloc(&H, n, h, 1, alpha)) return -2;
    natural_to_padded(n, S, H.lv[0].S);
    mgopt_t o = {nu1, nu2, 400, 1e-6};
    if (warm_start)
        natural_to_padded(n, phi, H.lv[0].phi);
    else
        nested_start(&H, &o, 1);
    const int rc = drive(&H, &o, max_cycles, tol, hist, hist_len, cycles_out, relres_out);
    padded_to_natural(n, H.lv[0].phi, phi);
    double mean = 0.0;
    for (int64_t c = 0; c < cells; ++c) mean += phi[c];
    mean /= (double)cells;
    for (int64_t c = 0; c < cells; ++c) phi[c] -= mean;
    hier_free(&H);
    return rc;
}

/*
 * Refined patch (Sec. III.A): nc^3 cells of size h_c, S natural nc^3, the
 * parent field (periodic natural np^3, or padded (np+2)^3) that supplies the
 * fixed boundary values and the initial guess by interpolation.  phi_pad
 * ((nc+2)^3) receives the solution with its ghost shell.  interp_only != 0 is
 * the truncated mode of Sec. III.B: the interpolated guess is the answer.
 */
int oracle_solve_patch(int nc, double hc, double alpha, const double *S, const double *parent,
                       int np, int parent_periodic, const int origin[3], double *phi_pad,
                       int max_cycles, double tol, int nu1, int nu2, int interp_only,
                       const unsigned char *mask,
                       double *hist, int hist_len, int *cycles_out, double *relres_out)
{
    if (oracle_interpolate(parent, np, parent_periodic, origin, 0, nc, phi_pad, 0)) return -1;
    if (interp_only) {
        if (cycles_out) *cycles_out = 0;
        if (relres_out) *relres_out = -1.0;
        return 0;
    }
    hier_t H;
    if (hier_alloc(&H, nc, hc, 0, alpha)) return -2;
    /* boundary values of every multigrid level: the parent interpolated at
       that level's ghost-cell centres (the finest of them equal phi_pad's). */
    for (int l = 0; l < H.nl; ++l) {
        if (oracle_interpolate(parent, np, parent_periodic, origin, l, H.lv[l].n, H.lv[l].ghost, 1)) {
            hier_free(&H);
            return -1;
        }
    }
    const int64_t pc = (int64_t)(nc + 2) * (nc + 2) * (nc + 2);
    memcpy(H.lv[0].phi, phi_pad, sizeof(double) * (size_t)pc);
    natural_to_padded(nc, S, H.lv[0].S);
    H.lv[0].mask = mask;
    /* coarse levels hold a cell if any of its eight children is held: the
       coarse correction is then zero wherever it would reach a held fine cell,
       so the held regions act as fixed boundaries on every level of the cycle.
       (Iterating a coarse cell with any iterated child instead lets corrections
       that do not vanish at the held cells leak into their iterated neighbours:
       the cycles then stagnate near 1e-4 on screened patches, and diverge with
       no coarse masks at all.) */
    for (int l = 1; mask && l < H.nl; ++l) {
        const int n = H.lv[l].n, nf = H.lv[l - 1].n;
        const unsigned char *mf = H.lv[l - 1].mask;
        unsigned char *mc = (unsigned char *)malloc((size_t)n * n * n);
        if (!mc) {
            hier_free(&H);
            return -2;
        }
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int all = 1;
                    for (int c = 0; c < 8; ++c)
                        all &= mf[((int64_t)(2 * k + (c >> 2)) * nf + 2 * j + ((c >> 1) & 1)) * nf
                                  + 2 * i + (c & 1)] != 0;
                    mc[((int64_t)k * n + j) * n + i] = (unsigned char)all;
                }
        H.lv[l].mask_own = mc;
        H.lv[l].mask = mc;
    }
    mgopt_t o = {nu1, nu2, 400, 1e-6};
    double snorm = sum_sq_interior(nc, H.lv[0].S);
    int rc = 0;
    if (snorm > 0.0) {
        rc = drive(&H, &o, max_cycles, tol, hist, hist_len, cycles_out, relres_out);
    } else {
        /* S = 0 on the patch: relax until the residual stops falling in
           absolute terms (the boundary values still drive the field) */
        for (int c = 0; c < max_cycles; ++c) vcycle(&H, 0, &o);
        if (cycles_out) *cycles_out = max_cycles;
        if (relres_out) *relres_out = sqrt(residual(&H, &H.lv[0]));
    }
    memcpy(phi_pad, H.lv[0].phi, sizeof(double) * (size_t)pc);
    hier_free(&H);
    return rc;
}

/*
 * Cell-wise truncation, the generalisation Sec. III.C proposes: a cell of a
 * refinement is iterated only if the fifth force on its parent cell is still
 * large, |F_5th| >= threshold |F_GR|, with F_5th = -grad(phi)/2 and
 * F_GR = -grad(Psi_N) by central differences on the parent level.  Written
 * without roots or divisions (the spacing cancels):
 *     sum_a (phi[P+e_a] - phi[P-e_a])^2  >=  (2 threshold)^2 sum_a (psi[P+e_a] - psi[P-e_a])^2
 * The child box (nc^3, ratio 2, lower corner `origin` in parent cells) lies
 * inside the parent; child cell i has parent cell origin + floor(i/2).  Parent
 * arrays are periodic natural (np^3) or padded ((np+2)^3).  mask is natural
 * nc^3: 1 = iterate, 0 = hold the interpolated value.  Returns -1 if a needed
 * parent cell is outside the parent.
 */
int oracle_cell_mask(const double *phi_parent, const double *psi_parent, int np,
                     int parent_periodic, const int origin[3], int nc, double threshold,
                     unsigned char *mask)
{
    const double t2 = (2.0 * threshold) * (2.0 * threshold);
    for (int k = 0; k < nc; ++k)
        for (int j = 0; j < nc; ++j)
            for (int i = 0; i < nc; ++i) {
                const int P[3] = {origin[0] + i / 2, origin[1] + j / 2, origin[2] + k / 2};
                double gphi = 0.0, gpsi = 0.0;
                for (int a = 0; a < 3; ++a) {
                    int up[3] = {P[0], P[1], P[2]}, dn[3] = {P[0], P[1], P[2]};
                    up[a] += 1;
                    dn[a] -= 1;
                    int64_t qu, qd;
                    if (parent_periodic) {
                        qu = ((int64_t)wrap(up[2], np) * np + wrap(up[1], np)) * np + wrap(up[0], np);
                        qd = ((int64_t)wrap(dn[2], np) * np + wrap(dn[1], np)) * np + wrap(dn[0], np);
                    } else {
                        for (int b = 0; b < 3; ++b)
                            if (up[b] > np || dn[b] < -1) return -1;
                        qu = pidx(np, up[0], up[1], up[2]);
                        qd = pidx(np, dn[0], dn[1], dn[2]);
                    }
                    const double dp = phi_parent[qu] - phi_parent[qd];
                    const double ds = psi_parent[qu] - psi_parent[qd];
                    gphi += dp * dp;
                    gpsi += ds * ds;
                }
                mask[((int64_t)k * nc + j) * nc + i] = gphi >= t2 * gpsi ? 1 : 0;
            }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* public: fifth force, Sec. III.B: F = -grad(phi) / 2 by central differences */

void oracle_force(int n, double h, double *phi_pad, int periodic, double *f /* 3 x n^3 */)
{
    if (periodic) fill_periodic(n, phi_pad);
    const int64_t cells = (int64_t)n * n * n;
    const int64_t e[3] = {1, (int64_t)n + 2, ((int64_t)n + 2) * ((int64_t)n + 2)};
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const int64_t c = pidx(n, i, j, k);
                const int64_t o = ((int64_t)k * n + j) * n + i;
                for (int a = 0; a < 3; ++a)
                    f[a * cells + o] = -0.5 * (phi_pad[c + e[a]] - phi_pad[c - e[a]]) / (2.0 * h);
            }
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
