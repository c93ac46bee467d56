// ndgp_kernels.hip -- HIP kernels for gfx950 (CDNA4) of the nDGP multigrid solve.
//
// Every kernel works in cell units (spacing 1 on its level): alpha is
// alpha_phys / h^2 and the source is h^2 S_phys, so the same code serves all
// levels.  Equation: Sec. II Eq. (eomvarphi) of arXiv:1511.08200; residual:
// Eq. (eomgen-disc); relaxation: per-cell root of the cell's own equation, the
// fixed point of the Newton iteration of Eq. (newton); multigrid transfers:
// Sec. III.A; interpolation of refinements: Sec. III.A/III.B; force: Sec. III.B.
//
// Memory is HBM-bound everywhere (a few flops per byte, no dense contraction),
// so nothing here uses MFMA.  Reductions are deterministic: a fixed grid of
// kReduceBlocks blocks, a fixed per-thread order, in-wave xor-shuffle trees
// and a fixed combination across waves.

#include "ndgp_internal.h"

namespace ndgp {
namespace {

// ------------------------------------------------------------------------
// indexing: periodic levels are natural n^3 with wrap-around (n a power of
// two, so wrap is a mask); Dirichlet levels are padded (n+2)^3.

template <bool PER>
struct Ix {
    int n, lg, p;
    __device__ __forceinline__ int operator()(int i, int j, int k) const {
        if constexpr (PER) {
            const int m = n - 1;
            return ((((k & m) << lg) | (j & m)) << lg) | (i & m);
        } else {
            return ((k + 1) * p + (j + 1)) * p + (i + 1);
        }
    }
};

template <bool PER>
inline Ix<PER> make_ix(int n, int lg) {
    return Ix<PER>{n, lg, n + 2};
}

inline int log2i(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

inline unsigned blocks_for(size_t total) {
    return (unsigned)((total + kBlock - 1) / kBlock);
}

// ------------------------------------------------------------------------
// the 19-point stencil
//
// v[0] centre; v[1..6] faces x+ x- y+ y- z+ z-; v[7..18] edges, by plane and
// corner (s,t) in the order ++ +- -+ --: xy (7-10), xz (11-14), yz (15-18).

template <bool PER>
__device__ __forceinline__ void gather(const double *__restrict__ a, const Ix<PER> &ix, int i,
                                       int j, int k, double v[19]) {
    v[0] = a[ix(i, j, k)];
    v[1] = a[ix(i + 1, j, k)];
    v[2] = a[ix(i - 1, j, k)];
    v[3] = a[ix(i, j + 1, k)];
    v[4] = a[ix(i, j - 1, k)];
    v[5] = a[ix(i, j, k + 1)];
    v[6] = a[ix(i, j, k - 1)];
    v[7] = a[ix(i + 1, j + 1, k)];
    v[8] = a[ix(i + 1, j - 1, k)];
    v[9] = a[ix(i - 1, j + 1, k)];
    v[10] = a[ix(i - 1, j - 1, k)];
    v[11] = a[ix(i + 1, j, k + 1)];
    v[12] = a[ix(i + 1, j, k - 1)];
    v[13] = a[ix(i - 1, j, k + 1)];
    v[14] = a[ix(i - 1, j, k - 1)];
    v[15] = a[ix(i, j + 1, k + 1)];
    v[16] = a[ix(i, j + 1, k - 1)];
    v[17] = a[ix(i, j - 1, k + 1)];
    v[18] = a[ix(i, j - 1, k - 1)];
}

// Pieces of the discrete operator at one cell (spacing 1):
//   lap = D_xx + D_yy + D_zz, D_aa = second difference along a;
//   nl  = sum_{a<b} D_aa D_bb - (1/4) sum over the 12 corner mixed
//         differences C^2, C = phi[c+s e_a+t e_b] - phi[c+s e_a] - phi[c+t e_b] + phi[c];
//   see = sum over the 12 edge neighbours of (phi_edge - phi[c]).
// L[phi] = lap + 2 alpha nl.
struct Terms {
    double lap, nl, see;
};

__device__ __forceinline__ Terms stencil_terms(const double v[19]) {
    const double u = v[0];
    const double dxp = v[1] - u, dxm = v[2] - u;
    const double dyp = v[3] - u, dym = v[4] - u;
    const double dzp = v[5] - u, dzm = v[6] - u;
    const double Dxx = dxp + dxm, Dyy = dyp + dym, Dzz = dzp + dzm;
    double e, c, c2, see;
    e = v[7] - u;  see = e;  c = e - dxp - dyp; c2 = c * c;
    e = v[8] - u;  see += e; c = e - dxp - dym; c2 = fma(c, c, c2);
    e = v[9] - u;  see += e; c = e - dxm - dyp; c2 = fma(c, c, c2);
    e = v[10] - u; see += e; c = e - dxm - dym; c2 = fma(c, c, c2);
    e = v[11] - u; see += e; c = e - dxp - dzp; c2 = fma(c, c, c2);
    e = v[12] - u; see += e; c = e - dxp - dzm; c2 = fma(c, c, c2);
    e = v[13] - u; see += e; c = e - dxm - dzp; c2 = fma(c, c, c2);
    e = v[14] - u; see += e; c = e - dxm - dzm; c2 = fma(c, c, c2);
    e = v[15] - u; see += e; c = e - dyp - dzp; c2 = fma(c, c, c2);
    e = v[16] - u; see += e; c = e - dyp - dzm; c2 = fma(c, c, c2);
    e = v[17] - u; see += e; c = e - dym - dzp; c2 = fma(c, c, c2);
    e = v[18] - u; see += e; c = e - dym - dzm; c2 = fma(c, c, c2);
    Terms t;
    t.lap = (Dxx + Dyy) + Dzz;
    t.nl = fma(Dxx, Dyy, fma(Dxx, Dzz, Dyy * Dzz)) - 0.25 * c2;
    t.see = see;
    return t;
}

__device__ __forceinline__ double apply_L(const Terms &t, double al) {
    return fma(2.0 * al, t.nl, t.lap);
}

// New value of the centre cell: the root of its own equation T(u') = 0 that is
// continuous with the linear case.  Moving u by du shifts every D_aa by -2 du
// and every corner difference by +du, so with dt = 2 du
//     T(dt) = r - B dt + (9/2) alpha dt^2,   r = L - s,
//     B = 3 + 4 alpha lap + 2 alpha M,  M = (1/4) sum C = see/4 - lap,
// and the root is dt = 2 r / (B + sqrt(B^2 - 18 alpha r)) (no cancellation).
// B <= 0: the linearised operator is not elliptic at this cell; it waits for
// its neighbours.  No real root: move to the vertex dt = B / (9 alpha).
__device__ __forceinline__ double relax_cell(const double v[19], double s, double al,
                                             unsigned &fallbacks) {
    const Terms t = stencil_terms(v);
    const double r = apply_L(t, al) - s;
    const double B = fma(al, fma(2.0, t.lap, 0.5 * t.see), 3.0);
    if (!(B > 0.0)) return v[0];
    const double D = fma(B, B, -18.0 * al * r);
    if (D < 0.0) {
        ++fallbacks;
        return v[0] + B / (18.0 * al);
    }
    return v[0] + r / (B + sqrt(D));
}

// ------------------------------------------------------------------------
// deterministic block sum (kBlock = 256 threads = 4 waves of 64)

__device__ __forceinline__ double block_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __shared__ double wsum[kBlock / 64];
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
    return r;
}

// ------------------------------------------------------------------------
// kernels

template <bool PER>
__global__ void __launch_bounds__(kBlock)
k_smooth_half(const double *__restrict__ pin, double *__restrict__ pout,
              const double *__restrict__ s, Ix<PER> ix, double al, int colour,
              unsigned *__restrict__ fallbacks) {
    const int n = ix.n, lg = ix.lg;
    const int half = n >> 1;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= (half << (2 * lg))) return;
    const int m = t & (half - 1);
    const int row = t >> (lg - 1);
    const int j = row & (n - 1);
    const int k = row >> lg;
    const int off = (colour ^ j ^ k) & 1; // parity of i of the cell of this colour
    const int iu = 2 * m + off;
    const int ic = 2 * m + 1 - off;
    double v[19];
    gather(pin, ix, iu, j, k, v);
    unsigned fb = 0;
    const double un = relax_cell(v, s[((k << lg) + j) * n + iu], al, fb);
    pout[ix(iu, j, k)] = un;
    pout[ix(ic, j, k)] = pin[ix(ic, j, k)];
    if (fb) atomicAdd(fallbacks, fb);
}

template <bool PER>
__global__ void __launch_bounds__(kBlock)
k_residual_sumsq(const double *__restrict__ phi, const double *__restrict__ s, Ix<PER> ix,
                 double al, double *__restrict__ partials, double *__restrict__ r_out,
                 double r_scale) {
    const int n = ix.n, lg = ix.lg;
    const int total = 1 << (3 * lg);
    double acc = 0.0;
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < total; c += gridDim.x * kBlock) {
        const int i = c & (n - 1), j = (c >> lg) & (n - 1), k = c >> (2 * lg);
        double v[19];
        gather(phi, ix, i, j, k, v);
        const double r = s[c] - apply_L(stencil_terms(v), al);
        acc = fma(r, r, acc);
        if (r_out) r_out[c] = r * r_scale;
    }
    const double b = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

__global__ void __launch_bounds__(kBlock)
k_partial_sums(const double *__restrict__ a, size_t count, int squares,
               double *__restrict__ partials) {
    double acc = 0.0;
    for (size_t c = (size_t)blockIdx.x * kBlock + threadIdx.x; c < count;
         c += (size_t)gridDim.x * kBlock) {
        const double x = a[c];
        acc = squares ? fma(x, x, acc) : acc + x;
    }
    const double b = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

__global__ void __launch_bounds__(kBlock)
k_diff_partials(const double *__restrict__ a, const double *__restrict__ b, size_t count,
                double *__restrict__ partials) {
    double dd = 0.0, aa = 0.0, bb = 0.0;
    for (size_t c = (size_t)blockIdx.x * kBlock + threadIdx.x; c < count;
         c += (size_t)gridDim.x * kBlock) {
        const double x = a[c];
        const double y = b ? b[c] : 0.0;
        dd = fma(x - y, x - y, dd);
        aa = fma(x, x, aa);
        bb = fma(y, y, bb);
    }
    const double s0 = block_sum(dd);
    __syncthreads();
    const double s1 = block_sum(aa);
    __syncthreads();
    const double s2 = block_sum(bb);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = s0;
        partials[kReduceBlocks + blockIdx.x] = s1;
        partials[2 * kReduceBlocks + blockIdx.x] = s2;
    }
}

__global__ void __launch_bounds__(kBlock)
k_reduce_final(const double *__restrict__ partials, double *__restrict__ out) {
    double acc = 0.0;
    for (int q = threadIdx.x; q < kReduceBlocks; q += kBlock) acc += partials[q];
    const double b = block_sum(acc);
    if (threadIdx.x == 0) out[0] = b;
}

// FAS restriction fused with the residual: one thread per coarse cell holds
// the 4x4x4 block of fine values around its 8 children (the 8 block corners
// are never part of a child's 19-point stencil and are not loaded).
template <bool PER>
__global__ void __launch_bounds__(kBlock)
k_restrict_residual(const double *__restrict__ phi_f, const double *__restrict__ s_f,
                    Ix<PER> ixf, double al_f, double *__restrict__ hat_c,
                    double *__restrict__ s_c, Ix<PER> ixc) {
    const int nc = ixc.n, lgc = ixc.lg, nf = ixf.n;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= (1 << (3 * lgc))) return;
    const int I = t & (nc - 1), J = (t >> lgc) & (nc - 1), K = t >> (2 * lgc);
    const int i0 = 2 * I - 1, j0 = 2 * J - 1, k0 = 2 * K - 1;
    double b[4][4][4];
#pragma unroll
    for (int dk = 0; dk < 4; ++dk)
#pragma unroll
        for (int dj = 0; dj < 4; ++dj)
#pragma unroll
            for (int di = 0; di < 4; ++di) {
                const bool corner = (dk == 0 || dk == 3) && (dj == 0 || dj == 3) && (di == 0 || di == 3);
                b[dk][dj][di] = corner ? 0.0 : phi_f[ixf(i0 + di, j0 + dj, k0 + dk)];
            }
    double sphi = 0.0, sr = 0.0;
#pragma unroll
    for (int ck = 0; ck < 2; ++ck)
#pragma unroll
        for (int cj = 0; cj < 2; ++cj)
#pragma unroll
            for (int ci = 0; ci < 2; ++ci) {
                const int x = 1 + ci, y = 1 + cj, z = 1 + ck;
                const double v[19] = {
                    b[z][y][x],
                    b[z][y][x + 1], b[z][y][x - 1], b[z][y + 1][x], b[z][y - 1][x],
                    b[z + 1][y][x], b[z - 1][y][x],
                    b[z][y + 1][x + 1], b[z][y - 1][x + 1], b[z][y + 1][x - 1], b[z][y - 1][x - 1],
                    b[z + 1][y][x + 1], b[z - 1][y][x + 1], b[z + 1][y][x - 1], b[z - 1][y][x - 1],
                    b[z + 1][y + 1][x], b[z - 1][y + 1][x], b[z + 1][y - 1][x], b[z - 1][y - 1][x]};
                const int fi = 2 * I + ci, fj = 2 * J + cj, fk = 2 * K + ck;
                const double r = s_f[((size_t)fk * nf + fj) * nf + fi] - apply_L(stencil_terms(v), al_f);
                sphi += v[0];
                sr += r;
            }
    hat_c[ixc(I, J, K)] = sphi * 0.125;
    s_c[t] = sr * 0.5; // 4 * mean: the coarse cell is twice as wide
}

template <bool PER>
__global__ void __launch_bounds__(kBlock)
k_coarse_source(const double *__restrict__ hat, double *__restrict__ phi,
                double *__restrict__ s, Ix<PER> ix, double al) {
    const int n = ix.n, lg = ix.lg;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= (1 << (3 * lg))) return;
    const int i = t & (n - 1), j = (t >> lg) & (n - 1), k = t >> (2 * lg);
    double v[19];
    gather(hat, ix, i, j, k, v);
    s[t] = apply_L(stencil_terms(v), al) + s[t];
    phi[ix(i, j, k)] = v[0];
}

// Trilinear cell-centred transfer: a fine cell centre sits a quarter coarse
// cell from its parent's centre on every axis, so the parent weighs 3/4 and
// the neighbour on the fine cell's side 1/4 per axis (27/64 ... 1/64).
template <bool PER, bool CORRECT>
__global__ void __launch_bounds__(kBlock)
k_prolong(double *__restrict__ phi_f, Ix<PER> ixf, const double *__restrict__ phi_c,
          const double *__restrict__ hat_c, Ix<PER> ixc) {
    const int n = ixf.n, lg = ixf.lg;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= (1 << (3 * lg))) return;
    const int i = t & (n - 1), j = (t >> lg) & (n - 1), k = t >> (2 * lg);
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const double w = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (c ? 0.25 : 0.75);
                const int q = ixc(I + a * si, J + b * sj, K + c * sk);
                const double val = CORRECT ? phi_c[q] - hat_c[q] : phi_c[q];
                acc = fma(w, val, acc);
            }
    if (CORRECT)
        phi_f[ixf(i, j, k)] += acc;
    else
        phi_f[ixf(i, j, k)] = acc;
}

__global__ void __launch_bounds__(kBlock)
k_restrict_source(const double *__restrict__ s_f, int nf, double *__restrict__ s_c, int lgc) {
    const int nc = 1 << lgc;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= (1 << (3 * lgc))) return;
    const int I = t & (nc - 1), J = (t >> lgc) & (nc - 1), K = t >> (2 * lgc);
    double acc = 0.0;
#pragma unroll
    for (int dk = 0; dk < 2; ++dk)
#pragma unroll
        for (int dj = 0; dj < 2; ++dj)
#pragma unroll
            for (int di = 0; di < 2; ++di)
                acc += s_f[((size_t)(2 * K + dk) * nf + (2 * J + dj)) * nf + (2 * I + di)];
    s_c[t] = acc * 0.5;
}

// Coarsest level (<= 8^3 cells): one workgroup, both colours in LDS,
// ping-ponging between two buffers so that every half sweep reads the
// values of its start (same semantics as k_smooth_half).
template <bool PER>
__global__ void __launch_bounds__(512)
k_coarsest(double *__restrict__ phi, const double *__restrict__ s, Ix<PER> ix, double al,
           int sweeps, unsigned *__restrict__ fallbacks) {
    __shared__ double A[(kCoarsestMax + 2) * (kCoarsestMax + 2) * (kCoarsestMax + 2)];
    __shared__ double B[(kCoarsestMax + 2) * (kCoarsestMax + 2) * (kCoarsestMax + 2)];
    const int n = ix.n, lg = ix.lg;
    const int cells = 1 << (3 * lg);
    const int slots = PER ? cells : (n + 2) * (n + 2) * (n + 2);
    for (int q = threadIdx.x; q < slots; q += blockDim.x) {
        const double x = phi[q];
        A[q] = x;
        B[q] = x;
    }
    __syncthreads();
    const int t = threadIdx.x;
    const bool active = t < cells;
    int i = 0, j = 0, k = 0;
    double sc = 0.0;
    if (active) {
        i = t & (n - 1);
        j = (t >> lg) & (n - 1);
        k = t >> (2 * lg);
        sc = s[t];
    }
    const int mycol = (i + j + k) & 1;
    unsigned fb = 0;
    for (int sw = 0; sw < sweeps; ++sw) {
#pragma unroll
        for (int col = 0; col < 2; ++col) {
            const double *src = col ? B : A;
            double *dst = col ? A : B;
            if (active) {
                const int me = ix(i, j, k);
                double val;
                if (mycol == col) {
                    double v[19];
                    gather(src, ix, i, j, k, v);
                    val = relax_cell(v, sc, al, fb);
                } else {
                    val = src[me];
                }
                dst[me] = val;
            }
            __syncthreads();
        }
    }
    if (active) phi[ix(i, j, k)] = A[ix(i, j, k)];
    if (fb) atomicAdd(fallbacks, fb);
}

__global__ void __launch_bounds__(kBlock)
k_source(const double *__restrict__ delta, size_t count, const double *__restrict__ sum,
         double inv_count_mean, double f, double *__restrict__ s) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= count) return;
    const double mean = sum[0] * inv_count_mean;
    s[t] = f * (delta[t] - mean);
}

__global__ void __launch_bounds__(kBlock)
k_shift_by_mean(double *__restrict__ a, size_t count, const double *__restrict__ sum,
                double inv_count) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= count) return;
    a[t] -= sum[0] * inv_count;
}

__global__ void __launch_bounds__(kBlock)
k_fill(double *__restrict__ a, size_t count, double v) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < count) a[t] = v;
}

__global__ void __launch_bounds__(kBlock)
k_copy(const double *__restrict__ src, double *__restrict__ dst, size_t count) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < count) dst[t] = src[t];
}

// Value of the parent at continuous coordinate X (parent cell c centred at
// c) by trilinear interpolation; the child box's cells are 2^m / 2 parent
// cells wide, so every coordinate and weight is an exact binary fraction.
template <bool PPER>
__global__ void __launch_bounds__(kBlock)
k_interpolate(const double *__restrict__ parent, int np, int lgp, ChildBox bx,
              double *__restrict__ child, int ghosts_only) {
    const int pc = bx.nc + 2;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= pc * pc * pc) return;
    const int ii = t % pc, jj = (t / pc) % pc, kk = t / (pc * pc);
    const int ijk[3] = {ii - 1, jj - 1, kk - 1};
    const bool interior = ijk[0] >= 0 && ijk[0] < bx.nc && ijk[1] >= 0 && ijk[1] < bx.nc &&
                          ijk[2] >= 0 && ijk[2] < bx.nc;
    if (ghosts_only && interior) return;
    const double q = ldexp(1.0, bx.m - 1);
    int i0[3];
    double w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double X = bx.origin[a] + (ijk[a] + 0.5) * q - 0.5;
        const double f = floor(X);
        i0[a] = (int)f;
        w[a] = X - f;
    }
    const int msk = np - 1, pp = np + 2;
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const double wt = (a ? w[0] : 1.0 - w[0]) * (b ? w[1] : 1.0 - w[1]) *
                                  (c ? w[2] : 1.0 - w[2]);
                const int x = i0[0] + a, y = i0[1] + b, z = i0[2] + c;
                int q2;
                if (PPER)
                    q2 = (((z & msk) << lgp | (y & msk)) << lgp) | (x & msk);
                else
                    q2 = ((z + 1) * pp + (y + 1)) * pp + (x + 1);
                v += wt * parent[q2];
            }
    child[t] = v;
}

template <bool PER>
__global__ void __launch_bounds__(kBlock)
k_force(const double *__restrict__ phi, Ix<PER> ix, double c4h, double *__restrict__ f) {
    const int n = ix.n, lg = ix.lg;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int cells = 1 << (3 * lg);
    if (t >= cells) return;
    const int i = t & (n - 1), j = (t >> lg) & (n - 1), k = t >> (2 * lg);
    f[t] = -(phi[ix(i + 1, j, k)] - phi[ix(i - 1, j, k)]) * c4h;
    f[(size_t)cells + t] = -(phi[ix(i, j + 1, k)] - phi[ix(i, j - 1, k)]) * c4h;
    f[2 * (size_t)cells + t] = -(phi[ix(i, j, k + 1)] - phi[ix(i, j, k - 1)]) * c4h;
}

} // namespace

// ------------------------------------------------------------------------
// launchers

void launch_smooth_half(const Level &L, const double *pin, double *pout, int colour,
                        unsigned *fallbacks, hipStream_t st) {
    const unsigned nb = blocks_for(L.cells() / 2);
    if (L.periodic)
        k_smooth_half<true><<<nb, kBlock, 0, st>>>(pin, pout, L.s, make_ix<true>(L.n, L.lg),
                                                   L.alpha, colour, fallbacks);
    else
        k_smooth_half<false><<<nb, kBlock, 0, st>>>(pin, pout, L.s, make_ix<false>(L.n, L.lg),
                                                    L.alpha, colour, fallbacks);
}

void launch_residual_sumsq(const Level &L, double *partials, double *r_out, double r_scale,
                           hipStream_t st) {
    if (L.periodic)
        k_residual_sumsq<true><<<kReduceBlocks, kBlock, 0, st>>>(
            L.phi, L.s, make_ix<true>(L.n, L.lg), L.alpha, partials, r_out, r_scale);
    else
        k_residual_sumsq<false><<<kReduceBlocks, kBlock, 0, st>>>(
            L.phi, L.s, make_ix<false>(L.n, L.lg), L.alpha, partials, r_out, r_scale);
}

void launch_partial_sums(const double *a, size_t count, bool squares, double *partials,
                         hipStream_t st) {
    k_partial_sums<<<kReduceBlocks, kBlock, 0, st>>>(a, count, squares ? 1 : 0, partials);
}

void launch_diff_partials(const double *a, const double *b, size_t count, double *partials,
                          hipStream_t st) {
    k_diff_partials<<<kReduceBlocks, kBlock, 0, st>>>(a, b, count, partials);
}

void launch_reduce_final(const double *partials, double *out, hipStream_t st) {
    k_reduce_final<<<1, kBlock, 0, st>>>(partials, out);
}

void launch_restrict_residual(const Level &F, const Level &C, hipStream_t st) {
    const unsigned nb = blocks_for(C.cells());
    if (F.periodic)
        k_restrict_residual<true><<<nb, kBlock, 0, st>>>(F.phi, F.s, make_ix<true>(F.n, F.lg),
                                                         F.alpha, C.hat, C.s,
                                                         make_ix<true>(C.n, C.lg));
    else
        k_restrict_residual<false><<<nb, kBlock, 0, st>>>(F.phi, F.s, make_ix<false>(F.n, F.lg),
                                                          F.alpha, C.hat, C.s,
                                                          make_ix<false>(C.n, C.lg));
}

void launch_coarse_source(const Level &C, hipStream_t st) {
    const unsigned nb = blocks_for(C.cells());
    if (C.periodic)
        k_coarse_source<true><<<nb, kBlock, 0, st>>>(C.hat, C.phi, C.s, make_ix<true>(C.n, C.lg),
                                                     C.alpha);
    else
        k_coarse_source<false><<<nb, kBlock, 0, st>>>(C.hat, C.phi, C.s,
                                                      make_ix<false>(C.n, C.lg), C.alpha);
}

void launch_prolong_correct(const Level &F, const Level &C, hipStream_t st) {
    const unsigned nb = blocks_for(F.cells());
    if (F.periodic)
        k_prolong<true, true><<<nb, kBlock, 0, st>>>(F.phi, make_ix<true>(F.n, F.lg), C.phi,
                                                     C.hat, make_ix<true>(C.n, C.lg));
    else
        k_prolong<false, true><<<nb, kBlock, 0, st>>>(F.phi, make_ix<false>(F.n, F.lg), C.phi,
                                                      C.hat, make_ix<false>(C.n, C.lg));
}

void launch_prolong_full(const Level &F, const Level &C, hipStream_t st) {
    const unsigned nb = blocks_for(F.cells());
    if (F.periodic)
        k_prolong<true, false><<<nb, kBlock, 0, st>>>(F.phi, make_ix<true>(F.n, F.lg), C.phi,
                                                      nullptr, make_ix<true>(C.n, C.lg));
    else
        k_prolong<false, false><<<nb, kBlock, 0, st>>>(F.phi, make_ix<false>(F.n, F.lg), C.phi,
                                                       nullptr, make_ix<false>(C.n, C.lg));
}

void launch_restrict_source(const Level &F, const Level &C, hipStream_t st) {
    k_restrict_source<<<blocks_for(C.cells()), kBlock, 0, st>>>(F.s, F.n, C.s, C.lg);
}

void launch_coarsest(const Level &L, int sweeps, unsigned *fallbacks, hipStream_t st) {
    const int threads = L.cells() < 64 ? 64 : (int)L.cells();
    if (L.periodic)
        k_coarsest<true><<<1, threads, 0, st>>>(L.phi, L.s, make_ix<true>(L.n, L.lg), L.alpha,
                                                sweeps, fallbacks);
    else
        k_coarsest<false><<<1, threads, 0, st>>>(L.phi, L.s, make_ix<false>(L.n, L.lg), L.alpha,
                                                 sweeps, fallbacks);
}

void launch_source(const double *delta, size_t count, const double *sum, double inv_count_mean,
                   double f, double *s, hipStream_t st) {
    k_source<<<blocks_for(count), kBlock, 0, st>>>(delta, count, sum, inv_count_mean, f, s);
}

void launch_shift_by_mean(double *a, size_t count, const double *sum, hipStream_t st) {
    k_shift_by_mean<<<blocks_for(count), kBlock, 0, st>>>(a, count, sum, 1.0 / (double)count);
}

void launch_fill(double *a, size_t count, double v, hipStream_t st) {
    k_fill<<<blocks_for(count), kBlock, 0, st>>>(a, count, v);
}

void launch_copy(const double *src, double *dst, size_t count, hipStream_t st) {
    k_copy<<<blocks_for(count), kBlock, 0, st>>>(src, dst, count);
}

void launch_interpolate(const double *parent, int np, bool parent_periodic, const ChildBox &b,
                        double *child_pad, bool ghosts_only, hipStream_t st) {
    const size_t pc = (size_t)b.nc + 2;
    const unsigned nb = blocks_for(pc * pc * pc);
    if (parent_periodic)
        k_interpolate<true><<<nb, kBlock, 0, st>>>(parent, np, log2i(np), b, child_pad,
                                                   ghosts_only ? 1 : 0);
    else
        k_interpolate<false><<<nb, kBlock, 0, st>>>(parent, np, log2i(np), b, child_pad,
                                                    ghosts_only ? 1 : 0);
}

void launch_force(const double *phi, int n, bool periodic, double h, double *f, hipStream_t st) {
    const int lg = log2i(n);
    const unsigned nb = blocks_for((size_t)n * n * n);
    if (periodic)
        k_force<true><<<nb, kBlock, 0, st>>>(phi, make_ix<true>(n, lg), 0.25 / h, f);
    else
        k_force<false><<<nb, kBlock, 0, st>>>(phi, make_ix<false>(n, lg), 0.25 / h, f);
}

} // namespace ndgp
