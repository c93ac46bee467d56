// ndgp_stats.hip -- total force and G_eff statistics per refinement level
// (arXiv:1511.08200, Eq. modpoisson and Sec. III.B; the per-level view of
// Sec. IV.B, Fig. 3, taken over grid cells instead of particles).
//
// The dynamical potential is Psi = Psi_N + phi/2 (Eq. modpoisson), so the
// total force is F = -grad(Psi_N) - grad(phi)/2 and the effective strength of
// gravity G_eff = 1 + |F_5th| / |F_GR| (Sec. III.B) with F_5th = -grad(phi)/2
// and F_GR = -grad(Psi_N).  All gradients are central differences on the
// level; patch levels use their ghost shells.  A cell of level l that a finer
// patch covers is left out of level l's statistics: each cell counts on the
// finest level that holds it, as a particle does in Fig. 3.

#include "ndgp_device.h"

namespace ndgp {
namespace {

using namespace dev;

template <bool PER>
__global__ void __launch_bounds__(kBlock)
k_total_force(const double *__restrict__ phi, const double *__restrict__ psi, Ix<PER> ix,
              double c2h, double c4h, double *__restrict__ f) {
    const int n = ix.n, lg = ix.lg;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int cells = 1 << (3 * lg);
    if (t >= cells) return;
    const int i = t & (n - 1), j = (t >> lg) & (n - 1), k = t >> (2 * lg);
    const int up[3] = {ix(i + 1, j, k), ix(i, j + 1, k), ix(i, j, k + 1)};
    const int dn[3] = {ix(i - 1, j, k), ix(i, j - 1, k), ix(i, j, k - 1)};
#pragma unroll
    for (int a = 0; a < 3; ++a)
        f[(size_t)a * cells + t] = -((psi[up[a]] - psi[dn[a]]) * c2h) - (phi[up[a]] - phi[dn[a]]) * c4h;
}

// G_eff - 1 of one cell: |F_5th| / |F_GR| = sqrt(sum dphi^2 / sum dpsi^2) / 2
// (the spacing cancels); a cell without Newtonian force counts as 0 if it has
// no fifth force either, else as +inf.
template <bool PER>
__device__ __forceinline__ double geff_minus_one(const double *__restrict__ phi,
                                                 const double *__restrict__ psi, const Ix<PER> &ix,
                                                 int i, int j, int k) {
    const int up[3] = {ix(i + 1, j, k), ix(i, j + 1, k), ix(i, j, k + 1)};
    const int dn[3] = {ix(i - 1, j, k), ix(i, j - 1, k), ix(i, j, k - 1)};
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double dp = phi[up[q]] - phi[dn[q]];
        const double ds = psi[up[q]] - psi[dn[q]];
        a = a + dp * dp;
        b = b + ds * ds;
    }
    if (b == 0.0) return a == 0.0 ? 0.0 : INFINITY;
    return 0.5 * sqrt(a / b);
}

// Per-block count, sum, sum of squares, min and max of G_eff - 1 over the
// level's cells outside the child box (cells [o, o + half) per axis, wrapped
// on a periodic level; half = 0: no child), and the histogram over the bins
// cut by `edges` (bin b holds edges[b-1] <= x < edges[b]), counted in LDS and
// added to `hist` with integer atomics (exact, so in any order).
template <bool PER>
__global__ void __launch_bounds__(kBlock)
k_geff_partials(const double *__restrict__ phi, const double *__restrict__ psi, Ix<PER> ix,
                int ox, int oy, int oz, int half, const double *__restrict__ edges, int n_edges,
                double *__restrict__ partials, unsigned long long *__restrict__ hist) {
    __shared__ unsigned int bins[kGeffMaxEdges + 1];
    __shared__ double E[kGeffMaxEdges];
    for (int b = threadIdx.x; b <= n_edges; b += kBlock) bins[b] = 0u;
    for (int b = threadIdx.x; b < n_edges; b += kBlock) E[b] = edges[b];
    __syncthreads();
    const int n = ix.n, lg = ix.lg;
    const int total = 1 << (3 * lg);
    double cnt = 0.0, s1 = 0.0, s2 = 0.0, lo = INFINITY, hi = -INFINITY;
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < total; c += gridDim.x * kBlock) {
        const int i = c & (n - 1), j = (c >> lg) & (n - 1), k = c >> (2 * lg);
        if (half > 0) {
            const unsigned di = PER ? (unsigned)((i - ox) & (n - 1)) : (unsigned)(i - ox);
            const unsigned dj = PER ? (unsigned)((j - oy) & (n - 1)) : (unsigned)(j - oy);
            const unsigned dk = PER ? (unsigned)((k - oz) & (n - 1)) : (unsigned)(k - oz);
            if (di < (unsigned)half && dj < (unsigned)half && dk < (unsigned)half) continue;
        }
        const double x = geff_minus_one(phi, psi, ix, i, j, k);
        cnt += 1.0;
        s1 += x;
        s2 = fma(x, x, s2);
        lo = fmin(lo, x);
        hi = fmax(hi, x);
        int b0 = 0, b1 = n_edges; // first edge above x: upper bound by bisection
        while (b0 < b1) {
            const int mid = (b0 + b1) >> 1;
            if (E[mid] <= x)
                b0 = mid + 1;
            else
                b1 = mid;
        }
        atomicAdd(&bins[b0], 1u);
    }
    const double c_b = block_sum(cnt);
    __syncthreads();
    const double s1_b = block_sum(s1);
    __syncthreads();
    const double s2_b = block_sum(s2);
    __shared__ double wlo[kBlock / 64], whi[kBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        wlo[threadIdx.x >> 6] = lo;
        whi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = c_b;
        partials[kReduceBlocks + blockIdx.x] = s1_b;
        partials[2 * kReduceBlocks + blockIdx.x] = s2_b;
        partials[3 * kReduceBlocks + blockIdx.x] = fmin(fmin(wlo[0], wlo[1]), fmin(wlo[2], wlo[3]));
        partials[4 * kReduceBlocks + blockIdx.x] = fmax(fmax(whi[0], whi[1]), fmax(whi[2], whi[3]));
    }
    for (int b = threadIdx.x; b <= n_edges; b += kBlock)
        if (bins[b]) atomicAdd(&hist[b], (unsigned long long)bins[b]);
}

// out[0..2] = fixed-order sums of count, sum, sum of squares; out[3], out[4]
// = min and max over the blocks.
__global__ void __launch_bounds__(kBlock)
k_geff_final(const double *__restrict__ partials, double *__restrict__ out) {
    double acc[3] = {0.0, 0.0, 0.0};
    double lo = INFINITY, hi = -INFINITY;
    for (int q = threadIdx.x; q < kReduceBlocks; q += kBlock) {
#pragma unroll
        for (int r = 0; r < 3; ++r) acc[r] += partials[r * kReduceBlocks + q];
        lo = fmin(lo, partials[3 * kReduceBlocks + q]);
        hi = fmax(hi, partials[4 * kReduceBlocks + q]);
    }
    const double c = block_sum(acc[0]);
    __syncthreads();
    const double s1 = block_sum(acc[1]);
    __syncthreads();
    const double s2 = block_sum(acc[2]);
    __shared__ double wlo[kBlock / 64], whi[kBlock / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        wlo[threadIdx.x >> 6] = lo;
        whi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = c;
        out[1] = s1;
        out[2] = s2;
        out[3] = fmin(fmin(wlo[0], wlo[1]), fmin(wlo[2], wlo[3]));
        out[4] = fmax(fmax(whi[0], whi[1]), fmax(whi[2], whi[3]));
    }
}

__global__ void __launch_bounds__(kBlock)
k_zero_u64(unsigned long long *__restrict__ a, int count) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < count) a[t] = 0ull;
}

} // namespace

void launch_total_force(const double *phi, const double *psi, int n, bool periodic, double h,
                        double *f, hipStream_t st) {
    const unsigned nb = blocks_for((size_t)n * n * n);
    const int lg = log2i(n);
    if (periodic)
        k_total_force<true><<<nb, kBlock, 0, st>>>(phi, psi, make_ix<true>(n, lg), 0.5 / h,
                                                   0.25 / h, f);
    else
        k_total_force<false><<<nb, kBlock, 0, st>>>(phi, psi, make_ix<false>(n, lg), 0.5 / h,
                                                    0.25 / h, f);
}

void launch_geff_level(const double *phi, const double *psi, int n, bool periodic,
                       const int child_origin[3], int child_half, const double *edges,
                       int n_edges, double *partials, unsigned long long *hist, double *out,
                       hipStream_t st) {
    const int lg = log2i(n);
    k_zero_u64<<<blocks_for((size_t)n_edges + 1), kBlock, 0, st>>>(hist, n_edges + 1);
    if (periodic)
        k_geff_partials<true><<<kReduceBlocks, kBlock, 0, st>>>(
            phi, psi, make_ix<true>(n, lg), child_origin[0], child_origin[1], child_origin[2],
            child_half, edges, n_edges, partials, hist);
    else
        k_geff_partials<false><<<kReduceBlocks, kBlock, 0, st>>>(
            phi, psi, make_ix<false>(n, lg), child_origin[0], child_origin[1], child_origin[2],
            child_half, edges, n_edges, partials, hist);
    k_geff_final<<<1, kBlock, 0, st>>>(partials, out);
}

} // namespace ndgp
