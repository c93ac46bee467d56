// ndgp_particles.hip -- cloud-in-cell transfers between equal-mass particles
// and the grid levels (arXiv:1511.08200, Sec. IV.A: the density and the forces
// go back and forth between particles and cells by cloud-in-cell).
//
// A particle is a cube of one cell's size centred on its position: along each
// axis the cell whose centre lies below it gets 1 - t and the next one t (t:
// distance from that centre in cells), and a cell gets the product of its
// three axis weights.  Level 0 is the periodic domain; a patch level takes
// the particles whose cube overlaps its cells, comparing positions with the
// patch modulo the box (a patch may wrap the domain).
//
// Deposit: the weights are added as 64-bit fixed-point integers (2^-36 of a
// particle), so the sums are exact and the same in any order -- the density
// is bit for bit reproducible although thousands of threads add into one
// cell.  Gather: every particle reads the finest level whose eight cells
// around it all lie inside that level.

#include "ndgp_device.h"

#include <cmath>

namespace ndgp {
namespace {

using namespace dev;

constexpr double kCicOne = 68719476736.0; // 2^36: one particle in fixed point

// The cells along one axis (up to two images of the particle, two cells each)
// that lie in [0, m) of the level, with their weights.
__device__ __forceinline__ int cic_axis(double x01, int n, double corner, double cells_per_domain,
                                        int m, bool periodic, int idx[4], double w[4]) {
    double d = x01 * (double)n - corner;
    d = d - (double)n * floor(d / (double)n); // [0, n)
    int cnt = 0;
#pragma unroll
    for (int img = 0; img < 2; ++img) {
        if (periodic && img) break;
        const double u = (img ? d - (double)n : d) * cells_per_domain - 0.5;
        const double f = floor(u);
        const double t = u - f;
        const int i0 = (int)f;
#pragma unroll
        for (int off = 0; off < 2; ++off) {
            int i = i0 + off;
            if (periodic) i &= m - 1;
            else if (i < 0 || i >= m) continue;
            idx[cnt] = i;
            w[cnt] = off ? t : 1.0 - t;
            ++cnt;
        }
    }
    return cnt;
}

// One thread per particle.  Particles whose eight cells are all in the level
// (the usual case) are keyed by their lower cell; lanes of a wave that hold a
// contiguous run of equal keys -- particles sorted by cell, as a tree code
// keeps them, in a dense region -- first add their fixed-point weights with
// shuffles (a segmented scan), and only the run's last lane sends the eight
// atomics.  Integer sums: the same bits whatever the grouping.
__global__ void __launch_bounds__(kBlock)
k_cic_deposit(const double *__restrict__ pos, long long np, int n, double cx, double cy, double cz,
              double cells_per_domain, int m, int periodic,
              unsigned long long *__restrict__ acc) {
    const long long p = (long long)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int ix[4], iy[4], iz[4];
    double wx[4], wy[4], wz[4];
    int nx = 0, ny = 0, nz = 0;
    if (p < np) {
        nx = cic_axis(pos[p], n, cx, cells_per_domain, m, periodic != 0, ix, wx);
        ny = cic_axis(pos[np + p], n, cy, cells_per_domain, m, periodic != 0, iy, wy);
        nz = cic_axis(pos[2 * np + p], n, cz, cells_per_domain, m, periodic != 0, iz, wz);
    }
    const bool whole = nx == 2 && ny == 2 && nz == 2 && ix[1] == ((ix[0] + 1) & (m - 1)) &&
                       iy[1] == ((iy[0] + 1) & (m - 1)) && iz[1] == ((iz[0] + 1) & (m - 1));
    if (!whole) { // partial overlap with a patch, or no particle: direct atomics
        for (int c = 0; c < nz; ++c)
            for (int b = 0; b < ny; ++b)
                for (int a = 0; a < nx; ++a) {
                    const double w = (wx[a] * wy[b]) * wz[c];
                    const unsigned long long q = __double2ull_rn(w * kCicOne);
                    if (q) atomicAdd(&acc[((size_t)iz[c] * m + iy[b]) * m + ix[a]], q);
                }
    }
    // the eight weights of a whole particle, in fixed point
    unsigned long long q[8];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                q[(c * 2 + b) * 2 + a] = whole ? __double2ull_rn(((wx[a] * wy[b]) * wz[c]) * kCicOne) : 0ull;
    // key: lower cell of a whole particle, else unique to the lane
    const long long key = whole ? (long long)(((size_t)iz[0] * m + iy[0]) * m + ix[0]) : -1 - lane;
    const long long kprev = __shfl_up(key, 1, 64);
    const bool head = lane == 0 || kprev != key;
    // start lane of this lane's run of equal keys (max over heads at or below)
    int seg = head ? lane : 0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(seg, off, 64);
        if (lane >= off) seg = seg > o ? seg : o;
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int so = __shfl_up(seg, off, 64);
        unsigned long long qo[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) qo[r] = __shfl_up(q[r], off, 64);
        if (lane >= off && so == seg) {
#pragma unroll
            for (int r = 0; r < 8; ++r) q[r] += qo[r];
        }
    }
    const int snext = __shfl_down(seg, 1, 64);
    const bool tail = lane == 63 || snext != seg;
    if (whole && tail) {
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const unsigned long long v = q[(c * 2 + b) * 2 + a];
                    if (v) atomicAdd(&acc[((size_t)iz[c] * m + iy[b]) * m + ix[a]], v);
                }
    }
}

__global__ void __launch_bounds__(kBlock)
k_cic_finish(const unsigned long long *__restrict__ acc, size_t cells, double scale,
             double *__restrict__ delta) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < cells) delta[t] = (double)acc[t] * scale - 1.0;
}

__global__ void __launch_bounds__(kBlock)
k_zero_acc(unsigned long long *__restrict__ a, size_t count) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < count) a[t] = 0ull;
}

// The lower cell and weight along one axis if all of the particle's cells lie
// inside the level (for a patch: the image whose two cells are in [0, m)).
__device__ __forceinline__ bool cic_inside(double x01, int n, double corner,
                                           double cells_per_domain, int m, bool periodic,
                                           int &i0, double &t) {
    double d = x01 * (double)n - corner;
    d = d - (double)n * floor(d / (double)n);
#pragma unroll
    for (int img = 0; img < 2; ++img) {
        if (periodic && img) break;
        const double u = (img ? d - (double)n : d) * cells_per_domain - 0.5;
        const double f = floor(u);
        const int i = (int)f;
        if (periodic || (i >= 0 && i + 1 <= m - 1)) {
            i0 = i;
            t = u - f;
            return true;
        }
    }
    return false;
}

__global__ void __launch_bounds__(kBlock)
k_cic_gather(const double *__restrict__ pos, long long np, CicLevels lv,
             double *__restrict__ out) {
    const long long p = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (p >= np) return;
    const double x = pos[p], y = pos[np + p], z = pos[2 * np + p];
    for (int q = lv.levels - 1; q >= 0; --q) {
        const bool per = q == 0;
        const int m = lv.m[q];
        const double cpd = lv.cells_per_domain[q];
        int i0, j0, k0;
        double tx, ty, tz;
        if (!cic_inside(x, lv.n, lv.corner[q][0], cpd, m, per, i0, tx)) continue;
        if (!cic_inside(y, lv.n, lv.corner[q][1], cpd, m, per, j0, ty)) continue;
        if (!cic_inside(z, lv.n, lv.corner[q][2], cpd, m, per, k0, tz)) continue;
        const double *f = lv.force[q];
        const size_t cells = (size_t)m * m * m;
        double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx) {
                    const double w = ((dx ? tx : 1.0 - tx) * (dy ? ty : 1.0 - ty)) * (dz ? tz : 1.0 - tz);
                    int ci = i0 + dx, cj = j0 + dy, ck = k0 + dz;
                    if (per) {
                        ci &= m - 1;
                        cj &= m - 1;
                        ck &= m - 1;
                    }
                    const size_t c = ((size_t)ck * m + cj) * m + ci;
#pragma unroll
                    for (int a = 0; a < 3; ++a) acc[a] = fma(w, f[a * cells + c], acc[a]);
                }
#pragma unroll
        for (int a = 0; a < 3; ++a) out[a * np + p] = acc[a];
        return;
    }
}

// Refinement criterion of Sec. IV.A: a cell is refined when the particles in
// its volume number more than n_ref.  count = (delta + 1) mean with mean the
// level's particles per cell; per-block counts of flagged cells.
__global__ void __launch_bounds__(kBlock)
k_refine_flags(const double *__restrict__ delta, size_t cells, double mean, double n_ref,
               unsigned char *__restrict__ flags, double *__restrict__ partials) {
    double nflag = 0.0;
    for (size_t c = (size_t)blockIdx.x * kBlock + threadIdx.x; c < cells;
         c += (size_t)gridDim.x * kBlock) {
        const bool f = (delta[c] + 1.0) * mean > n_ref;
        flags[c] = f ? 1 : 0;
        nflag += f ? 1.0 : 0.0;
    }
    const double b = block_sum(nflag);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

} // namespace

void launch_refine_flags(const double *delta, size_t cells, double mean, double n_ref,
                         unsigned char *flags, double *partials, hipStream_t st) {
    k_refine_flags<<<kReduceBlocks, kBlock, 0, st>>>(delta, cells, mean, n_ref, flags, partials);
}

void launch_cic_deposit(const double *pos, long long np, int n, const double corner[3], int q,
                        int m, unsigned long long *acc, double *delta, hipStream_t st) {
    const size_t cells = (size_t)m * m * m;
    k_zero_acc<<<blocks_for(cells), kBlock, 0, st>>>(acc, cells);
    if (np > 0)
        k_cic_deposit<<<(unsigned)((np + kBlock - 1) / kBlock), kBlock, 0, st>>>(
            pos, np, n, corner[0], corner[1], corner[2], std::ldexp(1.0, q), m, q == 0 ? 1 : 0,
            acc);
    // delta = count / mean - 1, mean = np / (n 2^q)^3 particles per cell
    const double cells_equiv = std::ldexp((double)n * n * n, 3 * q);
    const double scale = np > 0 ? cells_equiv / ((double)np * kCicOne) : 0.0;
    k_cic_finish<<<blocks_for(cells), kBlock, 0, st>>>(acc, cells, scale, delta);
}

void launch_cic_gather(const double *pos, long long np, const CicLevels &lv, double *out,
                       hipStream_t st) {
    if (np > 0)
        k_cic_gather<<<(unsigned)((np + kBlock - 1) / kBlock), kBlock, 0, st>>>(pos, np, lv, out);
}

} // namespace ndgp
