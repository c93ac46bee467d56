// ndgp_device.h -- device-side helpers shared by the library's kernel files:
// indexing, the 19-point stencil, the per-cell root, fast reciprocal and square
// root, and the deterministic block sum.  Not part of the public ABI.
#pragma once

#include "ndgp_internal.h"

namespace ndgp {
namespace dev {

// ------------------------------------------------------------------------
// z-streamed sweeps: ring slots, opaque per-thread values, plane addressing

// A plane of a fused sweep's z-chunk named by its offset from the chunk's first
// plane, as a type: LDS ring slots derived from it are compile-time constants,
// so every LDS access is the thread's base address plus an immediate offset
// (the LDS-streamed fused sweeps).
template <int D>
struct Plane {
    static constexpr int d = D;
};
constexpr int ring_slot(int a, int p) { return ((a % p) + p) % p; }
constexpr int floor_half(int a) { return a >= 0 ? a / 2 : -((1 - a) / 2); }

// The same per-thread value, opaque to the optimiser at this point: addresses
// derived from it are formed here, one instruction each, instead of being
// hoisted out of the z loop and held in registers the stencil needs.
__device__ __forceinline__ int fresh(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Cell i of one z-plane, the plane's address uniform across the workgroup (in
// scalar registers) and i a 32-bit offset inside it (a padded 1024^2 plane is
// 8.4 MB): one vector register per address instead of two.
__device__ __forceinline__ const double *plane_at(const double *plane, unsigned i) {
    return reinterpret_cast<const double *>(reinterpret_cast<const char *>(plane) + i * 8u);
}
__device__ __forceinline__ double *plane_at(double *plane, unsigned i) {
    return reinterpret_cast<double *>(reinterpret_cast<char *>(plane) + i * 8u);
}
__device__ __forceinline__ const float *plane_at(const float *plane, unsigned i) {
    return reinterpret_cast<const float *>(reinterpret_cast<const char *>(plane) + i * 4u);
}
__device__ __forceinline__ float *plane_at(float *plane, unsigned i) {
    return reinterpret_cast<float *>(reinterpret_cast<char *>(plane) + i * 4u);
}

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

template <bool PER, class T>
__device__ __forceinline__ void gather(const T *__restrict__ a, const Ix<PER> &ix, int i,
                                       int j, int k, T v[19]) {
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
    // corner (s,t) of plane a-b: C = v_st - (d_a,s + f_b,t), with f_b,t = v[face]
    double c, c2, sv;
    c = v[7] - (dxp + v[3]);  c2 = c * c;          sv = v[7];
    c = v[8] - (dxp + v[4]);  c2 = fma(c, c, c2);  sv += v[8];
    c = v[9] - (dxm + v[3]);  c2 = fma(c, c, c2);  sv += v[9];
    c = v[10] - (dxm + v[4]); c2 = fma(c, c, c2);  sv += v[10];
    c = v[11] - (dxp + v[5]); c2 = fma(c, c, c2);  sv += v[11];
    c = v[12] - (dxp + v[6]); c2 = fma(c, c, c2);  sv += v[12];
    c = v[13] - (dxm + v[5]); c2 = fma(c, c, c2);  sv += v[13];
    c = v[14] - (dxm + v[6]); c2 = fma(c, c, c2);  sv += v[14];
    c = v[15] - (dyp + v[5]); c2 = fma(c, c, c2);  sv += v[15];
    c = v[16] - (dyp + v[6]); c2 = fma(c, c, c2);  sv += v[16];
    c = v[17] - (dym + v[5]); c2 = fma(c, c, c2);  sv += v[17];
    c = v[18] - (dym + v[6]); c2 = fma(c, c, c2);  sv += v[18];
    Terms t;
    t.lap = (Dxx + Dyy) + Dzz;
    t.nl = fma(Dxx, Dyy, fma(Dxx, Dzz, Dyy * Dzz)) - 0.25 * c2;
    t.see = fma(-12.0, u, sv);
    return t;
}

__device__ __forceinline__ double apply_L(const Terms &t, double al) {
    return fma(2.0 * al, t.nl, t.lap);
}

// New value of the centre cell: the root of its own equation T(u') = 0 on the
// elliptic branch.  Moving u by du shifts every D_aa by -2 du and every corner
// difference by +du, so with dt = 2 du
//     T(dt) = r - B dt + (9/2) alpha dt^2,   r = L - s,
//     B = 3 + 4 alpha lap + 2 alpha M,  M = (1/4) sum C = see/4 - lap,
// and B itself falls by 9 alpha dt: the linearised operator is elliptic at the
// cell (dL/du < 0) left of the parabola's vertex dt = B / (9 alpha).  The root
// there is dt = (B - sqrt(B^2 - 18 alpha r)) / (9 alpha), written as
// 2 r / (B + sqrt(...)) when B > 0 (no cancellation; continuous with the
// linear case) and as it stands when B <= 0 (the value was past the vertex).
// No real root: move to the vertex.
// Reciprocal and square root from the hardware estimates plus one Newton
// step each (relative error near 1e-16).  The relaxation only needs them to
// pick its step: the fixed point L[phi] = s does not depend on how they round.
__device__ __forceinline__ double fast_rcp(double q) {
    const double y = __builtin_amdgcn_rcp(q);
    return fma(y, fma(-q, y, 1.0), y);
}

// fast_sqrt takes d >= 0 (the relaxation calls it only there): the estimate
// of 1/sqrt(d) is capped at 2^511, its value at the smallest normal double,
// so that d = 0 gives 0 (0 x 2^511) with no select, and every d >= 2^-1022 is
// unchanged.
__device__ __forceinline__ double fast_sqrt(double d) {
    const double rs = fmin(__builtin_amdgcn_rsq(d), 0x1p511);
    const double s0 = d * rs;
    const double e = fma(-s0, 0.5 * rs, 0.5);
    return fma(s0, e, s0);
}

// Relaxation events a thread counts in one unsigned: a visit with no real
// root adds 1, a visit of a cell past its vertex (not elliptic there) adds
// kPastVertexEvent (a thread relaxes far fewer than 2^16 cells per launch, so
// the halves never carry into each other).  flush_events adds them to the
// launch's two counters: counters[0] = no real root, counters[1] = past the
// vertex.
constexpr unsigned kPastVertexEvent = 1u << 16;

__device__ __forceinline__ void flush_events(unsigned *counters, unsigned ev) {
    if (ev & 0xffffu) atomicAdd(counters, ev & 0xffffu);
    if (ev >> 16) atomicAdd(counters + 1, ev >> 16);
}

// New value of one cell: the root of its own quadratic with the neighbours
// held, u + w * du.  w = 1 takes the root itself (w * r is then exactly r);
// w < 1 damps the step, for the safeguarded iteration of the driver (every
// branch is damped the same way).
__device__ __forceinline__ double relax_cell(const double v[19], double s, double al, double w,
                                             unsigned &events) {
    const Terms t = stencil_terms(v);
    const double r = apply_L(t, al) - s;
    const double B = fma(al, fma(2.0, t.lap, 0.5 * t.see), 3.0);
    const double D = fma(B, B, -18.0 * al * r);
    if (D < 0.0) {
        ++events;
        return fma(w, B / (18.0 * al), v[0]);
    }
    if (B > 0.0) return fma(w * r, fast_rcp(B + fast_sqrt(D)), v[0]);
    events += kPastVertexEvent;
    return fma(w, (B - fast_sqrt(D)) / (18.0 * al), v[0]);
}

// Coarse levels of a refinement: the ghosts whose correction is taken from
// interior cell (i,j,k).  The correction phi - hat is extrapolated linearly
// through zero at the fine boundary position (half a fine cell outside), which
// puts -1/3 of it on the coarse ghost per axis along which the ghost lies
// outside.  Every ghost has exactly one such interior cell, so each is
// written by one thread.
//
// ghost_slots: q[0] the cell itself, q[m] (m = 1..7, bit 0 x, bit 1 y, bit 2
// z) the ghost reached by leaving the grid along the axes of m; an axis along
// which the cell is not on the boundary keeps the cell's own index (always in
// range).  Returns the bit set of the slots that are ghosts of this cell.
template <bool PER>
__device__ __forceinline__ unsigned ghost_slots(const Ix<PER> &ix, int i, int j, int k, int q[8]) {
    const int n = ix.n;
    const bool bx = i == 0 || i == n - 1, by = j == 0 || j == n - 1, bz = k == 0 || k == n - 1;
    const int gx = bx ? (i == 0 ? -1 : n) : i, gy = by ? (j == 0 ? -1 : n) : j,
              gz = bz ? (k == 0 ? -1 : n) : k;
    unsigned own = 0;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        q[m] = ix(m & 1 ? gx : i, m & 2 ? gy : j, m & 4 ? gz : k);
        const bool ok = m != 0 && !((m & 1) && !bx) && !((m & 2) && !by) && !((m & 4) && !bz);
        own |= ok ? 1u << m : 0u;
    }
    return own;
}

// ghost value from the cell's new value, with h[m] = hat[q[m]] of ghost_slots
__device__ __forceinline__ void store_owned_ghosts(double *__restrict__ out, const int q[8],
                                                   const double h[8], unsigned own, double val) {
    const double e = val - h[0];
#pragma unroll
    for (int m = 1; m < 8; ++m) {
        if (!(own >> m & 1u)) continue;
        const int d = (m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1);
        const double f = d == 1 ? -1.0 / 3.0 : (d == 2 ? 1.0 / 9.0 : -1.0 / 27.0);
        out[q[m]] = h[m] + f * e;
    }
}

// Write the ghosts of cell (i,j,k) now holding `val`.  Every hat value is
// loaded before the first store, so that a boundary cell waits for memory
// once, not once per ghost.
template <bool PER>
__device__ __forceinline__ void write_owned_ghosts(double *__restrict__ out,
                                                   const double *__restrict__ hat,
                                                   const Ix<PER> &ix, int i, int j, int k,
                                                   double val) {
    if constexpr (!PER) {
        const int n = ix.n;
        if (!(i == 0 || i == n - 1 || j == 0 || j == n - 1 || k == 0 || k == n - 1)) return;
        int q[8];
        double h[8];
        const unsigned own = ghost_slots(ix, i, j, k, q);
#pragma unroll
        for (int m = 0; m < 8; ++m) h[m] = hat[q[m]];
        store_owned_ghosts(out, q, h, own, val);
    }
}

// Cell-centred trilinear interpolation of a parent level at the padded slot
// (ii, jj, kk) of a child box (bx: lower corner in parent cells, the box's
// cells 2^(m-1) parent cells wide, nc cells per side; slot 0 and nc+1 are
// the ghost shell).  Parent: natural and periodic (PPER) or padded.
template <bool PPER>
__device__ __forceinline__ double interpolate_slot(const double *__restrict__ parent, int np,
                                                   int lgp, const ChildBox &bx, int ii, int jj,
                                                   int kk) {
    const int ijk[3] = {ii - 1, jj - 1, kk - 1};
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
    return v;
}

// Workgroups of a launch are dealt to the 8 XCDs of the chip round robin
// (workgroup id modulo 8), and each XCD has its own L2.  Renumber so that XCD
// x runs a contiguous run of logical tiles: spatial neighbours then share the
// L2 that holds their common halo lines.  Identity when the grid is not a
// multiple of 8.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_local_id(int lin, int total) {
    if (total % kXcds) return lin;
    return (lin % kXcds) * (total / kXcds) + lin / kXcds;
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

} // namespace dev
} // namespace ndgp
