// ndgp_mixed.hip -- FP32 kernels of the mixed-precision solve.
//
// The FP64 outer loop computes r = s - L[phi] and adds corrections to phi.
// The correction e solves L[phi + e] - L[phi] = r, relaxed here in FP32 with
// the same red-black per-cell root and full-approximation multigrid as the
// FP64 path.  An FP32 copy of phi alone cannot carry the solution (its
// second differences keep only a few of FP32's digits), so the operator is
// never formed as a difference of two full evaluations: writing w = phi + e,
//   L[w] - L[phi] = lap e + 2 alpha ( sum_{a<b} (Dw_a De_b + De_a Dphi_b)
//                                     - 1/4 sum_corners (Cw + Cphi) Ce ),
// every term carries a factor of e, so FP32 rounding stays relative to the
// correction.  The phi terms only set the coefficients, where FP32's
// accuracy is ample.  The quadratic's discriminant, the root and every
// FP64-field update are in FP64.  Periodic levels only.

#include "ndgp_device.h"

namespace ndgp {
namespace {

using namespace dev;

struct CorrTerms {
    float A;    // L[phi + e] - L[phi] at the cell
    float lapw; // lap of w = phi + e
    float seew; // sum over edges of (w_edge - w_centre)
};

__device__ __forceinline__ CorrTerms corr_terms(const float vp[19], const float ve[19], float al) {
    const float up = vp[0], ue = ve[0];
    const float pxp = vp[1] - up, pxm = vp[2] - up, pyp = vp[3] - up, pym = vp[4] - up;
    const float pzp = vp[5] - up, pzm = vp[6] - up;
    const float exp_ = ve[1] - ue, exm = ve[2] - ue, eyp = ve[3] - ue, eym = ve[4] - ue;
    const float ezp = ve[5] - ue, ezm = ve[6] - ue;
    const float Dpx = pxp + pxm, Dpy = pyp + pym, Dpz = pzp + pzm;
    const float Dex = exp_ + exm, Dey = eyp + eym, Dez = ezp + ezm;
    const float Dwx = Dpx + Dex, Dwy = Dpy + Dey, Dwz = Dpz + Dez;
    const float pair = fmaf(Dwx, Dey, Dex * Dpy) + fmaf(Dwx, Dez, Dex * Dpz) +
                       fmaf(Dwy, Dez, Dey * Dpz);
    // corner (s, t) of plane a-b: C = (v_st - v_s) - (v_t - v_centre), the
    // first difference exact for neighbouring values (Sterbenz), for phi and
    // for e; the sum of the corner differences of w is the edge sum less
    // 4 lap w (every face neighbour sits in four corners)
    float cs = 0.f, sw = 0.f;
    auto corner = [&](int q, int s_face, float pb, float eb) {
        const float Cp = (vp[q] - vp[s_face]) - pb, Ce = (ve[q] - ve[s_face]) - eb;
        const float Cw = Cp + Ce;
        sw += Cw;
        cs = fmaf(Cw + Cp, Ce, cs);
    };
    corner(7, 1, pyp, eyp);
    corner(8, 1, pym, eym);
    corner(9, 2, pyp, eyp);
    corner(10, 2, pym, eym);
    corner(11, 1, pzp, ezp);
    corner(12, 1, pzm, ezm);
    corner(13, 2, pzp, ezp);
    corner(14, 2, pzm, ezm);
    corner(15, 3, pzp, ezp);
    corner(16, 3, pzm, ezm);
    corner(17, 4, pzp, ezp);
    corner(18, 4, pzm, ezm);
    CorrTerms t;
    t.A = fmaf(2.f * al, pair - 0.25f * cs, (Dex + Dey) + Dez);
    t.lapw = (Dwx + Dwy) + Dwz;
    t.seew = fmaf(4.f, t.lapw, sw);
    return t;
}

// New correction at the cell: the root of its own quadratic (same algebra as
// relax_cell, with w = phi + e in place of phi), discriminant and root in FP64.
__device__ __forceinline__ float relax_corr_cell(const float vp[19], const float ve[19], float r,
                                                 float al, double w, unsigned &fallbacks) {
    const CorrTerms t = corr_terms(vp, ve, al);
    const double ad = (double)al;
    const double rT = (double)t.A - (double)r;
    const double B = fma(ad, fma(2.0, (double)t.lapw, 0.5 * (double)t.seew), 3.0);
    const double D = fma(B, B, -18.0 * ad * rT);
    if (D < 0.0) {
        ++fallbacks;
        return (float)fma(w, B / (18.0 * ad), (double)ve[0]);
    }
    if (B > 0.0) return (float)fma(w * rT, fast_rcp(B + fast_sqrt(D)), (double)ve[0]);
    fallbacks += kPastVertexEvent;
    return (float)fma(w, (B - fast_sqrt(D)) / (18.0 * ad), (double)ve[0]);
}

using IxP = Ix<true>;

__global__ void __launch_bounds__(kBlock)
k_residual_to32(const double *__restrict__ phi, const double *__restrict__ s, IxP ix, double al,
                float *__restrict__ r32, double *__restrict__ partials) {
    const int n = ix.n, lg = ix.lg;
    const int total = 1 << (3 * lg);
    double acc = 0.0;
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < total; c += gridDim.x * kBlock) {
        const int i = c & (n - 1), j = (c >> lg) & (n - 1), k = c >> (2 * lg);
        double v[19];
        gather(phi, ix, i, j, k, v);
        const double r = s[c] - apply_L(stencil_terms(v), al);
        acc = fma(r, r, acc);
        r32[c] = (float)r;
    }
    const double b = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

__global__ void __launch_bounds__(kBlock)
k_to32(const double *__restrict__ a, float *__restrict__ b, size_t count) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < count) b[t] = (float)a[t];
}

__global__ void __launch_bounds__(kBlock)
k_add32(double *__restrict__ phi, const float *__restrict__ e, size_t count) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < count) phi[t] += (double)e[t];
}

// phi += e, and the FP32 copy of the result for the next outer iteration
__global__ void __launch_bounds__(kBlock)
k_add_to32(double *__restrict__ phi, const float *__restrict__ e, float *__restrict__ phi32,
           size_t count) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= count) return;
    const double v = phi[t] + (double)e[t];
    phi[t] = v;
    phi32[t] = (float)v;
}

__global__ void __launch_bounds__(kBlock)
k_fill32(float *__restrict__ a, size_t count, float v) {
    const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (t < count) a[t] = v;
}

__global__ void __launch_bounds__(kBlock)
k_avg32(const float *__restrict__ f, int nf, float *__restrict__ c, int lgc) {
    const int nc = 1 << lgc;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= (1 << (3 * lgc))) return;
    const int I = t & (nc - 1), J = (t >> lgc) & (nc - 1), K = t >> (2 * lgc);
    float acc = 0.f;
#pragma unroll
    for (int dk = 0; dk < 2; ++dk)
#pragma unroll
        for (int dj = 0; dj < 2; ++dj)
#pragma unroll
            for (int di = 0; di < 2; ++di)
                acc += f[((size_t)(2 * K + dk) * nf + (2 * J + dj)) * nf + (2 * I + di)];
    c[t] = acc * 0.125f;
}

__global__ void __launch_bounds__(kBlock)
k_corr_half(const float *__restrict__ ein, float *__restrict__ eout,
            const float *__restrict__ phi, const float *__restrict__ r, IxP ix, float al,
            double w, int colour, unsigned *__restrict__ fallbacks) {
    const int n = ix.n, lg = ix.lg;
    const int half = n >> 1;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= (half << (2 * lg))) return;
    const int m = t & (half - 1);
    const int row = t >> (lg - 1);
    const int j = row & (n - 1);
    const int k = row >> lg;
    const int off = (colour ^ j ^ k) & 1;
    const int iu = 2 * m + off, ic = 2 * m + 1 - off;
    float vp[19], ve[19];
    gather(phi, ix, iu, j, k, vp);
    gather(ein, ix, iu, j, k, ve);
    unsigned fb = 0;
    const int me = ix(iu, j, k);
    eout[me] = relax_corr_cell(vp, ve, r[me], al, w, fb);
    eout[ix(ic, j, k)] = ein[ix(ic, j, k)];
    if (fb) flush_events(fallbacks, fb);
}

__global__ void __launch_bounds__(kBlock)
k_corr_restrict(const float *__restrict__ e_f, const float *__restrict__ phi_f,
                const float *__restrict__ r_f, IxP ixf, float al_f, float *__restrict__ ehat_c,
                float *__restrict__ r_c, int lgc) {
    const int nc = 1 << lgc;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= (1 << (3 * lgc))) return;
    const int I = t & (nc - 1), J = (t >> lgc) & (nc - 1), K = t >> (2 * lgc);
    float se = 0.f, sr = 0.f;
#pragma unroll
    for (int ck = 0; ck < 2; ++ck)
#pragma unroll
        for (int cj = 0; cj < 2; ++cj)
#pragma unroll
            for (int ci = 0; ci < 2; ++ci) {
                const int i = 2 * I + ci, j = 2 * J + cj, k = 2 * K + ck;
                float vp[19], ve[19];
                gather(phi_f, ixf, i, j, k, vp);
                gather(e_f, ixf, i, j, k, ve);
                const CorrTerms ct = corr_terms(vp, ve, al_f);
                se += ve[0];
                sr += r_f[ixf(i, j, k)] - ct.A;
            }
    ehat_c[t] = se * 0.125f;
    r_c[t] = sr * 0.5f; // 4 * mean: the coarse cell is twice as wide
}

__global__ void __launch_bounds__(kBlock)
k_corr_coarse_source(const float *__restrict__ ehat, const float *__restrict__ phi,
                     float *__restrict__ r, float *__restrict__ e, IxP ix, float al) {
    const int n = ix.n, lg = ix.lg;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= (1 << (3 * lg))) return;
    const int i = t & (n - 1), j = (t >> lg) & (n - 1), k = t >> (2 * lg);
    float vp[19], ve[19];
    gather(phi, ix, i, j, k, vp);
    gather(ehat, ix, i, j, k, ve);
    r[t] = corr_terms(vp, ve, al).A + r[t];
    e[t] = ve[0];
}

// e_f += P(e_c - ehat_c): trilinear prolongation of the coarse-grid
// correction (weights 3/4, 1/4 per axis towards the nearer coarse cells),
// summed for each fine cell over its 8 coarse cells in a fixed order.  One
// thread per coarse cell: the 27 coarse differences around it are loaded
// once and serve its 8 children (54 coarse loads per 8 fine cells instead of
// 16 per fine cell with a thread per fine cell); the children are updated as
// x-pairs (8-byte accesses, consecutive across the wave).
__global__ void __launch_bounds__(kBlock)
k_corr_prolong_blocks(float *__restrict__ e_f, int lgf, const float *__restrict__ e_c,
                      const float *__restrict__ ehat_c, IxP ixc) {
    const int lgc = ixc.lg, mc = ixc.n - 1;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= (1 << (3 * lgc))) return;
    const int I = t & mc, J = (t >> lgc) & mc, K = t >> (2 * lgc);
    float d[27];
#pragma unroll
    for (int z = 0; z < 3; ++z)
#pragma unroll
        for (int y = 0; y < 3; ++y)
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                const int q = ixc(I + x - 1, J + y - 1, K + z - 1);
                d[(z * 3 + y) * 3 + x] = e_c[q] - ehat_c[q];
            }
#pragma unroll
    for (int ck = 0; ck < 2; ++ck)
#pragma unroll
        for (int cj = 0; cj < 2; ++cj) {
            const int sk = ck ? 1 : -1, sj = cj ? 1 : -1;
            const size_t row = ((size_t)(((2 * K + ck) << lgf) + 2 * J + cj)) << lgf;
            float2 *p = reinterpret_cast<float2 *>(e_f + row + 2 * I);
            const float2 old = *p;
            float out[2] = {old.x, old.y};
#pragma unroll
            for (int ci = 0; ci < 2; ++ci) {
                const int si = ci ? 1 : -1;
                float acc = 0.f;
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int a = 0; a < 2; ++a) {
                            const float w =
                                (a ? 0.25f : 0.75f) * (b ? 0.25f : 0.75f) * (c ? 0.25f : 0.75f);
                            acc = fmaf(w, d[((1 + c * sk) * 3 + (1 + b * sj)) * 3 + (1 + a * si)],
                                       acc);
                        }
                out[ci] += acc;
            }
            *p = make_float2(out[0], out[1]);
        }
}

__global__ void __launch_bounds__(512)
k_corr_coarsest(float *__restrict__ e, const float *__restrict__ phi, const float *__restrict__ r,
                IxP ix, float al, double w, int sweeps, unsigned *__restrict__ fallbacks) {
    constexpr int MAXC = kCoarsestMax * kCoarsestMax * kCoarsestMax;
    __shared__ float A[MAXC], B[MAXC], Ph[MAXC];
    const int n = ix.n, lg = ix.lg;
    const int cells = 1 << (3 * lg);
    for (int q = threadIdx.x; q < cells; q += blockDim.x) {
        A[q] = e[q];
        B[q] = e[q];
        Ph[q] = phi[q];
    }
    __syncthreads();
    const int t = threadIdx.x;
    const bool active = t < cells;
    int i = 0, j = 0, k = 0;
    float rc = 0.f;
    if (active) {
        i = t & (n - 1);
        j = (t >> lg) & (n - 1);
        k = t >> (2 * lg);
        rc = r[t];
    }
    float vp[19];
    if (active) gather(Ph, ix, i, j, k, vp);
    const int mycol = (i + j + k) & 1;
    unsigned fb = 0;
    for (int sw = 0; sw < sweeps; ++sw) {
#pragma unroll
        for (int col = 0; col < 2; ++col) {
            const float *src = col ? B : A;
            float *dst = col ? A : B;
            if (active) {
                const int me = ix(i, j, k);
                float val;
                if (mycol == col) {
                    float ve[19];
                    gather(src, ix, i, j, k, ve);
                    val = relax_corr_cell(vp, ve, rc, al, w, fb);
                } else {
                    val = src[me];
                }
                dst[me] = val;
            }
            __syncthreads();
        }
    }
    if (active) e[t] = A[t];
    if (fb) flush_events(fallbacks, fb);
}

// One full red-black sweep of the correction e on a large level in one
// launch: the LDS-streamed z pipeline of the FP64 k_sweep_fused with FP32
// planes of phi (both colours, static during the sweep) and of e (old red on
// 3 planes, old black on 5, red after the red pass on 3), and the cell update
// of k_corr_half, so the result is bit for bit two k_corr_half launches.  As
// in the FP64 sweep, the rings of 5 planes (phi, old black e) have 6 slots and
// the z loop is unrolled by 6, so every LDS slot is a compile-time constant.
// With PRO the sweep starts from e plus the interpolated coarse-grid
// correction P(e_c - ehat_c), added as each old e value is loaded, with the
// arithmetic of k_corr_prolong_blocks (three coarse planes of e_c - ehat_c in
// an LDS ring E): the same bits as that launch followed by the sweep.  With ZE
// the old e is zero everywhere (the first sweep of an outer iteration) and is
// not read: the same bits as zero-filling ein first.
template <int TX, int TY, int TZ, int NT, bool PRO = false, bool ZE = false>
__global__ void __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(4))) // two workgroups per CU: at most 128 VGPRs
k_corr_sweep_fused(const float *__restrict__ ein, float *__restrict__ eout,
                   const float *__restrict__ phi, const float *__restrict__ rr_in, int lg,
                   float al, double w, unsigned *__restrict__ fallbacks,
                   const float *__restrict__ e_c = nullptr,
                   const float *__restrict__ ehat_c = nullptr) {
    constexpr int PX = TX + 4, PY = TY + 4, HX = PX / 2, PLANE = PX * PY;
    constexpr int PRE = (PLANE / 2 + NT - 1) / NT; // pairs of cells per thread
    constexpr int RED_ROW = (TX + 2) / 2, RED_CELLS = RED_ROW * (TY + 2);
    constexpr int EX = TX / 2 + 4, EY = TY / 2 + 4; // coarse cells under the plane, +-1
    static_assert(TX % 2 == 0 && TY % 2 == 0 && TX * TY / 2 == NT, "one black cell per thread");
    static_assert(RED_CELLS <= 2 * NT, "at most two red cells per thread");
    static_assert(EX * EY <= NT, "one coarse value per thread");
    static_assert(!(PRO && ZE), "the correction is added after the first sweep");
    __shared__ float F[6][2][PY][HX]; // phi, both colours, planes k-2 .. k+2
    __shared__ float ER[3][PY][HX];   // old e, red cells
    __shared__ float EB[6][PY][HX];   // old e, black cells, planes k-2 .. k+2
    __shared__ float R[3][PY][HX];    // e after the red pass, red cells
    __shared__ float E[PRO ? 3 : 1][EY * EX]; // (PRO) e_c - ehat_c under the tile

    const int n = 1 << lg, m = n - 1;
    const int ntx = n / TX;
    const int tiles = ntx * (n / TY);
    const int logical = xcd_local_id(blockIdx.x, gridDim.x);
    const int tile = logical % tiles;
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY, z0 = (logical / tiles) * TZ;
    const int tid = threadIdx.x;
    unsigned fb = 0;
    auto zoff = [&](int z) { return (size_t)(z & m) << (2 * lg); };

    // pairs of cells (columns 2j, 2j+1 of a row: one red, one black, split
    // index j), loaded 8 bytes at a time
    int pxy[PRE], pidx[PRE], ppar[PRE], eat[PRE], edy[PRE];
#pragma unroll
    for (int e = 0; e < PRE; ++e) {
        const int q = tid + e * NT;
        const int r = q / HX, j = q - r * HX;
        pxy[e] = (((y0 - 2 + r) & m) << lg) | ((x0 - 2 + 2 * j) & m);
        pidx[e] = q < PLANE / 2 ? r * HX + j : -1;
        ppar[e] = r & 1; // colour of column 2j = ppar ^ (z & 1)
        // (PRO) fine x0-2+2j+i lies in coarse cell x0/2-1+j, E column j+1;
        // the neighbour column is on the left for i = 0, on the right for
        // i = 1, the neighbour row below for an even fine row
        eat[e] = ((r >> 1) + 1) * EX + j + 1;
        edy[e] = (r & 1) ? EX : -EX;
    }
    float2 pre_p[PRE], pre_e[PRE];
    auto fetch = [&](int z) {
        const float *pp = phi + zoff(z), *pe = ein + zoff(z);
#pragma unroll
        for (int e = 0; e < PRE; ++e)
            if (pidx[e] >= 0) {
                pre_p[e] = *reinterpret_cast<const float2 *>(plane_at(pp, pxy[e]));
                if constexpr (ZE)
                    pre_e[e] = make_float2(0.f, 0.f);
                else
                    pre_e[e] = *reinterpret_cast<const float2 *>(plane_at(pe, pxy[e]));
            }
    };
    auto commit = [&](auto pl) {
        constexpr int d = decltype(pl)::d; // the plane z0 + d, z0 even
        float *f0 = &F[ring_slot(d, 6)][0][0][0], *f1 = &F[ring_slot(d, 6)][1][0][0];
        float *red = &ER[ring_slot(d, 3)][0][0], *blk = &EB[ring_slot(d, 6)][0][0];
        constexpr int zp = ring_slot(d, 2);
        const float *e0 = nullptr, *e1 = nullptr;
        if constexpr (PRO) {
            // parent plane (offset from z0 / 2) and the neighbour side
            constexpr int K = floor_half(d), sk = zp ? 1 : -1;
            e0 = E[ring_slot(K, 3)];
            e1 = E[ring_slot(K + sk, 3)];
        }
#pragma unroll
        for (int e = 0; e < PRE; ++e)
            if (pidx[e] >= 0) {
                float ev[2] = {pre_e[e].x, pre_e[e].y};
                if constexpr (PRO) {
                    // the own and the neighbour coarse row, one column to the left
                    const int er[2] = {fresh(eat[e] - 1), fresh(eat[e] + edy[e] - 1)};
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        const int edx = i ? 1 : -1;
                        float acc = 0.f;
#pragma unroll
                        for (int cz = 0; cz < 2; ++cz) {
                            const float *ep = cz ? e1 : e0;
#pragma unroll
                            for (int b = 0; b < 2; ++b)
#pragma unroll
                                for (int a = 0; a < 2; ++a) {
                                    const float wt = (a ? 0.25f : 0.75f) * (b ? 0.25f : 0.75f) *
                                                     (cz ? 0.25f : 0.75f);
                                    acc = fmaf(wt, ep[er[b] + 1 + a * edx], acc);
                                }
                        }
                        ev[i] += acc;
                    }
                }
                const bool fb1 = (ppar[e] ^ zp) != 0; // column 2j black
                const int at = fresh(pidx[e]);
                f0[at] = fb1 ? pre_p[e].y : pre_p[e].x;
                f1[at] = fb1 ? pre_p[e].x : pre_p[e].y;
                red[at] = fb1 ? ev[1] : ev[0];
                blk[at] = fb1 ? ev[0] : ev[1];
            }
    };
    // (PRO) coarse plane K of the correction: loaded into registers, then
    // stored into its E slot
    const int mc = (n >> 1) - 1, lgc = lg - 1;
    const int eq = PRO && tid < EX * EY ? tid : -1;
    const int exy = (((y0 / 2 - 2 + tid / EX) & mc) << lgc) | ((x0 / 2 - 2 + tid % EX) & mc);
    float ea = 0.f, eb = 0.f;
    auto e_load = [&](int K) {
        if (eq >= 0) {
            const int q = ((K & mc) << (2 * lgc)) | exy;
            ea = e_c[q];
            eb = ehat_c[q];
        }
    };
    auto e_store = [&](auto kpl) { // kpl: the coarse plane's offset from z0 / 2
        if (eq >= 0) E[ring_slot(decltype(kpl)::d, 3)][eq] = ea - eb;
    };

    // red cells of the halo-1 region (row rr, split index jj + 1 - p at plane
    // parity p; red_low: row rr - 1 at split index jj, the lowest LDS index
    // the stencil reads)
    int red_rr[2], red_jj[2], red_low[2];
    bool red_on[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int q = tid + e * NT;
        red_on[e] = q < RED_CELLS;
        red_rr[e] = 1 + q / RED_ROW;
        red_jj[e] = q - (red_rr[e] - 1) * RED_ROW;
        red_low[e] = (red_rr[e] - 1) * HX + red_jj[e];
    }
    auto red_sources = [&](int z, auto pl, float out[2]) {
        const float *rp = rr_in + zoff(z);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int rr = red_rr[e];
            const int p = (rr + ring_slot(decltype(pl)::d, 2)) & 1;
            const int gx = x0 - 2 + 2 * (red_jj[e] + 1 - p) + p, gy = y0 - 2 + rr;
            // in bounds also when !red_on[e]
            out[e] = *plane_at(rp, (unsigned)(((gy & m) << lg) | (gx & m)));
        }
    };
    auto red_plane = [&](auto pl, const float src[2]) {
        constexpr int d = decltype(pl)::d;
        const float *pm0 = F[ring_slot(d - 1, 6)][0][0], *pm1 = F[ring_slot(d - 1, 6)][1][0];
        const float *pc0 = F[ring_slot(d, 6)][0][0], *pc1 = F[ring_slot(d, 6)][1][0];
        const float *pp0 = F[ring_slot(d + 1, 6)][0][0], *pp1 = F[ring_slot(d + 1, 6)][1][0];
        const float *m0 = ER[ring_slot(d - 1, 3)][0], *m1 = EB[ring_slot(d - 1, 6)][0];
        const float *c0 = ER[ring_slot(d, 3)][0], *c1 = EB[ring_slot(d, 6)][0];
        const float *p0 = ER[ring_slot(d + 1, 3)][0], *p1 = EB[ring_slot(d + 1, 6)][0];
        float *rz = R[ring_slot(d, 3)][0];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            if (!red_on[e]) continue;
            // red cell at split index j = jj + 1 - p; its x neighbours at
            // a = jj + 1 and b = jj
            const int p = (red_rr[e] + ring_slot(d, 2)) & 1;
            const int lo = fresh(red_low[e]); // row rr - 1, split index b
            const int lj = lo + 1 - p;        // row rr - 1, split index j
            const float vp[19] = {
                pc0[lj + HX], pc1[lo + HX + 1], pc1[lo + HX], pc1[lj + 2 * HX], pc1[lj],
                pp1[lj + HX], pm1[lj + HX],
                pc0[lo + 2 * HX + 1], pc0[lo + 1], pc0[lo + 2 * HX], pc0[lo],
                pp0[lo + HX + 1], pm0[lo + HX + 1], pp0[lo + HX], pm0[lo + HX],
                pp0[lj + 2 * HX], pm0[lj + 2 * HX], pp0[lj], pm0[lj]};
            const float ve[19] = {
                c0[lj + HX], c1[lo + HX + 1], c1[lo + HX], c1[lj + 2 * HX], c1[lj],
                p1[lj + HX], m1[lj + HX],
                c0[lo + 2 * HX + 1], c0[lo + 1], c0[lo + 2 * HX], c0[lo],
                p0[lo + HX + 1], m0[lo + HX + 1], p0[lo + HX], m0[lo + HX],
                p0[lj + 2 * HX], m0[lj + 2 * HX], p0[lj], m0[lj]};
            rz[lj + HX] = relax_corr_cell(vp, ve, src[e], al, w, fb);
        }
    };

    const int rt = 2 + tid / (TX / 2), jt = 1 + tid % (TX / 2);
    const int yt = y0 - 2 + rt;
    const int xy_t = (yt << lg) | (x0 - 2 + 2 * jt);
    const int black_low = (rt - 1) * HX + jt; // LDS index of row rt - 1, split index jt
    auto black_source = [&](int k, auto pl) {
        const int pb = (1 + rt + ring_slot(decltype(pl)::d, 2)) & 1;
        return *plane_at(rr_in + zoff(k), (unsigned)(xy_t | pb));
    };
    auto black_and_store = [&](int k, auto pl, float sv) {
        constexpr int d = decltype(pl)::d;
        const float *pm0 = F[ring_slot(d - 1, 6)][0][0], *pm1 = F[ring_slot(d - 1, 6)][1][0];
        const float *pc0 = F[ring_slot(d, 6)][0][0], *pc1 = F[ring_slot(d, 6)][1][0];
        const float *pp0 = F[ring_slot(d + 1, 6)][0][0], *pp1 = F[ring_slot(d + 1, 6)][1][0];
        const float *rm = R[ring_slot(d - 1, 3)][0], *r0 = R[ring_slot(d, 3)][0],
                    *rp = R[ring_slot(d + 1, 3)][0];
        const float *m1 = EB[ring_slot(d - 1, 6)][0], *c1 = EB[ring_slot(d, 6)][0],
                    *p1 = EB[ring_slot(d + 1, 6)][0];
        const int pb = (1 + rt + ring_slot(d, 2)) & 1; // black cell at column 2jt + pb
        // its x neighbours at split indices a = jt + pb, b = jt + pb - 1
        const int lo = fresh(black_low); // row rt - 1, split index jt
        const int lb = lo + pb - 1;      // row rt - 1, split index b
        const float vp[19] = {
            pc1[lo + HX], pc0[lb + HX + 1], pc0[lb + HX], pc0[lo + 2 * HX], pc0[lo],
            pp0[lo + HX], pm0[lo + HX],
            pc1[lb + 2 * HX + 1], pc1[lb + 1], pc1[lb + 2 * HX], pc1[lb],
            pp1[lb + HX + 1], pm1[lb + HX + 1], pp1[lb + HX], pm1[lb + HX],
            pp1[lo + 2 * HX], pm1[lo + 2 * HX], pp1[lo], pm1[lo]};
        const float ve[19] = {
            c1[lo + HX], r0[lb + HX + 1], r0[lb + HX], r0[lo + 2 * HX], r0[lo],
            rp[lo + HX], rm[lo + HX],
            c1[lb + 2 * HX + 1], c1[lb + 1], c1[lb + 2 * HX], c1[lb],
            p1[lb + HX + 1], m1[lb + HX + 1], p1[lb + HX], m1[lb + HX],
            p1[lo + 2 * HX], m1[lo + 2 * HX], p1[lo], m1[lo]};
        const float vb = relax_corr_cell(vp, ve, sv, al, w, fb);
        const float vr = r0[lo + HX];
        float *dst = plane_at(eout + zoff(k), (unsigned)xy_t);
        dst[0] = pb ? vr : vb;
        dst[1] = pb ? vb : vr;
    };

    // the FP64 kernel's schedule: phi and old e on planes z0-2 .. z0+TZ+1;
    // with PRO the coarse planes z0/2-2 .. z0/2+TZ/2+1
    const int c0 = z0 >> 1;
    if constexpr (PRO) {
        e_load(c0 - 2);
        e_store(Plane<-2>{});
        e_load(c0 - 1);
        e_store(Plane<-1>{});
        e_load(c0);
        e_store(Plane<0>{});
        __syncthreads();
    }
    fetch(z0 - 2);
    commit(Plane<-2>{});
    fetch(z0 - 1);
    commit(Plane<-1>{});
    fetch(z0);
    commit(Plane<0>{});
    float ra[2], rb[2], ba, bb;
    red_sources(z0 - 1, Plane<-1>{}, ra);
    fetch(z0 + 1);
    if constexpr (PRO) e_load(c0 + 1);
    __syncthreads();
    red_plane(Plane<-1>{}, ra);
    __syncthreads(); // red(z0-1) has read the red slot that plane z0+1 takes
    if constexpr (PRO) {
        e_store(Plane<1>{}); // the slot of coarse plane c0-2, last used by plane z0-2
        __syncthreads();
    }
    commit(Plane<1>{});
    red_sources(z0, Plane<0>{}, ra);
    fetch(z0 + 2);
    __syncthreads();
    red_plane(Plane<0>{}, ra);
    __syncthreads();
    red_sources(z0 + 1, Plane<1>{}, ra);
    ba = black_source(z0, Plane<0>{});
    if constexpr (PRO) e_load(c0 + 2);
    // (PRO) an even step stores coarse plane k/2+2 (first needed by plane
    // k+3, in the slot of plane k/2-1, last needed by plane k) and an odd
    // step loads the next one
    auto step = [&](int k, auto pl, const float (&use_r)[2], float use_b, float (&next_r)[2],
                    float &next_b) {
        constexpr int d = decltype(pl)::d; // k = z0 + d modulo the ring period
        commit(Plane<d + 2>{}); // red e slot of plane k-1, black e and phi slots of plane k-4
        red_sources(k + 2, Plane<d + 2>{}, next_r);
        next_b = black_source(k + 1, Plane<d + 1>{});
        if constexpr (PRO && (d & 1)) e_load((k + 1) / 2 + 2);
        fetch(k + 3);
        __syncthreads();
        if constexpr (PRO && !(d & 1)) e_store(Plane<d / 2 + 2>{});
        red_plane(Plane<d + 1>{}, use_r);
        __syncthreads();
        black_and_store(k, Plane<d>{}, use_b);
    };
    static_assert(TZ % 2 == 0, "steps alternate between two register sets");
    constexpr int G = 6; // ring period: a multiple of 3 and of 6 planes
    int k = z0;
    for (int g = 0; g < TZ / G; ++g, k += G) {
        step(k, Plane<0>{}, ra, ba, rb, bb);
        step(k + 1, Plane<1>{}, rb, bb, ra, ba);
        step(k + 2, Plane<2>{}, ra, ba, rb, bb);
        step(k + 3, Plane<3>{}, rb, bb, ra, ba);
        step(k + 4, Plane<4>{}, ra, ba, rb, bb);
        step(k + 5, Plane<5>{}, rb, bb, ra, ba);
    }
    // the last TZ mod 6 planes
    if constexpr (TZ % G >= 2) {
        step(k, Plane<0>{}, ra, ba, rb, bb);
        step(k + 1, Plane<1>{}, rb, bb, ra, ba);
    }
    if constexpr (TZ % G >= 4) {
        step(k + 2, Plane<2>{}, ra, ba, rb, bb);
        step(k + 3, Plane<3>{}, rb, bb, ra, ba);
    }
    if (fb) flush_events(fallbacks, fb);
}

// Restriction of the correction equation on a large level through LDS: phi
// and e planes (one-cell halo) stream along z as in the FP64 k_restrict_tiled,
// one thread per coarse cell finishing its 4 children per fine plane, with
// k_corr_restrict's expressions and summation order (same bits).
template <int TX, int TY>
__global__ void __launch_bounds__(kBlock)
k_corr_restrict_tiled(const float *__restrict__ e_f, const float *__restrict__ phi_f,
                      const float *__restrict__ r_f, int lg, int tz, float al_f,
                      float *__restrict__ ehat_c, float *__restrict__ r_c) {
    constexpr int PX = TX + 2, PY = TY + 2, PLANE = PX * PY;
    constexpr int PRE = (PLANE + kBlock - 1) / kBlock;
    static_assert(TX * TY == 4 * kBlock, "one coarse cell per thread");
    __shared__ float PP[4][PLANE], PE[4][PLANE];
    const int n = 1 << lg, m = n - 1, lgc = lg - 1;
    const int ntx = n / TX;
    const int tiles = ntx * (n / TY);
    const int logical = xcd_local_id(blockIdx.x, gridDim.x);
    const int tile = logical % tiles;
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY, z0 = (logical / tiles) * tz;
    const int tid = threadIdx.x;
    int pq[PRE], pxy[PRE];
#pragma unroll
    for (int e = 0; e < PRE; ++e) {
        const int q = tid + e * kBlock;
        pq[e] = q < PLANE ? q : -1;
        const int yy = q / PX, xx = q - yy * PX;
        pxy[e] = (((y0 - 1 + yy) & m) << lg) | ((x0 - 1 + xx) & m);
    }
    float pre_p[PRE], pre_e[PRE];
    auto fetch = [&](int z) {
        const int zo = (z & m) << (2 * lg);
#pragma unroll
        for (int e = 0; e < PRE; ++e)
            if (pq[e] >= 0) {
                pre_p[e] = phi_f[zo | pxy[e]];
                pre_e[e] = e_f[zo | pxy[e]];
            }
    };
    auto commit = [&](int z) {
#pragma unroll
        for (int e = 0; e < PRE; ++e)
            if (pq[e] >= 0) {
                PP[z & 3][pq[e]] = pre_p[e];
                PE[z & 3][pq[e]] = pre_e[e];
            }
    };
    const int ic = tid % (TX / 2), jc = tid / (TX / 2);
    float se = 0.f, sr = 0.f;
    fetch(z0 - 1);
    commit(z0 - 1);
    fetch(z0);
    commit(z0);
    fetch(z0 + 1);
    for (int k = z0; k < z0 + tz; ++k) {
        commit(k + 1); // slot of plane k-3, last read at step k-2
        if (k + 2 <= z0 + tz) fetch(k + 2);
        __syncthreads();
        const float(*fm)[PX] = reinterpret_cast<const float(*)[PX]>(PP[(k - 1) & 3]);
        const float(*f0)[PX] = reinterpret_cast<const float(*)[PX]>(PP[k & 3]);
        const float(*fp)[PX] = reinterpret_cast<const float(*)[PX]>(PP[(k + 1) & 3]);
        const float(*em)[PX] = reinterpret_cast<const float(*)[PX]>(PE[(k - 1) & 3]);
        const float(*e0)[PX] = reinterpret_cast<const float(*)[PX]>(PE[k & 3]);
        const float(*ep)[PX] = reinterpret_cast<const float(*)[PX]>(PE[(k + 1) & 3]);
        if ((k & 1) == 0) {
            se = 0.f;
            sr = 0.f;
        }
#pragma unroll
        for (int cj = 0; cj < 2; ++cj)
#pragma unroll
            for (int ci = 0; ci < 2; ++ci) {
                const int xt = 2 * ic + ci, yt = 2 * jc + cj;
                const int rr = yt + 1, c = xt + 1;
                const float vp[19] = {
                    f0[rr][c], f0[rr][c + 1], f0[rr][c - 1], f0[rr + 1][c], f0[rr - 1][c],
                    fp[rr][c], fm[rr][c],
                    f0[rr + 1][c + 1], f0[rr - 1][c + 1], f0[rr + 1][c - 1], f0[rr - 1][c - 1],
                    fp[rr][c + 1], fm[rr][c + 1], fp[rr][c - 1], fm[rr][c - 1],
                    fp[rr + 1][c], fm[rr + 1][c], fp[rr - 1][c], fm[rr - 1][c]};
                const float ve[19] = {
                    e0[rr][c], e0[rr][c + 1], e0[rr][c - 1], e0[rr + 1][c], e0[rr - 1][c],
                    ep[rr][c], em[rr][c],
                    e0[rr + 1][c + 1], e0[rr - 1][c + 1], e0[rr + 1][c - 1], e0[rr - 1][c - 1],
                    ep[rr][c + 1], em[rr][c + 1], ep[rr][c - 1], em[rr][c - 1],
                    ep[rr + 1][c], em[rr + 1][c], ep[rr - 1][c], em[rr - 1][c]};
                const CorrTerms ct = corr_terms(vp, ve, al_f);
                const int g = ((k << lg | (y0 + yt)) << lg) | (x0 + xt);
                se += ve[0];
                sr += r_f[g] - ct.A;
            }
        if (k & 1) {
            const int q = (((k >> 1) << lgc | (y0 / 2 + jc)) << lgc) | (x0 / 2 + ic);
            ehat_c[q] = se * 0.125f;
            r_c[q] = sr * 0.5f; // 4 * mean: the coarse cell is twice as wide
        }
    }
}

inline unsigned nblocks(size_t total) { return (unsigned)((total + kBlock - 1) / kBlock); }

inline IxP ixp(int n, int lg) { return IxP{n, lg, n + 2}; }

} // namespace

void launch_residual_to32(const Level &L, float *r32, double *partials, hipStream_t st) {
    if (residual_tiled_ok(L)) {
        launch_residual_tiled_to32(L, r32, partials, st);
        return;
    }
    k_residual_to32<<<kReduceBlocks, kBlock, 0, st>>>(L.phi, L.s, ixp(L.n, L.lg), L.alpha, r32,
                                                      partials);
}

void launch_to32(const double *a, float *b, size_t count, hipStream_t st) {
    k_to32<<<nblocks(count), kBlock, 0, st>>>(a, b, count);
}

void launch_avg32(const Level32 &F, const Level32 &C, hipStream_t st) {
    k_avg32<<<nblocks(C.cells()), kBlock, 0, st>>>(F.phi, F.n, C.phi, C.lg);
}

void launch_add32(double *phi, const float *e, size_t count, hipStream_t st) {
    k_add32<<<nblocks(count), kBlock, 0, st>>>(phi, e, count);
}

void launch_add_to32(double *phi, const float *e, float *phi32, size_t count, hipStream_t st) {
    k_add_to32<<<nblocks(count), kBlock, 0, st>>>(phi, e, phi32, count);
}

void launch_fill32(float *a, size_t count, float v, hipStream_t st) {
    k_fill32<<<nblocks(count), kBlock, 0, st>>>(a, count, v);
}

void launch_corr_half(const Level32 &L, const float *ein, float *eout, int colour,
                      unsigned *fallbacks, hipStream_t st) {
    k_corr_half<<<nblocks(L.cells() / 2), kBlock, 0, st>>>(ein, eout, L.phi, L.r, ixp(L.n, L.lg),
                                                          (float)L.alpha, L.omega, colour,
                                                          fallbacks);
}

bool corr_fused_ok(const Level32 &L) { return L.n >= 128; }

template <bool PRO, bool ZE>
void corr_sweep_fused(const Level32 &L, const float *ein, float *eout, unsigned *fallbacks,
                      const float *e_c, const float *ehat_c, hipStream_t st) {
    constexpr int TX = 64, TY = 16, NT = 512;
    const int tiles = (L.n / TX) * (L.n / TY);
    if (L.n >= 256) {
        constexpr int TZ = 32;
        k_corr_sweep_fused<TX, TY, TZ, NT, PRO, ZE><<<tiles * (L.n / TZ), NT, 0, st>>>(
            ein, eout, L.phi, L.r, L.lg, (float)L.alpha, L.omega, fallbacks, e_c, ehat_c);
    } else {
        constexpr int TZ = 8;
        k_corr_sweep_fused<TX, TY, TZ, NT, PRO, ZE><<<tiles * (L.n / TZ), NT, 0, st>>>(
            ein, eout, L.phi, L.r, L.lg, (float)L.alpha, L.omega, fallbacks, e_c, ehat_c);
    }
}

void launch_corr_sweep_fused(const Level32 &L, const float *ein, float *eout,
                             unsigned *fallbacks, hipStream_t st) {
    corr_sweep_fused<false, false>(L, ein, eout, fallbacks, nullptr, nullptr, st);
}

void launch_corr_sweep_fused_from_zero(const Level32 &L, float *eout, unsigned *fallbacks,
                                       hipStream_t st) {
    corr_sweep_fused<false, true>(L, nullptr, eout, fallbacks, nullptr, nullptr, st);
}

void launch_corr_sweep_fused_prolong(const Level32 &L, const Level32 &C, const float *ein,
                                     float *eout, unsigned *fallbacks, hipStream_t st) {
    corr_sweep_fused<true, false>(L, ein, eout, fallbacks, C.e, C.ehat, st);
}

void launch_corr_restrict(const Level32 &F, const Level32 &C, bool tiled, hipStream_t st) {
    if (tiled && F.n >= 128) {
        constexpr int TX = 64, TY = 16;
        const int tz = F.n >= 256 ? 8 : 4;
        const int tiles = (F.n / TX) * (F.n / TY);
        k_corr_restrict_tiled<TX, TY><<<tiles * (F.n / tz), kBlock, 0, st>>>(
            F.e, F.phi, F.r, F.lg, tz, (float)F.alpha, C.ehat, C.r);
        return;
    }
    k_corr_restrict<<<nblocks(C.cells()), kBlock, 0, st>>>(F.e, F.phi, F.r, ixp(F.n, F.lg),
                                                          (float)F.alpha, C.ehat, C.r, C.lg);
}

void launch_corr_coarse_source(const Level32 &C, hipStream_t st) {
    k_corr_coarse_source<<<nblocks(C.cells()), kBlock, 0, st>>>(C.ehat, C.phi, C.r, C.e,
                                                               ixp(C.n, C.lg), (float)C.alpha);
}

void launch_corr_prolong(const Level32 &F, const Level32 &C, hipStream_t st) {
    k_corr_prolong_blocks<<<nblocks(C.cells()), kBlock, 0, st>>>(F.e, F.lg, C.e, C.ehat,
                                                                ixp(C.n, C.lg));
}

void launch_corr_coarsest(const Level32 &L, int sweeps, unsigned *fallbacks, hipStream_t st) {
    const int threads = L.cells() < 64 ? 64 : (int)L.cells();
    k_corr_coarsest<<<1, threads, 0, st>>>(L.e, L.phi, L.r, ixp(L.n, L.lg), (float)L.alpha,
                                           L.omega, sweeps, fallbacks);
}

} // namespace ndgp
