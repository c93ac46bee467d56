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

#include "ndgp_device.h"

namespace ndgp {
namespace {

using namespace dev;

// ------------------------------------------------------------------------
// kernels

template <bool PER>
__global__ void __launch_bounds__(kBlock)
k_smooth_half(const double *__restrict__ pin, double *__restrict__ pout,
              const double *__restrict__ s, Ix<PER> ix, double al, double w, int colour,
              unsigned *__restrict__ fallbacks, const double *__restrict__ hat, int dyn_bc,
              const unsigned char *__restrict__ mask,
              const unsigned char *__restrict__ active) {
    // a block whose cells of this colour are all held has nothing to do: both
    // ping-pong arrays already hold their (fixed) values
    if (active && !active[colour * gridDim.x + blockIdx.x]) return;
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
    unsigned fb = 0;
    double un;
    if (mask && !mask[((k << lg) + j) * n + iu]) { // held (cell-wise truncation)
        un = pin[ix(iu, j, k)];
    } else {
        double v[19];
        gather(pin, ix, iu, j, k, v);
        un = relax_cell(v, s[((k << lg) + j) * n + iu], al, w, fb);
    }
    const double uc = pin[ix(ic, j, k)];
    pout[ix(iu, j, k)] = un;
    pout[ix(ic, j, k)] = uc;
    if (!PER && dyn_bc) {
        write_owned_ghosts(pout, hat, ix, iu, j, k, un);
        write_owned_ghosts(pout, hat, ix, ic, j, k, uc);
    }
    if (fb) flush_events(fallbacks, fb);
}

// One full red-black sweep of a periodic level in one launch, with the same
// semantics as two k_smooth_half launches (colour 0 from pin, then colour 1
// from that result; same-colour neighbours always at their pass-start
// values), bit for bit.  With PRO the sweep starts from pin plus the
// interpolated coarse-grid correction P(phi_c - hat_c), added as each old
// value is loaded, with the arithmetic of k_prolong8: the same bits as a
// k_prolong8 launch followed by the sweep, without the extra pass over HBM.
//
// A workgroup owns a TX x TY column of the x-y plane over TZ planes and
// streams along z.  LDS keeps every plane split by colour, so that lanes
// working on consecutive cells of one colour touch consecutive words (no
// bank conflicts):
//   PR, PB: the old field's red and black cells, tile + 2-cell halo, red on
//           planes k .. k+2 (3 slots), black on planes k-2 .. k+2 (6 slots);
//   R:  red cells after the red pass, planes k-1 .. k+1 (3 slots);
//   E:  (PRO) the coarse correction under the tile, three coarse planes.
// A plane's slot is its offset from the chunk's first plane modulo the ring
// size; the z loop is unrolled by 6 (a multiple of every ring), so the slots
// are constants: an LDS address is a per-thread base plus an immediate.
// Step k relaxes the red cells of plane k+1 over the tile plus a 1-cell halo
// (the black cells at the tile's edge need them), then the black cells of
// plane k over the tile (red neighbours from R, black ones from PB), and
// writes plane k.  The next old plane is read into registers meanwhile.  HBM
// sees each old value and each source value once and each new value once:
// 24 bytes per cell and sweep (PRO: + 2 x 8 bytes per coarse cell); tiles
// are ordered per XCD so that their halo lines are shared in L2.
//
// PER = false: the finest level of a refinement, in its padded layout with a
// fixed ghost shell (no correction on load).  Cells of the halo that lie in
// the shell keep their value instead of being relaxed, loads beyond the shell
// (needed only to relax such cells) are clamped to it, and pairs are moved
// as two 8-byte values (padded rows do not keep a pair 16-byte aligned); the
// shell itself is never written (both ping-pong arrays hold it).  With a
// mask (cell-wise truncation) a held cell keeps its value like a shell cell,
// and a workgroup whose own cells are all held (tile_on 0) returns at once:
// both ping-pong arrays hold the held values, so there is nothing to write.
template <int TX, int TY, int TZ, int NT, bool PRO, bool PER = true>
__global__ void __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu(4))) // two workgroups per CU: at most 128 VGPRs
k_sweep_fused(const double *__restrict__ pin, double *__restrict__ pout,
              const double *__restrict__ s, int lg, double al, double w,
              unsigned *__restrict__ fallbacks, const double *__restrict__ phi_c,
              const double *__restrict__ hat_c, const unsigned char *__restrict__ mask,
              const unsigned char *__restrict__ tile_on) {
    constexpr int PX = TX + 4, PY = TY + 4;   // plane with halo 2
    constexpr int HX = PX / 2;                // cells of one colour per row
    constexpr int PLANE = PX * PY;
    constexpr int RED_ROW = (TX + 2) / 2;     // red cells per row of the halo-1 region
    constexpr int RED_CELLS = RED_ROW * (TY + 2);
    constexpr int EX = TX / 2 + 4, EY = TY / 2 + 4; // coarse cells under the plane, +-1
    static_assert(TX % 2 == 0 && TY % 2 == 0 && TX * TY / 2 == NT, "one black cell per thread");
    static_assert(RED_CELLS <= 2 * NT, "at most two red cells per thread");
    static_assert(EX * EY <= NT, "one coarse value per thread");
    static_assert(PER || !PRO, "refinements add the coarse correction in its own launch");
    __shared__ double PR[3][PY][HX];
    __shared__ double PB[6][PY][HX];
    __shared__ double R[3][PY][HX];
    __shared__ double E[PRO ? 3 : 1][EY * EX];

    const int n = 1 << lg, m = n - 1;
    const int ntx = n / TX;
    const int tiles = ntx * (n / TY);
    const int logical = xcd_local_id(blockIdx.x, gridDim.x); // tile fastest, then z-chunk
    const int tile = logical % tiles;
    const int x0 = (tile % ntx) * TX;
    const int y0 = (tile / ntx) * TY;
    const int z0 = (logical / tiles) * TZ;
    const int tid = threadIdx.x;
    unsigned fb = 0;
    if constexpr (!PER)
        if (tile_on && !tile_on[logical]) return;

    // padded layout (PER = false): row pitch n + 2, cell (x, y, z) at
    // ((z + 1) pitch + y + 1) pitch + x + 1, every coordinate clamped to [-1, n]
    const int pitch = n + 2;
    auto cl = [&](int v) { return v < -1 ? -1 : (v > n ? n : v); };
    auto zoff = [&](int z) {
        if constexpr (PER) return (size_t)(z & m) << (2 * lg);
        else return (size_t)(cl(z) + 1) * pitch * pitch;
    };
    // sources (and mask): plane of z and the offset of (x, y) in it, clamped
    // inside the level where PER = false
    auto inside = [&](int v) { return v < 0 ? 0 : (v > m ? m : v); };
    auto splane = [&](int z) {
        if constexpr (PER) return (size_t)(z & m) << (2 * lg);
        else return (size_t)inside(z) << (2 * lg);
    };
    auto sxy = [&](int x, int y) {
        if constexpr (PER) return (unsigned)(((y & m) << lg) | (x & m));
        else return (unsigned)((inside(y) << lg) | inside(x));
    };
    // a cell of the ghost shell: kept, not relaxed
    auto ghost = [&](int x, int y, int z) {
        if constexpr (PER) return false;
        else return (unsigned)x >= (unsigned)n || (unsigned)y >= (unsigned)n ||
                    (unsigned)z >= (unsigned)n;
    };
    // a held cell (mask 0, loaded with its source a step ahead): kept
    auto held_at = [&](size_t plane, unsigned at) {
        if constexpr (PER) return false;
        else return mask != nullptr && mask[plane + at] == 0;
    };

    // this thread's share of a plane, in 16-byte pairs of cells (columns 2j,
    // 2j+1 of a row: one red, one black, both at split index j): global x-y
    // offset, LDS split position, colour of the pair's first cell, and (PRO)
    // their coarse cell in E with the step towards the neighbour row
    constexpr int PAIRS = PLANE / 2;
    constexpr int PRE2 = (PAIRS + NT - 1) / NT;
    int pxy[PRE2], pxy1[PRE2], pidx[PRE2], ppar[PRE2], eat[PRE2], edy[PRE2];
#pragma unroll
    for (int e = 0; e < PRE2; ++e) {
        const int q = tid + e * NT;
        const int r = q / HX, j = q - r * HX;
        if constexpr (PER) {
            pxy[e] = (((y0 - 2 + r) & m) << lg) | ((x0 - 2 + 2 * j) & m);
            pxy1[e] = 0;
        } else {
            const int y = cl(y0 - 2 + r), x = x0 - 2 + 2 * j;
            pxy[e] = (y + 1) * pitch + cl(x) + 1;
            pxy1[e] = (y + 1) * pitch + cl(x + 1) + 1;
        }
        pidx[e] = q < PAIRS ? r * HX + j : -1;
        ppar[e] = r & 1; // colour of column 2j = ppar ^ (z & 1)  (x0, y0 even)
        // fine x0-2+2j+i lies in coarse cell x0/2-1+j, E column j+1; the
        // neighbour column is on the left for i = 0, on the right for i = 1
        eat[e] = ((r >> 1) + 1) * EX + j + 1;
        edy[e] = (r & 1) ? EX : -EX;
    }
    double2 pre[PRE2];
    auto fetch = [&](int z) {
        const double *plane = pin + zoff(z);
#pragma unroll
        for (int e = 0; e < PRE2; ++e)
            if (pidx[e] >= 0) {
                if constexpr (PER) {
                    pre[e] = *reinterpret_cast<const double2 *>(plane_at(plane, pxy[e]));
                } else {
                    pre[e].x = *plane_at(plane, pxy[e]);
                    pre[e].y = *plane_at(plane, pxy1[e]);
                }
            }
    };
    auto commit = [&](int z, auto pl) {
        constexpr int d = decltype(pl)::d; // z = z0 + d, z0 even
        double *red = &PR[ring_slot(d, 3)][0][0], *blk = &PB[ring_slot(d, 6)][0][0];
        constexpr int zp = ring_slot(d, 2);
        const double *e0 = nullptr, *e1 = nullptr;
        if constexpr (PRO) {
            // parent plane (offset from z0 / 2) and the neighbour side
            constexpr int K = floor_half(d), sk = zp ? 1 : -1;
            e0 = E[ring_slot(K, 3)];
            e1 = E[ring_slot(K + sk, 3)];
        }
#pragma unroll
        for (int e = 0; e < PRE2; ++e)
            if (pidx[e] >= 0) {
                double v[2] = {pre[e].x, pre[e].y};
                if constexpr (PRO) {
                    // the own and the neighbour coarse row, one column to the left
                    const int er[2] = {fresh(eat[e] - 1), fresh(eat[e] + edy[e] - 1)};
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        const int edx = i ? 1 : -1;
                        double acc = 0.0;
#pragma unroll
                        for (int cz = 0; cz < 2; ++cz) {
                            const double *ep = cz ? e1 : e0;
#pragma unroll
                            for (int b = 0; b < 2; ++b)
#pragma unroll
                                for (int a = 0; a < 2; ++a) {
                                    const double w = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (cz ? 0.25 : 0.75);
                                    acc = fma(w, ep[er[b] + 1 + a * edx], acc);
                                }
                        }
                        v[i] = v[i] + acc;
                    }
                }
                const bool first_black = (ppar[e] ^ zp) != 0;
                const int at = fresh(pidx[e]);
                red[at] = first_black ? v[1] : v[0];
                blk[at] = first_black ? v[0] : v[1];
            }
    };
    // (PRO) coarse plane K of the correction: loaded into registers, then
    // stored into its E slot
    const int nc = n >> 1, mc = nc - 1, lgc = lg - 1;
    const int eq = PRO && tid < EX * EY ? tid : -1;
    const int exy = (((y0 / 2 - 2 + tid / EX) & mc) << lgc) | ((x0 / 2 - 2 + tid % EX) & mc);
    double ea = 0.0, eb = 0.0;
    auto e_load = [&](int K) {
        if (eq >= 0) {
            const int q = ((K & mc) << (2 * lgc)) | exy;
            ea = phi_c[q];
            eb = hat_c[q];
        }
    };
    auto e_store = [&](auto kpl) { // kpl: the coarse plane's offset from z0 / 2
        if (eq >= 0) E[ring_slot(decltype(kpl)::d, 3)][eq] = ea - eb;
    };

    // red cells of the halo-1 region: thread slot e covers q = tid + e * NT
    // (row rr, split index jj + 1 - p at plane parity p; red_low: row rr - 1
    // at split index jj, the lowest LDS index its stencil reads)
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
    // the sources of plane z's red cells, loaded a step ahead of their use
    auto red_sources = [&](int z, auto pl, double out[2], bool hold[2]) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int rr = red_rr[e];
            const int p = (rr + ring_slot(decltype(pl)::d, 2)) & 1;
            const int gx = x0 - 2 + 2 * (red_jj[e] + 1 - p) + p, gy = y0 - 2 + rr;
            const size_t plane = splane(z);
            const unsigned at = sxy(gx, gy); // in bounds also when !red_on[e]
            out[e] = *plane_at(s + plane, at);
            hold[e] = held_at(plane, at);
        }
    };
    // red cells of plane z over the tile + 1-cell halo -> R(z)
    auto red_plane = [&](int z, auto pl, const double src[2], const bool hold[2]) {
        constexpr int d = decltype(pl)::d;
        const double *m0 = PR[ring_slot(d - 1, 3)][0], *m1 = PB[ring_slot(d - 1, 6)][0];
        const double *c0 = PR[ring_slot(d, 3)][0], *c1 = PB[ring_slot(d, 6)][0];
        const double *p0 = PR[ring_slot(d + 1, 3)][0], *p1 = PB[ring_slot(d + 1, 6)][0];
        double *rz = R[ring_slot(d, 3)][0];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            if (!red_on[e]) continue;
            // red cell at column c = 2j + p, j = jj + 1 - p in [1, PX-2];
            // columns c+1, c-1 at split indices a = jj + 1, b = jj
            const int p = (red_rr[e] + ring_slot(d, 2)) & 1;
            const int lo = fresh(red_low[e]); // row rr - 1, split index b
            const int lj = lo + 1 - p;        // row rr - 1, split index j
            const double v[19] = {
                c0[lj + HX], c1[lo + HX + 1], c1[lo + HX], c1[lj + 2 * HX], c1[lj],
                p1[lj + HX], m1[lj + HX],
                c0[lo + 2 * HX + 1], c0[lo + 1], c0[lo + 2 * HX], c0[lo],
                p0[lo + HX + 1], m0[lo + HX + 1], p0[lo + HX], m0[lo + HX],
                p0[lj + 2 * HX], m0[lj + 2 * HX], p0[lj], m0[lj]};
            if constexpr (PER) {
                rz[lj + HX] = relax_cell(v, src[e], al, w, fb);
            } else {
                const int gx = x0 - 2 + 2 * (red_jj[e] + 1 - p) + p, gy = y0 - 2 + red_rr[e];
                rz[lj + HX] = ghost(gx, gy, z) || hold[e] ? v[0] : relax_cell(v, src[e], al, w, fb);
            }
        }
    };

    // this thread's black cell: row rt, split index jt (pair of columns 2jt, 2jt+1)
    const int rt = 2 + tid / (TX / 2), jt = 1 + tid % (TX / 2);
    const int yt = y0 - 2 + rt;
    const int xy_t = (yt << lg) | (x0 - 2 + 2 * jt);
    const int pxy_t = (yt + 1) * pitch + x0 - 2 + 2 * jt + 1; // padded (PER = false)
    const int black_low = (rt - 1) * HX + jt; // LDS index of row rt - 1, split index jt
    auto black_source = [&](int k, auto pl, bool &hold) {
        const int pb = (1 + rt + ring_slot(decltype(pl)::d, 2)) & 1;
        if constexpr (PER) {
            hold = false;
            return *plane_at(s + splane(k), (unsigned)(xy_t | pb));
        } else {
            const size_t plane = (size_t)(k < n ? k : m) << (2 * lg); // plane n: loaded, unused
            const unsigned at = (unsigned)(xy_t + pb);
            hold = held_at(plane, at);
            return *plane_at(s + plane, at);
        }
    };
    auto black_and_store = [&](int k, auto pl, double sv, bool hold) {
        constexpr int d = decltype(pl)::d;
        const double *rm = R[ring_slot(d - 1, 3)][0], *r0 = R[ring_slot(d, 3)][0],
                     *rp = R[ring_slot(d + 1, 3)][0];
        const double *m1 = PB[ring_slot(d - 1, 6)][0], *c1 = PB[ring_slot(d, 6)][0],
                     *p1 = PB[ring_slot(d + 1, 6)][0];
        const int pb = (1 + rt + ring_slot(d, 2)) & 1; // black cell at column 2jt + pb
        // columns 2jt + pb +- 1 at split indices a = jt + pb, b = jt + pb - 1
        const int lo = fresh(black_low); // row rt - 1, split index jt
        const int lb = lo + pb - 1;      // row rt - 1, split index b
        const double v[19] = {
            c1[lo + HX], r0[lb + HX + 1], r0[lb + HX], r0[lo + 2 * HX], r0[lo],
            rp[lo + HX], rm[lo + HX],
            c1[lb + 2 * HX + 1], c1[lb + 1], c1[lb + 2 * HX], c1[lb],
            p1[lb + HX + 1], m1[lb + HX + 1], p1[lb + HX], m1[lb + HX],
            p1[lo + 2 * HX], m1[lo + 2 * HX], p1[lo], m1[lo]};
        const double vb = hold ? v[0] : relax_cell(v, sv, al, w, fb);
        const double vr = r0[lo + HX]; // the red cell of the pair, column 2jt + 1 - pb
        // the pair as one 16-byte non-temporal store: the new field is not
        // read again in this sweep, so it need not displace the halo lines
        // that neighbouring tiles read from L2 (3% faster at 256^3)
        typedef double pair_t __attribute__((ext_vector_type(2)));
        pair_t o;
        o.x = pb ? vr : vb;
        o.y = pb ? vb : vr;
        if constexpr (PER) {
            __builtin_nontemporal_store(o, reinterpret_cast<pair_t *>(plane_at(pout + zoff(k),
                                                                                (unsigned)xy_t)));
        } else {
            double *q = plane_at(pout + zoff(k), (unsigned)pxy_t);
            __builtin_nontemporal_store(o.x, q);
            __builtin_nontemporal_store(o.y, q + 1);
        }
    };

    // Planes needed: old z0-2 .. z0+TZ+1 (black) / z0-1 .. z0+TZ+1 (red), R
    // z0-1 .. z0+TZ; with PRO the coarse planes z0/2-2 .. z0/2+TZ/2+1.  Old
    // plane z needs coarse planes z/2-1, z/2 (z even) or (z-1)/2, (z+1)/2.
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
    commit(z0 - 2, Plane<-2>{});
    fetch(z0 - 1);
    commit(z0 - 1, Plane<-1>{});
    fetch(z0);
    commit(z0, Plane<0>{});
    double ra[2], rb[2], ba, bb;
    bool ha[2], hb[2], hba, hbb;
    red_sources(z0 - 1, Plane<-1>{}, ra, ha);
    fetch(z0 + 1);
    if constexpr (PRO) e_load(c0 + 1);
    __syncthreads();
    red_plane(z0 - 1, Plane<-1>{}, ra, ha);
    __syncthreads(); // red(z0-1) has read the red slot that plane z0+1 takes
    if constexpr (PRO) {
        e_store(Plane<1>{}); // the slot of coarse plane c0-2, last used by plane z0-2
        __syncthreads();
    }
    commit(z0 + 1, Plane<1>{});
    red_sources(z0, Plane<0>{}, ra, ha);
    fetch(z0 + 2);
    __syncthreads();
    red_plane(z0, Plane<0>{}, ra, ha);
    __syncthreads(); // red(z0) has read the red slot that plane z0+2 takes
    red_sources(z0 + 1, Plane<1>{}, ra, ha);
    ba = black_source(z0, Plane<0>{}, hba);
    if constexpr (PRO) e_load(c0 + 2);
    // one step: red(k+1), black(k); loads the sources of red(k+2), black(k+1)
    // and the field of plane k+3 (on the last step one plane past the ones
    // used: in bounds, never committed).  With PRO an even step stores
    // coarse plane k/2+2 (first needed by plane k+3, in the slot of plane
    // k/2-1, last needed by plane k) and an odd step loads the next one.
    auto step = [&](int k, auto pl, const double (&use_r)[2], const bool (&use_rh)[2],
                    double use_b, bool use_bh, double (&next_r)[2], bool (&next_rh)[2],
                    double &next_b, bool &next_bh) {
        constexpr int d = decltype(pl)::d; // k = z0 + d modulo the ring period
        commit(k + 2, Plane<d + 2>{}); // red slot of plane k-1 (last read by red(k)), black of k-4
        red_sources(k + 2, Plane<d + 2>{}, next_r, next_rh);
        next_b = black_source(k + 1, Plane<d + 1>{}, next_bh);
        if constexpr (PRO && (d & 1)) e_load((k + 1) / 2 + 2);
        fetch(k + 3);
        __syncthreads();
        if constexpr (PRO && !(d & 1)) e_store(Plane<d / 2 + 2>{});
        // writes the R slot of plane k-2, last read by black(k-1)
        red_plane(k + 1, Plane<d + 1>{}, use_r, use_rh);
        __syncthreads();
        black_and_store(k, Plane<d>{}, use_b, use_bh);
    };
    static_assert(TZ % 2 == 0, "steps alternate between two register sets");
    constexpr int G = 6; // ring period: a multiple of 3 and of 6 planes
    int k = z0;
    for (int g = 0; g < TZ / G; ++g, k += G) {
        step(k, Plane<0>{}, ra, ha, ba, hba, rb, hb, bb, hbb);
        step(k + 1, Plane<1>{}, rb, hb, bb, hbb, ra, ha, ba, hba);
        step(k + 2, Plane<2>{}, ra, ha, ba, hba, rb, hb, bb, hbb);
        step(k + 3, Plane<3>{}, rb, hb, bb, hbb, ra, ha, ba, hba);
        step(k + 4, Plane<4>{}, ra, ha, ba, hba, rb, hb, bb, hbb);
        step(k + 5, Plane<5>{}, rb, hb, bb, hbb, ra, ha, ba, hba);
    }
    // the last TZ mod 6 planes
    if constexpr (TZ % G >= 2) {
        step(k, Plane<0>{}, ra, ha, ba, hba, rb, hb, bb, hbb);
        step(k + 1, Plane<1>{}, rb, hb, bb, hbb, ra, ha, ba, hba);
    }
    if constexpr (TZ % G >= 4) {
        step(k + 2, Plane<2>{}, ra, ha, ba, hba, rb, hb, bb, hbb);
        step(k + 3, Plane<3>{}, rb, hb, bb, hbb, ra, ha, ba, hba);
    }
    if (fb) flush_events(fallbacks, fb);
}

// FAS restriction with the residual on a large periodic level, through LDS:
// a workgroup streams a TX x TY fine column along z over tz planes (tz even)
// as k_residual_tiled does, and each thread owns one coarse cell of the
// tile, whose 4 children in a fine plane it finishes per step.  Per coarse
// cell the sums run over the children in restrict_cell's order, so the
// coarse values are bit for bit k_restrict_residual's.
template <int TX, int TY>
__global__ void __launch_bounds__(kBlock)
k_restrict_tiled(const double *__restrict__ phi, const double *__restrict__ s, int lg, int tz,
                 double al, double *__restrict__ hat_c, double *__restrict__ s_c) {
    constexpr int PX = TX + 2, PY = TY + 2, PLANE = PX * PY;
    constexpr int PRE = (PLANE + kBlock - 1) / kBlock;
    static_assert(TX * TY == 4 * kBlock, "one coarse cell per thread");
    __shared__ double P[4][PLANE];
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
    double pre[PRE];
    auto fetch = [&](int z) {
        const int zo = (z & m) << (2 * lg);
#pragma unroll
        for (int e = 0; e < PRE; ++e)
            if (pq[e] >= 0) pre[e] = phi[zo | pxy[e]];
    };
    auto commit = [&](int z) {
        double *dst = P[z & 3];
#pragma unroll
        for (int e = 0; e < PRE; ++e)
            if (pq[e] >= 0) dst[pq[e]] = pre[e];
    };
    // this thread's coarse cell: (x0/2 + ic, y0/2 + jc); children 2ic + ci, 2jc + cj
    const int ic = tid % (TX / 2), jc = tid / (TX / 2);
    double sphi = 0.0, sr = 0.0;
    fetch(z0 - 1);
    commit(z0 - 1);
    fetch(z0);
    commit(z0);
    fetch(z0 + 1);
    for (int k = z0; k < z0 + tz; ++k) {
        commit(k + 1); // slot of plane k-3, last read at step k-2
        if (k + 2 <= z0 + tz) fetch(k + 2);
        __syncthreads();
        const double(*pm)[PX] = reinterpret_cast<const double(*)[PX]>(P[(k - 1) & 3]);
        const double(*p0)[PX] = reinterpret_cast<const double(*)[PX]>(P[k & 3]);
        const double(*pp)[PX] = reinterpret_cast<const double(*)[PX]>(P[(k + 1) & 3]);
        if ((k & 1) == 0) {
            sphi = 0.0;
            sr = 0.0;
        }
#pragma unroll
        for (int cj = 0; cj < 2; ++cj)
#pragma unroll
            for (int ci = 0; ci < 2; ++ci) {
                const int xt = 2 * ic + ci, yt = 2 * jc + cj;
                const int rr = yt + 1, c = xt + 1;
                const double v[19] = {
                    p0[rr][c], p0[rr][c + 1], p0[rr][c - 1], p0[rr + 1][c], p0[rr - 1][c],
                    pp[rr][c], pm[rr][c],
                    p0[rr + 1][c + 1], p0[rr - 1][c + 1], p0[rr + 1][c - 1], p0[rr - 1][c - 1],
                    pp[rr][c + 1], pm[rr][c + 1], pp[rr][c - 1], pm[rr][c - 1],
                    pp[rr + 1][c], pm[rr + 1][c], pp[rr - 1][c], pm[rr - 1][c]};
                const int g = ((k << lg | (y0 + yt)) << lg) | (x0 + xt);
                const double r = s[g] - apply_L(stencil_terms(v), al);
                sphi += v[0];
                sr += r;
            }
        if (k & 1) {
            const int q = (((k >> 1) << lgc | (y0 / 2 + jc)) << lgc) | (x0 / 2 + ic);
            hat_c[q] = sphi * 0.125;
            s_c[q] = sr * 0.5; // 4 * mean: the coarse cell is twice as wide
        }
    }
}

// FAS coarse source on a large periodic level, through LDS: s = L[hat] + s
// and phi = hat, streaming hat planes with a one-cell halo as
// k_residual_tiled does.  Same expression per cell as k_coarse_source, so the
// same bits; hat is read from HBM about once instead of through 19 gathers.
template <int TX, int TY>
__global__ void __launch_bounds__(kBlock)
k_coarse_source_tiled(const double *__restrict__ hat, double *__restrict__ phi,
                      double *__restrict__ s, int lg, int tz, double al) {
    constexpr int PX = TX + 2, PY = TY + 2, PLANE = PX * PY;
    constexpr int PRE = (PLANE + kBlock - 1) / kBlock;
    constexpr int CELLS = TX * TY / kBlock; // output cells per thread per plane
    static_assert(TX * TY % kBlock == 0, "tile");
    __shared__ double P[4][PLANE];
    const int n = 1 << lg, m = n - 1;
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
    double pre[PRE];
    auto fetch = [&](int z) {
        const int zo = (z & m) << (2 * lg);
#pragma unroll
        for (int e = 0; e < PRE; ++e)
            if (pq[e] >= 0) pre[e] = hat[zo | pxy[e]];
    };
    auto commit = [&](int z) {
        double *dst = P[z & 3];
#pragma unroll
        for (int e = 0; e < PRE; ++e)
            if (pq[e] >= 0) dst[pq[e]] = pre[e];
    };
    fetch(z0 - 1);
    commit(z0 - 1);
    fetch(z0);
    commit(z0);
    fetch(z0 + 1);
    for (int k = z0; k < z0 + tz; ++k) {
        commit(k + 1); // slot of plane k-3, last read at step k-2
        if (k + 2 <= z0 + tz) fetch(k + 2);
        __syncthreads();
        const double(*pm)[PX] = reinterpret_cast<const double(*)[PX]>(P[(k - 1) & 3]);
        const double(*p0)[PX] = reinterpret_cast<const double(*)[PX]>(P[k & 3]);
        const double(*pp)[PX] = reinterpret_cast<const double(*)[PX]>(P[(k + 1) & 3]);
#pragma unroll
        for (int e = 0; e < CELLS; ++e) {
            const int q = tid + e * kBlock;
            const int yt = q / TX, xt = q - yt * TX;
            const int rr = yt + 1, c = xt + 1;
            const double v[19] = {
                p0[rr][c], p0[rr][c + 1], p0[rr][c - 1], p0[rr + 1][c], p0[rr - 1][c],
                pp[rr][c], pm[rr][c],
                p0[rr + 1][c + 1], p0[rr - 1][c + 1], p0[rr + 1][c - 1], p0[rr - 1][c - 1],
                pp[rr][c + 1], pm[rr][c + 1], pp[rr][c - 1], pm[rr][c - 1],
                pp[rr + 1][c], pm[rr + 1][c], pp[rr - 1][c], pm[rr - 1][c]};
            const int g = ((k << lg | (y0 + yt)) << lg) | (x0 + xt);
            s[g] = apply_L(stencil_terms(v), al) + s[g];
            phi[g] = v[0];
        }
    }
}

// Residual norm of a large periodic level through LDS: a workgroup streams a
// TX x TY column along z over tz planes, holding four planes of phi with a
// one-cell halo; each phi and S value is read from HBM about once.  One
// partial sum per workgroup (fixed order), optional r_out = r * scale (FP64,
// or rounded to FP32 for the mixed-precision loop).
template <int TX, int TY, class OutT, bool PER = true>
__global__ void __launch_bounds__(kBlock)
k_residual_tiled(const double *__restrict__ phi, const double *__restrict__ s, int lg, int tz,
                 double al, double *__restrict__ partials, OutT *__restrict__ r_out,
                 double r_scale, const unsigned char *__restrict__ mask = nullptr) {
    constexpr int PX = TX + 2, PY = TY + 2, PLANE = PX * PY;
    constexpr int PRE = (PLANE + kBlock - 1) / kBlock;
    constexpr int CELLS = TX * TY / kBlock; // output cells per thread per plane
    static_assert(TX * TY % kBlock == 0, "tile");
    __shared__ double P[4][PLANE];
    const int n = 1 << lg, m = n - 1;
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
        // periodic: wrapped natural index; Dirichlet: padded (n+2)^3, whose
        // ghost shell holds the halo beyond the level's faces
        pxy[e] = PER ? (((y0 - 1 + yy) & m) << lg) | ((x0 - 1 + xx) & m)
                     : (y0 + yy) * (n + 2) + (x0 + xx);
    }
    double pre[PRE];
    auto fetch = [&](int z) {
        const int zo = PER ? (z & m) << (2 * lg) : (z + 1) * (n + 2) * (n + 2);
#pragma unroll
        for (int e = 0; e < PRE; ++e)
            if (pq[e] >= 0) pre[e] = phi[zo + pxy[e]];
    };
    auto commit = [&](int z) {
        double *dst = P[z & 3];
#pragma unroll
        for (int e = 0; e < PRE; ++e)
            if (pq[e] >= 0) dst[pq[e]] = pre[e];
    };
    double acc = 0.0;
    fetch(z0 - 1);
    commit(z0 - 1);
    fetch(z0);
    commit(z0);
    fetch(z0 + 1);
    for (int k = z0; k < z0 + tz; ++k) {
        commit(k + 1); // slot of plane k-3, last read at step k-2
        if (k + 2 <= z0 + tz) fetch(k + 2);
        __syncthreads();
        const double(*pm)[PX] = reinterpret_cast<const double(*)[PX]>(P[(k - 1) & 3]);
        const double(*p0)[PX] = reinterpret_cast<const double(*)[PX]>(P[k & 3]);
        const double(*pp)[PX] = reinterpret_cast<const double(*)[PX]>(P[(k + 1) & 3]);
#pragma unroll
        for (int e = 0; e < CELLS; ++e) {
            const int q = tid + e * kBlock;
            const int yt = q / TX, xt = q - yt * TX;
            const int rr = yt + 1, c = xt + 1;
            const double v[19] = {
                p0[rr][c], p0[rr][c + 1], p0[rr][c - 1], p0[rr + 1][c], p0[rr - 1][c],
                pp[rr][c], pm[rr][c],
                p0[rr + 1][c + 1], p0[rr - 1][c + 1], p0[rr + 1][c - 1], p0[rr - 1][c - 1],
                pp[rr][c + 1], pm[rr][c + 1], pp[rr][c - 1], pm[rr][c - 1],
                pp[rr + 1][c], pm[rr + 1][c], pp[rr - 1][c], pm[rr - 1][c]};
            const int g = ((k << lg | (y0 + yt)) << lg) | (x0 + xt);
            // a held cell (cell-wise truncation) is not part of the equations
            const double r = !PER && mask && !mask[g] ? 0.0 : s[g] - apply_L(stencil_terms(v), al);
            acc = fma(r, r, acc);
            if (r_out) r_out[g] = (OutT)(r * r_scale);
        }
    }
    const double b = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

template <bool PER>
__global__ void __launch_bounds__(kBlock)
k_residual_sumsq(const double *__restrict__ phi, const double *__restrict__ s, Ix<PER> ix,
                 double al, double *__restrict__ partials, double *__restrict__ r_out,
                 double r_scale, const unsigned char *__restrict__ mask) {
    const int n = ix.n, lg = ix.lg;
    const int total = 1 << (3 * lg);
    double acc = 0.0;
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < total; c += gridDim.x * kBlock) {
        const int i = c & (n - 1), j = (c >> lg) & (n - 1), k = c >> (2 * lg);
        double r = 0.0; // a held cell is not part of the equations solved
        if (!mask || mask[c]) {
            double v[19];
            gather(phi, ix, i, j, k, v);
            r = s[c] - apply_L(stencil_terms(v), al);
        }
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

// out = (sum r^2, sum s^2, relative norm) from sums[1] = sum s^2 and
// sums[2] = sum r^2, the relative norm as the blocking residual computes it
// on the host (IEEE division and square root: the same bits)
__global__ void k_residual_norms(const double *__restrict__ sums, double *__restrict__ out) {
    const double ss = sums[1], rr = sums[2];
    out[0] = rr;
    out[1] = ss;
    out[2] = ss > 0.0 ? sqrt(rr / ss) : sqrt(rr);
}

// FAS restriction fused with the residual, for one coarse cell (I, J, K): the
// mean of its 8 children's phi and 4 x the mean of their residuals s - L[phi],
// from the 4x4x4 block of fine values around the children (the 8 block
// corners are never part of a child's 19-point stencil and are not loaded).
template <bool PER>
__device__ __forceinline__ void restrict_cell(const double *__restrict__ phi_f,
                                              const double *__restrict__ s_f, const Ix<PER> &ixf,
                                              int nf, double al_f, int I, int J, int K,
                                              double &hat, double &sc,
                                              const unsigned char *__restrict__ mask_f) {
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
                const size_t fc = ((size_t)fk * nf + fj) * nf + fi;
                const double r = mask_f && !mask_f[fc]
                                     ? 0.0 // held: no residual
                                     : s_f[fc] - apply_L(stencil_terms(v), al_f);
                sphi += v[0];
                sr += r;
            }
    hat = sphi * 0.125;
    sc = sr * 0.5; // 4 * mean: the coarse cell is twice as wide
}

// one thread per coarse cell
template <bool PER>
__global__ void __launch_bounds__(kBlock)
k_restrict_residual(const double *__restrict__ phi_f, const double *__restrict__ s_f,
                    Ix<PER> ixf, double al_f, double *__restrict__ hat_c,
                    double *__restrict__ s_c, Ix<PER> ixc, const unsigned char *__restrict__ mask_f) {
    const int nc = ixc.n, lgc = ixc.lg;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= (1 << (3 * lgc))) return;
    const int I = t & (nc - 1), J = (t >> lgc) & (nc - 1), K = t >> (2 * lgc);
    double hat, sc;
    restrict_cell(phi_f, s_f, ixf, ixf.n, al_f, I, J, K, hat, sc, mask_f);
    hat_c[ixc(I, J, K)] = hat;
    s_c[t] = sc;
}

template <bool PER>
__global__ void __launch_bounds__(kBlock)
k_coarse_source(const double *__restrict__ hat, double *__restrict__ phi,
                double *__restrict__ s, Ix<PER> ix, double al, int dyn_bc) {
    const int n = ix.n, lg = ix.lg;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= (1 << (3 * lg))) return;
    const int i = t & (n - 1), j = (t >> lg) & (n - 1), k = t >> (2 * lg);
    double v[19];
    gather(hat, ix, i, j, k, v);
    s[t] = apply_L(stencil_terms(v), al) + s[t];
    phi[ix(i, j, k)] = v[0];
    if (!PER && dyn_bc) write_owned_ghosts(phi, hat, ix, i, j, k, v[0]); // zero correction
}

// Trilinear cell-centred transfer: a fine cell centre sits a quarter coarse
// cell from its parent's centre on every axis, so the parent weighs 3/4 and
// the neighbour on the fine cell's side 1/4 per axis (27/64 ... 1/64).
template <bool PER, bool CORRECT>
__global__ void __launch_bounds__(kBlock)
k_prolong(double *__restrict__ phi_f, Ix<PER> ixf, const double *__restrict__ phi_c,
          const double *__restrict__ hat_c, Ix<PER> ixc, const double *__restrict__ hat_f,
          int dyn_bc_f) {
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
    const int me = ixf(i, j, k);
    const double val = CORRECT ? phi_f[me] + acc : acc;
    phi_f[me] = val;
    if (!PER && dyn_bc_f) write_owned_ghosts(phi_f, hat_f, ixf, i, j, k, val);
}

// The same transfer with one thread per COARSE cell: its 27 coarse values are
// loaded once and its 8 children written, the two x-children of a row as one
// 16-byte access on periodic levels.  Each child gets exactly the arithmetic
// of k_prolong (same weights, same order of the fma chain).
template <bool PER, bool CORRECT>
__global__ void __launch_bounds__(kBlock)
k_prolong8(double *__restrict__ phi_f, Ix<PER> ixf, const double *__restrict__ phi_c,
           const double *__restrict__ hat_c, Ix<PER> ixc, const double *__restrict__ hat_f,
           int dyn_bc_f, const unsigned char *__restrict__ mask_f) {
    const int nc = ixc.n, lgc = ixc.lg;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= (1 << (3 * lgc))) return;
    const int I = t & (nc - 1), J = (t >> lgc) & (nc - 1), K = t >> (2 * lgc);
    double cv[3][3][3];
#pragma unroll
    for (int dk = 0; dk < 3; ++dk)
#pragma unroll
        for (int dj = 0; dj < 3; ++dj)
#pragma unroll
            for (int di = 0; di < 3; ++di) {
                const int q = ixc(I + di - 1, J + dj - 1, K + dk - 1);
                cv[dk][dj][di] = CORRECT ? phi_c[q] - hat_c[q] : phi_c[q];
            }
    // Dirichlet levels: the children's masks and old values are loaded with
    // the coarse values, before any store (one wait for memory, not one per
    // child)
    unsigned char it[2][2][2];
    double old8[2][2][2] = {};
    if constexpr (!PER) {
#pragma unroll
        for (int ck = 0; ck < 2; ++ck)
#pragma unroll
            for (int cj = 0; cj < 2; ++cj)
#pragma unroll
                for (int ci = 0; ci < 2; ++ci) {
                    it[ck][cj][ci] = 1;
                    if (CORRECT) old8[ck][cj][ci] = phi_f[ixf(2 * I + ci, 2 * J + cj, 2 * K + ck)];
                }
        if (mask_f)
#pragma unroll
            for (int ck = 0; ck < 2; ++ck)
#pragma unroll
                for (int cj = 0; cj < 2; ++cj) {
                    const size_t row = ((size_t)(2 * K + ck) * ixf.n + 2 * J + cj) * ixf.n + 2 * I;
                    it[ck][cj][0] = mask_f[row];
                    it[ck][cj][1] = mask_f[row + 1];
                }
    }
    double val8[2][2][2];
#pragma unroll
    for (int ck = 0; ck < 2; ++ck)
#pragma unroll
        for (int cj = 0; cj < 2; ++cj) {
            double out[2];
#pragma unroll
            for (int ci = 0; ci < 2; ++ci) {
                const int si = ci ? 1 : -1, sj = cj ? 1 : -1, sk = ck ? 1 : -1;
                double acc = 0.0;
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int a = 0; a < 2; ++a) {
                            const double w = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (c ? 0.25 : 0.75);
                            acc = fma(w, cv[1 + c * sk][1 + b * sj][1 + a * si], acc);
                        }
                out[ci] = acc;
            }
            const int i = 2 * I, j = 2 * J + cj, k = 2 * K + ck;
            const int q0 = ixf(i, j, k);
            if constexpr (PER) {
                double2 *p2 = reinterpret_cast<double2 *>(phi_f + q0);
                double2 old = CORRECT ? *p2 : make_double2(0.0, 0.0);
                if (CORRECT) {
                    old.x += out[0];
                    old.y += out[1];
                } else {
                    old.x = out[0];
                    old.y = out[1];
                }
                *p2 = old;
            } else {
#pragma unroll
                for (int ci = 0; ci < 2; ++ci) {
                    const double val = CORRECT ? old8[ck][cj][ci] + out[ci] : out[ci];
                    val8[ck][cj][ci] = val;
                    if (it[ck][cj][ci]) phi_f[ixf(i + ci, j, k)] = val; // else held: kept
                }
            }
        }
    // the ghosts of the children on the boundary of a coarse level of a
    // refinement, four children at a time: their hat values first, then the
    // stores
    if constexpr (!PER) {
        if (!dyn_bc_f || !(I == 0 || I == nc - 1 || J == 0 || J == nc - 1 || K == 0 || K == nc - 1))
            return;
#pragma unroll
        for (int ck = 0; ck < 2; ++ck) {
            int q[2][2][8];
            double h[2][2][8];
            unsigned own[2][2];
#pragma unroll
            for (int cj = 0; cj < 2; ++cj)
#pragma unroll
                for (int ci = 0; ci < 2; ++ci) {
                    own[cj][ci] = ghost_slots(ixf, 2 * I + ci, 2 * J + cj, 2 * K + ck, q[cj][ci]);
                    if (!it[ck][cj][ci]) own[cj][ci] = 0; // a held cell writes nothing
#pragma unroll
                    for (int m = 0; m < 8; ++m) h[cj][ci][m] = hat_f[q[cj][ci][m]];
                }
#pragma unroll
            for (int cj = 0; cj < 2; ++cj)
#pragma unroll
                for (int ci = 0; ci < 2; ++ci)
                    store_owned_ghosts(phi_f, q[cj][ci], h[cj][ci], own[cj][ci], val8[ck][cj][ci]);
        }
    }
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
k_coarsest(double *__restrict__ phi, const double *__restrict__ s, Ix<PER> ix, double al, double w,
           int sweeps, unsigned *__restrict__ fallbacks, const double *__restrict__ hat,
           int dyn_bc, const unsigned char *__restrict__ mask) {
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
    const bool held = active && mask && !mask[t];
    unsigned fb = 0;
    for (int sw = 0; sw < sweeps; ++sw) {
#pragma unroll
        for (int col = 0; col < 2; ++col) {
            const double *src = col ? B : A;
            double *dst = col ? A : B;
            if (active) {
                const int me = ix(i, j, k);
                double val;
                if (mycol == col && !held) {
                    double v[19];
                    gather(src, ix, i, j, k, v);
                    val = relax_cell(v, sc, al, w, fb);
                } else {
                    val = src[me];
                }
                dst[me] = val;
                if (!PER && dyn_bc) write_owned_ghosts(dst, hat, ix, i, j, k, val);
            }
            __syncthreads();
        }
    }
    for (int q = threadIdx.x; q < slots; q += blockDim.x) phi[q] = A[q];
    if (fb) flush_events(fallbacks, fb);
}

// The bottom of a periodic V-cycle in one workgroup: every level from one of
// at most 16^3 cells down to the coarsest, with all its arrays in LDS, so
// that the small levels cost one launch instead of about a dozen per cycle.
// Each step has exactly the arithmetic, in the same order, of the per-level
// kernels (k_smooth_half, k_restrict_residual, k_coarse_source, k_coarsest,
// k_prolong), so the result is bit for bit the one of those launches.  A
// half sweep computes the new values of its colour into registers, waits for
// the whole workgroup, then stores them: every read sees the values of the
// start of the half sweep, as with the out-of-place kernels.
constexpr int kBottomThreads = 512;
constexpr int kBottomPerThread = 2048 / kBottomThreads; // cells of one colour at 16^3
constexpr int kBottomCells = 4096 + 512 + 64 + 8;       // 16^3 + 8^3 + 4^3 + 2^3

__global__ void __launch_bounds__(kBottomThreads)
k_bottom(double *__restrict__ phi, const double *__restrict__ s, int lg0, BottomLevels bl,
         int nu1, int nu2, int csweeps, unsigned *__restrict__ fallbacks) {
    __shared__ double PHI[kBottomCells];
    __shared__ double SRC[kBottomCells];
    __shared__ double HAT[kBottomCells - 4096];
    const int tid = threadIdx.x;
    const int nb = bl.levels;
    // level q starts at off(q) in PHI and SRC, at hoff(q) in HAT (q >= 1)
    auto off = [&](int q) {
        int o = 0;
        for (int p = 0; p < q; ++p) o += 1 << (3 * (lg0 - p));
        return o;
    };
    auto hoff = [&](int q) { return off(q) - (1 << (3 * lg0)); };
    auto alpha = [&](int q) {
        return q == 0 ? bl.alpha[0] : q == 1 ? bl.alpha[1] : q == 2 ? bl.alpha[2] : bl.alpha[3];
    };
    unsigned fb = 0;
    const int cells0 = 1 << (3 * lg0);
    for (int t = tid; t < cells0; t += kBottomThreads) {
        PHI[t] = phi[t];
        SRC[t] = s[t];
    }
    __syncthreads();

    auto smooth = [&](int q, int sweeps) {
        const int lg = lg0 - q, n = 1 << lg, half = n >> 1;
        const Ix<true> ix = {n, lg, n + 2};
        double *ph = PHI + off(q);
        const double *sr = SRC + off(q);
        const double al = alpha(q);
        const int ncol = (n * n * n) >> 1; // cells of one colour
        // new value of the t-th cell of colour col, or at = -1 past the last
        auto cell = [&](int t, int col, double &val, int &at) {
            at = -1;
            if (t >= ncol) return;
            const int m = t & (half - 1);
            const int row = t >> (lg - 1);
            const int j = row & (n - 1), k = row >> lg;
            const int i = 2 * m + ((col ^ j ^ k) & 1);
            double v[19];
            gather(ph, ix, i, j, k, v);
            val = relax_cell(v, sr[((k << lg) + j) * n + i], al, bl.omega, fb);
            at = ix(i, j, k);
        };
        for (int sw = 0; sw < sweeps; ++sw)
            for (int col = 0; col < 2; ++col) {
                double v[kBottomPerThread];
                int at[kBottomPerThread];
#pragma unroll
                for (int c = 0; c < kBottomPerThread; ++c) {
                    v[c] = 0.0;
                    cell(tid + c * kBottomThreads, col, v[c], at[c]);
                    __builtin_amdgcn_sched_barrier(0); // one cell at a time: no spills
                }
                __syncthreads();
#pragma unroll
                for (int c = 0; c < kBottomPerThread; ++c)
                    if (at[c] >= 0) ph[at[c]] = v[c];
                __syncthreads();
            }
    };

    for (int q = 0; q + 1 < nb; ++q) {
        smooth(q, nu1);
        const int lgf = lg0 - q, lgc = lgf - 1, nc = 1 << lgc;
        const Ix<true> ixf = {1 << lgf, lgf, (1 << lgf) + 2};
        const Ix<true> ixc = {nc, lgc, nc + 2};
        double *hc = HAT + hoff(q + 1), *sc = SRC + off(q + 1), *pc = PHI + off(q + 1);
        for (int t = tid; t < nc * nc * nc; t += kBottomThreads) {
            const int I = t & (nc - 1), J = (t >> lgc) & (nc - 1), K = t >> (2 * lgc);
            // restrict_cell's sums, each child's stencil gathered on its own
            const double *pf = PHI + off(q), *sf = SRC + off(q);
            const int nf = 1 << lgf;
            double sphi = 0.0, sr = 0.0;
#pragma unroll 1
            for (int ch = 0; ch < 8; ++ch) {
                const int fi = 2 * I + (ch & 1), fj = 2 * J + ((ch >> 1) & 1),
                          fk = 2 * K + (ch >> 2);
                double v[19];
                gather(pf, ixf, fi, fj, fk, v);
                const double r = sf[(fk * nf + fj) * nf + fi] - apply_L(stencil_terms(v), alpha(q));
                sphi += v[0];
                sr += r;
            }
            hc[t] = sphi * 0.125;
            sc[t] = sr * 0.5;
        }
        __syncthreads();
        for (int t = tid; t < nc * nc * nc; t += kBottomThreads) {
            const int i = t & (nc - 1), j = (t >> lgc) & (nc - 1), k = t >> (2 * lgc);
            double v[19];
            gather(hc, ixc, i, j, k, v);
            sc[t] = apply_L(stencil_terms(v), alpha(q + 1)) + sc[t];
            pc[t] = v[0];
        }
        __syncthreads();
    }
    smooth(nb - 1, csweeps);
    for (int q = nb - 2; q >= 0; --q) {
        const int lgf = lg0 - q, nf = 1 << lgf, lgc = lgf - 1, nc = 1 << lgc;
        const Ix<true> ixc = {nc, lgc, nc + 2};
        const double *pc = PHI + off(q + 1), *hc = HAT + hoff(q + 1);
        double *pf = PHI + off(q);
        for (int t = tid; t < nf * nf * nf; t += kBottomThreads) {
            const int i = t & (nf - 1), j = (t >> lgf) & (nf - 1), k = t >> (2 * lgf);
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
                        const int qq = ixc(I + a * si, J + b * sj, K + c * sk);
                        acc = fma(w, pc[qq] - hc[qq], acc);
                    }
            pf[t] = pf[t] + acc;
        }
        __syncthreads();
        smooth(q, nu2);
    }
    for (int t = tid; t < cells0; t += kBottomThreads) phi[t] = PHI[t];
    if (fb) flush_events(fallbacks, fb);
}

// The bottom of a refinement's V-cycle in one workgroup: its coarse levels
// from one of at most 16^3 cells down to the coarsest, padded with their
// ghost shells, all arrays in LDS.  Each step has the arithmetic, in the same
// order, of the per-level kernels of those levels (k_smooth_half,
// k_restrict_residual, k_coarse_source, k_coarsest, k_prolong8), so the result
// is bit for bit theirs.  Those kernels rewrite the ghosts of every cell they
// write from its new value (write_owned_ghosts); a ghost is thus always the
// same function of its interior cell's current value, and the half sweeps
// here, done in place (new values of one colour into registers, wait, store),
// rewrite only the ghosts of the cells they change.  Held cells (mask 0) keep
// their values, take no residual and no correction.
constexpr int kBottomDirThreads = 1024;
constexpr int kBottomDirPerThread = 2048 / kBottomDirThreads; // cells of one colour at 16^3
constexpr int kBottomDirPad = 18 * 18 * 18 + 10 * 10 * 10 + 6 * 6 * 6 + 4 * 4 * 4;
constexpr int kBottomDirCells = 4096 + 512 + 64 + 8;

__global__ void __launch_bounds__(kBottomDirThreads)
k_bottom_dir(BottomDirLevels bl, int nu1, int nu2, int csweeps, unsigned *__restrict__ fallbacks) {
    __shared__ double PHI[kBottomDirPad];
    __shared__ double HAT[kBottomDirPad];
    __shared__ double SRC[kBottomDirCells];
    __shared__ unsigned char MSK[kBottomDirCells];
    const int tid = threadIdx.x;
    const int nb = bl.levels, lg0 = bl.lg0;
    auto pad = [&](int q) {
        const int m = (1 << (lg0 - q)) + 2;
        return m * m * m;
    };
    // level q starts at poff(q) in PHI and HAT, at coff(q) in SRC and MSK
    auto poff = [&](int q) {
        int o = 0;
        for (int p = 0; p < q; ++p) o += pad(p);
        return o;
    };
    auto coff = [&](int q) {
        int o = 0;
        for (int p = 0; p < q; ++p) o += 1 << (3 * (lg0 - p));
        return o;
    };
    auto alpha = [&](int q) {
        return q == 0 ? bl.alpha[0] : q == 1 ? bl.alpha[1] : q == 2 ? bl.alpha[2] : bl.alpha[3];
    };
    auto ixq = [&](int q) {
        const int lg = lg0 - q;
        return Ix<false>{1 << lg, lg, (1 << lg) + 2};
    };
    unsigned fb = 0;
    for (int q = 0; q < nb; ++q) {
        const double *hg = q == 0 ? bl.hat[0] : q == 1 ? bl.hat[1] : q == 2 ? bl.hat[2] : bl.hat[3];
        const unsigned char *mg =
            q == 0 ? bl.mask[0] : q == 1 ? bl.mask[1] : q == 2 ? bl.mask[2] : bl.mask[3];
        double *hl = HAT + poff(q);
        for (int t = tid; t < pad(q); t += kBottomDirThreads) hl[t] = hg[t];
        unsigned char *ml = MSK + coff(q);
        for (int t = tid; t < (1 << (3 * (lg0 - q))); t += kBottomDirThreads)
            ml[t] = mg ? mg[t] : (unsigned char)1;
    }
    for (int t = tid; t < pad(0); t += kBottomDirThreads) PHI[t] = bl.phi0[t];
    for (int t = tid; t < (1 << (3 * lg0)); t += kBottomDirThreads) SRC[t] = bl.s0[t];
    __syncthreads();

    auto smooth = [&](int q, int sweeps) {
        const Ix<false> ix = ixq(q);
        const int lg = ix.lg, n = ix.n, half = n >> 1;
        double *ph = PHI + poff(q);
        const double *hh = HAT + poff(q);
        const double *sr = SRC + coff(q);
        const unsigned char *mk = MSK + coff(q);
        const double al = alpha(q);
        const int ncol = (n * n * n) >> 1; // cells of one colour
        for (int sw = 0; sw < sweeps; ++sw)
            for (int col = 0; col < 2; ++col) {
                double v[kBottomDirPerThread];
                int cell[kBottomDirPerThread]; // natural index, or -1: nothing to store
#pragma unroll
                for (int c = 0; c < kBottomDirPerThread; ++c) {
                    v[c] = 0.0;
                    cell[c] = -1;
                    const int t = tid + c * kBottomDirThreads;
                    if (t < ncol) {
                        const int m = t & (half - 1);
                        const int row = t >> (lg - 1);
                        const int j = row & (n - 1), k = row >> lg;
                        const int i = 2 * m + ((col ^ j ^ k) & 1);
                        const int nat = ((k << lg) + j) * n + i;
                        if (mk[nat]) { // a held cell keeps its value (and its ghosts)
                            double g[19];
                            gather(ph, ix, i, j, k, g);
                            v[c] = relax_cell(g, sr[nat], al, bl.omega, fb);
                            cell[c] = nat;
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0); // one cell at a time: no spills
                }
                __syncthreads();
#pragma unroll
                for (int c = 0; c < kBottomDirPerThread; ++c)
                    if (cell[c] >= 0) {
                        const int i = cell[c] & (n - 1), j = (cell[c] >> lg) & (n - 1),
                                  k = cell[c] >> (2 * lg);
                        ph[ix(i, j, k)] = v[c];
                        write_owned_ghosts(ph, hh, ix, i, j, k, v[c]);
                    }
                __syncthreads();
            }
    };

    for (int q = 0; q + 1 < nb; ++q) {
        smooth(q, nu1);
        const Ix<false> ixf = ixq(q), ixc = ixq(q + 1);
        const int nc = ixc.n, lgc = ixc.lg;
        double *pc = PHI + poff(q + 1), *hc = HAT + poff(q + 1), *sc = SRC + coff(q + 1);
        for (int t = tid; t < nc * nc * nc; t += kBottomDirThreads) {
            const int I = t & (nc - 1), J = (t >> lgc) & (nc - 1), K = t >> (2 * lgc);
            // restrict_cell's sums (children in its order), each child's
            // stencil gathered on its own
            const double *pf = PHI + poff(q), *sf = SRC + coff(q);
            const unsigned char *mf = MSK + coff(q);
            const int nf = ixf.n;
            double sphi = 0.0, sr = 0.0;
#pragma unroll 1
            for (int ch = 0; ch < 8; ++ch) {
                const int fi = 2 * I + (ch & 1), fj = 2 * J + ((ch >> 1) & 1), fk = 2 * K + (ch >> 2);
                double v[19];
                gather(pf, ixf, fi, fj, fk, v);
                const int fc = (fk * nf + fj) * nf + fi;
                const double r = !mf[fc] ? 0.0 : sf[fc] - apply_L(stencil_terms(v), alpha(q));
                sphi += v[0];
                sr += r;
            }
            hc[ixc(I, J, K)] = sphi * 0.125;
            sc[t] = sr * 0.5;
        }
        __syncthreads();
        for (int t = tid; t < nc * nc * nc; t += kBottomDirThreads) {
            const int i = t & (nc - 1), j = (t >> lgc) & (nc - 1), k = t >> (2 * lgc);
            double v[19];
            gather(hc, ixc, i, j, k, v);
            sc[t] = apply_L(stencil_terms(v), alpha(q + 1)) + sc[t];
            pc[ixc(i, j, k)] = v[0];
            write_owned_ghosts(pc, hc, ixc, i, j, k, v[0]); // zero correction
        }
        __syncthreads();
    }
    smooth(nb - 1, csweeps);
    for (int q = nb - 2; q >= 0; --q) {
        const Ix<false> ixf = ixq(q), ixc = ixq(q + 1);
        const int nf = ixf.n, lgf = ixf.lg;
        const double *pc = PHI + poff(q + 1), *hc = HAT + poff(q + 1);
        double *pf = PHI + poff(q);
        const double *hf = HAT + poff(q);
        const unsigned char *mk = MSK + coff(q);
        for (int t = tid; t < nf * nf * nf; t += kBottomDirThreads) {
            if (!mk[t]) continue; // held: no correction
            const int i = t & (nf - 1), j = (t >> lgf) & (nf - 1), k = t >> (2 * lgf);
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
                        const int qq = ixc(I + a * si, J + b * sj, K + c * sk);
                        acc = fma(w, pc[qq] - hc[qq], acc);
                    }
            const int me = ixf(i, j, k);
            const double val = pf[me] + acc;
            pf[me] = val;
            write_owned_ghosts(pf, hf, ixf, i, j, k, val);
        }
        __syncthreads();
        smooth(q, nu2);
    }
    for (int t = tid; t < pad(0); t += kBottomDirThreads) bl.phi0[t] = PHI[t];
    if (fb) flush_events(fallbacks, fb);
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
    const bool interior = ii >= 1 && ii <= bx.nc && jj >= 1 && jj <= bx.nc && kk >= 1 &&
                          kk <= bx.nc;
    if (ghosts_only && interior) return;
    child[t] = interpolate_slot<PPER>(parent, np, lgp, bx, ii, jj, kk);
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

// Force on a large periodic level through LDS: a workgroup streams a TX x TY
// column along z over tz planes with a ring of four planes (one-cell halo in
// x and y) as k_residual_tiled does, so phi is read from HBM about once
// instead of once per difference direction; each component is k_force's
// expression (same bits).
template <int TX, int TY>
__global__ void __launch_bounds__(kBlock)
k_force_tiled(const double *__restrict__ phi, int lg, int tz, double c4h,
              double *__restrict__ f) {
    constexpr int PX = TX + 2, PY = TY + 2, PLANE = PX * PY;
    constexpr int PRE = (PLANE + kBlock - 1) / kBlock;
    constexpr int CELLS = TX * TY / kBlock; // output cells per thread per plane
    static_assert(TX * TY % kBlock == 0, "tile");
    __shared__ double P[4][PLANE];
    const int n = 1 << lg, m = n - 1;
    const size_t cells = (size_t)1 << (3 * lg);
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
    double pre[PRE];
    auto fetch = [&](int z) {
        const double *plane = phi + ((size_t)(z & m) << (2 * lg));
#pragma unroll
        for (int e = 0; e < PRE; ++e)
            if (pq[e] >= 0) pre[e] = *plane_at(plane, (unsigned)pxy[e]);
    };
    auto commit = [&](int z) {
        double *dst = P[z & 3];
#pragma unroll
        for (int e = 0; e < PRE; ++e)
            if (pq[e] >= 0) dst[pq[e]] = pre[e];
    };
    fetch(z0 - 1);
    commit(z0 - 1);
    fetch(z0);
    commit(z0);
    fetch(z0 + 1);
    for (int k = z0; k < z0 + tz; ++k) {
        commit(k + 1); // slot of plane k-3, last read at step k-2
        if (k + 2 <= z0 + tz) fetch(k + 2);
        __syncthreads();
        const double(*pm)[PX] = reinterpret_cast<const double(*)[PX]>(P[(k - 1) & 3]);
        const double(*p0)[PX] = reinterpret_cast<const double(*)[PX]>(P[k & 3]);
        const double(*pp)[PX] = reinterpret_cast<const double(*)[PX]>(P[(k + 1) & 3]);
        double *fx = f + ((size_t)k << (2 * lg));
#pragma unroll
        for (int e = 0; e < CELLS; ++e) {
            const int q = tid + e * kBlock;
            const int yt = q / TX, xt = q - yt * TX;
            const int rr = yt + 1, c = xt + 1;
            const unsigned g = (unsigned)(((y0 + yt) << lg) | (x0 + xt)); // in plane k
            *plane_at(fx, g) = -(p0[rr][c + 1] - p0[rr][c - 1]) * c4h;
            *plane_at(fx + cells, g) = -(p0[rr + 1][c] - p0[rr - 1][c]) * c4h;
            *plane_at(fx + 2 * cells, g) = -(pp[rr][c] - pm[rr][c]) * c4h;
        }
    }
}

// Cell-wise truncation (the generalisation proposed in Sec. III.C): child
// cell (i, j, k) of a ratio-2 box is iterated only if its parent cell P =
// origin + (i, j, k) / 2 has |F_5th| >= threshold |F_GR|, F_5th = -grad(phi)/2
// and F_GR = -grad(psi) by central differences on the parent level, compared
// as sum (dphi)^2 >= (2 threshold)^2 sum (dpsi)^2 (no roots, no divisions;
// the spacing cancels).  One grid-stride pass over the child cells with a
// fixed grid, so the per-block counts of iterated cells sum deterministically.
template <bool PER>
__global__ void __launch_bounds__(kBlock)
k_cell_mask(const double *__restrict__ phi, const double *__restrict__ psi, Ix<PER> ixp, int ox,
            int oy, int oz, int lgc, double t2, unsigned char *__restrict__ mask,
            double *__restrict__ partials) {
    const int nc = 1 << lgc;
    const int total = 1 << (3 * lgc);
    double count = 0.0;
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < total; c += gridDim.x * kBlock) {
        const int i = c & (nc - 1), j = (c >> lgc) & (nc - 1), k = c >> (2 * lgc);
        const int P = ox + (i >> 1), Q = oy + (j >> 1), R = oz + (k >> 1);
        const int up[3] = {ixp(P + 1, Q, R), ixp(P, Q + 1, R), ixp(P, Q, R + 1)};
        const int dn[3] = {ixp(P - 1, Q, R), ixp(P, Q - 1, R), ixp(P, Q, R - 1)};
        double gphi = 0.0, gpsi = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double dp = phi[up[a]] - phi[dn[a]];
            const double ds = psi[up[a]] - psi[dn[a]];
            gphi = fma(dp, dp, gphi);
            gpsi = fma(ds, ds, gpsi);
        }
        const bool on = gphi >= t2 * gpsi;
        mask[c] = on ? 1 : 0;
        count += on ? 1.0 : 0.0;
    }
    const double b = block_sum(count);
    if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

// Coarse level of a masked hierarchy: a coarse cell is iterated only if all
// eight of its children are, so that no coarse correction reaches a held
// fine cell's neighbourhood from a coarse cell that straddles it (the held
// regions act as fixed boundaries on every level).
__global__ void __launch_bounds__(kBlock)
k_mask_restrict(const unsigned char *__restrict__ mf, int lgc, unsigned char *__restrict__ mc) {
    const int nc = 1 << lgc, nf = 2 * nc;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= (1 << (3 * lgc))) return;
    const int I = t & (nc - 1), J = (t >> lgc) & (nc - 1), K = t >> (2 * lgc);
    bool all = true;
#pragma unroll
    for (int ch = 0; ch < 8; ++ch)
        all = all && mf[((size_t)(2 * K + (ch >> 2)) * nf + 2 * J + ((ch >> 1) & 1)) * nf +
                        2 * I + (ch & 1)] != 0;
    mc[t] = all ? 1 : 0;
}

// Tile activity of a masked level for the fused sweep: on[b] = 1 if the
// cells that workgroup b of the sweep writes (a 64 x 16 column of tz planes,
// numbered as the sweep numbers them) include any relaxed cell.
__global__ void __launch_bounds__(kBlock)
k_tile_activity(const unsigned char *__restrict__ mask, int lg, int tz,
                unsigned char *__restrict__ on) {
    const int n = 1 << lg, ntx = n / 64, tiles = ntx * (n / 16);
    const int b = blockIdx.x, tile = b % tiles;
    const int x0 = (tile % ntx) * 64, y0 = (tile / ntx) * 16, z0 = (b / tiles) * tz;
    bool it = false;
    for (int q = threadIdx.x; q < 64 * 16 * tz; q += kBlock) {
        const int x = q & 63, y = (q >> 6) & 15, z = q >> 10;
        it = it || mask[((size_t)((z0 + z) << lg) + y0 + y) * n + x0 + x] != 0;
    }
    const int any = __syncthreads_or(it ? 1 : 0);
    if (threadIdx.x == 0) on[b] = any ? 1 : 0;
}

// Block activity of a masked level for k_smooth_half: active[c * blocks + b]
// = 1 if block b of the colour-c launch relaxes any cell (same cell order).
__global__ void __launch_bounds__(kBlock)
k_block_activity(const unsigned char *__restrict__ mask, int lg,
                 unsigned char *__restrict__ active) {
    const int n = 1 << lg, half = n >> 1, colour = blockIdx.y;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    bool it = false;
    if (t < (half << (2 * lg))) {
        const int m = t & (half - 1), row = t >> (lg - 1);
        const int j = row & (n - 1), k = row >> lg;
        const int iu = 2 * m + ((colour ^ j ^ k) & 1);
        it = mask[((k << lg) + j) * n + iu] != 0;
    }
    const int any = __syncthreads_or(it ? 1 : 0);
    if (threadIdx.x == 0) active[colour * gridDim.x + blockIdx.x] = any ? 1 : 0;
}

// guard bands of the workspace (debugging aid): fill, then count changed words
__global__ void k_guard_fill(uint64_t *__restrict__ g, int words, uint64_t w) {
    if ((int)threadIdx.x < words) g[threadIdx.x] = w;
}

__global__ void k_guard_check(const uint64_t *__restrict__ g, int words, uint64_t w,
                              unsigned *__restrict__ bad) {
    if ((int)threadIdx.x < words && g[threadIdx.x] != w) atomicAdd(bad, 1u);
}

} // namespace

// ------------------------------------------------------------------------
// launchers

void launch_guard_fill(void *band, int words, uint64_t word, hipStream_t st) {
    k_guard_fill<<<1, 64, 0, st>>>(static_cast<uint64_t *>(band), words, word);
}

void launch_guard_check(const void *band, int words, uint64_t word, unsigned *bad,
                        hipStream_t st) {
    k_guard_check<<<1, 64, 0, st>>>(static_cast<const uint64_t *>(band), words, word, bad);
}

// planes per workgroup of the fused sweep on a level of n cells per side
// (tiles of 64 x 16 cells), and its number of workgroups
int fused_tz(int n) { return n >= 256 ? 32 : 4; }
size_t fused_tiles(int n) {
    return n >= 128 ? (size_t)(n / 64) * (n / 16) * (n / fused_tz(n)) : 0;
}

// the half-sweep blocks of both colours, then the fused sweep's workgroups
size_t block_activity_bytes(int n) {
    return 2 * (size_t)blocks_for((size_t)n * n * n / 2) + fused_tiles(n);
}

const unsigned char *tile_activity(const unsigned char *active, int n) {
    return active + 2 * (size_t)blocks_for((size_t)n * n * n / 2);
}

void launch_block_activity(const unsigned char *mask, int n, unsigned char *active,
                           hipStream_t st) {
    const unsigned nb = blocks_for((size_t)n * n * n / 2);
    k_block_activity<<<dim3(nb, 2), kBlock, 0, st>>>(mask, log2i(n), active);
    if (fused_tiles(n))
        k_tile_activity<<<(unsigned)fused_tiles(n), kBlock, 0, st>>>(mask, log2i(n), fused_tz(n),
                                                                    active + 2 * (size_t)nb);
}

void launch_cell_mask(const double *phi_parent, const double *psi_parent, int np,
                      bool parent_periodic, const ChildBox &b, double threshold,
                      unsigned char *mask, double *partials, hipStream_t st) {
    const double t2 = (2.0 * threshold) * (2.0 * threshold);
    const int lgp = log2i(np), lgc = log2i(b.nc);
    if (parent_periodic)
        k_cell_mask<true><<<kReduceBlocks, kBlock, 0, st>>>(
            phi_parent, psi_parent, make_ix<true>(np, lgp), b.origin[0], b.origin[1],
            b.origin[2], lgc, t2, mask, partials);
    else
        k_cell_mask<false><<<kReduceBlocks, kBlock, 0, st>>>(
            phi_parent, psi_parent, make_ix<false>(np, lgp), b.origin[0], b.origin[1],
            b.origin[2], lgc, t2, mask, partials);
}

void launch_mask_restrict(const unsigned char *mask_f, int nc, unsigned char *mask_c,
                          hipStream_t st) {
    k_mask_restrict<<<blocks_for((size_t)nc * nc * nc), kBlock, 0, st>>>(mask_f, log2i(nc), mask_c);
}

void launch_smooth_half(const Level &L, const double *pin, double *pout, int colour,
                        unsigned *fallbacks, hipStream_t st) {
    const unsigned nb = blocks_for(L.cells() / 2);
    if (L.periodic)
        k_smooth_half<true><<<nb, kBlock, 0, st>>>(pin, pout, L.s, make_ix<true>(L.n, L.lg),
                                                   L.alpha, L.omega, colour, fallbacks, nullptr,
                                                   0, nullptr, nullptr);
    else
        k_smooth_half<false><<<nb, kBlock, 0, st>>>(pin, pout, L.s, make_ix<false>(L.n, L.lg),
                                                    L.alpha, L.omega, colour, fallbacks, L.hat,
                                                    L.dyn_bc ? 1 : 0, L.mask,
                                                    L.dyn_bc ? nullptr : L.active);
}

// (on 32^3 and 64^3 the one-workgroup-per-tile pipeline is slower than two
// short launches: its prologue latency is not amortised over enough planes)
// periodic levels, and the finest level of a refinement (fixed ghost shell,
// held cells of the cell-wise mode kept), from 128^3 on
bool fused_sweep_ok(const Level &L) { return L.n >= 128 && (L.periodic || !L.dyn_bc); }
bool fused_prolong_ok(const Level &L) { return L.periodic && L.n >= 128; }

template <int TX, int TY, int TZ, int NT, bool PRO, bool PER>
void sweep_fused_tiles(const Level &L, const double *pin, double *pout, unsigned *fallbacks,
                       const double *phi_c, const double *hat_c, hipStream_t st) {
    const int tiles = (L.n / TX) * (L.n / TY);
    k_sweep_fused<TX, TY, TZ, NT, PRO, PER><<<tiles * (L.n / TZ), NT, 0, st>>>(
        pin, pout, L.s, L.lg, L.alpha, L.omega, fallbacks, phi_c, hat_c,
        PER ? nullptr : L.mask, PER ? nullptr : L.tile_on);
}

template <bool PRO, bool PER>
void sweep_fused_layout(const Level &L, const double *pin, double *pout, unsigned *fallbacks,
                        const double *phi_c, const double *hat_c, hipStream_t st) {
    if (fused_tz(L.n) == 32) // n >= 256: long z-chunks, the halo planes are a small share
        sweep_fused_tiles<64, 16, 32, 512, PRO, PER>(L, pin, pout, fallbacks, phi_c, hat_c, st);
    else // 128^3: short chunks, two workgroups per CU (4 planes: 5% faster than 8)
        sweep_fused_tiles<64, 16, 4, 512, PRO, PER>(L, pin, pout, fallbacks, phi_c, hat_c, st);
}

template <bool PRO>
void sweep_fused(const Level &L, const double *pin, double *pout, unsigned *fallbacks,
                 const double *phi_c, const double *hat_c, hipStream_t st) {
    if (L.periodic)
        sweep_fused_layout<PRO, true>(L, pin, pout, fallbacks, phi_c, hat_c, st);
    else if constexpr (!PRO)
        sweep_fused_layout<false, false>(L, pin, pout, fallbacks, phi_c, hat_c, st);
}

void launch_sweep_fused(const Level &L, const double *pin, double *pout, unsigned *fallbacks,
                        hipStream_t st) {
    sweep_fused<false>(L, pin, pout, fallbacks, nullptr, nullptr, st);
}

void launch_sweep_fused_prolong(const Level &L, const Level &C, const double *pin, double *pout,
                                unsigned *fallbacks, hipStream_t st) {
    sweep_fused<true>(L, pin, pout, fallbacks, C.phi, C.hat, st);
}

template <class OutT>
void residual_tiled(const Level &L, double *partials, OutT *r_out, double r_scale,
                    hipStream_t st) {
    constexpr int TX = 64, TY = 16;
    const int tiles = (L.n / TX) * (L.n / TY);
    // z-chunks of 8 planes (4 at 128^3: enough workgroups to fill the chip), at
    // most kReduceBlocks workgroups
    int chunks = L.n >= 256 ? L.n / 8 : L.n / 4;
    while (tiles * chunks > kReduceBlocks) chunks /= 2;
    // blocks beyond the grid contribute zeros to the fixed-size final sum
    const size_t unused = (size_t)(kReduceBlocks - tiles * chunks);
    if (unused) k_fill<<<blocks_for(unused), kBlock, 0, st>>>(partials + tiles * chunks, unused, 0.0);
    if (L.periodic)
        k_residual_tiled<TX, TY, OutT, true><<<tiles * chunks, kBlock, 0, st>>>(
            L.phi, L.s, L.lg, L.n / chunks, L.alpha, partials, r_out, r_scale, nullptr);
    else
        k_residual_tiled<TX, TY, OutT, false><<<tiles * chunks, kBlock, 0, st>>>(
            L.phi, L.s, L.lg, L.n / chunks, L.alpha, partials, r_out, r_scale, L.mask);
}

void launch_residual_sumsq(const Level &L, double *partials, double *r_out, double r_scale,
                           hipStream_t st) {
    if (L.n >= 128) { // periodic levels and the finest levels of refinements
        residual_tiled<double>(L, partials, r_out, r_scale, st);
        return;
    }
    if (L.periodic)
        k_residual_sumsq<true><<<kReduceBlocks, kBlock, 0, st>>>(
            L.phi, L.s, make_ix<true>(L.n, L.lg), L.alpha, partials, r_out, r_scale, nullptr);
    else
        k_residual_sumsq<false><<<kReduceBlocks, kBlock, 0, st>>>(
            L.phi, L.s, make_ix<false>(L.n, L.lg), L.alpha, partials, r_out, r_scale, L.mask);
}

bool residual_tiled_ok(const Level &L) { return L.periodic && L.n >= 128; }

void launch_residual_tiled_to32(const Level &L, float *r32, double *partials, hipStream_t st) {
    residual_tiled<float>(L, partials, r32, 1.0, st);
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

void launch_residual_norms(const double *sums, double *out, hipStream_t st) {
    k_residual_norms<<<1, 1, 0, st>>>(sums, out);
}

void launch_restrict_residual(const Level &F, const Level &C, bool tiled, hipStream_t st) {
    const unsigned nb = blocks_for(C.cells());
    if (tiled && F.periodic && F.n >= 128) {
        constexpr int TX = 64, TY = 16;
        const int tz = F.n >= 256 ? 8 : 4; // 128^3: enough workgroups to fill the chip
        const int tiles = (F.n / TX) * (F.n / TY);
        k_restrict_tiled<TX, TY><<<tiles * (F.n / tz), kBlock, 0, st>>>(F.phi, F.s, F.lg, tz,
                                                                       F.alpha, C.hat, C.s);
    } else if (F.periodic)
        k_restrict_residual<true><<<nb, kBlock, 0, st>>>(F.phi, F.s, make_ix<true>(F.n, F.lg),
                                                         F.alpha, C.hat, C.s,
                                                         make_ix<true>(C.n, C.lg), nullptr);
    else
        k_restrict_residual<false><<<nb, kBlock, 0, st>>>(F.phi, F.s, make_ix<false>(F.n, F.lg),
                                                          F.alpha, C.hat, C.s,
                                                          make_ix<false>(C.n, C.lg), F.mask);
}

void launch_coarse_source(const Level &C, bool tiled, hipStream_t st) {
    const unsigned nb = blocks_for(C.cells());
    if (tiled && C.periodic && C.n >= 128) {
        constexpr int TX = 64, TY = 16;
        const int tz = C.n >= 256 ? 8 : 4;
        const int tiles = (C.n / TX) * (C.n / TY);
        k_coarse_source_tiled<TX, TY><<<tiles * (C.n / tz), kBlock, 0, st>>>(C.hat, C.phi, C.s,
                                                                            C.lg, tz, C.alpha);
    } else if (C.periodic)
        k_coarse_source<true><<<nb, kBlock, 0, st>>>(C.hat, C.phi, C.s, make_ix<true>(C.n, C.lg),
                                                     C.alpha, 0);
    else
        k_coarse_source<false><<<nb, kBlock, 0, st>>>(C.hat, C.phi, C.s,
                                                      make_ix<false>(C.n, C.lg), C.alpha,
                                                      C.dyn_bc ? 1 : 0);
}

void launch_prolong_correct(const Level &F, const Level &C, hipStream_t st) {
    const unsigned nb = blocks_for(C.cells());
    if (F.periodic)
        k_prolong8<true, true><<<nb, kBlock, 0, st>>>(F.phi, make_ix<true>(F.n, F.lg), C.phi,
                                                      C.hat, make_ix<true>(C.n, C.lg), nullptr, 0,
                                                      nullptr);
    else
        k_prolong8<false, true><<<nb, kBlock, 0, st>>>(F.phi, make_ix<false>(F.n, F.lg), C.phi,
                                                       C.hat, make_ix<false>(C.n, C.lg), F.hat,
                                                       F.dyn_bc ? 1 : 0, F.mask);
}

void launch_prolong_full(const Level &F, const Level &C, hipStream_t st) {
    const unsigned nb = blocks_for(C.cells());
    if (F.periodic)
        k_prolong8<true, false><<<nb, kBlock, 0, st>>>(F.phi, make_ix<true>(F.n, F.lg), C.phi,
                                                       nullptr, make_ix<true>(C.n, C.lg), nullptr,
                                                       0, nullptr);
    else
        k_prolong8<false, false><<<nb, kBlock, 0, st>>>(F.phi, make_ix<false>(F.n, F.lg), C.phi,
                                                        nullptr, make_ix<false>(C.n, C.lg),
                                                        F.hat, F.dyn_bc ? 1 : 0, nullptr);
}

void launch_restrict_source(const Level &F, const Level &C, hipStream_t st) {
    k_restrict_source<<<blocks_for(C.cells()), kBlock, 0, st>>>(F.s, F.n, C.s, C.lg);
}

void launch_coarsest(const Level &L, int sweeps, unsigned *fallbacks, hipStream_t st) {
    const int threads = L.cells() < 64 ? 64 : (int)L.cells();
    if (L.periodic)
        k_coarsest<true><<<1, threads, 0, st>>>(L.phi, L.s, make_ix<true>(L.n, L.lg), L.alpha,
                                                L.omega, sweeps, fallbacks, nullptr, 0, nullptr);
    else
        k_coarsest<false><<<1, threads, 0, st>>>(L.phi, L.s, make_ix<false>(L.n, L.lg), L.alpha,
                                                 L.omega, sweeps, fallbacks, L.hat,
                                                 L.dyn_bc ? 1 : 0, L.mask);
}

bool bottom_ok(const Level *H, int l, int nl) {
    if (l + 1 >= nl || nl - l > kBottomMaxLevels) return false;
    for (int q = l; q < nl; ++q)
        if (!H[q].periodic) return false;
    return H[l].n <= 16 && H[nl - 1].n >= 2;
}

void launch_bottom(const Level *H, int l, int nl, int nu1, int nu2, int csweeps,
                   unsigned *fallbacks, hipStream_t st) {
    BottomLevels bl{};
    bl.levels = nl - l;
    for (int q = 0; q < bl.levels; ++q) bl.alpha[q] = H[l + q].alpha;
    bl.omega = H[l].omega;
    k_bottom<<<1, kBottomThreads, 0, st>>>(H[l].phi, H[l].s, H[l].lg, bl, nu1, nu2, csweeps,
                                           fallbacks);
}

bool bottom_dir_ok(const Level *H, int l, int nl) {
    if (l + 1 >= nl || nl - l > kBottomMaxLevels) return false;
    for (int q = l; q < nl; ++q)
        if (H[q].periodic || !H[q].dyn_bc) return false;
    return H[l].n <= 16 && H[nl - 1].n >= 2;
}

void launch_bottom_dir(const Level *H, int l, int nl, int nu1, int nu2, int csweeps,
                       unsigned *fallbacks, hipStream_t st) {
    BottomDirLevels bl{};
    bl.levels = nl - l;
    bl.lg0 = H[l].lg;
    bl.omega = H[l].omega;
    bl.phi0 = H[l].phi;
    bl.s0 = H[l].s;
    for (int q = 0; q < bl.levels; ++q) {
        bl.alpha[q] = H[l + q].alpha;
        bl.hat[q] = H[l + q].hat;
        bl.mask[q] = H[l + q].mask;
    }
    k_bottom_dir<<<1, kBottomDirThreads, 0, st>>>(bl, nu1, nu2, csweeps, fallbacks);
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
    if (periodic && n >= 128) {
        constexpr int TX = 64, TY = 16;
        const int tz = n >= 256 ? 8 : 4; // 128^3: enough workgroups to fill the chip
        const int tiles = (n / TX) * (n / TY);
        k_force_tiled<TX, TY><<<tiles * (n / tz), kBlock, 0, st>>>(phi, lg, tz, 0.25 / h, f);
        return;
    }
    const unsigned nb = blocks_for((size_t)n * n * n);
    if (periodic)
        k_force<true><<<nb, kBlock, 0, st>>>(phi, make_ix<true>(n, lg), 0.25 / h, f);
    else
        k_force<false><<<nb, kBlock, 0, st>>>(phi, make_ix<false>(n, lg), 0.25 / h, f);
}

} // namespace ndgp
