// ndgp_amr.hip -- placement of refinement patches (host code).
//
// Sec. IV.A of arXiv:1511.08200 refines every cell that holds more than N_ref
// particles; ndgp_refine_flags marks those cells.  Here the marked cells of one
// level are grouped into rectangular clusters by the point-clustering
// algorithm of Berger & Rigoutsos ("An algorithm for point clustering and grid
// generation", IEEE Trans. Syst. Man Cybern. 21, 1991), and each cluster is
// turned into cubic patches of 2^k cells at twice the resolution, the shape
// the solver's per-patch multigrid needs.  The cubes sit on an octree lattice,
// where two cubes either nest or lie apart: keeping the larger of any two that
// meet leaves siblings that never hold two values for one place.

#include "ndgp.h"
#include "ndgp_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

namespace {

using ndgp::child_fits_axis;
using ndgp::default_levels;

struct Cluster {
    int lo[3], hi[3]; // half-open, in the (cut-open) parent cell coordinates
    int extent(int a) const { return hi[a] - lo[a]; }
};

// The flags of one level, read through the cut that opens a periodic level:
// coordinate u along axis a is parent cell (u + shift[a]) mod n.
struct FlagView {
    const uint8_t *f;
    int n;
    int shift[3];
    bool at(int u, int v, int w) const {
        const int i = (u + shift[0]) % n, j = (v + shift[1]) % n, k = (w + shift[2]) % n;
        return f[((size_t)k * n + j) * n + i] != 0;
    }
};

// signatures of the flags inside c: sig[a][t] = flagged cells in slab t of axis a
void signatures(const FlagView &F, const Cluster &c, std::vector<int64_t> sig[3], int64_t &count) {
    for (int a = 0; a < 3; ++a) sig[a].assign(c.extent(a), 0);
    count = 0;
    for (int w = c.lo[2]; w < c.hi[2]; ++w)
        for (int v = c.lo[1]; v < c.hi[1]; ++v)
            for (int u = c.lo[0]; u < c.hi[0]; ++u)
                if (F.at(u, v, w)) {
                    ++sig[0][u - c.lo[0]];
                    ++sig[1][v - c.lo[1]];
                    ++sig[2][w - c.lo[2]];
                    ++count;
                }
}

void berger_rigoutsos(const FlagView &F, Cluster c, double efficiency, int min_width,
                      std::vector<Cluster> &out) {
    std::vector<int64_t> sig[3];
    int64_t count = 0;
    signatures(F, c, sig, count);
    if (count == 0) return;
    // shrink to the bounding box of the flags (slabs without flags leave the
    // other axes' signatures unchanged)
    for (int a = 0; a < 3; ++a) {
        int b = 0, e = c.extent(a);
        while (sig[a][b] == 0) ++b;
        while (sig[a][e - 1] == 0) --e;
        sig[a] = std::vector<int64_t>(sig[a].begin() + b, sig[a].begin() + e);
        c.hi[a] = c.lo[a] + e;
        c.lo[a] += b;
    }
    const double volume = (double)c.extent(0) * c.extent(1) * c.extent(2);
    const int widest = std::max({c.extent(0), c.extent(1), c.extent(2)});
    if ((double)count >= efficiency * volume || widest <= min_width) {
        out.push_back(c);
        return;
    }
    int axis = -1, cut = 0; // split into [lo, lo + cut) and [lo + cut (+1 at a hole), hi)
    bool hole = false;
    // 1. a hole in a signature: the slab nearest the middle of its axis
    int best_off = 1 << 30;
    for (int a = 0; a < 3; ++a)
        for (int t = 1; t + 1 < c.extent(a); ++t)
            if (sig[a][t] == 0) {
                const int off = std::abs(2 * t - c.extent(a));
                if (off < best_off || (off == best_off && c.extent(a) > c.extent(axis))) {
                    best_off = off;
                    axis = a;
                    cut = t;
                    hole = true;
                }
            }
    // 2. the strongest sign change of the signatures' second difference
    if (axis < 0) {
        int64_t best = 0;
        for (int a = 0; a < 3; ++a) {
            const int e = c.extent(a);
            if (e < 4) continue;
            std::vector<int64_t> lap(e, 0);
            for (int t = 1; t + 1 < e; ++t) lap[t] = sig[a][t - 1] - 2 * sig[a][t] + sig[a][t + 1];
            for (int t = 1; t + 2 < e; ++t)
                if ((lap[t] < 0 && lap[t + 1] > 0) || (lap[t] > 0 && lap[t + 1] < 0)) {
                    const int64_t strength = std::abs(lap[t + 1] - lap[t]);
                    const int off = std::abs(2 * (t + 1) - e);
                    if (strength > best || (strength == best && axis >= 0 && off < best_off)) {
                        best = strength;
                        best_off = off;
                        axis = a;
                        cut = t + 1;
                    }
                }
        }
    }
    // 3. the middle of the longest side
    if (axis < 0) {
        axis = 0;
        for (int a = 1; a < 3; ++a)
            if (c.extent(a) > c.extent(axis)) axis = a;
        cut = c.extent(axis) / 2;
    }
    Cluster left = c, right = c;
    left.hi[axis] = c.lo[axis] + cut;
    right.lo[axis] = c.lo[axis] + cut + (hole ? 1 : 0);
    berger_rigoutsos(F, left, efficiency, min_width, out);
    berger_rigoutsos(F, right, efficiency, min_width, out);
}

struct Cube {
    Cluster c;     // the flagged cells it must cover
    int w = 0;     // child cells per side
    int o[3] = {}; // lower corner, cut-open parent coordinates
};

// the widest cube a level can hold: at most 512 cells and twice the level's
// cells per side, and on a patch parent one that fits inside it
int widest_cube(int n, bool periodic) {
    int w = 512;
    while (w > 2 * n) w /= 2;
    if (!periodic)
        while (w >= 8) {
            const int nlev = default_levels(w);
            bool any = false;
            for (int o = -n; o <= n && !any; ++o) any = child_fits_axis(n, o, w, nlev);
            if (any) break;
            w /= 2;
        }
    return w;
}

bool overlap(const Cube &x, const Cube &y) {
    for (int a = 0; a < 3; ++a)
        if (!(x.o[a] < y.o[a] + y.w / 2 && y.o[a] < x.o[a] + x.w / 2)) return false;
    return true;
}

int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Cubes on an octree lattice: a cube of w child cells (w/2 parent cells, a
// power of two >= 8) sits at L0 + t w/2 along each axis.  Two lattice cubes
// either nest or lie apart, so overlaps are removed by keeping the larger.
// On a periodic level the lattice starts at the cut (L0 = 0 in cut-open
// coordinates) and tiles it exactly; on a patch parent L0 is the lowest
// corner at which the widest cube fits, and only cubes that fit the parent
// with room for their stencils are used (flagged cells that none reaches,
// next to the parent's boundary, stay unrefined).
struct Lattice {
    int n, L0, wmax;
    bool periodic;
    bool fits(const Cube &q) const {
        if (periodic) return true;
        for (int a = 0; a < 3; ++a)
            if (!child_fits_axis(n, q.o[a], q.w, default_levels(q.w))) return false;
        return true;
    }
};

// lattice cubes of width w that meet the flags of c (each with the part of c
// it holds), and whether they all fit
bool lattice_tiles(const FlagView &F, const Lattice &L, const Cluster &c, int w,
                   std::vector<Cube> &tiles) {
    const int span = w / 2;
    int t0[3], t1[3];
    for (int a = 0; a < 3; ++a) {
        t0[a] = floor_div(c.lo[a] - L.L0, span);
        t1[a] = floor_div(c.hi[a] - 1 - L.L0, span);
    }
    bool all_fit = true;
    for (int tk = t0[2]; tk <= t1[2]; ++tk)
        for (int tj = t0[1]; tj <= t1[1]; ++tj)
            for (int ti = t0[0]; ti <= t1[0]; ++ti) {
                Cube g;
                g.w = w;
                g.o[0] = L.L0 + ti * span;
                g.o[1] = L.L0 + tj * span;
                g.o[2] = L.L0 + tk * span;
                Cluster t;
                for (int a = 0; a < 3; ++a) {
                    t.lo[a] = std::max(c.lo[a], g.o[a]);
                    t.hi[a] = std::min(c.hi[a], g.o[a] + span);
                }
                std::vector<int64_t> sig[3];
                int64_t count = 0;
                signatures(F, t, sig, count);
                if (count == 0) continue;
                g.c = t;
                if (L.fits(g))
                    tiles.push_back(g);
                else
                    all_fit = false;
            }
    return all_fit;
}

// A cluster's cubes: of the lattice cubes just wide enough for it (as tiles)
// and the smallest single lattice cube around it, the choice with the smaller
// volume; narrower tiles where wide ones do not fit the parent.
void fit_cluster(const FlagView &F, const Lattice &L, const Cluster &c, std::vector<Cube> &out) {
    if (L.wmax < 8) return;
    const int e = std::max({c.extent(0), c.extent(1), c.extent(2)});
    int wc = 8;
    while (wc < 2 * e && wc < L.wmax) wc *= 2;
    Cube single;
    for (int w = wc; w <= L.wmax && single.w == 0; w *= 2) {
        Cube q;
        q.c = c;
        q.w = w;
        bool ok = true;
        for (int a = 0; a < 3 && ok; ++a) {
            q.o[a] = L.L0 + floor_div(c.lo[a] - L.L0, w / 2) * (w / 2);
            ok = q.o[a] + w / 2 >= c.hi[a];
        }
        if (ok && L.fits(q)) single = q;
    }
    for (int w = wc; w >= 8; w /= 2) {
        std::vector<Cube> tiles;
        const bool all_fit = lattice_tiles(F, L, c, w, tiles);
        if (!all_fit && w > 8) continue;
        const double vt = (double)tiles.size() * (w / 2) * (w / 2) * (w / 2);
        const double vs = single.w ? std::pow(single.w / 2.0, 3) : 1e300;
        if (single.w && vs <= vt)
            out.push_back(single);
        else
            out.insert(out.end(), tiles.begin(), tiles.end());
        return;
    }
}

ndgp_status refine_boxes_impl(const unsigned char *flags, int on_device, int n, int periodic,
                              int parent_index, double efficiency, int min_width, ndgp_box *boxes,
                              int max_boxes, int *n_boxes, hipStream_t st) {
    auto fail = [](ndgp_status s, const std::string &m) {
        ndgp::set_last_error(m.c_str());
        return s;
    };
    if (!flags || !boxes || !n_boxes) return fail(NDGP_EINVAL, "flags, boxes and n_boxes must not be NULL");
    if (n < 8 || n > 1024 || (n & (n - 1))) return fail(NDGP_EINVAL, "n must be a power of two in [8, 1024]");
    if (!(efficiency > 0.0 && efficiency <= 1.0) || min_width < 1)
        return fail(NDGP_EINVAL, "need 0 < efficiency <= 1 and min_width >= 1");
    if (parent_index < -1 || max_boxes < 0) return fail(NDGP_EINVAL, "bad parent_index or max_boxes");
    const size_t cells = (size_t)n * n * n;
    std::vector<uint8_t> f(cells);
    if (on_device) {
        hipError_t e = hipMemcpyAsync(f.data(), flags, cells, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            return fail(NDGP_EDEVICE, std::string("flags copy: ") + hipGetErrorString(e));
    } else {
        std::memcpy(f.data(), flags, cells);
    }
    FlagView F{f.data(), n, {0, 0, 0}};
    if (periodic) { // cut each axis open in the middle of its widest empty slab
        for (int a = 0; a < 3; ++a) {
            std::vector<int64_t> sig(n, 0);
            for (int k = 0; k < n; ++k)
                for (int j = 0; j < n; ++j)
                    for (int i = 0; i < n; ++i)
                        if (f[((size_t)k * n + j) * n + i]) ++sig[a == 0 ? i : (a == 1 ? j : k)];
            int best_len = 0, best_mid = 0;
            for (int t = 0; t < n; ++t) {
                if (sig[t] != 0 || sig[(t + n - 1) % n] == 0) continue; // start of an empty run
                int len = 0;
                while (len < n && sig[(t + len) % n] == 0) ++len;
                if (len > best_len) {
                    best_len = len;
                    best_mid = (t + len / 2) % n;
                }
            }
            F.shift[a] = best_len > 0 ? best_mid : 0;
        }
    }
    std::vector<Cluster> clusters;
    berger_rigoutsos(F, Cluster{{0, 0, 0}, {n, n, n}}, efficiency, min_width, clusters);
    Lattice L{n, 0, widest_cube(n, periodic != 0), periodic != 0};
    if (!periodic)
        for (int o = -n; o <= n; ++o)
            if (L.wmax >= 8 && child_fits_axis(n, o, L.wmax, default_levels(L.wmax))) {
                L.L0 = o;
                break;
            }
    std::vector<Cube> cubes;
    for (const Cluster &c : clusters) fit_cluster(F, L, c, cubes);
    // lattice cubes nest or lie apart: drop every cube inside a larger (or an
    // equal, earlier) one
    std::vector<Cube> kept;
    for (size_t x = 0; x < cubes.size(); ++x) {
        bool inside = false;
        for (size_t y = 0; y < cubes.size() && !inside; ++y)
            if (y != x && overlap(cubes[x], cubes[y]) &&
                (cubes[y].w > cubes[x].w || (cubes[y].w == cubes[x].w && y < x)))
                inside = true;
        if (!inside) kept.push_back(cubes[x]);
    }
    cubes.swap(kept);
    if ((int)cubes.size() > max_boxes)
        return fail(NDGP_ENOMEM, "the flags need " + std::to_string(cubes.size()) +
                                     " boxes, more than max_boxes");
    // a deterministic order: by corner (z, y, x)
    std::sort(cubes.begin(), cubes.end(), [](const Cube &x, const Cube &y) {
        for (int a = 2; a >= 0; --a)
            if (x.o[a] != y.o[a]) return x.o[a] < y.o[a];
        return x.w < y.w;
    });
    for (size_t b = 0; b < cubes.size(); ++b) {
        ndgp_box &B = boxes[b];
        B.parent = parent_index;
        B.n = cubes[b].w;
        for (int a = 0; a < 3; ++a) {
            const int o = cubes[b].o[a] + F.shift[a];
            B.origin[a] = periodic ? ((o % n) + n) % n : o;
        }
    }
    *n_boxes = (int)cubes.size();
    return NDGP_OK;
}

} // namespace

extern "C" ndgp_status ndgp_refine_boxes(const unsigned char *flags, int32_t flags_on_device,
                                         int32_t n, int32_t periodic, int32_t parent_index,
                                         double efficiency, int32_t min_width, ndgp_box *boxes,
                                         int32_t max_boxes, int32_t *n_boxes,
                                         hipStream_t stream) {
    try {
        return refine_boxes_impl(flags, flags_on_device, n, periodic, parent_index, efficiency,
                                 min_width, boxes, max_boxes, n_boxes, stream);
    } catch (const std::exception &e) {
        ndgp::set_last_error(e.what());
        return NDGP_EDEVICE;
    }
}
