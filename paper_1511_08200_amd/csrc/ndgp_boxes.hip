// ndgp_boxes.hip -- the small boxes of an adaptive refinement tree solved
// together (Sec. IV.A: every refinement relaxed from its parent): one
// workgroup per box runs that box's whole solve -- interpolation from the
// parent, source, FAS V-cycles to the tolerance with the safeguard -- so
// that all small boxes of one tree level cost one launch instead of about
// forty launches and a host round trip per cycle each.
//
// Every step has the arithmetic, in the same order, of the per-level path
// (k_interpolate, k_source, k_partial_sums / k_residual_sumsq with
// k_reduce_final, k_smooth_half, k_restrict_residual, k_coarse_source,
// k_coarsest, k_prolong8, and the host's CycleMonitor), including the order
// of every reduction, so a box's result, cycle count and event counts are
// bit for bit those of relax_patch.  The finest level of a box of at most
// 16^3 cells and every 8^3 level live in LDS and are relaxed in place (a half
// sweep writes its colour's new values to an LDS buffer, waits, copies them
// in; ghosts of the coarse levels rewritten from their interior cell as
// write_owned_ghosts does); the 32^3 and 16^3 levels of a 32^3 box stay in
// global memory (L2, the box's scratch) and ping-pong like k_smooth_half.
#include "ndgp_device.h"

namespace ndgp {
namespace {

using namespace dev;

constexpr int kBoxThreads = 512;
constexpr int kPad16 = 18 * 18 * 18, kPad8 = 10 * 10 * 10;
constexpr int kMaxWaveSums = 32768 / 64; // one per wave of cells at 32^3

// one level of a box's hierarchy, as the workgroup sees it
struct BoxLevel {
    double *phi, *alt; // alt: levels in global memory only (out-of-place half sweeps)
    double *hat;       // levels >= 1
    double *s;
    Ix<false> ix;
    double al;
    bool dyn; // a coarse level: ghosts follow the interior
};

// the per-wave tree of block_sum (lanes combined by xor distance 32 .. 1)
__device__ __forceinline__ double wave_tree(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// LDS of one workgroup.  A 16^3 level lives here only as the finest level of
// a 16^3 box (phi and source; no hat); the 8^3 level always does.  newv holds
// the new values of one colour of an LDS level during a half sweep; the rest
// is the reduction scratch.
struct BoxShared {
    double phi16[kPad16], src16[4096], newv[2048];
    double phi8[kPad8], hat8[kPad8], src8[512];
    double ws[kMaxWaveSums], part[128], w4[4], bcast;
};

// The whole solve of one box of N0 cells per side (8, 16 or 32; 1, 2 or 3
// levels), by the workgroup; N0 fixes where each level lives.
template <int N0>
__device__ __forceinline__ void solve_box(const BoxJob &J, const BoxRun &R, BoxShared &S,
                                          BoxResult &out, unsigned &fb) {
    constexpr int NL = N0 == 8 ? 1 : N0 == 16 ? 2 : 3;
    const int tid = threadIdx.x;
    auto level = [&](int q) __attribute__((always_inline)) {
        BoxLevel V;
        const int n = N0 >> q, lg = 31 - __clz(n);
        V.ix = Ix<false>{n, lg, n + 2};
        V.al = q == 0 ? J.alpha[0] : q == 1 ? J.alpha[1] : J.alpha[2];
        V.dyn = q > 0;
        V.alt = nullptr;
        V.hat = nullptr;
        if (n == 32) {
            V.phi = J.phi;
            V.alt = J.alt;
            V.s = J.s0;
        } else if (n == 16 && q > 0) { // the middle level of a 32^3 box: global scratch
            V.phi = J.phi1;
            V.alt = J.alt1;
            V.hat = J.hat1;
            V.s = J.s1;
        } else if (n == 16) {
            V.phi = S.phi16;
            V.s = S.src16;
        } else {
            V.phi = S.phi8;
            V.hat = q ? S.hat8 : nullptr;
            V.s = S.src8;
        }
        return V;
    };
    const BoxLevel L0 = level(0), L1 = level(NL > 1 ? 1 : 0), L2 = level(NL > 2 ? 2 : 0);
    constexpr int cells0 = N0 * N0 * N0, pad0 = (N0 + 2) * (N0 + 2) * (N0 + 2);
    const int lgp = 31 - __clz(J.np);

    auto interp = [&](const ChildBox &bx, int slot) __attribute__((always_inline)) {
        const int pc = bx.nc + 2;
        const int ii = slot % pc, jj = (slot / pc) % pc, kk = slot / (pc * pc);
        return J.parent_periodic
                   ? interpolate_slot<true>(J.parent, J.np, lgp, bx, ii, jj, kk)
                   : interpolate_slot<false>(J.parent, J.np, lgp, bx, ii, jj, kk);
    };
    // the finest level from the parent, every slot (and the partner's shell)
    auto interpolate_level0 = [&](bool partner) __attribute__((always_inline)) {
        const ChildBox b0{{J.origin[0], J.origin[1], J.origin[2]}, 0, N0};
#pragma unroll 1
        for (int t = tid; t < pad0; t += kBoxThreads) {
            const double v = interp(b0, t);
            L0.phi[t] = v;
            if (N0 == 32 && partner) L0.alt[t] = v; // interior overwritten by every half sweep
        }
    };

    // The sum that k_partial_sums (or k_residual_sumsq) and k_reduce_final form
    // of per-cell values: cell c is thread c % 256 of block c / 256, each
    // block sums its four waves' trees as (w0 + w1) + (w2 + w3), the final
    // block takes block b's sum on thread b (cells0 / 256 <= 128 blocks;
    // every other partial is zero) and sums the same way.
    auto finish_sum = [&]() __attribute__((always_inline)) {
        __syncthreads();
        constexpr int nblk = cells0 >> 8;
        if (tid < nblk)
            S.part[tid] = (S.ws[4 * tid] + S.ws[4 * tid + 1]) + (S.ws[4 * tid + 2] + S.ws[4 * tid + 3]);
        __syncthreads();
        if (tid < 256) {
            const double acc = tid < nblk ? 0.0 + S.part[tid] : 0.0;
            const double v = wave_tree(acc);
            if ((tid & 63) == 0) S.w4[tid >> 6] = v;
        }
        __syncthreads();
        if (tid == 0) S.bcast = (S.w4[0] + S.w4[1]) + (S.w4[2] + S.w4[3]);
        __syncthreads();
        const double total = S.bcast;
        __syncthreads(); // the scratch is free again
        return total;
    };
    auto wave_sum_store = [&](int c, double v) __attribute__((always_inline)) {
        v = wave_tree(v);
        if ((tid & 63) == 0 && c < cells0) S.ws[c >> 6] = v;
    };
    auto source_sumsq = [&]() __attribute__((always_inline)) {
#pragma unroll 1
        for (int c = tid; c < ((cells0 + kBoxThreads - 1) / kBoxThreads) * kBoxThreads;
             c += kBoxThreads) {
            double v = 0.0;
            if (c < cells0) {
                const double a = L0.s[c];
                v = fma(a, a, 0.0);
            }
            wave_sum_store(c, v);
        }
        return finish_sum();
    };
    auto residual_sumsq = [&]() __attribute__((always_inline)) {
#pragma unroll 1
        for (int c = tid; c < ((cells0 + kBoxThreads - 1) / kBoxThreads) * kBoxThreads;
             c += kBoxThreads) {
            double v = 0.0;
            if (c < cells0) {
                const int i = c & (N0 - 1), j = (c >> L0.ix.lg) & (N0 - 1), k = c >> (2 * L0.ix.lg);
                double g[19];
                gather(L0.phi, L0.ix, i, j, k, g);
                const double r = L0.s[c] - apply_L(stencil_terms(g), L0.al);
                v = fma(r, r, 0.0);
            }
            wave_sum_store(c, v);
        }
        return finish_sum();
    };

    // `sweeps` red-black sweeps of a level with step factor w
    auto smooth = [&](const BoxLevel &V, int sweeps, double w) __attribute__((always_inline)) {
        const int n = V.ix.n, lg = V.ix.lg, half = n >> 1;
        const int ncol = (n * n * n) >> 1;
        if (V.alt) { // a level in global memory: out of place, as k_smooth_half
            double *pin = V.phi, *pout = V.alt;
            for (int h = 0; h < 2 * sweeps; ++h) {
                const int col = h & 1;
#pragma unroll 1
                for (int t = tid; t < ncol; t += kBoxThreads) {
                    const int m = t & (half - 1), row = t >> (lg - 1);
                    const int j = row & (n - 1), k = row >> lg;
                    const int off = (col ^ j ^ k) & 1;
                    const int iu = 2 * m + off, ic = 2 * m + 1 - off;
                    double g[19];
                    gather(pin, V.ix, iu, j, k, g);
                    const double un = relax_cell(g, V.s[((k << lg) + j) * n + iu], V.al, w, fb);
                    const double uc = pin[V.ix(ic, j, k)];
                    pout[V.ix(iu, j, k)] = un;
                    pout[V.ix(ic, j, k)] = uc;
                    if (V.dyn) {
                        write_owned_ghosts(pout, V.hat, V.ix, iu, j, k, un);
                        write_owned_ghosts(pout, V.hat, V.ix, ic, j, k, uc);
                    }
                }
                __syncthreads();
                double *tmp = pin;
                pin = pout;
                pout = tmp;
            }
            return; // an even number of half sweeps: back in V.phi
        }
        // in LDS, in place: the new values of the colour go to newv, then in
        for (int h = 0; h < 2 * sweeps; ++h) {
            const int col = h & 1;
#pragma unroll 1
            for (int t = tid; t < ncol; t += kBoxThreads) {
                const int m = t & (half - 1), row = t >> (lg - 1);
                const int j = row & (n - 1), k = row >> lg;
                const int i = 2 * m + ((col ^ j ^ k) & 1);
                double g[19];
                gather(V.phi, V.ix, i, j, k, g);
                S.newv[t] = relax_cell(g, V.s[((k << lg) + j) * n + i], V.al, w, fb);
            }
            __syncthreads();
#pragma unroll 1
            for (int t = tid; t < ncol; t += kBoxThreads) {
                const int m = t & (half - 1), row = t >> (lg - 1);
                const int j = row & (n - 1), k = row >> lg;
                const int i = 2 * m + ((col ^ j ^ k) & 1);
                const double v = S.newv[t];
                V.phi[V.ix(i, j, k)] = v;
                if (V.dyn) write_owned_ghosts(V.phi, V.hat, V.ix, i, j, k, v);
            }
            __syncthreads();
        }
    };

    // FAS restriction with the residual (F -> C) and the coarse source
    auto restrict_level = [&](const BoxLevel &F, const BoxLevel &C) __attribute__((always_inline)) {
        const int nc = C.ix.n, lgc = C.ix.lg, nf = F.ix.n;
#pragma unroll 1
        for (int t = tid; t < nc * nc * nc; t += kBoxThreads) {
            const int I = t & (nc - 1), J2 = (t >> lgc) & (nc - 1), K = t >> (2 * lgc);
            // restrict_cell's sums (children in its order), each child's stencil gathered
            double sphi = 0.0, sr = 0.0;
#pragma unroll 1
            for (int ch = 0; ch < 8; ++ch) {
                const int fi = 2 * I + (ch & 1), fj = 2 * J2 + ((ch >> 1) & 1), fk = 2 * K + (ch >> 2);
                double v[19];
                gather(F.phi, F.ix, fi, fj, fk, v);
                const double r = F.s[(fk * nf + fj) * nf + fi] - apply_L(stencil_terms(v), F.al);
                sphi += v[0];
                sr += r;
            }
            C.hat[C.ix(I, J2, K)] = sphi * 0.125;
            C.s[t] = sr * 0.5;
        }
        __syncthreads();
#pragma unroll 1
        for (int t = tid; t < nc * nc * nc; t += kBoxThreads) {
            const int i = t & (nc - 1), j = (t >> lgc) & (nc - 1), k = t >> (2 * lgc);
            double v[19];
            gather(C.hat, C.ix, i, j, k, v);
            C.s[t] = apply_L(stencil_terms(v), C.al) + C.s[t];
            C.phi[C.ix(i, j, k)] = v[0];
            write_owned_ghosts(C.phi, C.hat, C.ix, i, j, k, v[0]); // zero correction
        }
        __syncthreads();
    };

    // F += trilinear(phi - hat of C)
    auto prolong_level = [&](const BoxLevel &F, const BoxLevel &C) __attribute__((always_inline)) {
        const int nf = F.ix.n, lgf = F.ix.lg;
#pragma unroll 1
        for (int t = tid; t < nf * nf * nf; t += kBoxThreads) {
            const int i = t & (nf - 1), j = (t >> lgf) & (nf - 1), k = t >> (2 * lgf);
            const int I = i >> 1, J2 = j >> 1, K = k >> 1;
            const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        const double wt = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (c ? 0.25 : 0.75);
                        const int qq = C.ix(I + a * si, J2 + b * sj, K + c * sk);
                        acc = fma(wt, C.phi[qq] - C.hat[qq], acc);
                    }
            const int me = F.ix(i, j, k);
            const double val = F.phi[me] + acc;
            F.phi[me] = val;
            if (F.dyn) write_owned_ghosts(F.phi, F.hat, F.ix, i, j, k, val);
        }
        __syncthreads();
    };

    // vcycle(H, nl, 0) of the per-level path, written out for one to three levels
    auto vcycle = [&](double w) __attribute__((always_inline)) {
        if constexpr (NL == 1) {
            smooth(L0, R.csweeps, w);
        } else {
            smooth(L0, R.nu1, w);
            restrict_level(L0, L1);
            if constexpr (NL == 2) {
                smooth(L1, R.csweeps, w);
            } else {
                smooth(L1, R.nu1, w);
                restrict_level(L1, L2);
                smooth(L2, R.csweeps, w);
                prolong_level(L1, L2);
                smooth(L1, R.nu2, w);
            }
            prolong_level(L0, L1);
            smooth(L0, R.nu2, w);
        }
    };

    // ---- set-up: the finest level, the coarse levels' hat shells, the source
    interpolate_level0(true);
    auto hat_shell = [&](const BoxLevel &V, int q) __attribute__((always_inline)) {
        const ChildBox bq{{J.origin[0], J.origin[1], J.origin[2]}, q, V.ix.n};
        const int pc = V.ix.n + 2;
#pragma unroll 1
        for (int t = tid; t < pc * pc * pc; t += kBoxThreads) {
            const int ii = t % pc, jj = (t / pc) % pc, kk = t / (pc * pc);
            const bool interior = ii >= 1 && ii <= bq.nc && jj >= 1 && jj <= bq.nc && kk >= 1 &&
                                  kk <= bq.nc;
            if (!interior) V.hat[t] = interp(bq, t);
        }
    };
    if constexpr (NL > 1) hat_shell(L1, 1);
    if constexpr (NL > 2) hat_shell(L2, 2);
    {
        const double mean = R.dsum[0] * R.inv_cells0;
#pragma unroll 1
        for (int t = tid; t < cells0; t += kBoxThreads) L0.s[t] = J.f * (J.delta[t] - mean);
    }
    __syncthreads();

    double sn2 = source_sumsq();
    if (!__builtin_isfinite(sn2)) {
        out.status = kBoxBadSource;
    } else {
        if (sn2 == 0.0) {
            const double rr = residual_sumsq();
            sn2 = rr < 1e-300 ? 1e-300 : rr; // std::max(rr, 1e-300)
        }
        double w = 1.0;
        if (R.damped_start) {
            w = kDampedStep;
            out.damped_from = 1;
        }
        // the cycles of relax_patch's drive(), twice when the safeguard asks
        for (int pass = 0; pass < 2; ++pass) {
            const bool may_restart = pass == 0;
            CycleMonitor m{R.tol, R.maxc};
            m.damped = w != 1.0;
            m.start(sqrt(residual_sumsq() / sn2));
            bool restart = false;
            int code = 0;
            while (out.cycles < m.maxc && !m.converged()) {
                vcycle(w);
                ++out.cycles;
                const double r = sqrt(residual_sumsq() / sn2);
                const bool again = m.record(r);
                if (again && may_restart) {
                    restart = true;
                    break;
                }
                if (m.diverged()) {
                    code = kBoxDiverged;
                    break;
                }
                if (m.stalled()) break;
            }
            out.rel = m.rel;
            if (!restart) {
                out.status = code ? code : m.verdict_code();
                break;
            }
            // the safeguard: from the interpolated guess again, damped
            w = kDampedStep;
            out.damped_from = out.cycles + 1;
            interpolate_level0(false);
            __syncthreads();
        }
    }
    // a finest level held in LDS goes back to the box's array
    if constexpr (N0 <= 16)
#pragma unroll 1
        for (int t = tid; t < pad0; t += kBoxThreads) J.phi[t] = L0.phi[t];
}

__global__ void __launch_bounds__(kBoxThreads)
k_solve_boxes(const BoxJob *__restrict__ jobs, BoxResult *__restrict__ results, BoxRun R) {
    __shared__ BoxShared S;
    const BoxJob J = jobs[blockIdx.x];
    BoxResult out{0, 0, 0, 0.0};
    unsigned fb = 0;
    if (J.n == 8)
        solve_box<8>(J, R, S, out, fb);
    else if (J.n == 16)
        solve_box<16>(J, R, S, out, fb);
    else
        solve_box<32>(J, R, S, out, fb);
    if (threadIdx.x == 0) results[blockIdx.x] = out;
    if (fb) flush_events(R.fallbacks, fb);
}

} // namespace

void launch_solve_boxes(const BoxJob *jobs, BoxResult *results, int count, const BoxRun &run,
                        hipStream_t st) {
    if (count > 0) k_solve_boxes<<<count, kBoxThreads, 0, st>>>(jobs, results, run);
}

} // namespace ndgp
