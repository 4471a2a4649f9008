// Batched solvers for the projected shifted Sternheimer equations
//   Q (H - s_j) Q z_j = b_j,   b_j in range(Q),  z_j(0) = 0        (Eq. (3.6))
// H = -1/2 Delta_h + diag(V_eff), Q = I - Phi Phi^T.
//
// Design (gfx950):
//  * Each workgroup owns one tile of 16 systems for the whole solve and all
//    N_g rows, so every reduction of the method (Phi^T y, p^T A p, |r|^2) is
//    workgroup-local: no grid synchronisation, no per-iteration launches, and a
//    tile leaves the loop as soon as its 16 systems have converged.
//  * Vectors use the 16-column row-interleaved layout: one grid row of a tile
//    is a 128-byte line, so a wave touching 4 rows x 16 systems issues fully
//    coalesced loads, and the 64 values a wave holds are exactly the B operand
//    of one v_mfma_f64_16x16x4 (k = row, n = system).
//  * The stencil (8th-order Laplacian + V_eff - shift) is fused with the
//    projector: pass 1 forms p, y = (H - s) p and C = Phi^T y on the matrix
//    cores (waves split the orbital blocks, y staged through LDS); pass 2
//    recomputes y from p, forms A p = y - Phi C on the matrix cores and updates
//    x and r in the same sweep.  y and A p never touch memory.
//  * p^T A p is taken as p^T y: p stays in range(Q) to rounding, and the
//    neglected term (Phi^T p)^T (Phi^T y) is second order in that rounding.
//
// CG (the operator is positive definite on range(Q) when every shift lies
// below the lowest unoccupied eigenvalue): 8 vector sweeps per iteration
// (read r, p_old; write p | read p, x, r; write x, r).  p is double-buffered so
// the stencil in pass 1 can recompute p = r + beta p_old at neighbour rows
// without a race.
//
// MINRES (the solver the paper uses, Sec. 2.2 after Eq. (2.18)): Lanczos
// three-term recurrence with the tridiagonal least-squares problem reduced by
// Givens rotations, per system; three sweeps per iteration.
#include "acp_internal.h"

namespace acp {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NW = 8;             // waves per workgroup (2 per SIMD)
constexpr int NT = 64 * NW;       // threads per workgroup
constexpr int MAXNB = 16;         // up to 256 (padded) orbitals

__device__ __forceinline__ int wrap(int i, int n) {
    if (i < 0) i += n;
    if (i >= n) i -= n;
    return i;
}

// Neighbour rows of the 4-row group R..R+3 of one system, for the 8th-order
// stencil.  1D: rows R-4 .. R+7 (12 rows, periodic).  2D: for each of the 4 rows
// its 8 x-neighbours and 8 y-neighbours.  Every index is clamped into [0, ng)
// so that all loads can be issued unconditionally (rows past the end of the grid
// in the last block are computed but never stored).
template <int DIM>
struct Nbr {
    static constexpr int N = DIM == 1 ? 12 : 4 * 17;
    int idx[N];
    __device__ __forceinline__ Nbr(int R, const GridDesc &g) {
        if (DIM == 1) {
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                int rr = R - 4 + q;
                rr = rr < 0 ? rr + g.ng : rr;
                rr = rr >= g.ng ? rr - g.ng : rr;
                idx[q] = rr < g.ng ? rr : g.ng - 1;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int row = R + j;
                row = row < g.ng ? row : g.ng - 1;
                const int ix = row % g.nx, iy = row - ix;
                idx[17 * j] = row;
#pragma unroll
                for (int k = 1; k <= 4; ++k) {
                    idx[17 * j + k] = iy + wrap(ix + k, g.nx);
                    idx[17 * j + 4 + k] = iy + wrap(ix - k, g.nx);
                    const int iyk = iy / g.nx;
                    idx[17 * j + 8 + k] = wrap(iyk + k, g.ny) * g.nx + ix;
                    idx[17 * j + 12 + k] = wrap(iyk - k, g.ny) * g.nx + ix;
                }
            }
        }
    }
};

// y = (H - s) p at rows R..R+3 from gathered values w[] laid out as in Nbr.
template <int DIM>
__device__ __forceinline__ void stencil_from(const double (&w)[Nbr<DIM>::N], int R,
                                             const GridDesc &g, const double *__restrict__ V,
                                             double s, double (&y)[4], double (&pc)[4]) {
    const double c2 = -0.5 / (g.h * g.h);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int row = R + j;
        const bool ok = row < g.ng;
        const double v = V[ok ? row : g.ng - 1];
        double c, lap;
        if (DIM == 1) {
            c = w[4 + j];
            lap = fd8(0) * c;
#pragma unroll
            for (int k = 1; k <= 4; ++k) lap += fd8(k) * (w[4 + j + k] + w[4 + j - k]);
        } else {
            c = w[17 * j];
            lap = 2.0 * fd8(0) * c;
#pragma unroll
            for (int k = 1; k <= 4; ++k)
                lap += fd8(k) * (w[17 * j + k] + w[17 * j + 4 + k] + w[17 * j + 8 + k] + w[17 * j + 12 + k]);
        }
        pc[j] = ok ? c : 0.0;
        y[j] = ok ? (c2 * lap + (v - s) * c) : 0.0;
    }
}

// Sum over the threads of one column (threads t with t % 16 == col) of a
// per-thread value, in a fixed order; the total lands in red_out[col].
__device__ __forceinline__ void column_reduce(double v, double *red, double *red_out) {
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < kTile) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NT / kTile; ++k) s += red[threadIdx.x + kTile * k];
        red_out[threadIdx.x] = s;
    }
    __syncthreads();
}

// LDS slots for the cross-wave reduction of C = Phi^T y (64 KB in total).
template <int NB>
struct Slots {
    static constexpr int NEP = NB * 16;
    static constexpr int N = (512 / NEP) < NW ? (512 / NEP) : NW;
    static constexpr int ELEMS = NEP * kTile;
};

// Pass 1 of the projected apply.  Each wave owns the 16-row blocks b = wave,
// wave + NW, ...; lane l (q = l/16) computes p and y = (H - s) p at the four
// consecutive rows 16 b + 4 q + j of system l % 16 and feeds y(row) to the
// MFMA k-step j, whose k index q stands for that row (the contraction runs
// over rows, so any row order works as long as the A operand follows it).
// C = Phi^T y is reduced across waves in LDS into slots[0] (orbital-major,
// 16 systems per orbital).  Returns this thread's share of p^T y.
template <int DIM, int NB>
__device__ __forceinline__ double apply_pass1(const double *__restrict__ rv, const double *__restrict__ pv,
                                              double beta, const KrylovArgs &a, double s,
                                              double *slots, double *__restrict__ pstore) {
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int col = lane & 15;
    const int q = lane >> 4;
    constexpr int nep = NB * 16;
    constexpr int NN = Nbr<DIM>::N;
    d4 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = d4{0.0, 0.0, 0.0, 0.0};
    double pty = 0.0;
    for (int blk = wave; blk * 16 < a.g.ng; blk += NW) {
        const int R = blk * 16 + 4 * q;
        const Nbr<DIM> nb(R, a.g);
        // issue every load of the block before any use
        double w[NN], wp[NN];
#pragma unroll
        for (int k = 0; k < NN; ++k) w[k] = rv[nb.idx[k] * kTile + col];
        if (pv) {
#pragma unroll
            for (int k = 0; k < NN; ++k) wp[k] = pv[nb.idx[k] * kTile + col];
        }
        double av[4][NB];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = R + j < a.g.ng ? R + j : a.g.ng - 1;
            const double *ph = a.phi_rm + (long long)row * nep + col;
#pragma unroll
            for (int mb = 0; mb < NB; ++mb) av[j][mb] = ph[mb * 16];
        }
        if (pv) {
#pragma unroll
            for (int k = 0; k < NN; ++k) w[k] += beta * wp[k];
        }
        double y[4], pc[4];
        stencil_from<DIM>(w, R, a.g, a.veff, s, y, pc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            pty += pc[j] * y[j];
            if (pstore && R + j < a.g.ng) pstore[(R + j) * kTile + col] = pc[j];
        }
        // rows past the end contribute y = 0, so their (clamped) Phi rows are harmless
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int mb = 0; mb < NB; ++mb)
                acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j][mb], y[j], acc[mb], 0, 0, 0);
    }
    // deterministic cross-wave reduction: phases of Slots::N waves
    using S = Slots<NB>;
#pragma unroll 1
    for (int ph = 0; ph < NW / S::N; ++ph) {
        if (wave / S::N == ph) {
            double *dst = slots + (wave % S::N) * S::ELEMS;
#pragma unroll
            for (int mb = 0; mb < NB; ++mb)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int idx = (mb * 16 + q + 4 * e) * kTile + col;
                    if (ph == 0) dst[idx] = acc[mb][e];
                    else dst[idx] += acc[mb][e];
                }
        }
        __syncthreads();
    }
    for (int idx = t; idx < S::ELEMS; idx += NT) {
        double v = slots[idx];
#pragma unroll
        for (int k = 1; k < S::N; ++k) v += slots[k * S::ELEMS + idx];
        slots[idx] = v;
    }
    return pty;
}

// Pass 2 helper: for the 16-row block starting at row0, D = Phi(rows,:) C on
// the matrix cores.  The f64 MFMA returns D[l/16 + 4 e][l%16] to lane l, so the
// A operand feeds grid row 4 (m % 4) + m / 4 into MFMA row m: lane l then holds
// the consecutive grid rows row0 + 4*(l/16) + e of system l % 16.
template <int NB>
__device__ __forceinline__ d4 project_block(const KrylovArgs &a, const double *Cs, int row0) {
    const int lane = threadIdx.x & 63;
    constexpr int nep = NB * 16;
    const int m = lane & 15;
    int row = row0 + 4 * (m & 3) + (m >> 2);
    row = row < a.g.ng ? row : a.g.ng - 1;   // clamped rows feed outputs that are never stored
    const double *ph = a.phi_cm + row + (long long)(lane >> 4) * a.g.ng;
    double av[nep / 4];
#pragma unroll
    for (int k = 0; k < nep / 4; ++k) av[k] = ph[(long long)(4 * k) * a.g.ng];
    d4 d = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < nep / 4; ++k) {
        const double bv = Cs[(4 * k + (lane >> 4)) * kTile + (lane & 15)];
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(av[k], bv, d, 0, 0, 0);
    }
    return d;
}

// Gather the stencil neighbourhood of rows R..R+3 of one system from v.
template <int DIM>
__device__ __forceinline__ void gather(const double *__restrict__ v, int R, const GridDesc &g,
                                       int col, double (&w)[Nbr<DIM>::N]) {
    const Nbr<DIM> nb(R, g);
#pragma unroll
    for (int k = 0; k < Nbr<DIM>::N; ++k) w[k] = v[nb.idx[k] * kTile + col];
}

template <int DIM, int NB>
__global__ __launch_bounds__(NT) void cg_kernel(KrylovArgs a) {
    __shared__ double slots[Slots<NB>::N * Slots<NB>::ELEMS];
    __shared__ double red[NT];
    __shared__ double s_rr[kTile], s_alpha[kTile], s_beta[kTile], s_bn[kTile], s_tmp[kTile];
    __shared__ int s_active[kTile], s_iters[kTile], s_flag[kTile], s_any;

    const int tile = blockIdx.x;
    const int t = threadIdx.x;
    const int col = t & 15;
    const int lane = t & 63;
    const int wave = t >> 6;
    const long long base = (long long)tile * a.g.ng * kTile;
    const double *__restrict__ b = a.rhs + (long long)(tile % a.rhs_tiles) * a.g.ng * kTile;
    double *__restrict__ x = a.x + base;
    double *__restrict__ r = a.r + base;
    double *pA = a.pa + base;
    double *pB = a.pb + base;
    const double s = a.shift[tile * kTile + col];

    // init: x = 0, r = b, p_old = 0, rr = |b|^2
    double part = 0.0;
    for (int idx = t; idx < a.g.ng * kTile; idx += NT) {
        const double bv = b[idx];
        x[idx] = 0.0;
        r[idx] = bv;
        pA[idx] = 0.0;
        part += bv * bv;   // idx % 16 == t % 16 == col since NT % 16 == 0
    }
    column_reduce(part, red, s_rr);
    if (t < kTile) {
        s_bn[t] = sqrt(s_rr[t]);
        s_beta[t] = 0.0;
        s_iters[t] = 0;
        s_flag[t] = 0;
        s_active[t] = (s_bn[t] > 0.0) ? 1 : 0;
    }
    __syncthreads();

    int it = 0;
    for (; it < a.max_iter; ++it) {
        if (t == 0) {
            int any = 0;
            for (int c = 0; c < kTile; ++c) any |= s_active[c];
            s_any = any;
        }
        __syncthreads();
        if (!s_any) break;
        // ---- pass 1: p = r + beta p_old (into pB), y = (H - s) p, C = Phi^T y, p^T y
        const double beta = s_beta[col];
        const double pty = apply_pass1<DIM, NB>(r, pA, beta, a, s, slots, pB);
        column_reduce(pty, red, s_tmp);
        if (t < kTile) {
            double al = 0.0;
            if (s_active[t]) {
                if (s_tmp[t] > 0.0) {
                    al = s_rr[t] / s_tmp[t];
                } else {
                    s_flag[t] |= 2;
                    s_active[t] = 0;
                }
            }
            s_alpha[t] = al;
        }
        __syncthreads();
        // ---- pass 2: A p = y - Phi C; x += alpha p; r -= alpha A p; |r|^2
        double rr_part = 0.0;
        const double al = s_alpha[col];
        for (int blk = wave; blk * 16 < a.g.ng; blk += NW) {
            const int row0 = blk * 16;
            const int R = row0 + 4 * (lane >> 4);
            double w[Nbr<DIM>::N];
            gather<DIM>(pB, R, a.g, col, w);
            double xo[4], ro[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = R + e < a.g.ng ? R + e : a.g.ng - 1;
                xo[e] = x[row * kTile + col];
                ro[e] = r[row * kTile + col];
            }
            const d4 d = project_block<NB>(a, slots, row0);
            double y[4], pc[4];
            stencil_from<DIM>(w, R, a.g, a.veff, s, y, pc);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double ap = y[e] - d[e];
                const double xn = xo[e] + al * pc[e];
                const double rn = ro[e] - al * ap;
                if (R + e < a.g.ng) {
                    x[(R + e) * kTile + col] = xn;
                    r[(R + e) * kTile + col] = rn;
                    rr_part += rn * rn;
                }
            }
        }
        column_reduce(rr_part, red, s_tmp);
        if (t < kTile) {
            if (s_active[t]) {
                s_beta[t] = s_tmp[t] / s_rr[t];
                s_rr[t] = s_tmp[t];
                s_iters[t] += 1;
                if (sqrt(s_rr[t]) <= a.tol * s_bn[t]) s_active[t] = 0;
            } else {
                s_beta[t] = 0.0;
            }
        }
        __syncthreads();
        double *tmp = pA; pA = pB; pB = tmp;
    }
    if (t < kTile) {
        const int gc = tile * kTile + t;
        a.iters[gc] = s_iters[t];
        a.resid[gc] = (s_bn[t] > 0.0) ? sqrt(s_rr[t]) / s_bn[t] : 0.0;
        a.flags[gc] = s_flag[t] | (s_active[t] ? 1 : 0);
    }
    if (t == 0) a.tile_iters[tile] = it;
}

// MINRES: v (current Lanczos vector), vo (previous, overwritten by the next),
// w, wo (direction vectors), x.  Buffers: pa = v, pb = vo, w1 = w, w2 = wo.
template <int DIM, int NB>
__global__ __launch_bounds__(NT) void minres_kernel(KrylovArgs a) {
    __shared__ double slots[Slots<NB>::N * Slots<NB>::ELEMS];
    __shared__ double red[NT];
    __shared__ double s_beta[kTile], s_alpha[kTile], s_bn[kTile], s_tmp[kTile];
    __shared__ double s_cs[kTile], s_sn[kTile], s_dbar[kTile], s_epsn[kTile], s_phibar[kTile];
    __shared__ double s_delta[kTile], s_gamma[kTile], s_epsk[kTile], s_phi[kTile], s_binv[kTile];
    __shared__ int s_active[kTile], s_iters[kTile], s_flag[kTile], s_any;

    const int tile = blockIdx.x;
    const int t = threadIdx.x;
    const int col = t & 15;
    const int lane = t & 63;
    const int wave = t >> 6;
    const long long base = (long long)tile * a.g.ng * kTile;
    const double *__restrict__ b = a.rhs + (long long)(tile % a.rhs_tiles) * a.g.ng * kTile;
    double *__restrict__ x = a.x + base;
    double *v = a.pa + base;
    double *vo = a.pb + base;
    double *w = a.w1 + base;
    double *wo = a.w2 + base;
    const double s = a.shift[tile * kTile + col];

    double part = 0.0;
    for (int idx = t; idx < a.g.ng * kTile; idx += NT) {
        const double bv = b[idx];
        part += bv * bv;
    }
    column_reduce(part, red, s_tmp);
    if (t < kTile) {
        const double bn = sqrt(s_tmp[t]);
        s_bn[t] = bn;
        s_binv[t] = bn > 0.0 ? 1.0 / bn : 0.0;
        s_beta[t] = bn;
        s_cs[t] = -1.0;
        s_sn[t] = 0.0;
        s_dbar[t] = 0.0;
        s_epsn[t] = 0.0;
        s_phibar[t] = bn;
        s_iters[t] = 0;
        s_flag[t] = 0;
        s_active[t] = bn > 0.0 ? 1 : 0;
    }
    __syncthreads();
    for (int idx = t; idx < a.g.ng * kTile; idx += NT) {
        x[idx] = 0.0;
        v[idx] = b[idx] * s_binv[col];
        vo[idx] = 0.0;
        w[idx] = 0.0;
        wo[idx] = 0.0;
    }
    __syncthreads();

    int it = 0;
    for (; it < a.max_iter; ++it) {
        if (t == 0) {
            int any = 0;
            for (int c = 0; c < kTile; ++c) any |= s_active[c];
            s_any = any;
        }
        __syncthreads();
        if (!s_any) break;
        // ---- pass 1: y = (H - s) v, C = Phi^T y, alpha = v^T y
        const double vty = apply_pass1<DIM, NB>(v, nullptr, 0.0, a, s, slots, nullptr);
        column_reduce(vty, red, s_alpha);
        // ---- pass 2: v_new = (y - Phi C) - alpha v - beta v_old  (into vo), |v_new|^2
        double nn = 0.0;
        const double al = s_alpha[col], be = s_beta[col];
        for (int blk = wave; blk * 16 < a.g.ng; blk += NW) {
            const int row0 = blk * 16;
            const int R = row0 + 4 * (lane >> 4);
            double w[Nbr<DIM>::N];
            gather<DIM>(v, R, a.g, col, w);
            double vold[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = R + e < a.g.ng ? R + e : a.g.ng - 1;
                vold[e] = vo[row * kTile + col];
            }
            const d4 d = project_block<NB>(a, slots, row0);
            double y[4], pc[4];
            stencil_from<DIM>(w, R, a.g, a.veff, s, y, pc);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double vn = (y[e] - d[e]) - al * pc[e] - be * vold[e];
                if (R + e < a.g.ng) {
                    vo[(R + e) * kTile + col] = vn;
                    nn += vn * vn;
                }
            }
        }
        column_reduce(nn, red, s_tmp);
        // ---- rotations (per system)
        if (t < kTile) {
            const double beta_new = sqrt(s_tmp[t]);
            const double alk = s_alpha[t];
            const double cs = s_cs[t], sn = s_sn[t];
            const double epsk = s_epsn[t];
            const double delta = cs * s_dbar[t] + sn * alk;
            const double gbar = sn * s_dbar[t] - cs * alk;
            const double epsn = sn * beta_new;
            const double dbar = -cs * beta_new;
            double gamma = sqrt(gbar * gbar + beta_new * beta_new);
            if (!(gamma > 0.0)) gamma = 1e-300;
            const double csn = gbar / gamma, snn = beta_new / gamma;
            const double phi = csn * s_phibar[t];
            s_delta[t] = delta;
            s_epsk[t] = epsk;
            s_gamma[t] = gamma;
            s_phi[t] = s_active[t] ? phi : 0.0;
            if (s_active[t]) {
                s_phibar[t] = snn * s_phibar[t];
                s_cs[t] = csn;
                s_sn[t] = snn;
                s_epsn[t] = epsn;
                s_dbar[t] = dbar;
                s_beta[t] = beta_new;
                s_binv[t] = beta_new > 0.0 ? 1.0 / beta_new : 0.0;
                s_iters[t] += 1;
            }
        }
        __syncthreads();
        // ---- pass 3: w_new = (v - eps_k wo - delta w) / gamma (into wo); x += phi w_new;
        //      v_old <- v, v <- v_new / beta_new
        if (s_active[col]) {
            const double ek = s_epsk[col], dl = s_delta[col], gi = 1.0 / s_gamma[col];
            const double ph = s_phi[col], bi = s_binv[col];
            for (int idx = t; idx < a.g.ng * kTile; idx += NT) {
                const double vv = v[idx];
                const double wn = (vv - ek * wo[idx] - dl * w[idx]) * gi;
                wo[idx] = w[idx];
                w[idx] = wn;
                x[idx] += ph * wn;
                const double vn = vo[idx] * bi;
                vo[idx] = vv;
                v[idx] = vn;
            }
        }
        __syncthreads();
        if (t < kTile && s_active[t]) {
            if (fabs(s_phibar[t]) <= a.tol * s_bn[t]) s_active[t] = 0;
        }
        __syncthreads();
    }
    if (t < kTile) {
        const int gc = tile * kTile + t;
        a.iters[gc] = s_iters[t];
        a.resid[gc] = (s_bn[t] > 0.0) ? fabs(s_phibar[t]) / s_bn[t] : 0.0;
        a.flags[gc] = s_flag[t] | (s_active[t] ? 1 : 0);
    }
    if (t == 0) a.tile_iters[tile] = it;
}

#define ACP_NB_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

hipError_t launch_cg_impl(const KrylovArgs &a, hipStream_t s) {
    const int nb = (a.ne + 15) / 16;
    dim3 grid(a.ntiles), block(NT);
#define CASE(N)                                                                              \
    if (nb == N) {                                                                           \
        if (a.g.dim == 1) hipLaunchKernelGGL((cg_kernel<1, N>), grid, block, 0, s, a);       \
        else hipLaunchKernelGGL((cg_kernel<2, N>), grid, block, 0, s, a);                    \
        return hipGetLastError();                                                            \
    }
    ACP_NB_CASES(CASE)
#undef CASE
    return hipErrorInvalidValue;
}

hipError_t launch_minres_impl(const KrylovArgs &a, hipStream_t s) {
    const int nb = (a.ne + 15) / 16;
    dim3 grid(a.ntiles), block(NT);
#define CASE(N)                                                                              \
    if (nb == N) {                                                                           \
        if (a.g.dim == 1) hipLaunchKernelGGL((minres_kernel<1, N>), grid, block, 0, s, a);   \
        else hipLaunchKernelGGL((minres_kernel<2, N>), grid, block, 0, s, a);                \
        return hipGetLastError();                                                            \
    }
    ACP_NB_CASES(CASE)
#undef CASE
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_cg_fp64(const KrylovArgs &a, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    if (a.ne > MAXNB * 16) return hipErrorInvalidValue;
    return launch_cg_impl(a, s);
}

hipError_t launch_minres_fp64(const KrylovArgs &a, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    if (a.ne > MAXNB * 16) return hipErrorInvalidValue;
    return launch_minres_impl(a, s);
}

}  // namespace acp
