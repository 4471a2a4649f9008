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
#include "krylov_common.h"

namespace acp {

namespace {

using namespace kry;

template <int DIM, int NB, typename T>
__global__ __launch_bounds__(NT) void cg_kernel(KrylovArgsT<T> a) {
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
    const T *__restrict__ b = a.rhs + (long long)(tile % a.rhs_tiles) * a.g.ng * kTile;
    double *__restrict__ x = a.x + base;
    T *__restrict__ r = a.r + base;
    T *pA = a.pa + base;
    T *pB = a.pb + base;
    const double s = a.shift[tile * kTile + col];

    // init: x = 0, r = b, p_old = 0, rr = |b|^2
    double part = 0.0;
    for (int idx = t; idx < a.g.ng * kTile; idx += NT) {
        const double bv = (double)b[idx];
        x[idx] = 0.0;
        r[idx] = (T)bv;
        pA[idx] = (T)0.0;
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
        const double pty = apply_pass1<DIM, NB, T>(r, pA, beta, a, s, slots, pB);
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
                ro[e] = (double)r[row * kTile + col];
            }
            const d4 d = project_block<NB, T>(a.phi_cm, a.g.ng, slots, row0);
            double y[4], pc[4];
            stencil_from<DIM>(w, R, a.g, a.veff, s, y, pc);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double ap = y[e] - d[e];
                const double xn = xo[e] + al * pc[e];
                const double rn = ro[e] - al * ap;
                if (R + e < a.g.ng) {
                    x[(R + e) * kTile + col] = xn;
                    r[(R + e) * kTile + col] = (T)rn;
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
        T *tmp = pA; pA = pB; pB = tmp;
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
        const double vty = apply_pass1<DIM, NB, double>(v, nullptr, 0.0, a, s, slots, nullptr);
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
            const d4 d = project_block<NB, double>(a.phi_cm, a.g.ng, slots, row0);
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

template <typename T>
hipError_t launch_cg_impl(const KrylovArgsT<T> &a, hipStream_t s) {
    const int nb = (a.ne + 15) / 16;
    dim3 grid(a.ntiles), block(NT);
#define CASE(N)                                                                              \
    if (nb == N) {                                                                           \
        if (a.g.dim == 1) hipLaunchKernelGGL((cg_kernel<1, N, T>), grid, block, 0, s, a);    \
        else hipLaunchKernelGGL((cg_kernel<2, N, T>), grid, block, 0, s, a);                 \
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

hipError_t launch_cg_fp32(const KrylovArgsT<float> &a, hipStream_t s) {
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
