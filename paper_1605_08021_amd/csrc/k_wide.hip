// Kernels of the multi-shift CG for many orbitals (the "wide" form): the
// Krylov vectors are column-major N_g x n blocks and the projector of
// Eq. (3.6) is applied by two GEMMs (C = Phi^T y, y <- y - Phi C) on the
// matrix cores, which keep a whole block of right-hand sides per pass over Phi
// instead of one 16-column tile (Phi is read once per GEMM tile column, not once
// per 16 systems); the stencil sweep, the dot products, the base CG step and
// the shifted updates are the kernels below.
//
// Scalars of column j (one right-hand side b_j): rr = r.r, bn = |b|, al / alp =
// alpha_k / alpha_{k-1}, btp = beta_{k-1}, colact (any shift still running);
// per shift c and column j: z / zp = zeta_k / zeta_{k-1} of Jegerlehner's
// collinear residuals r_c = zeta_c r (the base shift has zeta = 1), act, the
// step coefficients of this iteration (ac = alpha^c_k, zn = zeta_{k+1},
// bc = beta^c_k), upd (bit 0: x_c moves, bit 1: p_c moves), iterations and the
// final recurrence residual.
//
// Deferred updates: the base shift's search direction p (the stencil's input)
// moves every iteration; its solution, and every other shift's p_c and x_c,
// move once per window of kWideWindow iterations (the base's p at the window's
// start is kept for that).  Within a window started at k0,
//   p_c^k = B p_c^{k0} + sum_{s} gamma_s r^{k0+1+s},
//   x_c^k = x_c^{k0} + A p_c^{k0} + sum_{s} chi_s r^{k0+1+s},
// with the coefficients advanced by each step (A += a B, chi += a gamma, then
// B *= b, gamma *= b, gamma_w = zeta_{k+1}); the residuals of the window stay
// in a ring (r^k in slot k mod kWideWindow), and one sweep at the window's end
// reads them once for all shifts.
#include "acp_internal.h"

namespace acp {
namespace {

__global__ void wide_init_kernel(int nb, int nc, const double *bsq, double *rr, double *bn, double *alp,
                                 double *btp, int *colact, double *z, double *zp, int *act, int *it,
                                 double *res) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    const double b2 = bsq[j];
    rr[j] = b2;
    bn[j] = sqrt(b2);
    alp[j] = 1.0;
    btp[j] = 0.0;
    const int live = b2 > 0.0;   // a zero right-hand side has the solution 0
    colact[j] = live;
    for (int c = 0; c < nc; ++c) {
        z[c * nb + j] = 1.0;
        zp[c * nb + j] = 1.0;
        act[c * nb + j] = live;
        it[c * nb + j] = 0;
        res[c * nb + j] = 0.0;
    }
}

// alpha_k = r.r / p.Ap; a non-positive curvature stops the column (flag bit 1).
__global__ void wide_alpha_kernel(int nb, const double *rr, const double *pw, int *colact, double *al,
                                  int *flags) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    double a = 0.0;
    if (colact[j]) {
        if (pw[j] > 0.0) {
            a = rr[j] / pw[j];
        } else {
            colact[j] = 0;
            atomicOr(flags, 2);
        }
    }
    al[j] = a;
}

// rn(:, j) = r(:, j) - alpha_j w(:, j) and rrn_j = |rn(:, j)|^2 (one block per
// column, fixed reduction order).
__global__ __launch_bounds__(256) void wide_residual_kernel(int ng, const double *al, const int *colact,
                                                            const double *w, const double *r, double *rn,
                                                            double *rrn) {
    const int j = blockIdx.x;
    __shared__ double red[256];
    double acc = 0.0;
    if (colact[j]) {
        const double a = al[j];
        const double *wj = w + (long long)j * ng;
        const double *rj = r + (long long)j * ng;
        double *rnj = rn + (long long)j * ng;
        if ((ng & 1) == 0) {   // pairs of rows: 16-byte accesses (even N_g keeps them aligned)
            for (int i = 2 * threadIdx.x; i < ng; i += 512) {
                const double2 rv = *(const double2 *)(rj + i), wv = *(const double2 *)(wj + i);
                const double2 v = make_double2(rv.x - a * wv.x, rv.y - a * wv.y);
                *(double2 *)(rnj + i) = v;
                acc += v.x * v.x + v.y * v.y;
            }
        } else {
            for (int i = threadIdx.x; i < ng; i += 256) {
                const double v = rj[i] - a * wj[i];
                rnj[i] = v;
                acc += v * v;
            }
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) rrn[j] = colact[j] ? red[0] : 0.0;
}

// The step of iteration k for every (shift, column): Jegerlehner's
//   zeta_{k+1} = zeta_k zeta_{k-1} a_{k-1} /
//                (a_k b_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} a_{k-1} (1 + sigma a_k)),
//   a^c_k = a_k zeta_{k+1} / zeta_k,  b^c_k = b_k (zeta_{k+1} / zeta_k)^2,
// with sigma_c = s_base - s_c >= 0 and b_k = |r_{k+1}|^2 / |r_k|^2; a shift
// converges when |zeta_{k+1}| |r_{k+1}| <= tol |b|.  The base shift keeps
// moving its search direction while any shift of the column runs.
__global__ void wide_shift_scalars_kernel(int nb, int nc, int base, const double *sig, double tol, int iter,
                                          int wpos, const double *al, const double *alp, const double *btp,
                                          const double *rr, const double *rrn, const double *bn, const int *colact,
                                          double *z, double *zp, int *act, int *upd, double *ac, double *zn,
                                          double *bc, int *it, double *res, double *coef, int *touched) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nb * nc) return;
    const int c = idx / nb, j = idx % nb;
    constexpr int W = kWideWindow;
    double *co = coef + (size_t)idx * (2 + 2 * W);   // B, A, gamma[W], chi[W]
    if (wpos == 0) {   // a new window: every shift starts from its stored p_c, x_c
        touched[idx] = 0;
        co[0] = 1.0;
        co[1] = 0.0;
        for (int q = 0; q < 2 * W; ++q) co[2 + q] = 0.0;
    }
    if (!colact[j]) {
        upd[idx] = 0;
        act[idx] = 0;
        return;
    }
    const double a = al[j];
    const double beta = rr[j] > 0.0 ? rrn[j] / rr[j] : 0.0;
    const bool live = act[idx] != 0;
    if (c == base) {
        // p moves every iteration (it feeds the operator); x is deferred to the
        // window's flush like the other shifts' (zeta = 1: a_c = alpha, b_c = beta),
        // its coefficients advancing only while the base shift is live
        upd[idx] = 2;
        ac[idx] = a;
        zn[idx] = 1.0;
        bc[idx] = beta;
        if (live) {
            touched[idx] = 1;
            co[1] += a * co[0];
            for (int q = 0; q < wpos; ++q) co[2 + W + q] += a * co[2 + q];
        }
        co[0] *= beta;
        for (int q = 0; q < wpos; ++q) co[2 + q] *= beta;
        co[2 + wpos] = 1.0;
        if (live) {
            it[idx] = iter + 1;
            if (sqrt(rrn[j]) <= tol * bn[j]) {
                act[idx] = 0;
                res[idx] = sqrt(rrn[j]) / bn[j];
            }
        }
        return;
    }
    if (!live) {
        upd[idx] = 0;
        return;
    }
    const double zk = z[idx], zkm = zp[idx], ap = alp[j], bp = btp[j];
    const double den = a * bp * (zkm - zk) + zkm * ap * (1.0 + sig[c] * a);
    const double znew = den != 0.0 ? zk * zkm * ap / den : 0.0;
    const double ratio = zk != 0.0 ? znew / zk : 0.0;
    const double a_c = a * ratio, b_c = beta * ratio * ratio;
    upd[idx] = 3;
    ac[idx] = a_c;
    zn[idx] = znew;
    bc[idx] = b_c;
    // window coefficients: x_c^{k+1} = x_c^k + a_c p_c^k, p_c^{k+1} = zeta_{k+1} r^{k+1} + b_c p_c^k
    touched[idx] = 1;
    co[1] += a_c * co[0];
    for (int q = 0; q < wpos; ++q) co[2 + W + q] += a_c * co[2 + q];
    co[0] *= b_c;
    for (int q = 0; q < wpos; ++q) co[2 + q] *= b_c;
    co[2 + wpos] = znew;
    zp[idx] = zk;
    z[idx] = znew;
    it[idx] = iter + 1;
    const double rc = fabs(znew) * sqrt(rrn[j]);
    if (rc <= tol * bn[j]) {
        act[idx] = 0;
        res[idx] = rc / bn[j];
    }
}

// The base shift every iteration: p = r^{k+1} + b_k p (its x moves at the
// window's flush); at a window's first iteration the old p is kept in P0 for
// that flush.  With pb0 the new p is also written as its BF16 split at
// j ldpb + i (two terms with pb1, else one).
__global__ void wide_base_update_kernel(int ng, int nb, int base, const int *upd, const double *ac,
                                        const double *bc, const double *rn, double *P, double *X,
                                        unsigned short *pb0, unsigned short *pb1, long long ldpb, double *P0,
                                        int save_p0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= ng) return;
    const int u = upd[base * nb + j];
    if (!u) return;
    const long long off = (long long)j * ng + i;
    const double p = P[off];
    if (save_p0) P0[off] = p;
    if (u & 1) X[off] += ac[base * nb + j] * p;
    if (u & 2) {
        const double pn = rn[off] + bc[base * nb + j] * p;
        P[off] = pn;
        if (pb0) {
            const unsigned short h = f64_to_bf16(pn);
            pb0[(long long)j * ldpb + i] = h;
            if (pb1) pb1[(long long)j * ldpb + i] = f64_to_bf16(pn - bf16_to_f64(h));
        }
    }
}

// End of a window of wl steps started at k0: for every shift touched in it,
// x_c += A p_c + sum_s chi_s r^{k0+1+s}, and for the others than the base
// p_c = B p_c + sum_s gamma_s r^{k0+1+s} (the base's p_c at the window start is
// P0; its current p was kept up to date every iteration).
__global__ void wide_flush1_kernel(int ng, int nb, int nc, int base, int k0, int wl, const double *ring,
                                   long long rs, const double *coef, const int *touched, double *P, double *X,
                                   long long xs, const double *P0) {
    constexpr int W = kWideWindow;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= ng) return;
    const long long off = (long long)j * ng + i;
    const long long cs = (long long)nb * ng;
    double rv[W];
#pragma unroll
    for (int q = 0; q < W; ++q) rv[q] = q < wl ? ring[((k0 + 1 + q) % W) * rs + off] : 0.0;
    for (int c = 0; c < nc; ++c) {
        if (!touched[c * nb + j]) continue;
        const double *co = coef + (size_t)(c * nb + j) * (2 + 2 * W);
        const double p = c == base ? P0[off] : P[c * cs + off];
        double xn = X[c * xs + off] + co[1] * p, pn = co[0] * p;
#pragma unroll
        for (int q = 0; q < W; ++q) {
            xn += co[2 + W + q] * rv[q];
            pn += co[2 + q] * rv[q];
        }
        X[c * xs + off] = xn;
        if (c != base) P[c * cs + off] = pn;
    }
}

// The same with two consecutive rows per thread (16-byte accesses; for even
// N_g, where every column's pairs of rows are aligned).
__global__ void wide_flush_kernel(int ng, int nb, int nc, int base, int k0, int wl, const double *ring,
                                  long long rs, const double *coef, const int *touched, double *P, double *X,
                                  long long xs, const double *P0) {
    constexpr int W = kWideWindow;
    const int i = 2 * (blockIdx.x * blockDim.x + threadIdx.x);
    const int j = blockIdx.y;
    if (i >= ng) return;
    const long long off = (long long)j * ng + i;
    const long long cs = (long long)nb * ng;
    double2 rv[W];
#pragma unroll
    for (int q = 0; q < W; ++q)
        rv[q] = q < wl ? *(const double2 *)(ring + ((k0 + 1 + q) % W) * rs + off) : make_double2(0.0, 0.0);
    for (int c = 0; c < nc; ++c) {
        if (!touched[c * nb + j]) continue;
        const double *co = coef + (size_t)(c * nb + j) * (2 + 2 * W);
        const double2 p = *(const double2 *)(c == base ? P0 + off : P + c * cs + off);
        const double2 x = *(const double2 *)(X + c * xs + off);
        double2 xn = make_double2(x.x + co[1] * p.x, x.y + co[1] * p.y);
        double2 pn = make_double2(co[0] * p.x, co[0] * p.y);
#pragma unroll
        for (int q = 0; q < W; ++q) {
            xn.x += co[2 + W + q] * rv[q].x;
            xn.y += co[2 + W + q] * rv[q].y;
            pn.x += co[2 + q] * rv[q].x;
            pn.y += co[2 + q] * rv[q].y;
        }
        *(double2 *)(X + c * xs + off) = xn;
        if (c != base) *(double2 *)(P + c * cs + off) = pn;
    }
}

// End of iteration: the base scalars move on; a column stays live while any
// of its shifts runs; nactive counts the live columns.
__global__ void wide_column_kernel(int nb, int nc, const int *act, int *colact, double *rr, const double *rrn,
                                   double *alp, const double *al, double *btp, int *nactive) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    if (!colact[j]) return;
    btp[j] = rr[j] > 0.0 ? rrn[j] / rr[j] : 0.0;
    rr[j] = rrn[j];
    alp[j] = al[j];
    int any = 0;
    for (int c = 0; c < nc; ++c) any |= act[c * nb + j];
    colact[j] = any;
    if (any) atomicAdd(nactive, 1);
}

}  // namespace

hipError_t wide_init(int nb, int nc, const double *bsq, const WideScalars &w, hipStream_t s) {
    hipLaunchKernelGGL(wide_init_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, nb, nc, bsq, w.rr, w.bn, w.alp,
                       w.btp, w.colact, w.z, w.zp, w.act, w.it, w.res);
    return hipGetLastError();
}

hipError_t wide_step(int ng, int nb, int nc, int base, const double *sig, double tol, int iter, int k0,
                     const double *pw, const double *w_vec, const double *r, double *rn, double *P, double *X,
                     long long xs, const WideScalars &w, double *P0, hipStream_t s, unsigned short *const *pb,
                     long long ldpb) {
    hipLaunchKernelGGL(wide_alpha_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, nb, (const double *)w.rr, pw,
                       w.colact, w.al, w.flags);
    hipLaunchKernelGGL(wide_residual_kernel, dim3(nb), dim3(256), 0, s, ng, (const double *)w.al,
                       (const int *)w.colact, w_vec, r, rn, w.rrn);
    hipLaunchKernelGGL(wide_shift_scalars_kernel, dim3((nb * nc + 255) / 256), dim3(256), 0, s, nb, nc, base, sig,
                       tol, iter, iter - k0, (const double *)w.al, (const double *)w.alp, (const double *)w.btp,
                       (const double *)w.rr, (const double *)w.rrn, (const double *)w.bn, (const int *)w.colact,
                       w.z, w.zp, w.act, w.upd, w.ac, w.zn, w.bc, w.it, w.res, w.coef, w.touched);
    hipLaunchKernelGGL(wide_base_update_kernel, dim3((ng + 255) / 256, nb), dim3(256), 0, s, ng, nb, base,
                       (const int *)w.upd, (const double *)w.ac, (const double *)w.bc, (const double *)rn,
                       P + (size_t)base * nb * ng, X + (size_t)base * xs, pb ? pb[0] : nullptr,
                       pb ? pb[1] : nullptr, ldpb, P0, iter == k0 ? 1 : 0);
    hipLaunchKernelGGL(wide_column_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, nb, nc, (const int *)w.act,
                       w.colact, w.rr, (const double *)w.rrn, w.alp, (const double *)w.al, w.btp, w.nactive);
    return hipGetLastError();
}

hipError_t wide_flush(int ng, int nb, int nc, int base, int k0, int wl, const double *ring, double *P, double *X,
                      long long xs, const WideScalars &w, const double *P0, hipStream_t s) {
    if (wl <= 0) return hipSuccess;
    if (ng & 1) {
        hipLaunchKernelGGL(wide_flush1_kernel, dim3((ng + 255) / 256, nb), dim3(256), 0, s, ng, nb, nc, base, k0, wl,
                           ring, (long long)ng * nb, (const double *)w.coef, (const int *)w.touched, P, X, xs, P0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(wide_flush_kernel, dim3((ng / 2 + 255) / 256, nb), dim3(256), 0, s, ng, nb, nc, base, k0, wl, ring,
                       (long long)ng * nb, (const double *)w.coef, (const int *)w.touched, P, X, xs, P0);
    return hipGetLastError();
}

}  // namespace acp
