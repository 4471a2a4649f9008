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

// r(:, j) -= alpha_j w(:, j) and rrn_j = |r(:, j)|^2 (one block per column,
// fixed reduction order).
__global__ __launch_bounds__(256) void wide_residual_kernel(int ng, const double *al, const int *colact,
                                                            const double *w, double *r, double *rrn) {
    const int j = blockIdx.x;
    __shared__ double red[256];
    double acc = 0.0;
    if (colact[j]) {
        const double a = al[j];
        const double *wj = w + (long long)j * ng;
        double *rj = r + (long long)j * ng;
        for (int i = threadIdx.x; i < ng; i += 256) {
            const double v = rj[i] - a * wj[i];
            rj[i] = v;
            acc += v * v;
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
                                          const double *al, const double *alp, const double *btp, const double *rr,
                                          const double *rrn, const double *bn, const int *colact, double *z,
                                          double *zp, int *act, int *upd, double *ac, double *zn, double *bc,
                                          int *it, double *res) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nb * nc) return;
    const int c = idx / nb, j = idx % nb;
    if (!colact[j]) {
        upd[idx] = 0;
        act[idx] = 0;
        return;
    }
    const double a = al[j];
    const double beta = rr[j] > 0.0 ? rrn[j] / rr[j] : 0.0;
    const bool live = act[idx] != 0;
    if (c == base) {
        upd[idx] = (live ? 1 : 0) | 2;
        ac[idx] = a;
        zn[idx] = 1.0;
        bc[idx] = beta;
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
    upd[idx] = 3;
    ac[idx] = a * ratio;
    zn[idx] = znew;
    bc[idx] = beta * ratio * ratio;
    zp[idx] = zk;
    z[idx] = znew;
    it[idx] = iter + 1;
    const double rc = fabs(znew) * sqrt(rrn[j]);
    if (rc <= tol * bn[j]) {
        act[idx] = 0;
        res[idx] = rc / bn[j];
    }
}

// x_c += a^c_k p_c (with the old p_c), p_c = zeta_{k+1} r_{k+1} + b^c_k p_c.
__global__ void wide_shift_update_kernel(int ng, int nb, int nc, const int *upd, const double *ac, const double *zn,
                                         const double *bc, const double *r, double *P, double *X, long long xs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= ng) return;
    const long long off = (long long)j * ng + i;
    const long long cs = (long long)nb * ng;
    const double rv = r[off];
    for (int c = 0; c < nc; ++c) {
        const int u = upd[c * nb + j];
        if (!u) continue;
        const double p = P[c * cs + off];
        if (u & 1) X[c * xs + off] += ac[c * nb + j] * p;
        if (u & 2) P[c * cs + off] = zn[c * nb + j] * rv + bc[c * nb + j] * p;
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

hipError_t wide_step(int ng, int nb, int nc, int base, const double *sig, double tol, int iter, const double *pw,
                     const double *w_vec, double *r, double *P, double *X, long long xs, const WideScalars &w,
                     hipStream_t s) {
    hipLaunchKernelGGL(wide_alpha_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, nb, (const double *)w.rr, pw,
                       w.colact, w.al, w.flags);
    hipLaunchKernelGGL(wide_residual_kernel, dim3(nb), dim3(256), 0, s, ng, (const double *)w.al,
                       (const int *)w.colact, w_vec, r, w.rrn);
    hipLaunchKernelGGL(wide_shift_scalars_kernel, dim3((nb * nc + 255) / 256), dim3(256), 0, s, nb, nc, base, sig,
                       tol, iter, (const double *)w.al, (const double *)w.alp, (const double *)w.btp,
                       (const double *)w.rr, (const double *)w.rrn, (const double *)w.bn, (const int *)w.colact,
                       w.z, w.zp, w.act, w.upd, w.ac, w.zn, w.bc, w.it, w.res);
    hipLaunchKernelGGL(wide_shift_update_kernel, dim3((ng + 255) / 256, nb), dim3(256), 0, s, ng, nb, nc,
                       (const int *)w.upd, (const double *)w.ac, (const double *)w.zn, (const double *)w.bc,
                       (const double *)r, P, X, xs);
    hipLaunchKernelGGL(wide_column_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, nb, nc, (const int *)w.act,
                       w.colact, w.rr, (const double *)w.rrn, w.alp, (const double *)w.al, w.btp, w.nactive);
    return hipGetLastError();
}

}  // namespace acp
