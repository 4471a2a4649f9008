// Lowest eigenpairs of H = -1/2 Delta_h + diag(V) on the periodic grid: the
// occupied orbitals and energies that the shifted equations of Eq. (3.6) and
// the weights of Eq. (3.4) take as input (the paper obtains them with LOBPCG
// inside an SCF loop, Sec. 4).  Here: Chebyshev-filtered subspace iteration
// (Zhou, Saad, Tiago and Chelikowsky, J. Comput. Phys. 219 (2006)), every step
// on the device:
//
//   subspace X of k = n_want + n_guard vectors (seeded Gaussian start);
//   repeat: Y = p_m(H) X, the degree-m Chebyshev polynomial that is small on
//           [a, b] (a = the largest Ritz value of the subspace, capped, b an upper
//           bound of the spectrum) and scaled to 1 at the lowest Ritz value,
//           by the three-term recurrence (one stencil sweep and one axpby per
//           degree);
//           Rayleigh-Ritz: orthonormalise Y twice through the eigenvectors of
//           its Gram matrix (Y <- Y W D^{-1/2}), project H, diagonalise, rotate;
//   until every wanted Ritz pair has ||H x - lambda x||_2 <= tol.
//
// The guard vectors keep the filter's cut-off a above the wanted eigenvalues
// (a gap to the wanted set speeds the convergence); only the n_want lowest
// pairs are returned, plus the next Ritz value as an estimate of
// eigenvalue n_want + 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "acp_internal.h"

namespace acp {

thread_local std::string g_free_error;   // last error of the calls without a context

namespace {

// splitmix64 (Steele, Lea and Flood 2014): a counter-based 64-bit generator.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// X[i] ~ N(0, 1) by the Box-Muller transform of two uniforms drawn from the
// counter 2 i (+1) and the seed.
__global__ void randn_kernel(long long n, unsigned long long seed, double *X) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const unsigned long long k = seed * 0x2545F4914F6CDD1Dull + 2ull * (unsigned long long)i;
    const double u1 = ((splitmix64(k) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = ((splitmix64(k + 1) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    X[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// W(:, j) /= sqrt(d[j]) (d floored at 1e-300: a vanishing direction becomes a
// normalised rounding pattern that the second pass orthonormalises).
__global__ void scale_cols_rsqrt_kernel(int m, int n, double *W, int ldw, const double *d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= m) return;
    W[i + (long long)j * ldw] /= sqrt(fmax(d[j], 1e-300));
}

// A = (A + A^T) / 2 in place.
__global__ void symmetrize_kernel(int n, double *A, int lda) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= n || i >= j) return;
    const double v = 0.5 * (A[i + (long long)j * lda] + A[j + (long long)i * lda]);
    A[i + (long long)j * lda] = v;
    A[j + (long long)i * lda] = v;
}

__global__ void fill_kernel(int n, double v, double *x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

struct Eig {
    int ng, k, want;
    GridDesc g;
    const double *V;
    hipStream_t s;
    DevBuf buf[4], S, W, d, lam, work, ones, norms, splitk;
    std::string err;

    ~Eig() {
        for (auto &b : buf) release(b);
        release(S), release(W), release(d), release(lam), release(work), release(ones), release(norms),
            release(splitk);
    }
    double *B(int i) { return (double *)buf[i].p; }
};

#define EIGCHK(x)                                                                            \
    do {                                                                                     \
        hipError_t e_ = (x);                                                                 \
        if (e_ != hipSuccess) {                                                              \
            e.err = std::string(#x) + ": " + hipGetErrorString(e_);                          \
            return ACP_EDEVICE;                                                              \
        }                                                                                    \
    } while (0)

// Y <- Y W D^{-1/2}, with W D W^T = Y^T Y: the columns become orthonormal
// (to rounding times cond(Y)^2; a second call restores full accuracy).
acp_status orthonormalise(Eig &e, double *Y, double *out) {
    const int ng = e.ng, k = e.k;
    EIGCHK(gemm_splitk(Op::T, Op::N, k, k, ng, 1.0, Y, ng, Y, ng, 0.0, (double *)e.S.p, k,
                       (double *)e.splitk.p, e.splitk.bytes / 8, e.s));
    EIGCHK(sym_eig_jacobi(k, (double *)e.S.p, k, (double *)e.d.p, (double *)e.W.p, k, (double *)e.work.p, 30,
                          1e-15, e.s, nullptr));
    hipLaunchKernelGGL(scale_cols_rsqrt_kernel, dim3((k + 255) / 256, k), dim3(256), 0, e.s, k, k,
                       (double *)e.W.p, k, (const double *)e.d.p);
    EIGCHK(hipGetLastError());
    EIGCHK(gemm(Op::N, Op::N, ng, k, k, 1.0, Y, ng, 0, (const double *)e.W.p, k, 0, 0.0, out, ng, 0, 1, e.s));
    return ACP_OK;
}

// Rayleigh-Ritz on the span of buf[iy]: Ritz vectors into buf[ix], H times
// them into buf[ih], Ritz values into lam (device, ascending); the fourth
// buffer is scratch.  Returns the wanted residual norms^2 in norms (device).
acp_status rayleigh_ritz(Eig &e, int iy, int ix, int ih, int it) {
    const int ng = e.ng, k = e.k;
    acp_status st;
    if ((st = orthonormalise(e, e.B(iy), e.B(it))) != ACP_OK) return st;
    if ((st = orthonormalise(e, e.B(it), e.B(iy))) != ACP_OK) return st;
    // HY (Y orthonormal), Hs = Y^T H Y
    EIGCHK(launch_stencil(e.g, k, e.B(iy), ng, e.B(it), ng, e.V, -0.5, 1.0, 0.0, nullptr, e.s));
    EIGCHK(gemm_splitk(Op::T, Op::N, k, k, ng, 1.0, e.B(iy), ng, e.B(it), ng, 0.0, (double *)e.S.p, k,
                       (double *)e.splitk.p, e.splitk.bytes / 8, e.s));
    hipLaunchKernelGGL(symmetrize_kernel, dim3((k + 255) / 256, k), dim3(256), 0, e.s, k, (double *)e.S.p, k);
    EIGCHK(hipGetLastError());
    EIGCHK(sym_eig_jacobi(k, (double *)e.S.p, k, (double *)e.lam.p, (double *)e.W.p, k, (double *)e.work.p, 30,
                          1e-15, e.s, nullptr));
    EIGCHK(gemm(Op::N, Op::N, ng, k, k, 1.0, e.B(iy), ng, 0, (const double *)e.W.p, k, 0, 0.0, e.B(ix), ng, 0, 1,
                e.s));
    EIGCHK(gemm(Op::N, Op::N, ng, k, k, 1.0, e.B(it), ng, 0, (const double *)e.W.p, k, 0, 0.0, e.B(ih), ng, 0, 1,
                e.s));
    // residuals of the wanted pairs: H x_j - lambda_j x_j
    EIGCHK(launch_scale_copy(1, e.want, -1.0, (const double *)e.lam.p, 1, (double *)e.d.p, 1, e.s));
    EIGCHK(launch_col_axpby(ng, e.want, (const double *)e.d.p, e.B(ix), ng, (const double *)e.ones.p, e.B(ih), ng,
                            e.s));
    EIGCHK(launch_col_sqnorm(ng, e.want, e.B(ih), ng, (double *)e.norms.p, e.s));
    return ACP_OK;
}

}  // namespace

acp_status lowest_eigenpairs(const acp_grid *grid, const double *veff, const acp_eig_opts *opts, double *X_out,
                             double *lambda, double *lambda_next, int *passes_out, double *resid_out,
                             hipStream_t s, std::string &err) {
    if (!grid || !veff || !opts || !X_out || !lambda) {
        err = "null argument";
        return ACP_EINVAL;
    }
    if ((grid->dim != 1 && grid->dim != 2) || grid->n[0] < 9 || (grid->dim == 2 && grid->n[1] < 9) ||
        !(grid->h > 0)) {
        err = "grid";
        return ACP_EINVAL;
    }
    Eig e;
    e.g.dim = grid->dim;
    e.g.nx = grid->n[0];
    e.g.ny = grid->dim == 2 ? grid->n[1] : 1;
    e.g.ng = e.g.nx * e.g.ny;
    e.g.h = grid->h;
    e.ng = e.g.ng;
    e.want = opts->n_want;
    const int guard = opts->n_guard > 0 ? opts->n_guard : std::max(16, e.want / 10);
    e.k = e.want + guard;
    const int degree = opts->degree > 0 ? opts->degree : 20;
    const int max_pass = opts->max_pass > 0 ? opts->max_pass : 60;
    const double tol = opts->tol > 0 ? opts->tol : 1e-10;
    if (e.want < 1 || e.k >= e.ng) {
        err = "n_want + n_guard must be below the number of grid points";
        return ACP_EINVAL;
    }
    e.V = veff;
    e.s = s;
    const int ng = e.ng, k = e.k;
    // upper bound of the spectrum: the largest eigenvalue of -1/2 Delta_h (its
    // symbol at the Nyquist mode, per axis) plus max V
    std::vector<double> vh(ng);
    if (hipMemcpyAsync(vh.data(), veff, (size_t)ng * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        err = "reading V";
        return ACP_EDEVICE;
    }
    const double vmax = *std::max_element(vh.begin(), vh.end());
    double nyq = -fd8(0);
    for (int q = 1; q <= 4; ++q) nyq -= 2.0 * fd8(q) * ((q & 1) ? -1.0 : 1.0);
    const double b = 0.5 * grid->dim * nyq / (grid->h * grid->h) + vmax;
    for (auto &bb : e.buf)
        if (!ensure(bb, (size_t)ng * k * 8)) {
            err = "device allocation failed";
            return ACP_ENOMEM;
        }
    if (!ensure(e.S, (size_t)k * k * 8) || !ensure(e.W, (size_t)k * k * 8) || !ensure(e.d, (size_t)k * 8) ||
        !ensure(e.lam, (size_t)k * 8) || !ensure(e.work, sym_eig_work_doubles(k, true) * 8) ||
        !ensure(e.ones, (size_t)k * 8) || !ensure(e.norms, (size_t)k * 8) ||
        !ensure(e.splitk, (size_t)8 * k * k * 8)) {
        err = "device allocation failed";
        return ACP_ENOMEM;
    }
    acp_status st = ACP_OK;
    auto fail_dev = [&]() {
        err = e.err;
        return ACP_EDEVICE;
    };
    hipLaunchKernelGGL(fill_kernel, dim3((k + 255) / 256), dim3(256), 0, s, k, 1.0, (double *)e.ones.p);
    const long long tot = (long long)ng * k;
    hipLaunchKernelGGL(randn_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, tot, opts->seed, e.B(0));
    if (hipGetLastError() != hipSuccess) return fail_dev();
    int ix = 1, ih = 2;
    if ((st = rayleigh_ritz(e, 0, ix, ih, 3)) != ACP_OK) return fail_dev();
    std::vector<double> lam(k), nrm(e.want);
    int pass = 0;
    double worst = INFINITY;
    while (true) {
        if (hipMemcpyAsync(lam.data(), e.lam.p, (size_t)k * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(nrm.data(), e.norms.p, (size_t)e.want * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            err = "reading Ritz values";
            return ACP_EDEVICE;
        }
        worst = 0.0;
        for (double v : nrm) worst = std::max(worst, std::sqrt(v));
        if (worst <= tol || pass >= max_pass) break;
        ++pass;
        // filter on [a, b], scaled at a0 (Zhou-Saad scaled recurrence)
        const double a0 = lam[0];
        const double a = std::min(lam[k - 1], a0 + 0.1 * (b - a0));
        const double half = 0.5 * (b - a), c = 0.5 * (b + a);
        double sigma = half / (a0 - c);
        const double sigma1 = sigma;
        // buffers: p (previous term, starts as the Ritz vectors X), y (current
        // term, starts in the buffer of H X, no longer needed), two free ones
        int fr0[2], nf0 = 0;
        for (int q = 0; q < 4; ++q)
            if (q != ix && q != ih) fr0[nf0++] = q;
        int ip = ix, iy = ih, fa = fr0[0], fb = fr0[1];
        const double al = sigma1 / half;   // y = (sigma1 / half)(H - c) x
        if (launch_stencil(e.g, k, e.B(ip), ng, e.B(iy), ng, veff, -0.5 * al, al, -al * c, nullptr, s) !=
            hipSuccess)
            return fail_dev();
        for (int deg = 2; deg <= degree; ++deg) {
            const double sigma2 = 1.0 / (2.0 / sigma1 - sigma);
            const double al2 = 2.0 * sigma2 / half;
            const int it = fa;   // t = al2 (H - c) y - sigma sigma2 p
            if (launch_stencil(e.g, k, e.B(iy), ng, e.B(it), ng, veff, -0.5 * al2, al2, -al2 * c, nullptr, s) !=
                    hipSuccess ||
                launch_axpby(ng, k, -sigma * sigma2, e.B(ip), ng, 1.0, e.B(it), ng, s) != hipSuccess)
                return fail_dev();
            fa = fb;
            fb = ip;
            ip = iy;
            iy = it;
            sigma = sigma2;
        }
        // Rayleigh-Ritz on y; Ritz vectors into one free buffer, H X into another
        int fr[3], nf = 0;
        for (int q = 0; q < 4; ++q)
            if (q != iy) fr[nf++] = q;
        ix = fr[0];
        ih = fr[1];
        if ((st = rayleigh_ritz(e, iy, ix, ih, fr[2])) != ACP_OK) return fail_dev();
    }
    if (hipMemcpyAsync(X_out, e.B(ix), (size_t)ng * e.want * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail_dev();
    std::memcpy(lambda, lam.data(), (size_t)e.want * 8);
    if (lambda_next) *lambda_next = lam[e.want];
    if (passes_out) *passes_out = pass;
    if (resid_out) *resid_out = worst;
    if (worst > tol) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "largest residual %.3e above tol after %d passes", worst, pass);
        err = buf;
        return ACP_ENOCONV;
    }
    return ACP_OK;
}

}  // namespace acp

extern "C" acp_status acp_lowest_eigenpairs(const acp_grid *grid, const double *veff, const acp_eig_opts *opts,
                                            double *psi, double *lambda, double *lambda_next, int *passes,
                                            double *max_resid, void *stream) {
    std::string err;
    const acp_status st = acp::lowest_eigenpairs(grid, veff, opts, psi, lambda, lambda_next, passes, max_resid,
                                                 (hipStream_t)stream, err);
    acp::g_free_error = err;
    return st;
}
