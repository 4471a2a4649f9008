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
#include <cstdlib>
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

// rho(a) = scale sum_{i < n} X(a, i)^2
__global__ void density_kernel(int ng, int n, double scale, const double *X, double *rho) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= ng) return;
    double acc = 0.0;
    for (int i = 0; i < n; ++i) {
        const double v = X[a + (long long)i * ng];
        acc += v * v;
    }
    rho[a] = scale * acc;
}

// Symbol of v_c = (4 pi / eps0)(-Delta_h + kappa^2)^{-1} (kind 0) or of the
// Kerker preconditioner q^2 / (q^2 + q0^2) with q^2 the symbol of -Delta_h
// (kind 1), on the real Fourier basis of launch_fourier_basis (column c of an
// n-point axis carries the wave number (c + 1) / 2).
__device__ double axis_symbol(int c, int n, double h) {
    const int kf = (c + 1) / 2;
    const double th = 2.0 * 3.141592653589793 * kf / n;
    double v = -fd8(0);
    for (int q = 1; q <= 4; ++q) v -= 2.0 * fd8(q) * cos(q * th);
    return v / (h * h);
}

__global__ void grid_symbol_kernel(int nx, int ny, double h, int kind, double p0, double p1, double *S) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nx * ny) return;
    double lam = axis_symbol(idx % nx, nx, h);
    if (ny > 1) lam += axis_symbol(idx / nx, ny, h);
    S[idx] = kind == 0 ? (4.0 * 3.141592653589793 / p0) / (lam + p1 * p1) : lam / (lam + p1 * p1);
}

// part[b] = {max |R|, max |rho|} over the block's rows.
__global__ void maxabs2_kernel(int ng, const double *R, const double *rho, double *part) {
    __shared__ double r0[256], r1[256];
    double a = 0.0, b = 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < ng; i += gridDim.x * 256) {
        a = fmax(a, fabs(R[i]));
        b = fmax(b, fabs(rho[i]));
    }
    r0[threadIdx.x] = a;
    r1[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            r0[threadIdx.x] = fmax(r0[threadIdx.x], r0[threadIdx.x + w]);
            r1[threadIdx.x] = fmax(r1[threadIdx.x], r1[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = r0[0];
        part[2 * blockIdx.x + 1] = r1[0];
    }
}

struct Eig {
    int ng, k, want;
    GridDesc g;
    const double *V;
    hipStream_t s;
    DevBuf buf[4], S, W, d, lam, work, ones, norms, splitk;
    int ix = -1;                  // buffer of the current Ritz vectors (-1: none yet)
    std::vector<double> lamh;     // Ritz values on the host
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

// Buffers and sizes of one eigenpair problem (kept across the SCF iterations).
acp_status eig_prepare(Eig &e, const acp_grid *grid, int want, int guard, hipStream_t s, std::string &err) {
    if (!grid || (grid->dim != 1 && grid->dim != 2) || grid->n[0] < 9 || (grid->dim == 2 && grid->n[1] < 9) ||
        !(grid->h > 0)) {
        err = "grid";
        return ACP_EINVAL;
    }
    e.g.dim = grid->dim;
    e.g.nx = grid->n[0];
    e.g.ny = grid->dim == 2 ? grid->n[1] : 1;
    e.g.ng = e.g.nx * e.g.ny;
    e.g.h = grid->h;
    e.ng = e.g.ng;
    e.want = want;
    e.k = want + (guard > 0 ? guard : std::max(16, want / 10));
    e.s = s;
    e.ix = -1;
    if (e.want < 1 || e.k >= e.ng) {
        err = "n_want + n_guard must be below the number of grid points";
        return ACP_EINVAL;
    }
    const int ng = e.ng, k = e.k;
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
    hipLaunchKernelGGL(fill_kernel, dim3((k + 255) / 256), dim3(256), 0, s, k, 1.0, (double *)e.ones.p);
    if (hipGetLastError() != hipSuccess) {
        err = "fill";
        return ACP_EDEVICE;
    }
    e.lamh.assign(k, 0.0);
    return ACP_OK;
}

// Filter passes until every wanted Ritz pair of H[veff] has residual <= tol;
// the first call starts from a seeded Gaussian block, later calls from the
// current Ritz vectors (warm start).
acp_status eig_solve(Eig &e, const double *veff, int degree, int max_pass, double tol, unsigned long long seed,
                     int *passes_out, double *resid_out, std::string &err) {
    const int ng = e.ng, k = e.k;
    hipStream_t s = e.s;
    e.V = veff;
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
    const double b = 0.5 * e.g.dim * nyq / (e.g.h * e.g.h) + vmax;
    acp_status st = ACP_OK;
    auto fail_dev = [&]() {
        err = e.err;
        return ACP_EDEVICE;
    };
    int ix, ih;
    if (e.ix < 0) {
        const long long tot = (long long)ng * k;
        hipLaunchKernelGGL(randn_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, tot, seed, e.B(0));
        if (hipGetLastError() != hipSuccess) return fail_dev();
        ix = 1;
        ih = 2;
        if ((st = rayleigh_ritz(e, 0, ix, ih, 3)) != ACP_OK) return fail_dev();
    } else {
        int fr[3], nf = 0;
        for (int q = 0; q < 4; ++q)
            if (q != e.ix) fr[nf++] = q;
        ix = fr[0];
        ih = fr[1];
        if ((st = rayleigh_ritz(e, e.ix, ix, ih, fr[2])) != ACP_OK) return fail_dev();
    }
    std::vector<double> &lam = e.lamh;
    std::vector<double> nrm(e.want);
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
    e.ix = ix;
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

acp_status lowest_eigenpairs(const acp_grid *grid, const double *veff, const acp_eig_opts *opts, double *X_out,
                             double *lambda, double *lambda_next, int *passes_out, double *resid_out,
                             hipStream_t s, std::string &err) {
    if (!grid || !veff || !opts || !X_out || !lambda) {
        err = "null argument";
        return ACP_EINVAL;
    }
    Eig e;
    acp_status st = eig_prepare(e, grid, opts->n_want, opts->n_guard, s, err);
    if (st != ACP_OK) return st;
    st = eig_solve(e, veff, opts->degree > 0 ? opts->degree : 20, opts->max_pass > 0 ? opts->max_pass : 60,
                   opts->tol > 0 ? opts->tol : 1e-10, opts->seed, passes_out, resid_out, err);
    if (st != ACP_OK && st != ACP_ENOCONV) return st;
    if (hipMemcpyAsync(X_out, e.B(e.ix), (size_t)e.ng * e.want * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        err = "copy";
        return ACP_EDEVICE;
    }
    std::memcpy(lambda, e.lamh.data(), (size_t)e.want * 8);
    if (lambda_next) *lambda_next = e.lamh[e.want];
    return st;
}

// Diagonal operator of the grid in the real Fourier basis: Y = F diag(S) F^T X
// for one grid vector (F = Fx, or Fy (x) Fx in 2D); T is scratch.
struct GridFourier {
    int nx, ny;
    DevBuf fx, fy, T, Y;
    ~GridFourier() { release(fx), release(fy), release(T), release(Y); }
};

hipError_t fourier_apply(GridFourier &f, const double *S, const double *X, double *Y, hipStream_t s) {
    const int nx = f.nx, ny = f.ny;
    double *T = (double *)f.T.p;
    hipError_t e;
    if ((e = gemm(Op::T, Op::N, nx, ny, nx, 1.0, (const double *)f.fx.p, nx, 0, X, nx, 0, 0.0, T, nx, 0, 1, s)))
        return e;
    if (ny > 1) {
        double *W = (double *)f.Y.p;
        if ((e = gemm(Op::N, Op::N, nx, ny, ny, 1.0, T, nx, 0, (const double *)f.fy.p, ny, 0, 0.0, W, nx, 0, 1, s)))
            return e;
        if ((e = launch_mul_symbol(nx * ny, 1, S, W, s))) return e;
        if ((e = gemm(Op::N, Op::T, nx, ny, ny, 1.0, W, nx, 0, (const double *)f.fy.p, ny, 0, 0.0, T, nx, 0, 1, s)))
            return e;
    } else if ((e = launch_mul_symbol(nx, 1, S, T, s))) {
        return e;
    }
    return gemm(Op::N, Op::N, nx, ny, nx, 1.0, (const double *)f.fx.p, nx, 0, T, nx, 0, 0.0, Y, nx, 0, 1, s);
}

acp_status scf(const acp_grid *grid, const double *m, const double *rho0, int n_e, const acp_scf_opts *o,
               double *psi, double *eps, double *veff, double *rho, int *iters_out, double *res_out, hipStream_t s,
               std::string &err) {
    if (!grid || !m || !o || !psi || !eps || !veff || !rho || n_e < 1) {
        err = "null argument";
        return ACP_EINVAL;
    }
    if (!(grid->kappa > 0) || !(grid->eps0 > 0) || !(grid->occ > 0)) {
        err = "kappa, eps0, occ must be > 0";
        return ACP_EINVAL;
    }
    Eig e;
    acp_status st = eig_prepare(e, grid, n_e, o->eig.n_guard, s, err);
    if (st != ACP_OK) return st;
    const int ng = e.ng, nx = e.g.nx, ny = e.g.ny;
    const double dv = std::pow(grid->h, grid->dim);
    const int max_iter = o->max_iter > 0 ? o->max_iter : 200;
    const double tol = o->tol > 0 ? o->tol : 1e-10;
    const double beta = o->beta > 0 ? o->beta : 0.3;
    const int hist = o->history == 0 ? 12 : std::max(0, std::min(o->history, 32));
    const double q0 = o->kerker_q0 == 0 ? 0.3 : o->kerker_q0;
    const double eig_tol = o->eig.tol > 0 ? o->eig.tol : 1e-10;
    const int degree = o->eig.degree > 0 ? o->eig.degree : 20;
    const int max_pass = o->eig.max_pass > 0 ? o->eig.max_pass : 60;
    GridFourier f;
    f.nx = nx;
    f.ny = ny;
    DevBuf Svc, Sker, rin, rout, R, tmp, Xh, Fh, part;
    auto cleanup = [&]() { release(Svc), release(Sker), release(rin), release(rout), release(R), release(tmp),
                           release(Xh), release(Fh), release(part); };
    if (!ensure(f.fx, (size_t)nx * nx * 8) || (ny > 1 && !ensure(f.fy, (size_t)ny * ny * 8)) ||
        !ensure(f.T, (size_t)ng * 8) || !ensure(f.Y, (size_t)ng * 8) || !ensure(Svc, (size_t)ng * 8) ||
        !ensure(Sker, (size_t)ng * 8) || !ensure(rin, (size_t)ng * 8) || !ensure(rout, (size_t)ng * 8) ||
        !ensure(R, (size_t)ng * 8) || !ensure(tmp, (size_t)ng * 8) ||
        !ensure(Xh, (size_t)(hist + 1) * ng * 8) || !ensure(Fh, (size_t)(hist + 1) * ng * 8) ||
        !ensure(part, 2 * 256 * 8)) {
        cleanup();
        err = "device allocation failed";
        return ACP_ENOMEM;
    }
    double *pin = (double *)rin.p, *pout = (double *)rout.p, *pr = (double *)R.p, *pt = (double *)tmp.p;
    double *X = (double *)Xh.p, *F = (double *)Fh.p;
    auto dev_fail = [&](const char *what) {
        cleanup();
        err = what;
        return ACP_EDEVICE;
    };
    if (launch_fourier_basis(nx, (double *)f.fx.p, s) || (ny > 1 && launch_fourier_basis(ny, (double *)f.fy.p, s)))
        return dev_fail("Fourier basis");
    hipLaunchKernelGGL(grid_symbol_kernel, dim3((ng + 255) / 256), dim3(256), 0, s, nx, ny, grid->h, 0, grid->eps0,
                       grid->kappa, (double *)Svc.p);
    hipLaunchKernelGGL(grid_symbol_kernel, dim3((ng + 255) / 256), dim3(256), 0, s, nx, ny, grid->h, 1, 0.0,
                       q0 > 0 ? q0 : 0.0, (double *)Sker.p);
    // start: rho0, or the neutral start -m scaled to f n_e electrons
    if (rho0) {
        if (hipMemcpyAsync(pin, rho0, (size_t)ng * 8, hipMemcpyDeviceToDevice, s)) return dev_fail("copy");
    } else {
        std::vector<double> mh(ng);
        if (hipMemcpyAsync(mh.data(), m, (size_t)ng * 8, hipMemcpyDeviceToHost, s) || hipStreamSynchronize(s))
            return dev_fail("copy");
        double q = 0.0;
        for (double v : mh) q -= v;
        q *= dv;
        const double sc = q != 0.0 ? grid->occ * n_e / q : 0.0;
        for (double &v : mh) v *= -sc;
        if (hipMemcpyAsync(pin, mh.data(), (size_t)ng * 8, hipMemcpyHostToDevice, s) || hipStreamSynchronize(s))
            return dev_fail("copy");
    }
    int nh = 0, it = 0;
    double res = INFINITY;
    std::vector<double> hp(512);
    for (it = 1; it <= max_iter; ++it) {
        // V = v_c (rho_in + m), its lowest n_e eigenpairs, rho_out
        if (launch_axpby(ng, 1, 1.0, m, ng, 0.0, pt, ng, s) || launch_axpby(ng, 1, 1.0, pin, ng, 1.0, pt, ng, s) ||
            fourier_apply(f, (const double *)Svc.p, pt, veff, s))
            return dev_fail("potential");
        st = eig_solve(e, veff, degree, max_pass, eig_tol, o->eig.seed, nullptr, nullptr, err);
        if (st != ACP_OK) {
            cleanup();
            return st;
        }
        hipLaunchKernelGGL(density_kernel, dim3((ng + 255) / 256), dim3(256), 0, s, ng, n_e, grid->occ / dv,
                           (const double *)e.B(e.ix), pout);
        // residual R = rho_out - rho_in, max |R| / max |rho_out|
        if (hipMemcpyAsync(pr, pout, (size_t)ng * 8, hipMemcpyDeviceToDevice, s) ||
            launch_axpby(ng, 1, -1.0, pin, ng, 1.0, pr, ng, s))
            return dev_fail("residual");
        hipLaunchKernelGGL(maxabs2_kernel, dim3(256), dim3(256), 0, s, ng, (const double *)pr, (const double *)pout,
                           (double *)part.p);
        if (hipMemcpyAsync(hp.data(), part.p, 512 * 8, hipMemcpyDeviceToHost, s) || hipStreamSynchronize(s))
            return dev_fail("reduction");
        double ar = 0.0, ao = 0.0;
        for (int b = 0; b < 256; ++b) {
            ar = std::max(ar, hp[2 * b]);
            ao = std::max(ao, hp[2 * b + 1]);
        }
        res = ao > 0 ? ar / ao : 0.0;
        if (std::getenv("ACP_SCF_VERBOSE")) std::fprintf(stderr, "[scf] %d %.3e\n", it, res);
        if (res <= tol) break;
        // Anderson mixing of the density (Kerker-preconditioned step):
        //   gamma = argmin |R - dF gamma|, rho_bar = rho_in - dX gamma,
        //   R_bar = R - dF gamma, rho_in <- rho_bar + beta K(R_bar)
        // with dX, dF the differences of the last stored (rho_in, R) pairs.
        const int slot = (it - 1) % (hist + 1);
        if (hist > 0) {
            if (hipMemcpyAsync(X + (size_t)slot * ng, pin, (size_t)ng * 8, hipMemcpyDeviceToDevice, s) ||
                hipMemcpyAsync(F + (size_t)slot * ng, pr, (size_t)ng * 8, hipMemcpyDeviceToDevice, s))
                return dev_fail("history");
            nh = std::min(nh + 1, hist + 1);
        }
        const int nd = nh - 1;   // differences between consecutive stored pairs
        std::vector<double> gam(std::max(nd, 0), 0.0);
        if (nd > 0) {
            // dF_l = F(slot_l+1) - F(slot_l) for the nd consecutive pairs ending at `slot`
            std::vector<int> sl(nh);
            for (int l = 0; l < nh; ++l) sl[l] = ((slot - (nh - 1 - l)) % (hist + 1) + hist + 1) % (hist + 1);
            // Gram of dF and dF^T R through the stored F (dots on the device)
            DevBuf dots;
            if (!ensure(dots, (size_t)(nh * nh + nh) * 8)) {
                cleanup();
                err = "device allocation failed";
                return ACP_ENOMEM;
            }
            double *dd = (double *)dots.p;
            for (int a = 0; a < nh; ++a) {
                for (int b = 0; b <= a; ++b)
                    if (launch_col_dot(ng, 1, F + (size_t)sl[a] * ng, ng, F + (size_t)sl[b] * ng, ng, dd + a * nh + b,
                                       s))
                        return dev_fail("dots");
                if (launch_col_dot(ng, 1, F + (size_t)sl[a] * ng, ng, pr, ng, dd + nh * nh + a, s)) return dev_fail("dots");
            }
            std::vector<double> h((size_t)nh * nh + nh);
            if (hipMemcpyAsync(h.data(), dd, h.size() * 8, hipMemcpyDeviceToHost, s) || hipStreamSynchronize(s))
                return dev_fail("dots");
            release(dots);
            auto g = [&](int a, int b) { return a >= b ? h[a * nh + b] : h[b * nh + a]; };
            // A(l, m) = dF_l . dF_m, rhs(l) = dF_l . R with dF_l = F_{l+1} - F_l
            std::vector<double> A((size_t)nd * nd), rhs(nd);
            for (int l = 0; l < nd; ++l) {
                for (int q = 0; q < nd; ++q)
                    A[l * nd + q] = g(l + 1, q + 1) - g(l + 1, q) - g(l, q + 1) + g(l, q);
                rhs[l] = h[(size_t)nh * nh + l + 1] - h[(size_t)nh * nh + l];
            }
            double tr = 0.0;
            for (int l = 0; l < nd; ++l) tr += A[l * nd + l];
            for (int l = 0; l < nd; ++l) A[l * nd + l] += 1e-12 * tr / nd;
            // Gaussian elimination with partial pivoting (nd <= 32)
            std::vector<int> pv(nd);
            bool ok = true;
            for (int c = 0; c < nd && ok; ++c) {
                int p = c;
                for (int r = c + 1; r < nd; ++r)
                    if (std::fabs(A[r * nd + c]) > std::fabs(A[p * nd + c])) p = r;
                if (!(std::fabs(A[p * nd + c]) > 0)) {
                    ok = false;
                    break;
                }
                if (p != c) {
                    for (int q = 0; q < nd; ++q) std::swap(A[c * nd + q], A[p * nd + q]);
                    std::swap(rhs[c], rhs[p]);
                }
                for (int r = c + 1; r < nd; ++r) {
                    const double l = A[r * nd + c] / A[c * nd + c];
                    for (int q = c; q < nd; ++q) A[r * nd + q] -= l * A[c * nd + q];
                    rhs[r] -= l * rhs[c];
                }
            }
            if (ok) {
                for (int c = nd - 1; c >= 0; --c) {
                    double v = rhs[c];
                    for (int q = c + 1; q < nd; ++q) v -= A[c * nd + q] * gam[q];
                    gam[c] = v / A[c * nd + c];
                }
            }
            // rho_bar = rho_in - sum gam_l (X_{l+1} - X_l), R_bar = R - sum gam_l (F_{l+1} - F_l)
            for (int l = 0; l < nd && ok; ++l) {
                if (launch_axpby(ng, 1, -gam[l], X + (size_t)sl[l + 1] * ng, ng, 1.0, pin, ng, s) ||
                    launch_axpby(ng, 1, gam[l], X + (size_t)sl[l] * ng, ng, 1.0, pin, ng, s) ||
                    launch_axpby(ng, 1, -gam[l], F + (size_t)sl[l + 1] * ng, ng, 1.0, pr, ng, s) ||
                    launch_axpby(ng, 1, gam[l], F + (size_t)sl[l] * ng, ng, 1.0, pr, ng, s))
                    return dev_fail("mixing");
            }
        }
        // rho_in <- rho_bar + beta K(R_bar)
        if (q0 > 0) {
            if (fourier_apply(f, (const double *)Sker.p, pr, pt, s) || launch_axpby(ng, 1, beta, pt, ng, 1.0, pin, ng, s))
                return dev_fail("Kerker step");
        } else if (launch_axpby(ng, 1, beta, pr, ng, 1.0, pin, ng, s)) {
            return dev_fail("step");
        }
    }
    // outputs: the orbitals and energies of V[rho_in], and rho_in (= rho_out to tol)
    if (hipMemcpyAsync(psi, e.B(e.ix), (size_t)ng * n_e * 8, hipMemcpyDeviceToDevice, s) ||
        hipMemcpyAsync(rho, pout, (size_t)ng * 8, hipMemcpyDeviceToDevice, s) || hipStreamSynchronize(s))
        return dev_fail("copy");
    std::memcpy(eps, e.lamh.data(), (size_t)(n_e + 1) * 8);
    if (iters_out) *iters_out = std::min(it, max_iter);
    if (res_out) *res_out = res;
    cleanup();
    if (res > tol) {
        char buf[96];
        std::snprintf(buf, sizeof buf, "SCF residual %.3e above tol", res);
        err = buf;
        return ACP_ENOCONV;
    }
    return ACP_OK;
}

hipError_t launch_col_scale_rsqrt(int m, int n, double *W, int ldw, const double *d, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_cols_rsqrt_kernel, dim3((m + 255) / 256, n), dim3(256), 0, s, m, n, W, ldw, d);
    return hipGetLastError();
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

extern "C" acp_status acp_scf(const acp_grid *grid, const double *m, const double *rho0, int n_e,
                              const acp_scf_opts *opts, double *psi, double *eps, double *veff, double *rho,
                              int *iters, double *max_res, void *stream) {
    std::string err;
    const acp_status st = acp::scf(grid, m, rho0, n_e, opts, psi, eps, veff, rho, iters, max_res,
                                   (hipStream_t)stream, err);
    acp::g_free_error = err;
    return st;
}
