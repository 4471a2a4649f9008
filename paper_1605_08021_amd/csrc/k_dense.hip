// Point selection for the interpolative decomposition and small dense FP64
// algebra on the GPU.
//
// ISDF (Alg. 2 with the sketch of the Remark after it).  The rows of the
// sketched matrix are M~(alpha, :) = G~(alpha, :) (x) phi(alpha, :), so the Gram
// matrix of those rows factorises as a Hadamard product
//     K(alpha, beta) = (phi(alpha,:) . phi(beta,:)) * (G~(alpha,:) . G~(beta,:)).
// Column-pivoted QR of M~^T picks, at step k, the row of largest residual norm
// after projecting out the rows already chosen.  Greedy pivoted Cholesky of K
// with the largest remaining diagonal as pivot makes the same choices in exact
// arithmetic (the residual diagonal of K is the squared residual row norm) and
// its factor L satisfies L(Pi,:) = R11^T and L(rest,:) = R12^T, so the
// interpolation vectors Xi^T = R11^{-1} [R11 R12] (Alg. 2 step 4) are
//     Xi = L L11^{-1},  with Xi(Pi, :) = I set exactly.
// M~ is never formed: each step costs one column of K (N_g (N_e + r)) and one
// update with the previous columns of L (N_g k).
//
// Dense algebra: Gauss-Jordan elimination with partial pivoting for the
// N_mu x N_mu system of the Sherman-Morrison-Woodbury update (Eq. (3.13)),
// triangular inversion, cyclic Jacobi for the eigenvalues of the dynamical
// matrix, and the assembly D = M^{-1/2} (sym(h^d G^T U) + K_local) M^{-1/2}.
#include "acp_internal.h"

namespace acp {
namespace {

inline unsigned nblk(long long tot, int b) { return (unsigned)((tot + b - 1) / b); }

// diag(alpha) = |phi(alpha,:)|^2 |G~(alpha,:)|^2
__global__ void isdf_diag_kernel(int ng, int ne, int r, const double *phi, int ldphi,
                                 const double *gt, int ldg, double *diag) {
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= ng) return;
    double s1 = 0.0, s2 = 0.0;
    for (int i = 0; i < ne; ++i) {
        double v = phi[a + (long long)i * ldphi];
        s1 += v * v;
    }
    for (int j = 0; j < r; ++j) {
        double v = gt[a + (long long)j * ldg];
        s2 += v * v;
    }
    diag[a] = s1 * s2;
}

// One workgroup: pivot for step k = argmax diag (ties -> smallest index), unless a
// forced selection is given.  state[0] = number of accepted pivots, state[1] = stop flag.
// dvals[0] = first pivot value (for the rank rule).
__global__ void isdf_pivot_kernel(int ng, int k, const double *diag, int *sel, const int *forced,
                                  double tol2, int *state, double *dvals) {
    __shared__ double bv[1024];
    __shared__ int bi[1024];
    const int t = threadIdx.x;
    if (state[1]) return;
    double best = -1.0;
    int besti = 0x7fffffff;
    if (forced) {
        if (t == 0) { best = diag[forced[k]]; besti = forced[k]; }
    } else {
        for (int a = t; a < ng; a += 1024) {
            double v = diag[a];
            if (v > best) { best = v; besti = a; }   // ascending a: first max kept
        }
    }
    bv[t] = best;
    bi[t] = besti;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) {
            double o = bv[t + w];
            int oi = bi[t + w];
            if (o > bv[t] || (o == bv[t] && oi < bi[t])) { bv[t] = o; bi[t] = oi; }
        }
        __syncthreads();
    }
    if (t == 0) {
        double piv = bv[0];
        if (k == 0) dvals[0] = piv;
        bool stop = !(piv > 0.0);
        if (!forced && tol2 > 0.0 && k > 0 && piv < tol2 * dvals[0]) stop = true;
        if (stop) {
            state[1] = 1;
        } else {
            sel[k] = bi[0];
            dvals[1] = piv;
            state[0] = k + 1;
        }
    }
}

// Column k of L: L(a,k) = (K(a,p) - sum_{j<k} L(a,j) L(p,j)) / sqrt(d_p);
// diag(a) -= L(a,k)^2; the pivot row is retired.
__global__ void isdf_column_kernel(int ng, int ne, int r, int k, const double *phi, int ldphi,
                                   const double *gt, int ldg, double *L, int ldl, double *diag,
                                   const int *sel, const int *state, const double *dvals) {
    if (state[0] != k + 1) return;   // stopped before this step
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= ng) return;
    const int p = sel[k];
    double s1 = 0.0, s2 = 0.0;
    for (int i = 0; i < ne; ++i) s1 += phi[a + (long long)i * ldphi] * phi[p + (long long)i * ldphi];
    for (int j = 0; j < r; ++j) s2 += gt[a + (long long)j * ldg] * gt[p + (long long)j * ldg];
    double g = s1 * s2;
    for (int j = 0; j < k; ++j) g -= L[a + (long long)j * ldl] * L[p + (long long)j * ldl];
    const double piv = dvals[1];
    const double lk = g / sqrt(piv);
    L[a + (long long)k * ldl] = lk;
    if (a == p) diag[a] = -1.0;
    else diag[a] -= lk * lk;
}

// L11(i, j) = L(sel[i], j) for j <= i, 0 above the diagonal.
__global__ void gather_lower_kernel(int n, const int *sel, const double *L, int ldl, double *L11) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * n) return;
    int i = (int)(idx % n);
    int j = (int)(idx / n);
    L11[idx] = (j <= i) ? L[sel[i] + (long long)j * ldl] : 0.0;
}

// Inverse of a lower-triangular matrix, one thread per column.
__global__ void tri_inverse_lower_kernel(int n, const double *L, int ldl, double *X) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double *x = X + (long long)j * n;
    for (int i = 0; i < j; ++i) x[i] = 0.0;
    x[j] = 1.0 / L[j + (long long)j * ldl];
    for (int i = j + 1; i < n; ++i) {
        double s = 0.0;
        for (int l = j; l < i; ++l) s += L[i + (long long)l * ldl] * x[l];
        x[i] = -s / L[i + (long long)i * ldl];
    }
}

// ------------------------------------------------------------ Gauss-Jordan
// Step k, part 1 (one workgroup): partial pivot in column k, swap rows k and p
// of [A | B].
__global__ void gj_pivot_kernel(int n, int nrhs, int k, double *A, int lda, double *B, int ldb) {
    __shared__ double bv[1024];
    __shared__ int bi[1024];
    __shared__ int s_p;
    const int t = threadIdx.x;
    double best = -1.0;
    int besti = k;
    for (int i = k + t; i < n; i += 1024) {
        double v = fabs(A[i + (long long)k * lda]);
        if (v > best) { best = v; besti = i; }
    }
    bv[t] = best;
    bi[t] = besti;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) {
            if (bv[t + w] > bv[t] || (bv[t + w] == bv[t] && bi[t + w] < bi[t])) {
                bv[t] = bv[t + w];
                bi[t] = bi[t + w];
            }
        }
        __syncthreads();
    }
    if (t == 0) s_p = bi[0];
    __syncthreads();
    const int p = s_p;
    if (p != k) {
        for (int j = t; j < n; j += 1024) {
            double a = A[k + (long long)j * lda];
            A[k + (long long)j * lda] = A[p + (long long)j * lda];
            A[p + (long long)j * lda] = a;
        }
        for (int j = t; j < nrhs; j += 1024) {
            double b = B[k + (long long)j * ldb];
            B[k + (long long)j * ldb] = B[p + (long long)j * ldb];
            B[p + (long long)j * ldb] = b;
        }
    }
}

// Step k, part 2: eliminate column k from every other row (columns > k of A, all of B).
__global__ void gj_eliminate_kernel(int n, int nrhs, int k, double *A, int lda, double *B,
                                    int ldb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;   // row
    const int jj = blockIdx.y;                               // column group
    if (i >= n || i == k) return;
    const double f = A[i + (long long)k * lda] / A[k + (long long)k * lda];
    if (f == 0.0) return;
    const int ncols = (n - k - 1) + nrhs;
    for (int q = jj; q < ncols; q += gridDim.y) {
        if (q < n - k - 1) {
            const int j = k + 1 + q;
            A[i + (long long)j * lda] -= f * A[k + (long long)j * lda];
        } else {
            const int j = q - (n - k - 1);
            B[i + (long long)j * ldb] -= f * B[k + (long long)j * ldb];
        }
    }
}

__global__ void gj_finish_kernel(int n, int nrhs, const double *A, int lda, double *B, int ldb) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * nrhs) return;
    int i = (int)(idx % n);
    long long j = idx / n;
    B[i + j * ldb] /= A[i + (long long)i * lda];
}

// ------------------------------------------------------------ Jacobi eigenvalues
// Cyclic Jacobi with round-robin (tournament) ordering: N-1 rounds of N/2
// disjoint rotations per sweep (N = n rounded up to even; a pair containing the
// extra position is a bye), each zeroing A(p,q) with the classical choice
// t = sign(theta) / (|theta| + sqrt(theta^2 + 1)), theta = (A_qq - A_pp) / (2 A_pq).
// One workgroup; A (n x n) in global memory.  work holds N doubles + N ints.
__global__ void jacobi_kernel(int n, double *A, int lda, double *eig, double *work, int max_sweeps,
                              double tol) {
    const int N = n + (n & 1);
    const int half = N / 2;
    double *cs = work;
    double *sn = work + half;
    int *pq = (int *)(work + N);
    __shared__ double red[1024];
    __shared__ int s_done;
    const int t = threadIdx.x;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (long long idx = t; idx < (long long)n * n; idx += 1024) {
            int i = (int)(idx % n), j = (int)(idx / n);
            double v = A[i + (long long)j * lda];
            tot += v * v;
            if (i != j) off += v * v;
        }
        red[t] = off;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) { if (t < w) red[t] += red[t + w]; __syncthreads(); }
        const double offs = red[0];
        __syncthreads();
        red[t] = tot;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) { if (t < w) red[t] += red[t + w]; __syncthreads(); }
        const double tots = red[0];
        if (t == 0) s_done = (offs <= tol * tol * tots) ? 1 : 0;
        __syncthreads();
        if (s_done) break;
        for (int round = 0; round < N - 1; ++round) {
            for (int k = t; k < half; k += 1024) {
                int a = (k == 0) ? 0 : 1 + (k - 1 + round) % (N - 1);
                int b = 1 + (N - 2 - k + round) % (N - 1);
                int p = a < b ? a : b, q = a < b ? b : a;
                double c = 1.0, s = 0.0;
                if (q < n) {
                    double apq = A[p + (long long)q * lda];
                    if (apq != 0.0) {
                        double app = A[p + (long long)p * lda], aqq = A[q + (long long)q * lda];
                        double theta = (aqq - app) / (2.0 * apq);
                        double tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(tt * tt + 1.0);
                        s = tt * c;
                    }
                } else {
                    q = -1;   // bye
                }
                pq[2 * k] = p;
                pq[2 * k + 1] = q;
                cs[k] = c;
                sn[k] = s;
            }
            __syncthreads();
            // columns: A <- A J
            for (long long idx = t; idx < (long long)half * n; idx += 1024) {
                int k = (int)(idx / n), i = (int)(idx % n);
                int p = pq[2 * k], q = pq[2 * k + 1];
                if (q < 0) continue;
                double c = cs[k], s = sn[k];
                double aip = A[i + (long long)p * lda], aiq = A[i + (long long)q * lda];
                A[i + (long long)p * lda] = c * aip - s * aiq;
                A[i + (long long)q * lda] = s * aip + c * aiq;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (long long idx = t; idx < (long long)half * n; idx += 1024) {
                int k = (int)(idx / n), j = (int)(idx % n);
                int p = pq[2 * k], q = pq[2 * k + 1];
                if (q < 0) continue;
                double c = cs[k], s = sn[k];
                double apj = A[p + (long long)j * lda], aqj = A[q + (long long)j * lda];
                A[p + (long long)j * lda] = c * apj - s * aqj;
                A[q + (long long)j * lda] = s * apj + c * aqj;
            }
            __syncthreads();
        }
    }
    // rank sort of the diagonal (ties broken by index)
    for (int i = t; i < n; i += 1024) {
        double v = A[i + (long long)i * lda];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            double u = A[j + (long long)j * lda];
            if (u < v || (u == v && j < i)) ++rank;
        }
        eig[rank] = v;
    }
}

// D = M^{-1/2} ((Phi + Phi^T)/2 + K) M^{-1/2}; asym2 = {||Phi - Phi^T||^2, ||Phi||^2}.
__global__ void dynmat_assemble_kernel(int np, int dim, const double *Phi, const double *K,
                                       const double *mass, double *D, int ldd, double *asym2) {
    __shared__ double r0[1024], r1[1024];
    const int t = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (long long idx = t; idx < (long long)np * np; idx += 1024) {
        int i = (int)(idx % np), j = (int)(idx / np);
        double pij = Phi[i + (long long)j * np], pji = Phi[j + (long long)i * np];
        double h = 0.5 * (pij + pji) + (K ? K[i + (long long)j * np] : 0.0);
        double mi = mass ? mass[i / dim] : 1.0, mj = mass ? mass[j / dim] : 1.0;
        D[i + (long long)j * ldd] = h / sqrt(mi * mj);
        a += (pij - pji) * (pij - pji);
        b += pij * pij;
    }
    r0[t] = a;
    r1[t] = b;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) { r0[t] += r0[t + w]; r1[t] += r1[t + w]; }
        __syncthreads();
    }
    if (t == 0) { asym2[0] = r0[0]; asym2[1] = r1[0]; }
}

}  // namespace

hipError_t isdf_pivoted_cholesky(int ng, int ne, int r, const double *phi, int ldphi,
                                 const double *gt, int ldg, int nmu_max, double tol, double *L,
                                 int ldl, double *diag, int *sel_dev, const int *forced,
                                 int *nmu_out_host, void *scratch, hipStream_t s) {
    // scratch: int state[2] | pad | double dvals[2]
    int *state = (int *)scratch;
    double *dvals = (double *)((char *)scratch + 16);
    hipError_t e = hipMemsetAsync(state, 0, 2 * sizeof(int), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(isdf_diag_kernel, dim3(nblk(ng, 256)), dim3(256), 0, s, ng, ne, r, phi,
                       ldphi, gt, ldg, diag);
    const double tol2 = tol * tol;
    for (int k = 0; k < nmu_max; ++k) {
        hipLaunchKernelGGL(isdf_pivot_kernel, dim3(1), dim3(1024), 0, s, ng, k, diag, sel_dev,
                           forced, tol2, state, dvals);
        hipLaunchKernelGGL(isdf_column_kernel, dim3(nblk(ng, 256)), dim3(256), 0, s, ng, ne, r, k,
                           phi, ldphi, gt, ldg, L, ldl, diag, sel_dev, state, dvals);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    int hstate[2];
    e = hipMemcpyAsync(hstate, state, sizeof(hstate), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (nmu_out_host) *nmu_out_host = hstate[0];
    return hipSuccess;
}

hipError_t launch_tri_inverse_lower(int n, const double *L, int ldl, double *Linv, hipStream_t s) {
    hipLaunchKernelGGL(tri_inverse_lower_kernel, dim3(nblk(n, 64)), dim3(64), 0, s, n, L, ldl,
                       Linv);
    return hipGetLastError();
}

hipError_t launch_gather_lower(int n, const int *sel, const double *L, int ldl, double *L11,
                               hipStream_t s) {
    long long tot = (long long)n * n;
    hipLaunchKernelGGL(gather_lower_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, n, sel, L, ldl,
                       L11);
    return hipGetLastError();
}

hipError_t gauss_jordan_solve(int n, int nrhs, double *A, int lda, double *B, int ldb,
                              int * /*piv_scratch*/, hipStream_t s) {
    for (int k = 0; k < n; ++k) {
        hipLaunchKernelGGL(gj_pivot_kernel, dim3(1), dim3(1024), 0, s, n, nrhs, k, A, lda, B, ldb);
        int ncols = (n - k - 1) + nrhs;
        int gy = ncols < 64 ? (ncols > 0 ? ncols : 1) : 64;
        hipLaunchKernelGGL(gj_eliminate_kernel, dim3(nblk(n, 256), gy), dim3(256), 0, s, n, nrhs,
                           k, A, lda, B, ldb);
    }
    long long tot = (long long)n * nrhs;
    hipLaunchKernelGGL(gj_finish_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, n, nrhs, A, lda,
                       B, ldb);
    return hipGetLastError();
}

hipError_t jacobi_eigvals(int n, double *A, int lda, double *eig, double *work, hipStream_t s) {
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(1024), 0, s, n, A, lda, eig, work, 40, 1e-15);
    return hipGetLastError();
}

hipError_t launch_dynmat_assemble(int np, int dim, const double *Phi_el, const double *K_local,
                                  const double *mass, double *D, double *asym2, hipStream_t s) {
    hipLaunchKernelGGL(dynmat_assemble_kernel, dim3(1), dim3(1024), 0, s, np, dim, Phi_el, K_local,
                       mass, D, np, asym2);
    return hipGetLastError();
}

}  // namespace acp
