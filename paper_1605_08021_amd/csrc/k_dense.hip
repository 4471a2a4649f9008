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

// The ISDF kernels work on row-major data: phi_rm (N_g x nep), gt_rm (N_g x r)
// and L_rm (N_g x ldl), so that one grid row is contiguous.  A wave handles 4
// rows with 16 lanes per row; dot products over orbitals, sketch columns and
// previous pivots are split over the 16 lanes and reduced by shuffles in a
// fixed order.  Each block leaves its best remaining diagonal entry as a
// candidate (value, row); every block of the next step reduces the candidates
// itself, so one launch per pivot suffices.
constexpr int ISDF_NT = 256;
constexpr int ISDF_ROWS = ISDF_NT / 16;   // rows per block

struct Cand {
    double v;
    int i;
    int pad;
};

__device__ __forceinline__ double sum16(double v) {
#pragma unroll
    for (int m = 8; m > 0; m >>= 1) v += __shfl_xor(v, m, 16);
    return v;
}

__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
    return v > bv || (v == bv && i < bi);
}

// Block-level candidate of the rows owned by this block (LDS reduction).
__device__ void block_candidate(double v, int i, Cand *out) {
    __shared__ double sv[ISDF_ROWS];
    __shared__ int si[ISDF_ROWS];
    const int t = threadIdx.x;
    if ((t & 15) == 0) { sv[t >> 4] = v; si[t >> 4] = i; }
    __syncthreads();
    if (t == 0) {
        double bv = sv[0];
        int bi = si[0];
        for (int k = 1; k < ISDF_ROWS; ++k)
            if (better(sv[k], si[k], bv, bi)) { bv = sv[k]; bi = si[k]; }
        out[blockIdx.x].v = bv;
        out[blockIdx.x].i = bi;
    }
}

// diag(alpha) = |phi(alpha,:)|^2 |G~(alpha,:)|^2 and the first candidates.
__global__ __launch_bounds__(ISDF_NT) void isdf_init_kernel(int ng, int nep, int r,
                                                            const double *phi_rm, const double *gt_rm,
                                                            double *diag, Cand *cand) {
    const int t = threadIdx.x;
    const int l16 = t & 15;
    const int a = blockIdx.x * ISDF_ROWS + (t >> 4);
    double s1 = 0.0, s2 = 0.0;
    if (a < ng) {
        for (int i = l16; i < nep; i += 16) { const double v = phi_rm[(long long)a * nep + i]; s1 += v * v; }
        for (int j = l16; j < r; j += 16) { const double v = gt_rm[(long long)a * r + j]; s2 += v * v; }
    }
    s1 = sum16(s1);
    s2 = sum16(s2);
    const double d = s1 * s2;
    if (a < ng && l16 == 0) diag[a] = d;
    block_candidate(a < ng ? d : -2.0, a < ng ? a : 0x7fffffff, cand);
}

// Step k of the greedy pivoted Cholesky of K = (Phi Phi^T) o (G~ G~^T):
//   p = argmax diag (ties -> smallest index), or forced[k];
//   L(a,k) = (K(a,p) - sum_{j<k} L(a,j) L(p,j)) / sqrt(diag(p)), diag(a) -= L(a,k)^2.
// state[0] = accepted pivots, state[1] = stopped; dvals[0] = first pivot value.
__global__ __launch_bounds__(ISDF_NT) void isdf_step_kernel(
    int ng, int nep, int r, int k, int nblk, const double *phi_rm, const double *gt_rm, double *L,
    int ldl, double *diag, int *sel, const int *forced, double tol2, int *state, double *dvals,
    const Cand *cand_in, Cand *cand_out) {
    __shared__ double s_piv;
    __shared__ int s_p, s_stop;
    __shared__ double rv[ISDF_NT];
    __shared__ int ri[ISDF_NT];
    const int t = threadIdx.x;
    const int stopped = state[1];
    if (!forced && !stopped) {
        // every block reduces the previous step's candidates (fixed tree order)
        double bv = -2.0;
        int bi = 0x7fffffff;
        for (int b = t; b < nblk; b += ISDF_NT)
            if (better(cand_in[b].v, cand_in[b].i, bv, bi)) { bv = cand_in[b].v; bi = cand_in[b].i; }
        rv[t] = bv;
        ri[t] = bi;
        __syncthreads();
        for (int w = ISDF_NT / 2; w > 0; w >>= 1) {
            if (t < w && better(rv[t + w], ri[t + w], rv[t], ri[t])) { rv[t] = rv[t + w]; ri[t] = ri[t + w]; }
            __syncthreads();
        }
    }
    if (t == 0) {
        int stop = stopped;
        double bv = -2.0;
        int bi = 0x7fffffff;
        if (!stop) {
            if (forced) {
                bi = forced[k];
                bv = diag[bi];
            } else {
                bv = rv[0];
                bi = ri[0];
            }
            if (!(bv > 0.0)) stop = 1;
            if (!forced && tol2 > 0.0 && k > 0 && bv < tol2 * dvals[0]) stop = 1;
        }
        s_piv = bv;
        s_p = bi;
        s_stop = stop;
        if (blockIdx.x == 0) {
            if (stop) {
                state[1] = 1;
            } else {
                sel[k] = bi;
                state[0] = k + 1;
                if (k == 0) dvals[0] = bv;
            }
        }
    }
    __syncthreads();
    if (s_stop) return;
    const int p = s_p;
    const double rsq = 1.0 / sqrt(s_piv);
    const int l16 = t & 15;
    const int a = blockIdx.x * ISDF_ROWS + (t >> 4);
    const int ac = a < ng ? a : ng - 1;
    double s1 = 0.0, s2 = 0.0, y = 0.0;
    for (int i = l16; i < nep; i += 16) s1 += phi_rm[(long long)ac * nep + i] * phi_rm[(long long)p * nep + i];
    for (int j = l16; j < r; j += 16) s2 += gt_rm[(long long)ac * r + j] * gt_rm[(long long)p * r + j];
    for (int j = l16; j < k; j += 16) y += L[(long long)ac * ldl + j] * L[(long long)p * ldl + j];
    s1 = sum16(s1);
    s2 = sum16(s2);
    y = sum16(y);
    double dnew = -2.0;
    if (a < ng) {
        const double lk = (s1 * s2 - y) * rsq;
        dnew = (a == p) ? -1.0 : diag[a] - lk * lk;
        if (l16 == 0) {
            L[(long long)a * ldl + k] = lk;
            diag[a] = dnew;
        }
    }
    block_candidate(dnew, a < ng ? a : 0x7fffffff, cand_out);
}

// L11(i, j) = L(sel[i], j) for j <= i, 0 above the diagonal (L row-major, ld ldl).
__global__ void gather_lower_kernel(int n, const int *sel, const double *L, int ldl, double *L11) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * n) return;
    int i = (int)(idx % n);
    int j = (int)(idx / n);
    L11[idx] = (j <= i) ? L[(long long)sel[i] * ldl + j] : 0.0;
}

// Inverse of the lower-triangular L11 (row i = L_rm(sel[i], 0..i)), one wave per
// column j:  x_j = 1 / L_jj,  x_i = -(sum_{l=j}^{i-1} L_il x_l) / L_ii.  Each dot
// product is split over the 64 lanes (contiguous row of L) and reduced by
// shuffles in a fixed order; x lives in LDS.
constexpr int TRI_MAX = 4096;
__global__ __launch_bounds__(64) void tri_inverse_rows_kernel(int n, const int *sel, const double *L,
                                                              int ldl, double *X) {
    __shared__ double x[TRI_MAX];
    const int j = blockIdx.x;
    const int lane = threadIdx.x;
    for (int i = lane; i < n; i += 64) x[i] = 0.0;
    __syncthreads();
    const double *Lj = L + (long long)sel[j] * ldl;
    if (lane == 0) x[j] = 1.0 / Lj[j];
    __syncthreads();
    for (int i = j + 1; i < n; ++i) {
        const double *Li = L + (long long)sel[i] * ldl;
        double sacc = 0.0;
        for (int l = j + lane; l < i; l += 64) sacc += Li[l] * x[l];
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) sacc += __shfl_xor(sacc, m, 64);
        if (lane == 0) x[i] = -sacc / Li[i];
        __syncthreads();
    }
    for (int i = lane; i < n; i += 64) X[i + (long long)j * n] = x[i];
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
    __shared__ int s_rot;
    const int t = threadIdx.x;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        if (t == 0) s_rot = 0;
        __syncthreads();
        for (int round = 0; round < N - 1; ++round) {
            for (int k = t; k < half; k += 1024) {
                int a = (k == 0) ? 0 : 1 + (k - 1 + round) % (N - 1);
                int b = 1 + (N - 2 - k + round) % (N - 1);
                int p = a < b ? a : b, q = a < b ? b : a;
                double c = 1.0, s = 0.0;
                if (q < n) {
                    double apq = A[p + (long long)q * lda];
                    double app = A[p + (long long)p * lda], aqq = A[q + (long long)q * lda];
                    if (fabs(apq) > tol * sqrt(fabs(app * aqq)) && apq != 0.0) {
                        atomicAdd(&s_rot, 1);
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
        if (s_rot == 0) break;
        __syncthreads();
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

hipError_t isdf_pivoted_cholesky(int ng, int nep, int r, const double *phi_rm, const double *gt_rm,
                                 int nmu_max, double tol, double *L, int ldl, double *diag,
                                 int *sel_dev, const int *forced, int *nmu_out_host, void *scratch,
                                 hipStream_t s) {
    // scratch: int state[2] | pad | double dvals[2] | Cand[2][nblk]
    const int nblk = (ng + ISDF_ROWS - 1) / ISDF_ROWS;
    int *state = (int *)scratch;
    double *dvals = (double *)((char *)scratch + 16);
    Cand *c0 = (Cand *)((char *)scratch + 32);
    Cand *c1 = c0 + nblk;
    hipError_t e = hipMemsetAsync(state, 0, 2 * sizeof(int), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(isdf_init_kernel, dim3(nblk), dim3(ISDF_NT), 0, s, ng, nep, r, phi_rm, gt_rm,
                       diag, c0);
    const double tol2 = tol * tol;
    for (int k = 0; k < nmu_max; ++k) {
        hipLaunchKernelGGL(isdf_step_kernel, dim3(nblk), dim3(ISDF_NT), 0, s, ng, nep, r, k, nblk,
                           phi_rm, gt_rm, L, ldl, diag, sel_dev, forced, tol2, state, dvals,
                           (k & 1) ? c1 : c0, (k & 1) ? c0 : c1);
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

size_t isdf_scratch_bytes(int ng) {
    const int nblk = (ng + ISDF_ROWS - 1) / ISDF_ROWS;
    return 32 + 2 * (size_t)nblk * sizeof(Cand);
}

hipError_t launch_tri_inverse_rows(int n, const int *sel, const double *L, int ldl, double *Linv,
                                  hipStream_t s) {
    if (n > TRI_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tri_inverse_rows_kernel, dim3(n), dim3(64), 0, s, n, sel, L, ldl, Linv);
    return hipGetLastError();
}

hipError_t launch_gather_lower(int n, const int *sel, const double *L, int ldl, double *L11,
                               hipStream_t s) {
    long long tot = (long long)n * n;
    hipLaunchKernelGGL(gather_lower_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, n, sel, L, ldl,
                       L11);
    return hipGetLastError();
}

// ------------------------------------------------------------ blocked LU solve
// A X = B by a right-looking blocked LU with partial pivoting applied to the
// augmented [A | B] (A n x n, B n x nrhs, column-major, in place): panels of
// LU_NB columns are factored by one workgroup with the panel in LDS; their row
// interchanges are applied to the other columns, the block row is solved with
// the unit lower triangle, and the trailing matrix (and B) is updated by a GEMM
// on the matrix cores.  Back substitution then proceeds by blocks.
constexpr int LU_NB = 32;
constexpr int LU_MAXM = 576;      // panel rows held in LDS (LU_MAXM x LU_NB doubles)
constexpr int LU_NT = 1024;

__global__ __launch_bounds__(LU_NT) void lu_panel_kernel(int m, int nb, double *A, int lda, int *piv) {
    __shared__ double P[LU_MAXM * LU_NB];    // P[c * m + r]
    __shared__ double wv[LU_NT / 64];
    __shared__ int wi[LU_NT / 64];
    __shared__ int s_p;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int i = t; i < m * nb; i += LU_NT) {
        const int c = i / m, r = i % m;
        P[i] = A[r + (long long)c * lda];
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        // pivot: largest |P[r][j]|, r >= j, ties to the smallest row (m <= LU_NT:
        // one row per thread, wave shuffles, then the 16 wave results)
        double bv = -1.0;
        int bi = 0x7fffffff;
        if (t >= j && t < m) {
            bv = fabs(P[j * m + t]);
            bi = t;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane == 0) {
            wv[wave] = bv;
            wi[wave] = bi;
        }
        __syncthreads();
        if (t == 0) {
            double b = wv[0];
            int bi0 = wi[0];
            for (int w = 1; w < LU_NT / 64; ++w)
                if (wv[w] > b || (wv[w] == b && wi[w] < bi0)) {
                    b = wv[w];
                    bi0 = wi[w];
                }
            s_p = bi0;
            piv[j] = bi0;
        }
        __syncthreads();
        const int p = s_p;
        // the pivot row's entries (after the swap) and the multipliers, from
        // values read before any thread writes
        const double piv_jj = P[j * m + p];
        double lr = 0.0;
        int r = -1;
        if (t > j && t < m) {
            r = t;
            const int src = (r == p) ? j : r;           // row r after the swap
            lr = P[j * m + src] / piv_jj;
        }
        __syncthreads();
        if (t < nb && p != j) {
            const double a = P[t * m + j];
            P[t * m + j] = P[t * m + p];
            P[t * m + p] = a;
        }
        __syncthreads();
        if (r >= 0) {
            P[j * m + r] = lr;
            for (int c = j + 1; c < nb; ++c) P[c * m + r] -= lr * P[c * m + j];
        }
        __syncthreads();
    }
    for (int i = t; i < m * nb; i += LU_NT) {
        const int c = i / m, r = i % m;
        A[r + (long long)c * lda] = P[i];
    }
}

// Row interchanges of panel k0 (rows k0 + j <-> k0 + piv[j], in order) on every
// column outside the panel, and on B.  One thread per column.
__global__ void lu_swap_kernel(int n, int nrhs, int k0, int nb, const int *piv, double *A, int lda,
                               double *B, int ldb) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n + nrhs) return;
    if (c >= k0 && c < k0 + nb) return;
    double *col = c < n ? A + (long long)c * lda : B + (long long)(c - n) * ldb;
    for (int j = 0; j < nb; ++j) {
        const int p = piv[j];
        if (p != j) {
            const double a = col[k0 + j];
            col[k0 + j] = col[k0 + p];
            col[k0 + p] = a;
        }
    }
}

// Block row k0: X = L11^{-1} X for the columns right of the panel and for B
// (L11 unit lower, nb x nb, staged in LDS).  One thread per column.
__global__ __launch_bounds__(64) void lu_trsm_lower_kernel(int n, int nrhs, int k0, int nb, const double *A,
                                                           int lda, double *Aw, double *B, int ldb) {
    __shared__ double L[LU_NB * LU_NB];
    for (int i = threadIdx.x; i < LU_NB * LU_NB; i += 64) {
        const int r = i % LU_NB, c = i / LU_NB;
        L[r * LU_NB + c] = (r < nb && c < nb) ? A[(k0 + r) + (long long)(k0 + c) * lda] : 0.0;
    }
    __syncthreads();
    const int c0 = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncols = (n - k0 - nb) + nrhs;
    if (c0 >= ncols) return;
    double *col = c0 < n - k0 - nb ? Aw + (long long)(k0 + nb + c0) * lda : B + (long long)(c0 - (n - k0 - nb)) * ldb;
    double x[LU_NB];
#pragma unroll
    for (int i = 0; i < LU_NB; ++i) x[i] = i < nb ? col[k0 + i] : 0.0;
#pragma unroll
    for (int i = 1; i < LU_NB; ++i) {
        double sacc = x[i];
#pragma unroll
        for (int j = 0; j < i; ++j) sacc -= L[i * LU_NB + j] * x[j];
        x[i] = sacc;
    }
    for (int i = 0; i < nb; ++i) col[k0 + i] = x[i];
}

// Back substitution on block rows r0..r0+nb-1: X = U11^{-1} X for every column
// of B (U11 staged in LDS).  One thread per column.
__global__ __launch_bounds__(64) void lu_trsm_upper_kernel(int nrhs, int r0, int nb, const double *A, int lda,
                                                           double *B, int ldb) {
    __shared__ double U[LU_NB * LU_NB];
    for (int i = threadIdx.x; i < LU_NB * LU_NB; i += 64) {
        const int r = i % LU_NB, c = i / LU_NB;
        U[r * LU_NB + c] = (r < nb && c < nb) ? A[(r0 + r) + (long long)(r0 + c) * lda] : (r == c ? 1.0 : 0.0);
    }
    __syncthreads();
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    double *col = B + (long long)c * ldb;
    double x[LU_NB];
#pragma unroll
    for (int i = 0; i < LU_NB; ++i) x[i] = i < nb ? col[r0 + i] : 0.0;
#pragma unroll
    for (int i = LU_NB - 1; i >= 0; --i) {
        double sacc = x[i];
#pragma unroll
        for (int j = i + 1; j < LU_NB; ++j) sacc -= U[i * LU_NB + j] * x[j];
        x[i] = sacc / U[i * LU_NB + i];
    }
    for (int i = 0; i < nb; ++i) col[r0 + i] = x[i];
}

hipError_t lu_solve(int n, int nrhs, double *A, int lda, double *B, int ldb, int *piv, hipStream_t s) {
    if (n > LU_MAXM) return gauss_jordan_solve(n, nrhs, A, lda, B, ldb, nullptr, s);
    hipError_t e;
    for (int k0 = 0; k0 < n; k0 += LU_NB) {
        const int nb = std::min(LU_NB, n - k0), m = n - k0;
        hipLaunchKernelGGL(lu_panel_kernel, dim3(1), dim3(LU_NT), 0, s, m, nb,
                           A + k0 + (long long)k0 * lda, lda, piv + k0);
        hipLaunchKernelGGL(lu_swap_kernel, dim3(nblk(n + nrhs, 256)), dim3(256), 0, s, n, nrhs, k0, nb,
                           (const int *)(piv + k0), A, lda, B, ldb);
        const int ncols = (n - k0 - nb) + nrhs;
        hipLaunchKernelGGL(lu_trsm_lower_kernel, dim3(nblk(ncols, 64)), dim3(64), 0, s, n, nrhs, k0, nb,
                           (const double *)A, lda, A, B, ldb);
        const int mr = n - k0 - nb;
        if (mr > 0) {
            if ((e = gemm(Op::N, Op::N, mr, mr, nb, -1.0, A + (k0 + nb) + (long long)k0 * lda, lda, 0,
                          A + k0 + (long long)(k0 + nb) * lda, lda, 0, 1.0,
                          A + (k0 + nb) + (long long)(k0 + nb) * lda, lda, 0, 1, s)) != hipSuccess)
                return e;
            if ((e = gemm(Op::N, Op::N, mr, nrhs, nb, -1.0, A + (k0 + nb) + (long long)k0 * lda, lda, 0,
                          B + k0, ldb, 0, 1.0, B + (k0 + nb), ldb, 0, 1, s)) != hipSuccess)
                return e;
        }
    }
    const int nblocks = (n + LU_NB - 1) / LU_NB;
    for (int kb = nblocks - 1; kb >= 0; --kb) {
        const int r0 = kb * LU_NB, nb = std::min(LU_NB, n - r0);
        hipLaunchKernelGGL(lu_trsm_upper_kernel, dim3(nblk(nrhs, 64)), dim3(64), 0, s, nrhs, r0, nb,
                           (const double *)A, lda, B, ldb);
        if (r0 > 0 &&
            (e = gemm(Op::N, Op::N, r0, nrhs, nb, -1.0, A + (long long)r0 * lda, lda, 0, B + r0, ldb, 0, 1.0,
                      B, ldb, 0, 1, s)) != hipSuccess)
            return e;
    }
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

// Largest matrix whose eigenvalues are computed in one workgroup's LDS.
constexpr int JAC_LDS_MAX = 128;

// Eigenvalues of a symmetric n x n matrix (n <= JAC_LDS_MAX), one workgroup:
// Householder reduction to tridiagonal form in LDS (lower triangle, textbook
// two-sided update A <- A - v w^T - w v^T with w = p - (beta/2)(v^T p) v,
// p = beta A v, beta = 2 / v^T v), then every eigenvalue by bisection on the
// Sturm sequence count (one thread per eigenvalue, Gershgorin bracket).
__global__ __launch_bounds__(1024) void tridiag_bisect_kernel(int n, const double *Ain, int lda, double *eig) {
    __shared__ double A[JAC_LDS_MAX * (JAC_LDS_MAX + 1)];
    __shared__ double v[JAC_LDS_MAX], p[JAC_LDS_MAX], dd[JAC_LDS_MAX], ee[JAC_LDS_MAX];
    __shared__ double red[1024];
    __shared__ double s_beta, s_alpha, s_k;
    const int t = threadIdx.x;
    const int ld = n + 1;
    for (int idx = t; idx < n * n; idx += 1024) {
        const int i = idx % n, j = idx / n;
        A[i + j * ld] = Ain[i + (long long)j * lda];
    }
    __syncthreads();
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;        // rows k+1 .. n-1
        // ||x||^2, x = A[k+1:, k]
        double sq = 0.0;
        for (int i = t; i < m; i += 1024) { const double x = A[(k + 1 + i) + k * ld]; sq += x * x; }
        red[t] = sq;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if (t < w) red[t] += red[t + w];
            __syncthreads();
        }
        if (t == 0) {
            const double x0 = A[(k + 1) + k * ld];
            const double nrm = sqrt(red[0]);
            const double alpha = x0 >= 0.0 ? -nrm : nrm;
            const double vtv = red[0] - x0 * x0 + (x0 - alpha) * (x0 - alpha);
            s_alpha = alpha;
            s_beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
            dd[k] = A[k + k * ld];
            ee[k] = alpha;
        }
        __syncthreads();
        for (int i = t; i < m; i += 1024) v[i] = A[(k + 1 + i) + k * ld] - (i == 0 ? s_alpha : 0.0);
        __syncthreads();
        const double beta = s_beta;
        // p = beta A22 v: 8 threads per row, then the partial sums
        for (int idx = t; idx < m * 8; idx += 1024) {
            const int i = idx >> 3, part = idx & 7;
            double acc = 0.0;
            for (int j = part; j < m; j += 8) acc += A[(k + 1 + i) + (k + 1 + j) * ld] * v[j];
            red[idx] = acc;
        }
        __syncthreads();
        for (int i = t; i < m; i += 1024) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc += red[i * 8 + q];
            p[i] = beta * acc;
        }
        __syncthreads();
        double vp = 0.0;
        for (int i = t; i < m; i += 1024) vp += v[i] * p[i];
        red[t] = vp;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if (t < w) red[t] += red[t + w];
            __syncthreads();
        }
        if (t == 0) s_k = 0.5 * beta * red[0];
        __syncthreads();
        for (int i = t; i < m; i += 1024) p[i] -= s_k * v[i];      // p <- w
        __syncthreads();
        for (int idx = t; idx < m * m; idx += 1024) {
            const int i = idx % m, j = idx / m;
            A[(k + 1 + i) + (k + 1 + j) * ld] -= v[i] * p[j] + p[i] * v[j];
        }
        __syncthreads();
    }
    if (t == 0) {
        if (n >= 2) {
            dd[n - 2] = A[(n - 2) + (n - 2) * ld];
            ee[n - 2] = A[(n - 1) + (n - 2) * ld];
        }
        dd[n - 1] = A[(n - 1) + (n - 1) * ld];
    }
    __syncthreads();
    // Gershgorin bracket
    double lo = 0.0, hi = 0.0;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(ee[i]) : 0.0);
        lo = i == 0 ? dd[i] - r : fmin(lo, dd[i] - r);
        hi = i == 0 ? dd[i] + r : fmax(hi, dd[i] + r);
    }
    const double scale = fmax(fabs(lo), fabs(hi));
    const double tiny = 1e-300 + 1e-30 * scale;
    for (int idx = t; idx < n; idx += 1024) {
        // the idx-th smallest: count(x) = #{eigenvalues < x}
        double a = lo, b = hi;
        for (int it = 0; it < 200 && b - a > 4e-16 * scale; ++it) {
            const double x = 0.5 * (a + b);
            int cnt = 0;
            double q = dd[0] - x;
            if (q == 0.0) q = -tiny;
            cnt += q < 0.0;
            for (int i = 1; i < n; ++i) {
                q = dd[i] - x - ee[i - 1] * ee[i - 1] / q;
                if (q == 0.0) q = -tiny;
                cnt += q < 0.0;
            }
            if (cnt > idx) b = x; else a = x;
        }
        eig[idx] = 0.5 * (a + b);
    }
}

hipError_t sym_eigvals(int n, double *A, int lda, double *eig, double *work, hipStream_t s) {
    if (n <= JAC_LDS_MAX) {
        hipLaunchKernelGGL(tridiag_bisect_kernel, dim3(1), dim3(1024), 0, s, n, (const double *)A, lda, eig);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(1024), 0, s, n, A, lda, eig, work, 40, 1e-16);
    return hipGetLastError();
}

hipError_t launch_dynmat_assemble(int np, int dim, const double *Phi_el, const double *K_local,
                                  const double *mass, double *D, double *asym2, hipStream_t s) {
    hipLaunchKernelGGL(dynmat_assemble_kernel, dim3(1), dim3(1024), 0, s, np, dim, Phi_el, K_local,
                       mass, D, np, asym2);
    return hipGetLastError();
}

}  // namespace acp
