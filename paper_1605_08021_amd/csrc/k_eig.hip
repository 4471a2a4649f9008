// Symmetric eigenvalues and eigenvectors of a dense FP64 matrix by cyclic
// Jacobi, spread over the whole device: every round of a sweep is one set of
// N/2 disjoint rotations (round-robin tournament ordering, N = n rounded up to
// even, the pair holding the extra position is a bye).  A round is three
// launches: the rotations (one thread per pair, from the current A_pp, A_qq,
// A_pq), the two-sided update A <- J^T A J (one thread per 2 x 2 block of the
// rows of one pair and the columns of another, so that rotations of different
// pairs never touch the same element twice), and V <- V J for the
// eigenvectors.  A sweep ends with one read-back of the number of rotations
// that were still above the threshold; the iteration stops on a sweep without
// any.
//
// Rotation of the pair (p, q): t = sign(theta) / (|theta| + sqrt(theta^2 + 1)),
// theta = (A_qq - A_pp) / (2 A_pq), c = 1 / sqrt(t^2 + 1), s = t c; columns
// A(:, p) <- c A(:, p) - s A(:, q), A(:, q) <- s A(:, p) + c A(:, q), rows the
// same, which zeroes A_pq (Golub and Van Loan, Sec. 8.5).  A pair is rotated
// while |A_pq| exceeds both tol sqrt(|A_pp A_qq|) and tol ||A||_F / sqrt(n).
#include "acp_internal.h"

namespace acp {
namespace {

// Pair k of round r among N positions.
__device__ __forceinline__ void tournament_pair(int k, int r, int N, int &p, int &q) {
    const int a = (k == 0) ? 0 : 1 + (k - 1 + r) % (N - 1);
    const int b = 1 + (N - 2 - k + r) % (N - 1);
    p = a < b ? a : b;
    q = a < b ? b : a;
}

__global__ void jacobi_rotations_kernel(int n, int N, int round, const double *A, int lda, double tol,
                                        const double *fro, double *cs, double *sn, int *pairs,
                                        unsigned *count) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N / 2) return;
    int p, q;
    tournament_pair(k, round, N, p, q);
    double c = 1.0, s = 0.0;
    if (q < n) {
        const double apq = A[p + (long long)q * lda];
        const double app = A[p + (long long)p * lda], aqq = A[q + (long long)q * lda];
        // relative to the pair's diagonal, with a floor tol ||A||_F / sqrt(n) at
        // the level of the rounding that every rotation leaves in its rows and
        // columns (without it, pairs of near-zero eigenvalues rotate forever);
        // the neglected elements change no eigenvalue by more than tol ||A||_F
        if (fabs(apq) > tol * sqrt(fabs(app * aqq)) && fabs(apq) > tol * fro[0] * rsqrt((double)n)) {
            atomicAdd(count, 1u);
            const double theta = (aqq - app) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
        }
    } else {
        q = -1;   // bye: no rotation
    }
    cs[k] = c;
    sn[k] = s;
    pairs[2 * k] = p;
    pairs[2 * k + 1] = q;
}

// Thread (k1, k2): rows {p1, q1} x columns {p2, q2} <- R1 M R2^T with
// R = [c -s; s c] (a bye contributes its single position untouched).
__global__ void jacobi_apply_kernel(int half, double *A, int lda, const double *cs, const double *sn,
                                    const int *pairs) {
    const int k1 = blockIdx.x * blockDim.x + threadIdx.x;
    const int k2 = blockIdx.y;
    if (k1 >= half) return;
    const int p1 = pairs[2 * k1], q1 = pairs[2 * k1 + 1];
    const int p2 = pairs[2 * k2], q2 = pairs[2 * k2 + 1];
    const double c1 = cs[k1], s1 = sn[k1], c2 = cs[k2], s2 = sn[k2];
    if (q1 < 0 && q2 < 0) return;   // byes only: nothing moves
    double *col_p = A + (long long)p2 * lda;
    double m00 = col_p[p1];
    double m10 = q1 >= 0 ? col_p[q1] : 0.0;
    double m01 = 0.0, m11 = 0.0;
    double *col_q = q2 >= 0 ? A + (long long)q2 * lda : nullptr;
    if (col_q) {
        m01 = col_q[p1];
        m11 = q1 >= 0 ? col_q[q1] : 0.0;
    }
    // rows: [r0; r1] = R1 [m0x; m1x]
    const double a00 = c1 * m00 - s1 * m10, a10 = s1 * m00 + c1 * m10;
    const double a01 = c1 * m01 - s1 * m11, a11 = s1 * m01 + c1 * m11;
    // columns: [x0 x1] = [a_x0 a_x1] R2^T
    col_p[p1] = c2 * a00 - s2 * a01;
    if (q1 >= 0) col_p[q1] = c2 * a10 - s2 * a11;
    if (col_q) {
        col_q[p1] = s2 * a00 + c2 * a01;
        if (q1 >= 0) col_q[q1] = s2 * a10 + c2 * a11;
    }
}

// V <- V J: thread (row i, pair k).
__global__ void jacobi_vectors_kernel(int n, double *V, int ldv, const double *cs, const double *sn,
                                      const int *pairs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = blockIdx.y;
    if (i >= n) return;
    const int p = pairs[2 * k], q = pairs[2 * k + 1];
    if (q < 0) return;
    const double c = cs[k], s = sn[k];
    double *vp = V + (long long)p * ldv + i, *vq = V + (long long)q * ldv + i;
    const double a = *vp, b = *vq;
    *vp = c * a - s * b;
    *vq = s * a + c * b;
}

// Frobenius norm (partial sums per block, then one block in a fixed order).
__global__ void frob_partial_kernel(int n, const double *A, int lda, double *part) {
    __shared__ double red[256];
    double acc = 0.0;
    for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < (long long)n * n;
         idx += (long long)gridDim.x * 256) {
        const double v = A[(idx % n) + (idx / n) * lda];
        acc += v * v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void frob_final_kernel(int nparts, const double *part, double *out) {
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int i = 0; i < nparts; ++i) acc += part[i];
        out[0] = sqrt(acc);
    }
}

__global__ void identity_kernel(int n, double *V, int ldv) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * n) return;
    const int i = (int)(idx % n), j = (int)(idx / n);
    V[i + (long long)j * ldv] = (i == j) ? 1.0 : 0.0;
}

// eig ascending (ties by index) from the diagonal; perm[rank] = index.
__global__ void diag_rank_kernel(int n, const double *A, int lda, double *eig, int *perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = A[i + (long long)i * lda];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
        const double u = A[j + (long long)j * lda];
        rank += (u < v || (u == v && j < i));
    }
    eig[rank] = v;
    perm[rank] = i;
}

__global__ void permute_cols_kernel(int n, const double *W, int ldw, const int *perm, double *V, int ldv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= n) return;
    V[i + (long long)j * ldv] = W[i + (long long)perm[j] * ldw];
}

}  // namespace

size_t sym_eig_work_doubles(int n, bool vectors) {
    const size_t N = (size_t)n + (n & 1);
    // cs, sn (N/2 each), pairs (N ints), perm (n ints), counter, norm partials (257), [W n x n]
    return N + (N + n + 2) / 2 + 2 + 257 + (vectors ? (size_t)n * n : 0);
}

hipError_t sym_eig_jacobi(int n, double *A, int lda, double *eig, double *V, int ldv, double *work,
                          int max_sweeps, double tol, hipStream_t s, int *sweeps_out) {
    if (n < 1) return hipSuccess;
    const int N = n + (n & 1), half = N / 2;
    double *cs = work, *sn = work + half;
    int *pairs = (int *)(work + N);
    int *perm = pairs + N;
    unsigned *count = (unsigned *)(perm + n);
    double *fro = work + N + (N + n + 2) / 2 + 2;   // [0]: the norm, [1..256]: partials
    double *W = V ? fro + 257 : nullptr;
    hipError_t e;
    hipLaunchKernelGGL(frob_partial_kernel, dim3(256), dim3(256), 0, s, n, (const double *)A, lda, fro + 1);
    hipLaunchKernelGGL(frob_final_kernel, dim3(1), dim3(64), 0, s, 256, (const double *)(fro + 1), fro);
    if (W) {
        hipLaunchKernelGGL(identity_kernel, dim3((unsigned)(((long long)n * n + 255) / 256)), dim3(256), 0, s,
                           n, W, n);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        if ((e = hipMemsetAsync(count, 0, sizeof(unsigned), s)) != hipSuccess) return e;
        for (int r = 0; r < N - 1; ++r) {
            hipLaunchKernelGGL(jacobi_rotations_kernel, dim3((half + 255) / 256), dim3(256), 0, s, n, N, r,
                               (const double *)A, lda, tol, (const double *)fro, cs, sn, pairs, count);
            hipLaunchKernelGGL(jacobi_apply_kernel, dim3((half + 255) / 256, half), dim3(256), 0, s, half, A,
                               lda, (const double *)cs, (const double *)sn, (const int *)pairs);
            if (W)
                hipLaunchKernelGGL(jacobi_vectors_kernel, dim3((n + 255) / 256, half), dim3(256), 0, s, n, W, n,
                                   (const double *)cs, (const double *)sn, (const int *)pairs);
        }
        unsigned h = 0;
        if ((e = hipMemcpyAsync(&h, count, sizeof(unsigned), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        if (h == 0) {
            ++sweep;
            break;
        }
    }
    if (sweeps_out) *sweeps_out = sweep;
    hipLaunchKernelGGL(diag_rank_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, (const double *)A, lda, eig,
                       perm);
    if (W)
        hipLaunchKernelGGL(permute_cols_kernel, dim3((n + 255) / 256, n), dim3(256), 0, s, n, (const double *)W, n,
                           (const int *)perm, V, ldv);
    return hipGetLastError();
}

}  // namespace acp
