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
// Dense algebra: a blocked LU with partial pivoting for the N_mu x N_mu system
// of the Sherman-Morrison-Woodbury update (Eq. (3.13); Gauss-Jordan above 1024
// unknowns), the blocked inverse of the triangular factor L11, Householder
// tridiagonalisation with Sturm bisection for the eigenvalues of the dynamical
// matrix (in one workgroup up to 128, over the device above), and the assembly
// D = M^{-1/2} (sym(h^d G^T U) + K_local) M^{-1/2}.
#include "acp_internal.h"

namespace acp {
namespace {

inline unsigned nblk(long long tot, int b) { return (unsigned)((tot + b - 1) / b); }

// One step of a wave-wide argmax (largest value, ties to the smallest index)
// with the partner lane chosen by a DPP control; lanes outside row_mask keep
// their own pair.
template <int CTRL, int ROWM>
__device__ __forceinline__ void argmax_dpp_step(double &v, int &i) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, ROWM, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, ROWM, 0xf, false);
    const int oi = __builtin_amdgcn_update_dpp(i, i, CTRL, ROWM, 0xf, false);
    const double ov = __hiloint2double(hi, lo);
    if (ov > v || (ov == v && oi < i)) {
        v = ov;
        i = oi;
    }
}

// Wave argmax, valid in lane 63: pairs within quads (quad_perm 1,0,3,2 and
// 2,3,0,1), half rows (row_half_mirror), rows (row_mirror), then rows 0-1 and
// 2-3 (row_bcast:15) and all four (row_bcast:31).
__device__ __forceinline__ void wave_argmax(double &v, int &i) {
    argmax_dpp_step<0xB1, 0xf>(v, i);
    argmax_dpp_step<0x4E, 0xf>(v, i);
    argmax_dpp_step<0x141, 0xf>(v, i);
    argmax_dpp_step<0x140, 0xf>(v, i);
    argmax_dpp_step<0x142, 0xa>(v, i);
    argmax_dpp_step<0x143, 0xc>(v, i);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}


// The ISDF kernels read column-major data with leading dimension N_g: Phi
// (N_g x n_e), G~ (N_g x r) and the factor L (N_g x N_mu; step k writes column
// k), so that 16 consecutive grid rows of one column form one 128-byte segment.
// A block owns 16 grid rows; its 512 threads form 32 streams of 16 lanes, and
// stream s takes the columns s, s + 32, ... of each of the three dot products
// of a step, summed over the streams afterwards in a fixed order.  The pivot
// row's entries are staged in LDS.  Each block leaves its best remaining
// diagonal entry as a candidate (value, row); every block of the next step
// reduces the candidates itself, so one launch per pivot suffices.  Block b
// owns the same rows at every step, so it re-reads its slice of Phi, G~ and L
// on the same XCD.
constexpr int ISDF_NT = 512;
constexpr int ISDF_ROWS = 16;
constexpr int ISDF_NS = ISDF_NT / ISDF_ROWS;   // column streams per block
constexpr int ISDF_VCH = 4096;                 // pivot-row entries staged per pass

struct Cand {
    double v;
    int i;
    int pad;
};

__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
    return v > bv || (v == bv && i < bi);
}

// Candidates of the previous step, 8 per thread and pass (thread pos of
// `stride` threads takes b0 + pos + stride i): a pass issues all its loads
// before any comparison (one memory round trip), and the comparisons can wait
// until other independent loads are in flight.  The order of comparisons does
// not matter: better() is a total order.
struct CandPass {
    static constexpr int CPL = 8;
    double v[CPL];
    int ix[CPL];
    __device__ __forceinline__ void load(const Cand *cand, int n, int b0, int pos, int stride) {
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
            const int b = b0 + pos + stride * i;
            const Cand c = cand[b < n ? b : n - 1];
            v[i] = c.v;
            ix[i] = c.i;
        }
    }
    __device__ __forceinline__ void reduce(int n, int b0, int pos, int stride, double &bv, int &bi) const {
#pragma unroll
        for (int i = 0; i < CPL; ++i)
            if (b0 + pos + stride * i < n && better(v[i], ix[i], bv, bi)) {
                bv = v[i];
                bi = ix[i];
            }
    }
};

// This lane's best (value, row) over cand[0..n); the caller reduces across the wave.
__device__ __forceinline__ void lane_best_candidate(const Cand *cand, int n, double &bv, int &bi) {
    CandPass cp;
    const int lane = threadIdx.x & 63;
    for (int b0 = 0; b0 < n; b0 += 64 * CandPass::CPL) {
        cp.load(cand, n, b0, lane, 64);
        cp.reduce(n, b0, lane, 64, bv, bi);
    }
}

// Best (value, row) over threads 0..15 (the block's rows); thread 0 writes it.
__device__ __forceinline__ void block_candidate16(double v, int i, Cand *out) {
    if (threadIdx.x < 64) {
#pragma unroll
        for (int m = 8; m > 0; m >>= 1) {
            const double ov = __shfl_xor(v, m, 16);
            const int oi = __shfl_xor(i, m, 16);
            if (better(ov, oi, v, i)) {
                v = ov;
                i = oi;
            }
        }
        if (threadIdx.x == 0) {
            out[blockIdx.x].v = v;
            out[blockIdx.x].i = i;
        }
    }
}

// sum_j col0[j ng] v[j] over this stream's columns j = st, st + 32, ... < n
// (four independent accumulators, combined in a fixed order).
__device__ __forceinline__ double stream_dot(const double *col0, int ng, const double *v, int n, int st) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int j = st;
    for (; j + 3 * ISDF_NS < n; j += 4 * ISDF_NS) {
        a0 += col0[(long long)j * ng] * v[j];
        a1 += col0[(long long)(j + ISDF_NS) * ng] * v[j + ISDF_NS];
        a2 += col0[(long long)(j + 2 * ISDF_NS) * ng] * v[j + 2 * ISDF_NS];
        a3 += col0[(long long)(j + 3 * ISDF_NS) * ng] * v[j + 3 * ISDF_NS];
    }
    for (; j < n; j += ISDF_NS) a0 += col0[(long long)j * ng] * v[j];
    return (a0 + a1) + (a2 + a3);
}

// Row a's dot product with row p over the n columns of M (column-major, ld ng),
// this stream's share: the pivot row is staged in LDS ISDF_VCH entries at a time.
__device__ double stream_row_dot(const double *M, int ng, int n, int p, long long a, int st, double *vp) {
    double acc = 0.0;
    for (int c0 = 0; c0 < n; c0 += ISDF_VCH) {
        const int cn = min(ISDF_VCH, n - c0);
        __syncthreads();
        for (int j = threadIdx.x; j < cn; j += ISDF_NT) vp[j] = M[p + (long long)(c0 + j) * ng];
        __syncthreads();
        acc += stream_dot(M + a + (long long)c0 * ng, ng, vp, cn, st);
    }
    return acc;
}

// diag(alpha) = |phi(alpha,:)|^2 |G~(alpha,:)|^2 and the first candidates.
__global__ __launch_bounds__(ISDF_NT) void isdf_init_kernel(int ng, int ne, int r, const double *phi,
                                                            const double *gt, double *diag, Cand *cand) {
    __shared__ double red[2][ISDF_NT];
    const int t = threadIdx.x, st = t / ISDF_ROWS;
    const int a = blockIdx.x * ISDF_ROWS + t % ISDF_ROWS;
    const long long ac = a < ng ? a : ng - 1;
    double s1 = 0.0, s2 = 0.0;
    for (int i = st; i < ne; i += ISDF_NS) {
        const double v = phi[ac + (long long)i * ng];
        s1 += v * v;
    }
    for (int j = st; j < r; j += ISDF_NS) {
        const double v = gt[ac + (long long)j * ng];
        s2 += v * v;
    }
    red[0][t] = s1;
    red[1][t] = s2;
    __syncthreads();
    double d = -2.0;
    int idx = 0x7fffffff;
    if (t < ISDF_ROWS) {
        double a1 = 0.0, a2 = 0.0;
        for (int k = 0; k < ISDF_NS; ++k) {
            a1 += red[0][k * ISDF_ROWS + t];
            a2 += red[1][k * ISDF_ROWS + t];
        }
        if (a < ng) {
            d = a1 * a2;
            diag[a] = d;
            idx = a;
        }
    }
    block_candidate16(d, idx, cand);
}

// Step k of the greedy pivoted Cholesky of K = (Phi Phi^T) o (G~ G~^T):
//   p = argmax diag (ties -> smallest index), or forced[k];
//   L(a,k) = (K(a,p) - sum_{j<k} L(a,j) L(p,j)) / sqrt(diag(p)), diag(a) -= L(a,k)^2.
// state[0] = accepted pivots, state[1] = stopped; dvals[0] = first pivot value.
__global__ __launch_bounds__(ISDF_NT) void isdf_step_kernel(
    int ng, int ne, int r, int k, int nblk, const double *phi, const double *pgram, const double *gt,
    double *L, double *diag, int *sel, const int *forced, double tol2, int *state, double *dvals,
    const Cand *cand_in, Cand *cand_out) {
    __shared__ double vp[ISDF_VCH];
    __shared__ double red[3][ISDF_NT];
    const int t = threadIdx.x;
    if (state[1]) return;   // stopped at an earlier step
    // the pivot: every wave reduces the previous step's candidates itself
    // (same order in every wave, so every thread holds the same pivot)
    double bv = -2.0;
    int bi = 0x7fffffff;
    if (forced) {
        bi = forced[k];
        bv = diag[bi];
    } else {
        lane_best_candidate(cand_in, nblk, bv, bi);
        wave_argmax(bv, bi);
        bv = readlane_f64(bv, 63);
        bi = __builtin_amdgcn_readlane(bi, 63);
    }
    const bool stop = !(bv > 0.0) || (!forced && tol2 > 0.0 && k > 0 && bv < tol2 * dvals[0]);
    if (blockIdx.x == 0 && t == 0) {
        if (stop) {
            state[1] = 1;
        } else {
            sel[k] = bi;
            state[0] = k + 1;
            if (k == 0) dvals[0] = bv;
        }
    }
    if (stop) return;
    const int p = bi;
    const int st = t / ISDF_ROWS;
    const int a = blockIdx.x * ISDF_ROWS + t % ISDF_ROWS;
    const long long ac = a < ng ? a : ng - 1;
    // with the Gram matrix Phi Phi^T at hand, phi(a,:).phi(p,:) is one entry of its column p
    if (pgram) ne = 0;
    if (ne + r + k <= ISDF_VCH) {
        // one staging pass: vp = [phi(p,:) | G~(p,:) | L(p, 0..k-1)]
        for (int j = t; j < ne + r + k; j += ISDF_NT) {
            const double *src = j < ne ? phi + (long long)j * ng
                                : j < ne + r ? gt + (long long)(j - ne) * ng
                                             : L + (long long)(j - ne - r) * ng;
            vp[j] = src[p];
        }
        __syncthreads();
        red[0][t] = stream_dot(phi + ac, ng, vp, ne, st);
        red[1][t] = stream_dot(gt + ac, ng, vp + ne, r, st);
        red[2][t] = stream_dot(L + ac, ng, vp + ne + r, k, st);
    } else {
        red[0][t] = stream_row_dot(phi, ng, ne, p, ac, st, vp);
        red[1][t] = stream_row_dot(gt, ng, r, p, ac, st, vp);
        red[2][t] = stream_row_dot(L, ng, k, p, ac, st, vp);
    }
    __syncthreads();
    double dnew = -2.0;
    int idx = 0x7fffffff;
    if (t < ISDF_ROWS && a < ng) {
        double s1 = 0.0, s2 = 0.0, y = 0.0;
        for (int q = 0; q < ISDF_NS; ++q) {
            s1 += red[0][q * ISDF_ROWS + t];
            s2 += red[1][q * ISDF_ROWS + t];
            y += red[2][q * ISDF_ROWS + t];
        }
        if (pgram) s1 = pgram[a + (long long)p * ng];
        const double lk = (s1 * s2 - y) / sqrt(bv);
        dnew = (a == p) ? -1.0 : diag[a] - lk * lk;
        L[a + (long long)k * ng] = lk;
        diag[a] = dnew;
        idx = a;
    }
    block_candidate16(dnew, idx, cand_out);
}

// The greedy step with Phi Phi^T at hand and this thread's share of its row in
// registers.  The loads are ordered by need: the previous step's candidates
// first, then the virtual columns v = st + 32 i (i < MAXR) of [G~ | L(:, 0..k-1)]
// (independent of the pivot, in flight during the candidate reduction), then,
// once the pivot p is known, its row (staged in LDS) and Phi Phi^T(a, p).  The
// launch picks the smallest MAXR with r + k <= 32 MAXR.
template <int MAXR>
__global__ __launch_bounds__(ISDF_NT) void isdf_step_gram_kernel(
    int ng, int r, int k, int nblk, const double *pgram, const double *gt, double *L, double *diag,
    int *sel, double tol2, int *state, double *dvals, const Cand *cand_in, Cand *cand_out) {
    constexpr int NV = ISDF_NS * MAXR;
    __shared__ double vp[NV];
    __shared__ double red[2][ISDF_NT];
    const int t = threadIdx.x;
    const int st = t / ISDF_ROWS;
    const int a = blockIdx.x * ISDF_ROWS + t % ISDF_ROWS;
    const long long ac = a < ng ? a : ng - 1;
    const int ntot = r + k;
    const int stopped = state[1];
    __shared__ double s_cv[ISDF_NT / 64];
    __shared__ int s_ci[ISDF_NT / 64];
    double bv = -2.0;
    int bi = 0x7fffffff;
    // up to 512 candidates every wave reads them all in one pass (no barrier);
    // beyond, the block shares them out (thread t takes t, t + 512, ...: one
    // pass up to 4096, each read once per block) and the waves' winners meet
    // in LDS
    const bool shared = nblk > 64 * CandPass::CPL;   // uniform over the launch
    const int pos = shared ? t : (t & 63), stride = shared ? ISDF_NT : 64;
    CandPass cp;
    cp.load(cand_in, nblk, 0, pos, stride);
    auto column = [&](int v) -> const double * {
        return v < r ? gt + (long long)v * ng : v < ntot ? L + (long long)(v - r) * ng : gt;
    };
    double x[MAXR];
#pragma unroll
    for (int i = 0; i < MAXR; ++i) x[i] = column(st + ISDF_NS * i)[ac];
    const double dold = diag[ac];
    cp.reduce(nblk, 0, pos, stride, bv, bi);
    for (int b0 = stride * CandPass::CPL; b0 < nblk; b0 += stride * CandPass::CPL) {
        cp.load(cand_in, nblk, b0, pos, stride);
        cp.reduce(nblk, b0, pos, stride, bv, bi);
    }
    if (stopped) return;
    wave_argmax(bv, bi);
    if (shared) {
        if ((t & 63) == 63) {
            s_cv[t >> 6] = bv;
            s_ci[t >> 6] = bi;
        }
        __syncthreads();
        bv = (t & 63) < ISDF_NT / 64 ? s_cv[t & 63] : -2.0;
        bi = (t & 63) < ISDF_NT / 64 ? s_ci[t & 63] : 0x7fffffff;
        wave_argmax(bv, bi);
    }
    bv = readlane_f64(bv, 63);
    bi = __builtin_amdgcn_readlane(bi, 63);
    const bool stop = !(bv > 0.0) || (tol2 > 0.0 && k > 0 && bv < tol2 * dvals[0]);
    if (blockIdx.x == 0 && t == 0) {
        if (stop) {
            state[1] = 1;
        } else {
            sel[k] = bi;
            state[0] = k + 1;
            if (k == 0) dvals[0] = bv;
        }
    }
    if (stop) return;
    const int p = bi;
    const double kp = pgram[ac + (long long)p * ng];
    for (int v = t; v < NV; v += ISDF_NT) vp[v] = v < ntot ? column(v)[p] : 0.0;
    __syncthreads();
    double s2 = 0.0, y = 0.0;
#pragma unroll
    for (int i = 0; i < MAXR; ++i) {
        const int v = st + ISDF_NS * i;
        const double pr = x[i] * vp[v];
        s2 += v < r ? pr : 0.0;
        y += v >= r ? pr : 0.0;
    }
    red[0][t] = s2;
    red[1][t] = y;
    __syncthreads();
    double dnew = -2.0;
    int idx = 0x7fffffff;
    if (t < ISDF_ROWS && a < ng) {
        double a2 = 0.0, a3 = 0.0;
        for (int q = 0; q < ISDF_NS; ++q) {
            a2 += red[0][q * ISDF_ROWS + t];
            a3 += red[1][q * ISDF_ROWS + t];
        }
        const double lk = (kp * a2 - a3) / sqrt(bv);
        dnew = (a == p) ? -1.0 : dold - lk * lk;
        L[a + (long long)k * ng] = lk;
        diag[a] = dnew;
        idx = a;
    }
    block_candidate16(dnew, idx, cand_out);
}

// X (n2 x n2, column-major) = [L11 0; 0 I] with L11(i, j) = L(sel[i], j) for
// j <= i and 0 above the diagonal (L column-major, leading dimension ng).
__global__ void gather_l11_kernel(int n, int n2, const int *sel, const double *L, int ng, double *X) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n2 * n2) return;
    const int i = (int)(idx % n2);
    const int j = (int)(idx / n2);
    double v;
    if (i < n && j < n) v = (j <= i) ? L[sel[i] + (long long)j * ng] : 0.0;
    else v = (i == j) ? 1.0 : 0.0;
    X[idx] = v;
}

// In place inverse of every 32 x 32 lower-triangular diagonal block of X
// (one workgroup per block, one thread per column, forward substitution in LDS).
constexpr int TRI_B = 32;
__global__ __launch_bounds__(TRI_B) void tri_diag_inverse_kernel(int n2, double *X) {
    __shared__ double A[TRI_B][TRI_B + 1];
    const int c = threadIdx.x;
    double *blk = X + (long long)blockIdx.x * TRI_B * (n2 + 1);
    for (int i = 0; i < TRI_B; ++i) A[i][c] = blk[i + (long long)c * n2];
    __syncthreads();
    double x[TRI_B];
#pragma unroll
    for (int i = 0; i < TRI_B; ++i) {
        double sacc = (i == c) ? 1.0 : 0.0;
#pragma unroll
        for (int l = 0; l < i; ++l) sacc -= A[i][l] * x[l];
        x[i] = (i < c) ? 0.0 : sacc / A[i][i];
    }
#pragma unroll
    for (int i = 0; i < TRI_B; ++i) blk[i + (long long)c * n2] = x[i];
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

hipError_t isdf_pivoted_cholesky(int ng, int ne, int r, const double *phi, const double *pgram,
                                 const double *gt, int nmu_max, double tol, double *L, double *diag,
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
    hipLaunchKernelGGL(isdf_init_kernel, dim3(nblk), dim3(ISDF_NT), 0, s, ng, ne, r, phi, gt, diag, c0);
    const double tol2 = tol * tol;
    for (int k = 0; k < nmu_max; ++k) {
        const Cand *cin = (k & 1) ? c1 : c0;
        Cand *cout = (k & 1) ? c0 : c1;
        if (pgram && !forced) {
            const int nreg = (r + k + ISDF_NS - 1) / ISDF_NS;
#define ISDF_GRAM(M)                                                                                     \
    if (nreg <= M) {                                                                                     \
        hipLaunchKernelGGL(isdf_step_gram_kernel<M>, dim3(nblk), dim3(ISDF_NT), 0, s, ng, r, k, nblk, pgram, \
                           gt, L, diag, sel_dev, tol2, state, dvals, cin, cout);                         \
        continue;                                                                                        \
    }
            ISDF_GRAM(2) ISDF_GRAM(4) ISDF_GRAM(6) ISDF_GRAM(8) ISDF_GRAM(10) ISDF_GRAM(12) ISDF_GRAM(14)
            ISDF_GRAM(16) ISDF_GRAM(18) ISDF_GRAM(20) ISDF_GRAM(24) ISDF_GRAM(28) ISDF_GRAM(32)
#undef ISDF_GRAM
        }
        hipLaunchKernelGGL(isdf_step_kernel, dim3(nblk), dim3(ISDF_NT), 0, s, ng, ne, r, k, nblk, phi,
                           forced ? nullptr : pgram, gt, L, diag, sel_dev, forced, tol2, state, dvals, cin, cout);
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

int tri_inverse_order(int n) {
    int n2 = TRI_B;
    while (n2 < n) n2 *= 2;
    return n2;
}

// Inverse of a lower-triangular matrix by blocks: the 32 x 32 diagonal blocks
// are inverted directly, then pairs of inverted blocks are joined level by level,
//     [A 0; B C]^{-1} = [A^{-1} 0; -C^{-1} B A^{-1}  C^{-1}],
// two batched GEMMs per level (T = B A^{-1}, then B <- -C^{-1} T).
hipError_t launch_isdf_l11_inverse(int n, const int *sel, const double *L, int ng, double *X, double *T,
                                   hipStream_t s) {
    const int n2 = tri_inverse_order(n);
    const long long tot = (long long)n2 * n2;
    hipLaunchKernelGGL(gather_l11_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, n, n2, sel, L, ng, X);
    hipLaunchKernelGGL(tri_diag_inverse_kernel, dim3(n2 / TRI_B), dim3(TRI_B), 0, s, n2, X);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int sz = 2 * TRI_B; sz <= n2; sz *= 2) {
        const int h = sz / 2, np = n2 / sz;
        const long long sd = (long long)sz * (n2 + 1), st = (long long)h * h;
        if ((e = gemm(Op::N, Op::N, h, h, h, 1.0, X + h, n2, sd, X, n2, sd, 0.0, T, h, st, np, s)) !=
            hipSuccess)
            return e;
        if ((e = gemm(Op::N, Op::N, h, h, h, -1.0, X + h + (long long)h * n2, n2, sd, T, h, st, 0.0, X + h,
                      n2, sd, np, s)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------ blocked LU solve
// A X = B by a right-looking blocked LU with partial pivoting applied to the
// augmented [A | B] (A n x n, B n x nrhs, column-major, in place): panels of
// LU_NB columns are factored by one workgroup that keeps one panel row per
// thread in registers; the panel's row permutation is applied to the columns
// right of it (and to B) together with the solve by its unit lower triangle,
// and the trailing matrix and B are updated by a GEMM on the matrix cores.
// Columns left of a panel are not permuted: B is eliminated along with A, so
// the multipliers of earlier panels are never used again.  Back substitution
// then proceeds by blocks of LU_NB rows (U does not depend on where the panels
// began).  Panels of more than LU_MAXM rows go through lu_panel_tall_kernel.
constexpr int LU_NB = 32;
constexpr int LU_MAXM = 1024;     // panel rows, one per thread
constexpr int LU_NT = 1024;
// Per-panel permutation record: position i < LU_NB of the permuted panel rows
// holds original row top[i]; ndisp rows at or below LU_NB receive another row:
// row dst[e] <- original row src[e] (panel-relative indices).
constexpr int LU_PI_TOP = 0, LU_PI_ND = LU_NB, LU_PI_DST = LU_NB + 1, LU_PI_SRC = 2 * LU_NB + 1;
constexpr int LU_PINFO = 4 * LU_NB;

struct LuPanelShared {
    double rows[2][2][LU_NB];   // [parity][row j | pivot row]
    double wv[2][LU_NT / 64];
    int wi[2][LU_NT / 64];
    int idx[LU_MAXM];           // original row at each position of the permuted panel
    int nd;
};

// Column J of the panel (static J, so the row stays in registers); the block
// has nw waves.
template <int J>
__device__ __forceinline__ void lu_panel_column(double (&P)[LU_NB], LuPanelShared &sh, int nb, bool own, int nw) {
    if constexpr (J < LU_NB) {
        const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
        if (J < nb) {
            constexpr int par = J & 1;
            // pivot: largest |P[r][J]|, r >= J, ties to the smallest row
            double bv = -1.0;
            int bi = 0x7fffffff;
            if (own && t >= J) {
                bv = fabs(P[J]);
                bi = t;
            }
            wave_argmax(bv, bi);
            if (lane == 63) {
                sh.wv[par][wave] = bv;
                sh.wi[par][wave] = bi;
            }
            __syncthreads();
            // every wave reduces the per-wave winners itself, one per lane
            double b = lane < nw ? sh.wv[par][lane] : -2.0;
            int p = lane < nw ? sh.wi[par][lane] : 0x7fffffff;
            wave_argmax(b, p);
            p = __builtin_amdgcn_readlane(p, 63);
            if (t == J) {
#pragma unroll
                for (int c = 0; c < LU_NB; ++c) sh.rows[par][0][c] = P[c];
            }
            if (t == p) {
#pragma unroll
                for (int c = 0; c < LU_NB; ++c) sh.rows[par][1][c] = P[c];
            }
            if (t == 0) {
                const int a = sh.idx[J];
                sh.idx[J] = sh.idx[p];
                sh.idx[p] = a;
            }
            __syncthreads();
            if (p != J) {
                if (t == J) {
#pragma unroll
                    for (int c = 0; c < LU_NB; ++c) P[c] = sh.rows[par][1][c];
                } else if (t == p) {
#pragma unroll
                    for (int c = 0; c < LU_NB; ++c) P[c] = sh.rows[par][0][c];
                }
            }
            if (own && t > J) {
                const double l = P[J] / sh.rows[par][1][J];
                P[J] = l;
#pragma unroll
                for (int c = J + 1; c < LU_NB; ++c) P[c] -= l * sh.rows[par][1][c];
            }
        }
        lu_panel_column<J + 1>(P, sh, nb, own, nw);
    }
}

__global__ __launch_bounds__(LU_NT) void lu_panel_kernel(int m, int nb, double *A, int lda, int *pinfo) {
    __shared__ LuPanelShared sh;
    const int t = threadIdx.x;
    const bool own = t < m;
    double P[LU_NB];
#pragma unroll
    for (int c = 0; c < LU_NB; ++c) P[c] = (own && c < nb) ? A[t + (long long)c * lda] : 0.0;
    if (own) sh.idx[t] = t;
    if (t == 0) sh.nd = 0;
    __syncthreads();
    lu_panel_column<0>(P, sh, nb, own, (int)(blockDim.x >> 6));
#pragma unroll
    for (int c = 0; c < LU_NB; ++c)
        if (own && c < nb) A[t + (long long)c * lda] = P[c];
    __syncthreads();
    if (t < nb) pinfo[LU_PI_TOP + t] = sh.idx[t];
    if (own && t >= nb && sh.idx[t] != t) {
        const int e = atomicAdd(&sh.nd, 1);   // at most nb displaced rows
        pinfo[LU_PI_DST + e] = t;
        pinfo[LU_PI_SRC + e] = sh.idx[t];
    }
    __syncthreads();
    if (t == 0) pinfo[LU_PI_ND] = sh.nd;
}

// Panels of more than LU_MAXM rows (up to LU_TALL_MAXM): LU_TALL_NB columns,
// each thread keeping the LU_TALL_R rows t, t + LU_NT, ... in registers; the
// same pivot rule (largest magnitude, ties to the smallest row) and the same
// permutation record as lu_panel_kernel.  Launched with LU_NT threads.
constexpr int LU_TALL_NB = 8;
constexpr int LU_TALL_R = 4;
constexpr int LU_TALL_MAXM = LU_TALL_R * LU_NT;

struct LuTallShared {
    double rows[2][2][LU_TALL_NB];   // [parity][row J | pivot row]
    double wv[2][LU_NT / 64];
    int wi[2][LU_NT / 64];
    int idx[LU_TALL_MAXM];
    int nd;
};

__global__ __launch_bounds__(LU_NT) void lu_panel_tall_kernel(int m, int nb, double *A, int lda, int *pinfo) {
    __shared__ LuTallShared sh;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int nw = LU_NT / 64;
    double P[LU_TALL_R][LU_TALL_NB];
#pragma unroll
    for (int r = 0; r < LU_TALL_R; ++r) {
        const int i = t + LU_NT * r;
#pragma unroll
        for (int c = 0; c < LU_TALL_NB; ++c) P[r][c] = (i < m && c < nb) ? A[i + (long long)c * lda] : 0.0;
    }
    for (int i = t; i < m; i += LU_NT) sh.idx[i] = i;
    if (t == 0) sh.nd = 0;
    __syncthreads();
#pragma unroll
    for (int J = 0; J < LU_TALL_NB; ++J) {
        if (J < nb) {
            const int par = J & 1;
            double bv = -1.0;
            int bi = 0x7fffffff;
#pragma unroll
            for (int r = 0; r < LU_TALL_R; ++r) {
                const int i = t + LU_NT * r;
                if (i < m && i >= J && fabs(P[r][J]) > bv) {
                    bv = fabs(P[r][J]);
                    bi = i;
                }
            }
            wave_argmax(bv, bi);
            if (lane == 63) {
                sh.wv[par][wave] = bv;
                sh.wi[par][wave] = bi;
            }
            __syncthreads();
            double b = lane < nw ? sh.wv[par][lane] : -2.0;
            int p = lane < nw ? sh.wi[par][lane] : 0x7fffffff;
            wave_argmax(b, p);
            p = __builtin_amdgcn_readlane(p, 63);
            if (p >= m) p = J;   // no comparable entry (NaN column): no exchange
            const int pt = p % LU_NT, pr = p / LU_NT;
            if (t == J) {   // row J < LU_TALL_NB is slot 0 of thread J
#pragma unroll
                for (int c = 0; c < LU_TALL_NB; ++c) sh.rows[par][0][c] = P[0][c];
            }
            if (t == pt) {
#pragma unroll
                for (int r = 0; r < LU_TALL_R; ++r)
                    if (r == pr) {
#pragma unroll
                        for (int c = 0; c < LU_TALL_NB; ++c) sh.rows[par][1][c] = P[r][c];
                    }
            }
            if (t == 0) {
                const int a = sh.idx[J];
                sh.idx[J] = sh.idx[p];
                sh.idx[p] = a;
            }
            __syncthreads();
            if (p != J) {
                if (t == J) {
#pragma unroll
                    for (int c = 0; c < LU_TALL_NB; ++c) P[0][c] = sh.rows[par][1][c];
                }
                if (t == pt) {
#pragma unroll
                    for (int r = 0; r < LU_TALL_R; ++r)
                        if (r == pr) {
#pragma unroll
                            for (int c = 0; c < LU_TALL_NB; ++c) P[r][c] = sh.rows[par][0][c];
                        }
                }
            }
            const double piv = sh.rows[par][1][J];
#pragma unroll
            for (int r = 0; r < LU_TALL_R; ++r) {
                const int i = t + LU_NT * r;
                if (i < m && i > J) {
                    const double l = P[r][J] / piv;
                    P[r][J] = l;
#pragma unroll
                    for (int c = J + 1; c < LU_TALL_NB; ++c) P[r][c] -= l * sh.rows[par][1][c];
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < LU_TALL_R; ++r) {
        const int i = t + LU_NT * r;
#pragma unroll
        for (int c = 0; c < LU_TALL_NB; ++c)
            if (i < m && c < nb) A[i + (long long)c * lda] = P[r][c];
    }
    __syncthreads();
    if (t < nb) pinfo[LU_PI_TOP + t] = sh.idx[t];
    for (int i = t; i < m; i += LU_NT)
        if (i >= nb && sh.idx[i] != i) {
            const int e = atomicAdd(&sh.nd, 1);   // at most nb displaced rows
            pinfo[LU_PI_DST + e] = i;
            pinfo[LU_PI_SRC + e] = sh.idx[i];
        }
    __syncthreads();
    if (t == 0) pinfo[LU_PI_ND] = sh.nd;
}

// col[0..nb) = x[0..nb) for nb <= LU_NB; a partial block goes through the
// caller's LDS staging area (one column per thread).
__device__ __forceinline__ void store_block(double *col, const double (&x)[LU_NB], int nb,
                                            double (*stage)[64]) {
    if (nb == LU_NB) {
#pragma unroll
        for (int i = 0; i < LU_NB; ++i) col[i] = x[i];
    } else {
#pragma unroll
        for (int i = 0; i < LU_NB; ++i) stage[i][threadIdx.x] = x[i];
        for (int i = 0; i < nb; ++i) col[i] = stage[i][threadIdx.x];
    }
}

// Block row k0 for every column right of the panel and for B: the panel's row
// permutation, then X = L11^{-1} X (L11 unit lower, staged in LDS).  One thread
// per column; every read of a column precedes every write to it (displaced
// rows pass through LDS).
__global__ __launch_bounds__(64) void lu_rowblock_kernel(int n, int nrhs, int k0, int nb, double *A, int lda,
                                                         double *B, int ldb, const int *pinfo) {
    __shared__ double L[LU_NB][LU_NB + 1];
    __shared__ double dv[LU_NB][64];
    __shared__ int pi[LU_PINFO];
    for (int i = threadIdx.x; i < LU_NB * LU_NB; i += 64) {
        const int r = i % LU_NB, c = i / LU_NB;
        L[r][c] = (r < nb && c < r) ? A[(k0 + r) + (long long)(k0 + c) * lda] : 0.0;
    }
    for (int i = threadIdx.x; i < LU_PINFO; i += 64) pi[i] = pinfo[i];
    __syncthreads();
    const int c0 = blockIdx.x * blockDim.x + threadIdx.x;
    const int nright = n - k0 - nb;
    if (c0 >= nright + nrhs) return;
    double *col = c0 < nright ? A + (long long)(k0 + nb + c0) * lda : B + (long long)(c0 - nright) * ldb;
    col += k0;
    const int nd = pi[LU_PI_ND];
    // (loads and stores of x without branches on nb: per-element branches make
    // the register allocator spill x)
    double x[LU_NB];
#pragma unroll
    for (int i = 0; i < LU_NB; ++i) {
        const double v = col[pi[LU_PI_TOP + (i < nb ? i : 0)]];
        x[i] = i < nb ? v : 0.0;
    }
    for (int e = 0; e < nd; ++e) dv[e][threadIdx.x] = col[pi[LU_PI_SRC + e]];
    for (int e = 0; e < nd; ++e) col[pi[LU_PI_DST + e]] = dv[e][threadIdx.x];
#pragma unroll
    for (int i = 1; i < LU_NB; ++i) {
        double sacc = x[i];
#pragma unroll
        for (int j = 0; j < i; ++j) sacc -= L[i][j] * x[j];
        x[i] = sacc;
    }
    store_block(col, x, nb, dv);
}

// Back substitution on block rows r0..r0+nb-1: X = U11^{-1} X for every column
// of B (U11 staged in LDS).  One thread per column.
__global__ __launch_bounds__(64) void lu_trsm_upper_kernel(int nrhs, int r0, int nb, const double *A, int lda,
                                                           double *B, int ldb) {
    __shared__ double U[LU_NB][LU_NB + 1];
    __shared__ double stage[LU_NB][64];
    for (int i = threadIdx.x; i < LU_NB * LU_NB; i += 64) {
        const int r = i % LU_NB, c = i / LU_NB;
        U[r][c] = (r < nb && c < nb) ? A[(r0 + r) + (long long)(r0 + c) * lda] : (r == c ? 1.0 : 0.0);
    }
    __syncthreads();
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nrhs) return;
    double *col = B + (long long)c * ldb + r0;
    double x[LU_NB];
#pragma unroll
    for (int i = 0; i < LU_NB; ++i) {
        const double v = col[i < nb ? i : 0];
        x[i] = i < nb ? v : 0.0;
    }
#pragma unroll
    for (int i = LU_NB - 1; i >= 0; --i) {
        double sacc = x[i];
#pragma unroll
        for (int j = i + 1; j < LU_NB; ++j) sacc -= U[i][j] * x[j];
        x[i] = sacc / U[i][i];
    }
    store_block(col, x, nb, stage);
}

// Panels: LU_TALL_NB columns while more than LU_MAXM rows remain, LU_NB after.
size_t lu_pinfo_ints(int n) {
    const int tall = n > LU_MAXM ? (n - LU_MAXM + LU_TALL_NB - 1) / LU_TALL_NB : 0;
    return (size_t)(tall + (LU_MAXM + LU_NB - 1) / LU_NB + 1) * LU_PINFO;
}

hipError_t lu_solve(int n, int nrhs, double *A, int lda, double *B, int ldb, int *pinfo, hipStream_t s) {
    if (n > LU_TALL_MAXM) return gauss_jordan_solve(n, nrhs, A, lda, B, ldb, nullptr, s);
    hipError_t e;
    // B stored right after A with the same leading dimension: one GEMM updates both
    const bool joint = B == A + (long long)n * lda && ldb == lda;
    int npanel = 0;
    for (int k0 = 0, nb = 0; k0 < n; k0 += nb) {
        const int m = n - k0;
        nb = std::min(m > LU_MAXM ? LU_TALL_NB : LU_NB, m);
        int *pi = pinfo + (size_t)(npanel++) * LU_PINFO;
        if (m > LU_MAXM)
            hipLaunchKernelGGL(lu_panel_tall_kernel, dim3(1), dim3(LU_NT), 0, s, m, nb, A + k0 + (long long)k0 * lda,
                               lda, pi);
        else
            hipLaunchKernelGGL(lu_panel_kernel, dim3(1), dim3((m + 63) / 64 * 64), 0, s, m, nb,
                               A + k0 + (long long)k0 * lda, lda, pi);
        const int ncols = (n - k0 - nb) + nrhs;
        hipLaunchKernelGGL(lu_rowblock_kernel, dim3(nblk(ncols, 64)), dim3(64), 0, s, n, nrhs, k0, nb, A, lda,
                           B, ldb, (const int *)pi);
        const int mr = n - k0 - nb;
        if (mr > 0) {
            const double *L21 = A + (k0 + nb) + (long long)k0 * lda;
            if ((e = gemm(Op::N, Op::N, mr, joint ? mr + nrhs : mr, nb, -1.0, L21, lda, 0,
                          A + k0 + (long long)(k0 + nb) * lda, lda, 0, 1.0,
                          A + (k0 + nb) + (long long)(k0 + nb) * lda, lda, 0, 1, s)) != hipSuccess)
                return e;
            if (!joint && (e = gemm(Op::N, Op::N, mr, nrhs, nb, -1.0, L21, lda, 0, B + k0, ldb, 0, 1.0,
                                    B + (k0 + nb), ldb, 0, 1, s)) != hipSuccess)
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

// ---- the same reduction for larger n over the whole device (A in global
// memory, overwritten): per column k, the reflector (one workgroup), p = A22 v
// by row blocks x column chunks into partial sums, w = beta p - K v (one
// workgroup, fixed order), the rank-2 update of A22; then every eigenvalue of
// the tridiagonal (d, e) by Sturm bisection, one thread each.
constexpr int TRI_CHUNKS = 8;

namespace {

__global__ __launch_bounds__(1024) void tri_reflector_kernel(int n, int k, const double *A, int lda, double *v,
                                                             double *d, double *e, double *sc) {
    __shared__ double red[1024];
    const int t = threadIdx.x;
    const int m = n - k - 1;
    const double *x = A + (k + 1) + (long long)k * lda;
    double sq = 0.0;
    for (int i = t; i < m; i += 1024) sq += x[i] * x[i];
    red[t] = sq;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    const double x0 = x[0];
    const double nrm = sqrt(red[0]);
    const double alpha = x0 >= 0.0 ? -nrm : nrm;
    const double vtv = red[0] - x0 * x0 + (x0 - alpha) * (x0 - alpha);
    for (int i = t; i < m; i += 1024) v[i] = x[i] - (i == 0 ? alpha : 0.0);
    if (t == 0) {
        d[k] = A[k + (long long)k * lda];
        e[k] = alpha;
        sc[0] = vtv > 0.0 ? 2.0 / vtv : 0.0;   // beta
    }
}

// part[c][i] = sum over the c-th chunk of columns j of A22(i, j) v[j]
__global__ __launch_bounds__(256) void tri_matvec_kernel(int n, int k, const double *A, int lda, const double *v,
                                                         double *part) {
    const int m = n - k - 1;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    const int jlen = (m + TRI_CHUNKS - 1) / TRI_CHUNKS;
    const int j0 = c * jlen, j1 = min(m, j0 + jlen);
    if (i >= m) return;
    const double *a = A + (k + 1 + i) + (long long)(k + 1) * lda;
    double acc = 0.0;
    for (int j = j0; j < j1; ++j) acc += a[(long long)j * lda] * v[j];
    part[(long long)c * n + i] = acc;
}

// p = beta sum_c part, K = beta v.p / 2, w = p - K v (fixed order)
__global__ __launch_bounds__(1024) void tri_w_kernel(int n, int k, const double *part, const double *v, double *w,
                                                     const double *sc) {
    __shared__ double red[1024];
    const int t = threadIdx.x;
    const int m = n - k - 1;
    const double beta = sc[0];
    double vp = 0.0;
    for (int i = t; i < m; i += 1024) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < TRI_CHUNKS; ++c) acc += part[(long long)c * n + i];
        const double p = beta * acc;
        w[i] = p;
        vp += v[i] * p;
    }
    red[t] = vp;
    __syncthreads();
    for (int s2 = 512; s2 > 0; s2 >>= 1) {
        if (t < s2) red[t] += red[t + s2];
        __syncthreads();
    }
    const double K = 0.5 * beta * red[0];
    for (int i = t; i < m; i += 1024) w[i] -= K * v[i];
}

// A22 -= v w^T + w v^T
__global__ __launch_bounds__(256) void tri_update_kernel(int n, int k, double *A, int lda, const double *v,
                                                         const double *w) {
    const int m = n - k - 1;
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= m || j >= m) return;
    A[(k + 1 + i) + (long long)(k + 1 + j) * lda] -= v[i] * w[j] + w[i] * v[j];
}

// the last 2 x 2 block's diagonal and off-diagonal
__global__ void tri_tail_kernel(int n, const double *A, int lda, double *d, double *e) {
    if (n >= 2) {
        d[n - 2] = A[(n - 2) + (long long)(n - 2) * lda];
        e[n - 2] = A[(n - 1) + (long long)(n - 2) * lda];
    }
    d[n - 1] = A[(n - 1) + (long long)(n - 1) * lda];
}

// eig[idx] = the idx-th smallest eigenvalue of the tridiagonal (d, e): bisection
// on the Sturm count inside the Gershgorin bracket (d, e staged in LDS).
__global__ __launch_bounds__(256) void tri_bisect_kernel(int n, const double *dg, const double *eg, double *eig) {
    extern __shared__ double sh[];
    double *dd = sh, *ee = sh + n;
    for (int i = threadIdx.x; i < n; i += 256) {
        dd[i] = dg[i];
        ee[i] = i + 1 < n ? eg[i] : 0.0;
    }
    __syncthreads();
    double lo = 0.0, hi = 0.0;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < n ? fabs(ee[i]) : 0.0);
        lo = i == 0 ? dd[i] - r : fmin(lo, dd[i] - r);
        hi = i == 0 ? dd[i] + r : fmax(hi, dd[i] + r);
    }
    const double scale = fmax(fabs(lo), fabs(hi));
    const double tiny = 1e-300 + 1e-30 * scale;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= n) return;
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

}  // namespace

size_t sym_eigvals_work_doubles(int n) { return (size_t)(TRI_CHUNKS + 4) * n + 8; }

hipError_t sym_eigvals(int n, double *A, int lda, double *eig, double *work, hipStream_t s) {
    if (n <= JAC_LDS_MAX) {
        hipLaunchKernelGGL(tridiag_bisect_kernel, dim3(1), dim3(1024), 0, s, n, (const double *)A, lda, eig);
        return hipGetLastError();
    }
    if ((size_t)2 * n * 8 > 64 * 1024) return hipErrorInvalidValue;   // d, e in one workgroup's LDS
    double *v = work, *w = v + n, *d = w + n, *e = d + n, *part = e + n, *sc = part + (size_t)TRI_CHUNKS * n;
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;
        hipLaunchKernelGGL(tri_reflector_kernel, dim3(1), dim3(1024), 0, s, n, k, (const double *)A, lda, v, d, e,
                           sc);
        hipLaunchKernelGGL(tri_matvec_kernel, dim3((m + 255) / 256, TRI_CHUNKS), dim3(256), 0, s, n, k,
                           (const double *)A, lda, (const double *)v, part);
        hipLaunchKernelGGL(tri_w_kernel, dim3(1), dim3(1024), 0, s, n, k, (const double *)part, (const double *)v,
                           w, (const double *)sc);
        hipLaunchKernelGGL(tri_update_kernel, dim3((m + 255) / 256, m), dim3(256), 0, s, n, k, A, lda,
                           (const double *)v, (const double *)w);
    }
    hipLaunchKernelGGL(tri_tail_kernel, dim3(1), dim3(1), 0, s, n, (const double *)A, lda, d, e);
    hipLaunchKernelGGL(tri_bisect_kernel, dim3((n + 255) / 256), dim3(256), (size_t)2 * n * 8, s, n,
                       (const double *)d, (const double *)e, eig);
    return hipGetLastError();
}

hipError_t launch_dynmat_assemble(int np, int dim, const double *Phi_el, const double *K_local,
                                  const double *mass, double *D, double *asym2, hipStream_t s) {
    hipLaunchKernelGGL(dynmat_assemble_kernel, dim3(1), dim3(1024), 0, s, np, dim, Phi_el, K_local,
                       mass, D, np, asym2);
    return hipGetLastError();
}

}  // namespace acp
