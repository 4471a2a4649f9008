// Greedy pivoted Cholesky of the implicit Hadamard Gram matrix
//     K(a, b) = (phi(a,:) . phi(b,:)) (G~(a,:) . G~(b,:))
// (the point selection of Alg. 2, see k_dense.hip) in panels, for grids whose
// Phi Phi^T is not kept.  The step-by-step form reads all of Phi and all
// previous columns of the factor L for every pivot (N_g (N_e + r + k) values);
// here a pool S of the rows with the largest remaining diagonal is chosen, and
// their residual Gram columns
//     Kp(:, S) = (Phi Phi(S,:)^T) o (G~ G~(S,:)^T) - L(:, 0..k0) L(S, 0..k0)^T
// are formed by three GEMMs on the matrix cores.  The next pivots are then
// taken from the pool, each step reading one column of Kp and the at most b
// columns of L added since the pool was formed.
//
// The pivots are exactly those of the step-by-step greedy rule: the remaining
// diagonal only decreases, every row outside S had a diagonal of at most theta
// (the largest outside S) when the pool was formed, so while the best row of S
// is still above theta it is the best row of the whole grid.  A step whose best
// pool row has fallen to theta ends the panel; the next pool is formed from the
// current diagonal.
#include <algorithm>

#include "acp_internal.h"

namespace acp {
namespace {

constexpr int PNT = 256;   // threads per block of the step kernel (one grid row each)

__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
    return v > bv || (v == bv && i < bi);
}

__device__ __forceinline__ void wave_best(double &v, int &i) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        const double ov = __shfl_xor(v, m, 64);
        const int oi = __shfl_xor(i, m, 64);
        if (better(ov, oi, v, i)) {
            v = ov;
            i = oi;
        }
    }
}

// diag(a) = |phi(a,:)|^2 |G~(a,:)|^2
__global__ void panel_diag_kernel(int ng, int ne, int r, const double *phi, const double *gt, double *diag) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= ng) return;
    double s1 = 0.0, s2 = 0.0;
    for (int i = 0; i < ne; ++i) {
        const double v = phi[a + (long long)i * ng];
        s1 += v * v;
    }
    for (int j = 0; j < r; ++j) {
        const double v = gt[a + (long long)j * ng];
        s2 += v * v;
    }
    diag[a] = s1 * s2;
}

// Block sums of 1024 threads (every thread gets the total).
__device__ double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

__device__ double block_max(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

// One block of 1024 threads: the pool S = the rows whose diagonal is at least
// a threshold t (found by bisection so that at most m rows pass; with more than
// m rows at the maximum, the first m of them), in index order; theta = the
// largest diagonal outside S (-inf if none), dS[pos] = diag(S[pos]),
// spos[S[pos]] = pos (spos is -1 elsewhere on entry).  info[0] = |S|.
__global__ __launch_bounds__(1024) void pool_select_kernel(int ng, int m, const double *diag, int *S, int *spos,
                                                           double *dS, double *theta, int *info) {
    __shared__ double red[1024];
    __shared__ int wcnt[16];
    __shared__ int s_base;
    const int t = threadIdx.x;
    double vmax = -INFINITY;
    for (int a = t; a < ng; a += 1024) vmax = fmax(vmax, diag[a]);
    vmax = block_max(vmax, red);
    if (!(vmax > 0.0)) {
        if (t == 0) {
            info[0] = 0;
            theta[0] = -INFINITY;
        }
        return;
    }
    // bisection on t in (0, vmax]: count(diag >= t) <= m at hi
    double lo = 0.0, hi = vmax;
    for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        double c = 0.0;
        for (int a = t; a < ng; a += 1024) c += diag[a] >= mid ? 1.0 : 0.0;
        c = block_sum(c, red);
        if (c > m) {
            lo = mid;
        } else {
            hi = mid;
            if (2 * c >= m) break;   // a pool at least half full is enough
        }
    }
    // compaction in index order (at most m rows); theta = the largest diagonal left out
    if (t == 0) s_base = 0;
    __syncthreads();
    double out_max = -INFINITY;
    const int lane = t & 63, wave = t >> 6;
    for (int a0 = 0; a0 < ng; a0 += 1024) {
        const int a = a0 + t;
        const double v = a < ng ? diag[a] : -INFINITY;
        const bool f = a < ng && v >= hi;
        const unsigned long long bal = __ballot(f);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wcnt[wave] = __popcll(bal);
        __syncthreads();
        int off = s_base;
        for (int w = 0; w < wave; ++w) off += wcnt[w];
        const int pos = off + before;
        if (f && pos < m) {
            S[pos] = a;
            spos[a] = pos;
            dS[pos] = v;
        } else if (a < ng) {
            out_max = fmax(out_max, v);
        }
        __syncthreads();
        if (t == 0) {
            int tot = 0;
            for (int w = 0; w < 16; ++w) tot += wcnt[w];
            s_base += tot;
        }
        __syncthreads();
    }
    out_max = block_max(out_max, red);
    if (t == 0) {
        info[0] = s_base < m ? s_base : m;
        theta[0] = out_max;
    }
}

// Pivot k of a panel started at k0: p = the best row of the pool (ties to the
// smallest index); it must lie above theta (else the panel ends: state[2] = 1)
// and satisfy the stopping rules (a positive remaining diagonal; with tol2 > 0,
// diag(p) >= tol2 diag(first pivot), the rank rule of Alg. 2 step 3).  Then for
// every row a:  L(a, k) = (Kp(a, pos(p)) - sum_{k0 <= j < k} L(a, j) L(p, j)) / sqrt(diag(p)),
// diag(a) -= L(a, k)^2 (diag(p) = -1), and the pool's diagonal goes to dS_out.
__global__ __launch_bounds__(PNT) void panel_step_kernel(int ng, int k, int k0, int ns, int skip_theta,
                                                         const int *S, const double *theta, const double *Kp,
                                                         double *L, double *diag, const int *spos,
                                                         const double *dS_in, double *dS_out, int *sel,
                                                         double tol2, int *state, double *dvals) {
    __shared__ double lp[kIsdfPanel];
    if (state[1] || state[2]) return;
    const int t = threadIdx.x;
    double bv = -INFINITY;
    int bi = 0x7fffffff;
    for (int q = t & 63; q < ns; q += 64) {
        const double v = dS_in[q];
        const int i = S[q];
        if (better(v, i, bv, bi)) {
            bv = v;
            bi = i;
        }
    }
    wave_best(bv, bi);
    const bool stop = !(bv > 0.0) || (tol2 > 0.0 && k > 0 && bv < tol2 * dvals[0]);
    const bool brk = !stop && !skip_theta && !(bv > theta[0]);
    if (blockIdx.x == 0 && t == 0) {
        if (stop) {
            state[1] = 1;
        } else if (brk) {
            state[2] = 1;
        } else {
            sel[k] = bi;
            state[0] = k + 1;
            if (k == 0) dvals[0] = bv;
        }
    }
    if (stop || brk) return;
    const int nj = k - k0;
    for (int j = t; j < nj; j += PNT) lp[j] = L[bi + (long long)(k0 + j) * ng];
    __syncthreads();
    const int a = blockIdx.x * PNT + t;
    if (a >= ng) return;
    double y = 0.0;
    for (int j = 0; j < nj; ++j) y += L[a + (long long)(k0 + j) * ng] * lp[j];
    const double lk = (Kp[a + (long long)spos[bi] * ng] - y) / sqrt(bv);
    const double dnew = (a == bi) ? -1.0 : diag[a] - lk * lk;
    L[a + (long long)k * ng] = lk;
    diag[a] = dnew;
    const int q = spos[a];
    if (q >= 0) dS_out[q] = dnew;
}

}  // namespace

size_t isdf_panel_scratch_bytes(int ng, int ne, int r, int nmu) {
    const size_t m = kIsdfPool;
    return 8 * ((size_t)2 * ng * m            // P1, Kp
                + m * (ne + r + nmu)           // gathered rows of Phi, G~, L
                + 2 * m + 8)                   // dS ping-pong, theta
           + 4 * ((size_t)ng + m + 8);         // spos, S, info, state
}

hipError_t isdf_panel_cholesky(int ng, int ne, int r, const double *phi, const double *gt, int nmu_max, double tol,
                               double *L, double *diag, int *sel_dev, int *nmu_out_host, void *scratch,
                               hipStream_t s) {
    const int m = kIsdfPool;
    double *P1 = (double *)scratch;
    double *Kp = P1 + (size_t)ng * m;
    double *Rphi = Kp + (size_t)ng * m;
    double *Rg = Rphi + (size_t)m * ne;
    double *RL = Rg + (size_t)m * r;
    double *dS = RL + (size_t)m * nmu_max;
    double *theta = dS + 2 * m;
    double *dvals = theta + 4;
    int *spos = (int *)(dvals + 4);
    int *S = spos + ng;
    int *info = S + m;
    int *state = info + 4;
    hipError_t e;
    if ((e = launch_fill_i32(state, 4, 0, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(panel_diag_kernel, dim3((ng + 255) / 256), dim3(256), 0, s, ng, ne, r, phi, gt, diag);
    const double tol2 = tol * tol;
    int k = 0, skip_theta = 0;
    while (k < nmu_max) {
        if ((e = launch_fill_i32(spos, ng, -1, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(pool_select_kernel, dim3(1), dim3(1024), 0, s, ng, m, (const double *)diag, S, spos, dS,
                           theta, info);
        int hinfo[4];
        if ((e = hipMemcpyAsync(hinfo, info, 4 * sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        const int ns = hinfo[0];
        if (ns == 0) break;   // no positive diagonal left
        // residual Gram columns of the pool
        if ((e = launch_gather_rows(ns, ne, S, phi, ng, Rphi, m, s)) != hipSuccess) return e;
        if ((e = launch_gather_rows(ns, r, S, gt, ng, Rg, m, s)) != hipSuccess) return e;
        if ((e = gemm(Op::N, Op::T, ng, ns, ne, 1.0, phi, ng, 0, Rphi, m, 0, 0.0, P1, ng, 0, 1, s)) != hipSuccess)
            return e;
        if ((e = hipMemsetAsync(Kp, 0, (size_t)ng * ns * 8, s)) != hipSuccess) return e;
        if ((e = gemm(Op::N, Op::T, ng, ns, r, 1.0, gt, ng, 0, Rg, m, 0, 0.0, Kp, ng, 0, 1, s, Epi::HadamardAcc, P1, ng,
                      0)) != hipSuccess)
            return e;
        if (k > 0) {
            if ((e = launch_gather_rows(ns, k, S, L, ng, RL, m, s)) != hipSuccess) return e;
            if ((e = gemm(Op::N, Op::T, ng, ns, k, -1.0, L, ng, 0, RL, m, 0, 1.0, Kp, ng, 0, 1, s)) != hipSuccess)
                return e;
        }
        if ((e = launch_fill_i32(state + 2, 1, 0, s)) != hipSuccess) return e;
        const int b = skip_theta ? 1 : std::min(kIsdfPanel, nmu_max - k);
        for (int i = 0; i < b; ++i) {
            const double *din = dS + (i & 1) * m;
            double *dout = dS + ((i + 1) & 1) * m;
            hipLaunchKernelGGL(panel_step_kernel, dim3((ng + PNT - 1) / PNT), dim3(PNT), 0, s, ng, k + i, k, ns,
                               skip_theta, (const int *)S, (const double *)theta, (const double *)Kp, L, diag,
                               (const int *)spos, din, dout, sel_dev, tol2, state, dvals);
        }
        int hs[4];
        if ((e = hipMemcpyAsync(hs, state, 4 * sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        if (hs[1]) {
            k = hs[0];
            break;
        }
        // no progress only when the best pool rows tie with theta: the next step
        // takes the pool's best (still a largest remaining diagonal)
        skip_theta = hs[0] == k;
        k = hs[0];
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (nmu_out_host) *nmu_out_host = k;
    return hipSuccess;
}

}  // namespace acp
