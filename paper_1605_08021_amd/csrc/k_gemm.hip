// FP64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4_f64).
//
// Used for every dense contraction around the solve: the right-hand sides
// -Q Xi (Alg. 3 step 2), the W assembly of Eq. (3.7) (Hadamard-accumulate
// epilogue), the interpolation vectors of Alg. 2, the Fourier form of v_c, the
// Dyson update of Eq. (3.13) and G^T U of Eq. (2.11).
//
// Tile 64 x 64 x 16, 256 threads (4 waves of 64).  Each wave owns a 32 x 32
// quarter = 2 x 2 MFMA blocks of 16 x 16.  Operands are staged k-major in LDS so
// that the 16 lanes feeding one MFMA row read consecutive addresses.  The next
// k-slab is prefetched into registers while the current one is multiplied.  The
// epilogue goes through LDS so global stores are coalesced along columns.
//
// MFMA f64 16x16x4 lane layout (measured on gfx950): lane l supplies A[l%16][l/16]
// and B[l/16][l%16] and receives D[l/16 + 4 j][l%16], j = 0..3.
#include "acp_internal.h"

namespace acp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;
constexpr int LDA_S = BM + 2;   // padded LDS strides (elements)
constexpr int LDB_S = BN + 2;
constexpr int LDC_S = BM + 1;

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(NT) void gemm_f64_kernel(
    int M, int N, int K, double alpha, const double *__restrict__ A, int lda, long long sa,
    const double *__restrict__ B, int ldb, long long sb, double beta, double *__restrict__ C,
    int ldc, long long sc, const double *__restrict__ E, int lde, long long se) {
    __shared__ double smem[2 * BK * LDA_S > BN * LDC_S ? 2 * BK * LDA_S : BN * LDC_S];
    double *As = smem;                  // [BK][LDA_S]
    double *Bs = smem + BK * LDA_S;     // [BK][LDB_S]

    const int bz = blockIdx.z;
    A += bz * sa;
    B += bz * sb;
    C += bz * sc;
    if (EPI == 1) E += bz * se;

    // XCD-aware tile order: workgroup b runs on XCD b mod 8, so each XCD takes a
    // contiguous range of the tile sequence, in which the index over the
    // dimension with fewer tiles runs fastest: consecutive tiles of one XCD share
    // a panel of the other operand, which its L2 then serves to all of them.
    int bm, bn;
    {
        const int mt = gridDim.x, nt = gridDim.y;
        const int T = mt * nt;
        const int lin = blockIdx.x + mt * blockIdx.y;
        const int x = lin & 7, slot = lin >> 3;
        const int q = T >> 3, rem = T & 7;
        const int tile = x * q + (x < rem ? x : rem) + slot;
        if (mt <= nt) {
            bm = tile % mt;
            bn = tile / mt;
        } else {
            bn = tile % nt;
            bm = tile / nt;
        }
    }
    const int m0 = bm * BM;
    const int n0 = bn * BN;
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int wm = (wave & 1) * 32;
    const int wn = (wave >> 1) * 32;

    d4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    double ra[4], rb[4];
    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int mm, kk;
            if (!TA) { mm = t & 63; kk = (t >> 6) + 4 * q; }
            else     { kk = t & 15; mm = (t >> 4) + 16 * q; }
            int gm = m0 + mm, gk = k0 + kk;
            double v = 0.0;
            if (gm < M && gk < K) v = TA ? A[gk + (long long)gm * lda] : A[gm + (long long)gk * lda];
            ra[q] = v;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int nn, kk;
            if (!TB) { kk = t & 15; nn = (t >> 4) + 16 * q; }
            else     { nn = t & 63; kk = (t >> 6) + 4 * q; }
            int gn = n0 + nn, gk = k0 + kk;
            double v = 0.0;
            if (gn < N && gk < K) v = TB ? B[gn + (long long)gk * ldb] : B[gk + (long long)gn * ldb];
            rb[q] = v;
        }
    };
    auto store_tiles = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int mm, kk;
            if (!TA) { mm = t & 63; kk = (t >> 6) + 4 * q; }
            else     { kk = t & 15; mm = (t >> 4) + 16 * q; }
            As[kk * LDA_S + mm] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int nn, kk;
            if (!TB) { kk = t & 15; nn = (t >> 4) + 16 * q; }
            else     { nn = t & 63; kk = (t >> 6) + 4 * q; }
            Bs[kk * LDB_S + nn] = rb[q];
        }
    };

    load_tiles(0);
    for (int k0 = 0; k0 < K; k0 += BK) {
        __syncthreads();
        store_tiles();
        __syncthreads();
        if (k0 + BK < K) load_tiles(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int ka = kk + (lane >> 4);
            double a0 = As[ka * LDA_S + wm + (lane & 15)];
            double a1 = As[ka * LDA_S + wm + 16 + (lane & 15)];
            double b0 = Bs[ka * LDB_S + wn + (lane & 15)];
            double b1 = Bs[ka * LDB_S + wn + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
    }

    // epilogue through LDS: Cs[col][row]
    __syncthreads();
    double *Cs = smem;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int row = wm + 16 * i + (lane >> 4) + 4 * e;
                int col = wn + 16 * j + (lane & 15);
                Cs[col * LDC_S + row] = acc[i][j][e];
            }
    __syncthreads();
    for (int idx = t; idx < BM * BN; idx += NT) {
        int row = idx & (BM - 1);
        int col = idx >> 6;
        int gm = m0 + row, gn = n0 + col;
        if (gm < M && gn < N) {
            double v = alpha * Cs[col * LDC_S + row];
            double *cp = C + gm + (long long)gn * ldc;
            if (EPI != 1) {
                if (beta != 0.0) v += beta * (*cp);
                *cp = v;
            } else {
                *cp += v * E[gm + (long long)gn * lde];
            }
        }
    }
}

// The same product with 128 x 128 x 16 tiles for large outputs: each wave owns a
// 64 x 64 quarter = 4 x 4 MFMA blocks, halving the operand bytes per flop that
// the tiles request from L2; the epilogue goes through LDS in two halves of 64
// columns.
constexpr int BM2 = 128, BN2 = 128, LDA2 = BM2 + 2, LDB2 = BN2 + 2, LDC2 = BM2 + 1;
constexpr int SMEM2 = 2 * BK * LDA2 > (BN2 / 2) * LDC2 ? 2 * BK * LDA2 : (BN2 / 2) * LDC2;

template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(NT, 2) void gemm_f64_big_kernel(
    int M, int N, int K, double alpha, const double *__restrict__ A, int lda, long long sa,
    const double *__restrict__ B, int ldb, long long sb, double beta, double *__restrict__ C,
    int ldc, long long sc, const double *__restrict__ E, int lde, long long se) {
    __shared__ double smem[SMEM2];
    double *As = smem;                   // [BK][LDA2]
    double *Bs = smem + BK * LDA2;       // [BK][LDB2]

    const int bz = blockIdx.z;
    A += bz * sa;
    B += bz * sb;
    C += bz * sc;
    if (EPI == 1) E += bz * se;

    int bm, bn;
    {   // XCD-aware tile order, as in gemm_f64_kernel
        const int mt = gridDim.x, nt = gridDim.y;
        const int T = mt * nt;
        const int lin = blockIdx.x + mt * blockIdx.y;
        const int x = lin & 7, slot = lin >> 3;
        const int q = T >> 3, rem = T & 7;
        const int tile = x * q + (x < rem ? x : rem) + slot;
        if (mt <= nt) {
            bm = tile % mt;
            bn = tile / mt;
        } else {
            bn = tile % nt;
            bm = tile / nt;
        }
    }
    const int m0 = bm * BM2, n0 = bn * BN2;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;

    d4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    double ra[8], rb[8];
    auto load_tiles = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int mm, kk;
            if (!TA) { mm = t & 127; kk = (t >> 7) + 2 * q; }
            else     { kk = t & 15; mm = (t >> 4) + 16 * q; }
            const int gm = m0 + mm, gk = k0 + kk;
            double v = 0.0;
            if (gm < M && gk < K) v = TA ? A[gk + (long long)gm * lda] : A[gm + (long long)gk * lda];
            ra[q] = v;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int nn, kk;
            if (!TB) { kk = t & 15; nn = (t >> 4) + 16 * q; }
            else     { nn = t & 127; kk = (t >> 7) + 2 * q; }
            const int gn = n0 + nn, gk = k0 + kk;
            double v = 0.0;
            if (gn < N && gk < K) v = TB ? B[gn + (long long)gk * ldb] : B[gk + (long long)gn * ldb];
            rb[q] = v;
        }
    };
    auto store_tiles = [&]() {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int mm, kk;
            if (!TA) { mm = t & 127; kk = (t >> 7) + 2 * q; }
            else     { kk = t & 15; mm = (t >> 4) + 16 * q; }
            As[kk * LDA2 + mm] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            int nn, kk;
            if (!TB) { kk = t & 15; nn = (t >> 4) + 16 * q; }
            else     { nn = t & 127; kk = (t >> 7) + 2 * q; }
            Bs[kk * LDB2 + nn] = rb[q];
        }
    };

    load_tiles(0);
    for (int k0 = 0; k0 < K; k0 += BK) {
        __syncthreads();
        store_tiles();
        __syncthreads();
        if (k0 + BK < K) load_tiles(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int ka = kk + (lane >> 4);
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[ka * LDA2 + wm + 16 * i + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[ka * LDB2 + wn + 16 * j + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }

    // epilogue through LDS, 64 columns at a time: Cs[col][row]
    double *Cs = smem;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        __syncthreads();
        if (wn == 64 * h) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int row = wm + 16 * i + (lane >> 4) + 4 * e;
                        const int col = 16 * j + (lane & 15);
                        Cs[col * LDC2 + row] = acc[i][j][e];
                    }
        }
        __syncthreads();
        for (int idx = t; idx < BM2 * (BN2 / 2); idx += NT) {
            const int row = idx & (BM2 - 1);
            const int col = idx >> 7;
            const int gm = m0 + row, gn = n0 + 64 * h + col;
            if (gm < M && gn < N) {
                double v = alpha * Cs[col * LDC2 + row];
                double *cp = C + gm + (long long)gn * ldc;
                if (EPI != 1) {
                    if (beta != 0.0) v += beta * (*cp);
                    *cp = v;
                } else {
                    *cp += v * E[gm + (long long)gn * lde];
                }
            }
        }
    }
}

template <bool TA, bool TB>
hipError_t dispatch_epi(int m, int n, int k, double alpha, const double *A, int lda, long long sa,
                        const double *B, int ldb, long long sb, double beta, double *C, int ldc,
                        long long sc, int batch, hipStream_t s, Epi epi, const double *E,
                        int lde, long long se) {
    // large outputs (at least ~2 tiles of 128 x 128 per CU) take the 128-wide tiles
    const long long big_tiles = (long long)((m + BM2 - 1) / BM2) * ((n + BN2 - 1) / BN2) * batch;
    if (m >= BM2 && n >= BN2 && big_tiles >= 512) {
        dim3 grid((m + BM2 - 1) / BM2, (n + BN2 - 1) / BN2, batch);
        if (epi == Epi::Store)
            hipLaunchKernelGGL((gemm_f64_big_kernel<TA, TB, 0>), grid, dim3(NT), 0, s, m, n, k, alpha, A, lda, sa, B,
                               ldb, sb, beta, C, ldc, sc, E, lde, se);
        else if (epi == Epi::StoreProjector)
            hipLaunchKernelGGL((gemm_f64_big_kernel<TA, TB, 2>), grid, dim3(NT), 0, s, m, n, k, alpha, A, lda, sa, B,
                               ldb, sb, beta, C, ldc, sc, E, lde, se);
        else
            hipLaunchKernelGGL((gemm_f64_big_kernel<TA, TB, 1>), grid, dim3(NT), 0, s, m, n, k, alpha, A, lda, sa, B,
                               ldb, sb, beta, C, ldc, sc, E, lde, se);
        return hipGetLastError();
    }
    dim3 grid((m + BM - 1) / BM, (n + BN - 1) / BN, batch);
    if (epi == Epi::Store)
        hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, 0>), grid, dim3(NT), 0, s, m, n, k, alpha, A,
                           lda, sa, B, ldb, sb, beta, C, ldc, sc, E, lde, se);
    else if (epi == Epi::StoreProjector)   // same code; its own symbol, so profiles separate it
        hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, 2>), grid, dim3(NT), 0, s, m, n, k, alpha, A,
                           lda, sa, B, ldb, sb, beta, C, ldc, sc, E, lde, se);
    else
        hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, 1>), grid, dim3(NT), 0, s, m, n, k, alpha, A,
                           lda, sa, B, ldb, sb, beta, C, ldc, sc, E, lde, se);
    return hipGetLastError();
}

__global__ void scale_kernel(int m, int n, double beta, double *C, int ldc) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long tot = (long long)m * n;
    if (idx < tot) {
        int i = (int)(idx % m);
        long long j = idx / m;
        double *p = C + i + j * ldc;
        *p = (beta == 0.0) ? 0.0 : beta * (*p);
    }
}

// C = alpha * sum_s W_s + beta C over the split-K partial products W (fixed order).
__global__ void splitk_reduce_kernel(int m, int n, int nsplit, const double *W, double alpha,
                                     double beta, double *C, int ldc) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long tot = (long long)m * n;
    if (idx >= tot) return;
    int i = (int)(idx % m);
    long long j = idx / m;
    double v = 0.0;
    for (int sidx = 0; sidx < nsplit; ++sidx) v += W[sidx * tot + idx];
    double *cp = C + i + j * ldc;
    *cp = alpha * v + ((beta != 0.0) ? beta * (*cp) : 0.0);
}

}  // namespace

hipError_t gemm_splitk(Op ta, Op tb, int m, int n, int k, double alpha, const double *A, int lda,
                       const double *B, int ldb, double beta, double *C, int ldc, double *work,
                       size_t work_elems, hipStream_t s, Epi epi) {
    // split so that the grid has >= ~512 workgroups; each slice handles a multiple
    // of 64 of K.  The slices of equal length run as one batched launch (batch
    // index = slice), a shorter last slice as a second launch.
    const int tiles = ((m + BM - 1) / BM) * ((n + BN - 1) / BN);
    int nsplit = (512 + tiles - 1) / tiles;
    const int kmax_split = (k + 63) / 64;
    if (nsplit > kmax_split) nsplit = kmax_split;
    while (nsplit > 1 && (size_t)nsplit * m * n > work_elems) --nsplit;
    if (nsplit <= 1)
        return gemm(ta, tb, m, n, k, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1, s, epi);
    const int kc = ((k + nsplit - 1) / nsplit + 63) / 64 * 64;
    const int nfull = k / kc;
    const int rem = k - nfull * kc;
    nsplit = nfull + (rem > 0 ? 1 : 0);
    const long long sa = (ta == Op::N) ? (long long)kc * lda : kc;
    const long long sb = (tb == Op::N) ? kc : (long long)kc * ldb;
    const long long sc = (long long)m * n;
    hipError_t e = gemm(ta, tb, m, n, kc, 1.0, A, lda, sa, B, ldb, sb, 0.0, work, m, sc, nfull, s, epi);
    if (e != hipSuccess) return e;
    if (rem > 0) {
        e = gemm(ta, tb, m, n, rem, 1.0, A + nfull * sa, lda, 0, B + nfull * sb, ldb, 0, 0.0,
                 work + (size_t)nfull * m * n, m, 0, 1, s, epi);
        if (e != hipSuccess) return e;
    }
    long long tot = (long long)m * n;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       m, n, nsplit, work, alpha, beta, C, ldc);
    return hipGetLastError();
}

hipError_t gemm(Op ta, Op tb, int m, int n, int k, double alpha, const double *A, int lda,
                long long sa, const double *B, int ldb, long long sb, double beta, double *C,
                int ldc, long long sc, int batch, hipStream_t s, Epi epi, const double *E,
                int lde, long long se) {
    if (m <= 0 || n <= 0 || batch <= 0) return hipSuccess;
    if (k <= 0) {
        if (epi == Epi::HadamardAcc) return hipSuccess;
        for (int b = 0; b < batch; ++b) {
            long long tot = (long long)m * n;
            hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                               m, n, beta, C + b * sc, ldc);
        }
        return hipGetLastError();
    }
    if (ta == Op::N && tb == Op::N)
        return dispatch_epi<false, false>(m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc,
                                          batch, s, epi, E, lde, se);
    if (ta == Op::T && tb == Op::N)
        return dispatch_epi<true, false>(m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc,
                                         batch, s, epi, E, lde, se);
    if (ta == Op::N && tb == Op::T)
        return dispatch_epi<false, true>(m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc,
                                         batch, s, epi, E, lde, se);
    return dispatch_epi<true, true>(m, n, k, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc,
                                    batch, s, epi, E, lde, se);
}

}  // namespace acp
