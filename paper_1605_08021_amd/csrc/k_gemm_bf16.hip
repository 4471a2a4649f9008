// BF16 GEMM on the CDNA4 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation) for the projector of the many-orbital solver in its
// reduced-precision form, and the conversions that feed it.
//
// Both operands are K-major ("TN"): A_s[m lda + k], B_s[n ldb + k], so every
// lane's MFMA fragment (8 consecutive k) is one 16-byte load.  An operand can be
// split into up to three BF16 terms x = x_0 + x_1 + x_2 (x_0 = bf16(x),
// x_1 = bf16(x - x_0), ...); the kernel sums the products A_a B_b with
// a + b < max(NA, NB) (the dropped cross terms are below the last kept one), so
// two terms per operand carry ~16 significant bits and three ~24.
//
// Tile 128 x 128 x 64, 256 threads = 4 waves in 2 x 2, each wave 64 x 64 =
// 4 x 4 blocks of 16 x 16.  The slab of every term is staged in LDS with rows
// padded to 72 elements (144 bytes: the 16 lanes of one fragment read hit
// disjoint banks); the next slab is prefetched into registers while the current
// one is multiplied.
//
// MFMA bf16 16x16x32 lane layout: lane l supplies A[l%16][8(l/16) + j] and
// B[8(l/16) + j][l%16], j = 0..7, and receives D[4(l/16) + r][l%16], r = 0..3.
//
// Epilogues: 0 stores the FP32 tile into split-K slice blockIdx.z of P
// (P[z psz + n ldp + m]); 1 adds alpha * tile to a column-major FP64 matrix
// (W[n ldw + m] += ...): per 16 x 16 block each column receives 4 lanes x 4
// consecutive rows = one 128-byte line.
#include "acp_internal.h"

namespace acp {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

constexpr int TM = 128, TN = 128, TK = 64, NTH = 256;
constexpr int LK = TK + 8;            // LDS row stride (elements)
constexpr int CHUNKS = TM * TK / 8 / NTH;   // 16-byte chunks per thread per term (4)

// Split column-major X (m x n, leading dimension ldx) into nt BF16 terms
// written with leading dimension ldo; rows m..ldo-1 of the output are zeroed.
__global__ void split_bf16_kernel(int m, int n, const double *__restrict__ X, long long ldx, int nt,
                                  unsigned short *__restrict__ O0, unsigned short *__restrict__ O1,
                                  unsigned short *__restrict__ O2, long long ldo) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= ldo) return;
    const long long o = (long long)j * ldo + i;
    if (i >= m) {
        O0[o] = 0;
        if (nt > 1) O1[o] = 0;
        if (nt > 2) O2[o] = 0;
        return;
    }
    double x = X[(long long)j * ldx + i];
    const unsigned short h0 = f64_to_bf16(x);
    O0[o] = h0;
    if (nt > 1) {
        x -= bf16_to_f64(h0);
        const unsigned short h1 = f64_to_bf16(x);
        O1[o] = h1;
        if (nt > 2) {
            x -= bf16_to_f64(h1);
            O2[o] = f64_to_bf16(x);
        }
    }
}

// Row-major split: X column-major (m x n, ldx) -> O_s[i ldo + j] (the
// transpose of the column-major split), columns n..ldo-1 zeroed.  One block
// transposes a 32 x 32 tile through LDS.
__global__ void split_bf16_transpose_kernel(int m, int n, const double *__restrict__ X, long long ldx, int nt,
                                            unsigned short *__restrict__ O0, unsigned short *__restrict__ O1,
                                            unsigned short *__restrict__ O2, long long ldo) {
    __shared__ double tile[32][33];
    const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + tx, j = j0 + r;
        tile[r][tx] = (i < m && j < n) ? X[(long long)j * ldx + i] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + r, j = j0 + tx;
        if (i >= m || j >= ldo) continue;
        double x = tile[tx][r];
        const long long o = (long long)i * ldo + j;
        const unsigned short h0 = f64_to_bf16(x);
        O0[o] = h0;
        if (nt > 1) {
            x -= bf16_to_f64(h0);
            const unsigned short h1 = f64_to_bf16(x);
            O1[o] = h1;
            if (nt > 2) {
                x -= bf16_to_f64(h1);
                O2[o] = f64_to_bf16(x);
            }
        }
    }
}

struct TermPtrs {
    const unsigned short *p[3];
};

template <int NA, int NB, int EPI>
__global__ __launch_bounds__(NTH, 2) void gemm_bf16_tn_kernel(int M, int N, int K, TermPtrs A, long long lda,
                                                          TermPtrs B, long long ldb, int kslice,
                                                          float *__restrict__ P, long long ldp, long long psz,
                                                          double *__restrict__ Wd, long long ldw, double alpha) {
    constexpr int NP = NA > NB ? NA : NB;
    __shared__ __attribute__((aligned(16))) unsigned short lds[(NA + NB) * TM * LK];
    unsigned short *As = lds;                    // [NA][TM][LK]
    unsigned short *Bs = lds + NA * TM * LK;     // [NB][TN][LK]

    int bm, bn;
    {   // XCD-aware tile order (workgroup b runs on XCD b mod 8): each XCD takes a
        // contiguous range of tiles, the dimension with fewer tiles fastest
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
    const int m0 = bm * TM, n0 = bn * TN;
    const int kbeg = blockIdx.z * kslice;
    const int kend = min(K, kbeg + kslice);
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;

    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    u4 ra[NA][CHUNKS], rb[NB][CHUNKS];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < CHUNKS; ++q) {
            const int c = t + NTH * q;
            const int row = c >> 3, kc = (c & 7) * 8;
            const int gk = k0 + kc;
            const bool kin = gk < kend;   // K and every slice boundary are multiples of 8
            const int gm = m0 + row, gn = n0 + row;
#pragma unroll
            for (int a = 0; a < NA; ++a)
                ra[a][q] = (kin && gm < M) ? *(const u4 *)(A.p[a] + (long long)gm * lda + gk) : u4{0u, 0u, 0u, 0u};
#pragma unroll
            for (int b = 0; b < NB; ++b)
                rb[b][q] = (kin && gn < N) ? *(const u4 *)(B.p[b] + (long long)gn * ldb + gk) : u4{0u, 0u, 0u, 0u};
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < CHUNKS; ++q) {
            const int c = t + NTH * q;
            const int row = c >> 3, kc = (c & 7) * 8;
#pragma unroll
            for (int a = 0; a < NA; ++a) *(u4 *)(As + (a * TM + row) * LK + kc) = ra[a][q];
#pragma unroll
            for (int b = 0; b < NB; ++b) *(u4 *)(Bs + (b * TN + row) * LK + kc) = rb[b][q];
        }
    };

    const int fr = lane & 15, fk = (lane >> 4) * 8;
    load(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
        __syncthreads();
        store();
        __syncthreads();
        if (k0 + TK < kend) load(k0 + TK);
#pragma unroll
        for (int kk = 0; kk < TK; kk += 32) {
            bf8 bfr[NB][4];
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    bfr[b][j] = *(const bf8 *)(Bs + (b * TN + wn + 16 * j + fr) * LK + kk + fk);
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const bf8 afr = *(const bf8 *)(As + (a * TM + wm + 16 * i + fr) * LK + kk + fk);
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        if (a + b >= NP) continue;
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[b][j], acc[i][j], 0, 0, 0);
                    }
                }
        }
    }

#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + wn + 16 * j + fr;
            const int mb = m0 + wm + 16 * i + (lane >> 4) * 4;
            if (n >= N) continue;
            if (EPI == 0) {
                float *pp = P + (long long)blockIdx.z * psz + (long long)n * ldp + mb;
                if (mb + 3 < M) {
                    *(f4 *)pp = acc[i][j];
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (mb + r < M) pp[r] = acc[i][j][r];
                }
            } else {
                double *wp = Wd + (long long)n * ldw + mb;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (mb + r < M) wp[r] += alpha * (double)acc[i][j][r];
            }
        }
}

// C'(i, j) = bf16((T - eps_i) * sum_z P[z psz + j ldp + i]) for i < m (T alone
// without eps), zero for m <= i < ldc (the padding the next GEMM reads as K).
__global__ void deflate_coef_kernel(int m, int n, int nsplit, const float *__restrict__ P, long long ldp,
                                    long long psz, const double *__restrict__ eps, double T,
                                    unsigned short *__restrict__ Cb, long long ldc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= ldc) return;
    double v = 0.0;
    if (i < m) {
        for (int z = 0; z < nsplit; ++z) v += (double)P[(long long)z * psz + (long long)j * ldp + i];
        v *= eps ? T - eps[i] : T;
    }
    Cb[(long long)j * ldc + i] = f64_to_bf16(v);
}

template <int NA, int NB, int EPI>
hipError_t launch_tn(int M, int N, int K, const unsigned short *const *A, long long lda,
                     const unsigned short *const *B, long long ldb, int nsplit, float *P, long long ldp,
                     double *Wd, long long ldw, double alpha, hipStream_t s) {
    TermPtrs ta{}, tb{};
    for (int a = 0; a < NA; ++a) ta.p[a] = A[a];
    for (int b = 0; b < NB; ++b) tb.p[b] = B[b];
    int kslice = (K + nsplit - 1) / nsplit;
    kslice = (kslice + TK - 1) / TK * TK;
    const int nz = (K + kslice - 1) / kslice;
    dim3 grid((M + TM - 1) / TM, (N + TN - 1) / TN, nz);
    hipLaunchKernelGGL((gemm_bf16_tn_kernel<NA, NB, EPI>), grid, dim3(NTH), 0, s, M, N, K, ta, lda, tb, ldb,
                       kslice, P, ldp, (long long)ldp * N, Wd, ldw, alpha);
    return hipGetLastError();
}

}  // namespace

int bf16_split_count(int K, int nsplit) {
    int kslice = (K + nsplit - 1) / nsplit;
    kslice = (kslice + TK - 1) / TK * TK;
    return (K + kslice - 1) / kslice;
}

hipError_t launch_split_bf16(int m, int n, const double *X, long long ldx, int nt, unsigned short *const *O,
                             long long ldo, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    if (nt < 1 || nt > 3 || ldo < m) return hipErrorInvalidValue;
    hipLaunchKernelGGL(split_bf16_kernel, dim3((unsigned)((ldo + 255) / 256), n), dim3(256), 0, s, m, n, X, ldx,
                       nt, O[0], nt > 1 ? O[1] : nullptr, nt > 2 ? O[2] : nullptr, ldo);
    return hipGetLastError();
}

hipError_t launch_split_bf16_transpose(int m, int n, const double *X, long long ldx, int nt,
                                       unsigned short *const *O, long long ldo, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    if (nt < 1 || nt > 3 || ldo < n) return hipErrorInvalidValue;
    hipLaunchKernelGGL(split_bf16_transpose_kernel, dim3((m + 31) / 32, (unsigned)((ldo + 31) / 32)), dim3(256), 0,
                       s, m, n, X, ldx, nt, O[0], nt > 1 ? O[1] : nullptr, nt > 2 ? O[2] : nullptr, ldo);
    return hipGetLastError();
}

hipError_t gemm_bf16_tn(int na, int nb, int epi, int M, int N, int K, const unsigned short *const *A, long long lda,
                        const unsigned short *const *B, long long ldb, int nsplit, float *P, long long ldp,
                        double *Wd, long long ldw, double alpha, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    if ((K & 7) || (lda & 7) || (ldb & 7)) return hipErrorInvalidValue;
    if (epi == 0 && (ldp < M || (ldp & 3))) return hipErrorInvalidValue;
    if (epi == 1 && nsplit != 1) return hipErrorInvalidValue;
    if (na == 2 && nb == 2 && epi == 0)
        return launch_tn<2, 2, 0>(M, N, K, A, lda, B, ldb, nsplit, P, ldp, Wd, ldw, alpha, s);
    if (na == 1 && nb == 1 && epi == 0)
        return launch_tn<1, 1, 0>(M, N, K, A, lda, B, ldb, nsplit, P, ldp, Wd, ldw, alpha, s);
    if (na == 3 && nb == 1 && epi == 1)
        return launch_tn<3, 1, 1>(M, N, K, A, lda, B, ldb, 1, P, ldp, Wd, ldw, alpha, s);
    if (na == 3 && nb == 1 && epi == 0)
        return launch_tn<3, 1, 0>(M, N, K, A, lda, B, ldb, 1, P, ldp, Wd, ldw, alpha, s);
    if (na == 3 && nb == 2 && epi == 1)
        return launch_tn<3, 2, 1>(M, N, K, A, lda, B, ldb, 1, P, ldp, Wd, ldw, alpha, s);
    if (na == 2 && nb == 1 && epi == 1)
        return launch_tn<2, 1, 1>(M, N, K, A, lda, B, ldb, 1, P, ldp, Wd, ldw, alpha, s);
    if (na == 1 && nb == 1 && epi == 1)
        return launch_tn<1, 1, 1>(M, N, K, A, lda, B, ldb, 1, P, ldp, Wd, ldw, alpha, s);
    return hipErrorInvalidValue;
}

hipError_t launch_deflate_coef(int m, int n, int nsplit, const float *P, long long ldp, const double *eps, double T,
                               unsigned short *Cb, long long ldc, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(deflate_coef_kernel, dim3((unsigned)((ldc + 255) / 256), n), dim3(256), 0, s, m, n, nsplit,
                       P, ldp, (long long)ldp * n, eps, T, Cb, ldc);
    return hipGetLastError();
}

}  // namespace acp
