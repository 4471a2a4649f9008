// Device helpers shared by the Krylov kernels (included by k_krylov.hip and
// k_mscg.hip only).
#pragma once
#include "acp_internal.h"

namespace acp {
namespace kry {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int NW = 8;             // waves per workgroup (2 per SIMD)
constexpr int NT = 64 * NW;       // threads per workgroup
constexpr int MAXNB = 16;         // up to 256 (padded) orbitals

__device__ __forceinline__ int wrap(int i, int n) {
    if (i < 0) i += n;
    if (i >= n) i -= n;
    return i;
}

// Neighbour rows of the 4-row group R..R+3 of one system, for the 8th-order
// stencil.  1D: rows R-4 .. R+7 (12 rows, periodic).  2D: for each of the 4 rows
// its 8 x-neighbours and 8 y-neighbours.  DIM = 3 is the 2D grid with n_x a
// multiple of 4, where the 4 rows of a group share one grid line: the x-window
// x-4 .. x+7 of that line (12 values) and the 8 y-neighbours of each row (32).
// Every index is clamped into [0, ng) so that all loads can be issued
// unconditionally (rows past the end of the grid in the last block are
// computed but never stored).
template <int DIM>
struct Nbr {
    static constexpr int N = DIM == 1 ? 12 : DIM == 3 ? 12 + 32 : 4 * 17;
    int idx[N];
    __device__ __forceinline__ Nbr(int R, const GridDesc &g) {
        if (DIM == 3) {
            const int r0 = R + 3 < g.ng ? R : g.ng - 4;   // whole group inside the grid
            const int ix = r0 % g.nx, iy = r0 / g.nx;
            const int line = iy * g.nx;
#pragma unroll
            for (int o = -4; o < 8; ++o) idx[4 + o] = line + wrap(ix + o, g.nx);
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int k = 1; k <= 4; ++k) {
                    idx[12 + 8 * j + (k - 1)] = wrap(iy + k, g.ny) * g.nx + ix + j;
                    idx[12 + 8 * j + 4 + (k - 1)] = wrap(iy - k, g.ny) * g.nx + ix + j;
                }
        } else if (DIM == 1) {
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                int rr = R - 4 + q;
                rr = rr < 0 ? rr + g.ng : rr;
                rr = rr >= g.ng ? rr - g.ng : rr;
                idx[q] = rr < g.ng ? rr : g.ng - 1;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int row = R + j;
                row = row < g.ng ? row : g.ng - 1;
                const int ix = row % g.nx, iy = row - ix;
                idx[17 * j] = row;
#pragma unroll
                for (int k = 1; k <= 4; ++k) {
                    idx[17 * j + k] = iy + wrap(ix + k, g.nx);
                    idx[17 * j + 4 + k] = iy + wrap(ix - k, g.nx);
                    const int iyk = iy / g.nx;
                    idx[17 * j + 8 + k] = wrap(iyk + k, g.ny) * g.nx + ix;
                    idx[17 * j + 12 + k] = wrap(iyk - k, g.ny) * g.nx + ix;
                }
            }
        }
    }
};

// y = (H - s) p at rows R..R+3 from gathered values w[] laid out as in Nbr.
template <int DIM>
__device__ __forceinline__ void stencil_from(const double (&w)[Nbr<DIM>::N], int R,
                                             const GridDesc &g, const double *__restrict__ V,
                                             double s, double (&y)[4], double (&pc)[4]) {
    const double c2 = -0.5 / (g.h * g.h);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int row = R + j;
        const bool ok = row < g.ng;
        const double v = V[ok ? row : g.ng - 1];
        double c, lap;
        if (DIM == 1) {
            c = w[4 + j];
            lap = fd8(0) * c;
#pragma unroll
            for (int k = 1; k <= 4; ++k) lap += fd8(k) * (w[4 + j + k] + w[4 + j - k]);
        } else if (DIM == 3) {
            c = w[4 + j];
            lap = 2.0 * fd8(0) * c;
#pragma unroll
            for (int k = 1; k <= 4; ++k)
                lap += fd8(k) * (w[4 + j + k] + w[4 + j - k] + w[12 + 8 * j + (k - 1)] + w[12 + 8 * j + 4 + (k - 1)]);
        } else {
            c = w[17 * j];
            lap = 2.0 * fd8(0) * c;
#pragma unroll
            for (int k = 1; k <= 4; ++k)
                lap += fd8(k) * (w[17 * j + k] + w[17 * j + 4 + k] + w[17 * j + 8 + k] + w[17 * j + 12 + k]);
        }
        pc[j] = ok ? c : 0.0;
        y[j] = ok ? (c2 * lap + (v - s) * c) : 0.0;
    }
}

// Sum over the threads of one column (threads t with t % 16 == col) of a
// per-thread value, in a fixed order; the total lands in red_out[col].
__device__ __forceinline__ void column_reduce(double v, double *red, double *red_out) {
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < kTile) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NT / kTile; ++k) s += red[threadIdx.x + kTile * k];
        red_out[threadIdx.x] = s;
    }
    __syncthreads();
}

// LDS slots for the cross-wave reduction of C = Phi^T y (at most 64 KB): the
// waves write their partial C in NW / N phases of N slots, so N divides NW.
template <int NB>
struct Slots {
    static constexpr int NEP = NB * 16;
    static constexpr int FIT = 512 / NEP;   // partials of NEP x 16 doubles in 64 KB
    static constexpr int N = FIT >= 8 ? 8 : FIT >= 4 ? 4 : FIT >= 2 ? 2 : 1;
    static constexpr int ELEMS = NEP * kTile;
    static_assert(NW % N == 0, "every wave has a slot in some phase");
};

// Pass 1 of the projected apply.  Each wave owns the 16-row blocks b = wave,
// wave + NW, ...; lane l (q = l/16) computes p and y = (H - s) p at the four
// consecutive rows 16 b + 4 q + j of system l % 16 and feeds y(row) to the
// MFMA k-step j, whose k index q stands for that row (the contraction runs
// over rows, so any row order works as long as the A operand follows it).
// C = Phi^T y is reduced across waves in LDS into slots[0] (orbital-major,
// 16 systems per orbital).  Returns this thread's share of p^T y.
template <int DIM, int NB, typename T>
__device__ __forceinline__ double apply_pass1(const T *__restrict__ rv, const T *__restrict__ pv,
                                              double beta, const KrylovArgsT<T> &a, double s,
                                              double *slots, T *__restrict__ pstore) {
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int col = lane & 15;
    const int q = lane >> 4;
    constexpr int nep = NB * 16;
    constexpr int NN = Nbr<DIM>::N;
    d4 acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = d4{0.0, 0.0, 0.0, 0.0};
    double pty = 0.0;
    for (int blk = wave; blk * 16 < a.g.ng; blk += NW) {
        const int R = blk * 16 + 4 * q;
        const Nbr<DIM> nb(R, a.g);
        // issue every load of the block before any use
        double w[NN], wp[NN];
#pragma unroll
        for (int k = 0; k < NN; ++k) w[k] = (double)rv[nb.idx[k] * kTile + col];
        if (pv) {
#pragma unroll
            for (int k = 0; k < NN; ++k) wp[k] = (double)pv[nb.idx[k] * kTile + col];
        }
        double av[4][NB];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int row = R + j < a.g.ng ? R + j : a.g.ng - 1;
            const T *ph = a.phi_rm + (long long)row * nep + col;
#pragma unroll
            for (int mb = 0; mb < NB; ++mb) av[j][mb] = (double)ph[mb * 16];
        }
        if (pv) {
#pragma unroll
            for (int k = 0; k < NN; ++k) w[k] += beta * wp[k];
        }
        double y[4], pc[4];
        stencil_from<DIM>(w, R, a.g, a.veff, s, y, pc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            pty += pc[j] * y[j];
            if (pstore && R + j < a.g.ng) pstore[(R + j) * kTile + col] = (T)pc[j];
        }
        // rows past the end contribute y = 0, so their (clamped) Phi rows are harmless
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int mb = 0; mb < NB; ++mb)
                acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j][mb], y[j], acc[mb], 0, 0, 0);
    }
    // deterministic cross-wave reduction: phases of Slots::N waves
    using S = Slots<NB>;
#pragma unroll 1
    for (int ph = 0; ph < NW / S::N; ++ph) {
        if (wave / S::N == ph) {
            double *dst = slots + (wave % S::N) * S::ELEMS;
#pragma unroll
            for (int mb = 0; mb < NB; ++mb)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int idx = (mb * 16 + q + 4 * e) * kTile + col;
                    if (ph == 0) dst[idx] = acc[mb][e];
                    else dst[idx] += acc[mb][e];
                }
        }
        __syncthreads();
    }
    for (int idx = t; idx < S::ELEMS; idx += NT) {
        double v = slots[idx];
#pragma unroll
        for (int k = 1; k < S::N; ++k) v += slots[k * S::ELEMS + idx];
        slots[idx] = v;
    }
    return pty;
}

// Pass 2 helper: for the 16-row block starting at row0, D = Phi(rows,:) C on
// the matrix cores.  The f64 MFMA returns D[l/16 + 4 e][l%16] to lane l, so the
// A operand feeds grid row 4 (m % 4) + m / 4 into MFMA row m: lane l then holds
// the consecutive grid rows row0 + 4*(l/16) + e of system l % 16.
template <int NB, typename T>
__device__ __forceinline__ d4 project_block(const T *__restrict__ phi_cm, int ng,
                                            const double *Cs, int row0) {
    const int lane = threadIdx.x & 63;
    constexpr int nep = NB * 16;
    const int m = lane & 15;
    int row = row0 + 4 * (m & 3) + (m >> 2);
    row = row < ng ? row : ng - 1;   // clamped rows feed outputs that are never stored
    const T *ph = phi_cm + row + (long long)(lane >> 4) * ng;
    double av[nep / 4];
#pragma unroll
    for (int k = 0; k < nep / 4; ++k) av[k] = (double)ph[(long long)(4 * k) * ng];
    d4 d = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < nep / 4; ++k) {
        const double bv = Cs[(4 * k + (lane >> 4)) * kTile + (lane & 15)];
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(av[k], bv, d, 0, 0, 0);
    }
    return d;
}

// Gather the stencil neighbourhood of rows R..R+3 of one system from v.
template <int DIM, typename T>
__device__ __forceinline__ void gather(const T *__restrict__ v, int R, const GridDesc &g,
                                       int col, double (&w)[Nbr<DIM>::N]) {
    const Nbr<DIM> nb(R, g);
#pragma unroll
    for (int k = 0; k < Nbr<DIM>::N; ++k) w[k] = (double)v[nb.idx[k] * kTile + col];
}


}  // namespace kry
}  // namespace acp
