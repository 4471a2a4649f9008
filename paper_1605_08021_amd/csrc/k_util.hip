// Grid operators and small device utilities.
//
//  * stencil (column-major): Y = c_lap Delta_h X + (c_v V + c_0 - shift_j) X with the
//    periodic 8th-order central Laplacian; used for H - shift (Eq. (2.5) on the
//    grid) and for v_c^{-1} = (eps0/4pi)(-Delta_h + kappa^2), the change of
//    variables B = v_hxc^{-1} G of Sec. 3.2.
//  * the real orthonormal Fourier basis and the symbol of v_c, which turn
//    v_c X into dense products on the matrix cores.
//  * conversions between column-major grid vectors and the 16-column
//    row-interleaved layout of the Krylov kernels, gathers, scatters and
//    deterministic reductions.
#include "acp_internal.h"

namespace acp {

namespace {

__global__ void stencil_kernel(int dim, int nx, int ny, int ng, int n, const double *__restrict__ X,
                               int ldx, double *__restrict__ Y, int ldy,
                               const double *__restrict__ V, double c_lap_h2, double c_v,
                               double c_0, const double *__restrict__ shift, const float *__restrict__ add,
                               long long ld_add) {
    int row = blockIdx.x * blockDim.x + threadIdx.x;
    int col = blockIdx.y;
    if (row >= ng || col >= n) return;
    const double *x = X + (long long)col * ldx;
    int ix = row % nx;
    int iy = row / nx;
    double lap = 0.0;
    double xc = x[row];
    // x direction
    {
        double s = fd8(0) * xc;  // c_0 x, once per axis
#pragma unroll
        for (int k = 1; k <= 4; ++k) {
            int ip = ix + k; if (ip >= nx) ip -= nx;
            int im = ix - k; if (im < 0) im += nx;
            s += fd8(k) * (x[iy * nx + ip] + x[iy * nx + im]);
        }
        lap += s;
    }
    if (dim == 2) {
        double s = fd8(0) * xc;
#pragma unroll
        for (int k = 1; k <= 4; ++k) {
            int jp = iy + k; if (jp >= ny) jp -= ny;
            int jm = iy - k; if (jm < 0) jm += ny;
            s += fd8(k) * (x[jp * nx + ix] + x[jm * nx + ix]);
        }
        lap += s;
    }
    double diag = c_0 - (shift ? shift[col] : 0.0);
    if (c_v != 0.0) diag += c_v * V[row];
    double y = c_lap_h2 * lap + diag * xc;
    if (add) y += (double)add[(long long)col * ld_add + row];
    Y[(long long)col * ldy + row] = y;
}

// 2D stencil through LDS: a block computes a 64 x 16 tile of one column
// (threads 64 x 4, four rows each) from the tile and its 4-point periodic halo
// staged in LDS (24 x 72 doubles), so that each input is read from memory about
// 1.7 times instead of 17.
constexpr int ST_TX = 64, ST_TY = 16, ST_LX = ST_TX + 8, ST_LY = ST_TY + 8;
// WRAP1: every halo index lies within one period of the grid (nx >= 68 and
// ny >= 20 for these tiles), so that one conditional add or subtract wraps it;
// otherwise the remainder is taken.
template <bool WRAP1>
__global__ __launch_bounds__(256) void stencil2d_tile_kernel(int nx, int ny, const double *__restrict__ X, int ldx,
                                                             double *__restrict__ Y, int ldy,
                                                             const double *__restrict__ V, double c_lap_h2,
                                                             double c_v, double c_0,
                                                             const double *__restrict__ shift,
                                                             const float *__restrict__ add, long long ld_add,
                                                             double *__restrict__ dot_part) {
    __shared__ double tile[ST_LY][ST_LX + 1];
    __shared__ double red[4];
    const int col = blockIdx.z;
    const int x0 = blockIdx.x * ST_TX, y0 = blockIdx.y * ST_TY;
    const double *x = X + (long long)col * ldx;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int ix = x0 + tx;
    // this thread's potential and correction, read before the barrier so that
    // the loads overlap the staging of the tile
    double vr[4];
    float ar[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int iy = y0 + ty + 4 * r;
        const bool in = ix < nx && iy < ny;
        const int row = iy * nx + ix;
        vr[r] = (in && c_v != 0.0) ? V[row] : 0.0;
        ar[r] = (in && add) ? add[(long long)col * ld_add + row] : 0.0f;
    }
    for (int idx = threadIdx.x; idx < ST_LY * ST_LX; idx += 256) {
        const int ly = idx / ST_LX, lx = idx - ly * ST_LX;
        int gx = x0 + lx - 4, gy = y0 + ly - 4;
        if (WRAP1) {
            gx += gx < 0 ? nx : (gx >= nx ? -nx : 0);
            gy += gy < 0 ? ny : (gy >= ny ? -ny : 0);
        } else {
            gx %= nx;
            gy %= ny;
            if (gx < 0) gx += nx;
            if (gy < 0) gy += ny;
        }
        tile[ly][lx] = x[gy * nx + gx];
    }
    __syncthreads();
    const double d0 = c_0 - (shift ? shift[col] : 0.0);
    double xy = 0.0;   // this thread's share of x.y over the tile
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ly = ty + 4 * r, iy = y0 + ly;
        if (ix >= nx || iy >= ny) break;
        const double xc = tile[ly + 4][tx + 4];
        double sx = fd8(0) * xc, sy = fd8(0) * xc;
#pragma unroll
        for (int k = 1; k <= 4; ++k) {
            sx += fd8(k) * (tile[ly + 4][tx + 4 + k] + tile[ly + 4][tx + 4 - k]);
            sy += fd8(k) * (tile[ly + 4 + k][tx + 4] + tile[ly + 4 - k][tx + 4]);
        }
        const int row = iy * nx + ix;
        const double y = c_lap_h2 * (sx + sy) + (d0 + c_v * vr[r]) * xc + (double)ar[r];
        Y[(long long)col * ldy + row] = y;
        xy += xc * y;
    }
    if (dot_part) {   // the tile's x.y: butterfly within each wave, then the 4 waves in order
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) xy += __shfl_xor(xy, o, 64);
        if (tx == 0) red[ty] = xy;
        __syncthreads();
        if (threadIdx.x == 0)
            dot_part[(long long)col * gridDim.x * gridDim.y + blockIdx.y * gridDim.x + blockIdx.x] =
                (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// out[j] = sum_t part[j m + t] (fixed order), one block per column.
__global__ __launch_bounds__(256) void col_sum_kernel(int m, const double *part, double *out) {
    __shared__ double red[256];
    const double *pc = part + (long long)blockIdx.x * m;
    double acc = 0.0;
    for (int t = threadIdx.x; t < m; t += 256) acc += pc[t];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ void scale_copy_kernel(int m, int n, double alpha, const double *X, int ldx, double *Y,
                                  int ldy) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)m * n) return;
    int i = (int)(idx % m);
    long long j = idx / m;
    Y[i + j * ldy] = alpha * X[i + j * ldx];
}

__global__ void gather_rows_kernel(int nsel, int n, const int *sel, const double *X, int ldx,
                                   double *Y, int ldy) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)nsel * n) return;
    int i = (int)(idx % nsel);
    long long j = idx / nsel;
    Y[i + j * ldy] = X[sel[i] + j * ldx];
}

__global__ void scatter_identity_kernel(int nsel, const int *sel, double *Xi, int ld) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)nsel * nsel) return;
    int k = (int)(idx % nsel);      // row index in sel
    long long j = idx / nsel;       // column
    Xi[sel[k] + j * ld] = (k == j) ? 1.0 : 0.0;
}

__global__ void add_identity_neg_kernel(int n, double *T, int ld) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * n) return;
    int i = (int)(idx % n);
    long long j = idx / n;
    double *p = T + i + j * ld;
    *p = ((i == j) ? 1.0 : 0.0) - *p;
}

// One block per column; fixed-order tree reduction (deterministic).
__global__ void col_sqnorm_kernel(int m, const double *X, int ldx, double *out) {
    __shared__ double red[256];
    const double *x = X + (long long)blockIdx.x * ldx;
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) s += x[i] * x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// One block per column: out[j] = X(:,j) . Y(:,j) (deterministic).
__global__ void col_dot_kernel(int m, const double *X, int ldx, const double *Y, int ldy, double *out) {
    __shared__ double red[256];
    const double *x = X + (long long)blockIdx.x * ldx;
    const double *y = Y + (long long)blockIdx.x * ldy;
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) s += x[i] * y[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Y(:,j) = a[j] X(:,j) + b[j] Y(:,j); a null means 1, b null means 1.
__global__ void col_axpby_kernel(int m, int n, const double *__restrict__ a, const double *X, int ldx,
                                 const double *__restrict__ b, double *Y, int ldy) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)m * n) return;
    const int j = (int)(i / m), r = (int)(i % m);
    const double av = a ? a[j] : 1.0, bv = b ? b[j] : 1.0;
    double *y = Y + (long long)j * ldy + r;
    *y = av * X[(long long)j * ldx + r] + bv * *y;
}

// dst(:, i) = src(:, idx[i]), i < n.
__global__ void col_gather_kernel(int m, int n, const double *__restrict__ src, int lds,
                                  const int *__restrict__ idx, double *dst, int ldd) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)m * n) return;
    const int j = (int)(i / m), r = (int)(i % m);
    dst[(long long)j * ldd + r] = src[(long long)idx[j] * lds + r];
}

// Y(:, idx[i]) += a[i] X(:, i), i < n (the idx[i] distinct).
__global__ void col_axpy_scatter_kernel(int m, int n, const double *__restrict__ a, const double *X, int ldx,
                                        const int *__restrict__ idx, double *Y, int ldy) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)m * n) return;
    const int j = (int)(i / m), r = (int)(i % m);
    Y[(long long)idx[j] * ldy + r] += a[j] * X[(long long)j * ldx + r];
}

// One block per column: out[j] = ||X(:,j) - Y(:,j)||^2 (deterministic).
__global__ void col_diff_sqnorm_kernel(int m, const double *X, int ldx, const double *Y, int ldy,
                                       double *out) {
    __shared__ double red[256];
    const double *x = X + (long long)blockIdx.x * ldx;
    const double *y = Y + (long long)blockIdx.x * ldy;
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) {
        double d = x[i] - y[i];
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ void axpby_kernel(int m, int n, double a, const double *X, int ldx, double b, double *Y,
                             int ldy) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)m * n) return;
    int i = (int)(idx % m);
    long long j = idx / m;
    Y[i + j * ldy] = a * X[i + j * ldx] + b * Y[i + j * ldy];
}

// Bc(i, mu) = L(i) * phi(sel[mu], i): the N_e x N_mu factor diag(L_c) Phi(Pi,:)^T of Eq. (3.7).
__global__ void weighted_rows_kernel(int ne, int nmu, const double *L, const int *sel,
                                     const double *phi, int ldphi, double *Bc) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)ne * nmu) return;
    int i = (int)(idx % ne);
    long long mu = idx / ne;
    Bc[i + mu * ne] = L[i] * phi[sel[mu] + (long long)i * ldphi];
}

// max |G - I| of a n x n matrix (single block).
__global__ void max_dev_identity_kernel(int n, const double *G, double *out) {
    __shared__ double red[256];
    double m = 0.0;
    for (long long idx = threadIdx.x; idx < (long long)n * n; idx += 256) {
        int i = (int)(idx % n);
        long long j = idx / n;
        double v = fabs(G[idx] - ((i == j) ? 1.0 : 0.0));
        m = fmax(m, v);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// Column-major (ld = ldx) -> 16-column row-interleaved tiles; padded columns are zero.
// Block: 16 columns x 64 rows through LDS.
// Column-major -> 16-column tiles; TO = double, or float for the inner solves of
// the mixed-precision form; colscale (optional) multiplies each column.
template <typename TO>
__global__ void to_tiled_kernel(int ng, int ncols, const double *__restrict__ X, int ldx,
                                const double *__restrict__ colscale, TO *__restrict__ T) {
    __shared__ double buf[kTile][65];
    const int tile = blockIdx.y;
    const int r0 = blockIdx.x * 64;
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int r = t & 63, c = (t >> 6) + 4 * q;
        int gr = r0 + r, gc = tile * kTile + c;
        double v = 0.0;
        if (gr < ng && gc < ncols) v = X[gr + (long long)gc * ldx] * (colscale ? colscale[gc] : 1.0);
        buf[c][r] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int c = t & 15, r = (t >> 4) + 16 * q;
        int gr = r0 + r;
        if (gr < ng) T[((long long)tile * ng + gr) * kTile + c] = (TO)buf[c][r];
    }
}

// 16-column tiles -> column-major; ADD accumulates into X.
template <bool ADD>
__global__ void from_tiled_kernel(int ng, int ncols, const double *__restrict__ T,
                                  double *__restrict__ X, int ldx) {
    __shared__ double buf[kTile][65];
    const int tile = blockIdx.y;
    const int r0 = blockIdx.x * 64;
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int c = t & 15, r = (t >> 4) + 16 * q;
        int gr = r0 + r;
        buf[c][r] = (gr < ng) ? T[((long long)tile * ng + gr) * kTile + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int r = t & 63, c = (t >> 6) + 4 * q;
        int gr = r0 + r, gc = tile * kTile + c;
        if (gr < ng && gc < ncols) {
            if (ADD) X[gr + (long long)gc * ldx] += buf[c][r];
            else X[gr + (long long)gc * ldx] = buf[c][r];
        }
    }
}

// Rows Pi of a translation-invariant (periodic) operator with first column g:
// K(mu, a) = g(x(Pi_mu) - x(a), y(Pi_mu) - y(a)) (indices mod the grid),
// K column-major with leading dimension nsel.
__global__ void circulant_rows_kernel(int nsel, const int *__restrict__ sel, int nx, int ny,
                                      const double *__restrict__ g, double *__restrict__ K) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long ng = (long long)nx * ny;
    if (i >= (long long)nsel * ng) return;
    const int mu = (int)(i % nsel);
    const long long a = i / nsel;
    const int p = sel[mu];
    const int ax = (int)(a % nx), ay = (int)(a / nx);
    const int px = p % nx, py = p / nx;
    int dx = px - ax, dy = py - ay;
    if (dx < 0) dx += nx;
    if (dy < 0) dy += ny;
    K[i] = g[(long long)dy * nx + dx];
}

__global__ void to_f32_kernel(long long n, const double *__restrict__ X, float *__restrict__ Y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) Y[i] = (float)X[i];
}

// Real orthonormal Fourier basis of R^n: column 0 constant, columns 2k-1 / 2k
// cos / sin of frequency k, and for even n the alternating column last.
__device__ int mode_freq(int c, int n) {
    if (c == 0) return 0;
    if ((n % 2 == 0) && c == n - 1) return n / 2;
    return (c + 1) / 2;
}

__global__ void fourier_basis_kernel(int n, double *F) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)n * n) return;
    int j = (int)(idx % n);     // grid point
    int c = (int)(idx / n);     // basis column
    double v;
    if (c == 0) {
        v = 1.0 / sqrt((double)n);
    } else if ((n % 2 == 0) && c == n - 1) {
        v = ((j & 1) ? -1.0 : 1.0) / sqrt((double)n);
    } else {
        int k = (c + 1) / 2;
        long long kj = ((long long)k * j) % n;
        double arg = 2.0 * (double)kj / (double)n;   // in units of pi
        v = sqrt(2.0 / n) * ((c & 1) ? cospi(arg) : sinpi(arg));
    }
    F[idx] = v;
}

__device__ double neg_lap_symbol(int k, int n, double h) {
    double s = -fd8(0);
#pragma unroll
    for (int q = 1; q <= 4; ++q) {
        long long kq = ((long long)k * q) % n;
        s -= 2.0 * fd8(q) * cospi(2.0 * (double)kq / (double)n);
    }
    return s / (h * h);
}

__global__ void fourier_symbol_kernel(int nx, int ny, double h, double kappa, double eps0,
                                      double *S) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nx * ny) return;
    int cx = idx % nx, cy = idx / nx;
    double lam = neg_lap_symbol(mode_freq(cx, nx), nx, h);
    if (ny > 1) lam += neg_lap_symbol(mode_freq(cy, ny), ny, h);
    S[idx] = (4.0 * M_PI / eps0) / (lam + kappa * kappa);
}

__global__ void mul_symbol_kernel(int ng, long long tot, const double *S, double *X) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= tot) return;
    X[idx] *= S[idx % ng];
}

// B = A^T (A m x n, B n x m), 32 x 32 tiles through LDS.
__global__ void transpose_kernel(int m, int n, const double *A, int lda, double *B, int ldb) {
    __shared__ double tileb[32][33];
    int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
    for (int k = ty; k < 32; k += 8) {
        int i = bx + tx, j = by + k;
        tileb[k][tx] = (i < m && j < n) ? A[i + (long long)j * lda] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        int j = by + tx, i = bx + k;
        if (i < m && j < n) B[j + (long long)i * ldb] = tileb[tx][k];
    }
}

__global__ void fill_u32_kernel(unsigned *p, size_t n, unsigned v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned nblk(long long tot, int b) { return (unsigned)((tot + b - 1) / b); }


// Columns of tile-interleaved vectors (tile-major, then row, then the 16
// columns of the tile): destination column m (tile m / 16, position m % 16) of
// each of the gridDim.y vectors takes source column map[m]; a negative entry
// writes zero (zero_missing) or leaves the destination column as it is.
template <typename T>
__global__ void tilecol_gather_kernel(int rows, int ncols, const int *map, const T *src,
                                      long long src_vstride, T *dst, long long dst_vstride,
                                      int zero_missing) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)rows * ncols) return;
    const int pos = (int)(idx & 15);
    const long long rest = idx >> 4;
    const int row = (int)(rest % rows);
    const long long tile = rest / rows;
    const long long ts = (long long)rows * 16;
    const int sm = map[tile * 16 + pos];
    T *d = dst + (long long)blockIdx.y * dst_vstride + tile * ts + (long long)row * 16 + pos;
    if (sm < 0) {
        if (zero_missing) *d = (T)0;
        return;
    }
    *d = src[(long long)blockIdx.y * src_vstride + (long long)(sm >> 4) * ts + (long long)row * 16 + (sm & 15)];
}

}  // namespace

// Fills by kernel rather than hipMemsetAsync, so that they may be recorded in a graph.
hipError_t launch_fill_u32(unsigned *p, size_t n, unsigned v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(nblk((long long)n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *p, size_t n, int v, hipStream_t s) {
    return launch_fill_u32((unsigned *)p, n, (unsigned)v, s);
}

hipError_t launch_transpose(int m, int n, const double *A, int lda, double *B, int ldb,
                            hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid(nblk(m, 32), nblk(n, 32));
    hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, s, m, n, A, lda, B, ldb);
    return hipGetLastError();
}

size_t stencil_dot_work_doubles(const GridDesc &g, int n) {
    return g.dim == 2 ? (size_t)nblk(g.nx, ST_TX) * nblk(g.ny, ST_TY) * n : 0;
}

hipError_t launch_stencil(const GridDesc &g, int n, const double *X, int ldx, double *Y, int ldy,
                          const double *V, double c_lap, double c_v, double c_0,
                          const double *shift_dev, hipStream_t s, const float *add, long long ld_add,
                          double *dot, double *dot_work) {
    if (n <= 0) return hipSuccess;
    if (dot && g.dim != 2) return hipErrorInvalidValue;
    if (g.dim == 2) {
        const int tiles = (int)(nblk(g.nx, ST_TX) * nblk(g.ny, ST_TY));
        for (int c0 = 0; c0 < n; c0 += 65535) {   // columns in grid z
            const int nc = std::min(65535, n - c0);
            dim3 grid(nblk(g.nx, ST_TX), nblk(g.ny, ST_TY), nc);
            const bool wrap1 = g.nx >= ST_TX + 4 && g.ny >= ST_TY + 4;
            hipLaunchKernelGGL(wrap1 ? stencil2d_tile_kernel<true> : stencil2d_tile_kernel<false>, grid, dim3(256),
                               0, s, g.nx, g.ny, X + (long long)c0 * ldx,
                               ldx, Y + (long long)c0 * ldy, ldy, V, c_lap / (g.h * g.h), c_v, c_0,
                               shift_dev ? shift_dev + c0 : nullptr, add ? add + (long long)c0 * ld_add : nullptr,
                               ld_add, dot ? dot_work + (long long)c0 * tiles : nullptr);
        }
        if (dot) hipLaunchKernelGGL(col_sum_kernel, dim3(n), dim3(256), 0, s, tiles, dot_work, dot);
        return hipGetLastError();
    }
    dim3 grid(nblk(g.ng, 256), n);
    hipLaunchKernelGGL(stencil_kernel, grid, dim3(256), 0, s, g.dim, g.nx, g.ny, g.ng, n, X, ldx,
                       Y, ldy, V, c_lap / (g.h * g.h), c_v, c_0, shift_dev, add, ld_add);
    return hipGetLastError();
}

hipError_t launch_scale_copy(int m, int n, double alpha, const double *X, int ldx, double *Y,
                             int ldy, hipStream_t s) {
    long long tot = (long long)m * n;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(scale_copy_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, m, n, alpha, X,
                       ldx, Y, ldy);
    return hipGetLastError();
}

hipError_t launch_gather_rows(int nsel, int n, const int *sel, const double *X, int ldx, double *Y,
                              int ldy, hipStream_t s) {
    long long tot = (long long)nsel * n;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, nsel, n, sel, X,
                       ldx, Y, ldy);
    return hipGetLastError();
}

hipError_t launch_scatter_identity(int nsel, const int *sel, double *Xi, int ld, hipStream_t s) {
    long long tot = (long long)nsel * nsel;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_identity_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, nsel, sel,
                       Xi, ld);
    return hipGetLastError();
}

hipError_t launch_add_identity_neg(int n, double *T, int ld, hipStream_t s) {
    long long tot = (long long)n * n;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(add_identity_neg_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, n, T, ld);
    return hipGetLastError();
}

hipError_t launch_col_sqnorm(int m, int n, const double *X, int ldx, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(col_sqnorm_kernel, dim3(n), dim3(256), 0, s, m, X, ldx, out);
    return hipGetLastError();
}

hipError_t launch_col_dot(int m, int n, const double *X, int ldx, const double *Y, int ldy,
                          double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(col_dot_kernel, dim3(n), dim3(256), 0, s, m, X, ldx, Y, ldy, out);
    return hipGetLastError();
}

hipError_t launch_col_axpby(int m, int n, const double *a, const double *X, int ldx, const double *b,
                            double *Y, int ldy, hipStream_t s) {
    const long long tot = (long long)m * n;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(col_axpby_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, m, n, a, X, ldx, b, Y, ldy);
    return hipGetLastError();
}

template <typename T>
static hipError_t tilecol_gather(int rows, int ncols, const int *map, const T *src, long long svs, T *dst,
                                 long long dvs, int nvec, bool zero_missing, hipStream_t s) {
    const long long tot = (long long)rows * ncols;
    if (tot <= 0 || nvec <= 0) return hipSuccess;
    hipLaunchKernelGGL(tilecol_gather_kernel<T>, dim3(nblk(tot, 256), nvec), dim3(256), 0, s, rows, ncols, map,
                       src, svs, dst, dvs, zero_missing ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_tilecol_gather(int rows, int ncols, const int *map, const double *src, long long svs,
                                 double *dst, long long dvs, int nvec, bool zero_missing, hipStream_t s) {
    return tilecol_gather(rows, ncols, map, src, svs, dst, dvs, nvec, zero_missing, s);
}

hipError_t launch_tilecol_gather(int rows, int ncols, const int *map, const float *src, long long svs,
                                 float *dst, long long dvs, int nvec, bool zero_missing, hipStream_t s) {
    return tilecol_gather(rows, ncols, map, src, svs, dst, dvs, nvec, zero_missing, s);
}

hipError_t launch_col_gather(int m, int n, const double *src, int lds, const int *idx, double *dst, int ldd,
                             hipStream_t s) {
    const long long tot = (long long)m * n;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(col_gather_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, m, n, src, lds, idx, dst, ldd);
    return hipGetLastError();
}

hipError_t launch_col_axpy_scatter(int m, int n, const double *a, const double *X, int ldx, const int *idx,
                                   double *Y, int ldy, hipStream_t s) {
    const long long tot = (long long)m * n;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(col_axpy_scatter_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, m, n, a, X, ldx, idx, Y,
                       ldy);
    return hipGetLastError();
}

hipError_t launch_col_diff_sqnorm(int m, int n, const double *X, int ldx, const double *Y,
                                  int ldy, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(col_diff_sqnorm_kernel, dim3(n), dim3(256), 0, s, m, X, ldx, Y, ldy, out);
    return hipGetLastError();
}

hipError_t launch_axpby(int m, int n, double a, const double *X, int ldx, double b, double *Y,
                        int ldy, hipStream_t s) {
    long long tot = (long long)m * n;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(axpby_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, m, n, a, X, ldx, b, Y,
                       ldy);
    return hipGetLastError();
}

hipError_t launch_weighted_rows(int ne, int nmu, const double *L, const int *sel,
                                const double *phi, int ldphi, double *Bc, hipStream_t s) {
    long long tot = (long long)ne * nmu;
    hipLaunchKernelGGL(weighted_rows_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, ne, nmu, L,
                       sel, phi, ldphi, Bc);
    return hipGetLastError();
}

hipError_t launch_gram_check(int n, int /*unused*/, const double *G, double *maxdev,
                             hipStream_t s) {
    hipLaunchKernelGGL(max_dev_identity_kernel, dim3(1), dim3(256), 0, s, n, G, maxdev);
    return hipGetLastError();
}

hipError_t launch_to_tiled(int ng, int ncols, int ncols_pad, const double *X, int ldx, double *T,
                           hipStream_t s) {
    dim3 grid(nblk(ng, 64), ncols_pad / kTile);
    hipLaunchKernelGGL(to_tiled_kernel<double>, grid, dim3(256), 0, s, ng, ncols, X, ldx,
                       (const double *)nullptr, T);
    return hipGetLastError();
}

hipError_t launch_to_tiled_f32(int ng, int ncols, int ncols_pad, const double *X, int ldx,
                               const double *colscale, float *T, hipStream_t s) {
    dim3 grid(nblk(ng, 64), ncols_pad / kTile);
    hipLaunchKernelGGL(to_tiled_kernel<float>, grid, dim3(256), 0, s, ng, ncols, X, ldx, colscale, T);
    return hipGetLastError();
}

hipError_t launch_from_tiled(int ng, int ncols, const double *T, double *X, int ldx,
                             hipStream_t s) {
    dim3 grid(nblk(ng, 64), (ncols + kTile - 1) / kTile);
    hipLaunchKernelGGL(from_tiled_kernel<false>, grid, dim3(256), 0, s, ng, ncols, T, X, ldx);
    return hipGetLastError();
}

hipError_t launch_from_tiled_add(int ng, int ncols, const double *T, double *X, int ldx,
                                 hipStream_t s) {
    dim3 grid(nblk(ng, 64), (ncols + kTile - 1) / kTile);
    hipLaunchKernelGGL(from_tiled_kernel<true>, grid, dim3(256), 0, s, ng, ncols, T, X, ldx);
    return hipGetLastError();
}

hipError_t launch_circulant_rows(int nsel, const int *sel, int nx, int ny, const double *g, double *K,
                                 hipStream_t s) {
    const long long tot = (long long)nsel * nx * ny;
    hipLaunchKernelGGL(circulant_rows_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, nsel, sel, nx, ny, g, K);
    return hipGetLastError();
}

hipError_t launch_to_f32(size_t n, const double *X, float *Y, hipStream_t s) {
    hipLaunchKernelGGL(to_f32_kernel, dim3(nblk((long long)n, 256)), dim3(256), 0, s, (long long)n, X, Y);
    return hipGetLastError();
}

hipError_t launch_fourier_basis(int n, double *F, hipStream_t s) {
    long long tot = (long long)n * n;
    hipLaunchKernelGGL(fourier_basis_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, n, F);
    return hipGetLastError();
}

hipError_t launch_fourier_symbol(const GridDesc &g, double kappa, double eps0, double *S,
                                 hipStream_t s) {
    hipLaunchKernelGGL(fourier_symbol_kernel, dim3(nblk(g.ng, 256)), dim3(256), 0, s, g.nx, g.ny,
                       g.h, kappa, eps0, S);
    return hipGetLastError();
}

hipError_t launch_mul_symbol(int ng, int n, const double *S, double *X, hipStream_t s) {
    long long tot = (long long)ng * n;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(mul_symbol_kernel, dim3(nblk(tot, 256)), dim3(256), 0, s, ng, tot, S, X);
    return hipGetLastError();
}

namespace {
// One thread per frequency point; the modes' frequencies staged in LDS.
__global__ void phonon_dos_kernel(const double *omega2, int n, double scale, double inv2s2, const double *w, int nw,
                                  double *dos) {
    __shared__ double wk[256];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const double x = p < nw ? w[p] : 0.0;
    double acc = 0.0;
    for (int k0 = 0; k0 < n; k0 += 256) {
        __syncthreads();
        if (k0 + (int)threadIdx.x < n) {
            const double l = omega2[k0 + threadIdx.x];
            wk[threadIdx.x] = l < 0.0 ? -sqrt(-l) : sqrt(l);
        }
        __syncthreads();
        const int m = min(256, n - k0);
        for (int k = 0; k < m; ++k) {
            const double d = x - wk[k];
            acc += exp(-d * d * inv2s2);
        }
    }
    if (p < nw) dos[p] = scale * acc;
}
}  // namespace

hipError_t launch_phonon_dos(const double *omega2, int n, int n_modes, double sigma, const double *w, int nw,
                             double *dos, hipStream_t s) {
    if (nw <= 0) return hipSuccess;
    const double scale = 1.0 / (n_modes * sqrt(2.0 * M_PI * sigma * sigma));
    hipLaunchKernelGGL(phonon_dos_kernel, dim3(nblk(nw, 256)), dim3(256), 0, s, omega2, n, scale,
                       1.0 / (2.0 * sigma * sigma), w, nw, dos);
    return hipGetLastError();
}

}  // namespace acp
