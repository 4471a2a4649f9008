// The learned preconditioner's network on the matrix cores (BF16 operands, FP32
// accumulation): four periodic convolutions of width 5 per grid axis, channels
// 2 -> 32 -> 32 -> 32 -> 1, ReLU after the first three.  A convolution
//   out[co, a] = b[co] + sum_ci sum_t W[co, ci, t] in[ci, a + off(t)]
// is an implicit GEMM over k = ci * T + t (T = 5 taps in 1D, 25 in 2D):
// D(co, position) += W(co, k) * im2col(k, position).
//
// Layouts: activations [sample][channel][grid point] in BF16; forward weights
// [cout][KP] in BF16 with KP = T cin rounded up to 16 (zero padded); the
// network's parameters theta in FP32 as [cout][cin][taps] then [cout] per
// layer (the ABI weight format).
//
// One workgroup (4 waves) computes a tile of 128 grid points (1D: 128
// consecutive points; 2D: 8 rows x 16 columns) for one sample and every output
// channel.  The input tile and its halo of 2 (periodic wrap) and the weights are
// staged in LDS; each wave owns 32 points (two 16-point MFMA column blocks) and
// all output channels (one or two 16-channel row blocks) and walks k in steps
// of 16 with v_mfma_f32_16x16x16bf16_1k:
//   A (weights): lane l holds W(16 mb + l % 16, k0 + 4 (l / 16) + e), e < 4;
//   B (im2col):  lane l holds im2col(k0 + 4 (l / 16) + e, 16 nb + l % 16);
//   D: lane l, register e holds D(16 mb + 4 (l / 16) + e, 16 nb + l % 16).
// The same kernel computes the data gradient of a layer (the adjoint of a
// periodic correlation is the correlation with the flipped kernel, channels
// swapped) with the ReLU mask of the layer below applied in the epilogue.
// Weight gradients are a second implicit GEMM, contracting over grid points:
// dW(co, k) = sum_samples sum_points g(co, point) im2col(k, point).
#include "acp_internal.h"

namespace acp {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NNT = 256;        // threads per workgroup (4 waves)
constexpr int TP = 128;         // grid points per tile

__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ __forceinline__ unsigned short f2bf(float f) {
    // round to nearest even (finite values)
    const unsigned u = __float_as_uint(f);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

template <int DIM>
struct Geom {
    static constexpr int T = DIM == 1 ? 5 : 25;        // taps
    static constexpr int TY = DIM == 1 ? 1 : 8;        // tile rows
    static constexpr int TX = DIM == 1 ? 128 : 16;     // tile columns
    static constexpr int HY = DIM == 1 ? 1 : TY + 4;   // staged rows (with halo)
    static constexpr int HX = TX + 4;                  // staged columns (with halo)
    static __device__ __forceinline__ int dy(int t) { return DIM == 1 ? 0 : t / 5 - 2; }
    static __device__ __forceinline__ int dx(int t) { return DIM == 1 ? t - 2 : t % 5 - 2; }
};

__device__ __forceinline__ int wrapi(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// Stage channels [0, C) of one sample's tile at (y0, x0) with a halo of 2 into
// lds[C][HY][HX] (BF16, periodic wrap).
template <int DIM, int C>
__device__ __forceinline__ void stage_tile(const unsigned short *__restrict__ src, int nx, int ny,
                                           int y0, int x0, unsigned short *lds) {
    using G = Geom<DIM>;
    const long long n = (long long)nx * ny;
    for (int i = threadIdx.x; i < C * G::HY * G::HX; i += NNT) {
        const int c = i / (G::HY * G::HX);
        const int rem = i % (G::HY * G::HX);
        const int jy = rem / G::HX, jx = rem % G::HX;
        const int gy = DIM == 1 ? 0 : wrapi(y0 - 2 + jy, ny);
        const int gx = wrapi(x0 - 2 + jx, nx);
        lds[i] = src[(long long)c * n + (long long)gy * nx + gx];
    }
}

// im2col value for k = ci * T + t at tile point p (clamped for padded k).
template <int DIM, int C>
__device__ __forceinline__ unsigned short im2col(const unsigned short *lds, int k, int p) {
    using G = Geom<DIM>;
    int ci = k / G::T;
    const int t = k - ci * G::T;
    ci = ci < C ? ci : C - 1;   // padded k: any finite value (its weight is zero)
    const int py = DIM == 1 ? 0 : p / G::TX, px = DIM == 1 ? p : p % G::TX;
    return lds[(ci * G::HY + py + (DIM == 1 ? 0 : 2 + G::dy(t))) * G::HX + px + 2 + G::dx(t)];
}

enum { MODE_RELU_BF16 = 0, MODE_LINEAR_F32 = 1, MODE_MASK_BF16 = 2 };

struct ConvArgs {
    int nx, ny;                     // grid (ny = 1 in 1D)
    const unsigned short *in;       // [B][CIN][N]
    const unsigned short *w;        // [COUT][KP]
    const float *bias;              // [COUT] (forward modes)
    void *out;                      // [B][COUT][N], BF16 or FP32
    const unsigned short *mask;     // [B][COUT][N] (MODE_MASK_BF16): keep where mask > 0
};

template <int DIM, int CIN, int COUT, int MODE>
__global__ __launch_bounds__(NNT) void conv_kernel(ConvArgs a) {
    using G = Geom<DIM>;
    constexpr int K = CIN * G::T;
    constexpr int KP = (K + 15) / 16 * 16;
    constexpr int MB = (COUT + 15) / 16;
    __shared__ unsigned short s_in[CIN * G::HY * G::HX];
    __shared__ __align__(16) unsigned short s_w[MB * 16 * KP];
    const int b = blockIdx.y;
    const int ntx = (a.nx + G::TX - 1) / G::TX;
    const int y0 = (blockIdx.x / ntx) * G::TY, x0 = (blockIdx.x % ntx) * G::TX;
    const long long n = (long long)a.nx * a.ny;
    stage_tile<DIM, CIN>(a.in + (long long)b * CIN * n, a.nx, a.ny, y0, x0, s_in);
    for (int i = threadIdx.x; i < MB * 16 * KP; i += NNT)
        s_w[i] = (i / KP) < COUT ? a.w[i] : (unsigned short)0;
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, r16 = lane & 15;
    f4 acc[MB][2];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < KP; k0 += 16) {
        s4 av[MB], bv[2];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const unsigned short *wp = s_w + (mb * 16 + r16) * KP + k0 + 4 * q;
#pragma unroll
            for (int e = 0; e < 4; ++e) av[mb][e] = (short)wp[e];
        }
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            const int p = (2 * wave + nb) * 16 + r16;
#pragma unroll
            for (int e = 0; e < 4; ++e) bv[nb][e] = (short)im2col<DIM, CIN>(s_in, k0 + 4 * q + e, p);
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[mb], bv[nb], acc[mb][nb], 0, 0, 0);
    }
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        const int p = (2 * wave + nb) * 16 + r16;
        const int gy = y0 + (DIM == 1 ? 0 : p / G::TX), gx = x0 + (DIM == 1 ? p : p % G::TX);
        if (gy >= a.ny || gx >= a.nx) continue;
        const long long pos = (long long)gy * a.nx + gx;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int co = mb * 16 + 4 * q + e;
                if (co >= COUT) continue;
                const long long o = ((long long)b * COUT + co) * n + pos;
                float v = acc[mb][nb][e];
                if (MODE == MODE_RELU_BF16) {
                    v += a.bias[co];
                    ((unsigned short *)a.out)[o] = f2bf(v > 0.f ? v : 0.f);
                } else if (MODE == MODE_LINEAR_F32) {
                    ((float *)a.out)[o] = v + a.bias[co];
                } else {
                    ((unsigned short *)a.out)[o] = bf2f(a.mask[o]) > 0.f ? f2bf(v) : (unsigned short)0;
                }
            }
    }
}

struct WgradArgs {
    int nx, ny, B;
    const unsigned short *g;        // [B][COUT][N] gradient w.r.t. the layer's output
    const unsigned short *act;      // [B][CIN][N] the layer's input
    float *part;                    // [groups][COUT][K]
    float *bpart;                   // [groups][COUT]
    int items_per_group;            // (sample, tile) items per workgroup
};

// dW partials: workgroup (x = group, y = chunk of 16-wide k blocks) accumulates
// over its (sample, tile) items; the four waves' partials are summed in LDS in
// wave order, and the group's partial is written for a fixed-order reduction.
constexpr int WG_NBC = 10;      // k blocks per workgroup chunk

template <int DIM, int CIN, int COUT>
__global__ __launch_bounds__(NNT) void wgrad_kernel(WgradArgs a) {
    using G = Geom<DIM>;
    constexpr int K = CIN * G::T;
    constexpr int NBK = (K + 15) / 16;
    constexpr int MB = (COUT + 15) / 16;
    __shared__ unsigned short s_act[CIN * G::HY * G::HX];
    __shared__ __align__(16) unsigned short s_g[MB * 16 * TP];
    __shared__ float s_red[MB * 16 * WG_NBC * 16];
    __shared__ float s_bias[4][MB * 16];
    const int ntx = (a.nx + G::TX - 1) / G::TX, nty = (a.ny + G::TY - 1) / G::TY;
    const int tiles = ntx * nty;
    const long long n = (long long)a.nx * a.ny;
    const int kb0 = blockIdx.y * WG_NBC;
    const int nbc = NBK - kb0 < WG_NBC ? NBK - kb0 : WG_NBC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, r16 = lane & 15;
    f4 acc[MB][WG_NBC];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int j = 0; j < WG_NBC; ++j) acc[mb][j] = f4{0.f, 0.f, 0.f, 0.f};
    float bsum[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) bsum[mb] = 0.f;
    const int it0 = blockIdx.x * a.items_per_group;
    const int it1 = min(it0 + a.items_per_group, a.B * tiles);
    for (int it = it0; it < it1; ++it) {
        const int b = it / tiles, tile = it % tiles;
        const int y0 = (tile / ntx) * G::TY, x0 = (tile % ntx) * G::TX;
        __syncthreads();   // the previous item's LDS reads are done
        stage_tile<DIM, CIN>(a.act + (long long)b * CIN * n, a.nx, a.ny, y0, x0, s_act);
        for (int i = threadIdx.x; i < MB * 16 * TP; i += NNT) {
            const int co = i / TP, p = i % TP;
            const int gy = y0 + (DIM == 1 ? 0 : p / G::TX), gx = x0 + (DIM == 1 ? p : p % G::TX);
            unsigned short v = 0;
            if (co < COUT && gy < a.ny && gx < a.nx)
                v = a.g[((long long)b * COUT + co) * n + (long long)gy * a.nx + gx];
            s_g[i] = v;
        }
        __syncthreads();
        // this wave's 32 points: two k-steps of 16 points
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int pbase = (2 * wave + ks) * 16;
            s4 av[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const unsigned short *gp = s_g + (mb * 16 + r16) * TP + pbase + 4 * q;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    av[mb][e] = (short)gp[e];
                    if (blockIdx.y == 0) bsum[mb] += bf2f(gp[e]);
                }
            }
#pragma unroll
            for (int j = 0; j < WG_NBC; ++j) {
                if (j < nbc) {
                    s4 bv;
                    const int k = (kb0 + j) * 16 + r16;
#pragma unroll
                    for (int e = 0; e < 4; ++e) bv[e] = (short)im2col<DIM, CIN>(s_act, k, pbase + 4 * q + e);
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
                        acc[mb][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[mb], bv, acc[mb][j], 0, 0, 0);
                }
            }
        }
    }
    // waves' partials summed in LDS in wave order
    constexpr int RW = WG_NBC * 16;
    for (int w = 0; w < 4; ++w) {
        __syncthreads();
        if (wave == w) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int j = 0; j < WG_NBC; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int idx = (mb * 16 + 4 * q + e) * RW + j * 16 + r16;
                        if (w == 0) s_red[idx] = acc[mb][j][e];
                        else s_red[idx] += acc[mb][j][e];
                    }
        }
    }
    // bias: lanes of one output channel (r16) across the four lane groups, then waves
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        float v = bsum[mb];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (q == 0) s_bias[wave][mb * 16 + r16] = v;
    }
    __syncthreads();
    float *part = a.part + (long long)blockIdx.x * COUT * K;
    for (int i = threadIdx.x; i < COUT * nbc * 16; i += NNT) {
        const int co = i / (nbc * 16), kk = i % (nbc * 16);
        const int k = kb0 * 16 + kk;
        if (k < K) part[co * K + k] = s_red[co * RW + kk];
    }
    if (blockIdx.y == 0 && threadIdx.x < COUT) {
        const int co = threadIdx.x;
        a.bpart[(long long)blockIdx.x * COUT + co] =
            s_bias[0][co] + s_bias[1][co] + s_bias[2][co] + s_bias[3][co];
    }
}

// grad[j] = sum_g part[g][j] in group order (one layer's weights, then biases).
__global__ void reduce_parts_kernel(int groups, int nw, const float *__restrict__ part, int nb,
                                    const float *__restrict__ bpart, float *__restrict__ grad) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < nw) {
        float s = 0.f;
        for (int g = 0; g < groups; ++g) s += part[(long long)g * nw + j];
        grad[j] = s;
    } else if (j < nw + nb) {
        const int c = j - nw;
        float s = 0.f;
        for (int g = 0; g < groups; ++g) s += bpart[(long long)g * nb + c];
        grad[j] = s;
    }
}

// Network input of column j of R (FP64, column-major, leading dimension ldr):
// channel 0 = r / rms(r), channel 1 = shat[j]; rms[j] returned.  One workgroup
// per column.
__global__ __launch_bounds__(NNT) void features_kernel(int n, const double *__restrict__ R, int ldr,
                                                       const double *__restrict__ shat,
                                                       unsigned short *__restrict__ X,
                                                       double *__restrict__ rms) {
    __shared__ double red[NNT];
    const int j = blockIdx.x;
    const double *r = R + (long long)j * ldr;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += NNT) s += r[i] * r[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = NNT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double rm = sqrt(red[0] / n);
    const double inv = rm > 0.0 ? 1.0 / rm : 0.0;
    if (threadIdx.x == 0) rms[j] = rm;
    unsigned short *x = X + (long long)j * 2 * n;
    const unsigned short sh = f2bf((float)shat[j]);
    for (int i = threadIdx.x; i < n; i += NNT) {
        x[i] = f2bf((float)(r[i] * inv));
        x[n + i] = sh;
    }
}

// Gradient w.r.t. the network output as BF16 samples: g[b][x] = G(x, b) scale[b]
// (G FP64 column-major).
__global__ void grad_out_kernel(int n, int B, const double *__restrict__ G, int ldg,
                                const double *__restrict__ scale, unsigned short *__restrict__ g) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * B) return;
    const int b = (int)(i / n), x = (int)(i % n);
    g[i] = f2bf((float)(G[(long long)b * ldg + x] * scale[b]));
}

// D(:, b) = out[b] * rms[b]  (FP64 column-major)
__global__ void scale_out_kernel(int n, int B, const float *__restrict__ out,
                                 const double *__restrict__ rms, double *__restrict__ D, int ldd) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long long)n * B) return;
    const int b = (int)(i / n), x = (int)(i % n);
    D[(long long)b * ldd + x] = (double)out[i] * rms[b];
}

// Adam (Kingma and Ba 2015) on the FP32 master parameters.
__global__ void adam_kernel(int np, float *__restrict__ theta, float *__restrict__ m,
                            float *__restrict__ v, const float *__restrict__ g, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 weights of one layer from theta: forward [cout][KP] (k = ci T + t), and
// the data-gradient weights [cin][KPb] (k = co T + t') = W[co][ci][T - 1 - t'].
__global__ void pack_weights_kernel(int cin, int cout, int T, const float *__restrict__ W,
                                    unsigned short *__restrict__ wf, int kp,
                                    unsigned short *__restrict__ wb, int kpb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cout * kp) {
        const int co = i / kp, k = i % kp;
        wf[i] = k < cin * T ? f2bf(W[co * cin * T + k]) : (unsigned short)0;
    }
    if (wb && i < cin * kpb) {
        const int ci = i / kpb, k = i % kpb;
        unsigned short v = 0;
        if (k < cout * T) {
            const int co = k / T, tp = k % T;
            v = f2bf(W[(co * cin + ci) * T + (T - 1 - tp)]);
        }
        wb[i] = v;
    }
}

inline unsigned nblocks(long long tot, int b) { return (unsigned)((tot + b - 1) / b); }

template <int DIM, int CIN, int COUT, int MODE>
hipError_t conv_launch(const NnShape &sh, int B, const unsigned short *in, const unsigned short *w,
                       const float *bias, void *out, const unsigned short *mask, hipStream_t s) {
    using G = Geom<DIM>;
    ConvArgs a{sh.nx, sh.ny, in, w, bias, out, mask};
    const int tiles = ((sh.nx + G::TX - 1) / G::TX) * ((sh.ny + G::TY - 1) / G::TY);
    hipLaunchKernelGGL((conv_kernel<DIM, CIN, COUT, MODE>), dim3(tiles, B), dim3(NNT), 0, s, a);
    return hipGetLastError();
}

template <int DIM, int CIN, int COUT>
hipError_t wgrad_launch(const NnShape &sh, int B, const unsigned short *g, const unsigned short *act,
                        float *part, float *bpart, int groups_max, float *grad, hipStream_t s) {
    using G = Geom<DIM>;
    constexpr int K = CIN * G::T;
    constexpr int NBK = (K + 15) / 16;
    const int tiles = ((sh.nx + G::TX - 1) / G::TX) * ((sh.ny + G::TY - 1) / G::TY);
    const int items = B * tiles;
    const int per = (items + groups_max - 1) / groups_max;
    const int groups = (items + per - 1) / per;
    WgradArgs a{sh.nx, sh.ny, B, g, act, part, bpart, per};
    hipLaunchKernelGGL((wgrad_kernel<DIM, CIN, COUT>), dim3(groups, (NBK + WG_NBC - 1) / WG_NBC),
                       dim3(NNT), 0, s, a);
    const int nw = COUT * K, nb = COUT;
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(nblocks(nw + nb, 256)), dim3(256), 0, s, groups, nw,
                       (const float *)part, nb, (const float *)bpart, grad);
    return hipGetLastError();
}

template <int DIM>
hipError_t forward_impl(const NnShape &sh, int B, const NnBuffers &nb, hipStream_t s) {
    hipError_t e;
    if ((e = conv_launch<DIM, 2, 32, MODE_RELU_BF16>(sh, B, nb.act[0], nb.wf[0], nb.bias[0], nb.act[1], nullptr, s)) != hipSuccess) return e;
    if ((e = conv_launch<DIM, 32, 32, MODE_RELU_BF16>(sh, B, nb.act[1], nb.wf[1], nb.bias[1], nb.act[2], nullptr, s)) != hipSuccess) return e;
    if ((e = conv_launch<DIM, 32, 32, MODE_RELU_BF16>(sh, B, nb.act[2], nb.wf[2], nb.bias[2], nb.act[3], nullptr, s)) != hipSuccess) return e;
    return conv_launch<DIM, 32, 1, MODE_LINEAR_F32>(sh, B, nb.act[3], nb.wf[3], nb.bias[3], nb.out, nullptr, s);
}

template <int DIM>
hipError_t backward_impl(const NnShape &sh, int B, const NnBuffers &nb, hipStream_t s) {
    hipError_t e;
    // layer 4 (32 -> 1): weight gradient, then the gradient w.r.t. act[3] (masked)
    if ((e = wgrad_launch<DIM, 32, 1>(sh, B, nb.g[3], nb.act[3], nb.part, nb.bpart, nb.groups_max, nb.grad + nb.off[3], s)) != hipSuccess) return e;
    if ((e = conv_launch<DIM, 1, 32, MODE_MASK_BF16>(sh, B, nb.g[3], nb.wb[3], nullptr, nb.g[2], nb.act[3], s)) != hipSuccess) return e;
    if ((e = wgrad_launch<DIM, 32, 32>(sh, B, nb.g[2], nb.act[2], nb.part, nb.bpart, nb.groups_max, nb.grad + nb.off[2], s)) != hipSuccess) return e;
    if ((e = conv_launch<DIM, 32, 32, MODE_MASK_BF16>(sh, B, nb.g[2], nb.wb[2], nullptr, nb.g[1], nb.act[2], s)) != hipSuccess) return e;
    if ((e = wgrad_launch<DIM, 32, 32>(sh, B, nb.g[1], nb.act[1], nb.part, nb.bpart, nb.groups_max, nb.grad + nb.off[1], s)) != hipSuccess) return e;
    if ((e = conv_launch<DIM, 32, 32, MODE_MASK_BF16>(sh, B, nb.g[1], nb.wb[1], nullptr, nb.g[0], nb.act[1], s)) != hipSuccess) return e;
    return wgrad_launch<DIM, 2, 32>(sh, B, nb.g[0], nb.act[0], nb.part, nb.bpart, nb.groups_max, nb.grad + nb.off[0], s);
}

}  // namespace

const int kNnChannels[5] = {2, 32, 32, 32, 1};

int nn_taps(int dim) { return dim == 1 ? 5 : 25; }

hipError_t nn_features(int n, int B, const double *R, int ldr, const double *shat, unsigned short *X,
                       double *rms, hipStream_t s) {
    hipLaunchKernelGGL(features_kernel, dim3(B), dim3(NNT), 0, s, n, R, ldr, shat, X, rms);
    return hipGetLastError();
}

hipError_t nn_scale_out(int n, int B, const float *out, const double *rms, double *D, int ldd,
                        hipStream_t s) {
    hipLaunchKernelGGL(scale_out_kernel, dim3(nblocks((long long)n * B, 256)), dim3(256), 0, s, n, B,
                       out, rms, D, ldd);
    return hipGetLastError();
}

hipError_t nn_grad_out(int n, int B, const double *G, int ldg, const double *scale, unsigned short *g,
                       hipStream_t s) {
    hipLaunchKernelGGL(grad_out_kernel, dim3(nblocks((long long)n * B, 256)), dim3(256), 0, s, n, B, G, ldg,
                       scale, g);
    return hipGetLastError();
}

hipError_t nn_pack_weights(int dim, const float *theta, const NnBuffers &nb, hipStream_t s) {
    const int T = nn_taps(dim);
    for (int l = 0; l < 4; ++l) {
        const int ci = kNnChannels[l], co = kNnChannels[l + 1];
        const int kp = (ci * T + 15) / 16 * 16, kpb = (co * T + 15) / 16 * 16;
        const int tot = std::max(co * kp, ci * kpb);
        hipLaunchKernelGGL(pack_weights_kernel, dim3(nblocks(tot, 256)), dim3(256), 0, s, ci, co, T,
                           theta + nb.off[l], nb.wf[l], kp, l > 0 ? nb.wb[l] : nullptr, kpb);
    }
    return hipGetLastError();
}

hipError_t nn_forward(int dim, const NnShape &sh, int B, const NnBuffers &nb, hipStream_t s) {
    return dim == 1 ? forward_impl<1>(sh, B, nb, s) : forward_impl<2>(sh, B, nb, s);
}

hipError_t nn_backward(int dim, const NnShape &sh, int B, const NnBuffers &nb, hipStream_t s) {
    return dim == 1 ? backward_impl<1>(sh, B, nb, s) : backward_impl<2>(sh, B, nb, s);
}

hipError_t nn_adam(int np, float *theta, float *m, float *v, const float *g, float lr, int step,
                   hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(nblocks(np, 256)), dim3(256), 0, s, np, theta, m, v, g, lr, b1,
                       b2, 1e-8f, c1, c2);
    return hipGetLastError();
}

}  // namespace acp
