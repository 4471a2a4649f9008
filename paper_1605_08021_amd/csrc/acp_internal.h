// Internal declarations shared by the host orchestration and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/acp.h"

namespace acp {

// Column tile width of the Krylov layout: a tile holds 16 consecutive systems,
// stored row-interleaved (element (row, col) at ((col/16) * N_g + row) * 16 + col%16),
// so that one grid row of a tile is one 128-byte line.
constexpr int kTile = 16;

// 8th-order central coefficients of the second derivative, c_0 .. c_4:
// u''(x) ~ h^-2 sum_{s=-4..4} c_|s| u(x + s h).
__host__ __device__ constexpr double fd8(int k) {
    return k == 0 ? -205.0 / 72.0
         : k == 1 ? 8.0 / 5.0
         : k == 2 ? -1.0 / 5.0
         : k == 3 ? 8.0 / 315.0
                  : -1.0 / 560.0;
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Error text of the last call without a context (acp_last_error(NULL)).
extern thread_local std::string g_free_error;

// Grow-only device buffer; returns nullptr on failure.
void *ensure(DevBuf &b, size_t bytes);
void release(DevBuf &b);

struct GridDesc {
    int dim;
    int nx, ny;       // ny = 1 in 1D
    int ng;
    double h;
};

// ---------------------------------------------------------------- stencil (K1)
// Y(:,j) = c_lap * Delta_h X(:,j) + (c_v * V + c_0 - shift[j]) X(:,j), column-major;
// with add (FP32, leading dimension ld_add) also + add(:,j); with dot (2D only)
// dot[j] = X(:,j).Y(:,j) through per-tile partials in dot_work
// (stencil_dot_work_doubles(g, n)), summed in a fixed order.
hipError_t launch_stencil(const GridDesc &g, int n, const double *X, int ldx, double *Y,
                          int ldy, const double *V, double c_lap, double c_v, double c_0,
                          const double *shift_dev, hipStream_t s, const float *add = nullptr,
                          long long ld_add = 0, double *dot = nullptr, double *dot_work = nullptr);
size_t stencil_dot_work_doubles(const GridDesc &g, int n);

// ---------------------------------------------------------------- GEMM (FP64 MFMA)
enum class Op { N, T };
enum class Epi { Store, HadamardAcc, StoreProjector };
// C = alpha op(A) op(B) + beta C   (Store; StoreProjector is the same product
//                                  under its own kernel symbol: the projector
//                                  GEMMs of the many-orbital Krylov solver)
// C += alpha (op(A) op(B)) o E     (HadamardAcc; beta ignored)
// batched with strides sa, sb, sc, se (in elements).
hipError_t gemm(Op ta, Op tb, int m, int n, int k, double alpha, const double *A, int lda,
                long long sa, const double *B, int ldb, long long sb, double beta, double *C,
                int ldc, long long sc, int batch, hipStream_t s, Epi epi = Epi::Store,
                const double *E = nullptr, int lde = 0, long long se = 0);

// Same product for outputs with few 64 x 64 tiles and a long K: the K range is
// split into slices whose partial products (work, >= nsplit m n elements) are
// summed in a fixed order.  Op::N/Op::T as above; beta applies to C.
hipError_t gemm_splitk(Op ta, Op tb, int m, int n, int k, double alpha, const double *A, int lda,
                       const double *B, int ldb, double beta, double *C, int ldc, double *work,
                       size_t work_elems, hipStream_t s, Epi epi = Epi::Store);

// ---------------------------------------------------------------- small utilities
hipError_t launch_scale_copy(int m, int n, double alpha, const double *X, int ldx, double *Y,
                             int ldy, hipStream_t s);                      // Y = alpha X
hipError_t launch_gather_rows(int nsel, int n, const int *sel, const double *X, int ldx,
                              double *Y, int ldy, hipStream_t s);          // Y = X(sel, :)
hipError_t launch_scatter_identity(int nsel, const int *sel, double *Xi, int ld,
                                   hipStream_t s);                         // Xi(sel,:) = I
hipError_t launch_add_identity_neg(int n, double *T, int ld, hipStream_t s);  // T = I - T
hipError_t launch_col_sqnorm(int m, int n, const double *X, int ldx, double *out,
                             hipStream_t s);                               // out[j] = ||X(:,j)||^2
hipError_t launch_col_diff_sqnorm(int m, int n, const double *X, int ldx, const double *Y,
                                  int ldy, double *out, hipStream_t s);  // ||X(:,j)-Y(:,j)||^2
hipError_t launch_axpby(int m, int n, double a, const double *X, int ldx, double b, double *Y,
                        int ldy, hipStream_t s);                           // Y = a X + b Y
hipError_t launch_weighted_rows(int ne, int nmu, const double *L, const int *sel,
                                const double *phi, int ldphi, double *Bc, hipStream_t s);
hipError_t launch_gram_check(int n, int unused, const double *G, double *maxdev, hipStream_t s);
hipError_t launch_transpose(int m, int n, const double *A, int lda, double *B, int ldb,
                            hipStream_t s);                                // B = A^T

// ---------------------------------------------------------------- Krylov layout
hipError_t launch_to_tiled(int ng, int ncols, int ncols_pad, const double *X, int ldx,
                           double *T, hipStream_t s);
hipError_t launch_from_tiled(int ng, int ncols, const double *T, double *X, int ldx,
                             hipStream_t s);
// FP32 tiles of X (each column scaled by colscale[j] when given), X += tiles,
// and an elementwise FP64 -> FP32 copy: the mixed-precision form.
hipError_t launch_to_tiled_f32(int ng, int ncols, int ncols_pad, const double *X, int ldx,
                               const double *colscale, float *T, hipStream_t s);
hipError_t launch_from_tiled_add(int ng, int ncols, const double *T, double *X, int ldx,
                                 hipStream_t s);
hipError_t launch_to_f32(size_t n, const double *X, float *Y, hipStream_t s);
// K(mu, a) = g((x, y)(sel[mu]) - (x, y)(a)) on the periodic nx x ny grid: the rows
// sel of the translation-invariant operator whose first column is g.
hipError_t launch_circulant_rows(int nsel, const int *sel, int nx, int ny, const double *g, double *K,
                                 hipStream_t s);

// T is the storage type of Phi, the right-hand sides and the Krylov vectors
// (double, or float for the inner solves of the mixed-precision form); the
// solution x is always accumulated in double, and all arithmetic is FP64.
template <typename T>
struct KrylovArgsT {
    GridDesc g;
    int ne;
    int ntiles;             // number of 16-column tiles to solve
    int rhs_tiles;          // tiles of the right-hand side; tile t uses rhs tile t % rhs_tiles
    const T *phi_rm;        // N_g x N_e row-major (orbitals contiguous)
    const T *phi_cm;        // N_g x N_e column-major
    const double *veff;     // N_g
    const double *shift;    // per column (ntiles * 16)
    const T *rhs;           // tiled right-hand sides
    double *x;              // tiled solution
    T *r, *pa, *pb;         // tiled state
    T *w1, *w2, *w3;        // extra tiled vectors (MINRES)
    int *iters;             // per column
    double *resid;          // per column: final recurrence residual / ||b||
    int *flags;             // per column: bit0 not converged, bit1 non-positive curvature
    double tol;
    int max_iter;
    int *tile_iters;        // per tile: iterations executed by its workgroup
};
using KrylovArgs = KrylovArgsT<double>;
hipError_t launch_cg_fp64(const KrylovArgs &a, hipStream_t s);
hipError_t launch_cg_fp32(const KrylovArgsT<float> &a, hipStream_t s);

// Multi-shift CG: every tile of 16 right-hand sides solves all nshift shifts;
// a group of K workgroups shares a tile (cooperative launch of ntiles * K).
template <typename T>
struct MsArgsT {
    GridDesc g;
    int ne;                 // padded orbital count (multiple of 16)
    int ntiles;             // right-hand-side tiles
    int K;                  // workgroups per tile
    int nshift, base;       // shifts; index of the base (largest) shift
    const double *shift;    // device, nshift
    const T *phi_rm, *phi_cm;
    const double *veff;
    const T *rhs;           // tiled right-hand sides, ntiles tiles
    double *x;              // [nshift][ntiles] tiles (always double)
    T *p;                   // [nshift][ntiles] tiles
    T *r;                   // residual ring: [kMsWindow][ntiles] tiles
    T *pa, *pb;             // ntiles tiles each (pa: s = A p of the base sequence)
    double *gbuf;           // ntiles * 2 * K * slot doubles
    unsigned *cnt;          // ntiles counters, zero at launch
    int sg;                 // lockstep: tiles t, t + ntiles/sg, ... share one barrier (<= 1: off)
    int *active;            // lockstep: per super-group tiles not yet done, sg at launch
    int *hflag;             // halo flags: [ntiles][K], zero at launch (K > 1)
    int *abort_flag;        // set if a group barrier wait expired
    int *iters;             // [nshift][ntiles * 16]
    double *resid;
    int *flags;
    int *tile_iters;        // ntiles
    double tol;
    int max_iter;
    unsigned long long *phase_clock;   // 8 phase timers of workgroup 0 (ACP_PHASE_CLOCKS builds)
    // Suspend and resume at window boundaries (both multiples of the window
    // length): it0 > 0 resumes every tile at iteration it0 from the vectors in
    // x, p, pa and ring slot it0 of r and from the scalars in state; stop_at > 0
    // suspends a tile still running at the top of iteration stop_at, leaving
    // its scalars in state.  state: [ntiles][kMsStateFields][16] doubles, then
    // [ntiles][16] carry flags (1: suspended and still live).
    int it0, stop_at;
    double *state;
};
using MsArgs = MsArgsT<double>;
// Scalar state of one right-hand side of a tile: its base-sequence scalars
// (fields 0-7: r.r, |b|, b_{k-1}, a_{k-1}, flags, live, suspended, unused),
// then six per shift (zeta_k, zeta_{k-1}, b^c, converged residual, live,
// iterations).
constexpr int kMsStateFields = 8 + 6 * 16;
// Longest window of the deferred solution updates of the multi-shift solver (16
// iterations with at most 8 shifts, else 8); the residual ring holds this many
// residuals per tile.
constexpr int kMsWindow = 16;
constexpr int kMsMaxGroup = 16;   // workgroups per right-hand-side tile
hipError_t launch_mscg_fp64(const MsArgs &a, hipStream_t s);
hipError_t launch_mscg_fp32(const MsArgsT<float> &a, hipStream_t s);
// Persistent ragged batch: systems[] are device descriptors of systems with the
// same dim (3: 2D grids whose lines hold a multiple of 4 points, the compact
// stencil gather) whose orbital blocks are padded to ne_pad (each with its own group
// size K); the work list (work_sys[w], work_tile[w] = tile * kMsMaxGroup + kg,
// the K members of a tile consecutive) is consumed in order through *queue
// (zero at launch); grid >= the largest K.
hipError_t launch_mscg_batch_fp64(int dim, int ne_pad, const MsArgs *systems, const int *work_sys,
                                  const int *work_tile, int n_work, unsigned *queue, int grid,
                                  hipStream_t s);
int mscg_resident_capacity(int dim, int ne, bool fp32);   // workgroups the device can hold at once
size_t mscg_group_slot(int ne);                // doubles per group partial
hipError_t launch_fill_u32(unsigned *p, size_t n, unsigned v, hipStream_t s);
hipError_t launch_fill_i32(int *p, size_t n, int v, hipStream_t s);
hipError_t launch_minres_fp64(const KrylovArgs &a, hipStream_t s);

// ---------------------------------------------------------------- multi-shift CG, many orbitals
// Scalar state of the wide multi-shift CG (k_wide.hip): per column j (nb) and
// per (shift c, column j) at c * nb + j.
constexpr int kWideWindow = 16;  // iterations between the deferred updates (flush)
struct WideScalars {
    double *rr, *rrn, *bn, *al, *alp, *btp;          // nb each
    double *z, *zp, *ac, *zn, *bc, *res;             // nc * nb each
    double *coef;                                    // nc * nb * (2 + 2 kWideWindow): window coefficients
    int *colact;                                     // nb
    int *act, *upd, *it, *touched;                   // nc * nb each
    int *flags, *nactive;                            // 1 each
};
// rr = |b|^2 from bsq, every shift live for b != 0, zeta = 1.
hipError_t wide_init(int nb, int nc, const double *bsq, const WideScalars &w, hipStream_t s);
// One CG step after w = A p (p = P block `base`) and pw = p.w, iteration `iter`
// of the window started at k0: alpha, rn = r - alpha w (r = r^iter, rn = r^{iter+1},
// ring slots), the shifted coefficients (advanced in the window), the base
// shift's x and p, the column state (nactive += live columns).  P: nc blocks of
// N_g x nb (stride N_g nb); X: nc blocks with stride xs.
// With pb (two arrays, leading dimension ldpb) the base p is also written as
// its two-term BF16 split (the operand of the reduced-precision projector).
// The base shift's x is deferred to the flush: at a window's first iteration
// (iter == k0) its p is kept in P0 (N_g x nb).
hipError_t wide_step(int ng, int nb, int nc, int base, const double *sig, double tol, int iter, int k0,
                     const double *pw, const double *w_vec, const double *r, double *rn, double *P, double *X,
                     long long xs, const WideScalars &w, double *P0, hipStream_t s, unsigned short *const *pb = nullptr,
                     long long ldpb = 0);
// End of a window of wl steps started at k0: the other shifts' p_c and x_c from
// the ring of residuals (slot q holds r^k for k mod kWideWindow = q, stride N_g nb).
hipError_t wide_flush(int ng, int nb, int nc, int base, int k0, int wl, const double *ring, double *P, double *X,
                      long long xs, const WideScalars &w, const double *P0, hipStream_t s);

// dos[p] = (1 / n_modes) sum_k exp(-(w[p] - w_k)^2 / (2 sigma^2)) / sqrt(2 pi sigma^2),
// w_k = sign(omega2_k) sqrt(|omega2_k|) (all on the device).
hipError_t launch_phonon_dos(const double *omega2, int n, int n_modes, double sigma, const double *w, int nw,
                             double *dos, hipStream_t s);

// ---------------------------------------------------------------- flexible CG scalars (k_fcg.hip)
// Columns in compact order i (system cols[i]); done, iters in system order;
// squared norms throughout (bn2 = |b|^2, sref = |r|^2 at the last halving).
hipError_t fcg_init(int n, const double *bn2, int *act, int *done, int *iters, double *sref, int *sit,
                    hipStream_t s);
hipError_t fcg_alpha(int w, const double *pq, const double *rz, int *act, double *al, double *nal, int mode,
                     int *flags, hipStream_t s);
hipError_t fcg_conv(int w, int k, const double *rr, const double *bn2, double tol, int *act, int *done,
                    const int *cols, int *iters, double *sref, int *sit, int mode, int kstall, int *nopen,
                    hipStream_t s);
hipError_t fcg_beta(int w, const int *act, const double *al, const double *zq, const double *rzn, double *rz,
                    double *be, hipStream_t s);

// ---------------------------------------------------------------- BF16 projector (k_gemm_bf16.hip)
// bf16 of x: FP64 -> FP32 (nearest), then nearest-even to 8 significant bits.
// Splitting needs no exact rounding: x - bf16(x) is exact in FP64, and the next
// term carries it.
__device__ inline unsigned short f64_to_bf16(double x) {
    unsigned int fb = __float_as_uint((float)x);
    if ((fb & 0x7f800000u) == 0x7f800000u) return (unsigned short)((fb >> 16) | ((fb & 0xffffu) ? 0x40u : 0u));
    fb += 0x7fffu + ((fb >> 16) & 1u);
    return (unsigned short)(fb >> 16);
}
__device__ inline double bf16_to_f64(unsigned short h) { return (double)__uint_as_float((unsigned int)h << 16); }
// X column-major (m x n, ldx) -> nt (1..3) BF16 terms O[s][j ldo + i], rows
// m..ldo-1 zero.
hipError_t launch_split_bf16(int m, int n, const double *X, long long ldx, int nt, unsigned short *const *O,
                             long long ldo, hipStream_t s);
// The same split written transposed: O[s][i ldo + j], columns n..ldo-1 zero.
hipError_t launch_split_bf16_transpose(int m, int n, const double *X, long long ldx, int nt,
                                       unsigned short *const *O, long long ldo, hipStream_t s);
// D = sum_{a + b < max(na, nb)} A_a B_b^T with A_a[m lda + k] (M x K) and
// B_b[n ldb + k] (N x K), BF16 operands, FP32 accumulation on the matrix cores.
// epi 0: split-K over nsplit slices, slice z stored to P[z ldp N + n ldp + m]
// (FP32; ldp a multiple of 4); epi 1 (nsplit = 1): Wd[n ldw + m] += alpha D.
// K, lda, ldb multiples of 8; supported (na, nb, epi): (1,1,*), (2,2,0),
// (3,1,*), (3,2,1), (2,1,1).
hipError_t gemm_bf16_tn(int na, int nb, int epi, int M, int N, int K, const unsigned short *const *A, long long lda,
                        const unsigned short *const *B, long long ldb, int nsplit, float *P, long long ldp,
                        double *Wd, long long ldw, double alpha, hipStream_t s);
// Number of split-K slices gemm_bf16_tn actually uses for K and nsplit.
int bf16_split_count(int K, int nsplit);
// Cb[j ldc + i] = bf16((T - eps_i) sum_z P[z ldp n + j ldp + i]) for i < m (T alone
// when eps is null), 0 below ldc.
hipError_t launch_deflate_coef(int m, int n, int nsplit, const float *P, long long ldp, const double *eps, double T,
                               unsigned short *Cb, long long ldc, hipStream_t s);

// ---------------------------------------------------------------- DFPT comparator (k_dfpt.hip)
// P(:, i + ne j) = phi_i o V(:, j);  Y(:, j) = scale sum_i phi_i o Z(:, i + ne j).
hipError_t launch_dfpt_products(int ng, int ne, int n, const double *phi, const double *V, double *P, hipStream_t s);
hipError_t launch_dfpt_response(int ng, int ne, int n, double scale, const double *phi, const double *Z, double *Y,
                                hipStream_t s);

// ---------------------------------------------------------------- learned preconditioner
// Network of four periodic convolutions (channels kNnChannels), BF16 operands on
// the matrix cores, FP32 accumulation (k_nn.hip).
extern const int kNnChannels[5];
int nn_taps(int dim);
struct NnShape {
    int nx, ny;                 // grid (ny = 1 in 1D)
};
struct NnBuffers {
    unsigned short *act[4];     // act[0] = features [B][2][N]; act[1..3] = hidden [B][32][N]
    float *out;                 // network output [B][N]
    unsigned short *g[4];       // g[l] = dL/d(output of layer l) (g[3]: [B][1][N], others [B][32][N])
    unsigned short *wf[4];      // forward weights [cout][KP]
    unsigned short *wb[4];      // data-gradient weights [cin][KPb] (layers 1..3)
    const float *bias[4];       // into theta
    float *grad;                // [n_params], theta layout
    int off[4];                 // offset of layer l in theta
    float *part, *bpart;        // weight-gradient partials
    int groups_max;
};
hipError_t nn_features(int n, int B, const double *R, int ldr, const double *shat, unsigned short *X,
                       double *rms, hipStream_t s);
hipError_t nn_scale_out(int n, int B, const float *out, const double *rms, double *D, int ldd,
                        hipStream_t s);
hipError_t nn_grad_out(int n, int B, const double *G, int ldg, const double *scale, unsigned short *g,
                       hipStream_t s);
hipError_t nn_pack_weights(int dim, const float *theta, const NnBuffers &nb, hipStream_t s);
hipError_t nn_forward(int dim, const NnShape &sh, int B, const NnBuffers &nb, hipStream_t s);
hipError_t nn_backward(int dim, const NnShape &sh, int B, const NnBuffers &nb, hipStream_t s);
hipError_t nn_adam(int np, float *theta, float *m, float *v, const float *g, float lr, int step,
                   hipStream_t s);
hipError_t launch_col_dot(int m, int n, const double *X, int ldx, const double *Y, int ldy,
                          double *out, hipStream_t s);                     // out[j] = X(:,j).Y(:,j)
// dst(:, i) = src(:, idx[i]) and Y(:, idx[i]) += a[i] X(:, i) for i < n (idx on the device).
// Columns of tile-interleaved vectors ([tile][row][16]): destination column m
// of each of nvec vectors (strides svs, dvs elements) takes source column map[m];
// map[m] < 0 writes zero (zero_missing) or skips the column.  ncols = 16 x tiles.
hipError_t launch_tilecol_gather(int rows, int ncols, const int *map, const double *src, long long svs,
                                 double *dst, long long dvs, int nvec, bool zero_missing, hipStream_t s);
hipError_t launch_tilecol_gather(int rows, int ncols, const int *map, const float *src, long long svs,
                                 float *dst, long long dvs, int nvec, bool zero_missing, hipStream_t s);
hipError_t launch_col_gather(int m, int n, const double *src, int lds, const int *idx, double *dst, int ldd,
                             hipStream_t s);
hipError_t launch_col_axpy_scatter(int m, int n, const double *a, const double *X, int ldx, const int *idx,
                                   double *Y, int ldy, hipStream_t s);
hipError_t launch_col_axpby(int m, int n, const double *a, const double *X, int ldx, const double *b,
                            double *Y, int ldy, hipStream_t s);  // Y(:,j) = a[j] X(:,j) + b[j] Y(:,j)

// ---------------------------------------------------------------- ISDF (K4)
// Greedy pivoted Cholesky of the implicit Hadamard Gram matrix (column-major
// inputs phi N_g x n_e and gt N_g x r, leading dimension N_g; pgram: Phi Phi^T
// (N_g x N_g) or null; factor L column-major N_g x nmu_max, leading dimension
// N_g); forced (dev, nmu_max entries) replaces the argmax by the given pivots.
hipError_t isdf_pivoted_cholesky(int ng, int ne, int r, const double *phi, const double *pgram,
                                 const double *gt, int nmu_max, double tol, double *L, double *diag,
                                 int *sel_dev, const int *forced, int *nmu_out_host, void *scratch,
                                 hipStream_t s);
size_t isdf_scratch_bytes(int ng);
// The same selection in panels (k_isdf_panel.hip), for grids whose Phi Phi^T
// is not kept: pools of kIsdfPool rows with the largest remaining diagonal,
// their residual Gram columns by GEMMs, up to kIsdfPanel pivots per pool, the
// same pivots as the step-by-step rule.  Unforced only; scratch of
// isdf_panel_scratch_bytes bytes.
constexpr int kIsdfPool = 256;
constexpr int kIsdfPanel = 64;
size_t isdf_panel_scratch_bytes(int ng, int ne, int r, int nmu);
hipError_t isdf_panel_cholesky(int ng, int ne, int r, const double *phi, const double *gt, int nmu_max, double tol,
                               double *L, double *diag, int *sel_dev, int *nmu_out_host, void *scratch,
                               hipStream_t s);
// Order n2 >= n (32 times a power of two) of the padded inverse below.
int tri_inverse_order(int n);
// X (n2 x n2, leading dimension n2) = [L11 0; 0 I]^{-1} for L11(i, j) = L(sel[i], j),
// j <= i (L column-major, leading dimension ng); T: n2 * n2 / 4 doubles of scratch.
hipError_t launch_isdf_l11_inverse(int n, const int *sel, const double *L, int ng, double *X, double *T,
                                   hipStream_t s);

// ---------------------------------------------------------------- dense FP64
// Solve A X = B in place (A n x n, B n x nrhs) by Gauss-Jordan with partial pivoting.
hipError_t gauss_jordan_solve(int n, int nrhs, double *A, int lda, double *B, int ldb,
                              int *piv_scratch, hipStream_t s);
// A X = B (A n x n, B n x nrhs, column-major, both overwritten: B <- X) by a
// blocked LU with partial pivoting; pinfo: device scratch of lu_pinfo_ints(n)
// ints.  B = A + n lda with ldb = lda lets one GEMM update both.  Panels of 8
// columns while more than 1024 rows remain, 32 after; Gauss-Jordan above 4096
// unknowns.
size_t lu_pinfo_ints(int n);
hipError_t lu_solve(int n, int nrhs, double *A, int lda, double *B, int ldb, int *pinfo, hipStream_t s);
// Symmetric eigenvalues by Householder reduction to tridiagonal form and Sturm
// bisection: in one workgroup's LDS up to n = 128, over the whole device above
// (n <= 4096); A overwritten; eig ascending; work: sym_eigvals_work_doubles(n).
hipError_t sym_eigvals(int n, double *A, int lda, double *eig, double *work, hipStream_t s);
size_t sym_eigvals_work_doubles(int n);
// Symmetric eigenvalues (ascending, eig dev n) and, when V is not null, the
// eigenvectors (V dev n x n, column j for eig[j]) by cyclic Jacobi over the
// whole device (k_eig.hip); A is overwritten; work: sym_eig_work_doubles(n, V
// != null) doubles.  Stops after a sweep with no rotation above the threshold
// |A_pq| > tol sqrt(|A_pp A_qq|) or after max_sweeps (the sweeps performed go to
// *sweeps_out).  Synchronises the stream once per sweep.
size_t sym_eig_work_doubles(int n, bool vectors);
// W(:, j) /= sqrt(d[j]) (d floored at 1e-300), m x n, d on the device.
hipError_t launch_col_scale_rsqrt(int m, int n, double *W, int ldw, const double *d, hipStream_t s);
hipError_t sym_eig_jacobi(int n, double *A, int lda, double *eig, double *V, int ldv, double *work,
                          int max_sweeps, double tol, hipStream_t s, int *sweeps_out);
hipError_t launch_dynmat_assemble(int np, int dim, const double *Phi_el, const double *K_local,
                                  const double *mass, double *D, double *asym2,
                                  hipStream_t s);

// ---------------------------------------------------------------- v_c by Fourier GEMMs
hipError_t launch_fourier_basis(int n, double *F, hipStream_t s);
hipError_t launch_fourier_symbol(const GridDesc &g, double kappa, double eps0, double *S,
                                 hipStream_t s);
hipError_t launch_mul_symbol(int ng, int n, const double *S, double *X, hipStream_t s);

}  // namespace acp
