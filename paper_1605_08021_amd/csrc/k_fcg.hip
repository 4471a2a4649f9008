// Per-column scalar steps of the flexible CG of the learned form, on the device
// so that the iteration runs without a host round trip: alpha from p.Ap, the
// convergence and stagnation tests after r -= alpha Ap, beta from z'.Ap.
// Columns are in the solver's compact order i (system cols[i]); done and iters
// are in system order.
#include "acp_internal.h"

namespace acp {
namespace {

__global__ void fcg_init_kernel(int n, const double *bn2, int *act, int *done, int *iters, double *sref, int *sit) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int live = bn2[j] > 0.0;
    act[j] = live;
    done[j] = !live;
    iters[j] = 0;
    sref[j] = bn2[j];
    sit[j] = 0;
}

// alpha = r.z / p.Ap; p.Ap <= 0 stops the column (mode 1: left for the FP64
// solver; otherwise flags |= 2).  nal = -alpha; both 0 for stopped columns.
__global__ void fcg_alpha_kernel(int w, const double *pq, const double *rz, int *act, double *al, double *nal,
                                 int mode, int *flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= w) return;
    double a = 0.0;
    if (act[i]) {
        if (pq[i] > 0.0) {
            a = rz[i] / pq[i];
        } else {
            act[i] = 0;
            if (mode != 1) atomicOr(flags, 2);
        }
    }
    al[i] = a;
    nal[i] = -a;
}

// After r -= alpha Ap (rr = r.r): a live column counts an iteration and stops
// at |r| <= tol |b| (done), or, with the network (mode 1), when |r| has not
// halved in kstall iterations; nopen counts the columns still live.
__global__ void fcg_conv_kernel(int w, int k, const double *rr, const double *bn2, double tol2, int *act, int *done,
                                const int *cols, int *iters, double *sref, int *sit, int mode, int kstall,
                                int *nopen) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= w || !act[i]) return;
    const int j = cols[i];
    iters[j] += 1;
    const double r2 = rr[i];
    if (r2 <= tol2 * bn2[i]) {
        act[i] = 0;
        done[j] = 1;
        return;
    }
    if (r2 <= 0.25 * sref[i]) {
        sref[i] = r2;
        sit[i] = k;
    } else if (mode == 1 && k - sit[i] >= kstall) {
        act[i] = 0;
        return;
    }
    atomicAdd(nopen, 1);
}

// beta = -alpha z'.Ap / r.z for live columns (0 for the others); rz = r'.z'.
__global__ void fcg_beta_kernel(int w, const int *act, const double *al, const double *zq, const double *rzn,
                                double *rz, double *be) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= w) return;
    be[i] = (act[i] && rz[i] != 0.0) ? -al[i] * zq[i] / rz[i] : 0.0;
    rz[i] = rzn[i];
}

inline unsigned blocks(int n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t fcg_init(int n, const double *bn2, int *act, int *done, int *iters, double *sref, int *sit,
                    hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fcg_init_kernel, dim3(blocks(n)), dim3(256), 0, s, n, bn2, act, done, iters, sref, sit);
    return hipGetLastError();
}

hipError_t fcg_alpha(int w, const double *pq, const double *rz, int *act, double *al, double *nal, int mode,
                     int *flags, hipStream_t s) {
    if (w <= 0) return hipSuccess;
    hipLaunchKernelGGL(fcg_alpha_kernel, dim3(blocks(w)), dim3(256), 0, s, w, pq, rz, act, al, nal, mode, flags);
    return hipGetLastError();
}

hipError_t fcg_conv(int w, int k, const double *rr, const double *bn2, double tol, int *act, int *done,
                    const int *cols, int *iters, double *sref, int *sit, int mode, int kstall, int *nopen,
                    hipStream_t s) {
    if (w <= 0) return hipSuccess;
    hipLaunchKernelGGL(fcg_conv_kernel, dim3(blocks(w)), dim3(256), 0, s, w, k, rr, bn2, tol * tol, act, done, cols,
                       iters, sref, sit, mode, kstall, nopen);
    return hipGetLastError();
}

hipError_t fcg_beta(int w, const int *act, const double *al, const double *zq, const double *rzn, double *rz,
                    double *be, hipStream_t s) {
    if (w <= 0) return hipSuccess;
    hipLaunchKernelGGL(fcg_beta_kernel, dim3(blocks(w)), dim3(256), 0, s, w, act, al, zq, rzn, rz, be);
    return hipGetLastError();
}

}  // namespace acp
