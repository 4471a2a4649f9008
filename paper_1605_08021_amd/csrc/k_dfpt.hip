// Element-wise kernels of the DFPT comparator (Alg. 1): the right-hand sides
// phi_i o v_j of the Sternheimer equations at the occupied energies, and the
// density response sum_i phi_i o z_ij.  Column (i, j) of the N_e n block is
// i + N_e j.
#include "acp_internal.h"

namespace acp {
namespace {

// P(a, i + ne j) = phi_i(a) v_j(a)
__global__ void dfpt_products_kernel(int ng, int ne, const double *phi, const double *V, double *P) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int col = blockIdx.y;
    if (a >= ng) return;
    const int i = col % ne, j = col / ne;
    P[a + (long long)col * ng] = phi[a + (long long)i * ng] * V[a + (long long)j * ng];
}

// Y(a, j) = scale sum_i phi_i(a) Z(a, i + ne j)
__global__ void dfpt_response_kernel(int ng, int ne, double scale, const double *phi, const double *Z, double *Y) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (a >= ng) return;
    double acc = 0.0;
    for (int i = 0; i < ne; ++i) acc += phi[a + (long long)i * ng] * Z[a + (long long)(i + (long long)ne * j) * ng];
    Y[a + (long long)j * ng] = scale * acc;
}

}  // namespace

hipError_t launch_dfpt_products(int ng, int ne, int n, const double *phi, const double *V, double *P, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dfpt_products_kernel, dim3((ng + 255) / 256, ne * n), dim3(256), 0, s, ng, ne, phi, V, P);
    return hipGetLastError();
}

hipError_t launch_dfpt_response(int ng, int ne, int n, double scale, const double *phi, const double *Z, double *Y,
                                hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dfpt_response_kernel, dim3((ng + 255) / 256, n), dim3(256), 0, s, ng, ne, scale, phi, Z, Y);
    return hipGetLastError();
}

}  // namespace acp
