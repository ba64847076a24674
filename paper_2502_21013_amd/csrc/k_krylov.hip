// Space-time vector kernels of the Newton outer loop's Krylov solve: dot products with a
// fixed-order reduction, and the update y = alpha x + beta y, on node-major time fields
// ([nodes][N] doubles, boundary entries 0). Grid-stride, two doubles per thread step.
#include "pt_device.h"

namespace pt {

__global__ void __launch_bounds__(kBlock) k_tdot(const double2* __restrict__ a, const double2* __restrict__ b,
                                                 size_t n2, double* part) {
    double s = 0.0;
    for (size_t id = blockIdx.x * (size_t)kBlock + threadIdx.x; id < n2; id += (size_t)gridDim.x * kBlock) {
        const double2 x = a[id], y = b[id];
        s = __builtin_fma(x.x, y.x, s);
        s = __builtin_fma(x.y, y.y, s);
    }
    __shared__ double red[kBlock];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * (size_t)blockIdx.x] = red[0];
        part[2 * (size_t)blockIdx.x + 1] = 0.0;
    }
}

__global__ void __launch_bounds__(kBlock) k_taxpby(double alpha, const double2* __restrict__ x, double beta,
                                                   double2* __restrict__ y, size_t n2) {
    for (size_t id = blockIdx.x * (size_t)kBlock + threadIdx.x; id < n2; id += (size_t)gridDim.x * kBlock) {
        const double2 v = x[id];
        double2 w = beta == 0.0 ? make_double2(0.0, 0.0) : y[id];
        w.x = alpha * v.x + beta * w.x;
        w.y = alpha * v.y + beta * w.y;
        y[id] = w;
    }
}

static int tgrid(size_t n2) {
    size_t g = (n2 + kBlock - 1) / kBlock;
    if (g > (size_t)kAdjBlocks) g = kAdjBlocks;
    if (g < 1) g = 1;
    return (int)g;
}

int launch_tdot(const Plan& p, const double* a, const double* b, double* part, hipStream_t st) {
    const size_t n2 = p.nodes * (size_t)p.N / 2;
    const int g = tgrid(n2);
    hipLaunchKernelGGL(k_tdot, dim3(g), dim3(kBlock), 0, st, (const double2*)a, (const double2*)b, n2, part);
    return g;
}

void launch_taxpby(const Plan& p, double alpha, const double* x, double beta, double* y, hipStream_t st) {
    const size_t n2 = p.nodes * (size_t)p.N / 2;
    hipLaunchKernelGGL(k_taxpby, dim3(tgrid(n2)), dim3(kBlock), 0, st, alpha, (const double2*)x, beta, (double2*)y,
                       n2);
}

}  // namespace pt
