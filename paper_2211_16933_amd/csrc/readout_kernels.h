// Readout kernels beyond the per-cell moments.
#pragma once

#include <hip/hip_runtime.h>

namespace elb {

constexpr int AMP_THREADS = 1024;

// Fourier amplitudes of the density over the cells (Sec. IV.A, the projection of the
// density perturbation): out[0] = (2/nx) sum_i n_i sin(k x_i), out[1] = (2/nx) sum_i n_i
// cos(k x_i), x_i = x0 + (i + 1/2) dx.  One block; FP64 sums in a fixed order (strided
// partial sums, then a tree over the threads), so repeated calls agree bit for bit.
__global__ __launch_bounds__(AMP_THREADS) void k_amplitudes(const double *n, int nx, double x0,
                                                            double dx, double k, double *out)
{
    __shared__ double ps[AMP_THREADS], pc[AMP_THREADS];
    const int tid = threadIdx.x;
    double s = 0.0, c = 0.0;
    for (int i = tid; i < nx; i += AMP_THREADS) {
        double sv, cv;
        sincos(k * (x0 + (i + 0.5) * dx), &sv, &cv);
        s = fma(n[i], sv, s);
        c = fma(n[i], cv, c);
    }
    ps[tid] = s;
    pc[tid] = c;
    __syncthreads();
    for (int h = AMP_THREADS / 2; h > 0; h >>= 1) {
        if (tid < h) {
            ps[tid] += ps[tid + h];
            pc[tid] += pc[tid + h];
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[0] = 2.0 * ps[0] / nx;
        out[1] = 2.0 * pc[0] / nx;
    }
}

}  // namespace elb
