// Vector kernels of the least-squares inverse (conjugate gradients on the
// normal equations of the forward transform): squared norms and updates of
// complex vectors.  Sums are binary64 on both precision paths.
#pragma once

#include "fmm_device.h"

namespace fn {

constexpr int SOLVE_BLOCKS = 256; // workgroups (and partial sums) of a norm

// part[b] = sum over workgroup b's share of |x_i|^2 (binary64).
template <typename R>
__global__ void __launch_bounds__(256) k_sqnorm(int64_t n, const cx<R> *x, double *part)
{
    __shared__ double red[4];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = (double)x[i].re, b = (double)x[i].im;
        s = fma(a, a, fma(b, b, s));
    }
    for (int d = 32; d > 0; d >>= 1)
        s += __shfl_down(s, d);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// y += a x (real a).
template <typename R>
__global__ void k_axpy(int64_t n, double a, const cx<R> *x, cx<R> *y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const cx<R> xv = x[i];
        cx<R> yv = y[i];
        yv.re = (R)((double)yv.re + a * (double)xv.re);
        yv.im = (R)((double)yv.im + a * (double)xv.im);
        y[i] = yv;
    }
}

// p = s + b p (real b).
template <typename R>
__global__ void k_xpby(int64_t n, const cx<R> *s, double b, cx<R> *p)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const cx<R> sv = s[i];
        cx<R> pv = p[i];
        pv.re = (R)((double)sv.re + b * (double)pv.re);
        pv.im = (R)((double)sv.im + b * (double)pv.im);
        p[i] = pv;
    }
}

} // namespace fn
