// Autocorrelation of photodissociation packets: C_k = <u_0|u_k> of every step
// (the overlap of Eqs. fourier-transform and chebyshev-transform), where the R
// pass does not form it (general kernels, learned-potential pass) and for C_0.
// One launch per packet and step writes per-workgroup partial sums; the rows of
// a chunk of steps are summed in a fixed order when the chunk's norms are read
// back.
#pragma once
#include <hip/hip_runtime.h>

namespace tdwp {

constexpr int kAcfThreads = 256;
constexpr int kAcfPerBlock = 4096;   // values per workgroup before the grid stops growing
constexpr int kAcfMaxBlocks = 512;

// part[blockIdx.x] = partial sum of a[i] b[i] over this workgroup's grid-stride
// share of [0, n).  Four independent accumulators per lane keep four loads of
// each operand in flight.
__global__ void __launch_bounds__(kAcfThreads)
k_dot_partial(const double* __restrict__ a, const double* __restrict__ b, size_t n,
              double* __restrict__ part) {
  const size_t stride = (size_t)gridDim.x * kAcfThreads;
  size_t i = (size_t)blockIdx.x * kAcfThreads + threadIdx.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (; i + 3 * stride < n; i += 4 * stride) {
    s0 += a[i] * b[i];
    s1 += a[i + stride] * b[i + stride];
    s2 += a[i + 2 * stride] * b[i + 2 * stride];
    s3 += a[i + 3 * stride] * b[i + 3 * stride];
  }
  for (; i < n; i += stride) s0 += a[i] * b[i];
  double s = (s0 + s1) + (s2 + s3);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  __shared__ double wave_sum[kAcfThreads / 64];
  if ((threadIdx.x & 63) == 0) wave_sum[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kAcfThreads / 64; ++w) t += wave_sum[w];
    part[blockIdx.x] = t;
  }
}

// out[r] = sum_{q < nb} part[r * stride + q] for r < rows (fixed order).
__global__ void k_rows_sum(const double* __restrict__ part, size_t stride, int nb, int rows,
                           double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const double* src = part + (size_t)r * stride;
  double s = 0.0;
  for (int q = 0; q < nb; ++q) s += src[q];
  out[r] = s;
}

// out[i] = a out[i] + b in[i]: H u = dE (H_s u) + E0 u from a step's H_s u.
__global__ void k_affine(double* __restrict__ out, const double* __restrict__ in, double a,
                         double b, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = a * out[i] + b * in[i];
}

// y = a y + b x + c z (y may alias x; y is not read when a = 0, z not when c = 0):
// the vector updates of the bound-state Lanczos iteration.
__global__ void k_lincomb(double* y, double a, const double* x, double b, const double* z,
                          double c, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    double v = b * x[i];
    if (a != 0.0) v += a * y[i];
    if (c != 0.0) v += c * z[i];
    y[i] = v;
  }
}

}  // namespace tdwp
