// Learned diabatic potential: a 3 -> 128 -> 128 -> 128 -> n_pair network (SiLU)
// of the three internuclear distances, trained on the device (FP32 forward,
// backward and Adam kernels) and evaluated on the fly inside the step with
// BF16 weights on the matrix cores (FP32 accumulation).
//
//   f = (d - 4 bohr) / 3 bohr;  a_k = silu(a_{k-1} W_k + b_k) (k = 1..3);
//   V = 0.1 hartree * (a_3 W_4 + b_4),  silu(x) = x / (1 + e^-x).
// Parameter layout (FP32, flat): W1[3][128] b1 W2[128][128] b2 W3[128][128] b3
// W4[128][n_pair] b4, W stored [in][out].
#pragma once
#include <hip/hip_runtime.h>

#include "fast_kernels.hpp"

namespace tdwp {

constexpr int kMlpH = 128;
constexpr float kFeatCenter = 4.0f, kFeatScale = 3.0f;
constexpr double kOutScale = 0.1;
constexpr int kMlpLd = 136;   // per-wave activation tile row stride (bf16), 16-byte aligned rows

__device__ __forceinline__ float silu_f(float x) { return x / (1.0f + __expf(-x)); }
__device__ __forceinline__ float dsilu_f(float x) {
  const float s = 1.0f / (1.0f + __expf(-x));
  return s * (1.0f + x * (1.0f - s));
}

// Distances (r_AB, r_BC, r_AC) of Jacobi point (r, R, cos gamma): B at -cB r, C at +cC r
// along r from the BC centre of mass, A at R.
__device__ __forceinline__ void jacobi_distances(double r, double R, double x, double cB, double cC,
                                                 float* d) {
  const double dB = cB * r, dC = cC * r;
  d[0] = (float)sqrt(fmax(R * R + dB * dB + 2.0 * R * dB * x, 0.0));
  d[1] = (float)r;
  d[2] = (float)sqrt(fmax(R * R + dC * dC - 2.0 * R * dC * x, 0.0));
}

// ---- training (FP32) ----------------------------------------------------------------

// Minibatch features and normalised targets: rows order[(e0 + b) % n] of the samples.
__global__ void k_mlp_batch(const long* __restrict__ sample_idx, const int* __restrict__ order,
                            int n_samples, long e0, int B, const double* __restrict__ V, int npair,
                            size_t plane, const double* __restrict__ rg, const double* __restrict__ Rg,
                            const double* __restrict__ xg, int nR, int nr, double cB, double cC,
                            float* __restrict__ X, float* __restrict__ T) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const long s = sample_idx[order[(e0 + b) % n_samples]];
  const int n = (int)(s / ((long)nR * nr)), m = (int)((s / nr) % nR), i = (int)(s % nr);
  float d[3];
  jacobi_distances(rg[i], Rg[m], xg[n], cB, cC, d);
  for (int c = 0; c < 3; ++c) X[b * 3 + c] = (d[c] - kFeatCenter) / kFeatScale;
  for (int p = 0; p < npair; ++p) T[b * npair + p] = (float)(V[(size_t)p * plane + s] / kOutScale);
}

// Features and normalised targets of given points (gradient checks).
__global__ void k_mlp_feats(const double* __restrict__ dist, const double* __restrict__ v, int n,
                            int npair, float* __restrict__ X, float* __restrict__ T) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  for (int c = 0; c < 3; ++c) X[b * 3 + c] = ((float)dist[b * 3 + c] - kFeatCenter) / kFeatScale;
  for (int p = 0; p < npair; ++p) T[b * npair + p] = (float)(v[b * npair + p] / kOutScale);
}

// Z = A W + b, Aout = silu(Z) (act) or Z.
__global__ void k_dense_fwd(const float* __restrict__ A, int in, const float* __restrict__ W,
                            const float* __restrict__ bias, int out, int B, float* __restrict__ Z,
                            float* __restrict__ Aout, int act) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= B * out) return;
  const int b = q / out, j = q % out;
  float s = bias[j];
  for (int i = 0; i < in; ++i) s += A[b * in + i] * W[i * out + j];
  Z[q] = s;
  Aout[q] = act ? silu_f(s) : s;
}

// dZ = 2 (Y - T) / (B n);  partial sums of the squared error per block.
__global__ void k_mse_grad(const float* __restrict__ Y, const float* __restrict__ T, int n_total,
                           float inv, float* __restrict__ dZ, float* __restrict__ part) {
  __shared__ float red[256];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  float e = 0.0f;
  if (q < n_total) {
    const float d = Y[q] - T[q];
    dZ[q] = 2.0f * d * inv;
    e = d * d;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// dZprev = (dZ W^T) * silu'(Zprev)
__global__ void k_dense_bwd_data(const float* __restrict__ dZ, const float* __restrict__ W, int in,
                                 int out, int B, const float* __restrict__ Zprev,
                                 float* __restrict__ dZprev) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= B * in) return;
  const int b = q / in, i = q % in;
  float s = 0.0f;
  for (int j = 0; j < out; ++j) s += dZ[b * out + j] * W[i * out + j];
  dZprev[q] = s * dsilu_f(Zprev[q]);
}

// gW = A^T dZ, gb = column sums of dZ (thread per weight, i == in gives the bias).
__global__ void k_dense_bwd_w(const float* __restrict__ A, const float* __restrict__ dZ, int in,
                              int out, int B, float* __restrict__ gW, float* __restrict__ gb) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (in + 1) * out) return;
  const int i = q / out, j = q % out;
  float s = 0.0f;
  if (i < in) {
    for (int b = 0; b < B; ++b) s += A[b * in + i] * dZ[b * out + j];
    gW[i * out + j] = s;
  } else {
    for (int b = 0; b < B; ++b) s += dZ[b * out + j];
    gb[j] = s;
  }
}

__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float gq = g[q];
  const float a = b1 * m1[q] + (1.0f - b1) * gq;
  const float v = b2 * m2[q] + (1.0f - b2) * gq * gq;
  m1[q] = a;
  m2[q] = v;
  th[q] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// ---- inference (BF16 weights on the matrix cores) ------------------------------------

struct MlpNet {
  const __bf16* w1t;   // [128][32]   W1^T, inputs padded to 32
  const __bf16* w2t;   // [128][128]  W2^T
  const __bf16* w3t;   // [128][128]  W3^T
  const __bf16* w4t;   // [16][128]   W4^T, outputs padded to 16
  const float* b1;
  const float* b2;
  const float* b3;
  const float* b4;     // [16]
  int npair;
  int s1 = 32;         // row strides (elements) of w1t and of w2t, w3t, w4t
  int s2 = kMlpH;
};

// Packs FP32 master parameters into the inference layout.
__global__ void k_mlp_pack(const float* __restrict__ th, int npair, __bf16* __restrict__ w1t,
                           __bf16* __restrict__ w2t, __bf16* __restrict__ w3t,
                           __bf16* __restrict__ w4t, float* __restrict__ bs) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const float* W1 = th;
  const float* b1 = W1 + 3 * kMlpH;
  const float* W2 = b1 + kMlpH;
  const float* b2 = W2 + kMlpH * kMlpH;
  const float* W3 = b2 + kMlpH;
  const float* b3 = W3 + kMlpH * kMlpH;
  const float* W4 = b3 + kMlpH;
  const float* b4 = W4 + kMlpH * npair;
  if (q < kMlpH * 32) {   // W1^T
    const int o = q / 32, k = q % 32;
    w1t[q] = (__bf16)(k < 3 ? W1[k * kMlpH + o] : 0.0f);
  }
  if (q < kMlpH * kMlpH) {
    const int o = q / kMlpH, k = q % kMlpH;
    w2t[q] = (__bf16)W2[k * kMlpH + o];
    w3t[q] = (__bf16)W3[k * kMlpH + o];
  }
  if (q < 16 * kMlpH) {
    const int o = q / kMlpH, k = q % kMlpH;
    w4t[q] = (__bf16)(o < npair ? W4[k * npair + o] : 0.0f);
  }
  if (q < kMlpH) {
    bs[q] = b1[q];
    bs[kMlpH + q] = b2[q];
    bs[2 * kMlpH + q] = b3[q];
  }
  if (q < 16) bs[3 * kMlpH + q] = q < npair ? b4[q] : 0.0f;
}

__device__ __forceinline__ v8bf ld8(const __bf16* p) { return *reinterpret_cast<const v8bf*>(p); }

// One wavefront evaluates the network on 16 MTP points (MTP tiles of 16).  Lane l
// supplies the features of point 16 mt + l % 16 of each tile (feat[mt], already
// normalised).  Hs: per-wave LDS tile [16 MTP][kMlpLd] bf16; Vs: per-wave LDS
// [16 MTP][16] float receiving V (hartree).  Every weight fragment is read once
// and applied to all MTP tiles; per point the arithmetic does not depend on MTP.
template <int MTP>
__device__ __forceinline__ void mlp_wave(const MlpNet& N, const float (&feat)[MTP][3], __bf16* Hs,
                                         float* Vs, int l) {
  const int row = l & 15, kq = 8 * (l >> 4);
  v4f acc[MTP][8];
  // layer 1: K = 3 (padded to 32)
  {
    v8bf a[MTP];
#pragma unroll
    for (int mt = 0; mt < MTP; ++mt)
#pragma unroll
      for (int t = 0; t < 8; ++t) a[mt][t] = (__bf16)((kq + t) < 3 ? feat[mt][kq + t] : 0.0f);
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
      const v8bf b = ld8(N.w1t + (nt * 16 + row) * N.s1 + kq);
#pragma unroll
      for (int mt = 0; mt < MTP; ++mt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b, v4f{0, 0, 0, 0}, 0, 0, 0);
    }
  }
#pragma unroll
  for (int layer = 0; layer < 3; ++layer) {
    const float* bl = layer == 0 ? N.b1 : (layer == 1 ? N.b2 : N.b3);
    const __bf16* wl = layer == 0 ? N.w2t : N.w3t;
    // bias + SiLU, store as the next A operand (row = point, k = unit)
#pragma unroll
    for (int mt = 0; mt < MTP; ++mt)
#pragma unroll
      for (int nt = 0; nt < 8; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int pr = 16 * mt + 4 * (l >> 4) + v, col = nt * 16 + row;
          Hs[pr * kMlpLd + col] = (__bf16)silu_f(acc[mt][nt][v] + bl[col]);
        }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    v8bf a[MTP][4];
#pragma unroll
    for (int mt = 0; mt < MTP; ++mt)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) a[mt][ks] = ld8(Hs + (16 * mt + row) * kMlpLd + ks * 32 + kq);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (layer < 2) {
#pragma unroll
      for (int nt = 0; nt < 8; ++nt) {
#pragma unroll
        for (int mt = 0; mt < MTP; ++mt) acc[mt][nt] = v4f{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          const v8bf b = ld8(wl + (nt * 16 + row) * N.s2 + ks * 32 + kq);
#pragma unroll
          for (int mt = 0; mt < MTP; ++mt)
            acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt][ks], b, acc[mt][nt], 0, 0, 0);
        }
      }
    } else {
      v4f o[MTP];
#pragma unroll
      for (int mt = 0; mt < MTP; ++mt) o[mt] = v4f{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const v8bf b = ld8(N.w4t + row * N.s2 + ks * 32 + kq);
#pragma unroll
        for (int mt = 0; mt < MTP; ++mt)
          o[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt][ks], b, o[mt], 0, 0, 0);
      }
#pragma unroll
      for (int mt = 0; mt < MTP; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int pr = 16 * mt + 4 * (l >> 4) + v;
          Vs[pr * 16 + row] = (float)kOutScale * (o[mt][v] + N.b4[row]);
        }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void mlp_wave16(const MlpNet& N, const float* feat, __bf16* Hs,
                                           float* Vs, int l) {
  const float f[1][3] = {{feat[0], feat[1], feat[2]}};
  mlp_wave<1>(N, f, Hs, Vs, l);
}

// Inference on arbitrary points (tests, bounds): one wave per 16 points.
__global__ __launch_bounds__(256) void k_mlp_eval(MlpNet N, const double* __restrict__ dist,
                                                  int n_pts, double* __restrict__ out) {
  __shared__ __align__(16) __bf16 hs[4][16 * kMlpLd];
  __shared__ float vs[4][16 * 16];
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int p0 = (blockIdx.x * 4 + w) * 16;
  if (p0 >= n_pts) return;
  const int p = p0 + (l & 15);
  float f[3];
  for (int c = 0; c < 3; ++c) f[c] = p < n_pts ? ((float)dist[(size_t)p * 3 + c] - kFeatCenter) / kFeatScale : 0.0f;
  mlp_wave16(N, f, hs[w], vs[w], l);
  if (l < 16 && p < n_pts)
    for (int q = 0; q < N.npair; ++q) out[(size_t)p * N.npair + q] = (double)vs[w][l * 16 + q];
}

// Same grid-point evaluation: V for every point of the grid, [pair][gamma][R][r].
__global__ __launch_bounds__(256) void k_mlp_grid(MlpNet N, const double* __restrict__ rg,
                                                  const double* __restrict__ Rg,
                                                  const double* __restrict__ xg, int ng, int nR,
                                                  int nr, double cB, double cC,
                                                  double* __restrict__ out) {
  __shared__ __align__(16) __bf16 hs[4][16 * kMlpLd];
  __shared__ float vs[4][16 * 16];
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long n_pts = (long)ng * nR * nr;
  const long p0 = ((long)blockIdx.x * 4 + w) * 16;
  if (p0 >= n_pts) return;
  const long p = p0 + (l & 15);
  float d[3] = {0.f, 0.f, 0.f};
  if (p < n_pts) {
    const int n = (int)(p / ((long)nR * nr)), m = (int)((p / nr) % nR), i = (int)(p % nr);
    jacobi_distances(rg[i], Rg[m], xg[n], cB, cC, d);
  }
  for (int c = 0; c < 3; ++c) d[c] = (d[c] - kFeatCenter) / kFeatScale;
  mlp_wave16(N, d, hs[w], vs[w], l);
  if (l < 16 && p < n_pts)
    for (int q = 0; q < N.npair; ++q) out[(size_t)q * n_pts + p] = (double)vs[w][l * 16 + q];
}

// ---- the step with the potential evaluated by the network --------------------------
// Runs after k_radR_epi<P, NE, true>, which leaves y = T_R u + h in h's place.
// Resident workgroups (the weights staged in LDS once each) take blocks of 256
// grid points (gamma, R, r); a wave evaluates the network on 32 points at a time,
// once per point for every packet and helicity, then finishes the step there:
//   u_{k+1} = D (2 (y + sum_l' V_ll' u_l' - E0 u_l)/dE - D u_{k-1})   (first step: D w).
// Norm partials: one per (workgroup, packet), at normpart_row[packet * gridDim.x + block].
constexpr int kMlpW1Ld = 40;   // LDS row strides of the staged weights (bf16)
constexpr int kMlpWLd = 136;
constexpr size_t kMlpEpiWeights = (size_t)(kMlpH * kMlpW1Ld + 2 * kMlpH * kMlpWLd + 16 * kMlpWLd) * 2 +
                                  (3 * kMlpH + 16) * 4;
constexpr size_t kMlpEpiWave = (size_t)32 * kMlpLd * 2 + 32 * 16 * 4;

__host__ __device__ constexpr size_t mlp_epi_lds(int n_pk) {
  return kMlpEpiWeights + 4 * kMlpEpiWave + (size_t)4 * n_pk * sizeof(double);
}

template <int P, int NE>
__global__ __launch_bounds__(256) void k_mlp_epi(
    MlpNet gnet, const double* __restrict__ rg, const double* __restrict__ Rg,
    const double* __restrict__ xg, double cB, double cC, int ng, int nR, int nr,
    const PkDesc* __restrict__ pks, int n_pk, const double* __restrict__ uk_all,
    double* __restrict__ uprev_all, const typename HType<P>::T* __restrict__ y_all,
    const double* __restrict__ Dsep, double E0, double inv_dE, int first,
    double* __restrict__ normpart, size_t n_wg_total, int* __restrict__ counters,
    int norm_rows, int recorded) {
  constexpr int NPAIR = NE * (NE + 1) / 2;
  extern __shared__ __align__(16) double lds[];
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  __bf16* W1 = reinterpret_cast<__bf16*>(lds);
  __bf16* W2 = W1 + kMlpH * kMlpW1Ld;
  __bf16* W3 = W2 + kMlpH * kMlpWLd;
  __bf16* W4 = W3 + kMlpH * kMlpWLd;
  float* Bs = reinterpret_cast<float*>(W4 + 16 * kMlpWLd);
  char* wbase = reinterpret_cast<char*>(lds) + kMlpEpiWeights;
  __bf16* Hs = reinterpret_cast<__bf16*>(wbase + (size_t)w * kMlpEpiWave);
  float* Vs = reinterpret_cast<float*>(reinterpret_cast<char*>(Hs) + (size_t)32 * kMlpLd * 2);
  double* red = reinterpret_cast<double*>(wbase + 4 * kMlpEpiWave);   // [4][n_pk]
  // stage the weights (16-byte chunks) and biases
  for (int q = threadIdx.x; q < kMlpH * 4; q += 256) {
    const int r = q >> 2, c = (q & 3) * 8;
    *reinterpret_cast<uint4*>(W1 + r * kMlpW1Ld + c) = *reinterpret_cast<const uint4*>(gnet.w1t + r * 32 + c);
  }
  for (int q = threadIdx.x; q < kMlpH * 16; q += 256) {
    const int r = q >> 4, c = (q & 15) * 8;
    *reinterpret_cast<uint4*>(W2 + r * kMlpWLd + c) = *reinterpret_cast<const uint4*>(gnet.w2t + r * kMlpH + c);
    *reinterpret_cast<uint4*>(W3 + r * kMlpWLd + c) = *reinterpret_cast<const uint4*>(gnet.w3t + r * kMlpH + c);
  }
  for (int q = threadIdx.x; q < 16 * 16; q += 256) {
    const int r = q >> 4, c = (q & 15) * 8;
    *reinterpret_cast<uint4*>(W4 + r * kMlpWLd + c) = *reinterpret_cast<const uint4*>(gnet.w4t + r * kMlpH + c);
  }
  for (int q = threadIdx.x; q < 3 * kMlpH + 16; q += 256)
    Bs[q] = q < kMlpH ? gnet.b1[q] : (q < 2 * kMlpH ? gnet.b2[q - kMlpH]
                                                     : (q < 3 * kMlpH ? gnet.b3[q - 2 * kMlpH] : gnet.b4[q - 3 * kMlpH]));
  for (int q = threadIdx.x; q < 4 * n_pk; q += 256) red[q] = 0.0;
  MlpNet net;
  net.w1t = W1;
  net.w2t = W2;
  net.w3t = W3;
  net.w4t = W4;
  net.b1 = Bs;
  net.b2 = Bs + kMlpH;
  net.b3 = Bs + 2 * kMlpH;
  net.b4 = Bs + 3 * kMlpH;
  net.npair = gnet.npair;
  net.s1 = kMlpW1Ld;
  net.s2 = kMlpWLd;
  __syncthreads();
  const int nrow_ix = counters[1];
  double* __restrict__ normpart_row =
      (nrow_ix >= 0 && nrow_ix < norm_rows) ? normpart + (size_t)nrow_ix * n_wg_total : nullptr;
  const long plane = (long)nR * nr;
  const long n_pts = (long)ng * plane;
  const size_t es = (size_t)ng * plane;   // one (helicity, elec) block of a packet
  const int row = l & 15, pl = l & 31, hf = l >> 5;
  for (long b = blockIdx.x; b * 256 < n_pts; b += gridDim.x) {
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
      const long p0 = b * 256 + w * 64 + pass * 32;
      float f[2][3];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) {
        long p = p0 + 16 * mt + row;
        p = p < n_pts ? p : n_pts - 1;
        const int n = (int)(p / plane), m = (int)((p / nr) % nR), i = (int)(p % nr);
        float d[3];
        jacobi_distances(rg[i], Rg[m], xg[n], cB, cC, d);
#pragma unroll
        for (int c = 0; c < 3; ++c) f[mt][c] = (d[c] - kFeatCenter) / kFeatScale;
      }
      mlp_wave<2>(net, f, Hs, Vs, l);
      // lane l finishes point p0 + l % 32 for the helicities of parity l / 32
      const long p = p0 + pl;
      const bool ok = p < n_pts;
      const long pc = ok ? p : n_pts - 1;
      const double dmp = Dsep[pc % nr] * Dsep[nr + (pc % plane) / nr];   // exp(-phi_r) exp(-phi_R)
      double V[NPAIR];
#pragma unroll
      for (int q = 0; q < NPAIR; ++q) V[q] = (double)Vs[pl * 16 + q];
      for (int pk = 0; pk < n_pk; ++pk) {
        const PkDesc d = pks[pk];
        double nsum = 0.0;
        for (int o = hf; o < d.n_om; o += 2) {
          const size_t base = d.off + (size_t)o * NE * es + (size_t)pc;
          double u[NE], y[NE], up[NE];
#pragma unroll
          for (int le = 0; le < NE; ++le) {
            u[le] = uk_all[base + le * es];
            y[le] = (double)y_all[base + le * es];
            up[le] = first ? 0.0 : uprev_all[base + le * es];
          }
#pragma unroll
          for (int le = 0; le < NE; ++le) {
            double sacc = y[le];
#pragma unroll
            for (int l2 = 0; l2 < NE; ++l2) {
              const int a0 = le < l2 ? le : l2, a1 = le < l2 ? l2 : le;
              const int pi = a0 * NE - a0 * (a0 - 1) / 2 + (a1 - a0);
              sacc += V[pi] * u[l2];
            }
            const double wv = (sacc - E0 * u[le]) * inv_dE;
            const double un = first ? dmp * wv : dmp * (2.0 * wv - dmp * up[le]);
            if (ok) {
              uprev_all[base + le * es] = un;
              nsum += un * un;
            }
          }
        }
        for (int off = 32; off > 0; off >>= 1) nsum += __shfl_down(nsum, off, 64);
        if (l == 0) red[w * n_pk + pk] += nsum;
      }
    }
  }
  __syncthreads();
  for (int pk = threadIdx.x; pk < n_pk; pk += 256)
    if (normpart_row)
      normpart_row[(size_t)pk * gridDim.x + blockIdx.x] =
          red[pk] + red[n_pk + pk] + red[2 * n_pk + pk] + red[3 * n_pk + pk];
  if (threadIdx.x == 0) advance_if_last(counters, recorded);
}

}  // namespace tdwp
