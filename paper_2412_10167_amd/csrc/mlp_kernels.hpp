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

// One wavefront evaluates the network on 16 points.  Lane l supplies the
// features of point l % 16 (feat, already normalised).  Hs: per-wave LDS tile
// [16][kMlpLd] bf16; Vs: per-wave LDS [16][16] float receiving V (hartree).
__device__ __forceinline__ void mlp_wave16(const MlpNet& N, const float* feat, __bf16* Hs,
                                           float* Vs, int l) {
  const int row = l & 15, kq = 8 * (l >> 4);
  v4f acc[8];
  // layer 1: K = 3 (padded to 32)
  {
    v8bf a;
#pragma unroll
    for (int t = 0; t < 8; ++t) a[t] = (__bf16)((kq + t) < 3 ? feat[kq + t] : 0.0f);
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
      acc[nt] = v4f{0, 0, 0, 0};
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, ld8(N.w1t + (nt * 16 + row) * 32 + kq), acc[nt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int layer = 0; layer < 3; ++layer) {
    const float* bl = layer == 0 ? N.b1 : (layer == 1 ? N.b2 : N.b3);
    const __bf16* wl = layer == 0 ? N.w2t : N.w3t;
    // bias + SiLU, store as the next A operand (row = point, k = unit)
#pragma unroll
    for (int nt = 0; nt < 8; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int pr = 4 * (l >> 4) + v, col = nt * 16 + row;
        Hs[pr * kMlpLd + col] = (__bf16)silu_f(acc[nt][v] + bl[col]);
      }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    v8bf a[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) a[ks] = ld8(Hs + row * kMlpLd + ks * 32 + kq);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (layer < 2) {
#pragma unroll
      for (int nt = 0; nt < 8; ++nt) {
        acc[nt] = v4f{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              a[ks], ld8(wl + (nt * 16 + row) * kMlpH + ks * 32 + kq), acc[nt], 0, 0, 0);
      }
    } else {
      v4f o = v4f{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ks], ld8(N.w4t + row * kMlpH + ks * 32 + kq), o, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int pr = 4 * (l >> 4) + v;
        Vs[pr * 16 + row] = (float)kOutScale * (o[v] + N.b4[row]);
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
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

// Row selector of the accumulator layout: the item v of lane l that holds tile row rr, or -1.
template <int P> __device__ __forceinline__ int vsel(int l, int rr) {
  if (P == kP64) return ((l >> 4) == (rr & 3)) ? (rr >> 2) : -1;
  return ((l >> 4) == (rr >> 2)) ? (rr & 3) : -1;
}

template <class A> __device__ __forceinline__ double pick(const A& a, int v) {
  return (double)(v == 0 ? a[0] : v == 1 ? a[1] : v == 2 ? a[2] : a[3]);
}

constexpr int kMlpMaxMT = 2;   // R M-tiles per wave (n_R <= 256)
constexpr int kMlpMaxElec = 4;

// k_radR_epi with the potential evaluated by the network at every point of the
// tile instead of read from a table.  Phase 1 forms T_R u for every elec (results
// kept in registers); phase 2 walks the tile rows 16 points at a time: one
// network evaluation per point serves every elec.
template <int P>
__global__ __launch_bounds__(256) void k_radR_epi_mlp(
    const double* __restrict__ uk_all, double* __restrict__ uprev_all,
    const typename HType<P>::T* __restrict__ h_all, const PkDesc* __restrict__ pks,
    const int* __restrict__ blk_start, int n_pk, const typename Fmt<P>::E* __restrict__ Ts,
    const typename Fmt<P>::E* __restrict__ Td, int ldt, int pst, MlpNet net,
    const double* __restrict__ rg, const double* __restrict__ Rg, const double* __restrict__ xg,
    double cB, double cC, const double* __restrict__ D, int ne, int ng, int nR, int nr,
    double E0, double inv_dE, int first, double* __restrict__ normpart, size_t n_wg_total,
    const int* __restrict__ counters, int norm_rows) {
  const int nrow_ix = counters[1];
  double* __restrict__ normpart_row =
      (nrow_ix >= 0 && nrow_ix < norm_rows) ? normpart + (size_t)nrow_ix * n_wg_total : nullptr;
  using M = Mma<P>;
  using F = Fmt<P>;
  using E = typename F::E;
  constexpr int CH = Chunk<P>::CH;
  constexpr int RT = 16;
  extern __shared__ __align__(16) double lds[];
  __shared__ double red[4];
  const int pk = find_packet(blk_start, n_pk, blockIdx.x);
  const int local = blockIdx.x - blk_start[pk];
  const PkDesc dsc = pks[pk];
  const double* __restrict__ uk = uk_all + dsc.off;
  double* __restrict__ uprev = uprev_all + dsc.off;
  const typename HType<P>::T* __restrict__ h = h_all + dsc.off;
  const int nrt = (nr + RT - 1) / RT;
  const int nh = nR >> 1;
  const int kp = round_up(nh, M::KS);
  const int ld = tile_ld<P>(kp);
  const int ps = 2 * RT * ld;
  const int i0 = (local % nrt) * RT;
  const int slab = local / nrt;
  const int o = slab / ng, n = slab % ng;
  const size_t plane = (size_t)nR * nr;
  double* X = lds;                                             // [le][nR][RT]
  E* SD = reinterpret_cast<E*>(lds + (size_t)ne * nR * RT);    // S^T, D^T of one elec
  const size_t sd_bytes = ((size_t)F::PLANES * ps * sizeof(E) + 15) / 16 * 16;
  char* scratch = reinterpret_cast<char*>(SD) + sd_bytes;
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  __bf16* Hs = reinterpret_cast<__bf16*>(scratch + (size_t)w * (16 * kMlpLd * 2 + 16 * 16 * 4));
  float* Vs = reinterpret_cast<float*>(reinterpret_cast<char*>(Hs) + 16 * kMlpLd * 2);
  {
    const int tt = threadIdx.x & 15, r0 = threadIdx.x >> 4;
    const int ii = i0 + tt;
    for (int le = 0; le < ne; ++le) {
      const double* src = uk + ((size_t)(o * ne + le) * ng + n) * plane + ii;
      double* dst = X + (size_t)le * nR * RT + tt;
      for (int mm = r0; mm < nR; mm += 16) dst[mm * RT] = (ii < nr) ? src[(size_t)mm * nr] : 0.0;
    }
  }
  const int MT = (nh + 15) >> 4;
  typename M::acc_t acc[kMlpMaxMT][kMlpMaxElec][2];
#pragma unroll
  for (int le = 0; le < kMlpMaxElec; ++le) {
    if (le >= ne) break;
    __syncthreads();
    const double* Xl = X + (size_t)le * nR * RT;
    {
      const int tt = threadIdx.x & 15;
      for (int k = threadIdx.x >> 4; k < kp; k += 16) {
        double a = 0.0, b = 0.0;
        if (k < nh) {
          a = Xl[k * RT + tt];
          b = Xl[(nR - 1 - k) * RT + tt];
        }
        F::put(SD, ps, tt * ld + k, a + b);
        F::put(SD, ps, RT * ld + tt * ld + k, a - b);
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kMlpMaxMT; ++r) {
      const int mt = w + 4 * r;
      if (mt >= MT) break;
      const E* As = Ts + (size_t)mt * 16 * ldt;
      const E* Ad = Td + (size_t)mt * 16 * ldt;
      acc[r][le][0] = M::zero();
      acc[r][le][1] = M::zero();
      for (int k0 = 0; k0 < kp; k0 += CH * M::KS) {
        typename M::frag_t fs[CH], fd[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q)
          if (k0 + q * M::KS < kp) {
            fs[q] = F::frag(As, ldt, pst, l, k0 + q * M::KS);
            fd[q] = F::frag(Ad, ldt, pst, l, k0 + q * M::KS);
          }
#pragma unroll
        for (int q = 0; q < CH; ++q)
          if (k0 + q * M::KS < kp) {
            M::mma(acc[r][le][0], fs[q], F::frag(SD, ld, ps, l, k0 + q * M::KS));
            M::mma(acc[r][le][1], fd[q], F::frag(SD + RT * ld, ld, ps, l, k0 + q * M::KS));
          }
      }
    }
  }
  const int t = l & 15;
  const int i = i0 + t;
  const double xn = xg[n];
  const double ri = rg[i < nr ? i : nr - 1];
  double nsum = 0.0;
#pragma unroll
  for (int r = 0; r < kMlpMaxMT; ++r) {
    const int mt = w + 4 * r;
    if (mt >= MT) break;
    for (int side = 0; side < 2; ++side)
      for (int rr = 0; rr < 16; ++rr) {
        const int a = mt * 16 + rr;
        if (a >= nh) break;
        const int mm = side ? nR - 1 - a : a;
        float f[3];
        jacobi_distances(ri, Rg[mm], xn, cB, cC, f);
        for (int c = 0; c < 3; ++c) f[c] = (f[c] - kFeatCenter) / kFeatScale;
        mlp_wave16(net, f, Hs, Vs, l);
        const int v = vsel<P>(l, rr);
        if (v < 0 || i >= nr) continue;
        const size_t pt = (size_t)n * plane + (size_t)mm * nr + i;
        double Vm[kMlpMaxElec * (kMlpMaxElec + 1) / 2];
        for (int q = 0; q < net.npair; ++q) Vm[q] = (double)Vs[t * 16 + q];
#pragma unroll
        for (int le = 0; le < kMlpMaxElec; ++le) {
          if (le >= ne) break;
          const double ys = pick(acc[r][le][0], v) * M::kUnscale;
          const double yd = pick(acc[r][le][1], v) * M::kUnscale;
          const size_t idx = (size_t)(o * ne + le) * ng * plane + pt;
          const double ukv = X[((size_t)le * nR + mm) * RT + t];
          double sacc = (side ? ys - yd : ys + yd) + (double)h[idx];
          for (int l2 = 0; l2 < ne; ++l2) {
            const int a0 = le < l2 ? le : l2, a1 = le < l2 ? l2 : le;
            const int pi = a0 * ne - a0 * (a0 - 1) / 2 + (a1 - a0);
            sacc += Vm[pi] * X[((size_t)l2 * nR + mm) * RT + t];
          }
          const double wv = (sacc - E0 * ukv) * inv_dE;
          const double dmp = D[(size_t)mm * nr + i];
          const double un = first ? dmp * wv : dmp * (2.0 * wv - dmp * uprev[idx]);
          uprev[idx] = un;
          nsum += un * un;
        }
      }
  }
  for (int off = 32; off > 0; off >>= 1) nsum += __shfl_down(nsum, off, 64);
  if (l == 0) red[w] = nsum;
  __syncthreads();
  if (threadIdx.x == 0 && normpart_row) normpart_row[dsc.wg_off + local] = red[0] + red[1] + red[2] + red[3];
}

}  // namespace tdwp
