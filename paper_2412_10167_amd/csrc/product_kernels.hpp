// Product line of J = 0 packets (Sec. "Analysis of final states", reactant-
// coordinate-based method): the packet's function on the product points,
//   line[p] = f_p sum_n L[p][n] sum_m wR[p][m] sum_i wr[p][i] u[n][m][i],
// in FP64 (an analysis line, like the flux and R_inf lines), written into the
// ring row after the packet's R_inf line and accumulated in energy with them.
//
// Stage 1 (k_prod_contract): for one (packet, state, gamma node n) and 64
// product points, T[m][p] = sum_i u[n][m][i] wr[p][i] on the FP64 matrix cores
// (rows m of the packet plane, columns p), then Z[n][p] = sum_m wR[p][m] T[m][p]
// reduced in a fixed order (lanes, then waves through LDS).
// Stage 2 (k_prod_finish): line[p] = f_p sum_n L[p][n] Z[n][p], one thread per
// (packet, state, point), into the ring row counters[0].
#pragma once
#include <hip/hip_runtime.h>

#include "mfma.hpp"

namespace tdwp {

constexpr int kProdPts = 64;   // product points per stage-1 workgroup (4 column tiles)
constexpr int kProdMTW = 4;    // row tiles (m) per wave work item

struct ProdDesc {
  unsigned long u_off;     // packet offset in u (values)
  unsigned long line_off;  // offset of the product line in a ring row
  unsigned long z_off;     // offset of the packet's partial contractions in Z
};

// grid: n_pk * ne * ng * ceil(P / 64) workgroups of 256 threads
__global__ __launch_bounds__(256) void k_prod_contract(
    const double* __restrict__ u_all, const ProdDesc* __restrict__ pd, int ne, int ng, int nR,
    int nr, const double* __restrict__ wr, int kr, const double* __restrict__ wR, int kR, int P,
    double* __restrict__ Z) {
  using M = Mma<kP64>;
  __shared__ double red[kProdPts * 16];   // [m-group][point]: at most 16 m-groups
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int npc = (P + kProdPts - 1) / kProdPts;
  int b = blockIdx.x;
  const int pc = b % npc;
  b /= npc;
  const int n = b % ng;
  b /= ng;
  const int le = b % ne;
  const int pk = b / ne;
  const ProdDesc d = pd[pk];
  const size_t plane = (size_t)nR * nr;
  const double* __restrict__ U = u_all + d.u_off + ((size_t)le * ng + n) * plane;
  const int p0 = pc * kProdPts;
  const int MT = (nR + 15) >> 4;
  const int MG = (MT + kProdMTW - 1) / kProdMTW;
  // work items: (m-group mg, column tile ct), ct over the four 16-point tiles
  for (int g = w; g < MG * 4; g += 4) {
    const int mg = g >> 2, ct = g & 3;
    const int pcol = p0 + ct * 16 + (l & 15);
    const int pc_ok = pcol < P ? pcol : P - 1;   // clamped, in-range row of the tables
    M::acc_t acc[kProdMTW];
#pragma unroll
    for (int a = 0; a < kProdMTW; ++a) acc[a] = M::zero();
    for (int k0 = 0; k0 < nr; k0 += 4) {
      const int k = k0 + (l >> 4);
      const int kc = k < nr ? k : nr - 1;
      // B = wr^T: B(k, p) = wr[p][k] (zero-padded to kr; clamped here)
      const double bv = (k < nr) ? wr[(size_t)pc_ok * kr + kc] : 0.0;
#pragma unroll
      for (int a = 0; a < kProdMTW; ++a) {
        const int mt = mg * kProdMTW + a;
        if (mt >= MT) break;
        const int mrow = mt * 16 + (l & 15);
        const double av = (k < nr && mrow < nR) ? U[(size_t)mrow * nr + kc] : 0.0;
        M::mma(acc[a], av, bv);
      }
    }
    // Z partial over this wave's rows m: sum_m wR[p][m] T[m][p]
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < kProdMTW; ++a) {
      const int mt = mg * kProdMTW + a;
      if (mt >= MT) break;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int mrow = mt * 16 + M::row(l, v);
        if (mrow < nR) s += wR[(size_t)pc_ok * kR + mrow] * acc[a][v];
      }
    }
    // lanes l, l ^ 16, l ^ 32, l ^ 48 hold the same point
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    if (l < 16) red[mg * kProdPts + ct * 16 + l] = s;
  }
  __syncthreads();
  if (threadIdx.x < kProdPts) {
    const int p = p0 + threadIdx.x;
    double s = 0.0;
    for (int mg = 0; mg < MG; ++mg) s += red[mg * kProdPts + threadIdx.x];
    if (p < P) Z[d.z_off + ((size_t)le * ng + n) * P + p] = s;
  }
}

// grid: ceil(n_pk * ne * P / 256) workgroups of 256 threads
__global__ __launch_bounds__(256) void k_prod_finish(const ProdDesc* __restrict__ pd, int n_pk,
                                                     int ne, int ng, int P,
                                                     const double* __restrict__ Z,
                                                     const double* __restrict__ wL,
                                                     const double* __restrict__ factor,
                                                     double* __restrict__ ring_base,
                                                     size_t ring_stride, const int* counters,
                                                     int ring_len) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long)n_pk * ne * P) return;
  const int crow = counters[0];
  if (crow < 0 || crow >= ring_len) return;
  const int p = (int)(q % P);
  const int le = (int)((q / P) % ne);
  const int pk = (int)(q / ((long)P * ne));
  const ProdDesc d = pd[pk];
  const double* __restrict__ z = Z + d.z_off + (size_t)le * ng * P + p;
  double s = 0.0;
  for (int n = 0; n < ng; ++n) s += wL[(size_t)p * ng + n] * z[(size_t)n * P];
  ring_base[(size_t)crow * ring_stride + d.line_off + (size_t)le * P + p] = factor[p] * s;
}

}  // namespace tdwp
