// Matrix-core form of one Chebyshev step (even n_r, n_R, n_gamma).
//
// Both sine-DVR kinetic matrices are symmetric and persymmetric
// (T[N-1-i][N-1-j] = T[i][j]), and the Gauss-Legendre DVR->FBR rows satisfy
// P[j][ng-1-n] = (-1)^(j+Omega) P[j][n].  In the sum/difference basis
// s = x_a + x_(N-1-a), d = x_a - x_(N-1-a) each contraction therefore splits
// exactly into two half-size ones:
//   (T x)_a = Ts s + Td d,  (T x)_(N-1-a) = Ts s - Td d,  Ts,Td = (A +- B)/2,
// with A, B the upper-left and upper-right (column-reversed) quarters of T;
// and the FBR coefficients of class c = (j + Omega) mod 2 only see s (c = 0)
// or d (c = 1).  This halves the arithmetic of every dense contraction.
//
// Passes per packet and step (Sec. 2.1 items 1-5, Sec. 2.2 Eq. wvp-k):
//   k_radr<P>      h  = T_r u                       (lines along r)
//   k_ang<P>       h += angular + Coriolis terms    (per R, r tile, elec)
//   k_radR_epi<P>  u_{k+1} = D(2 (T_R u + h + V u - E0 u)/dE - D u_{k-1})
//                  (first step: D (...)/dE), plus one norm partial per workgroup.
#pragma once
#include <hip/hip_runtime.h>

#include "mfma.hpp"

namespace tdwp {

constexpr int kRadrLines = 32;   // lines of r per k_radr workgroup (2 M-tiles)
constexpr int kRadRMaxAcc = 12;  // 16x16 accumulators per wave in k_radR_epi (checked on the host)

// ---- h = T_r u along r --------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_radr(const double* __restrict__ u,
                                              typename HType<P>::T* __restrict__ h,
                                              const double* __restrict__ Ts,
                                              const double* __restrict__ Td, int nr, int nhk,
                                              long nlines) {
  using M = Mma<P>;
  extern __shared__ double lds[];
  const int nh = nr >> 1;
  const int kp = round_up(nh, M::KS);
  const int ld = kp + 1;
  double* S = lds;
  double* Dd = lds + kRadrLines * ld;
  const long line0 = (long)blockIdx.x * kRadrLines;
  for (int q = threadIdx.x; q < kRadrLines * kp; q += blockDim.x) {
    const int li = q / kp, k = q % kp;
    const long gl = line0 + li;
    double a = 0.0, b = 0.0;
    if (gl < nlines && k < nh) {
      const double* p = u + gl * nr;
      a = p[k];
      b = p[nr - 1 - k];
    }
    S[li * ld + k] = a + b;
    Dd[li * ld + k] = a - b;
  }
  __syncthreads();
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int NT = (nh + 15) >> 4;
  const int mt = w & 1;
  const double* Sw = S + (16 * mt) * ld;
  const double* Dw = Dd + (16 * mt) * ld;
  auto As = [&](int i, int k) { return Sw[i * ld + k]; };
  auto Ad = [&](int i, int k) { return Dw[i * ld + k]; };
  for (int ntb = (w >> 1); ntb < NT; ntb += 8) {
    typename M::acc_t cs[4], cd[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      cs[g] = M::zero();
      cd[g] = M::zero();
    }
    for (int k0 = 0; k0 < kp; k0 += M::KS) {
      const auto fs = M::load_a(As, k0, l);
      const auto fd = M::load_a(Ad, k0, l);
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int nt = ntb + 2 * g;
        if (nt < NT) {
          auto Bs = [&](int k, int j) { return Ts[(size_t)k * nhk + nt * 16 + j]; };
          auto Bd = [&](int k, int j) { return Td[(size_t)k * nhk + nt * 16 + j]; };
          M::mma(cs[g], fs, M::load_b(Bs, k0, l));
          M::mma(cd[g], fd, M::load_b(Bd, k0, l));
        }
      }
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int nt = ntb + 2 * g;
      if (nt >= NT) continue;
      const int a = nt * 16 + (l & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const long gl = line0 + 16 * mt + M::row(l, v);
        if (gl < nlines && a < nh) {
          const double ys = (double)cs[g][v] * M::kUnscale;
          const double yd = (double)cd[g][v] * M::kUnscale;
          h[gl * nr + a] = (typename HType<P>::T)(ys + yd);
          h[gl * nr + nr - 1 - a] = (typename HType<P>::T)(ys - yd);
        }
      }
    }
  }
}

// ---- h += angular + Coriolis terms -----------------------------------------------
// One workgroup per (r tile of 16, R index m, elec l) of one packet; all helicities.
// Pc: [omega][class][jj][n'] = P^omega[omega + class + 2 jj][n'] (n' < ng/2), zero padded
// to ngk x ngk per (omega, class).
template <int P>
__global__ __launch_bounds__(256) void k_ang(const double* __restrict__ u,
                                             typename HType<P>::T* __restrict__ h, int n_om,
                                             int om_lo, int ne, int ng, int nR, int nr,
                                             const double* __restrict__ Pc, int ngk,
                                             const double* __restrict__ U,
                                             const double* __restrict__ ell,
                                             const int* __restrict__ ang_off,
                                             const int* __restrict__ ell_off,
                                             const int* __restrict__ n_om_j,
                                             const double* __restrict__ Br,
                                             const double* __restrict__ BR, double rot_cut) {
  using M = Mma<P>;
  extern __shared__ double lds[];
  const int ngh = ng >> 1;
  const int kpa = round_up(ngh, M::KS);
  const int i0 = blockIdx.x * 16;
  const int m = blockIdx.y;
  const int le = blockIdx.z;
  const size_t plane = (size_t)nR * nr;
  double* Xp = lds;                               // [o][kpa][16]
  double* Xm = Xp + (size_t)n_om * kpa * 16;      // [o][kpa][16]
  double* C = Xm + (size_t)n_om * kpa * 16;       // [o][ng][16]
  for (int q = threadIdx.x; q < n_om * kpa * 16; q += blockDim.x) {
    const int t = q & 15, k = (q >> 4) % kpa, o = (q >> 4) / kpa;
    const int i = i0 + t;
    double a = 0.0, b = 0.0;
    if (k < ngh && i < nr) {
      const size_t col = (size_t)(o * ne + le) * ng;
      a = u[(col + k) * plane + (size_t)m * nr + i];
      b = u[(col + ng - 1 - k) * plane + (size_t)m * nr + i];
    }
    Xp[q] = a + b;
    Xm[q] = a - b;
  }
  for (int q = threadIdx.x; q < n_om * ng * 16; q += blockDim.x) C[q] = 0.0;
  __syncthreads();
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  // forward: C[o][Omega + c + 2jj][t] = sum_n' Pc[Omega][c][jj][n'] X_c[o][n'][t]
  {
    int item = 0;
    for (int o = 0; o < n_om; ++o) {
      const int Om = om_lo + o;
      for (int c = 0; c < 2; ++c) {
        const int njc = (ng - 1 - (Om + c)) >= 0 ? (ng - 1 - (Om + c)) / 2 + 1 : 0;
        for (int mt = 0; mt * 16 < njc; ++mt, ++item) {
          if ((item & 3) != w) continue;
          const double* Ab = Pc + ((size_t)(Om * 2 + c) * ngk + mt * 16) * ngk;
          const double* Bb = (c ? Xm : Xp) + (size_t)o * kpa * 16;
          auto A = [&](int i, int k) { return Ab[(size_t)i * ngk + k]; };
          auto B = [&](int k, int j) { return Bb[k * 16 + j]; };
          typename M::acc_t acc = M::zero();
          for (int k0 = 0; k0 < kpa; k0 += M::KS) M::mma(acc, M::load_a(A, k0, l), M::load_b(B, k0, l));
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int jj = mt * 16 + M::row(l, v);
            if (jj < njc) C[((size_t)o * ng + Om + c + 2 * jj) * 16 + (l & 15)] = (double)acc[v] * M::kUnscale;
          }
        }
      }
    }
  }
  __syncthreads();
  // Omega mixing at fixed j: U diag(min(B_r j(j+1) + B_R ell_a, rot_cut)) U^T
  const double bR = BR[m];
  for (int q = threadIdx.x; q < ng * 16; q += blockDim.x) {
    const int t = q & 15, j = q >> 4;
    const int nj = n_om_j[j];
    if (nj <= 0 || i0 + t >= nr) continue;
    const double rot = Br[i0 + t] * (double)j * (double)(j + 1);
    const double* Uj = U + ang_off[j];
    const double* lj = ell + ell_off[j];
    double cv[kMaxOmega], tt[kMaxOmega];
    for (int a = 0; a < nj; ++a) cv[a] = C[((size_t)a * ng + j) * 16 + t];
    for (int b = 0; b < nj; ++b) {
      double s = 0.0;
      for (int a = 0; a < nj; ++a) s += Uj[a * nj + b] * cv[a];
      double e = rot + bR * lj[b];
      if (rot_cut > 0.0) e = fmin(e, rot_cut);
      tt[b] = s * e;
    }
    for (int a = 0; a < nj; ++a) {
      double s = 0.0;
      for (int b = 0; b < nj; ++b) s += Uj[a * nj + b] * tt[b];
      C[((size_t)a * ng + j) * 16 + t] = s;
    }
  }
  __syncthreads();
  // back: H_c[o][n'][t] = sum_jj Pc[Omega][c][jj][n'] C[o][Omega + c + 2jj][t]
  {
    int item = 0;
    const int NTh = (ngh + 15) >> 4;
    for (int o = 0; o < n_om; ++o) {
      const int Om = om_lo + o;
      const int nj0 = (ng - 1 - Om) >= 0 ? (ng - 1 - Om) / 2 + 1 : 0;
      const int nj1 = (ng - 2 - Om) >= 0 ? (ng - 2 - Om) / 2 + 1 : 0;
      const int kb = round_up(nj0 > nj1 ? nj0 : nj1, M::KS);
      for (int mt = 0; mt < NTh; ++mt, ++item) {
        if ((item & 3) != w) continue;
        typename M::acc_t acc[2] = {M::zero(), M::zero()};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int njc = c ? nj1 : nj0;
          const double* Ab = Pc + (size_t)(Om * 2 + c) * ngk * ngk + mt * 16;
          const double* Cb = C + ((size_t)o * ng + Om + c) * 16;
          auto A = [&](int i, int k) { return Ab[(size_t)k * ngk + i]; };
          auto B = [&](int k, int j) { return k < njc ? Cb[(size_t)(2 * k) * 16 + j] : 0.0; };
          for (int k0 = 0; k0 < kb; k0 += M::KS) M::mma(acc[c], M::load_a(A, k0, l), M::load_b(B, k0, l));
        }
        const int t = l & 15;
        const int i = i0 + t;
        if (i >= nr) continue;
        const size_t col = (size_t)(o * ne + le) * ng;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = mt * 16 + M::row(l, v);
          if (n >= ngh) continue;
          const double h0 = (double)acc[0][v] * M::kUnscale, h1 = (double)acc[1][v] * M::kUnscale;
          const size_t ia = (col + n) * plane + (size_t)m * nr + i;
          const size_t ib = (col + ng - 1 - n) * plane + (size_t)m * nr + i;
          h[ia] = (typename HType<P>::T)((double)h[ia] + h0 + h1);
          h[ib] = (typename HType<P>::T)((double)h[ib] + h0 - h1);
        }
      }
    }
  }
}

// ---- T_R along R, potential, scaling, recursion, damping, norm partial ---------------
// One workgroup per (r tile of 16*NTR, slab (omega, gamma)) of one packet, all elec.
template <int P, int NTR>
__global__ __launch_bounds__(256) void k_radR_epi(
    const double* __restrict__ uk, double* __restrict__ uprev,
    const typename HType<P>::T* __restrict__ h, const double* __restrict__ Ts,
    const double* __restrict__ Td, int nhk, const double* __restrict__ V,
    const double* __restrict__ D, int ne, int ng, int nR, int nr, double E0, double inv_dE,
    int first, double* __restrict__ normpart) {
  using M = Mma<P>;
  constexpr int RT = 16 * NTR;
  extern __shared__ double lds[];
  __shared__ double red[4];
  const int nh = nR >> 1;
  const int kp = round_up(nh, M::KS);
  const int i0 = blockIdx.x * RT;
  const int o = blockIdx.y / ng, n = blockIdx.y % ng;
  const size_t plane = (size_t)nR * nr;
  double* S = lds;                        // [l][kp][RT]
  double* Dd = lds + (size_t)ne * kp * RT;  // [l][kp][RT]
  for (int q = threadIdx.x; q < ne * kp * RT; q += blockDim.x) {
    const int t = q % RT, b = (q / RT) % kp, le = q / (RT * kp);
    const int i = i0 + t;
    double a = 0.0, c = 0.0;
    if (b < nh && i < nr) {
      const double* base = uk + ((size_t)(o * ne + le) * ng + n) * plane + i;
      a = base[(size_t)b * nr];
      c = base[(size_t)(nR - 1 - b) * nr];
    }
    S[q] = a + c;
    Dd[q] = a - c;
  }
  __syncthreads();
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int MT = (nh + 15) >> 4;
  // Work items (elec, g in {sum, diff}, M-tile), NTR accumulators each, item it on
  // wave it % 4.  Results stay in registers until every wave has read S and Dd.
  const int n_items = ne * 2 * MT;
  constexpr int RES = kRadRMaxAcc / NTR;
  typename M::acc_t res[RES][NTR];
#pragma unroll
  for (int r = 0; r < RES; ++r) {
    const int it = w + 4 * r;
    if (it >= n_items) break;
    const int mt = it % MT, g = (it / MT) & 1, le = it / (2 * MT);
    const double* Ab = (g ? Td : Ts) + (size_t)(mt * 16) * nhk;
    const double* Bb = (g ? Dd : S) + (size_t)le * kp * RT;
    auto A = [&](int i, int k) { return Ab[(size_t)i * nhk + k]; };
#pragma unroll
    for (int nt = 0; nt < NTR; ++nt) res[r][nt] = M::zero();
    for (int k0 = 0; k0 < kp; k0 += M::KS) {
      const auto fa = M::load_a(A, k0, l);
#pragma unroll
      for (int nt = 0; nt < NTR; ++nt) {
        auto B = [&](int k, int j) { return Bb[(size_t)k * RT + nt * 16 + j]; };
        M::mma(res[r][nt], fa, M::load_b(B, k0, l));
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RES; ++r) {
    const int it = w + 4 * r;
    if (it >= n_items) break;
    const int mt = it % MT, g = (it / MT) & 1, le = it / (2 * MT);
    double* Y = (g ? Dd : S) + (size_t)le * kp * RT;
#pragma unroll
    for (int nt = 0; nt < NTR; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = mt * 16 + M::row(l, v);
        if (a < kp) Y[(size_t)a * RT + nt * 16 + (l & 15)] = (double)res[r][nt][v] * M::kUnscale;
      }
  }
  __syncthreads();
  double nsum = 0.0;
  for (int q = threadIdx.x; q < ne * nR * RT; q += blockDim.x) {
    const int t = q % RT, mm = (q / RT) % nR, le = q / (RT * nR);
    const int i = i0 + t;
    if (i >= nr) continue;
    const int a = mm < nh ? mm : nR - 1 - mm;
    const double ys = S[((size_t)le * kp + a) * RT + t];
    const double yd = Dd[((size_t)le * kp + a) * RT + t];
    const size_t pt = (size_t)n * plane + (size_t)mm * nr + i;
    const size_t idx = (size_t)(o * ne + le) * ng * plane + pt;
    double s = (mm < nh ? ys + yd : ys - yd) + (double)h[idx];
    const double ukv = uk[idx];
    for (int l2 = 0; l2 < ne; ++l2) {
      const int a0 = le < l2 ? le : l2, a1 = le < l2 ? l2 : le;
      const int pi = a0 * ne - a0 * (a0 - 1) / 2 + (a1 - a0);
      const double ul2 = (l2 == le) ? ukv : uk[(size_t)(o * ne + l2) * ng * plane + pt];
      s += V[(size_t)pi * ng * plane + pt] * ul2;
    }
    const double wv = (s - E0 * ukv) * inv_dE;
    const double d = D[(size_t)mm * nr + i];
    const double un = first ? d * wv : d * (2.0 * wv - d * uprev[idx]);
    uprev[idx] = un;
    nsum += un * un;
  }
  for (int off = 32; off > 0; off >>= 1) nsum += __shfl_down(nsum, off, 64);
  if (l == 0) red[w] = nsum;
  __syncthreads();
  if (threadIdx.x == 0) normpart[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// ---- energy accumulation: acc[c e][s] += sum_b coef[c e][b] ring[b][s] ----------------
// M = 2 n_E rows (real and imaginary parts), K = buffered steps, N = slice values.
// One workgroup per 32 slice values; wave w owns M-tiles w, w+4, ...
constexpr int kAccMaxMT = 8;   // M-tiles per wave (2 n_E <= 512)
__global__ __launch_bounds__(256) void k_accum_mfma(double* __restrict__ acc,
                                                    const double* __restrict__ coef, int ldc,
                                                    const double* __restrict__ ring,
                                                    size_t ring_stride, int n_slice, int rows,
                                                    int count) {
  using M = Mma<kP64>;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int s0 = blockIdx.x * 32;
  const int MT = (rows + 15) >> 4;
  M::acc_t c[kAccMaxMT][2];
#pragma unroll
  for (int a = 0; a < kAccMaxMT; ++a) c[a][0] = c[a][1] = M::zero();
  const int kc = round_up(count, 4);
  for (int k0 = 0; k0 < kc; k0 += 4) {
    const int kb = k0 + (l >> 4);
    double b[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int s = s0 + nt * 16 + (l & 15);
      b[nt] = (kb < count && s < n_slice) ? ring[(size_t)kb * ring_stride + s] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < kAccMaxMT; ++a) {
      const int mt = w + 4 * a;
      if (mt >= MT) break;
      const int r = mt * 16 + (l & 15);
      const double av = (r < rows && kb < count) ? coef[(size_t)r * ldc + kb] : 0.0;
      M::mma(c[a][0], av, b[0]);
      M::mma(c[a][1], av, b[1]);
    }
  }
#pragma unroll
  for (int a = 0; a < kAccMaxMT; ++a) {
    const int mt = w + 4 * a;
    if (mt >= MT) break;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int s = s0 + nt * 16 + (l & 15);
      if (s >= n_slice) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = mt * 16 + M::row(l, v);
        if (r < rows) acc[(size_t)r * n_slice + s] += c[a][nt][v];
      }
    }
  }
}

}  // namespace tdwp
