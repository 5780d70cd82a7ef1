// Device kernels of the Chebyshev wave-packet step (FP64 form); included by tdwp.hip.
//
// Packet layout: u[omega][elec][gamma][R][r], r fastest.  One Chebyshev step
// H_s u_k -> u_{k+1} (Sec. 2.2, Eq. wvp-k) is three launches per packet:
//   k_angular_pot : angular + Coriolis terms in the Legendre FBR and the
//                   diabatic potential (Sec. 2.1, items 3-5), -> h
//   k_radial_epi  : sine-DVR kinetic terms along R and r (item 2), plus h,
//                   scaling, three-term recursion and damping, norm partials
//   k_slices      : flux line at r* and analysis line at R_inf of u_{k+1}
// and every kRing steps the energy accumulation (Eq. wvf-chebyshev).
#pragma once
#include <hip/hip_runtime.h>

#include "plan.h"

namespace tdwp {

__device__ __forceinline__ int pair_index(int a, int b, int ne) {
  if (a > b) { int t = a; a = b; b = t; }
  return a * ne - a * (a - 1) / 2 + (b - a);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Angular + Coriolis + potential for one (R index, r tile) of one packet.
// LDS: X[col][n][t] (the packet) and C[col][j][t] (its FBR coefficients),
// col = omega_index * ne + elec.
__global__ void k_angular_pot(const double* __restrict__ u, double* __restrict__ h, int n_om,
                              int om_lo, int ne, int ng, int nR, int nr, int rt,
                              const double* __restrict__ P, const double* __restrict__ U,
                              const double* __restrict__ ell, const int* __restrict__ ang_off,
                              const int* __restrict__ ell_off, const int* __restrict__ n_om_j,
                              const double* __restrict__ Br, const double* __restrict__ BR,
                              double rot_cut, const double* __restrict__ V) {
  extern __shared__ double lds[];
  const int m = blockIdx.y;
  const int i0 = blockIdx.x * rt;
  const int nt = min(rt, nr - i0);
  const int ncol = n_om * ne;
  const int nq = ncol * ng * rt;
  double* X = lds;
  double* C = lds + nq;
  const size_t plane = (size_t)nR * nr;
  const size_t row = (size_t)m * nr + i0;
  for (int q = threadIdx.x; q < nq; q += blockDim.x) {
    const int t = q % rt;
    const int cn = q / rt;
    X[q] = (t < nt) ? u[(size_t)cn * plane + row + t] : 0.0;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nq; q += blockDim.x) {
    const int t = q % rt;
    const int j = (q / rt) % ng;
    const int col = q / (rt * ng);
    const int Om = om_lo + col / ne;
    double s = 0.0;
    if (j >= Om) {
      const double* p = P + ((size_t)Om * ng + j) * ng;
      const double* x = X + (size_t)col * ng * rt + t;
      for (int n = 0; n < ng; ++n) s += p[n] * x[n * rt];
    }
    C[q] = s;
  }
  __syncthreads();
  const double bR = BR[m];
  for (int q = threadIdx.x; q < ne * ng * rt; q += blockDim.x) {
    const int t = q % rt;
    const int j = (q / rt) % ng;
    const int l = q / (rt * ng);
    const int nj = n_om_j[j];
    if (nj <= 0 || t >= nt) continue;
    const double rot = Br[i0 + t] * (double)j * (double)(j + 1);
    const double* Uj = U + ang_off[j];
    const double* lj = ell + ell_off[j];
    double c[kMaxOmega], tt[kMaxOmega];
    for (int a = 0; a < nj; ++a) c[a] = C[((size_t)(a * ne + l) * ng + j) * rt + t];
    for (int b = 0; b < nj; ++b) {
      double s = 0.0;
      for (int a = 0; a < nj; ++a) s += Uj[a * nj + b] * c[a];
      double e = rot + bR * lj[b];
      if (rot_cut > 0.0) e = fmin(e, rot_cut);
      tt[b] = s * e;
    }
    for (int a = 0; a < nj; ++a) {
      double s = 0.0;
      for (int b = 0; b < nj; ++b) s += Uj[a * nj + b] * tt[b];
      C[((size_t)(a * ne + l) * ng + j) * rt + t] = s;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nq; q += blockDim.x) {
    const int t = q % rt;
    if (t >= nt) continue;
    const int n = (q / rt) % ng;
    const int col = q / (rt * ng);
    const int o = col / ne, l = col % ne;
    const int Om = om_lo + o;
    double s = 0.0;
    const double* c = C + (size_t)col * ng * rt + t;
    for (int j = Om; j < ng; ++j) s += P[((size_t)Om * ng + j) * ng + n] * c[j * rt];
    const size_t pt = (size_t)n * plane + row + t;
    for (int l2 = 0; l2 < ne; ++l2)
      s += V[(size_t)pair_index(l, l2, ne) * ng * plane + pt] * X[((size_t)(o * ne + l2) * ng + n) * rt + t];
    h[(size_t)col * ng * plane + pt] = s;
  }
}

// Radial kinetic terms of one R-row tile of one (omega, elec, gamma) slab,
// then w = (h + T u - E0 u)/dE and u_{k+1} = D w (first step) or
// D (2 w - D u_{k-1}), written over u_{k-1}.  One norm partial per workgroup.
__global__ void k_radial_epi(const double* __restrict__ uk, double* __restrict__ uprev,
                             const double* __restrict__ h, const double* __restrict__ TR,
                             const double* __restrict__ Tr, const double* __restrict__ D, int nR,
                             int nr, int rows, double E0, double inv_dE, int first,
                             double* __restrict__ normpart) {
  extern __shared__ double lds[];
  double* X = lds;               // [rows][nr]
  double* Trow = lds + rows * nr;  // [rows][nR]
  __shared__ double red[16];
  const int m0 = blockIdx.x * rows;
  const size_t base = (size_t)blockIdx.y * nR * nr;
  const int nrow = min(rows, nR - m0);
  for (int q = threadIdx.x; q < rows * nr; q += blockDim.x) {
    const int a = q / nr;
    X[q] = (a < nrow) ? uk[base + (size_t)(m0 + a) * nr + q % nr] : 0.0;
  }
  for (int q = threadIdx.x; q < rows * nR; q += blockDim.x) {
    const int a = q / nR;
    Trow[q] = (a < nrow) ? TR[(size_t)(m0 + a) * nR + q % nR] : 0.0;
  }
  __syncthreads();
  double nsum = 0.0;
  for (int q = threadIdx.x; q < nrow * nr; q += blockDim.x) {
    const int a = q / nr, i = q % nr, mm = m0 + a;
    double s = 0.0;
    const double* tr = Trow + a * nR;
    for (int k = 0; k < nR; ++k) s += tr[k] * uk[base + (size_t)k * nr + i];
    const double* xr = X + a * nr;
    for (int k = 0; k < nr; ++k) s += xr[k] * Tr[(size_t)k * nr + i];
    const size_t idx = base + (size_t)mm * nr + i;
    const double wv = (s + h[idx] - E0 * xr[i]) * inv_dE;
    const double d = D[(size_t)mm * nr + i];
    const double un = first ? d * wv : d * (2.0 * wv - d * uprev[idx]);
    uprev[idx] = un;
    nsum += un * un;
  }
  nsum = wave_sum(nsum);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = nsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    normpart[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

// Flux line (a . u, d . u along r for every (omega, elec, gamma, R)) and the
// R_inf line of one packet into its slot of a ring row.  One wavefront per line.
// Lines of every packet are contiguous (line_start[p] .. line_start[p+1]);
// slice_off[p] places the packet's values in the ring row.
__global__ void k_slices(const double* __restrict__ u_all, const long* __restrict__ line_start,
                         const unsigned long* __restrict__ slice_off, int n_pk, int nR, int nr,
                         int m_inf, const double* __restrict__ arow,
                         const double* __restrict__ drow, double inv_sqrt_dR,
                         double* __restrict__ ring_row) {
  const long gline = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (gline >= line_start[n_pk]) return;
  int lo = 0, hi = n_pk - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (line_start[mid] <= gline) lo = mid;
    else hi = mid - 1;
  }
  const int nlines = (int)(line_start[lo + 1] - line_start[lo]);
  const int line = (int)(gline - line_start[lo]);
  const double* u = u_all + (size_t)line_start[lo] * nr;
  double* out = ring_row + slice_off[lo];
  const double* p = u + (size_t)line * nr;
  double sv = 0.0, sd = 0.0;
  for (int i = lane; i < nr; i += 64) {
    const double v = p[i];
    sv += arow[i] * v;
    sd += drow[i] * v;
  }
  sv = wave_sum(sv);
  sd = wave_sum(sd);
  if (lane == 0) {
    out[line] = sv;
    out[nlines + line] = sd;
  }
  if (line % nR == m_inf) {
    double* wout = out + 2 * (size_t)nlines + (size_t)(line / nR) * nr;
    for (int i = lane; i < nr; i += 64) wout[i] = p[i] * inv_sqrt_dR;
  }
}

// Chebyshev energy coefficients c_k(E) = (2 - delta_k0) e^{-ik theta}/(dE sin theta),
// theta = arccos((E_col + E_v0j0 - E0)/dE), for k = k0 .. k0 + count - 1.
// coef layout [2][n_E][kRing] (real, imaginary).
// One launch for every packet: coef[p][2][n_E][ldc] with the packet's E_v0j0.
__global__ void k_coef(double* __restrict__ coef_all, int ldc, int nE, double ecol_min,
                       double ecol_step, const double* __restrict__ E_v0j0, int n_pk, double E0,
                       double dE, long k0, int count) {
  // one thread per (packet, energy, buffered step) of the ldc columns: the columns
  // past count are zeroed, so that the matrix-core accumulation may read whole
  // fragments without masking them
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nE * ldc * n_pk) return;
  const int p = q / (nE * ldc);
  const int e = (q / ldc) % nE, b = q % ldc;
  double* coef = coef_all + (size_t)p * 2 * nE * ldc;
  if (b >= count) {
    coef[(size_t)e * ldc + b] = 0.0;
    coef[((size_t)nE + e) * ldc + b] = 0.0;
    return;
  }
  const double Es = (ecol_min + e * ecol_step + E_v0j0[p] - E0) / dE;
  const double th = acos(Es);
  const long kk = k0 + b;
  const double f = (kk == 0 ? 1.0 : 2.0) / (dE * sin(th));
  const double ph = (double)kk * th;
  coef[(size_t)e * ldc + b] = f * cos(ph);
  coef[((size_t)nE + e) * ldc + b] = -f * sin(ph);
}

// acc[c][e][s] += sum_b coef[c][e][b] ring[b][s] for one packet (s < n_slice).
__global__ void k_accumulate(double* __restrict__ acc, const double* __restrict__ coef,
                             const double* __restrict__ ring, size_t ring_stride, int n_slice,
                             int nE, int e_per_block, int count) {
  __shared__ double cs[2 * 8 * kRing];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int e0 = blockIdx.y * e_per_block;
  const int ne = min(e_per_block, nE - e0);
  for (int q = threadIdx.x; q < 2 * ne * kRing; q += blockDim.x) {
    const int c = q / (ne * kRing), rem = q % (ne * kRing);
    cs[q] = coef[((size_t)c * nE + e0) * kRing + rem];
  }
  __syncthreads();
  if (s >= n_slice) return;
  double x[kRing];
  for (int b = 0; b < count; ++b) x[b] = ring[(size_t)b * ring_stride + s];
  for (int e = 0; e < ne; ++e) {
    double re = 0.0, im = 0.0;
    const double* cr = cs + (size_t)e * kRing;
    const double* ci = cs + (size_t)(ne + e) * kRing;
    for (int b = 0; b < count; ++b) {
      re += cr[b] * x[b];
      im += ci[b] * x[b];
    }
    acc[(size_t)(e0 + e) * n_slice + s] += re;
    acc[((size_t)nE + e0 + e) * n_slice + s] += im;
  }
}

// snap[c][e][t] = acc[c][e][w_off + t]: the analysis-line amplitudes summed over k < k_min_elastic.
__global__ void k_snapshot(double* __restrict__ snap, const double* __restrict__ acc, int nE,
                           int n_slice, int w_off, int n_w) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (size_t)2 * nE * n_w) return;
  const size_t ce = q / n_w, t = q % n_w;
  snap[q] = acc[ce * n_slice + w_off + t];
}

// norms[p][kk] = sum of the packet's workgroup partials of step kk (fixed order).
__global__ void k_norm_reduce(double* __restrict__ norms, const double* __restrict__ part,
                              size_t n_wg_total, const size_t* __restrict__ wg_off,
                              const int* __restrict__ n_wg, int n_packets, int steps) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_packets * steps) return;
  const int p = q / steps, kk = q % steps;
  const double* src = part + (size_t)kk * n_wg_total + wg_off[p];
  double s = 0.0;
  for (int i = 0; i < n_wg[p]; ++i) s += src[i];
  norms[(size_t)p * kNormChunk + kk] = s;
}

// u_0 = pj[n] g[m] chi[i] in block (o0, l0); every other block zero.
__global__ void k_build_packet(double* __restrict__ u, double* __restrict__ uprev, size_t n_values,
                               int o0l0, int ng, int nR, int nr, const double* __restrict__ pj,
                               const double* __restrict__ g, const double* __restrict__ chi) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_values) return;
  const size_t blk = (size_t)ng * nR * nr;
  const size_t col = q / blk, rem = q % blk;
  double v = 0.0;
  if ((int)col == o0l0) {
    const int n = (int)(rem / ((size_t)nR * nr));
    const int mm = (int)((rem / nr) % nR);
    const int i = (int)(rem % nr);
    v = pj[n] * g[mm] * chi[i];
  }
  u[q] = v;
  uprev[q] = 0.0;
}

// Inelastic |S|^2: one workgroup per (channel f, energy e).  chan_i: per channel
// {omega index, elec, j, omega, initial flag}; chan_d: {energy}.
__global__ void k_project(double* __restrict__ p_inel, const double* __restrict__ acc,
                          const double* __restrict__ snap, int snap_valid,
                          const double* __restrict__ chi, const int* __restrict__ chan_i,
                          const double* __restrict__ chan_e, const double* __restrict__ P,
                          const double* __restrict__ g, int n_ch, int nE, int ne, int ng, int nR,
                          int nr, int n_slice, int w_off, int n_w, double ecol_min,
                          double ecol_step, double E_v0j0, double mu, double R_min, double dR,
                          double R_inf) {
  __shared__ double red[4][16];
  const int f = blockIdx.x, e = blockIdx.y;
  const int oi = chan_i[f * 5 + 0], l = chan_i[f * 5 + 1], j = chan_i[f * 5 + 2];
  const int Om = chan_i[f * 5 + 3], initial = chan_i[f * 5 + 4];
  const double* ar = acc + (size_t)e * n_slice + w_off;
  const double* ai = acc + ((size_t)nE + e) * n_slice + w_off;
  const double* sr = snap + (size_t)e * n_w;
  const double* si = snap + ((size_t)nE + e) * n_w;
  const bool late = initial != 0;
  const size_t colbase = (size_t)(oi * ne + l) * ng * nr;
  double re = 0.0, im = 0.0, gre = 0.0, gim = 0.0;
  const double Ecol = ecol_min + e * ecol_step;
  const double K0 = sqrt(2.0 * mu * Ecol);
  if (j >= Om) {
    for (int q = threadIdx.x; q < ng * nr; q += blockDim.x) {
      const int n = q / nr, i = q % nr;
      const double wgt = chi[(size_t)f * nr + i] * P[((size_t)Om * ng + j) * ng + n];
      double vr = ar[colbase + q], vi = ai[colbase + q];
      if (late) {
        if (snap_valid) {
          vr -= sr[colbase + q];
          vi -= si[colbase + q];
        } else {
          vr = 0.0;
          vi = 0.0;
        }
      }
      re += wgt * vr;
      im += wgt * vi;
    }
  }
  for (int mm = threadIdx.x; mm < nR; mm += blockDim.x) {
    const double Rm = R_min + mm * dR;
    const double a = sqrt(dR) * g[mm];
    gre += a * cos(K0 * Rm);
    gim += a * sin(K0 * Rm);
  }
  re = wave_sum(re);
  im = wave_sum(im);
  gre = wave_sum(gre);
  gim = wave_sum(gim);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = re;
    red[1][wv] = im;
    red[2][wv] = gre;
    red[3][wv] = gim;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s[4] = {0, 0, 0, 0};
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k)
      for (int c = 0; c < 4; ++c) s[c] += red[c][k];
    const double Ef = Ecol + E_v0j0 - chan_e[f];
    double out = 0.0;
    if (Ef > 0.0 && j >= Om) {
      const double Kf = sqrt(2.0 * mu * Ef);
      // |S|^2 = K0 Kf |Phi_f|^2 / (mu^2 |g^(K0)|^2); the phase e^{-i Kf R_inf} has unit modulus.
      const double num = K0 * Kf * (s[0] * s[0] + s[1] * s[1]);
      const double den = mu * mu * (s[2] * s[2] + s[3] * s[3]);
      out = num / den;
      (void)R_inf;
    }
    p_inel[(size_t)f * nE + e] = out;
  }
}

// Reactive flux per diabatic state: one workgroup per (elec l, energy e).
__global__ void k_flux(double* __restrict__ p_reac, const double* __restrict__ acc,
                       const double* __restrict__ g, int n_om, int nE, int ne, int ng, int nR,
                       int n_slice, int n_sv, double ecol_min, double ecol_step, double mu,
                       double m_red, double R_min, double dR) {
  __shared__ double red[3][16];
  const int l = blockIdx.x, e = blockIdx.y;
  const double* vr = acc + (size_t)e * n_slice;
  const double* vi = acc + ((size_t)nE + e) * n_slice;
  const double Ecol = ecol_min + e * ecol_step;
  const double K0 = sqrt(2.0 * mu * Ecol);
  double f = 0.0, gre = 0.0, gim = 0.0;
  const int per = ng * nR;
  for (int q = threadIdx.x; q < n_om * per; q += blockDim.x) {
    const int o = q / per, rem = q % per;
    const size_t s = (size_t)(o * ne + l) * per + rem;
    f += vr[s] * vi[n_sv + s] - vi[s] * vr[n_sv + s];
  }
  for (int mm = threadIdx.x; mm < nR; mm += blockDim.x) {
    const double Rm = R_min + mm * dR;
    const double a = sqrt(dR) * g[mm];
    gre += a * cos(K0 * Rm);
    gim += a * sin(K0 * Rm);
  }
  f = wave_sum(f);
  gre = wave_sum(gre);
  gim = wave_sum(gim);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = f;
    red[1][wv] = gre;
    red[2][wv] = gim;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s[3] = {0, 0, 0};
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k)
      for (int c = 0; c < 3; ++c) s[c] += red[c][k];
    p_reac[(size_t)l * nE + e] = K0 * (s[0] / m_red) / (mu * (s[1] * s[1] + s[2] * s[2]));
  }
}

}  // namespace tdwp
