// Both radial kinetic terms in one pass over whole (R, r) planes, for one
// electronic state in the mixed-precision forms (Sec. 2.1 items 1-2, then the
// potential, scaling, recursion and damping of Eq. wvp-k).
//
// A plane (packet, Omega, gamma) of u_k is read once from HBM, as FP64 rows of r:
// the flux line at r* (a . u, d . u along r, FP64) and the R_inf line are taken
// from those rows, and an FP32 copy of the plane stays in LDS.  From that one
// copy the matrix cores form
//     C[R][r] = sum_R' T_R[R][R'] u[R'][r] + sum_r' u[R][r'] T_r[r'][r]
// into the same accumulators: the first term takes the operator as the A
// operand and a column of the plane as B, the second the plane's row as A and
// the (symmetric) operator's row as B, so both yield C in (R, r) orientation.
// The epilogue adds the angular terms h of the preceding pass and finishes the
// step as the R pass does: u_{k+1} = D (2 (C + h + V u - E0 u)/dE - D u_{k-1}),
// one norm partial per workgroup.  Against an r pass plus an R pass this drops
// one read of u_k and a read and a write of h per value (and the partial-sum
// buffer of T_r u).
//
// The plane is the unit of work because each contraction needs a whole line of
// its axis: the tile must hold all of R for every r it finishes and all of r for
// every R, so nothing smaller than a plane closes both.  It fits in LDS for
// the batched workload's 128 x 128 planes (66.5 KB in FP32, two workgroups per
// CU); larger planes keep the two-pass form.
#pragma once
#include <hip/hip_runtime.h>

#include "fast_kernels.hpp"
#include "mfma.hpp"

namespace tdwp {

constexpr int kPlaneThreads = 512;   // eight waves per plane
constexpr int kPlaneMTW = 4;         // 16-row tiles (R) per wave work item
constexpr int kPlaneNTW = 2;         // 16-column tiles (r) per wave work item
constexpr int kPlaneRowsPerBatch = 8;   // plane rows whose loads a wave issues together
constexpr int kPlaneMaxCols = 4;        // r values per lane and row: n_r <= 256

__host__ __device__ constexpr int plane_pad(int n, int ks) { return round_up(round_up(n, 16), ks); }
__host__ __device__ constexpr int plane_ld(int cols) { return cols + 2; }   // floats; rows 8 apart 16 banks apart

struct PlaneArgs {
  const double* uk_all;
  double* uprev_all;
  const float* h_all;
  const PkDesc* pks;
  const int* blk_start;     // planes per packet, prefix sums (n_pk + 1)
  int n_pk;
  const void* TRf;          // T_R [rows_R][kR] in compute format (planes psR apart)
  const void* Trf;          // T_r [rows_r][kr]
  int kR, kr, psR, psr;     // padded contraction lengths (row pitch of the tables)
  const float* V;           // FP32 potential [gamma][R][r]
  const double* Dsep;       // damping factors [r (n_r), R (n_R)]
  int ng, nR, nr;
  double E0, inv_dE;
  int first;
  double* normpart;
  size_t n_wg_total;
  int* counters;
  int norm_rows;
  // analysis lines of u_k (the ring row is counters[0])
  int record;
  const unsigned long* slice_off;   // per packet, in a ring row
  const long* line_start;           // per packet: first r-line (n_pk + 1)
  const double* arow;               // flux rows over r (value, derivative)
  const double* drow;
  int m_inf;
  double inv_sqrt_dR;
  double* ring_base;
  size_t ring_stride;
  int ring_len;
};

template <int P>
__global__ __launch_bounds__(kPlaneThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_plane_epi(PlaneArgs A) {
  using M = Mma<P>;
  using F = Fmt<P>;
  using E = typename F::E;
  extern __shared__ __align__(16) double lds[];
  float* __restrict__ X = reinterpret_cast<float*>(lds);
  __shared__ double red[kPlaneThreads / 64];
  const int nR = A.nR, nr = A.nr, ng = A.ng;
  const int rows_x = plane_pad(nR, M::KS), cols_x = plane_pad(nr, M::KS);
  const int ldx = plane_ld(cols_x);
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = kPlaneThreads / 64;
  const int nrow_ix = A.counters[1];
  double* __restrict__ normpart_row =
      (nrow_ix >= 0 && nrow_ix < A.norm_rows) ? A.normpart + (size_t)nrow_ix * A.n_wg_total : nullptr;
  const int crow = A.record ? A.counters[0] : -1;
  const bool rec_ok = crow >= 0 && crow < A.ring_len;
  double* ring_row = rec_ok ? A.ring_base + (size_t)crow * A.ring_stride : nullptr;
  // zero padding of the tile (rows >= n_R, columns >= n_r): never overwritten
  for (int q = threadIdx.x; q < rows_x * ldx; q += kPlaneThreads) {
    const int row = q / ldx, col = q - row * ldx;
    if (row >= nR || col >= nr) X[q] = 0.0f;
  }
  // per-lane column pairs of a row (c = 2 l + 128 j, n_r even) and their flux-row
  // entries
  constexpr int kPairs = kPlaneMaxCols / 2;
  const int ppl = (nr + 127) >> 7;
  double ar[kPlaneMaxCols], dr[kPlaneMaxCols];
#pragma unroll
  for (int j = 0; j < kPlaneMaxCols; ++j) {
    const int c = 2 * l + 128 * (j >> 1) + (j & 1);
    const bool ok = (j >> 1) < ppl && c < nr;
    ar[j] = (rec_ok && ok) ? A.arow[c] : 0.0;
    dr[j] = (rec_ok && ok) ? A.drow[c] : 0.0;
  }
  const size_t plane = (size_t)nR * nr;
  const int MT = (nR + 15) >> 4, NT = (nr + 15) >> 4;
  const int MG = (MT + kPlaneMTW - 1) / kPlaneMTW, NG = (NT + kPlaneNTW - 1) / kPlaneNTW;
  const int nblk = A.blk_start[A.n_pk];
  double nsum = 0.0;
  int local = 0;
  PkDesc dsc{};
  for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    __syncthreads();   // the previous plane's tile has been read
    const int pk = find_packet(A.blk_start, A.n_pk, blk);
    local = blk - A.blk_start[pk];
    dsc = A.pks[pk];
    const int n = local % ng;               // gamma index; local / ng is the helicity block
    const size_t poff = dsc.off + (size_t)local * plane;   // one state: plane = (omega, gamma)
    const double* __restrict__ uk = A.uk_all + poff;
    // ---- load the plane: FP64 rows -> FP32 tile; flux and R_inf lines ----------
    const long lidx0 = (long)local * nR;   // r-line index of row 0 within the packet
    unsigned long soff = 0;
    long nsv = 0;
    if (rec_ok) {
      soff = A.slice_off[pk];
      nsv = A.line_start[pk + 1] - A.line_start[pk];
    }
    typedef double v2d __attribute__((ext_vector_type(2)));
    typedef float v2f __attribute__((ext_vector_type(2)));
    for (int m0 = w; m0 < nR; m0 += nw * kPlaneRowsPerBatch) {
      // 16-byte loads of column pairs (n_r even; rows start at even offsets)
      v2d v[kPlaneRowsPerBatch][kPairs];
#pragma unroll
      for (int b = 0; b < kPlaneRowsPerBatch; ++b) {
        const int m = m0 + nw * b;
        const int mc = m < nR ? m : nR - 1;
#pragma unroll
        for (int j = 0; j < kPairs; ++j) {
          const int c = 2 * l + 128 * j;
          v[b][j] = (j < ppl) ? *reinterpret_cast<const v2d*>(uk + (size_t)mc * nr + (c < nr ? c : nr - 2))
                              : v2d{0.0, 0.0};
        }
      }
#pragma unroll
      for (int b = 0; b < kPlaneRowsPerBatch; ++b) {
        const int m = m0 + nw * b;
        if (m >= nR) break;
        double sv = 0.0, sd = 0.0;
#pragma unroll
        for (int j = 0; j < kPairs; ++j) {
          const int c = 2 * l + 128 * j;
          if (j < ppl && c < nr) {
            const v2d x = v[b][j];
            *reinterpret_cast<v2f*>(X + m * ldx + c) = v2f{(float)x[0], (float)x[1]};
            sv += ar[2 * j] * x[0] + ar[2 * j + 1] * x[1];
            sd += dr[2 * j] * x[0] + dr[2 * j + 1] * x[1];
            if (rec_ok && m == A.m_inf)
              *reinterpret_cast<v2d*>(ring_row + soff + 2 * nsv + (size_t)local * nr + c) =
                  v2d{x[0] * A.inv_sqrt_dR, x[1] * A.inv_sqrt_dR};
          }
        }
        if (rec_ok) {
          for (int off = 32; off > 0; off >>= 1) {
            sv += __shfl_down(sv, off, 64);
            sd += __shfl_down(sd, off, 64);
          }
          if (l == 0) {
            ring_row[soff + lidx0 + m] = sv;
            ring_row[soff + nsv + lidx0 + m] = sd;
          }
        }
      }
    }
    __syncthreads();
    // ---- contractions and epilogue, one work item of MTW x NTW tiles at a time ---
    for (int g = w; g < MG * NG; g += nw) {
      const int mg = g / NG, ngi = g % NG;
      typename M::acc_t acc[kPlaneMTW][kPlaneNTW];
#pragma unroll
      for (int a = 0; a < kPlaneMTW; ++a)
#pragma unroll
        for (int b = 0; b < kPlaneNTW; ++b) acc[a][b] = M::zero();
      // T_R u: A = operator rows (global), B = plane columns (LDS)
      const E* TRf = reinterpret_cast<const E*>(A.TRf);
      for (int k0 = 0; k0 < A.kR; k0 += M::KS) {
        typename M::frag_t fb[kPlaneNTW];
#pragma unroll
        for (int b = 0; b < kPlaneNTW; ++b) {
          const int nt = ngi * kPlaneNTW + b;   // past the last tile: loaded, not used
          const int c0 = (nt < NT ? nt : NT - 1) * 16;
          fb[b] = M::load_b([&](int k, int c) { return X[k * ldx + c0 + c]; }, k0, l);
        }
#pragma unroll
        for (int a = 0; a < kPlaneMTW; ++a) {
          const int mt = mg * kPlaneMTW + a;
          if (mt >= MT) break;
          const typename M::frag_t fa = F::frag(TRf + (size_t)mt * 16 * A.kR, A.kR, A.psR, l, k0);
#pragma unroll
          for (int b = 0; b < kPlaneNTW; ++b)
            if ((ngi * kPlaneNTW + b) < NT) M::mma(acc[a][b], fa, fb[b]);
        }
      }
      // u T_r: A = plane rows (LDS), B = operator rows (global; T_r is symmetric)
      const E* Trf = reinterpret_cast<const E*>(A.Trf);
      for (int k0 = 0; k0 < A.kr; k0 += M::KS) {
        typename M::frag_t fb[kPlaneNTW];
#pragma unroll
        for (int b = 0; b < kPlaneNTW; ++b) {
          const int nt = ngi * kPlaneNTW + b;
          fb[b] = F::frag(Trf + (size_t)(nt < NT ? nt : NT - 1) * 16 * A.kr, A.kr, A.psr, l, k0);
        }
#pragma unroll
        for (int a = 0; a < kPlaneMTW; ++a) {
          const int mt = mg * kPlaneMTW + a;
          if (mt >= MT) break;
          const int r0 = mt * 16;
          const typename M::frag_t fa =
              M::load_a([&](int row, int k) { return X[(r0 + row) * ldx + k]; }, k0, l);
#pragma unroll
          for (int b = 0; b < kPlaneNTW; ++b)
            if ((ngi * kPlaneNTW + b) < NT) M::mma(acc[a][b], fa, fb[b]);
        }
      }
      // epilogue of this work item's outputs
#pragma unroll
      for (int a = 0; a < kPlaneMTW; ++a) {
        const int mt = mg * kPlaneMTW + a;
        if (mt >= MT) break;
#pragma unroll
        for (int b = 0; b < kPlaneNTW; ++b) {
          const int nt = ngi * kPlaneNTW + b;
          const int i = nt * 16 + (l & 15);
          if (nt >= NT || i >= nr) continue;
          const double dr_i = A.Dsep[i];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int mm = mt * 16 + M::row(l, v);
            if (mm >= nR) continue;
            const size_t idx = poff + (size_t)mm * nr + i;
            const double ukv = (double)X[mm * ldx + i];
            const double hv = (double)A.h_all[idx];
            const double vv = (double)A.V[(size_t)n * plane + (size_t)mm * nr + i];
            const double pv = A.first ? 0.0 : A.uprev_all[idx];
            const double sacc = (double)acc[a][b][v] * M::kUnscale + hv + vv * ukv;
            const double wv = (sacc - A.E0 * ukv) * A.inv_dE;
            const double dmp = A.Dsep[nr + mm] * dr_i;
            const double un = A.first ? dmp * wv : dmp * (2.0 * wv - dmp * pv);
            A.uprev_all[idx] = un;
            nsum += un * un;
          }
        }
      }
    }
    // ---- norm partial of this plane ------------------------------------------------
    for (int off = 32; off > 0; off >>= 1) nsum += __shfl_down(nsum, off, 64);
    if (l == 0) red[w] = nsum;
    nsum = 0.0;
    __syncthreads();
    if (threadIdx.x == 0 && normpart_row) {
      double s = 0.0;
      for (int q = 0; q < nw; ++q) s += red[q];
      normpart_row[dsc.wg_off + local] = s;
    }
  }
  if (threadIdx.x == 0) advance_if_last(A.counters, A.record);
}

}  // namespace tdwp
