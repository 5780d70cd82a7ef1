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

#include <type_traits>

#include "fast_kernels.hpp"
#include "mfma.hpp"

namespace tdwp {

constexpr int kPlaneThreads = 512;   // eight waves per plane
constexpr int kPlaneMTW = 4;         // 16-row tiles (R) per wave work item
constexpr int kPlaneNTW = 2;         // 16-column tiles (r) per wave work item
constexpr int kPlaneRowsPerBatch = 8;   // plane rows whose loads a wave issues together
constexpr int kPlaneMaxCols = 4;        // r values per lane and row: n_r <= 256
constexpr int kPlaneEpiTiles = 2;       // row tiles whose epilogue operands are loaded together

__host__ __device__ constexpr int plane_pad(int n, int ks) { return round_up(round_up(n, 16), ks); }
__host__ __device__ constexpr int plane_ld(int cols) { return cols + 2; }   // floats; rows 8 apart 16 banks apart
__host__ __device__ constexpr size_t plane_tile_bytes(int rows, int cols) {
  return (size_t)rows * plane_ld(cols) * sizeof(float);
}

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

// Bytes of the FP64 rows staged ahead of the tile: the damping factors (r, then
// R) and the flux rows a and d over r, padded to 16 bytes.
__host__ __device__ constexpr int plane_aux_bytes(int nr, int nR) {
  return (int)(((((nr + nR + 1) & ~1) + 2 * nr) * sizeof(double) + 15) / 16 * 16);
}

template <int P>
__global__ __launch_bounds__(kPlaneThreads) __attribute__((amdgpu_waves_per_eu(4)))
void k_plane_epi(PlaneArgs A) {
  using M = Mma<P>;
  using F = Fmt<P>;
  using E = typename F::E;
  extern __shared__ __align__(16) double lds[];
  const int nR = A.nR, nr = A.nr, ng = A.ng;
  double* __restrict__ Ds = lds;                // damping: r factors, then R factors
  double* __restrict__ Fa = lds + ((nr + nR + 1) & ~1);   // flux rows over r (value, derivative)
  double* __restrict__ Fd = Fa + nr;
  float* __restrict__ X = reinterpret_cast<float*>(reinterpret_cast<char*>(lds) + plane_aux_bytes(nr, nR));
  __shared__ double red[kPlaneThreads / 64];
  const int rows_x = plane_pad(nR, M::KS), cols_x = plane_pad(nr, M::KS);
  const int ldx = plane_ld(cols_x);
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = kPlaneThreads / 64;
  const int nrow_ix = A.counters[1];
  double* __restrict__ normpart_row =
      (nrow_ix >= 0 && nrow_ix < A.norm_rows) ? A.normpart + (size_t)nrow_ix * A.n_wg_total : nullptr;
  const int crow = A.record ? A.counters[0] : -1;
  const bool rec_ok = crow >= 0 && crow < A.ring_len;
  double* ring_row = rec_ok ? A.ring_base + (size_t)crow * A.ring_stride : nullptr;
  for (int q = threadIdx.x; q < nr + nR; q += kPlaneThreads) Ds[q] = A.Dsep[q];
  for (int q = threadIdx.x; q < nr; q += kPlaneThreads) {
    Fa[q] = rec_ok ? A.arow[q] : 0.0;
    Fd[q] = rec_ok ? A.drow[q] : 0.0;
  }
  // zero padding of the tile read by the contractions (rows n_R .. rows_x - 1,
  // columns n_r .. cols_x - 1): never overwritten; none for 16-multiple planes
  for (int q = threadIdx.x; q < (rows_x - nR) * cols_x; q += kPlaneThreads)
    X[(nR + q / cols_x) * ldx + q % cols_x] = 0.0f;
  for (int q = threadIdx.x; q < nR * (cols_x - nr); q += kPlaneThreads)
    X[(q / (cols_x - nr)) * ldx + nr + q % (cols_x - nr)] = 0.0f;
  // per-lane column pairs of a row (c = 2 l + 128 j, n_r even) and their flux-row
  // entries
  constexpr int kPairs = kPlaneMaxCols / 2;
  constexpr int RB = kPlaneRowsPerBatch;
  static_assert(RB == 1 || RB == 2 || RB == 4 || RB == 8, "rows per batch");
  const int ppl = (nr + 127) >> 7;
  const size_t plane = (size_t)nR * nr;
  const int MT = (nR + 15) >> 4, NT = (nr + 15) >> 4;
  const int NG = (NT + kPlaneNTW - 1) / kPlaneNTW;
  const int MG = (MT + kPlaneMTW - 1) / kPlaneMTW;
  const int nblk = A.blk_start[A.n_pk];
  double nsum = 0.0;
  int local = 0;
  PkDesc dsc{};
  for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    __syncthreads();   // the previous plane's tile has been read
    // The lane index as an opaque value of this iteration: per-lane offsets are
    // formed where they are used rather than hoisted out of the loop (which holds
    // them in registers across it and spills them).
    int l = lane;
    asm volatile("" : "+v"(l));
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
    for (int m0 = w; m0 < nR; m0 += nw * RB) {
      // 16-byte loads of column pairs (n_r even; rows start at even offsets)
      v2d v[RB][kPairs];
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const int m = m0 + nw * b;
        const int mc = m < nR ? m : nR - 1;
#pragma unroll
        for (int j = 0; j < kPairs; ++j) {
          const int c = 2 * l + 128 * j;
          // byte offset within the plane (32-bit: see the epilogue)
          const unsigned ob = ((unsigned)mc * (unsigned)nr + (unsigned)(c < nr ? c : nr - 2)) * 8u;
          v[b][j] = (j < ppl) ? __builtin_nontemporal_load(reinterpret_cast<const v2d*>(
                                    reinterpret_cast<const char*>(uk) + ob))
                              : v2d{0.0, 0.0};
        }
      }
      // t[2b] = this lane's part of a . u on row b, t[2b + 1] the part of d . u
      double t[2 * RB];
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const int m = m0 + nw * b;
        double sv = 0.0, sd = 0.0;
#pragma unroll
        for (int j = 0; j < kPairs; ++j) {
          const int c = 2 * l + 128 * j;
          if (j < ppl && c < nr && m < nR) {
            const v2d x = v[b][j];
            const v2d fa = *reinterpret_cast<const v2d*>(Fa + c);
            const v2d fd = *reinterpret_cast<const v2d*>(Fd + c);
            *reinterpret_cast<v2f*>(X + m * ldx + c) = v2f{(float)x[0], (float)x[1]};
            sv += fa[0] * x[0] + fa[1] * x[1];
            sd += fd[0] * x[0] + fd[1] * x[1];
            if (rec_ok && m == A.m_inf)
              *reinterpret_cast<v2d*>(ring_row + soff + 2 * nsv + (size_t)local * nr + c) =
                  v2d{x[0] * A.inv_sqrt_dR, x[1] * A.inv_sqrt_dR};
          }
        }
        t[2 * b] = sv;
        t[2 * b + 1] = sd;
      }
      if (rec_ok) {
        // All 2 RB lane sums at once: each exchange over lane bit o halves the
        // quantities a lane holds (it keeps the half its bit selects and adds the
        // partner's copy of it), so after the exchanges over bits 5, 4, ... lane l
        // holds quantity (l >> kLo) & (2 RB - 1) summed over those bits; the low
        // bits finish the sum.
        constexpr int kSteps = RB == 8 ? 4 : RB == 4 ? 3 : RB == 2 ? 2 : 1;
        constexpr int kLo = 6 - kSteps;
#pragma unroll
        for (int st = 0; st < kSteps; ++st) {
          const int o = 32 >> st, half = RB >> st;   // quantities per lane: 2 * half -> half
          const bool up = (l & o) != 0;
#pragma unroll
          for (int q = 0; q < half; ++q) {
            const double keep = up ? t[q + half] : t[q];
            const double send = up ? t[q] : t[q + half];
            t[q] = keep + __shfl_xor(send, o, 64);
          }
        }
        double s = t[0];
#pragma unroll
        for (int o = (1 << kLo) >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        const int q = (l >> kLo) & (2 * RB - 1), b = q >> 1;
        const int m = m0 + nw * b;
        if ((l & ((1 << kLo) - 1)) == 0 && m < nR)
          ring_row[soff + ((q & 1) ? nsv : 0) + lidx0 + m] = s;
      }
    }
    __syncthreads();
    // ---- contractions and epilogue, one work item of MTW x NTW tiles at a time ---
    // Tiles past the plane's last one (ragged sizes) are computed on the last
    // tile's data and not stored.
    for (int g = w; g < MG * NG; g += nw) {
      const int mg = g / NG, ngi = g % NG;
      int mtc[kPlaneMTW], ntc[kPlaneNTW];
#pragma unroll
      for (int a = 0; a < kPlaneMTW; ++a) mtc[a] = min(mg * kPlaneMTW + a, MT - 1);
#pragma unroll
      for (int b = 0; b < kPlaneNTW; ++b) ntc[b] = min(ngi * kPlaneNTW + b, NT - 1);
      typename M::acc_t acc[kPlaneMTW][kPlaneNTW];
#pragma unroll
      for (int a = 0; a < kPlaneMTW; ++a)
#pragma unroll
        for (int b = 0; b < kPlaneNTW; ++b) acc[a][b] = M::zero();
      // T_R u: A = operator rows (global), B = plane columns (LDS)
      const E* TRf = reinterpret_cast<const E*>(A.TRf);
      for (int k0 = 0; k0 < A.kR; k0 += M::KS) {
        typename M::frag_t fa[kPlaneMTW], fb[kPlaneNTW];
#pragma unroll
        for (int a = 0; a < kPlaneMTW; ++a)
          fa[a] = F::frag(TRf + (size_t)mtc[a] * 16 * A.kR, A.kR, A.psR, l, k0);
#pragma unroll
        for (int b = 0; b < kPlaneNTW; ++b) {
          const int c0 = ntc[b] * 16;
          fb[b] = M::load_b([&](int k, int c) { return X[k * ldx + c0 + c]; }, k0, l);
        }
#pragma unroll
        for (int a = 0; a < kPlaneMTW; ++a)
#pragma unroll
          for (int b = 0; b < kPlaneNTW; ++b) M::mma(acc[a][b], fa[a], fb[b]);
      }
      // u T_r: A = plane rows (LDS), B = operator rows (global; T_r is symmetric)
      const E* Trf = reinterpret_cast<const E*>(A.Trf);
      for (int k0 = 0; k0 < A.kr; k0 += M::KS) {
        typename M::frag_t fa[kPlaneMTW], fb[kPlaneNTW];
#pragma unroll
        for (int b = 0; b < kPlaneNTW; ++b)
          fb[b] = F::frag(Trf + (size_t)ntc[b] * 16 * A.kr, A.kr, A.psr, l, k0);
#pragma unroll
        for (int a = 0; a < kPlaneMTW; ++a) {
          const int r0 = mtc[a] * 16;
          fa[a] = M::load_a([&](int row, int k) { return X[(r0 + row) * ldx + k]; }, k0, l);
        }
#pragma unroll
        for (int a = 0; a < kPlaneMTW; ++a)
#pragma unroll
          for (int b = 0; b < kPlaneNTW; ++b) M::mma(acc[a][b], fa[a], fb[b]);
      }
      // epilogue of this work item's outputs: the operands of a group of tiles are
      // loaded together (clamped to the plane), then the outputs are formed and
      // stored where they lie inside it
      // uniform bases of this plane's arrays and 32-bit per-lane byte offsets (a
      // plane fits in LDS as FP32, so 8 n_R n_r is far below 2^32): the loads and
      // stores take the scalar-base form, and no 64-bit lane addresses are held
      const char* __restrict__ hp = reinterpret_cast<const char*>(A.h_all + poff);
      const char* __restrict__ vp = reinterpret_cast<const char*>(A.V + (size_t)n * plane);
      char* __restrict__ pp = reinterpret_cast<char*>(A.uprev_all + poff);
      auto epilogue = [&](auto first_tag) {
        constexpr bool FIRST = decltype(first_tag)::value;
        constexpr int GA = kPlaneEpiTiles;   // row tiles per load group
#pragma unroll
        for (int b = 0; b < kPlaneNTW; ++b) {
          const int nt = ngi * kPlaneNTW + b;
          const int i = nt * 16 + (l & 15);
          const int ic = i < nr ? i : nr - 1;
          const bool col_ok = nt < NT && i < nr;
          const double dr_i = Ds[ic];
#pragma unroll
          for (int a0 = 0; a0 < kPlaneMTW; a0 += GA) {
            float hv[GA][4], vv[GA][4];
            double pv[GA][4];
#pragma unroll
            for (int a = 0; a < GA; ++a)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int mm = (mg * kPlaneMTW + a0 + a) * 16 + M::row(l, v);
                const int mc = mm < nR ? mm : nR - 1;
                const unsigned o = (unsigned)mc * (unsigned)nr + (unsigned)ic;
                hv[a][v] = __builtin_nontemporal_load(reinterpret_cast<const float*>(hp + 4u * o));
                vv[a][v] = *reinterpret_cast<const float*>(vp + 4u * o);
                pv[a][v] = FIRST ? 0.0
                                 : __builtin_nontemporal_load(reinterpret_cast<const double*>(pp + 8u * o));
              }
#pragma unroll
            for (int a = 0; a < GA; ++a)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int mm = (mg * kPlaneMTW + a0 + a) * 16 + M::row(l, v);
                if (!col_ok || mm >= nR) continue;
                const unsigned o = (unsigned)mm * (unsigned)nr + (unsigned)i;
                const double ukv = (double)X[mm * ldx + i];
                const double sacc = (double)acc[a0 + a][b][v] * M::kUnscale + (double)hv[a][v] +
                                    (double)vv[a][v] * ukv;
                const double wv = (sacc - A.E0 * ukv) * A.inv_dE;
                const double dmp = Ds[nr + mm] * dr_i;
                const double un = FIRST ? dmp * wv : dmp * (2.0 * wv - dmp * pv[a][v]);
                __builtin_nontemporal_store(un, reinterpret_cast<double*>(pp + 8u * o));
                nsum += un * un;
              }
          }
        }
      };
      if (A.first)
        epilogue(std::true_type{});
      else
        epilogue(std::false_type{});
    }
    // ---- norm partial of this plane ------------------------------------------------
    for (int off = 32; off > 0; off >>= 1) nsum += __shfl_down(nsum, off, 64);
    if (lane == 0) red[w] = nsum;
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
