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
//   k_ang<P>       h  = angular + Coriolis terms    (per R, r tile, elec)
//   k_radr<P>      h += T_r u                       (lines along r)
//   k_radR_epi<P>  u_{k+1} = D(2 (T_R u + h + V u - E0 u)/dE - D u_{k-1})
//                  (first step: D (...)/dE), plus one norm partial per workgroup.
#pragma once
#include <hip/hip_runtime.h>

#include "mfma.hpp"

namespace tdwp {

// Per-packet description for the batched launches: one launch of each pass
// covers every packet of every unit of the plan.
struct PkDesc {
  unsigned long off;      // offset of the packet in u / h (values)
  unsigned long wg_off;   // first norm partial of the packet
  int n_om, om_lo;
  const double* U;        // angular blocks of the packet's unit
  const double* ell;
  const int* ang_off;
  const int* ell_off;
  const int* n_om_j;
  int n_U, n_ell;         // sizes of U and ell (staged into LDS by k_ang)
  // padded blocks of the register mixing ([j][b][a] with a < the kernel's MAXOM,
  // b < n_om; eigenvalues [j][MAXOM]) in FP64 and FP32, and their sizes
  // the tridiagonal blocks ([j][2 MAXOM + 2]: diagonal, coupling of helicities o and
  // o + 1, smallest and largest eigenvalue)
  const double* mixU;
  const double* mixell;
  const double* mixL;
  const float* mixUf;
  const float* mixellf;
  const float* mixLf;
  int n_mixL;
};

// Index p with start[p] <= b < start[p + 1] (start has n + 1 entries).
// Workgroups are dealt to the eight XCDs of the device in turn.  xcd_order gives
// each XCD a contiguous run of the n blocks (a bijection on the first 8 floor(n/8),
// the rest unchanged), so that neighbouring column tiles, which share cache lines
// of the FP32 arrays, are read through the same L2 (the R pass, whose 16-column
// tiles read h and V in 64-byte runs; for the angular pass it helps some shapes
// and not others, so it is a choice of the autotuner there).
__device__ __forceinline__ int xcd_order(int b, int n) {
  const int n8 = n & ~7;
  return b < n8 ? (b & 7) * (n8 >> 3) + (b >> 3) : b;
}

__device__ __forceinline__ int find_packet(const int* __restrict__ start, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

constexpr int kRadrLines = 32;   // lines of r per k_radr workgroup (2 M-tiles)

// Operand fragments of CH consecutive k-steps are loaded together, so one
// memory latency is paid per CH matrix-core steps instead of per step.
template <int P> struct Chunk { static constexpr int CH = (Mma<P>::KS == 4) ? 8 : 2; };

template <int P> __host__ __device__ constexpr int tile_ld(int kp) {
  return kp + (P == kPBF || P == kPF16 ? 8 : 1);
}

// ---- h += T_r u along r (h holds the angular terms already) ----------------------
// One workgroup per 32 lines (2 M-tiles) of length n_r.  LDS holds the sum and
// difference halves of the lines in compute format; the half-size operators come
// from global tables in compute format (symmetric, so their rows are the
// transposed B operand).  Wave w takes M-tile w % 2 and N-tiles w/2, w/2 + 2, ...
// With record != 0 the workgroup also writes the flux line (a . u, d . u via the
// sum/difference halves of the flux rows) and, for lines at R index m_inf, the
// R_inf line of every packet into the ring row (the same layout k_slices uses).
struct SliceArgs {
  int record;
  int slices_only;                 // record and return (no T_r contraction)
  const long* line_start;          // first line of each packet (n_pk + 1 entries)
  const unsigned long* slice_off;  // packet slice offsets in a ring row
  int n_pk, nR, m_inf;
  const double* a_s;               // flux rows split into sum / difference halves
  const double* a_d;
  const double* d_s;
  const double* d_d;
  double inv_sqrt_dR;
  double* ring_base;               // ring row = ring_base + counters[0] * ring_stride
  size_t ring_stride;
  const int* counters;             // device step counters: [0] ring row, [1] norm row
  int ring_len;                    // rows of the ring (a counter outside 0..ring_len-1 records nothing)
  const int* blk_pk;               // packet holding the first line of each workgroup
};

// ACC: h += T_r u (h holds the angular terms); otherwise h receives T_r u alone
// (the r pass then runs beside the angular pass and the R pass adds both).
// Blocks bid0, bid0 + bstride, ... of the pass.
template <int P, bool ACC>
__device__ __forceinline__ void radr_blk(const double* __restrict__ u,
                                         typename HType<P>::T* __restrict__ h,
                                         const typename Fmt<P>::E* __restrict__ Ts,
                                         const typename Fmt<P>::E* __restrict__ Td, int ldt,
                                         int pst, int nr, long nlines, const SliceArgs& sa,
                                         long bid0, long bstride) {
  using M = Mma<P>;
  using F = Fmt<P>;
  using E = typename F::E;
  constexpr int CH = Chunk<P>::CH;
  extern __shared__ __align__(16) double lds[];
  const int nh = nr >> 1;
  const int kp = round_up(nh, M::KS);
  const int ld = tile_ld<P>(kp);
  const int ps = kRadrLines * ld;
  E* S = reinterpret_cast<E*>(lds);
  E* Dd = S + F::PLANES * ps;
  const int crow = sa.record ? sa.counters[0] : -1;
  const bool rec_ok = crow >= 0 && crow < sa.ring_len;
  double* ring_row = rec_ok ? sa.ring_base + (size_t)crow * sa.ring_stride : nullptr;
  const long nblk = (nlines + kRadrLines - 1) / kRadrLines;
  for (long blk = bid0; blk < nblk; blk += bstride) {
  __syncthreads();   // the previous block's operands have been read
  const long line0 = blk * kRadrLines;
  // wave w loads lines w, w+4, ...; lanes run along the half line; the loads of
  // a group of G lines are issued before any of them is used.  Beside the angular
  // pass (few r blocks per CU) a wave's eight lines go in one group, so twice the
  // bytes are in flight; the standalone pass keeps groups of four (eight would
  // take it past 128 VGPRs, to three waves per SIMD).
  constexpr int LPW = kRadrLines / 4;
  constexpr int G = ACC ? 4 : 8;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  // packet of the block's first line and its bounds (block-uniform loads); a
  // line past the packet's end (a block straddling two packets) looks up its own
  int pk0 = 0;
  long ls0 = 0, ls1 = 0;
  unsigned long so0 = 0;
  if (rec_ok) {
    pk0 = sa.blk_pk[blk];
    ls0 = sa.line_start[pk0];
    ls1 = sa.line_start[pk0 + 1];
    so0 = sa.slice_off[pk0];
  }
  // slice values per packet and the packet's offset in the ring row
  auto nsv_of = [&](int pp) { return pp == pk0 ? ls1 - ls0 : sa.line_start[pp + 1] - sa.line_start[pp]; };
  auto soff_of = [&](int pp) { return pp == pk0 ? so0 : sa.slice_off[pp]; };
#pragma unroll 1
  for (int g0 = 0; g0 < LPW; g0 += G) {
    int pkx[G];
    int lidx[G];
    bool rinf[G];
    double sv[G], sd[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const long gl = line0 + wv + 4 * (g0 + q);
      pkx[q] = 0;
      lidx[q] = 0;
      rinf[q] = false;
      sv[q] = sd[q] = 0.0;
      if (rec_ok && gl < nlines) {
        int pp = pk0;
        long base = ls0;
        if (gl >= ls1) {
          while (pp + 1 < sa.n_pk && sa.line_start[pp + 1] <= gl) ++pp;
          base = sa.line_start[pp];
        }
        pkx[q] = pp;
        lidx[q] = (int)(gl - base);
        rinf[q] = (lidx[q] % sa.nR) == sa.m_inf;
      }
    }
    for (int kc = 0; kc < kp; kc += 64) {
      const int k = kc + lane;
      const int kcl = k < nh ? k : nh - 1;   // loads use clamped, in-range addresses
      double av[G], bv[G];
#pragma unroll
      for (int q = 0; q < G; ++q) {
        long gl = line0 + wv + 4 * (g0 + q);
        gl = gl < nlines ? gl : nlines - 1;
        av[q] = u[gl * nr + kcl];
        bv[q] = u[gl * nr + nr - 1 - kcl];
      }
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const int li = wv + 4 * (g0 + q);
        const long gl = line0 + li;
        const bool ok = gl < nlines && k < nh;
        const double a = ok ? av[q] : 0.0, b = ok ? bv[q] : 0.0;
        if (rec_ok && gl < nlines && k < nh) {
          sv[q] += sa.a_s[k] * (a + b) + sa.a_d[k] * (a - b);
          sd[q] += sa.d_s[k] * (a + b) + sa.d_d[k] * (a - b);
          if (rinf[q]) {
            const long nsv = nsv_of(pkx[q]);
            double* wline = ring_row + soff_of(pkx[q]) + 2 * nsv + (lidx[q] / sa.nR) * nr;
            wline[k] = a * sa.inv_sqrt_dR;
            wline[nr - 1 - k] = b * sa.inv_sqrt_dR;
          }
        }
        if (k < kp) {
          F::put(S, ps, li * ld + k, a + b);
          F::put(Dd, ps, li * ld + k, a - b);
        }
      }
    }
    if (rec_ok) {
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const long gl = line0 + wv + 4 * (g0 + q);
        if (gl >= nlines) continue;
        double x = sv[q], y = sd[q];
        for (int off = 32; off > 0; off >>= 1) {
          x += __shfl_down(x, off, 64);
          y += __shfl_down(y, off, 64);
        }
        if (lane == 0) {
          const long nsv = nsv_of(pkx[q]);
          double* out = ring_row + soff_of(pkx[q]);
          out[lidx[q]] = x;
          out[nsv + lidx[q]] = y;
        }
      }
    }
  }
  if (sa.slices_only) continue;
  __syncthreads();
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int NT = (nh + 15) >> 4;
  const int mt = w & 1;
  const E* Sw = S + 16 * mt * ld;
  const E* Dw = Dd + 16 * mt * ld;
  for (int nt = (w >> 1); nt < NT; nt += 2) {
    // the angular pass has written h already: read this lane's 8 values first
    // (clamped, in-range addresses; outputs outside the range are skipped below)
    typename HType<P>::T hp[4] = {}, hm[4] = {};
    if constexpr (ACC) {
      int a = nt * 16 + (l & 15);
      a = a < nh ? a : nh - 1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        long gl = line0 + 16 * mt + M::row(l, v);
        gl = gl < nlines ? gl : nlines - 1;
        hp[v] = h[gl * nr + a];
        hm[v] = h[gl * nr + nr - 1 - a];
      }
    }
    typename M::acc_t cs = M::zero(), cd = M::zero();
    const E* Bs = Ts + (size_t)nt * 16 * ldt;
    const E* Bd = Td + (size_t)nt * 16 * ldt;
    for (int k0 = 0; k0 < kp; k0 += CH * M::KS) {
      typename M::frag_t bs[CH], bd[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c)
        if (k0 + c * M::KS < kp) {
          bs[c] = F::frag(Bs, ldt, pst, l, k0 + c * M::KS);
          bd[c] = F::frag(Bd, ldt, pst, l, k0 + c * M::KS);
        }
#pragma unroll
      for (int c = 0; c < CH; ++c)
        if (k0 + c * M::KS < kp) {
          M::mma(cs, F::frag(Sw, ld, ps, l, k0 + c * M::KS), bs[c]);
          M::mma(cd, F::frag(Dw, ld, ps, l, k0 + c * M::KS), bd[c]);
        }
    }
    const int a = nt * 16 + (l & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const long gl = line0 + 16 * mt + M::row(l, v);
      if (gl < nlines && a < nh) {
        const double ys = (double)cs[v] * M::kUnscale;
        const double yd = (double)cd[v] * M::kUnscale;
        if constexpr (ACC) {
          h[gl * nr + a] = (typename HType<P>::T)((double)hp[v] + ys + yd);
          h[gl * nr + nr - 1 - a] = (typename HType<P>::T)((double)hm[v] + ys - yd);
        } else {
          h[gl * nr + a] = (typename HType<P>::T)(ys + yd);
          h[gl * nr + nr - 1 - a] = (typename HType<P>::T)(ys - yd);
        }
      }
    }
  }
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_radr(const double* __restrict__ u,
                                              typename HType<P>::T* __restrict__ h,
                                              const typename Fmt<P>::E* __restrict__ Ts,
                                              const typename Fmt<P>::E* __restrict__ Td,
                                              int ldt, int pst, int nr, long nlines,
                                              SliceArgs sa) {
  radr_blk<P, true>(u, h, Ts, Td, ldt, pst, nr, nlines, sa, blockIdx.x, gridDim.x);
}

// Loads the sums / differences of mirrored Gauss-Legendre nodes of every helicity of
// one (R index m, r tile, elec le) column block: X[o][class][t][k] in compute format.
// Each thread owns one column t and the node pairs (k, k + 1) for k = 2 (kf + kstep q);
// the (helicity, q) sequence is the same for every thread, so its bookkeeping is
// wave-uniform, and the block base is uniform with 32-bit per-lane offsets (a packet
// holds fewer than 2^29 values).  Addresses are clamped in range; items are loaded
// four pairs (16 values) at a time.
template <int P, int RT>
__device__ __forceinline__ void ang_load(typename Fmt<P>::E* __restrict__ X,
                                         const double* __restrict__ u, int n_om, int ne, int le,
                                         int ng, int kpa, int ld, int tile, int ps, int m,
                                         int i0, int nr, size_t plane) {
  using F = Fmt<P>;
  using E = typename F::E;
  constexpr int kstep = 256 / RT;   // threads per column
  constexpr int B = 4;
  const int ngh = ng >> 1;
  const int t = threadIdx.x % RT, kf = threadIdx.x / RT;
  const int nq = ((kpa >> 1) + kstep - 1) / kstep;   // pairs per thread and helicity
  const int n_items = n_om * nq;
  const bool okc = i0 + t < nr;
  const double* __restrict__ ub = u + ((size_t)le * ng * plane + (size_t)m * nr + i0);
  const unsigned pl = (unsigned)plane;
  const unsigned tcol = (unsigned)(okc ? t : nr - 1 - i0);
  const unsigned lastp = (unsigned)(ngh - 1) * pl, topp = (unsigned)(ng - 1) * pl;
  const unsigned kfp = (unsigned)(2 * kf) * pl, q_step = (unsigned)(2 * kstep) * pl;
  const unsigned o_step = (unsigned)(ne * ng) * pl;
  E* __restrict__ Xt = X + t * ld + 2 * kf;
  int o_next = 0, q_next = 0;
  for (int it0 = 0; it0 < n_items; it0 += B) {
    int ob[B], qb[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      ob[b] = o_next;
      qb[b] = q_next;
      if (++q_next == nq) {
        q_next = 0;
        ++o_next;
      }
    }
    double av[B][2], bv[B][2];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const bool in = it0 + b < n_items;
      const int o = in ? ob[b] : n_om - 1, q = in ? qb[b] : nq - 1;
      const unsigned so = (unsigned)o * o_step + tcol;
      const unsigned r0 = min(kfp + (unsigned)q * q_step, lastp);
      const unsigned r1 = min(r0 + pl, lastp);
      av[b][0] = ub[so + r0];
      av[b][1] = ub[so + r1];
      bv[b][0] = ub[so + (topp - r0)];
      bv[b][1] = ub[so + (topp - r1)];
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int k = 2 * (kf + kstep * qb[b]);
      if (it0 + b < n_items && k < kpa) {
        const bool ok0 = okc && k < ngh, ok1 = okc && k + 1 < ngh;
        const double a0 = ok0 ? av[b][0] : 0.0, c0 = ok0 ? bv[b][0] : 0.0;
        const double a1 = ok1 ? av[b][1] : 0.0, c1 = ok1 ? bv[b][1] : 0.0;
        E* x = Xt + (ob[b] * 2) * tile + 2 * kstep * qb[b];
        F::put2(x, ps, 0, a0 + c0, a1 + c1);
        F::put2(x + tile, ps, 0, a0 - c0, a1 - c1);
      }
    }
  }
}

__device__ __forceinline__ int n_class(int ng, int Om, int c) {
  const int top = ng - 1 - (Om + c);
  return top >= 0 ? top / 2 + 1 : 0;
}

// Back transform FBR -> DVR of one column block and the h stores:
// H_c[o][n'][t] = sum_jj PcT[Omega][c][n'][jj] C[o][c][t][jj] (C in X's place),
// h[n'] = H_0 + H_1, h[ng-1-n'] = H_0 - H_1.
template <int P, int NT>
__device__ __forceinline__ void ang_back(const typename Fmt<P>::E* __restrict__ X,
                                         typename HType<P>::T* __restrict__ h,
                                         const typename Fmt<P>::E* __restrict__ PcT, size_t tab,
                                         int ngk, int psp, int n_om, int om_lo, int ne, int le,
                                         int ng, int ld, int tile, int ps, int m, int i0, int nr,
                                         size_t plane) {
  using M = Mma<P>;
  using F = Fmt<P>;
  using E = typename F::E;
  constexpr int CH = Chunk<P>::CH;
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ngh = ng >> 1;
  const int NTh = (ngh + 15) >> 4;
  for (int it = w; it < n_om * NTh; it += 4) {
    const int o = it / NTh, mt = it % NTh;
    const int Om = om_lo + o;
    const int nj0 = n_class(ng, Om, 0), nj1 = n_class(ng, Om, 1);
    const int kb = round_up(nj0 > nj1 ? nj0 : nj1, M::KS);
    typename M::acc_t acc[2][NT];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const E* Ab = PcT + (size_t)(Om * 2 + c) * tab + (size_t)mt * 16 * ngk;
      const E* Bb = X + (o * 2 + c) * tile;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[c][nt] = M::zero();
      for (int k0 = 0; k0 < kb; k0 += CH * M::KS) {
        typename M::frag_t fa[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q)
          if (k0 + q * M::KS < kb) fa[q] = F::frag(Ab, ngk, psp, l, k0 + q * M::KS);
#pragma unroll
        for (int q = 0; q < CH; ++q)
          if (k0 + q * M::KS < kb) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
              M::mma(acc[c][nt], fa[q], F::frag(Bb + nt * 16 * ld, ld, ps, l, k0 + q * M::KS));
          }
      }
    }
    // uniform block base, 32-bit per-lane offsets (a packet holds < 2^29 values);
    // the unscaling and the sum / difference in h's precision
    using HT = typename HType<P>::T;
    HT* __restrict__ hb = h + ((size_t)(o * ne + le) * ng * plane + (size_t)m * nr + i0);
    const unsigned pl = (unsigned)plane;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int tc = nt * 16 + (l & 15);
      if (i0 + tc >= nr) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int n = mt * 16 + M::row(l, v);
        if (n >= ngh) continue;
        const HT h0 = (HT)acc[0][nt][v] * (HT)M::kUnscale;
        const HT h1 = (HT)acc[1][nt][v] * (HT)M::kUnscale;
        hb[(unsigned)n * pl + tc] = h0 + h1;
        hb[(unsigned)(ng - 1 - n) * pl + tc] = h0 - h1;
      }
    }
  }
}

// ---- h = angular + Coriolis terms (the first pass of a step) ---------------------
// One workgroup per (r tile of 16 NT columns, R index m, elec l) of one packet,
// all helicities.  Pc / PcT: [omega][class][jj][n'] and [omega][class][n'][jj]
// with P^omega[omega + class + 2 jj][n'] (n' < ng/2), compute format, zero padded
// to ngk x ngk.  LDS tiles X[o][class][t][n'] (sums / differences of mirrored
// nodes) are replaced by the FBR coefficients C[o][class][t][jj] once every wave
// has finished reading them (forward results are held in registers meanwhile).
constexpr int kAngMaxAcc = 12;   // 16x16 accumulators per wave held across the barrier

template <int P, int NT, int MAXOM>
__device__ __forceinline__ void ang_blk(const double* __restrict__ u_all,
                                        typename HType<P>::T* __restrict__ h_all,
                                        const PkDesc* __restrict__ pks,
                                        const int* __restrict__ blk_start, int n_pk, int ne,
                                        int ng, int nR, int nr,
                                        const typename Fmt<P>::E* __restrict__ Pc,
                                        const typename Fmt<P>::E* __restrict__ PcT, int ngk,
                                        int psp, const double* __restrict__ Br,
                                        const double* __restrict__ BR, double rot_cut, int bid,
                                        int xcd) {
  using M = Mma<P>;
  using F = Fmt<P>;
  using E = typename F::E;
  constexpr int CH = Chunk<P>::CH;
  constexpr int RT = 16 * NT;
  constexpr int RES = kAngMaxAcc / NT;
  extern __shared__ __align__(16) double lds[];
  if (xcd) bid = xcd_order(bid, blk_start[n_pk]);
  const int pk = find_packet(blk_start, n_pk, bid);
  const int local = bid - blk_start[pk];
  const PkDesc d = pks[pk];
  const double* __restrict__ u = u_all + d.off;
  typename HType<P>::T* __restrict__ h = h_all + d.off;
  const int n_om = d.n_om, om_lo = d.om_lo;
  const int nrt = (nr + RT - 1) / RT;
  const int ngh = ng >> 1;
  const int kpa = round_up(ngh, M::KS);
  const int ld = tile_ld<P>(kpa);
  const int tile = RT * ld;                 // one (o, class) tile, per plane
  const int ps = n_om * 2 * tile;           // plane stride
  const int i0 = (local % nrt) * RT;
  const int m = (local / nrt) % nR;
  const int le = local / (nrt * nR);
  const size_t plane = (size_t)nR * nr;
  E* X = reinterpret_cast<E*>(lds);         // [o][class][t][k], then C
  // angular blocks of the unit, after the tiles (16-byte aligned)
  double* Ul = lds + (((size_t)F::PLANES * ps * sizeof(E) + 15) / 16) * 2;
  double* elll = Ul + d.n_U;
  for (int q = threadIdx.x; q < d.n_U; q += blockDim.x) Ul[q] = d.U[q];
  for (int q = threadIdx.x; q < d.n_ell; q += blockDim.x) elll[q] = d.ell[q];
  ang_load<P, RT>(X, u, n_om, ne, le, ng, kpa, ld, tile, ps, m, i0, nr, plane);
  __syncthreads();
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int mt_per = (kpa + 15) >> 4;   // forward M-tiles per (omega, class): rows up to kpa
  const size_t tab = (size_t)ngk * ngk;
  typename M::acc_t res[RES][NT];
#pragma unroll
  for (int r = 0; r < RES; ++r) {
    const int it = w + 4 * r;
    const int o = it / (2 * mt_per), c = (it / mt_per) & 1, mt = it % mt_per;
    if (o >= n_om) break;
    const int Om = om_lo + o;
    const E* Ab = Pc + (size_t)(Om * 2 + c) * tab + (size_t)mt * 16 * ngk;
    const E* Bb = X + (o * 2 + c) * tile;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) res[r][nt] = M::zero();
    for (int k0 = 0; k0 < kpa; k0 += CH * M::KS) {
      typename M::frag_t fa[CH];
#pragma unroll
      for (int q = 0; q < CH; ++q)
        if (k0 + q * M::KS < kpa) fa[q] = F::frag(Ab, ngk, psp, l, k0 + q * M::KS);
#pragma unroll
      for (int q = 0; q < CH; ++q)
        if (k0 + q * M::KS < kpa) {
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            M::mma(res[r][nt], fa[q], F::frag(Bb + nt * 16 * ld, ld, ps, l, k0 + q * M::KS));
        }
    }
  }
  __syncthreads();
  // C[o][class][t][jj], jj < kpa (rows past the class size come out zero:
  // the table rows there are zero).  With one helicity the mixing is the factor
  // min(B_r j(j+1) + B_R ell, rot_cut) of each coefficient, applied here.
  const double bR = BR[m];
#pragma unroll
  for (int r = 0; r < RES; ++r) {
    const int it = w + 4 * r;
    const int o = it / (2 * mt_per), c = (it / mt_per) & 1, mt = it % mt_per;
    if (o >= n_om) break;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jj = mt * 16 + M::row(l, v);
        if (jj >= kpa) continue;
        const int t = nt * 16 + (l & 15);
        double val = (double)res[r][nt][v] * M::kUnscale;
        if constexpr (MAXOM == 1) {
          const int j = 2 * jj + om_lo + c;   // FBR index of row jj of class c
          if (j < ng && i0 + t < nr && d.n_om_j[j] > 0) {
            double e = Br[i0 + t] * (double)j * (double)(j + 1) + bR * elll[d.ell_off[j]];
            if (rot_cut > 0.0) e = fmin(e, rot_cut);
            val *= e;
          }
        }
        F::put(X, ps, (o * 2 + c) * tile + t * ld + jj, val);
      }
  }
  __syncthreads();
  // Omega mixing at fixed j: U diag(min(B_r j(j+1) + B_R ell_a, rot_cut)) U^T
  if constexpr (MAXOM > 1)
  for (int q = threadIdx.x; q < ng * RT; q += blockDim.x) {
    const int t = q % RT, j = q / RT;
    const int nj = d.n_om_j[j];
    if (nj <= 0 || i0 + t >= nr) continue;
    const double rot = Br[i0 + t] * (double)j * (double)(j + 1);
    const double* Uj = Ul + d.ang_off[j];
    const double* lj = elll + d.ell_off[j];
    auto pos = [&](int a) {
      const int Om = om_lo + a, c = (j + Om) & 1;
      return (a * 2 + c) * tile + t * ld + (j - Om - c) / 2;
    };
    if (MAXOM == 1 || nj == 1) {   // a single helicity: U = [1]
      double e = rot + bR * lj[0];
      if (rot_cut > 0.0) e = fmin(e, rot_cut);
      F::put(X, ps, pos(0), F::get(X, ps, pos(0)) * e);
      continue;
    }
    if constexpr (MAXOM > 1) {
      double cv[MAXOM], tt[MAXOM];
      for (int a = 0; a < nj; ++a) cv[a] = F::get(X, ps, pos(a));
      for (int b = 0; b < nj; ++b) {
        double sacc = 0.0;
        for (int a = 0; a < nj; ++a) sacc += Uj[a * nj + b] * cv[a];
        double e = rot + bR * lj[b];
        if (rot_cut > 0.0) e = fmin(e, rot_cut);
        tt[b] = sacc * e;
      }
      for (int a = 0; a < nj; ++a) {
        double sacc = 0.0;
        for (int b = 0; b < nj; ++b) sacc += Uj[a * nj + b] * tt[b];
        F::put(X, ps, pos(a), sacc);
      }
    }
  }
  if constexpr (MAXOM > 1) __syncthreads();
  ang_back<P, NT>(X, h, PcT, tab, ngk, psp, n_om, om_lo, ne, le, ng, ld, tile, ps, m, i0, nr,
                  plane);
}

// ---- h = angular + Coriolis terms, helicity mixing in registers -----------------
// Same column blocks as k_ang.  The forward transform is indexed by the absolute
// FBR index j: C[o][j][t] = sum_n' Pf[Omega][0][j][n'] s[o][n'][t]
//                         + sum_n' Pf[Omega][1][j][n'] d[o][n'][t],
// where Pf[Omega][c] keeps the rows of P^Omega whose (j + Omega) mod 2 is c and is
// zero elsewhere (rows j < Omega or j >= ng are zero too).  A wave computes one
// (j tile, t tile) for every helicity, so a lane holds C[.][j][t] for all Omega of
// its rows j and the mixing U diag(min(B_r j(j+1) + B_R ell_a, rot_cut)) U^T runs in
// registers (U and ell staged in LDS).  The mixed coefficients go to
// C[o][class][t][jj] in X's place for the back transform of ang_back.  TPW tiles
// per wave times MAXOM helicities bound the accumulators held across the barrier.
template <int P, int NT, int MAXOM, int TPW>
__device__ __forceinline__ void angr_blk(const double* __restrict__ u_all,
                                         typename HType<P>::T* __restrict__ h_all,
                                         const PkDesc* __restrict__ pks,
                                         const int* __restrict__ blk_start, int n_pk, int ne,
                                         int ng, int nR, int nr,
                                         const typename Fmt<P>::E* __restrict__ Pf, int ngr,
                                         int psf, const typename Fmt<P>::E* __restrict__ PcT,
                                         int ngk, int psp, const double* __restrict__ Br,
                                         const double* __restrict__ BR, double rot_cut, int bid,
                                         int xcd) {
  using M = Mma<P>;
  using F = Fmt<P>;
  using E = typename F::E;
  constexpr int CH = Chunk<P>::CH;
  constexpr int RT = 16 * NT;
  static_assert(TPW * MAXOM <= 16, "accumulators per wave");
  extern __shared__ __align__(16) double lds[];
  if (xcd) bid = xcd_order(bid, blk_start[n_pk]);
  const int pk = find_packet(blk_start, n_pk, bid);
  const int local = bid - blk_start[pk];
  const PkDesc d = pks[pk];
  const double* __restrict__ u = u_all + d.off;
  typename HType<P>::T* __restrict__ h = h_all + d.off;
  const int n_om = d.n_om, om_lo = d.om_lo;
  const int nrt = (nr + RT - 1) / RT;
  const int ngh = ng >> 1;
  const int kpa = round_up(ngh, M::KS);
  const int ld = tile_ld<P>(kpa);
  const int tile = RT * ld;
  const int ps = n_om * 2 * tile;
  const int i0 = (local % nrt) * RT;
  const int m = (local / nrt) % nR;
  const int le = local / (nrt * nR);
  const size_t plane = (size_t)nR * nr;
  E* X = reinterpret_cast<E*>(lds);
  // the unit's tridiagonal l^2 blocks ([j][2 MAXOM + 2]) in the mixing precision,
  // staged after the tiles; the padded eigenvectors stay in global memory
  using MX = typename HType<P>::T;
  MX* Ll = reinterpret_cast<MX*>(reinterpret_cast<char*>(lds) +
                                 ((size_t)F::PLANES * ps * sizeof(E) + 15) / 16 * 16);
  const MX* gU;
  const MX* gl;
  {
    const MX* gL;
    if constexpr (P == kP64) {
      gL = d.mixL;
      gU = d.mixU;
      gl = d.mixell;
    } else {
      gL = d.mixLf;
      gU = d.mixUf;
      gl = d.mixellf;
    }
    for (int q = threadIdx.x; q < d.n_mixL; q += 256) Ll[q] = gL[q];
  }
  ang_load<P, RT>(X, u, n_om, ne, le, ng, kpa, ld, tile, ps, m, i0, nr, plane);
  __syncthreads();
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int MTj = (ng + 15) >> 4;
  const int n_tiles = MTj * NT;
  typename M::acc_t acc[TPW][MAXOM];
#pragma unroll
  for (int tp = 0; tp < TPW; ++tp) {
    const int tix = w + 4 * tp;
    if (tix >= n_tiles) break;
    const int mt = tix % MTj, nt = tix / MTj;
#pragma unroll
    for (int o = 0; o < MAXOM; ++o) {
      acc[tp][o] = M::zero();
      if (o >= n_om) continue;
      const int Om = om_lo + o;
      const E* Ae = Pf + ((size_t)(Om * 2 + 0) * ngr + mt * 16) * ngk;
      const E* Ao = Pf + ((size_t)(Om * 2 + 1) * ngr + mt * 16) * ngk;
      const E* Bs = X + (o * 2 + 0) * tile + nt * 16 * ld;
      const E* Bd = X + (o * 2 + 1) * tile + nt * 16 * ld;
      typename M::acc_t c = M::zero();
      for (int k0 = 0; k0 < kpa; k0 += CH * M::KS) {
        typename M::frag_t fe[CH], fo[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q)
          if (k0 + q * M::KS < kpa) {
            fe[q] = F::frag(Ae, ngk, psf, l, k0 + q * M::KS);
            fo[q] = F::frag(Ao, ngk, psf, l, k0 + q * M::KS);
          }
#pragma unroll
        for (int q = 0; q < CH; ++q)
          if (k0 + q * M::KS < kpa) {
            M::mma(c, fe[q], F::frag(Bs, ld, ps, l, k0 + q * M::KS));
            M::mma(c, fo[q], F::frag(Bd, ld, ps, l, k0 + q * M::KS));
          }
      }
      acc[tp][o] = c;
    }
  }
  __syncthreads();   // X is read by every wave before the coefficients replace it
  const MX bRm = (MX)BR[m];
  const MX cap = (MX)rot_cut;
  const int om_hi = om_lo + n_om - 1;
#pragma unroll
  for (int tp = 0; tp < TPW; ++tp) {
    const int tix = w + 4 * tp;
    if (tix >= n_tiles) break;
    const int mt = tix % MTj, nt = tix / MTj;
    const int t = nt * 16 + (l & 15);
    const int i = i0 + t;
    const MX br = (MX)Br[i < nr ? i : nr - 1];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = mt * 16 + M::row(l, v);
      const int nj = (j < ng) ? (j < om_hi ? j : om_hi) - om_lo + 1 : 0;
      if (nj <= 0) continue;
      // mixing in the accumulation precision (FP64 form: FP64; mixed forms: FP32)
      MX cv[MAXOM];
#pragma unroll
      for (int o = 0; o < MAXOM; ++o)
        cv[o] = (o < nj) ? (MX)acc[tp][o][v] * (MX)M::kUnscale : (MX)0;
      const MX rot = br * (MX)(j * (j + 1));
      const MX* __restrict__ Lj = Ll + j * (2 * MAXOM + 2);
      // The factor is min(rot + B_R l, cap) on the eigenvalues l of the l^2 block.
      // Below the cap for all of them it is rot + B_R L with L the tridiagonal block
      // itself; at the cap for all of them it is the cap.  Otherwise (a band of
      // (j, r) only) the eigenvectors are applied, from global memory.
      const MX elo = rot + bRm * Lj[2 * MAXOM], ehi = rot + bRm * Lj[2 * MAXOM + 1];
      if (MAXOM == 1) {
        MX e = elo;
        if (rot_cut > 0.0) e = e < cap ? e : cap;
        cv[0] *= e;
      } else if (rot_cut <= 0.0 || ehi <= cap) {
        MX outv[MAXOM];
#pragma unroll
        for (int a = 0; a < MAXOM; ++a) {
          MX s = Lj[a] * cv[a];
          if (a > 0) s += Lj[MAXOM + a - 1] * cv[a - 1];
          if (a + 1 < MAXOM) s += Lj[MAXOM + a] * cv[a + 1];
          outv[a] = rot * cv[a] + bRm * s;
        }
#pragma unroll
        for (int a = 0; a < MAXOM; ++a) cv[a] = outv[a];
      } else if (elo >= cap) {
#pragma unroll
        for (int a = 0; a < MAXOM; ++a) cv[a] *= cap;
      } else {
        // one eigenvector column per iteration: project, scale, scatter back.  The
        // padded block is the identity outside the j's own nj x nj block and the
        // coefficients there are zero, so the sums over all MAXOM entries and the
        // unit's n_om columns (a wave-uniform count) add exact zeros only.
        const MX* __restrict__ Uj = gU + (size_t)j * n_om * MAXOM;
        const MX* __restrict__ lj = gl + j * MAXOM;
        MX outv[MAXOM];
#pragma unroll
        for (int a = 0; a < MAXOM; ++a) outv[a] = (MX)0;
        for (int b = 0; b < n_om; ++b) {
          MX uc[MAXOM];
#pragma unroll
          for (int a = 0; a < MAXOM; ++a) uc[a] = Uj[b * MAXOM + a];
          MX sacc = (MX)0;
#pragma unroll
          for (int a = 0; a < MAXOM; ++a) sacc += uc[a] * cv[a];
          MX e = rot + bRm * lj[b];
          if (rot_cut > 0.0) e = e < cap ? e : cap;
          const MX tb = sacc * e;
#pragma unroll
          for (int a = 0; a < MAXOM; ++a) outv[a] += uc[a] * tb;
        }
#pragma unroll
        for (int a = 0; a < MAXOM; ++a) cv[a] = outv[a];
      }
#pragma unroll
      for (int o = 0; o < MAXOM; ++o)
        if (o < nj) {
          const int Om = om_lo + o, c = (j + Om) & 1;
          F::put(X, ps, (o * 2 + c) * tile + t * ld + ((j - Om - c) >> 1), (double)cv[o]);
        }
    }
  }
  __syncthreads();
  ang_back<P, NT>(X, h, PcT, (size_t)ngk * ngk, ngk, psp, n_om, om_lo, ne, le, ng, ld, tile, ps,
                  m, i0, nr, plane);
}

// Arguments of the angular pass and of the r pass, for the launches that run
// both side by side.
struct AngArgs {
  const double* u_all;
  void* h_all;
  const PkDesc* pks;
  const int* blk_start;
  int n_pk, ne, ng, nR, nr;
  const void* Pfwd;   // forward table: Pc (LDS-mixing kernel) or Pf (register mixing)
  int ngr, psf;
  const void* PcT;
  int ngk, psp;
  const double* Br;
  const double* BR;
  double rot_cut;
  int xcd;   // blocks in XCD order (xcd_order)
};
struct RadrArgs {
  const double* u;
  void* h2;           // receives T_r u
  const void* Ts;
  const void* Td;
  int ldt, pst, nr;
  long nlines;
  SliceArgs sa;
};

template <int P, int NT, int MAXOM>
__global__ __launch_bounds__(256) void k_ang(AngArgs a) {
  using E = typename Fmt<P>::E;
  ang_blk<P, NT, MAXOM>(a.u_all, (typename HType<P>::T*)a.h_all, a.pks, a.blk_start, a.n_pk, a.ne,
                        a.ng, a.nR, a.nr, (const E*)a.Pfwd, (const E*)a.PcT, a.ngk, a.psp, a.Br,
                        a.BR, a.rot_cut, blockIdx.x, a.xcd);
}
template <int P, int NT, int MAXOM, int TPW>
__global__ __launch_bounds__(256) void k_angr(AngArgs a) {
  using E = typename Fmt<P>::E;
  angr_blk<P, NT, MAXOM, TPW>(a.u_all, (typename HType<P>::T*)a.h_all, a.pks, a.blk_start, a.n_pk,
                              a.ne, a.ng, a.nR, a.nr, (const E*)a.Pfwd, a.ngr, a.psf,
                              (const E*)a.PcT, a.ngk, a.psp, a.Br, a.BR, a.rot_cut, blockIdx.x, a.xcd);
}
// The angular pass (blocks 0 .. n_ang-1) and the r pass (the rest) in one launch:
// neither reads what the other writes, so their memory latencies overlap.  With one
// helicity the mixed forms ask for four waves per SIMD (the register allocator then
// fits both bodies in 128 registers without spilling; the FP64 form would spill).
template <int P, int MAXOM>
constexpr int fused_waves() { return (P != kP64 && MAXOM <= 1) ? 4 : 1; }

template <int P, int NT, int MAXOM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(fused_waves<P, MAXOM>())))
void k_ang_radr(AngArgs a, RadrArgs r, int n_ang) {
  using E = typename Fmt<P>::E;
  using HT = typename HType<P>::T;
  if ((int)blockIdx.x < n_ang)
    ang_blk<P, NT, MAXOM>(a.u_all, (HT*)a.h_all, a.pks, a.blk_start, a.n_pk, a.ne, a.ng, a.nR,
                          a.nr, (const E*)a.Pfwd, (const E*)a.PcT, a.ngk, a.psp, a.Br, a.BR,
                          a.rot_cut, blockIdx.x, a.xcd);
  else
    radr_blk<P, false>(r.u, (HT*)r.h2, (const E*)r.Ts, (const E*)r.Td, r.ldt, r.pst, r.nr,
                       r.nlines, r.sa, (long)blockIdx.x - n_ang, (long)gridDim.x - n_ang);
}
template <int P, int NT, int MAXOM, int TPW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(fused_waves<P, MAXOM>())))
void k_angr_radr(AngArgs a, RadrArgs r, int n_ang) {
  using E = typename Fmt<P>::E;
  using HT = typename HType<P>::T;
  if ((int)blockIdx.x < n_ang)
    angr_blk<P, NT, MAXOM, TPW>(a.u_all, (HT*)a.h_all, a.pks, a.blk_start, a.n_pk, a.ne, a.ng,
                                a.nR, a.nr, (const E*)a.Pfwd, a.ngr, a.psf, (const E*)a.PcT, a.ngk,
                                a.psp, a.Br, a.BR, a.rot_cut, blockIdx.x, a.xcd);
  else
    radr_blk<P, false>(r.u, (HT*)r.h2, (const E*)r.Ts, (const E*)r.Td, r.ldt, r.pst, r.nr,
                       r.nlines, r.sa, (long)blockIdx.x - n_ang, (long)gridDim.x - n_ang);
}

// ---- T_R along R, potential, scaling, recursion, damping, norm partial ---------------
// (SPLIT: only y = T_R u + h is formed and stored in h's place; the learned-potential
// pass k_mlp_epi adds the potential and finishes the step.)
// One workgroup per (r tile of 16 columns, slab (omega, gamma)) of one packet, all
// NE electronic states.  The raw tile X[elec][R][t] of u_k stays in LDS for the
// epilogue; per elec the sum/difference operand (rows t, contraction over R) is
// built in compute format, and each M-tile work item finishes rows a and n_R-1-a
// from its accumulators.  Global loads are issued in independent batches (the
// tile in groups of kLoadBatch rows; the epilogue operands of an M-tile before its
// contraction) so that one memory latency is paid per batch, not per element.
constexpr int kLoadBatch = 8;

// Called by thread 0 of every workgroup of a step's last pass after its last
// read of the counters: the workgroup that finishes last advances the ring row
// by `recorded` and the norm row by one, and re-arms the arrival count
// counters[2] (every other workgroup has read counters[0..1] by then).
__device__ __forceinline__ void advance_if_last(int* counters, int recorded) {
  const unsigned done = atomicAdd(reinterpret_cast<unsigned*>(counters + 2), 1u);
  if (done == gridDim.x - 1) {
    counters[0] += recorded;
    counters[1] += 1;
    counters[2] = 0;
  }
}
// Row stride (entries) of the u_k tile (padding it to 18, 20 or 24 measured no
// faster while it costs occupancy).
constexpr int kXLd = 16;

// The u_k tile is kept in LDS in h's precision: FP64 in the FP64 form; FP32 in the
// mixed forms, where it feeds the split contraction operand and the local V u and
// E0 u terms of H u (rounding at 2^-24, below the contraction's own error).  The
// mixed forms load one operator chunk at a time and, with one electronic state, ask
// for four waves per SIMD so that registers do not bound occupancy (measured: with
// two or more states the request costs more in spills than it gains).
template <int P, int NE>
constexpr int radR_waves() { return (P == kP64 || NE > 1) ? 1 : 4; }

// ACF: also the partial sums of <u_0|u_{k+1}> of every packet (u_0 in u0_all, packet
// layout; the photodissociation autocorrelation), one per workgroup beside the
// norm partial, in acfpart with the norm partials' layout.
template <int P, int NE, bool SPLIT = false, bool TWO = false, bool ACF = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(radR_waves<P, NE>())))
void k_radR_epi(
    const double* __restrict__ uk_all, double* __restrict__ uprev_all,
    typename HType<P>::T* __restrict__ h_all, const typename HType<P>::T* __restrict__ h2_all,
    const PkDesc* __restrict__ pks,
    const int* __restrict__ blk_start, int n_pk, const typename Fmt<P>::E* __restrict__ Ts,
    const typename Fmt<P>::E* __restrict__ Td, int ldt, int pst,
    const typename HType<P>::T* __restrict__ V,
    const double* __restrict__ Dsep, int ng, int nR, int nr, double E0, double inv_dE,
    int first, double* __restrict__ normpart, size_t n_wg_total, int* __restrict__ counters,
    int norm_rows, int recorded, const double* __restrict__ u0_all,
    double* __restrict__ acfpart) {
  using M = Mma<P>;
  using F = Fmt<P>;
  using E = typename F::E;
  using HT = typename HType<P>::T;
  static_assert(!(ACF && SPLIT), "the overlap needs u_{k+1}, formed only by the full epilogue");
  constexpr int CH = (M::KS == 4) ? Chunk<P>::CH : 1;
  using XT = typename HType<P>::T;
  constexpr int RT = 16;
  extern __shared__ __align__(16) double lds[];
  const int nrow_ix = counters[1];
  double* __restrict__ normpart_row =
      (nrow_ix >= 0 && nrow_ix < norm_rows) ? normpart + (size_t)nrow_ix * n_wg_total : nullptr;
  __shared__ double red[4];
  __shared__ double red_acf[ACF ? 4 : 1];
  const int nblk = blk_start[n_pk];
  // a workgroup takes blocks blockIdx.x, blockIdx.x + gridDim.x, ...
  for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
  __syncthreads();   // the previous block's tile and partials have been read
  const int bx = xcd_order(blk, nblk);
  const int pk = find_packet(blk_start, n_pk, bx);
  const int local = bx - blk_start[pk];
  const PkDesc dsc = pks[pk];
  const double* __restrict__ uk = uk_all + dsc.off;
  double* __restrict__ uprev = uprev_all + dsc.off;
  HT* __restrict__ h = h_all + dsc.off;
  // TWO: T_r u in a separate buffer (the r pass ran beside the angular pass)
  const HT* __restrict__ h2 = TWO ? h2_all + dsc.off : h;
  const int nrt = (nr + RT - 1) / RT;
  const int nh = nR >> 1;
  const int kp = round_up(nh, M::KS);
  const int ld = tile_ld<P>(kp);
  const int ps = 2 * RT * ld;
  const int i0 = (local % nrt) * RT;
  const int slab = local / nrt;
  const int o = slab / ng, n = slab % ng;
  const size_t plane = (size_t)nR * nr;
  XT* X = reinterpret_cast<XT*>(lds);   // [le][nR][kXLd]
  E* SD = reinterpret_cast<E*>(reinterpret_cast<char*>(lds) +
                               (size_t)NE * nR * kXLd * sizeof(XT));   // S^T [t][k], then D^T
  {
    const int tt = threadIdx.x & 15, r0 = threadIdx.x >> 4;
    const int ii = i0 + tt;
    const bool okc = ii < nr;
    const int iic = okc ? ii : nr - 1;   // loads use clamped, in-range addresses
#pragma unroll
    for (int le = 0; le < NE; ++le) {
      const double* src = uk + ((size_t)(o * NE + le) * ng + n) * plane + iic;
      XT* dst = X + (size_t)le * nR * kXLd + tt;
      for (int m0 = r0; m0 < nR; m0 += 16 * kLoadBatch) {
        double vb[kLoadBatch];
#pragma unroll
        for (int b = 0; b < kLoadBatch; ++b) {
          const int mm = m0 + 16 * b;
          vb[b] = src[(size_t)(mm < nR ? mm : nR - 1) * nr];
        }
#pragma unroll
        for (int b = 0; b < kLoadBatch; ++b) {
          const int mm = m0 + 16 * b;
          if (mm < nR) dst[mm * kXLd] = okc ? (XT)vb[b] : (XT)0;
        }
      }
    }
  }
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int MT = (nh + 15) >> 4;
  const int t = l & 15;
  const int i = i0 + t;
  const double dr_i = Dsep[i < nr ? i : nr - 1];   // damping exp(-phi_r(r_i))
  double nsum = 0.0, asum = 0.0;
#pragma unroll 1
  for (int le = 0; le < NE; ++le) {
    __syncthreads();
    const XT* Xl = X + (size_t)le * nR * kXLd;
    {
      const int tt = threadIdx.x & 15;
      for (int k = threadIdx.x >> 4; k < kp; k += 16) {
        double a = 0.0, b = 0.0;
        if (k < nh) {
          a = (double)Xl[k * kXLd + tt];
          b = (double)Xl[(nR - 1 - k) * kXLd + tt];
        }
        F::put(SD, ps, tt * ld + k, a + b);
        F::put(SD, ps, RT * ld + tt * ld + k, a - b);
      }
    }
    __syncthreads();
    for (int mt = w; mt < MT; mt += 4) {
      // epilogue operands of this lane's 8 outputs (rows a and n_R-1-a), loaded
      // before the contraction so their latency overlaps it
      // (addresses clamped into range; outputs outside it are skipped below)
      HT hv[8];
      double dv[8], pv[8];
      HT vv[8][NE];   // the potential in h's precision
      const int ic = i < nr ? i : nr - 1;
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          const int q = 2 * v + side;
          const int a0r = mt * 16 + M::row(l, v);
          const int a = a0r < nh ? a0r : nh - 1;
          const int mm = side ? nR - 1 - a : a;
          const size_t pt = (size_t)n * plane + (size_t)mm * nr + ic;
          const size_t idx = (size_t)(o * NE + le) * ng * plane + pt;
          // with the r pass beside the angular one: h + T_r u, summed in h's precision
          if constexpr (TWO) hv[q] = h[idx] + h2[idx];
          else hv[q] = h[idx];
          if constexpr (!SPLIT) {
            dv[q] = Dsep[nr + mm];   // damping exp(-phi_R(R)); times the r factor below
            pv[q] = first ? 0.0 : uprev[idx];
#pragma unroll
            for (int l2 = 0; l2 < NE; ++l2) {
              const int a0 = le < l2 ? le : l2, a1 = le < l2 ? l2 : le;
              const int pi = a0 * NE - a0 * (a0 - 1) / 2 + (a1 - a0);
              vv[q][l2] = V[(size_t)pi * ng * plane + pt];
            }
          }
        }
      const E* As = Ts + (size_t)mt * 16 * ldt;
      const E* Ad = Td + (size_t)mt * 16 * ldt;
      typename M::acc_t cs = M::zero(), cd = M::zero();
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
            M::mma(cs, fs[q], F::frag(SD, ld, ps, l, k0 + q * M::KS));
            M::mma(cd, fd[q], F::frag(SD + RT * ld, ld, ps, l, k0 + q * M::KS));
          }
      }
      if (i >= nr) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = mt * 16 + M::row(l, v);
        if (a >= nh) continue;
        const double ys = (double)cs[v] * M::kUnscale, yd = (double)cd[v] * M::kUnscale;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          const int q = 2 * v + side;
          const int mm = side ? nR - 1 - a : a;
          const size_t idx = (size_t)(o * NE + le) * ng * plane + (size_t)n * plane + (size_t)mm * nr + i;
          double sacc = (side ? ys - yd : ys + yd) + (double)hv[q];
          if constexpr (SPLIT) {   // T_R u + h only; the potential and the recursion follow
            h[idx] = (HT)sacc;
            continue;
          }
          const double ukv = (double)Xl[mm * kXLd + t];
#pragma unroll
          for (int l2 = 0; l2 < NE; ++l2)
            sacc += (double)vv[q][l2] * (double)X[((size_t)l2 * nR + mm) * kXLd + t];
          const double wv = (sacc - E0 * ukv) * inv_dE;
          const double dmp = dv[q] * dr_i;
          const double un = first ? dmp * wv : dmp * (2.0 * wv - dmp * pv[q]);
          uprev[idx] = un;
          nsum += un * un;
          if constexpr (ACF) asum += u0_all[dsc.off + idx] * un;
        }
      }
    }
  }
  if constexpr (!SPLIT) {
    for (int off = 32; off > 0; off >>= 1) nsum += __shfl_down(nsum, off, 64);
    if (l == 0) red[w] = nsum;
    if constexpr (ACF) {
      for (int off = 32; off > 0; off >>= 1) asum += __shfl_down(asum, off, 64);
      if (l == 0) red_acf[w] = asum;
    }
    __syncthreads();
    if (threadIdx.x == 0 && normpart_row) normpart_row[dsc.wg_off + local] = red[0] + red[1] + red[2] + red[3];
    if constexpr (ACF) {
      if (threadIdx.x == 0 && normpart_row)
        acfpart[(size_t)nrow_ix * n_wg_total + dsc.wg_off + local] =
            red_acf[0] + red_acf[1] + red_acf[2] + red_acf[3];
    }
  }
  }
  if constexpr (!SPLIT) {
    if (threadIdx.x == 0) advance_if_last(counters, recorded);
  }
}

// FP32 copy of an FP64 array (the potential table read by the mixed forms' R pass).
__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, size_t n) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x)
    dst[q] = (float)src[q];
}

// Converts an FP64 operator table to compute format (planes ps elements apart).
template <int P>
__global__ void k_to_format(const double* __restrict__ src, typename Fmt<P>::E* __restrict__ dst,
                            size_t n, int ps) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) Fmt<P>::put(dst, ps, (int)q, src[q]);
}

// ---- energy accumulation: acc[c e][s] += sum_b coef[c e][b] ring[b][s] ----------------
// M = 2 n_E rows (real and imaginary parts), K = buffered steps, N = slice values.
// One workgroup of eight waves per 32 slice values; wave w owns M-tiles w, w+8, ...
// (four waves per SIMD with two workgroups a CU, so one wave's coefficient loads
// hide behind the others' products).
// The workgroup's slab of the ring (K x 32 values, 64 KB at K = 256) is loaded
// into LDS with every load in flight at once, so the ring's HBM latency is paid
// once per workgroup.  The coefficients (shared by all workgroups of a packet,
// L2-resident) are read in chunks of eight ring rows (two matrix-core k-steps):
// within a chunk lane l takes rows 2 (l/16) and 2 (l/16) + 1 for both operands
// (any pairing of k between the operands' fragments is a valid contraction as
// long as it is the same for A and B), so its two coefficients are one 16-byte
// load, and the next chunk's loads are issued before the current chunk's
// products (two register buffers).
constexpr int kAccThreads = 512;                  // eight waves
constexpr int kAccWaves = kAccThreads / 64;
constexpr int kAccMaxMT = 4;                      // M-tiles per wave (2 n_E <= 16 * 4 * 8)
constexpr int kAccCols = 32;                      // slice values per workgroup
constexpr int kAccChunks = 32;                    // chunks of eight steps in a full ring
struct AccDesc {
  unsigned long acc_off;    // accumulators of the packet [2 n_E][n_slice]
  unsigned long slice_off;  // the packet's slice values in a ring row
  int n_slice;
};

__global__ __launch_bounds__(kAccThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_accum_mfma(double* __restrict__ acc_all,
                                                       const double* __restrict__ coef_all, int ldc,
                                                       const double* __restrict__ ring_all,
                                                       size_t ring_stride,
                                                       const AccDesc* __restrict__ ads,
                                                       const int* __restrict__ blk_start, int n_pk,
                                                       int rows, int count) {
  using M = Mma<kP64>;
  typedef double v2d __attribute__((ext_vector_type(2)));
  extern __shared__ __align__(16) double slab[];   // [8 * nch][kAccCols]
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int pk = find_packet(blk_start, n_pk, blockIdx.x);
  const AccDesc ad = ads[pk];
  double* __restrict__ acc = acc_all + ad.acc_off;
  const double* __restrict__ coef = coef_all + (size_t)pk * rows * ldc;
  const double* __restrict__ ring = ring_all + ad.slice_off;
  const int n_slice = ad.n_slice;
  const int s0 = (blockIdx.x - blk_start[pk]) * kAccCols;
  const int MT = (rows + 15) >> 4;
  const int kq = 2 * (l >> 4);
  const int nch = (count + 7) >> 3;
  // ---- the ring slab: rows [0, 8 nch), columns s0 .. s0 + 31 (zero outside) ----
  {
    const int col = threadIdx.x & (kAccCols - 1);
    const int s = s0 + col;
    const bool sok = s < n_slice;
    const int sc = sok ? s : n_slice - 1;   // clamped, in-range address
    constexpr int kRows = kAccThreads / kAccCols;   // rows per pass of the workgroup
    const int r0 = threadIdx.x / kAccCols;
    constexpr int kBatch = 16;                       // rows kRows * kBatch = 256 per thread batch
    for (int rb = 0; rb < 8 * nch; rb += kRows * kBatch) {
      double x[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const int k = rb + r0 + kRows * q;
        const int kc = k < count ? k : count - 1;
        x[q] = ring[(size_t)kc * ring_stride + sc];
      }
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const int k = rb + r0 + kRows * q;
        if (k < 8 * nch) slab[k * kAccCols + col] = (k < count && sok) ? x[q] : 0.0;
      }
    }
  }
  __syncthreads();
  // The wave's M-tiles are w, w + 8, ...: their count NT is the same for the
  // whole wave, and each count has a body of its own, so no tile loop branches
  // (branches would break the straight-line code the waits are counted in).
  const int ntile = (MT - w + kAccWaves - 1) / kAccWaves;
  auto body = [&](auto ntag) __attribute__((always_inline)) {
    constexpr int NT = decltype(ntag)::value;
    M::acc_t c[NT][2];
#pragma unroll
    for (int a = 0; a < NT; ++a) c[a][0] = c[a][1] = M::zero();
    // coefficient fragments of one chunk: A[tile] = (row r, ring rows kb, kb + 1)
    v2d A0[NT], A1[NT];
    auto load = [&](v2d (&A)[NT], int ch) __attribute__((always_inline)) {
      const int kb = 8 * ch + kq;   // even; kb + 1 < 8 * nch <= ldc
#pragma unroll
      for (int a = 0; a < NT; ++a) {
        // rows past the last are clamped (their products are not stored); columns
        // past count are zero in the coefficient table, so fragments load whole
        const int r = min((w + kAccWaves * a) * 16 + (l & 15), rows - 1);
        A[a] = *reinterpret_cast<const v2d*>(coef + (size_t)r * ldc + kb);
      }
    };
    auto compute = [&](const v2d (&A)[NT], int ch) __attribute__((always_inline)) {
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const int k = 8 * ch + kq + cc;
        const double b0 = slab[k * kAccCols + (l & 15)];
        const double b1 = slab[k * kAccCols + 16 + (l & 15)];
#pragma unroll
        for (int a = 0; a < NT; ++a) {
          M::mma(c[a][0], A[a][cc], b0);
          M::mma(c[a][1], A[a][cc], b1);
        }
      }
    };
    if (nch == kAccChunks) {
      // a full ring: straight-line code, each wait covering only the chunk about
      // to be used while the next chunk's loads stay in flight (the scheduling
      // barriers keep each prefetch ahead of the products it overlaps)
      load(A0, 0);
#pragma unroll
      for (int ch = 0; ch < kAccChunks; ch += 2) {
        load(A1, ch + 1);
        __builtin_amdgcn_sched_barrier(0);
        compute(A0, ch);
        if (ch + 2 < kAccChunks) load(A0, ch + 2);
        __builtin_amdgcn_sched_barrier(0);
        compute(A1, ch + 1);
      }
    } else {
      if (nch > 0) load(A0, 0);
      for (int ch = 0; ch < nch; ch += 2) {
        if (ch + 1 < nch) load(A1, ch + 1);
        compute(A0, ch);
        if (ch + 2 < nch) load(A0, ch + 2);
        if (ch + 1 < nch) compute(A1, ch + 1);
      }
    }
    // accumulators of one M-tile: all eight loads in flight, then the stores
    // (without per-lane conditions when the tile lies inside the slice and rows)
    const bool cols_full = s0 + kAccCols <= n_slice;
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const int mt = w + kAccWaves * a;
      if (cols_full && (mt + 1) * 16 <= rows) {
        double* __restrict__ base = acc + (size_t)mt * 16 * n_slice + s0 + (l & 15);
        double old[2][4];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v) old[nt][v] = base[(size_t)M::row(l, v) * n_slice + nt * 16];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            base[(size_t)M::row(l, v) * n_slice + nt * 16] = old[nt][v] + c[a][nt][v];
        continue;
      }
      double old[2][4];
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int s = s0 + nt * 16 + (l & 15), r = mt * 16 + M::row(l, v);
          old[nt][v] = (s < n_slice && r < rows) ? acc[(size_t)r * n_slice + s] : 0.0;
        }
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int s = s0 + nt * 16 + (l & 15), r = mt * 16 + M::row(l, v);
          if (s < n_slice && r < rows) acc[(size_t)r * n_slice + s] = old[nt][v] + c[a][nt][v];
        }
    }
  };
  static_assert(kAccMaxMT == 4, "bodies for one to four M-tiles per wave");
  if (ntile >= 4) body(std::integral_constant<int, 4>{});
  else if (ntile == 3) body(std::integral_constant<int, 3>{});
  else if (ntile == 2) body(std::integral_constant<int, 2>{});
  else if (ntile == 1) body(std::integral_constant<int, 1>{});
}

}  // namespace tdwp

namespace tdwp {
// Advances the device step counters after a step: ring row if slices were recorded,
// norm-partial row always.
__global__ void k_advance(int* counters, int recorded, int stepped) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    counters[0] += recorded;
    counters[1] += stepped;
  }
}

__global__ void k_set_counters(int* counters, int ring_row, int norm_row) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    counters[0] = ring_row;
    counters[1] = norm_row;
    counters[2] = 0;
  }
}
}  // namespace tdwp
