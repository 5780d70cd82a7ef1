// Angular pass with every wave holding its own columns (split forms): the
// rotational / Coriolis part of H u (Sec. 2.1 item 3, the angular terms of the
// Hamiltonian in the body-fixed frame).
//
// A wave owns one (packet, state, R point, 16 r values) block and all of its
// helicities and gamma nodes.  It reads that block straight from HBM into
// registers (no LDS tile, no barriers in the pass):
//   forward   C[Omega][j][r] = sum_n P^Omega[j][n] u[Omega][n][r], with the
//             gamma grid's symmetry: the rows of even (j + Omega) take
//             s[n] = u[n] + u[ng-1-n], the odd ones d[n] = u[n] - u[ng-1-n], n < ng/2;
//   mixing    per (j, r): U diag(min(B_r j(j+1) + B_R l_a, cap)) U^T over the
//             helicities (the tridiagonal l^2 block applied directly when no
//             eigenvalue is capped), in the wave's accumulator registers;
//   back      h[Omega][n][r] = sum_j P^Omega[j][n] C'[Omega][j][r] as the
//             even and odd parts h0 +- h1 at n and ng-1-n.
// The back transform takes its B operand from the accumulators as they lie:
// a lane holds rows 4 (l/16) + v of each 16-row j tile, so k-step s of the
// contraction pairs slot t of lane group g with
//   j = 32 s + 4 g + t (t < 4),   j = 32 s + 16 + 4 g + (t - 4) (t >= 4),
// and the back table is stored with its columns in that order (rows j of the
// other parity, and j < Omega, are zero).  Any pairing of k between the two
// operands is a valid contraction as long as both use it.
//
// Registers: MTJ j tiles x MAXOM helicities of accumulators; two waves per SIMD.
#pragma once
#include <hip/hip_runtime.h>

#include "fast_kernels.hpp"
#include "mfma.hpp"

namespace tdwp {

constexpr int kAngwThreads = 256;   // four waves, one column block each

struct AngwArgs {
  const double* u_all;
  float* h_all;
  const PkDesc* pks;
  const int* blk_start;   // workgroups per packet, prefix sums (n_pk + 1)
  int n_pk, ne, ng, nR, nr;
  const void* Pf;         // forward rows [Omega][class][ngr][ngk] (compute format)
  int ngr, ngk, psf;
  const void* Pb;         // back rows [Omega][class][nbr][kbk], columns in slot order
  int nbr, kbk, psb;
  const double* Br;
  const double* BR;
  double rot_cut;
};

// Slot t of lane group g in k-step s of the back contraction -> row j.
__host__ __device__ constexpr int angw_slot_j(int s, int g, int t) {
  return 32 * s + (t < 4 ? 4 * g + t : 16 + 4 * g + (t - 4));
}

template <int P, int MAXOM, int MTJ>
__global__ __launch_bounds__(kAngwThreads) __attribute__((amdgpu_waves_per_eu(2)))
void k_angw(AngwArgs A) {
  using M = Mma<P>;
  using F = Fmt<P>;
  using E = typename F::E;
  using V = decltype(M::frag_t::hi);
  static_assert(P == kPF16 || P == kPBF, "split forms");
  static_assert(MTJ >= 1 && MTJ <= 4, "n_gamma <= 64");
  extern __shared__ __align__(16) float Ll[];   // the unit's tridiagonal l^2 blocks [j][2 MAXOM + 2]
  const int l = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int pk = find_packet(A.blk_start, A.n_pk, blockIdx.x);
  const PkDesc d = A.pks[pk];
  for (int q = threadIdx.x; q < d.n_mixL; q += kAngwThreads) Ll[q] = d.mixLf[q];
  __syncthreads();
  const int ng = A.ng, nR = A.nR, nr = A.nr;
  const int nrt = (nr + 15) >> 4;
  const int local = (blockIdx.x - A.blk_start[pk]) * (kAngwThreads / 64) + w;
  if (local >= A.ne * nR * nrt) return;   // the packet's last workgroup may be partial
  const int i0 = (local % nrt) * 16, m = (local / nrt) % nR, le = local / (nrt * nR);
  const size_t plane = (size_t)nR * nr;
  const size_t o_step = (size_t)A.ne * ng * plane;
  const size_t base = d.off + (size_t)le * ng * plane + (size_t)m * nr;
  const double* __restrict__ u = A.u_all + base;
  float* __restrict__ h = A.h_all + base;
  const int g = l >> 4, col = l & 15;
  const int i = i0 + col, ic = i < nr ? i : nr - 1;
  const int ngh = ng >> 1;
  const int n_om = d.n_om, om_lo = d.om_lo;
  const E* Pf = reinterpret_cast<const E*>(A.Pf);
  const E* Pb = reinterpret_cast<const E*>(A.Pb);
  // ---- forward: C[o][jt] ---------------------------------------------------------
  typename M::acc_t acc[MTJ][MAXOM];
#pragma unroll
  for (int o = 0; o < MAXOM; ++o)
#pragma unroll
    for (int jt = 0; jt < MTJ; ++jt) acc[jt][o] = M::zero();
  // software pipeline over the helicities: the next block's 16 loads a lane are in
  // flight while this one is transformed
  double ab[2][16];
  auto fetch = [&](double (&x)[16], int o) __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int n = 8 * g + t;   // k slot = gamma pair index n < ng / 2
      const int nc = n < ngh ? n : 0;
      x[t] = u[(size_t)o * o_step + (size_t)nc * plane + ic];
      x[8 + t] = u[(size_t)o * o_step + (size_t)(ng - 1 - nc) * plane + ic];
    }
  };
  fetch(ab[0], 0);
#pragma unroll
  for (int o = 0; o < MAXOM; ++o) {
    if (o >= n_om) break;
    if (o + 1 < MAXOM && o + 1 < n_om) fetch(ab[(o + 1) & 1], o + 1);
    const int Om = om_lo + o;
    typename M::frag_t fe[MTJ], fo[MTJ];
#pragma unroll
    for (int jt = 0; jt < MTJ; ++jt) {
      fe[jt] = F::frag(Pf + ((size_t)(Om * 2 + 0) * A.ngr + jt * 16) * A.ngk, A.ngk, A.psf, l, 0);
      fo[jt] = F::frag(Pf + ((size_t)(Om * 2 + 1) * A.ngr + jt * 16) * A.ngk, A.ngk, A.psf, l, 0);
    }
    const double(&x)[16] = ab[o & 1];
    typename M::frag_t fs, fd;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const bool ok = 8 * g + t < ngh;
      const float vs = ok ? (float)(x[t] + x[8 + t]) * F::kScale : 0.0f;
      const float vd = ok ? (float)(x[t] - x[8 + t]) * F::kScale : 0.0f;
      const E hs = (E)vs, hd = (E)vd;
      fs.hi[t] = hs;
      fs.lo[t] = (E)(vs - (float)hs);
      fd.hi[t] = hd;
      fd.lo[t] = (E)(vd - (float)hd);
    }
#pragma unroll
    for (int jt = 0; jt < MTJ; ++jt) {
      M::mma(acc[jt][o], fe[jt], fs);
      M::mma(acc[jt][o], fo[jt], fd);
    }
  }
  // ---- helicity mixing per (j, r), in place -----------------------------------------
  const float bRm = (float)A.BR[m];
  const float cap = (float)A.rot_cut;
  const int om_hi = om_lo + n_om - 1;
  const float br = (float)A.Br[ic];
  const float* __restrict__ gU = d.mixUf;
  const float* __restrict__ gl = d.mixellf;
#pragma unroll
  for (int jt = 0; jt < MTJ; ++jt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = jt * 16 + M::row(l, v);
      const int nj = (j < ng) ? (j < om_hi ? j : om_hi) - om_lo + 1 : 0;
      float cv[MAXOM];
#pragma unroll
      for (int o = 0; o < MAXOM; ++o) cv[o] = (o < nj) ? acc[jt][o][v] * (float)M::kUnscale : 0.0f;
      if (nj > 0) {
        const float rot = br * (float)(j * (j + 1));
        const float* __restrict__ Lj = Ll + j * (2 * MAXOM + 2);
        // min(rot + B_R l, cap) on the eigenvalues l of the l^2 block: below the cap
        // for all of them, rot + B_R L with L the tridiagonal block; at the cap for
        // all of them, the cap; otherwise the eigenvectors are applied
        const float elo = rot + bRm * Lj[2 * MAXOM], ehi = rot + bRm * Lj[2 * MAXOM + 1];
        if (MAXOM == 1) {
          float e = elo;
          if (A.rot_cut > 0.0) e = e < cap ? e : cap;
          cv[0] *= e;
        } else if (A.rot_cut <= 0.0 || ehi <= cap) {
          float outv[MAXOM];
#pragma unroll
          for (int a = 0; a < MAXOM; ++a) {
            float s = Lj[a] * cv[a];
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
          // one eigenvector column per iteration: project, scale, scatter back (the
          // padded block is the identity outside the j's own nj x nj block, where the
          // coefficients are zero)
          const float* __restrict__ Uj = gU + (size_t)j * n_om * MAXOM;
          const float* __restrict__ lj = gl + j * MAXOM;
          float outv[MAXOM];
#pragma unroll
          for (int a = 0; a < MAXOM; ++a) outv[a] = 0.0f;
          for (int b = 0; b < n_om; ++b) {
            float uc[MAXOM];
#pragma unroll
            for (int a = 0; a < MAXOM; ++a) uc[a] = Uj[b * MAXOM + a];
            float sacc = 0.0f;
#pragma unroll
            for (int a = 0; a < MAXOM; ++a) sacc += uc[a] * cv[a];
            float e = rot + bRm * lj[b];
            if (A.rot_cut > 0.0) e = e < cap ? e : cap;
            const float tb = sacc * e;
#pragma unroll
            for (int a = 0; a < MAXOM; ++a) outv[a] += uc[a] * tb;
          }
#pragma unroll
          for (int a = 0; a < MAXOM; ++a) cv[a] = outv[a];
        }
      }
#pragma unroll
      for (int o = 0; o < MAXOM; ++o) acc[jt][o][v] = (o < nj) ? cv[o] : 0.0f;
    }
  // ---- back: h0 +- h1 at n and ng-1-n --------------------------------------------------
  constexpr int KB = (MTJ + 1) / 2;   // k-steps of 32 j slots
  const int NBT = (ngh + 15) >> 4;    // 16-row tiles of n < ng / 2 (at most 2)
#pragma unroll
  for (int o = 0; o < MAXOM; ++o) {
    if (o >= n_om) break;
    const int Om = om_lo + o;
    typename M::frag_t fb[KB];
#pragma unroll
    for (int s = 0; s < KB; ++s)
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int jt = 2 * s + (t >> 2);
        const float x = jt < MTJ ? acc[jt < MTJ ? jt : 0][o][t & 3] * F::kScale : 0.0f;
        const E hx = (E)x;
        fb[s].hi[t] = hx;
        fb[s].lo[t] = (E)(x - (float)hx);
      }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      if (nt >= NBT) break;
      typename M::frag_t fa[2][KB];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int s = 0; s < KB; ++s)
          fa[c][s] = F::frag(Pb + ((size_t)(Om * 2 + c) * A.nbr + nt * 16) * A.kbk, A.kbk, A.psb, l, 32 * s);
      typename M::acc_t hc[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        hc[c] = M::zero();
#pragma unroll
        for (int s = 0; s < KB; ++s) M::mma(hc[c], fa[c][s], fb[s]);
      }
      if (i < nr) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int n = nt * 16 + M::row(l, v);
          if (n >= ngh) continue;
          const float h0 = hc[0][v] * (float)M::kUnscale, h1 = hc[1][v] * (float)M::kUnscale;
          h[(size_t)o * o_step + (size_t)n * plane + i] = h0 + h1;
          h[(size_t)o * o_step + (size_t)(ng - 1 - n) * plane + i] = h0 - h1;
        }
      }
    }
  }
}

}  // namespace tdwp
