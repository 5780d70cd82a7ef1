// C ABI of the tdwp library: plan construction, potential and packet set-up,
// the propagation loop, energy analysis.  See include/tdwp.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "host_tables.h"
#include "plan.h"
#include "fast_kernels.hpp"
#include "mlp_kernels.hpp"
#include "photo_kernels.hpp"
#include "plane_kernels.hpp"
#include "angw_kernels.hpp"
#include "product_kernels.hpp"
#include "products.h"
#include "step_kernels.hpp"

using namespace tdwp;

namespace {

constexpr size_t kLdsBudget = 64 * 1024;       // general kernels
size_t kLdsMax = 64 * 1024;                    // queried per device in tdwp_plan
int kNumCU = 256;                              // compute units, queried per device

// helicity width of the register-mixing angular kernel (its MAXOM) for units of
// up to n_om helicity blocks
int mix_width(int n_om) { return n_om <= 1 ? 1 : (n_om <= 8 ? 8 : 16); }

// With TDWP_DEBUG set in the environment, HIP errors are reported on stderr.
int hip_fail(hipError_t e, const char* what, int line) {
  if (std::getenv("TDWP_DEBUG"))
    std::fprintf(stderr, "tdwp: %s failed at line %d: %s\n", what, line, hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? TDWP_ENOMEM : TDWP_EDEVICE;
}

#define HIP_TRY(expr)                                     \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return hip_fail(e_, #expr, __LINE__); \
  } while (0)

#define TRY(expr)                 \
  do {                            \
    int s_ = (expr);              \
    if (s_ != TDWP_OK) return s_; \
  } while (0)

int dev_alloc(Plan* P, void** ptr, size_t bytes) {
  *ptr = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return e == hipErrorOutOfMemory ? TDWP_ENOMEM : TDWP_EDEVICE;
  }
  P->allocations.push_back(*ptr);
  return TDWP_OK;
}

// Releases one allocation of the plan before the plan itself is destroyed.
void dev_release(Plan* P, void** ptr) {
  if (!*ptr) return;
  for (auto& a : P->allocations)
    if (a == *ptr) a = nullptr;
  (void)hipFree(*ptr);
  *ptr = nullptr;
}

// The potential table (FP64, and its FP32 copy in the mixed forms of the
// matrix-core path), allocated while the plan holds one.
int ensure_table(Plan* P) {
  const size_t n = (size_t)P->npair * P->ng * P->nR * P->nr;
  if (!P->d_V) TRY(dev_alloc(P, (void**)&P->d_V, n * sizeof(double)));
  if (!P->d_Vf && P->fast && P->cfg.precision != TDWP_FP64)
    TRY(dev_alloc(P, (void**)&P->d_Vf, n * sizeof(float)));
  return TDWP_OK;
}

template <class T>
int alloc_copy(Plan* P, T** dptr, const std::vector<T>& h) {
  TRY(dev_alloc(P, (void**)dptr, h.size() * sizeof(T)));
  if (!h.empty()) HIP_TRY(hipMemcpy(*dptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return TDWP_OK;
}

void drop_graphs(Plan* P) {
  for (int c = 0; c < 2; ++c) {
    if (P->graph_exec[c]) (void)hipGraphExecDestroy(P->graph_exec[c]);
    if (P->graph[c]) (void)hipGraphDestroy(P->graph[c]);
    P->graph_exec[c] = nullptr;
    P->graph[c] = nullptr;
  }
}

void free_plan(Plan* P) {
  if (!P) return;
  if (P->stream) (void)hipStreamSynchronize(P->stream);
  drop_graphs(P);
  for (void* a : P->allocations) (void)hipFree(a);
  if (P->own_stream && P->stream) (void)hipStreamDestroy(P->stream);
  delete P;
}

int omega_lo(const tdwp_unit& u) { return (u.parity * ((u.J % 2) ? -1 : 1) == 1) ? 0 : 1; }

int validate(const tdwp_config* c) {
  if (!c) return TDWP_EINVAL;
  if (c->n_r < 2 || c->n_R < 2 || c->n_gamma < 2) return TDWP_EINVAL;
  if (c->n_r > 1024 || c->n_R > 1024 || c->n_gamma > 256) return TDWP_EINVAL;
  if (!(c->r_min > 0) || !(c->r_max > c->r_min) || !(c->R_min > 0) || !(c->R_max > c->R_min))
    return TDWP_EINVAL;
  if (!(c->mass_A > 0) || !(c->mass_B > 0) || !(c->mass_C > 0)) return TDWP_EINVAL;
  if (c->n_elec < 1 || c->n_elec > kMaxElec) return TDWP_EINVAL;
  if (c->abs_r_power < 1 || c->abs_R_power < 1) return TDWP_EINVAL;
  if (c->abs_r_strength < 0 || c->abs_R_strength < 0) return TDWP_EINVAL;
  if (!(c->r_flux >= c->r_min && c->r_flux <= c->r_max)) return TDWP_EINVAL;
  if (!(c->R_inf >= c->R_min && c->R_inf <= c->R_max)) return TDWP_EINVAL;
  if (c->n_energy < 2 || !(c->ecol_min > 0) || !(c->ecol_max > c->ecol_min)) return TDWP_EINVAL;
  if (c->n_units < 1 || !c->units) return TDWP_EINVAL;
  if (!(c->e_min == 0 && c->e_max == 0) && !(c->e_max > c->e_min)) return TDWP_EINVAL;
  if (c->precision < TDWP_FP64 || c->precision > TDWP_FP16X3) return TDWP_EINVAL;
  for (int i = 0; i < c->n_units; ++i) {
    const tdwp_unit& u = c->units[i];
    if (u.J < 0 || (u.parity != 1 && u.parity != -1)) return TDWP_EINVAL;
    if (u.omega_max < 0 || u.omega_max > u.J || u.omega_max >= kMaxOmega) return TDWP_EINVAL;
    if (u.omega_max > c->n_gamma - 1) return TDWP_EINVAL;
    if (omega_lo(u) > u.omega_max) return TDWP_EINVAL;
    if (u.n_packets < 1 || u.n_packets > 64) return TDWP_EINVAL;
  }
  return TDWP_OK;
}

double absorb(double x, double start, double strength, int power) {
  if (x <= start) return 0.0;
  return strength * std::pow(x - start, power);
}

int build_tables(Plan* P) {
  const tdwp_config& c = P->cfg;
  P->nr = c.n_r;
  P->nR = c.n_R;
  P->ng = c.n_gamma;
  P->ne = c.n_elec;
  P->npair = P->ne * (P->ne + 1) / 2;
  const double M = c.mass_A + c.mass_B + c.mass_C;
  P->mu = c.mass_A * (c.mass_B + c.mass_C) / M;
  P->m = c.mass_B * c.mass_C / (c.mass_B + c.mass_C);
  P->dr = (c.r_max - c.r_min) / (P->nr - 1);
  P->dR = (c.R_max - c.R_min) / (P->nR - 1);
  P->Lr = (P->nr + 1) * P->dr;
  P->LR = (P->nR + 1) * P->dR;
  P->r_wall = c.r_min - P->dr;
  P->R_wall = c.R_min - P->dR;
  P->r.resize(P->nr);
  P->R.resize(P->nR);
  for (int i = 0; i < P->nr; ++i) P->r[i] = c.r_min + P->dr * i;
  for (int i = 0; i < P->nR; ++i) P->R[i] = c.R_min + P->dR * i;
  gauss_legendre(P->ng, P->x, P->w);
  sine_kinetic(P->nr, P->Lr, P->m, c.rad_cut, P->Tr, P->er);
  sine_kinetic(P->nR, P->LR, P->mu, c.rad_cut, P->TR, P->eR);
  P->Br.resize(P->nr);
  P->BR.resize(P->nR);
  for (int i = 0; i < P->nr; ++i) P->Br[i] = 1.0 / (2.0 * P->m * P->r[i] * P->r[i]);
  for (int i = 0; i < P->nR; ++i) P->BR[i] = 1.0 / (2.0 * P->mu * P->R[i] * P->R[i]);
  // damping D(R, r) = exp(-phi_r(r) - phi_R(R)), and its two factors
  // [exp(-phi_r(r_i)) ..., exp(-phi_R(R_m)) ...] for the matrix-core R pass
  P->Dsep.resize((size_t)P->nr + P->nR);
  for (int i = 0; i < P->nr; ++i)
    P->Dsep[i] = std::exp(-absorb(P->r[i], c.abs_r_start, c.abs_r_strength, c.abs_r_power));
  for (int mm = 0; mm < P->nR; ++mm)
    P->Dsep[P->nr + mm] = std::exp(-absorb(P->R[mm], c.abs_R_start, c.abs_R_strength, c.abs_R_power));
  P->D.resize((size_t)P->nR * P->nr);
  for (int mm = 0; mm < P->nR; ++mm)
    for (int i = 0; i < P->nr; ++i)
      P->D[(size_t)mm * P->nr + i] =
          std::exp(-absorb(P->r[i], c.abs_r_start, c.abs_r_strength, c.abs_r_power) -
                   absorb(P->R[mm], c.abs_R_start, c.abs_R_strength, c.abs_R_power));
  // flux rows from the plain sine basis sqrt(2/L) sin(n pi (r - r_wall)/L)
  {
    const double pi = std::acos(-1.0);
    const int n = P->nr;
    P->arow.assign(n, 0.0);
    P->drow.assign(n, 0.0);
    const double cS = std::sqrt(2.0 / (n + 1)), cB = std::sqrt(2.0 / P->Lr);
    for (int a = 1; a <= n; ++a) {
      const double ka = pi * a / P->Lr;
      const double phi = cB * std::sin(ka * (c.r_flux - P->r_wall));
      const double dphi = cB * ka * std::cos(ka * (c.r_flux - P->r_wall));
      for (int i = 1; i <= n; ++i) {
        long prod = (long)a * i % (2L * (n + 1));
        const double s = cS * std::sin(pi * (double)prod / (n + 1));
        P->arow[i - 1] += s * phi;
        P->drow[i - 1] += s * dphi;
      }
    }
  }
  P->m_inf = (int)std::floor((c.R_inf - c.R_min) / P->dR + 0.5);
  // Legendre FBR tables for every Omega in use
  P->max_om = 0;
  for (auto& u : P->units_in) P->max_om = std::max(P->max_om, u.omega_max);
  P->Ptab.assign((size_t)(P->max_om + 1) * P->ng * P->ng, 0.0);
  for (int om = 0; om <= P->max_om; ++om) {
    std::vector<double> rows;
    legendre_fbr_rows(P->ng - 1, om, P->x, P->w, rows);
    for (int j = om; j < P->ng; ++j)
      for (int n = 0; n < P->ng; ++n)
        P->Ptab[((size_t)om * P->ng + j) * P->ng + n] = rows[(size_t)(j - om) * P->ng + n];
  }
  // angular blocks per unit and j
  P->units.clear();
  for (auto& u : P->units_in) {
    UnitInfo U;
    U.J = u.J;
    U.parity = u.parity;
    U.om_lo = omega_lo(u);
    U.om_hi = u.omega_max;
    U.n_om = U.om_hi - U.om_lo + 1;
    U.n_packets = u.n_packets;
    for (int j = 0; j < P->ng; ++j) {
      const int hi = std::min(U.om_hi, j);
      const int nj = hi - U.om_lo + 1;
      U.ang_off.push_back((int)U.ang_U.size());
      U.ell_off.push_back((int)U.ang_ell.size());
      U.n_om_j.push_back(std::max(nj, 0));
      if (nj <= 0) continue;
      std::vector<double> L, ev, vec;
      ell2_block(U.J, j, U.om_lo, hi, L);
      jacobi_eigh(nj, L, ev, vec);
      U.ang_U.insert(U.ang_U.end(), vec.begin(), vec.end());
      U.ang_ell.insert(U.ang_ell.end(), ev.begin(), ev.end());
    }
    P->units.push_back(U);
  }
  // padded blocks of the register mixing (k_angr): width = the kernel's MAXOM
  {
    int max_n = 0;
    for (auto& U : P->units) max_n = std::max(max_n, U.n_om);
    const int S = mix_width(max_n);
    for (auto& U : P->units) {
      U.mix_U.assign((size_t)P->ng * U.n_om * S, 0.0);
      U.mix_ell.assign((size_t)P->ng * S, 0.0);
      U.mix_L.assign((size_t)P->ng * (2 * S + 2), 0.0);
      for (int j = 0; j < P->ng; ++j) {
        const int nj = U.n_om_j[j];
        if (nj > 0) {
          std::vector<double> L;
          ell2_block(U.J, j, U.om_lo, U.om_lo + nj - 1, L);
          double* row = U.mix_L.data() + (size_t)j * (2 * S + 2);
          double lmin = 0.0, lmax = 0.0;
          for (int a = 0; a < nj; ++a) {
            row[a] = L[(size_t)a * nj + a];
            if (a + 1 < nj) row[S + a] = L[(size_t)a * nj + a + 1];
            const double e = U.ang_ell[U.ell_off[j] + a];
            lmin = a ? std::min(lmin, e) : e;
            lmax = a ? std::max(lmax, e) : e;
          }
          row[2 * S] = lmin;
          row[2 * S + 1] = lmax;
        }
        for (int b = 0; b < U.n_om; ++b)
          for (int a = 0; a < S; ++a)
            U.mix_U[((size_t)j * U.n_om + b) * S + a] =
                (a < nj && b < nj) ? U.ang_U[U.ang_off[j] + a * nj + b] : (a == b ? 1.0 : 0.0);
        for (int b = 0; b < nj; ++b) U.mix_ell[(size_t)j * S + b] = U.ang_ell[U.ell_off[j] + b];
      }
    }
  }
  // half-size operators of the matrix-core path (even sizes only)
  if (P->nr % 2 == 0 && P->nR % 2 == 0 && P->ng % 2 == 0) {
    auto split = [](const std::vector<double>& T, int N, int nhk, std::vector<double>& Ts,
                    std::vector<double>& Td) {
      const int h = N / 2;
      Ts.assign((size_t)nhk * nhk, 0.0);
      Td.assign((size_t)nhk * nhk, 0.0);
      for (int i = 0; i < h; ++i)
        for (int j = 0; j < h; ++j) {
          const double a = T[(size_t)i * N + j], b = T[(size_t)i * N + (N - 1 - j)];
          Ts[(size_t)i * nhk + j] = 0.5 * (a + b);
          Td[(size_t)i * nhk + j] = 0.5 * (a - b);
        }
    };
    P->nrhk = round_up(P->nr / 2, 32);
    P->nRhk = round_up(P->nR / 2, 32);
    P->ngk = round_up(P->ng / 2, 32);
    split(P->Tr, P->nr, P->nrhk, P->Trs, P->Trd);
    split(P->TR, P->nR, P->nRhk, P->TRs, P->TRd);
    const int ngh = P->ng / 2, ngk = P->ngk;
    P->Pc.assign((size_t)(P->max_om + 1) * 2 * ngk * ngk, 0.0);
    for (int om = 0; om <= P->max_om; ++om)
      for (int c = 0; c < 2; ++c)
        for (int jj = 0; om + c + 2 * jj < P->ng; ++jj)
          for (int n = 0; n < ngh; ++n)
            P->Pc[(((size_t)om * 2 + c) * ngk + jj) * ngk + n] =
                P->Ptab[((size_t)om * P->ng + om + c + 2 * jj) * P->ng + n];
    P->PcT.assign(P->Pc.size(), 0.0);
    for (size_t b = 0; b < (size_t)(P->max_om + 1) * 2; ++b)
      for (int x = 0; x < ngk; ++x)
        for (int y = 0; y < ngk; ++y)
          P->PcT[(b * ngk + y) * ngk + x] = P->Pc[(b * ngk + x) * ngk + y];
    // forward rows by absolute j, split by the parity of j + omega
    P->ngr = round_up(P->ng, 16);
    const int ngr = P->ngr;
    P->Pf.assign((size_t)(P->max_om + 1) * 2 * ngr * ngk, 0.0);
    for (int om = 0; om <= P->max_om; ++om)
      for (int j = om; j < P->ng; ++j) {
        const int c = (j + om) & 1;
        for (int n = 0; n < ngh; ++n)
          P->Pf[(((size_t)om * 2 + c) * ngr + j) * ngk + n] =
              P->Ptab[((size_t)om * P->ng + j) * P->ng + n];
      }
    // back rows of k_angw: [omega][parity][n][slot], the row j of a slot given by
    // the accumulator layout (zero for j of the other parity, j < omega, j >= n_gamma)
    if (P->ng <= 64) {
      P->nbr = round_up(ngh, 16);
      P->kbk = round_up(P->ng, 32);
      const int nbr = P->nbr, kbk = P->kbk;
      P->Pb.assign((size_t)(P->max_om + 1) * 2 * nbr * kbk, 0.0);
      for (int om = 0; om <= P->max_om; ++om)
        for (int c = 0; c < 2; ++c)
          for (int n = 0; n < ngh; ++n)
            for (int q = 0; q < kbk; ++q) {
              const int j = angw_slot_j(q / 32, (q % 32) / 8, q % 8);
              if (j < om || j >= P->ng || ((j + om) & 1) != c) continue;
              P->Pb[(((size_t)om * 2 + c) * nbr + n) * kbk + q] =
                  P->Ptab[((size_t)om * P->ng + j) * P->ng + n];
            }
    }
  }
  return TDWP_OK;
}

size_t ks_of(int prec) { return (prec == TDWP_BF16X3 || prec == TDWP_FP16X3) ? 32 : 4; }

size_t elem_bytes(int prec) {
  return prec == TDWP_FP64 ? 8 : (prec == TDWP_FP32 ? 4 : 2);
}
int planes_of(int prec) { return (prec == TDWP_BF16X3 || prec == TDWP_FP16X3) ? 2 : 1; }
int ld_of(int prec, int kp) { return kp + ((prec == TDWP_BF16X3 || prec == TDWP_FP16X3) ? 8 : 1); }

// Angular kernel for a tile width of 16 nt columns: k_angr (helicity mixing in
// registers) when its accumulators fit, else k_ang.  Returns false if neither fits.
bool ang_config(Plan* P, int nt, int* regs, size_t* lds) {
  const int prec = P->cfg.precision;
  const size_t eb = elem_bytes(prec) * planes_of(prec);
  const int kpa = round_up(P->ng / 2, (int)ks_of(prec));
  int max_om = 0;
  size_t ang_tab = 0, mix_n = 0;
  for (auto& U : P->units) {
    max_om = std::max(max_om, U.n_om);
    ang_tab = std::max(ang_tab, (U.ang_U.size() + U.ang_ell.size()) * sizeof(double));
    mix_n = std::max(mix_n, U.mix_L.size());
  }
  const size_t tiles = ((size_t)max_om * 2 * 16 * nt * ld_of(prec, kpa) * eb + 15) / 16 * 16;
  const int mom = mix_width(max_om);
  const int tpw = ((P->ng + 15) / 16 * nt + 3) / 4;
  // k_angr stages the tridiagonal blocks in the mixing precision (FP64 form: double, else float)
  const size_t mix_tab = mix_n * (prec == TDWP_FP64 ? sizeof(double) : sizeof(float));
  if (P->ang_pref != 1 && max_om <= kMaxOmega && tpw <= 16 / mom && tiles + mix_tab <= kLdsMax) {
    *regs = mom;
    *lds = tiles + mix_tab;
    return true;
  }
  if (P->ang_pref == 2) return false;
  const int mt_per = (kpa + 15) / 16;
  const int per_wave = (max_om * 2 * mt_per + 3) / 4;
  if (per_wave * nt > kAngMaxAcc || tiles + ang_tab > kLdsMax) return false;
  *regs = 0;
  *lds = tiles + ang_tab;
  return true;
}

// Decides whether the matrix-core kernels apply and sizes their tiles and LDS.
void choose_fast_path(Plan* P) {
  P->fast = false;
  if (P->nr % 2 || P->nR % 2 || P->ng % 2) return;
  const int prec = P->cfg.precision;
  const int ks = (int)ks_of(prec);
  const size_t eb = elem_bytes(prec) * planes_of(prec);
  const int kpr = round_up(P->nr / 2, ks), kpR = round_up(P->nR / 2, ks);
  const int kpa = round_up(P->ng / 2, ks);
  const size_t soft = std::min<size_t>(80 * 1024, kLdsMax);   // two workgroups per CU
  int max_om = 0;
  for (auto& U : P->units) {
    max_om = std::max(max_om, U.n_om);
    // the step kernels address a packet with 32-bit byte offsets of doubles
    if ((size_t)U.n_om * P->ne * P->ng * P->nR * P->nr >= ((size_t)1 << 29)) return;
  }
  P->lds_radr = (size_t)2 * kRadrLines * ld_of(prec, kpr) * eb;
  (void)kpa;
  (void)max_om;
  P->nta = 0;
  for (int nt : {4, 2, 1}) {
    int regs = 0;
    size_t lds = 0;
    if (!ang_config(P, nt, &regs, &lds)) continue;
    if (lds <= soft || nt == 1) {
      P->nta = nt;
      P->ang_regs = regs;
      P->lds_ang = lds;
      break;
    }
  }
  if (P->nta == 0) return;
  P->ntr = 1;
  P->lds_radR = (size_t)P->ne * P->nR * kXLd * (prec == TDWP_FP64 ? sizeof(double) : sizeof(float)) +
                (size_t)2 * 16 * ld_of(prec, kpR) * eb;
  if (P->lds_radr > kLdsMax || P->lds_ang > kLdsMax || P->lds_radR > kLdsMax) return;
  P->fast = true;
}

template <int PR>
int upload_formatted(Plan* P, void** dst, const std::vector<double>& src) {
  using E = typename Fmt<PR>::E;
  double* tmp = nullptr;
  TRY(alloc_copy(P, &tmp, src));
  TRY(dev_alloc(P, dst, src.size() * Fmt<PR>::PLANES * sizeof(E)));
  hipLaunchKernelGGL(k_to_format<PR>, dim3((unsigned)((src.size() + 255) / 256)), dim3(256), 0,
                     P->stream, tmp, (E*)*dst, src.size(), (int)src.size());
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(P->stream));
  return TDWP_OK;
}

template <int PR>
int upload_tables(Plan* P) {
  TRY(upload_formatted<PR>(P, &P->d_TrsF, P->Trs));
  TRY(upload_formatted<PR>(P, &P->d_TrdF, P->Trd));
  TRY(upload_formatted<PR>(P, &P->d_TRsF, P->TRs));
  TRY(upload_formatted<PR>(P, &P->d_TRdF, P->TRd));
  TRY(upload_formatted<PR>(P, &P->d_PcF, P->Pc));
  TRY(upload_formatted<PR>(P, &P->d_PcTF, P->PcT));
  TRY(upload_formatted<PR>(P, &P->d_PfF, P->Pf));
  if (!P->Pb.empty()) TRY(upload_formatted<PR>(P, &P->d_PbF, P->Pb));
  return TDWP_OK;
}

// Kernel choice for the angular pass alone (Plain) or with the r pass (Fused).
struct PlainAng {};
struct FusedAng {};
template <int PR, int NT, int M, int TPW>
auto angr_ptr(PlainAng) { return k_angr<PR, NT, M, TPW>; }
template <int PR, int NT, int M, int TPW>
auto angr_ptr(FusedAng) { return k_angr_radr<PR, NT, M, TPW>; }
template <int PR, int NT, int M>
auto ang_ptr(PlainAng) { return k_ang<PR, NT, M>; }
template <int PR, int NT, int M>
auto ang_ptr(FusedAng) { return k_ang_radr<PR, NT, M>; }

// Calls f with the register-mixing angular kernel for tile width nt, helicity width
// mom and at least tpw column tiles per wave.
template <int PR, class Tag, class F>
void with_angr(int nt, int mom, int tpw, Tag tag, F&& f) {
  auto by_nt = [&](auto ntc) {
    constexpr int NT = decltype(ntc)::value;
    if (mom == 1) {
      if (tpw <= 4) f(angr_ptr<PR, NT, 1, 4>(tag));
      else if (tpw <= 8) f(angr_ptr<PR, NT, 1, 8>(tag));
      else f(angr_ptr<PR, NT, 1, 16>(tag));
    } else if (mom == 8) {
      if (tpw <= 1) f(angr_ptr<PR, NT, 8, 1>(tag));
      else f(angr_ptr<PR, NT, 8, 2>(tag));
    } else {
      f(angr_ptr<PR, NT, 16, 1>(tag));
    }
  };
  if (nt == 4) by_nt(std::integral_constant<int, 4>{});
  else if (nt == 2) by_nt(std::integral_constant<int, 2>{});
  else by_nt(std::integral_constant<int, 1>{});
}

// Calls f with the per-wave angular kernel for helicity width mom (1 or 8) and
// mtj 16-row j tiles (1 .. 4).
template <int PR, class F>
void with_angw(int mom, int mtj, F&& f) {
  auto by = [&](auto mc) {
    constexpr int MOM = decltype(mc)::value;
    if (mtj == 1) f(k_angw<PR, MOM, 1>);
    else if (mtj == 2) f(k_angw<PR, MOM, 2>);
    else if (mtj == 3) f(k_angw<PR, MOM, 3>);
    else f(k_angw<PR, MOM, 4>);
  };
  if (mom == 1) by(std::integral_constant<int, 1>{});
  else by(std::integral_constant<int, 8>{});
}

// The same for the LDS-mixing angular kernel (one helicity or up to kMaxOmega).
template <int PR, class Tag, class F>
void with_ang(int nt, bool single, Tag tag, F&& f) {
  auto by_nt = [&](auto ntc) {
    constexpr int NT = decltype(ntc)::value;
    if (single) f(ang_ptr<PR, NT, 1>(tag));
    else f(ang_ptr<PR, NT, kMaxOmega>(tag));
  };
  if (nt == 4) by_nt(std::integral_constant<int, 4>{});
  else if (nt == 2) by_nt(std::integral_constant<int, 2>{});
  else by_nt(std::integral_constant<int, 1>{});
}

// Raises the dynamic-LDS limit of the matrix-core kernels above the 64 KB
// default where the device allows it; a refusal only matters if a launch
// actually needs more, which choose_fast_path has already excluded.
template <int PR>
void set_lds_limits() {
  if (kLdsMax <= 64 * 1024) return;
  const void* fns[13] = {(const void*)k_radr<PR>,         (const void*)k_radR_epi<PR, 1>,
                         (const void*)k_radR_epi<PR, 2>,  (const void*)k_radR_epi<PR, 3>,
                         (const void*)k_radR_epi<PR, 4>,  (const void*)k_mlp_epi<PR, 1>,
                         (const void*)k_mlp_epi<PR, 2>,   (const void*)k_mlp_epi<PR, 3>,
                         (const void*)k_mlp_epi<PR, 4>,
                         (const void*)k_radR_epi<PR, 1, false, true>,
                         (const void*)k_radR_epi<PR, 2, false, true>,
                         (const void*)k_radR_epi<PR, 3, false, true>,
                         (const void*)k_radR_epi<PR, 4, false, true>};
  std::vector<const void*> all(fns, fns + 13);
  auto add = [&](auto kern) { all.push_back((const void*)kern); };
  add(k_radR_epi<PR, 1, false, false, true>);
  add(k_radR_epi<PR, 2, false, false, true>);
  add(k_radR_epi<PR, 3, false, false, true>);
  add(k_radR_epi<PR, 4, false, false, true>);
  add(k_radR_epi<PR, 1, false, true, true>);
  add(k_radR_epi<PR, 2, false, true, true>);
  add(k_radR_epi<PR, 3, false, true, true>);
  add(k_radR_epi<PR, 4, false, true, true>);
  for (int nt : {1, 2, 4}) {
    for (bool single : {true, false}) {
      with_ang<PR>(nt, single, PlainAng{}, add);
      with_ang<PR>(nt, single, FusedAng{}, add);
    }
    for (int mom : {1, 8, 16})
      for (int tpw : {1, 2, 4, 8, 16}) {
        with_angr<PR>(nt, mom, tpw, PlainAng{}, add);
        with_angr<PR>(nt, mom, tpw, FusedAng{}, add);
      }
  }
  if constexpr (PR != kP64) add(k_plane_epi<PR>);
  for (const void* f : all) {
    // the dynamic share is what the device allows beyond the kernel's static LDS
    hipFuncAttributes fa{};
    size_t stat = 0;
    if (hipFuncGetAttributes(&fa, f) == hipSuccess) stat = fa.sharedSizeBytes;
    (void)hipGetLastError();
    if (stat >= kLdsMax) continue;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(kLdsMax - stat));
    if (e != hipSuccess) {
      hip_fail(e, "hipFuncSetAttribute", __LINE__);
      (void)hipGetLastError();
    }
  }
}

void query_lds_limit() {
  int dev = 0, a = 0, b = 0;
  if (hipGetDevice(&dev) != hipSuccess) { (void)hipGetLastError(); return; }
  if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) a = 0;
  if (hipDeviceGetAttribute(&b, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) b = 0;
  (void)hipGetLastError();
  const size_t lim = (size_t)std::max(a, b);
  if (lim >= 64 * 1024) kLdsMax = lim;
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
    kNumCU = cu;
  (void)hipGetLastError();
}

// Full-size radial operators padded to the plane pass's tile (rows to 16, the
// contraction to the matrix-core k-step), in compute format.
template <int PR>
int plane_tables(Plan* P) {
  using M = Mma<PR>;
  const int nR = P->nR, nr = P->nr;
  P->plane_kR = plane_pad(nR, M::KS);
  P->plane_kr = plane_pad(nr, M::KS);
  auto padded = [](const std::vector<double>& T, int n, int kp) {
    std::vector<double> out((size_t)round_up(n, 16) * kp, 0.0);
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) out[(size_t)a * kp + b] = T[(size_t)a * n + b];
    return out;
  };
  TRY(upload_formatted<PR>(P, &P->d_TRfullF, padded(P->TR, nR, P->plane_kR)));
  TRY(upload_formatted<PR>(P, &P->d_TrfullF, padded(P->Tr, nr, P->plane_kr)));
  const int rows_x = plane_pad(nR, M::KS), cols_x = plane_pad(nr, M::KS);
  P->lds_plane = (size_t)plane_aux_bytes(nr, nR) + plane_tile_bytes(rows_x, cols_x);
  hipFuncAttributes fa{};
  size_t stat = 0;
  if (hipFuncGetAttributes(&fa, (const void*)k_plane_epi<PR>) == hipSuccess) stat = fa.sharedSizeBytes;
  (void)hipGetLastError();
  P->plane_ok = P->lds_plane + stat <= kLdsMax;
  return TDWP_OK;
}

// The plane pass (one electronic state, mixed forms, r lines of at most 256):
// tables, block map and norm-partial counts.
int plane_setup(Plan* P) {
  P->plane_ok = false;
  if (P->ne != 1 || P->cfg.precision == TDWP_FP64 || P->nr > 64 * kPlaneMaxCols) return TDWP_OK;
  switch (P->cfg.precision) {
    case TDWP_FP32: TRY(plane_tables<kP32>(P)); break;
    case TDWP_BF16X3: TRY(plane_tables<kPBF>(P)); break;
    default: TRY(plane_tables<kPF16>(P)); break;
  }
  std::vector<int> bp(1, 0), nw;
  for (auto& pk : P->packets) {
    const int n_planes = P->units[pk.unit].n_om * P->ng;
    bp.push_back(bp.back() + n_planes);
    nw.push_back(n_planes);
  }
  P->blocks_plane = bp.back();
  TRY(alloc_copy(P, &P->d_blk_plane, bp));
  TRY(alloc_copy(P, &P->d_n_wg_plane, nw));
  return TDWP_OK;
}

int layout_and_allocate(Plan* P) {
  const int nr = P->nr, nR = P->nR, ng = P->ng, ne = P->ne;
  // kernel tiles
  int max_col = 0;
  for (auto& U : P->units) max_col = std::max(max_col, U.n_om * ne);
  P->rt_ang = 0;
  for (int rt : {64, 32, 16, 8, 4, 2, 1}) {
    if (rt > nr && rt > 1) continue;
    if ((size_t)2 * max_col * ng * rt * sizeof(double) <= kLdsBudget) {
      P->rt_ang = rt;
      break;
    }
  }
  if (P->rt_ang == 0) return TDWP_ENOMEM;
  P->rt_rad = 0;
  for (int rows : {8, 4, 2, 1})
    if ((size_t)rows * (nr + nR) * sizeof(double) <= kLdsBudget) {
      P->rt_rad = rows;
      break;
    }
  if (P->rt_rad == 0) return TDWP_ENOMEM;
  const int n_tiles_R = (nR + P->rt_rad - 1) / P->rt_rad;
  choose_fast_path(P);
  if (!P->fast && P->cfg.precision != TDWP_FP64) return TDWP_EINVAL;
  if (P->cfg.prod_arrangement != 0) {
    if (!P->fast) return TDWP_EINVAL;   // the product line is recorded by the matrix-core path
    TRY(build_product_tables(P));
  }
  P->fast_accum = P->cfg.n_energy <= 16 * kAccMaxMT * kAccWaves / 2;
  static_assert(kAccChunks * 8 == kRingFast, "a full ring is kAccChunks chunks of eight steps");
  P->ring_len = P->fast_accum ? kRingFast : kRing;
  const int rtf = 16 * P->ntr;
  // packets
  P->packets.clear();
  size_t off = 0, soff = 0, aoff = 0, snoff = 0, wgoff = 0;
  const int nE = P->cfg.n_energy;
  for (int ui = 0; ui < (int)P->units.size(); ++ui) {
    const UnitInfo& U = P->units[ui];
    for (int s = 0; s < U.n_packets; ++s) {
      PacketInfo pk;
      pk.unit = ui;
      pk.slot = s;
      pk.off = off;
      pk.n_values = (size_t)U.n_om * ne * ng * nR * nr;
      pk.n_sv = U.n_om * ne * ng * nR;
      pk.n_w = U.n_om * ne * ng * nr;
      pk.n_p = (P->prod_np > 0 && U.J == 0 && U.n_om == 1) ? ne * P->prod_np : 0;
      pk.prod_idx = pk.n_p > 0 ? P->prod_n_pk++ : -1;
      pk.n_slice = 2 * pk.n_sv + pk.n_w + pk.n_p;
      pk.slice_off = soff;
      pk.acc_off = aoff;
      pk.snap_off = snoff;
      pk.wg_off = wgoff;
      pk.n_wg = P->fast ? U.n_om * ng * ((nr + rtf - 1) / rtf) : U.n_om * ne * ng * n_tiles_R;
      off += pk.n_values;
      soff += pk.n_slice;
      aoff += (size_t)2 * nE * pk.n_slice;
      snoff += (size_t)2 * nE * pk.n_w;
      wgoff += pk.n_wg;
      P->packets.push_back(pk);
    }
  }
  P->n_total = off;
  P->slice_total = soff;
  P->acc_total = aoff;
  P->snap_total = snoff;
  P->n_wg_total = wgoff;
  // the learned-potential pass writes one norm partial per (resident workgroup, packet)
  P->mlp_grid = kNumCU;
  P->n_wg_total = std::max(P->n_wg_total, (size_t)P->packets.size() * (size_t)P->mlp_grid);
  // device buffers
  TRY(dev_alloc(P, (void**)&P->d_u[0], P->n_total * sizeof(double)));
  TRY(dev_alloc(P, (void**)&P->d_u[1], P->n_total * sizeof(double)));
  TRY(dev_alloc(P, (void**)&P->d_h, P->n_total * sizeof(double)));
  if (P->fast) TRY(dev_alloc(P, (void**)&P->d_h2, P->n_total * sizeof(double)));
  TRY(ensure_table(P));
  TRY(alloc_copy(P, &P->d_Tr, P->Tr));
  TRY(alloc_copy(P, &P->d_TR, P->TR));
  TRY(alloc_copy(P, &P->d_P, P->Ptab));
  TRY(alloc_copy(P, &P->d_D, P->D));
  TRY(alloc_copy(P, &P->d_Dsep, P->Dsep));
  TRY(alloc_copy(P, &P->d_Br, P->Br));
  TRY(alloc_copy(P, &P->d_rg, P->r));
  TRY(alloc_copy(P, &P->d_Rg, P->R));
  TRY(alloc_copy(P, &P->d_xg, P->x));
  TRY(alloc_copy(P, &P->d_BR, P->BR));
  TRY(alloc_copy(P, &P->d_arow, P->arow));
  TRY(alloc_copy(P, &P->d_drow, P->drow));
  for (auto& U : P->units) {
    std::vector<double> Uv = U.ang_U.empty() ? std::vector<double>{0.0} : U.ang_U;
    std::vector<double> lv = U.ang_ell.empty() ? std::vector<double>{0.0} : U.ang_ell;
    TRY(alloc_copy(P, &U.d_U, Uv));
    TRY(alloc_copy(P, &U.d_ell, lv));
    TRY(alloc_copy(P, &U.d_mixU, U.mix_U));
    TRY(alloc_copy(P, &U.d_mixell, U.mix_ell));
    TRY(alloc_copy(P, &U.d_mixL, U.mix_L));
    TRY(alloc_copy(P, &U.d_mixUf, std::vector<float>(U.mix_U.begin(), U.mix_U.end())));
    TRY(alloc_copy(P, &U.d_mixellf, std::vector<float>(U.mix_ell.begin(), U.mix_ell.end())));
    TRY(alloc_copy(P, &U.d_mixLf, std::vector<float>(U.mix_L.begin(), U.mix_L.end())));
    TRY(alloc_copy(P, &U.d_ang_off, U.ang_off));
    TRY(alloc_copy(P, &U.d_ell_off, U.ell_off));
    TRY(alloc_copy(P, &U.d_n_om_j, U.n_om_j));
  }
  TRY(dev_alloc(P, (void**)&P->d_ring, (size_t)P->ring_len * P->slice_total * sizeof(double)));
  TRY(dev_alloc(P, (void**)&P->d_acc, P->acc_total * sizeof(double)));
  TRY(dev_alloc(P, (void**)&P->d_snap, P->snap_total * sizeof(double)));
  TRY(dev_alloc(P, (void**)&P->d_coef, P->packets.size() * 2 * nE * P->ring_len * sizeof(double)));
  if (P->prod_n_pk > 0) {
    TRY(alloc_copy(P, &P->d_prod_wr, P->prod_wr));
    TRY(alloc_copy(P, &P->d_prod_wR, P->prod_wR));
    TRY(alloc_copy(P, &P->d_prod_wL, P->prod_wL));
    TRY(alloc_copy(P, &P->d_prod_factor, P->prod_factor));
    const size_t zper = (size_t)ne * ng * P->prod_np;
    TRY(dev_alloc(P, (void**)&P->d_prod_Z, (size_t)P->prod_n_pk * zper * sizeof(double)));
    std::vector<ProdDesc> pdv;
    for (auto& pk : P->packets)
      if (pk.prod_idx >= 0)
        pdv.push_back(ProdDesc{pk.off, pk.slice_off + 2 * (size_t)pk.n_sv + pk.n_w,
                               (size_t)pk.prod_idx * zper});
    ProdDesc* dpd = nullptr;
    TRY(alloc_copy(P, &dpd, pdv));
    P->d_prod_desc = dpd;
  }
  if (P->fast) {
    {
      const int h2 = nr / 2;
      std::vector<double> fs((size_t)4 * h2);
      for (int k = 0; k < h2; ++k) {
        fs[k] = 0.5 * (P->arow[k] + P->arow[nr - 1 - k]);
        fs[h2 + k] = 0.5 * (P->arow[k] - P->arow[nr - 1 - k]);
        fs[2 * h2 + k] = 0.5 * (P->drow[k] + P->drow[nr - 1 - k]);
        fs[3 * h2 + k] = 0.5 * (P->drow[k] - P->drow[nr - 1 - k]);
      }
      TRY(alloc_copy(P, &P->d_flux_split, fs));
    }
    TRY(alloc_copy(P, &P->d_Trs, P->Trs));
    TRY(alloc_copy(P, &P->d_Trd, P->Trd));
    TRY(alloc_copy(P, &P->d_TRs, P->TRs));
    TRY(alloc_copy(P, &P->d_TRd, P->TRd));
    TRY(alloc_copy(P, &P->d_Pc, P->Pc));
    switch (P->cfg.precision) {
      case TDWP_FP64: set_lds_limits<kP64>(); TRY(upload_tables<kP64>(P)); break;
      case TDWP_FP32: set_lds_limits<kP32>(); TRY(upload_tables<kP32>(P)); break;
      case TDWP_BF16X3: set_lds_limits<kPBF>(); TRY(upload_tables<kPBF>(P)); break;
      default: set_lds_limits<kPF16>(); TRY(upload_tables<kPF16>(P)); break;
    }
    TRY(plane_setup(P));
  }
  TRY(dev_alloc(P, (void**)&P->d_normpart, (size_t)kNormChunk * P->n_wg_total * sizeof(double)));
  TRY(dev_alloc(P, (void**)&P->d_norms, P->packets.size() * kNormChunk * sizeof(double)));
  TRY(dev_alloc(P, (void**)&P->d_g, P->packets.size() * nR * sizeof(double)));
  std::vector<size_t> wg_off;
  std::vector<int> n_wg;
  for (auto& pk : P->packets) {
    wg_off.push_back(pk.wg_off);
    n_wg.push_back(pk.n_wg);
  }
  TRY(alloc_copy(P, &P->d_wg_off, wg_off));
  TRY(alloc_copy(P, &P->d_n_wg, n_wg));
  for (size_t ip = 0; ip < P->packets.size(); ++ip) {
    wg_off[ip] = ip * (size_t)P->mlp_grid;
    n_wg[ip] = P->mlp_grid;
  }
  TRY(alloc_copy(P, &P->d_wg_off_mlp, wg_off));
  TRY(alloc_copy(P, &P->d_n_wg_mlp, n_wg));
  // batched-launch index maps
  std::vector<long> line_start(1, 0);
  std::vector<unsigned long> slice_off;
  std::vector<int> blk_acc(1, 0);
  std::vector<AccDesc> ad;
  for (auto& pk : P->packets) {
    line_start.push_back(line_start.back() + pk.n_sv);
    slice_off.push_back(pk.slice_off);
    blk_acc.push_back(blk_acc.back() + (pk.n_slice + kAccCols - 1) / kAccCols);
    ad.push_back(AccDesc{pk.acc_off, pk.slice_off, pk.n_slice});
  }
  P->blocks_acc = blk_acc.back();
  TRY(alloc_copy(P, &P->d_line_start, line_start));
  {
    const long nlines = (long)(P->n_total / nr);
    const long nblk = (nlines + kRadrLines - 1) / kRadrLines;
    std::vector<int> bp((size_t)std::max<long>(nblk, 1), 0);
    int q = 0;
    for (long b = 0; b < nblk; ++b) {
      while (q + 1 < (int)P->packets.size() && line_start[q + 1] <= b * kRadrLines) ++q;
      bp[b] = q;
    }
    TRY(alloc_copy(P, &P->d_radr_pk, bp));
  }
  TRY(alloc_copy(P, &P->d_slice_off, slice_off));
  TRY(alloc_copy(P, &P->d_blk_acc, blk_acc));
  AccDesc* dad = nullptr;
  TRY(alloc_copy(P, &dad, ad));
  P->d_accdesc = dad;
  TRY(dev_alloc(P, (void**)&P->d_E, P->packets.size() * sizeof(double)));
  TRY(dev_alloc(P, (void**)&P->d_counters, 4 * sizeof(int)));
  hipLaunchKernelGGL(k_set_counters, dim3(1), dim3(64), 0, P->stream, P->d_counters, 0, 0);
  HIP_TRY(hipGetLastError());
  if (P->fast) {
    std::vector<PkDesc> pd;
    std::vector<int> ba(1, 0), br(1, 0), bw(1, 0);
    const int nrt_w = (nr + 15) / 16;
    constexpr int kWaves = kAngwThreads / 64;
    const int nrt_a = (nr + 16 * P->nta - 1) / (16 * P->nta);
    const int nrt_r = (nr + 16 * P->ntr - 1) / (16 * P->ntr);
    P->lds_ang_max = P->lds_ang;
    for (auto& pk : P->packets) {
      const UnitInfo& U = P->units[pk.unit];
      pd.push_back(PkDesc{pk.off, pk.wg_off, U.n_om, U.om_lo, U.d_U, U.d_ell, U.d_ang_off,
                          U.d_ell_off, U.d_n_om_j, (int)U.ang_U.size(), (int)U.ang_ell.size(),
                          U.d_mixU, U.d_mixell, U.d_mixL, U.d_mixUf, U.d_mixellf, U.d_mixLf,
                          (int)U.mix_L.size()});
      ba.push_back(ba.back() + nrt_a * nR * ne);
      bw.push_back(bw.back() + (nrt_w * nR * ne + kWaves - 1) / kWaves);
      P->lds_angw = std::max(P->lds_angw, U.mix_L.size() * sizeof(float));
      br.push_back(br.back() + nrt_r * U.n_om * ng);
    }
    P->blocks_ang = ba.back();
    P->blocks_radR = br.back();
    PkDesc* dpd = nullptr;
    TRY(alloc_copy(P, &dpd, pd));
    P->d_pkdesc = dpd;
    TRY(alloc_copy(P, &P->d_blk_ang, ba));
    P->blocks_angw = bw.back();
    TRY(alloc_copy(P, &P->d_blk_angw, bw));
    {
      int max_om = 0;
      for (auto& U : P->units) max_om = std::max(max_om, U.n_om);
      const int prec = P->cfg.precision;
      P->angw_ok = (prec == TDWP_FP16X3 || prec == TDWP_BF16X3) && !P->Pb.empty() &&
                   mix_width(max_om) <= 8 && P->lds_angw <= kLdsMax;
    }
    TRY(alloc_copy(P, &P->d_blk_radR, br));
  }
  return TDWP_OK;
}

// Device memory owned by one library call and released when it returns.
struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    if (ptrs.empty()) return;
    (void)hipDeviceSynchronize();   // no kernel may still use the memory
    for (void* q : ptrs) (void)hipFree(q);
  }
  int get(void** out, size_t bytes) {
    *out = nullptr;
    hipError_t e = hipMalloc(out, bytes ? bytes : 8);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *out = nullptr;
      return e == hipErrorOutOfMemory ? TDWP_ENOMEM : TDWP_EDEVICE;
    }
    ptrs.push_back(*out);
    return TDWP_OK;
  }
};

int ensure_staging(Plan* P, double** buf, size_t* cap, size_t need) {
  if (*cap >= need) return TDWP_OK;
  void* p = nullptr;
  TRY(dev_alloc(P, &p, need * sizeof(double)));
  *buf = (double*)p;
  *cap = need;
  return TDWP_OK;
}

// Angular-kernel tile width (16 nt columns): block prefix sums and LDS size.
int set_ang_tiles(Plan* P, int nt) {
  HIP_TRY(hipStreamSynchronize(P->stream));
  int regs = 0;
  size_t lds = 0;
  if (!ang_config(P, nt, &regs, &lds)) return TDWP_EINVAL;
  std::vector<int> ba(1, 0);
  const int nrt_a = (P->nr + 16 * nt - 1) / (16 * nt);
  for (auto& pk : P->packets) {
    (void)pk;
    ba.push_back(ba.back() + nrt_a * P->nR * P->ne);
  }
  HIP_TRY(hipMemcpy(P->d_blk_ang, ba.data(), ba.size() * sizeof(int), hipMemcpyHostToDevice));
  P->blocks_ang = ba.back();
  P->nta = nt;
  P->ang_regs = regs;
  P->lds_ang = P->lds_ang_max = lds;
  return TDWP_OK;
}

std::string tune_key(Plan* P) {
  int max_om = 0;
  for (auto& U : P->units) max_om = std::max(max_om, U.n_om);
  char buf[160];
  std::snprintf(buf, sizeof buf, "ang p%d r%d R%d g%d e%d om%d", P->cfg.precision, P->nr, P->nR,
                P->ng, P->ne, max_om);
  return buf;
}

// Cached tile choice from the file named by TDWP_TUNE_CACHE (lines "key=value").
int cached_tile(Plan* P) {
  const char* path = std::getenv("TDWP_TUNE_CACHE");
  if (!path) return 0;
  FILE* f = std::fopen(path, "r");
  if (!f) return 0;
  const std::string key = tune_key(P) + "=";
  char line[256];
  int val = 0;
  while (std::fgets(line, sizeof line, f))
    if (std::strncmp(line, key.c_str(), key.size()) == 0) val = std::atoi(line + key.size());
  std::fclose(f);
  return val;
}

void store_tile(Plan* P, int nt) {
  const char* path = std::getenv("TDWP_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s=%d\n", tune_key(P).c_str(), nt);
  std::fclose(f);
}

// ---- propagation -----------------------------------------------------------

struct Timing {
  hipEvent_t ev[2];
  double ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  long calls[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

int timed_begin(Plan* P, Timing* T) {
  if (T) HIP_TRY(hipEventRecord(T->ev[0], P->stream));
  return TDWP_OK;
}

int timed_end(Plan* P, Timing* T, int kind) {
  if (!T) return TDWP_OK;
  HIP_TRY(hipEventRecord(T->ev[1], P->stream));
  HIP_TRY(hipEventSynchronize(T->ev[1]));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, T->ev[0], T->ev[1]));
  T->ms[kind] += ms;
  T->calls[kind] += 1;
  return TDWP_OK;
}

int record_slices(Plan* P, int row) {
  const long nlines = (long)(P->n_total / P->nr);
  const long threads = nlines * 64;
  hipLaunchKernelGGL(k_slices, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, P->stream,
                     P->d_u[P->cur], P->d_line_start, P->d_slice_off, (int)P->packets.size(),
                     P->nR, P->nr, P->m_inf, P->d_arow, P->d_drow, 1.0 / std::sqrt(P->dR),
                     P->d_ring + (size_t)row * P->slice_total);
  HIP_TRY(hipGetLastError());
  return TDWP_OK;
}

// Mirrors the host's ring row and norm row into the device counters.
int sync_counters(Plan* P) {
  hipLaunchKernelGGL(k_set_counters, dim3(1), dim3(64), 0, P->stream, P->d_counters,
                     P->ring_count, P->norm_row);
  HIP_TRY(hipGetLastError());
  return TDWP_OK;
}

int flush_ring(Plan* P) {
  if (P->ring_count == 0) return TDWP_OK;
  const tdwp_config& c = P->cfg;
  const int nE = c.n_energy;
  const double step = (c.ecol_max - c.ecol_min) / (nE - 1);
  const int np = (int)P->packets.size();
  const int nq = nE * P->ring_len * np;
  hipLaunchKernelGGL(k_coef, dim3((nq + 255) / 256), dim3(256), 0, P->stream, P->d_coef,
                     P->ring_len, nE, c.ecol_min, step, P->d_E, np, P->E0, P->dE, P->ring_k0,
                     P->ring_count);
  if (P->fast_accum) {
    const size_t slab = (size_t)8 * ((P->ring_count + 7) / 8) * kAccCols * sizeof(double);
    hipLaunchKernelGGL(k_accum_mfma, dim3(P->blocks_acc), dim3(kAccThreads), slab, P->stream, P->d_acc,
                       P->d_coef, P->ring_len, P->d_ring, P->slice_total,
                       (const AccDesc*)P->d_accdesc, P->d_blk_acc, np, 2 * nE, P->ring_count);
  } else {
    for (size_t ip = 0; ip < P->packets.size(); ++ip) {
      auto& pk = P->packets[ip];
      const int epb = 8;
      dim3 grid((pk.n_slice + 255) / 256, (nE + epb - 1) / epb);
      hipLaunchKernelGGL(k_accumulate, grid, dim3(256), 0, P->stream, P->d_acc + pk.acc_off,
                         P->d_coef + ip * 2 * nE * P->ring_len, P->d_ring + pk.slice_off,
                         P->slice_total, pk.n_slice, nE, epb, P->ring_count);
    }
  }
  HIP_TRY(hipGetLastError());
  P->ring_k0 += P->ring_count;
  P->ring_count = 0;
  return sync_counters(P);
}

int take_snapshots(Plan* P) {
  const int nE = P->cfg.n_energy;
  for (auto& pk : P->packets) {
    if (pk.snap_taken || pk.pk.k_min_elastic != P->k) continue;
    const size_t n = (size_t)2 * nE * pk.n_w;
    hipLaunchKernelGGL(k_snapshot, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, P->stream,
                       P->d_snap + pk.snap_off, P->d_acc + pk.acc_off, nE, pk.n_slice,
                       2 * pk.n_sv, pk.n_w);
    pk.snap_taken = true;
  }
  HIP_TRY(hipGetLastError());
  return TDWP_OK;
}

MlpNet mlp_net(Plan* P) {
  const __bf16* w = (const __bf16*)P->d_mlp_w;
  MlpNet N;
  N.w1t = w;
  N.w2t = w + kMlpH * 32;
  N.w3t = N.w2t + kMlpH * kMlpH;
  N.w4t = N.w3t + kMlpH * kMlpH;
  N.b1 = P->d_mlp_b;
  N.b2 = P->d_mlp_b + kMlpH;
  N.b3 = P->d_mlp_b + 2 * kMlpH;
  N.b4 = P->d_mlp_b + 3 * kMlpH;
  N.npair = P->npair;
  return N;
}

int mlp_param_count(int npair) {
  return 3 * kMlpH + kMlpH + 2 * (kMlpH * kMlpH + kMlpH) + kMlpH * npair + npair;
}

// Device work buffers of one forward/backward pass on a batch of B points.
struct MlpPass {
  float *X, *T, *Z1, *A1, *Z2, *A2, *Z3, *A3, *Z4, *Y, *dZ4, *dZ3, *dZ2, *dZ1, *part;
};

int mlp_alloc_pass(Scratch& S, Plan* P, int B, MlpPass* q) {
  const int np = P->npair;
  const size_t sizes[15] = {(size_t)B * 3, (size_t)B * np, (size_t)B * kMlpH, (size_t)B * kMlpH,
                            (size_t)B * kMlpH, (size_t)B * kMlpH, (size_t)B * kMlpH,
                            (size_t)B * kMlpH, (size_t)B * np, (size_t)B * np, (size_t)B * np,
                            (size_t)B * kMlpH, (size_t)B * kMlpH, (size_t)B * kMlpH,
                            (size_t)(B * np + 255) / 256 + 1};
  float** ptrs[15] = {&q->X, &q->T, &q->Z1, &q->A1, &q->Z2, &q->A2, &q->Z3, &q->A3, &q->Z4,
                      &q->Y, &q->dZ4, &q->dZ3, &q->dZ2, &q->dZ1, &q->part};
  for (int i = 0; i < 15; ++i) TRY(S.get((void**)ptrs[i], sizes[i] * sizeof(float)));
  return TDWP_OK;
}

// Forward + backward on the batch already in q.X / q.T; gradient into g (layout of theta).
int mlp_fwd_bwd(Plan* P, const float* th, float* g, int B, const MlpPass& q) {
  const int np = P->npair, H = kMlpH;
  const float* W1 = th;
  const float* b1 = W1 + 3 * H;
  const float* W2 = b1 + H;
  const float* b2 = W2 + H * H;
  const float* W3 = b2 + H;
  const float* b3 = W3 + H * H;
  const float* W4 = b3 + H;
  const float* b4 = W4 + H * np;
  float* gW1 = g;
  float* gb1 = gW1 + 3 * H;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + H * H;
  float* gW3 = gb2 + H;
  float* gb3 = gW3 + H * H;
  float* gW4 = gb3 + H;
  float* gb4 = gW4 + H * np;
  auto grid = [](long n) { return dim3((unsigned)((n + 255) / 256)); };
  hipStream_t st = P->stream;
  hipLaunchKernelGGL(k_dense_fwd, grid((long)B * H), dim3(256), 0, st, q.X, 3, W1, b1, H, B, q.Z1, q.A1, 1);
  hipLaunchKernelGGL(k_dense_fwd, grid((long)B * H), dim3(256), 0, st, q.A1, H, W2, b2, H, B, q.Z2, q.A2, 1);
  hipLaunchKernelGGL(k_dense_fwd, grid((long)B * H), dim3(256), 0, st, q.A2, H, W3, b3, H, B, q.Z3, q.A3, 1);
  hipLaunchKernelGGL(k_dense_fwd, grid((long)B * np), dim3(256), 0, st, q.A3, H, W4, b4, np, B, q.Z4, q.Y, 0);
  hipLaunchKernelGGL(k_mse_grad, grid((long)B * np), dim3(256), 0, st, q.Y, q.T, B * np,
                     1.0f / (float)(B * np), q.dZ4, q.part);
  hipLaunchKernelGGL(k_dense_bwd_w, grid((long)(H + 1) * np), dim3(256), 0, st, q.A3, q.dZ4, H, np, B, gW4, gb4);
  hipLaunchKernelGGL(k_dense_bwd_data, grid((long)B * H), dim3(256), 0, st, q.dZ4, W4, H, np, B, q.Z3, q.dZ3);
  hipLaunchKernelGGL(k_dense_bwd_w, grid((long)(H + 1) * H), dim3(256), 0, st, q.A2, q.dZ3, H, H, B, gW3, gb3);
  hipLaunchKernelGGL(k_dense_bwd_data, grid((long)B * H), dim3(256), 0, st, q.dZ3, W3, H, H, B, q.Z2, q.dZ2);
  hipLaunchKernelGGL(k_dense_bwd_w, grid((long)(H + 1) * H), dim3(256), 0, st, q.A1, q.dZ2, H, H, B, gW2, gb2);
  hipLaunchKernelGGL(k_dense_bwd_data, grid((long)B * H), dim3(256), 0, st, q.dZ2, W2, H, H, B, q.Z1, q.dZ1);
  hipLaunchKernelGGL(k_dense_bwd_w, grid((long)4 * H), dim3(256), 0, st, q.X, q.dZ1, 3, H, B, gW1, gb1);
  HIP_TRY(hipGetLastError());
  return TDWP_OK;
}

// Before slices of the current k are recorded: flush a full ring, and flush
// then snapshot where an elastic-channel window opens at this k.
int prepare_record(Plan* P, Timing* T) {
  bool opens = false;
  for (auto& pk : P->packets)
    if (!pk.snap_taken && pk.pk.k_min_elastic == P->k) opens = true;
  if (P->ring_count == P->ring_len || opens) {
    TRY(timed_begin(P, T));
    TRY(flush_ring(P));
    TRY(take_snapshots(P));
    TRY(timed_end(P, T, 3));
  }
  return TDWP_OK;
}

// Workgroups of a radial pass over n blocks (each workgroup loops over its blocks).
unsigned radial_blocks(const Plan* P, long n) {
  return (unsigned)((P->radial_grid > 0 && P->radial_grid < n) ? P->radial_grid : n);
}

// Whether this step runs the plane pass (both radial terms, one launch) after
// the angular pass: chosen, feasible, a tabulated potential, and no overlaps to
// form in the R pass.
bool use_plane(const Plan* P) {
  return P->fast && P->plane_ok && P->plane_r && P->pot_mode == TDWP_POT_TABLE && !P->acf_in_pass;
}

// Whether the angular pass runs the per-wave kernel (chosen, feasible, and its
// launch not shared with the r pass).
bool use_angw(const Plan* P) {
  return P->fast && P->angw_ok && P->ang_wave && !(P->fuse_r && !use_plane(P));
}

// The product lines of u in d_u[cur] into the ring row counters[0] (J = 0 packets
// of a plan with a product arrangement); nothing otherwise.
int launch_product_lines(Plan* P, int cur) {
  if (P->prod_n_pk == 0) return TDWP_OK;
  const int np = P->prod_np;
  const unsigned g1 = (unsigned)((size_t)P->prod_n_pk * P->ne * P->ng * ((np + kProdPts - 1) / kProdPts));
  hipLaunchKernelGGL(k_prod_contract, dim3(g1), dim3(256), 0, P->stream, P->d_u[cur],
                     (const ProdDesc*)P->d_prod_desc, P->ne, P->ng, P->nR, P->nr, P->d_prod_wr,
                     P->prod_kr, P->d_prod_wR, P->prod_kR, np, P->d_prod_Z);
  const long n2 = (long)P->prod_n_pk * P->ne * np;
  hipLaunchKernelGGL(k_prod_finish, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, P->stream,
                     (const ProdDesc*)P->d_prod_desc, P->prod_n_pk, P->ne, P->ng, np, P->d_prod_Z,
                     P->d_prod_wL, P->d_prod_factor, P->d_ring, P->slice_total, P->d_counters,
                     P->ring_len);
  HIP_TRY(hipGetLastError());
  return TDWP_OK;
}

// Launches the kernels of one step of the matrix-core path (no host state change):
// u_k in d_u[cur], u_{k-1} in d_u[1 - cur]; rec: record the slices of u_k.
template <int PR>
int enqueue_step(Plan* P, int cur, int first, int rec, Timing* T) {
  using HT = typename HType<PR>::T;
  using E = typename Fmt<PR>::E;
  const double* uk = P->d_u[cur];
  double* uo = P->d_u[1 - cur];
  HT* h = reinterpret_cast<HT*>(P->d_h);
  const int nr = P->nr, nR = P->nR, ng = P->ng, ne = P->ne;
  const int np = (int)P->packets.size();
  const PkDesc* pkd = (const PkDesc*)P->d_pkdesc;
  const long nlines = (long)(P->n_total / nr);
  const int nrh = nr / 2;
  SliceArgs sa{rec, 0, P->d_line_start, P->d_slice_off, np, nR, P->m_inf,
               P->d_flux_split, P->d_flux_split + nrh, P->d_flux_split + 2 * nrh,
               P->d_flux_split + 3 * nrh, 1.0 / std::sqrt(P->dR), P->d_ring, P->slice_total,
               P->d_counters, P->ring_len, P->d_radr_pk};
  const unsigned nblk_r = radial_blocks(P, (nlines + kRadrLines - 1) / kRadrLines);
  const bool plane = use_plane(P);
  const bool fuse = P->fuse_r && !plane;
  HT* h2 = fuse ? reinterpret_cast<HT*>(P->d_h2) : nullptr;
  // the potential table in h's precision (an FP32 copy in the mixed forms)
  const HT* vtab = reinterpret_cast<const HT*>(PR == kP64 ? (const void*)P->d_V : (const void*)P->d_Vf);
  TRY(timed_begin(P, T));
  {
    AngArgs aa{uk, h, pkd, P->d_blk_ang, np, ne, ng, nR, nr, nullptr, P->ngr, (int)P->Pf.size(),
               P->d_PcTF, P->ngk, (int)P->Pc.size(), P->d_Br, P->d_BR, P->cfg.rot_cut,
               P->ang_xcd ? 1 : 0};
    RadrArgs ra{uk, h2, P->d_TrsF, P->d_TrdF, P->nrhk, P->nrhk * P->nrhk, nr, nlines, sa};
    auto plain = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(P->blocks_ang), dim3(256), P->lds_ang_max, P->stream, aa);
    };
    // the r-pass blocks follow the angular blocks in the same grid
    auto fused = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(P->blocks_ang + nblk_r), dim3(256),
                         std::max(P->lds_ang_max, P->lds_radr), P->stream, aa, ra,
                         (int)P->blocks_ang);
    };
    int max_om = 0;
    for (auto& U : P->units) max_om = std::max(max_om, U.n_om);
    bool wave = false;
    if constexpr (PR == kPF16 || PR == kPBF) {
      if (use_angw(P)) {
        wave = true;
        AngwArgs wa{uk, reinterpret_cast<float*>(h), pkd, P->d_blk_angw, np, ne, ng, nR, nr,
                    P->d_PfF, P->ngr, P->ngk, (int)P->Pf.size(), P->d_PbF, P->nbr, P->kbk,
                    (int)P->Pb.size(), P->d_Br, P->d_BR, P->cfg.rot_cut};
        with_angw<PR>(mix_width(max_om), (ng + 15) / 16, [&](auto kern) {
          hipLaunchKernelGGL(kern, dim3(P->blocks_angw), dim3(kAngwThreads), P->lds_angw, P->stream,
                             wa);
        });
      }
    }
    if (wave) {
    } else if (P->ang_regs) {
      aa.Pfwd = P->d_PfF;
      // column tiles per wave: (j tiles) x (r tiles) over the four waves
      const int tpw = ((ng + 15) / 16 * P->nta + 3) / 4;
      if (fuse) with_angr<PR>(P->nta, P->ang_regs, tpw, FusedAng{}, fused);
      else with_angr<PR>(P->nta, P->ang_regs, tpw, PlainAng{}, plain);
    } else {
      aa.Pfwd = P->d_PcF;
      if (fuse) with_ang<PR>(P->nta, max_om == 1, FusedAng{}, fused);
      else with_ang<PR>(P->nta, max_om == 1, PlainAng{}, plain);
    }
  }
  HIP_TRY(hipGetLastError());
  TRY(timed_end(P, T, 0));
  if (rec && P->prod_n_pk > 0) {   // before the step's last pass advances the ring row
    TRY(timed_begin(P, T));
    TRY(launch_product_lines(P, cur));
    TRY(timed_end(P, T, 7));
  }
  if constexpr (PR != kP64) {
    if (plane) {
      // T_r and T_R over whole planes, potential, recursion, damping, norm, slices
      TRY(timed_begin(P, T));
      PlaneArgs pa{uk, uo, reinterpret_cast<const float*>(P->d_h), pkd, P->d_blk_plane, np,
                   P->d_TRfullF, P->d_TrfullF, P->plane_kR, P->plane_kr,
                   round_up(nR, 16) * P->plane_kR, round_up(nr, 16) * P->plane_kr,
                   P->d_Vf, P->d_Dsep, ng, nR, nr, P->E0, 1.0 / P->dE, first, P->d_normpart,
                   P->n_wg_total, P->d_counters, kNormChunk, rec, P->d_slice_off,
                   P->d_line_start, P->d_arow, P->d_drow, P->m_inf, 1.0 / std::sqrt(P->dR),
                   P->d_ring, P->slice_total, P->ring_len};
      hipLaunchKernelGGL(k_plane_epi<PR>, dim3(radial_blocks(P, P->blocks_plane)),
                         dim3(kPlaneThreads), P->lds_plane, P->stream, pa);
      HIP_TRY(hipGetLastError());
      TRY(timed_end(P, T, 6));
      return TDWP_OK;
    }
  }
  if (!fuse) {
    TRY(timed_begin(P, T));
    hipLaunchKernelGGL(k_radr<PR>, dim3(nblk_r), dim3(256), P->lds_radr, P->stream, uk, h,
                       (const E*)P->d_TrsF, (const E*)P->d_TrdF, P->nrhk, P->nrhk * P->nrhk, nr,
                       nlines, sa);
    HIP_TRY(hipGetLastError());
    TRY(timed_end(P, T, 4));
  }
  TRY(timed_begin(P, T));
  if (P->pot_mode == TDWP_POT_MLP) {
    // y = T_R u + h in h's place, then the network and the rest of the step per point
    auto split = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(radial_blocks(P, P->blocks_radR)), dim3(256), P->lds_radR,
                         P->stream, uk, uo, h, (const HT*)h2, pkd, P->d_blk_radR, np,
                         (const E*)P->d_TRsF,
                         (const E*)P->d_TRdF, P->nRhk, P->nRhk * P->nRhk, vtab, P->d_Dsep, ng, nR,
                         nr, P->E0, 1.0 / P->dE, first, P->d_normpart, P->n_wg_total,
                         P->d_counters, kNormChunk, rec, (const double*)nullptr, (double*)nullptr);
    };
    const double mbc = P->cfg.mass_B + P->cfg.mass_C;
    auto epi = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(P->mlp_grid), dim3(256), mlp_epi_lds(np), P->stream,
                         mlp_net(P), P->d_rg, P->d_Rg, P->d_xg, P->cfg.mass_C / mbc,
                         P->cfg.mass_B / mbc, ng, nR, nr, pkd, np, uk, uo, (const HT*)h, P->d_Dsep,
                         P->E0, 1.0 / P->dE, first, P->d_normpart, P->n_wg_total,
                         P->d_counters, kNormChunk, rec);
    };
    switch (ne) {
      case 1: fuse ? split(k_radR_epi<PR, 1, true, true>) : split(k_radR_epi<PR, 1, true>); epi(k_mlp_epi<PR, 1>); break;
      case 2: fuse ? split(k_radR_epi<PR, 2, true, true>) : split(k_radR_epi<PR, 2, true>); epi(k_mlp_epi<PR, 2>); break;
      case 3: fuse ? split(k_radR_epi<PR, 3, true, true>) : split(k_radR_epi<PR, 3, true>); epi(k_mlp_epi<PR, 3>); break;
      default: fuse ? split(k_radR_epi<PR, 4, true, true>) : split(k_radR_epi<PR, 4, true>); epi(k_mlp_epi<PR, 4>); break;
    }
  } else {
    // photodissociation packets: the R pass also forms <u_0|u_{k+1}>
    const bool acf = P->acf_in_pass;
    auto launch = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(radial_blocks(P, P->blocks_radR)), dim3(256), P->lds_radR,
                         P->stream, uk, uo,
                         h, (const HT*)h2, pkd, P->d_blk_radR, np, (const E*)P->d_TRsF,
                         (const E*)P->d_TRdF,
                         P->nRhk, P->nRhk * P->nRhk, vtab, P->d_Dsep, ng, nR, nr, P->E0,
                         1.0 / P->dE, first, P->d_normpart, P->n_wg_total, P->d_counters,
                         kNormChunk, rec, acf ? (const double*)P->d_u0 : nullptr,
                         acf ? P->d_acfwg : nullptr);
    };
    auto by_ne = [&](auto two, auto withacf) {
      constexpr bool TW = decltype(two)::value, AC = decltype(withacf)::value;
      switch (ne) {
        case 1: launch(k_radR_epi<PR, 1, false, TW, AC>); break;
        case 2: launch(k_radR_epi<PR, 2, false, TW, AC>); break;
        case 3: launch(k_radR_epi<PR, 3, false, TW, AC>); break;
        default: launch(k_radR_epi<PR, 4, false, TW, AC>); break;
      }
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    if (fuse) acf ? by_ne(T_{}, T_{}) : by_ne(T_{}, F_{});
    else acf ? by_ne(F_{}, T_{}) : by_ne(F_{}, F_{});
  }
  HIP_TRY(hipGetLastError());   // the pass's last workgroup has advanced the counters
  TRY(timed_end(P, T, 1));
  return TDWP_OK;
}

template <int PR>
int fast_step(Plan* P, int chunk_row, Timing* T) {
  (void)chunk_row;
  const int first = (P->k == 0) ? 1 : 0;
  const bool rec = P->rec_k < P->k;
  if (rec) TRY(prepare_record(P, T));
  TRY(enqueue_step<PR>(P, P->cur, first, rec ? 1 : 0, T));
  if (rec) {
    P->ring_count += 1;
    P->rec_k = P->k;
  }
  P->norm_row += 1;
  return TDWP_OK;
}

// Two steady-state steps (slices recorded, not the first step) captured once per
// buffer parity and replayed; every per-step argument lives in the device counters.
template <int PR>
int graph_two_steps(Plan* P) {
  const int c = P->cur;
  if (!P->graph_exec[c]) {
    HIP_TRY(hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal));
    int st = enqueue_step<PR>(P, c, 0, 1, nullptr);
    if (st == TDWP_OK) st = enqueue_step<PR>(P, 1 - c, 0, 1, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(P->stream, &g);
    if (st != TDWP_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __LINE__);
    P->graph[c] = g;
    HIP_TRY(hipGraphInstantiate(&P->graph_exec[c], g, nullptr, nullptr, 0));
  }
  HIP_TRY(hipGraphLaunch(P->graph_exec[c], P->stream));
  P->ring_count += 2;
  P->rec_k = P->k + 1;
  P->k += 2;
  P->norm_row += 2;
  P->graph_steps += 2;
  return TDWP_OK;
}

int after_step(Plan* P, Timing* T);

int one_step(Plan* P, int chunk_row, Timing* T) {
  if (P->fast) {
    switch (P->cfg.precision) {
      case TDWP_FP64: TRY(fast_step<kP64>(P, chunk_row, T)); break;
      case TDWP_FP32: TRY(fast_step<kP32>(P, chunk_row, T)); break;
      case TDWP_BF16X3: TRY(fast_step<kPBF>(P, chunk_row, T)); break;
      default: TRY(fast_step<kPF16>(P, chunk_row, T)); break;
    }
    return after_step(P, T);
  }
  const int first = (P->k == 0) ? 1 : 0;
  double* uk = P->d_u[P->cur];
  double* uo = P->d_u[1 - P->cur];
  TRY(timed_begin(P, T));
  for (auto& pk : P->packets) {
    const UnitInfo& U = P->units[pk.unit];
    const int ntile = (P->nr + P->rt_ang - 1) / P->rt_ang;
    const size_t lds = (size_t)2 * U.n_om * P->ne * P->ng * P->rt_ang * sizeof(double);
    hipLaunchKernelGGL(k_angular_pot, dim3(ntile, P->nR), dim3(256), lds, P->stream, uk + pk.off,
                       P->d_h + pk.off, U.n_om, U.om_lo, P->ne, P->ng, P->nR, P->nr, P->rt_ang,
                       P->d_P, U.d_U, U.d_ell, U.d_ang_off, U.d_ell_off, U.d_n_om_j, P->d_Br,
                       P->d_BR, P->cfg.rot_cut, P->d_V);
  }
  HIP_TRY(hipGetLastError());
  TRY(timed_end(P, T, 0));
  TRY(timed_begin(P, T));
  const int n_tiles_R = (P->nR + P->rt_rad - 1) / P->rt_rad;
  const size_t lds_rad = (size_t)P->rt_rad * (P->nr + P->nR) * sizeof(double);
  for (auto& pk : P->packets) {
    const UnitInfo& U = P->units[pk.unit];
    const int slabs = U.n_om * P->ne * P->ng;
    hipLaunchKernelGGL(k_radial_epi, dim3(n_tiles_R, slabs), dim3(256), lds_rad, P->stream,
                       uk + pk.off, uo + pk.off, P->d_h + pk.off, P->d_TR, P->d_Tr, P->d_D,
                       P->nR, P->nr, P->rt_rad, P->E0, 1.0 / P->dE, first,
                       P->d_normpart + (size_t)chunk_row * P->n_wg_total + pk.wg_off);
  }
  HIP_TRY(hipGetLastError());
  TRY(timed_end(P, T, 1));
  return after_step(P, T);
}

// Swaps the packet buffers; the general path records the slices of the new u_k
// here, the matrix-core path inside the next step's k_radr (or finish_slices).
int after_step(Plan* P, Timing* T) {
  P->cur = 1 - P->cur;
  P->k += 1;
  if (P->fast) return TDWP_OK;
  TRY(prepare_record(P, T));
  TRY(timed_begin(P, T));
  TRY(record_slices(P, P->ring_count));
  P->ring_count += 1;
  P->rec_k = P->k;
  TRY(timed_end(P, T, 2));
  return TDWP_OK;
}

// Slices of u_k through k_radr's recording path (same arithmetic as in a step).
template <int PR>
int record_via_radr(Plan* P) {
  using E = typename Fmt<PR>::E;
  const int nr = P->nr, h2 = nr / 2;
  const long nlines = (long)(P->n_total / nr);
  SliceArgs sa{1, 1, P->d_line_start, P->d_slice_off, (int)P->packets.size(), P->nR, P->m_inf,
               P->d_flux_split, P->d_flux_split + h2, P->d_flux_split + 2 * h2,
               P->d_flux_split + 3 * h2, 1.0 / std::sqrt(P->dR), P->d_ring, P->slice_total,
               P->d_counters, P->ring_len, P->d_radr_pk};
  hipLaunchKernelGGL(k_radr<PR>, dim3(radial_blocks(P, (nlines + kRadrLines - 1) / kRadrLines)),
                     dim3(256), P->lds_radr, P->stream, P->d_u[P->cur],
                     reinterpret_cast<typename HType<PR>::T*>(P->d_h), (const E*)P->d_TrsF,
                     (const E*)P->d_TrdF, P->nrhk, P->nrhk * P->nrhk, nr, nlines, sa);
  TRY(launch_product_lines(P, P->cur));
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, P->stream, P->d_counters, 1, 0);
  HIP_TRY(hipGetLastError());
  return TDWP_OK;
}

// Records the slices of the current u_k if that has not happened yet.
int finish_slices(Plan* P, Timing* T) {
  if (P->rec_k >= P->k) return TDWP_OK;
  TRY(prepare_record(P, T));
  TRY(timed_begin(P, T));
  if (P->fast) {
    switch (P->cfg.precision) {
      case TDWP_FP64: TRY(record_via_radr<kP64>(P)); break;
      case TDWP_FP32: TRY(record_via_radr<kP32>(P)); break;
      case TDWP_BF16X3: TRY(record_via_radr<kPBF>(P)); break;
      default: TRY(record_via_radr<kPF16>(P)); break;
    }
  } else {
    TRY(record_slices(P, P->ring_count));
  }
  P->ring_count += 1;
  P->rec_k = P->k;
  TRY(timed_end(P, T, 2));
  return TDWP_OK;
}

// Whether the next two steps are steady state: matrix-core path, not the first
// step, slices recorded in both, no ring flush or elastic snapshot in between.
bool graph_ready(Plan* P, int left, Timing* T) {
  if (!P->use_graphs || !P->fast || T || left < 2 || P->k < 1 || (P->n_photo && !P->acf_in_pass))
    return false;
  if (P->rec_k >= P->k || P->ring_count + 2 > P->ring_len) return false;
  for (auto& pk : P->packets)
    if (!pk.snap_taken && (pk.pk.k_min_elastic == P->k || pk.pk.k_min_elastic == P->k + 1)) return false;
  return true;
}

// ---- autocorrelation of photodissociation packets -------------------------------

int acf_blocks(size_t n) {
  const size_t nb = (n + kAcfPerBlock - 1) / kAcfPerBlock;
  return (int)std::min<size_t>(std::max<size_t>(nb, 1), kAcfMaxBlocks);
}

// Partial-sum layout of every photodissociation packet: rows of acf_nb_total.
// The buffers are sized first; on an allocation failure nothing is changed.
int acf_layout(Plan* P) {
  size_t tot = 0;
  int idx = 0;
  for (auto& pk : P->packets)
    if (pk.photo) {
      tot += acf_blocks(pk.n_values);
      ++idx;
    }
  const bool in_pass = idx > 0 && P->fast && P->pot_mode != TDWP_POT_MLP;
  if (idx) {
    TRY(ensure_staging(P, &P->d_acfpart, &P->acfpart_cap, (size_t)kNormChunk * tot));
    TRY(ensure_staging(P, &P->d_acf, &P->acf_cap, (size_t)kNormChunk * P->packets.size()));
  }
  if (in_pass) TRY(ensure_staging(P, &P->d_acfwg, &P->acfwg_cap, (size_t)kNormChunk * P->n_wg_total));
  if (in_pass != P->acf_in_pass) drop_graphs(P);   // captured steps launch the other R pass
  P->acf_in_pass = in_pass;
  tot = 0;
  idx = 0;
  for (auto& pk : P->packets) {
    if (!pk.photo) continue;
    pk.acf_nb = acf_blocks(pk.n_values);
    pk.acf_part_off = tot;
    pk.acf_idx = idx++;
    tot += pk.acf_nb;
  }
  P->acf_nb_total = tot;
  P->n_photo = idx;
  return TDWP_OK;
}

// Row `row` of the partials: <u_0|u_k> of packet pk with u_k the current buffer.
void acf_dot(Plan* P, const PacketInfo& pk, int row) {
  hipLaunchKernelGGL(k_dot_partial, dim3(pk.acf_nb), dim3(kAcfThreads), 0, P->stream,
                     P->d_u0 + pk.off, P->d_u[P->cur] + pk.off, pk.n_values,
                     P->d_acfpart + (size_t)row * P->acf_nb_total + pk.acf_part_off);
}

int acf_enqueue(Plan* P, int row, Timing* T) {
  TRY(timed_begin(P, T));
  for (auto& pk : P->packets)
    if (pk.photo) acf_dot(P, pk, row);
  HIP_TRY(hipGetLastError());
  TRY(timed_end(P, T, 5));
  return TDWP_OK;
}

// Sums rows [0, rows) of packet pk and appends them to its series (synchronises).
int acf_collect(Plan* P, PacketInfo& pk, int rows) {
  double* out = P->d_acf + (size_t)pk.acf_idx * kNormChunk;
  hipLaunchKernelGGL(k_rows_sum, dim3((rows + 255) / 256), dim3(256), 0, P->stream,
                     P->d_acfpart + pk.acf_part_off, P->acf_nb_total, pk.acf_nb, rows, out);
  HIP_TRY(hipGetLastError());
  const size_t n0 = pk.acf.size();
  pk.acf.resize(n0 + rows);
  HIP_TRY(hipMemcpyAsync(pk.acf.data() + n0, out, rows * sizeof(double), hipMemcpyDeviceToHost,
                         P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return TDWP_OK;
}

// Sum of a[i] b[i] over n values (device arrays), to the host.
int dev_dot(Plan* P, const double* a, const double* b, size_t n, double* out) {
  const int nb = acf_blocks(n);
  TRY(ensure_staging(P, &P->d_dotpart, &P->dotpart_cap, (size_t)nb + 1));
  hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(kAcfThreads), 0, P->stream, a, b, n,
                     P->d_dotpart);
  hipLaunchKernelGGL(k_rows_sum, dim3(1), dim3(256), 0, P->stream, P->d_dotpart, (size_t)nb, nb, 1,
                     P->d_dotpart + nb);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out, P->d_dotpart + nb, sizeof(double), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return TDWP_OK;
}

// y = a y + b x + c z on the device (z may be null when c = 0).
int dev_axpbypcz(Plan* P, double* y, double a, const double* x, double b, const double* z,
                 double c, size_t n) {
  hipLaunchKernelGGL(k_lincomb, dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)), dim3(256),
                     0, P->stream, y, a, x, b, z, c, n);
  HIP_TRY(hipGetLastError());
  return TDWP_OK;
}

// Lowest eigenvalue of the symmetric tridiagonal matrix (diagonal al[0..m-1],
// off-diagonal be[1..m-1]) by bisection on the Sturm count.
double tridiag_lowest(const std::vector<double>& al, const std::vector<double>& be, int m) {
  double lo = al[0], hi = al[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i ? std::fabs(be[i]) : 0.0) + (i + 1 < m ? std::fabs(be[i + 1]) : 0.0);
    lo = std::min(lo, al[i] - r);
    hi = std::max(hi, al[i] + r);
  }
  auto below = [&](double x) {   // eigenvalues < x
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < m; ++i) {
      const double b2 = i ? be[i] * be[i] : 0.0;
      d = (al[i] - x) - (i ? b2 / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid) >= 1) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Eigenvector of the tridiagonal matrix for eigenvalue lam: inverse iteration with
// Gaussian elimination and row pivoting on (T - lam I), normalised.
std::vector<double> tridiag_vector(const std::vector<double>& al, const std::vector<double>& be,
                                   int m, double lam) {
  double scale = 0.0;
  for (int i = 0; i < m; ++i) scale = std::max(scale, std::fabs(al[i]) + (i ? std::fabs(be[i]) : 0));
  const double shift = lam - 1e-13 * std::max(scale, 1e-300);
  std::vector<double> y(m, 1.0), dl(m), d(m), du(m), du2(m);
  std::vector<int> piv(m);
  // LU with partial pivoting of the tridiagonal (T - shift I), as in a banded solver
  for (int i = 0; i < m; ++i) {
    d[i] = al[i] - shift;
    du[i] = i + 1 < m ? be[i + 1] : 0.0;
    dl[i] = i + 1 < m ? be[i + 1] : 0.0;
    du2[i] = 0.0;
  }
  for (int i = 0; i + 1 < m; ++i) {
    if (std::fabs(d[i]) >= std::fabs(dl[i])) {   // no interchange
      piv[i] = 0;
      const double f = d[i] != 0.0 ? dl[i] / d[i] : 0.0;
      dl[i] = f;
      d[i + 1] -= f * du[i];
    } else {   // interchange rows i and i+1
      piv[i] = 1;
      const double f = d[i] / dl[i];
      d[i] = dl[i];
      dl[i] = f;
      const double t = du[i];
      du[i] = d[i + 1];
      d[i + 1] = t - f * d[i + 1];
      du2[i] = i + 2 < m ? du[i + 1] : 0.0;
      if (i + 2 < m) du[i + 1] = -f * du[i + 1];
    }
  }
  if (d[m - 1] == 0.0) d[m - 1] = 1e-300;
  for (int it = 0; it < 4; ++it) {
    for (int i = 0; i + 1 < m; ++i) {   // forward: apply L^-1 with the interchanges
      if (piv[i]) std::swap(y[i], y[i + 1]);
      y[i + 1] -= dl[i] * y[i];
    }
    for (int i = m - 1; i >= 0; --i) {   // back: U^-1 (diagonal, two superdiagonals)
      double v = y[i];
      if (i + 1 < m) v -= du[i] * y[i + 1];
      if (i + 2 < m) v -= du2[i] * y[i + 2];
      y[i] = v / (d[i] != 0.0 ? d[i] : 1e-300);
    }
    double nrm = 0.0;
    for (double v : y) nrm += v * v;
    nrm = std::sqrt(nrm);
    for (double& v : y) v /= nrm;
  }
  return y;
}

// Checks for the calls that use the packet buffers as scratch (H applied alone):
// potential installed, packet (unit, slot) exists (its index in *ip), none set.
int h_scratch_ready(Plan* P, int unit, int slot, int* ip) {
  if (!P->have_potential) return TDWP_ESTATE;
  *ip = -1;
  for (size_t i = 0; i < P->packets.size(); ++i)
    if (P->packets[i].unit == unit && P->packets[i].slot == slot) *ip = (int)i;
  if (*ip < 0) return TDWP_EINVAL;
  for (auto& pk : P->packets)
    if (pk.set) return TDWP_ESTATE;
  if (!P->d_ones) {
    const std::vector<double> ones((size_t)P->nR * P->nr + P->nR + P->nr, 1.0);
    TRY(alloc_copy(P, &P->d_ones, ones));
    P->ones_cap = ones.size();
  }
  return TDWP_OK;
}

int one_step(Plan* P, int chunk_row, Timing* T);
void reset_propagation(Plan* P);

// out = H in for packet ip (device arrays of its size, outside the packet
// buffers): the first step of the plan with the damping factors set to one
// leaves H_s in in the new buffer, and H in = dE H_s in + E0 in.
int apply_h_dev(Plan* p, int ip, const double* in, double* out) {
  const PacketInfo& P = p->packets[ip];
  const size_t n = P.n_values;
  reset_propagation(p);
  HIP_TRY(hipMemsetAsync(p->d_u[0], 0, p->n_total * sizeof(double), p->stream));
  HIP_TRY(hipMemsetAsync(p->d_u[1], 0, p->n_total * sizeof(double), p->stream));
  HIP_TRY(hipMemcpyAsync(p->d_u[p->cur] + P.off, in, n * sizeof(double), hipMemcpyDeviceToDevice,
                         p->stream));
  double* const keep_D = p->d_D;
  double* const keep_Dsep = p->d_Dsep;
  p->d_D = p->d_ones;
  p->d_Dsep = p->d_ones;
  int st = p->fast ? sync_counters(p) : TDWP_OK;
  if (st == TDWP_OK) st = one_step(p, 0, nullptr);
  p->d_D = keep_D;
  p->d_Dsep = keep_Dsep;
  if (st == TDWP_OK) {
    hipLaunchKernelGGL(k_affine, dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)), dim3(256),
                       0, p->stream, p->d_u[p->cur] + P.off, p->d_u[1 - p->cur] + P.off, p->dE,
                       p->E0, n);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(out, p->d_u[p->cur] + P.off, n * sizeof(double), hipMemcpyDeviceToDevice,
                         p->stream);
    if (e != hipSuccess) st = hip_fail(e, "apply_h_dev", __LINE__);
  }
  reset_propagation(p);
  return st;
}

// The R pass's overlap partials of rows [0, rows), summed per packet in the norm
// partials' fixed order, appended to each photodissociation packet's series.
int acf_collect_pass(Plan* P, int rows) {
  const int np = (int)P->packets.size();
  hipLaunchKernelGGL(k_norm_reduce, dim3((np * rows + 255) / 256), dim3(256), 0, P->stream,
                     P->d_acf, P->d_acfwg, P->n_wg_total, P->d_wg_off, P->d_n_wg, np, rows);
  HIP_TRY(hipGetLastError());
  for (int ip = 0; ip < np; ++ip) {
    PacketInfo& pk = P->packets[ip];
    if (!pk.photo) continue;
    const size_t n0 = pk.acf.size();
    pk.acf.resize(n0 + rows);
    HIP_TRY(hipMemcpyAsync(pk.acf.data() + n0, P->d_acf + (size_t)ip * kNormChunk,
                           rows * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  }
  HIP_TRY(hipStreamSynchronize(P->stream));
  return TDWP_OK;
}

int run_steps(Plan* P, long n_steps, double* norms_out, Timing* T) {
  if (!P->have_potential) return TDWP_ESTATE;
  for (auto& pk : P->packets)
    if (!pk.set) return TDWP_ESTATE;
  const int np = (int)P->packets.size();
  std::vector<double> hn;
  long done = 0;
  while (done < n_steps) {
    const int chunk = (int)std::min<long>(kNormChunk, n_steps - done);
    P->norm_row = 0;
    if (P->fast) TRY(sync_counters(P));
    for (int s = 0; s < chunk;) {
      if (graph_ready(P, chunk - s, T)) {
        switch (P->cfg.precision) {
          case TDWP_FP64: TRY(graph_two_steps<kP64>(P)); break;
          case TDWP_FP32: TRY(graph_two_steps<kP32>(P)); break;
          case TDWP_BF16X3: TRY(graph_two_steps<kPBF>(P)); break;
          default: TRY(graph_two_steps<kPF16>(P)); break;
        }
        s += 2;
      } else {
        TRY(one_step(P, s, T));
        if (P->n_photo && !P->acf_in_pass) TRY(acf_enqueue(P, s, T));
        s += 1;
      }
    }
    const int nq = np * chunk;
    const bool mlp_layout = P->fast && P->pot_mode == TDWP_POT_MLP;
    const bool plane_layout = use_plane(P);
    hipLaunchKernelGGL(k_norm_reduce, dim3((nq + 255) / 256), dim3(256), 0, P->stream,
                       P->d_norms, P->d_normpart, P->n_wg_total,
                       mlp_layout ? P->d_wg_off_mlp : P->d_wg_off,
                       mlp_layout ? P->d_n_wg_mlp : (plane_layout ? P->d_n_wg_plane : P->d_n_wg),
                       np, chunk);
    HIP_TRY(hipGetLastError());
    hn.resize((size_t)np * kNormChunk);
    HIP_TRY(hipMemcpyAsync(hn.data(), P->d_norms, hn.size() * sizeof(double),
                           hipMemcpyDeviceToHost, P->stream));
    HIP_TRY(hipStreamSynchronize(P->stream));
    bool bad = false;
    for (int p = 0; p < np; ++p)
      for (int s = 0; s < chunk; ++s) {
        const double v = hn[(size_t)p * kNormChunk + s];
        if (!std::isfinite(v) || v > 1e6) bad = true;
        if (norms_out) norms_out[(size_t)p * n_steps + done + s] = v;
      }
    if (P->acf_in_pass) TRY(acf_collect_pass(P, chunk));
    else
      for (auto& pk : P->packets)
        if (pk.photo) TRY(acf_collect(P, pk, chunk));
    done += chunk;
    if (bad) return TDWP_ERANGE;
  }
  // the slices of the final u_k are recorded by the next step's r pass, or by the
  // analysis (tdwp_state_to_state) if it comes first: a chunked caller pays no
  // extra pass per call
  return TDWP_OK;
}

void reset_propagation(Plan* P) {
  P->k = 0;
  P->rec_k = -1;
  P->norm_row = 0;
  P->cur = 0;
  P->ring_count = 0;
  P->ring_k0 = 0;
  for (auto& pk : P->packets) {
    pk.set = false;
    pk.snap_taken = false;
    pk.photo = false;
    pk.acf.clear();
  }
  P->n_photo = 0;
  P->acf_nb_total = 0;
  if (P->acf_in_pass) drop_graphs(P);
  P->acf_in_pass = false;
}

}  // namespace

// ---- C ABI -------------------------------------------------------------------

// ---- fixed scratch of the network inference without allocation ------------------
// Device memory for tdwp_mlp_eval_noalloc: the distances of the call, then its
// outputs.  Each GPU holds its own copy for the life of the process; the host
// reaches it only through the address hipGetSymbolAddress returns on that
// device (the array's name is a host-side stand-in, not a device address).
constexpr size_t kNoAllocDoubles = (size_t)1 << 19;   // 4 MiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kMaxDevices = 64;
double* g_scratch_dev[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Once per device, with that device current: the device address of its copy.
int scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return TDWP_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev]) return TDWP_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return TDWP_EDEVICE;
  }
  g_scratch_dev[dev] = static_cast<double*>(ptr);
  return TDWP_OK;
}
}  // namespace

extern "C" int bounds_from_table(tdwp_plan_t p, const double* v);

extern "C" {

int tdwp_plan(const tdwp_config* cfg, tdwp_plan_t* out) {
  if (!out) return TDWP_EINVAL;
  *out = nullptr;
  TRY(validate(cfg));
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return TDWP_EDEVICE;
  }
  query_lds_limit();
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return TDWP_EDEVICE;
  }
  TRY(scratch_setup(dev));
  Plan* P = new (std::nothrow) Plan();
  if (!P) return TDWP_ENOMEM;
  P->device = dev;
  P->cfg = *cfg;
  P->units_in.assign(cfg->units, cfg->units + cfg->n_units);
  P->cfg.units = nullptr;
  P->bounds_given = !(cfg->e_min == 0 && cfg->e_max == 0);
  P->use_graphs = std::getenv("TDWP_NO_GRAPHS") == nullptr;
  if (cfg->stream) {
    P->stream = (hipStream_t)cfg->stream;
  } else {
    if (hipStreamCreate(&P->stream) != hipSuccess) {
      delete P;
      return TDWP_EDEVICE;
    }
    P->own_stream = true;
  }
  int st = build_tables(P);
  if (st == TDWP_OK) st = layout_and_allocate(P);
  if (st != TDWP_OK) {
    free_plan(P);
    return st;
  }
  if (P->fast) {
    // cached choice: 1000 * (angular blocks in XCD order) + 100 * (r pass fused) +
    // 10 * kernel + tile (kernel 1: LDS mixing, 2: register mixing, 3: columns per wave)
    const int c = cached_tile(P);
    const int nt = c % 10, kern = (c / 10) % 10, fz = (c / 100) % 10, xo = (c / 1000) % 10;
    const int pl = c / 10000;
    if ((nt == 1 || nt == 2 || nt == 4) && kern <= 3 && fz <= 1 && xo <= 1 && pl <= 1) {
      P->fuse_r = fz == 1;
      P->ang_xcd = xo == 1;
      P->plane_r = pl == 1 && P->plane_ok;
      P->ang_wave = kern == 3 && P->angw_ok;
      const int keep = P->ang_pref;
      P->ang_pref = kern == 3 ? 2 : kern;
      if (set_ang_tiles(P, nt) != TDWP_OK) {
        P->ang_pref = keep;
        (void)set_ang_tiles(P, P->nta);
      }
    }
  }
  if (P->bounds_given) {
    P->e_min = cfg->e_min;
    P->e_max = cfg->e_max;
    P->E0 = 0.5 * (P->e_max + P->e_min);
    P->dE = 0.5 * (P->e_max - P->e_min);
  }
  *out = P;
  return TDWP_OK;
}

int tdwp_grid(tdwp_plan_t p, double* r, double* R, double* cos_gamma, double* gl_weights) {
  if (!p) return TDWP_EINVAL;
  if (r) std::memcpy(r, p->r.data(), p->nr * sizeof(double));
  if (R) std::memcpy(R, p->R.data(), p->nR * sizeof(double));
  if (cos_gamma) std::memcpy(cos_gamma, p->x.data(), p->ng * sizeof(double));
  if (gl_weights) std::memcpy(gl_weights, p->w.data(), p->ng * sizeof(double));
  return TDWP_OK;
}

int tdwp_diatomic_states(tdwp_plan_t p, const double* v_asym, int j, int n_states,
                         double* energies, double* chi) {
  if (!p || !v_asym || j < 0 || n_states < 1 || n_states > p->nr) return TDWP_EINVAL;
  const int n = p->nr;
  std::vector<double> A(p->Tr);
  for (int i = 0; i < n; ++i) {
    double rot = p->Br[i] * (double)j * (j + 1);
    if (p->cfg.rot_cut > 0) rot = std::min(rot, p->cfg.rot_cut);
    A[(size_t)i * n + i] += v_asym[i] + rot;
  }
  std::vector<double> ev, vec;
  jacobi_eigh(n, A, ev, vec);
  for (int s = 0; s < n_states; ++s) {
    if (energies) energies[s] = ev[s];
    if (!chi) continue;
    double mx = 0.0, nrm = 0.0;
    for (int i = 0; i < n; ++i) {
      mx = std::max(mx, std::fabs(vec[(size_t)i * n + s]));
      nrm += vec[(size_t)i * n + s] * vec[(size_t)i * n + s];
    }
    double sign = 1.0;
    for (int i = 0; i < n; ++i)
      if (std::fabs(vec[(size_t)i * n + s]) > 1e-3 * mx) {
        sign = vec[(size_t)i * n + s] < 0 ? -1.0 : 1.0;
        break;
      }
    const double scale = sign / std::sqrt(nrm);
    for (int i = 0; i < n; ++i) chi[(size_t)s * n + i] = vec[(size_t)i * n + s] * scale;
  }
  return TDWP_OK;
}

int tdwp_set_potential(tdwp_plan_t p, int mode, const double* v, size_t n_values) {
  if (!p || !v) return TDWP_EINVAL;
  if (mode != TDWP_POT_TABLE) return TDWP_EINVAL;
  const size_t plane = (size_t)p->ng * p->nR * p->nr;
  if (n_values != (size_t)p->npair * plane) return TDWP_EINVAL;
  TRY(ensure_table(p));
  HIP_TRY(hipMemcpyAsync(p->d_V, v, n_values * sizeof(double), hipMemcpyHostToDevice, p->stream));
  if (p->d_Vf) {
    hipLaunchKernelGGL(k_to_f32, dim3(1024), dim3(256), 0, p->stream, p->d_V, p->d_Vf, n_values);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (!p->bounds_given) TRY(bounds_from_table(p, v));
  drop_graphs(p);
  p->pot_mode = TDWP_POT_TABLE;
  p->have_potential = true;
  reset_propagation(p);
  return TDWP_OK;
}

int bounds_from_table(tdwp_plan_t p, const double* v) {
  const size_t plane = (size_t)p->ng * p->nR * p->nr;
  {
    // Gershgorin range of the per-point diabatic matrix
    const int ne = p->ne;
    double lo = INFINITY, hi = -INFINITY;
    for (size_t q = 0; q < plane; ++q) {
      for (int a = 0; a < ne; ++a) {
        double off = 0.0, dia = 0.0;
        for (int b = 0; b < ne; ++b) {
          const int i0 = std::min(a, b), i1 = std::max(a, b);
          const int pi = i0 * ne - i0 * (i0 - 1) / 2 + (i1 - i0);
          const double val = v[(size_t)pi * plane + q];
          if (a == b) dia = val;
          else off += std::fabs(val);
        }
        lo = std::min(lo, dia - off);
        hi = std::max(hi, dia + off);
      }
    }
    if (!std::isfinite(lo) || !std::isfinite(hi)) return TDWP_EINVAL;
    double ang = 0.0;
    for (auto& U : p->units)
      for (int j = 0; j < p->ng; ++j) {
        const int nj = U.n_om_j[j];
        if (nj <= 0) continue;
        const double lmax = U.ang_ell[U.ell_off[j] + nj - 1];
        double e = p->Br[0] * (double)j * (j + 1) + p->BR[0] * lmax;
        if (p->cfg.rot_cut > 0) e = std::min(e, p->cfg.rot_cut);
        ang = std::max(ang, e);
      }
    const double tmax = *std::max_element(p->er.begin(), p->er.end()) +
                        *std::max_element(p->eR.begin(), p->eR.end());
    p->e_min = lo;
    p->e_max = hi + tmax + ang;
    p->E0 = 0.5 * (p->e_max + p->e_min);
    p->dE = 0.5 * (p->e_max - p->e_min);
  }
  return TDWP_OK;
}

int tdwp_spectral_bounds(tdwp_plan_t p, double* e_min, double* e_max) {
  if (!p) return TDWP_EINVAL;
  if (!p->have_potential && !p->bounds_given) return TDWP_ESTATE;
  if (e_min) *e_min = p->e_min;
  if (e_max) *e_max = p->e_max;
  return TDWP_OK;
}

int tdwp_set_initial_packet(tdwp_plan_t p, const tdwp_packet* pk, const double* chi0) {
  if (!p || !pk || !chi0) return TDWP_EINVAL;
  if (!p->have_potential) return TDWP_ESTATE;
  if (pk->unit < 0 || pk->unit >= (int)p->units.size()) return TDWP_EINVAL;
  const UnitInfo& U = p->units[pk->unit];
  if (pk->slot < 0 || pk->slot >= U.n_packets) return TDWP_EINVAL;
  if (pk->omega0 < U.om_lo || pk->omega0 > U.om_hi) return TDWP_EINVAL;
  if (pk->j0 < pk->omega0 || pk->j0 > p->ng - 1) return TDWP_EINVAL;
  if (pk->elec0 < 0 || pk->elec0 >= p->ne) return TDWP_EINVAL;
  if (!(pk->width > 0) || !(pk->ecol_mean > 0) || pk->k_min_elastic < 0) return TDWP_EINVAL;
  if (p->k > 0) reset_propagation(p);
  int ip = -1;
  for (size_t i = 0; i < p->packets.size(); ++i)
    if (p->packets[i].unit == pk->unit && p->packets[i].slot == pk->slot) ip = (int)i;
  PacketInfo& P = p->packets[ip];
  P.pk = *pk;
  if (P.photo) {
    P.photo = false;
    P.acf.clear();
    TRY(acf_layout(p));
  }
  const int nr = p->nr, nR = p->nR, ng = p->ng;
  // factor vectors: Legendre row, DVR-weighted Gaussian, channel function
  std::vector<double> pj(ng), g(nR), chi(nr);
  double s = 0.0;
  for (int n = 0; n < ng; ++n) {
    pj[n] = p->Ptab[((size_t)pk->omega0 * ng + pk->j0) * ng + n];
    s += pj[n] * pj[n];
  }
  for (auto& v : pj) v /= std::sqrt(s);
  const double k0 = std::sqrt(2.0 * p->mu * pk->ecol_mean);
  s = 0.0;
  for (int mm = 0; mm < nR; ++mm) {
    const double d = p->R[mm] - pk->R0;
    g[mm] = std::sqrt(p->dR) * std::exp(-d * d / (2.0 * pk->width * pk->width)) * 2.0 *
            std::cos(k0 * p->R[mm]);
    s += g[mm] * g[mm];
  }
  if (!(s > 0)) return TDWP_EINVAL;
  for (auto& v : g) v /= std::sqrt(s);
  s = 0.0;
  for (int i = 0; i < nr; ++i) {
    chi[i] = chi0[i];
    s += chi[i] * chi[i];
  }
  if (!(s > 0) || !std::isfinite(s)) return TDWP_EINVAL;
  for (auto& v : chi) v /= std::sqrt(s);
  P.g = g;
  std::vector<double> stage;
  stage.insert(stage.end(), pj.begin(), pj.end());
  stage.insert(stage.end(), g.begin(), g.end());
  stage.insert(stage.end(), chi.begin(), chi.end());
  TRY(ensure_staging(p, &p->d_chan, &p->chan_cap, stage.size()));
  HIP_TRY(hipMemcpyAsync(p->d_chan, stage.data(), stage.size() * sizeof(double),
                         hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(p->d_g + (size_t)ip * nR, g.data(), nR * sizeof(double),
                         hipMemcpyHostToDevice, p->stream));
  const int col = (pk->omega0 - U.om_lo) * p->ne + pk->elec0;
  hipLaunchKernelGGL(k_build_packet, dim3((unsigned)((P.n_values + 255) / 256)), dim3(256), 0,
                     p->stream, p->d_u[p->cur] + P.off, p->d_u[1 - p->cur] + P.off, P.n_values,
                     col, ng, nR, nr, p->d_chan, p->d_chan + ng, p->d_chan + ng + nR);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemsetAsync(p->d_acc + P.acc_off, 0, (size_t)2 * p->cfg.n_energy * P.n_slice * sizeof(double), p->stream));
  HIP_TRY(hipMemsetAsync(p->d_snap + P.snap_off, 0, (size_t)2 * p->cfg.n_energy * P.n_w * sizeof(double), p->stream));
  P.snap_taken = (pk->k_min_elastic == 0);
  HIP_TRY(hipMemcpyAsync(p->d_E + ip, &pk->E_v0j0, sizeof(double), hipMemcpyHostToDevice, p->stream));
  // k = 0 slices: the matrix-core path records them inside the first step (or in
  // finish_slices), once for all packets; the general path records them here into
  // ring row 0 (packets not yet set are overwritten when they are)
  p->ring_count = 0;
  p->norm_row = 0;
  p->ring_k0 = 0;
  if (p->fast) {
    TRY(sync_counters(p));
    p->rec_k = -1;
  } else {
    TRY(record_slices(p, 0));
    p->ring_count = 1;
    p->rec_k = 0;
  }
  P.set = true;
  HIP_TRY(hipStreamSynchronize(p->stream));
  return TDWP_OK;
}

int tdwp_propagate(tdwp_plan_t p, long n_steps, double* norms) {
  if (!p || n_steps < 0) return TDWP_EINVAL;
  return run_steps(p, n_steps, norms, nullptr);
}

int tdwp_set_packet_values(tdwp_plan_t p, int unit, int slot, const double* u0) {
  if (!p || !u0) return TDWP_EINVAL;
  if (!p->have_potential) return TDWP_ESTATE;
  int ip = -1;
  for (size_t i = 0; i < p->packets.size(); ++i)
    if (p->packets[i].unit == unit && p->packets[i].slot == slot) ip = (int)i;
  if (ip < 0) return TDWP_EINVAL;
  const size_t n = p->packets[ip].n_values;
  double s = 0.0;
  for (size_t q = 0; q < n; ++q) s += u0[q] * u0[q];
  if (!(s > 0) || !std::isfinite(s)) return TDWP_EINVAL;
  if (!p->d_u0) {   // zeros for every packet that is not a photodissociation packet
    TRY(ensure_staging(p, &p->d_u0, &p->u0_cap, p->n_total));
    HIP_TRY(hipMemsetAsync(p->d_u0, 0, p->n_total * sizeof(double), p->stream));
  }
  {   // the autocorrelation buffers for this packet besides the others (no-op if they fit)
    const bool was = p->packets[ip].photo;
    p->packets[ip].photo = true;
    const int st = acf_layout(p);
    p->packets[ip].photo = was;
    if (st != TDWP_OK) {
      (void)acf_layout(p);   // the previous layout fits the existing buffers
      return st;
    }
  }
  if (p->k > 0) reset_propagation(p);
  PacketInfo& P = p->packets[ip];
  P.pk = tdwp_packet{};
  P.pk.unit = unit;
  P.pk.slot = slot;
  HIP_TRY(hipMemcpyAsync(p->d_u0 + P.off, u0, n * sizeof(double), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(p->d_u[p->cur] + P.off, p->d_u0 + P.off, n * sizeof(double),
                         hipMemcpyDeviceToDevice, p->stream));
  HIP_TRY(hipMemsetAsync(p->d_u[1 - p->cur] + P.off, 0, n * sizeof(double), p->stream));
  HIP_TRY(hipMemsetAsync(p->d_acc + P.acc_off, 0, (size_t)2 * p->cfg.n_energy * P.n_slice * sizeof(double), p->stream));
  HIP_TRY(hipMemsetAsync(p->d_snap + P.snap_off, 0, (size_t)2 * p->cfg.n_energy * P.n_w * sizeof(double), p->stream));
  P.snap_taken = true;   // no elastic-channel window
  const double zero = 0.0;
  HIP_TRY(hipMemcpyAsync(p->d_E + ip, &zero, sizeof(double), hipMemcpyHostToDevice, p->stream));
  p->ring_count = 0;
  p->norm_row = 0;
  p->ring_k0 = 0;
  if (p->fast) {
    TRY(sync_counters(p));
    p->rec_k = -1;
  } else {
    TRY(record_slices(p, 0));
    p->ring_count = 1;
    p->rec_k = 0;
  }
  P.photo = true;
  P.acf.clear();
  TRY(acf_layout(p));
  acf_dot(p, P, 0);   // C_0 = <u_0|u_0>
  HIP_TRY(hipGetLastError());
  TRY(acf_collect(p, P, 1));
  P.set = true;
  return TDWP_OK;
}

int tdwp_apply_hamiltonian(tdwp_plan_t p, int unit, int slot, const double* in, double* out) {
  if (!p || !in || !out) return TDWP_EINVAL;
  int ip = -1;
  TRY(h_scratch_ready(p, unit, slot, &ip));
  const PacketInfo& P = p->packets[ip];
  const size_t n = P.n_values;
  TRY(ensure_staging(p, &p->d_lz, &p->lz_cap, 4 * n));
  HIP_TRY(hipMemcpyAsync(p->d_lz, in, n * sizeof(double), hipMemcpyHostToDevice, p->stream));
  int st = apply_h_dev(p, ip, p->d_lz, p->d_lz + n);
  if (st == TDWP_OK) {
    hipError_t e = hipMemcpyAsync(out, p->d_lz + n, n * sizeof(double), hipMemcpyDeviceToHost,
                                  p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) st = hip_fail(e, "tdwp_apply_hamiltonian", __LINE__);
  }
  return st;
}

int tdwp_lowest_state(tdwp_plan_t p, int unit, int slot, const double* guess, int n_iter,
                      double* energy, double* psi, double* residual) {
  if (!p || !guess || !energy || n_iter < 2) return TDWP_EINVAL;
  int ip = -1;
  TRY(h_scratch_ready(p, unit, slot, &ip));
  const size_t n = p->packets[ip].n_values;
  TRY(ensure_staging(p, &p->d_lz, &p->lz_cap, 4 * n));
  double* q = p->d_lz;          // q_j
  double* w = p->d_lz + n;      // H q_j, then the next residual
  double* qp = p->d_lz + 2 * n; // q_{j-1}
  double* x = p->d_lz + 3 * n;  // Ritz vector
  // Lanczos without reorthogonalisation (as the preparatory stage's bound-state
  // program does), from the normalised guess; a second pass rebuilds the q_j for
  // the Ritz vector, so only three vectors are kept.
  auto restart = [&](double* nrm_out) -> int {
    HIP_TRY(hipMemcpyAsync(q, guess, n * sizeof(double), hipMemcpyHostToDevice, p->stream));
    HIP_TRY(hipMemsetAsync(qp, 0, n * sizeof(double), p->stream));
    double s = 0.0;
    TRY(dev_dot(p, q, q, n, &s));
    if (!(s > 0) || !std::isfinite(s)) return TDWP_EINVAL;
    TRY(dev_axpbypcz(p, q, 1.0 / std::sqrt(s), q, 0.0, nullptr, 0.0, n));
    if (nrm_out) *nrm_out = s;
    return TDWP_OK;
  };
  std::vector<double> al, be(1, 0.0);
  TRY(restart(nullptr));
  for (int j = 0; j < n_iter; ++j) {
    TRY(apply_h_dev(p, ip, q, w));
    double a = 0.0;
    TRY(dev_dot(p, w, q, n, &a));
    TRY(dev_axpbypcz(p, w, 1.0, q, -a, qp, -be[j], n));   // w = H q - a q - b qp
    double b2 = 0.0;
    TRY(dev_dot(p, w, w, n, &b2));
    al.push_back(a);
    const double b = std::sqrt(b2);
    if (j + 1 == n_iter || !(b > 1e-14 * std::fabs(a))) break;   // invariant subspace found
    be.push_back(b);
    TRY(dev_axpbypcz(p, qp, 0.0, q, 1.0, nullptr, 0.0, n));      // qp = q
    TRY(dev_axpbypcz(p, q, 0.0, w, 1.0 / b, nullptr, 0.0, n));   // q = w / b
  }
  const int m = (int)al.size();
  const double lam = tridiag_lowest(al, be, m);
  const std::vector<double> y = tridiag_vector(al, be, m, lam);
  // second pass: x = sum_j y_j q_j with the same recursion coefficients
  TRY(restart(nullptr));
  HIP_TRY(hipMemsetAsync(x, 0, n * sizeof(double), p->stream));
  for (int j = 0; j < m; ++j) {
    TRY(dev_axpbypcz(p, x, 1.0, q, y[j], nullptr, 0.0, n));
    if (j + 1 == m) break;
    TRY(apply_h_dev(p, ip, q, w));
    TRY(dev_axpbypcz(p, w, 1.0, q, -al[j], qp, -be[j], n));
    TRY(dev_axpbypcz(p, qp, 0.0, q, 1.0, nullptr, 0.0, n));
    TRY(dev_axpbypcz(p, q, 0.0, w, 1.0 / be[j + 1], nullptr, 0.0, n));
  }
  double xx = 0.0;
  TRY(dev_dot(p, x, x, n, &xx));
  if (!(xx > 0) || !std::isfinite(xx)) return TDWP_ERANGE;
  TRY(dev_axpbypcz(p, x, 1.0 / std::sqrt(xx), x, 0.0, nullptr, 0.0, n));
  // Rayleigh quotient and residual of the normalised Ritz vector
  TRY(apply_h_dev(p, ip, x, w));
  double e = 0.0;
  TRY(dev_dot(p, x, w, n, &e));
  *energy = e;
  if (residual) {
    TRY(dev_axpbypcz(p, w, 1.0, x, -e, nullptr, 0.0, n));
    double r2 = 0.0;
    TRY(dev_dot(p, w, w, n, &r2));
    *residual = std::sqrt(r2);
  }
  if (psi) {
    HIP_TRY(hipMemcpyAsync(psi, x, n * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  return TDWP_OK;
}

int tdwp_autocorrelation(tdwp_plan_t p, int unit, int slot, long n, double* out) {
  if (!p || n < 0 || (n > 0 && !out)) return TDWP_EINVAL;
  for (auto& pk : p->packets)
    if (pk.unit == unit && pk.slot == slot) {
      if (!pk.set || !pk.photo) return TDWP_ESTATE;
      if ((size_t)n > pk.acf.size()) return TDWP_EINVAL;
      std::copy(pk.acf.begin(), pk.acf.begin() + n, out);
      return TDWP_OK;
    }
  return TDWP_EINVAL;
}

int tdwp_step_index(tdwp_plan_t p, long* k) {
  if (!p || !k) return TDWP_EINVAL;
  *k = p->k;
  return TDWP_OK;
}

int tdwp_get_packet(tdwp_plan_t p, int unit, int slot, int which, double* out) {
  if (!p || !out || (which != 0 && which != 1)) return TDWP_EINVAL;
  for (auto& pk : p->packets)
    if (pk.unit == unit && pk.slot == slot) {
      if (!pk.set) return TDWP_ESTATE;
      const double* src = p->d_u[which == 0 ? p->cur : 1 - p->cur] + pk.off;
      HIP_TRY(hipMemcpyAsync(out, src, pk.n_values * sizeof(double), hipMemcpyDeviceToHost, p->stream));
      HIP_TRY(hipStreamSynchronize(p->stream));
      return TDWP_OK;
    }
  return TDWP_EINVAL;
}

int tdwp_state_to_state(tdwp_plan_t p, int unit, int slot, int n_ch, const tdwp_channel* ch,
                        const double* chi, double* p_inel, double* p_reac) {
  if (!p || n_ch < 0 || (n_ch > 0 && (!ch || !chi))) return TDWP_EINVAL;
  int ip = -1;
  for (size_t i = 0; i < p->packets.size(); ++i)
    if (p->packets[i].unit == unit && p->packets[i].slot == slot) ip = (int)i;
  if (ip < 0) return TDWP_EINVAL;
  PacketInfo& P = p->packets[ip];
  if (!P.set || P.photo) return TDWP_ESTATE;
  const UnitInfo& U = p->units[unit];
  const tdwp_config& c = p->cfg;
  const int nE = c.n_energy;
  const double step = (c.ecol_max - c.ecol_min) / (nE - 1);
  for (int f = 0; f < n_ch; ++f) {
    if (ch[f].elec < 0 || ch[f].elec >= p->ne || ch[f].j < 0 || ch[f].j > p->ng - 1) return TDWP_EINVAL;
    if (ch[f].omega < U.om_lo || ch[f].omega > U.om_hi) return TDWP_EINVAL;
  }
  TRY(finish_slices(p, nullptr));
  TRY(flush_ring(p));
  const size_t need_out = (size_t)(n_ch + p->ne) * nE;
  TRY(ensure_staging(p, &p->d_out, &p->out_cap, need_out));
  if (p_reac) {
    hipLaunchKernelGGL(k_flux, dim3(p->ne, nE), dim3(256), 0, p->stream, p->d_out + (size_t)n_ch * nE,
                       p->d_acc + P.acc_off, p->d_g + (size_t)ip * p->nR, U.n_om, nE, p->ne, p->ng,
                       p->nR, P.n_slice, P.n_sv, c.ecol_min, step, p->mu, p->m, c.R_min, p->dR);
    HIP_TRY(hipGetLastError());
  }
  if (n_ch > 0 && p_inel) {
    // staging: chi [n_ch][nr], energies [n_ch], then int records [n_ch][5]
    const size_t nd = (size_t)n_ch * p->nr + n_ch;
    const size_t ni_d = ((size_t)n_ch * 5 * sizeof(int) + sizeof(double) - 1) / sizeof(double);
    TRY(ensure_staging(p, &p->d_chan, &p->chan_cap, nd + ni_d));
    std::vector<double> host(nd + ni_d, 0.0);
    std::memcpy(host.data(), chi, (size_t)n_ch * p->nr * sizeof(double));
    std::vector<int> rec((size_t)n_ch * 5);
    for (int f = 0; f < n_ch; ++f) {
      host[(size_t)n_ch * p->nr + f] = ch[f].energy;
      const bool initial = ch[f].elec == P.pk.elec0 && ch[f].v == P.pk.v0 && ch[f].j == P.pk.j0 &&
                           ch[f].omega == P.pk.omega0;
      rec[f * 5 + 0] = ch[f].omega - U.om_lo;
      rec[f * 5 + 1] = ch[f].elec;
      rec[f * 5 + 2] = ch[f].j;
      rec[f * 5 + 3] = ch[f].omega;
      rec[f * 5 + 4] = initial ? 1 : 0;
    }
    std::memcpy(host.data() + nd, rec.data(), rec.size() * sizeof(int));
    HIP_TRY(hipMemcpyAsync(p->d_chan, host.data(), host.size() * sizeof(double),
                           hipMemcpyHostToDevice, p->stream));
    const int snap_valid = P.snap_taken ? 1 : 0;
    hipLaunchKernelGGL(k_project, dim3(n_ch, nE), dim3(256), 0, p->stream, p->d_out,
                       p->d_acc + P.acc_off, p->d_snap + P.snap_off, snap_valid, p->d_chan,
                       (const int*)(p->d_chan + nd), p->d_chan + (size_t)n_ch * p->nr, p->d_P,
                       p->d_g + (size_t)ip * p->nR, n_ch, nE, p->ne, p->ng, p->nR, p->nr,
                       P.n_slice, 2 * P.n_sv, P.n_w, c.ecol_min, step, P.pk.E_v0j0, p->mu,
                       c.R_min, p->dR, p->R[p->m_inf]);
    HIP_TRY(hipGetLastError());
  }
  std::vector<double> h(need_out);
  HIP_TRY(hipMemcpyAsync(h.data(), p->d_out, need_out * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (p_inel && n_ch > 0) std::memcpy(p_inel, h.data(), (size_t)n_ch * nE * sizeof(double));
  if (p_reac) std::memcpy(p_reac, h.data() + (size_t)n_ch * nE, (size_t)p->ne * nE * sizeof(double));
  return TDWP_OK;
}

int tdwp_time_kernels(tdwp_plan_t p, long n_steps, int n_max, double* avg_us, char* names,
                      size_t names_len) {
  if (!p || n_steps < 1 || n_max < 0) return TDWP_EINVAL;
  Timing T;
  HIP_TRY(hipEventCreate(&T.ev[0]));
  HIP_TRY(hipEventCreate(&T.ev[1]));
  int st = run_steps(p, n_steps, nullptr, &T);
  (void)hipEventDestroy(T.ev[0]);
  (void)hipEventDestroy(T.ev[1]);
  if (st != TDWP_OK) return st;
  static const char* kinds[8] = {"angular", "radial_R_epilogue", "slices", "accumulate", "radial_r",
                                 "autocorrelation", "radial_rR_epilogue", "products"};
  std::string joined;
  for (int i = 0; i < 8; ++i) {
    if (i < n_max && avg_us) avg_us[i] = T.calls[i] ? 1000.0 * T.ms[i] / T.calls[i] : 0.0;
    if (i) joined += ";";
    joined += kinds[i];
  }
  if (names && names_len) {
    std::strncpy(names, joined.c_str(), names_len - 1);
    names[names_len - 1] = 0;
  }
  return 8;
}

int tdwp_autotune(tdwp_plan_t p, int steps, char* report, size_t report_len) {
  if (!p || steps < 1) return TDWP_EINVAL;
  if (!p->have_potential) return TDWP_ESTATE;
  for (auto& pk : p->packets)
    if (pk.set) return TDWP_ESTATE;
  if (!p->fast) return TDWP_OK;
  Timing T;
  HIP_TRY(hipEventCreate(&T.ev[0]));
  HIP_TRY(hipEventCreate(&T.ev[1]));
  // the timed steps run on zeroed buffers (no packet is installed yet)
  HIP_TRY(hipMemsetAsync(p->d_u[0], 0, p->n_total * sizeof(double), p->stream));
  HIP_TRY(hipMemsetAsync(p->d_u[1], 0, p->n_total * sizeof(double), p->stream));
  std::string rep;
  const int keep_pref = p->ang_pref, keep_nt = p->nta;
  const bool keep_fuse = p->fuse_r, keep_xcd = p->ang_xcd, keep_plane = p->plane_r;
  const bool keep_wave = p->ang_wave;
  int best_k = -1, best_nt = keep_nt, best_f = keep_fuse ? 1 : 0, best_x = keep_xcd ? 1 : 0;
  int best_p = keep_plane ? 1 : 0;
  double best_us = 1e300;
  // both radial terms in one plane pass, or the r pass beside the angular pass or
  // after it x angular kernel (3: columns held per wave, 2: helicity mixing in
  // registers, 1: through LDS) x tile width; the kernels of whole steps are timed
  for (int pl : {1, 0})
  for (int xo : {0, 1})
  for (int fz : {1, 0})
  for (int kern : {3, 2, 1})
    for (int nt : {4, 2, 1}) {
      if (pl && (!p->plane_ok || fz)) continue;   // the plane pass follows a plain angular pass
      // the per-wave kernel has no tile width, no XCD order and no fused form
      if (kern == 3 && (!p->angw_ok || fz || nt != 1 || xo)) continue;
      p->plane_r = pl == 1;
      p->ang_xcd = xo == 1;
      p->fuse_r = fz == 1;
      p->ang_wave = kern == 3;
      p->ang_pref = kern == 3 ? 2 : kern;
      if (set_ang_tiles(p, nt) != TDWP_OK) continue;
      reset_propagation(p);
      int st = sync_counters(p);
      for (int s2 = 0; s2 < steps + 1 && st == TDWP_OK; ++s2) {   // the first step warms up
        if (s2 <= 1)
          for (int q : {0, 1, 4, 6}) {
            T.ms[q] = 0.0;
            T.calls[q] = 0;
          }
        st = one_step(p, 0, &T);
      }
      reset_propagation(p);
      if (st != TDWP_OK) {
        (void)hipEventDestroy(T.ev[0]);
        (void)hipEventDestroy(T.ev[1]);
        p->ang_pref = keep_pref;
        p->fuse_r = keep_fuse;
        p->ang_xcd = keep_xcd;
        p->plane_r = keep_plane;
        p->ang_wave = keep_wave;
        (void)set_ang_tiles(p, keep_nt);
        return st;
      }
      // the whole step: the launch form also changes what the later passes read
      const double us =
          1000.0 * (T.ms[0] + T.ms[1] + T.ms[4] + T.ms[6]) / std::max<long>(T.calls[0], 1);
      char buf[80];
      std::snprintf(buf, sizeof buf, "%sp%d_x%d_f%d_k%d_nt%d:%.1fus", rep.empty() ? "" : ";", pl,
                    xo, fz, kern, nt, us);
      rep += buf;
      if (us < best_us) {
        best_us = us;
        best_k = kern;
        best_nt = nt;
        best_f = fz;
        best_x = xo;
        best_p = pl;
      }
    }
  (void)hipEventDestroy(T.ev[0]);
  (void)hipEventDestroy(T.ev[1]);
  if (best_k < 0) {   // no variant fits: keep the plan's choice
    p->ang_pref = keep_pref;
    p->fuse_r = keep_fuse;
    p->ang_xcd = keep_xcd;
    p->plane_r = keep_plane;
    p->ang_wave = keep_wave;
    TRY(set_ang_tiles(p, keep_nt));
  } else {
    p->ang_wave = best_k == 3;
    p->ang_pref = best_k == 3 ? 2 : best_k;
    p->fuse_r = best_f == 1;
    p->ang_xcd = best_x == 1;
    p->plane_r = best_p == 1;
    TRY(set_ang_tiles(p, best_nt));
    store_tile(p, 10000 * best_p + 1000 * best_x + 100 * best_f + 10 * best_k + best_nt);
  }
  drop_graphs(p);
  reset_propagation(p);
  if (report && report_len) {
    rep += ";chosen=p" + std::to_string(use_plane(p) ? 1 : 0) + "_x" +
           std::to_string(p->ang_xcd ? 1 : 0) + "_f" + std::to_string(p->fuse_r ? 1 : 0) +
           "_k" + std::to_string(use_angw(p) ? 3 : (p->ang_regs ? 2 : 1)) + "_nt" +
           std::to_string(p->nta);
    std::strncpy(report, rep.c_str(), report_len - 1);
    report[report_len - 1] = 0;
  }
  return TDWP_OK;
}

int tdwp_set_option(tdwp_plan_t p, int option, long value) {
  if (!p) return TDWP_EINVAL;
  switch (option) {
    case TDWP_OPT_GRAPHS:
      if (value != 0 && value != 1) return TDWP_EINVAL;
      p->use_graphs = value != 0;
      return TDWP_OK;
    case TDWP_OPT_ANG_TILE:
      if (!p->fast || (value != 1 && value != 2 && value != 4)) return TDWP_EINVAL;
      TRY(set_ang_tiles(p, (int)value));
      drop_graphs(p);
      return TDWP_OK;
    case TDWP_OPT_ANG_KERNEL: {
      if (!p->fast || value < 0 || value > 3) return TDWP_EINVAL;
      if (value == 3) {
        if (!p->angw_ok) return TDWP_EINVAL;
        p->ang_wave = true;
        drop_graphs(p);
        return TDWP_OK;
      }
      p->ang_wave = false;
      const int keep = p->ang_pref;
      p->ang_pref = (int)value;
      int regs = 0;
      size_t lds = 0;
      if (!ang_config(p, p->nta, &regs, &lds)) {
        p->ang_pref = keep;
        return TDWP_EINVAL;
      }
      TRY(set_ang_tiles(p, p->nta));
      drop_graphs(p);
      return TDWP_OK;
    }
    case TDWP_OPT_ANG_XCD:
      if (value != 0 && value != 1) return TDWP_EINVAL;
      p->ang_xcd = value != 0;
      drop_graphs(p);
      return TDWP_OK;
    case TDWP_OPT_FUSE_R:
      if (value != 0 && value != 1) return TDWP_EINVAL;
      p->fuse_r = value != 0;
      drop_graphs(p);
      return TDWP_OK;
    case TDWP_OPT_PLANE_R:
      if (value != 0 && value != 1) return TDWP_EINVAL;
      if (value == 1 && !(p->fast && p->plane_ok)) return TDWP_EINVAL;
      p->plane_r = value != 0;
      drop_graphs(p);
      return TDWP_OK;
    case TDWP_OPT_RADIAL_GRID:
      if (value < 0 || value > (1L << 30)) return TDWP_EINVAL;
      p->radial_grid = value;
      drop_graphs(p);
      return TDWP_OK;
    default:
      return TDWP_EINVAL;
  }
}

int tdwp_get_stat(tdwp_plan_t p, int stat, long* value) {
  if (!p || !value) return TDWP_EINVAL;
  switch (stat) {
    case TDWP_STAT_GRAPH_STEPS: *value = p->graph_steps; return TDWP_OK;
    case TDWP_STAT_ANG_TILE: *value = p->fast ? p->nta : 0; return TDWP_OK;
    case TDWP_STAT_ANG_KERNEL:
      *value = p->fast ? (use_angw(p) ? 3 : (p->ang_regs ? 2 : 1)) : 0;
      return TDWP_OK;
    case TDWP_STAT_MATRIX_CORE_PATH: *value = p->fast ? 1 : 0; return TDWP_OK;
    case TDWP_STAT_FUSE_R: *value = (p->fast && p->fuse_r) ? 1 : 0; return TDWP_OK;
    case TDWP_STAT_RING_LEN: *value = p->ring_len; return TDWP_OK;
    case TDWP_STAT_PLANE_R: *value = use_plane(p) ? 1 : 0; return TDWP_OK;
    case TDWP_STAT_POTENTIAL_BYTES: {
      const size_t n = (size_t)p->npair * p->ng * p->nR * p->nr;
      size_t b = (p->d_V ? n * sizeof(double) : 0) + (p->d_Vf ? n * sizeof(float) : 0);
      if (p->pot_mode == TDWP_POT_MLP)
        b += (size_t)p->mlp_nparams * sizeof(float) +
             ((size_t)kMlpH * 32 + 2 * kMlpH * kMlpH + 16 * kMlpH) * sizeof(__bf16) +
             (size_t)(3 * kMlpH + 16) * sizeof(float);
      *value = (long)b;
      return TDWP_OK;
    }
    default: return TDWP_EINVAL;
  }
}

int tdwp_mlp_n_params(tdwp_plan_t p) {
  if (!p) return TDWP_EINVAL;
  return mlp_param_count(p->npair);
}

int tdwp_set_potential_mlp(tdwp_plan_t p, const double* v, size_t n_values,
                           const tdwp_mlp_options* o, double* report) {
  if (!p || !v || !o) return TDWP_EINVAL;
  const size_t plane = (size_t)p->ng * p->nR * p->nr;
  if (n_values != (size_t)p->npair * plane) return TDWP_EINVAL;
  if (o->n_samples < 1 || !o->sample_idx || !o->init_params || !o->order) return TDWP_EINVAL;
  if (o->batch < 1 || o->batch > 4096 || o->batch > o->n_samples || o->epochs < 0) return TDWP_EINVAL;
  if (!(o->lr > 0) || !(o->lr_final >= 0) || o->lr_final > o->lr) return TDWP_EINVAL;
  if (!p->fast || p->ne > kMaxElec || mlp_epi_lds((int)p->packets.size()) > kLdsMax) return TDWP_EINVAL;
  for (int i = 0; i < o->n_samples; ++i) {
    if (o->sample_idx[i] < 0 || (size_t)o->sample_idx[i] >= plane) return TDWP_EINVAL;
    if (o->order[i] < 0 || o->order[i] >= o->n_samples) return TDWP_EINVAL;
  }
  TRY(ensure_table(p));   // the training targets
  HIP_TRY(hipMemcpyAsync(p->d_V, v, n_values * sizeof(double), hipMemcpyHostToDevice, p->stream));
  const int npar = mlp_param_count(p->npair);
  p->mlp_nparams = npar;
  if (!p->d_mlp_theta) {
    TRY(dev_alloc(p, (void**)&p->d_mlp_theta, (size_t)npar * sizeof(float)));
    const size_t nw = (size_t)kMlpH * 32 + 2 * kMlpH * kMlpH + 16 * kMlpH;
    TRY(dev_alloc(p, &p->d_mlp_w, nw * sizeof(__bf16)));
    TRY(dev_alloc(p, (void**)&p->d_mlp_b, (size_t)(3 * kMlpH + 16) * sizeof(float)));
  }
  Scratch S;
  float *g = nullptr, *m1 = nullptr, *m2 = nullptr;
  long* d_idx = nullptr;
  int* d_ord = nullptr;
  TRY(S.get((void**)&g, (size_t)npar * sizeof(float)));
  TRY(S.get((void**)&m1, (size_t)npar * sizeof(float)));
  TRY(S.get((void**)&m2, (size_t)npar * sizeof(float)));
  TRY(S.get((void**)&d_idx, (size_t)o->n_samples * sizeof(long)));
  TRY(S.get((void**)&d_ord, (size_t)o->n_samples * sizeof(int)));
  HIP_TRY(hipMemcpyAsync(p->d_mlp_theta, o->init_params, (size_t)npar * sizeof(float), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(d_idx, o->sample_idx, (size_t)o->n_samples * sizeof(long), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(d_ord, o->order, (size_t)o->n_samples * sizeof(int), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipMemsetAsync(m1, 0, (size_t)npar * sizeof(float), p->stream));
  HIP_TRY(hipMemsetAsync(m2, 0, (size_t)npar * sizeof(float), p->stream));
  MlpPass q;
  const int B = o->batch;
  TRY(mlp_alloc_pass(S, p, B, &q));
  const double mbc = p->cfg.mass_B + p->cfg.mass_C;
  const double cB = p->cfg.mass_C / mbc, cC = p->cfg.mass_B / mbc;
  const int nb = o->n_samples / B;
  long step = 0;
  const double b1 = 0.9, b2 = 0.999;
  for (int e = 0; e < o->epochs; ++e)
    for (int b = 0; b < nb; ++b) {
      const long e0 = (long)e * o->n_samples + (long)b * B;
      hipLaunchKernelGGL(k_mlp_batch, dim3((B + 255) / 256), dim3(256), 0, p->stream, d_idx, d_ord,
                         o->n_samples, e0, B, p->d_V, p->npair, plane, p->d_rg, p->d_Rg, p->d_xg,
                         p->nR, p->nr, cB, cC, q.X, q.T);
      TRY(mlp_fwd_bwd(p, p->d_mlp_theta, g, B, q));
      ++step;
      const float c1 = (float)(1.0 - std::pow(b1, (double)step));
      const float c2 = (float)(1.0 - std::pow(b2, (double)step));
      // cosine decay from lr to lr_final over the run (constant when lr_final is 0)
      const double frac = (o->epochs * (long)nb > 1) ? (double)(step - 1) / (double)(o->epochs * (long)nb - 1) : 0.0;
      const double lr = o->lr_final > 0
                            ? o->lr_final + 0.5 * (o->lr - o->lr_final) * (1.0 + std::cos(M_PI * frac))
                            : o->lr;
      hipLaunchKernelGGL(k_adam, dim3((npar + 255) / 256), dim3(256), 0, p->stream, p->d_mlp_theta, g,
                         m1, m2, npar, (float)lr, (float)b1, (float)b2, 1e-8f, c1, c2);
      HIP_TRY(hipGetLastError());
    }
  // final training loss over every sample (forward only; the gradient is discarded)
  double loss_sum = 0.0;
  {
    const int nparts = (B * p->npair + 255) / 256;
    std::vector<float> part(nparts);
    for (int b = 0; b < nb; ++b) {
      hipLaunchKernelGGL(k_mlp_batch, dim3((B + 255) / 256), dim3(256), 0, p->stream, d_idx, d_ord,
                         o->n_samples, (long)b * B, B, p->d_V, p->npair, plane, p->d_rg, p->d_Rg,
                         p->d_xg, p->nR, p->nr, cB, cC, q.X, q.T);
      TRY(mlp_fwd_bwd(p, p->d_mlp_theta, g, B, q));
      HIP_TRY(hipMemcpyAsync(part.data(), q.part, nparts * sizeof(float), hipMemcpyDeviceToHost, p->stream));
      HIP_TRY(hipStreamSynchronize(p->stream));
      for (float x : part) loss_sum += x;
    }
    loss_sum /= (double)nb * B * p->npair;
  }
  hipLaunchKernelGGL(k_mlp_pack, dim3((kMlpH * kMlpH + 255) / 256), dim3(256), 0, p->stream,
                     p->d_mlp_theta, p->npair, (__bf16*)p->d_mlp_w,
                     (__bf16*)p->d_mlp_w + kMlpH * 32,
                     (__bf16*)p->d_mlp_w + kMlpH * 32 + kMlpH * kMlpH,
                     (__bf16*)p->d_mlp_w + kMlpH * 32 + 2 * kMlpH * kMlpH, p->d_mlp_b);
  HIP_TRY(hipGetLastError());
  // the network on the whole grid: error against the table, and spectral bounds
  double* d_vm = nullptr;
  TRY(S.get((void**)&d_vm, (size_t)p->npair * plane * sizeof(double)));
  const long n_pts = (long)plane;
  hipLaunchKernelGGL(k_mlp_grid, dim3((unsigned)((n_pts + 63) / 64)), dim3(256), 0, p->stream,
                     mlp_net(p), p->d_rg, p->d_Rg, p->d_xg, p->ng, p->nR, p->nr, cB, cC, d_vm);
  HIP_TRY(hipGetLastError());
  std::vector<double> vm((size_t)p->npair * plane);
  HIP_TRY(hipMemcpyAsync(vm.data(), d_vm, vm.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  double se = 0.0, mx = 0.0;
  for (size_t q2 = 0; q2 < vm.size(); ++q2) {
    const double d = vm[q2] - v[q2];
    se += d * d;
    mx = std::max(mx, std::fabs(d));
  }
  if (!p->bounds_given) TRY(bounds_from_table(p, vm.data()));
  if (report) {
    report[0] = loss_sum;
    report[1] = std::sqrt(se / (double)vm.size());
    report[2] = mx;
  }
  drop_graphs(p);
  // the steps evaluate the network: the table is no longer held
  HIP_TRY(hipStreamSynchronize(p->stream));
  dev_release(p, (void**)&p->d_V);
  dev_release(p, (void**)&p->d_Vf);
  p->pot_mode = TDWP_POT_MLP;
  p->have_potential = true;
  reset_propagation(p);
  return TDWP_OK;
}

int tdwp_mlp_params(tdwp_plan_t p, float* params) {
  if (!p || !params) return TDWP_EINVAL;
  if (!p->d_mlp_theta) return TDWP_ESTATE;
  HIP_TRY(hipMemcpyAsync(params, p->d_mlp_theta, (size_t)p->mlp_nparams * sizeof(float),
                         hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return TDWP_OK;
}

int tdwp_mlp_gradient(tdwp_plan_t p, const float* params, int n_pts, const double* dist,
                      const double* v, double* loss, float* grad) {
  if (!p || !params || !dist || !v || n_pts < 1 || n_pts > 65536) return TDWP_EINVAL;
  const int npar = mlp_param_count(p->npair);
  Scratch S;
  float *th = nullptr, *g = nullptr;
  double *dd = nullptr, *dv = nullptr;
  TRY(S.get((void**)&th, (size_t)npar * sizeof(float)));
  TRY(S.get((void**)&g, (size_t)npar * sizeof(float)));
  TRY(S.get((void**)&dd, (size_t)n_pts * 3 * sizeof(double)));
  TRY(S.get((void**)&dv, (size_t)n_pts * p->npair * sizeof(double)));
  MlpPass q;
  TRY(mlp_alloc_pass(S, p, n_pts, &q));
  HIP_TRY(hipMemcpyAsync(th, params, (size_t)npar * sizeof(float), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(dd, dist, (size_t)n_pts * 3 * sizeof(double), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(dv, v, (size_t)n_pts * p->npair * sizeof(double), hipMemcpyHostToDevice, p->stream));
  hipLaunchKernelGGL(k_mlp_feats, dim3((n_pts + 255) / 256), dim3(256), 0, p->stream, dd, dv, n_pts,
                     p->npair, q.X, q.T);
  TRY(mlp_fwd_bwd(p, th, g, n_pts, q));
  const int nparts = (n_pts * p->npair + 255) / 256;
  std::vector<float> part(nparts);
  HIP_TRY(hipMemcpyAsync(part.data(), q.part, nparts * sizeof(float), hipMemcpyDeviceToHost, p->stream));
  if (grad) HIP_TRY(hipMemcpyAsync(grad, g, (size_t)npar * sizeof(float), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  double s = 0.0;
  for (float x : part) s += x;
  if (loss) *loss = s / ((double)n_pts * p->npair);
  return TDWP_OK;
}

int tdwp_mlp_eval(tdwp_plan_t p, int n_pts, const double* dist, double* v_out) {
  if (!p || !dist || !v_out || n_pts < 1) return TDWP_EINVAL;
  if (!p->d_mlp_theta || p->pot_mode != TDWP_POT_MLP) return TDWP_ESTATE;
  Scratch S;
  double *dd = nullptr, *dv = nullptr;
  TRY(S.get((void**)&dd, (size_t)n_pts * 3 * sizeof(double)));
  TRY(S.get((void**)&dv, (size_t)n_pts * p->npair * sizeof(double)));
  HIP_TRY(hipMemcpyAsync(dd, dist, (size_t)n_pts * 3 * sizeof(double), hipMemcpyHostToDevice, p->stream));
  hipLaunchKernelGGL(k_mlp_eval, dim3((n_pts + 63) / 64), dim3(256), 0, p->stream, mlp_net(p), dd,
                     n_pts, dv);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(v_out, dv, (size_t)n_pts * p->npair * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return TDWP_OK;
}

int tdwp_mlp_eval_noalloc(tdwp_plan_t p, int n_pts, const double* dist, double* v_out) {
  if (!p || !dist || !v_out || n_pts < 1) return TDWP_EINVAL;
  if (!p->d_mlp_theta || p->pot_mode != TDWP_POT_MLP) return TDWP_ESTATE;
  const size_t need = (size_t)n_pts * (3 + (size_t)p->npair);
  if (need > kNoAllocDoubles) return TDWP_ESCRATCH;
  double* base = (p->device >= 0 && p->device < kMaxDevices) ? g_scratch_dev[p->device] : nullptr;
  if (!base) return TDWP_EDEVICE;
  double* dd = base;                          // [n_pts][3] distances
  double* dv = base + (size_t)n_pts * 3;      // [n_pts][n_pair] outputs (every entry written)
  HIP_TRY(hipMemcpyAsync(dd, dist, (size_t)n_pts * 3 * sizeof(double), hipMemcpyHostToDevice, p->stream));
  hipLaunchKernelGGL(k_mlp_eval, dim3((n_pts + 63) / 64), dim3(256), 0, p->stream, mlp_net(p), dd,
                     n_pts, dv);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(v_out, dv, (size_t)n_pts * p->npair * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return TDWP_OK;
}

int tdwp_mlp_grid(tdwp_plan_t p, double* v_out) {
  if (!p || !v_out) return TDWP_EINVAL;
  if (!p->d_mlp_theta || p->pot_mode != TDWP_POT_MLP) return TDWP_ESTATE;
  const size_t plane = (size_t)p->ng * p->nR * p->nr;
  Scratch S;
  double* dv = nullptr;
  TRY(S.get((void**)&dv, (size_t)p->npair * plane * sizeof(double)));
  const double mbc = p->cfg.mass_B + p->cfg.mass_C;
  hipLaunchKernelGGL(k_mlp_grid, dim3((unsigned)((plane + 63) / 64)), dim3(256), 0, p->stream,
                     mlp_net(p), p->d_rg, p->d_Rg, p->d_xg, p->ng, p->nR, p->nr,
                     p->cfg.mass_C / mbc, p->cfg.mass_B / mbc, dv);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(v_out, dv, (size_t)p->npair * plane * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return TDWP_OK;
}

int tdwp_product_grid(tdwp_plan_t p, double* r_prod, double* cos_gamma_prod, double* weights) {
  if (!p || p->prod_np == 0) return TDWP_EINVAL;
  if (r_prod) std::copy(p->prod_r.begin(), p->prod_r.end(), r_prod);
  if (cos_gamma_prod) std::copy(p->prod_x.begin(), p->prod_x.end(), cos_gamma_prod);
  if (weights) std::copy(p->prod_w.begin(), p->prod_w.end(), weights);
  return TDWP_OK;
}

int tdwp_product_diatomic_states(tdwp_plan_t p, const double* v_asym, int j, int n_states,
                                 double* energies, double* chi) {
  if (!p || p->prod_np == 0) return TDWP_EINVAL;
  return product_channels(p, v_asym, j, n_states, energies, chi);
}

int tdwp_state_to_state_products(tdwp_plan_t p, int unit, int slot, int n_ch,
                                 const tdwp_channel* ch, const double* chi, double* p_prod) {
  if (!p || n_ch < 0 || (n_ch > 0 && (!ch || !chi || !p_prod))) return TDWP_EINVAL;
  if (p->prod_np == 0) return TDWP_EINVAL;
  int ip = -1;
  for (size_t i = 0; i < p->packets.size(); ++i)
    if (p->packets[i].unit == unit && p->packets[i].slot == slot) ip = (int)i;
  if (ip < 0) return TDWP_EINVAL;
  PacketInfo& P = p->packets[ip];
  if (P.prod_idx < 0) return TDWP_EINVAL;   // no product line: a J > 0 unit
  if (!P.set || P.photo) return TDWP_ESTATE;
  const int npg = p->cfg.prod_n_gamma, npr = p->cfg.prod_n_r, np = p->prod_np;
  for (int f = 0; f < n_ch; ++f)
    if (ch[f].elec < 0 || ch[f].elec >= p->ne || ch[f].j < 0 || ch[f].j > npg - 1 || ch[f].omega != 0)
      return TDWP_EINVAL;
  TRY(finish_slices(p, nullptr));
  TRY(flush_ring(p));
  const tdwp_config& c = p->cfg;
  const int nE = c.n_energy;
  const size_t w = (size_t)p->ne * np;
  const size_t col0 = 2 * (size_t)P.n_sv + P.n_w;
  std::vector<double> A((size_t)2 * nE * w), g(p->nR);
  HIP_TRY(hipMemcpy2DAsync(A.data(), w * sizeof(double), p->d_acc + P.acc_off + col0,
                           (size_t)P.n_slice * sizeof(double), w * sizeof(double), (size_t)2 * nE,
                           hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipMemcpyAsync(g.data(), p->d_g + (size_t)ip * p->nR, p->nR * sizeof(double),
                         hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  const double step = (c.ecol_max - c.ecol_min) / (nE - 1);
  std::vector<double> K0(nE), g2(nE);
  for (int e = 0; e < nE; ++e) {
    K0[e] = std::sqrt(2.0 * p->mu * (c.ecol_min + e * step));
    double gr = 0.0, gi = 0.0;
    for (int m = 0; m < p->nR; ++m) {
      const double a = std::sqrt(p->dR) * g[m], Rm = c.R_min + m * p->dR;
      gr += a * std::cos(K0[e] * Rm);
      gi += a * std::sin(K0[e] * Rm);
    }
    g2[e] = gr * gr + gi * gi;
  }
  for (int f = 0; f < n_ch; ++f) {
    // the channel's product-line weights: Legendre row of j times chi (Eq. final-states)
    std::vector<double> wf(np);
    for (int n = 0; n < npg; ++n)
      for (int i = 0; i < npr; ++i)
        wf[(size_t)n * npr + i] = p->prod_P[(size_t)ch[f].j * npg + n] * chi[(size_t)f * npr + i];
    const size_t off = (size_t)ch[f].elec * np;
    for (int e = 0; e < nE; ++e) {
      double re = 0.0, im = 0.0;
      const double* ar = A.data() + (size_t)e * w + off;
      const double* ai = A.data() + (size_t)(nE + e) * w + off;
      for (int q = 0; q < np; ++q) {
        re += wf[q] * ar[q];
        im += wf[q] * ai[q];
      }
      const double Ef = c.ecol_min + e * step + P.pk.E_v0j0 - ch[f].energy;
      double prob = 0.0;
      if (Ef > 0) {
        const double Kf = std::sqrt(2.0 * p->prod_mu * Ef);
        prob = K0[e] * Kf * (re * re + im * im) / (p->mu * p->prod_mu * g2[e]);
      }
      p_prod[(size_t)f * nE + e] = prob;
    }
  }
  return TDWP_OK;
}

void tdwp_destroy(tdwp_plan_t p) { free_plan(p); }

const char* tdwp_strerror(int code) {
  switch (code) {
    case TDWP_OK: return "ok";
    case TDWP_EINVAL: return "invalid argument";
    case TDWP_ENOMEM: return "out of device memory or plan too large";
    case TDWP_EDEVICE: return "HIP device error";
    case TDWP_ESTATE: return "call out of order";
    case TDWP_ERANGE: return "packet norm diverged (spectral bounds too narrow)";
    case TDWP_ESCRATCH: return "input larger than the fixed scratch area of a no-allocation call";
    default: return "unknown error";
  }
}

}  // extern "C"
