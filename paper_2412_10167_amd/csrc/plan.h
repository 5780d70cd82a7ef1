// Internal plan object of the tdwp library.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/tdwp.h"

namespace tdwp {

constexpr int kMaxOmega = 16;     // helicity blocks per unit (omega_max <= 15)
constexpr int kMaxElec = 4;       // diabatic states
constexpr int kRing = 64;         // slices buffered per flush, general accumulation kernel
constexpr int kRingFast = 256;    // slices buffered per flush, matrix-core accumulation
constexpr int kNormChunk = 4096;  // steps of norms held on the device per host read-back

struct UnitInfo {
  int J, parity, om_lo, om_hi, n_om, n_packets;
  // Angular blocks per j: n_omega_j = number of Omega <= j in [om_lo, om_hi];
  // eigenvectors U (n x n, column a = eigenvector a) and eigenvalues ell of l^2.
  std::vector<int> ang_off;   // per j: offset into ang_U (ell offset = ang_off/n? see ell_off)
  std::vector<int> ell_off;   // per j: offset into ang_ell
  std::vector<int> n_om_j;    // per j
  std::vector<double> ang_U, ang_ell;
  double* d_U = nullptr;
  double* d_ell = nullptr;
  // The same blocks padded for the register mixing: every j holds n_om columns b
  // of mix_ld entries a ([j][b][a], identity outside the j's own block) and
  // mix_ld eigenvalues ([j][b], zero outside), in FP64 and FP32.
  // and, per j, the tridiagonal l^2 block itself ([j][2 mix_ld + 2]: diagonal,
  // coupling of Omega and Omega + 1, smallest and largest eigenvalue), in FP64 and FP32.
  std::vector<double> mix_U, mix_ell, mix_L;
  double* d_mixU = nullptr;
  double* d_mixell = nullptr;
  double* d_mixL = nullptr;
  float* d_mixUf = nullptr;
  float* d_mixellf = nullptr;
  float* d_mixLf = nullptr;
  int* d_ang_off = nullptr;
  int* d_ell_off = nullptr;
  int* d_n_om_j = nullptr;
};

struct PacketInfo {
  int unit, slot;
  size_t off;          // offset of this packet in the packet arrays (doubles)
  size_t n_values;
  size_t slice_off;    // offset of this packet's slice vector in a ring row
  int n_sv;            // flux-line values per packet: n_om * n_elec * n_gamma * n_R
  int n_w;             // analysis-line values: n_om * n_elec * n_gamma * n_r
  int n_slice;         // 2 * n_sv + n_w
  size_t acc_off;      // offset of this packet's accumulators [2][n_E][n_slice]
  size_t snap_off;     // offset of the elastic snapshot [2][n_E][n_w]
  int n_p = 0;         // product-line values (n_elec * prod points; J = 0 units), after the R_inf line
  int prod_idx = -1;   // index among the packets with a product line
  size_t wg_off;       // offset of this packet's workgroups in the norm partials
  int n_wg;
  bool set = false;
  bool snap_taken = false;
  tdwp_packet pk{};
  std::vector<double> g;   // DVR-weighted unit-normalised g_m
  // photodissociation packets (installed from caller values): autocorrelation
  bool photo = false;
  int acf_nb = 0;            // workgroups of its partial sums
  size_t acf_part_off = 0;   // offset of its partials within a row of d_acfpart
  int acf_idx = -1;          // its row block in d_acf
  std::vector<double> acf;   // C_0 .. C_k
};

}  // namespace tdwp

// The opaque plan handle of the C ABI.
struct tdwp_plan_s {
  using UnitInfo = tdwp::UnitInfo;
  using PacketInfo = tdwp::PacketInfo;
  tdwp_config cfg{};
  std::vector<tdwp_unit> units_in;
  std::vector<UnitInfo> units;
  std::vector<PacketInfo> packets;
  int nr = 0, nR = 0, ng = 0, ne = 0, npair = 0;
  double mu = 0, m = 0, dr = 0, dR = 0, Lr = 0, LR = 0, r_wall = 0, R_wall = 0;
  std::vector<double> r, R, x, w, Tr, TR, er, eR, Br, BR, D, Dsep, arow, drow;
  std::vector<double> Ptab;   // [omega 0..max_om][j 0..ng-1][n], zero rows for j < omega
  int max_om = 0;
  int m_inf = 0;
  double e_min = 0, e_max = 0, E0 = 0, dE = 0;
  bool bounds_given = false, have_potential = false;
  size_t n_total = 0;        // doubles per packet buffer (all packets)
  size_t slice_total = 0;    // doubles per ring row
  size_t acc_total = 0, snap_total = 0;
  size_t n_wg_total = 0;     // norm partials per step
  int rt_ang = 1;            // r-tile of the angular kernel (general path)
  int rt_rad = 1;            // R-rows per workgroup of the radial kernel (general path)
  // matrix-core path (even n_r, n_R, n_gamma)
  bool fast = false;
  bool fast_accum = false;
  int ntr = 1;               // 16-column tiles per k_radR_epi workgroup
  int nta = 1;               // 16-column tiles per angular workgroup
  int ang_regs = 0;          // angular kernel: 0 k_ang, else k_angr with this many helicities
  long radial_grid = 0;      // workgroups of the two radial passes (0: one per block)
  int ang_pref = 0;          // angular kernel: 0 automatic, 1 k_ang, 2 k_angr
  bool fuse_r = true;        // angular and r passes in one launch (T_r u into d_h2)
  bool ang_xcd = false;      // angular blocks in XCD order
  // angular pass with every wave holding its own columns (k_angw, split forms)
  bool angw_ok = false;      // the shapes and the form allow it
  bool ang_wave = false;     // in use when the r pass is not fused (option / autotuner)
  int* d_blk_angw = nullptr; // workgroups per packet, prefix sums
  int blocks_angw = 0;
  size_t lds_angw = 0;       // the largest unit's tridiagonal blocks (FP32)
  // both radial terms in one pass over whole (R, r) planes (one state, mixed forms)
  bool plane_ok = false;     // the plane fits the device's LDS and the form allows it
  bool plane_r = false;      // in use (option / autotuner)
  int plane_kR = 0, plane_kr = 0;   // padded contraction lengths of the full operator tables
  size_t lds_plane = 0;
  void* d_TRfullF = nullptr;  // T_R [rows][plane_kR], compute format
  void* d_TrfullF = nullptr;  // T_r [rows][plane_kr], compute format
  int* d_blk_plane = nullptr; // planes per packet, prefix sums
  int blocks_plane = 0;
  int* d_n_wg_plane = nullptr;   // norm partials per packet of the plane pass
  // product-arrangement analysis (reactant-coordinate based, J = 0 units)
  int prod_np = 0;                // product points per state: prod_n_r * prod_n_gamma
  double prod_mu = 0, prod_m = 0; // reduced masses of Z + XY and of XY
  double prod_dr = 0, prod_L = 0, prod_wall = 0;
  std::vector<double> prod_r, prod_x, prod_w, prod_T, prod_Br, prod_P;
  std::vector<double> prod_wr, prod_wR, prod_wL, prod_factor;   // interpolation tables
  int prod_kr = 0, prod_kR = 0;   // row pitch of the r and R weight tables (padded to 4)
  int prod_n_pk = 0;              // packets with a product line
  double* d_prod_wr = nullptr;    // [P][prod_kr]  sine-DVR functions of r at the points
  double* d_prod_wR = nullptr;    // [P][prod_kR]  ... of R
  double* d_prod_wL = nullptr;    // [P][n_gamma]  Legendre DVR functions at cos gamma
  double* d_prod_factor = nullptr;// [P] r'R'/(rR) sqrt(dr' w')
  double* d_prod_Z = nullptr;     // [prod_n_pk][n_elec][n_gamma][P] partial contractions
  void* d_prod_desc = nullptr;    // ProdDesc[prod_n_pk]
  int nrhk = 0, nRhk = 0, ngk = 0, ngr = 0;
  size_t lds_radr = 0, lds_ang = 0, lds_radR = 0;
  std::vector<double> Trs, Trd, TRs, TRd, Pc;
  double* d_Trs = nullptr;
  double* d_Trd = nullptr;
  double* d_TRs = nullptr;
  double* d_TRd = nullptr;
  double* d_Pc = nullptr;
  std::vector<double> PcT;
  std::vector<double> Pf;    // [omega][parity][j < ngr][n' < ngk], rows of one parity of j + omega
  std::vector<double> Pb;    // [omega][parity][n < nbr][slot < kbk], back rows in k_angw slot order
  int nbr = 0, kbk = 0;
  // operator tables in the compute format of the plan's precision
  void* d_TrsF = nullptr;
  void* d_TrdF = nullptr;
  void* d_TRsF = nullptr;
  void* d_TRdF = nullptr;
  void* d_PcF = nullptr;
  void* d_PcTF = nullptr;
  void* d_PfF = nullptr;
  void* d_PbF = nullptr;
  // propagation state
  long k = 0;
  int cur = 0;               // u_k lives in d_u[cur], u_{k-1} in d_u[1 - cur]
  int ring_count = 0;
  long rec_k = -1;           // highest Chebyshev index whose slices are recorded
  int ring_len = tdwp::kRing;
  long ring_k0 = 0;
  // device
  int device = -1;           // HIP device current when the plan was made
  hipStream_t stream = nullptr;
  bool own_stream = false;
  double* d_u[2] = {nullptr, nullptr};
  double* d_h = nullptr;
  double* d_h2 = nullptr;    // T_r u when the r pass shares the angular launch
  double* d_V = nullptr;
  double* d_Tr = nullptr;
  double* d_TR = nullptr;
  double* d_P = nullptr;
  double* d_D = nullptr;
  double* d_Dsep = nullptr;   // damping factors [r (n_r), R (n_R)]
  float* d_Vf = nullptr;      // FP32 copy of the potential table (mixed forms)
  double* d_Br = nullptr;
  double* d_BR = nullptr;
  double* d_arow = nullptr;
  double* d_flux_split = nullptr;   // a_s, a_d, d_s, d_d (n_r/2 each)
  double* d_drow = nullptr;
  double* d_ring = nullptr;
  double* d_acc = nullptr;
  double* d_snap = nullptr;
  double* d_coef = nullptr;       // [n_packets][2][n_E][ring_len]
  double* d_normpart = nullptr;   // [kNormChunk][n_wg_total]
  double* d_norms = nullptr;      // [n_packets][kNormChunk]
  double* d_chan = nullptr;       // staging for channel functions
  size_t chan_cap = 0;
  double* d_out = nullptr;        // staging for analysis outputs
  size_t out_cap = 0;
  double* d_u0 = nullptr;         // initial photodissociation packets, packet layout
  size_t u0_cap = 0;
  double* d_acfpart = nullptr;    // [kNormChunk][acf_nb_total] autocorrelation partials
  size_t acfpart_cap = 0;
  double* d_acf = nullptr;        // [n_photo][kNormChunk] summed autocorrelation rows
  size_t acf_cap = 0;
  size_t acf_nb_total = 0;
  int n_photo = 0;
  double* d_acfwg = nullptr;      // [kNormChunk][n_wg_total] overlaps formed by the R pass
  size_t acfwg_cap = 0;
  bool acf_in_pass = false;       // the R pass forms the overlaps (else a kernel of its own)
  double* d_ones = nullptr;       // ones in place of the damping factors (H applied alone)
  size_t ones_cap = 0;
  double* d_lz = nullptr;         // vectors of H u and of the bound-state Lanczos iteration
  size_t lz_cap = 0;
  double* d_dotpart = nullptr;    // partial sums of a dot product, then its sum
  size_t dotpart_cap = 0;
  double* d_g = nullptr;          // [n_packets][n_R]
  // batched-launch index maps (one launch per pass covers every packet)
  void* d_pkdesc = nullptr;       // PkDesc[n_packets]
  int* d_blk_ang = nullptr;       // block prefix sums per packet, k_ang
  int* d_blk_radR = nullptr;      // block prefix sums per packet, k_radR_epi
  void* d_accdesc = nullptr;      // AccDesc[n_packets]
  int* d_blk_acc = nullptr;       // block prefix sums per packet, k_accum_mfma
  long* d_line_start = nullptr;   // first r-line of each packet (n_packets + 1)
  int* d_radr_pk = nullptr;       // packet of the first line of each k_radr workgroup
  unsigned long* d_slice_off = nullptr;
  double* d_E = nullptr;          // E_v0j0 per packet
  int blocks_ang = 0, blocks_radR = 0, blocks_acc = 0;
  size_t lds_ang_max = 0;
  size_t* d_wg_off = nullptr;     // per packet: first norm partial
  int* d_n_wg = nullptr;          // per packet: number of norm partials
  // learned potential
  int pot_mode = 0;               // TDWP_POT_TABLE or TDWP_POT_MLP
  int mlp_nparams = 0;
  float* d_mlp_theta = nullptr;   // FP32 master parameters
  void* d_mlp_w = nullptr;        // packed BF16 weights (w1t, w2t, w3t, w4t)
  float* d_mlp_b = nullptr;       // biases [3*128 + 16]
  double* d_rg = nullptr;         // grids on the device (r, R, cos gamma)
  double* d_Rg = nullptr;
  double* d_xg = nullptr;
  int mlp_grid = 0;               // resident workgroups of the learned-potential pass
  size_t* d_wg_off_mlp = nullptr; // its norm-partial layout (per packet: offset, count)
  int* d_n_wg_mlp = nullptr;
  // device step counters ([0] ring row, [1] norm-partial row) and captured steps
  int* d_counters = nullptr;
  int norm_row = 0;
  bool use_graphs = true;
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};   // two steps, starting from cur = 0 / 1
  hipGraph_t graph[2] = {nullptr, nullptr};
  long graph_steps = 0;        // steps taken by graph replay (diagnostics)
  std::vector<void*> allocations;
};

namespace tdwp {
using Plan = ::tdwp_plan_s;
}  // namespace tdwp
