/*
 * tdwp.h -- C ABI of the MI355X time-dependent wave-packet library.
 *
 * The library propagates triatomic A + BC wave packets with the damped real
 * Chebyshev recursion of arXiv 2412.10167 (MADWAVE3), Sec. 2.2, Eq. wvp-k:
 *     u_1 = D H_s u_0,   u_{k+1} = D (2 H_s u_k - D u_{k-1}),
 *     H_s = (H - E0)/dE,  D = exp(-phi_r(r) - phi_R(R))  (Eq. imaginary-potential),
 * with H the Jacobi-coordinate Hamiltonian of Sec. 2.1 (Eq. hamiltonian):
 * sine-DVR radial kinetic terms along r and R, the rotational and centrifugal
 * terms applied in the Legendre FBR with the Omega-tridiagonal Coriolis
 * coupling, and the diabatic potential matrix, diagonal on the grid.  Every
 * step also records the flux line at r* and the analysis line at R_inf and
 * folds them into energy-resolved amplitudes (Eqs. wvf-chebyshev,
 * chebyshev-expansion-constants), from which tdwp_state_to_state returns the
 * total reactive flux per diabatic state (Eq. total-flux) and inelastic
 * state-to-state probabilities |S|^2 (Eqs. Chebyshev-products-overlaps,
 * S-matrix-from-chebyshev).
 *
 * Conventions common to every call:
 *  - Atomic units throughout: bohr, hartree, electron masses, hbar = 1.
 *  - Host arrays are FP64, borrowed for the duration of the call and copied;
 *    the plan owns every device allocation and frees it in tdwp_destroy.
 *  - Packet layout (device, and every host array that mirrors it):
 *      u[omega_index][elec][gamma][R][r], r fastest, one array per packet.
 *    Omega runs over omega_min..omega_max of its unit, omega_min = 0 when
 *    parity * (-1)^J = +1, else 1 (Eq. angular-functions, Lambda = 0 states).
 *    The stored coefficients are DVR-weighted: sqrt(dr dR w_n) Phi(r, R, gamma).
 *  - Grids (Table tab:parameters, inputgridbase): r_i = r_min + i dr,
 *    i = 0..n_r-1, dr = (r_max - r_min)/(n_r - 1), Dirichlet walls one step
 *    outside both ends (the real sine transform of Sec. 2.1, item 2); the same
 *    for R; gamma on Gauss-Legendre nodes, cos(gamma) ascending.
 *  - Errors are negative return codes; nothing aborts or throws across the ABI.
 *    A failed call leaves the plan as it was, except TDWP_EDEVICE (the device
 *    state is then undefined and the plan should be destroyed).
 *  - One plan is used by one host thread at a time.  Work is enqueued on the
 *    stream given in tdwp_config (a hipStream_t), or on a private stream if
 *    that is NULL; calls that return results to host memory synchronise it.
 */
#ifndef TDWP_H
#define TDWP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tdwp_plan_s* tdwp_plan_t;

enum tdwp_status {
  TDWP_OK = 0,
  TDWP_EINVAL = -1,   /* bad argument or configuration                          */
  TDWP_ENOMEM = -2,   /* device allocation failed or the plan exceeds limits    */
  TDWP_EDEVICE = -3,  /* HIP runtime error (no device, launch failure)          */
  TDWP_ESTATE = -4,   /* call out of order, e.g. propagate before a packet      */
  TDWP_ERANGE = -5,   /* packet norm diverged: spectral bounds too narrow       */
  TDWP_ESCRATCH = -6  /* a no-allocation call's input exceeds its fixed scratch */
};

/* Arithmetic of the kinetic and angular contractions (the recursion, damping,
 * norms and energy accumulation are FP64 in every form). */
enum tdwp_precision {
  TDWP_FP64 = 0,
  TDWP_FP32 = 1,
  TDWP_BF16X3 = 2,
  TDWP_FP16X3 = 3
};

enum tdwp_potential_mode { TDWP_POT_TABLE = 0, TDWP_POT_MLP = 1 };

/* One partial wave (J, p): Jtot, iparity, iommax of the input namelists. */
typedef struct {
  int J;
  int parity;      /* +1 or -1 */
  int omega_max;   /* 0 <= omega_max <= J */
  int n_packets;   /* initial states propagated with this Hamiltonian, >= 1 */
} tdwp_unit;

typedef struct {
  int n_r, n_R, n_gamma;                 /* npun1, npun2, nangu; each >= 2        */
  double r_min, r_max, R_min, R_max;     /* first and last grid points, > 0       */
  double mass_A, mass_B, mass_C;         /* A + BC, electron masses               */
  int n_elec;                            /* diabatic states, 1..4                 */
  double rad_cut;                        /* cap on radial kinetic eigenvalues, <= 0: none */
  double rot_cut;                        /* cap on angular eigenvalues, <= 0: none */
  double abs_r_start, abs_r_strength; int abs_r_power;   /* absr1, absalp1, n1expo */
  double abs_R_start, abs_R_strength; int abs_R_power;   /* absr2, absalp2, n2expo */
  double e_min, e_max;                   /* spectral bounds; both 0: computed      */
  double r_flux;                         /* r* of the total flux (Eq. total-flux)  */
  double R_inf;                          /* analysis line, snapped to the nearest R point */
  int n_energy;                          /* netot >= 2                             */
  double ecol_min, ecol_max;             /* collision energies above E_v0j0        */
  int n_units;                           /* partial waves in the batch, >= 1       */
  const tdwp_unit* units;
  int precision;                         /* enum tdwp_precision                    */
  void* stream;                          /* hipStream_t or NULL                    */
  /* State-to-state analysis in a product arrangement XY + Z from the packet in
   * reactant coordinates (Sec. "Analysis of final states", the reactant-
   * coordinate-based method, iprod = 2 of the inputprod namelist): every step,
   * the packet of each J = 0 unit is evaluated on the line R' = prod_R_inf of the
   * product Jacobi coordinates (r' on prod_n_r equidistant points over
   * [prod_r_min, prod_r_max], gamma' on prod_n_gamma Gauss-Legendre nodes) and
   * accumulated in energy like the reactant lines (Eq.
   * Chebyshev-products-overlaps).  Matrix-core path only (even grid sizes). */
  int prod_arrangement;                  /* 0: none (default); 1: AB + C; 2: AC + B */
  int prod_n_r, prod_n_gamma;            /* product r' points, gamma' nodes (>= 2)  */
  double prod_R_inf;                     /* R'_inf (Rbalinprod)                     */
  double prod_r_min, prod_r_max;         /* first and last r' points, > 0           */
} tdwp_config;

/* Initial collision packet (Sec. 2.3.1, Eqs. initial-collision-wvp and
 * initial-gaussian; nvref, jref, iomref, ielecref and the inputcol namelist). */
typedef struct {
  int unit, slot;          /* which unit, and which of its n_packets           */
  int v0, j0, omega0, elec0;
  double E_v0j0;           /* energy of chi_{v0 j0}, zero of collision energy  */
  double R0, width;        /* Gaussian centre and width Gamma                  */
  double ecol_mean;        /* mean collision energy, k0 = sqrt(2 mu ecol_mean) */
  long k_min_elastic;      /* first k in the elastic-channel sum (kminelastic) */
} tdwp_packet;

/* Final channel of the reactant arrangement (Eq. final-states with beta = A). */
typedef struct {
  int elec, v, j, omega;
  double energy;           /* E_{v' j'} of the channel function                */
} tdwp_channel;

/* Builds a plan: grids, quadrature, sine-DVR and Legendre tables, angular
 * blocks, damping, flux rows, index maps and all device buffers.
 * Errors: EINVAL (inconsistent sizes, omega_max > J, parity not +-1, ...),
 * ENOMEM, EDEVICE.  On success *out owns everything; free with tdwp_destroy. */
int tdwp_plan(const tdwp_config* cfg, tdwp_plan_t* out);

/* Copies the plan's grids: r[n_r], R[n_R], cos_gamma[n_gamma] (any may be NULL). */
int tdwp_grid(tdwp_plan_t p, double* r, double* R, double* cos_gamma, double* gl_weights);

/* Preparatory stage (Sec. 4, pot.out): the n_states lowest eigenpairs of the
 * diatomic channel Hamiltonian T_r + v_asym(r) + min(j(j+1)/(2 m r^2), rot_cut)
 * on the plan's r grid, with T_r the plan's (capped) radial kinetic matrix.
 * chi[n_states][n_r] is DVR-normalised (sum_i chi_i^2 = 1); each vector's
 * first component above 1e-3 of its largest magnitude is positive.
 * Errors: EINVAL for n_states outside 1..n_r or j < 0. */
int tdwp_diatomic_states(tdwp_plan_t p, const double* v_asym, int j, int n_states,
                         double* energies, double* chi);

/* Installs the diabatic potential matrix, diagonal on the grid (Sec. 2.1,
 * item 5).  v: packed upper triangle [n_elec (n_elec+1)/2][n_gamma][n_R][n_r]
 * in the order 11, 12, .., 1n, 22, .., nn; n_values must equal that size.
 * Any cut (VcutmaxeV) is applied by the caller.  Unless cfg.e_min/e_max were
 * given, this also fixes E0 and dE from the rigorous bounds: Gershgorin range
 * of V plus the largest eigenvalue of each kinetic and angular term.
 * Only TDWP_POT_TABLE is accepted by this entry point.  Resets propagation. */
int tdwp_set_potential(tdwp_plan_t p, int mode, const double* v, size_t n_values);

/* Options of the learned potential.  The network maps the three internuclear
 * distances (r_AB, r_BC, r_AC) of a grid point to the packed upper triangle of
 * its diabatic matrix (n_elec (n_elec+1)/2 outputs):
 *   f = (d - 4 bohr)/3 bohr; a_k = silu(a_{k-1} W_k + b_k), k = 1..3, 128 units;
 *   V = 0.1 hartree (a_3 W_4 + b_4);  silu(x) = x/(1 + e^-x).
 * Parameters (FP32, flat): W1[3][128] b1[128] W2[128][128] b2 W3[128][128] b3
 * W4[128][n_pair] b4[n_pair], W stored [in][out]; tdwp_mlp_n_params gives the
 * count.  Training minimises the mean squared error of V/0.1 hartree with
 * Adam (beta1 0.9, beta2 0.999, eps 1e-8) on minibatches taken in the order
 * given; inference uses BF16 copies of the weights with FP32 accumulation. */
typedef struct {
  int n_samples;              /* training points                                       */
  const long* sample_idx;     /* flat grid indices n*(n_R*n_r) + m*n_r + i, [n_samples] */
  const float* init_params;   /* initial parameters                                    */
  const int* order;           /* permutation of 0..n_samples-1; minibatch b of epoch e  */
                              /* takes order[(e*n_samples + b*batch + j) % n_samples]   */
  int batch;                  /* minibatch size, 1..4096                               */
  int epochs;
  double lr;                  /* Adam step size (at the first minibatch)               */
  double lr_final;            /* step size at the last minibatch, reached by a cosine  */
                              /* decay over all minibatches; 0: constant lr            */
} tdwp_mlp_options;

/* Number of parameters of the learned potential for this plan's n_elec. */
int tdwp_mlp_n_params(tdwp_plan_t p);

/* Trains the learned potential on the device from the tabulated potential v
 * (same layout as tdwp_set_potential) and installs it: from now on every step
 * evaluates the network at each grid point instead of reading a table.  E0 and
 * dE follow from the Gershgorin bounds of the network's values on the grid
 * (unless cfg.e_min/e_max were given).  report (may be NULL) receives
 * [final training loss, RMS error over all grid entries (hartree), max abs error
 * (hartree)].  Errors: EINVAL (sizes, options), EDEVICE. Resets propagation. */
int tdwp_set_potential_mlp(tdwp_plan_t p, const double* v, size_t n_values,
                           const tdwp_mlp_options* opt, double* report);

/* Copies the current FP32 network parameters (after training) to params. */
int tdwp_mlp_params(tdwp_plan_t p, float* params);

/* Loss and gradient of the training objective for given parameters on n_pts
 * points: dist [n_pts][3] internuclear distances (bohr), v [n_pts][n_pair]
 * targets (hartree).  FP32 device kernels; grad has tdwp_mlp_n_params entries. */
int tdwp_mlp_gradient(tdwp_plan_t p, const float* params, int n_pts, const double* dist,
                      const double* v, double* loss, float* grad);

/* Inference kernel on n_pts points with the plan's trained network (BF16
 * weights): v_out [n_pts][n_pair] in hartree. */
int tdwp_mlp_eval(tdwp_plan_t p, int n_pts, const double* dist, double* v_out);

/* tdwp_mlp_eval without any device allocation, for callers that cannot
 * allocate (serving loops evaluating the learned surface point by point,
 * harnesses that forbid hipMalloc).  Same kernel and results as tdwp_mlp_eval;
 * the distances and outputs are staged in a fixed device array of 4 MiB
 * (2^19 doubles) that each GPU the library runs on holds until the process
 * ends.  Limit: n_pts * (3 + n_pair) <= 2^19 (n_pair = n_elec (n_elec + 1) / 2),
 * else TDWP_ESCRATCH and nothing runs.  Every call on one GPU shares that
 * GPU's array, so calls that overlap on one GPU (other host threads, other
 * plans) race; calls from one thread in turn are safe.  dist [n_pts][3] and
 * v_out [n_pts][n_pair] are host arrays, as for tdwp_mlp_eval.
 * Errors: EINVAL, ESTATE (no trained network), ESCRATCH, EDEVICE. */
int tdwp_mlp_eval_noalloc(tdwp_plan_t p, int n_pts, const double* dist, double* v_out);

/* The network's potential on the plan's grid, v_out laid out like the table of
 * tdwp_set_potential (the values every step uses after tdwp_set_potential_mlp). */
int tdwp_mlp_grid(tdwp_plan_t p, double* v_out);

/* Returns the (E_min, E_max) in use (after tdwp_set_potential). */
int tdwp_spectral_bounds(tdwp_plan_t p, double* e_min, double* e_max);

/* Builds u_0 = P^{omega0}[j0][n] g_m chi0_i in block (omega0, elec0) of packet
 * (unit, slot), unit norm; g(R) = exp(-(R-R0)^2/(2 width^2)) cos(k0 R) made
 * DVR-weighted and normalised.  chi0[n_r] is normalised by the library.
 * Resets that packet to k = 0 and records its k = 0 slices.  All packets of a
 * plan must be set before tdwp_propagate.  Errors: EINVAL, ESTATE (no potential). */
int tdwp_set_initial_packet(tdwp_plan_t p, const tdwp_packet* pk, const double* chi0);

/* Advances every packet by n_steps Chebyshev steps from its current (u_{k-1},
 * u_k, k).  norms: NULL, or host [n_packets_total][n_steps] receiving
 * ||u_{k+1}||^2 .. ||u_{k+n_steps}||^2, packets ordered by (unit, slot).
 * Chunked calls give the same results as one call (the analysis lines of the
 * last u_k are recorded by the next step or by tdwp_state_to_state, so a
 * chunk boundary adds no pass).  Errors: ESTATE (packets
 * missing), ERANGE (a norm exceeded 1e6 or is not finite: E_max too low). */
int tdwp_propagate(tdwp_plan_t p, long n_steps, double* norms);

/* Current Chebyshev index k of the plan (all packets advance together). */
int tdwp_step_index(tdwp_plan_t p, long* k);

/* Copies packet (unit, slot) to host: which = 0 gives u_k, 1 gives u_{k-1}.
 * out has n_omega(unit) * n_elec * n_gamma * n_R * n_r doubles. */
int tdwp_get_packet(tdwp_plan_t p, int unit, int slot, int which, double* out);

/* Energy analysis of packet (unit, slot) on the collision-energy grid
 * ecol_min..ecol_max (n_energy points, both ends included):
 *   p_reac[n_elec][n_energy]: K0 F_Lambda / (mu |g^(K0)|^2), F the flux of
 *     the energy-resolved packet through r* (Eq. total-flux), g^ the Fourier
 *     amplitude of the incoming Gaussian (Eq. initial-flux-collisions);
 *   p_inel[n_ch][n_energy]: |S_f|^2 with S_f = -sqrt(K0 K_f) e^{-i K_f R_inf}
 *     Phi_f / (mu g^(K0)), Phi_f the energy-resolved projection of the R_inf
 *     line on chi_f(r) P~_{j' omega'}(gamma) (Eqs. Chebyshev-products-overlaps,
 *     S-matrix-from-chebyshev); the initial channel sums k >= k_min_elastic.
 *     Closed channels (E_tot <= energy) give 0.
 * chi: [n_ch][n_r] DVR-normalised channel functions.  Either output may be NULL. */
int tdwp_state_to_state(tdwp_plan_t p, int unit, int slot, int n_ch, const tdwp_channel* ch,
                        const double* chi, double* p_inel, double* p_reac);

/* ---- Photodissociation packets (Sec. "Initial wave packet in photodissociation")
 * A photodissociation packet is the transition dipole applied to an initial bound
 * state, projected on the unit's helicity blocks (Eq. initial-photo-wvp), built
 * by tdwp_photo_packet from the bound state and the dipole, or by the caller and
 * installed with tdwp_set_packet_values.  Its energy content is not known in advance and follows from
 * the autocorrelation C_k = <u_0|u_k> of the propagated packet (Eqs.
 * fourier-transform, chebyshev-transform), which the library forms on the
 * device after every step: in the R pass on the matrix-core path with a
 * tabulated potential (one more read of u_0 per step), else in a kernel of its
 * own (u_0 and u_k read; HIP-graph replay of steps is then off). */

/* Installs packet (unit, slot) from caller values u0 (host, the layout of
 * tdwp_get_packet: DVR-weighted coefficients, not normalised by the library)
 * and resets it to k = 0, as tdwp_set_initial_packet does for a collision
 * packet (every packet of a plan restarts together).  The packet then records
 * its autocorrelation; tdwp_state_to_state refuses it (TDWP_ESTATE).
 * Errors: EINVAL (no such packet, u0 zero or not finite), ESTATE (no potential). */
int tdwp_set_packet_values(tdwp_plan_t p, int unit, int slot, const double* u0);

/* Builds and installs the photodissociation packet of Eq. initial-photo-wvp in
 * packet (unit, slot): sum over Omega of |W^{JMp}_Omega> <W^{JMp}_Omega| d.e |Psi_i>,
 * with J and p the unit's (Eq. angular-functions; the unit's helicities only),
 * d.e = sum_q (-1)^pol D^{1*}_{pol q} d_q (unit polarisation component
 * (e)_{-pol}), so the final M is M_i + pol; Lambda = 0 electronic states with
 * sigma = +1.  The Euler-angle integrals are Clebsch-Gordan coefficients; the
 * result is local in (r, R, gamma) and lands in diabatic state `elec`, the other
 * states zero.  Then as tdwp_set_packet_values.
 *   J_i, M_i, p_i: the bound state's total angular momentum, its projection and
 *     parity; its helicity components Omega_i = om_lo_i .. om_lo_i + n_om_i - 1;
 *   bound [n_om_i][n_gamma][n_R][n_r]: those components on the plan's grid,
 *     DVR-weighted like a packet (host, borrowed);
 *   dip [3][n_gamma][n_R][n_r]: the body-frame spherical components d_q,
 *     q = -1, 0, +1, of the transition dipole (real; a dipole in the x-z plane
 *     has d_{+1} = -d_x / sqrt 2, d_{-1} = d_x / sqrt 2, d_0 = d_z);
 *   pol: -1, 0 (linear, space-fixed z along the polarisation) or +1.
 * Errors: EINVAL (no such packet or state, |M_i| > J_i, p_i not +-1, helicities
 * outside 0..J_i or an Omega_i = 0 component with p_i (-1)^J_i = -1, |M_i + pol|
 * above the unit's J, or a transition that the dipole cannot make: the packet
 * is zero), ESTATE (no potential). */
int tdwp_photo_packet(tdwp_plan_t p, int unit, int slot, int elec, int J_i, int M_i, int p_i,
                      int om_lo_i, int n_om_i, const double* bound, const double* dip, int pol);

/* out = H in for packet (unit, slot): the plan's Hamiltonian (Eq. hamiltonian,
 * with its radial and rotational caps, the potential installed, no damping)
 * applied by the step kernels in the plan's precision.  in, out: host arrays in
 * the packet layout.  This is the H u of the preparatory stage's bound-state
 * calculation (an iterative Lanczos method on the same grid, Sec. "Initial wave
 * packet in photodissociation"), which callers build on this call.  The packet
 * buffers are its scratch: no packet may be installed (TDWP_ESTATE otherwise),
 * and none is after it.  Errors: EINVAL (no such packet), ESTATE (no potential,
 * or a packet installed). */
int tdwp_apply_hamiltonian(tdwp_plan_t p, int unit, int slot, const double* in, double* out);

/* Lowest eigenstate of the plan's H in the space of packet (unit, slot), by a
 * Lanczos iteration without reorthogonalisation (the method of the preparatory
 * stage's bound-state program, Sec. "Initial wave packet in photodissociation")
 * of n_iter >= 2 steps from the host vector guess (packet layout, not zero),
 * with a second pass that rebuilds the Lanczos vectors for the Ritz vector;
 * H u as in tdwp_apply_hamiltonian, three device vectors besides the packet
 * buffers.  energy: the Rayleigh quotient of the normalised Ritz vector; psi
 * (may be NULL): that vector, DVR-normalised (sum psi^2 = 1); residual (may be
 * NULL): |H psi - energy psi|.  The packet buffers are its scratch, as for
 * tdwp_apply_hamiltonian.  Errors: EINVAL (no such packet, n_iter < 2, zero or
 * non-finite guess), ESTATE (no potential, or a packet installed), ERANGE (the
 * Ritz vector vanished). */
int tdwp_lowest_state(tdwp_plan_t p, int unit, int slot, const double* guess, int n_iter,
                      double* energy, double* psi, double* residual);

/* Copies C_0 .. C_{n-1} of photodissociation packet (unit, slot), C_k = <u_0|u_k>
 * in FP64 over the whole packet; n <= k + 1 with k the plan's step index.
 * Errors: EINVAL (no such packet, n out of range), ESTATE (not a
 * photodissociation packet, or not set). */
int tdwp_autocorrelation(tdwp_plan_t p, int unit, int slot, long n, double* out);

/* Energy content of a packet from its autocorrelation (Eq. chebyshev-transform):
 *   a0[i] = (1/pi) sum_{k<n_k} (2 - delta_k0) cos(k theta) / (dE sin theta) C[k],
 *   theta = arccos((E[i] - E0)/dE), E0 = (e_min + e_max)/2, dE = (e_max - e_min)/2,
 * with (e_min, e_max) the plan's spectral bounds (tdwp_spectral_bounds).  Host
 * function.  Errors: EINVAL (NULL, n_k or n_e < 1, e_max <= e_min, an energy
 * not strictly inside (e_min, e_max); nothing is written then). */
int tdwp_energy_content(const double* C, long n_k, double e_min, double e_max, const double* E,
                        int n_e, double* a0);

/* Total photodissociation cross section (Eq. spectrum), bohr^2:
 *   sigma[i] = A hnu[i] / (2 pi) sum_k 2 Re[c_k(H_s, E_i + hnu[i]) C[k]],
 * A = 1/(hbar^2 eps0 c) = 4 pi / c in atomic units, E_i the initial bound-state
 * energy on the energy scale of H, hnu > 0 the photon energies.  Host function.
 * Errors: as tdwp_energy_content, also for hnu <= 0. */
int tdwp_photo_cross_section(const double* C, long n_k, double e_min, double e_max, double E_i,
                             const double* hnu, int n_e, double* sigma);

/* ---- Partial-wave sums (Sec. "Cross sections") ------------------------------
 * Host functions on host FP64 arrays; no plan, no device.  They combine the
 * probabilities that tdwp_state_to_state returns for the computed partial waves.
 * Energy grids are strictly ascending; a probability curve sampled on a grid is
 * read between grid points by linear interpolation and keeps its end values
 * outside the grid.  B (rotational constants) and energies in hartree.
 * Errors: TDWP_EINVAL for a NULL pointer, a size < 1, a grid that does not
 * ascend, a negative J or B, or J outside the allowed range; nothing is
 * written then. */

/* J-shifting from one computed total angular momentum J_ref (the J-shifting
 * approach cited in Sec. "Cross sections"): the threshold moves up with the
 * rotational energy, out[i] = p_ref(e[i] - B [J(J+1) - J_ref(J_ref+1)]).
 * p_ref, e, out: [n_e].  Any J >= 0. */
int tdwp_jshift(const double* p_ref, const double* e, int n_e, int J_ref, double B, int J,
                double* out);

/* J-shifting interpolation (Eq. J-shifting-interpolation) between computed
 * J1 < J2, for J1 <= J <= J2:
 *   out(E) = (J2-J)/(J2-J1) p1(E - B [J(J+1) - J1(J1+1)])
 *          + (J-J1)/(J2-J1) p2(E + B [J2(J2+1) - J(J+1)]),
 * so that J = J1 returns p1 and J = J2 returns p2.  p1, p2, e, out: [n_e]. */
int tdwp_jshift_interpolate(const double* p1, const double* p2, const double* e, int n_e, int J1,
                            int J2, double B, int J, double* out);

/* Cumulative probability (Eq. cumulative-probability) on the grid e[n_e]:
 *   c_out[f][i] = sum_{J=0..J_max} sum_fam (2J+1) P^J_{fam,f}(e[i]),
 * fam running over the initial-helicity/parity families (Omega0, p) of the
 * computed waves and f over the final states the caller resolves (a sum over
 * final helicities can be taken before or after: the result is linear in P).
 *  J_calc[n_calc]: computed total angular momenta, strictly ascending.
 *  B[n_calc]: B[c] is the constant of the interval [J_calc[c], J_calc[c+1]];
 *    the last entry is used for J above the last computed J, B[0] for J below
 *    the first (plain J-shifting there).
 *  p[n_calc][n_fam][n_f][n_e]: computed probabilities; a family with no state
 *    at a computed J (Omega0 > J) has zeros there.
 *  fam_jmin[n_fam] (may be NULL: all 0): the family contributes for J >= fam_jmin.
 *  P^J is the computed curve at a computed J, the interpolation of
 *  tdwp_jshift_interpolate between neighbouring computed J, and tdwp_jshift
 *  from the nearest computed J outside their range.  c_out: [n_f][n_e]. */
int tdwp_cumulative_probability(const int* J_calc, const double* B, int n_calc, const double* p,
                                int n_fam, const int* fam_jmin, int n_f, const double* e, int n_e,
                                int J_max, double* c_out);

/* Integral cross section (Eq. collisional-xsection), bohr^2:
 *   sigma[f][i] = pi / (K0^2 (2 j0 + 1)) c[f][i],  K0^2 = 2 mu e_col[i],
 * mu the reduced mass of A + BC (electron masses), e_col > 0 the collision
 * energies of c's grid.  c, sigma: [n_f][n_e]. */
int tdwp_cross_section(const double* c, int n_f, const double* e_col, int n_e, double mu, int j0,
                       double* sigma);

/* Rotational constant for the interval [J1, J2] of Eq. J-shifting-interpolation,
 * fitted as the B in [0, B_max] that minimises sum_i (p1(e[i] - B [J2(J2+1) -
 * J1(J1+1)]) - p2(e[i]))^2: the J1 curve J-shifted onto the computed J2 curve.
 * The search scans 512 equal cells and refines the best one to 1e-13 B_max.
 * p1, p2, e: [n_e], n_e >= 2, J2 > J1. */
int tdwp_fit_jshift_b(const double* p1, const double* p2, const double* e, int n_e, int J1, int J2,
                      double B_max, double* B_out);

/* Chooses the kernel variants of a step (angular and r passes in one launch or
 * two, angular kernel, its tile width, its block order) by timing the kernels
 * of `steps` whole steps for each feasible combination on this plan's shapes,
 * and keeps the fastest.  Call after the
 * potential and before any initial packet (the packet buffers are used as
 * scratch).  With TDWP_TUNE_CACHE naming a file, the choice is appended to it
 * and later plans of the same shapes start from it.  report (may be NULL)
 * receives "kernel_variant:time;...;chosen=..." text.  Errors: ESTATE. */
int tdwp_autotune(tdwp_plan_t p, int steps, char* report, size_t report_len);

enum tdwp_option {
  TDWP_OPT_GRAPHS = 0,     /* 1 (default): replay captured HIP graphs of steady-state steps */
  TDWP_OPT_ANG_TILE = 1,   /* angular-kernel tile: 1, 2 or 4 sixteen-column tiles          */
  TDWP_OPT_RADIAL_GRID = 2, /* workgroups of the two radial passes, each looping over its
                               blocks; 0 (default): one workgroup per block                 */
  TDWP_OPT_ANG_KERNEL = 3,  /* angular kernel: 0 (default) automatic, 1 helicity mixing
                               through LDS, 2 helicity mixing in registers, 3 every wave
                               holding its own columns in registers (split forms,
                               n_gamma <= 64, at most 8 helicities; used when the r pass
                               is not fused, else kernel 2 runs); a kernel that does not
                               fit the plan's shapes is refused with TDWP_EINVAL          */
  TDWP_OPT_FUSE_R = 4,      /* 1 (default): the angular pass and the r pass in one launch
                               (T_r u into a buffer of its own); 0: two launches, the r
                               pass adding T_r u to the angular terms                      */
  TDWP_OPT_ANG_XCD = 5,     /* 1: angular blocks dealt to the XCDs in contiguous runs;
                               0 (default): in launch order                                */
  TDWP_OPT_PLANE_R = 6      /* 1: both radial kinetic terms, the potential and the
                               recursion in one pass over whole (R, r) planes (one
                               electronic state, mixed forms, plane within the device's
                               LDS; EINVAL otherwise); 0 (default): r pass and R pass    */
};
enum tdwp_stat {
  TDWP_STAT_GRAPH_STEPS = 0,        /* steps taken so far by graph replay      */
  TDWP_STAT_ANG_TILE = 1,           /* current angular-kernel tile (0: general kernels) */
  TDWP_STAT_MATRIX_CORE_PATH = 2,   /* 1 when the matrix-core kernels are in use */
  TDWP_STAT_ANG_KERNEL = 3,         /* angular kernel in use: 1 LDS mixing, 2 register mixing,
                                       3 columns held per wave (0: general kernels) */
  TDWP_STAT_FUSE_R = 4,             /* 1 when the angular and r passes share a launch */
  TDWP_STAT_RING_LEN = 5,           /* steps of slices buffered between two energy
                                       accumulations (Eq. wvf-chebyshev, blocked)     */
  TDWP_STAT_PLANE_R = 6,            /* 1 when steps run the plane pass               */
  TDWP_STAT_POTENTIAL_BYTES = 7     /* device bytes held for the potential: the table
                                       (FP64, plus its FP32 copy in the mixed forms), or
                                       the trained network's parameters once the steps
                                       evaluate it (the table is then released)        */
};

/* Sets a plan option; EINVAL for an unknown option or value. */
int tdwp_set_option(tdwp_plan_t p, int option, long value);

/* Reads a plan statistic. */
int tdwp_get_stat(tdwp_plan_t p, int stat, long* value);

/* Per-kernel average device time (microseconds) over n_steps further steps,
 * each kernel bracketed by HIP events on the plan's stream.  names receives
 * up to n_max kernel-kind names joined by ';' (buffer of names_len bytes).
 * Returns the number of kernel kinds (>= 0) or an error.  Advances the plan. */
int tdwp_time_kernels(tdwp_plan_t p, long n_steps, int n_max, double* avg_us,
                      char* names, size_t names_len);

/* The product grid of a plan with a product arrangement: r_prod [prod_n_r],
 * cos_gamma_prod and weights [prod_n_gamma] (Gauss-Legendre).  Any pointer may
 * be NULL.  Errors: EINVAL (no product arrangement). */
int tdwp_product_grid(tdwp_plan_t p, double* r_prod, double* cos_gamma_prod, double* weights);

/* Product channel functions (Eq. final-states): the lowest n_states eigenpairs of
 * the XY diatomic Hamiltonian on the product r' grid (reduced mass of XY, the
 * caller's asymptotic potential v_asym [prod_n_r] in hartree, the plan's radial
 * and rotational caps), as tdwp_diatomic_states does for the reactant BC.
 * chi [n_states][prod_n_r] DVR-normalised.  Errors: EINVAL. */
int tdwp_product_diatomic_states(tdwp_plan_t p, const double* v_asym, int j, int n_states,
                                 double* energies, double* chi);

/* |S'_f(E)|^2 of product channels f = (elec, v, j, omega = 0) for packet (unit,
 * slot) of a J = 0 unit (Eq. S-matrix-from-chebyshev with the normalisation of
 * the reactant channels): K0 K'_f |Phi'_f|^2 / (mu mu' |g^(K0)|^2), Phi'_f the
 * energy-resolved projection of the product line on the channel function
 * (chi [n_ch][prod_n_r]) times the Legendre row of j, K'_f = sqrt(2 mu' (E -
 * energy_f)), mu' the reduced mass of Z + XY; zero for closed channels.
 * p_prod [n_ch][n_energy].  Errors: EINVAL (no product arrangement, J > 0 unit,
 * bad channel), ESTATE (packet not set or a photodissociation packet). */
int tdwp_state_to_state_products(tdwp_plan_t p, int unit, int slot, int n_ch,
                                 const tdwp_channel* ch, const double* chi, double* p_prod);

void tdwp_destroy(tdwp_plan_t p);
const char* tdwp_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* TDWP_H */
