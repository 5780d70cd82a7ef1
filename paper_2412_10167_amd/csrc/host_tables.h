// Host-side construction of the plan's tables (quadrature, DVR/FBR matrices,
// angular blocks, channel eigenproblems).  Plain FP64 C++, run once per plan.
#pragma once
#include <vector>

namespace tdwp {

// Gauss-Legendre nodes (ascending) and weights on [-1, 1].
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// Rows j = omega..jmax of sqrt(w_n) * Ptilde_{j omega}(x_n), L2-normalised
// associated Legendre functions without the Condon-Shortley phase.
// out is (jmax - omega + 1) x n, row-major.
void legendre_fbr_rows(int jmax, int omega, const std::vector<double>& x,
                       const std::vector<double>& w, std::vector<double>& out);

// Sine-DVR kinetic matrix S diag(min(k_n^2 / 2M, cap)) S (n x n, row-major),
// k_n = n pi / L, S the orthogonal DST-I matrix; cap <= 0 disables the cap.
// Also returns the (capped) FBR eigenvalues.
void sine_kinetic(int n, double length, double mass, double cap, std::vector<double>& T,
                  std::vector<double>& eig);

// Symmetric eigen-decomposition by cyclic Jacobi rotations.  a is n x n
// row-major (destroyed); on return evals ascending and evecs column k
// (evecs[i*n + k]) the k-th eigenvector.
void jacobi_eigh(int n, std::vector<double>& a, std::vector<double>& evals,
                 std::vector<double>& evecs);

// <J Omega j| l^2 |J Omega' j> over Omega = om_lo..om_hi (om_hi <= j), including
// the sqrt(2) factor between parity-adapted Omega = 0 and 1.
void ell2_block(int J, int j, int om_lo, int om_hi, std::vector<double>& L);

}  // namespace tdwp
