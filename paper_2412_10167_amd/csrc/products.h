// Host side of the product-arrangement analysis (products.cpp).
#pragma once

struct tdwp_plan_s;

namespace tdwp {

// Product grid, channel Hamiltonian pieces and the interpolation tables of the
// product line (no-op without a product arrangement).  Errors: EINVAL.
int build_product_tables(tdwp_plan_s* P);

// Lowest n_states eigenpairs of the XY diatomic Hamiltonian on the product grid.
int product_channels(const tdwp_plan_s* P, const double* v_asym, int j, int n_states,
                     double* energies, double* chi);

}  // namespace tdwp
