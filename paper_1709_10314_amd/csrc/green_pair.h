// The Sec. 3 setup for a complex-conjugate pair kappa = alpha +- i beta at order 2 in the basis
// (g, U g) (setup.hip).
#pragma once

#include "smf_internal.h"

namespace smf {

// Green's-function tables of kappa_1 = alpha + i beta into hp / hn (each 2 * n_theta * (m_rows + 1)
// doubles: complex values interleaved), then every factor set from them (as launch_factors_green).
hipError_t launch_green_pair(const Geometry& g, double alpha, double beta, const double* z_dev, int south,
                              double* hp, double* hn, double* f64, float* f32, hipStream_t st);

}  // namespace smf
