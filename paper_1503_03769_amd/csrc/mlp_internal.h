// Internal interface between the filter (pphd.hip) and the learned proposal
// (mlp.hip), and the layout of the mixture table they share.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/pphd_mlp.h"

namespace pphd {

// Mixture table: for measurement p and component c, TAB doubles at
// tab[(p*4 + c)*TAB]: log pi_c, cumulative sum of pi over components 0..c,
// log(pi_c) minus the log of the Gaussian's normaliser (so that
// pi_c N(x) = exp(t[2] - |(x - mean) / sigma|^2 / 2)), padding, mean[4],
// sigma[4], 1/sigma[4] (state units, order x, vx, y, vy).
constexpr int MIX_TAB = 16;

// Sets the thread's last-error message and returns s.
pphd_status set_error(pphd_status s, const char* msg);

// Runs the network on M measurements (device double[M][2]) and writes their
// mixture table (device, M*4*MIX_TAB doubles), on stream.
pphd_status mlp_mixture_table(pphd_mlp* h, hipStream_t stream, const double* dz, int M, double* tab);

// Writes the mixture table of given network outputs (device float[M][36]).
pphd_status mlp_head_table(const pphd_model& m, hipStream_t stream, const double* dz, const float* raw, int M,
                           double* tab);

}  // namespace pphd
