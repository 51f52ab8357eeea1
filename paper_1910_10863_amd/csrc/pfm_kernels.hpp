// Kernel launchers of the periodic FMM (implemented in pfm_kernels.hip).
#pragma once
#include "pfm_internal.hpp"

namespace pfm {

bool supported_p(int p);

hipError_t launch_discretise(Problem& pb, double* d_ends);
hipError_t launch_tables(Problem& pb);                 // htab, jtab (per k)
hipError_t launch_lattice_sums(Problem& pb);           // per (k, theta)
hipError_t launch_near_blocks(Problem& pb);            // per (k, theta)
hipError_t launch_rhs(Problem& pb, cd* d_b);
hipError_t launch_fields(Problem& pb, const cd* d_psi, int n_orders, cd* d_out);
hipError_t launch_bessel_test(const double* d_x, int n, double* d_out, hipStream_t s);

// y = (I - A) psi.  When ev != nullptr, events ev[0..6] bracket the stages.
hipError_t apply_operator(Problem& pb, const cd* d_psi, cd* d_y, hipEvent_t* ev);
// the same with the near field in complex64 (FP32 accumulation)
hipError_t apply_operator_mixed(Problem& pb, const cd* d_psi, cd* d_y);
// complex128 near blocks -> complex64 copy
hipError_t launch_near_to_c64(Problem& pb);
// upward pass only (P2M and M2M), for tests
hipError_t apply_upward(Problem& pb, const cd* d_psi);

// GMRES building blocks (deterministic two-stage reductions)
hipError_t launch_dots(Problem& pb, const cd* V, long long ldv, int cnt, const cd* w, int n, cd* d_out);
hipError_t launch_update(Problem& pb, cd* w, const cd* V, long long ldv, int cnt, const cd* d_h, int n);
hipError_t launch_axpby(Problem& pb, cd* y, cd a, const cd* x, cd b, int n);   // y = a x + b y
hipError_t launch_gemv_acc(Problem& pb, cd* x, const cd* V, long long ldv, int cnt, const cd* d_c, int n);

}  // namespace pfm
