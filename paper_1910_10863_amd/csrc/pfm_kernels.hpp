// Kernel launchers of the periodic FMM (implemented in pfm_kernels.hip).
#pragma once
#include "pfm_internal.hpp"

namespace pfm {

bool supported_p(int p);

hipError_t launch_discretise(Problem& pb, double* d_ends);
hipError_t launch_tables(Problem& pb);                 // htab, jtab (per k)
// lattice sums of members 0..B-1 (phase steps pb.d_betas) into their tables
hipError_t launch_lattice_sums(Problem& pb, int B);
// near blocks; phase_free: image phases left out (applied per member by the batched P2P)
hipError_t launch_near_blocks(Problem& pb, bool phase_free);
// per-fibre block preconditioner: coefficients from the circulant rows, and
// out = P^{-1} in (inverse) or P in, for B stacked vectors of 2 M N
hipError_t launch_precond_setup(Problem& pb);
int reduction_blocks(long long n);
hipError_t launch_precond(Problem& pb, const cd* in, cd* out, bool inverse, int B = 1, hipStream_t st = nullptr);
hipError_t launch_rhs(Problem& pb, double theta, cd* d_b);
hipError_t launch_fields(Problem& pb, const cd* d_psi, int n_orders, cd* d_out);
hipError_t launch_bessel_test(const double* d_x, int n, double* d_out, hipStream_t s);

// y = (I - A) psi.  When ev != nullptr, events ev[0..6] bracket the stages.
hipError_t apply_operator(Problem& pb, const cd* d_psi, cd* d_y, hipEvent_t* ev);
// the same with the near-field blocks stored in complex64 (sums in FP64)
hipError_t apply_operator_mixed(Problem& pb, const cd* d_psi, cd* d_y);
// B = pb.B members at once over phase-free near blocks; vectors [B][2E]
hipError_t apply_operator_batch(Problem& pb, const cd* d_psi, cd* d_y, hipEvent_t* ev);
// zero bytes (a multiple of 16) at p on stream s
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
// complex128 near blocks -> complex64 copy
hipError_t launch_near_to_c64(Problem& pb);
// upward pass only (P2M and M2M), for tests
hipError_t apply_upward(Problem& pb, const cd* d_psi);
// one stage of the FMM chain (0 P2M, 1 M2M, 2 M2L, 3 downward pass) launched
// reps times back to back between events e0 and e1
hipError_t time_chain_stage(Problem& pb, const cd* d_psi, int stage, int reps, hipEvent_t e0, hipEvent_t e1);

// GMRES building blocks (deterministic two-stage reductions)
hipError_t launch_dots(Problem& pb, const cd* V, long long ldv, int cnt, const cd* w, int n, cd* d_out);
hipError_t launch_update(Problem& pb, cd* w, const cd* V, long long ldv, int cnt, const cd* d_h, int n);
hipError_t launch_axpby(Problem& pb, cd* y, cd a, const cd* x, cd b, long long n);   // y = a x + b y
// batched forms: B members, member z reads its vectors at base + z * (stride)
hipError_t launch_dots_b(Problem& pb, int B, const cd* V, long long ldv, long long vsb, int cnt, const cd* w,
                         long long wsb, int n, cd* d_out, long long osb);
hipError_t launch_update_b(Problem& pb, int B, cd* w, long long wsb, const cd* V, long long ldv, long long vsb,
                           int cnt, const cd* d_h, long long hsb, int n);
hipError_t launch_gemv_acc_b(Problem& pb, int B, cd* x, long long xsb, const cd* V, long long ldv, long long vsb,
                             int cnt, const cd* d_c, long long csb, int n);
// one CGS2 Arnoldi step of B members (fused: five launches)
hipError_t launch_dcgs_step(Problem& pb, int B, cd* V, long long ldv, long long vsb, int j, cd* W, long long wsb,
                            int n, long long hsb);
hipError_t launch_dcgs_finish(Problem& pb, int B, cd* V, long long ldv, long long vsb, int jl, int n,
                              long long hsb);
hipError_t launch_arnoldi_step(Problem& pb, int B, const cd* V, long long ldv, long long vsb, int j, cd* W,
                               long long wsb, int n, cd* hcol, long long hsb);
// B members: g = v^H c, c -= g v, store g and ||c||^2 (augmented GMRES)
hipError_t launch_project_out(Problem& pb, int B, const cd* v, cd* c, long long wsb, int n, cd* gout, cd* nout,
                              long long hsb);
hipError_t launch_normalize_b(Problem& pb, int B, cd* out, const cd* in, long long sb, const cd* d_nrm,
                              long long nsb, int n);
hipError_t launch_gemv_acc(Problem& pb, cd* x, const cd* V, long long ldv, int cnt, const cd* d_c, int n);

}  // namespace pfm
