// C ABI of the periodic FM-BEM library (declared in include/pfmbem.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>
#include <map>
#include <cstdint>
#include <array>

#include "pfm_kernels.hpp"

using namespace pfm;


// The fixed device array behind pfm_matvec_static: its per-apply scratch
// (multipole moments, M2L partial expansions and their sums, the lattice
// convolution's spectra, the far part, split P2P partial rows).  Each GPU the
// library runs on holds one copy until the process ends.  In host code the
// name stands for a host-side shadow, never for device memory: the device
// address comes from hipGetSymbolAddress, once per device, at pfm_create.
static __device__ __align__(256) unsigned char scratch[PFM_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
void* g_scratch_addr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up once per device).
hipError_t static_scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

const char* status_name(pfm_status s) {
  switch (s) {
    case PFM_OK: return "ok";
    case PFM_EINVAL: return "invalid argument";
    case PFM_ENOMEM: return "out of memory";
    case PFM_EDEVICE: return "device error";
    case PFM_ENOCONV: return "no convergence";
    case PFM_EWOOD: return "Wood anomaly";
    case PFM_ENUMERIC: return "non-finite value";
    case PFM_ESTATE: return "call order";
  }
  return "?";
}

pfm_status fail(Problem& pb, pfm_status s, const std::string& msg) {
  pb.err = std::string(status_name(s)) + ": " + msg;
  return s;
}

#define HIPCHK(pb, call)                                                                     \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(pb, e_ == hipErrorOutOfMemory ? PFM_ENOMEM : PFM_EDEVICE,                  \
                  std::string(#call) + ": " + hipGetErrorString(e_));                        \
  } while (0)

// Device allocation of plan data and of the library-owned workspace block;
// counted so that callers (and tests) can see that nothing is allocated after
// a workspace is bound.
hipError_t dev_alloc(Problem& pb, void** d, size_t bytes) {
  hipError_t e = hipMalloc(d, bytes);
  if (e == hipSuccess) {
    pb.n_dev_allocs++;
    pb.dev_alloc_bytes += (double)bytes;
  }
  return e;
}

template <typename T>
hipError_t upload(Problem& pb, T** d, const std::vector<T>& h) {
  size_t bytes = std::max<size_t>(1, h.size()) * sizeof(T);
  hipError_t e = dev_alloc(pb, (void**)d, bytes);
  if (e != hipSuccess) return e;
  if (!h.empty()) e = hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

template <typename T>
void dfree(T*& d) {
  if (d) (void)hipFree((void*)d);
  d = nullptr;
}

size_t ws_align(size_t b) { return (b + 255) & ~(size_t)255; }

size_t ws_slot_bytes(const Problem::WsSlot& s, int B) {
  return ws_align(std::max<size_t>(1, s.fixed + (size_t)B * s.per_member));
}

// Register a workspace buffer of fixed + per_member * B bytes (B: batch capacity).
void ws_add(Problem& pb, void* pptr, size_t fixed, size_t per_member, bool zero = false) {
  pb.ws.push_back(Problem::WsSlot{(void**)pptr, fixed, per_member, zero});
}

size_t ws_size(const Problem& pb, int B) {
  size_t t = 0;
  for (const auto& s : pb.ws) t += ws_slot_bytes(s, B);
  return t;
}

// Point every slot into base (ws_size(B) bytes) and clear the slots that must
// start at zero, on stream st.
hipError_t ws_carve(Problem& pb, void* base, int B, hipStream_t st) {
  char* p = (char*)base;
  for (const auto& s : pb.ws) {
    const size_t b = ws_slot_bytes(s, B);
    *s.ptr = p;
    if (s.zero) {
      hipError_t e = hipMemsetAsync(p, 0, b, st);
      if (e != hipSuccess) return e;
    }
    p += b;
  }
  pb.ws_base = base;
  pb.ws_bytes = ws_size(pb, B);
  pb.max_batch = B;
  // the lattice rows follow the explicit M2L rows inside each member's table
  pb.d_lat = pb.d_htab ? pb.d_htab + (pb.hp.off_xy.size() / 2) * (size_t)(4 * pb.opt.p + 1) : nullptr;
  return hipSuccess;
}

void ws_release(Problem& pb) {
  for (const auto& s : pb.ws) *s.ptr = nullptr;
  pb.d_lat = nullptr;
  if (pb.ws_own) (void)hipFree(pb.ws_own);
  pb.ws_own = nullptr;
  pb.ws_base = nullptr;
  pb.ws_bytes = 0;
}

void free_all(Problem& pb) {
  ws_release(pb);
  dfree(pb.d_centres); dfree(pb.d_radii);
  dfree(pb.d_mx); dfree(pb.d_my); dfree(pb.d_tx); dfree(pb.d_ty); dfree(pb.d_h);
  dfree(pb.d_gl); dfree(pb.d_gl16); dfree(pb.d_elem_of); dfree(pb.d_psi_idx);
  dfree(pb.d_e_src); dfree(pb.d_e_off); dfree(pb.d_e_m); dfree(pb.d_chunks); dfree(pb.d_cc_ptr);
  dfree(pb.d_part); dfree(pb.d_epart); dfree(pb.d_mchunks);
  dfree(pb.d_up_cells); dfree(pb.d_up_ptr); dfree(pb.d_up_src); dfree(pb.d_up_off);
  dfree(pb.d_ldesc); dfree(pb.d_lanc); dfree(pb.d_tgeo); dfree(pb.d_trh); dfree(pb.d_far);
  dfree(pb.d_cx); dfree(pb.d_cy); dfree(pb.d_ebeg); dfree(pb.d_eend);
  dfree(pb.d_first_child); dfree(pb.d_n_child); dfree(pb.d_cell_joff); dfree(pb.d_parent);
  dfree(pb.d_leaves); dfree(pb.d_root_of_fibre); dfree(pb.d_fibre_of_cell);
  dfree(pb.d_m2l_ptr); dfree(pb.d_m2l_src); dfree(pb.d_m2l_off); dfree(pb.d_m2l_m);
  dfree(pb.d_m2li_ptr); dfree(pb.d_m2li_src); dfree(pb.d_m2li_off);
  dfree(pb.d_near_ptr); dfree(pb.d_near_src); dfree(pb.d_near_m); dfree(pb.d_near_tgt);
  dfree(pb.d_near_blk); dfree(pb.d_leaf_blk); dfree(pb.d_cols_ptr); dfree(pb.d_col_psi); dfree(pb.d_col_m);
  dfree(pb.d_p2p_items); dfree(pb.d_p2p_rowtasks); dfree(pb.d_p2p_rowoff); dfree(pb.d_leaf_near_t0);
  dfree(pb.d_ccols_ptr); dfree(pb.d_ccol_psi); dfree(pb.d_ccol_loc); dfree(pb.d_cwin); dfree(pb.d_circ);
  dfree(pb.d_pc_fwd); dfree(pb.d_pc_inv); dfree(pb.d_pc_tw); dfree(pb.d_pc_x); dfree(pb.d_kress);
  dfree(pb.d_lat_cell); dfree(pb.d_lat_slot); dfree(pb.d_lat_key); dfree(pb.d_lat_shat); dfree(pb.d_lat_xhat);
  dfree(pb.d_lat_lhat);
  dfree(pb.d_near_uniq); dfree(pb.d_near_cp_src); dfree(pb.d_near_cp_dst); dfree(pb.d_near_cp_len);
  dfree(pb.d_spec_rng); dfree(pb.d_dptr); dfree(pb.d_danc);
  dfree(pb.d_vchunks); dfree(pb.d_mfma_items); dfree(pb.d_mfma_cols);
  dfree(pb.d_mcell); dfree(pb.d_dldesc);
  dfree(pb.d_alpha_one); dfree(pb.d_gin); dfree(pb.d_gout); dfree(pb.d_p2ppart);
  if (pb.graph) (void)hipGraphExecDestroy(pb.graph);
  pb.graph = nullptr;
  if (pb.cap) (void)hipStreamDestroy(pb.cap);
  pb.cap = nullptr;
  dfree(pb.d_root_pair_off); dfree(pb.d_root_mrange);
  dfree(pb.d_off_xy); dfree(pb.d_joff_xy); dfree(pb.d_root_off_xy);
  dfree(pb.d_near); dfree(pb.d_near32); dfree(pb.d_ir_r); dfree(pb.d_ir_d); dfree(pb.d_ir_aug); dfree(pb.d_cperp); dfree(pb.d_htab); dfree(pb.d_jtab); pb.d_lat = nullptr; dfree(pb.d_alpha);
  dfree(pb.d_srule); dfree(pb.d_betas); dfree(pb.d_thetas); dfree(pb.d_latpart);
  dfree(pb.d_mpole);
  dfree(pb.d_V); dfree(pb.d_w); dfree(pb.d_r); dfree(pb.d_b); dfree(pb.d_tmp);
  dfree(pb.d_red); dfree(pb.d_hcol); dfree(pb.d_fields);
  if (pb.h_hcol) (void)hipHostFree(pb.h_hcol);
  pb.h_hcol = nullptr;
  if (pb.h_hall) (void)hipHostFree(pb.h_hall);
  pb.h_hall = nullptr;
  dfree(pb.d_npart); dfree(pb.d_dcoef); dfree(pb.d_hall);
  if (pb.events) {
    for (int i = 0; i < 16; ++i) (void)hipEventDestroy(pb.ev[i]);
    (void)hipEventDestroy(pb.ev_fork);
    (void)hipEventDestroy(pb.ev_join);
  }
  pb.events = false;
  if (pb.side) (void)hipStreamDestroy(pb.side);
  pb.side = nullptr;
}

double wood_distance(double k, double H, double th) {
  double best = 1e300;
  for (int s = -1; s <= 1; s += 2) {
    double v = k * H * (1.0 + s * std::sin(th)) / (2.0 * PI);
    best = std::min(best, std::fabs(v - std::nearbyint(v)));
  }
  return best;
}

// Composite Gauss-Legendre rule in s for the lattice-sum tails: panels
// graded quadratically towards s = 0, where a near-Wood pole of
// 1/(1 - e^{+-i beta - mu H}) sits, up to s_max where the Gaussian factor
// exp(-((q+1)H - |Y|) s^2) has removed the integrand.
constexpr int LAT_RULE_POINTS = 1024;   // points of the lattice tail rule

void tail_rule(double k, double H, double gap, double xmax, int nu_max, std::vector<double>& rule) {
  double smax = 1.0;
  auto logmag = [&](double s) {
    return -gap * s * s + std::sqrt(k) * xmax * s + nu_max * std::log(1.0 + (2.0 * s * s + k) / k);
  };
  while (logmag(smax) > -60.0) smax *= 1.2;
  const int npan = LAT_RULE_POINTS / 16, ng = 16;
  std::vector<double> x, w;
  gauss_legendre(ng, x, w);
  rule.assign(2 * npan * ng, 0.0);
  for (int p = 0; p < npan; ++p) {
    double a = smax * std::pow((double)p / npan, 2.0);
    double b = smax * std::pow((double)(p + 1) / npan, 2.0);
    for (int g = 0; g < ng; ++g) {
      rule[p * ng + g] = 0.5 * (a + b) + 0.5 * (b - a) * x[g];
      rule[npan * ng + p * ng + g] = 0.5 * (b - a) * w[g];
    }
  }
}

}  // namespace

namespace {
// 64-bit FNV-1a over the bytes of values
struct Fnv {
  unsigned long long h = 1469598103934665603ULL;
  template <typename T>
  void add(const T& v) {
    const unsigned char* b = reinterpret_cast<const unsigned char*>(&v);
    for (size_t i = 0; i < sizeof(T); ++i) {
      h ^= b[i];
      h *= 1099511628211ULL;
    }
  }
  template <typename T>
  void vec(const std::vector<T>& v) {
    add(v.size());
    for (const T& x : v) add(x);
  }
};
}  // namespace

extern "C" {

pfm_status pfm_create(const pfm_geometry* geo, const pfm_material* mat, const pfm_options* opt,
                      pfm_problem** out) {
  if (!out) return PFM_EINVAL;
  *out = nullptr;
  pfm_problem* h = new (std::nothrow) pfm_problem();
  if (!h) return PFM_ENOMEM;
  Problem& pb = h->p;
  auto bail = [&](pfm_status s) {
    // keep the handle so that the caller can read the message
    *out = h;
    return s;
  };
  if (!geo || !mat || !opt) return bail(fail(pb, PFM_EINVAL, "null argument"));
  if (geo->lattice != PFM_SQUARE && geo->lattice != PFM_HEXAGON)
    return bail(fail(pb, PFM_EINVAL, "lattice must be square or hexagon"));
  if (!(geo->a > 0) || geo->M_L < 1 || geo->M_H < 1 || geo->n_elem < 8)
    return bail(fail(pb, PFM_EINVAL, "need a > 0, M_L >= 1, M_H >= 1, n_elem >= 8"));
  if ((long long)geo->M_L * geo->M_H * geo->n_elem > (1LL << 26))
    return bail(fail(pb, PFM_EINVAL, "too many elements"));
  if (!supported_p(opt->p)) return bail(fail(pb, PFM_EINVAL, "p must be one of 8,12,16,20,24,32,40"));
  if (opt->leaf_max < 1 || opt->leaf_max > 64) return bail(fail(pb, PFM_EINVAL, "leaf_max must be 1..64"));
  if (!(opt->mac > 0.0 && opt->mac < 1.0)) return bail(fail(pb, PFM_EINVAL, "mac must be in (0,1)"));
  if (opt->g_far < 1 || opt->g_far > 16) return bail(fail(pb, PFM_EINVAL, "g_far must be 1..16"));
  if (opt->restart < 1 || opt->restart > 200 || opt->max_iter < 1 || !(opt->tol > 0))
    return bail(fail(pb, PFM_EINVAL, "restart 1..200, max_iter >= 1, tol > 0"));
  if (opt->store_self_blocks != 0 && opt->store_self_blocks != 1)
    return bail(fail(pb, PFM_EINVAL, "store_self_blocks must be 0 or 1"));
  if (opt->p2p_cached_rows != 0 && opt->p2p_cached_rows != 1)
    return bail(fail(pb, PFM_EINVAL, "p2p_cached_rows must be 0 or 1"));
  if (opt->direct_lattice_m2l != 0 && opt->direct_lattice_m2l != 1)
    return bail(fail(pb, PFM_EINVAL, "direct_lattice_m2l must be 0 or 1"));
  if (opt->precision != PFM_FP64 && opt->precision != PFM_MIXED)
    return bail(fail(pb, PFM_EINVAL, "precision must be PFM_FP64 or PFM_MIXED"));
  if (opt->precond != 0 && opt->precond != 1) return bail(fail(pb, PFM_EINVAL, "precond must be 0 or 1"));
  if (opt->self_mode < 0 || opt->self_mode > 2) return bail(fail(pb, PFM_EINVAL, "self_mode must be 0, 1 or 2"));
  if (opt->tree_on_host != 0 && opt->tree_on_host != 1)
    return bail(fail(pb, PFM_EINVAL, "tree_on_host must be 0 or 1"));
  if (opt->m2l_vector != 0 && opt->m2l_vector != 1)
    return bail(fail(pb, PFM_EINVAL, "m2l_vector must be 0 or 1"));
  if (opt->tree_shape != PFM_TREE_SQUARE && opt->tree_shape != PFM_TREE_TRIANGLE)
    return bail(fail(pb, PFM_EINVAL, "tree_shape must be PFM_TREE_SQUARE or PFM_TREE_TRIANGLE"));
  if (opt->tree_shape == PFM_TREE_TRIANGLE && geo->lattice != PFM_HEXAGON)
    return bail(fail(pb, PFM_EINVAL, "PFM_TREE_TRIANGLE needs the hexagonal lattice"));
  if (opt->discretisation != PFM_CHORDS && opt->discretisation != PFM_NYSTROM)
    return bail(fail(pb, PFM_EINVAL, "discretisation must be PFM_CHORDS or PFM_NYSTROM"));
  if (opt->discretisation == PFM_NYSTROM &&
      (geo->shape != PFM_CIRCLE || geo->n_elem < 8 || geo->n_elem > 512 || (geo->n_elem & (geo->n_elem - 1)) != 0 ||
       opt->self_mode == 1 || opt->store_self_blocks))
    return bail(fail(pb, PFM_EINVAL, "PFM_NYSTROM needs circles, N a power of two in 8..512, self_mode 0 or 2 "
                                     "and store_self_blocks 0"));
  if (opt->precond == 1 && (geo->n_elem < 8 || geo->n_elem > 512 || (geo->n_elem & (geo->n_elem - 1)) != 0))
    return bail(fail(pb, PFM_EINVAL, "precond = 1 needs n_elem a power of two in 8..512"));
  if (opt->max_batch < 0 || opt->max_batch > PFM_MAX_BATCH || (opt->use_graph != 0 && opt->use_graph != 1))
    return bail(fail(pb, PFM_EINVAL, "max_batch must be 0..16 and use_graph 0 or 1"));
  if (opt->p2p_blocks_per_cu < 0 || opt->p2p_blocks_per_cu > 8 ||
      !(opt->p2p_unroll == 0 || opt->p2p_unroll == 1 || opt->p2p_unroll == 2 || opt->p2p_unroll == 4))
    return bail(fail(pb, PFM_EINVAL, "p2p_blocks_per_cu must be 0..8 and p2p_unroll 0, 1, 2 or 4"));
  if (!(mat->rho_fiber > 0 && mat->c_fiber > 0 && mat->rho_matrix > 0 && mat->c_matrix > 0))
    return bail(fail(pb, PFM_EINVAL, "materials must be positive"));

  pb.lattice = geo->lattice;
  pb.a = geo->a;
  pb.ML = geo->M_L;
  pb.MH = geo->M_H;
  pb.M = pb.ML * pb.MH;
  pb.N = geo->n_elem;
  pb.E = pb.M * pb.N;
  pb.opt = *opt;
  if (!(pb.opt.inner_tol > 0 && pb.opt.inner_tol < 1)) pb.opt.inner_tol = 0;   // relaxation point from tol
  pb.max_batch = std::max(1, opt->max_batch);
  pb.max_batch_create = pb.max_batch;
  // Every fibre is a circle cut into N equal chords, so its own image-0 block
  // (both wavenumbers, near and far pairs) is block circulant; with N a power
  // of two it is applied by the FFTs of the preconditioner's transforms.
  pb.self_fft = opt->self_mode != 1 && !opt->store_self_blocks && geo->shape == PFM_CIRCLE && pb.N >= 8 &&
                pb.N <= 512 && (pb.N & (pb.N - 1)) == 0;
  // Nystrom: the point rule at the nodes for every smooth kernel
  pb.nystrom = opt->discretisation == PFM_NYSTROM;
  if (pb.nystrom) pb.opt.g_far = 1;

  pb.rho_f = mat->rho_fiber;
  pb.c_f = mat->c_fiber;
  pb.rho_m = mat->rho_matrix;
  pb.c_m = mat->c_matrix;
  pb.eta_user = mat->eta;
  if (geo->shape != PFM_CIRCLE && geo->shape != PFM_ROUND_SQUARE)
    return bail(fail(pb, PFM_EINVAL, "shape must be PFM_CIRCLE or PFM_ROUND_SQUARE"));
  pb.shape = geo->shape;
  if (pb.shape != PFM_CIRCLE) {
    // the chords of a non-circular fibre are not rotations of each other: no
    // circulant rows, every near pair is a stored block
    if (opt->precond) return bail(fail(pb, PFM_EINVAL, "precond = 1 needs circular fibres"));
    pb.opt.store_self_blocks = 1;
  }
  // farthest point of the boundary curve from the fibre centre, per unit r
  const double reach = pb.shape == PFM_ROUND_SQUARE ? 4.0 : 1.0;
  pb.radii.resize(pb.M);
  for (int f = 0; f < pb.M; ++f) {
    double r = geo->radii ? geo->radii[f] : geo->r0;
    if (!(r > 0) || !(2.0 * reach * r < pb.a))
      return bail(fail(pb, PFM_EINVAL, "fibre size must satisfy 0 < 2 (reach) r < a (fibres may not touch)"));
    pb.radii[f] = r;
  }
  pb.centres.resize(2 * pb.M);
  const double s3 = std::sqrt(3.0) / 2.0;
  for (int j = 0; j < pb.MH; ++j)
    for (int i = 0; i < pb.ML; ++i) {
      int f = j * pb.ML + i;
      if (pb.lattice == PFM_SQUARE) {
        pb.centres[2 * f] = (i + 0.5) * pb.a;
        pb.centres[2 * f + 1] = (j + 0.5) * pb.a;
      } else {
        pb.centres[2 * f] = (i + 0.5) * s3 * pb.a;
        pb.centres[2 * f + 1] = (j + 0.5 + 0.5 * (i % 2)) * pb.a;
      }
    }
  pb.L = pb.lattice == PFM_SQUARE ? pb.ML * pb.a : pb.ML * s3 * pb.a;
  pb.H = pb.MH * pb.a;

  {
    // P2P runs as a persistent grid of a few workgroups per compute unit (set
    // once the near pairs are classified), leaving room on every CU for the
    // concurrent FMM chain
    int dev = 0;
    if (!(hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&pb.n_cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess))
      pb.n_cu = 0;
    pb.device = dev;
    // with the own blocks by FFT the P2P stream is a few leaves of stored
    // blocks, bound by load latency: four columns' loads in flight per wave
    pb.p2p_unroll = opt->p2p_unroll > 0 ? opt->p2p_unroll : (pb.self_fft ? 4 : 1);
    // this device's address of the fixed scratch array of pfm_matvec_static
    hipError_t e = static_scratch_address(dev, &pb.static_scratch);
    if (e != hipSuccess)
      return bail(fail(pb, PFM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)));
  }
  // discretisation on the device
  int E = pb.E;
#define CK(call) do { hipError_t e_ = (call); if (e_ != hipSuccess) { free_all(pb); \
    return bail(fail(pb, e_ == hipErrorOutOfMemory ? PFM_ENOMEM : PFM_EDEVICE, \
                     std::string(#call) + ": " + hipGetErrorString(e_))); } } while (0)
  CK(upload(pb, &pb.d_centres, pb.centres));
  CK(upload(pb, &pb.d_radii, pb.radii));
  CK(dev_alloc(pb, (void**)&pb.d_mx, E * sizeof(double)));
  CK(dev_alloc(pb, (void**)&pb.d_my, E * sizeof(double)));
  CK(dev_alloc(pb, (void**)&pb.d_tx, E * sizeof(double)));
  CK(dev_alloc(pb, (void**)&pb.d_ty, E * sizeof(double)));
  CK(dev_alloc(pb, (void**)&pb.d_h, E * sizeof(double)));
  double* d_ends = nullptr;
  CK(dev_alloc(pb, (void**)&d_ends, 4 * (size_t)E * sizeof(double)));
  CK(launch_discretise(pb, d_ends));
  // quadtrees and interaction lists: GPU kernels, or the host construction
  // (asked for, or where the GPU build does not apply)
  std::vector<double> mx(E), my(E);
  CK(hipMemcpy(mx.data(), pb.d_mx, E * sizeof(double), hipMemcpyDeviceToHost));
  CK(hipMemcpy(my.data(), pb.d_my, E * sizeof(double), hipMemcpyDeviceToHost));
  bool planned = false;
  pb.tree_on_device = false;
  if (!opt->tree_on_host && opt->tree_shape == PFM_TREE_SQUARE) {
    std::string why;
    planned = build_device_plan(pb, pb.d_mx, pb.d_my, d_ends, why);
    pb.tree_on_device = planned;
    if (!planned && why.find("leaf holds more than 64") != std::string::npos) {
      (void)hipFree(d_ends);
      free_all(pb);
      return bail(fail(pb, PFM_EINVAL, "tree construction failed"));
    }
    if (!planned && why.rfind("more than", 0) != 0 && why.rfind("a level", 0) != 0) {
      (void)hipFree(d_ends);
      free_all(pb);
      return bail(fail(pb, PFM_EDEVICE, "GPU tree build: " + why));
    }
  }
  if (!planned) {
    std::vector<double> ends(4 * (size_t)E), mid(2 * (size_t)E);
    CK(hipMemcpy(ends.data(), d_ends, ends.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int e = 0; e < E; ++e) {
      mid[2 * e] = mx[e];
      mid[2 * e + 1] = my[e];
    }
    if (!build_host_plan(pb, mid, ends)) {
      (void)hipFree(d_ends);
      free_all(pb);
      return bail(fail(pb, PFM_EINVAL, "tree construction failed"));
    }
  }
  (void)hipFree(d_ends);
  const HostPlan& hp = pb.hp;
  int nc = (int)hp.cells.size();
  std::vector<double> cx(nc), cy(nc);
  std::vector<int> eb(nc), ee(nc), fc(nc), nch(nc), par(nc), fib(nc);
  for (int i = 0; i < nc; ++i) {
    const Cell& c = hp.cells[i];
    cx[i] = c.cx; cy[i] = c.cy; eb[i] = c.ebeg; ee[i] = c.eend;
    fc[i] = c.first_child; nch[i] = c.n_child; par[i] = c.parent; fib[i] = c.fiber;
  }
  CK(upload(pb, &pb.d_elem_of, hp.elem_of));
  {
    std::vector<int> pidx(E);
    for (int t = 0; t < E; ++t) {
      int e = hp.elem_of[t], f = e / pb.N;
      pidx[t] = 2 * f * pb.N + (e - f * pb.N);
    }
    CK(upload(pb, &pb.d_psi_idx, pidx));
  }
  CK(upload(pb, &pb.d_cx, cx)); CK(upload(pb, &pb.d_cy, cy));
  CK(upload(pb, &pb.d_ebeg, eb)); CK(upload(pb, &pb.d_eend, ee));
  CK(upload(pb, &pb.d_first_child, fc)); CK(upload(pb, &pb.d_n_child, nch));
  CK(upload(pb, &pb.d_parent, par)); CK(upload(pb, &pb.d_fibre_of_cell, fib));

  CK(upload(pb, &pb.d_leaves, hp.leaves));
  CK(upload(pb, &pb.d_root_of_fibre, hp.root_of_fibre));
  CK(upload(pb, &pb.d_m2l_ptr, hp.m2l_ptr)); CK(upload(pb, &pb.d_m2l_src, hp.m2l_src));
  CK(upload(pb, &pb.d_m2l_off, hp.m2l_off)); CK(upload(pb, &pb.d_m2l_m, hp.m2l_m));
  CK(upload(pb, &pb.d_m2li_ptr, hp.m2li_ptr)); CK(upload(pb, &pb.d_m2li_src, hp.m2li_src));
  CK(upload(pb, &pb.d_m2li_off, hp.m2li_off));
  CK(upload(pb, &pb.d_near_ptr, hp.near_ptr)); CK(upload(pb, &pb.d_near_src, hp.near_src));
  CK(upload(pb, &pb.d_near_m, hp.near_m)); CK(upload(pb, &pb.d_near_tgt, hp.near_tgt));
  // Near pairs of one fibre with itself (m = 0) are circulant: the chords of
  // a circle are rotations of each other, so the 2x2 block of target element
  // a and source element b depends only on (b - a) mod N, and one row per
  // fibre (pfm_set_wave fills it) stands for all of them.  The other pairs
  // (another fibre, or an image) keep stored blocks; store_self_blocks = 1
  // stores every pair.
  const int npairs_all = (int)hp.near_src.size();
  std::vector<char> circ(npairs_all, 0);
  long long n_circ_entries = 0;
  for (int q = 0; q < npairs_all; ++q) {
    const Cell& D = hp.cells[hp.leaves[hp.near_tgt[q]]];
    const Cell& C = hp.cells[hp.near_src[q]];
    circ[q] = !pb.opt.store_self_blocks && C.fiber == D.fiber && hp.near_m[q] == 0;
    if (circ[q]) n_circ_entries += (long long)(D.eend - D.ebeg) * (C.eend - C.ebeg);
  }
  pb.n_near_circ = n_circ_entries;
  // with mostly circulant pairs P2P is the short branch of the overlapped apply
  {
    long long stored_entries = 0;
    for (int q = 0; q < npairs_all; ++q)
      if (!circ[q]) {
        const Cell& D = hp.cells[hp.leaves[hp.near_tgt[q]]];
        const Cell& C = hp.cells[hp.near_src[q]];
        stored_entries += (long long)(D.eend - D.ebeg) * (C.eend - C.ebeg);
      }
    // with the self blocks applied by FFT, the FFT apply and the P2P of the
    // remaining stored pairs form the short branch
    pb.p2p_on_side = pb.self_fft || n_circ_entries > stored_entries;
    // default grid: two workgroups per CU stream stored blocks at full HBM
    // rate without starving the chain; the light circulant P2P on the side
    // stream takes four (measured fastest for the overlapped apply)
    if (pb.n_cu > 0)
      pb.p2p_grid = (opt->p2p_blocks_per_cu > 0 ? opt->p2p_blocks_per_cu : (pb.p2p_on_side ? 3 : 2)) * pb.n_cu;
  }
  std::vector<long long> leaf_blk_host;   // per leaf: start of its stored region (entries)
  std::vector<int> near_t0_host;          // per leaf: its first P2P row task (-1: none)
  // near-block storage of the other pairs: per target leaf its stored pairs
  // one after the other; with equal fibres, a region (the stored blocks of one
  // target leaf) is stored once for every leaf that has the same region
  {
    // Equal fibres (same radius, so the same chords and the same tree about
    // each centre): a near block depends only on the two leaves' places in
    // their fibres' trees, on the offset between the fibres and, through the
    // quasi-periodic phase alpha^m, on the image m.
    const int npairs = npairs_all;
    const int nl = (int)hp.leaves.size();
    bool equal = pb.M > 1 && npairs > 0;
    for (int f = 1; f < pb.M && equal; ++f) equal = pb.radii[f] == pb.radii[0];
    std::vector<std::vector<int>> leaves_of(pb.M);
    std::vector<int> local(hp.cells.size(), -1);
    if (equal) {
      for (int li = 0; li < nl; ++li) {
        const Cell& c = hp.cells[hp.leaves[li]];
        local[hp.leaves[li]] = (int)leaves_of[c.fiber].size();
        leaves_of[c.fiber].push_back(hp.leaves[li]);
      }
      for (int f = 1; f < pb.M && equal; ++f) {
        if (leaves_of[f].size() != leaves_of[0].size()) { equal = false; break; }
        for (size_t j = 0; j < leaves_of[f].size() && equal; ++j) {
          const Cell& a = hp.cells[leaves_of[0][j]];
          const Cell& b = hp.cells[leaves_of[f][j]];
          if (std::fabs((a.cx - pb.centres[0]) - (b.cx - pb.centres[2 * f])) > 1e-12 ||
              std::fabs((a.cy - pb.centres[1]) - (b.cy - pb.centres[2 * f + 1])) > 1e-12 ||
              a.eend - a.ebeg != b.eend - b.ebeg) {
            equal = false;
            break;
          }
          for (int t = 0; t < a.eend - a.ebeg; ++t)
            if (hp.elem_of[a.ebeg + t] != hp.elem_of[b.ebeg + t] - f * pb.N) { equal = false; break; }
        }
      }
    }
    std::vector<long long> blk(npairs, 0), leaf_blk(nl, 0);
    std::vector<int> uniq, cp_len;
    std::vector<long long> cp_src, cp_dst;
    long long stored = 0;
    auto pair_len = [&](int q) {
      const Cell& D = hp.cells[hp.leaves[hp.near_tgt[q]]];
      const Cell& C = hp.cells[hp.near_src[q]];
      return (long long)(D.eend - D.ebeg) * (C.eend - C.ebeg);
    };
    if (equal) {
      // key of a pair: (target's place, source's place, offset, image)
      auto pair_key = [&](int q) {
        const Cell& D = hp.cells[hp.leaves[hp.near_tgt[q]]];
        const Cell& C = hp.cells[hp.near_src[q]];
        double ox = pb.centres[2 * C.fiber] - pb.centres[2 * D.fiber];
        double oy = pb.centres[2 * C.fiber + 1] - pb.centres[2 * D.fiber + 1] + hp.near_m[q] * pb.H;
        return std::array<long long, 5>{local[hp.leaves[hp.near_tgt[q]]], local[hp.near_src[q]],
                                        std::llround(ox * 1e9), std::llround(oy * 1e9), (long long)hp.near_m[q]};
      };
      std::map<std::vector<long long>, int> region_first;
      std::map<std::array<long long, 5>, long long> pair_first;
      for (int li = 0; li < nl; ++li) {
        std::vector<long long> rkey = {local[hp.leaves[li]]};
        for (int q = hp.near_ptr[li]; q < hp.near_ptr[li + 1]; ++q) {
          if (circ[q]) continue;
          auto k = pair_key(q);
          rkey.insert(rkey.end(), k.begin() + 1, k.end());
        }
        auto it = region_first.find(rkey);
        if (it != region_first.end()) {
          const int lf = it->second;
          leaf_blk[li] = leaf_blk[lf];
          for (int q = hp.near_ptr[li], r = hp.near_ptr[lf]; q < hp.near_ptr[li + 1]; ++q) {
            if (circ[q]) continue;
            while (circ[r]) ++r;
            blk[q] = blk[r++];
          }
          continue;
        }
        region_first.emplace(rkey, li);
        leaf_blk[li] = stored;
        for (int q = hp.near_ptr[li]; q < hp.near_ptr[li + 1]; ++q) {
          if (circ[q]) continue;
          const long long len = pair_len(q);
          blk[q] = stored;
          stored += len;
          auto k = pair_key(q);
          auto pf = pair_first.find(k);
          if (pf == pair_first.end()) {
            pair_first.emplace(k, blk[q]);
            uniq.push_back(q);
          } else {
            cp_src.push_back(pf->second);
            cp_dst.push_back(blk[q]);
            cp_len.push_back((int)(4 * len));
          }
        }
      }
    } else {
      for (int li = 0; li < nl; ++li) {
        leaf_blk[li] = stored;
        for (int q = hp.near_ptr[li]; q < hp.near_ptr[li + 1]; ++q) {
          if (circ[q]) continue;
          blk[q] = stored;
          stored += pair_len(q);
          uniq.push_back(q);
        }
      }
    }
    pb.n_near_stored = stored;
    pb.n_near_uniq = (int)uniq.size();
    pb.n_near_copies = (int)cp_src.size();
    CK(upload(pb, &pb.d_near_blk, blk));
    CK(upload(pb, &pb.d_leaf_blk, leaf_blk));
    leaf_blk_host = leaf_blk;
    CK(upload(pb, &pb.d_near_uniq, uniq));
    if (!cp_src.empty()) {
      CK(upload(pb, &pb.d_near_cp_src, cp_src)); CK(upload(pb, &pb.d_near_cp_dst, cp_dst));
      CK(upload(pb, &pb.d_near_cp_len, cp_len));
    }
  }
  {
    // flattened source columns of every target leaf: the stored pairs' columns
    // in storage order, and the circulant pairs' columns with the source's
    // place on its circle
    int nl = (int)hp.leaves.size();
    std::vector<int> cptr(nl + 1, 0), cpsi, cm, qptr(nl + 1, 0), qpsi, qloc;
    for (int li = 0; li < nl; ++li) {
      for (int q = hp.near_ptr[li]; q < hp.near_ptr[li + 1]; ++q) {
        const Cell& C = hp.cells[hp.near_src[q]];
        for (int t = C.ebeg; t < C.eend; ++t) {
          int e = hp.elem_of[t], f = e / pb.N;
          if (circ[q]) {
            qpsi.push_back(2 * f * pb.N + (e - f * pb.N));
            qloc.push_back(e - f * pb.N);
          } else {
            cpsi.push_back(2 * f * pb.N + (e - f * pb.N));
            cm.push_back(hp.near_m[q]);
          }
        }
      }
      cptr[li + 1] = (int)cpsi.size();
      qptr[li + 1] = (int)qpsi.size();
    }
    {
      // with the own blocks by FFT P2P adds into the rows only where a leaf
      // has stored near columns
      std::vector<int> items, rowtasks, near_t0(std::max(1, nl), -1);
      std::vector<long long> rowoff;
      for (int li = 0; li < nl; ++li)
        if (cptr[li + 1] > cptr[li] || qptr[li + 1] > qptr[li]) {
          items.push_back(li);
          const Cell& L = hp.cells[hp.leaves[li]];
          const int rows = L.eend - L.ebeg;
          near_t0[li] = (int)(rowtasks.size() / 4);
          for (int r = 0; r < rows; ++r) {
            const int e = hp.elem_of[L.ebeg + r], f = e / pb.N;
            rowtasks.push_back(2 * f * pb.N + (e - f * pb.N));
            rowtasks.push_back(cptr[li]);
            rowtasks.push_back(cptr[li + 1] - cptr[li]);
            rowtasks.push_back(rows);
            rowoff.push_back(4 * leaf_blk_host[li] + r);
          }
        }
      pb.n_p2p_items = (int)items.size();
      pb.n_p2p_rowtasks = (int)(rowtasks.size() / 4);
      CK(upload(pb, &pb.d_p2p_items, items));
      CK(upload(pb, &pb.d_p2p_rowtasks, rowtasks));
      CK(upload(pb, &pb.d_p2p_rowoff, rowoff));
      CK(upload(pb, &pb.d_leaf_near_t0, near_t0));
      near_t0_host = near_t0;
      if (pb.self_fft) ws_add(pb, &pb.d_near_rows, 2 * (size_t)std::max(1, pb.n_p2p_rowtasks) * sizeof(cd), 0);
    }
    CK(upload(pb, &pb.d_cols_ptr, cptr));
    CK(upload(pb, &pb.d_col_psi, cpsi));
    CK(upload(pb, &pb.d_col_m, cm));
    CK(upload(pb, &pb.d_ccols_ptr, qptr));
    CK(upload(pb, &pb.d_ccol_psi, qpsi));
    CK(upload(pb, &pb.d_ccol_loc, qloc));
    // LDS windows of the circulant rows.  Target leaf li reads the entries
    // (b - a) + N of its fibre's rows for its rows a and circulant columns b;
    // counted from the start of the arc that holds them (after the largest
    // gap on the circle), a' = a - rot and b' = b - rot (mod N) keep b - a
    // mod N, and the entries N - a' + b' form one range of
    // (a'_max - a'_min) + (b'_max - b'_min) + 1 entries.  Leaves whose range
    // exceeds P2P_WCAP read the entries through the caches.
    std::vector<int> cwin(3 * (size_t)std::max(1, nl), 0);
    pb.p2p_wmax = 0;
    pb.n_win_leaves = 0;
    for (int li = 0; li < nl; ++li) {
      if (qptr[li + 1] == qptr[li]) continue;
      const Cell& L = hp.cells[hp.leaves[li]];
      std::vector<int> u;
      for (int t = L.ebeg; t < L.eend; ++t) u.push_back(hp.elem_of[t] % pb.N);
      for (int q = qptr[li]; q < qptr[li + 1]; ++q) u.push_back(qloc[q]);
      std::sort(u.begin(), u.end());
      u.erase(std::unique(u.begin(), u.end()), u.end());
      int rot = u[0], gap = u[0] + pb.N - u.back();
      for (size_t i = 1; i < u.size(); ++i)
        if (u[i] - u[i - 1] > gap) {
          gap = u[i] - u[i - 1];
          rot = u[i];
        }
      auto place = [&](int x) { return x >= rot ? x - rot : x - rot + pb.N; };
      int amin = pb.N, amax = -1, bmin = pb.N, bmax = -1;
      for (int t = L.ebeg; t < L.eend; ++t) {
        int a = place(hp.elem_of[t] % pb.N);
        amin = std::min(amin, a);
        amax = std::max(amax, a);
      }
      for (int q = qptr[li]; q < qptr[li + 1]; ++q) {
        int b = place(qloc[q]);
        bmin = std::min(bmin, b);
        bmax = std::max(bmax, b);
      }
      const int elo = pb.N - amax + bmin, wl = (bmax - bmin) + (amax - amin) + 1;
      cwin[3 * (size_t)li] = rot;
      cwin[3 * (size_t)li + 1] = elo;
      if (!pb.opt.p2p_cached_rows && wl <= P2P_WCAP) {
        cwin[3 * (size_t)li + 2] = wl;
        pb.p2p_wmax = std::max(pb.p2p_wmax, wl);
        pb.n_win_leaves++;
      }
    }
    CK(upload(pb, &pb.d_cwin, cwin));
    // split the columns of each target leaf when there are too few leaves to
    // fill the P2P grid, keeping at least 32 columns per split on average
    const long long ncols = (long long)cpsi.size() + (long long)qpsi.size();
    int S = 1;
    if (pb.p2p_grid > 0 && nl > 0 && nl < pb.p2p_grid) S = std::min(8, (pb.p2p_grid + nl - 1) / nl);
    while (S > 1 && ncols / ((long long)nl * S) < 32) --S;
    if (pb.self_fft) S = 1;             // P2P adds into the rows the FFT apply wrote
    pb.p2p_split = S;
    ws_add(pb, &pb.d_p2ppart, S > 1 ? 0 : sizeof(cd), S > 1 ? (size_t)S * 2 * (size_t)pb.E * sizeof(cd) : 0);
    // circulant rows [fibre][component][2N] (the second copy spares the wrap)
    ws_add(pb, &pb.d_circ, (size_t)std::max(1, pb.M) * 8 * pb.N * sizeof(cd), 0);
  }
  if (pb.opt.precond || pb.self_fft) {
    // per (fibre, mode) 2x2 blocks of the fibres' self blocks and of their
    // inverses, twiddles exp(2 pi i j / N), and (preconditioned GMRES) the
    // vector P^{-1} v of the preconditioned apply
    ws_add(pb, &pb.d_pc_fwd, (size_t)pb.M * pb.N * 4 * sizeof(cd), 0);
    ws_add(pb, &pb.d_pc_inv, (size_t)pb.M * pb.N * 4 * sizeof(cd), 0);
    if (pb.opt.precond) ws_add(pb, &pb.d_pc_x, 0, 2 * (size_t)pb.E * sizeof(cd));
    std::vector<cd> tw(pb.N);
    for (int j = 0; j < pb.N; ++j) {
      const double t = 2.0 * M_PI * j / pb.N;
      tw[j] = mkc(std::cos(t), std::sin(t));
    }
    CK(upload(pb, &pb.d_pc_tw, tw));
    pb.pc_logN = 0;
    while ((1 << pb.pc_logN) < pb.N) ++pb.pc_logN;
  }
  if (pb.nystrom) {
    // Kress's logarithmic weights R(t_d), t_d = 2 pi d / N, of the spectral
    // Nystrom rule for the log-singular kernels (the paper's refs. 2 and 4)
    std::vector<double> R(pb.N);
    for (int d = 0; d < pb.N; ++d) {
      double acc = 0.0;
      for (int m = 1; m < pb.N / 2; ++m) acc += std::cos(2.0 * M_PI * (double)m * d / pb.N) / m;
      R[d] = -(4.0 * M_PI / pb.N) * acc - (4.0 * M_PI / ((double)pb.N * pb.N)) * (d % 2 ? -1.0 : 1.0);
    }
    CK(upload(pb, &pb.d_kress, R));
  }
  CK(upload(pb, &pb.d_root_pair_off, hp.root_pair_off));
  CK(upload(pb, &pb.d_root_mrange, hp.root_off_mrange));
  CK(upload(pb, &pb.d_off_xy, hp.off_xy)); CK(upload(pb, &pb.d_joff_xy, hp.joff_xy));
  CK(upload(pb, &pb.d_root_off_xy, hp.root_off_xy));
  // quadrature rules: far rule, then 16-point near rule and 8-point field rule
  {
    std::vector<double> x, w, t;
    gauss_legendre(pb.opt.g_far, x, w);
    t = x;
    t.insert(t.end(), w.begin(), w.end());
    CK(upload(pb, &pb.d_gl, t));
    std::vector<double> x16, w16, x8, w8;
    gauss_legendre(16, x16, w16);
    gauss_legendre(8, x8, w8);
    std::vector<double> u = x16;
    u.insert(u.end(), w16.begin(), w16.end());
    u.insert(u.end(), x8.begin(), x8.end());
    u.insert(u.end(), w8.begin(), w8.end());
    CK(upload(pb, &pb.d_gl16, u));
  }
  const int NP = 2 * pb.opt.p + 1, NT = 4 * pb.opt.p + 1;
  const size_t MB = (size_t)pb.max_batch;   // per-member buffers: one copy per batch member
  ws_add(pb, &pb.d_mpole, 0, (size_t)nc * 2 * NP * sizeof(cd), true);
  size_t n_ent = std::max<long long>(1, pb.n_near_stored);
  ws_add(pb, &pb.d_near, 4 * n_ent * sizeof(cd), 0);
  if (pb.opt.precision == PFM_MIXED) {
    ws_add(pb, &pb.d_near32, 4 * n_ent * sizeof(float2), 0);
    ws_add(pb, &pb.d_ir_r, 2 * (size_t)E * sizeof(cd), 0);
    ws_add(pb, &pb.d_ir_d, 2 * (size_t)E * sizeof(cd), 0);
  }
  int n_off = std::max<int>(1, (int)hp.off_xy.size() / 2);
  int n_joff = std::max<int>(1, (int)hp.joff_xy.size() / 2);
  int n_roff = std::max<int>(1, (int)hp.root_off_xy.size() / 2);
  // translation table rows per channel: explicit M2L offsets, then lattice offsets
  int n_off_real = (int)hp.off_xy.size() / 2;
  pb.n_tab = n_off_real + n_roff;
  ws_add(pb, &pb.d_htab, 0, 2 * (size_t)pb.n_tab * NT * sizeof(cd), true);
  ws_add(pb, &pb.d_jtab, (size_t)2 * n_joff * NT * sizeof(cd), 0);
  ws_add(pb, &pb.d_betas, 0, sizeof(double));
  ws_add(pb, &pb.d_thetas, 0, sizeof(double));
  ws_add(pb, &pb.d_latpart, 0, (size_t)n_roff * ((LAT_RULE_POINTS + 255) / 256) * NT * sizeof(cd));
  ws_add(pb, &pb.d_srule, 2 * (size_t)LAT_RULE_POINTS * sizeof(double), 0);
  (void)n_off;
  // fibre roots by their Fourier modes (with the own blocks by FFT): a fibre
  // is a tree fibre when a cell of it below the root is the target or the
  // source of an M2L entry, or when one of its leaves or cells is in a near
  // pair; the others are spectral fibres.  Root cells come first in the
  // level-major order (root of fibre f = cell f), which the moments' DFT
  // launch relies on.
  std::vector<char> tree_fib(pb.M, 0);
  pb.spec_root = pb.self_fft && opt->self_mode == 0;
  for (int f = 0; f < pb.M && pb.spec_root; ++f)
    if (hp.root_of_fibre[f] != f) pb.spec_root = false;
  if (pb.spec_root) {
    for (int c = 0; c < nc; ++c) {
      for (int q = hp.m2l_ptr[c]; q < hp.m2l_ptr[c + 1]; ++q) {
        if (hp.cells[c].level != 0) tree_fib[hp.cells[c].fiber] = 1;
        const Cell& S = hp.cells[hp.m2l_src[q]];
        if (S.level != 0) tree_fib[S.fiber] = 1;
      }
      for (int q = hp.m2li_ptr[c]; q < hp.m2li_ptr[c + 1]; ++q) {
        tree_fib[hp.cells[c].fiber] = 1;
        tree_fib[hp.cells[hp.m2li_src[q]].fiber] = 1;
      }
    }
    for (size_t q = 0; q < hp.near_src.size(); ++q) {
      tree_fib[hp.cells[hp.leaves[hp.near_tgt[q]]].fiber] = 1;
      tree_fib[hp.cells[hp.near_src[q]].fiber] = 1;
    }
  }
  if (pb.spec_root) {
    ws_add(pb, &pb.d_spec_tab, (size_t)pb.M * 4 * NP * sizeof(cd), 0);
    ws_add(pb, &pb.d_spec_hat, 0, 2 * (size_t)E * sizeof(cd));
  }
  {
    // M2L work: per (channel, cell) the entries (source cell, table row, image),
    // contiguous, cut into chunks of at most M2L_CHUNK entries (one wavefront
    // each); one sum per (channel, cell) with entries adds its chunks' partial
    // expansions in order, so the downward pass reads one sum per cell.  A
    // root's M lattice entries go in chunks of M2L_LAT_CHUNK once M >= 128,
    // where one-entry chunks would write M partial expansions per root.
    std::vector<int> esrc, eoff, em, mchunks, sums, ccptr(2 * (size_t)nc + 1, 0);
    std::vector<int> fibre_of_root(nc, -1);
    for (int f = 0; f < pb.M; ++f) fibre_of_root[hp.root_of_fibre[f]] = f;
    // Fibre grid of the lattice M2L convolution.  Fibre f = j M_L + i sits in
    // column i, row j; on the hexagonal lattice odd columns are half a
    // spacing higher, so the column parity is a sublattice and gx = i / 2.
    // Every root pair's lattice row must depend only on (sublattices, grid
    // displacement); that is checked here, else the pairs stay M2L entries.
    const bool hexl = pb.lattice == PFM_HEXAGON;
    const int lns = hexl ? 2 : 1, lgx = hexl ? (pb.ML + 1) / 2 : pb.ML, lgy = pb.MH;
    const int lpx = 2 * lgx, lpy = 2 * lgy;
    auto lsub = [&](int f) { return hexl ? (f % pb.ML) & 1 : 0; };
    auto lgxf = [&](int f) { return hexl ? (f % pb.ML) >> 1 : f % pb.ML; };
    auto lgyf = [&](int f) { return f / pb.ML; };
    std::vector<int> lkey((size_t)lns * lns * (2 * lgy - 1) * (2 * lgx - 1), -1);
    pb.lat_fft = pb.M >= 128 && !pb.opt.direct_lattice_m2l && lpx <= 64 && lpy <= 64 && lpx * lpy <= LAT_PXY_MAX;
    for (int i = 0; pb.lat_fft && i < pb.M; ++i)
      for (int j = 0; j < pb.M; ++j) {
        const size_t kk = (((size_t)lsub(i) * lns + lsub(j)) * (2 * lgy - 1) + (lgyf(i) - lgyf(j) + lgy - 1)) *
                              (2 * lgx - 1) + (lgxf(i) - lgxf(j) + lgx - 1);
        const int id = hp.root_pair_off[(size_t)i * pb.M + j];
        if (lkey[kk] < 0) lkey[kk] = id;
        else if (lkey[kk] != id) pb.lat_fft = false;
      }
    std::vector<int> lcell((size_t)lns * lgy * lgx, -1), lslot((size_t)lns * lgy * lgx, -1);
    for (int f = 0; f < pb.M; ++f) lcell[((size_t)lsub(f) * lgy + lgyf(f)) * lgx + lgxf(f)] = hp.root_of_fibre[f];
    for (int ch = 0; ch < 2; ++ch) {
      for (int c = 0; c < nc; ++c) {
        int first = (int)esrc.size();
        bool lattice_root = false;
        if (ch == 0) {
          for (int q = hp.m2l_ptr[c]; q < hp.m2l_ptr[c + 1]; ++q) {
            esrc.push_back(hp.m2l_src[q]); eoff.push_back(hp.m2l_off[q]); em.push_back(hp.m2l_m[q]);
          }
          int fi = fibre_of_root[c];
          lattice_root = fi >= 0;
          if (fi >= 0 && !pb.lat_fft)
            for (int j = 0; j < pb.M; ++j) {
              esrc.push_back(hp.root_of_fibre[j]);
              eoff.push_back(n_off_real + hp.root_pair_off[(size_t)fi * pb.M + j]);
              em.push_back(0);
            }
        } else {
          for (int q = hp.m2li_ptr[c]; q < hp.m2li_ptr[c + 1]; ++q) {
            esrc.push_back(hp.m2li_src[q]); eoff.push_back(hp.m2li_off[q]); em.push_back(0);
          }
        }
        int last = (int)esrc.size();
        int chunk0 = (int)(mchunks.size() / 4);
        const int csz = lattice_root && pb.M >= 128 ? M2L_LAT_CHUNK : M2L_CHUNK;
        for (int b = first; b < last; b += csz) {
          mchunks.push_back(c); mchunks.push_back(ch); mchunks.push_back(b);
          mchunks.push_back(std::min(csz, last - b));
        }
        if (ch == 0 && lattice_root && pb.lat_fft) {
          // the root's lattice M2L arrives from the grid convolution as one more
          // partial expansion, after its explicit entries (an empty chunk that
          // k_m2l leaves alone)
          const int f = fibre_of_root[c];
          lslot[((size_t)lsub(f) * lgy + lgyf(f)) * lgx + lgxf(f)] = (int)(mchunks.size() / 4);
          mchunks.push_back(c); mchunks.push_back(ch); mchunks.push_back(last); mchunks.push_back(0);
        }
        int chunk1 = (int)(mchunks.size() / 4);
        if (chunk1 > chunk0) {
          sums.push_back(c); sums.push_back(ch); sums.push_back(chunk0); sums.push_back(chunk1 - chunk0);
        }
        ccptr[(size_t)ch * nc + c + 1] = (int)(sums.size() / 4);
      }
    }
    pb.n_chunks = (int)(sums.size() / 4);
    pb.n_mchunks = (int)(mchunks.size() / 4);
    {
      // one-entry chunks grouped by translation (channel, table row) for the
      // matrix cores, 16 entries per item; the other chunks stay with k_m2l
      std::map<std::pair<int, int>, std::vector<int>> groups;
      std::vector<int> vch;
      for (int c = 0; c < pb.n_mchunks; ++c) {
        const int ch = mchunks[4 * (size_t)c + 1], b = mchunks[4 * (size_t)c + 2], cnt = mchunks[4 * (size_t)c + 3];
        if (cnt == 0) continue;                      // the lattice convolution's slot
        if (cnt == 1 && !opt->m2l_vector) groups[{ch, eoff[b]}].push_back(c);
        else vch.push_back(c);
      }
      // columns stored 16 per item (unused ones repeat the item's first, so
      // that their source and image stay valid indices)
      std::vector<int> items, cols;
      int n_cols = 0;
      for (const auto& g : groups)
        for (size_t j0 = 0; j0 < g.second.size(); j0 += 16) {
          const int n = (int)std::min<size_t>(16, g.second.size() - j0);
          items.push_back(g.first.first); items.push_back(g.first.second);
          items.push_back((int)(cols.size() / 4)); items.push_back(n);
          for (int j = 0; j < 16; ++j) {
            const int c = g.second[j0 + (j < n ? j : 0)];
            const int b = mchunks[4 * (size_t)c + 2];
            cols.push_back(esrc[b]); cols.push_back(c); cols.push_back(em[b]); cols.push_back(0);
          }
          n_cols += n;
        }
      pb.n_vchunks = (int)vch.size();
      pb.n_mfma_items = (int)(items.size() / 4);
      pb.n_mfma_cols = n_cols;
      if (vch.empty()) vch.assign(1, 0);
      if (items.empty()) items.assign(4, 0), cols.assign(4, 0);
      CK(upload(pb, &pb.d_vchunks, vch)); CK(upload(pb, &pb.d_mfma_items, items)); CK(upload(pb, &pb.d_mfma_cols, cols));
    }
    CK(upload(pb, &pb.d_e_src, esrc)); CK(upload(pb, &pb.d_e_off, eoff)); CK(upload(pb, &pb.d_e_m, em));
    CK(upload(pb, &pb.d_mchunks, mchunks)); CK(upload(pb, &pb.d_chunks, sums)); CK(upload(pb, &pb.d_cc_ptr, ccptr));
    // leaf descriptors of P2M and the downward pass: everything a leaf's
    // workgroup reads is one load away from its index (no chain leaf -> cell
    // -> element -> geometry, or cell -> sum row)
    const int nl = (int)hp.leaves.size();
    std::vector<int> ldesc(8 * (size_t)nl), lanc;
    std::vector<double> tgeo(4 * (size_t)E), trh(E), tx(E), ty(E), hh(E);
    CK(hipMemcpy(tx.data(), pb.d_tx, E * sizeof(double), hipMemcpyDeviceToHost));
    CK(hipMemcpy(ty.data(), pb.d_ty, E * sizeof(double), hipMemcpyDeviceToHost));
    CK(hipMemcpy(hh.data(), pb.d_h, E * sizeof(double), hipMemcpyDeviceToHost));
    auto sum_row = [&](int ch, int c) {
      size_t i = (size_t)ch * nc + c;
      return ccptr[i + 1] > ccptr[i] ? ccptr[i] : -1;
    };
    // the M2L chunks (first, count) of a (channel, cell), count 0 if none
    auto chunk_rng = [&](int ch, int c) {
      const int r = sum_row(ch, c);
      return r < 0 ? std::make_pair(0, 0) : std::make_pair(sums[4 * (size_t)r + 2], sums[4 * (size_t)r + 3]);
    };
    if (pb.spec_root) {
      // every fibre's root local expansion (the sum of the root's M2L
      // chunks) is evaluated at its midpoints by the synthesis of the last
      // own-block launch
      std::vector<int> rng(2 * (size_t)pb.M, 0);
      pb.n_spec = 0;
      for (int f = 0; f < pb.M; ++f) {
        const auto cr = chunk_rng(0, hp.root_of_fibre[f]);
        rng[2 * (size_t)f] = cr.first;
        rng[2 * (size_t)f + 1] = cr.second;
        if (!tree_fib[f]) pb.n_spec++;
      }
      CK(upload(pb, &pb.d_spec_rng, rng));
    }
    for (int li = 0; li < nl; ++li) {
      const Cell& L = hp.cells[hp.leaves[li]];
      int* d = &ldesc[8 * (size_t)li];
      d[0] = L.ebeg;
      d[1] = L.eend - L.ebeg;
      for (int ch = 0; ch < 2; ++ch) {
        d[2 + ch] = sum_row(ch, hp.leaves[li]);
        d[4 + 2 * ch] = (int)(lanc.size() / 2);
        for (int q = hp.anc_ptr[li]; q < hp.anc_ptr[li + 1]; ++q) {
          int r = sum_row(ch, hp.anc[q]);
          if (r < 0) continue;
          lanc.push_back(r);
          lanc.push_back(hp.anc_off[q]);
        }
        d[5 + 2 * ch] = (int)(lanc.size() / 2);
      }
      for (int t = L.ebeg; t < L.eend; ++t) {
        int e = hp.elem_of[t];
        tgeo[4 * (size_t)t] = mx[e] - L.cx;
        tgeo[4 * (size_t)t + 1] = my[e] - L.cy;
        tgeo[4 * (size_t)t + 2] = tx[e];
        tgeo[4 * (size_t)t + 3] = ty[e];
        trh[t] = hh[e];
      }
    }
    if (pb.spec_root) {
      // P2M: the tree fibres' leaves below the root (rows in tree order,
      // offsets from the leaf's centre; a root's moments come from the
      // transforms, also when the root is a leaf).  Downward pass, grouped by
      // fibre: the tree fibres' leaves with a far part from below the root
      // (M2L chunks of their own or of an ancestor other than the root, whose
      // expansion the synthesis evaluates) or with stored near pairs; each
      // with its ancestors' (chunks, J-table row) without the root.  A leaf
      // that is its fibre's root keeps only its near rows here.
      // Every cell of a tree fibre below its root gets its moments directly
      // from per-frequency P2M weights of its elements (cells between the
      // leaves and the root first: they have the most elements), so that no
      // M2M runs: [cell, first row, rows, first table row]
      std::vector<int> mc;
      int trows = 0;
      for (int pass = 0; pass < 2; ++pass)
        for (int c = 0; c < nc; ++c) {
          const Cell& C = hp.cells[c];
          if (!tree_fib[C.fiber] || C.level == 0 || (pass == 0) == (C.leaf != 0)) continue;
          const int rows = C.eend - C.ebeg;     // <= N <= 512 (the own blocks by FFT)
          mc.push_back(c); mc.push_back(C.ebeg); mc.push_back(rows); mc.push_back(trows);
          trows += rows;
        }
      pb.n_mcells = (int)(mc.size() / 4);
      ws_add(pb, &pb.d_p2m_tab, (size_t)std::max(1, trows) * (pb.opt.p + 1) * 2 * sizeof(cd), 0);
      if (mc.empty()) mc.assign(4, 0);
      CK(upload(pb, &pb.d_mcell, mc));
      std::vector<std::vector<int>> by_fib(pb.M);
      std::vector<int> da;
      for (int li = 0; li < nl; ++li) {
        const Cell& L = hp.cells[hp.leaves[li]];
        if (!tree_fib[L.fiber]) continue;
        const auto own = L.level == 0 ? std::make_pair(0, 0) : chunk_rng(0, hp.leaves[li]);
        const int a0 = (int)(da.size() / 4);
        for (int q = hp.anc_ptr[li]; q < hp.anc_ptr[li + 1]; ++q) {
          const auto ar = chunk_rng(0, hp.anc[q]);
          if (ar.second == 0 || hp.cells[hp.anc[q]].level == 0) continue;
          da.push_back(ar.first); da.push_back(ar.second); da.push_back(hp.anc_off[q]); da.push_back(0);
        }
        const int a1 = (int)(da.size() / 4);
        const int t0 = near_t0_host.empty() ? -1 : near_t0_host[li];
        if (own.second == 0 && a1 == a0 && t0 < 0) continue;
        std::vector<int>& v = by_fib[L.fiber];
        v.insert(v.end(), {L.ebeg, L.eend - L.ebeg, own.first, own.second, a0, a1, t0, 0});
      }
      std::vector<int> dptr(pb.M + 1, 0), dd;
      for (int f = 0; f < pb.M; ++f) {
        dd.insert(dd.end(), by_fib[f].begin(), by_fib[f].end());
        dptr[f + 1] = (int)(dd.size() / 8);
      }
      pb.n_dleaves = dptr[pb.M];
      // each down leaf's first row in the per-frequency L2P table (desc[7])
      int lrows = 0;
      for (int q = 0; q < pb.n_dleaves; ++q) {
        dd[8 * (size_t)q + 7] = lrows;
        lrows += dd[8 * (size_t)q + 1];
      }
      ws_add(pb, &pb.d_l2p_tab, (size_t)std::max(1, lrows) * (pb.opt.p + 2) * sizeof(cd), 0);
      if (dd.empty()) dd.assign(8, 0);
      if (da.empty()) da.assign(4, 0);
      CK(upload(pb, &pb.d_dptr, dptr)); CK(upload(pb, &pb.d_dldesc, dd)); CK(upload(pb, &pb.d_danc, da));
    }
    if (lanc.empty()) lanc.assign(2, 0);
    CK(upload(pb, &pb.d_ldesc, ldesc)); CK(upload(pb, &pb.d_lanc, lanc)); CK(upload(pb, &pb.d_tgeo, tgeo)); CK(upload(pb, &pb.d_trh, trh));
    ws_add(pb, &pb.d_part, 0, (size_t)std::max(1, pb.n_chunks) * NP * sizeof(cd));
    ws_add(pb, &pb.d_epart, 0, (size_t)std::max(1, pb.n_mchunks) * NP * sizeof(cd));
    if (pb.lat_fft) {
      pb.lat_ns = lns; pb.lat_gx = lgx; pb.lat_gy = lgy; pb.lat_px = lpx; pb.lat_py = lpy;
      const size_t pxy = (size_t)lpx * lpy;
      CK(upload(pb, &pb.d_lat_cell, lcell)); CK(upload(pb, &pb.d_lat_slot, lslot)); CK(upload(pb, &pb.d_lat_key, lkey));
      ws_add(pb, &pb.d_lat_shat, 0, (size_t)lns * lns * pxy * NT * sizeof(cd));
      ws_add(pb, &pb.d_lat_xhat, 0, (size_t)lns * pxy * NP * sizeof(cd));
      ws_add(pb, &pb.d_lat_lhat, 0, (size_t)lns * pxy * NP * sizeof(cd));
    }
  }
  {
    CK(upload(pb, &pb.d_up_cells, hp.up_cells)); CK(upload(pb, &pb.d_up_ptr, hp.up_ptr));
    CK(upload(pb, &pb.d_up_src, hp.up_src)); CK(upload(pb, &pb.d_up_off, hp.up_off));
    pb.n_up = (int)hp.up_cells.size();
    ws_add(pb, &pb.d_far, 0, 2 * (size_t)E * sizeof(cd));
  }
  {
    size_t na = (size_t)(hp.m_max - hp.m_min + 1);
    ws_add(pb, &pb.d_alpha, 0, na * sizeof(cd));
    std::vector<cd> ones(na, mkc(1.0, 0.0));
    CK(upload(pb, &pb.d_alpha_one, ones));
  }
  // GMRES workspace (batched solves use MB members of each vector)
  size_t n = 2 * (size_t)E;
  ws_add(pb, &pb.d_V, 0, (size_t)(pb.opt.restart + 1) * n * sizeof(cd));
  ws_add(pb, &pb.d_w, 0, n * sizeof(cd));
  ws_add(pb, &pb.d_r, 0, n * sizeof(cd));
  ws_add(pb, &pb.d_b, 0, n * sizeof(cd));
  ws_add(pb, &pb.d_tmp, 0, n * sizeof(cd));
  ws_add(pb, &pb.d_gin, 0, n * sizeof(cd));
  ws_add(pb, &pb.d_ir_aug, 0, n * sizeof(cd));
  ws_add(pb, &pb.d_cperp, 0, n * sizeof(cd));
  ws_add(pb, &pb.d_gout, 0, n * sizeof(cd));
  pb.red_blocks = reduction_blocks((long long)n);
  ws_add(pb, &pb.d_npart, 0, ((n + 63) / 64) * sizeof(double));
  ws_add(pb, &pb.d_dcoef, 0, (2 * (size_t)pb.opt.restart + 4) * sizeof(cd));
  // restart + 1 columns: DCGS2 leaves the last reorthogonalisation of a cycle in column restart
  ws_add(pb, &pb.d_hall, 0, ((size_t)pb.opt.restart + 1) * (2 * pb.opt.restart + 4) * sizeof(cd));
  CK(hipHostMalloc((void**)&pb.h_hall, ((size_t)pb.opt.restart + 1) * MB * (2 * pb.opt.restart + 4) * sizeof(cd)));
  // dot partials [member][vector][block], then (long vectors) the reduced [member][vector]
  ws_add(pb, &pb.d_red, 0, (size_t)(pb.red_blocks + 1) * (2 * pb.opt.restart + 8) * sizeof(cd));
  ws_add(pb, &pb.d_hcol, 0, (size_t)(2 * pb.opt.restart + 8) * sizeof(cd));
  CK(hipHostMalloc((void**)&pb.h_hcol, MB * (2 * pb.opt.restart + 8) * sizeof(cd)));
  ws_add(pb, &pb.d_fields, (size_t)2 * 512 * sizeof(cd), 0);
  // the library's own workspace block, sized for max_batch members (a caller
  // may later bind a block of its own with pfm_bind)
  {
    const size_t wsb = ws_size(pb, pb.max_batch);
    CK(dev_alloc(pb, &pb.ws_own, wsb));
    CK(ws_carve(pb, pb.ws_own, pb.max_batch, nullptr));
    CK(hipDeviceSynchronize());
  }
  for (int i = 0; i < 16; ++i) CK(hipEventCreate(&pb.ev[i]));
  CK(hipEventCreateWithFlags(&pb.ev_fork, hipEventDisableTiming));
  CK(hipEventCreateWithFlags(&pb.ev_join, hipEventDisableTiming));
  pb.events = true;
  CK(hipStreamCreateWithFlags(&pb.side, hipStreamNonBlocking));
  CK(hipStreamCreateWithFlags(&pb.cap, hipStreamNonBlocking));
#undef CK
  *out = h;
  return PFM_OK;
}

pfm_status pfm_set_stream(pfm_problem* h, void* stream) {
  if (!h) return PFM_EINVAL;
  h->p.stream = (hipStream_t)stream;
  return PFM_OK;
}

}  // extern "C"

namespace {

void drop_graph(Problem& pb) {
  if (pb.graph) (void)hipGraphExecDestroy(pb.graph);
  pb.graph = nullptr;
}

// Wavenumbers and coupling of a frequency (no device work).
void set_frequency(Problem& pb, double ka) {
  pb.k = ka / pb.a;
  pb.k1 = pb.k * pb.c_m / pb.c_f;
  pb.varrho = pb.rho_m / pb.rho_f;
  pb.eta = pb.eta_user > 0 ? pb.eta_user : pb.k;
}

std::vector<cd> image_phases(const Problem& pb, double beta) {
  const HostPlan& hp = pb.hp;
  std::vector<cd> al(hp.m_max - hp.m_min + 1);
  for (int m = hp.m_min; m <= hp.m_max; ++m) al[m - hp.m_min] = mkc(std::cos(m * beta), std::sin(m * beta));
  return al;
}

// Angle-independent per-frequency work: lattice cut-off q and tail rule
// (they depend on k and the geometry only), translation tables of member 0.
pfm_status frequency_tables(Problem& pb) {
  const HostPlan& hp = pb.hp;
  // lattice-sum cut-off q: all excluded images inside |m| <= q, (q+1)H - |Y| >= H/2,
  // and the contour factor exp(k X^2 / (4 ((q+1)H - |Y|))) held below e^2
  double xmax = 0.0, ymax = 0.0;
  int mex = 0;
  int n_roff = (int)hp.root_off_xy.size() / 2;
  for (int o = 0; o < n_roff; ++o) {
    xmax = std::max(xmax, std::fabs(hp.root_off_xy[2 * o]));
    ymax = std::max(ymax, std::fabs(hp.root_off_xy[2 * o + 1]));
    if (hp.root_off_mrange[2 * o] <= hp.root_off_mrange[2 * o + 1])
      mex = std::max(mex, std::max(std::abs(hp.root_off_mrange[2 * o]), std::abs(hp.root_off_mrange[2 * o + 1])));
  }
  int q = std::max(3, mex + 1);
  while (true) {
    double gap = (q + 1) * pb.H - ymax;
    if (gap >= 0.5 * pb.H && pb.k * xmax * xmax / (4.0 * gap) <= 2.0) break;
    ++q;
  }
  pb.lattice_q = q;
  std::vector<double> rule;
  tail_rule(pb.k, pb.H, (q + 1) * pb.H - ymax, xmax, 2 * pb.opt.p, rule);
  if (rule.size() != 2 * (size_t)LAT_RULE_POINTS) return fail(pb, PFM_ENUMERIC, "lattice tail rule size");
  HIPCHK(pb, hipMemcpyAsync(pb.d_srule, rule.data(), rule.size() * sizeof(double), hipMemcpyHostToDevice,
                            pb.stream));
  pb.n_srule = (int)rule.size() / 2;
  HIPCHK(pb, launch_tables(pb));
  return PFM_OK;
}

pfm_status check_wood(Problem& pb, double theta) {
  double wd = wood_distance(pb.k, pb.H, theta);
  if (pb.opt.wood_margin > 0 && wd < pb.opt.wood_margin)
    return fail(pb, PFM_EWOOD, "k H (1 +- sin theta) / (2 pi) is " + std::to_string(wd) + " from an integer");
  return PFM_OK;
}

// Capture the batched apply d_gin -> d_gout of the current batch into a graph.
pfm_status capture_batch_graph(Problem& pb) {
  drop_graph(pb);
  hipStream_t saved = pb.stream;
  pb.stream = pb.cap;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(pb.cap, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    hipError_t ea = apply_operator_batch(pb, pb.d_gin, pb.d_gout, nullptr);
    e = hipStreamEndCapture(pb.cap, &g);
    if (ea != hipSuccess) e = ea;
  }
  pb.stream = saved;
  if (e == hipSuccess) e = hipGraphInstantiate(&pb.graph, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    pb.graph = nullptr;
    return fail(pb, PFM_EDEVICE, std::string("graph capture of the batched apply: ") + hipGetErrorString(e));
  }
  return PFM_OK;
}

}  // namespace

extern "C" {

pfm_status pfm_set_wave(pfm_problem* h, double ka, double theta) {
  if (!h) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!(ka > 0) || !(std::fabs(theta) < 0.5 * PI))
    return fail(pb, PFM_EINVAL, "need ka > 0 and |theta| < pi/2");
  pb.wave_ready = false;
  pb.batch_ready = false;
  drop_graph(pb);
  set_frequency(pb, ka);
  pb.theta = theta;
  pb.beta = pb.k * pb.H * std::sin(theta);
  pfm_status st = check_wood(pb, theta);
  if (st != PFM_OK) return st;
  std::vector<cd> al = image_phases(pb, pb.beta);
  HIPCHK(pb, hipMemcpyAsync(pb.d_alpha, al.data(), al.size() * sizeof(cd), hipMemcpyHostToDevice, pb.stream));
  st = frequency_tables(pb);
  if (st != PFM_OK) return st;
  HIPCHK(pb, hipMemcpyAsync(pb.d_betas, &pb.beta, sizeof(double), hipMemcpyHostToDevice, pb.stream));
  HIPCHK(pb, launch_lattice_sums(pb, 1));
  HIPCHK(pb, launch_near_blocks(pb, false));
  if (pb.opt.precision == PFM_MIXED) HIPCHK(pb, launch_near_to_c64(pb));
  if (pb.opt.precond || pb.self_fft) HIPCHK(pb, launch_precond_setup(pb));
  HIPCHK(pb, hipStreamSynchronize(pb.stream));
  pb.wave_ready = true;
  return PFM_OK;
}

pfm_status pfm_set_batch(pfm_problem* h, double ka, int B, const double* theta) {
  if (!h) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!theta || B < 1 || B > pb.max_batch)
    return fail(pb, PFM_EINVAL, "need 1 <= B <= max_batch and a theta array");
  if (!(ka > 0)) return fail(pb, PFM_EINVAL, "need ka > 0");
  for (int b = 0; b < B; ++b)
    if (!(std::fabs(theta[b]) < 0.5 * PI)) return fail(pb, PFM_EINVAL, "need |theta| < pi/2");
  pb.wave_ready = false;
  pb.batch_ready = false;
  drop_graph(pb);
  set_frequency(pb, ka);
  for (int b = 0; b < B; ++b) {
    pfm_status st = check_wood(pb, theta[b]);
    if (st != PFM_OK) return st;
  }
  pb.B = B;
  pb.thetas.assign(theta, theta + B);
  pb.theta = theta[0];
  pb.beta = pb.k * pb.H * std::sin(theta[0]);
  const HostPlan& hp = pb.hp;
  const size_t na = (size_t)(hp.m_max - hp.m_min + 1);
  std::vector<cd> al(na * B);
  for (int b = 0; b < B; ++b) {
    std::vector<cd> ab = image_phases(pb, pb.k * pb.H * std::sin(theta[b]));
    std::copy(ab.begin(), ab.end(), al.begin() + b * na);
  }
  HIPCHK(pb, hipMemcpyAsync(pb.d_alpha, al.data(), al.size() * sizeof(cd), hipMemcpyHostToDevice, pb.stream));
  pfm_status st = frequency_tables(pb);
  if (st != PFM_OK) return st;
  // every member starts from member 0's tables; their lattice rows are then replaced
  const size_t tab = (size_t)2 * pb.n_tab * (4 * pb.opt.p + 1);
  for (int b = 1; b < B; ++b)
    HIPCHK(pb, hipMemcpyAsync(pb.d_htab + b * tab, pb.d_htab, tab * sizeof(cd), hipMemcpyDeviceToDevice,
                              pb.stream));
  std::vector<double> betas(B);
  for (int b = 0; b < B; ++b) betas[b] = pb.k * pb.H * std::sin(theta[b]);
  HIPCHK(pb, hipMemcpyAsync(pb.d_betas, betas.data(), B * sizeof(double), hipMemcpyHostToDevice, pb.stream));
  HIPCHK(pb, launch_lattice_sums(pb, B));
  HIPCHK(pb, launch_near_blocks(pb, true));
  if (pb.opt.precond || pb.self_fft) HIPCHK(pb, launch_precond_setup(pb));
  HIPCHK(pb, hipStreamSynchronize(pb.stream));
  if (pb.opt.use_graph) {
    st = capture_batch_graph(pb);
    if (st != PFM_OK) return st;
  }
  pb.batch_ready = true;
  return PFM_OK;
}

pfm_status pfm_matvec_batch(pfm_problem* h, const void* d_psi, void* d_y) {
  if (!h || !d_psi || !d_y) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!pb.batch_ready) return fail(pb, PFM_ESTATE, "pfm_set_batch first");
  HIPCHK(pb, apply_operator_batch(pb, (const cd*)d_psi, (cd*)d_y, nullptr));
  return PFM_OK;
}

pfm_status pfm_rhs_batch(pfm_problem* h, void* d_b) {
  if (!h || !d_b) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!pb.batch_ready) return fail(pb, PFM_ESTATE, "pfm_set_batch first");
  for (int b = 0; b < pb.B; ++b) HIPCHK(pb, launch_rhs(pb, pb.thetas[b], (cd*)d_b + (size_t)b * 2 * pb.E));
  return PFM_OK;
}

pfm_status pfm_matvec_batch_timed(pfm_problem* h, const void* d_psi, void* d_y, int reps, double* stage_ms,
                                  double* total_ms) {
  if (!h || !d_psi || !d_y || reps < 1) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!pb.batch_ready) return fail(pb, PFM_ESTATE, "pfm_set_batch first");
  double acc[6] = {0, 0, 0, 0, 0, 0}, tot = 0.0;
  for (int r = 0; r < reps; ++r) {
    HIPCHK(pb, apply_operator_batch(pb, (const cd*)d_psi, (cd*)d_y, pb.ev));
    HIPCHK(pb, hipEventSynchronize(pb.ev[6]));
    for (int s = 0; s < 6; ++s) {
      float ms = 0.f;
      HIPCHK(pb, hipEventElapsedTime(&ms, pb.ev[s], pb.ev[s + 1]));
      acc[s] += ms;
    }
    float all = 0.f;
    HIPCHK(pb, hipEventElapsedTime(&all, pb.ev[0], pb.ev[6]));
    tot += all;
  }
  if (stage_ms)
    for (int s = 0; s < 6; ++s) stage_ms[s] = acc[s] / reps;
  if (total_ms) *total_ms = tot / reps;
  return PFM_OK;
}

pfm_status pfm_matvec(pfm_problem* h, const void* d_psi, void* d_y) {
  if (!h || !d_psi || !d_y) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!pb.wave_ready) return fail(pb, PFM_ESTATE, "pfm_set_wave first");
  HIPCHK(pb, apply_operator(pb, (const cd*)d_psi, (cd*)d_y, nullptr));
  return PFM_OK;
}

pfm_status pfm_matvec_static(pfm_problem* h, const void* d_psi, void* d_y) {
  if (!h || !d_psi || !d_y) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!pb.wave_ready) return fail(pb, PFM_ESTATE, "pfm_set_wave first");
  if (!pb.static_scratch) return fail(pb, PFM_EDEVICE, "no address of the static scratch array");
  int dev = -1;
  HIPCHK(pb, hipGetDevice(&dev));
  if (dev != pb.device) return fail(pb, PFM_EINVAL, "the handle's GPU is not the current device");
  const size_t NP = 2 * (size_t)pb.opt.p + 1;
  const size_t nc = pb.hp.cells.size();
  const size_t pxy = (size_t)pb.lat_px * pb.lat_py;
  struct Use {
    cd** ptr;
    size_t bytes;
  } use[] = {
      {&pb.d_mpole, nc * 2 * NP * sizeof(cd)},
      {&pb.d_epart, (size_t)std::max(1, pb.n_mchunks) * NP * sizeof(cd)},
      {&pb.d_part, (size_t)std::max(1, pb.n_chunks) * NP * sizeof(cd)},
      {&pb.d_far, 2 * (size_t)pb.E * sizeof(cd)},
      {&pb.d_p2ppart, pb.p2p_split > 1 ? (size_t)pb.p2p_split * 2 * pb.E * sizeof(cd) : sizeof(cd)},
      {&pb.d_lat_xhat, pb.lat_fft ? (size_t)pb.lat_ns * pxy * NP * sizeof(cd) : 0},
      {&pb.d_lat_lhat, pb.lat_fft ? (size_t)pb.lat_ns * pxy * NP * sizeof(cd) : 0},
      {&pb.d_spec_hat, pb.spec_root ? 2 * (size_t)pb.E * sizeof(cd) : 0},
  };
  size_t total = 0;
  for (const Use& u : use) total += ws_align(u.bytes);
  if (total > (size_t)PFM_STATIC_SCRATCH_BYTES)
    return fail(pb, PFM_EINVAL, "the apply needs " + std::to_string(total) + " bytes of scratch, above the " +
                                    std::to_string((size_t)PFM_STATIC_SCRATCH_BYTES) + " of the static array");
  // point the apply's scratch buffers into the array for this call only (the
  // kernels take the addresses as arguments when they are queued)
  cd* saved[sizeof(use) / sizeof(use[0])];
  char* at = (char*)pb.static_scratch;
  for (size_t i = 0; i < sizeof(use) / sizeof(use[0]); ++i) {
    saved[i] = *use[i].ptr;
    if (use[i].bytes) *use[i].ptr = (cd*)at;
    at += ws_align(use[i].bytes);
  }
  // the moments start from zero as in a fresh workspace (the array keeps the
  // last call's contents)
  hipError_t e = launch_fill_zero(pb.d_mpole, use[0].bytes, pb.stream);
  if (e == hipSuccess) e = apply_operator(pb, (const cd*)d_psi, (cd*)d_y, nullptr);
  for (size_t i = 0; i < sizeof(use) / sizeof(use[0]); ++i) *use[i].ptr = saved[i];
  HIPCHK(pb, e);
  return PFM_OK;
}

pfm_status pfm_matvec_mixed(pfm_problem* h, const void* d_psi, void* d_y) {
  if (!h || !d_psi || !d_y) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!pb.wave_ready) return fail(pb, PFM_ESTATE, "pfm_set_wave first");
  if (pb.opt.precision != PFM_MIXED) return fail(pb, PFM_ESTATE, "handle was not created with PFM_MIXED");
  HIPCHK(pb, apply_operator_mixed(pb, (const cd*)d_psi, (cd*)d_y));
  return PFM_OK;
}

pfm_status pfm_matvec_timed(pfm_problem* h, const void* d_psi, void* d_y, int reps, double* stage_ms,
                            double* total_ms) {
  if (!h || !d_psi || !d_y || reps < 1) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!pb.wave_ready) return fail(pb, PFM_ESTATE, "pfm_set_wave first");
  double acc[6] = {0, 0, 0, 0, 0, 0}, tot = 0.0;
  for (int r = 0; r < reps; ++r) {
    HIPCHK(pb, apply_operator(pb, (const cd*)d_psi, (cd*)d_y, pb.ev));
    HIPCHK(pb, hipEventSynchronize(pb.ev[6]));
    for (int s = 0; s < 6; ++s) {
      float ms = 0.f;
      HIPCHK(pb, hipEventElapsedTime(&ms, pb.ev[s], pb.ev[s + 1]));
      acc[s] += ms;
    }
    float all = 0.f;
    HIPCHK(pb, hipEventElapsedTime(&all, pb.ev[0], pb.ev[6]));
    tot += all;
  }
  if (stage_ms)
    for (int s = 0; s < 6; ++s) stage_ms[s] = acc[s] / reps;
  if (total_ms) *total_ms = tot / reps;
  return PFM_OK;
}

pfm_status pfm_matvec_stage_timed(pfm_problem* h, const void* d_psi, int stage, int reps, double* ms_per_launch) {
  if (!h || !d_psi || !ms_per_launch || stage < 0 || stage > 3 || reps < 1) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!pb.wave_ready) return fail(pb, PFM_ESTATE, "pfm_set_wave first");
  HIPCHK(pb, time_chain_stage(pb, (const cd*)d_psi, stage, reps, pb.ev[0], pb.ev[1]));
  HIPCHK(pb, hipEventSynchronize(pb.ev[1]));
  float ms = 0.f;
  HIPCHK(pb, hipEventElapsedTime(&ms, pb.ev[0], pb.ev[1]));
  *ms_per_launch = ms / reps;
  return PFM_OK;
}

pfm_status pfm_rhs(pfm_problem* h, void* d_b) {
  if (!h || !d_b) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!pb.wave_ready) return fail(pb, PFM_ESTATE, "pfm_set_wave first");
  HIPCHK(pb, launch_rhs(pb, pb.theta, (cd*)d_b));
  return PFM_OK;
}

}  // extern "C"

namespace {

struct GmresStats {
  int iters = 0, matvecs = 0;
  double rel = 1.0;              // true relative residual ||b - A x|| / ||b|| of the returned x
};

// Batched apply of the current batch: from the captured graph (fixed in/out
// buffers, copies around it) or launched kernel by kernel.
// Whether right preconditioning can run inside the apply: with the roots by
// Fourier modes the fibres' forward transforms are the only reader of the
// densities unless a fibre has tree work (cells below its root, down leaves)
// or there are stored near pairs (row tasks, batched P2P); then P^{-1} z is
// needed only as its spectrum, the mode blocks of P^{-1} times that of z.
bool pc_fusable(const Problem& pb) {
  return pb.spec_root && pb.n_mcells == 0 && pb.n_dleaves == 0 && pb.n_p2p_rowtasks == 0 && pb.n_p2p_items == 0;
}

hipError_t batch_apply(Problem& pb, const cd* in, cd* out) {
  if (!pb.graph) return apply_operator_batch(pb, in, out, nullptr);
  const size_t bytes = (size_t)pb.B * 2 * pb.E * sizeof(cd);
  hipError_t e = hipMemcpyAsync(pb.d_gin, in, bytes, hipMemcpyDeviceToDevice, pb.stream);
  if (e == hipSuccess) e = hipGraphLaunch(pb.graph, pb.stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, pb.d_gout, bytes, hipMemcpyDeviceToDevice, pb.stream);
  return e;
}

// Restarted GMRES(m) for B systems in lockstep (B = 1: a single system).
// apply(in, out) applies the B operators to B stacked vectors.  Every
// iteration is one apply and one fused CGS2 Arnoldi step for all members;
// the Hessenberg columns stay on the device and are read back two
// iterations at a time while the next two are already queued, so the host
// never waits on a single iteration.  The small least-squares problems
// (Givens rotations) are per member on the host.  A member stops taking part
// when its estimate meets the tolerance; the cycle ends when no member is
// left (a member may have up to three extra queued iterations, which are
// discarded).  Every cycle starts with the true residual b - A x, which also
// decides convergence.  Basis layout: V[(j * B + b) * n].
template <typename Apply>
pfm_status gmres_lockstep(Problem& pb, int B, Apply&& apply, const cd* b, cd* x, bool use_x0, double tol,
                          int max_iter, std::vector<GmresStats>& gs, std::vector<pfm_status>& st,
                          std::vector<int>* fallback = nullptr, const cd* aug = nullptr,
                          double* est_track = nullptr) {
  typedef std::complex<double> C;
  const int n = 2 * pb.E;
  const long long nb = (long long)n;
  const long long ldv = (long long)B * n;
  const int m = pb.opt.restart;
  const long long hs = 2 * m + 8;           // d_hcol stride per member
  const long long hs2 = 2 * m + 4;          // column stride per member in d_hall
  const int LOOK = 4;                        // iterations per read-back group
  cd* V = pb.d_V;
  cd* W = pb.d_w;
  cd* R = pb.d_r;
  cd* hc = pb.d_hcol;
  cd* hh = pb.h_hcol;
  gs.assign(B, GmresStats());
  st.assign(B, PFM_OK);
  std::vector<double> bnorm(B), beta(B);
  std::vector<char> done(B, 0), cyc(B, 0);
  std::vector<int> jj(B, 0);
  std::vector<C> Hm((size_t)B * (m + 1) * m), g((size_t)B * (m + 1)), cs((size_t)B * m), sn((size_t)B * m);
  std::vector<C> Hraw((size_t)B * (m + 1) * m);   // DCGS2: the Hessenberg matrix before the rotations
  auto sync_norms = [&](const cd* vec, std::vector<double>& out) -> hipError_t {
    hipError_t e = launch_dots_b(pb, B, vec, nb, nb, 1, vec, nb, n, hc, hs);
    if (e == hipSuccess) e = hipMemcpyAsync(hh, hc, (size_t)B * hs * sizeof(cd), hipMemcpyDeviceToHost, pb.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pb.stream);
    for (int i = 0; i < B; ++i) out[i] = std::sqrt(std::max(0.0, hh[i * hs].x));
    return e;
  };
  HIPCHK(pb, sync_norms(b, bnorm));
  if (!use_x0) HIPCHK(pb, hipMemsetAsync(x, 0, (size_t)B * n * sizeof(cd), pb.stream));
  // Augmented first cycle (aug != nullptr): minimise the residual over
  // span{u} + K_j(A, b) with u = aug.  With c = A u split as c = V g + c_perp
  // against the Arnoldi basis, the least-squares problem in (y, alpha) reduces,
  // after the Givens rotations of the Hessenberg matrix (also applied to g,
  // giving s), to the scalar alpha = conj(s_j1) t_j1 / (|s_j1|^2 + |c_perp|^2)
  // and the residual |t_j1| |c_perp| / sqrt(|s_j1|^2 + |c_perp|^2), never more
  // than the plain GMRES estimate |t_j1|.  c_perp is kept as a vector (each
  // new basis vector projected out, modified Gram-Schmidt) so that its norm
  // does not suffer the cancellation of ||c||^2 - ||g||^2.
  cd* Cv = pb.d_tmp;                             // c = A u
  cd* Cp = pb.d_cperp;                           // c_perp
  std::vector<double> cp2(B, 0.0);
  std::vector<C> sv((size_t)B * (m + 1)), alpha(B, 0.0);
  bool augmenting = aug != nullptr;
  if (augmenting) HIPCHK(pb, apply(aug, Cv));
  bool first = true;
  while (true) {
    // true residuals R = b - A x
    if (first && !use_x0) {
      HIPCHK(pb, hipMemcpyAsync(R, b, (size_t)B * n * sizeof(cd), hipMemcpyDeviceToDevice, pb.stream));
    } else {
      HIPCHK(pb, apply(x, W));
      for (int i = 0; i < B; ++i)
        if (!done[i]) ++gs[i].matvecs;
      HIPCHK(pb, hipMemcpyAsync(R, b, (size_t)B * n * sizeof(cd), hipMemcpyDeviceToDevice, pb.stream));
      HIPCHK(pb, launch_axpby(pb, R, mkc(-1, 0), W, mkc(1, 0), (long long)B * n));
    }
    HIPCHK(pb, sync_norms(R, beta));
    if (est_track && bnorm[0] > 0) *est_track = beta[0] / bnorm[0];
    if (first && use_x0 && fallback) {
      // a start vector that does not beat zero is replaced by zero
      for (int i = 0; i < B; ++i) {
        if (std::isfinite(beta[i]) && beta[i] < bnorm[i]) continue;
        (*fallback)[i] = 1;
        HIPCHK(pb, hipMemsetAsync(x + (size_t)i * n, 0, n * sizeof(cd), pb.stream));
        HIPCHK(pb, hipMemcpyAsync(R + (size_t)i * n, b + (size_t)i * n, n * sizeof(cd), hipMemcpyDeviceToDevice,
                                  pb.stream));
        beta[i] = bnorm[i];
      }
      HIPCHK(pb, launch_dots_b(pb, B, R, nb, nb, 1, R, nb, n, hc, hs));   // squared norms for V_0
    }
    first = false;
    bool all_done = true;
    for (int i = 0; i < B; ++i) {
      if (done[i]) continue;
      if (!std::isfinite(beta[i])) {
        st[i] = fail(pb, PFM_ENUMERIC, "non-finite residual norm");
        done[i] = 1;
        continue;
      }
      gs[i].rel = bnorm[i] > 0 ? beta[i] / bnorm[i] : 0.0;
      if (bnorm[i] == 0.0 || beta[i] / bnorm[i] <= tol) {
        done[i] = 1;
        continue;
      }
      if (gs[i].iters >= max_iter) {
        st[i] = fail(pb, PFM_ENOCONV, "GMRES stopped at relative residual " + std::to_string(gs[i].rel));
        done[i] = 1;
        continue;
      }
      all_done = false;
    }
    if (all_done) return PFM_OK;
    // V_0 = R / ||R|| per member (the squared norms are still in d_hcol)
    HIPCHK(pb, launch_normalize_b(pb, B, V, R, nb, hc, hs, n));
    if (augmenting) {
      // g_0 = v_0^H c, c_perp = c - g_0 v_0
      HIPCHK(pb, hipMemcpyAsync(Cp, Cv, (size_t)B * n * sizeof(cd), hipMemcpyDeviceToDevice, pb.stream));
      HIPCHK(pb, launch_project_out(pb, B, V, Cp, nb, n, hc, hc + 1, hs));
      HIPCHK(pb, hipMemcpyAsync(hh, hc, (size_t)B * hs * sizeof(cd), hipMemcpyDeviceToHost, pb.stream));
      HIPCHK(pb, hipStreamSynchronize(pb.stream));
      for (int i = 0; i < B; ++i) {
        sv[(size_t)i * (m + 1)] = C(hh[i * hs].x, hh[i * hs].y);
        cp2[i] = std::max(0.0, hh[i * hs + 1].x);
      }
    }
    int budget = 0;      // iterations any member may still take
    for (int i = 0; i < B; ++i) {
      cyc[i] = !done[i];
      jj[i] = 0;
      for (int r = 0; r <= m; ++r) g[(size_t)i * (m + 1) + r] = 0.0;
      g[(size_t)i * (m + 1)] = beta[i];
      if (cyc[i]) budget = std::max(budget, max_iter - gs[i].iters);
    }
    const int jmax = std::min(m, budget);
    // plain cycles orthogonalise with delayed reorthogonalisation (DCGS2: two
    // passes over the basis per step, column j final after step j + 1); the
    // augmented first cycle keeps CGS2 (four passes, column j final at once)
    const bool dcgs = !augmenting;
    auto enqueue = [&](int j) -> hipError_t {
      cd* Vj = V + (size_t)j * ldv;
      cd* Wj = V + (size_t)(j + 1) * ldv;
      hipError_t e = apply(Vj, Wj);
      if (e != hipSuccess) return e;
      if (dcgs) return launch_dcgs_step(pb, B, V, ldv, nb, j, Wj, nb, n, hs2);
      cd* hcol = pb.d_hall + (size_t)j * B * hs2;
      e = launch_arnoldi_step(pb, B, V, ldv, nb, j, Wj, nb, n, hcol, hs2);
      if (e != hipSuccess || !augmenting) return e;
      // g_{j+1} = v_{j+1}^H c_perp into slot 2j+3, c_perp -= g_{j+1} v_{j+1},
      // ||c_perp||^2 into slot 2j+4
      return launch_project_out(pb, B, Wj, Cp, nb, n, hcol + 2 * (j + 1) + 1, hcol + 2 * (j + 1) + 2, hs2);
    };
    auto readback = [&](int j0, int j1) -> hipError_t {
      return hipMemcpyAsync(pb.h_hall + (size_t)j0 * B * hs2, pb.d_hall + (size_t)j0 * B * hs2,
                            (size_t)(j1 - j0) * B * hs2 * sizeof(cd), hipMemcpyDeviceToHost, pb.stream);
    };
    int j_enq = 0, j_proc = 0, c_sched = 0;
    int grp = 0;
    hipEvent_t gev[2] = {pb.ev[14], pb.ev[15]};
    int gbeg[2] = {0, 0}, gend[2] = {0, 0};
    // Queue up to LOOK more steps and the read-back of the columns they make
    // final (DCGS2: one behind, all at the end of the cycle), as group `slot`.
    auto queue_group = [&](int slot) -> hipError_t {
      int stop = std::min(jmax, j_enq + LOOK);
      for (; j_enq < stop; ++j_enq) {
        hipError_t e = enqueue(j_enq);
        if (e != hipSuccess) return e;
      }
      if (dcgs && j_enq == jmax && jmax > 0) {
        hipError_t e = launch_dcgs_finish(pb, B, V, ldv, nb, jmax - 1, n, hs2);
        if (e != hipSuccess) return e;
      }
      const int c1 = std::max(c_sched, dcgs && j_enq < jmax ? j_enq - 1 : j_enq);
      gbeg[slot] = c_sched;
      gend[slot] = c1;
      if (c1 > c_sched) {
        // DCGS2 also needs the raw column c1 (the next step's a and gamma)
        hipError_t e = readback(c_sched, dcgs ? c1 + 1 : c1);
        if (e != hipSuccess) return e;
      }
      c_sched = c1;
      return hipEventRecord(gev[slot], pb.stream);
    };
    HIPCHK(pb, queue_group(0));
    bool any = true;
    while (j_proc < jmax && any) {
      // queue the next group before waiting for the current one
      int nxt = grp ^ 1;
      gbeg[nxt] = gend[nxt] = c_sched;
      if (j_enq < jmax) HIPCHK(pb, queue_group(nxt));
      HIPCHK(pb, hipEventSynchronize(gev[grp]));
      for (int j = gbeg[grp]; j < gend[grp] && any; ++j) {
        any = false;
        for (int i = 0; i < B; ++i) {
          if (!cyc[i]) continue;
          const cd* hv = pb.h_hall + ((size_t)j * B + i) * hs2;
          std::vector<C> col(j + 2);
          double hn;
          if (dcgs) {
            // raw step data of j and j + 1 -> column j of H (see launch_dcgs_step):
            // h = ((b, s) - H[0..j][0..j-1] a) / gamma, plus a' of step j + 1,
            // subdiagonal gamma' (u_{j+1} = w1 is not normalised)
            const cd* rn = pb.h_hall + ((size_t)(j + 1) * B + i) * hs2;
            const double gam = hv[2 * j + 1].x;
            const double gam1 = rn[2 * (j + 1) + 1].x;
            C* Hr = &Hraw[(size_t)i * (m + 1) * m];
            for (int r = 0; r <= j; ++r) {
              C gr = 0.0;
              for (int c = std::max(r - 1, 0); c < j; ++c) gr += Hr[(size_t)r * m + c] * C(hv[c].x, hv[c].y);
              const C br = r < j ? C(hv[j + r].x, hv[j + r].y) : C(hv[2 * j].x, hv[2 * j].y);
              const C hrj = (br - gr) / gam + C(rn[r].x, rn[r].y);
              Hr[(size_t)r * m + j] = hrj;
              col[r] = hrj;
            }
            hn = gam1;
            Hr[(size_t)(j + 1) * m + j] = hn;
          } else {
            for (int r = 0; r <= j; ++r) col[r] = C(hv[r].x + hv[j + 1 + r].x, hv[r].y + hv[j + 1 + r].y);
            hn = std::sqrt(std::max(0.0, hv[2 * (j + 1)].x));
          }
          if (!std::isfinite(hn)) {
            st[i] = fail(pb, PFM_ENUMERIC, "non-finite Arnoldi norm");
            cyc[i] = 0;
            done[i] = 1;
            continue;
          }
          col[j + 1] = hn;
          C* csi = &cs[(size_t)i * m];
          C* sni = &sn[(size_t)i * m];
          C* gi = &g[(size_t)i * (m + 1)];
          for (int r = 0; r < j; ++r) {
            C a = col[r], bb = col[r + 1];
            col[r] = csi[r] * a + sni[r] * bb;
            col[r + 1] = -std::conj(sni[r]) * a + csi[r] * bb;
          }
          C a = col[j], bb = col[j + 1];
          double t = std::sqrt(std::norm(a) + std::norm(bb));
          if (std::abs(a) == 0.0) {
            csi[j] = 0.0;
            sni[j] = 1.0;
            col[j] = bb;
          } else {
            C ph = a / std::abs(a);
            csi[j] = std::abs(a) / t;
            sni[j] = ph * std::conj(bb) / t;
            col[j] = ph * t;
          }
          gi[j + 1] = -std::conj(sni[j]) * gi[j];
          gi[j] = csi[j] * gi[j];
          for (int r = 0; r <= j; ++r) Hm[((size_t)i * (m + 1) + r) * m + j] = col[r];
          ++gs[i].iters;
          ++gs[i].matvecs;
          jj[i] = j + 1;
          double est = std::abs(gi[j + 1]) / bnorm[i];
          if (augmenting) {
            C* s_ = &sv[(size_t)i * (m + 1)];
            C gnew(hv[2 * (j + 1) + 1].x, hv[2 * (j + 1) + 1].y);
            cp2[i] = std::max(0.0, hv[2 * (j + 1) + 2].x);
            C a2 = s_[j];
            s_[j] = csi[j] * a2 + sni[j] * gnew;
            s_[j + 1] = -std::conj(sni[j]) * a2 + csi[j] * gnew;
            double den = std::norm(s_[j + 1]) + cp2[i];
            alpha[i] = den > 0 ? std::conj(s_[j + 1]) * gi[j + 1] / den : C(0.0);
            double r2 = den > 0 ? std::norm(gi[j + 1]) * cp2[i] / den : 0.0;
            est = std::sqrt(r2) / bnorm[i];
          }
          // the caller may read the residual estimate of member 0 (relative
          // to ||b||) when it queues the next applies
          if (est_track && i == 0) *est_track = est;
          if (est <= 0.7 * tol || gs[i].iters >= max_iter || hn == 0.0) cyc[i] = 0;
          any = any || cyc[i];
        }
        j_proc = j + 1;
      }
      grp ^= 1;
    }
    // drain what is still queued before the basis is used
    HIPCHK(pb, hipStreamSynchronize(pb.stream));
    // x_b += V_b y_b, y_b from the triangular systems (zeros past a member's jj)
    int cnt = 0;
    for (int i = 0; i < B; ++i) {
      cd* yv = hh + i * hs;
      for (int r = 0; r < m; ++r) yv[r] = mkc(0, 0);
      std::vector<C> y(jj[i]);
      for (int r = jj[i] - 1; r >= 0; --r) {
        C acc = g[(size_t)i * (m + 1) + r];
        if (augmenting) acc -= alpha[i] * sv[(size_t)i * (m + 1) + r];
        for (int l = r + 1; l < jj[i]; ++l) acc -= Hm[((size_t)i * (m + 1) + r) * m + l] * y[l];
        y[r] = acc / Hm[((size_t)i * (m + 1) + r) * m + r];
        yv[r] = mkc(y[r].real(), y[r].imag());
      }
      cnt = std::max(cnt, jj[i]);
    }
    if (cnt > 0) {
      HIPCHK(pb, hipMemcpyAsync(hc, hh, (size_t)B * hs * sizeof(cd), hipMemcpyHostToDevice, pb.stream));
      HIPCHK(pb, launch_gemv_acc_b(pb, B, x, nb, V, ldv, nb, cnt, hc, hs, n));
    }
    if (augmenting) {
      // x_b += alpha_b u_b, then plain restarts
      for (int i = 0; i < B; ++i) {
        C a = jj[i] > 0 ? alpha[i] : C(0.0);
        HIPCHK(pb, launch_axpby(pb, x + (size_t)i * n, mkc(a.real(), a.imag()), aug + (size_t)i * n, mkc(1, 0), n));
      }
      augmenting = false;
    }
  }
}

}  // namespace

extern "C" {

pfm_status pfm_solve(pfm_problem* h, const void* d_b_in, void* d_x_io, int use_x0, pfm_info* info) {
  if (!h || !d_x_io || use_x0 < 0 || use_x0 > 3) return PFM_EINVAL;
  Problem& pb = h->p;
  if (use_x0 == 3 && pb.opt.precision == PFM_MIXED)
    return fail(pb, PFM_EINVAL, "augmentation (use_x0 = 3) needs precision PFM_FP64");
  if (!pb.wave_ready) return fail(pb, PFM_ESTATE, "pfm_set_wave first");
  auto t0 = std::chrono::steady_clock::now();
  const int n = 2 * pb.E;
  cd* x = (cd*)d_x_io;
  cd* b = pb.d_b;
  if (d_b_in) HIPCHK(pb, hipMemcpyAsync(b, d_b_in, n * sizeof(cd), hipMemcpyDeviceToDevice, pb.stream));
  else HIPCHK(pb, launch_rhs(pb, pb.theta, b));
  auto apply64 = [&](const cd* in, cd* out) { return apply_operator(pb, in, out, nullptr); };
  GmresStats gs;
  pfm_status st = PFM_OK;
  int outer = 0;
  int fell_back = 0;
  int matvecs_low = 0;
  if (pb.opt.precision == PFM_MIXED) {
    // FP64 iterative refinement: r = b - A x with the FP64 apply, A d = r
    // solved by GMRES, x += d.  Inside GMRES the apply is relaxed (inexact
    // Krylov: Simoncini & Szyld 2003, Bouras & Fraysse 2005): an apply error
    // E_k at iteration k moves the final residual by about ||E_k|| ||y_k||,
    // and ||y_k|| shrinks with the residual r_{k-1}, so the FP64 operator is
    // used while the estimated residual (relative to ||B||) is above the
    // relaxation point and the complex64 near field after it.  The bound
    // alone would allow the switch near tol / 2^-22; the perturbed Arnoldi
    // steps then slow the convergence, and the default point 1e4 tol (capped
    // at 0.1) is where the measured iterations stay those of FP64.  The
    // restart residuals of GMRES and the refinement residual are always
    // FP64, so the returned residual is exact.
    auto apply32 = [&](const cd* in, cd* out) { return apply_operator_mixed(pb, in, out); };
    const double relax = pb.opt.inner_tol > 0 ? pb.opt.inner_tol : std::min(0.1, 1e4 * pb.opt.tol);
    cd* rr = pb.d_ir_r;
    cd* d = pb.d_ir_d;
    if (use_x0) {
      HIPCHK(pb, apply64(x, pb.d_w));
      ++gs.matvecs;
      HIPCHK(pb, hipMemcpyAsync(rr, b, n * sizeof(cd), hipMemcpyDeviceToDevice, pb.stream));
      HIPCHK(pb, launch_axpby(pb, rr, mkc(-1, 0), pb.d_w, mkc(1, 0), n));
    } else {
      HIPCHK(pb, hipMemsetAsync(x, 0, n * sizeof(cd), pb.stream));
      HIPCHK(pb, hipMemcpyAsync(rr, b, n * sizeof(cd), hipMemcpyDeviceToDevice, pb.stream));
    }
    cd* nn = pb.h_hcol;
    HIPCHK(pb, launch_dots(pb, b, n, 1, b, n, pb.d_hcol));
    HIPCHK(pb, launch_dots(pb, rr, n, 1, rr, n, pb.d_hcol + 1));
    HIPCHK(pb, hipMemcpyAsync(nn, pb.d_hcol, 2 * sizeof(cd), hipMemcpyDeviceToHost, pb.stream));
    HIPCHK(pb, hipStreamSynchronize(pb.stream));
    double bnorm = std::sqrt(std::max(0.0, nn[0].x)), rnorm = std::sqrt(std::max(0.0, nn[1].x));
    gs.rel = bnorm > 0 ? rnorm / bnorm : 0.0;
    const int max_outer = 30;
    while (true) {
      if (!std::isfinite(rnorm)) { st = fail(pb, PFM_ENUMERIC, "non-finite residual norm"); break; }
      if (bnorm == 0.0 || rnorm / bnorm <= pb.opt.tol) { st = PFM_OK; break; }
      if (gs.iters >= pb.opt.max_iter || outer >= max_outer) {
        st = fail(pb, PFM_ENOCONV, "refinement stopped at relative residual " + std::to_string(gs.rel));
        break;
      }
      // the inner solve aims at the outer tolerance; est is its residual
      // estimate relative to ||r||, so relative to ||B|| it is est ||r|| / ||B||
      const double tin = 0.5 * pb.opt.tol * bnorm / rnorm;
      const double scale = rnorm / bnorm;
      double est = 1.0;
      auto apply_in = [&](const cd* in, cd* out) -> hipError_t {
        // with the preconditioner the inner system is (I - A) P^{-1} z = r;
        // the relaxation test looks at the vector GMRES hands over (its own
        // iterate d gets the FP64 apply for the true residual)
        const cd* v = in;
        if (pb.opt.precond) {
          hipError_t e = launch_precond(pb, in, pb.d_pc_x, true);
          if (e != hipSuccess) return e;
          v = pb.d_pc_x;
        }
        if (in != d && est * scale <= relax) {
          ++matvecs_low;
          return apply32(v, out);
        }
        return apply64(v, out);
      };
      std::vector<GmresStats> gi;
      std::vector<pfm_status> sti;
      pfm_status si = gmres_lockstep(pb, 1, apply_in, rr, d, false, tin, pb.opt.max_iter - gs.iters, gi, sti,
                                     nullptr, nullptr, &est);
      if (pb.opt.precond) HIPCHK(pb, launch_precond(pb, d, d, true));      // d = P^{-1} z
      gs.iters += gi[0].iters;
      gs.matvecs += gi[0].matvecs;
      if (si != PFM_OK) { st = si; break; }
      if (sti[0] != PFM_OK && sti[0] != PFM_ENOCONV) { st = sti[0]; break; }
      HIPCHK(pb, launch_axpby(pb, x, mkc(1, 0), d, mkc(1, 0), n));
      HIPCHK(pb, apply64(x, pb.d_w));
      ++gs.matvecs;
      HIPCHK(pb, hipMemcpyAsync(rr, b, n * sizeof(cd), hipMemcpyDeviceToDevice, pb.stream));
      HIPCHK(pb, launch_axpby(pb, rr, mkc(-1, 0), pb.d_w, mkc(1, 0), n));
      HIPCHK(pb, launch_dots(pb, rr, n, 1, rr, n, pb.d_hcol));
      HIPCHK(pb, hipMemcpyAsync(nn, pb.d_hcol, sizeof(cd), hipMemcpyDeviceToHost, pb.stream));
      HIPCHK(pb, hipStreamSynchronize(pb.stream));
      rnorm = std::sqrt(std::max(0.0, nn[0].x));
      if (std::isfinite(rnorm)) gs.rel = rnorm / bnorm;
      ++outer;
    }
  } else {
    std::vector<GmresStats> g1;
    std::vector<pfm_status> s1;
    std::vector<int> fb(1, 0);
    if (pb.opt.precond) {
      // right preconditioning: GMRES for (I - A) P^{-1} z = B, then Psi = P^{-1} z;
      // the residual B - (I - A) P^{-1} z is that of Psi, so the stop test and
      // the reported residual are those of the unpreconditioned system.  A
      // start vector or an augmenting guess u enters as P u, since
      // (I - A) P^{-1} (P u) = (I - A) u.
      const bool fused = pc_fusable(pb);
      auto apply_pc = [&](const cd* in, cd* out) -> hipError_t {
        if (fused) {
          pb.pc_fused_inv = pb.d_pc_inv;
          hipError_t e = apply_operator(pb, in, out, nullptr);
          pb.pc_fused_inv = nullptr;
          return e;
        }
        hipError_t e = launch_precond(pb, in, pb.d_pc_x, true);
        if (e == hipSuccess) e = apply_operator(pb, pb.d_pc_x, out, nullptr);
        return e;
      };
      if (use_x0 == 3) {
        HIPCHK(pb, launch_precond(pb, x, pb.d_ir_aug, false));
        st = gmres_lockstep(pb, 1, apply_pc, b, x, false, pb.opt.tol, pb.opt.max_iter, g1, s1, nullptr,
                            pb.d_ir_aug);
      } else {
        if (use_x0) HIPCHK(pb, launch_precond(pb, x, x, false));     // z0 = P Psi0
        st = gmres_lockstep(pb, 1, apply_pc, b, x, use_x0 != 0, pb.opt.tol, pb.opt.max_iter, g1, s1,
                            use_x0 == 2 ? &fb : nullptr);
      }
      HIPCHK(pb, launch_precond(pb, x, x, true));
    } else if (use_x0 == 3) {
      HIPCHK(pb, hipMemcpyAsync(pb.d_ir_aug, x, n * sizeof(cd), hipMemcpyDeviceToDevice, pb.stream));
      st = gmres_lockstep(pb, 1, apply64, b, x, false, pb.opt.tol, pb.opt.max_iter, g1, s1, nullptr, pb.d_ir_aug);
    } else {
      st = gmres_lockstep(pb, 1, apply64, b, x, use_x0 != 0, pb.opt.tol, pb.opt.max_iter, g1, s1,
                          use_x0 == 2 ? &fb : nullptr);
    }
    gs = g1[0];
    if (st == PFM_OK) st = s1[0];
    fell_back = fb[0];
  }
  HIPCHK(pb, hipStreamSynchronize(pb.stream));
  auto t1 = std::chrono::steady_clock::now();
  if (info) {
    info->status = st;
    info->iters = gs.iters;
    info->matvecs = gs.matvecs;
    info->rel_residual = gs.rel;
    info->t_solve_s = std::chrono::duration<double>(t1 - t0).count();
    info->outer = outer;
    info->fallback = fell_back;
    info->matvecs_mixed = matvecs_low;
  }
  return st;
}

pfm_status pfm_precond_apply(pfm_problem* h, const void* d_in, void* d_out, int inverse) {
  if (!h || !d_in || !d_out || (inverse != 0 && inverse != 1)) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!pb.opt.precond) return fail(pb, PFM_ESTATE, "the handle was created with precond = 0");
  if (!pb.wave_ready) return fail(pb, PFM_ESTATE, "pfm_set_wave first");
  HIPCHK(pb, launch_precond(pb, (const cd*)d_in, (cd*)d_out, inverse != 0));
  return PFM_OK;
}

pfm_status pfm_solve_batch(pfm_problem* h, const void* d_b_in, void* d_x_io, int use_x0, pfm_info* infos) {
  if (!h || !d_x_io || use_x0 < 0 || use_x0 > 3) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!pb.batch_ready) return fail(pb, PFM_ESTATE, "pfm_set_batch first");
  auto t0 = std::chrono::steady_clock::now();
  const size_t n = 2 * (size_t)pb.E;
  cd* b = pb.d_b;
  if (d_b_in)
    HIPCHK(pb, hipMemcpyAsync(b, d_b_in, pb.B * n * sizeof(cd), hipMemcpyDeviceToDevice, pb.stream));
  else
    for (int i = 0; i < pb.B; ++i) HIPCHK(pb, launch_rhs(pb, pb.thetas[i], b + i * n));
  std::vector<GmresStats> gs;
  std::vector<pfm_status> st;
  auto apply = [&](const cd* in, cd* out) { return batch_apply(pb, in, out); };
  std::vector<int> fb(pb.B, 0);
  pfm_status s;
  if (pb.opt.precond) {
    // right preconditioning as in pfm_solve; the members share P (it does not
    // depend on the angle), and the preconditioner runs ahead of the
    // (possibly graph-replayed) batched apply
    cd* x = (cd*)d_x_io;
    // (a replayed graph holds its launches' arguments: it keeps the separate launch)
    const bool fused = !pb.graph && pc_fusable(pb);
    auto apply_pc = [&](const cd* in, cd* out) -> hipError_t {
      if (fused) {
        pb.pc_fused_inv = pb.d_pc_inv;
        hipError_t e = batch_apply(pb, in, out);
        pb.pc_fused_inv = nullptr;
        return e;
      }
      hipError_t e = launch_precond(pb, in, pb.d_pc_x, true, pb.B);
      if (e == hipSuccess) e = batch_apply(pb, pb.d_pc_x, out);
      return e;
    };
    if (use_x0 == 3) {
      HIPCHK(pb, launch_precond(pb, x, pb.d_ir_aug, false, pb.B));
      s = gmres_lockstep(pb, pb.B, apply_pc, b, x, false, pb.opt.tol, pb.opt.max_iter, gs, st, nullptr,
                         pb.d_ir_aug);
    } else {
      if (use_x0) HIPCHK(pb, launch_precond(pb, x, x, false, pb.B));
      s = gmres_lockstep(pb, pb.B, apply_pc, b, x, use_x0 != 0, pb.opt.tol, pb.opt.max_iter, gs, st,
                         use_x0 == 2 ? &fb : nullptr);
    }
    HIPCHK(pb, launch_precond(pb, x, x, true, pb.B));
  } else if (use_x0 == 3) {
    HIPCHK(pb, hipMemcpyAsync(pb.d_ir_aug, d_x_io, pb.B * n * sizeof(cd), hipMemcpyDeviceToDevice, pb.stream));
    s = gmres_lockstep(pb, pb.B, apply, b, (cd*)d_x_io, false, pb.opt.tol, pb.opt.max_iter, gs, st, nullptr,
                       pb.d_ir_aug);
  } else {
    s = gmres_lockstep(pb, pb.B, apply, b, (cd*)d_x_io, use_x0 != 0, pb.opt.tol, pb.opt.max_iter, gs, st,
                       use_x0 == 2 ? &fb : nullptr);
  }
  HIPCHK(pb, hipStreamSynchronize(pb.stream));
  double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  pfm_status worst = s;
  for (int i = 0; i < pb.B && i < (int)st.size(); ++i) {
    if (infos) {
      infos[i].status = st[i];
      infos[i].iters = gs[i].iters;
      infos[i].matvecs = gs[i].matvecs;
      infos[i].rel_residual = gs[i].rel;
      infos[i].t_solve_s = dt;
      infos[i].outer = 0;
      infos[i].fallback = fb[i];
      infos[i].matvecs_mixed = 0;
    }
    if (worst == PFM_OK && st[i] != PFM_OK) worst = st[i];
  }
  return worst;
}

pfm_status pfm_sweep(pfm_problem* h, int n_ka, const double* ka, int B, const double* theta, void* d_x,
                     pfm_info* infos) {
  if (!h || !ka || !theta || !d_x || n_ka < 0) return PFM_EINVAL;
  Problem& pb = h->p;
  const size_t n = 2 * (size_t)pb.E;
  pfm_status worst = PFM_OK;
  for (int i = 0; i < n_ka; ++i) {
    cd* x = (cd*)d_x + (size_t)i * B * n;
    pfm_info* inf = infos ? infos + (size_t)i * B : nullptr;
    pfm_status s = pfm_set_batch(h, ka[i], B, theta);
    if (s == PFM_EWOOD) {
      HIPCHK(pb, hipMemsetAsync(x, 0, B * n * sizeof(cd), pb.stream));
      if (inf)
        for (int b = 0; b < B; ++b) {
          inf[b] = pfm_info();
          inf[b].status = PFM_EWOOD;
        }
      if (worst == PFM_OK || worst == PFM_ENOCONV) worst = PFM_EWOOD;
      continue;
    }
    if (s != PFM_OK) return s;
    s = pfm_solve_batch(h, nullptr, x, 0, inf);
    if (s != PFM_OK && s != PFM_ENOCONV && s != PFM_ENUMERIC) return s;
    if (s != PFM_OK && worst == PFM_OK) worst = s;
  }
  HIPCHK(pb, hipStreamSynchronize(pb.stream));
  return worst;
}

pfm_status pfm_fields(pfm_problem* h, const void* d_psi, int n_orders, double* R, double* T, double* etc,
                      double* energy_residual) {
  if (!h || !d_psi || n_orders < 0 || n_orders > 255) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!pb.wave_ready) return fail(pb, PFM_ESTATE, "pfm_set_wave first");
  int no = 2 * n_orders + 1;
  HIPCHK(pb, launch_fields(pb, (const cd*)d_psi, n_orders, pb.d_fields));
  std::vector<cd> v(2 * no);
  HIPCHK(pb, hipMemcpyAsync(v.data(), pb.d_fields, 2 * no * sizeof(cd), hipMemcpyDeviceToHost, pb.stream));
  HIPCHK(pb, hipStreamSynchronize(pb.stream));
  double flux = 0.0;
  std::vector<std::complex<double>> Tn(no), gam(no);
  std::vector<double> kap(no);
  for (int i = 0; i < no; ++i) {
    int nn = i - n_orders;
    if (R) { R[2 * i] = v[2 * i].x; R[2 * i + 1] = v[2 * i].y; }
    if (T) { T[2 * i] = v[2 * i + 1].x; T[2 * i + 1] = v[2 * i + 1].y; }
    kap[i] = pb.k * std::sin(pb.theta) + 2.0 * PI * nn / pb.H;
    double g2 = pb.k * pb.k - kap[i] * kap[i];
    gam[i] = g2 >= 0 ? std::complex<double>(std::sqrt(g2), 0) : std::complex<double>(0, std::sqrt(-g2));
    Tn[i] = std::complex<double>(v[2 * i + 1].x, v[2 * i + 1].y) + (nn == 0 ? 1.0 : 0.0);
    if (g2 >= 0) {
      std::complex<double> Rn(v[2 * i].x, v[2 * i].y);
      flux += std::sqrt(g2) * (std::norm(Rn) + std::norm(Tn[i]));
    }
  }
  if (energy_residual) *energy_residual = flux / (pb.k * std::cos(pb.theta)) - 1.0;
  if (etc) {
    // (1/(kH)) int_0^H |du/dx1(L, x2)| dx2 on the modal expansion, trapezoid rule
    const int npts = 512;
    double s = 0.0;
    for (int t = 0; t < npts; ++t) {
      double x2 = t * pb.H / npts;
      std::complex<double> du = 0.0;
      for (int i = 0; i < no; ++i)
        du += std::complex<double>(0, 1) * gam[i] * Tn[i] *
              std::exp(std::complex<double>(0, 1) * (gam[i] * pb.L + kap[i] * x2));
      s += std::abs(du);
    }
    *etc = s * (pb.H / npts) / (pb.k * pb.H);
  }
  return PFM_OK;
}

pfm_status pfm_get_stats(const pfm_problem* h, pfm_stats* st) {
  if (!h || !st) return PFM_EINVAL;
  const Problem& pb = h->p;
  const HostPlan& hp = pb.hp;
  std::memset(st, 0, sizeof(*st));
  st->M = pb.M;
  st->N = pb.N;
  st->E = pb.E;
  st->n_unknowns = 2 * pb.E;
  st->n_cells = (int)hp.cells.size();
  st->n_leaves = (int)hp.leaves.size();
  st->depth = hp.depth;
  st->n_m2l_ext = (int)hp.m2l_src.size();
  st->n_m2l_int = (int)hp.m2li_src.size();
  st->n_near_pairs = (int)hp.near_src.size();
  st->n_near_entries = hp.n_near_entries;
  for (size_t q = 0; q < hp.near_src.size(); ++q)
    st->n_near_cols += hp.cells[hp.near_src[q]].eend - hp.cells[hp.near_src[q]].ebeg;
  st->n_root_offsets = (int)hp.root_off_xy.size() / 2;
  st->n_m2l_offsets = (int)hp.off_xy.size() / 2;
  st->near_bytes = 4.0 * 16.0 * (double)pb.n_near_stored;
  st->k = pb.k;
  st->k1 = pb.k1;
  st->eta = pb.eta;
  st->varrho = pb.varrho;
  st->theta = pb.theta;
  st->lattice_q = pb.lattice_q;
  st->p2p_split = pb.p2p_split;
  st->n_near_computed = pb.n_near_uniq;
  st->n_near_stored = pb.n_near_stored;
  st->n_near_circulant = pb.n_near_circ;
  st->p2p_window_leaves = pb.n_win_leaves;
  st->p2p_window_max = pb.p2p_wmax;
  st->lattice_m2l_grid = pb.lat_fft ? 1 : 0;
  st->workspace_bytes = (double)pb.ws_bytes;
  st->workspace_bound = pb.ws_bound ? 1 : 0;
  st->batch_capacity = pb.max_batch;
  st->n_device_allocs = pb.n_dev_allocs;
  st->device_alloc_bytes = pb.dev_alloc_bytes;
  st->self_fft = pb.self_fft ? 1 : 0;
  st->tree_on_device = pb.tree_on_device ? 1 : 0;
  st->spectral_roots = pb.spec_root ? 1 : 0;
  st->precond_in_apply = pb.opt.precond && pc_fusable(pb) ? 1 : 0;
  st->n_spectral_fibres = pb.spec_root ? pb.n_spec : 0;
  st->m2l_mfma_items = pb.n_mfma_items;
  st->m2l_vector_chunks = pb.n_vchunks;
  st->m2l_mfma_entries = pb.n_mfma_cols;
  return PFM_OK;
}


pfm_status pfm_test_plan_digest(const pfm_problem* h, unsigned long long* out) {
  if (!h || !out) return PFM_EINVAL;
  const HostPlan& hp = h->p.hp;
  Fnv d[8];
  for (const Cell& c : hp.cells) {
    d[0].add(c.cx); d[0].add(c.cy); d[0].add(c.half); d[0].add(c.rho);
    d[0].add(c.level); d[0].add(c.fiber); d[0].add(c.parent); d[0].add(c.first_child);
    d[0].add(c.n_child); d[0].add(c.ebeg); d[0].add(c.eend); d[0].add(c.leaf); d[0].add(c.leaf_index);
  }
  d[1].vec(hp.level_beg); d[1].vec(hp.elem_of); d[1].vec(hp.leaves); d[1].vec(hp.root_of_fibre);
  d[1].add(hp.depth);
  d[2].vec(hp.joff_xy); d[2].vec(hp.anc_ptr); d[2].vec(hp.anc); d[2].vec(hp.anc_off);
  d[3].vec(hp.up_cells); d[3].vec(hp.up_ptr); d[3].vec(hp.up_src); d[3].vec(hp.up_off);
  d[4].vec(hp.root_off_xy); d[4].vec(hp.root_off_mrange); d[4].vec(hp.root_pair_off);
  d[5].vec(hp.m2l_ptr); d[5].vec(hp.m2l_src); d[5].vec(hp.m2l_off); d[5].vec(hp.m2l_m); d[5].vec(hp.off_xy);
  d[6].vec(hp.m2li_ptr); d[6].vec(hp.m2li_src); d[6].vec(hp.m2li_off);
  d[7].vec(hp.near_ptr); d[7].vec(hp.near_src); d[7].vec(hp.near_m); d[7].vec(hp.near_tgt);
  d[7].vec(hp.near_blk); d[7].add(hp.n_near_entries); d[7].add(hp.m_min); d[7].add(hp.m_max);
  for (int i = 0; i < 8; ++i) out[i] = d[i].h;
  return PFM_OK;
}

pfm_status pfm_workspace_size(const pfm_problem* h, int batch, size_t* bytes) {
  if (!h || !bytes) return PFM_EINVAL;
  const Problem& pb = h->p;
  if (batch == 0) batch = pb.max_batch_create;
  if (batch < 1 || batch > pb.max_batch_create) return PFM_EINVAL;
  *bytes = ws_size(pb, batch);
  return PFM_OK;
}

pfm_status pfm_bind(pfm_problem* h, void* d_workspace, size_t bytes, void* hip_stream) {
  if (!h) return PFM_EINVAL;
  Problem& pb = h->p;
  int cap = pb.max_batch_create;
  if (d_workspace) {
    if (((uintptr_t)d_workspace & 255) != 0) return fail(pb, PFM_EINVAL, "workspace must be 256-byte aligned");
    while (cap >= 1 && ws_size(pb, cap) > bytes) --cap;
    if (cap < 1)
      return fail(pb, PFM_EINVAL, "workspace of " + std::to_string(bytes) + " bytes is below the " +
                                      std::to_string(ws_size(pb, 1)) + " bytes of one member");
  }
  // work queued on the old buffers ends first; then the wave or batch set up
  // in them (and a graph that holds their addresses) is dropped
  HIPCHK(pb, hipStreamSynchronize(pb.stream));
  HIPCHK(pb, hipStreamSynchronize(pb.side));
  drop_graph(pb);
  pb.wave_ready = false;
  pb.batch_ready = false;
  ws_release(pb);
  pb.ws_bound = false;
  pb.stream = (hipStream_t)hip_stream;
  void* base = d_workspace;
  if (!d_workspace) {
    HIPCHK(pb, dev_alloc(pb, &pb.ws_own, ws_size(pb, cap)));
    base = pb.ws_own;
  }
  HIPCHK(pb, ws_carve(pb, base, cap, pb.stream));
  pb.ws_bound = d_workspace != nullptr;
  return PFM_OK;
}

const char* pfm_last_error(const pfm_problem* h) { return h ? h->p.err.c_str() : "null handle"; }

void pfm_destroy(pfm_problem* h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  free_all(h->p);
  delete h;
}

pfm_status pfm_test_bessel(const double* d_x, int n, double* d_out) {
  if (!d_x || !d_out || n < 0) return PFM_EINVAL;
  if (launch_bessel_test(d_x, n, d_out, nullptr) != hipSuccess) return PFM_EDEVICE;
  if (hipDeviceSynchronize() != hipSuccess) return PFM_EDEVICE;
  return PFM_OK;
}

pfm_status pfm_test_lattice(pfm_problem* h, double* sums, double* offsets, int* mrange) {
  if (!h) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!pb.wave_ready) return fail(pb, PFM_ESTATE, "pfm_set_wave first");
  const HostPlan& hp = pb.hp;
  int n_roff = (int)hp.root_off_xy.size() / 2;
  int NT = 4 * pb.opt.p + 1;
  HIPCHK(pb, hipStreamSynchronize(pb.stream));
  if (sums) HIPCHK(pb, hipMemcpy(sums, pb.d_lat, (size_t)n_roff * NT * sizeof(cd), hipMemcpyDeviceToHost));
  if (offsets) std::memcpy(offsets, hp.root_off_xy.data(), hp.root_off_xy.size() * sizeof(double));
  if (mrange) std::memcpy(mrange, hp.root_off_mrange.data(), hp.root_off_mrange.size() * sizeof(int));
  return PFM_OK;
}

pfm_status pfm_test_moments(pfm_problem* h, const void* d_psi, double* moments, double* centres, int* levels,
                            int* elem_order) {
  if (!h || !d_psi) return PFM_EINVAL;
  Problem& pb = h->p;
  if (!pb.wave_ready) return fail(pb, PFM_ESTATE, "pfm_set_wave first");
  const HostPlan& hp = pb.hp;
  int nc = (int)hp.cells.size();
  int NP = 2 * pb.opt.p + 1;
  HIPCHK(pb, apply_upward(pb, (const cd*)d_psi));
  HIPCHK(pb, hipStreamSynchronize(pb.stream));
  if (moments) HIPCHK(pb, hipMemcpy(moments, pb.d_mpole, (size_t)nc * 2 * NP * sizeof(cd), hipMemcpyDeviceToHost));
  for (int i = 0; i < nc; ++i) {
    if (centres) { centres[2 * i] = hp.cells[i].cx; centres[2 * i + 1] = hp.cells[i].cy; }
    if (levels) {
      levels[4 * i] = hp.cells[i].level;
      levels[4 * i + 1] = hp.cells[i].fiber;
      levels[4 * i + 2] = hp.cells[i].ebeg;
      levels[4 * i + 3] = hp.cells[i].eend;
    }
  }
  if (elem_order) std::memcpy(elem_order, hp.elem_of.data(), hp.elem_of.size() * sizeof(int));
  return PFM_OK;
}

}  // extern "C"
