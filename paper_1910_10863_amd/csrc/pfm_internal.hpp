// Internal plan of the periodic FMM: tree, interaction lists, device buffers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pfmbem.h"
#include "pfm_math.hpp"

namespace pfm {

// One quadtree cell.  Cells of one fibre's tree are lattice-aligned squares:
// the root is the square of side a centred on the fibre (the basic tree of
// Sec. 3.1); children are quadrants.  rho is the tight radius: the largest
// distance from the centre to a chord end point of an element in the cell.
struct Cell {
  double cx, cy, half, rho;
  int level, fiber, parent;
  int first_child, n_child;   // children are contiguous after renumbering
  int ebeg, eend;             // range in the tree-ordered element list
  int leaf;                   // 1 for a leaf
  int leaf_index;             // index among leaves, or -1
};

struct M2LEntry { int tgt, src, off, m; };

// M2L entries are processed in chunks of at most this many entries of one (channel, cell)
constexpr int M2L_CHUNK = 1;
constexpr int M2L_LAT_CHUNK = 8;     // lattice entries of a root, for M >= 128 fibres
// largest padded fibre grid of the lattice M2L convolution (LDS per DFT;
// each axis at most 64 points)
constexpr int LAT_PXY_MAX = 1024;
// largest LDS window of a fibre's circulant rows that P2P stages per target
// leaf (entries; 4 components x 16 B each: 20 KB, so that four P2P
// workgroups still fit on a CU)
constexpr int P2P_WCAP = 320;
struct NearEntry { int tgt_leaf, src, m; };

struct HostPlan {
  std::vector<Cell> cells;              // level-major order
  std::vector<int> level_beg;           // cells of level l: [level_beg[l], level_beg[l+1])
  std::vector<int> elem_of;             // tree position -> natural element id
  std::vector<int> leaves;              // leaf cell ids
  std::vector<int> root_of_fibre;       // [M]
  // M2L (exterior, all images) and interior (same fibre, m = 0) lists, CSR by target cell
  std::vector<int> m2l_ptr, m2l_src, m2l_off, m2l_m;
  std::vector<int> m2li_ptr, m2li_src, m2li_off;
  std::vector<double> off_xy;           // unique M2L translation vectors [n_off][2]
  std::vector<double> joff_xy;          // unique leaf-to-ancestor offsets O_L - O_A [n_joff][2]
  std::vector<int> up_cells, up_ptr, up_src, up_off;   // per non-leaf cell: leaves below it
  std::vector<int> anc_ptr, anc, anc_off;              // per leaf: its ancestors
  // P2P near lists, CSR by target leaf
  std::vector<int> near_ptr, near_src, near_m, near_tgt;
  std::vector<long long> near_blk;      // block offset (entries) of each near pair
  long long n_near_entries = 0;
  // top-level lattice M2L
  std::vector<double> root_off_xy;      // unique fibre offsets [n_roff][2]
  std::vector<int> root_off_mrange;     // [n_roff][2]: explicit images m_lo..m_hi
  std::vector<int> root_pair_off;       // [M*M]: offset id of (target i, source j)
  int depth = 0;
  int m_min = 0, m_max = 0;             // image range used by explicit entries
};

struct Problem {
  // inputs
  int lattice = 0;
  double a = 1.0;
  int ML = 1, MH = 1, M = 1, N = 8, E = 8;
  int shape = PFM_CIRCLE;               // boundary curve of every fibre (pfm_shape)
  std::vector<double> radii, centres;   // [M] size parameters, [M][2]
  double L = 1.0, H = 1.0;
  double rho_f = 1, c_f = 1, rho_m = 1, c_m = 1, eta_user = 0;
  pfm_options opt{};
  // current wave (one angle) or batch (B angles at one frequency)
  bool wave_ready = false;
  bool batch_ready = false;
  int max_batch = 1;                    // capacity of the per-member buffers
  int B = 0;                            // members of the current batch
  std::vector<double> thetas;           // their incidence angles
  double k = 0, k1 = 0, eta = 0, varrho = 0, theta = 0, beta = 0;
  int lattice_q = 0;

  hipStream_t stream = nullptr;
  std::string err;
  HostPlan hp;

  // device buffers -----------------------------------------------------
  // elements (natural order), SoA
  double *d_centres = nullptr, *d_radii = nullptr;
  double *d_mx = nullptr, *d_my = nullptr, *d_tx = nullptr, *d_ty = nullptr, *d_h = nullptr;
  double *d_gl = nullptr;               // far-rule nodes [g_far], weights [g_far]
  double *d_gl16 = nullptr;             // near-rule nodes [16], weights [16]
  int *d_elem_of = nullptr;
  int *d_psi_idx = nullptr;             // tree position -> index of phi in Psi
  // cells
  double *d_cx = nullptr, *d_cy = nullptr;
  int *d_ebeg = nullptr, *d_eend = nullptr, *d_first_child = nullptr, *d_n_child = nullptr;
  int *d_cell_joff = nullptr, *d_parent = nullptr, *d_leaves = nullptr, *d_root_of_fibre = nullptr;
  int *d_fibre_of_cell = nullptr;
  // lists
  int *d_m2l_ptr = nullptr, *d_m2l_src = nullptr, *d_m2l_off = nullptr, *d_m2l_m = nullptr;
  int *d_m2li_ptr = nullptr, *d_m2li_src = nullptr, *d_m2li_off = nullptr;
  int *d_near_ptr = nullptr, *d_near_src = nullptr, *d_near_m = nullptr, *d_near_tgt = nullptr;
  long long *d_near_blk = nullptr;      // block offset (entries) of each stored near pair in d_near
  long long *d_leaf_blk = nullptr;      // per leaf: offset of its stored region
  long long n_near_stored = 0;          // element pairs stored in d_near
  long long n_near_circ = 0;            // element pairs taken from the circulant rows
  bool p2p_on_side = false;             // overlapped apply: P2P on the side stream, the chain on the caller's
  int *d_ccols_ptr = nullptr;           // per leaf: range of its circulant source columns
  int *d_ccol_psi = nullptr;            // circulant source columns: index of phi in Psi
  int *d_ccol_loc = nullptr;            // circulant source columns: element index on its circle
  int *d_cwin = nullptr;                // per leaf: [rotation, first row entry, entries] of its LDS window
  // root lattice M2L as a convolution over the fibre grid: fibre f sits at
  // (sublattice, gx, gy); a root pair's lattice row depends only on the two
  // sublattices and the grid displacement; DFTs over the zero-padded
  // lat_px x lat_py grid
  bool lat_fft = false;
  int lat_ns = 1, lat_gx = 1, lat_gy = 1, lat_px = 2, lat_py = 2;
  int* d_lat_cell = nullptr;            // [ns][gy][gx]: root cell at the grid point (-1: none)
  int* d_lat_slot = nullptr;            // [ns][gy][gx]: M2L partial slot of that root (-1: none)
  int* d_lat_key = nullptr;             // [ns][ns][2gy-1][2gx-1]: lattice row of the displacement (-1: none)
  cd* d_lat_shat = nullptr;             // [member][ns][ns][px py][4p+1]: DFT of the rows over the grid
  cd* d_lat_xhat = nullptr;             // [member][ns][px py][2p+1]: DFT of the root multipoles
  cd* d_lat_lhat = nullptr;             // [member][ns][px py][2p+1]: their product, before the inverse DFT
  int p2p_wmax = 0, n_win_leaves = 0;   // largest window; leaves with a window
  cd *d_circ = nullptr;                 // [fibre][B11, B12, B21, B22][2N] circulant near rows
  // block-Jacobi preconditioner (options.precond): for each fibre and Fourier
  // mode kappa of the element index, the 2x2 block of P and of P^{-1}
  cd *d_pc_fwd = nullptr, *d_pc_inv = nullptr;   // [fibre][kappa][4]
  // right preconditioning inside the apply: P^{-1}'s mode blocks while a
  // preconditioned GMRES applies its operator, nullptr otherwise (see
  // pc_fusable)
  const cd* pc_fused_inv = nullptr;
  cd *d_pc_tw = nullptr;                // [N]: exp(2 pi i j / N)
  cd *d_pc_x = nullptr;                 // [2 M N]: P^{-1} v inside the preconditioned apply
  int pc_logN = 0;
  // equal fibres: target leaves with the same near region (same place in
  // their fibres, same sources at the same offsets and images) read one
  // stored region; inside a stored region, pairs equal to an earlier pair are
  // computed once and copied
  int *d_near_uniq = nullptr;           // stored pair ids whose blocks are computed
  long long *d_near_cp_src = nullptr, *d_near_cp_dst = nullptr;   // block offsets (entries)
  int *d_near_cp_len = nullptr;         // complex values per copied block
  int n_near_uniq = 0, n_near_copies = 0;
  int *d_cols_ptr = nullptr;            // per leaf: range of its flattened near source columns
  int *d_col_psi = nullptr;             // flattened near source columns: index of phi in Psi
  int *d_col_m = nullptr;               // image index m of each flattened near source column
  int *d_root_pair_off = nullptr, *d_root_mrange = nullptr;
  double *d_off_xy = nullptr, *d_joff_xy = nullptr, *d_root_off_xy = nullptr;
  // per-wave data
  cd *d_near = nullptr;                 // near blocks, complex128
  float2 *d_near32 = nullptr;           // near blocks, complex64 (PFM_MIXED)
  cd *d_ir_r = nullptr, *d_ir_d = nullptr;   // refinement residual and correction
  cd *d_ir_aug = nullptr;               // augmentation vectors of the first GMRES cycle [member][2E]
  cd *d_cperp = nullptr;                // their images A u with the Krylov basis projected out
  cd *d_htab = nullptr;                 // [2 ch][n_tab][4p+1]
  cd *d_jtab = nullptr;                 // [2 ch][n_joff][4p+1]
  cd *d_lat = nullptr;                  // = d_htab + n_off rows: lattice sums [n_roff][4p+1]
  // M2L work split into chunks of at most M2L_CHUNK entries of one (cell, channel);
  // exterior entries of a root cell include one lattice entry per source fibre
  int *d_e_src = nullptr, *d_e_off = nullptr, *d_e_m = nullptr;
  int *d_chunks = nullptr;              // [n_chunks][4]: cell, channel, first entry chunk, chunk count (one per (ch, cell) with entries)
  int *d_cc_ptr = nullptr;              // [2*n_cells+1]: chunks of (channel, cell)
  cd *d_part = nullptr;                 // [n_chunks][2p+1] M2L sums of each (channel, cell)
  int n_chunks = 0;
  int *d_mchunks = nullptr;             // [n_mchunks][4]: cell, channel, first entry, count (<= M2L_CHUNK entries)
  int n_mchunks = 0;
  cd *d_epart = nullptr;                // [n_mchunks][2p+1] M2L result of each entry chunk
  int *d_vchunks = nullptr;             // the chunks k_m2l takes (vector ALU)
  int n_vchunks = 0;
  int *d_mfma_items = nullptr;          // [item][4]: channel, table row, first column, columns (<= 16)
  int *d_mfma_cols = nullptr;           // [column][4]: source cell, partial slot (chunk), image, 0
  int n_mfma_items = 0, n_mfma_cols = 0;
  int n_cu = 0;                         // compute units of the device
  int p2p_grid = 0;                     // workgroups of the P2P launch (0: one per work item)
  int p2p_split = 1;                    // column splits per target leaf
  int p2p_unroll = 1;                   // source columns in flight per P2P wavefront
  int* d_p2p_items = nullptr;           // self_fft: the target leaves with stored near columns
  int n_p2p_items = 0;
  int* d_p2p_rowtasks = nullptr;        // self_fft: per row of those leaves (phi index, first column,
                                        // columns, rows of the leaf)
  long long* d_p2p_rowoff = nullptr;    // and the entry offset of the row in the leaf's block region
  int n_p2p_rowtasks = 0;
  int* d_leaf_near_t0 = nullptr;        // per leaf: its first row task (-1: none)
  cd* d_near_rows = nullptr;            // [task][2] the row tasks' sums (one wave)
  // fibre roots by their Fourier modes (spec_root: with the own blocks by
  // FFT).  Every fibre's root moments come from the DFTs of its densities
  // and its root's local expansion is evaluated at its midpoints by a
  // synthesis over the orders; a spectral fibre (none of its cells below the
  // root in an M2L entry, none of its elements in a near pair) needs nothing
  // else; the others (tree fibres) keep P2M at their leaves, M2M into their
  // cells below the root and the downward pass of those cells' expansions.
  bool spec_root = false;
  int n_spec = 0;                       // spectral fibres
  cd* d_spec_tab = nullptr;             // [M][4][2p+1] per frequency
  cd* d_spec_hat = nullptr;             // [member][M][2N] spectrum of P psi between the own-block launches
  int n_mcells = 0;                     // the tree fibres' cells below their roots (P2M from weights)
  int *d_mcell = nullptr;               // [n_mcells][4]: cell, first row (tree order), rows, first table row
  cd* d_p2m_tab = nullptr;              // [table rows][p+1][2] the cells' P2M weights, per frequency
  cd* d_l2p_tab = nullptr;              // [down-leaf rows][p+2]: Jp_n(kap (x_e - O_leaf)), n = 0..p+1, per frequency
  int n_dleaves = 0;                    // tree fibres' leaves with a far part from below the root or near rows
  int *d_dptr = nullptr;                // [M + 1]: those leaves of fibre f are dptr[f] .. dptr[f + 1]
  int *d_dldesc = nullptr;              // [leaf][8]: first row, rows, own M2L chunks (first, count),
                                        // ancestor range in d_danc, first near row task (-1: none), 0
  int *d_danc = nullptr;                // [ancestor][4]: M2L chunks (first, count), J-table row, 0 (no root)
  int *d_spec_rng = nullptr;            // [M][2]: the root's M2L chunks (first, count)
  cd *d_p2ppart = nullptr;              // [split][member][2E] partial near rows (split > 1)
  // upward: per non-leaf cell the leaves below it; downward: per leaf its
  // ancestors; both with an index into the J translation table
  int *d_up_cells = nullptr, *d_up_ptr = nullptr, *d_up_src = nullptr, *d_up_off = nullptr;
  int n_up = 0;
  // P2M and downward pass, per leaf: [row begin, rows, own M2L sum row per channel,
  // ancestor range per channel] (8 ints), the ancestors' (M2L sum row, leaf
  // offset) pairs, and the targets' (x - O, y - O, tx, ty) in row order
  int *d_ldesc = nullptr, *d_lanc = nullptr;
  double *d_tgeo = nullptr, *d_trh = nullptr;   // [E][4] target geometry, [E] chord length, row order
  cd *d_far = nullptr;                  // far part of the rows, Psi order
  int n_tab = 0;                        // rows per channel of d_htab: M2L offsets, then lattice offsets
  cd *d_alpha = nullptr;                // alpha^m, m = m_min..m_max, per batch member
  cd *d_alpha_one = nullptr;            // ones: phase-free near blocks
  double *d_srule = nullptr;            // lattice tail rule: nodes, weights
  int n_srule = 0;
  double *d_betas = nullptr;            // k H sin(theta) per batch member
  double *d_thetas = nullptr;           // incidence angles per batch member (modal transforms)
  cd *d_latpart = nullptr;              // tail partial sums [member][offset][rule block][4p+1]
  // expansions
  cd *d_mpole = nullptr;                // [n_cells][2][2p+1]
  // GMRES workspace
  cd *d_V = nullptr;                    // [restart+1][n]
  cd *d_w = nullptr, *d_r = nullptr, *d_b = nullptr, *d_tmp = nullptr;
  cd *d_red = nullptr;                  // reduction partials
  double *d_npart = nullptr;            // per-block squared norms [member][block]
  cd *d_dcoef = nullptr;                // DCGS2 update coefficients [member][2 restart + 4]
  cd *d_hall = nullptr, *h_hall = nullptr;   // Arnoldi columns [restart][member][2 restart + 4]
  cd *d_hcol = nullptr;                 // column of dots
  cd *h_hcol = nullptr;                 // pinned host copy
  int red_blocks = 0;
  // fields
  cd *d_fields = nullptr;
  hipEvent_t ev[16];
  bool events = false;
  hipStream_t side = nullptr;           // FMM chain runs here, concurrent with P2P
  hipEvent_t ev_fork, ev_join;
  // batched solves: captured apply of the current batch (fixed in/out buffers)
  hipStream_t cap = nullptr;
  hipGraphExec_t graph = nullptr;
  cd *d_gin = nullptr, *d_gout = nullptr;

  // Workspace: the device buffers whose contents are per frequency or per
  // call (near blocks, circulant rows, tables, lattice sums, expansions, M2L
  // partials, far part, GMRES basis and vectors, reduction scratch).  Each
  // slot is fixed + per_member * (batch capacity) bytes, 256-byte aligned,
  // carved in registration order from one block that the library allocates
  // at create or that the caller binds (pfm_bind).  Plan metadata (elements,
  // tree, lists, rules) stays library-owned.
  struct WsSlot {
    void** ptr;
    size_t fixed, per_member;
    bool zero;                          // cleared when (re)carved
  };
  std::vector<WsSlot> ws;
  void* ws_own = nullptr;               // library-owned block (nullptr while a caller's block is bound)
  void* ws_base = nullptr;              // block the slots point into
  size_t ws_bytes = 0;                  // its size in use
  bool ws_bound = false;                // the caller's block is bound
  int max_batch_create = 1;             // max_batch of pfm_create (upper bound of any binding)
  long long n_dev_allocs = 0;           // device allocations made by the library so far
  double dev_alloc_bytes = 0;
  // each fibre's own image-0 block (both wavenumbers, near and far pairs)
  // applied by FFT as a block-circulant operator; the tree holds only the
  // pairs between fibres and with images, and only the exterior channel
  bool self_fft = false;
  // spectral Nystrom discretisation (PFM_NYSTROM): nodes as points, trapezoid
  // weights as lengths, each fibre's own block from Kress's quadrature
  bool nystrom = false;
  double *d_kress = nullptr;            // [N] logarithmic weights R(2 pi d / N)
  bool tree_on_device = false;          // the plan was built by the GPU kernels
  int device = 0;                       // the GPU the handle was created on
  void* static_scratch = nullptr;       // that GPU's address of the fixed scratch array (pfm_matvec_static)
};

bool build_host_plan(Problem& pb, const std::vector<double>& mid, const std::vector<double>& ends);
// The same plan built by GPU kernels from the device copies of the element
// midpoints (natural order) and chord end points [E][4]; false with the
// reason when the build does not apply (more than 4096 elements per fibre, a
// level of one fibre's tree with more than 512 cells) or fails.
bool build_device_plan(Problem& pb, const double* d_mx, const double* d_my, const double* d_ends, std::string& why);
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

}  // namespace pfm

// the opaque handle of the C interface
struct pfm_problem {
  pfm::Problem p;
};
