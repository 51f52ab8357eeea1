/*
 * pfmbem: periodic fast-multipole boundary element method for 2D acoustic
 * transmission through periodic fibre media, on AMD MI355X (gfx950).
 *
 * Operation (Meng & Liu, "A periodic FM-BEM for solving the acoustic
 * transmission problems in periodic media", Sec. 2 and 3):
 *   A fundamental block of M = M_L x M_H fibres, periodic along y with period
 *   H = M_H * a (eq. 3), quasi-periodic phase alpha = exp(i k H sin(theta)).
 *   Each fibre boundary is cut into N straight chord elements with constant
 *   densities and midpoint collocation.  The unknowns are the double-layer
 *   density phi and the single-layer density varphi of the Kress
 *   representation (eqs. 4-5), ordered per fibre as in eq. (9):
 *       Psi = (phi_1[N], varphi_1[N], ..., phi_M[N], varphi_M[N]),
 *   2*M*N complex128 values (interleaved re, im; 16 bytes each).
 *   The library applies and solves (I - A) Psi = B of eq. (9), where the
 *   exterior operators carry the infinite image sum (eqs. 7-8), by a fast
 *   multipole method: quadtree per fibre, multipole moments with J_n, M2L
 *   with H_n (Graf, eq. 10-13), and all far images folded into the top-level
 *   local expansion by lattice sums (Sec. 3.3).
 *
 * Units: k = ka / a is the matrix wavenumber, k1 = k c_matrix / c_fibre the
 * fibre wavenumber, varrho = rho_matrix / rho_fibre (eq. 6); theta is the
 * incidence angle from +x, in radians; u_inc = exp(i k x.(cos th, sin th)).
 *
 * Conventions: every pointer argument named d_* is DEVICE memory owned by
 * the caller (for example a torch tensor's data_ptr()); host arrays are
 * owned by the caller as well.  The library allocates device memory only in
 * pfm_create (plan metadata and, until the caller binds a block of its own
 * with pfm_bind, the workspace) and frees it in pfm_destroy; no other call
 * allocates.  All work is queued on the stream given to
 * pfm_set_stream (default: the null stream); calls that return host values
 * synchronise that stream.  Functions return PFM_OK or an error code; the
 * message of the last error of a handle is returned by pfm_last_error.
 * A handle is not thread-safe.
 */
#ifndef PFMBEM_H
#define PFMBEM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pfm_problem pfm_problem;

typedef enum {
  PFM_OK = 0,
  PFM_EINVAL = 1,       /* invalid argument (sizes, overlap, unsupported p) */
  PFM_ENOMEM = 2,       /* device or host allocation failed */
  PFM_EDEVICE = 3,      /* HIP runtime error */
  PFM_ENOCONV = 4,      /* GMRES did not reach the tolerance; best iterate written */
  PFM_EWOOD = 5,        /* too close to a Wood anomaly k H (1 +- sin th) = 2 pi n */
  PFM_ENUMERIC = 6,     /* NaN/Inf in a residual norm */
  PFM_ESTATE = 7        /* call order (e.g. matvec before pfm_set_wave) */
} pfm_status;

typedef enum { PFM_SQUARE = 0, PFM_HEXAGON = 1 } pfm_lattice;

/* Arithmetic of the operator apply inside the solver.  PFM_FP64: everything in
 * FP64.  PFM_MIXED: the near field (P2P, the bulk of the bytes) is stored as
 * complex64 (densities and sums FP64) inside FP64 iterative refinement; the
 * far-field expansions, lattice sums, self/near element integrals, GMRES
 * orthogonalisation and the refinement residual stay FP64.  The inner GMRES
 * applies the FP64 operator while its residual estimate (relative to ||B||)
 * is above the relaxation point inner_tol and the complex64 near field below
 * it (an inexact Krylov method: late applies may be less accurate). */
typedef enum { PFM_FP64 = 0, PFM_MIXED = 1 } pfm_precision;

/* Fibre lattice (Sec. 2, Fig. 1).  Square: fibre (col i, row j) centred at
 * ((i+1/2)a, (j+1/2)a).  Hexagon: ((i+1/2)(sqrt3/2)a, (j+1/2+(i mod 2)/2)a).
 * Fibre index f = j*M_L + i.  radii: host array of M size parameters r_f, or
 * NULL to use r0 for every fibre.  Boundary nodes c_f + gamma(r_f, t_e),
 * t_e = 2 pi e/N, counter-clockwise, with the curve gamma of `shape`:
 *   PFM_CIRCLE        r (cos t, sin t)
 *   PFM_ROUND_SQUARE  r ((3 + 2 sin^2 t) cos t, (3 + 2 cos^2 t) sin t), the
 *                     round-square scatterer of Sec. 4 (area 23 pi r^2 / 2,
 *                     farthest point 4 r from the centre, on the diagonals).
 * Fibres may not touch: twice the farthest distance of the curve from its
 * centre must stay below a.  Non-circular fibres keep every near pair as a
 * stored block (their chords are not rotations of each other), so the
 * circulant self rows, self_mode 0 and precond = 1 need PFM_CIRCLE. */
typedef enum { PFM_CIRCLE = 0, PFM_ROUND_SQUARE = 1 } pfm_shape;

/* Discretisation of the boundary integral equations of Sec. 2 (eqs. 6-9).
 * PFM_CHORDS: N straight chords per fibre between the nodes, constant
 * densities collocated at the chord midpoints, Gauss-Legendre rules on the
 * chords with exact integrals for the self and neighbouring elements (the
 * element method).  PFM_NYSTROM: the spectral Nystrom method of Kress (the
 * paper's refs. 2 and 4): densities at the N nodes t_e = 2 pi e / N of the
 * parametrisation, the trapezoidal rule for the smooth kernels (other fibres,
 * periodic images), and for each fibre's own operators Kress's logarithmic
 * splitting with the hypersingular operator by Maue's identity and
 * trigonometric differentiation; it converges exponentially in N where the
 * element method converges at first order.  PFM_NYSTROM needs PFM_CIRCLE
 * fibres with N a power of two, 8 <= N <= 512 (each fibre's own block is
 * applied by FFT: self_mode 0 or 2, store_self_blocks 0); g_far is taken as
 * 1 (the point rule at the nodes). */
typedef enum { PFM_CHORDS = 0, PFM_NYSTROM = 1 } pfm_discretisation;

/* Shape of each fibre's basic tree (Sec. 3.1).  PFM_TREE_SQUARE: the root is
 * the square of side a centred on the fibre, cut into quadrants.
 * PFM_TREE_TRIANGLE (hexagonal lattice only, Fig. 5): the root is the
 * fibre's hexagonal lattice cell (inradius a/2), cut into six equilateral
 * triangles, each cut into four by its edge midpoints; cell centres are the
 * centroids.  An element belongs to the cell holding its midpoint (node for
 * PFM_NYSTROM).  The admissibility test is the same radius test on either
 * tree.  The triangle tree is built on the host (pfm_stats.tree_on_device
 * is 0). */
typedef enum { PFM_TREE_SQUARE = 0, PFM_TREE_TRIANGLE = 1 } pfm_tree_shape;

typedef struct {
  int lattice;
  double a;
  int M_L, M_H;
  int n_elem;              /* N, elements per fibre, >= 8 */
  const double* radii;     /* host, M entries, or NULL */
  double r0;
  int shape;               /* pfm_shape */
} pfm_geometry;

/* Materials: fibre (rho_1, c_1), matrix (rho_2, c_2).  eta is the real
 * coupling constant of eqs. (4)-(5); eta <= 0 selects eta = k. */
typedef struct {
  double rho_fiber, c_fiber, rho_matrix, c_matrix;
  double eta;
} pfm_material;

/* Method settings.
 *  p          expansion truncation -p..p; one of 8, 12, 16, 20, 24, 32, 40
 *  leaf_max   maximum elements per quadtree leaf, 1..64
 *  mac        admissibility ratio: cells D, C interact by M2L when
 *             rho_D + rho_C <= mac * |O_D - O_C - m h|, 0 < mac < 1
 *  g_far      Gauss-Legendre points per element for the far rule (4)
 *  restart    GMRES restart length m (1..200); max_iter total iterations
 *  tol        GMRES stop: true relative residual ||B - (I-A)Psi|| / ||B||
 *  wood_margin  reject (PFM_EWOOD) when the distance of k H (1 +- sin th)/(2 pi)
 *             to an integer is below this; 0 disables the check
 *  precision  PFM_FP64 or PFM_MIXED (see pfm_precision)
 *  inner_tol  PFM_MIXED: relaxation point, the relative residual below which the
 *             inner GMRES applies the complex64 near field (<= 0 or >= 1:
 *             min(0.1, 1e4 tol), where the measured GMRES iterations stay
 *             those of the FP64 solve)
 *  max_batch  capacity of the batched calls: angles per frequency (0 -> 1, at
 *             most PFM_MAX_BATCH); per-member buffers are sized for it
 *  use_graph  batched solves replay the batched apply from a captured HIP
 *             graph (1) or launch it kernel by kernel (0)
 *  p2p_blocks_per_cu  workgroups per compute unit of the persistent P2P
 *             launch (0: 3 when most near pairs use circulant rows, else 2;
 *             at most 8)
 *  p2p_unroll  source columns whose block entries a P2P wavefront keeps in
 *             flight at once: 1, 2 or 4 (0: 4 with self_mode 0 in effect, else 1)
 *  store_self_blocks  0: near pairs of a fibre with itself (image 0) use one
 *             circulant row per fibre (the N chords of a circle are rotations
 *             of each other, so their 2x2 block depends only on the index
 *             difference mod N); 1: every near pair is a stored block
 *  p2p_cached_rows  0: for each target leaf, P2P copies the window of its
 *             fibre's circulant rows that the leaf reads (at most 320 entries)
 *             into LDS once; 1: every row entry is read through the caches.
 *             Both give the same sums in the same order.
 *  direct_lattice_m2l  0: from 128 fibres up, the root lattice M2L (Sec. 3.3)
 *             runs as a convolution over the fibre grid (a root pair's lattice
 *             sum depends only on the grid displacement and, on the hexagonal
 *             lattice, on the parities of the two columns), by zero-padded 2D
 *             DFTs: (2 M_L)(2 M_H) Toeplitz products per sublattice pair
 *             instead of M^2; 1: every root pair is an M2L entry.
 *  self_mode  how the pairs of a fibre with itself at image 0 (both
 *             wavenumbers) are applied.  0 (auto): when every fibre is a circle
 *             cut into N equal chords with N a power of two, 8 <= N <= 512, and
 *             store_self_blocks = 0, that 2N x 2N block of each fibre is block
 *             circulant (rotation by one chord maps element a to a + 1), so it
 *             is applied exactly, near and far pairs alike, by FFTs of length N
 *             per fibre (the preconditioner's transforms): the tree then
 *             carries only the pairs between different fibres and with
 *             images, and the interior wavenumber k1, which acts within one
 *             fibre only, leaves the FMM altogether.  1: those pairs go
 *             through the tree like the others (near pairs by P2P from the
 *             circulant rows or stored blocks, far pairs by M2L at k and k1).
 *             With 0, moreover, every fibre root's multipole moments come
 *             from the fibre's discrete Fourier modes (element e is element
 *             0 turned by 2 pi e / N, so the moment of order n is
 *             A_n phihat(n) + B_n varphihat(n)), and every root's local
 *             expansion is evaluated at the fibre's midpoints by a synthesis
 *             over the orders (added to the spectrum before the inverse
 *             transform of the fibre's own block).  A fibre whose cells take
 *             part only in M2L entries at its root (no near pairs, no entry
 *             below the root: its neighbours are farther away than the
 *             admissibility ratio allows for their radii) needs no P2M, M2M,
 *             L2L or L2P (pfm_stats.spectral_roots, n_spectral_fibres); the
 *             other fibres' cells below the root take their moments
 *             straight from per-frequency P2M weights of their elements (no
 *             M2M), and their leaves run the downward pass of those cells'
 *             expansions (L2P from per-frequency Bessel values of each
 *             row).  2: as 0 without this.
 *  precond    0: plain GMRES; 1: pfm_solve runs GMRES (with PFM_MIXED the
 *             inner GMRES of the refinement)
 *             right-preconditioned by the fibres' free-space self blocks of
 *             (I - A) (the block-Jacobi preconditioner of the paper's
 *             "preconditioned GMRES", Sec. 4): each is block circulant, so it
 *             is inverted per Fourier mode of the element index (one 2x2
 *             solve per mode, FFTs of length N per fibre).  The residual and
 *             the stop test are those of the unpreconditioned system.  Needs
 *             N a power of two, 8 <= N <= 512.  pfm_solve_batch and
 *             pfm_sweep use it too (the blocks do not depend on theta, so a
 *             batch shares them), as do start vectors and the augmented
 *             start (use_x0 = 3), whose guess u enters as P u.
 *  tree_on_host  0: the quadtrees and interaction lists (Sec. 3.1) are built
 *             by GPU kernels (element keys sorted per fibre, cells level by
 *             level, one dual traversal per fibre pair and image), which
 *             give the host construction's plan bit for bit; where they do not
 *             apply (more than 4096 elements per fibre, or a level of one
 *             fibre's tree with more than 512 cells) the host builds it
 *             (pfm_stats.tree_on_device tells which ran).  1: the host
 *             construction (the reference the GPU build is tested against).
 *  discretisation  PFM_CHORDS or PFM_NYSTROM (pfm_discretisation).
 *  tree_shape PFM_TREE_SQUARE or PFM_TREE_TRIANGLE (pfm_tree_shape).
 *  m2l_vector 0: the M2L entries (eq. 13) that share a translation (an offset
 *             between cells, or the lattice sum of a fibre offset, Sec. 3.3)
 *             are applied together as complex matrix products on the matrix
 *             cores (FP64 v_mfma, 16 entries per product); 1: every entry on
 *             the vector ALU (pfm_stats.m2l_mfma_items counts the products). */
typedef struct {
  int p;
  int leaf_max;
  double mac;
  int g_far;
  int restart;
  int max_iter;
  double tol;
  double wood_margin;
  int precision;
  double inner_tol;
  int max_batch;
  int use_graph;
  int p2p_blocks_per_cu;
  int p2p_unroll;
  int store_self_blocks;
  int p2p_cached_rows;
  int direct_lattice_m2l;
  int precond;
  int self_mode;
  int tree_on_host;
  int m2l_vector;
  int discretisation;      /* pfm_discretisation */
  int tree_shape;          /* pfm_tree_shape */
} pfm_options;

#define PFM_MAX_BATCH 16

typedef struct {
  int status;              /* pfm_status of the solve */
  int iters;               /* GMRES iterations (matvecs inside Arnoldi) */
  int matvecs;             /* total operator applications */
  double rel_residual;     /* true relative residual of the returned Psi */
  double t_solve_s;        /* wall time of the solve */
  int outer;               /* PFM_MIXED: refinement steps (0 in FP64) */
  int fallback;            /* use_x0 = 2: the start vector was replaced by zero */
  int matvecs_mixed;       /* PFM_MIXED: applies with the complex64 near field (0 in FP64) */
} pfm_info;

/* Sizes and counts of the built plan (for reports and tests). */
typedef struct {
  int M, N, E, n_unknowns;
  int n_cells, n_leaves, depth;
  int n_m2l_ext, n_m2l_int;    /* explicit M2L pairs, exterior / interior */
  int n_near_pairs;            /* leaf pairs handled by P2P */
  long long n_near_entries;    /* element pairs in P2P blocks */
  long long n_near_cols;       /* sum over near leaf pairs of source elements */
  int n_root_offsets;          /* distinct fibre offsets of the lattice M2L */
  int n_m2l_offsets;           /* distinct M2L translation vectors */
  double near_bytes;           /* bytes of the stored P2P blocks (n_near_stored x 64) */
  double k, k1, eta, varrho, theta;
  int lattice_q;               /* direct images of the lattice sums, |m| <= q */
  int p2p_split;               /* column splits per target leaf in the P2P launch */
  int n_near_computed;         /* stored near pairs whose blocks are computed (equal fibres share blocks) */
  long long n_near_stored;     /* element pairs stored: with equal fibres, target leaves with the
                                  same near region (the same sources at the same offsets and
                                  images) read one stored copy of it */
  long long n_near_circulant;  /* element pairs taken from the circulant rows of their fibre */
  int p2p_window_leaves;       /* target leaves whose circulant row entries P2P stages in LDS
                                  (one window of consecutive entries per leaf) */
  int p2p_window_max;          /* entries of the largest such window (at most 320) */
  int lattice_m2l_grid;        /* 1: the root lattice M2L runs as a convolution over the fibre grid */
  double workspace_bytes;      /* bytes of the workspace in use (library-owned or bound) */
  int workspace_bound;         /* 1: the caller's block is bound (pfm_bind) */
  int batch_capacity;          /* angles per batch the current workspace serves */
  long long n_device_allocs;   /* device allocations the library has made for this handle */
  double device_alloc_bytes;   /* their total size */
  int self_fft;                /* 1: each fibre's own image-0 block is applied by FFT (self_mode 0) */
  int tree_on_device;          /* 1: the plan's tree and lists were built by the GPU kernels */
  int spectral_roots;          /* 1: fibre roots' moments by Fourier modes (self_mode 0) */
  int n_spectral_fibres;       /* fibres whose far rows come from their root's local expansion alone */
  int m2l_mfma_items;          /* M2L matrix products on the matrix cores (m2l_vector = 0) */
  int m2l_vector_chunks;       /* M2L entry chunks on the vector ALU */
  int m2l_mfma_entries;        /* M2L entries in those products (columns) */
  int precond_in_apply;        /* 1: a preconditioned solve applies P^{-1} inside the apply's forward
                                  transforms (roots by Fourier modes, and no tree fibres, stored near
                                  pairs or other reader of the densities): one launch fewer per
                                  iteration; 0: a separate launch before each apply */
} pfm_stats;

/* Build the plan: discretisation, quadtrees and interaction lists (on the
 * GPU unless tree_on_host = 1).  Fills *out on success.  Errors: PFM_EINVAL for bad sizes,
 * overlapping fibres (2 r >= lattice spacing) or unsupported options. */
pfm_status pfm_create(const pfm_geometry* geo, const pfm_material* mat,
                      const pfm_options* opt, pfm_problem** out);

/* Caller-owned workspace (the problem statement of Sec. 2 fixes what a
 * caller supplies; device memory is the caller's too).  The workspace holds
 * every device buffer whose contents depend on the frequency or the call:
 * near blocks and circulant rows, translation tables, lattice sums and their
 * tail rule, multipole expansions, M2L partial expansions, the far part,
 * preconditioner blocks, the GMRES basis, vectors and reduction scratch.
 * Plan metadata (elements, tree, lists, quadrature rules) stays with the
 * handle.  pfm_create allocates one workspace block for max_batch angles.
 *
 * pfm_workspace_size: *bytes = size of the workspace for batches of up to
 * `batch` angles (1 <= batch <= max_batch; 0 means max_batch).
 *
 * pfm_bind: move the workspace into the caller's device block d_workspace of
 * `bytes` bytes (256-byte aligned, e.g. a torch uint8 CUDA tensor).  The
 * batch capacity becomes the largest batch (<= max_batch) whose workspace
 * fits; PFM_EINVAL when not even one angle fits.  Work queued on the handle
 * is finished first; the library's own block is freed; the state of
 * pfm_set_wave / pfm_set_batch is dropped (call them again); hip_stream
 * becomes the handle's stream (as pfm_set_stream).  From then on no call on
 * the handle allocates device memory (pfm_stats.n_device_allocs stays put).
 * The caller keeps the block alive, and does not write to it, until the
 * handle is destroyed or bound elsewhere.  d_workspace = NULL returns to a
 * library-owned block of max_batch angles. */
pfm_status pfm_workspace_size(const pfm_problem* pb, int batch, size_t* bytes);
pfm_status pfm_bind(pfm_problem* pb, void* d_workspace, size_t bytes, void* hip_stream);

/* Use this HIP stream (hipStream_t) for all later work; NULL = null stream. */
pfm_status pfm_set_stream(pfm_problem* pb, void* hip_stream);

/* Per-frequency setup for (ka, theta): P2P near blocks with the exact self and
 * near element integrals, M2L/M2M/L2L translation tables at k and k1, and the
 * lattice sums of the top-level M2L (Sec. 3.3).  Returns PFM_EWOOD before any
 * work when the Wood margin test fails. */
pfm_status pfm_set_wave(pfm_problem* pb, double ka, double theta);

/* d_y = (I - A) d_psi, both 2*M*N complex128 on the device.  No allocation. */
pfm_status pfm_matvec(pfm_problem* pb, const void* d_psi, void* d_y);

/* For callers that cannot allocate device memory at all (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * d_y = (I - A) d_psi exactly as pfm_matvec, with the apply's scratch
 * (multipole moments, M2L partial expansions and their sums, the lattice
 * convolution's spectra, the far part, split P2P partial rows) taken from a
 * fixed device array of PFM_STATIC_SCRATCH_BYTES that the library holds on
 * each GPU until the process ends, instead of from the handle's workspace.
 * Allocates nothing.  The handle's GPU must be the current device.
 * PFM_EINVAL when the apply needs more scratch than the array holds (the
 * message gives the size).  Every call on one GPU shares its array, and the
 * array keeps the last call's contents: calls that overlap on one GPU (other
 * streams, other handles) race. */
#define PFM_STATIC_SCRATCH_BYTES (64u << 20)
pfm_status pfm_matvec_static(pfm_problem* pb, const void* d_psi, void* d_y);

/* The same operator with the near-field blocks stored in complex64 (each
 * block entry widened to FP64 before its multiply-add; densities and sums
 * stay FP64) and the far field in FP64 (the apply used inside PFM_MIXED
 * refinement).
 * Requires a handle created with precision = PFM_MIXED. */
pfm_status pfm_matvec_mixed(pfm_problem* pb, const void* d_psi, void* d_y);

/* d_b = B of eq. (9) for the current wave. */
pfm_status pfm_rhs(pfm_problem* pb, void* d_b);

/* Restarted GMRES for (I - A) Psi = B with the FMM apply.  d_b: right-hand
 * side (NULL: B of eq. 9).  d_x: on entry the start vector when use_x0 != 0
 * (else zero is used), on return the solution.  use_x0 = 2: a start vector
 * whose true residual is not below ||B|| is replaced by zero (the cold start
 * is the fallback; info->fallback = 1).  use_x0 = 3: d_x holds a guess u that
 * augments the first cycle, which minimises the residual over
 * span{u} + K_j((I - A), B) starting from zero, so it never needs more
 * iterations than the cold start (FP64 precision only).  Returns PFM_ENOCONV when the
 * tolerance is not met in max_iter iterations (d_x holds the best iterate). */
pfm_status pfm_solve(pfm_problem* pb, const void* d_b, void* d_x, int use_x0,
                     pfm_info* info);

/* Block-Jacobi preconditioner of the current wave (options.precond = 1):
 * d_out = P^{-1} d_in (inverse = 1) or d_out = P d_in (inverse = 0), where P
 * is block diagonal with, for each fibre, its free-space self block of
 * (I - A): the 2N x 2N block of its own elements at image 0, near and far
 * pairs alike (Sec. 2, the operators of eq. 6 with the row scaling of eq. 9).
 * d_in, d_out: device vectors of 2 M N complex128 in the layout of Psi;
 * they may be the same buffer.  Enqueued on the bound stream.  PFM_ESTATE
 * without pfm_set_wave or when the handle was created with precond = 0. */
pfm_status pfm_precond_apply(pfm_problem* pb, const void* d_in, void* d_out, int inverse);

/* Reflected and transmitted Bragg amplitudes for orders -n_orders..n_orders
 * (host arrays of 2*(2*n_orders+1) doubles, interleaved complex), the energy
 * transmission coefficient of Sec. 4 and the flux-balance residual
 * sum_prop gamma_n (|R_n|^2 + |delta_n0 + T_n|^2) / (k cos th) - 1. */
pfm_status pfm_fields(pfm_problem* pb, const void* d_psi, int n_orders,
                      double* R, double* T, double* etc, double* energy_residual);

pfm_status pfm_get_stats(const pfm_problem* pb, pfm_stats* st);

/* Apply the operator reps times with every stage in order on the bound
 * stream and return the mean duration (milliseconds, HIP events) of each
 * stage: stage_ms[6] = [P2M, M2M, M2L including the lattice sums, downward
 * pass with L2P, near part (each fibre's own block by FFT and P2P of the
 * stored pairs), join of near and far parts], and of the whole apply in
 * *total_ms.  The stages write the far part to a buffer of their own and a
 * join kernel adds it (pfm_matvec fuses the join into the downward pass).
 * With the roots by Fourier modes (pfm_stats.spectral_roots) the launches
 * are those of pfm_matvec, bracketed: [forward transforms of the own blocks
 * with the roots' moments and the other tree-fibre cells' moments from
 * their P2M weights, M2M (no launch), M2L, inverse transforms with the
 * roots' far part and the tree fibres' downward pass (and near rows),
 * 0, 0]. */
pfm_status pfm_matvec_timed(pfm_problem* pb, const void* d_psi, void* d_y,
                            int reps, double* stage_ms, double* total_ms);

/* ---- batched sweep: B incidence angles at one frequency ------------------
 * The B members share the tree, the near-field blocks (stored once, without
 * the quasi-periodic image phase, which each member applies to its source
 * densities as alpha_b^m), the translation tables at k and k1 and the
 * orders of the expansions; each member has its own lattice sums (Sec. 3.3,
 * theta-dependent through alpha), image phases and right-hand side.
 * Batched vectors are [B][2*M*N] complex128, member after member. */

/* Per-frequency setup for the angles theta[0..B-1], 1 <= B <= max_batch.
 * Invalidates the single-angle state of pfm_set_wave (and vice versa).
 * PFM_EWOOD when any angle fails the Wood margin test (nothing is set up). */
pfm_status pfm_set_batch(pfm_problem* pb, double ka, int B, const double* theta);

/* d_y[b] = (I - A_b) d_psi[b] for every member b.  No allocation. */
pfm_status pfm_matvec_batch(pfm_problem* pb, const void* d_psi, void* d_y);

/* d_b[b] = B of eq. (9) for member b. */
pfm_status pfm_rhs_batch(pfm_problem* pb, void* d_b);

/* Restarted GMRES for all members in lockstep: one batched apply per
 * iteration, Arnoldi (CGS2) per member in FP64.  d_b: [B][2MN] right-hand
 * sides or NULL (eq. 9); d_x: [B][2MN] start vectors when use_x0 != 0, the
 * solutions on return (use_x0 = 2: per-member fallback to zero, 3:
 * per-member augmentation, as in pfm_solve); infos: host array of B records.  A member stops
 * when its true residual meets tol.  Returns PFM_ENOCONV when any member
 * misses the tolerance within max_iter iterations (its best iterate is
 * written), PFM_OK otherwise. */
pfm_status pfm_solve_batch(pfm_problem* pb, const void* d_b, void* d_x, int use_x0, pfm_info* infos);

/* Band sweep: for each ka[i] (i < n_ka), pfm_set_batch(ka[i], B, theta)
 * and pfm_solve_batch from zero.  d_x: [n_ka][B][2MN] solutions; infos:
 * host [n_ka][B].  Frequencies that fail the Wood test get status
 * PFM_EWOOD in their records and zero solutions; the sweep goes on.
 * Returns the first error that is neither PFM_ENOCONV nor PFM_EWOOD, else
 * PFM_ENOCONV / PFM_EWOOD if any record has it, else PFM_OK. */
pfm_status pfm_sweep(pfm_problem* pb, int n_ka, const double* ka, int B, const double* theta, void* d_x,
                     pfm_info* infos);

/* One stage of the FMM chain of the current wave (0 P2M, 1 M2M, 2 M2L
 * with the lattice sums, 3 downward pass with L2P; with the roots by
 * Fourier modes the stages of pfm_matvec_timed) launched reps times back
 * to back on the bound stream after one whole chain for d_psi, which leaves
 * every stage's inputs in place; *ms_per_launch = the mean duration of one
 * launch (HIP events around the reps launches).  For measuring a kernel
 * in steady state; PFM_EINVAL for a bad stage or reps < 1. */
pfm_status pfm_matvec_stage_timed(pfm_problem* pb, const void* d_psi, int stage, int reps, double* ms_per_launch);

/* Batched apply timed like pfm_matvec_timed (stage_ms[6], total_ms). */
pfm_status pfm_matvec_batch_timed(pfm_problem* pb, const void* d_psi, void* d_y, int reps, double* stage_ms,
                                  double* total_ms);

const char* pfm_last_error(const pfm_problem* pb);
void pfm_destroy(pfm_problem* pb);

/* ---- test hooks: expose single stages for parity tests ------------------ */

/* Bessel J0, J1, Y0, Y1 of n arguments d_x > 0 on the device:
 * d_out[4*i + (0..3)].  Special functions are written from DLMF 10.8
 * (series), 10.17 (Hankel asymptotics), 10.23 (Neumann series) and Miller's
 * backward recurrence (DLMF 3.6). */
pfm_status pfm_test_bessel(const double* d_x, int n, double* d_out);

/* Lattice sums of the current wave: host array [n_root_offsets][4p+1] complex,
 * the offsets [n_root_offsets][2] and the excluded image range [m_lo, m_hi]. */
pfm_status pfm_test_lattice(pfm_problem* pb, double* sums, double* offsets, int* mrange);

/* Multipole moments of every cell for d_psi after the upward pass (P2M and
 * M2M): host [n_cells][2 channels][2p+1] complex (channel 0: k, 1: k1), the
 * cell centres [n_cells][2], per cell (level, fibre, first, end) into the
 * tree-ordered element list, and that list (E natural element ids).
 * Any output pointer may be NULL. */
pfm_status pfm_test_moments(pfm_problem* pb, const void* d_psi, double* moments,
                            double* centres, int* cellinfo, int* elem_order);

/* Digests of the built plan (Sec. 3.1), for comparing the GPU tree build
 * with the host construction: out[0..7] = 64-bit FNV-1a hashes of, in order,
 * the cells (every field), the level ranges with the element order, leaves
 * and fibre roots, the leaf-to-ancestor lists with their offsets, the upward
 * lists, the fibre offsets with their image ranges and pair table, the M2L
 * lists with their translation vectors, the interior M2L lists, and the near
 * lists with their block offsets and the image range. */
pfm_status pfm_test_plan_digest(const pfm_problem* pb, unsigned long long* out);

#ifdef __cplusplus
}
#endif
#endif /* PFMBEM_H */
