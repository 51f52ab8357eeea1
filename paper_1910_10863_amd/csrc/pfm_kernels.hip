// Device kernels of the periodic FM-BEM (gfx950).
//
// Layouts: complex values are double2 (re, im).  Element data are SoA in
// natural order (fibre-major).  Expansion coefficients of cell c, channel
// ch (0: exterior wavenumber k, 1: interior wavenumber k1), order n in
// [-p, p] live at [(c * 2 + ch) * (2p+1) + n + p].  Translation tables hold
// orders nu in [-2p, 2p] at [nu + 2p].  P2P blocks hold four complex values
// (B11, B12, B21, B22) per (target, source) element pair, laid out per near
// leaf pair as [source column][component][target row]; the pairs of one
// target leaf follow each other, so the near field of a leaf is one
// contiguous stream and the lanes of a wavefront (target rows) read
// consecutive addresses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>

#include "pfm_kernels.hpp"

namespace pfm {

bool supported_p(int p) {
  return p == 8 || p == 12 || p == 16 || p == 20 || p == 24 || p == 32 || p == 40;
}

// ---------------------------------------------------------------------------
// discretisation: N chords per fibre between the nodes c + gamma(r, t_e),
// t_e = 2 pi e / N, of the fibre's boundary curve: a circle, or the round
// square of Sec. 4, r ((3 + 2 sin^2 t) cos t, (3 + 2 cos^2 t) sin t)
// ---------------------------------------------------------------------------
__device__ inline void boundary_point(int shape, double r, double t, double& x, double& y) {
  const double c = cos(t), s = sin(t);
  if (shape == PFM_ROUND_SQUARE) {
    x = r * (3.0 + 2.0 * s * s) * c;
    y = r * (3.0 + 2.0 * c * c) * s;
  } else {
    x = r * c;
    y = r * s;
  }
}

// nystrom = 0: chord e between the nodes at t_e and t_{e+1} (midpoint, unit
// tangent, length).  nystrom = 1 (circles): the node at t_e itself as the
// point, the circle's unit tangent, and the trapezoid weight r 2 pi / N as
// the length; both chord ends are the node (the tree's tight radii).
__global__ void k_discretise(int E, int N, int shape, int nystrom, const double* __restrict__ centres,
                             const double* __restrict__ radii, double* mx, double* my,
                             double* tx, double* ty, double* h, double* ends) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  int f = e / N, l = e - f * N;
  double t0 = 2.0 * PI * l / N, t1 = 2.0 * PI * (l + 1) / N;
  double cx = centres[2 * f], cy = centres[2 * f + 1], r = radii[f];
  if (nystrom) {
    double sv, cv;
    sincospi(2.0 * (double)l / (double)N, &sv, &cv);
    const double px = cx + r * cv, py = cy + r * sv;
    mx[e] = px;
    my[e] = py;
    tx[e] = -sv;
    ty[e] = cv;
    h[e] = 2.0 * PI * r / N;
    if (ends) {
      ends[4 * e + 0] = ends[4 * e + 2] = px;
      ends[4 * e + 1] = ends[4 * e + 3] = py;
    }
    return;
  }
  double ux, uy, vx, vy;
  boundary_point(shape, r, t0, ux, uy);
  boundary_point(shape, r, t1, vx, vy);
  double ax = cx + ux, ay = cy + uy;
  double bx = cx + vx, by = cy + vy;
  double dx = bx - ax, dy = by - ay;
  double hh = sqrt(dx * dx + dy * dy);
  mx[e] = 0.5 * (ax + bx);
  my[e] = 0.5 * (ay + by);
  tx[e] = dx / hh;
  ty[e] = dy / hh;
  h[e] = hh;
  if (ends) {
    ends[4 * e + 0] = ax;
    ends[4 * e + 1] = ay;
    ends[4 * e + 2] = bx;
    ends[4 * e + 3] = by;
  }
}

hipError_t launch_discretise(Problem& pb, double* d_ends) {
  int E = pb.E;
  hipLaunchKernelGGL(k_discretise, dim3((E + 255) / 256), dim3(256), 0, pb.stream, E, pb.N, pb.shape,
                     pb.nystrom ? 1 : 0, pb.d_centres, pb.d_radii, pb.d_mx, pb.d_my, pb.d_tx, pb.d_ty, pb.d_h,
                     d_ends);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// kernels S, D, K, T of the layer operators at one point pair (Sec. 2)
// ---------------------------------------------------------------------------
__device__ inline void kern_sdkt(double kap, double dx, double dy, double nux, double nuy,
                                 double nx, double ny, cd& S, cd& D, cd& K, cd& T) {
  double r = sqrt(dx * dx + dy * dy);
  cd H0, H1;
  hankel01(kap * r, H0, H1);
  double dnx = dx * nux + dy * nuy;      // d . nu_x
  double dny = dx * nx + dy * ny;        // d . n_y
  double nn = nux * nx + nuy * ny;
  double ir = 1.0 / r;
  S = mkc(-0.25 * H0.y, 0.25 * H0.x);                 // (i/4) H0
  cd ikH1 = mkc(-0.25 * kap * H1.y, 0.25 * kap * H1.x);  // (i kap/4) H1
  D = cscale(ikH1, dny * ir);
  K = cscale(ikH1, -dnx * ir);
  // (i kap/4) [ (kap H0/r - 2 H1/r^2) dnx dny / r + H1 nn / r ]
  cd a = csub(cscale(H0, kap * ir), cscale(H1, 2.0 * ir * ir));
  cd b = cadd(cscale(a, dnx * dny * ir), cscale(H1, nn * ir));
  T = cscale(mkc(-b.y, b.x), 0.25 * kap);
}

// Self element at its midpoint: S = (i/4) 2 int_0^{h/2} H0(kap s) ds by the
// term-wise integrated power series of J0 and Y0 (DLMF 10.8.1);
// T = kap^2 S - (i kap/2) H1(kap h/2) (straight-element Maue identity); D = K = 0.
__device__ inline void self_terms(double kap, double h, cd& S, cd& T) {
  double X = 0.5 * kap * h;
  double q = -0.25 * X * X;
  double lg = log(0.5 * X) + EULER_GAMMA;
  double ak = 1.0;        // (-1/4)^k / (k!)^2 * X^{2k}  (without the X factor)
  double Hk = 0.0;        // harmonic number
  double ij = 0.0, iy1 = 0.0, iy2 = 0.0;
  for (int k = 0; k < 60; ++k) {
    if (k > 0) {
      ak *= q / ((double)k * (double)k);
      Hk += 1.0 / k;
    }
    double inv = 1.0 / (2.0 * k + 1.0);
    double t = ak * X * inv;            // a_k X^{2k+1} / (2k+1)
    ij += t;
    iy1 += t * (lg - inv);
    iy2 += Hk * t;
    if (k > 2 && fabs(t) < 1e-18 * fabs(ij)) break;
  }
  double iy = (2.0 / PI) * (iy1 - iy2);
  // int_0^{h/2} H0(kap s) ds = (ij + i iy) / kap ; S = (i/2)(...)
  S = mkc(-0.5 * iy / kap, 0.5 * ij / kap);
  cd H0, H1;
  hankel01(X, H0, H1);
  T = csub(cscale(S, kap * kap), mkc(-0.5 * kap * H1.y, 0.5 * kap * H1.x));
}

// ---------------------------------------------------------------------------
// near-field blocks (per wave): one workgroup per near leaf pair
// ---------------------------------------------------------------------------
struct NearArgs {
  int N, g_far;
  double k, k1, eta, varrho, H;
  const double *mx, *my, *tx, *ty, *h, *gl, *gl16;
  const int *elem_of, *ebeg, *eend, *leaves, *near_tgt, *near_src, *near_m;
  const long long* near_blk;
  const cd* alpha;
  int m_min;
  long long n_entries;
  cd* out;
  const int* pair_ids;     // stored pair computed by each workgroup row
};

__device__ inline void far_rule(double kap, double x, double y, double nux, double nuy,
                                double cxm, double cym, double tx, double ty, double hh,
                                const double* gl, int G, cd& S, cd& D, cd& K, cd& T) {
  S = D = K = T = mkc(0, 0);
  double nx = ty, ny = -tx;
  for (int g = 0; g < G; ++g) {
    double s = 0.5 * hh * gl[g];
    double w = 0.5 * hh * gl[G + g];
    cd s_, d_, k_, t_;
    kern_sdkt(kap, x - (cxm + s * tx), y - (cym + s * ty), nux, nuy, nx, ny, s_, d_, k_, t_);
    S = cadd(S, cscale(s_, w));
    D = cadd(D, cscale(d_, w));
    K = cadd(K, cscale(k_, w));
    T = cadd(T, cscale(t_, w));
  }
}

// The 2x2 block of (I - A) for target element ea and source element eb
// (natural ids), source shifted by image m with phase ph.
__device__ inline void near_entry(const NearArgs& A, int ea, int eb, int m, cd ph, cd& B11, cd& B12, cd& B21,
                                  cd& B22) {
  cd c = mkc(0.0, -2.0 / (A.eta * (1.0 + A.varrho)));     // 2 / (i eta (1 + varrho))
  cd mieta = mkc(0.0, -A.eta);                              // -i eta
  double x = A.mx[ea], y = A.my[ea];
  double nux = A.ty[ea], nuy = -A.tx[ea];
  double sx = A.mx[eb], sy = A.my[eb] + m * A.H;
  double tx = A.tx[eb], ty = A.ty[eb], hh = A.h[eb];
  int fa = ea / A.N, fb = eb / A.N;
  if (fa == fb && m == 0) {
    int dl = abs((ea - fa * A.N) - (eb - fb * A.N));
    dl = min(dl, A.N - dl);
    cd S2, D2, K2, T2, S1, D1, K1, T1;
    if (dl == 0) {
      self_terms(A.k, hh, S2, T2);
      self_terms(A.k1, hh, S1, T1);
      D2 = K2 = D1 = K1 = mkc(0, 0);
    } else if (dl <= 2) {
      far_rule(A.k, x, y, nux, nuy, sx, sy, tx, ty, hh, A.gl16, 16, S2, D2, K2, T2);
      far_rule(A.k1, x, y, nux, nuy, sx, sy, tx, ty, hh, A.gl16, 16, S1, D1, K1, T1);
    } else {
      far_rule(A.k, x, y, nux, nuy, sx, sy, tx, ty, hh, A.gl, A.g_far, S2, D2, K2, T2);
      far_rule(A.k1, x, y, nux, nuy, sx, sy, tx, ty, hh, A.gl, A.g_far, S1, D1, K1, T1);
    }
    B11 = csub(D2, D1);
    B12 = cmul(mieta, csub(S2, S1));
    B21 = cmul(c, csub(T2, cscale(T1, A.varrho)));
    B22 = cmul(cmul(c, mieta), csub(K2, cscale(K1, A.varrho)));
  } else {
    cd S2, D2, K2, T2;
    far_rule(A.k, x, y, nux, nuy, sx, sy, tx, ty, hh, A.gl, A.g_far, S2, D2, K2, T2);
    B11 = cmul(ph, D2);
    B12 = cmul(cmul(mieta, ph), S2);
    B21 = cmul(cmul(c, ph), T2);
    B22 = cmul(cmul(cmul(c, mieta), ph), K2);
  }
}

__global__ void __launch_bounds__(128) k_near_blocks(NearArgs A) {
  int q = A.pair_ids[blockIdx.x];
  int D = A.leaves[A.near_tgt[q]];
  int C = A.near_src[q];
  int m = A.near_m[q];
  int db = A.ebeg[D], rows = A.eend[D] - db;
  int cb = A.ebeg[C], cols = A.eend[C] - cb;
  long long blk = A.near_blk[q];
  cd ph = A.alpha[m - A.m_min];
  // the pair's entries are spread over the y axis of the grid, one per thread
  for (int rc = blockIdx.y * blockDim.x + threadIdx.x; rc < rows * cols; rc += gridDim.y * blockDim.x) {
    int col = rc / rows, row = rc - col * rows;
    cd B11, B12, B21, B22;
    near_entry(A, A.elem_of[db + row], A.elem_of[cb + col], m, ph, B11, B12, B21, B22);
    long long idx = 4 * blk + (long long)col * 4 * rows + row;
    A.out[idx] = B11;
    A.out[idx + rows] = B12;
    A.out[idx + 2 * rows] = B21;
    A.out[idx + 3 * rows] = B22;
  }
}

// Circulant near rows: for fibre f the block of its element 0 with its
// element d (image 0) for d = 0..N-1, which is the block of any element a
// with element (a + d) mod N.  Layout [f][B11, B12, B21, B22][2N], entry d
// stored at d and at d + N so that the index (b - a) + N needs no wrap.
// 32 lanes per entry: lane bit 4 picks the wavenumber (k or k1), bits 0..3
// the Gauss point of the source element's rule (16 points for the two
// neighbours on each side, g_far <= 16 otherwise, the closed form for the
// element itself); the points are summed by a 16-lane butterfly.
constexpr int CR_ENTRIES = 8;            // entries per 256-thread workgroup

__global__ void __launch_bounds__(256) k_circ_rows(NearArgs A, cd* __restrict__ circ) {
  const int f = blockIdx.y, N = A.N;
  const int d = blockIdx.x * CR_ENTRIES + (threadIdx.x >> 5);
  const int sub = threadIdx.x & 31, kw = sub >> 4, g = sub & 15;
  if (d >= N) return;                    // the entry's 32 lanes leave together
  const int ea = f * N, eb = f * N + d;
  const double kap = kw ? A.k1 : A.k;
  const double x = A.mx[ea], y = A.my[ea];
  const double nux = A.ty[ea], nuy = -A.tx[ea];
  const double cxm = A.mx[eb], cym = A.my[eb];
  const double tx = A.tx[eb], ty = A.ty[eb], hh = A.h[eb];
  const int dl = min(d, N - d);
  cd S = mkc(0, 0), D = S, K = S, T = S;
  if (dl == 0) {
    if (g == 0) self_terms(kap, hh, S, T);
  } else {
    const double* gl = dl <= 2 ? A.gl16 : A.gl;
    const int G = dl <= 2 ? 16 : A.g_far;
    if (g < G) {
      const double sg = 0.5 * hh * gl[g], w = 0.5 * hh * gl[G + g];
      cd s_, d_, k_, t_;
      kern_sdkt(kap, x - (cxm + sg * tx), y - (cym + sg * ty), nux, nuy, ty, -tx, s_, d_, k_, t_);
      S = cscale(s_, w);
      D = cscale(d_, w);
      K = cscale(k_, w);
      T = cscale(t_, w);
    }
  }
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) {
    S.x += __shfl_xor(S.x, off, 64); S.y += __shfl_xor(S.y, off, 64);
    D.x += __shfl_xor(D.x, off, 64); D.y += __shfl_xor(D.y, off, 64);
    K.x += __shfl_xor(K.x, off, 64); K.y += __shfl_xor(K.y, off, 64);
    T.x += __shfl_xor(T.x, off, 64); T.y += __shfl_xor(T.y, off, 64);
  }
  // the interior (k1) sums of lane 16 to lane 0
  const cd S1 = mkc(__shfl_xor(S.x, 16, 64), __shfl_xor(S.y, 16, 64));
  const cd D1 = mkc(__shfl_xor(D.x, 16, 64), __shfl_xor(D.y, 16, 64));
  const cd K1 = mkc(__shfl_xor(K.x, 16, 64), __shfl_xor(K.y, 16, 64));
  const cd T1 = mkc(__shfl_xor(T.x, 16, 64), __shfl_xor(T.y, 16, 64));
  if (sub != 0) return;
  const cd c = mkc(0.0, -2.0 / (A.eta * (1.0 + A.varrho)));     // 2 / (i eta (1 + varrho))
  const cd mieta = mkc(0.0, -A.eta);                              // -i eta
  const cd B11 = csub(D, D1);
  const cd B12 = cmul(mieta, csub(S, S1));
  const cd B21 = cmul(c, csub(T, cscale(T1, A.varrho)));
  const cd B22 = cmul(cmul(c, mieta), csub(K, cscale(K1, A.varrho)));
  cd* row = circ + (size_t)f * 8 * N;
  row[d] = row[d + N] = B11;
  row[2 * N + d] = row[3 * N + d] = B12;
  row[4 * N + d] = row[5 * N + d] = B21;
  row[6 * N + d] = row[7 * N + d] = B22;
}

// copy of computed near blocks into the slots of the pairs that share them
__global__ void k_copy_blocks(const long long* __restrict__ src, const long long* __restrict__ dst,
                              const int* __restrict__ len, cd* blocks) {
  int c = blockIdx.x;
  const cd* s = blocks + 4 * src[c];
  cd* d = blocks + 4 * dst[c];
  for (int i = blockIdx.y * blockDim.x + threadIdx.x; i < len[c]; i += gridDim.y * blockDim.x) d[i] = s[i];
}

static hipError_t launch_circ_rows_nys(Problem& pb);

hipError_t launch_near_blocks(Problem& pb, bool phase_free) {
  const HostPlan& hp = pb.hp;
  int npairs = (int)hp.near_src.size();
  NearArgs A;
  A.N = pb.N;
  A.g_far = pb.opt.g_far;
  A.k = pb.k;
  A.k1 = pb.k1;
  A.eta = pb.eta;
  A.varrho = pb.varrho;
  A.H = pb.H;
  A.mx = pb.d_mx; A.my = pb.d_my; A.tx = pb.d_tx; A.ty = pb.d_ty; A.h = pb.d_h;
  A.gl = pb.d_gl; A.gl16 = pb.d_gl16;
  A.elem_of = pb.d_elem_of; A.ebeg = pb.d_ebeg; A.eend = pb.d_eend; A.leaves = pb.d_leaves;
  A.near_tgt = pb.d_near_tgt; A.near_src = pb.d_near_src; A.near_m = pb.d_near_m;
  A.near_blk = pb.d_near_blk;
  A.alpha = phase_free ? pb.d_alpha_one : pb.d_alpha;
  A.m_min = hp.m_min;
  A.n_entries = pb.n_near_stored;
  A.out = pb.d_near;
  int lm = pb.opt.leaf_max;
  A.pair_ids = pb.d_near_uniq;
  if (npairs > 0 && pb.n_near_uniq > 0)
    hipLaunchKernelGGL(k_near_blocks, dim3(pb.n_near_uniq, (lm * lm + 127) / 128), dim3(128), 0, pb.stream, A);
  if (npairs > 0 && pb.n_near_copies > 0)
    hipLaunchKernelGGL(k_copy_blocks, dim3(pb.n_near_copies, (4 * lm * lm + 255) / 256), dim3(256), 0, pb.stream,
                       pb.d_near_cp_src, pb.d_near_cp_dst, pb.d_near_cp_len, pb.d_near);
  if (pb.nystrom)
    return launch_circ_rows_nys(pb);
  if (pb.n_near_circ > 0 || pb.opt.precond || pb.self_fft)
    hipLaunchKernelGGL(k_circ_rows, dim3((pb.N + CR_ENTRIES - 1) / CR_ENTRIES, pb.M), dim3(256), 0, pb.stream, A,
                       pb.d_circ);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block-Jacobi preconditioner (the "preconditioned GMRES" of Sec. 4), one
// block per fibre: its free-space self block of (I - A), whose 2x2 block for
// elements a, b is I delta_ab + R((b - a) mod N) with R the circulant row
// (the row holds no identity).  The vectors e_kappa(a) = w^{kappa a},
// w = exp(2 pi i / N), diagonalise it: mode kappa sees the 2x2 matrix
// I + L(kappa), L(kappa) = sum_d R(d) w^{kappa d}.  With the forward DFT
// xhat(kappa) = sum_b x_b w^{-kappa b}, P x is the inverse DFT of
// (I + L(kappa)) xhat(kappa) and P^{-1} x that of (I + L(kappa))^{-1} xhat.
// The DFTs are Stockham transforms in LDS (radix 4, plus one radix-2 stage
// when log2 N is odd; natural order in and out, so no bit reversal), one
// workgroup per fibre.
// ---------------------------------------------------------------------------
constexpr int PC_THREADS = 512;

// nv vectors of length N = 2^logN at X + v N, transformed with Y (same size)
// as the other buffer of each stage; fwd: exponent -i (unscaled either way).
// Radix-4 stages: each splits every remaining sub-sequence of length n into
// four interleaved quarters (a 4-point DFT and the twiddles w^{j p s},
// j = 1..3), then one radix-2 stage when log2 N is odd.  Returns the buffer
// with the result.
__device__ cd* pc_fft(cd* X, cd* Y, int nv, int N, int logN, const cd* __restrict__ tw, bool fwd) {
  const int quarter = N >> 2;
  int lg = 0;
  for (; lg + 2 <= logN; lg += 2) {
    const int s = 1 << lg, m = quarter >> lg;
    for (int i = threadIdx.x; i < nv * quarter; i += blockDim.x) {
      const int v = i >> (logN - 2), r = i & (quarter - 1);
      const int p = r >> lg, q = r & (s - 1);
      cd w1 = tw[p * s], w2 = tw[2 * p * s], w3 = tw[3 * p * s];
      if (fwd) {
        w1.y = -w1.y;
        w2.y = -w2.y;
        w3.y = -w3.y;
      }
      const cd* x = X + v * N;
      cd* y = Y + v * N;
      const cd a0 = x[q + s * p], a1 = x[q + s * (p + m)], a2 = x[q + s * (p + 2 * m)], a3 = x[q + s * (p + 3 * m)];
      const cd b0 = cadd(a0, a2), b1 = csub(a0, a2), b2 = cadd(a1, a3), d = csub(a1, a3);
      const cd b3 = fwd ? mkc(d.y, -d.x) : mkc(-d.y, d.x);     // -i d (forward) or +i d
      y[q + 4 * s * p] = cadd(b0, b2);
      y[q + 4 * s * p + s] = cmul(cadd(b1, b3), w1);
      y[q + 4 * s * p + 2 * s] = cmul(csub(b0, b2), w2);
      y[q + 4 * s * p + 3 * s] = cmul(csub(b1, b3), w3);
    }
    __syncthreads();
    cd* t = X;
    X = Y;
    Y = t;
  }
  if (lg < logN) {                     // the last radix-2 stage (stride N / 2, no twiddle)
    const int half = N >> 1;
    for (int i = threadIdx.x; i < nv * half; i += blockDim.x) {
      const int v = i >> (logN - 1), q = i & (half - 1);
      const cd* x = X + v * N;
      cd* y = Y + v * N;
      const cd a = x[q], b = x[q + half];
      y[q] = cadd(a, b);
      y[q + half] = csub(a, b);
    }
    __syncthreads();
    cd* t = X;
    X = Y;
    Y = t;
  }
  return X;
}

// Circulant rows of the Nystrom discretisation (circles): the 2x2 blocks of
// (I - A) without the identity for node 0 of fibre f and its node d (image
// 0), d = 0..N-1, laid out as k_circ_rows.  On a circle of radius r every
// operator of Kress's quadrature depends on d only: with t = 2 pi d / N,
// R_d = kress[d] the logarithmic weight, lg = ln(4 sin^2(t/2)), the distance
// rho = 2 r |sin(t/2)|, and per wavenumber kap (k outside, k1 inside)
//   S   = R_d F1 + (2 pi/N)(F - F1 lg),  F = (i/4) H0(kap rho) r,       F1 = -J0 r / (4 pi)
//   D   ...                             F = (i kap/4) H1 (x - y).nt / rho, F1 = -(kap/4 pi) J1 (x - y).nt / rho
//   K   ...                             F = -(i kap/4) H1 (x - y).nu / rho r, F1 its J1 part
//   S0  ...                             F = (i/4) H0,   F1 = -J0 / (4 pi)   (for T)
//   Snu ...                             F = (i/4) H0 r cos t, F1 = -J0 r cos t / (4 pi)
// with (x - y).nt = -2 r^2 sin^2(t/2), (x - y).nu = 2 r sin^2(t/2), and at
// d = 0 the limits F - F1 lg -> (i/4 - C/(2 pi) - ln(kap r/2)/(2 pi)) r for S
// and Snu (without r for S0) and -1/(4 pi) for D and K (curvature 1/r).
// T = (1/r) D S0 D + kap^2 Snu by Maue's identity, with D the trigonometric
// differentiation: the circulant (1/r) D S0 D has the eigenvalues
// -q^2 lambda_S0(q) / r (q signed, 0 on the Nyquist mode), lambda(q) =
// sum_d row(d) w^{q d}; its row is (1/N) sum_q lambda(q) w^{-q d}.  One
// workgroup per fibre; the two S0 rows go through the block's transforms.
__global__ void __launch_bounds__(PC_THREADS) k_circ_rows_nys(int N, int logN, const double* __restrict__ radii,
                                                              double k, double k1, double eta, double varrho,
                                                              const double* __restrict__ kress,
                                                              const cd* __restrict__ tw, cd* __restrict__ circ) {
  extern __shared__ cd pcs[];
  const int f = blockIdx.x;
  const double r = radii[f];
  cd* X = pcs;                   // [2][N]: the S0 rows at k and k1
  cd* Y = pcs + 2 * N;
  const double w2 = 2.0 * PI / N;
  for (int d = threadIdx.x; d < N; d += blockDim.x) {
    double sv, cv, s2, c2;
    sincospi((double)d / (double)N, &s2, &c2);         // sin(t/2), cos(t/2)
    sincospi(2.0 * (double)d / (double)N, &sv, &cv);   // sin t, cos t
    const double R = kress[d];
    for (int ch = 0; ch < 2; ++ch) {
      const double kap = ch ? k1 : k;
      cd S0;
      if (d == 0) {
        const cd lnk = mkc(-EULER_GAMMA / (2.0 * PI) - log(0.5 * kap * r) / (2.0 * PI), 0.25);
        S0 = cadd(mkc(-R / (4.0 * PI), 0.0), cscale(lnk, w2));
      } else {
        const double rho = 2.0 * r * fabs(s2), lg = log(4.0 * s2 * s2);
        cd H0, H1;
        hankel01(kap * rho, H0, H1);
        const cd F = mkc(-0.25 * H0.y, 0.25 * H0.x);               // (i/4) H0
        const double F1 = -H0.x / (4.0 * PI);                      // -J0 / (4 pi)
        S0 = cadd(mkc(R * F1, 0.0), cscale(csub(F, mkc(F1 * lg, 0.0)), w2));
      }
      X[ch * N + d] = S0;
    }
  }
  __syncthreads();
  cd* L = pc_fft(X, Y, 2, N, logN, tw, false);           // eigenvalues of S0
  for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) {
    const int q = i & (N - 1);
    const int qs = 2 * q == N ? 0 : (2 * q < N ? q : q - N);
    L[i] = cscale(L[i], -(double)qs * (double)qs / r);
  }
  __syncthreads();
  const cd* Z = pc_fft(L, L == X ? Y : X, 2, N, logN, tw, true);   // N x rows of (1/r) D S0 D
  const cd c = mkc(0.0, -2.0 / (eta * (1.0 + varrho)));            // 2 / (i eta (1 + varrho))
  const cd mieta = mkc(0.0, -eta);
  cd* row = circ + (size_t)f * 8 * N;
  for (int d = threadIdx.x; d < N; d += blockDim.x) {
    double sv, cv, s2, c2;
    sincospi((double)d / (double)N, &s2, &c2);
    sincospi(2.0 * (double)d / (double)N, &sv, &cv);
    const double R = kress[d];
    cd S[2], Dv[2], Kv[2], T[2];
    for (int ch = 0; ch < 2; ++ch) {
      const double kap = ch ? k1 : k;
      cd Snu;
      if (d == 0) {
        const cd lnk = mkc(-EULER_GAMMA / (2.0 * PI) - log(0.5 * kap * r) / (2.0 * PI), 0.25);
        S[ch] = cadd(mkc(-R * r / (4.0 * PI), 0.0), cscale(lnk, w2 * r));
        Snu = S[ch];
        Dv[ch] = Kv[ch] = mkc(-w2 / (4.0 * PI), 0.0);
      } else {
        const double rho = 2.0 * r * fabs(s2), lg = log(4.0 * s2 * s2);
        cd H0, H1;
        hankel01(kap * rho, H0, H1);
        const double J0 = H0.x, J1r = H1.x / rho;
        const cd F = mkc(-0.25 * H0.y * r, 0.25 * H0.x * r);         // (i/4) H0 r
        const double F1 = -J0 * r / (4.0 * PI);
        S[ch] = cadd(mkc(R * F1, 0.0), cscale(csub(F, mkc(F1 * lg, 0.0)), w2));
        const cd Fn = cscale(F, cv);                                  // times cos t
        Snu = cadd(mkc(R * F1 * cv, 0.0), cscale(csub(Fn, mkc(F1 * cv * lg, 0.0)), w2));
        const double dnt = -2.0 * r * r * s2 * s2, dnu = 2.0 * r * s2 * s2;
        const cd ikH1 = mkc(-0.25 * kap * H1.y, 0.25 * kap * H1.x);  // (i kap/4) H1
        const cd FD = cscale(ikH1, dnt / rho);
        const double F1D = -(kap / (4.0 * PI)) * J1r * dnt;
        Dv[ch] = cadd(mkc(R * F1D, 0.0), cscale(csub(FD, mkc(F1D * lg, 0.0)), w2));
        const cd FK = cscale(ikH1, -dnu * r / rho);
        const double F1K = (kap / (4.0 * PI)) * J1r * dnu * r;
        Kv[ch] = cadd(mkc(R * F1K, 0.0), cscale(csub(FK, mkc(F1K * lg, 0.0)), w2));
      }
      T[ch] = cadd(cscale(Z[ch * N + d], 1.0 / N), cscale(Snu, kap * kap));
    }
    const cd B11 = csub(Dv[0], Dv[1]);
    const cd B12 = cmul(mieta, csub(S[0], S[1]));
    const cd B21 = cmul(c, csub(T[0], cscale(T[1], varrho)));
    const cd B22 = cmul(cmul(c, mieta), csub(Kv[0], cscale(Kv[1], varrho)));
    row[d] = row[d + N] = B11;
    row[2 * N + d] = row[3 * N + d] = B12;
    row[4 * N + d] = row[5 * N + d] = B21;
    row[6 * N + d] = row[7 * N + d] = B22;
  }
}

static hipError_t launch_circ_rows_nys(Problem& pb) {
  hipLaunchKernelGGL(k_circ_rows_nys, dim3(pb.M), dim3(PC_THREADS), 4 * (size_t)pb.N * sizeof(cd), pb.stream, pb.N,
                     pb.pc_logN, pb.d_radii, pb.k, pb.k1, pb.eta, pb.varrho, pb.d_kress, pb.d_pc_tw, pb.d_circ);
  return hipGetLastError();
}

// L(kappa) of fibre blockIdx.x for the two row components 2 blockIdx.y and
// 2 blockIdx.y + 1, written with the identity added as the blocks of P:
// pfwd[fibre][kappa][B11, B12, B21, B22].
__global__ void __launch_bounds__(PC_THREADS) k_pc_lambda(const cd* __restrict__ circ, const cd* __restrict__ tw,
                                                           int N, int logN, cd* __restrict__ pfwd) {
  extern __shared__ cd pcs[];
  const int f = blockIdx.x, h = blockIdx.y;
  cd* X = pcs;
  cd* Y = pcs + 2 * N;
  const cd* row = circ + (size_t)f * 8 * N;
  for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) {
    const int j = i >> logN, d = i & (N - 1);
    X[i] = row[(2 * h + j) * 2 * N + d];
  }
  __syncthreads();
  const cd* L = pc_fft(X, Y, 2, N, logN, tw, false);
  for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) {
    const int j = i >> logN, kk = i & (N - 1);
    cd v = L[i];
    if (j == h) v.x += 1.0;            // components B11 (h = 0, j = 0) and B22 (h = 1, j = 1)
    pfwd[((size_t)f * N + kk) * 4 + 2 * h + j] = v;
  }
}

// per (fibre, mode): P^{-1} block = adj(P block) / det
__global__ void k_pc_invert(const cd* __restrict__ pfwd, cd* __restrict__ pinv, long long n_modes) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_modes) return;
  const cd a = pfwd[4 * i], b = pfwd[4 * i + 1], c = pfwd[4 * i + 2], d = pfwd[4 * i + 3];
  const cd idet = cdiv(mkc(1.0, 0.0), csub(cmul(a, d), cmul(b, c)));
  pinv[4 * i] = cmul(d, idet);
  pinv[4 * i + 1] = cmul(cscale(b, -1.0), idet);
  pinv[4 * i + 2] = cmul(cscale(c, -1.0), idet);
  pinv[4 * i + 3] = cmul(a, idet);
}

// out = blockdiag(P_f) in or blockdiag(P_f^{-1}) in, one workgroup per
// (fibre, batch member): the blocks do not depend on the angle, so the
// members of a batch share them; in and out may alias (a workgroup reads its
// fibre whole before writing).
__global__ void __launch_bounds__(PC_THREADS) k_pc_apply(const cd* in, cd* out, const cd* __restrict__ coef,
                                                          const cd* __restrict__ tw, int N, int logN) {
  extern __shared__ cd pcs[];
  const int f = blockIdx.x;
  const size_t mem = (size_t)blockIdx.y * gridDim.x * 2 * N;   // member offset: 2 M N
  cd* X = pcs;
  cd* Y = pcs + 2 * N;
  const cd* src = in + mem + (size_t)f * 2 * N;  // phi_f then varphi_f
  for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) X[i] = src[i];
  // with one mode per thread (N <= PC_THREADS) the mode block's loads are
  // issued now and land while the forward transforms run
  const bool one = N <= (int)blockDim.x;
  const int kk = threadIdx.x;
  cd c0 = mkc(0, 0), c1 = c0, c2 = c0, c3 = c0;
  if (one && kk < N) {
    const cd* c = coef + ((size_t)f * N + kk) * 4;
    c0 = c[0]; c1 = c[1]; c2 = c[2]; c3 = c[3];
  }
  __syncthreads();
  cd* H = pc_fft(X, Y, 2, N, logN, tw, true);
  if (one) {
    if (kk < N) {
      const cd u = H[kk], v = H[N + kk];
      H[kk] = cadd(cmul(c0, u), cmul(c1, v));
      H[N + kk] = cadd(cmul(c2, u), cmul(c3, v));
    }
  } else {
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
      const cd* c = coef + ((size_t)f * N + m) * 4;
      const cd u = H[m], v = H[N + m];
      H[m] = cadd(cmul(c[0], u), cmul(c[1], v));
      H[N + m] = cadd(cmul(c[2], u), cmul(c[3], v));
    }
  }
  __syncthreads();
  const cd* Z = pc_fft(H, H == X ? Y : X, 2, N, logN, tw, false);
  const double sc = 1.0 / N;
  cd* dst = out + mem + (size_t)f * 2 * N;
  for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) dst[i] = cscale(Z[i], sc);
}

hipError_t launch_precond_setup(Problem& pb) {
  const int N = pb.N;
  const size_t lds = 4 * (size_t)N * sizeof(cd);
  hipLaunchKernelGGL(k_pc_lambda, dim3(pb.M, 2), dim3(PC_THREADS), lds, pb.stream, pb.d_circ, pb.d_pc_tw, N,
                     pb.pc_logN, pb.d_pc_fwd);
  const long long nm = (long long)pb.M * N;
  hipLaunchKernelGGL(k_pc_invert, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, pb.stream, pb.d_pc_fwd,
                     pb.d_pc_inv, nm);
  return hipGetLastError();
}

hipError_t launch_precond(Problem& pb, const cd* in, cd* out, bool inverse, int B, hipStream_t st) {
  const int N = pb.N;
  const size_t lds = 4 * (size_t)N * sizeof(cd);
  hipLaunchKernelGGL(k_pc_apply, dim3(pb.M, std::max(1, B)), dim3(PC_THREADS), lds, st ? st : pb.stream, in, out,
                     inverse ? pb.d_pc_inv : pb.d_pc_fwd, pb.d_pc_tw, N, pb.pc_logN);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// translation tables (per wave): Hp_nu(kap d) for M2L offsets, Jp_nu(kap delta)
// for child-parent offsets, nu = -2p..2p, both wavenumbers.
// ---------------------------------------------------------------------------
template <int P>
__global__ void k_htab(int n_off, int n_tab, const double* __restrict__ off, double k, double k1, cd* tab) {
  constexpr int NT = 4 * P + 1;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * n_off) return;
  int ch = i / n_off, o = i - ch * n_off;
  double kap = ch ? k1 : k;
  double dx = off[2 * o], dy = off[2 * o + 1];
  double r = sqrt(dx * dx + dy * dy);
  double x = kap * r;
  cd e1 = mkc(dx / r, dy / r);             // e^{i theta}
  cd Hm1, Hn;
  hankel01(x, Hm1, Hn);                    // H_0, H_1
  cd* out = tab + ((size_t)ch * n_tab + o) * NT + 2 * P;
  out[0] = Hm1;
  cd en = e1;                              // e^{i n theta}
  cd Hprev = Hm1;
  double sgn = -1.0;
  for (int n = 1; n <= 2 * P; ++n) {
    cd v = cmul(Hn, en);
    out[n] = v;
    out[-n] = cscale(cconj(cmul(cconj(Hn), en)), sgn);   // (-1)^n H_n e^{-i n theta}
    cd Hnext = csub(cscale(Hn, 2.0 * n / x), Hprev);
    Hprev = Hn;
    Hn = Hnext;
    en = cmul(en, e1);
    sgn = -sgn;
  }
}

template <int P>
__global__ void k_jtab(int n_off, const double* __restrict__ off, double k, double k1, cd* tab) {
  constexpr int NT = 4 * P + 1;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * n_off) return;
  int ch = i / n_off, o = i - ch * n_off;
  double kap = ch ? k1 : k;
  cd jp[2 * P + 1];
  jplus_seq<2 * P>(kap * off[2 * o], kap * off[2 * o + 1], jp);
  cd* out = tab + (size_t)i * NT + 2 * P;
  double sgn = 1.0;
#pragma unroll
  for (int n = 0; n <= 2 * P; ++n) {
    out[n] = jp[n];
    out[-n] = cscale(cconj(jp[n]), sgn);
    sgn = -sgn;
  }
}

// ---------------------------------------------------------------------------
// lattice sums of the top-level M2L (Sec. 3.3):
//   S_nu(o) = sum_{m outside [m_lo, m_hi]} alpha^m Hp_nu(k (o - m h))
// direct for |m| <= q, tails for |m| > q as contour integrals in s
// (t = +-s sqrt(s^2 - 2ik), mu = s^2 - ik, dt/mu = 2 ds / sqrt(s^2 - 2ik)).
// ---------------------------------------------------------------------------
// Tails of the lattice sums (both sides |m| > q), from the corrected contour
// integrals: for the rule point s with t = +-s sqrt(s^2 - 2ik), mu = s^2 - ik,
//   up:   exp(i X t + mu Y + (q+1)(i beta - mu H)) / (1 - e^{i beta - mu H}),
//   down: exp(i X t - mu Y - (q+1)(i beta + mu H)) / (1 - e^{-i beta - mu H}),
// times 2 w / sqrt(s^2 - 2ik) and the order factors (-i(t +- mu)/k)^nu
// (nu >= 0) or (i(t -+ mu)/k)^|nu| (nu < 0).  One thread per rule point
// carries all orders by running products.  The sums over the workgroup's 256
// points go through LDS a few orders at a time: every thread stores its terms
// of LT_NB orders (both signs), then 32 threads per term add eight points
// each and a 32-lane butterfly finishes the sum (far fewer cross-lane moves
// than a full-wave butterfly per order).  Partial sums per (member, offset,
// rule block) are added by k_lattice_direct.
// sum of a complex value over the 64 lanes of a wavefront (every lane gets it)
__device__ __forceinline__ cd wave_sum(cd v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}

constexpr int LAT_MAX_P = 40;           // largest expansion order (the options accept p <= 40)
constexpr int LAT_MAX_NT = 4 * LAT_MAX_P + 1;
constexpr int LT_NB = 4;                 // orders per LDS round of k_lattice_tails

__global__ void __launch_bounds__(256) k_lattice_tails(int P, int n_roff, const double* __restrict__ roff,
                                                       double k, double H, const double* __restrict__ betas,
                                                       int q, const double* __restrict__ rule, int n_rule,
                                                       cd* __restrict__ partial) {
  __shared__ cd sv[2 * LT_NB][256];
  const int NT = 4 * P + 1;
  const int o = blockIdx.x, rb = blockIdx.y, mb = blockIdx.z;
  const double beta = betas[mb];
  const double ox = roff[2 * o], oy = roff[2 * o + 1];
  const double invk = 1.0 / k;
  const int i = rb * 256 + threadIdx.x;
  // running products per branch: up/down x positive/negative orders
  cd aup[2], adn[2], bup[2], bdn[2];      // a*: orders >= 0, b*: orders < 0
  cd zup[2], zdn[2], yup[2], ydn[2];
  for (int br = 0; br < 2; ++br) {
    aup[br] = adn[br] = bup[br] = bdn[br] = mkc(0, 0);
    zup[br] = zdn[br] = yup[br] = ydn[br] = mkc(0, 0);
  }
  if (i < n_rule) {
    double s = rule[i], wgt = rule[n_rule + i];
    cd root = csqrt(mkc(s * s, -2.0 * k));
    cd mu = mkc(s * s, -k);
    cd jac = cdiv(mkc(2.0 * wgt, 0.0), root);
    cd emh = cexp(mkc(-mu.x * H, -mu.y * H));                  // e^{-mu H}
    cd eib = mkc(cos(beta), sin(beta));
    cd den_up = csub(mkc(1, 0), cmul(eib, emh));
    cd den_dn = csub(mkc(1, 0), cmul(cconj(eib), emh));
    for (int br = 0; br < 2; ++br) {
      cd tt = cscale(root, br ? -s : s);
      cd itx = cmul_i(cscale(tt, ox));
      cd ex_up = cadd(itx, cadd(cscale(mu, oy), cscale(csub(mkc(0, beta), cscale(mu, H)), q + 1.0)));
      cd ex_dn = cadd(itx, csub(cscale(mu, -oy), cscale(cadd(mkc(0, beta), cscale(mu, H)), q + 1.0)));
      cd fu = cmul(jac, cdiv(cexp(ex_up), den_up));
      cd fd = cmul(jac, cdiv(cexp(ex_dn), den_dn));
      cd tpm = cadd(tt, mu), tmm = csub(tt, mu);
      aup[br] = bup[br] = fu;
      adn[br] = bdn[br] = fd;
      zup[br] = cscale(mkc(tpm.y, -tpm.x), invk);     // -i (t + mu) / k
      zdn[br] = cscale(mkc(tmm.y, -tmm.x), invk);     // -i (t - mu) / k
      yup[br] = cscale(mkc(-tmm.y, tmm.x), invk);     //  i (t - mu) / k
      ydn[br] = cscale(mkc(-tpm.y, tpm.x), invk);     //  i (t + mu) / k
    }
  }
  cd* out = partial + (((size_t)mb * n_roff + o) * gridDim.y + rb) * NT;
  const int term = threadIdx.x >> 5, seg = threadIdx.x & 31;
  for (int nu0 = 0; nu0 <= 2 * P; nu0 += LT_NB) {
#pragma unroll
    for (int j = 0; j < LT_NB; ++j) {
      // order nu0 + j: term 2j holds +nu, term 2j + 1 holds -nu
      sv[2 * j][threadIdx.x] = cadd(cadd(aup[0], adn[0]), cadd(aup[1], adn[1]));
      sv[2 * j + 1][threadIdx.x] = cadd(cadd(bup[0], bdn[0]), cadd(bup[1], bdn[1]));
      for (int br = 0; br < 2; ++br) {
        aup[br] = cmul(aup[br], zup[br]);
        adn[br] = cmul(adn[br], zdn[br]);
        bup[br] = cmul(bup[br], yup[br]);
        bdn[br] = cmul(bdn[br], ydn[br]);
      }
    }
    __syncthreads();
    cd a = sv[term][seg];
#pragma unroll
    for (int r = 1; r < 8; ++r) a = cadd(a, sv[term][seg + 32 * r]);
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) {
      a.x += __shfl_xor(a.x, off, 64);
      a.y += __shfl_xor(a.y, off, 64);
    }
    const int nu = nu0 + (term >> 1);
    if (seg == 0 && nu <= 2 * P) {
      if (!(term & 1)) out[2 * P + nu] = a;
      else if (nu > 0) out[2 * P - nu] = a;
    }
    __syncthreads();
  }
}

// Direct part of the lattice sums, the images |m| <= q outside the explicit
// range [m_lo, m_hi] of the offset:
//   S_nu(o) = sum_m alpha^m Hp_nu(k (o - m H e_y)),  Hp_nu(v) = H_|nu|(|v|) e^{i nu arg v}
//             (times (-1)^nu for nu < 0),
// plus the tails of k_lattice_tails times 1/(i pi).  One workgroup per
// (offset, member).  The images go in chunks of LD_CH: one thread per image
// evaluates H_0, H_1 and the upward recurrence to H_{2P}, its angle and
// alpha^m into LDS; then one thread per order adds the chunk's images in
// increasing m.
constexpr int LD_CH = 16;

__global__ void __launch_bounds__(128) k_lattice_direct(int P, int n_roff, const double* __restrict__ roff,
                                                        const int* __restrict__ mrange, double k, double H,
                                                        const double* __restrict__ betas, int q, int n_rblk,
                                                        const cd* __restrict__ partial, cd* out,
                                                        long long out_stride) {
  __shared__ cd sH[LD_CH][2 * LAT_MAX_P + 1];
  __shared__ cd sAl[LD_CH];
  __shared__ double sTh[LD_CH];
  const int o = blockIdx.x, mb = blockIdx.y;
  const int NT = 4 * P + 1;
  const double beta = betas[mb];
  const double ox = roff[2 * o], oy = roff[2 * o + 1];
  const int mlo = mrange[2 * o], mhi = mrange[2 * o + 1];
  const int nex = mhi >= mlo ? mhi - mlo + 1 : 0;     // excluded images (inside [-q, q])
  const int n_img = 2 * q + 1 - nex;
  cd acc[2] = {mkc(0, 0), mkc(0, 0)};                 // orders threadIdx.x, threadIdx.x + 128
  for (int c0 = 0; c0 < n_img; c0 += LD_CH) {
    const int cnt = min(LD_CH, n_img - c0);
    if ((int)threadIdx.x < cnt) {
      int m = -q + c0 + (int)threadIdx.x;
      if (nex > 0 && m >= mlo) m += nex;
      const double vx = ox, vy = oy - m * H;
      const double x = k * sqrt(vx * vx + vy * vy);
      cd Hp, Hc;
      hankel01(x, Hp, Hc);
      cd* hr = sH[threadIdx.x];
      hr[0] = Hp;
      if (P > 0) hr[1] = Hc;
      for (int n = 1; n < 2 * P; ++n) {
        cd Hx = csub(cscale(Hc, 2.0 * n / x), Hp);
        Hp = Hc;
        Hc = Hx;
        hr[n + 1] = Hc;
      }
      sTh[threadIdx.x] = atan2(vy, vx);
      double sb, cb;
      sincos(m * beta, &sb, &cb);
      sAl[threadIdx.x] = mkc(cb, sb);
    }
    __syncthreads();
    for (int h = 0; h < 2; ++h) {
      const int t = threadIdx.x + 128 * h;
      if (t >= NT) break;
      const int nu = t - 2 * P;
      const int an = nu < 0 ? -nu : nu;
      cd a = acc[h];
      for (int j = 0; j < cnt; ++j) {
        double s, c;
        sincos(nu * sTh[j], &s, &c);
        cd v = cmul(sH[j][an], mkc(c, s));
        if (nu < 0 && (an & 1)) v = cscale(v, -1.0);
        a = cfma(sAl[j], v, a);
      }
      acc[h] = a;
    }
    __syncthreads();
  }
  const cd* part = partial + ((size_t)mb * n_roff + o) * n_rblk * NT;
  for (int h = 0; h < 2; ++h) {
    const int t = threadIdx.x + 128 * h;
    if (t >= NT) break;
    cd tail = mkc(0, 0);
    for (int rb = 0; rb < n_rblk; ++rb) tail = cadd(tail, part[(size_t)rb * NT + t]);
    // 1/(i pi) * tail
    tail = mkc(tail.y / PI, -tail.x / PI);
    out[mb * out_stride + (size_t)o * NT + t] = cadd(acc[h], tail);
  }
}

// ---------------------------------------------------------------------------
// Root lattice M2L (Sec. 3.3) as a convolution over the fibre grid.  With
// fibre f at (sublattice s, gx, gy) and the lattice row of a root pair
// depending only on (s_t, s_s, dgx, dgy), the M2L of every root,
//   L_l(t) = sum_s sum_n S_{n-l}(o_ts) M_n(s),
// is for each (l, n) a 2D linear convolution over the grid, done as a product
// of zero-padded DFTs on the px x py grid (px = 2 gx, py = 2 gy):
//   Shat_nu(xi) = DFT of S_nu over the displacements (once per frequency),
//   Xhat_n(xi) = DFT of M_n over the grid, Lhat_l(xi) = sum_n Shat_{n-l} Xhat_n,
// and L_l = inverse DFT of Lhat_l at the grid points.  The DFTs are direct sums
// over each grid axis (at most 64 points) with tabulated roots of unity.
// ---------------------------------------------------------------------------
__device__ __forceinline__ cd unit_root(int k, int n, double sign) {
  double s, c;
  sincospi(sign * 2.0 * (double)k / (double)n, &s, &c);
  return mkc(c, s);
}

// One block per (order nu, sublattice pair, member): the rows over the
// padded grid (K[y][x] at x = dgx mod px, y = dgy mod py), then DFT along x
// and along y into shat[member][pair][xi][nu].
__global__ void __launch_bounds__(256) k_lat_shat(const cd* __restrict__ lat, long long lat_stride,
                                                  const int* __restrict__ key, int ns, int gx, int gy, int px,
                                                  int py, int NT, cd* __restrict__ shat) {
  __shared__ cd sk[LAT_PXY_MAX], tmp[LAT_PXY_MAX], wx[64], wy[64];
  const int nu = blockIdx.x, pair = blockIdx.y, st = pair / ns, ss = pair - st * ns;
  const int pxy = px * py;
  lat += blockIdx.z * lat_stride;
  shat += ((size_t)blockIdx.z * ns * ns + pair) * pxy * NT;
  for (int i = threadIdx.x; i < px; i += 256) wx[i] = unit_root(i, px, -1.0);
  for (int i = threadIdx.x; i < py; i += 256) wy[i] = unit_root(i, py, -1.0);
  for (int idx = threadIdx.x; idx < pxy; idx += 256) {
    const int x = idx % px, y = idx / px;
    const int dx = x < gx ? x : x - px, dy = y < gy ? y : y - py;
    cd v = mkc(0, 0);
    if (dx > -gx && dy > -gy) {
      const int r = key[(((size_t)st * ns + ss) * (2 * gy - 1) + dy + gy - 1) * (2 * gx - 1) + dx + gx - 1];
      if (r >= 0) v = lat[(size_t)r * NT + nu];
    }
    sk[idx] = v;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < pxy; idx += 256) {
    const int fx = idx % px, y = idx / px;
    cd s = mkc(0, 0);
    for (int x = 0; x < px; ++x) s = cfma(sk[y * px + x], wx[(fx * x) % px], s);
    tmp[idx] = s;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < pxy; idx += 256) {
    const int fx = idx % px, fy = idx / px;
    cd s = mkc(0, 0);
    for (int y = 0; y < py; ++y) s = cfma(tmp[y * px + fx], wy[(fy * y) % py], s);
    shat[(size_t)idx * NT + nu] = s;
  }
}

// One block per (order n, sublattice, member): the roots' exterior multipoles
// on the grid, DFT along x and y into xhat[member][s][xi][n].
template <int P>
__global__ void __launch_bounds__(256) k_lat_fwd(const cd* __restrict__ mpole, long long mp_stride,
                                                 const int* __restrict__ cell, int ns, int gx, int gy, int px,
                                                 int py, cd* __restrict__ xhat) {
  constexpr int NP = 2 * P + 1;
  __shared__ cd sk[LAT_PXY_MAX], tmp[LAT_PXY_MAX], wx[64], wy[64];
  const int n = blockIdx.x, s = blockIdx.y, pxy = px * py;
  mpole += blockIdx.z * mp_stride;
  xhat += ((size_t)blockIdx.z * ns + s) * pxy * NP;
  for (int i = threadIdx.x; i < px; i += 256) wx[i] = unit_root(i, px, -1.0);
  for (int i = threadIdx.x; i < py; i += 256) wy[i] = unit_root(i, py, -1.0);
  for (int idx = threadIdx.x; idx < gx * gy; idx += 256) {
    const int c = cell[(size_t)s * gx * gy + idx];
    sk[idx] = c >= 0 ? mpole[((size_t)c * 2) * NP + n] : mkc(0, 0);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < gy * px; idx += 256) {
    const int fx = idx % px, y = idx / px;
    cd a = mkc(0, 0);
    for (int x = 0; x < gx; ++x) a = cfma(sk[y * gx + x], wx[(fx * x) % px], a);
    tmp[idx] = a;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < pxy; idx += 256) {
    const int fx = idx % px, fy = idx / px;
    cd a = mkc(0, 0);
    for (int y = 0; y < gy; ++y) a = cfma(tmp[y * px + fx], wy[(fy * y) % py], a);
    xhat[(size_t)idx * NP + n] = a;
  }
}

// One wavefront per (grid frequency, target sublattice, member), lane = order
// l: Lhat_l = sum over source sublattices and n of Shat_{n-l} Xhat_n.
template <int P>
__global__ void __launch_bounds__(64) k_lat_mul(const cd* __restrict__ shat, const cd* __restrict__ xhat, int ns,
                                                int pxy, cd* __restrict__ lhat) {
  constexpr int NP = 2 * P + 1, NT = 4 * P + 1;
  __shared__ cd sS[2][NT], sX[2][NP];
  const int xi = blockIdx.x, st = blockIdx.y, b = blockIdx.z, lane = threadIdx.x;
  for (int ss = 0; ss < ns; ++ss) {
    const cd* sr = shat + ((((size_t)b * ns + st) * ns + ss) * pxy + xi) * NT;
    const cd* xr = xhat + (((size_t)b * ns + ss) * pxy + xi) * NP;
    for (int i = lane; i < NT; i += 64) sS[ss][i] = sr[i];
    for (int i = lane; i < NP; i += 64) sX[ss][i] = xr[i];
  }
  __syncthreads();
  cd* out = lhat + (((size_t)b * ns + st) * pxy + xi) * NP;
  for (int l = lane; l < NP; l += 64) {
    cd a = mkc(0, 0);
    for (int ss = 0; ss < ns; ++ss)
      for (int n = 0; n < NP; ++n) a = cfma(sS[ss][n - l + 2 * P], sX[ss][n], a);
    out[l] = a;
  }
}

// One block per (order l, sublattice, member): inverse DFT along y and x at
// the grid points, scaled by 1 / (px py), into the roots' M2L partial slots.
template <int P>
__global__ void __launch_bounds__(256) k_lat_inv(const cd* __restrict__ lhat, const int* __restrict__ slot, int ns,
                                                 int gx, int gy, int px, int py, cd* __restrict__ epart,
                                                 long long ep_stride) {
  constexpr int NP = 2 * P + 1;
  __shared__ cd sk[LAT_PXY_MAX], tmp[LAT_PXY_MAX], wx[64], wy[64];
  const int l = blockIdx.x, s = blockIdx.y, pxy = px * py;
  lhat += ((size_t)blockIdx.z * ns + s) * pxy * NP;
  epart += blockIdx.z * ep_stride;
  for (int i = threadIdx.x; i < px; i += 256) wx[i] = unit_root(i, px, 1.0);
  for (int i = threadIdx.x; i < py; i += 256) wy[i] = unit_root(i, py, 1.0);
  for (int idx = threadIdx.x; idx < pxy; idx += 256) sk[idx] = lhat[(size_t)idx * NP + l];
  __syncthreads();
  for (int idx = threadIdx.x; idx < gy * px; idx += 256) {
    const int fx = idx % px, y = idx / px;
    cd a = mkc(0, 0);
    for (int fy = 0; fy < py; ++fy) a = cfma(sk[fy * px + fx], wy[(fy * y) % py], a);
    tmp[idx] = a;
  }
  __syncthreads();
  const double sc = 1.0 / (double)pxy;
  for (int idx = threadIdx.x; idx < gx * gy; idx += 256) {
    const int x = idx % gx, y = idx / gx;
    cd a = mkc(0, 0);
    for (int fx = 0; fx < px; ++fx) a = cfma(tmp[y * px + fx], wx[(fx * x) % px], a);
    const int sl = slot[(size_t)s * gx * gy + idx];
    if (sl >= 0) epart[(size_t)sl * NP + l] = cscale(a, sc);
  }
}

hipError_t launch_lattice_sums(Problem& pb, int B) {
  int n_roff = (int)pb.hp.root_off_xy.size() / 2;
  if (n_roff == 0) return hipSuccess;
  const int NT = 4 * pb.opt.p + 1;
  int n_rblk = (pb.n_srule + 255) / 256;
  hipLaunchKernelGGL(k_lattice_tails, dim3(n_roff, n_rblk, B), dim3(256), 0, pb.stream, pb.opt.p, n_roff,
                     pb.d_root_off_xy, pb.k, pb.H, pb.d_betas, pb.lattice_q, pb.d_srule, pb.n_srule,
                     pb.d_latpart);
  hipLaunchKernelGGL(k_lattice_direct, dim3(n_roff, B), dim3(128), 0, pb.stream, pb.opt.p, n_roff,
                     pb.d_root_off_xy, pb.d_root_mrange, pb.k, pb.H, pb.d_betas, pb.lattice_q, n_rblk,
                     pb.d_latpart, pb.d_lat, 2LL * pb.n_tab * NT);
  if (pb.lat_fft)
    hipLaunchKernelGGL(k_lat_shat, dim3(NT, pb.lat_ns * pb.lat_ns, B), dim3(256), 0, pb.stream, pb.d_lat,
                       2LL * pb.n_tab * NT, pb.d_lat_key, pb.lat_ns, pb.lat_gx, pb.lat_gy, pb.lat_px, pb.lat_py, NT,
                       pb.d_lat_shat);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// right-hand side B of eq. (9)
// ---------------------------------------------------------------------------
__global__ void k_rhs(int E, int N, const double* mx, const double* my, const double* tx,
                      const double* ty, double k, double th, double eta, double varrho, cd* b) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double d1 = cos(th), d2 = sin(th);
  double ph = k * (mx[e] * d1 + my[e] * d2);
  cd u = mkc(cos(ph), sin(ph));
  double dn = k * (ty[e] * d1 - tx[e] * d2);               // k (d . nu)
  cd du = cscale(cmul_i(u), dn);                            // i k (d.nu) u
  int f = e / N, l = e - f * N;
  b[2 * f * N + l] = mkc(-u.x, -u.y);
  double s = 2.0 / (eta * (1.0 + varrho));
  b[2 * f * N + N + l] = cscale(cmul_i(du), s);             // 2i/(eta(1+varrho)) du
}

hipError_t launch_rhs(Problem& pb, double theta, cd* d_b) {
  hipLaunchKernelGGL(k_rhs, dim3((pb.E + 255) / 256), dim3(256), 0, pb.stream, pb.E, pb.N, pb.d_mx,
                     pb.d_my, pb.d_tx, pb.d_ty, pb.k, theta, pb.eta, pb.varrho, d_b);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Bragg amplitudes: one workgroup per order, G = 8 Gauss points per element
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_fields(int E, int N, int n_orders, const double* mx,
                                                const double* my, const double* tx, const double* ty,
                                                const double* h, const double* gl8, int G, double k,
                                                double th, double H, double eta, const cd* psi,
                                                cd* out) {
  int n = (int)blockIdx.x - n_orders;
  double kap = k * sin(th) + 2.0 * PI * n / H;
  double g2 = k * k - kap * kap;
  cd gam = g2 >= 0 ? mkc(sqrt(g2), 0.0) : mkc(0.0, sqrt(-g2));
  cd accT = mkc(0, 0), accR = mkc(0, 0);
  for (int e = threadIdx.x; e < E; e += blockDim.x) {
    int f = e / N, l = e - f * N;
    cd ph = psi[2 * f * N + l], vp = psi[2 * f * N + N + l];
    double n1 = ty[e], n2 = -tx[e];
    for (int g = 0; g < G; ++g) {
      double s = 0.5 * h[e] * gl8[g], w = 0.5 * h[e] * gl8[G + g];
      double y1 = mx[e] + s * tx[e], y2 = my[e] + s * ty[e];
      // T: e^{-i(gam y1 + kap y2)} [ (gam n1 + kap n2) phi + eta varphi ]
      cd argT = cmul_i(mkc(-(gam.x * y1 + kap * y2), -gam.y * y1));
      cd fT = cadd(cmul(mkc(gam.x * n1 + kap * n2, gam.y * n1), ph), cscale(vp, eta));
      accT = cfma(cscale(cexp(argT), w), fT, accT);
      // R: e^{i(gam y1 - kap y2)} [ -(gam n1 - kap n2) phi + eta varphi ]
      cd argR = cmul_i(mkc(gam.x * y1 - kap * y2, gam.y * y1));
      cd fR = cadd(cmul(mkc(-(gam.x * n1 - kap * n2), -gam.y * n1), ph), cscale(vp, eta));
      accR = cfma(cscale(cexp(argR), w), fR, accR);
    }
  }
  __shared__ cd sT[256], sR[256];
  sT[threadIdx.x] = accT;
  sR[threadIdx.x] = accR;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sT[threadIdx.x] = cadd(sT[threadIdx.x], sT[threadIdx.x + s]);
      sR[threadIdx.x] = cadd(sR[threadIdx.x], sR[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cd den = cscale(gam, 2.0 * H);
    out[2 * blockIdx.x] = cdiv(sR[0], den);
    out[2 * blockIdx.x + 1] = cdiv(sT[0], den);
  }
}

hipError_t launch_fields(Problem& pb, const cd* d_psi, int n_orders, cd* d_out) {
  // the 8-point Gauss rule on every chord, or the Nystrom nodes (point rule)
  hipLaunchKernelGGL(k_fields, dim3(2 * n_orders + 1), dim3(256), 0, pb.stream, pb.E, pb.N, n_orders,
                     pb.d_mx, pb.d_my, pb.d_tx, pb.d_ty, pb.d_h, pb.nystrom ? pb.d_gl : pb.d_gl16 + 32,
                     pb.nystrom ? 1 : 8, pb.k, pb.theta, pb.H, pb.eta, d_psi, d_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Bessel test hook
// ---------------------------------------------------------------------------
__global__ void k_bessel(const double* x, int n, double* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a, b, c, d;
  bessel_jy01(x[i], a, b, c, d);
  out[4 * i] = a;
  out[4 * i + 1] = b;
  out[4 * i + 2] = c;
  out[4 * i + 3] = d;
}

hipError_t launch_bessel_test(const double* d_x, int n, double* d_out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bessel, dim3((n + 255) / 256), dim3(256), 0, s, d_x, n, d_out);
  return hipGetLastError();
}

// ===========================================================================
// The operator apply (hot path)
// ===========================================================================

// Distances between consecutive members of a batch in the per-member buffers.
struct BatchStrides { long long vec, mpole, part, epart, tab; int alpha; };
static BatchStrides batch_strides(const Problem& pb) {
  const int NP = 2 * pb.opt.p + 1, NT = 4 * pb.opt.p + 1;
  BatchStrides s;
  s.vec = 2LL * pb.E;
  s.mpole = (long long)pb.hp.cells.size() * 2 * NP;
  s.part = (long long)std::max(1, pb.n_chunks) * NP;
  s.epart = (long long)std::max(1, pb.n_mchunks) * NP;
  s.tab = 2LL * pb.n_tab * NT;
  s.alpha = pb.hp.m_max - pb.hp.m_min + 1;
  return s;
}

// P2M: multipole moments at the leaves, both wavenumbers (Sec. 3.2, MM of
// S-bar and D-bar combined as in the representation D phi - i eta S varphi):
//   M_n(C) = (i/4) sum_{e in C} sum_g w_g [ dJm_n/dn_y phi_e - i eta Jm_n varphi_e ],
//   dJm_n/dn_y = (kap/2) (conj(nu) Jm_{n-1} - nu Jm_{n+1}),  nu = n1 + i n2,
// i.e. per Gauss point M_n += w0 Jm_n + wm Jm_{n-1} + wp Jm_{n+1}.
// Two wavefronts per (leaf, channel): both walk every Gauss point of the leaf
// (one point per lane at a time) through the orders |n| = 0..p with a window
// of three Jm values; wavefront W accumulates the orders M_LO(W) <= |n| <= M_HI(W)
// in registers.  Orders m and -m share their products through
// Jm_{-j} = (-1)^j conj(Jm_j): with s = (-1)^m, K = Jm_{m-1} - conj(Jm_{m+1})
// and K' = Jm_{m-1} + conj(Jm_{m+1}) the lane keeps
//   Pm = (M_m + s M_{-m}) / 2 = sum w0 Re(Jm_m) + (wm K - wp conj(K)) / 2,
//   Qm = (M_m - s M_{-m}) / 2 = sum i w0 Im(Jm_m) + (wm K' + wp conj(K')) / 2,
// whose real and imaginary parts take 12 FMA with the point weights
// (wm + wp)/2 and (wm - wp)/2 (against 24 for M_m and M_{-m} apart), and
// turns them into M_m = Pm + Qm, M_{-m} = s (Pm - Qm) once at the end.  One
// LDS transpose per wavefront sums the lanes.
template <int P, int W>
struct P2MHalf {
  static constexpr int HALF = P / 2;
  static constexpr int LO = W == 0 ? 0 : HALF + 1;
  static constexpr int HI = W == 0 ? HALF : P;
  // slots: orders +m at [m - LO], orders -m (m >= max(LO,1)) after them
  static constexpr int NPOS = HI - LO + 1;
  static constexpr int NNEG = HI - (LO > 0 ? LO : 1) + 1;
  static constexpr int NS = NPOS + NNEG;
};

// A leaf's rows staged in LDS: element midpoint relative to the leaf centre,
// unit tangent, chord length and the two densities, plus the Gauss rule.
struct P2MRows {
  double x[64], y[64], tx[64], ty[64], h[64];
  cd phi[64], vphi[64];
  double gl[32];
};

// Accumulates into acc (the first H::NS slots; the caller zeroes them) the
// raw slot sums of this wavefront's half of the orders over its points;
// p2m_fold turns them into moments once every point is in.
template <int P, int W, int NA>
__device__ __forceinline__ void p2m_half(cd (&acc)[NA], int first, int stride, int npts, int G, double kap,
                                         double eta, const P2MRows& rw) {
  using H = P2MHalf<P, W>;
  static_assert(H::NS <= NA, "slots");
  constexpr int M1 = H::LO > 0 ? H::LO : 1;   // first order with a +- pair
  // slot of order +m: m - LO (Pm for m >= 1); slot of order -m: NPOS + m - M1 (Qm)
  for (int pt = first; pt < npts; pt += stride) {
    int q = pt / G;
    int g = pt - q * G;
    cd phi = rw.phi[q], vphi = rw.vphi[q];
    double etx = rw.tx[q], ety = rw.ty[q], hh = rw.h[q];
    double s = 0.5 * hh * rw.gl[g], w = 0.125 * hh * rw.gl[G + g];
    double vx = kap * (rw.x[q] + s * etx), vy = kap * (rw.y[q] + s * ety);
    // (i/4) w [ -i eta varphi | (kap/2) conj(nu) phi | -(kap/2) nu phi ], nu = (ty, -tx):
    // w0 = eta w varphi, wm = i (ty + i tx) phi sk, wp = -i (ty - i tx) phi sk, sk = kap w / 2
    const double sk = 0.5 * kap * w;
    cd w0 = cscale(vphi, eta * w);
    cd ah = cscale(phi, -sk * etx);                                // (wm + wp) / 2
    cd bh = mkc(-sk * ety * phi.y, sk * ety * phi.x);               // (wm - wp) / 2
    double gs[H::HI + 2];                                          // h_n = g_n / n!
    scaled_h<H::HI + 1>(0.25 * (vx * vx + vy * vy), gs);
    cd hv = mkc(0.5 * vx, -0.5 * vy);                              // conj(v)/2
    cd uu = hv;                                                    // (conj(v)/2)^n
    cd J0 = mkc(gs[0], 0.0);                                       // Jm_0
    cd J1 = cscale(uu, gs[1]);                                     // Jm_1
    cd Jprev = cscale(cconj(J1), -1.0);                            // Jm_{-1}
#pragma unroll
    for (int m = 0; m <= H::HI; ++m) {
      if (m >= H::LO) {
        if (m == 0) {
          cd wm = cadd(ah, bh), wp = csub(ah, bh);
          acc[0] = cfma(wp, J1, cfma(wm, Jprev, cfma(w0, J0, acc[0])));
        } else {
          const int jp = m - H::LO, jn = H::NPOS + m - M1;
          const double kx = Jprev.x - J1.x, ky = Jprev.y + J1.y;     // K
          const double kpx = Jprev.x + J1.x, kpy = Jprev.y - J1.y;   // K'
          acc[jp].x = fma(w0.x, J0.x, fma(bh.x, kx, fma(-ah.y, ky, acc[jp].x)));
          acc[jp].y = fma(w0.y, J0.x, fma(ah.x, ky, fma(bh.y, kx, acc[jp].y)));
          acc[jn].x = fma(-w0.y, J0.y, fma(ah.x, kpx, fma(-bh.y, kpy, acc[jn].x)));
          acc[jn].y = fma(w0.x, J0.y, fma(bh.x, kpy, fma(ah.y, kpx, acc[jn].y)));
        }
      }
      if (m < H::HI) {
        uu = cmul(uu, hv);
        Jprev = J0;
        J0 = J1;
        J1 = cscale(uu, gs[m + 2]);
      }
    }
  }
}

// The slot sums of p2m_half as moments: orders m and -m from the sums P_m
// and Q_m of their shared products.
template <int P, int W, int NA>
__device__ __forceinline__ void p2m_fold(cd (&acc)[NA]) {
  using H = P2MHalf<P, W>;
  constexpr int M1 = H::LO > 0 ? H::LO : 1;   // first order with a +- pair
#pragma unroll
  for (int m = M1; m <= H::HI; ++m) {
    const int jp = m - H::LO, jn = H::NPOS + m - M1;
    const cd pm = acc[jp], qm = acc[jn];
    acc[jp] = cadd(pm, qm);
    acc[jn] = cscale(csub(pm, qm), (m & 1) ? -1.0 : 1.0);
  }
}

// Sum over the 64 lanes of a wavefront of NA complex slots held by every
// lane, by recursive halving: at each step a lane keeps half of its live
// slots (the upper half when its lane bit m is set), sends the other half to
// lane ^ m and adds what that lane sends for the half it keeps.  With
// V = 32 live slots at the start (NA <= 32) five steps leave lanes 2s and
// 2s + 1 with halves of slot s, and one more exchange completes both; with
// V = 64 six steps leave lane s with slot s.  Slots past NA are zero.
// Returns the total of slot lane >> 1 (V = 32) or slot lane (V = 64).
template <int NA>
__device__ __forceinline__ cd wave_sum_slots(cd (&a)[NA], int lane) {
  constexpr int V = NA <= 32 ? 32 : 64;
  static_assert(NA <= 64, "at most 64 slots");
  constexpr int STEPS = V == 32 ? 5 : 6;
#pragma unroll
  for (int step = 0; step < STEPS; ++step) {
    const int h = (V >> step) >> 1, m = 32 >> step;
    const bool up = (lane & m) != 0;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      if (i >= h) break;
      const cd lo = i < NA ? a[i] : mkc(0, 0);
      const cd hi = i + h < NA ? a[i + h] : mkc(0, 0);
      const cd keep = up ? hi : lo, send = up ? lo : hi;
      cd got;
      got.x = __shfl_xor(send.x, m, 64);
      got.y = __shfl_xor(send.y, m, 64);
      if (i < NA) a[i] = cadd(keep, got);
    }
  }
  cd r = a[0];
  if (V == 32) {
    r.x += __shfl_xor(r.x, 1, 64);
    r.y += __shfl_xor(r.y, 1, 64);
  }
  return r;
}

// PS groups of two wavefronts per (leaf, channel): group g walks the Gauss
// points g*64 + lane, g*64 + lane + 64 PS, ...  Each wavefront sums its
// lanes' partial moments by a butterfly across the lanes (no LDS round
// trips); with PS > 1 the groups' sums meet in LDS in a fixed order.
// The moments of cell `cell` about its centre for channel ch and batch
// member `mem`, by the 128 PS threads of the calling workgroup: its `rows`
// elements are rows rb.. of the geometry arrays (offset from the cell's
// centre, tangent; chord length; index of phi in Psi), staged in LDS 64 at a
// time.
template <int P, int PS>
__device__ __forceinline__ void p2m_cell(int cell, int rb, int rows, int ch, int mem,
                                         const double4* __restrict__ tgeo, const double* __restrict__ trh,
                                         const int* __restrict__ psi_idx, const double* __restrict__ gl, int G,
                                         int N, double k, double k1, double eta, const cd* __restrict__ psi,
                                         cd* __restrict__ mpole, long long psi_stride, long long mp_stride) {
  constexpr int NP = 2 * P + 1;
  constexpr int NA = P2MHalf<P, 0>::NS > P2MHalf<P, 1>::NS ? P2MHalf<P, 0>::NS : P2MHalf<P, 1>::NS;
  constexpr int SPL = NA <= 32 ? 2 : 1;         // lanes per slot after the butterfly
  // each chunk of 64 rows is loaded once by the first wavefront; the point
  // loop then reads only LDS
  __shared__ P2MRows rw;
  __shared__ cd grp_sum[PS > 1 ? PS - 1 : 1][2][64];
  psi += mem * psi_stride;
  mpole += mem * mp_stride;
  double kap = ch ? k1 : k;
  int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int half = wv & 1, grp = wv >> 1;
  cd acc[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) acc[j] = mkc(0, 0);
  for (int r0 = 0; r0 < rows; r0 += 64) {
    const int nr = rows - r0 < 64 ? rows - r0 : 64;
    if (r0 > 0) __syncthreads();                // the previous chunk is consumed
    if (wv == 0) {
      if (lane < nr) {
        const double4 g = tgeo[rb + r0 + lane];
        const int pi = psi_idx[rb + r0 + lane];
        rw.x[lane] = g.x; rw.y[lane] = g.y; rw.tx[lane] = g.z; rw.ty[lane] = g.w;
        rw.h[lane] = trh[rb + r0 + lane];
        rw.phi[lane] = psi[pi];
        rw.vphi[lane] = psi[pi + N];
      }
    } else if (wv == 1 && lane < 2 * G && r0 == 0) {
      rw.gl[lane] = gl[lane];
    }
    __syncthreads();
    const int npts = nr * G;
    if (half == 0)
      p2m_half<P, 0, NA>(acc, grp * 64 + lane, 64 * PS, npts, G, kap, eta, rw);
    else
      p2m_half<P, 1, NA>(acc, grp * 64 + lane, 64 * PS, npts, G, kap, eta, rw);
  }
  if (half == 0)
    p2m_fold<P, 0, NA>(acc);
  else
    p2m_fold<P, 1, NA>(acc);
  cd tot = wave_sum_slots<NA>(acc, lane);
  const int slot = SPL == 2 ? lane >> 1 : lane;
  const bool writer = SPL == 2 ? (lane & 1) == 0 : true;
  if (PS > 1) {
    if (grp > 0 && writer && slot < NA) grp_sum[grp - 1][half][slot] = tot;
    __syncthreads();
    if (grp == 0)
      for (int g2 = 1; g2 < PS; ++g2)
        if (writer && slot < NA) tot = cadd(tot, grp_sum[g2 - 1][half][slot]);
  }
  // slot -> order of this wavefront's half: orders +m at [m - LO], then -m
  const int lo = half == 0 ? 0 : P / 2 + 1, hi = half == 0 ? P / 2 : P;
  const int npos = hi - lo + 1, nneg = hi - (lo > 0 ? lo : 1) + 1;
  if (grp == 0 && writer && slot < npos + nneg) {
    const int n = slot < npos ? lo + slot : -((lo > 0 ? lo : 1) + (slot - npos));
    mpole[((size_t)cell * 2 + ch) * NP + n + P] = tot;
  }
}

template <int P, int PS>
__global__ void __launch_bounds__(128 * PS) k_p2m(const int* __restrict__ leaves, const int* __restrict__ ldesc,
                                             const double4* __restrict__ tgeo, const double* __restrict__ trh,
                                             const int* __restrict__ psi_idx, const double* __restrict__ gl,
                                             int G, int N, double k, double k1, double eta,
                                             const cd* __restrict__ psi, cd* __restrict__ mpole,
                                             long long psi_stride, long long mp_stride) {
  p2m_cell<P, PS>(leaves[blockIdx.x], ldesc[8 * blockIdx.x], ldesc[8 * blockIdx.x + 1], blockIdx.y, blockIdx.z, tgeo,
                  trh, psi_idx, gl, G, N, k, k1, eta, psi, mpole, psi_stride, mp_stride);
}

// The value of lane `lane` (wave-uniform) of a complex register, through the
// scalar unit (four 32-bit lane reads); every lane receives it without LDS.
__device__ __forceinline__ cd lane_cd(cd v, int lane) {
  long long xr = __double_as_longlong(v.x), yr = __double_as_longlong(v.y);
  int xl = __builtin_amdgcn_readlane((int)xr, lane), xh = __builtin_amdgcn_readlane((int)(xr >> 32), lane);
  int yl = __builtin_amdgcn_readlane((int)yr, lane), yh = __builtin_amdgcn_readlane((int)(yr >> 32), lane);
  return mkc(__longlong_as_double(((long long)xh << 32) | (unsigned int)xl),
             __longlong_as_double(((long long)yh << 32) | (unsigned int)yl));
}

// M2M, directly from the leaves: every non-leaf cell C gathers the moments of
// the leaves below it, M_n(C) = sum_L sum_l M_l(L) Jm_{n-l}(kap (O_L - O_C))
// (Graf's theorem for J, eq. 10, as in the M2M translation of Sec. 3.2,
// applied across several levels at once), so the whole upward pass above
// the leaves is a single launch.  One workgroup of eight wavefronts per
// (non-leaf cell, channel); the wavefronts split the leaves and their
// partial sums meet in LDS in a fixed order.
constexpr int M2M_WAVES = 8;
template <int P>
__global__ void __launch_bounds__(64 * M2M_WAVES) k_m2m(const int* __restrict__ cells, const int* __restrict__ ptr,
                                             const int* __restrict__ src, const int* __restrict__ off,
                                             const cd* __restrict__ jtab, int n_joff, cd* mpole,
                                             long long mp_stride) {
  constexpr int NP = 2 * P + 1, NT = 4 * P + 1, NU = (NP + 63) / 64;
  __shared__ cd sj[M2M_WAVES][NT];
  __shared__ cd sr[M2M_WAVES][NP];
  mpole += blockIdx.z * mp_stride;              // batch member
  int ci = blockIdx.x, ch = blockIdx.y;
  int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int cell = cells[ci];
  cd acc[NU];
  for (int i = 0; i < NU; ++i) acc[i] = mkc(0, 0);
  constexpr int NTU = (NT + 63) / 64;
  // the next leaf's moments and translation row are loaded into registers
  // while the current leaf is translated (double buffering of the loads)
  const int qend = ptr[ci + 1];
  int q = ptr[ci] + w;
  cd mnext[NU], tnext[NTU];
  auto fetch = [&](int qq) {
    const cd* ms = mpole + ((size_t)src[qq] * 2 + ch) * NP;
    const cd* tj = jtab + ((size_t)ch * n_joff + off[qq]) * NT;
#pragma unroll
    for (int u = 0; u < NU; ++u) mnext[u] = lane + 64 * u < NP ? ms[lane + 64 * u] : mkc(0, 0);
#pragma unroll
    for (int u = 0; u < NTU; ++u) tnext[u] = lane + 64 * u < NT ? tj[lane + 64 * u] : mkc(0, 0);
  };
  if (q < qend) fetch(q);
  for (; q < qend; q += M2M_WAVES) {
    // the leaf's moments stay in registers and reach the lanes by lane reads
    cd mreg[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) mreg[u] = mnext[u];
#pragma unroll
    for (int u = 0; u < NTU; ++u)
      if (lane + 64 * u < NT) sj[w][lane + 64 * u] = tnext[u];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    if (q + M2M_WAVES < qend) fetch(q + M2M_WAVES);
#pragma unroll
    for (int i = 0; i < NU; ++i) {
      int n = min(lane + 64 * i - P, P);      // lanes past the last order repeat it
      cd s = acc[i];
#pragma unroll
      for (int sl = 0; sl < NU; ++sl) {
        const int hi = NP < 64 * sl + 64 ? NP : 64 * sl + 64;
        for (int idx = 64 * sl; idx < hi; ++idx)
          s = cfma_conj(sj[w][n - idx + 3 * P], lane_cd(mreg[sl], idx - 64 * sl), s);
      }
      acc[i] = s;
    }
    __builtin_amdgcn_wave_barrier();
  }
  for (int i = 0; i < NU; ++i) {
    int n = lane + 64 * i;
    if (n < NP) sr[w][n] = acc[i];
  }
  __syncthreads();
  cd* out = mpole + ((size_t)cell * 2 + ch) * NP;
  for (int n = threadIdx.x; n < NP; n += 64 * M2M_WAVES) {
    cd a = sr[0][n];
    for (int v = 1; v < M2M_WAVES; ++v) a = cadd(a, sr[v][n]);
    out[n] = a;
  }
}

// M2L over chunks of the interaction lists (eq. 13 with the index n - l):
//   part[c]_l = sum_{(C, t, m) in chunk c} alpha^m sum_n T_t[n - l] M_n(C),
// where T_t is Hp_nu(kap d) of an explicit pair (channel 0: exterior, with
// image m; channel 1: interior) or, for the roots, the lattice sum
// S_nu(c_i - c_j) that carries every far image of fibre j (Sec. 3.3).
// One wavefront per chunk; k_m2l_sum adds the chunks of each (channel, cell)
// in a fixed order, so the result does not depend on scheduling.
template <int P>
__global__ void __launch_bounds__(64) k_m2l(const int* __restrict__ chunks, const int* __restrict__ e_src,
                                            const int* __restrict__ e_off, const int* __restrict__ e_m,
                                            const cd* __restrict__ htab, int n_tab,
                                            const cd* __restrict__ alpha, int m_min,
                                            const cd* __restrict__ mpole, cd* __restrict__ part,
                                            long long mp_stride, long long part_stride, long long tab_stride,
                                            int alpha_stride, const int* __restrict__ ids) {
  constexpr int NP = 2 * P + 1, NT = 4 * P + 1;
  __shared__ cd sh[NT];
  // batch member: its multipoles, partial sums, lattice rows and image phases
  mpole += blockIdx.y * mp_stride;
  part += blockIdx.y * part_stride;
  htab += blockIdx.y * tab_stride;
  alpha += blockIdx.y * alpha_stride;
  // the chunks this launch takes (ids: those not on the matrix cores)
  int c = ids ? ids[blockIdx.x] : (int)blockIdx.x;
  int ch = chunks[4 * c + 1], b = chunks[4 * c + 2], e = b + chunks[4 * c + 3];
  if (e == b) return;                           // a root's slot for the lattice convolution
  constexpr int NU = (NP + 63) / 64;
  const int lane = threadIdx.x;
  cd acc[NU];
  for (int i = 0; i < NU; ++i) acc[i] = mkc(0, 0);
  constexpr int NTU = (NT + 63) / 64;
  // the next entry's moments, row and phase are loaded into registers while
  // the current entry is translated (double buffering of the loads)
  cd mnext[NU], tnext[NTU], pnext;
  auto fetch = [&](int qq) {
    const cd* ms = mpole + ((size_t)e_src[qq] * 2 + ch) * NP;
    const cd* th = htab + ((size_t)ch * n_tab + e_off[qq]) * NT;
#pragma unroll
    for (int u = 0; u < NU; ++u) mnext[u] = lane + 64 * u < NP ? ms[lane + 64 * u] : mkc(0, 0);
#pragma unroll
    for (int u = 0; u < NTU; ++u) tnext[u] = lane + 64 * u < NT ? th[lane + 64 * u] : mkc(0, 0);
    pnext = alpha[e_m[qq] - m_min];
  };
  if (b < e) fetch(b);
  for (int q = b; q < e; ++q) {
    // the source moments stay in registers (order n in lane n % 64 of slot
    // n / 64) and reach every lane through lane reads; only the translation
    // row goes through LDS
    cd mreg[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) mreg[u] = mnext[u];
#pragma unroll
    for (int u = 0; u < NTU; ++u)
      if (lane + 64 * u < NT) sh[lane + 64 * u] = tnext[u];
    cd ph = pnext;
    __syncthreads();
    if (q + 1 < e) fetch(q + 1);
#pragma unroll
    for (int i = 0; i < NU; ++i) {
      int l = min(lane + 64 * i - P, P);      // lanes past the last order repeat it
      cd s = mkc(0, 0);
#pragma unroll
      for (int sl = 0; sl < NU; ++sl) {
        const int hi = NP < 64 * sl + 64 ? NP : 64 * sl + 64;
        for (int idx = 64 * sl; idx < hi; ++idx)
          s = cfma(sh[idx - P - l + 2 * P], lane_cd(mreg[sl], idx - 64 * sl), s);
      }
      acc[i] = cfma(ph, s, acc[i]);
    }
    __syncthreads();
  }
  cd* out = part + (size_t)c * NP;
  for (int i = 0; i < NU; ++i) {
    int l = lane + 64 * i;
    if (l < NP) out[l] = acc[i];
  }
}

// M2L entries on the matrix cores.  The one-entry chunks that share a
// translation (channel and table row: one offset between cells, or one
// lattice sum of a fibre offset) form one complex matrix product, the
// Toeplitz matrix T[l][n] = t[n - l] of eq. 13 (index n - l) times the panel
// of their sources' moments, [2p+1 x entries], each result column then
// multiplied by its image phase alpha^m.  An item is one table row with up
// to 16 of its entries (columns, stored 16 per item, the unused ones
// repeating the first): one workgroup per (item, batch member) with NR =
// (2p + 15) / 16 wavefronts on the matrix cores, wavefront w computing the
// orders l = 16 w .. 16 w + 15 for the item's columns as one 16 x 16 tile of
// v_mfma_f64_16x16x4 steps over the source orders, four real products per
// complex step (re re, -im im, re im, im re).  When 2p + 1 = 16 NR + 1 (p =
// 8, 16, 24, 32, 40) one more wavefront computes the last order l = 2p
// (t[n] against every column) on the vector ALU meanwhile.  Lane layout of
// the f64 16 x 16 x 4 product: A[i][k] and B[k][j] in lane i + 16 k and
// j + 16 k, D[4 r + lane / 16][lane % 16] in accumulator r.  Loads come in
// two rounds: the item and its columns, then the translation row, every
// column's moments and the phases.  Each entry's result goes to its chunk's
// partial slot.
typedef double mfma_v4d __attribute__((ext_vector_type(4)));
constexpr int MFMA_COLS = 16;
template <int P>
constexpr int m2l_mfma_tiles() { return (2 * P + 15) / 16; }
template <int P>
constexpr int m2l_mfma_waves() { return m2l_mfma_tiles<P>() + (16 * m2l_mfma_tiles<P>() < 2 * P + 1 ? 1 : 0); }
template <int P>
__global__ void __launch_bounds__(64 * m2l_mfma_waves<P>()) k_m2l_mfma(
    const int4* __restrict__ items, const int4* __restrict__ cols, const cd* __restrict__ htab, int n_tab,
    const cd* __restrict__ alpha, int m_min, const cd* __restrict__ mpole, cd* __restrict__ part,
    long long mp_stride, long long part_stride, long long tab_stride, int alpha_stride) {
  constexpr int NP = 2 * P + 1, NT = 4 * P + 1, NR = m2l_mfma_tiles<P>(), NTH = 64 * m2l_mfma_waves<P>();
  constexpr int KS = (NP + 3) / 4, KP = 4 * KS + 1;   // source order steps; padded LDS row of a column
  constexpr int NFILL = MFMA_COLS * 4 * KS, PER = (NFILL + NTH - 1) / NTH;
  __shared__ cd sT[NT];
  __shared__ cd sB[MFMA_COLS * KP];
  __shared__ int4 sCol[MFMA_COLS];
  __shared__ int4 sIt;
  mpole += blockIdx.y * mp_stride;
  part += blockIdx.y * part_stride;
  htab += blockIdx.y * tab_stride;
  alpha += blockIdx.y * alpha_stride;
  if (threadIdx.x < MFMA_COLS) sCol[threadIdx.x] = cols[(size_t)MFMA_COLS * blockIdx.x + threadIdx.x];
  if (threadIdx.x == MFMA_COLS) sIt = items[blockIdx.x];    // channel, table row, -, columns
  __syncthreads();
  const int4 it = sIt;
  const int ch = it.x, ncol = it.w;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 15, kq = lane >> 4, l = 16 * w + i;
  const int4 mycol = sCol[i];
  const cd ph = alpha[mycol.z - m_min];               // this lane's column phase, used at the store
  const cd* t = htab + ((size_t)ch * n_tab + it.y) * NT;
  for (int q = threadIdx.x; q < NT; q += NTH) sT[q] = t[q];
  cd v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = threadIdx.x + u * NTH, j = min(q / (4 * KS), MFMA_COLS - 1), n = q - j * (4 * KS);
    v[u] = (q < NFILL && j < ncol && n < NP) ? mpole[((size_t)sCol[j].x * 2 + ch) * NP + n] : mkc(0, 0);
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int q = threadIdx.x + u * NTH, j = q / (4 * KS), n = q - j * (4 * KS);
    if (q < NFILL) sB[j * KP + n] = v[u];
  }
  __syncthreads();
  if (w < NR) {
    mfma_v4d dre = {0, 0, 0, 0}, dim = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int n = 4 * ks + kq;
      const cd a = (l < NP && n < NP) ? sT[n - l + 2 * P] : mkc(0, 0);
      const cd b = sB[i * KP + n];
      dre = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, dre, 0, 0, 0);
      dre = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, dre, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, dim, 0, 0, 0);
      dim = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, dim, 0, 0, 0);
    }
    if (i < ncol) {
      cd* out = part + (size_t)mycol.y * NP;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lo = 16 * w + 4 * r + kq;
        if (lo < NP) out[lo] = cmul(ph, mkc(dre[r], dim[r]));
      }
    }
  } else {
    // the last order (l = 2p: t[n] against column i), lanes kq = 0..3
    // taking n = kq, kq + 4, ..., then added across the column's four lanes
    cd tail = mkc(0, 0);
    for (int n = kq; n < NP; n += 4) tail = cfma(sT[n], sB[i * KP + n], tail);
#pragma unroll
    for (int o = 16; o < 64; o <<= 1) {
      tail.x += __shfl_xor(tail.x, o, 64);
      tail.y += __shfl_xor(tail.y, o, 64);
    }
    if (i < ncol && kq == 0) part[(size_t)mycol.y * NP + NP - 1] = cmul(ph, tail);
  }
}

// The M2L sum of each (channel, cell) with entries: the partial expansions
// of its chunks, their range cut into four consecutive quarters (one per
// wavefront, added in order with eight loads in flight), the quarters then
// added in order.  The downward pass then reads one sum per cell.
template <int P>
__global__ void __launch_bounds__(256) k_m2l_sum(const int* __restrict__ sums, const cd* __restrict__ epart,
                                                 cd* __restrict__ part, long long ep_stride, long long part_stride) {
  constexpr int NP = 2 * P + 1;
  __shared__ cd sq[4][NP];
  epart += blockIdx.y * ep_stride;
  part += blockIdx.y * part_stride;
  const int c = blockIdx.x, first = sums[4 * c + 2], cnt = sums[4 * c + 3];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q0 = first + (cnt * w) / 4, q1 = first + (cnt * (w + 1)) / 4;
  for (int l = lane; l < NP; l += 64) {
    cd s = mkc(0, 0);
#pragma unroll 8
    for (int e = q0; e < q1; ++e) s = cadd(s, epart[(size_t)e * NP + l]);
    sq[w][l] = s;
  }
  __syncthreads();
  for (int l = threadIdx.x; l < NP; l += 256)
    part[(size_t)c * NP + l] = cadd(cadd(sq[0][l], sq[1][l]), cadd(sq[2][l], sq[3][l]));
}

// Downward pass and L2P, one workgroup of two wavefronts (channels) per leaf
// (one, the exterior channel, when each fibre's own block is applied by FFT).
// The leaf's local expansion is its own M2L sum plus the own M2L sums of all
// its ancestors translated directly to it (L2L of Sec. 3.2 across several
// levels, Graf's theorem for J):
//   L_n(D) = own_n(D) + sum_A sum_l own_l(A) Jp_{l-n}(kap (O_D - O_A)),
// with own(A) the fixed-order sum of A's M2L chunks.  Then every target of
// the leaf evaluates (L2P)
//   u = sum_l L_l Jp_l(kap (x - O)),  dn = (kap/2) sum_l L_l (nu Jp_{l-1} - conj(nu) Jp_{l+1}),
// and the far part of the rows of (I - A) (eq. 9) is written:
//   far1 = u_ext - u_int,  far2 = 2/(i eta (1 + varrho)) (dn_ext - varrho dn_int).
// The kernel is bound by load latency, not arithmetic: the leaf descriptor
// names the sum rows and the target geometry directly, so the loads form two
// dependent steps, and each ancestor's sum and translation row are loaded
// while the previous ancestor is translated.
template <int P>
__global__ void __launch_bounds__(128) k_down(const int* __restrict__ ldesc, const int2* __restrict__ lanc,
                                              const double4* __restrict__ tgeo, const int* __restrict__ psi_idx,
                                              const cd* __restrict__ part, const cd* __restrict__ jtab, int n_joff,
                                              int N, double k, double k1, double eta, double varrho,
                                              cd* __restrict__ far, long long part_stride, long long far_stride,
                                              int add_into, const int* __restrict__ leaf_near_t0,
                                              const cd* __restrict__ near_buf) {
  constexpr int NP = 2 * P + 1, NT = 4 * P + 1, NU = (NP + 63) / 64, NTU = (NT + 63) / 64;
  __shared__ cd sJ[2][NT], sA[2][NP], sL[2][NP], sS[2][3][P + 2], sT[2][3][P + 2];
  __shared__ cd su[64], sd[64];
  part += blockIdx.y * part_stride;             // batch member
  far += blockIdx.y * far_stride;
  const int* dsc = ldesc + 8 * blockIdx.x;
  const int ch = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rb = dsc[0], rows = dsc[1], own = dsc[2 + ch];
  const int q0 = dsc[4 + 2 * ch], na = dsc[5 + 2 * ch] - q0;
  // independent loads first: target geometry, the leaf's own sum (order l in
  // lane l % 64 of slot l / 64) and the ancestors' (sum row, offset), one per lane
  double4 g = make_double4(0.0, 0.0, 0.0, 0.0);
  int pi = 0;
  if (lane < rows) {
    g = tgeo[rb + lane];
    pi = psi_idx[rb + lane];
  }
  cd acc[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    int i = lane + 64 * u;
    acc[u] = (own >= 0 && i < NP) ? part[(size_t)own * NP + i] : mkc(0, 0);
  }
  int2 an = make_int2(0, 0);
  if (lane < na) an = lanc[q0 + lane];
  cd anext[NU], tnext[NTU];
  auto fetch = [&](int q) {
    const int r = __builtin_amdgcn_readlane(an.x, q), o = __builtin_amdgcn_readlane(an.y, q);
    const cd* ps = part + (size_t)r * NP;
    const cd* tj = jtab + ((size_t)ch * n_joff + o) * NT;
#pragma unroll
    for (int u = 0; u < NU; ++u) anext[u] = lane + 64 * u < NP ? ps[lane + 64 * u] : mkc(0, 0);
#pragma unroll
    for (int u = 0; u < NTU; ++u) tnext[u] = lane + 64 * u < NT ? tj[lane + 64 * u] : mkc(0, 0);
  };
  if (na > 0) fetch(0);
  for (int q = 0; q < na; ++q) {                // wave-uniform trip count
#pragma unroll
    for (int u = 0; u < NU; ++u)
      if (lane + 64 * u < NP) sA[ch][lane + 64 * u] = anext[u];
#pragma unroll
    for (int u = 0; u < NTU; ++u)
      if (lane + 64 * u < NT) sJ[ch][lane + 64 * u] = tnext[u];
    if (q + 1 < na) fetch(q + 1);
    // the row is read only by this wavefront: its LDS stores must be done
    // (lgkmcnt 0), the loads of the next ancestor stay in flight
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      int n = min(lane + 64 * u - P, P);      // lanes past the last order repeat it
      cd sres = acc[u];
      for (int idx = 0; idx < NP; ++idx) sres = cfma(sA[ch][idx], sJ[ch][idx - n + P], sres);
      acc[u] = sres;
    }
    __builtin_amdgcn_wave_barrier();
  }
  for (int u = 0; u < NU; ++u) {
    int i = lane + 64 * u;
    if (i < NP) sL[ch][i] = acc[u];
  }
  __syncthreads();
  // L2P.  The three sums u = sum_n L_n Jp_n, A = sum_n L_{n+1} Jp_n and
  // B = sum_n L_{n-1} Jp_n (|n| <= P + 1; dn = (kap/2)(nu A - conj(nu) B))
  // fold order -n onto order n through Jp_{-n} = (-1)^n conj(Jp_n): with
  // Jp_n = x_n + i y_n and coefficients c_n,
  //   c_n Jp_n + c_{-n} Jp_{-n} = s_n x_n + t_n y_n,
  //   s_n = c_n + (-1)^n c_{-n},  t_n = i (c_n - (-1)^n c_{-n}),
  // so each target needs 4 real FMA per sum and order n >= 0.
  constexpr int K = P + 1;
  if (lane <= K) {
    const int n = lane;
    const double sg = (n & 1) ? -1.0 : 1.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int sh = j == 0 ? 0 : (j == 1 ? 1 : -1);
      const int lp = n + sh, lm = -n + sh;
      cd c = (lp >= -P && lp <= P) ? sL[ch][P + lp] : mkc(0, 0);
      cd e = (lm >= -P && lm <= P) ? cscale(sL[ch][P + lm], sg) : mkc(0, 0);
      cd d = csub(c, e);
      sS[ch][j][n] = n ? cadd(c, e) : c;
      sT[ch][j][n] = n ? mkc(-d.y, d.x) : mkc(0, 0);
    }
  }
  __syncthreads();
  cd u = mkc(0, 0), dv = mkc(0, 0);
  double kap = ch ? k1 : k;
  if (lane < rows) {
    double vx = kap * g.x, vy = kap * g.y;
    double gs[K + 1];                        // h_n = g_n / n!
    scaled_h<K>(0.25 * (vx * vx + vy * vy), gs);
    cd hv = mkc(0.5 * vx, 0.5 * vy);
    cd uu = mkc(1.0, 0.0);                   // (v/2)^n
    cd sa = mkc(0, 0), sb = mkc(0, 0);
#pragma unroll
    for (int n = 0; n <= K; ++n) {
      const double x = uu.x * gs[n], y = uu.y * gs[n];   // Jp_n
      cd s0 = sS[ch][0][n], t0 = sT[ch][0][n];
      cd s1 = sS[ch][1][n], t1 = sT[ch][1][n];
      cd s2 = sS[ch][2][n], t2 = sT[ch][2][n];
      u.x = fma(s0.x, x, fma(t0.x, y, u.x));
      u.y = fma(s0.y, x, fma(t0.y, y, u.y));
      sa.x = fma(s1.x, x, fma(t1.x, y, sa.x));
      sa.y = fma(s1.y, x, fma(t1.y, y, sa.y));
      sb.x = fma(s2.x, x, fma(t2.x, y, sb.x));
      sb.y = fma(s2.y, x, fma(t2.y, y, sb.y));
      if (n < K) uu = cmul(uu, hv);
    }
    cd nu = mkc(g.w, -g.z);
    dv = cscale(csub(cmul(nu, sa), cmul(cconj(nu), sb)), 0.5 * kap);
  }
  if (ch == 1) {
    su[lane] = u;
    sd[lane] = dv;
  } else if (blockDim.x == 64) {
    // one wavefront: the interior channel is applied outside the tree
    su[lane] = mkc(0, 0);
    sd[lane] = mkc(0, 0);
  }
  __syncthreads();
  if (ch == 0 && lane < rows) {
    cd c = mkc(0.0, -2.0 / (eta * (1.0 + varrho)));
    const cd f1 = csub(u, su[lane]), f2 = cmul(c, csub(dv, cscale(sd[lane], varrho)));
    if (add_into) {
      // far is the output y, which already holds psi + near (the join), or
      // P psi, with the near sums of this leaf's rows in near_buf
      cd y1 = far[pi], y2 = far[pi + N];
      const int t0 = leaf_near_t0 ? leaf_near_t0[blockIdx.x] : -1;
      if (t0 >= 0) {
        y1 = cadd(y1, near_buf[2 * (t0 + lane)]);
        y2 = cadd(y2, near_buf[2 * (t0 + lane) + 1]);
      }
      far[pi] = cadd(y1, f1);
      far[pi + N] = cadd(y2, f2);
    } else {
      far[pi] = f1;
      far[pi + N] = f2;
    }
  }
}

// The join of the near and far parts of the rows: y += far when the P2P
// wrote y = psi + near itself (S = 1), else y = psi + far + sum of the S
// partial near parts, added in split order.
__global__ void k_combine(long long n, const cd* __restrict__ far, const cd* __restrict__ psi,
                          const cd* __restrict__ part, int S, cd* __restrict__ y) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (S == 1) {
    y[i] = cadd(y[i], far[i]);
    return;
  }
  cd acc = part[i];
  for (int s = 1; s < S; ++s) acc = cadd(acc, part[s * n + i]);
  y[i] = cadd(cadd(psi[i], acc), far[i]);
}

// P2P with the stored near blocks plus the identity of (I - A):
//   y1 = phi + sum_b (B11 phi_b + B12 varphi_b),  y2 = varphi + sum_b (B21 phi_b + B22 varphi_b).
// One workgroup (4 wavefronts) per target leaf, lane = target row.  The
// densities of the leaf's source columns are first gathered into LDS (in
// segments), then the wavefronts take the columns in turn and stream the
// leaf's contiguous block region; partial rows meet in LDS.  Pure streaming:
// the kernel is HBM-bound.
constexpr int P2P_WAVES = 4;
constexpr int P2P_SEG = 256;

// Complex arithmetic of the batched P2P stream: FP64 (double2) or FP32 (float2).
__device__ __forceinline__ double2 p2p_fma(double2 a, double2 b, double2 c) { return cfma(a, b, c); }
__device__ __forceinline__ float2 p2p_fma(float2 a, float2 b, float2 c) { return cfmaf(a, b, c); }
template <typename C> __device__ __forceinline__ C p2p_cvt(cd v);
template <> __device__ __forceinline__ double2 p2p_cvt<double2>(cd v) { return v; }
template <> __device__ __forceinline__ float2 p2p_cvt<float2>(cd v) {
  float2 r;
  r.x = (float)v.x;
  r.y = (float)v.y;
  return r;
}
template <typename C> __device__ __forceinline__ cd p2p_wide(C v) { return mkc((double)v.x, (double)v.y); }

// Loads of the near-block stream.  The blocks are read once per apply and
// are far larger than the L2, so they are loaded non-temporally and do not
// evict the densities the P2P gathers or the expansions and tables of the
// concurrent FMM chain.
template <typename C> __device__ __forceinline__ C nt_load(const C* p);
template <> __device__ __forceinline__ double2 nt_load<double2>(const double2* p) {
  double2 r;
  r.x = __builtin_nontemporal_load(&p->x);
  r.y = __builtin_nontemporal_load(&p->y);
  return r;
}
template <> __device__ __forceinline__ float2 nt_load<float2>(const float2* p) {
  float2 r;
  r.x = __builtin_nontemporal_load(&p->x);
  r.y = __builtin_nontemporal_load(&p->y);
  return r;
}

template <typename C, int U>
// the persistent grid holds few workgroups per CU (p2p_blocks_per_cu), so the
// register budget is not cut for occupancy
__global__ void __launch_bounds__(64 * P2P_WAVES, 2) k_p2p(
    const int* __restrict__ leaves, const int* __restrict__ ebeg, const int* __restrict__ eend,
    const int* __restrict__ psi_idx, int N, const long long* __restrict__ leaf_blk,
    const int* __restrict__ cols_ptr, const int* __restrict__ col_psi, const C* __restrict__ blocks,
    const int* __restrict__ ccols_ptr, const int* __restrict__ ccol_psi, const int* __restrict__ ccol_loc,
    const cd* __restrict__ circ, const int* __restrict__ cwin, const cd* __restrict__ psi,
    cd* y, const cd* ybase, const int* __restrict__ item_leaf, int n_leaves, int S, cd* __restrict__ part,
    long long vec) {
  // the blocks are stored as C (complex128, or complex64 for PFM_MIXED); the
  // densities and the sums stay FP64, so the complex64 form only rounds the
  // stored blocks (the stream is bandwidth-bound either way)
  extern __shared__ cd swin[];                  // [B11, B12, B21, B22][P2P_WCAP] row window
  constexpr int WS = P2P_WCAP;
  __shared__ cd sp[P2P_SEG][2];
  __shared__ int sl[P2P_SEG];
  __shared__ cd r1[P2P_WAVES][64], r2[P2P_WAVES][64];
  // work item = (target leaf, column split); with S > 1 the splits write
  // partial rows that k_combine adds in a fixed order
  // work items run over n_leaves target leaves, all of them or (item_leaf)
  // the listed ones: when P2P adds into rows that already hold the rest
  // (ybase == y), only the leaves with near columns
  for (int item = blockIdx.x; item < n_leaves * S; item += gridDim.x) {
    int lw = item / S, sp_i = item - lw * S;
    int li = item_leaf ? item_leaf[lw] : lw;
    int k0 = cols_ptr[li], ncol = cols_ptr[li + 1] - k0;
    // a leaf without near columns has nothing to add (uniform over the workgroup)
    if (ybase == y && ncol == 0 && ccols_ptr[li + 1] == ccols_ptr[li]) continue;
    int D = leaves[li];
    int db = ebeg[D], rows = eend[D] - db;
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    cd a1 = mkc(0, 0), a2 = a1;
    int chunk = (ncol + S - 1) / S;
    int c_lo = min(ncol, sp_i * chunk), c_hi = min(ncol, c_lo + chunk);
    const C* bl = blocks + 4 * leaf_blk[li];
    const unsigned cstride = 4u * (unsigned)rows;
    bool act = lane < rows;
    // stored columns: stream the leaf's block region
    for (int seg = c_lo; seg < c_hi; seg += P2P_SEG) {
      int nseg = min(P2P_SEG, c_hi - seg);
      for (int i = threadIdx.x; i < nseg; i += 64 * P2P_WAVES) {
        int pi = col_psi[k0 + seg + i];
        sp[i][0] = psi[pi];
        sp[i][1] = psi[pi + N];
      }
      __syncthreads();
      const C* bs = bl + (size_t)seg * cstride + lane;
      if (act) {
        // U columns per step: their 4U block loads are issued before the FMAs
        int k = w;
        for (; k + (U - 1) * P2P_WAVES < nseg; k += U * P2P_WAVES) {
          C bb[U][4];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            unsigned o = (unsigned)(k + u * P2P_WAVES) * cstride;
            bb[u][0] = nt_load(bs + o);
            bb[u][1] = nt_load(bs + o + rows);
            bb[u][2] = nt_load(bs + o + 2 * rows);
            bb[u][3] = nt_load(bs + o + 3 * rows);
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            cd ph = sp[k + u * P2P_WAVES][0], vp = sp[k + u * P2P_WAVES][1];
            a1 = cfma(p2p_wide(bb[u][0]), ph, a1);
            a1 = cfma(p2p_wide(bb[u][1]), vp, a1);
            a2 = cfma(p2p_wide(bb[u][2]), ph, a2);
            a2 = cfma(p2p_wide(bb[u][3]), vp, a2);
          }
        }
        for (; k < nseg; k += P2P_WAVES) {
          unsigned o = (unsigned)k * cstride;
          C b11 = nt_load(bs + o), b12 = nt_load(bs + o + rows);
          C b21 = nt_load(bs + o + 2 * rows), b22 = nt_load(bs + o + 3 * rows);
          cd ph = sp[k][0], vp = sp[k][1];
          a1 = cfma(p2p_wide(b11), ph, a1);
          a1 = cfma(p2p_wide(b12), vp, a1);
          a2 = cfma(p2p_wide(b21), ph, a2);
          a2 = cfma(p2p_wide(b22), vp, a2);
        }
      }
      __syncthreads();
    }
    // circulant columns (same fibre, image 0): the block of target element a
    // and source element b is entry (b - a) mod N of the fibre's row.  Places
    // on the circle are counted from the leaf's rotation rot (a' = a - rot,
    // b' = b - rot mod N), so that the entries N - a' + b' the leaf reads form
    // one window [elo, elo + wl) of the doubled row; with wl > 0 it is staged
    // in LDS once per leaf (a Toeplitz block needs rows + columns - 1 entries,
    // not rows x columns loads), else the entries are read through the caches.
    // Both read the same entries and sum in the same order.
    {
      const int q0 = ccols_ptr[li], nq = ccols_ptr[li + 1] - q0;
      const int qchunk = (nq + S - 1) / S;
      const int q_lo = min(nq, sp_i * qchunk), q_hi = min(nq, q_lo + qchunk);
      const int rot = cwin[3 * li], elo = cwin[3 * li + 1], wl = cwin[3 * li + 2];
      const int pr = psi_idx[db + min(lane, rows - 1)];
      const int fD = pr / (2 * N), aloc = pr - 2 * fD * N;
      const int ar = aloc >= rot ? aloc - rot : aloc - rot + N;
      const cd* frow = circ + (size_t)fD * 8 * N;
      const cd* crow = frow + (N - ar);                 // + b': entry (b' - a') + N
      const int woff = N - ar - elo;                    // window slot of column b': woff + b'
      if (wl > 0 && q_lo < q_hi) {
        // visible after the barrier that follows the first column staging
        for (int i = threadIdx.x; i < 4 * wl; i += 64 * P2P_WAVES) {
          const int c = i / wl, j = i - c * wl;
          swin[c * WS + j] = frow[(size_t)c * 2 * N + elo + j];
        }
      }
      for (int seg = q_lo; seg < q_hi; seg += P2P_SEG) {
        int nseg = min(P2P_SEG, q_hi - seg);
        for (int i = threadIdx.x; i < nseg; i += 64 * P2P_WAVES) {
          int pi = ccol_psi[q0 + seg + i];
          sp[i][0] = psi[pi];
          sp[i][1] = psi[pi + N];
          const int bl = ccol_loc[q0 + seg + i];
          sl[i] = bl >= rot ? bl - rot : bl - rot + N;
        }
        __syncthreads();
        if (act && wl > 0) {
          // four columns per step, their row entries read from LDS
          constexpr int CU = 4;
          int k = w;
          for (; k + (CU - 1) * P2P_WAVES < nseg; k += CU * P2P_WAVES) {
            cd cc[CU][4];
#pragma unroll
            for (int u = 0; u < CU; ++u) {
              const cd* x = swin + woff + sl[k + u * P2P_WAVES];
              cc[u][0] = x[0];
              cc[u][1] = x[WS];
              cc[u][2] = x[2 * WS];
              cc[u][3] = x[3 * WS];
            }
#pragma unroll
            for (int u = 0; u < CU; ++u) {
              cd ph = sp[k + u * P2P_WAVES][0], vp = sp[k + u * P2P_WAVES][1];
              a1 = cfma(cc[u][0], ph, a1);
              a1 = cfma(cc[u][1], vp, a1);
              a2 = cfma(cc[u][2], ph, a2);
              a2 = cfma(cc[u][3], vp, a2);
            }
          }
          for (; k < nseg; k += P2P_WAVES) {
            const cd* x = swin + woff + sl[k];
            cd ph = sp[k][0], vp = sp[k][1];
            a1 = cfma(x[0], ph, a1);
            a1 = cfma(x[WS], vp, a1);
            a2 = cfma(x[2 * WS], ph, a2);
            a2 = cfma(x[3 * WS], vp, a2);
          }
        } else if (act) {
          // four columns' row entries in flight per wavefront (cached loads)
          constexpr int CU = 4;
          int k = w;
          for (; k + (CU - 1) * P2P_WAVES < nseg; k += CU * P2P_WAVES) {
            cd cc[CU][4];
#pragma unroll
            for (int u = 0; u < CU; ++u) {
              const cd* cr = crow + sl[k + u * P2P_WAVES];
              cc[u][0] = cr[0];
              cc[u][1] = cr[2 * N];
              cc[u][2] = cr[4 * N];
              cc[u][3] = cr[6 * N];
            }
#pragma unroll
            for (int u = 0; u < CU; ++u) {
              cd ph = sp[k + u * P2P_WAVES][0], vp = sp[k + u * P2P_WAVES][1];
              a1 = cfma(cc[u][0], ph, a1);
              a1 = cfma(cc[u][1], vp, a1);
              a2 = cfma(cc[u][2], ph, a2);
              a2 = cfma(cc[u][3], vp, a2);
            }
          }
          for (; k < nseg; k += P2P_WAVES) {
            const cd* cr = crow + sl[k];
            cd ph = sp[k][0], vp = sp[k][1];
            a1 = cfma(cr[0], ph, a1);
            a1 = cfma(cr[2 * N], vp, a1);
            a2 = cfma(cr[4 * N], ph, a2);
            a2 = cfma(cr[6 * N], vp, a2);
          }
        }
        __syncthreads();
      }
    }
    r1[w][lane] = a1;
    r2[w][lane] = a2;
    __syncthreads();
    if (w == 0 && act) {
      cd s1 = r1[0][lane], s2 = r2[0][lane];
#pragma unroll
      for (int v = 1; v < P2P_WAVES; ++v) {
        s1 = cadd(s1, r1[v][lane]);
        s2 = cadd(s2, r2[v][lane]);
      }
      int pi = psi_idx[db + lane];
      if (S == 1) {
        // ybase: psi (the identity of I - A), or y itself when the rows
        // already hold psi and the rest of the operator
        y[pi] = cadd(ybase[pi], s1);
        y[pi + N] = cadd(ybase[pi + N], s2);
      } else {
        cd* pp = part + (size_t)sp_i * vec;
        pp[pi] = s1;
        pp[pi + N] = s2;
      }
    }
    __syncthreads();
  }
}

// P2P of the stored near blocks by target row, when each fibre's own block
// is applied by FFT and only pairs between fibres or with images are stored
// (a few leaves): one wavefront per row of a leaf with stored columns, the
// lanes over the leaf's stored columns, the lanes' sums added by a butterfly.
// A row task is described by (index of phi of the row in Psi, first stored
// column of the leaf, stored columns, rows of the leaf) and the offset of its
// row in the leaf's block region (entries), so that the sums start two loads
// away from the task index.
template <typename C>
__device__ __forceinline__ void p2p_row_sums(const int4 d, const long long off, const int* __restrict__ col_psi,
                                             const C* __restrict__ blocks, const cd* __restrict__ psi, int N,
                                             int lane, cd& a1, cd& a2) {
  const int k0 = d.y, ncol = d.z, rows = d.w;
  const C* bl = blocks + off;
  const size_t cs = 4 * (size_t)rows;
  a1 = mkc(0, 0);
  a2 = mkc(0, 0);
  for (int k = lane; k < ncol; k += 64) {
    const C* b = bl + (size_t)k * cs;
    const int pi = col_psi[k0 + k];
    const cd ph = psi[pi], vp = psi[pi + N];
    a1 = cfma(p2p_wide(b[0]), ph, a1);
    a1 = cfma(p2p_wide(b[rows]), vp, a1);
    a2 = cfma(p2p_wide(b[2 * rows]), ph, a2);
    a2 = cfma(p2p_wide(b[3 * rows]), vp, a2);
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    a1.x += __shfl_xor(a1.x, m, 64);
    a1.y += __shfl_xor(a1.y, m, 64);
    a2.x += __shfl_xor(a2.x, m, 64);
    a2.y += __shfl_xor(a2.y, m, 64);
  }
}

// The row tasks added into y (which already holds the rest of the rows).
template <typename C>
__global__ void __launch_bounds__(64) k_p2p_rows(const int4* __restrict__ tasks, const long long* __restrict__ toff,
                                                 const int* __restrict__ col_psi, const C* __restrict__ blocks,
                                                 const cd* __restrict__ psi, int N, cd* y) {
  const int4 d = tasks[blockIdx.x];
  cd a1, a2;
  p2p_row_sums<C>(d, toff[blockIdx.x], col_psi, blocks, psi, N, threadIdx.x, a1, a2);
  if (threadIdx.x == 0) {
    y[d.x] = cadd(y[d.x], a1);
    y[d.x + N] = cadd(y[d.x + N], a2);
  }
}

// The first launch of the apply with each fibre's own block by FFT (one
// wave): workgroups f < M apply fibre f's block to its rows, y = P psi (as
// k_pc_apply); the workgroups after them take the row tasks of the stored
// near pairs, eight per workgroup (one per wavefront), and leave each row's
// sums in near_buf for the downward pass to add.
template <typename C>
__global__ void __launch_bounds__(PC_THREADS) k_self_apply(const cd* in, cd* out, const cd* __restrict__ coef,
                                                           const cd* __restrict__ tw, int N, int logN, int M,
                                                           const int4* __restrict__ tasks,
                                                           const long long* __restrict__ toff, int ntasks,
                                                           const int* __restrict__ col_psi,
                                                           const C* __restrict__ blocks, cd* __restrict__ near_buf) {
  extern __shared__ cd pcs[];
  if ((int)blockIdx.x >= M) {
    const int t = ((int)blockIdx.x - M) * (PC_THREADS / 64) + (threadIdx.x >> 6);
    if (t >= ntasks) return;
    cd a1, a2;
    p2p_row_sums<C>(tasks[t], toff[t], col_psi, blocks, in, N, threadIdx.x & 63, a1, a2);
    if ((threadIdx.x & 63) == 0) {
      near_buf[2 * t] = a1;
      near_buf[2 * t + 1] = a2;
    }
    return;
  }
  const int f = blockIdx.x;
  cd* X = pcs;
  cd* Y = pcs + 2 * N;
  const cd* src = in + (size_t)f * 2 * N;  // phi_f then varphi_f
  for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) X[i] = src[i];
  // with one mode per thread (N <= PC_THREADS) the mode block's loads are
  // issued now and land while the forward transforms run
  const bool one = N <= (int)blockDim.x;
  const int kk = threadIdx.x;
  cd c0 = mkc(0, 0), c1 = c0, c2 = c0, c3 = c0;
  if (one && kk < N) {
    const cd* c = coef + ((size_t)f * N + kk) * 4;
    c0 = c[0]; c1 = c[1]; c2 = c[2]; c3 = c[3];
  }
  __syncthreads();
  cd* H = pc_fft(X, Y, 2, N, logN, tw, true);
  if (one) {
    if (kk < N) {
      const cd u = H[kk], v = H[N + kk];
      H[kk] = cadd(cmul(c0, u), cmul(c1, v));
      H[N + kk] = cadd(cmul(c2, u), cmul(c3, v));
    }
  } else {
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
      const cd* c = coef + ((size_t)f * N + m) * 4;
      const cd u = H[m], v = H[N + m];
      H[m] = cadd(cmul(c[0], u), cmul(c[1], v));
      H[N + m] = cadd(cmul(c[2], u), cmul(c[3], v));
    }
  }
  __syncthreads();
  const cd* Z = pc_fft(H, H == X ? Y : X, 2, N, logN, tw, false);
  const double sc = 1.0 / N;
  cd* dst = out + (size_t)f * 2 * N;
  for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) dst[i] = cscale(Z[i], sc);
}

// ---------------------------------------------------------------------------
// Fibre roots through the fibre's Fourier modes.  On a circle cut into N
// equal chords, element e is element 0 turned by t_e = 2 pi e / N about the
// centre c, and under a turn by t the harmonics of Sec. 3.2 go as
//   Jm_n(R_t v) = Jm_n(v) e^{-i n t},  Jp_l(R_t v) = Jp_l(v) e^{i l t},
// with the normal turning along.  So the multipole moments of the whole
// fibre about its centre (the P2M sums over all its elements) are
//   M_n = A_n phihat(n mod N) + B_n varphihat(n mod N),
//   phihat(j) = sum_e phi_e e^{-2 pi i j e / N},
// A_n, B_n the P2M weights summed over element 0's Gauss points, and a local
// expansion L about c gives at the midpoints (L2P)
//   u_e  = sum_l L_l Jp_l(v_0) e^{i l t_e},
//   dn_e = sum_l L_l (kap/2)(nu_0 Jp_{l-1}(v_0) - conj(nu_0) Jp_{l+1}(v_0)) e^{i l t_e},
// v_0 = kap (x_0 - c), nu_0 the normal of element 0.  Every root's moments
// come from the partial DFTs (no M2M truncation).  A fibre whose cells take
// part only in root-to-root M2L entries (no near pairs, nothing below its
// root) needs nothing else: its far rows are the synthesis of its root's
// local expansion (no L2L truncation).  The other fibres keep P2M at their
// leaves, M2M into their cells below the root and the downward pass.
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ cd jp_signed(const cd (&jp)[K + 1], int j) {
  // Jp_{-j} = (-1)^j conj(Jp_j)
  if (j >= 0) return jp[j];
  const cd v = cconj(jp[-j]);
  return (j & 1) ? cscale(v, -1.0) : v;
}

// the same from a sequence Jp_0..Jp_K held in LDS
template <int K>
__device__ __forceinline__ cd jp_lds(const cd* jp, int j) {
  if (j >= 0) return jp[j];
  const cd v = cconj(jp[-j]);
  return (j & 1) ? cscale(v, -1.0) : v;
}

// tab[f][0][n] = A_n, [1][n] = B_n, [2][l] = Jp_l(v_0),
// [3][l] = (kap/2)(nu_0 Jp_{l-1}(v_0) - conj(nu_0) Jp_{l+1}(v_0)); n, l = -P..P.
// One workgroup per fibre: the Bessel sequences at the G Gauss points and
// at the element's centre once each into LDS, then one thread per order;
// the exterior wavenumber only.
template <int P>
__global__ void __launch_bounds__(128) k_spec_tables(int N, const double* __restrict__ centres,
                                                     const double* __restrict__ mx, const double* __restrict__ my,
                                                     const double* __restrict__ tx, const double* __restrict__ ty,
                                                     const double* __restrict__ h, const double* __restrict__ gl,
                                                     int G, double kap, double eta, cd* __restrict__ tab) {
  constexpr int NP = 2 * P + 1, K = P + 1;
  __shared__ cd sJ[17][K + 1];             // Jp_0..Jp_K at the G <= 16 points and at the element's centre
  const int f = blockIdx.x, i = threadIdx.x;
  const size_t e0 = (size_t)f * N;
  const double ex = tx[e0], ey = ty[e0], hh = h[e0];
  const double rx = mx[e0] - centres[2 * f], ry = my[e0] - centres[2 * f + 1];
  // one Bessel sequence per thread 0..G (thread G: the centre), shared by the orders
  if (i <= G) {
    cd jp[K + 1];
    const double s = i < G ? 0.5 * hh * gl[i] : 0.0;
    jplus_seq<K>(kap * (rx + s * ex), kap * (ry + s * ey), jp);
#pragma unroll
    for (int j = 0; j <= K; ++j) sJ[i][j] = jp[j];
  }
  __syncthreads();
  if (i >= NP) return;
  const int n = i - P;
  // P2M weights per unit phi and varphi (as k_p2m: w = h gl_w / 8 carries
  // the factor i/4 of the representation, sk = kap w / 2):
  //   A_n = sum_g sk (-tx + i ty) Jm_{n-1} + sk (-tx - i ty) Jm_{n+1},  B_n = sum_g eta w Jm_n
  cd A = mkc(0, 0), Bn = mkc(0, 0);
  for (int g = 0; g < G; ++g) {
    const double w = 0.125 * hh * gl[G + g], sk = 0.5 * kap * w;
    const cd jm0 = cconj(jp_lds<K>(sJ[g], n)), jmm = cconj(jp_lds<K>(sJ[g], n - 1)),
             jmp = cconj(jp_lds<K>(sJ[g], n + 1));
    A = cfma(mkc(-sk * ex, sk * ey), jmm, A);
    A = cfma(mkc(-sk * ex, -sk * ey), jmp, A);
    Bn = cadd(Bn, cscale(jm0, eta * w));
  }
  const cd nu = mkc(ey, -ex);
  const cd dl = cscale(csub(cmul(nu, jp_lds<K>(sJ[G], n - 1)), cmul(cconj(nu), jp_lds<K>(sJ[G], n + 1))),
                       0.5 * kap);
  cd* T = tab + (size_t)f * 4 * NP;
  T[i] = A;
  T[NP + i] = Bn;
  T[2 * NP + i] = jp_lds<K>(sJ[G], n);
  T[3 * NP + i] = dl;
}

// P2M weights of the tree fibres' cells below their roots (mcell = [cell,
// first row, rows, first table row]: the leaves and the cells between them
// and the root): tab[((toff + e) (p + 1) + n) 2 + {0, 1}] = A_n, B_n (n =
// 0..p) of the cell's element e (tree order) about the cell centre (as
// k_spec_tables, exterior wavenumber), so that M_n(cell) = sum_e A_n phi_e
// + B_n varphi_e.  The negative orders follow from Jm_{-j} = (-1)^j
// conj(Jm_j) with the real weight of B and the conjugate pair of weights in
// A: A_{-n} = (-1)^{n+1} conj(A_n), B_{-n} = (-1)^n conj(B_n).  One thread
// per (element, block of eight orders) of a cell, one Bessel sequence per
// Gauss point for its orders; the block's first order is a template
// constant so that the sequence stays in registers.  Workgroups of 64
// threads, P2M_TAB_SPLIT of them per cell.
constexpr int P2M_TAB_OB = 8;            // orders per thread
constexpr int P2M_TAB_SPLIT = 8;         // workgroups per cell

template <int P, int N0>
__device__ __forceinline__ void p2m_table_orders(double rx, double ry, double ex, double ey, double hh,
                                                 const double* __restrict__ gl, int G, double kap, double eta,
                                                 cd* __restrict__ t) {
  constexpr int NH = P + 1, K = P + 1, OB = P2M_TAB_OB;
  cd A[OB], Bn[OB];
#pragma unroll
  for (int o = 0; o < OB; ++o) A[o] = Bn[o] = mkc(0, 0);
  cd jp[K + 1];
  for (int g = 0; g < G; ++g) {
    const double s = 0.5 * hh * gl[g], w = 0.125 * hh * gl[G + g], sk = 0.5 * kap * w;
    jplus_seq<K>(kap * (rx + s * ex), kap * (ry + s * ey), jp);   // once for the thread's orders
#pragma unroll
    for (int o = 0; o < OB; ++o) {
      const int n = N0 + o < P ? N0 + o : P;
      const cd jm0 = cconj(jp_signed<K>(jp, n)), jmm = cconj(jp_signed<K>(jp, n - 1)),
               jmp = cconj(jp_signed<K>(jp, n + 1));
      A[o] = cfma(mkc(-sk * ex, sk * ey), jmm, A[o]);
      A[o] = cfma(mkc(-sk * ex, -sk * ey), jmp, A[o]);
      Bn[o] = cadd(Bn[o], cscale(jm0, eta * w));
    }
  }
#pragma unroll
  for (int o = 0; o < OB; ++o)
    if (N0 + o < NH) {
      t[2 * (N0 + o)] = A[o];
      t[2 * (N0 + o) + 1] = Bn[o];
    }
}

template <int P, int B>
__device__ __forceinline__ void p2m_table_block(int blk, double rx, double ry, double ex, double ey, double hh,
                                                const double* __restrict__ gl, int G, double kap, double eta,
                                                cd* __restrict__ t) {
  constexpr int NB = (P + 1 + P2M_TAB_OB - 1) / P2M_TAB_OB;
  if constexpr (B < NB) {
    if (blk == B)
      p2m_table_orders<P, B * P2M_TAB_OB>(rx, ry, ex, ey, hh, gl, G, kap, eta, t);
    else
      p2m_table_block<P, B + 1>(blk, rx, ry, ex, ey, hh, gl, G, kap, eta, t);
  }
}

template <int P>
__global__ void __launch_bounds__(64) k_p2m_tables(const int4* __restrict__ mcell, const int* __restrict__ elem_of,
                                                   const double* __restrict__ cx, const double* __restrict__ cy,
                                                   const double* __restrict__ mx, const double* __restrict__ my,
                                                   const double* __restrict__ tx, const double* __restrict__ ty,
                                                   const double* __restrict__ h, const double* __restrict__ gl,
                                                   int G, double kap, double eta, cd* __restrict__ tab) {
  constexpr int NH = P + 1, NB = (NH + P2M_TAB_OB - 1) / P2M_TAB_OB;   // order blocks
  const int4 mc = mcell[blockIdx.x];
  const int cell = mc.x, rb = mc.y, rows = mc.z, toff = mc.w;
  const double ox = cx[cell], oy = cy[cell];
  for (int q = blockIdx.y * blockDim.x + threadIdx.x; q < NB * rows; q += gridDim.y * blockDim.x) {
    const int e = q / NB, blk = q - e * NB;
    const int en = elem_of[rb + e];
    p2m_table_block<P, 0>(blk, mx[en] - ox, my[en] - oy, tx[en], ty[en], h[en], gl, G, kap, eta,
                          tab + ((size_t)toff + e) * NH * 2);
  }
}

// L2P values of the down leaves' rows (ddesc[8 q] = rb, rows, ..., ddesc[8 q
// + 7] = first table row): tab[(toff + e) (p + 2) + n] = Jp_n(kap (x_e -
// O_leaf)), n = 0..p+1, from the row's offset to its leaf centre (tgeo), as
// k_down_spec's L2P would compute them at every apply.  One thread per row.
template <int P>
__global__ void __launch_bounds__(64) k_l2p_tables(const int* __restrict__ ddesc, const double4* __restrict__ tgeo,
                                                   double k, cd* __restrict__ tab) {
  constexpr int K = P + 1;
  const int* d = ddesc + 8 * blockIdx.x;
  const int rb = d[0], rows = d[1], toff = d[7];
  const int lane = threadIdx.x;
  if (lane >= rows) return;
  const double4 g = tgeo[rb + lane];
  const double vx = k * g.x, vy = k * g.y;
  double gs[K + 1];                          // h_n = g_n / n!
  scaled_h<K>(0.25 * (vx * vx + vy * vy), gs);
  const cd hv = mkc(0.5 * vx, 0.5 * vy);
  cd uu = mkc(1.0, 0.0);                     // (v/2)^n
  cd* t = tab + (size_t)(toff + lane) * (K + 1);
  for (int n = 0; n <= K; ++n) {
    t[n] = mkc(uu.x * gs[n], uu.y * gs[n]);
    if (n < K) uu = cmul(uu, hv);
  }
}

// A tree fibre's cell moments from its P2M weights (k_p2m_tables): lane m of
// every wavefront takes the orders m and -m (m <= p), wavefront w a
// contiguous eighth of the cell's elements (eight at a time, the next
// eight's weights loaded while the current ones are used), and the eight
// wavefronts' sums meet in LDS in a fixed order.  The first weights' loads
// go out before the densities' (which wait for the rows' indices).
// The densities are staged in stage[0 .. 2 rows) (the launch's dynamic LDS:
// a cell has at most N elements, the launch holds 4N).
template <int P>
__device__ __forceinline__ void p2m_table_cell(int cell, int rb, int rows, const cd* __restrict__ tab,
                                               const int* __restrict__ psi_idx, int N, const cd* __restrict__ psi,
                                               cd* __restrict__ mpole, cd* stage) {
  constexpr int NH = P + 1, NW = PC_THREADS / 64;
  static_assert(NH <= 64, "one order per lane");
  __shared__ cd sPos[NW][NH], sNeg[NW][NH];
  cd* sPh = stage;
  cd* sVp = stage + rows;
  const int w = threadIdx.x >> 6, m = threadIdx.x & 63;
  const int per = (rows + NW - 1) / NW, e0 = min(rows, w * per), e1 = min(rows, e0 + per);
  cd a[8], b[8];
  auto load = [&](int e) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const bool ok = m < NH && e + q < e1;
      const cd* t = tab + ((size_t)(e + q) * NH + m) * 2;
      a[q] = ok ? t[0] : mkc(0, 0);
      b[q] = ok ? t[1] : mkc(0, 0);
    }
  };
  load(e0);
  for (int t = threadIdx.x; t < rows; t += PC_THREADS) {
    const int pi = psi_idx[rb + t];
    sPh[t] = psi[pi];
    sVp[t] = psi[pi + N];
  }
  __syncthreads();
  cd pos = mkc(0, 0), neg = mkc(0, 0);     // M_m and (-1)^m M_{-m} over this wavefront's elements
  for (int e = e0; e < e1; e += 8) {
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (e + q < e1) {
        const cd ph = sPh[e + q], vp = sVp[e + q];
        pos = cadd(pos, cadd(cmul(a[q], ph), cmul(b[q], vp)));
        neg = cadd(neg, csub(cmul(cconj(b[q]), vp), cmul(cconj(a[q]), ph)));
      }
    if (e + 8 < e1) load(e + 8);
  }
  if (m < NH) {
    sPos[w][m] = pos;
    sNeg[w][m] = neg;
  }
  __syncthreads();
  if (w == 0 && m < NH) {
    cd tp = sPos[0][m], tn = sNeg[0][m];
#pragma unroll
    for (int v = 1; v < NW; ++v) {
      tp = cadd(tp, sPos[v][m]);
      tn = cadd(tn, sNeg[v][m]);
    }
    cd* out = mpole + (size_t)cell * 2 * (2 * P + 1) + P;
    out[m] = tp;
    if (m > 0) out[-m] = (m & 1) ? cscale(tn, -1.0) : tn;
  }
}

// With the roots by Fourier modes, each fibre's own-block apply is split
// around the FMM chain so that one inverse transform serves both.  First
// launch: the first workgroups compute the moments of the tree fibres'
// cells below their roots from their P2M weights (p2m_table_cell; mcell =
// [cell, first row, rows, first table row] in the tree order), which thus
// run beside the transforms; the next M (one per fibre and member) take the forward
// transforms of the fibre's densities and write the root's moments and the
// spectrum of P psi, (I + L(kappa)) psihat(kappa), to spec; with one wave,
// the last `ntb` workgroups take the row tasks of the stored near pairs (as
// k_self_apply) and leave the sums in near_buf.
template <int P, typename C>
__global__ void __launch_bounds__(PC_THREADS) k_self_fwd(const cd* __restrict__ in, cd* __restrict__ spec,
                                                         long long vec_stride, const cd* __restrict__ coef,
                                                         const cd* __restrict__ tw, int N, int logN, int M,
                                                         const int4* __restrict__ tasks,
                                                         const long long* __restrict__ toff, int ntasks, int ntb,
                                                         const int* __restrict__ col_psi,
                                                         const C* __restrict__ blocks, cd* __restrict__ near_buf,
                                                         const cd* __restrict__ rtab, cd* __restrict__ mpole,
                                                         long long mp_stride, const int4* __restrict__ mcell,
                                                         const int* __restrict__ psi_idx,
                                                         const cd* __restrict__ p2m_tab,
                                                         const cd* __restrict__ pinv) {
  constexpr int NP = 2 * P + 1;
  extern __shared__ cd pcs[];
  // workgroups: the tree fibres' cells' P2M first (the longest), then the
  // fibres, then the row tasks
  const int nmc = (int)gridDim.x - M - ntb;
  if ((int)blockIdx.x < nmc) {
    const int4 mc = mcell[blockIdx.x];
    p2m_table_cell<P>(mc.x, mc.y, mc.z, p2m_tab + (size_t)mc.w * (P + 1) * 2, psi_idx, N,
                      in + (size_t)blockIdx.y * vec_stride, mpole + blockIdx.y * mp_stride, pcs);
    return;
  }
  if ((int)blockIdx.x >= nmc + M) {
    const int t = ((int)blockIdx.x - nmc - M) * (PC_THREADS / 64) + (threadIdx.x >> 6);
    if (t >= ntasks) return;
    cd a1, a2;
    p2p_row_sums<C>(tasks[t], toff[t], col_psi, blocks, in, N, threadIdx.x & 63, a1, a2);
    if ((threadIdx.x & 63) == 0) {
      near_buf[2 * t] = a1;
      near_buf[2 * t + 1] = a2;
    }
    return;
  }
  const int f = (int)blockIdx.x - nmc;
  const size_t mem = (size_t)blockIdx.y * vec_stride;
  cd* X = pcs;
  cd* Y = pcs + 2 * N;
  const cd* src = in + mem + (size_t)f * 2 * N;   // phi_f then varphi_f
  for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) X[i] = src[i];
  // the mode blocks and the table row do not depend on the transforms: their
  // loads are issued now and land while the transforms run (N <= 512 =
  // PC_THREADS: one mode per thread)
  const int kk = threadIdx.x;
  cd c0 = mkc(0, 0), c1 = c0, c2 = c0, c3 = c0, ta = c0, tb = c0;
  if (kk < N) {
    const cd* c = coef + ((size_t)f * N + kk) * 4;
    c0 = c[0]; c1 = c[1]; c2 = c[2]; c3 = c[3];
  }
  const cd* T = rtab + (size_t)f * 4 * NP;
  if (kk < NP) {
    ta = T[kk];
    tb = T[NP + kk];
  }
  // right preconditioning fused into the apply (pinv != nullptr, only when
  // no kernel of the apply reads the densities themselves): the input is
  // z and the operator acts on P^{-1} z, whose spectrum is the fibre's mode
  // blocks of P^{-1} times that of z
  cd q0 = mkc(0, 0), q1 = q0, q2 = q0, q3 = q0;
  if (pinv && kk < N) {
    const cd* q = pinv + ((size_t)f * N + kk) * 4;
    q0 = q[0]; q1 = q[1]; q2 = q[2]; q3 = q[3];
  }
  __syncthreads();
  cd* H = pc_fft(X, Y, 2, N, logN, tw, true);
  if (pinv) {
    if (kk < N) {
      const cd u = H[kk], v = H[N + kk];
      H[kk] = cadd(cmul(q0, u), cmul(q1, v));
      H[N + kk] = cadd(cmul(q2, u), cmul(q3, v));
    }
    __syncthreads();
  }
  // the root's exterior moments of order n = kk - p from the two densities'
  // transforms and the fibre's table row (A_n, B_n): M_n = A_n phihat(n mod N)
  // + B_n varphihat(n mod N)
  if (kk < NP) {
    const int j = ((kk - P) % N + N) % N;
    mpole[blockIdx.y * mp_stride + (size_t)f * 2 * NP + kk] = cadd(cmul(ta, H[j]), cmul(tb, H[N + j]));
  }
  cd* dst = spec + mem + (size_t)f * 2 * N;
  if (kk < N) {
    const cd u = H[kk], v = H[N + kk];
    dst[kk] = cadd(cmul(c0, u), cmul(c1, v));
    dst[N + kk] = cadd(cmul(c2, u), cmul(c3, v));
  }
}

// acc += the partial expansions of chunks c0 .. c0 + cnt - 1 (coefficient l
// of chunk c at part[c NP + l]), added in chunk order with eight chunks'
// loads in flight at once
template <int NP>
__device__ __forceinline__ cd add_chunks(cd acc, const cd* __restrict__ part, int c0, int cnt, int l) {
  for (int c = 0; c < cnt; c += 8) {
    cd v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = c + q < cnt ? part[(size_t)(c0 + c + q) * NP + l] : mkc(0, 0);
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (c + q < cnt) acc = cadd(acc, v[q]);
  }
  return acc;
}

// Downward pass and L2P of the tree fibres' leaves with a far part from
// below their roots (or stored near pairs), exterior channel only, one
// wavefront per (leaf, member), adding into y after the own-block launch has
// written it.  As k_down, but the M2L partial expansions are summed here
// (a cell's chunks are contiguous): the leaf's own (desc[2], desc[3]: first
// chunk, count) and each ancestor's below the root (anc[desc[4] ..
// desc[5]]: first chunk, count, J-table row), translated to the leaf by L2L;
// then L2P at its rows from their per-frequency values Jp_n (k_l2p_tables:
// table rows from desc[7]), y1 += u, y2 += 2/(i eta (1 + varrho)) dn, plus the
// stored near pairs' row sums (near_buf from task desc[6], one wave).
template <int P>
__global__ void __launch_bounds__(64) k_down_spec(const int* __restrict__ ddesc, const int4* __restrict__ anc,
                                                  const cd* __restrict__ epart, long long ep_stride,
                                                  const cd* __restrict__ jtab, const double4* __restrict__ tgeo,
                                                  const int* __restrict__ psi_idx, int N, double k, double eta,
                                                  double varrho, cd* __restrict__ y, long long y_stride,
                                                  const cd* __restrict__ near_buf, const cd* __restrict__ l2p_tab) {
  constexpr int NP = 2 * P + 1, NT = 4 * P + 1, NU = (NP + 63) / 64, NTU = (NT + 63) / 64, K = P + 1;
  // the L2P tables are indexed through wz (= 0, a lane value to the
  // compiler) so that their reads stay in the order loop instead of being
  // hoisted into registers all at once
  __shared__ cd sJ[NT], sA[NP], sL[NP], sS[1][3][P + 2], sT[1][3][P + 2];
  const int wz = threadIdx.x >> 6;
  epart += blockIdx.y * ep_stride;
  y += blockIdx.y * y_stride;
  const int* d = ddesc + 8 * blockIdx.x;
  const int lane = threadIdx.x;
  const int rb = d[0], rows = d[1], own0 = d[2], ownc = d[3], a0 = d[4], na = d[5] - d[4], t0 = d[6], toff = d[7];
  double4 g = make_double4(0.0, 0.0, 0.0, 0.0);
  int pi = 0;
  if (lane < rows) {
    g = tgeo[rb + lane];
    pi = psi_idx[rb + lane];
  }
  // the ancestors' descriptors (at most 64) come in with the leaf's own chunks
  __shared__ int4 sAn[64];
  if (lane < na) sAn[lane] = anc[a0 + lane];
  cd acc[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) acc[u] = mkc(0, 0);
#pragma unroll
  for (int u = 0; u < NU; ++u)
    if (lane + 64 * u < NP) acc[u] = add_chunks<NP>(acc[u], epart, own0, ownc, lane + 64 * u);
  __syncthreads();
  for (int q = 0; q < na; ++q) {                // wave-uniform trip count
    const int4 an = sAn[q];
    cd sa[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) sa[u] = mkc(0, 0);
#pragma unroll
    for (int u = 0; u < NU; ++u)
      if (lane + 64 * u < NP) sa[u] = add_chunks<NP>(sa[u], epart, an.x, an.y, lane + 64 * u);
    const cd* tj = jtab + (size_t)an.z * NT;
#pragma unroll
    for (int u = 0; u < NU; ++u)
      if (lane + 64 * u < NP) sA[lane + 64 * u] = sa[u];
#pragma unroll
    for (int u = 0; u < NTU; ++u)
      if (lane + 64 * u < NT) sJ[lane + 64 * u] = tj[lane + 64 * u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      int n = min(lane + 64 * u - P, P);      // lanes past the last order repeat it
      cd sres = acc[u];
      for (int idx = 0; idx < NP; ++idx) sres = cfma(sA[idx], sJ[idx - n + P], sres);
      acc[u] = sres;
    }
    __syncthreads();
  }
  for (int u = 0; u < NU; ++u) {
    int i = lane + 64 * u;
    if (i < NP) sL[i] = acc[u];
  }
  __syncthreads();
  // L2P with orders -n and n folded (as k_down)
  if (lane <= K) {
    const int n = lane;
    const double sg = (n & 1) ? -1.0 : 1.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int sh = j == 0 ? 0 : (j == 1 ? 1 : -1);
      const int lp = n + sh, lm = -n + sh;
      cd c = (lp >= -P && lp <= P) ? sL[P + lp] : mkc(0, 0);
      cd e = (lm >= -P && lm <= P) ? cscale(sL[P + lm], sg) : mkc(0, 0);
      cd dd = csub(c, e);
      sS[wz][j][n] = n ? cadd(c, e) : c;
      sT[wz][j][n] = n ? mkc(-dd.y, dd.x) : mkc(0, 0);
    }
  }
  __syncthreads();
  cd u = mkc(0, 0), dv = mkc(0, 0);
  if (lane < rows) {
    const cd* jt = l2p_tab + (size_t)(toff + lane) * (K + 1);   // Jp_n of this row (k_l2p_tables)
    cd sa = mkc(0, 0), sb = mkc(0, 0);
#pragma unroll
    for (int n = 0; n <= K; ++n) {
      const cd jn = jt[n];
      const double x = jn.x, yv = jn.y;                            // Jp_n
      cd s0 = sS[wz][0][n], tt0 = sT[wz][0][n];
      cd s1 = sS[wz][1][n], tt1 = sT[wz][1][n];
      cd s2 = sS[wz][2][n], tt2 = sT[wz][2][n];
      u.x = fma(s0.x, x, fma(tt0.x, yv, u.x));
      u.y = fma(s0.y, x, fma(tt0.y, yv, u.y));
      sa.x = fma(s1.x, x, fma(tt1.x, yv, sa.x));
      sa.y = fma(s1.y, x, fma(tt1.y, yv, sa.y));
      sb.x = fma(s2.x, x, fma(tt2.x, yv, sb.x));
      sb.y = fma(s2.y, x, fma(tt2.y, yv, sb.y));
    }
    cd nu = mkc(g.w, -g.z);
    dv = cscale(csub(cmul(nu, sa), cmul(cconj(nu), sb)), 0.5 * k);
  }
  // the rows of y are read and written after the order loop (read inside the
  // branch above, their loads would be hoisted over it and hold registers)
  __syncthreads();
  if (lane < rows) {
    cd c = mkc(0.0, -2.0 / (eta * (1.0 + varrho)));
    cd y1 = y[pi], y2 = y[pi + N];
    if (t0 >= 0 && near_buf) {
      y1 = cadd(y1, near_buf[2 * (t0 + lane)]);
      y2 = cadd(y2, near_buf[2 * (t0 + lane) + 1]);
    }
    y[pi] = cadd(y1, u);
    y[pi + N] = cadd(y2, cmul(c, dv));
  }
}

// Last launch, after the M2L: workgroup f (one per fibre and member) sums
// its root's M2L partial expansions (chunks rrng[f] = first, count: the
// root's local expansion L), loads the spectrum of P psi and adds N times
// the coefficients of L's far part,
//   u_e = sum_l L_l Jp_l(v_0) w^{l e},
//   far2_e = 2/(i eta (1 + varrho)) sum_l L_l (kap/2)(nu_0 Jp_{l-1} - conj(nu_0) Jp_{l+1}) w^{l e},
// at mode l mod N (orders that alias add up); one inverse transform then
// gives y = P psi + far for the fibre's rows (a tree fibre's downward pass,
// k_down_spec, then adds the far part of its cells below the root).
template <int P>
__global__ void __launch_bounds__(PC_THREADS) k_self_inv(const cd* __restrict__ spec, cd* __restrict__ out,
                                                         long long vec_stride, const cd* __restrict__ tw, int N,
                                                         int logN, const int2* __restrict__ rrng,
                                                         const cd* __restrict__ epart, long long ep_stride,
                                                         const cd* __restrict__ rtab, double eta, double varrho) {
  constexpr int NP = 2 * P + 1, NW = PC_THREADS / 64;
  extern __shared__ cd pcs[];
  __shared__ cd sLw[NW][NP];
  __shared__ cd sT23[2][NP];
  const int f = blockIdx.x;
  const size_t mem = (size_t)blockIdx.y * vec_stride;
  epart += blockIdx.y * ep_stride;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  cd* X = pcs;
  cd* Y = pcs + 2 * N;
  const cd* src = spec + mem + (size_t)f * 2 * N;
  for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) X[i] = src[i];
  // the synthesis rows of the fibre's table, loaded with the spectrum
  for (int i = threadIdx.x; i < 2 * NP; i += blockDim.x) sT23[i / NP][i % NP] = rtab[(size_t)f * 4 * NP + 2 * NP + i];
  // the root's local expansion: wavefront w adds chunks w, w + NW, ... (lane
  // = order), then the NW partial sums in order
  const int2 rr = rrng[f];
  for (int l = lane; l < NP; l += 64) {
    cd sacc = mkc(0, 0);
    for (int c = w; c < rr.y; c += 8 * NW) {   // eight chunks' loads in flight, added in order
      cd v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = c + q * NW < rr.y ? epart[(size_t)(rr.x + c + q * NW) * NP + l] : mkc(0, 0);
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (c + q * NW < rr.y) sacc = cadd(sacc, v[q]);
    }
    sLw[w][l] = sacc;
  }
  __syncthreads();
  if (rr.y > 0) {
    const int P_ = NP >> 1;
    const double nn = (double)N;
    const cd c = mkc(0.0, -2.0 * nn / (eta * (1.0 + varrho)));
    for (int kk = threadIdx.x; kk < N; kk += blockDim.x) {
      cd su = mkc(0, 0), sd = mkc(0, 0);
      for (int l = kk - ((kk + P_) / N) * N; l <= P_; l += N) {
        cd Ll = sLw[0][l + P_];
#pragma unroll
        for (int v = 1; v < NW; ++v) Ll = cadd(Ll, sLw[v][l + P_]);
        su = cfma(Ll, sT23[0][l + P_], su);
        sd = cfma(Ll, sT23[1][l + P_], sd);
      }
      X[kk] = cadd(X[kk], cscale(su, nn));
      X[N + kk] = cadd(X[N + kk], cmul(c, sd));
    }
    __syncthreads();
  }
  const cd* Z = pc_fft(X, Y, 2, N, logN, tw, false);
  const double sc = 1.0 / N;
  cd* dst = out + mem + (size_t)f * 2 * N;
  for (int i = threadIdx.x; i < 2 * N; i += blockDim.x) dst[i] = cscale(Z[i], sc);
}

// Batched P2P: the NB members of a batch share one set of near blocks
// stored without the quasi-periodic phase; member b sees image m of a source
// through alpha_b^m, applied to the densities as they are staged in LDS.
// Each block entry is read from HBM once and used for every member.
template <int NB> struct P2PBatchSeg { static constexpr int value = 1024 / NB; };

template <typename C, int NB>
__global__ void __launch_bounds__(64 * P2P_WAVES) k_p2p_batch(
    const int* __restrict__ leaves, const int* __restrict__ ebeg, const int* __restrict__ eend,
    const int* __restrict__ psi_idx, int N, const long long* __restrict__ leaf_blk,
    const int* __restrict__ cols_ptr, const int* __restrict__ col_psi, const int* __restrict__ col_m,
    const cd* __restrict__ alpha, int alpha_stride, int m_min, int B, long long stride,
    const C* __restrict__ blocks, const int* __restrict__ ccols_ptr, const int* __restrict__ ccol_psi,
    const int* __restrict__ ccol_loc, const cd* __restrict__ circ, const cd* __restrict__ psi,
    cd* y, const cd* ybase, const int* __restrict__ item_leaf, int n_leaves, int S, cd* __restrict__ part) {
  constexpr int SEG = P2PBatchSeg<NB>::value;
  __shared__ C sp[SEG][NB][2];
  __shared__ int sl[SEG];
  __shared__ cd r1[P2P_WAVES][64], r2[P2P_WAVES][64];
  // work item = (target leaf, column split); with S > 1 the splits write
  // partial rows [split][member][vector] that k_combine adds in a fixed order
  for (int item = blockIdx.x; item < n_leaves * S; item += gridDim.x) {
    int lw = item / S, sp_i = item - lw * S;
    int li = item_leaf ? item_leaf[lw] : lw;
    int k0 = cols_ptr[li], ncol = cols_ptr[li + 1] - k0;
    if (ybase == y && ncol == 0 && ccols_ptr[li + 1] == ccols_ptr[li]) continue;
    int D = leaves[li];
    int db = ebeg[D], rows = eend[D] - db;
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    C a1[NB], a2[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) a1[b] = a2[b] = p2p_cvt<C>(mkc(0, 0));
    int chunk = (ncol + S - 1) / S;
    int c_lo = min(ncol, sp_i * chunk), c_hi = min(ncol, c_lo + chunk);
    const C* bl = blocks + 4 * leaf_blk[li];
    const unsigned cstride = 4u * (unsigned)rows;
    bool act = lane < rows;
    for (int seg = c_lo; seg < c_hi; seg += SEG) {
      int nseg = min(SEG, c_hi - seg);
      for (int i = threadIdx.x; i < nseg * NB; i += 64 * P2P_WAVES) {
        int col = i / NB, b = i - col * NB;
        cd v0 = mkc(0, 0), v1 = mkc(0, 0);
        if (b < B) {
          int pi = col_psi[k0 + seg + col];
          cd ph = alpha[b * alpha_stride + col_m[k0 + seg + col] - m_min];
          v0 = cmul(ph, psi[b * stride + pi]);
          v1 = cmul(ph, psi[b * stride + pi + N]);
        }
        sp[col][b][0] = p2p_cvt<C>(v0);
        sp[col][b][1] = p2p_cvt<C>(v1);
      }
      __syncthreads();
      const C* bs = bl + (size_t)seg * cstride + lane;
      if (act) {
        for (int k = w; k < nseg; k += P2P_WAVES) {
          unsigned o = (unsigned)k * cstride;
          C b11 = nt_load(bs + o), b12 = nt_load(bs + o + rows);
          C b21 = nt_load(bs + o + 2 * rows), b22 = nt_load(bs + o + 3 * rows);
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            C ph = sp[k][b][0], vp = sp[k][b][1];
            a1[b] = p2p_fma(b11, ph, a1[b]);
            a1[b] = p2p_fma(b12, vp, a1[b]);
            a2[b] = p2p_fma(b21, ph, a2[b]);
            a2[b] = p2p_fma(b22, vp, a2[b]);
          }
        }
      }
      __syncthreads();
    }
    // circulant columns (same fibre, image 0, so no image phase), as in k_p2p
    {
      const int q0 = ccols_ptr[li], nq = ccols_ptr[li + 1] - q0;
      const int qchunk = (nq + S - 1) / S;
      const int q_lo = min(nq, sp_i * qchunk), q_hi = min(nq, q_lo + qchunk);
      const int pr = psi_idx[db + min(lane, rows - 1)];
      const int fD = pr / (2 * N), aloc = pr - 2 * fD * N;
      const cd* crow = circ + (size_t)fD * 8 * N + (N - aloc);
      for (int seg = q_lo; seg < q_hi; seg += SEG) {
        int nseg = min(SEG, q_hi - seg);
        for (int i = threadIdx.x; i < nseg * NB; i += 64 * P2P_WAVES) {
          int col = i / NB, b = i - col * NB;
          cd v0 = mkc(0, 0), v1 = mkc(0, 0);
          if (b < B) {
            int pi = ccol_psi[q0 + seg + col];
            v0 = psi[b * stride + pi];
            v1 = psi[b * stride + pi + N];
          }
          sp[col][b][0] = p2p_cvt<C>(v0);
          sp[col][b][1] = p2p_cvt<C>(v1);
          if (b == 0) sl[col] = ccol_loc[q0 + seg + col];
        }
        __syncthreads();
        if (act) {
          for (int k = w; k < nseg; k += P2P_WAVES) {
            const cd* cr = crow + sl[k];
            const C b11 = p2p_cvt<C>(cr[0]), b12 = p2p_cvt<C>(cr[2 * N]);
            const C b21 = p2p_cvt<C>(cr[4 * N]), b22 = p2p_cvt<C>(cr[6 * N]);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              C ph = sp[k][b][0], vp = sp[k][b][1];
              a1[b] = p2p_fma(b11, ph, a1[b]);
              a1[b] = p2p_fma(b12, vp, a1[b]);
              a2[b] = p2p_fma(b21, ph, a2[b]);
              a2[b] = p2p_fma(b22, vp, a2[b]);
            }
          }
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      r1[w][lane] = p2p_wide(a1[b]);
      r2[w][lane] = p2p_wide(a2[b]);
      __syncthreads();
      if (w == 0 && act && b < B) {
        cd s1 = r1[0][lane], s2 = r2[0][lane];
#pragma unroll
        for (int v = 1; v < P2P_WAVES; ++v) {
          s1 = cadd(s1, r1[v][lane]);
          s2 = cadd(s2, r2[v][lane]);
        }
        int pi = psi_idx[db + lane];
        if (S == 1) {
          const cd* pb_ = ybase + b * stride;
          cd* yb = y + b * stride;
          yb[pi] = cadd(pb_[pi], s1);
          yb[pi + N] = cadd(pb_[pi + N], s2);
        } else {
          cd* pp = part + ((size_t)sp_i * B + b) * stride;
          pp[pi] = s1;
          pp[pi + N] = s2;
        }
      }
      __syncthreads();
    }
  }
}

__global__ void k_to_c64(long long n, const cd* __restrict__ in, float2* __restrict__ out) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    float2 r;
    r.x = (float)in[i].x;
    r.y = (float)in[i].y;
    out[i] = r;
  }
}

// Clear a buffer of n16 16-byte words with vector stores (a kernel rather
// than a memset node, so that the clear may sit inside a captured graph).
__global__ void k_fill_zero(double2* __restrict__ p, long long n16) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) p[i] = make_double2(0.0, 0.0);
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  const long long n16 = (long long)(bytes / 16);
  if (n16 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, s, (double2*)p, n16);
  return hipGetLastError();
}

hipError_t launch_near_to_c64(Problem& pb) {
  long long n = 4 * pb.n_near_stored;
  if (n == 0 || !pb.d_near32) return hipSuccess;
  hipLaunchKernelGGL(k_to_c64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, pb.stream, n, pb.d_near,
                     pb.d_near32);
  return hipGetLastError();
}

template <int P>
static hipError_t tables_impl(Problem& pb) {
  const HostPlan& hp = pb.hp;
  int n_off = (int)hp.off_xy.size() / 2;
  int n_joff = (int)hp.joff_xy.size() / 2;
  if (n_off > 0)
    hipLaunchKernelGGL(k_htab<P>, dim3((2 * n_off + 63) / 64), dim3(64), 0, pb.stream, n_off, pb.n_tab,
                       pb.d_off_xy, pb.k, pb.k1, pb.d_htab);
  if (n_joff > 0)
    hipLaunchKernelGGL(k_jtab<P>, dim3((2 * n_joff + 63) / 64), dim3(64), 0, pb.stream, n_joff,
                       pb.d_joff_xy, pb.k, pb.k1, pb.d_jtab);
  if (pb.spec_root)
    hipLaunchKernelGGL(k_spec_tables<P>, dim3(pb.M), dim3(128), 0, pb.stream, pb.N, pb.d_centres, pb.d_mx, pb.d_my,
                       pb.d_tx, pb.d_ty, pb.d_h, pb.d_gl, pb.opt.g_far, pb.k, pb.eta, pb.d_spec_tab);
  if (pb.spec_root && pb.n_dleaves > 0)
    hipLaunchKernelGGL(k_l2p_tables<P>, dim3(pb.n_dleaves), dim3(64), 0, pb.stream, pb.d_dldesc,
                       reinterpret_cast<const double4*>(pb.d_tgeo), pb.k, pb.d_l2p_tab);
  if (pb.spec_root && pb.n_mcells > 0)
    hipLaunchKernelGGL(k_p2m_tables<P>, dim3(pb.n_mcells, P2M_TAB_SPLIT), dim3(64), 0, pb.stream,
                       reinterpret_cast<const int4*>(pb.d_mcell), pb.d_elem_of, pb.d_cx, pb.d_cy, pb.d_mx, pb.d_my,
                       pb.d_tx, pb.d_ty, pb.d_h, pb.d_gl, pb.opt.g_far, pb.k, pb.eta, pb.d_p2m_tab);
  return hipGetLastError();
}

// The FMM chain: P2M, M2M (leaves to every ancestor), M2L with the lattice
// sums, downward pass (every ancestor to the leaves) with L2P into the
// far-field buffer.
template <int P>
// join != nullptr: the stream waits for it before the downward pass, which
// then adds the far part into y_join (holding psi + near) instead of d_far.
// With each fibre's own block applied by FFT (pb.self_fft) only the exterior
// channel carries pairs, so the chain runs channel 0 alone (the upward pass of
// the test hook keeps both).
// only >= 0: launch stage `only` alone (0 P2M, 1 M2M, 2 M2L with the lattice
// sums, 3 downward pass with L2P into the far-field buffer) reps times back
// to back, for timing one kernel in steady state.
// With the roots by Fourier modes (pb.spec_root) the chain covers only the
// tree fibres' leaves and cells: the roots' moments and the spectral fibres'
// far rows come from the own-block launches around it (apply_spectral).
static void fmm_chain(Problem& pb, const cd* d_psi, hipStream_t s, hipEvent_t* ev, bool upward_only, int B,
                      hipEvent_t join = nullptr, cd* y_join = nullptr, bool near_in_down = false, int only = -1,
                      int reps = 1) {
  auto times = [&](int stage) { return only < 0 ? 1 : (only == stage ? reps : 0); };
  const HostPlan& hp = pb.hp;
  // fibre roots by their Fourier modes: every cell's moments come from the
  // first own-block launch (no P2M or M2M here), no M2L sums and no
  // downward pass here (the last own-block launch adds the partials and runs
  // it)
  const bool spec = pb.spec_root && !upward_only;
  int n_leaves = spec ? 0 : (int)hp.leaves.size();
  const int* leaves = pb.d_leaves;
  const int* ldesc = pb.d_ldesc;
  const int n_down = spec ? 0 : n_leaves;       // spectral: the downward pass runs in k_self_inv
  const int* ddesc = pb.d_ldesc;
  const int* near_t0 = pb.d_leaf_near_t0;
  const int n_up = spec ? 0 : pb.n_up;           // spectral: every moment comes from the first launch
  const int* up_cells = pb.d_up_cells;
  const int* up_ptr = pb.d_up_ptr;
  const int* up_src = pb.d_up_src;
  const int* up_off = pb.d_up_off;
  int n_joff = (int)hp.joff_xy.size() / 2;
  const BatchStrides bs = batch_strides(pb);
  const int nch = pb.self_fft && !upward_only ? 1 : 2;
  if (ev) (void)hipEventRecord(ev[0], s);
  // one group of two wavefronts per (leaf, channel): two groups (PS = 2)
  // were slower on the square 8x8 block with one channel (21.7 us against
  // 15.5 us in order)
  for (int r = 0; r < times(0); ++r) {
    // few leaves (the tree fibres of a mostly spectral block): four groups
    // of two wavefronts per (leaf, channel), each taking a quarter of the
    // Gauss points, so that the launch is not one long serial loop per leaf
    if (n_leaves > 0 && n_leaves * nch * B < 2 * pb.n_cu)
      hipLaunchKernelGGL((k_p2m<P, 4>), dim3(n_leaves, nch, B), dim3(512), 0, s, leaves, ldesc,
                         reinterpret_cast<const double4*>(pb.d_tgeo), pb.d_trh, pb.d_psi_idx, pb.d_gl,
                         pb.opt.g_far, pb.N, pb.k, pb.k1, pb.eta, d_psi, pb.d_mpole, bs.vec, bs.mpole);
    else if (n_leaves > 0)
      hipLaunchKernelGGL((k_p2m<P, 1>), dim3(n_leaves, nch, B), dim3(128), 0, s, leaves, ldesc,
                         reinterpret_cast<const double4*>(pb.d_tgeo), pb.d_trh, pb.d_psi_idx, pb.d_gl,
                         pb.opt.g_far, pb.N, pb.k, pb.k1, pb.eta, d_psi, pb.d_mpole, bs.vec, bs.mpole);
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  for (int r = 0; r < times(1) && n_up > 0; ++r)
    hipLaunchKernelGGL(k_m2m<P>, dim3(n_up, nch, B), dim3(64 * M2M_WAVES), 0, s, up_cells, up_ptr, up_src, up_off,
                       pb.d_jtab, n_joff, pb.d_mpole, bs.mpole);
  if (ev) (void)hipEventRecord(ev[2], s);
  if (upward_only) return;
  for (int r = 0; r < times(2) && pb.n_mchunks > 0; ++r) {
    if (pb.n_vchunks > 0)
      hipLaunchKernelGGL(k_m2l<P>, dim3(pb.n_vchunks, B), dim3(64), 0, s, pb.d_mchunks, pb.d_e_src, pb.d_e_off,
                         pb.d_e_m, pb.d_htab, pb.n_tab, pb.d_alpha, hp.m_min, pb.d_mpole, pb.d_epart, bs.mpole,
                         bs.epart, bs.tab, bs.alpha, pb.d_vchunks);
    if (pb.n_mfma_items > 0)
      hipLaunchKernelGGL(k_m2l_mfma<P>, dim3(pb.n_mfma_items, B), dim3(64 * m2l_mfma_waves<P>()), 0, s,
                         reinterpret_cast<const int4*>(pb.d_mfma_items),
                         reinterpret_cast<const int4*>(pb.d_mfma_cols), pb.d_htab, pb.n_tab, pb.d_alpha, hp.m_min,
                         pb.d_mpole, pb.d_epart, bs.mpole, bs.epart, bs.tab, bs.alpha);
    if (pb.lat_fft) {
      const int ns = pb.lat_ns, pxy = pb.lat_px * pb.lat_py;
      constexpr int NP = 2 * P + 1;
      hipLaunchKernelGGL(k_lat_fwd<P>, dim3(NP, ns, B), dim3(256), 0, s, pb.d_mpole, bs.mpole, pb.d_lat_cell, ns,
                         pb.lat_gx, pb.lat_gy, pb.lat_px, pb.lat_py, pb.d_lat_xhat);
      hipLaunchKernelGGL(k_lat_mul<P>, dim3(pxy, ns, B), dim3(64), 0, s, pb.d_lat_shat, pb.d_lat_xhat, ns, pxy,
                         pb.d_lat_lhat);
      hipLaunchKernelGGL(k_lat_inv<P>, dim3(NP, ns, B), dim3(256), 0, s, pb.d_lat_lhat, pb.d_lat_slot, ns,
                         pb.lat_gx, pb.lat_gy, pb.lat_px, pb.lat_py, pb.d_epart, bs.epart);
    }
    // with the roots by Fourier modes the consumers add the partials themselves
    if (!spec)
      hipLaunchKernelGGL(k_m2l_sum<P>, dim3(pb.n_chunks, B), dim3(256), 0, s, pb.d_chunks, pb.d_epart, pb.d_part,
                         bs.epart, bs.part);
  }
  if (ev) (void)hipEventRecord(ev[3], s);
  if (join) (void)hipStreamWaitEvent(s, join, 0);
  for (int r = 0; r < times(3) && n_down > 0; ++r)
    hipLaunchKernelGGL(k_down<P>, dim3(n_down, B), dim3(64 * nch), 0, s, ddesc,
                       reinterpret_cast<const int2*>(pb.d_lanc), reinterpret_cast<const double4*>(pb.d_tgeo),
                       pb.d_psi_idx, pb.d_part, pb.d_jtab, n_joff, pb.N, pb.k, pb.k1, pb.eta, pb.varrho,
                       y_join ? y_join : pb.d_far, bs.part, bs.vec, y_join ? 1 : 0,
                       near_in_down ? near_t0 : nullptr, pb.d_near_rows);
  if (ev) (void)hipEventRecord(ev[4], s);
}

template <int P, typename C>
static hipError_t apply_spectral(Problem& pb, const C* blocks, const cd* d_psi, cd* d_y, hipEvent_t* ev, int B,
                                 int only = -1, int reps = 1);

// One stage of the chain launched reps times back to back between events
// e0 and e1 on the handle's stream, after one whole chain that leaves every
// stage's inputs in place (each stage then rewrites the same outputs).
template <int P>
static hipError_t stage_timed_impl(Problem& pb, const cd* d_psi, int stage, int reps, hipEvent_t e0,
                                   hipEvent_t e1) {
  if (pb.spec_root) {
    // the stages of apply_spectral, with the far-part buffer as the output
    (void)apply_spectral<P, cd>(pb, pb.d_near, d_psi, pb.d_far, nullptr, 0);
    (void)hipEventRecord(e0, pb.stream);
    (void)apply_spectral<P, cd>(pb, pb.d_near, d_psi, pb.d_far, nullptr, 0, stage, reps);
    (void)hipEventRecord(e1, pb.stream);
    return hipGetLastError();
  }
  fmm_chain<P>(pb, d_psi, pb.stream, nullptr, false, 1);
  (void)hipEventRecord(e0, pb.stream);
  fmm_chain<P>(pb, d_psi, pb.stream, nullptr, false, 1, nullptr, nullptr, false, stage, reps);
  (void)hipEventRecord(e1, pb.stream);
  return hipGetLastError();
}

template <int P>
static hipError_t upward_impl(Problem& pb, const cd* d_psi, hipEvent_t* ev) {
  fmm_chain<P>(pb, d_psi, pb.stream, ev, true, 1);
  return hipGetLastError();
}

template <typename C, int NB>
static void launch_p2p_batch(Problem& pb, hipStream_t st, int grid, const C* blocks, const cd* d_psi, cd* d_y,
                             int B) {
  const BatchStrides bs = batch_strides(pb);
  hipLaunchKernelGGL((k_p2p_batch<C, NB>), dim3(grid), dim3(64 * P2P_WAVES), 0, st, pb.d_leaves,
                     pb.d_ebeg, pb.d_eend, pb.d_psi_idx, pb.N, pb.d_leaf_blk, pb.d_cols_ptr, pb.d_col_psi,
                     pb.d_col_m, pb.d_alpha, bs.alpha, pb.hp.m_min, B, bs.vec, blocks, pb.d_ccols_ptr,
                     pb.d_ccol_psi, pb.d_ccol_loc, pb.d_circ, d_psi, d_y, pb.self_fft ? d_y : d_psi,
                     pb.self_fft ? pb.d_p2p_items : nullptr,
                     pb.self_fft ? pb.n_p2p_items : (int)pb.hp.leaves.size(), pb.p2p_split, pb.d_p2ppart);
}

// y = (I - A) psi.  Without stage events the FMM chain runs on the side
// stream while the near field streams through HBM on the caller's stream;
// the far part is added after the join.  With stage events everything runs
// in order on the caller's stream so that each stage can be timed alone.
// B = 0: one wave, image phases inside the near blocks; B >= 1: a batch of
// B members (one per incidence angle) over phase-free near blocks.
template <int P, typename C>
static void launch_p2p_any(Problem& pb, hipStream_t ps, const C* blocks, const cd* d_psi, cd* d_y, int B) {
  // with the own blocks by FFT, only the leaves with stored near columns
  const int* item_leaf = pb.self_fft ? pb.d_p2p_items : nullptr;
  int n_leaves = pb.self_fft ? pb.n_p2p_items : (int)pb.hp.leaves.size();
  if (n_leaves == 0) return;
  if (pb.self_fft && B == 0) {
    // one wavefront per target row of those leaves
    hipLaunchKernelGGL((k_p2p_rows<C>), dim3(pb.n_p2p_rowtasks), dim3(64), 0, ps,
                       reinterpret_cast<const int4*>(pb.d_p2p_rowtasks), pb.d_p2p_rowoff, pb.d_col_psi, blocks,
                       d_psi, pb.N, d_y);
    return;
  }
  int items = n_leaves * pb.p2p_split;
  int p2p_grid = pb.p2p_grid > 0 ? std::min(pb.p2p_grid, items) : items;
  if (B == 0) {
#define PFM_P2P(U)                                                                                             \
  hipLaunchKernelGGL((k_p2p<C, U>), dim3(p2p_grid), dim3(64 * P2P_WAVES),                                      \
                     pb.p2p_wmax ? 4 * P2P_WCAP * sizeof(cd) : 0, ps, pb.d_leaves, pb.d_ebeg, pb.d_eend,       \
                     pb.d_psi_idx, pb.N, pb.d_leaf_blk, pb.d_cols_ptr, pb.d_col_psi, blocks, pb.d_ccols_ptr,    \
                     pb.d_ccol_psi, pb.d_ccol_loc, pb.d_circ, pb.d_cwin, d_psi, d_y,                           \
                     pb.self_fft ? d_y : d_psi, item_leaf, n_leaves, pb.p2p_split, pb.d_p2ppart, 2LL * pb.E)
    if (pb.p2p_unroll == 4) PFM_P2P(4);
    else if (pb.p2p_unroll == 2) PFM_P2P(2);
    else PFM_P2P(1);
#undef PFM_P2P
  } else if (B == 1) {
    launch_p2p_batch<C, 1>(pb, ps, p2p_grid, blocks, d_psi, d_y, B);
  } else if (B == 2) {
    launch_p2p_batch<C, 2>(pb, ps, p2p_grid, blocks, d_psi, d_y, B);
  } else if (B <= 4) {
    launch_p2p_batch<C, 4>(pb, ps, p2p_grid, blocks, d_psi, d_y, B);
  } else if (B <= 8) {
    launch_p2p_batch<C, 8>(pb, ps, p2p_grid, blocks, d_psi, d_y, B);
  } else {
    launch_p2p_batch<C, 16>(pb, ps, p2p_grid, blocks, d_psi, d_y, B);
  }
}

// The apply with the roots by Fourier modes (pb.spec_root), in order on the
// caller's stream:
//   1. k_self_fwd: forward transforms, roots' moments, spectrum of P psi
//      (one wave: also the stored near pairs' row sums), and in the same
//      launch P2M at the tree fibres' leaves;
//   2. M2M into the tree fibres' cells below their roots;
//   3. M2L with the lattice sums (partial expansions only: the consumers
//      add them);
//   4. k_self_inv: y = P psi plus the far part of each fibre's root local
//      expansion; k_down_spec: the downward pass of the tree fibres' leaves
//      adds the far part of their cells below the root (one wave: and the
//      near row sums); a batch: P2P of the stored pairs adds into y.
// With stage events the same launches are bracketed by ev[0..4] (ev[5] and
// ev[6] follow at once: the near part and the join are inside stages 1 and
// 4).  only >= 0 repeats that stage reps times (steady-state timing).
template <int P, typename C>
static hipError_t apply_spectral(Problem& pb, const C* blocks, const cd* d_psi, cd* d_y, hipEvent_t* ev, int B,
                                 int only, int reps) {
  auto times = [&](int stage) { return only < 0 ? 1 : (only == stage ? reps : 0); };
  const int nb = B > 0 ? B : 1;
  const BatchStrides bs = batch_strides(pb);
  const int ntask = B == 0 ? pb.n_p2p_rowtasks : 0, tpb = PC_THREADS / 64;
  const int extra = (ntask + tpb - 1) / tpb;
  const size_t lds = 4 * (size_t)pb.N * sizeof(cd);
  constexpr int NP = 2 * P + 1;
  if (ev) (void)hipEventRecord(ev[0], pb.stream);
  for (int r = 0; r < times(0); ++r) {
    const int ntb = B == 0 ? extra : 0;
    hipLaunchKernelGGL((k_self_fwd<P, C>), dim3(pb.M + ntb + pb.n_mcells, nb), dim3(PC_THREADS), lds, pb.stream,
                       d_psi, pb.d_spec_hat, bs.vec, pb.d_pc_fwd, pb.d_pc_tw, pb.N, pb.pc_logN, pb.M,
                       reinterpret_cast<const int4*>(pb.d_p2p_rowtasks), pb.d_p2p_rowoff, ntask, ntb, pb.d_col_psi,
                       blocks, pb.d_near_rows, pb.d_spec_tab, pb.d_mpole, bs.mpole,
                       reinterpret_cast<const int4*>(pb.d_mcell), pb.d_psi_idx,
                       pb.d_p2m_tab, pb.pc_fused_inv);
  }
  if (ev) (void)hipEventRecord(ev[1], pb.stream);
  for (int r = 0; r < times(1); ++r) fmm_chain<P>(pb, d_psi, pb.stream, nullptr, false, nb, nullptr, nullptr, false, 1, 1);
  if (ev) (void)hipEventRecord(ev[2], pb.stream);
  for (int r = 0; r < times(2); ++r) fmm_chain<P>(pb, d_psi, pb.stream, nullptr, false, nb, nullptr, nullptr, false, 2, 1);
  if (ev) (void)hipEventRecord(ev[3], pb.stream);
  for (int r = 0; r < times(3); ++r) {
    hipLaunchKernelGGL(k_self_inv<P>, dim3(pb.M, nb), dim3(PC_THREADS), lds, pb.stream, pb.d_spec_hat, d_y, bs.vec,
                       pb.d_pc_tw, pb.N, pb.pc_logN, reinterpret_cast<const int2*>(pb.d_spec_rng), pb.d_epart,
                       bs.epart, pb.d_spec_tab, pb.eta, pb.varrho);
    if (pb.n_dleaves > 0)
      hipLaunchKernelGGL(k_down_spec<P>, dim3(pb.n_dleaves, nb), dim3(64), 0, pb.stream, pb.d_dldesc,
                         reinterpret_cast<const int4*>(pb.d_danc), pb.d_epart, bs.epart, pb.d_jtab,
                         reinterpret_cast<const double4*>(pb.d_tgeo), pb.d_psi_idx, pb.N, pb.k, pb.eta, pb.varrho,
                         d_y, bs.vec, B == 0 ? pb.d_near_rows : nullptr, pb.d_l2p_tab);
    if (B > 0) launch_p2p_any<P, C>(pb, pb.stream, blocks, d_psi, d_y, B);
  }
  if (ev) {
    (void)hipEventRecord(ev[4], pb.stream);
    (void)hipEventRecord(ev[5], pb.stream);
    (void)hipEventRecord(ev[6], pb.stream);
  }
  return hipGetLastError();
}

// The apply with each fibre's own image-0 block applied by FFT (pb.self_fft):
//   y = P psi + near(psi) + far(psi),
// P the block-diagonal operator of the fibres' own blocks (identity included),
// near the stored P2P blocks of pairs between fibres or with images, far the
// exterior FMM chain.  Everything runs in order on the caller's stream: P
// writes y, P2P adds the near part, and the chain's downward pass adds the far
// part (a second stream for P and P2P was 4.5 us slower on the square 8x8
// block: the crossings between hardware queues cost more than the overlap
// gains).  With stage events the chain comes first and writes the far part to
// its buffer, P and P2P write y, and the join kernel adds the far part.
template <int P, typename C>
static hipError_t apply_self_fft(Problem& pb, const C* blocks, const cd* d_psi, cd* d_y, hipEvent_t* ev, int B) {
  if (pb.spec_root) return apply_spectral<P, C>(pb, blocks, d_psi, d_y, ev, B);
  const int nb = B > 0 ? B : 1;
  if (ev) {
    fmm_chain<P>(pb, d_psi, pb.stream, ev, false, nb);
    hipError_t e = launch_precond(pb, d_psi, d_y, false, nb, pb.stream);
    if (e != hipSuccess) return e;
    launch_p2p_any<P, C>(pb, pb.stream, blocks, d_psi, d_y, B);
    (void)hipEventRecord(ev[5], pb.stream);
    long long n = 2LL * pb.E * nb;
    hipLaunchKernelGGL(k_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, pb.stream, n, pb.d_far, d_psi,
                       pb.d_p2ppart, 1, d_y);
    (void)hipEventRecord(ev[6], pb.stream);
    return hipGetLastError();
  }
  if (B == 0) {
    // one launch for P psi and the stored pairs' row sums, which the
    // downward pass adds with the far part
    const int ntask = pb.n_p2p_rowtasks, tpb = PC_THREADS / 64;
    const int extra = (ntask + tpb - 1) / tpb;
    const size_t lds = 4 * (size_t)pb.N * sizeof(cd);
    hipLaunchKernelGGL((k_self_apply<C>), dim3(pb.M + extra), dim3(PC_THREADS), lds, pb.stream, d_psi, d_y,
                       pb.d_pc_fwd, pb.d_pc_tw, pb.N, pb.pc_logN, pb.M,
                       reinterpret_cast<const int4*>(pb.d_p2p_rowtasks), pb.d_p2p_rowoff, ntask, pb.d_col_psi,
                       blocks, pb.d_near_rows);
    fmm_chain<P>(pb, d_psi, pb.stream, nullptr, false, nb, nullptr, d_y, ntask > 0);
    return hipGetLastError();
  }
  hipError_t e = launch_precond(pb, d_psi, d_y, false, nb, pb.stream);
  if (e != hipSuccess) return e;
  launch_p2p_any<P, C>(pb, pb.stream, blocks, d_psi, d_y, B);
  fmm_chain<P>(pb, d_psi, pb.stream, nullptr, false, nb, nullptr, d_y);
  return hipGetLastError();
}

template <int P, typename C>
static hipError_t apply_impl_t(Problem& pb, const C* blocks, const cd* d_psi, cd* d_y, hipEvent_t* ev, int B) {
  if (pb.self_fft) return apply_self_fft<P, C>(pb, blocks, d_psi, d_y, ev, B);
  const HostPlan& hp = pb.hp;
  int n_leaves = (int)hp.leaves.size();
  int nb = B > 0 ? B : 1;
  // Overlapped: the longer branch runs on the caller's stream and the shorter
  // on the side stream, so that the join event has fired by the time the
  // caller's stream reaches it (crossing between hardware queues costs
  // microseconds at the fork and at the join).  P2P is the shorter branch
  // when most near pairs come from the circulant rows.
  const bool p2p_side = !ev && pb.p2p_on_side;
  hipStream_t ps = p2p_side ? pb.side : pb.stream;
  hipStream_t fs = (ev || p2p_side) ? pb.stream : pb.side;
  if (!ev) {
    (void)hipEventRecord(pb.ev_fork, pb.stream);
    (void)hipStreamWaitEvent(pb.side, pb.ev_fork, 0);
  }
  if (ev) fmm_chain<P>(pb, d_psi, fs, ev, false, nb);
  // P2P is queued first: on the side stream it starts while the chain is
  // queued; on the caller's stream the chain's side-stream launches follow
  int items = n_leaves * pb.p2p_split;
  int p2p_grid = pb.p2p_grid > 0 ? std::min(pb.p2p_grid, items) : items;
  if (B == 0) {
#define PFM_P2P(U)                                                                                             \
  hipLaunchKernelGGL((k_p2p<C, U>), dim3(p2p_grid), dim3(64 * P2P_WAVES),                                      \
                     pb.p2p_wmax ? 4 * P2P_WCAP * sizeof(cd) : 0, ps, pb.d_leaves, pb.d_ebeg, pb.d_eend,       \
                     pb.d_psi_idx, pb.N, pb.d_leaf_blk, pb.d_cols_ptr, pb.d_col_psi, blocks, pb.d_ccols_ptr,    \
                     pb.d_ccol_psi, pb.d_ccol_loc, pb.d_circ, pb.d_cwin, d_psi, d_y,                           \
                     pb.self_fft ? d_y : d_psi, nullptr, n_leaves, pb.p2p_split, pb.d_p2ppart, 2LL * pb.E)
    if (pb.p2p_unroll == 4) PFM_P2P(4);
    else if (pb.p2p_unroll == 2) PFM_P2P(2);
    else PFM_P2P(1);
#undef PFM_P2P
  } else if (B == 1) {
    launch_p2p_batch<C, 1>(pb, ps, p2p_grid, blocks, d_psi, d_y, B);
  } else if (B == 2) {
    launch_p2p_batch<C, 2>(pb, ps, p2p_grid, blocks, d_psi, d_y, B);
  } else if (B <= 4) {
    launch_p2p_batch<C, 4>(pb, ps, p2p_grid, blocks, d_psi, d_y, B);
  } else if (B <= 8) {
    launch_p2p_batch<C, 8>(pb, ps, p2p_grid, blocks, d_psi, d_y, B);
  } else {
    launch_p2p_batch<C, 16>(pb, ps, p2p_grid, blocks, d_psi, d_y, B);
  }
  if (ev) (void)hipEventRecord(ev[5], pb.stream);
  if (!ev && p2p_side && B == 0 && pb.p2p_split == 1) {
    // P2P wrote y = psi + near on the side stream: the chain waits for it
    // just before the downward pass, which adds the far part into y (P2P
    // has long finished by then, and no join kernel follows)
    (void)hipEventRecord(pb.ev_join, pb.side);
    fmm_chain<P>(pb, d_psi, fs, nullptr, false, nb, pb.ev_join, d_y);
    return hipGetLastError();
  }
  if (!ev) {
    fmm_chain<P>(pb, d_psi, fs, nullptr, false, nb);
    (void)hipEventRecord(pb.ev_join, pb.side);
    (void)hipStreamWaitEvent(pb.stream, pb.ev_join, 0);
  }
  long long n = 2LL * pb.E * nb;
  hipLaunchKernelGGL(k_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, pb.stream, n, pb.d_far, d_psi,
                     pb.d_p2ppart, pb.p2p_split, d_y);
  if (ev) (void)hipEventRecord(ev[6], pb.stream);
  return hipGetLastError();
}

template <int P>
static hipError_t apply_impl(Problem& pb, const cd* d_psi, cd* d_y, hipEvent_t* ev) {
  return apply_impl_t<P, double2>(pb, pb.d_near, d_psi, d_y, ev, 0);
}
template <int P>
static hipError_t apply_mixed_impl(Problem& pb, const cd* d_psi, cd* d_y) {
  return apply_impl_t<P, float2>(pb, pb.d_near32, d_psi, d_y, nullptr, 0);
}
template <int P>
static hipError_t apply_batch_impl(Problem& pb, const cd* d_psi, cd* d_y, hipEvent_t* ev) {
  return apply_impl_t<P, double2>(pb, pb.d_near, d_psi, d_y, ev, pb.B);
}

#define PFM_DISPATCH(fn, ...)                        \
  switch (pb.opt.p) {                                \
    case 8: return fn<8>(__VA_ARGS__);               \
    case 12: return fn<12>(__VA_ARGS__);             \
    case 16: return fn<16>(__VA_ARGS__);             \
    case 20: return fn<20>(__VA_ARGS__);             \
    case 24: return fn<24>(__VA_ARGS__);             \
    case 32: return fn<32>(__VA_ARGS__);             \
    case 40: return fn<40>(__VA_ARGS__);             \
    default: return hipErrorInvalidValue;            \
  }

hipError_t launch_tables(Problem& pb) { PFM_DISPATCH(tables_impl, pb) }
hipError_t apply_operator(Problem& pb, const cd* d_psi, cd* d_y, hipEvent_t* ev) {
  PFM_DISPATCH(apply_impl, pb, d_psi, d_y, ev)
}
hipError_t apply_upward(Problem& pb, const cd* d_psi) { PFM_DISPATCH(upward_impl, pb, d_psi, nullptr) }
hipError_t time_chain_stage(Problem& pb, const cd* d_psi, int stage, int reps, hipEvent_t e0, hipEvent_t e1) {
  PFM_DISPATCH(stage_timed_impl, pb, d_psi, stage, reps, e0, e1)
}
hipError_t apply_operator_mixed(Problem& pb, const cd* d_psi, cd* d_y) {
  PFM_DISPATCH(apply_mixed_impl, pb, d_psi, d_y)
}
hipError_t apply_operator_batch(Problem& pb, const cd* d_psi, cd* d_y, hipEvent_t* ev) {
  PFM_DISPATCH(apply_batch_impl, pb, d_psi, d_y, ev)
}

// ===========================================================================
// GMRES building blocks
// ===========================================================================
constexpr int RED_THREADS = 256;

constexpr int DOT_PER_LANE = 4;                 // w elements a lane keeps in registers
constexpr int DOT_CHUNK = 64 * DOT_PER_LANE;      // elements of one block's chunk

// blocks of the dot kernels along a vector of n elements (one chunk each up
// to 512 blocks)
int reduction_blocks(long long n) { return (int)std::min<long long>(512, (n + DOT_CHUNK - 1) / DOT_CHUNK); }

constexpr int DOT_VPW = 1;                      // vectors a wave reduces at once
constexpr int DOT_VPB = DOT_VPW * (RED_THREADS / 64);   // vectors per block

// partial[(z * cnt + i) * gridDim.x + blockIdx.x] = sum over the chunks of
// blockIdx.x of conj(V_i) w, for the vectors i of blockIdx.y and the batch
// member z = blockIdx.z (V and w advanced by vsb and wsb per member).  A
// chunk of w sits in registers (8 values per lane); each wave takes two
// vectors, keeps their 16 loads per lane in flight together and reduces with
// cross-lane sums, so there is no barrier.  The vector groups on the y axis
// keep enough waves resident to cover memory latency.
__global__ void __launch_bounds__(RED_THREADS) k_dots(const cd* __restrict__ V, long long ldv, long long vsb,
                                                      int cnt, const cd* __restrict__ w, long long wsb, int n,
                                                      cd* partial) {
  const int nblk = gridDim.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i0 = blockIdx.y * DOT_VPB + wv * DOT_VPW;
  if (i0 >= cnt) return;
  V += blockIdx.z * vsb;
  w += blockIdx.z * wsb;
  partial += (size_t)blockIdx.z * cnt * nblk;
  for (int c0 = blockIdx.x * DOT_CHUNK; c0 < n; c0 += nblk * DOT_CHUNK) {
    cd wr[DOT_PER_LANE];
#pragma unroll
    for (int s = 0; s < DOT_PER_LANE; ++s) {
      int t = c0 + lane + 64 * s;
      wr[s] = t < n ? w[t] : mkc(0, 0);
    }
    const bool first = c0 == blockIdx.x * DOT_CHUNK;
    cd acc[DOT_VPW];
#pragma unroll
    for (int u = 0; u < DOT_VPW; ++u) {
      acc[u] = mkc(0, 0);
      const int i = min(i0 + u, cnt - 1);
      const cd* v = V + (size_t)i * ldv + c0 + lane;
#pragma unroll
      for (int s = 0; s < DOT_PER_LANE; ++s)
        if (c0 + lane + 64 * s < n) acc[u] = cfma_conj(v[64 * s], wr[s], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < DOT_VPW; ++u) {
      cd r = wave_sum(acc[u]);
      if (lane == 0 && i0 + u < cnt) {
        cd* dst = partial + (size_t)(i0 + u) * nblk + blockIdx.x;
        *dst = first ? r : cadd(*dst, r);
      }
    }
  }
}

__global__ void __launch_bounds__(RED_THREADS) k_dots_final(const cd* partial, int nblk, int cnt, cd* out,
                                                            long long osb) {
  __shared__ cd s[RED_THREADS];
  int i = blockIdx.x;
  partial += (size_t)blockIdx.y * cnt * nblk;
  out += blockIdx.y * osb;
  cd acc = mkc(0, 0);
  for (int b = threadIdx.x; b < nblk; b += RED_THREADS) acc = cadd(acc, partial[(size_t)i * nblk + b]);
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int st = RED_THREADS / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) s[threadIdx.x] = cadd(s[threadIdx.x], s[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = s[0];
}

hipError_t launch_dots_b(Problem& pb, int B, const cd* V, long long ldv, long long vsb, int cnt, const cd* w,
                         long long wsb, int n, cd* d_out, long long osb) {
  int nblk = pb.red_blocks;
  dim3 grid(nblk, (cnt + DOT_VPB - 1) / DOT_VPB, B);
  hipLaunchKernelGGL(k_dots, grid, dim3(RED_THREADS), 0, pb.stream, V, ldv, vsb, cnt, w, wsb, n, pb.d_red);
  hipLaunchKernelGGL(k_dots_final, dim3(cnt, B), dim3(RED_THREADS), 0, pb.stream, pb.d_red, nblk, cnt, d_out,
                     osb);
  return hipGetLastError();
}

hipError_t launch_dots(Problem& pb, const cd* V, long long ldv, int cnt, const cd* w, int n, cd* d_out) {
  return launch_dots_b(pb, 1, V, ldv, 0, cnt, w, 0, n, d_out, 0);
}

// w -= sum_i h_i V_i   (member blockIdx.y: w, V, h advanced by their strides)
__global__ void k_update(cd* w, long long wsb, const cd* __restrict__ V, long long ldv, long long vsb, int cnt,
                         const cd* __restrict__ hcoef, long long hsb, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  w += blockIdx.y * wsb;
  V += blockIdx.y * vsb;
  hcoef += blockIdx.y * hsb;
  cd acc = w[t];
#pragma unroll 8
  for (int i = 0; i < cnt; ++i) {
    cd hv = hcoef[i];
    acc = csub(acc, cmul(hv, V[(size_t)i * ldv + t]));
  }
  w[t] = acc;
}

hipError_t launch_update_b(Problem& pb, int B, cd* w, long long wsb, const cd* V, long long ldv, long long vsb,
                           int cnt, const cd* d_h, long long hsb, int n) {
  hipLaunchKernelGGL(k_update, dim3((n + 255) / 256, B), dim3(256), 0, pb.stream, w, wsb, V, ldv, vsb, cnt, d_h,
                     hsb, n);
  return hipGetLastError();
}

hipError_t launch_update(Problem& pb, cd* w, const cd* V, long long ldv, int cnt, const cd* d_h, int n) {
  return launch_update_b(pb, 1, w, 0, V, ldv, 0, cnt, d_h, 0, n);
}

// x += sum_i c_i V_i   (member blockIdx.y)
__global__ void k_gemv_acc(cd* x, long long xsb, const cd* __restrict__ V, long long ldv, long long vsb, int cnt,
                           const cd* __restrict__ c, long long csb, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  x += blockIdx.y * xsb;
  V += blockIdx.y * vsb;
  c += blockIdx.y * csb;
  cd acc = x[t];
#pragma unroll 8
  for (int i = 0; i < cnt; ++i) acc = cfma(c[i], V[(size_t)i * ldv + t], acc);
  x[t] = acc;
}

hipError_t launch_gemv_acc_b(Problem& pb, int B, cd* x, long long xsb, const cd* V, long long ldv, long long vsb,
                             int cnt, const cd* d_c, long long csb, int n) {
  hipLaunchKernelGGL(k_gemv_acc, dim3((n + 255) / 256, B), dim3(256), 0, pb.stream, x, xsb, V, ldv, vsb, cnt,
                     d_c, csb, n);
  return hipGetLastError();
}

hipError_t launch_gemv_acc(Problem& pb, cd* x, const cd* V, long long ldv, int cnt, const cd* d_c, int n) {
  return launch_gemv_acc_b(pb, 1, x, 0, V, ldv, 0, cnt, d_c, 0, n);
}

__global__ void k_axpby(cd* y, cd a, const cd* __restrict__ x, cd b, long long n) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  cd yv = b.x == 0.0 && b.y == 0.0 ? mkc(0, 0) : cmul(b, y[t]);
  y[t] = x ? cfma(a, x[t], yv) : yv;
}

hipError_t launch_axpby(Problem& pb, cd* y, cd a, const cd* x, cd b, long long n) {
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, pb.stream, y, a, x, b, n);
  return hipGetLastError();
}

// out_b = in_b / sqrt(Re nrm[b * nsb]) for every member whose squared norm is
// positive; members with a zero norm get a zero vector.
__global__ void k_normalize_b(cd* out, const cd* __restrict__ in, long long sb, const cd* __restrict__ nrm,
                              long long nsb, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double q = nrm[blockIdx.y * nsb].x;
  double s = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  out[blockIdx.y * sb + t] = cscale(in[blockIdx.y * sb + t], s);
}

hipError_t launch_normalize_b(Problem& pb, int B, cd* out, const cd* in, long long sb, const cd* d_nrm,
                              long long nsb, int n) {
  hipLaunchKernelGGL(k_normalize_b, dim3((n + 255) / 256, B), dim3(256), 0, pb.stream, out, in, sb, d_nrm, nsb,
                     n);
  return hipGetLastError();
}

// ---- fused Arnoldi steps (the coefficient reductions are redone per block) ----

// w_b -= V_b h_b with h_b[i] = sum over the nblk dot partials of member b
// (partial[(b * cnt + i) * nblk + blk]); block 0 of each member stores h_b at
// hout + b * hsb.  With npart != nullptr every block also writes the squared
// norm of its updated chunk to npart[b * gridDim.x + blockIdx.x].
__global__ void __launch_bounds__(256) k_update_fused(cd* w, long long wsb, const cd* __restrict__ V, long long ldv,
                                                      long long vsb, int cnt, const cd* __restrict__ partial,
                                                      int nblk, cd* hout, long long hsb, int n, double* npart) {
  __shared__ cd sh[256];
  __shared__ double sn[256];
  const int b = blockIdx.y;
  const cd* pb_ = partial + (size_t)b * cnt * nblk;
  w += b * wsb;
  V += b * vsb;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  cd acc = t < n ? w[t] : mkc(0, 0);
  for (int i0 = 0; i0 < cnt; i0 += 256) {
    int c = min(256, cnt - i0);
    if ((int)threadIdx.x < c) {
      int i = i0 + threadIdx.x;
      cd hv = mkc(0, 0);
      for (int k = 0; k < nblk; ++k) hv = cadd(hv, pb_[(size_t)i * nblk + k]);
      sh[threadIdx.x] = hv;
      if (blockIdx.x == 0) hout[b * hsb + i] = hv;
    }
    __syncthreads();
    if (t < n) {
#pragma unroll 8
      for (int i = 0; i < c; ++i) acc = csub(acc, cmul(sh[i], V[(size_t)(i0 + i) * ldv + t]));
    }
    __syncthreads();
  }
  if (t < n) w[t] = acc;
  if (npart) {
    sn[threadIdx.x] = t < n ? cabs2(acc) : 0.0;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) sn[threadIdx.x] += sn[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) npart[(size_t)b * gridDim.x + blockIdx.x] = sn[0];
  }
}

// out_b = w_b / ||w_b|| with ||w_b||^2 the fixed-order sum of the np block
// partials of member b (npart[b * np + k]); block 0 stores ||w_b||^2 at
// nout + b * nsb (as a complex number with zero imaginary part).
__global__ void __launch_bounds__(256) k_normalize_fused(cd* w, long long wsb, const double* __restrict__ npart,
                                                         int np, cd* nout, long long nsb, int n) {
  __shared__ double sn[256];
  const int b = blockIdx.y;
  double q = 0.0;
  for (int k = threadIdx.x; k < np; k += 256) q += npart[(size_t)b * np + k];
  sn[threadIdx.x] = q;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sn[threadIdx.x] += sn[threadIdx.x + st];
    __syncthreads();
  }
  q = sn[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) nout[b * nsb] = mkc(q, 0.0);
  double s = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) w[b * wsb + t] = cscale(w[b * wsb + t], s);
}

// One CGS2 Arnoldi step for B members after W_b = A V_{j,b}:
// h1 = V^H W; W -= V h1; h2 = V^H W; W -= V h2; W /= ||W||.
// Column j of every member is stored at hcol + b * hsb: h1 in [0, j],
// h2 in [j+1, 2j+1], ||W||^2 in [2j+2].
// ---- Arnoldi with delayed reorthogonalisation (DCGS2: Bielich, Langou,
// Thomas, Swirydowicz, Yamazaki & Boman 2022) ----
// Step j holds v_0..v_{j-1} final and u_j (slot j) orthogonalised once (not
// normalised); w = Op u_j is in slot j+1.  One reduction gives
// a = V_{j-1}^H u_j, d = u_j^H u_j, b = V_{j-1}^H w, c = u_j^H w.  Then
//   gamma = sqrt(d - |a|^2),  v_j = (u_j - V_{j-1} a) / gamma      (second pass of step j-1)
//   s = v_j^H w = (c - a^H b) / gamma
//   w1 = (w - V_{j-1} b - s v_j) / gamma,  u_{j+1} = w1
// so every step reads the basis twice (one reduction, one update) instead of
// four times.  u_{j+1} is left unnormalised: the next step's gamma divides
// its norm out (scaling u_j by nu scales a, b, s, gamma and w by nu, and v_j
// and w1 not at all).  The Hessenberg column needs g = H[0..j][0..j-1] a (the
// Arnoldi relation applied to V_{j-1} a): h = ((b, s) - g) / gamma plus the
// next step's a, and the subdiagonal is the next step's gamma (w1 =
// gamma' v_{j+1} + V_j a').  That small dense algebra is left to the host,
// which reads per step j the raw column [a (j) | b (j) | s | gamma] from d_hall.

// partial[member][v * cnt + i][block] = V_i^H x_v over the block's chunks, x_0 = V_{cnt-1}
// (u_j), x_1 = w (NV = 2) or only x_0 (NV = 1)
template <int NV>
__global__ void __launch_bounds__(RED_THREADS) k_dots2(const cd* __restrict__ V, long long ldv, long long vsb,
                                                       int cnt, const cd* __restrict__ w, long long wsb, int n,
                                                       cd* partial) {
  const int nblk = gridDim.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i0 = blockIdx.y * DOT_VPB + wv * DOT_VPW;
  if (i0 >= cnt) return;
  V += blockIdx.z * vsb;
  w += blockIdx.z * wsb;
  partial += (size_t)blockIdx.z * NV * cnt * nblk;
  const cd* u = V + (size_t)(cnt - 1) * ldv;
  for (int c0 = blockIdx.x * DOT_CHUNK; c0 < n; c0 += nblk * DOT_CHUNK) {
    cd xr[NV][DOT_PER_LANE];
#pragma unroll
    for (int s = 0; s < DOT_PER_LANE; ++s) {
      int t = c0 + lane + 64 * s;
      xr[0][s] = t < n ? u[t] : mkc(0, 0);
      if (NV == 2) xr[NV - 1][s] = t < n ? w[t] : mkc(0, 0);
    }
    const bool first = c0 == blockIdx.x * DOT_CHUNK;
    cd acc[DOT_VPW][NV];
#pragma unroll
    for (int q = 0; q < DOT_VPW; ++q) {
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[q][v] = mkc(0, 0);
      const int i = min(i0 + q, cnt - 1);
      const cd* vi = V + (size_t)i * ldv + c0 + lane;
#pragma unroll
      for (int s = 0; s < DOT_PER_LANE; ++s)
        if (c0 + lane + 64 * s < n) {
          const cd a = vi[64 * s];
#pragma unroll
          for (int v = 0; v < NV; ++v) acc[q][v] = cfma_conj(a, xr[v][s], acc[q][v]);
        }
    }
#pragma unroll
    for (int q = 0; q < DOT_VPW; ++q)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        cd r = wave_sum(acc[q][v]);
        if (lane == 0 && i0 + q < cnt) {
          cd* dst = partial + ((size_t)v * cnt + i0 + q) * nblk + blockIdx.x;
          *dst = first ? r : cadd(*dst, r);
        }
      }
  }
}

// One block per member, from the reduced dots fin[member][NV cnt]: gamma, s,
// the update coefficients (coef: [0, j) a/gamma, [j, 2j) b/gamma, 2j s/gamma,
// 2j+1 1/gamma) and the raw column j of d_hall (slots [0, j) a, [j, 2j) b,
// 2j s, 2j+1 gamma).  NV = 1 (end of a cycle, x_0 = u_j): a and gamma only.
// gamma, s and the update coefficients of one member from its reduced dots
// fin (coef: [0, j) a/gamma, [j, 2j) b/gamma, 2j s/gamma, 2j+1 1/gamma) and,
// when hcol is given, the raw column j of d_hall (slots [0, j) a, [j, 2j) b,
// 2j s, 2j+1 gamma), by the 256 threads of the calling workgroup.  NV = 1
// (end of a cycle, x_0 = u_j): a and gamma only.
__device__ __forceinline__ void dcgs_coefficients(const cd* __restrict__ fin, int j, int NV, cd* hcol, cd* coef,
                                                  double* s_a2, cd* s_ab) {
  const int cnt = j + 1;
  double q2 = 0.0;
  cd ab = mkc(0, 0);
  for (int i = threadIdx.x; i < j; i += 256) {
    q2 += cabs2(fin[i]);
    if (NV == 2) ab = cfma_conj(fin[i], fin[cnt + i], ab);
  }
  s_a2[threadIdx.x] = q2;
  s_ab[threadIdx.x] = ab;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      s_a2[threadIdx.x] += s_a2[threadIdx.x + st];
      s_ab[threadIdx.x] = cadd(s_ab[threadIdx.x], s_ab[threadIdx.x + st]);
    }
    __syncthreads();
  }
  const double g2 = fin[j].x - s_a2[0];
  const double gamma = sqrt(g2 > 1e-300 ? g2 : 1e-300);
  const double ig = 1.0 / gamma;
  for (int i = threadIdx.x; i < j; i += 256) {
    coef[i] = cscale(fin[i], ig);
    if (hcol) hcol[i] = fin[i];
    if (NV == 2) {
      coef[j + i] = cscale(fin[cnt + i], ig);
      if (hcol) hcol[j + i] = fin[cnt + i];
    }
  }
  if (threadIdx.x == 0) {
    if (hcol) hcol[2 * j + 1] = mkc(gamma, 0.0);
    if (NV == 2) {
      const cd sv = cscale(csub(fin[cnt + j], s_ab[0]), ig);
      if (hcol) hcol[2 * j] = sv;
      coef[2 * j] = cscale(sv, ig);
      coef[2 * j + 1] = mkc(ig, 0.0);
    }
  }
}

// One block per member, from the reduced dots fin[member][NV cnt]: the
// coefficients into coef and the raw column into d_hall (the end of a cycle).
__global__ void __launch_bounds__(256) k_dcgs_coeff(const cd* __restrict__ fin, int j, int NV, cd* hcol,
                                                    long long hsb, cd* coef, long long csb) {
  __shared__ double s_a2[256];
  __shared__ cd s_ab[256];
  const int b = blockIdx.x;
  dcgs_coefficients(fin + (size_t)b * NV * (j + 1), j, NV, hcol + b * hsb, coef + b * csb, s_a2, s_ab);
}

// v_j = u_j / gamma - V_{j-1} (a / gamma) into slot j; w = w / gamma - V_{j-1} (b / gamma)
// - (s / gamma) v_j.  Every workgroup first forms the coefficients from the
// reduced dots fin[member][2 cnt] in LDS (dcgs_coefficients; workgroup 0
// also writes the raw column j of d_hall), which spares a launch.  A
// workgroup covers 64 elements; its four wavefronts take the basis vectors
// i = wv, wv + 4, ... (four times the loads in flight of one wavefront per
// element block), and their partial sums are added in wavefront order.
constexpr int UPD_ELEMS = 64;
__global__ void __launch_bounds__(256) k_dcgs_update(cd* V, long long ldv, long long vsb, int j, cd* w,
                                                     long long wsb, const cd* __restrict__ fin, cd* hcol,
                                                     long long hsb, int n) {
  __shared__ cd pv[4][UPD_ELEMS], pw[4][UPD_ELEMS];
  __shared__ cd coef[2 * 200 + 2];
  __shared__ double s_a2[256];
  __shared__ cd s_ab[256];
  const int b = blockIdx.y;
  V += b * vsb;
  w += b * wsb;
  dcgs_coefficients(fin + (size_t)b * 2 * (j + 1), j, 2, blockIdx.x == 0 ? hcol + b * hsb : nullptr, coef, s_a2,
                    s_ab);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int t = blockIdx.x * UPD_ELEMS + lane;
  const bool in = t < n;
  cd dv = mkc(0, 0), dw = mkc(0, 0);
  if (in) {
    const cd* vp = V + t;
#pragma unroll 4
    for (int i = wv; i < j; i += 4) {
      const cd vi = vp[(size_t)i * ldv];
      dv = cfma(coef[i], vi, dv);
      dw = cfma(coef[j + i], vi, dw);
    }
  }
  pv[wv][lane] = dv;
  pw[wv][lane] = dw;
  __syncthreads();
  if (wv != 0) return;
  const double ig = coef[2 * j + 1].x;
  const cd sv = cadd(cadd(pv[0][lane], pv[1][lane]), cadd(pv[2][lane], pv[3][lane]));
  const cd sw = cadd(cadd(pw[0][lane], pw[1][lane]), cadd(pw[2][lane], pw[3][lane]));
  if (in) {
    const cd vj = csub(cscale(V[(size_t)j * ldv + t], ig), sv);
    const cd wa = csub(csub(cscale(w[t], ig), sw), cmul(coef[2 * j], vj));
    V[(size_t)j * ldv + t] = vj;
    w[t] = wa;
  }
}

hipError_t launch_dcgs_step(Problem& pb, int B, cd* V, long long ldv, long long vsb, int j, cd* W, long long wsb,
                            int n, long long hsb) {
  const int cnt = j + 1;
  const int nblk = pb.red_blocks;
  const long long hcs = (long long)B * hsb;                 // column stride in d_hall
  cd* fin = pb.d_red + (size_t)B * 2 * cnt * nblk;          // [B][2 cnt] reduced dots
  hipLaunchKernelGGL(k_dots2<2>, dim3(nblk, (cnt + DOT_VPB - 1) / DOT_VPB, B), dim3(RED_THREADS), 0, pb.stream,
                     V, ldv, vsb, cnt, W, wsb, n, pb.d_red);
  hipLaunchKernelGGL(k_dots_final, dim3(2 * cnt, B), dim3(RED_THREADS), 0, pb.stream, pb.d_red, nblk, 2 * cnt, fin,
                     2LL * cnt);
  const int nup = (n + UPD_ELEMS - 1) / UPD_ELEMS;
  hipLaunchKernelGGL(k_dcgs_update, dim3(nup, B), dim3(256), 0, pb.stream, V, ldv, vsb, j, W, wsb, fin,
                     pb.d_hall + (size_t)j * hcs, hsb, n);
  return hipGetLastError();
}

// End of a cycle after step jl: the reorthogonalisation coefficients a and
// gamma of u_{jl+1} (slot jl + 1) into raw column jl + 1 of d_hall.
hipError_t launch_dcgs_finish(Problem& pb, int B, cd* V, long long ldv, long long vsb, int jl, int n,
                              long long hsb) {
  const int j = jl + 1, cnt = j + 1;
  const int nblk = pb.red_blocks;
  const long long hcs = (long long)B * hsb;
  cd* fin = pb.d_red + (size_t)B * cnt * nblk;
  hipLaunchKernelGGL(k_dots2<1>, dim3(nblk, (cnt + DOT_VPB - 1) / DOT_VPB, B), dim3(RED_THREADS), 0, pb.stream,
                     V, ldv, vsb, cnt, (const cd*)V, vsb, n, pb.d_red);
  hipLaunchKernelGGL(k_dots_final, dim3(cnt, B), dim3(RED_THREADS), 0, pb.stream, pb.d_red, nblk, cnt, fin,
                     (long long)cnt);
  hipLaunchKernelGGL(k_dcgs_coeff, dim3(B), dim3(256), 0, pb.stream, fin, j, 1, pb.d_hall + (size_t)j * hcs, hsb,
                     pb.d_dcoef, 2LL * pb.opt.restart + 4);
  return hipGetLastError();
}

hipError_t launch_arnoldi_step(Problem& pb, int B, const cd* V, long long ldv, long long vsb, int j, cd* W,
                               long long wsb, int n, cd* hcol, long long hsb) {
  const int cnt = j + 1;
  const int nblk = pb.red_blocks;
  const int nu = (n + 255) / 256;
  dim3 gd(nblk, (cnt + DOT_VPB - 1) / DOT_VPB, B), gu(nu, B);
  // Few dot partials per coefficient (short vectors): every update block sums
  // them itself.  Many (long vectors): one extra launch reduces them first.
  const bool fused = nblk <= 32;
  cd* fin = pb.d_red + (size_t)B * cnt * nblk;     // [B][cnt] reduced coefficients
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_dots, gd, dim3(RED_THREADS), 0, pb.stream, V, ldv, vsb, cnt, W, wsb, n, pb.d_red);
    const cd* part = pb.d_red;
    int np = nblk;
    if (!fused) {
      hipLaunchKernelGGL(k_dots_final, dim3(cnt, B), dim3(RED_THREADS), 0, pb.stream, pb.d_red, nblk, cnt, fin,
                         (long long)cnt);
      part = fin;
      np = 1;
    }
    hipLaunchKernelGGL(k_update_fused, gu, dim3(256), 0, pb.stream, W, wsb, V, ldv, vsb, cnt, part, np,
                       hcol + pass * cnt, hsb, n, pass ? pb.d_npart : (double*)nullptr);
  }
  hipLaunchKernelGGL(k_normalize_fused, gu, dim3(256), 0, pb.stream, W, wsb, pb.d_npart, nu, hcol + 2 * cnt, hsb,
                     n);
  return hipGetLastError();
}

// out[b * osb] = (sum of the np partials of member b, 0)
__global__ void __launch_bounds__(256) k_sum_parts(const double* __restrict__ npart, int np, cd* out, long long osb) {
  __shared__ double sn[256];
  const int b = blockIdx.x;
  double q = 0.0;
  for (int k = threadIdx.x; k < np; k += 256) q += npart[(size_t)b * np + k];
  sn[threadIdx.x] = q;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sn[threadIdx.x] += sn[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b * osb] = mkc(sn[0], 0.0);
}

// For B members: g = v^H c; c -= g v; g stored at gout + b*hsb and ||c||^2
// at nout + b*hsb (v, c: member stride wsb).
hipError_t launch_project_out(Problem& pb, int B, const cd* v, cd* c, long long wsb, int n, cd* gout, cd* nout,
                              long long hsb) {
  const int nblk = pb.red_blocks;
  const int nu = (n + 255) / 256;
  dim3 gd(nblk, 1, B), gu(nu, B);
  hipLaunchKernelGGL(k_dots, gd, dim3(RED_THREADS), 0, pb.stream, v, wsb, wsb, 1, c, wsb, n, pb.d_red);
  const cd* part = pb.d_red;
  int np = nblk;
  if (nblk > 32) {
    cd* fin = pb.d_red + (size_t)B * nblk;
    hipLaunchKernelGGL(k_dots_final, dim3(1, B), dim3(RED_THREADS), 0, pb.stream, pb.d_red, nblk, 1, fin, 1LL);
    part = fin;
    np = 1;
  }
  hipLaunchKernelGGL(k_update_fused, gu, dim3(256), 0, pb.stream, c, wsb, v, wsb, wsb, 1, part, np, gout, hsb, n,
                     pb.d_npart);
  hipLaunchKernelGGL(k_sum_parts, dim3(B), dim3(256), 0, pb.stream, pb.d_npart, nu, nout, hsb);
  return hipGetLastError();
}

}  // namespace pfm
