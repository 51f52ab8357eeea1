// The periodic tree and its interaction lists built by GPU kernels (Sec. 3.1).
//
// The result is the plan of the host construction (pfm_plan.cpp) bit for
// bit, so that either may serve:
//  * keys: every element gets the quadrant digits q = (x >= cx) + 2 (y >= cy)
//    of its midpoint at levels 1..24 of its fibre's tree (the same halving of
//    the root square as the host), most significant first, followed by its
//    index in the fibre; each fibre's keys are sorted in LDS (bitonic);
//  * cells: a fibre's cells of level L are the runs of equal level-L digit
//    prefixes inside the cells of level L - 1 that hold more than leaf_max
//    elements; one workgroup per fibre walks the levels (a first pass counts
//    the cells of each (fibre, level), the host turns the counts into the
//    level-major numbering, a second pass writes the cells, the leaves and
//    the element order, natural order inside a leaf);
//  * leaf-to-ancestor offsets, fibre offsets and M2L translation vectors get
//    ids in order of first occurrence, as the host's hash does: the entries'
//    rounded keys are sorted (stable radix sorts), each run's first position
//    found, and the runs ranked by it;
//  * the dual traversal of every (target fibre, source fibre, image) triple
//    runs in one thread with an explicit stack (children in order, depth
//    first), twice: counting, then writing at scanned positions, so the
//    entries come out in the host's order; the lists are then made CSR by a
//    stable sort on the target.
// Floating point: the file is compiled without contraction of multiplies and
// adds, and square roots are correctly rounded, so every distance and
// comparison is the host's.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <numeric>

#include "pfm_internal.hpp"

namespace pfm {

namespace {

constexpr int TREE_LEVELS = 24;       // deepest level (cells there are not split)
constexpr int TREE_NMAX = 4096;       // elements per fibre sorted in LDS
constexpr int TREE_LCAP = 512;        // cells of one level of one fibre
constexpr int TREE_THREADS = 512;
constexpr int TREE_STACK = 160;       // pending pairs of one traversal

typedef unsigned long long u64;

__device__ __forceinline__ double dist2d(double dx, double dy) {
  return __dsqrt_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)));
}

// digit of level L (1..24) of a key
__device__ __forceinline__ int key_digit(u64 k, int L) { return (int)((k >> (16 + 2 * (TREE_LEVELS - L))) & 3); }

__global__ void __launch_bounds__(TREE_THREADS) k_tree_sort(int N, double a, const double* __restrict__ centres,
                                                           const double* __restrict__ mx,
                                                           const double* __restrict__ my, u64* __restrict__ skey) {
  __shared__ u64 k[TREE_NMAX];
  const int f = blockIdx.x;
  int np = 1;
  while (np < N) np <<= 1;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    u64 key = ~0ULL;
    if (i < N) {
      const size_t e = (size_t)f * N + i;
      const double x = mx[e], y = my[e];
      double cx = centres[2 * f], cy = centres[2 * f + 1], half = 0.5 * a;
      u64 d = 0;
      for (int L = 1; L <= TREE_LEVELS; ++L) {
        const int q = (x >= cx ? 1 : 0) + (y >= cy ? 2 : 0);
        d = (d << 2) | (u64)q;
        half = 0.5 * half;
        cx = cx + ((q & 1) ? half : -half);
        cy = cy + ((q & 2) ? half : -half);
      }
      key = (d << 16) | (u64)i;
    }
    k[i] = key;
  }
  __syncthreads();
  for (int size = 2; size <= np; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < np; i += blockDim.x) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = (i & size) == 0;
          const u64 a0 = k[i], a1 = k[j];
          if ((a0 > a1) == up) {
            k[i] = a1;
            k[j] = a0;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < N; i += blockDim.x) skey[(size_t)f * N + i] = k[i];
}

// Cells written by the second pass (structure of arrays, global cell ids).
struct TreeCells {
  double *cx, *cy, *half, *rho;
  int *level, *fiber, *parent, *first_child, *n_child, *ebeg, *eend, *leaf, *leaf_index;
  int* leaves;
  int* elem_of;
};

// exclusive scan of v over the workgroup (TREE_THREADS values); returns the
// total; buf holds TREE_THREADS ints
__device__ int block_exscan(int v, int* buf, int& total) {
  const int t = threadIdx.x;
  buf[t] = v;
  __syncthreads();
  for (int off = 1; off < TREE_THREADS; off <<= 1) {
    const int add = t >= off ? buf[t - off] : 0;
    __syncthreads();
    buf[t] += add;
    __syncthreads();
  }
  const int incl = buf[t];
  total = buf[TREE_THREADS - 1];
  __syncthreads();
  return incl - v;
}

// emit = 0: cnt[f][L] = cells, lcnt[f][L] = leaves of fibre f at level L.
// emit = 1: the cells at ids cell_off[L][f] + local index, leaves at
// leaf_off[L][f] + local leaf index, and the element order.
// err: 1 a level of a fibre has more than TREE_LCAP cells, 2 a leaf has more
// than 64 elements.
__global__ void __launch_bounds__(TREE_THREADS) k_tree_levels(int M, int N, int leaf_max, double a,
                                                             const double* __restrict__ centres,
                                                             const double* __restrict__ ends,
                                                             const u64* __restrict__ skey, int emit, int* cnt,
                                                             int* lcnt, const int* __restrict__ cell_off,
                                                             const int* __restrict__ leaf_off, TreeCells out,
                                                             int* err) {
  __shared__ u64 k[TREE_NMAX];
  __shared__ int lb[2][TREE_LCAP], le[2][TREE_LCAP], lp[2][TREE_LCAP];
  __shared__ int sbuf[TREE_THREADS];
  const int f = blockIdx.x, t = threadIdx.x;
  for (int i = t; i < N; i += blockDim.x) k[i] = skey[(size_t)f * N + i];
  if (t == 0) {
    lb[0][0] = 0;
    le[0][0] = N;
    lp[0][0] = -1;
  }
  __syncthreads();
  int n_cur = 1, cur = 0;
  for (int L = 0; L <= TREE_LEVELS && n_cur > 0; ++L) {
    const bool mine = t < n_cur;
    const int b = mine ? lb[cur][t] : 0, e = mine ? le[cur][t] : 0;
    const int count = e - b;
    const bool split = mine && count > leaf_max && L < TREE_LEVELS;
    int cb[5] = {b, b, b, b, e};       // child q: [cb[q], cb[q + 1])
    int nk = 0;
    if (split) {
      for (int q = 1; q < 4; ++q) {
        int lo = cb[q - 1], hi = e;          // first index with digit >= q
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (key_digit(k[mid], L + 1) < q) lo = mid + 1;
          else hi = mid;
        }
        cb[q] = lo;
      }
      for (int q = 0; q < 4; ++q) nk += cb[q + 1] > cb[q];
    }
    int n_next = 0, n_leaf = 0;
    const int pos = block_exscan(nk, sbuf, n_next);
    const int lpos = block_exscan(mine && !split ? 1 : 0, sbuf, n_leaf);
    if (!emit && t == 0) {
      cnt[(size_t)f * (TREE_LEVELS + 1) + L] = n_cur;
      lcnt[(size_t)f * (TREE_LEVELS + 1) + L] = n_leaf;
    }
    if (n_next > TREE_LCAP) {
      if (t == 0) atomicMax(err, 1);
      return;
    }
    if (mine && emit) {
      const int id = cell_off[(size_t)L * M + f] + t;
      // centre from the root by the digits of the cell's first key
      double cx = centres[2 * f], cy = centres[2 * f + 1], half = 0.5 * a;
      for (int l = 1; l <= L; ++l) {
        const int q = key_digit(k[b], l);
        half = 0.5 * half;
        cx = cx + ((q & 1) ? half : -half);
        cy = cy + ((q & 2) ? half : -half);
      }
      double rho = 0.0;
      for (int i = b; i < e; ++i) {
        const size_t en = (size_t)f * N + (int)(k[i] & 0xFFFF);
        for (int s = 0; s < 2; ++s) {
          const double dx = ends[4 * en + 2 * s] - cx, dy = ends[4 * en + 2 * s + 1] - cy;
          rho = fmax(rho, dist2d(dx, dy));
        }
      }
      out.cx[id] = cx;
      out.cy[id] = cy;
      out.half[id] = half;
      out.rho[id] = rho;
      out.level[id] = L;
      out.fiber[id] = f;
      out.parent[id] = lp[cur][t];
      out.n_child[id] = nk;
      out.first_child[id] = nk ? cell_off[(size_t)(L + 1) * M + f] + pos : -1;
      out.ebeg[id] = f * N + b;
      out.eend[id] = f * N + e;
      out.leaf[id] = split ? 0 : 1;
      if (!split) {
        const int li = leaf_off[(size_t)L * M + f] + lpos;
        out.leaf_index[id] = li;
        out.leaves[li] = id;
        if (count > 64) atomicMax(err, 2);
        // natural order inside the leaf
        for (int i = b; i < e; ++i) {
          const int ii = (int)(k[i] & 0xFFFF);
          int r = 0;
          for (int j = b; j < e; ++j) r += (int)(k[j] & 0xFFFF) < ii;
          out.elem_of[(size_t)f * N + b + r] = f * N + ii;
        }
      } else {
        out.leaf_index[id] = -1;
      }
    }
    if (split) {
      const int nxt = cur ^ 1;
      int w = pos;
      const int id = emit ? cell_off[(size_t)L * M + f] + t : -1;
      for (int q = 0; q < 4; ++q) {
        if (cb[q + 1] == cb[q]) continue;
        lb[nxt][w] = cb[q];
        le[nxt][w] = cb[q + 1];
        lp[nxt][w] = id;
        ++w;
      }
    }
    __syncthreads();
    n_cur = n_next;
    cur ^= 1;
  }
}

// per leaf: its ancestors (parent first) and the rounded offsets O_L - O_A
__global__ void k_tree_anc(int n_leaves, const int* __restrict__ leaves, const int* __restrict__ anc_ptr,
                           const int* __restrict__ parent, const double* __restrict__ cx,
                           const double* __restrict__ cy, double scale, int* __restrict__ anc,
                           long long* __restrict__ kx, long long* __restrict__ ky, double* __restrict__ dxy) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_leaves) return;
  const int c = leaves[l];
  int q = anc_ptr[l];
  for (int p = parent[c]; p >= 0; p = parent[p], ++q) {
    const double dx = cx[c] - cx[p], dy = cy[c] - cy[p];
    anc[q] = p;
    kx[q] = llround(dx * scale);
    ky[q] = llround(dy * scale);
    dxy[2 * q] = dx;
    dxy[2 * q + 1] = dy;
  }
}

// fibre pair (i, j) = (q / M, q % M): its offset c_i - c_j
__global__ void k_tree_roots(int M, const double* __restrict__ centres, double scale, long long* __restrict__ kx,
                             long long* __restrict__ ky, double* __restrict__ dxy) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)M * M) return;
  const int i = (int)(q / M), j = (int)(q % M);
  const double ox = centres[2 * i] - centres[2 * j], oy = centres[2 * i + 1] - centres[2 * j + 1];
  kx[q] = llround(ox * scale);
  ky[q] = llround(oy * scale);
  dxy[2 * q] = ox;
  dxy[2 * q + 1] = oy;
}

// explicit images of each distinct fibre offset: the m with
// 2 rho_max > mac |o - m H e_y|
__global__ void k_tree_mrange(int n_roff, const double* __restrict__ off, double rho_max, double mac, double H,
                              double R, int* __restrict__ mrange) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n_roff) return;
  const double ox = off[2 * id], oy = off[2 * id + 1];
  int mlo = 1, mhi = 0;
  const int mc = (int)floor(oy / H);
  const int span = (int)ceil(R / H) + 2;
  for (int m = mc - span; m <= mc + span; ++m) {
    const double d = dist2d(ox, oy - m * H);
    if (!(2.0 * rho_max <= mac * d)) {
      if (mlo > mhi) {
        mlo = m;
        mhi = m;
      }
      mlo = min(mlo, m);
      mhi = max(mhi, m);
    }
  }
  mrange[2 * id] = mlo;
  mrange[2 * id + 1] = mhi;
}

// per fibre pair: traversals it starts (its explicit images, the fibre's own
// image 0 left out when that block is applied by FFT), and the image range
__global__ void k_tree_pair_count(int M, const int* __restrict__ pair_off, const int* __restrict__ mrange,
                                  int self_fft, int* __restrict__ ntrip, int* __restrict__ mminmax) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)M * M) return;
  const int i = (int)(q / M), j = (int)(q % M);
  const int id = pair_off[q];
  const int mlo = mrange[2 * id], mhi = mrange[2 * id + 1];
  int n = mhi >= mlo ? mhi - mlo + 1 : 0;
  if (n > 0) {
    atomicMin(&mminmax[0], mlo);
    atomicMax(&mminmax[1], mhi);
    if (self_fft && i == j && mlo <= 0 && 0 <= mhi) --n;
  }
  ntrip[q] = n;
}

__global__ void k_tree_pair_expand(int M, const int* __restrict__ pair_off, const int* __restrict__ mrange,
                                   int self_fft, const int* __restrict__ tbase, int4* __restrict__ trip) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)M * M) return;
  const int i = (int)(q / M), j = (int)(q % M);
  const int id = pair_off[q];
  int w = tbase[q];
  for (int m = mrange[2 * id]; m <= mrange[2 * id + 1]; ++m) {
    if (self_fft && i == j && m == 0) continue;
    trip[w++] = make_int4(i, j, m, i == j && m == 0 ? 1 : 0);
  }
}

struct TravCells {
  const double *cx, *cy, *rho;
  const int *leaf, *first_child, *n_child, *leaf_index;
};

// The dual traversal of one triple (target root, source root, image m).
// pass 0: counts of M2L and near entries; pass 1: the entries at the bases.
__global__ void k_tree_trav(int n_trip, const int4* __restrict__ trip, int M, TravCells c, double mac, double H,
                            double scale, int pass, int* __restrict__ n_m2l, int* __restrict__ n_near,
                            const int* __restrict__ m2l_base, const int* __restrict__ near_base,
                            int4* __restrict__ m2l_e, long long* __restrict__ m2l_kx,
                            long long* __restrict__ m2l_ky, double* __restrict__ m2l_d,
                            int4* __restrict__ near_e, int* err) {
  const int tq = blockIdx.x * blockDim.x + threadIdx.x;
  if (tq >= n_trip) return;
  const int4 tr = trip[tq];
  const int m = tr.z;
  int sd[TREE_STACK], sc[TREE_STACK];
  int top = 0;
  sd[top] = tr.x;                       // roots are cells 0..M-1, root of fibre f is f
  sc[top] = tr.y;
  ++top;
  int nm = 0, nn = 0;
  int wm = pass ? m2l_base[tq] : 0, wn = pass ? near_base[tq] : 0;
  while (top > 0) {
    --top;
    const int D = sd[top], C = sc[top];
    const double dx = c.cx[D] - c.cx[C];
    const double dy = c.cy[D] - c.cy[C] - m * H;
    const double d = dist2d(dx, dy);
    if (c.rho[D] + c.rho[C] <= mac * d) {
      if (pass) {
        m2l_e[wm] = make_int4(D, C, m, tr.w);
        m2l_kx[wm] = llround(dx * scale);
        m2l_ky[wm] = llround(dy * scale);
        m2l_d[2 * wm] = dx;
        m2l_d[2 * wm + 1] = dy;
        ++wm;
      }
      ++nm;
      continue;
    }
    const bool dl = c.leaf[D] != 0, cl = c.leaf[C] != 0;
    if (dl && cl) {
      if (pass) near_e[wn++] = make_int4(c.leaf_index[D], C, m, 0);
      ++nn;
      continue;
    }
    const bool split_src = dl || (!cl && c.rho[C] >= c.rho[D]);
    const int P = split_src ? C : D;
    const int n = c.n_child[P], f0 = c.first_child[P];
    if (top + n > TREE_STACK) {
      atomicMax(err, 3);
      return;
    }
    for (int kk = n - 1; kk >= 0; --kk) {     // child 0 on top: visited first
      sd[top] = split_src ? D : f0 + kk;
      sc[top] = split_src ? f0 + kk : C;
      ++top;
    }
  }
  if (!pass) {
    n_m2l[tq] = nm;
    n_near[tq] = nn;
  }
}

__global__ void k_iota(int n, int* v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

// signed 64-bit keys as unsigned in the same order
__global__ void k_flip_gather(int n, const long long* __restrict__ src, const int* __restrict__ idx,
                              u64* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (u64)(idx ? src[idx[i]] : src[i]) ^ 0x8000000000000000ULL;
}

// run starts of the (kx, ky)-sorted entries
__global__ void k_run_starts(int n, const u64* __restrict__ kxs, const long long* __restrict__ ky,
                             const int* __restrict__ pos, int* __restrict__ start) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  start[s] = s == 0 || kxs[s] != kxs[s - 1] || ky[pos[s]] != ky[pos[s - 1]];
}

__global__ void k_run_first(int n, const int* __restrict__ start, const int* __restrict__ run_incl,
                            const int* __restrict__ pos, int* __restrict__ first_pos, int* __restrict__ run_id) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  if (start[s]) {
    first_pos[run_incl[s] - 1] = pos[s];
    run_id[run_incl[s] - 1] = run_incl[s] - 1;
  }
}

__global__ void k_run_rank(int nu, const int* __restrict__ run_sorted, int* __restrict__ id_of_run) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nu) id_of_run[run_sorted[r]] = r;
}

__global__ void k_run_scatter(int n, const int* __restrict__ run_incl, const int* __restrict__ pos,
                              const int* __restrict__ id_of_run, int* __restrict__ ids) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) ids[pos[s]] = id_of_run[run_incl[s] - 1];
}

__global__ void k_gather_xy(int nu, const int* __restrict__ first_sorted, const double* __restrict__ dxy,
                            double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nu) return;
  out[2 * r] = dxy[2 * (size_t)first_sorted[r]];
  out[2 * r + 1] = dxy[2 * (size_t)first_sorted[r] + 1];
}

__global__ void k_count_keys(int n, const int* __restrict__ key, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[key[i] + 1], 1);
}

__global__ void k_m2l_split(int n, const int4* __restrict__ e, int* __restrict__ tgt, int* __restrict__ interior) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  tgt[i] = e[i].x;
  interior[i] = e[i].w;
}

__global__ void k_near_tgt(int n, const int4* __restrict__ e, int* __restrict__ tgt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) tgt[i] = e[i].x;
}

// entries in CSR order (perm = emission indices sorted by target)
__global__ void k_m2l_csr(int n, const int* __restrict__ perm, const int4* __restrict__ e,
                          const int* __restrict__ off_id, int* __restrict__ src, int* __restrict__ off,
                          int* __restrict__ mm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int4 v = e[perm[i]];
  src[i] = v.y;
  off[i] = off_id[perm[i]];
  if (mm) mm[i] = v.z;
}

__global__ void k_near_csr(int n, const int* __restrict__ perm, const int4* __restrict__ e,
                           const int* __restrict__ leaves, const int* __restrict__ ebeg,
                           const int* __restrict__ eend, int* __restrict__ src, int* __restrict__ mm,
                           int* __restrict__ tgt, long long* __restrict__ size) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int4 v = e[perm[i]];
  src[i] = v.y;
  mm[i] = v.z;
  tgt[i] = v.x;
  const int D = leaves[v.x];
  size[i] = (long long)(eend[D] - ebeg[D]) * (eend[v.y] - ebeg[v.y]);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

// Device buffers of one build, freed together.
struct Scratch {
  std::vector<void*> ptrs;
  hipError_t err = hipSuccess;
  template <typename T>
  T* alloc(size_t n) {
    void* p = nullptr;
    if (err == hipSuccess) err = hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T));
    if (err == hipSuccess) ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

#define TCK(call)                                     \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) {                           \
      why = std::string(#call) + ": " + hipGetErrorString(e_); \
      return false;                                   \
    }                                                 \
  } while (0)

inline unsigned nblk(long long n, int t = 256) { return (unsigned)std::max(1LL, (n + t - 1) / t); }

struct Builder {
  Scratch& s;
  hipStream_t st;
  std::string& why;

  template <typename K, typename V>
  bool sort_pairs(const K* kin, K* kout, const V* vin, V* vout, int n, int end_bit) {
    if (n == 0) return true;
    size_t bytes = 0;
    TCK(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, kin, kout, vin, vout, n, 0, end_bit, st));
    void* tmp = s.alloc<unsigned char>(bytes);
    TCK(s.err);
    TCK(hipcub::DeviceRadixSort::SortPairs(tmp, bytes, kin, kout, vin, vout, n, 0, end_bit, st));
    return true;
  }
  template <typename T>
  bool exscan(const T* in, T* out, int n) {
    if (n == 0) return true;
    size_t bytes = 0;
    TCK(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, n, st));
    void* tmp = s.alloc<unsigned char>(bytes);
    TCK(s.err);
    TCK(hipcub::DeviceScan::ExclusiveSum(tmp, bytes, in, out, n, st));
    return true;
  }
  template <typename T>
  bool inscan(const T* in, T* out, int n) {
    if (n == 0) return true;
    size_t bytes = 0;
    TCK(hipcub::DeviceScan::InclusiveSum(nullptr, bytes, in, out, n, st));
    void* tmp = s.alloc<unsigned char>(bytes);
    TCK(s.err);
    TCK(hipcub::DeviceScan::InclusiveSum(tmp, bytes, in, out, n, st));
    return true;
  }
  template <typename T>
  bool download(std::vector<T>& h, const T* d, size_t n) {
    h.resize(n);
    if (n) TCK(hipMemcpyAsync(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost, st));
    return true;
  }
  bool sync() {
    TCK(hipStreamSynchronize(st));
    return true;
  }

  // ids in order of first occurrence of the keys (kx, ky) of n entries, and
  // the values dxy of each id's first entry
  bool unique_first(int n, const long long* kx, const long long* ky, const double* dxy, int* ids, int& nu,
                    double*& uxy) {
    nu = 0;
    uxy = nullptr;
    if (n == 0) return true;
    int* pos0 = s.alloc<int>(n);
    int* pos1 = s.alloc<int>(n);
    int* pos2 = s.alloc<int>(n);
    u64* ka = s.alloc<u64>(n);
    u64* kb = s.alloc<u64>(n);
    int* start = s.alloc<int>(n);
    int* run = s.alloc<int>(n);
    int* first = s.alloc<int>(n);
    int* rid = s.alloc<int>(n);
    int* first_s = s.alloc<int>(n);
    int* rid_s = s.alloc<int>(n);
    int* id_of_run = s.alloc<int>(n);
    TCK(s.err);
    hipLaunchKernelGGL(k_iota, dim3(nblk(n)), dim3(256), 0, st, n, pos0);
    hipLaunchKernelGGL(k_flip_gather, dim3(nblk(n)), dim3(256), 0, st, n, ky, (const int*)nullptr, ka);
    if (!sort_pairs(ka, kb, pos0, pos1, n, 64)) return false;
    hipLaunchKernelGGL(k_flip_gather, dim3(nblk(n)), dim3(256), 0, st, n, kx, pos1, ka);
    if (!sort_pairs(ka, kb, pos1, pos2, n, 64)) return false;
    hipLaunchKernelGGL(k_run_starts, dim3(nblk(n)), dim3(256), 0, st, n, kb, ky, pos2, start);
    if (!inscan(start, run, n)) return false;
    std::vector<int> last;
    if (!download(last, run + n - 1, 1) || !sync()) return false;
    nu = last[0];
    hipLaunchKernelGGL(k_run_first, dim3(nblk(n)), dim3(256), 0, st, n, start, run, pos2, first, rid);
    if (!sort_pairs(first, first_s, rid, rid_s, nu, 32)) return false;
    hipLaunchKernelGGL(k_run_rank, dim3(nblk(nu)), dim3(256), 0, st, nu, rid_s, id_of_run);
    hipLaunchKernelGGL(k_run_scatter, dim3(nblk(n)), dim3(256), 0, st, n, run, pos2, id_of_run, ids);
    uxy = s.alloc<double>(2 * (size_t)nu);
    TCK(s.err);
    hipLaunchKernelGGL(k_gather_xy, dim3(nblk(nu)), dim3(256), 0, st, nu, first_s, dxy, uxy);
    TCK(hipGetLastError());
    return true;
  }

  // stable CSR order of n entries by key in [0, n_key): perm and ptr
  bool csr(int n, const int* key, int n_key, int*& perm, int*& ptr) {
    perm = s.alloc<int>(n);
    ptr = s.alloc<int>(n_key + 1);
    int* cnt = s.alloc<int>(n_key + 1);
    int* idx = s.alloc<int>(n);
    int* ks = s.alloc<int>(n);
    TCK(s.err);
    TCK(hipMemsetAsync(cnt, 0, (n_key + 1) * sizeof(int), st));
    if (n > 0) {
      hipLaunchKernelGGL(k_iota, dim3(nblk(n)), dim3(256), 0, st, n, idx);
      int bits = 1;
      while ((1LL << bits) < n_key) ++bits;
      if (!sort_pairs(key, ks, idx, perm, n, bits)) return false;
      hipLaunchKernelGGL(k_count_keys, dim3(nblk(n)), dim3(256), 0, st, n, key, cnt);
    }
    if (!inscan(cnt, ptr, n_key + 1)) return false;
    TCK(hipGetLastError());
    return true;
  }
};

}  // namespace

bool build_device_plan(Problem& pb, const double* d_mx, const double* d_my, const double* d_ends,
                       std::string& why) {
  const int M = pb.M, N = pb.N;
  if (N > TREE_NMAX) {
    why = "more than " + std::to_string(TREE_NMAX) + " elements per fibre";
    return false;
  }
  HostPlan& hp = pb.hp;
  hp = HostPlan();
  Scratch s;
  hipStream_t st = pb.stream;
  Builder bd{s, st, why};
  const int NL = TREE_LEVELS + 1;
  double* d_centres = s.alloc<double>(2 * (size_t)M);
  u64* skey = s.alloc<u64>((size_t)M * N);
  int* cnt = s.alloc<int>((size_t)M * NL);
  int* lcnt = s.alloc<int>((size_t)M * NL);
  int* err = s.alloc<int>(1);
  TCK(s.err);
  TCK(hipMemcpyAsync(d_centres, pb.centres.data(), 2 * (size_t)M * sizeof(double), hipMemcpyHostToDevice, st));
  TCK(hipMemsetAsync(cnt, 0, (size_t)M * NL * sizeof(int), st));
  TCK(hipMemsetAsync(lcnt, 0, (size_t)M * NL * sizeof(int), st));
  TCK(hipMemsetAsync(err, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_tree_sort, dim3(M), dim3(TREE_THREADS), 0, st, N, pb.a, d_centres, d_mx, d_my, skey);
  TreeCells none{};
  hipLaunchKernelGGL(k_tree_levels, dim3(M), dim3(TREE_THREADS), 0, st, M, N, pb.opt.leaf_max, pb.a, d_centres,
                     d_ends, skey, 0, cnt, lcnt, (const int*)nullptr, (const int*)nullptr, none, err);
  TCK(hipGetLastError());
  std::vector<int> hc, hl, herr;
  if (!bd.download(hc, cnt, (size_t)M * NL) || !bd.download(hl, lcnt, (size_t)M * NL) ||
      !bd.download(herr, err, 1) || !bd.sync())
    return false;
  if (herr[0]) {
    why = "a level of a fibre's tree has more than " + std::to_string(TREE_LCAP) + " cells";
    return false;
  }
  // level-major numbering: level L holds fibre 0's cells, then fibre 1's, ...
  std::vector<int> cell_off((size_t)NL * M), leaf_off((size_t)NL * M);
  hp.level_beg.assign(1, 0);
  int nc = 0, nleaf = 0;
  for (int L = 0; L < NL; ++L) {
    int lev = 0;
    for (int f = 0; f < M; ++f) {
      cell_off[(size_t)L * M + f] = nc + lev;
      lev += hc[(size_t)f * NL + L];
    }
    if (lev == 0) break;
    nc += lev;
    hp.level_beg.push_back(nc);
  }
  for (int L = 0; L < NL; ++L)
    for (int f = 0; f < M; ++f) {
      leaf_off[(size_t)L * M + f] = nleaf;
      nleaf += hl[(size_t)f * NL + L];
    }
  hp.depth = (int)hp.level_beg.size() - 2;
  int* d_cell_off = s.alloc<int>(cell_off.size());
  int* d_leaf_off = s.alloc<int>(leaf_off.size());
  TreeCells tc;
  tc.cx = s.alloc<double>(nc);
  tc.cy = s.alloc<double>(nc);
  tc.half = s.alloc<double>(nc);
  tc.rho = s.alloc<double>(nc);
  tc.level = s.alloc<int>(nc);
  tc.fiber = s.alloc<int>(nc);
  tc.parent = s.alloc<int>(nc);
  tc.first_child = s.alloc<int>(nc);
  tc.n_child = s.alloc<int>(nc);
  tc.ebeg = s.alloc<int>(nc);
  tc.eend = s.alloc<int>(nc);
  tc.leaf = s.alloc<int>(nc);
  tc.leaf_index = s.alloc<int>(nc);
  tc.leaves = s.alloc<int>(nleaf);
  tc.elem_of = s.alloc<int>((size_t)M * N);
  TCK(s.err);
  TCK(hipMemcpyAsync(d_cell_off, cell_off.data(), cell_off.size() * sizeof(int), hipMemcpyHostToDevice, st));
  TCK(hipMemcpyAsync(d_leaf_off, leaf_off.data(), leaf_off.size() * sizeof(int), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_tree_levels, dim3(M), dim3(TREE_THREADS), 0, st, M, N, pb.opt.leaf_max, pb.a, d_centres,
                     d_ends, skey, 1, cnt, lcnt, d_cell_off, d_leaf_off, tc, err);
  TCK(hipGetLastError());

  // leaf-to-ancestor lists: each leaf's ancestors, parent first
  std::vector<int> h_level, h_leaves;
  if (!bd.download(h_leaves, tc.leaves, nleaf) || !bd.download(h_level, tc.level, nc) ||
      !bd.download(herr, err, 1) || !bd.sync())
    return false;
  if (herr[0]) {
    why = herr[0] == 2 ? "a leaf holds more than 64 elements" : "tree levels overflow";
    return false;
  }
  hp.leaves = h_leaves;
  hp.anc_ptr.assign(nleaf + 1, 0);
  for (int l = 0; l < nleaf; ++l) hp.anc_ptr[l + 1] = hp.anc_ptr[l] + h_level[hp.leaves[l]];
  const int n_anc = hp.anc_ptr[nleaf];
  const double scale = std::ldexp(1.0, 36) / pb.a;
  int* d_anc_ptr = s.alloc<int>(nleaf + 1);
  int* d_anc = s.alloc<int>(n_anc);
  long long* akx = s.alloc<long long>(n_anc);
  long long* aky = s.alloc<long long>(n_anc);
  double* adxy = s.alloc<double>(2 * (size_t)n_anc);
  int* d_anc_off = s.alloc<int>(n_anc);
  TCK(s.err);
  TCK(hipMemcpyAsync(d_anc_ptr, hp.anc_ptr.data(), (nleaf + 1) * sizeof(int), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_tree_anc, dim3(nblk(nleaf)), dim3(256), 0, st, nleaf, tc.leaves, d_anc_ptr, tc.parent, tc.cx,
                     tc.cy, scale, d_anc, akx, aky, adxy);
  TCK(hipGetLastError());
  int n_joff = 0;
  double* d_joff = nullptr;
  if (!bd.unique_first(n_anc, akx, aky, adxy, d_anc_off, n_joff, d_joff)) return false;
  // upward lists: per non-leaf cell (id order) the leaves below it, in leaf order
  int *up_perm = nullptr, *up_ptr_all = nullptr;
  if (!bd.csr(n_anc, d_anc, nc, up_perm, up_ptr_all)) return false;

  // fibre offsets and their explicit image ranges
  const long long MM = (long long)M * M;
  long long* rkx = s.alloc<long long>(MM);
  long long* rky = s.alloc<long long>(MM);
  double* rdxy = s.alloc<double>(2 * MM);
  int* d_pair_off = s.alloc<int>(MM);
  TCK(s.err);
  hipLaunchKernelGGL(k_tree_roots, dim3(nblk(MM)), dim3(256), 0, st, M, d_centres, scale, rkx, rky, rdxy);
  int n_roff = 0;
  double* d_roff = nullptr;
  if (!bd.unique_first((int)MM, rkx, rky, rdxy, d_pair_off, n_roff, d_roff)) return false;
  std::vector<double> h_rho;
  if (!bd.download(h_rho, tc.rho, M) || !bd.sync()) return false;
  double rho_max = 0.0;
  for (int f = 0; f < M; ++f) rho_max = std::max(rho_max, h_rho[f]);
  const double R = 2.0 * rho_max / pb.opt.mac;
  int* d_mrange = s.alloc<int>(2 * (size_t)n_roff);
  int* ntrip = s.alloc<int>(MM);
  int* tbase = s.alloc<int>(MM);
  int* mminmax = s.alloc<int>(2);
  TCK(s.err);
  hipLaunchKernelGGL(k_tree_mrange, dim3(nblk(n_roff)), dim3(256), 0, st, n_roff, d_roff, rho_max, pb.opt.mac,
                     pb.H, R, d_mrange);
  {
    const int init[2] = {0, 0};
    TCK(hipMemcpyAsync(mminmax, init, sizeof(init), hipMemcpyHostToDevice, st));
  }
  const int self_fft = pb.self_fft ? 1 : 0;
  hipLaunchKernelGGL(k_tree_pair_count, dim3(nblk(MM)), dim3(256), 0, st, M, d_pair_off, d_mrange, self_fft, ntrip,
                     mminmax);
  if (!bd.exscan(ntrip, tbase, (int)MM)) return false;
  std::vector<int> tl, tn, hmm;
  if (!bd.download(tl, tbase + MM - 1, 1) || !bd.download(tn, ntrip + MM - 1, 1) || !bd.download(hmm, mminmax, 2) ||
      !bd.sync())
    return false;
  const int n_trip = tl[0] + tn[0];
  hp.m_min = hmm[0];
  hp.m_max = hmm[1];
  int4* trip = s.alloc<int4>(n_trip);
  int* tm = s.alloc<int>(n_trip);
  int* tn2 = s.alloc<int>(n_trip);
  int* bm = s.alloc<int>(n_trip);
  int* bn = s.alloc<int>(n_trip);
  TCK(s.err);
  hipLaunchKernelGGL(k_tree_pair_expand, dim3(nblk(MM)), dim3(256), 0, st, M, d_pair_off, d_mrange, self_fft, tbase,
                     trip);
  TravCells tcv{tc.cx, tc.cy, tc.rho, tc.leaf, tc.first_child, tc.n_child, tc.leaf_index};
  hipLaunchKernelGGL(k_tree_trav, dim3(nblk(n_trip, 64)), dim3(64), 0, st, n_trip, trip, M, tcv, pb.opt.mac, pb.H,
                     scale, 0, tm, tn2, (const int*)nullptr, (const int*)nullptr, (int4*)nullptr,
                     (long long*)nullptr, (long long*)nullptr, (double*)nullptr, (int4*)nullptr, err);
  if (!bd.exscan(tm, bm, n_trip) || !bd.exscan(tn2, bn, n_trip)) return false;
  std::vector<int> v1, v2, v3, v4;
  if (!bd.download(v1, bm + n_trip - 1, n_trip ? 1 : 0) || !bd.download(v2, tm + n_trip - 1, n_trip ? 1 : 0) ||
      !bd.download(v3, bn + n_trip - 1, n_trip ? 1 : 0) || !bd.download(v4, tn2 + n_trip - 1, n_trip ? 1 : 0) ||
      !bd.download(herr, err, 1) || !bd.sync())
    return false;
  if (herr[0]) {
    why = "traversal stack overflow";
    return false;
  }
  const int n_m2l = n_trip ? v1[0] + v2[0] : 0, n_near = n_trip ? v3[0] + v4[0] : 0;
  int4* m2l_e = s.alloc<int4>(n_m2l);
  long long* mkx = s.alloc<long long>(n_m2l);
  long long* mky = s.alloc<long long>(n_m2l);
  double* mdxy = s.alloc<double>(2 * (size_t)n_m2l);
  int4* near_e = s.alloc<int4>(n_near);
  int* m_off = s.alloc<int>(n_m2l);
  TCK(s.err);
  hipLaunchKernelGGL(k_tree_trav, dim3(nblk(n_trip, 64)), dim3(64), 0, st, n_trip, trip, M, tcv, pb.opt.mac, pb.H,
                     scale, 1, tm, tn2, bm, bn, m2l_e, mkx, mky, mdxy, near_e, err);
  TCK(hipGetLastError());
  int n_off = 0;
  double* d_off = nullptr;
  if (!bd.unique_first(n_m2l, mkx, mky, mdxy, m_off, n_off, d_off)) return false;
  // M2L lists, CSR by target cell; the interior entries (same fibre, m = 0) apart
  int* m_tgt = s.alloc<int>(n_m2l);
  int* m_int = s.alloc<int>(n_m2l);
  int* m_src_c = s.alloc<int>(n_m2l);
  int* m_off_c = s.alloc<int>(n_m2l);
  int* m_m_c = s.alloc<int>(n_m2l);
  TCK(s.err);
  hipLaunchKernelGGL(k_m2l_split, dim3(nblk(n_m2l)), dim3(256), 0, st, n_m2l, m2l_e, m_tgt, m_int);
  int *m_perm = nullptr, *m_ptr = nullptr;
  if (!bd.csr(n_m2l, m_tgt, nc, m_perm, m_ptr)) return false;
  hipLaunchKernelGGL(k_m2l_csr, dim3(nblk(n_m2l)), dim3(256), 0, st, n_m2l, m_perm, m2l_e, m_off, m_src_c, m_off_c,
                     m_m_c);
  TCK(hipGetLastError());
  // interior subset, in emission order
  std::vector<int4> h_m2l_e;
  std::vector<int> h_m_off;
  if (!bd.download(h_m2l_e, m2l_e, n_m2l) || !bd.download(h_m_off, m_off, n_m2l) || !bd.sync()) return false;
  std::vector<int> int_idx;
  for (int q = 0; q < n_m2l; ++q)
    if (h_m2l_e[q].w) int_idx.push_back(q);
  const int n_int = (int)int_idx.size();
  int* i_tgt = s.alloc<int>(n_int);
  int4* i_e = s.alloc<int4>(n_int);
  int* i_off = s.alloc<int>(n_int);
  int* i_src_c = s.alloc<int>(n_int);
  int* i_off_c = s.alloc<int>(n_int);
  TCK(s.err);
  {
    std::vector<int> it(n_int), io(n_int);
    std::vector<int4> ie(n_int);
    for (int q = 0; q < n_int; ++q) {
      ie[q] = h_m2l_e[int_idx[q]];
      it[q] = ie[q].x;
      io[q] = h_m_off[int_idx[q]];
    }
    if (n_int) {
      TCK(hipMemcpyAsync(i_tgt, it.data(), n_int * sizeof(int), hipMemcpyHostToDevice, st));
      TCK(hipMemcpyAsync(i_e, ie.data(), n_int * sizeof(int4), hipMemcpyHostToDevice, st));
      TCK(hipMemcpyAsync(i_off, io.data(), n_int * sizeof(int), hipMemcpyHostToDevice, st));
    }
    int *i_perm = nullptr, *i_ptr = nullptr;
    if (!bd.csr(n_int, i_tgt, nc, i_perm, i_ptr)) return false;
    hipLaunchKernelGGL(k_m2l_csr, dim3(nblk(n_int)), dim3(256), 0, st, n_int, i_perm, i_e, i_off, i_src_c, i_off_c,
                       (int*)nullptr);
    TCK(hipGetLastError());
    if (!bd.download(hp.m2li_ptr, i_ptr, nc + 1) || !bd.download(hp.m2li_src, i_src_c, n_int) ||
        !bd.download(hp.m2li_off, i_off_c, n_int) || !bd.sync())
      return false;
  }
  // near lists, CSR by target leaf, with the block offsets
  int* n_tgt = s.alloc<int>(n_near);
  int* n_src_c = s.alloc<int>(n_near);
  int* n_m_c = s.alloc<int>(n_near);
  int* n_tgt_c = s.alloc<int>(n_near);
  long long* n_size = s.alloc<long long>(n_near);
  long long* n_blk = s.alloc<long long>(n_near);
  TCK(s.err);
  hipLaunchKernelGGL(k_near_tgt, dim3(nblk(n_near)), dim3(256), 0, st, n_near, near_e, n_tgt);
  int *n_perm = nullptr, *n_ptr = nullptr;
  if (!bd.csr(n_near, n_tgt, nleaf, n_perm, n_ptr)) return false;
  hipLaunchKernelGGL(k_near_csr, dim3(nblk(n_near)), dim3(256), 0, st, n_near, n_perm, near_e, tc.leaves, tc.ebeg,
                     tc.eend, n_src_c, n_m_c, n_tgt_c, n_size);
  if (!bd.exscan(n_size, n_blk, n_near)) return false;
  TCK(hipGetLastError());

  // everything back into the host plan
  std::vector<double> hcx, hcy, hhalf, hrho;
  std::vector<int> hfib, hpar, hfc, hnch, heb, hee, hleaf, hli;
  if (!bd.download(hcx, tc.cx, nc) || !bd.download(hcy, tc.cy, nc) || !bd.download(hhalf, tc.half, nc) ||
      !bd.download(hrho, tc.rho, nc) || !bd.download(hfib, tc.fiber, nc) || !bd.download(hpar, tc.parent, nc) ||
      !bd.download(hfc, tc.first_child, nc) || !bd.download(hnch, tc.n_child, nc) ||
      !bd.download(heb, tc.ebeg, nc) || !bd.download(hee, tc.eend, nc) || !bd.download(hleaf, tc.leaf, nc) ||
      !bd.download(hli, tc.leaf_index, nc) || !bd.download(hp.elem_of, tc.elem_of, (size_t)M * N) ||
      !bd.download(hp.anc, d_anc, n_anc) || !bd.download(hp.anc_off, d_anc_off, n_anc) ||
      !bd.download(hp.joff_xy, d_joff, 2 * (size_t)n_joff) || !bd.download(hp.root_off_xy, d_roff, 2 * (size_t)n_roff) ||
      !bd.download(hp.root_off_mrange, d_mrange, 2 * (size_t)n_roff) ||
      !bd.download(hp.root_pair_off, d_pair_off, MM) || !bd.download(hp.m2l_ptr, m_ptr, nc + 1) ||
      !bd.download(hp.m2l_src, m_src_c, n_m2l) || !bd.download(hp.m2l_off, m_off_c, n_m2l) ||
      !bd.download(hp.m2l_m, m_m_c, n_m2l) || !bd.download(hp.off_xy, d_off, 2 * (size_t)n_off) ||
      !bd.download(hp.near_ptr, n_ptr, nleaf + 1) || !bd.download(hp.near_src, n_src_c, n_near) ||
      !bd.download(hp.near_m, n_m_c, n_near) || !bd.download(hp.near_tgt, n_tgt_c, n_near) ||
      !bd.download(hp.near_blk, n_blk, n_near))
    return false;
  std::vector<int> up_perm_h, up_ptr_h;
  if (!bd.download(up_perm_h, up_perm, n_anc) || !bd.download(up_ptr_h, up_ptr_all, nc + 1) || !bd.sync())
    return false;
  hp.cells.assign(nc, Cell{});
  for (int i = 0; i < nc; ++i) {
    Cell& c = hp.cells[i];
    c.cx = hcx[i];
    c.cy = hcy[i];
    c.half = hhalf[i];
    c.rho = hrho[i];
    c.level = h_level[i];
    c.fiber = hfib[i];
    c.parent = hpar[i];
    c.first_child = hfc[i];
    c.n_child = hnch[i];
    c.ebeg = heb[i];
    c.eend = hee[i];
    c.leaf = hleaf[i];
    c.leaf_index = hli[i];
  }
  hp.root_of_fibre.resize(M);
  std::iota(hp.root_of_fibre.begin(), hp.root_of_fibre.end(), 0);
  // non-leaf cells in id order with the leaves below each (the CSR of the
  // ancestor entries by ancestor: leaf order inside, as the host pushes them)
  hp.up_cells.clear();
  hp.up_ptr.assign(1, 0);
  hp.up_src.clear();
  hp.up_off.clear();
  std::vector<int> anc_leaf(n_anc);
  for (int l = 0; l < nleaf; ++l)
    for (int q = hp.anc_ptr[l]; q < hp.anc_ptr[l + 1]; ++q) anc_leaf[q] = hp.leaves[l];
  for (int c = 0; c < nc; ++c) {
    if (hp.cells[c].leaf) continue;
    hp.up_cells.push_back(c);
    for (int q = up_ptr_h[c]; q < up_ptr_h[c + 1]; ++q) {
      hp.up_src.push_back(anc_leaf[up_perm_h[q]]);
      hp.up_off.push_back(hp.anc_off[up_perm_h[q]]);
    }
    hp.up_ptr.push_back((int)hp.up_src.size());
  }
  hp.n_near_entries = 0;
  if (n_near > 0) {
    const Cell& D = hp.cells[hp.leaves[hp.near_tgt[n_near - 1]]];
    const Cell& C = hp.cells[hp.near_src[n_near - 1]];
    hp.n_near_entries = hp.near_blk[n_near - 1] + (long long)(D.eend - D.ebeg) * (C.eend - C.ebeg);
  }
  return true;
}

}  // namespace pfm
