// Learned warm start: MLP forward/backward/Adam in FP32, BF16 inference on
// the matrix cores, features and per-fibre modal transforms of the densities.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "../../include/pfmwarm.h"
#include "pfm_internal.hpp"

namespace pfm {
namespace warm {

// ---------------------------------------------------------------------------
// FP32 GEMM  C[M x N] = op(A)[M x K] op(B)[K x N]  with a fused epilogue.
// op(A)[m][k] = TA ? A[k * lda + m] : A[m * lda + k]
// op(B)[k][n] = TB ? B[n * ldb + k] : B[k * ldb + n]
// 64 x 64 tiles, 16-deep K slices staged in LDS, 4 x 4 outputs per thread.
// ---------------------------------------------------------------------------
enum Epi { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_TANH = 2, EPI_DTANH = 3 };

constexpr int GB = 64, GK = 16;

template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const float* __restrict__ A, int lda,
                                              const float* __restrict__ B, int ldb, float* __restrict__ C,
                                              int ldc, int epi, const float* __restrict__ bias,
                                              const float* __restrict__ H) {
  __shared__ float As[GK][GB + 4], Bs[GK][GB + 4];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.y * GB, n0 = blockIdx.x * GB;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += GK) {
    // each thread loads 4 elements of each tile
    for (int r = 0; r < 4; ++r) {
      int idx = threadIdx.x + 256 * r;      // 0..1023 over a 64 x 16 tile
      int mm, kk;
      if (TA) { mm = idx & 63; kk = idx >> 6; } else { kk = idx & 15; mm = idx >> 4; }
      int gm = m0 + mm, gk = k0 + kk;
      float v = 0.f;
      if (gm < M && gk < K) v = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
      As[kk][mm] = v;
      int nn, kb;
      if (TB) { kb = idx & 15; nn = idx >> 4; } else { nn = idx & 63; kb = idx >> 6; }
      int gn = n0 + nn, gkb = k0 + kb;
      float u = 0.f;
      if (gn < N && gkb < K) u = TB ? B[(size_t)gn * ldb + gkb] : B[(size_t)gkb * ldb + gn];
      Bs[kb][nn] = u;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int gm = m0 + ty * 4 + i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int gn = n0 + tx * 4 + j;
      if (gn >= N) continue;
      float v = acc[i][j];
      if (epi == EPI_BIAS || epi == EPI_BIAS_TANH) v += bias[gn];
      if (epi == EPI_BIAS_TANH) v = tanhf(v);
      if (epi == EPI_DTANH) {
        float h = H[(size_t)gm * ldc + gn];
        v *= 1.f - h * h;
      }
      C[(size_t)gm * ldc + gn] = v;
    }
  }
}

static void gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B,
                 int ldb, float* C, int ldc, int epi, const float* bias, const float* H) {
  dim3 grid((N + GB - 1) / GB, (M + GB - 1) / GB);
  if (!ta && tb)
    hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, epi, bias, H);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, epi, bias, H);
  else if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, epi, bias, H);
  else
    hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, epi, bias, H);
}

// column sums of a row-major [rows x cols] matrix, fixed row order
__global__ void k_colsum(int rows, int cols, const float* __restrict__ X, float* __restrict__ out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += X[(size_t)r * cols + c];
  out[c] = s;
}

// d = 2 (y - t) / n, and per-block partial sums of (y - t)^2
__global__ void __launch_bounds__(256) k_mse(long long n, const float* __restrict__ y, const float* __restrict__ t,
                                             float* __restrict__ d, float* __restrict__ part) {
  __shared__ float sh[256];
  long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  float e = 0.f;
  if (i < n) {
    float r = y[i] - t[i];
    d[i] = 2.f * r / (float)n;
    e = r * r;
  }
  sh[threadIdx.x] = e;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_partials(int n, const float* __restrict__ part, float scale, float* out) {
  __shared__ float sh[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0] * scale;
}

__global__ void k_adam(long long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float bc1, float bc2) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// SplitMix64 (Steele, Lea & Flood 2014): state += golden gamma, then two
// xor-shift-multiply rounds; the top 53 bits give a uniform double in [0, 1).
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void k_init_uniform(long long n, float* __restrict__ p, float scale, unsigned long long seed,
                               long long offset) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double u = (double)(splitmix64(seed + (unsigned long long)(offset + i)) >> 11) * (1.0 / 9007199254740992.0);
  p[i] = (float)((2.0 * u - 1.0) * scale);
}

// FP32 -> bfloat16 bits, round to nearest even (NaN kept quiet)
__device__ __forceinline__ unsigned short f32_to_bf16(float f) {
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__global__ void k_to_bf16(long long n, const float* __restrict__ src, unsigned short* __restrict__ dst) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = f32_to_bf16(src[i]);
}

// BF16 layer on the matrix cores: Y[M x N] = act(X[M x K] W^T + b) with W
// [N x K] in bfloat16, X rounded to bfloat16 as it is loaded, FP32
// accumulation.  One wavefront per 16 x 16 output tile, v_mfma_f32_16x16x16
// bf16: lane l supplies A[l % 16][4 (l / 16) + 0..3] and B[4 (l / 16) + 0..3][l % 16]
// and receives D[4 (l / 16) + 0..3][l % 16].
typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_gemm_bf16(int M, int N, int K, const float* __restrict__ X,
                                                   const unsigned short* __restrict__ W, const float* __restrict__ bias,
                                                   int act, float* __restrict__ Y) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 16, n0 = (blockIdx.x * 4 + w) * 16;
  if (n0 >= N) return;                       // wave-uniform
  const int i = lane & 15, kg = lane >> 4;
  const int row = m0 + i, col = n0 + i;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    v4s a, b;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int k = k0 + 4 * kg + r;
      float xv = (row < M && k < K) ? X[(size_t)row * K + k] : 0.f;
      a[r] = (short)f32_to_bf16(xv);
      b[r] = (short)((col < N && k < K) ? W[(size_t)col * K + k] : 0);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  const int c = n0 + i;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int rr = m0 + 4 * kg + r;
    if (rr < M && c < N) {
      float v = acc[r] + bias[c];
      Y[(size_t)rr * N + c] = act ? tanhf(v) : v;
    }
  }
}

// last layer y_o -> scale_o y_o + shift_o: row o of W and b_o scaled, shift added
__global__ void k_scale_output(int outw, int in, float* __restrict__ W, float* __restrict__ b,
                               const float* __restrict__ scale, const float* __restrict__ shift) {
  int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= outw) return;
  float s = scale[o];
  for (int i = 0; i < in; ++i) W[(size_t)o * in + i] *= s;
  b[o] = b[o] * s + shift[o];
}

// features: 2 (d - lo) / (hi - lo) - 1
__global__ void k_features(int n, const double* __restrict__ d, float* __restrict__ x) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 5 * n) return;
  const double lo[5] = {0.2, 0.0, 0.15, 0.5, 0.5};
  const double hi[5] = {8.0, 1.5707963267948966, 0.4, 20.0, 2.0};
  int c = i % 5;
  x[i] = (float)(2.0 * (d[i] - lo[c]) / (hi[c] - lo[c]) - 1.0);
}

// ---------------------------------------------------------------------------
// modal transforms, one workgroup per (fibre, density, member)
// ---------------------------------------------------------------------------
constexpr int MODES_MAX_N = 1024;

__global__ void __launch_bounds__(256) k_modes_analyse(int M, int N, int K, double k, const double* __restrict__ th,
                                                       const double* __restrict__ centres,
                                                       const cd* __restrict__ psi, float* __restrict__ vec) {
  __shared__ cd tw[MODES_MAX_N];
  __shared__ cd row[MODES_MAX_N];
  const int fs = blockIdx.x, b = blockIdx.y, f = fs >> 1, s = fs & 1;
  const size_t n2 = 2 * (size_t)M * N;
  const cd* src = psi + b * n2 + (size_t)(2 * f + s) * N;
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    double sn, cs;
    sincospi(-2.0 * j / N, &sn, &cs);
    tw[j] = mkc(cs, sn);                 // e^{-2 pi i j / N}
    row[j] = src[j];
  }
  __syncthreads();
  double ph = k * (centres[2 * f] * cos(th[b]) + centres[2 * f + 1] * sin(th[b]));
  double ps, pc;
  sincos(-ph, &ps, &pc);
  cd rot = mkc(pc / N, ps / N);          // e^{-i k c.d} / N
  float* out = vec + (size_t)b * 4 * M * K + (size_t)fs * 2 * K;
  for (int q = threadIdx.x; q < K; q += blockDim.x) {
    int n = q - K / 2;
    int step = ((n % N) + N) % N;
    cd acc = mkc(0, 0);
    int idx = 0;
    for (int e = 0; e < N; ++e) {
      acc = cfma(row[e], tw[idx], acc);
      idx += step;
      if (idx >= N) idx -= N;
    }
    acc = cmul(acc, rot);
    out[2 * q] = (float)acc.x;
    out[2 * q + 1] = (float)acc.y;
  }
}

__global__ void __launch_bounds__(256) k_modes_synthesise(int M, int N, int K, double k, const double* __restrict__ th,
                                                          const double* __restrict__ centres,
                                                          const float* __restrict__ vec, cd* __restrict__ psi) {
  __shared__ cd tw[MODES_MAX_N];
  __shared__ cd cf[MODES_MAX_N];
  const int fs = blockIdx.x, b = blockIdx.y, f = fs >> 1;
  const size_t n2 = 2 * (size_t)M * N;
  const float* in = vec + (size_t)b * 4 * M * K + (size_t)fs * 2 * K;
  double ph = k * (centres[2 * f] * cos(th[b]) + centres[2 * f + 1] * sin(th[b]));
  double ps, pc;
  sincos(ph, &ps, &pc);
  cd rot = mkc(pc, ps);                  // e^{i k c.d}
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * j / N, &sn, &cs);
    tw[j] = mkc(cs, sn);                 // e^{2 pi i j / N}
  }
  for (int q = threadIdx.x; q < K; q += blockDim.x) cf[q] = cmul(rot, mkc(in[2 * q], in[2 * q + 1]));
  __syncthreads();
  cd* dst = psi + b * n2 + (size_t)fs * N;
  for (int e = threadIdx.x; e < N; e += blockDim.x) {
    cd acc = mkc(0, 0);
    for (int q = 0; q < K; ++q) {
      int n = q - K / 2;
      int idx = (int)(((long long)n * e % N + N) % N);
      acc = cfma(cf[q], tw[idx], acc);
    }
    dst[e] = acc;
  }
}

// Column statistics of training targets t [n][m] (row-major): mean and
// standard deviation with n - 1 in the denominator, at least `floor`; sums
// in FP64, one thread per column (coalesced across the columns of a row).
__global__ void k_col_stats(const float* __restrict__ t, int n, int m, float floor_, float* __restrict__ mean,
                            float* __restrict__ sd) {
  int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= m) return;
  double s = 0.0;
  for (int r = 0; r < n; ++r) s += (double)t[(size_t)r * m + o];
  const double mu = s / n;
  double v = 0.0;
  for (int r = 0; r < n; ++r) {
    const double d = (double)t[(size_t)r * m + o] - mu;
    v += d * d;
  }
  const double sdv = n > 1 ? sqrt(v / (n - 1)) : 0.0;
  mean[o] = (float)mu;
  sd[o] = (float)fmax(sdv, (double)floor_);
}

__global__ void k_standardise(const float* __restrict__ t, long long total, int m, const float* __restrict__ mean,
                              const float* __restrict__ sd, float* __restrict__ out) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int o = (int)(i % m);
  out[i] = (t[i] - mean[o]) / sd[o];
}

// Per output column o over n validation rows: s_o = clamp(1 - sum (y - t)^2 /
// sum t^2, 0, 1) (the share of the column's power the network predicts);
// and the column's sums sum (s_o y - t)^2, sum t^2 for the relative error
// after the shrink.
__global__ void k_val_shrink(const float* __restrict__ y, const float* __restrict__ t, int n, int m,
                             float* __restrict__ shrink, double* __restrict__ err2, double* __restrict__ pow2) {
  int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= m) return;
  double e = 0.0, pw = 0.0;
  for (int r = 0; r < n; ++r) {
    const double yy = y[(size_t)r * m + o], tt = t[(size_t)r * m + o];
    e += (yy - tt) * (yy - tt);
    pw += tt * tt;
  }
  const double sh = fmin(1.0, fmax(0.0, 1.0 - e / fmax(pw, 1e-30)));
  double es = 0.0;
  for (int r = 0; r < n; ++r) {
    const double d = sh * (double)y[(size_t)r * m + o] - (double)t[(size_t)r * m + o];
    es += d * d;
  }
  shrink[o] = (float)sh;
  err2[o] = es;
  pow2[o] = pw;
}

}  // namespace warm
}  // namespace pfm

using namespace pfm;
using namespace pfm::warm;

struct pfm_mlp {
  int L = 0;                        // weight layers
  int sizes[PFM_MLP_MAX_LAYERS + 1] = {};
  int max_batch = 0;
  long long n_params = 0;
  long long woff[PFM_MLP_MAX_LAYERS] = {}, boff[PFM_MLP_MAX_LAYERS] = {};
  float *d_p = nullptr, *d_g = nullptr, *d_m = nullptr, *d_v = nullptr;
  float* d_act[PFM_MLP_MAX_LAYERS + 1] = {};   // activations, [0] = copy of the input
  float *d_d0 = nullptr, *d_d1 = nullptr;      // backprop deltas (ping-pong)
  float *d_part = nullptr, *d_loss = nullptr, *h_loss = nullptr;
  unsigned short* d_wbf = nullptr;             // bf16 weights (same offsets as d_p)
  float* d_tmp[2] = {nullptr, nullptr};        // bf16 inference ping-pong
  hipStream_t stream = nullptr;
};

namespace {

void mlp_free(pfm_mlp* m) {
  auto f = [](void* p) { if (p) (void)hipFree(p); };
  f(m->d_p); f(m->d_g); f(m->d_m); f(m->d_v);
  for (int l = 0; l <= PFM_MLP_MAX_LAYERS; ++l) f(m->d_act[l]);
  f(m->d_d0); f(m->d_d1); f(m->d_part); f(m->d_loss); f(m->d_wbf); f(m->d_tmp[0]); f(m->d_tmp[1]);
  if (m->h_loss) (void)hipHostFree(m->h_loss);
}

}  // namespace

extern "C" {

pfm_status pfm_mlp_create(const int* sizes, int n_layers, int max_batch, unsigned long long seed, pfm_mlp** out) {
  if (!out) return PFM_EINVAL;
  *out = nullptr;
  if (!sizes || n_layers < 1 || n_layers > PFM_MLP_MAX_LAYERS || max_batch < 1 || max_batch > (1 << 20))
    return PFM_EINVAL;
  for (int l = 0; l <= n_layers; ++l)
    if (sizes[l] < 1 || sizes[l] > PFM_MLP_MAX_WIDTH) return PFM_EINVAL;
  pfm_mlp* m = new (std::nothrow) pfm_mlp();
  if (!m) return PFM_ENOMEM;
  m->L = n_layers;
  m->max_batch = max_batch;
  int wmax = 0;
  for (int l = 0; l <= n_layers; ++l) {
    m->sizes[l] = sizes[l];
    wmax = std::max(wmax, sizes[l]);
  }
  long long o = 0;
  for (int l = 0; l < n_layers; ++l) {
    m->woff[l] = o;
    o += (long long)sizes[l] * sizes[l + 1];
    m->boff[l] = o;
    o += sizes[l + 1];
  }
  m->n_params = o;
#define CK(call) do { if ((call) != hipSuccess) { mlp_free(m); delete m; return PFM_ENOMEM; } } while (0)
  CK(hipMalloc((void**)&m->d_p, o * sizeof(float)));
  CK(hipMalloc((void**)&m->d_g, o * sizeof(float)));
  CK(hipMalloc((void**)&m->d_m, o * sizeof(float)));
  CK(hipMalloc((void**)&m->d_v, o * sizeof(float)));
  CK(hipMalloc((void**)&m->d_wbf, o * sizeof(unsigned short)));
  for (int l = 0; l <= n_layers; ++l) CK(hipMalloc((void**)&m->d_act[l], (size_t)max_batch * sizes[l] * sizeof(float)));
  CK(hipMalloc((void**)&m->d_d0, (size_t)max_batch * wmax * sizeof(float)));
  CK(hipMalloc((void**)&m->d_d1, (size_t)max_batch * wmax * sizeof(float)));
  CK(hipMalloc((void**)&m->d_tmp[0], (size_t)max_batch * wmax * sizeof(float)));
  CK(hipMalloc((void**)&m->d_tmp[1], (size_t)max_batch * wmax * sizeof(float)));
  long long nout = (long long)max_batch * sizes[n_layers];
  CK(hipMalloc((void**)&m->d_part, ((nout + 255) / 256 + 1) * sizeof(float)));
  CK(hipMalloc((void**)&m->d_loss, sizeof(float)));
  CK(hipHostMalloc((void**)&m->h_loss, sizeof(float)));
  CK(hipMemset(m->d_m, 0, o * sizeof(float)));
  CK(hipMemset(m->d_v, 0, o * sizeof(float)));
  CK(hipMemset(m->d_g, 0, o * sizeof(float)));
  for (int l = 0; l < n_layers; ++l) {
    float sc = 1.0f / std::sqrt((float)sizes[l]);
    long long nw = (long long)sizes[l] * sizes[l + 1] + sizes[l + 1];
    hipLaunchKernelGGL(k_init_uniform, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, nullptr, nw,
                       m->d_p + m->woff[l], sc, seed, m->woff[l]);
  }
  CK(hipGetLastError());
  CK(hipDeviceSynchronize());
#undef CK
  *out = m;
  return PFM_OK;
}

void pfm_mlp_destroy(pfm_mlp* m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  mlp_free(m);
  delete m;
}

pfm_status pfm_mlp_set_stream(pfm_mlp* m, void* s) {
  if (!m) return PFM_EINVAL;
  m->stream = (hipStream_t)s;
  return PFM_OK;
}

long long pfm_mlp_n_params(const pfm_mlp* m) { return m ? m->n_params : -1; }

pfm_status pfm_mlp_buffers(pfm_mlp* m, float** d_params, float** d_grads) {
  if (!m) return PFM_EINVAL;
  if (d_params) *d_params = m->d_p;
  if (d_grads) *d_grads = m->d_g;
  return PFM_OK;
}

static pfm_status copy_dd(pfm_mlp* m, void* dst, const void* src) {
  if (!m || !dst || !src) return PFM_EINVAL;
  if (hipMemcpyAsync(dst, src, m->n_params * sizeof(float), hipMemcpyDeviceToDevice, m->stream) != hipSuccess)
    return PFM_EDEVICE;
  return PFM_OK;
}

pfm_status pfm_mlp_get_params(pfm_mlp* m, float* d_dst) { return copy_dd(m, d_dst, m ? m->d_p : nullptr); }
pfm_status pfm_mlp_set_params(pfm_mlp* m, const float* d_src) { return copy_dd(m, m ? m->d_p : nullptr, d_src); }
pfm_status pfm_mlp_get_grads(pfm_mlp* m, float* d_dst) { return copy_dd(m, d_dst, m ? m->d_g : nullptr); }

pfm_status pfm_mlp_scale_output(pfm_mlp* m, const float* d_scale, const float* d_shift) {
  if (!m || !d_scale || !d_shift) return PFM_EINVAL;
  const int l = m->L - 1, in = m->sizes[l], outw = m->sizes[l + 1];
  hipLaunchKernelGGL(k_scale_output, dim3((outw + 255) / 256), dim3(256), 0, m->stream, outw, in,
                     m->d_p + m->woff[l], m->d_p + m->boff[l], d_scale, d_shift);
  return hipGetLastError() == hipSuccess ? PFM_OK : PFM_EDEVICE;
}

pfm_status pfm_mlp_target_stats(pfm_mlp* m, const float* d_t, int n, float* d_mean, float* d_std) {
  if (!m || !d_t || !d_mean || !d_std || n < 1) return PFM_EINVAL;
  const int w = m->sizes[m->L];
  hipLaunchKernelGGL(k_col_stats, dim3((w + 255) / 256), dim3(256), 0, m->stream, d_t, n, w, 1e-6f, d_mean, d_std);
  return hipGetLastError() == hipSuccess ? PFM_OK : PFM_EDEVICE;
}

pfm_status pfm_mlp_standardise(pfm_mlp* m, const float* d_t, int n, const float* d_mean, const float* d_std,
                               float* d_out) {
  if (!m || !d_t || !d_mean || !d_std || !d_out || n < 1) return PFM_EINVAL;
  const int w = m->sizes[m->L];
  const long long total = (long long)n * w;
  hipLaunchKernelGGL(k_standardise, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, m->stream, d_t, total, w,
                     d_mean, d_std, d_out);
  return hipGetLastError() == hipSuccess ? PFM_OK : PFM_EDEVICE;
}

pfm_status pfm_mlp_forward(pfm_mlp* m, const float* d_x, int B, float* d_y);

pfm_status pfm_mlp_validation_shrink(pfm_mlp* m, const float* d_x, const float* d_t, int n, float* d_shrink,
                                     float* h_rel_err) {
  if (!m || !d_x || !d_t || !d_shrink || n < 1 || n > m->max_batch || m->max_batch < 4) return PFM_EINVAL;
  const int w = m->sizes[m->L];
  // the FP32 forward of the validation rows (kept in the inference scratch)
  float* y = m->d_tmp[0];
  pfm_status st = pfm_mlp_forward(m, d_x, n, y);
  if (st != PFM_OK) return st;
  // per-column sums in the delta buffers (max_batch * widest layer floats each, >= 2 w doubles)
  double* e2 = reinterpret_cast<double*>(m->d_d0);
  double* p2 = e2 + w;
  hipLaunchKernelGGL(k_val_shrink, dim3((w + 255) / 256), dim3(256), 0, m->stream, y, d_t, n, w, d_shrink, e2, p2);
  if (hipGetLastError() != hipSuccess) return PFM_EDEVICE;
  if (h_rel_err) {
    std::vector<double> h(2 * (size_t)w);
    if (hipMemcpyAsync(h.data(), e2, 2 * (size_t)w * sizeof(double), hipMemcpyDeviceToHost, m->stream) != hipSuccess ||
        hipStreamSynchronize(m->stream) != hipSuccess)
      return PFM_EDEVICE;
    double se = 0.0, sp = 0.0;
    for (int o = 0; o < w; ++o) {
      se += h[o];
      sp += h[w + o];
    }
    *h_rel_err = (float)std::sqrt(se / std::max(sp, 1e-300));
  }
  // fold the shrink into the last layer
  std::vector<float> zeros(w, 0.0f);
  float* shift = m->d_d1;
  if (hipMemcpyAsync(shift, zeros.data(), (size_t)w * sizeof(float), hipMemcpyHostToDevice, m->stream) != hipSuccess)
    return PFM_EDEVICE;
  return pfm_mlp_scale_output(m, d_shrink, shift);
}

pfm_status pfm_mlp_forward(pfm_mlp* m, const float* d_x, int B, float* d_y) {
  if (!m || !d_x || !d_y || B < 1 || B > m->max_batch) return PFM_EINVAL;
  hipStream_t s = m->stream;
  if (hipMemcpyAsync(m->d_act[0], d_x, (size_t)B * m->sizes[0] * sizeof(float), hipMemcpyDeviceToDevice, s) !=
      hipSuccess)
    return PFM_EDEVICE;
  for (int l = 0; l < m->L; ++l) {
    int in = m->sizes[l], outw = m->sizes[l + 1];
    bool last = l == m->L - 1;
    gemm(s, false, true, B, outw, in, m->d_act[l], in, m->d_p + m->woff[l], in, m->d_act[l + 1], outw,
         last ? EPI_BIAS : EPI_BIAS_TANH, m->d_p + m->boff[l], nullptr);
  }
  if (hipMemcpyAsync(d_y, m->d_act[m->L], (size_t)B * m->sizes[m->L] * sizeof(float), hipMemcpyDeviceToDevice, s) !=
      hipSuccess)
    return PFM_EDEVICE;
  return hipGetLastError() == hipSuccess ? PFM_OK : PFM_EDEVICE;
}

pfm_status pfm_mlp_backward_mse(pfm_mlp* m, const float* d_t, int B, float* h_loss) {
  if (!m || !d_t || B < 1 || B > m->max_batch) return PFM_EINVAL;
  hipStream_t s = m->stream;
  const int L = m->L;
  long long nout = (long long)B * m->sizes[L];
  int nblk = (int)((nout + 255) / 256);
  float* d = m->d_d0;
  float* dn = m->d_d1;
  hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(256), 0, s, nout, m->d_act[L], d_t, d, m->d_part);
  if (h_loss) hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, nblk, m->d_part, 1.0f / (float)nout, m->d_loss);
  for (int l = L - 1; l >= 0; --l) {
    int in = m->sizes[l], outw = m->sizes[l + 1];
    // dW_l = d^T h_l, db_l = column sums of d
    gemm(s, true, false, outw, in, B, d, outw, m->d_act[l], in, m->d_g + m->woff[l], in, EPI_NONE, nullptr, nullptr);
    hipLaunchKernelGGL(k_colsum, dim3((outw + 255) / 256), dim3(256), 0, s, B, outw, d, m->d_g + m->boff[l]);
    if (l > 0) {
      // d_{l-1} = (d W_l) * (1 - h_l^2), h_l = tanh output of layer l-1
      gemm(s, false, false, B, in, outw, d, outw, m->d_p + m->woff[l], in, dn, in, EPI_DTANH, nullptr, m->d_act[l]);
      std::swap(d, dn);
    }
  }
  if (hipGetLastError() != hipSuccess) return PFM_EDEVICE;
  if (h_loss) {
    if (hipMemcpyAsync(m->h_loss, m->d_loss, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return PFM_EDEVICE;
    *h_loss = *m->h_loss;
  }
  return PFM_OK;
}

pfm_status pfm_mlp_adam(pfm_mlp* m, float lr, float b1, float b2, float eps, int t) {
  if (!m || t < 1) return PFM_EINVAL;
  float bc1 = 1.0f - std::pow(b1, (float)t), bc2 = 1.0f - std::pow(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((m->n_params + 255) / 256)), dim3(256), 0, m->stream, m->n_params,
                     m->d_p, m->d_g, m->d_m, m->d_v, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError() == hipSuccess ? PFM_OK : PFM_EDEVICE;
}

pfm_status pfm_mlp_to_bf16(pfm_mlp* m) {
  if (!m) return PFM_EINVAL;
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((m->n_params + 255) / 256)), dim3(256), 0, m->stream, m->n_params,
                     m->d_p, m->d_wbf);
  return hipGetLastError() == hipSuccess ? PFM_OK : PFM_EDEVICE;
}

pfm_status pfm_mlp_infer_bf16(pfm_mlp* m, const float* d_x, int B, float* d_y) {
  if (!m || !d_x || !d_y || B < 1 || B > m->max_batch) return PFM_EINVAL;
  const float* x = d_x;
  for (int l = 0; l < m->L; ++l) {
    int in = m->sizes[l], outw = m->sizes[l + 1];
    bool last = l == m->L - 1;
    float* y = last ? d_y : m->d_tmp[l & 1];
    dim3 grid((outw + 63) / 64, (B + 15) / 16);
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, m->stream, B, outw, in, x, m->d_wbf + m->woff[l],
                       m->d_p + m->boff[l], last ? 0 : 1, y);
    x = y;
  }
  return hipGetLastError() == hipSuccess ? PFM_OK : PFM_EDEVICE;
}

pfm_status pfm_warm_features(const double* d_draws, int B, float* d_x, void* stream) {
  if (!d_draws || !d_x || B < 1) return PFM_EINVAL;
  hipLaunchKernelGGL(k_features, dim3((5 * B + 255) / 256), dim3(256), 0, (hipStream_t)stream, B, d_draws, d_x);
  return hipGetLastError() == hipSuccess ? PFM_OK : PFM_EDEVICE;
}

static pfm_status modes_call(pfm_problem* h, int K, int B, const double* thetas, bool analyse, const void* in,
                             void* out) {
  if (!h || !thetas || !in || !out) return PFM_EINVAL;
  Problem& pb = h->p;
  if (K < 2 || (K & 1) || K > pb.N || pb.N > MODES_MAX_N || B < 1 || B > pb.max_batch) return PFM_EINVAL;
  if (!(pb.k > 0)) return PFM_ESTATE;
  if (hipMemcpyAsync(pb.d_thetas, thetas, B * sizeof(double), hipMemcpyHostToDevice, pb.stream) != hipSuccess)
    return PFM_EDEVICE;
  dim3 grid(2 * pb.M, B);
  if (analyse)
    hipLaunchKernelGGL(k_modes_analyse, grid, dim3(256), 0, pb.stream, pb.M, pb.N, K, pb.k, pb.d_thetas,
                       pb.d_centres, (const cd*)in, (float*)out);
  else
    hipLaunchKernelGGL(k_modes_synthesise, grid, dim3(256), 0, pb.stream, pb.M, pb.N, K, pb.k, pb.d_thetas,
                       pb.d_centres, (const float*)in, (cd*)out);
  // the host array of angles may go away once the copy has run
  if (hipStreamSynchronize(pb.stream) != hipSuccess) return PFM_EDEVICE;
  return hipGetLastError() == hipSuccess ? PFM_OK : PFM_EDEVICE;
}

pfm_status pfm_modes_analyse(pfm_problem* h, int K, int B, const double* thetas, const void* d_psi, float* d_vec) {
  return modes_call(h, K, B, thetas, true, d_psi, d_vec);
}

pfm_status pfm_modes_synthesise(pfm_problem* h, int K, int B, const double* thetas, const float* d_vec,
                                void* d_psi) {
  return modes_call(h, K, B, thetas, false, d_vec, d_psi);
}

}  // extern "C"
