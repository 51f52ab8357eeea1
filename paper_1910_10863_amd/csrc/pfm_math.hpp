// Complex arithmetic and FP64 cylinder functions for the FMM (host + device).
//
// Special functions are written from the series and expansions of the DLMF:
//   * J0, J1, Y0, Y1 by their ascending series for x <= 2,
//   * J0, J1 by Miller's backward recurrence normalised by
//     J0 + 2 sum_k J_2k = 1 (DLMF 10.12.4 at theta = 0, 3.6),
//   * Y0 from the same J values by Neumann's series
//     Y0 = (2/pi)(ln(x/2) + gamma) J0 - (4/pi) sum_k (-1)^k J_2k / k
//     (Abramowitz & Stegun 9.1.88), and Y1 = -Y0' term by term,
//   * the Hankel asymptotic expansion for large arguments (DLMF 10.17.3),
//   * scaled J_n sequences g_n(x) = n! (2/x)^n J_n(x) by their power series
//     (DLMF 10.2.2) at the top order and the scaled backward recurrence
//     g_{n-1} = g_n - (x^2/4) g_{n+1} / (n (n+1)) (from DLMF 10.6.1),
//   * H_n by the forward recurrence H_{n+1} = (2n/x) H_n - H_{n-1}
//     (DLMF 10.6.1), which is stable for the dominant Y part.
// The cylinder harmonics of the paper's expansions (Sec. 3.2) are
//   Hp_n(v) = H_n(|v|) e^{i n arg v},  Jp_n(v) = J_n(|v|) e^{i n arg v},
//   Jm_n(v) = J_n(|v|) e^{-i n arg v} = conj(Jp_n(v)),
//   Jp_{-n}(v) = (-1)^n conj(Jp_n(v)),  Hp_{-n}(v) = (-1)^n H_n e^{-i n arg v}.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace pfm {

typedef double2 cd;

__host__ __device__ __forceinline__ cd mkc(double r, double i) { cd z; z.x = r; z.y = i; return z; }
__host__ __device__ __forceinline__ cd cadd(cd a, cd b) { return mkc(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ cd csub(cd a, cd b) { return mkc(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ cd cmul(cd a, cd b) {
  return mkc(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ cd cconj(cd a) { return mkc(a.x, -a.y); }
__host__ __device__ __forceinline__ cd cscale(cd a, double s) { return mkc(a.x * s, a.y * s); }
// a*b + c
__host__ __device__ __forceinline__ cd cfma(cd a, cd b, cd c) {
  return mkc(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
// single-precision complex a*b + c
__host__ __device__ __forceinline__ float2 cfmaf(float2 a, float2 b, float2 c) {
  float2 r;
  r.x = fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x));
  r.y = fmaf(a.x, b.y, fmaf(a.y, b.x, c.y));
  return r;
}
// conj(a)*b + c
__host__ __device__ __forceinline__ cd cfma_conj(cd a, cd b, cd c) {
  return mkc(fma(a.x, b.x, fma(a.y, b.y, c.x)), fma(a.x, b.y, fma(-a.y, b.x, c.y)));
}
__host__ __device__ __forceinline__ cd cmul_i(cd a) { return mkc(-a.y, a.x); }   // i*a
__host__ __device__ __forceinline__ double cabs2(cd a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ __forceinline__ cd cexp(cd a) {
  double e = exp(a.x), s, c;
  sincos(a.y, &s, &c);
  return mkc(e * c, e * s);
}
__host__ __device__ __forceinline__ cd cdiv(cd a, cd b) {
  double d = b.x * b.x + b.y * b.y;
  return mkc((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
// principal square root
__host__ __device__ __forceinline__ cd csqrt(cd a) {
  double r = sqrt(a.x * a.x + a.y * a.y);
  double re = sqrt(fmax(0.5 * (r + a.x), 0.0));
  double im = sqrt(fmax(0.5 * (r - a.x), 0.0));
  if (a.y < 0) im = -im;
  return mkc(re, im);
}
// integer power by repeated squaring, n >= 0
__host__ __device__ __forceinline__ cd cpowi(cd a, int n) {
  cd r = mkc(1.0, 0.0);
  while (n > 0) {
    if (n & 1) r = cmul(r, a);
    a = cmul(a, a);
    n >>= 1;
  }
  return r;
}

constexpr double PI = 3.14159265358979323846;
constexpr double EULER_GAMMA = 0.57721566490153286061;

// J0, J1, Y0, Y1 for 0 < x <= 2 by their ascending series (DLMF 10.2.2, 10.8.1;
// Abramowitz & Stegun 9.1.10-9.1.11), q = x^2/4:
//   J0 = sum_k (-q)^k / (k!)^2,  J1 = (x/2) sum_k (-q)^k / (k! (k+1)!),
//   Y0 = (2/pi) (ln(x/2) + gamma) J0 + (2/pi) sum_{k>=1} (-1)^{k+1} H_k q^k / (k!)^2,
//   Y1 = -2/(pi x) + (2/pi) ln(x/2) J1 - (x/(2 pi)) sum_k (psi(k+1) + psi(k+2)) (-q)^k / (k! (k+1)!),
// with H_k the harmonic numbers and psi(k+1) = H_k - gamma.  For q <= 1 the
// terms fall below 1e-18 of the sum after 14 of them; the fixed count keeps
// the lanes of a wavefront together.
__host__ __device__ inline void bessel_jy01_series(double x, double& J0, double& J1, double& Y0, double& Y1) {
  const double q = 0.25 * x * x;
  double t0 = 1.0, t1 = 1.0;          // (-q)^k/(k!)^2 and (-q)^k/(k!(k+1)!)
  double sj0 = 1.0, sj1 = 1.0;
  double sy0 = 0.0;                   // sum (-1)^{k+1} H_k q^k/(k!)^2 = -sum H_k t0
  double sy1 = 1.0 - 2.0 * EULER_GAMMA; // k = 0 term: psi(1) + psi(2) = 1 - 2 gamma
  double hk = 0.0;
#pragma unroll
  for (int k = 1; k <= 14; ++k) {
    t0 *= -q * (1.0 / ((double)k * (double)k));
    t1 *= -q * (1.0 / ((double)k * (double)(k + 1)));
    hk += 1.0 / (double)k;
    sj0 += t0;
    sj1 += t1;
    sy0 -= hk * t0;
    // psi(k+1) + psi(k+2) = 2 H_k + 1/(k+1) - 2 gamma
    sy1 += (2.0 * hk + 1.0 / (double)(k + 1) - 2.0 * EULER_GAMMA) * t1;
  }
  const double lg = log(0.5 * x);
  J0 = sj0;
  J1 = 0.5 * x * sj1;
  Y0 = (2.0 / PI) * ((lg + EULER_GAMMA) * J0 + sy0);
  Y1 = -2.0 / (PI * x) + (2.0 / PI) * lg * J1 - (0.5 * x / PI) * sy1;
}

// J0, J1, Y0, Y1 for x > 0.
__host__ __device__ inline void bessel_jy01(double x, double& J0, double& J1, double& Y0, double& Y1) {
  if (x <= 2.0) {
    bessel_jy01_series(x, J0, J1, Y0, Y1);
    return;
  }
  if (x > 25.0) {
    // Hankel's expansion H_nu(x) ~ sqrt(2/(pi x)) e^{i w} sum_k i^k a_k(nu) / x^k,
    // a_k(nu) = prod_{j=1..k} (4 nu^2 - (2j-1)^2) / (k! 8^k),  w = x - nu pi/2 - pi/4.
    double pre = sqrt(2.0 / (PI * x));
    for (int nu = 0; nu <= 1; ++nu) {
      double mu = 4.0 * nu * nu;
      double tr = 1.0, ti = 0.0;     // running term i^k a_k / x^k
      double sr = 1.0, si = 0.0;
      double last = 1.0;
      for (int k = 1; k < 40; ++k) {
        double f = (mu - (2.0 * k - 1) * (2.0 * k - 1)) / (8.0 * k * x);
        // multiply by i * f
        double nr = -ti * f, ni = tr * f;
        tr = nr; ti = ni;
        double mag = fabs(tr) + fabs(ti);
        if (mag > last) break;       // asymptotic series starts to diverge
        sr += tr; si += ti;
        last = mag;
        if (mag < 1e-18) break;
      }
      double w = x - 0.5 * nu * PI - 0.25 * PI, s, c;
      sincos(w, &s, &c);
      // (sr + i si)(c + i s)
      double hr = pre * (sr * c - si * s);
      double hi = pre * (sr * s + si * c);
      if (nu == 0) { J0 = hr; Y0 = hi; } else { J1 = hr; Y1 = hi; }
    }
    return;
  }
  // Miller's algorithm.  Unnormalised values v_n ~ J_n; sums accumulated on the way down:
  //   norm = v_0 + 2 sum_{k>=1} v_2k,
  //   sy0  = sum_{k>=1} (-1)^k v_2k / k,
  //   sy1  = sum_{k>=1} (-1)^k (v_{2k-1} - v_{2k+1}) / k.
  int N = 2 * (int)((x + 24.0 + 9.0 * sqrt(x)) * 0.5) + 2;
  double two_over_x = 2.0 / x;
  double vp1 = 0.0;            // v_{n+1}
  double v = 1e-280;           // v_n at n = N
  double vp2 = 0.0;            // v_{n+2}
  double norm = 0.0, sy0 = 0.0, sy1 = 0.0;
  // v_N, v_{N+1} = 0: start with n = N
  // contributions that involve v_N (N even): norm, sy0; sy1 uses v_{2k+1} terms.
  for (int n = N; n >= 1; --n) {
    // here v = v_n, vp1 = v_{n+1}, vp2 = v_{n+2}
    if ((n & 1) == 0) {
      int k = n >> 1;
      norm += 2.0 * v;
      double sgn = (k & 1) ? -1.0 : 1.0;
      sy0 += sgn * v / k;
    } else {
      // n = 2k-1: term (-1)^k (v_{2k-1} - v_{2k+1}) / k with k = (n+1)/2
      int k = (n + 1) >> 1;
      double sgn = (k & 1) ? -1.0 : 1.0;
      sy1 += sgn * (v - vp2) / k;
    }
    double vm1 = n * two_over_x * v - vp1;
    vp2 = vp1;
    vp1 = v;
    v = vm1;
    if (fabs(v) > 1e250) {
      const double s = 1e-250;
      v *= s; vp1 *= s; vp2 *= s; norm *= s; sy0 *= s; sy1 *= s;
    }
  }
  // now v = v_0, vp1 = v_1
  norm += v;
  double inv = 1.0 / norm;
  J0 = v * inv;
  J1 = vp1 * inv;
  double lg = log(0.5 * x) + EULER_GAMMA;
  Y0 = (2.0 / PI) * lg * J0 - (4.0 / PI) * sy0 * inv;
  Y1 = -(2.0 / (PI * x)) * J0 + (2.0 / PI) * lg * J1 + (2.0 / PI) * sy1 * inv;
}

__host__ __device__ inline void hankel01(double x, cd& H0, cd& H1) {
  double j0, j1, y0, y1;
  bessel_jy01(x, j0, j1, y0, y1);
  H0 = mkc(j0, y0);
  H1 = mkc(j1, y1);
}

// Scaled Bessel sequence g_n(x) = n! (2/x)^n J_n(x), n = 0..NT (x >= 0), written to g[].
// q = x^2/4.  Power series g_n = sum_k (-q)^k n! / (k! (n+k)!) at NT and NT-1,
// then the scaled backward recurrence g_{n-1} = g_n - q g_{n+1} / (n (n+1)).
// All divisors are compile-time constants, so no division is executed; for
// q <= 10 the series is cut at 18 terms (remainder below 1e-17 for NT >= 9),
// larger arguments sum until the terms are negligible.
template <int NT>
__host__ __device__ __forceinline__ double scaled_j_series(double q) {
  double term = 1.0, sum = 1.0;
  if (q <= 10.0) {
#pragma unroll
    for (int k = 1; k <= 18; ++k) {
      term *= -q * (1.0 / ((double)k * (double)(NT + k)));
      sum += term;
    }
  } else {
    for (int k = 1; k < 400; ++k) {
      term *= -q / ((double)k * (double)(NT + k));
      sum += term;
      if (fabs(term) < 1e-17 * fabs(sum)) break;
    }
  }
  return sum;
}

template <int NT>
__host__ __device__ __forceinline__ void scaled_j(double q, double (&g)[NT + 1]) {
  g[NT] = scaled_j_series<NT>(q);
  g[NT - 1] = scaled_j_series<NT - 1>(q);
#pragma unroll
  for (int n = NT - 1; n >= 1; --n) {
    g[n - 1] = g[n] - q * g[n + 1] * (1.0 / ((double)n * (double)(n + 1)));
  }
}

// The same sequence divided by n!: h_n(x) = (2/x)^n J_n(x) = g_n / n!, so that
// Jp_n(v) = (v/2)^n h_n(|v|) needs no factorial in the power sequence.  Power
// series at NT and NT-1 (h_n = sum_k (-q)^k / (k! (n+k)!)); for q <= 1/4 eight
// terms leave a remainder below 1e-19 relative for n >= 4, else as scaled_j.
// Backward recurrence h_{n-1} = n h_n - q h_{n+1} (that of g_n times 1/(n-1)!).
__host__ __device__ constexpr double inv_factorial(int n) { return n <= 1 ? 1.0 : inv_factorial(n - 1) / n; }

template <int NT>
__host__ __device__ __forceinline__ double scaled_h_series(double q) {
  constexpr double f = inv_factorial(NT);
  double term = f, sum = f;
  if (q <= 0.25) {
#pragma unroll
    for (int k = 1; k <= 8; ++k) {
      term *= -q * (1.0 / ((double)k * (double)(NT + k)));
      sum += term;
    }
  } else if (q <= 10.0) {
#pragma unroll
    for (int k = 1; k <= 18; ++k) {
      term *= -q * (1.0 / ((double)k * (double)(NT + k)));
      sum += term;
    }
  } else {
    for (int k = 1; k < 400; ++k) {
      term *= -q / ((double)k * (double)(NT + k));
      sum += term;
      if (fabs(term) < 1e-17 * fabs(sum)) break;
    }
  }
  return sum;
}

template <int NT>
__host__ __device__ __forceinline__ void scaled_h(double q, double (&h)[NT + 1]) {
  static_assert(NT >= 5, "the eight-term series needs n >= 4");
  h[NT] = scaled_h_series<NT>(q);
  h[NT - 1] = scaled_h_series<NT - 1>(q);
#pragma unroll
  for (int n = NT - 1; n >= 1; --n) h[n - 1] = (double)n * h[n] - q * h[n + 1];
}

// Jp_n(v) for n = 0..NT at the complex point v (v = vx + i vy), into jp[].
template <int NT>
__host__ __device__ __forceinline__ void jplus_seq(double vx, double vy, cd (&jp)[NT + 1]) {
  double g[NT + 1];
  scaled_j<NT>(0.25 * (vx * vx + vy * vy), g);
  cd u = mkc(1.0, 0.0);        // (v/2)^n / n!
  cd h = mkc(0.5 * vx, 0.5 * vy);
#pragma unroll
  for (int n = 0; n <= NT; ++n) {
    jp[n] = cscale(u, g[n]);
    u = cscale(cmul(u, h), 1.0 / (double)(n + 1));
  }
}

}  // namespace pfm
