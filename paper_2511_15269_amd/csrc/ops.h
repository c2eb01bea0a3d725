// Device building blocks shared by the single- and multi-vector evaluation
// kernels: the real regular basis and its gradient (App. A.1, A.3), the
// rotation-based translations (Sec. II.D, App. B) in the normalised,
// radius-scaled coefficient basis (see tables.h and eval.hip), and small
// arithmetic helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "tables.h"

namespace fmm {
namespace ops {

constexpr double kInv4Pi = 0.079577471545947667884441881686257181;

template <int P>
struct K_ {
  static constexpr int value = (P + 1) * (P + 1);
};

// Opaque copy of a wave-uniform pointer: table reads through it are issued
// where they are used instead of being hoisted out of the interaction loop
// (hoisting them all would exceed the scalar register file and spill).
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;  // constant memory

template <typename T>
__device__ __forceinline__ cptr<T> local_ptr(const T* p) {
  asm volatile("" : "+s"(p));
  return (cptr<T>)p;
}

// Sequential reader of a constant table whose entries are consumed in
// storage order at compile-time-known positions (fully unrolled loops).
// Entries arrive through the scalar unit in 64-byte blocks, R blocks per
// batch, double-buffered: right after the first use of batch j the loads
// of batch j+1 are issued, so their latency overlaps the rest of batch j.
// (Scalar loads may complete out of order, so a wait is always a wait for
// every outstanding one; the first use of a batch comes before the next
// batch is requested for that reason.)  Reads up to 2 R blocks past the
// last entry used: the tables carry tab_pad() entries of padding.
template <typename T>
struct TabReader {
  static constexpr int B = 64 / sizeof(T);  // entries per block
  static constexpr int R = 2;               // blocks per batch
  static constexpr int BR = B * R;
  cptr<T> p;
  T buf[2][BR];
  __device__ __forceinline__ explicit TabReader(cptr<T> q) : p(q) { fetch(0); }
  __device__ __forceinline__ void fetch(int batch) {
#pragma unroll
    for (int i = 0; i < BR; ++i) buf[batch & 1][i] = p[batch * BR + i];
  }
  __device__ __forceinline__ T get(int o) const { return buf[(o / BR) & 1][o % BR]; }
  // call after the use of entry o
  __device__ __forceinline__ void used(int o) {
    if (o % BR == 0) {
      __builtin_amdgcn_sched_barrier(0);
      fetch(o / BR + 1);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
};

// The translation steps below (azimuth, apply_y, zshift, Turn) do not let
// the compiler fuse a product with an addition on its own: every fused
// multiply-add is written out, so the rounding of each coefficient is fixed
// by the source and the same wherever the steps are inlined (the one-lane
// and the wave-shared M2L forms give identical results).
//
// Degree masks (bit n: degree n) and order masks (bit |m|: orders +-m)
// restrict the steps to part of a coefficient vector; the default takes all
// of it.
template <int P>
struct All_ {
  static constexpr unsigned value = (1u << (P + 1)) - 1u;
};

// (v^m, v^{-m}) <- (a c + b s, b c - a s) for every degree, with
// (c, s) = (cos m g, sgn sin m g) after the quarter-turn shift q (m*q*pi/2
// added to the angle; q in {0, 1}): q = 1 maps (cos mg, sin mg) to
// (cos m(pi/2 - g), sin m(pi/2 - g)).  cos m g and sin m g are formed from
// (c1, s1) = (cos g, sin g) by repeated complex multiplication as m grows
// (the same values at every call, and no registers held between calls).
template <int P, typename T, int SGN, int Q, unsigned DM = All_<P>::value>
__device__ __forceinline__ void azimuth(T* v, T c1, T s1) {
#pragma clang fp contract(off)
  T cm = T(1), sm = T(0);
#pragma unroll
  for (int m = 1; m <= P; ++m) {
    if ((DM >> m) == 0) break;  // no degree >= m in the mask
    const T cn = fma(cm, c1, -(sm * s1));
    const T sn = fma(sm, c1, cm * s1);
    cm = cn;
    sm = sn;
    T c, s;
    if (Q == 0) {
      c = cm;
      s = sm;
    } else {
      switch (m & 3) {
        case 0: c = cm; s = -sm; break;
        case 1: c = sm; s = cm; break;
        case 2: c = -cm; s = sm; break;
        default: c = -sm; s = -cm; break;
      }
    }
    if (SGN < 0) s = -s;
#pragma unroll
    for (int n = m; n <= P; ++n) {
      if (!((DM >> n) & 1u)) continue;
      T a = v[cidx(n, m)], b = v[cidx(n, -m)];
      v[cidx(n, m)] = fma(a, c, b * s);
      v[cidx(n, -m)] = fma(b, c, -(a * s));
    }
  }
}

// v_n <- Y_n v_n (TR: Y_n^T v_n) over the nonzero entries, column by
// column: each input coefficient is scattered into the output rows it
// reaches, so consecutive multiply-adds go to different accumulators.  The
// column-major order of Y_n is the row-major order of Y_n^T, so the product
// with Y_n reads the stored Y_n^T rows and vice versa.  A run of consecutive
// degrees in the mask is read with one sequential table reader.  (The
// reader of degree 1 is set up even when degree 1 is not in the mask; its
// loads go unused.)
template <int P, bool TR, typename T, unsigned DM = All_<P>::value>
__device__ __forceinline__ void apply_y(T* v, const T* __restrict__ tab) {
#pragma clang fp contract(off)
  const T* base = tab + (TR ? tab_y(P) : tab_yt(P));
  TabReader<T> Y(local_ptr(base) + ycbase(1));
  int o = 0;
#pragma unroll
  for (int n = 1; n <= P; ++n) {
    if (!((DM >> n) & 1u)) continue;
    if (n > 1 && !((DM >> (n - 1)) & 1u)) {  // a new run of degrees
      Y = TabReader<T>(local_ptr(base) + ycbase(n));
      o = 0;
    }
    T u[2 * P + 1];
    bool live[2 * P + 1];
#pragma unroll
    for (int a = 0; a <= 2 * n; ++a) live[a] = false;
#pragma unroll
    for (int b = -n; b <= n; ++b) {
      const T vb = v[cidx(n, b)];
#pragma unroll
      for (int a = -n; a <= n; ++a) {
        if (!ynz(n, a, b)) continue;
        u[a + n] = live[a + n] ? fma(Y.get(o), vb, u[a + n]) : Y.get(o) * vb;
        live[a + n] = true;
        Y.used(o);
        ++o;
      }
    }
#pragma unroll
    for (int a = -n; a <= n; ++a) v[cidx(n, a)] = u[a + n];
  }
}

enum { kM2M = 0, kM2L = 1, kL2L = 2 };

// z-axis operators of App. B.3 in the normalised, radius-scaled basis, in
// place.  With r the shift length:
//   M2L (a = rho_src/r, b = rho_tgt/r):   out_n = b^{n+1} sum_k T_nk a^k v_k
//   M2M (a = r/rho_par, b = rho_chi/rho_par): out_n = sum_{k<=n} T_nk a^{n-k} b^k v_k
//   L2L (a = r/rho_par, b = rho_chi/rho_par): out_n = b^{n+1} sum_{k>=n} T_nk a^{k-n} v_k
template <int P, int KIND, typename T, unsigned OM = All_<P>::value>
__device__ __forceinline__ void zshift(T* v, T a, T b, const T* __restrict__ tab) {
#pragma clang fp contract(off)
  T pa[2 * P + 2], pb[P + 2];
  pa[0] = T(1);
  pb[0] = T(1);
#pragma unroll
  for (int j = 1; j <= P; ++j) pa[j] = pa[j - 1] * a;
#pragma unroll
  for (int j = 1; j <= P + 1; ++j) pb[j] = pb[j - 1] * b;
  if (KIND == kM2L) {
#pragma unroll
    for (int n = 0; n <= P; ++n)
#pragma unroll
      for (int m = -n; m <= n; ++m)
        if ((OM >> (m < 0 ? -m : m)) & 1u) v[cidx(n, m)] *= pa[n];
    // table column by column (k outer): independent accumulators; the
    // blocks of -m and +m are the same, read twice in a row
#pragma unroll
    for (int m = -P; m <= P; ++m) {
      const int am = m < 0 ? -m : m;
      if (!((OM >> am) & 1u)) continue;
      TabReader<T> tb(local_ptr(tab) + tab_tm2l(P) + zl_base(P, am));
      T o[P + 1];
      int c = 0;
#pragma unroll
      for (int k = am; k <= P; ++k) {
        const T vk = v[cidx(k, m)];
#pragma unroll
        for (int n = am; n <= P; ++n) {
          o[n] = k == am ? tb.get(c) * vk : fma(tb.get(c), vk, o[n]);
          tb.used(c);
          ++c;
        }
      }
#pragma unroll
      for (int n = am; n <= P; ++n) v[cidx(n, m)] = m < 0 ? -(o[n] * pb[n + 1]) : o[n] * pb[n + 1];
    }
  } else {
    if (KIND == kM2M) {
#pragma unroll
      for (int n = 0; n <= P; ++n)
#pragma unroll
        for (int m = -n; m <= n; ++m)
          if ((OM >> (m < 0 ? -m : m)) & 1u) v[cidx(n, m)] *= pb[n];
    }
#pragma unroll
    for (int m = -P; m <= P; ++m) {
      const int am = m < 0 ? -m : m;
      if (!((OM >> am) & 1u)) continue;
      TabReader<T> tb(local_ptr(tab) + (KIND == kM2M ? tab_tm2m(P) : tab_tl2l(P)) +
                      zt_base(P, am));
      T o[P + 1];
      int c = 0;
#pragma unroll
      for (int n = am; n <= P; ++n) {
        T acc = T(0);
        if (KIND == kM2M) {
#pragma unroll
          for (int k = am; k <= n; ++k) {
            acc = fma(tb.get(c) * pa[n - k], v[cidx(k, m)], acc);
            tb.used(c++);
          }
        } else {
#pragma unroll
          for (int k = n; k <= P; ++k) {
            acc = fma(tb.get(c) * pa[k - n], v[cidx(k, m)], acc);
            tb.used(c++);
          }
          acc *= pb[n + 1];
        }
        o[n] = acc;
      }
#pragma unroll
      for (int n = am; n <= P; ++n) v[cidx(n, m)] = o[n];
    }
  }
}

// Geometry of one translation: b = old centre - new centre, rho_old and
// rho_new the scale lengths of the two boxes.  Holds cosine and sine of the
// two rotation angles (azimuth A of b, polar angle B) and the z-shift
// ratios (a, b of zshift).
template <int P, int KIND, typename T>
struct Turn {
  T ca, sa, cb, sb;
  T a, b;
  __device__ __forceinline__ Turn(double bx, double by, double bz, double rho_old,
                                  double rho_new) {
#pragma clang fp contract(off)
    const double rxy2 = bx * bx + by * by;
    const double rxy = sqrt(rxy2);
    const double r = sqrt(rxy2 + bz * bz);
    // two reciprocals instead of six divisions
    const double ixy = rxy > 0.0 ? 1.0 / rxy : 0.0;
    const double ir = r > 0.0 ? 1.0 / r : 0.0;
    double dca = 1.0, dsa = 0.0, dcb = 1.0, dsb = 0.0;
    if (rxy > 0.0) {
      dca = bx * ixy;
      dsa = by * ixy;
    }
    if (r > 0.0) {
      dcb = bz * ir;
      dsb = rxy * ir;
    }
    double da, db;
    if (KIND == kM2L) {
      da = rho_old * ir;
      db = rho_new * ir;
    } else {
      const double ip = 1.0 / (KIND == kM2M ? rho_new : rho_old);
      da = r * ip;
      db = (KIND == kM2M ? rho_old : rho_new) * ip;
    }
    a = T(da);
    b = T(db);
    ca = T(dca);
    sa = T(dsa);
    cb = T(dcb);
    sb = T(dsb);
  }
};

// Rotation taking b onto +z: Rz(pi/2 - A), Y, Rz(-B), Y^T (sign
// conventions per kind), on the degrees of DM.
template <int P, int KIND, typename T, unsigned DM = All_<P>::value>
__device__ __forceinline__ void turn_forward(T* v, const Turn<P, KIND, T>& g,
                                             const T* __restrict__ tab) {
  if (KIND == kL2L)
    azimuth<P, T, -1, 1, DM>(v, g.ca, g.sa);
  else
    azimuth<P, T, +1, 1, DM>(v, g.ca, g.sa);
  apply_y<P, false, T, DM>(v, tab);
  if (KIND == kL2L)
    azimuth<P, T, +1, 0, DM>(v, g.cb, g.sb);
  else
    azimuth<P, T, -1, 0, DM>(v, g.cb, g.sb);
  apply_y<P, true, T, DM>(v, tab);
}

// The inverse rotation: Y, Rz(B), Y^T, Rz(A - pi/2), on the degrees of DM.
template <int P, int KIND, typename T, unsigned DM = All_<P>::value>
__device__ __forceinline__ void turn_back(T* v, const Turn<P, KIND, T>& g,
                                          const T* __restrict__ tab) {
  apply_y<P, false, T, DM>(v, tab);
  if (KIND == kM2M)
    azimuth<P, T, +1, 0, DM>(v, g.cb, g.sb);
  else
    azimuth<P, T, -1, 0, DM>(v, g.cb, g.sb);
  apply_y<P, true, T, DM>(v, tab);
  if (KIND == kM2M)
    azimuth<P, T, -1, 1, DM>(v, g.ca, g.sa);
  else
    azimuth<P, T, +1, 1, DM>(v, g.ca, g.sa);
}

// Rotate so that b points along +z, shift along z, rotate back.
// b = old centre - new centre; rho_old, rho_new the scale lengths of the
// two boxes.  M2L maps multipole (regular-basis sign convention) to local
// (singular-basis convention); M2M keeps the former, L2L the latter.
template <int P, int KIND, typename T>
__device__ __forceinline__ void rotate_shift(T* v, double bx, double by, double bz,
                                             double rho_old, double rho_new,
                                             const T* __restrict__ tab) {
  const Turn<P, KIND, T> g(bx, by, bz, rho_old, rho_new);
  turn_forward<P, KIND, T>(v, g, tab);
  zshift<P, KIND, T>(v, g.a, g.b, tab);
  turn_back<P, KIND, T>(v, g, tab);
}

// Source points in leaf order with their charges, one 32-byte record per
// point (so that a wave-uniform read is a single scalar load).  Positions
// stay FP64 in both forms: the FP32 form takes each pair difference in FP64
// and rounds it, so clustered points keep their separation and exactly
// coincident points give exactly zero.
template <typename T>
struct alignas(32) Src {
  double x, y, z;
  T q;
};

// Regular basis R-hat^m_n(x, y, z) in degree-major order by the App. A.1
// recursions; calls f(k, value) for k = 0..K-1 as values become available.
template <int P, typename T, typename F>
__device__ __forceinline__ void regular_basis(T x, T y, T z, F&& f) {
  const T r2 = x * x + y * y + z * z;
  T sc = T(1), ss = T(0);  // sectoral R^{m}_{m}, R^{-m}_{m}
#pragma unroll
  for (int m = 0; m <= P; ++m) {
    if (m == 1) {
      sc = x * T(0.5);
      ss = -y * T(0.5);
    } else if (m >= 2) {
      const T nc = (x * sc + y * ss) * T(1.0 / (2 * m));
      const T ns = (x * ss - y * sc) * T(1.0 / (2 * m));
      sc = nc;
      ss = ns;
    }
    f(cidx(m, m), sc);
    if (m > 0) f(cidx(m, -m), ss);
    T p2c = T(0), p2s = T(0), p1c = sc, p1s = ss;
#pragma unroll
    for (int n = m + 1; n <= P; ++n) {
      T c, s;
      if (n == m + 1) {
        c = z * p1c;
        s = z * p1s;
      } else {
        const T inv = T(1.0 / ((n - m) * (n + m)));
        c = (T(2 * n - 1) * z * p1c - r2 * p2c) * inv;
        s = (T(2 * n - 1) * z * p1s - r2 * p2s) * inv;
      }
      f(cidx(n, m), c);
      if (m > 0) f(cidx(n, -m), s);
      p2c = p1c;
      p2s = p1s;
      p1c = c;
      p1s = s;
    }
  }
}

// Regular basis R-hat^m_n and its gradient (App. A.1, A.3; the sectoral
// gradient without the printed leading minus) in order-major sweeps; calls
// f(k, value, d/dx, d/dy, d/dz) once per coefficient index k and
// band_end() after the last coefficient of every order m.
template <int P, typename T, typename F, typename E>
__device__ __forceinline__ void basis_with_gradient(T x, T y, T z, F&& f, E&& band_end) {
  const T r2 = x * x + y * y + z * z;
  // sectoral value and gradient (z component of a sectoral gradient is 0)
  T sc = T(1), ss = T(0), scx = T(0), scy = T(0), ssx = T(0), ssy = T(0);
#pragma unroll
  for (int m = 0; m <= P; ++m) {
    if (m == 1) {
      sc = x * T(0.5);
      ss = -y * T(0.5);
      scx = T(0.5);
      scy = T(0);
      ssx = T(0);
      ssy = T(-0.5);
    } else if (m >= 2) {
      const T fm = T(1.0 / (2 * m));
      const T nc = (x * sc + y * ss) * fm;
      const T ns = (x * ss - y * sc) * fm;
      const T ncx = (x * scx + y * ssx + sc) * fm;
      const T ncy = (x * scy + y * ssy + ss) * fm;
      const T nsx = (x * ssx - y * scx + ss) * fm;
      const T nsy = (x * ssy - y * scy - sc) * fm;
      sc = nc; ss = ns; scx = ncx; scy = ncy; ssx = nsx; ssy = nsy;
    }
    // keep each order's reads of the callback's operands inside its band
    __builtin_amdgcn_sched_barrier(0);
    f(cidx(m, m), sc, scx, scy, T(0));
    if (m > 0) f(cidx(m, -m), ss, ssx, ssy, T(0));
    // previous two degrees for +m (c) and -m (s): value, gradient
    T c2 = T(0), c2x = T(0), c2y = T(0), c2z = T(0);
    T s2 = T(0), s2x = T(0), s2y = T(0), s2z = T(0);
    T c1 = sc, c1x = scx, c1y = scy, c1z = T(0);
    T s1 = ss, s1x = ssx, s1y = ssy, s1z = T(0);
#pragma unroll
    for (int n = m + 1; n <= P; ++n) {
      T c, cxg, cyg, czg, s, sxg, syg, szg;
      if (n == m + 1) {
        c = z * c1; cxg = z * c1x; cyg = z * c1y; czg = z * c1z + c1;
        s = z * s1; sxg = z * s1x; syg = z * s1y; szg = z * s1z + s1;
      } else {
        const T inv = T(1.0 / ((n - m) * (n + m)));
        const T a = T(2 * n - 1);
        c = (a * z * c1 - r2 * c2) * inv;
        cxg = (a * (z * c1x) - r2 * c2x - T(2) * c2 * x) * inv;
        cyg = (a * (z * c1y) - r2 * c2y - T(2) * c2 * y) * inv;
        czg = (a * (z * c1z + c1) - r2 * c2z - T(2) * c2 * z) * inv;
        s = (a * z * s1 - r2 * s2) * inv;
        sxg = (a * (z * s1x) - r2 * s2x - T(2) * s2 * x) * inv;
        syg = (a * (z * s1y) - r2 * s2y - T(2) * s2 * y) * inv;
        szg = (a * (z * s1z + s1) - r2 * s2z - T(2) * s2 * z) * inv;
      }
      f(cidx(n, m), c, cxg, cyg, czg);
      if (m > 0) f(cidx(n, -m), s, sxg, syg, szg);
      c2 = c1; c2x = c1x; c2y = c1y; c2z = c1z;
      s2 = s1; s2x = s1x; s2y = s1y; s2z = s1z;
      c1 = c; c1x = cxg; c1y = cyg; c1z = czg;
      s1 = s; s1x = sxg; s1y = syg; s1z = szg;
    }
    band_end();
  }
}

template <int P, typename T, typename F>
__device__ __forceinline__ void basis_with_gradient(T x, T y, T z, F&& f) {
  basis_with_gradient<P, T>(x, y, z, f, [] {});
}

// Neumaier's compensated addition: s + c carries the running sum.
template <typename T>
__device__ __forceinline__ void neumaier(T& s, T& c, T x) {
  const T t = s + x;
  c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
  s = t;
}

// Regular basis values R-hat^m_n only, in the order-major sweeps of
// basis_with_gradient (the same recursions, the same values); calls f(n, k,
// value) and band_end() after the last coefficient of every order m.
template <int P, typename T, typename F, typename E>
__device__ __forceinline__ void basis_values_bands(T x, T y, T z, F&& f, E&& band_end) {
  const T r2 = x * x + y * y + z * z;
  T sc = T(1), ss = T(0);
#pragma unroll
  for (int m = 0; m <= P; ++m) {
    if (m == 1) {
      sc = x * T(0.5);
      ss = -y * T(0.5);
    } else if (m >= 2) {
      const T fm = T(1.0 / (2 * m));
      const T nc = (x * sc + y * ss) * fm;
      const T ns = (x * ss - y * sc) * fm;
      sc = nc;
      ss = ns;
    }
    __builtin_amdgcn_sched_barrier(0);
    f(m, cidx(m, m), sc);
    if (m > 0) f(m, cidx(m, -m), ss);
    T c2 = T(0), s2 = T(0), c1 = sc, s1 = ss;
#pragma unroll
    for (int n = m + 1; n <= P; ++n) {
      T c, s;
      if (n == m + 1) {
        c = z * c1;
        s = z * s1;
      } else {
        const T inv = T(1.0 / ((n - m) * (n + m)));
        const T a = T(2 * n - 1);
        c = (a * z * c1 - r2 * c2) * inv;
        s = (a * z * s1 - r2 * s2) * inv;
      }
      f(n, cidx(n, m), c);
      if (m > 0) f(n, cidx(n, -m), s);
      c2 = c1;
      s2 = s1;
      c1 = c;
      s1 = s;
    }
    band_end();
  }
}

// Gradient expansions of a local expansion: with u = sum_k w[k] R-hat_k,
// grad u = sum over degrees <= P-1 of (gx[k], gy[k], gz[k]) R-hat_k.  The
// regular basis of these recursions satisfies d/dz R_n^m = R_{n-1}^m and
// (d/dx + i d/dy) R_n^m = R_{n-1}^{m-1}, (d/dx - i d/dy) R_n^m = -R_{n-1}^{m+1}
// (R_n^m = cos part + i sin part for m >= 0, App. A.1), so every gradient
// coefficient of degree d and order m' is one or two coefficients of degree
// d + 1, orders m' +- 1, times +-1/2 (or +-1 next to order 0).  Entry k of
// g (k < P^2) for k = 0 .. P^2 - 1: gx, gy, gz.
template <int P, typename T>
__device__ __forceinline__ void grad_coeff(const T* __restrict__ w, int k, T& gx, T& gy, T& gz) {
  int d = 0;
  while ((d + 1) * (d + 1) <= k) ++d;
  const int m = k - d * d - d;  // signed order, |m| <= d
  const int am = m < 0 ? -m : m;
  const int n = d + 1;
  const T h = T(0.5);
  gz = w[cidx(n, m)];
  if (m >= 0) {  // cos part of order am
    const T up = w[cidx(n, am + 1)], ups = w[cidx(n, -(am + 1))];
    if (am == 0) {
      gx = h * up;
      gy = -(h * ups);
    } else if (am == 1) {
      gx = h * up - w[cidx(n, 0)];
      gy = -(h * ups);
    } else {
      gx = h * up - h * w[cidx(n, am - 1)];
      gy = -(h * ups) - h * w[cidx(n, -(am - 1))];
    }
  } else {  // sin part of order am >= 1
    const T up = w[cidx(n, am + 1)], ups = w[cidx(n, -(am + 1))];
    if (am == 1) {
      gx = h * ups;
      gy = h * up + w[cidx(n, 0)];
    } else {
      gx = h * ups - h * w[cidx(n, -(am - 1))];
      gy = h * up + h * w[cidx(n, am - 1)];
    }
  }
}

// pot = sum_k w[k] R-hat_k and grad = sum_k g[.][k] R-hat_k (g from
// grad_coeff, degrees <= P-1) over one value sweep of the basis.  In FP32
// the terms of each order m are summed on their own and the order sums are
// added with Neumaier compensation.
template <int P, typename T>
__device__ __forceinline__ void local_eval_grad(T x, T y, T z, const T* __restrict__ w,
                                                const T* __restrict__ gxw,
                                                const T* __restrict__ gyw,
                                                const T* __restrict__ gzw, T& pot, T& gx,
                                                T& gy, T& gz) {
  constexpr bool kComp = sizeof(T) == 4;
  T bp = T(0), bx = T(0), by = T(0), bz = T(0);
  T cp = T(0), cx = T(0), cy = T(0), cz = T(0);
  T& ap = kComp ? bp : pot;
  T& ax = kComp ? bx : gx;
  T& ay = kComp ? by : gy;
  T& az = kComp ? bz : gz;
  basis_values_bands<P, T>(
      x, y, z,
      [&](int n, int k, T v) {
        ap = fma(w[k], v, ap);
        if (n < P) {
          ax = fma(gxw[k], v, ax);
          ay = fma(gyw[k], v, ay);
          az = fma(gzw[k], v, az);
        }
      },
      [&] {
        if (kComp) {
          neumaier(pot, cp, bp);
          neumaier(gx, cx, bx);
          neumaier(gy, cy, by);
          neumaier(gz, cz, bz);
          bp = bx = by = bz = T(0);
        }
      });
  if (kComp) {
    pot += cp;
    gx += cx;
    gy += cy;
    gz += cz;
  }
}


// ---------------------------------------------------------------- P2P
__device__ __forceinline__ double inv_sqrt(double r2) {
  // hardware estimate refined by one Newton step
  const double y = __builtin_amdgcn_rsq(r2);
  return y * fma(-0.5 * r2, y * y, 1.5);
}
__device__ __forceinline__ float inv_sqrt(float r2) { return __builtin_amdgcn_rsqf(r2); }

// ------------------------------------------------------ M2L partial sums
// D[t][0..W) = sum over the M2L work items of box t (in item order) of
// their partial rows, for every box t in boxes[0..nb): one block per box,
// threads over the row.  The far-field local of every box starts here; the
// level-by-level L2L kernels then add the translated parent local.
template <typename T>
__global__ void k_psum(int64_t nb, const int32_t* __restrict__ boxes,
                       const int32_t* __restrict__ item_first, const int32_t* __restrict__ item_cnt,
                       const T* __restrict__ partial, int W, T* __restrict__ D) {
  const int64_t t = boxes[blockIdx.x];
  const int b = item_first[t], e = b + item_cnt[t];
  for (int k = threadIdx.x; k < W; k += blockDim.x) {
    T acc = T(0);
    int it = b;
    // four rows' loads in flight at a time; the sum keeps item order
    for (; it + 4 <= e; it += 4) {
      const T r0 = partial[(int64_t)it * W + k], r1 = partial[(int64_t)(it + 1) * W + k];
      const T r2 = partial[(int64_t)(it + 2) * W + k], r3 = partial[(int64_t)(it + 3) * W + k];
      acc += r0;
      acc += r1;
      acc += r2;
      acc += r3;
    }
    for (; it < e; ++it) acc += partial[(int64_t)it * W + k];
    D[t * W + k] = acc;
  }
}

// ------------------------------------------------------ block placement
// Workgroups are handed to the 8 XCDs round robin (block b to XCD b % 8),
// each XCD with its own L2.  This maps block b to a logical index so that
// every XCD works through one contiguous range of the logical blocks, and
// neighbouring work (which shares expansions and source points) shares an
// L2.  A bijection on [0, nb) for any nb.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  constexpr unsigned kXcd = 8;
  const unsigned q = nb / kXcd, r = nb % kXcd;
  const unsigned x = b % kXcd, j = b / kXcd;
  return x * q + (x < r ? x : r) + j;
}

// The same for blocks of unequal cost: logical blocks go to the XCDs in
// chunks of K consecutive ones, chunk c to XCD c % 8, so that neighbours
// still share an L2 while runs of expensive blocks spread over all XCDs;
// the tail that does not fill a round of 8 chunks is placed as xcd_block
// places it.  A bijection of [0, nb).
template <unsigned K>
__device__ __forceinline__ unsigned xcd_chunked(unsigned b, unsigned nb) {
  constexpr unsigned kXcd = 8;
  const unsigned full = nb / (kXcd * K);  // complete rounds
  const unsigned x = b % kXcd, j = b / kXcd;
  if (j < full * K) return ((j / K) * kXcd + x) * K + j % K;
  const unsigned base = full * kXcd * K;
  return base + xcd_block(b - base, nb - base);
}

// ------------------------------------------------------ lane reductions
// Cross-lane moves through the VALU's data-parallel primitives (no LDS).
// CTRL: quad_perm / row_mirror / row_bcast selector; RM: rows written (the
// others receive 0).
template <int CTRL, int RM = 0xF>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, RM, 0xF, false));
}
template <int CTRL, int RM = 0xF>
__device__ __forceinline__ double dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, RM, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, RM, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over each aligned group of LW lanes (LW a power of two <= 64), in a
// fixed order; the result is valid in the last lane of every group.
template <int LW, typename T>
__device__ __forceinline__ T group_sum(T v) {
  if (LW >= 2) v += dpp<0xB1>(v);        // quad_perm [1,0,3,2]: lane ^ 1
  if (LW >= 4) v += dpp<0x4E>(v);        // quad_perm [2,3,0,1]: lane ^ 2
  if (LW >= 8) v += dpp<0x141>(v);       // row_half_mirror: other quad of 8
  if (LW >= 16) v += dpp<0x140>(v);      // row_mirror: other half of 16
  if (LW >= 32) v += dpp<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
  if (LW >= 64) v += dpp<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
  return v;
}



}  // namespace ops
}  // namespace fmm
