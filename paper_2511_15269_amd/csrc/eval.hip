// FMM evaluation pass (stage order of Sec. III.A: sort, P2M, M2M, M2L, L2L,
// L2P, P2P), hand-written HIP kernels for gfx950.
//
// Coefficients are kept normalised (tables.h) and scaled per box by its
// radius rho (multipole degree n divided by rho^n, local degree n multiplied
// by rho^{n+1}), box-major: [box][(P+1)^2].  With this scaling every
// translation below multiplies by ratios of lengths that are at most 1
// (child/parent radius, centre offset/parent radius, radius/distance of an
// admissible pair), so single precision cannot overflow.
// All translations are rotation based (Sec. II.D, App. B): for a shift from
// an old centre to a new one with b = old - new = r (sin B cos A,
// sin B sin A, cos B), the coefficients are rotated so that b points along
// +z, shifted with the diagonal z-axis operators of App. B.3 and rotated
// back.  The rotation about y by B is factored as
//   Rz(-pi/2) Ry(-pi/2) Rz(B) Ry(pi/2) Rz(pi/2)
// so each interaction needs four products with the fixed per-degree block
// Y_n (or its transpose) and azimuthal 2x2 rotations (App. B.1) by angles
// built from A and B; the Rz(+-pi/2) next to the z-axis operator cancel
// because that operator commutes with rotations about z.  One thread owns
// one interaction (all of its coefficients sit in registers); the operator
// tables are wave-uniform and are read through the scalar cache.
//
//   M2L item: thread = (target box, up to 16 of its sources); partial sums
//             are added per target in a fixed order by the L2L kernel, so
//             results do not depend on scheduling (no atomics).
//   M2M:      thread = child box; the 2^s children of a parent sit in
//             adjacent lanes and are summed with cross-lane shuffles.
//   L2L:      thread = box of the level; adds its M2L partials and the
//             shifted local expansion of its parent.
//   P2M:      block = leaf, thread = point, LDS reduction over points.
//   L2P:      block = target leaf, thread = target point; writes outputs.
//   P2P:      block = target leaf, thread = target point; adds the near
//             field; the source points of the direct list are read with
//             wave-uniform (scalar) loads.
#include <cmath>

#include "internal.h"
#include "tables.h"

namespace fmm {
namespace {

constexpr double kInv4Pi = 0.079577471545947667884441881686257181;
constexpr int kM2LThreads = 64;

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

// cos(m g), sin(m g), m = 0..P, by repeated complex multiplication
template <int P, typename T>
__device__ __forceinline__ void powers(T c1, T s1, T* c, T* s) {
  c[0] = T(1);
  s[0] = T(0);
#pragma unroll
  for (int m = 1; m <= P; ++m) {
    c[m] = c[m - 1] * c1 - s[m - 1] * s1;
    s[m] = s[m - 1] * c1 + c[m - 1] * s1;
  }
}

// (v^m, v^{-m}) <- (a c + b s, b c - a s) for every degree, with
// (c, s) = (cm[m], sgn * sm[m]) after the quarter-turn shift q (m*q*pi/2
// added to the angle; q in {0, 1}): q = 1 maps (cos ma, sin ma) to
// (cos m(pi/2 - a), sin m(pi/2 - a)).
template <int P, typename T, int SGN, int Q>
__device__ __forceinline__ void azimuth(T* v, const T* cm, const T* sm) {
#pragma unroll
  for (int m = 1; m <= P; ++m) {
    T c, s;
    if (Q == 0) {
      c = cm[m];
      s = sm[m];
    } else {
      switch (m & 3) {
        case 0: c = cm[m]; s = -sm[m]; break;
        case 1: c = sm[m]; s = cm[m]; break;
        case 2: c = -cm[m]; s = sm[m]; break;
        default: c = -sm[m]; s = -cm[m]; break;
      }
    }
    if (SGN < 0) s = -s;
#pragma unroll
    for (int n = m; n <= P; ++n) {
      T a = v[cidx(n, m)], b = v[cidx(n, -m)];
      v[cidx(n, m)] = a * c + b * s;
      v[cidx(n, -m)] = b * c - a * s;
    }
  }
}

// v_n <- Y_n v_n (TR: Y_n^T v_n) over the stored nonzero entries
template <int P, bool TR, typename T>
__device__ __forceinline__ void apply_y(T* v, const T* __restrict__ tab) {
#pragma unroll
  for (int n = 1; n <= P; ++n) {
    cptr<T> Y = local_ptr(tab) + (TR ? tab_yt(P) : tab_y(P)) + ycbase(n);
    T u[2 * P + 1];
    int o = 0;
#pragma unroll
    for (int a = -n; a <= n; ++a) {
      T acc = T(0);
#pragma unroll
      for (int b = -n; b <= n; ++b) {
        if (!ynz(n, a, b)) continue;
        acc = fma(Y[o], v[cidx(n, b)], acc);
        ++o;
      }
      u[a + n] = acc;
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
template <int P, int KIND, typename T>
__device__ __forceinline__ void zshift(T* v, T a, T b, const T* __restrict__ tab) {
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
      for (int m = -n; m <= n; ++m) v[cidx(n, m)] *= pa[n];
#pragma unroll
    for (int m = -P; m <= P; ++m) {
      const int am = m < 0 ? -m : m;
      cptr<T> tb = local_ptr(tab) + tab_tm2l(P) + zl_base(P, am);
      T o[P + 1];
      int c = 0;
#pragma unroll
      for (int n = am; n <= P; ++n) {
        T acc = T(0);
#pragma unroll
        for (int k = am; k <= P; ++k) acc = fma(tb[c++], v[cidx(k, m)], acc);
        o[n] = acc * pb[n + 1];
      }
#pragma unroll
      for (int n = am; n <= P; ++n) v[cidx(n, m)] = m < 0 ? -o[n] : o[n];
    }
  } else {
    if (KIND == kM2M) {
#pragma unroll
      for (int n = 0; n <= P; ++n)
#pragma unroll
        for (int m = -n; m <= n; ++m) v[cidx(n, m)] *= pb[n];
    }
#pragma unroll
    for (int m = -P; m <= P; ++m) {
      const int am = m < 0 ? -m : m;
      cptr<T> tb = local_ptr(tab) + (KIND == kM2M ? tab_tm2m(P) : tab_tl2l(P)) + zt_base(P, am);
      T o[P + 1];
      int c = 0;
#pragma unroll
      for (int n = am; n <= P; ++n) {
        T acc = T(0);
        if (KIND == kM2M) {
#pragma unroll
          for (int k = am; k <= n; ++k) acc = fma(tb[c++] * pa[n - k], v[cidx(k, m)], acc);
        } else {
#pragma unroll
          for (int k = n; k <= P; ++k) acc = fma(tb[c++] * pa[k - n], v[cidx(k, m)], acc);
          acc *= pb[n + 1];
        }
        o[n] = acc;
      }
#pragma unroll
      for (int n = am; n <= P; ++n) v[cidx(n, m)] = o[n];
    }
  }
}

// Rotate so that b points along +z, shift along z, rotate back.
// b = old centre - new centre; rho_old, rho_new the scale lengths of the
// two boxes.  M2L maps multipole (regular-basis sign convention) to local
// (singular-basis convention); M2M keeps the former, L2L the latter.
template <int P, int KIND, typename T>
__device__ __forceinline__ void rotate_shift(T* v, double bx, double by, double bz,
                                             double rho_old, double rho_new,
                                             const T* __restrict__ tab) {
  const double rxy2 = bx * bx + by * by;
  const double rxy = sqrt(rxy2);
  const double r = sqrt(rxy2 + bz * bz);
  double ca = 1.0, sa = 0.0, cb = 1.0, sb = 0.0;
  if (rxy > 0.0) {
    ca = bx / rxy;
    sa = by / rxy;
  }
  if (r > 0.0) {
    cb = bz / r;
    sb = rxy / r;
  }
  double a, b;
  if (KIND == kM2L) {
    a = rho_old / r;
    b = rho_new / r;
  } else if (KIND == kM2M) {
    a = r / rho_new;
    b = rho_old / rho_new;
  } else {
    a = r / rho_old;
    b = rho_new / rho_old;
  }
  T am_c[P + 1], am_s[P + 1], bm_c[P + 1], bm_s[P + 1];
  powers<P, T>(T(ca), T(sa), am_c, am_s);
  powers<P, T>(T(cb), T(sb), bm_c, bm_s);
  // forward: Rz(pi/2 - A), Y, Rz(-B), Y^T   (sign conventions per kind)
  if (KIND == kL2L)
    azimuth<P, T, -1, 1>(v, am_c, am_s);
  else
    azimuth<P, T, +1, 1>(v, am_c, am_s);
  apply_y<P, false, T>(v, tab);
  if (KIND == kL2L)
    azimuth<P, T, +1, 0>(v, bm_c, bm_s);
  else
    azimuth<P, T, -1, 0>(v, bm_c, bm_s);
  apply_y<P, true, T>(v, tab);
  zshift<P, KIND, T>(v, T(a), T(b), tab);
  // back: Y, Rz(B), Y^T, Rz(A - pi/2)
  apply_y<P, false, T>(v, tab);
  if (KIND == kM2M)
    azimuth<P, T, +1, 0>(v, bm_c, bm_s);
  else
    azimuth<P, T, -1, 0>(v, bm_c, bm_s);
  apply_y<P, true, T>(v, tab);
  if (KIND == kM2M)
    azimuth<P, T, -1, 1>(v, am_c, am_s);
  else
    azimuth<P, T, +1, 1>(v, am_c, am_s);
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

// ---------------------------------------------------------------- P2M
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

// C_leaf = normc * sum_i q_i R-hat((x_i - c) / rho)  (scaled multipole)
template <int P, typename T>
__global__ __launch_bounds__(64) void k_p2m(
    int64_t leaf_box0, const int32_t* __restrict__ leaf_start,
    const double* __restrict__ xs, const double* __restrict__ ys,
    const double* __restrict__ zs, const Src<T>* __restrict__ src,
    const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const T* __restrict__ tab, T* __restrict__ C) {
  constexpr int K = K_<P>::value;
  __shared__ T red[K][65];
  const int leaf = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t g = leaf_box0 + leaf;
  const int st = leaf_start[leaf], en = leaf_start[leaf + 1];
  T acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = T(0);
  const double ox = cx[g], oy = cy[g], oz = cz[g], ir = 1.0 / scale[g];
  for (int j = st + lane; j < en; j += 64) {
    const T qj = src[j].q;
    regular_basis<P, T>(T((xs[j] - ox) * ir), T((ys[j] - oy) * ir), T((zs[j] - oz) * ir),
                        [&](int k, T v) { acc[k] = fma(qj, v, acc[k]); });
  }
#pragma unroll
  for (int k = 0; k < K; ++k) red[k][lane] = acc[k];
  __syncthreads();
  for (int k = lane; k < K; k += 64) {
    T s = T(0);
    for (int l = 0; l < 64; ++l) s += red[k][l];
    C[g * K + k] = s * tab[tab_normc(P) + k];
  }
}

// ---------------------------------------------------------------- M2M
template <int P, typename T>
__global__ __launch_bounds__(64) void k_m2m(
    int64_t nchild, int64_t child0, int64_t parent0, int s,
    const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const T* __restrict__ tab, T* C) {
  constexpr int K = K_<P>::value;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < nchild;
  const int64_t c = child0 + (live ? i : 0);
  const int64_t pa = parent0 + ((live ? i : 0) >> s);
  T v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = live ? C[c * K + k] : T(0);
  rotate_shift<P, kM2M, T>(v, cx[c] - cx[pa], cy[c] - cy[pa], cz[c] - cz[pa], scale[c],
                           scale[pa], tab);
  const int nch = 1 << s;
  for (int off = 1; off < nch; off <<= 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += __shfl_xor(v[k], off, 64);
  }
  if (live && (i & (nch - 1)) == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) C[pa * K + k] = v[k];
  }
}

// ---------------------------------------------------------------- M2L
template <int P, typename T>
__global__ __launch_bounds__(kM2LThreads) void k_m2l(
    int64_t nitems, const int32_t* __restrict__ item_tgt,
    const int32_t* __restrict__ item_begin, const int32_t* __restrict__ item_end,
    const int32_t* __restrict__ src, const double* __restrict__ cx,
    const double* __restrict__ cy, const double* __restrict__ cz,
    const double* __restrict__ scale, const T* __restrict__ C,
    const T* __restrict__ tab, T* __restrict__ partial) {
  constexpr int K = K_<P>::value;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nitems) return;
  const int t = item_tgt[i];
  const int jb = item_begin[i], je = item_end[i];
  const double tx = cx[t], ty = cy[t], tz = cz[t], rt = scale[t];
  T acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = T(0);
  for (int j = jb; j < je; ++j) {
    const int sidx = src[j];
    T v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = C[(int64_t)sidx * K + k];
    rotate_shift<P, kM2L, T>(v, cx[sidx] - tx, cy[sidx] - ty, cz[sidx] - tz, scale[sidx], rt,
                             tab);
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += v[k];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) partial[i * K + k] = acc[k];
}

// ---------------------------------------------------------------- L2L
// D_t = (M2L partials of t, in item order) + L2L(D_parent)
template <int P, typename T>
__global__ __launch_bounds__(64) void k_l2l(
    int64_t nb, int64_t box0, int64_t parent0, int s,
    const int32_t* __restrict__ item_ptr, const T* __restrict__ partial,
    const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const T* __restrict__ tab, T* D) {
  constexpr int K = K_<P>::value;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int64_t t = box0 + i;
  T acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = T(0);
  for (int it = item_ptr[t]; it < item_ptr[t + 1]; ++it) {
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += partial[(int64_t)it * K + k];
  }
  if (parent0 >= 0) {
    const int64_t pa = parent0 + (i >> s);
    T v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = D[pa * K + k];
    rotate_shift<P, kL2L, T>(v, cx[pa] - cx[t], cy[pa] - cy[t], cz[pa] - cz[t], scale[pa],
                             scale[t], tab);
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += v[k];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) D[t * K + k] = acc[k];
}

// ---------------------------------------------------------------- L2P
// Regular basis and its gradient (App. A.1, A.3; the sectoral gradient
// without the printed leading minus), accumulated against w[k] = weight *
// local coefficient: pot += w R, grad += w grad R.
template <int P, typename T>
__device__ __forceinline__ void local_eval(T x, T y, T z, const T* __restrict__ w,
                                           T& pot, T& gx, T& gy, T& gz) {
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
      const T f = T(1.0 / (2 * m));
      const T nc = (x * sc + y * ss) * f;
      const T ns = (x * ss - y * sc) * f;
      const T ncx = (x * scx + y * ssx + sc) * f;
      const T ncy = (x * scy + y * ssy + ss) * f;
      const T nsx = (x * ssx - y * scx + ss) * f;
      const T nsy = (x * ssy - y * scy - sc) * f;
      sc = nc; ss = ns; scx = ncx; scy = ncy; ssx = nsx; ssy = nsy;
    }
    {
      const T wc = w[cidx(m, m)];
      pot = fma(wc, sc, pot);
      gx = fma(wc, scx, gx);
      gy = fma(wc, scy, gy);
      if (m > 0) {
        const T ws = w[cidx(m, -m)];
        pot = fma(ws, ss, pot);
        gx = fma(ws, ssx, gx);
        gy = fma(ws, ssy, gy);
      }
    }
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
      const T wc = w[cidx(n, m)];
      pot = fma(wc, c, pot);
      gx = fma(wc, cxg, gx);
      gy = fma(wc, cyg, gy);
      gz = fma(wc, czg, gz);
      if (m > 0) {
        const T ws = w[cidx(n, -m)];
        pot = fma(ws, s, pot);
        gx = fma(ws, sxg, gx);
        gy = fma(ws, syg, gy);
        gz = fma(ws, szg, gz);
      }
      c2 = c1; c2x = c1x; c2y = c1y; c2z = c1z;
      s2 = s1; s2x = s1x; s2y = s1y; s2z = s1z;
      c1 = c; c1x = cxg; c1y = cyg; c1z = czg;
      s1 = s; s1x = sxg; s1y = syg; s1z = szg;
    }
  }
}

// L2P: u = -1/(4 pi) (1/rho) sum w_m D R-hat(y), y = (x - c)/rho, and
// field = -grad u (an extra 1/rho from the chain rule), at every point of the
// target leaf; writes (not adds) the outputs in input order.
template <int P, typename T, bool FIELD>
__global__ __launch_bounds__(64) void k_l2p(
    int64_t leaf_box0, const int32_t* __restrict__ leaf_start,
    const int32_t* __restrict__ perm, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs,
    const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const T* __restrict__ D, const T* __restrict__ tab, T* __restrict__ pot,
    T* __restrict__ field) {
  constexpr int K = K_<P>::value;
  __shared__ T w[K];
  const int leaf = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t g = leaf_box0 + leaf;
  for (int k = lane; k < K; k += 64) w[k] = D[g * K + k] * tab[tab_l2p(P) + k];
  __syncthreads();
  const int st = leaf_start[leaf], en = leaf_start[leaf + 1];
  const double ox = cx[g], oy = cy[g], oz = cz[g], ir = 1.0 / scale[g];
  const T fu = T(-kInv4Pi * ir), ff = T(kInv4Pi * ir * ir);
  for (int i = st + lane; i < en; i += 64) {
    T fp = T(0), fx = T(0), fy = T(0), fz = T(0);
    local_eval<P, T>(T((xs[i] - ox) * ir), T((ys[i] - oy) * ir), T((zs[i] - oz) * ir), w, fp,
                     fx, fy, fz);
    const int o = perm[i];
    pot[o] = fu * fp;
    if (FIELD) {
      field[3 * (int64_t)o + 0] = ff * fx;
      field[3 * (int64_t)o + 1] = ff * fy;
      field[3 * (int64_t)o + 2] = ff * fz;
    }
  }
}

// ---------------------------------------------------------------- P2P
__device__ __forceinline__ double inv_sqrt(double r2) {
  // hardware estimate refined by one Newton step
  const double y = __builtin_amdgcn_rsq(r2);
  return y * fma(-0.5 * r2, y * y, 1.5);
}
__device__ __forceinline__ float inv_sqrt(float r2) { return __builtin_amdgcn_rsqf(r2); }

// Neumaier's compensated addition: s + c carries the running sum.
template <typename T>
__device__ __forceinline__ void neumaier(T& s, T& c, T x) {
  const T t = s + x;
  c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
  s = t;
}

// One source point against the lane's target at (xi, yi, zi): the
// difference is taken in FP64 and rounded to T; pairs at distance 0
// contribute nothing.
template <typename T, bool FIELD>
__device__ __forceinline__ void p2p_pair(const Src<T>& s, double xi, double yi, double zi,
                                         T& u, T& gx, T& gy, T& gz) {
  const T dx = T(xi - s.x), dy = T(yi - s.y), dz = T(zi - s.z);
  const T r2 = dx * dx + dy * dy + dz * dz;
  const T inv0 = inv_sqrt(r2);
  const T inv = r2 > T(0) ? inv0 : T(0);
  const T qi = s.q * inv;
  u += qi;
  if (FIELD) {
    const T q3 = qi * inv * inv;
    gx = fma(q3, dx, gx);
    gy = fma(q3, dy, gy);
    gz = fma(q3, dz, gz);
  }
}

constexpr int kChunk = 8;

// P2P: adds -1/(4 pi) sum q/r and the matching field over the direct list.
// Block = target leaf, lane = target point.  G source groups: lanes
// [g*64/G, (g+1)*64/G) share targets with the other groups but walk every
// G-th source point starting at point g.  G = 1 keeps all source reads
// wave-uniform (scalar loads); G = 2, 4 fill the wave when leaves hold at
// most 32 or 16 points.  Per source leaf the partial sums are added to the
// running sums with Neumaier compensation (FP32 form); group sums are then
// combined with cross-lane shuffles in a fixed order.
template <typename T, bool FIELD, int G>
__global__ __launch_bounds__(64) void k_p2p(
    int64_t leaf_box0, const int32_t* __restrict__ leaf_start,
    const int32_t* __restrict__ perm, const Src<T>* __restrict__ src,
    const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const int32_t* __restrict__ p2p_ptr, const int32_t* __restrict__ p2p_src,
    T* __restrict__ pot, T* __restrict__ field) {
  constexpr int TL = 64 / G;  // targets per pass
  constexpr bool kComp = sizeof(T) == 4;  // FP32: compensated sums
  const int leaf = blockIdx.x;
  const int lane = threadIdx.x;
  const int g = G == 1 ? 0 : lane / TL;
  const int st = leaf_start[leaf], en = leaf_start[leaf + 1];
  const int pb = p2p_ptr[leaf], pe = p2p_ptr[leaf + 1];
  for (int i0 = st; i0 < en; i0 += TL) {
    const int i = i0 + lane % TL;
    const bool live = i < en;
    const Src<T> a = src[live ? i : st];
    T u = T(0), gx = T(0), gy = T(0), gz = T(0);
    T cu = T(0), cgx = T(0), cgy = T(0), cgz = T(0);
    for (int k = pb; k < pe; ++k) {
      const int sl = p2p_src[k];
      const int js = leaf_start[sl], cnt = leaf_start[sl + 1] - js;
      T lu = T(0), lx = T(0), ly = T(0), lz = T(0);
      const int full = cnt / G;  // points per group present in every group
      const Src<T>* base = src + js + g;
      int c = 0;
      for (; c + kChunk <= full; c += kChunk) {
        Src<T> r[kChunk];
#pragma unroll
        for (int t = 0; t < kChunk; ++t) r[t] = base[(c + t) * G];
#pragma unroll
        for (int t = 0; t < kChunk; ++t) p2p_pair<T, FIELD>(r[t], a.x, a.y, a.z, lu, lx, ly, lz);
      }
      for (; c < full; ++c) p2p_pair<T, FIELD>(base[c * G], a.x, a.y, a.z, lu, lx, ly, lz);
      if (G > 1 && g < cnt - full * G)
        p2p_pair<T, FIELD>(base[full * G], a.x, a.y, a.z, lu, lx, ly, lz);
      if (kComp) {
        neumaier(u, cu, lu);
        if (FIELD) {
          neumaier(gx, cgx, lx);
          neumaier(gy, cgy, ly);
          neumaier(gz, cgz, lz);
        }
      } else {
        u += lu;
        gx += lx;
        gy += ly;
        gz += lz;
      }
    }
    u += cu;
    gx += cgx;
    gy += cgy;
    gz += cgz;
#pragma unroll
    for (int off = TL; off < 64; off <<= 1) {
      u += __shfl_xor(u, off, 64);
      if (FIELD) {
        gx += __shfl_xor(gx, off, 64);
        gy += __shfl_xor(gy, off, 64);
        gz += __shfl_xor(gz, off, 64);
      }
    }
    if (live && g == 0) {
      const int o = perm[i];
      pot[o] += -T(kInv4Pi) * u;
      if (FIELD) {
        // field = -grad u;  grad of the near part is +(1/4pi) sum q d/r^3
        field[3 * (int64_t)o + 0] -= T(kInv4Pi) * gx;
        field[3 * (int64_t)o + 1] -= T(kInv4Pi) * gy;
        field[3 * (int64_t)o + 2] -= T(kInv4Pi) * gz;
      }
    }
  }
}

// sort stage: source records in leaf order with their charges
template <typename T>
__global__ void k_gather(int64_t n, const int32_t* __restrict__ perm,
                         const double* __restrict__ xs, const double* __restrict__ ys,
                         const double* __restrict__ zs, const T* __restrict__ q,
                         Src<T>* __restrict__ src) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) src[j] = Src<T>{xs[j], ys[j], zs[j], q[perm[j]]};
}

// d/dx_k of sum_i g_i u_i: g_k grad u(x_k) (x_k as a target of the forward
// pass) + q_k grad v(x_k) (x_k as a source, v = transposed pass with charges
// g); fields are -grad.
template <typename T>
__global__ void k_adjoint_combine(int64_t n, const T* __restrict__ q, const T* __restrict__ g,
                                  const T* __restrict__ ff, const T* __restrict__ ft,
                                  T* __restrict__ gx) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * n) return;
  const int64_t i = e / 3;
  gx[e] = -(g[i] * ff[e] + q[i] * ft[e]);
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <int P, typename T>
void run(fmm_plan* pl, const ListSet& Ls, const T* q, T* pot, T* field, hipStream_t st) {
  const int L = pl->L, s = pl->s;
  const T* tab = (const T*)pl->tables;
  Src<T>* src = (Src<T>*)pl->src;
  T* C = (T*)pl->C;
  T* D = (T*)pl->D;
  T* part = (T*)pl->partial;
  const int64_t n = pl->n;
  const int64_t leaf0 = pl->level_off[L];
  std::vector<hipEvent_t>* row = nullptr;
  if (pl->profiling) {
    pl->ev_rows.emplace_back();
    row = &pl->ev_rows.back();
    for (int k = 0; k <= FMM_NSTAGES; ++k) row->push_back(take_event(pl));
  }
  auto mark = [&](int k) {
    if (row) FMM_HIP(hipEventRecord((*row)[k], st));
  };
  mark(0);
  k_gather<T><<<blocks(n, 256), 256, 0, st>>>(n, pl->perm, pl->xs, pl->ys, pl->zs, q, src);
  mark(1);
  k_p2m<P, T><<<(unsigned)pl->nleaf, 64, 0, st>>>(leaf0, pl->leaf_start, pl->xs, pl->ys, pl->zs,
                                                  src, pl->cx, pl->cy, pl->cz, pl->scale, tab, C);
  mark(2);
  for (int l = L - 1; l >= 0; --l) {
    const int64_t nchild = pl->level_off[l + 2] - pl->level_off[l + 1];
    k_m2m<P, T><<<blocks(nchild, 64), 64, 0, st>>>(nchild, pl->level_off[l + 1], pl->level_off[l],
                                                   s, pl->cx, pl->cy, pl->cz, pl->scale, tab, C);
  }
  mark(3);
  if (Ls.n_items > 0)
    k_m2l<P, T><<<blocks(Ls.n_items, kM2LThreads), kM2LThreads, 0, st>>>(
        Ls.n_items, Ls.item_tgt, Ls.item_begin, Ls.item_end, Ls.m2l_src, pl->cx, pl->cy,
        pl->cz, pl->scale, C, tab, part);
  mark(4);
  for (int l = 0; l <= L; ++l) {
    const int64_t nb = pl->level_off[l + 1] - pl->level_off[l];
    k_l2l<P, T><<<blocks(nb, 64), 64, 0, st>>>(nb, pl->level_off[l],
                                               l > 0 ? pl->level_off[l - 1] : -1, s,
                                               Ls.item_ptr, part, pl->cx, pl->cy, pl->cz,
                                               pl->scale, tab, D);
  }
  mark(5);
  if (field)
    k_l2p<P, T, true><<<(unsigned)pl->nleaf, 64, 0, st>>>(
        leaf0, pl->leaf_start, pl->perm, pl->xs, pl->ys, pl->zs, pl->cx, pl->cy, pl->cz,
        pl->scale, D, tab, pot, field);
  else
    k_l2p<P, T, false><<<(unsigned)pl->nleaf, 64, 0, st>>>(
        leaf0, pl->leaf_start, pl->perm, pl->xs, pl->ys, pl->zs, pl->cx, pl->cy, pl->cz,
        pl->scale, D, tab, pot, field);
  mark(6);
  const int G = pl->max_leaf_count > 32 ? 1 : (pl->max_leaf_count > 16 ? 2 : 4);
  auto p2p = [&](auto kern) {
    kern<<<(unsigned)pl->nleaf, 64, 0, st>>>(leaf0, pl->leaf_start, pl->perm, src, pl->cx,
                                              pl->cy, pl->cz, pl->scale, Ls.p2p_ptr,
                                              Ls.p2p_src, pot, field);
  };
  if (field) {
    if (G == 1) p2p(k_p2p<T, true, 1>);
    else if (G == 2) p2p(k_p2p<T, true, 2>);
    else p2p(k_p2p<T, true, 4>);
  } else {
    if (G == 1) p2p(k_p2p<T, false, 1>);
    else if (G == 2) p2p(k_p2p<T, false, 2>);
    else p2p(k_p2p<T, false, 4>);
  }
  mark(7);
  FMM_HIP(hipGetLastError());
}

template <typename T>
void dispatch(int p, fmm_plan* pl, const ListSet& Ls, const T* q, T* pot, T* field,
              hipStream_t st) {
  switch (p) {
#define FMM_CASE(PP) \
  case PP:           \
    run<PP, T>(pl, Ls, q, pot, field, st); \
    break;
    FMM_CASE(1) FMM_CASE(2) FMM_CASE(3) FMM_CASE(4) FMM_CASE(5)
    FMM_CASE(6) FMM_CASE(7) FMM_CASE(8) FMM_CASE(9) FMM_CASE(10)
#undef FMM_CASE
    default:
      throw Error{FMM_ENOTSUP, "expansion order without compiled kernels"};
  }
}

}  // namespace

void evaluate(fmm_plan* pl, int dir, const void* q, int nrhs, void* pot, void* field,
              hipStream_t st) {
  const int64_t n = pl->n;
  const ListSet& Ls = pl->lists[dir];
  for (int r = 0; r < nrhs; ++r) {
    if (pl->prm.precision == FMM_FP32) {
      dispatch<float>(pl->prm.p, pl, Ls, (const float*)q + r * n, (float*)pot + r * n,
                      field ? (float*)field + 3 * r * n : nullptr, st);
    } else {
      dispatch<double>(pl->prm.p, pl, Ls, (const double*)q + r * n, (double*)pot + r * n,
                       field ? (double*)field + 3 * r * n : nullptr, st);
    }
  }
}

void adjoint_combine(fmm_plan* pl, const void* q, const void* g, const void* field_fwd,
                     const void* field_t, void* grad_x, hipStream_t st) {
  const int64_t n = pl->n;
  if (pl->prm.precision == FMM_FP32)
    k_adjoint_combine<float><<<blocks(3 * n, 256), 256, 0, st>>>(
        n, (const float*)q, (const float*)g, (const float*)field_fwd, (const float*)field_t,
        (float*)grad_x);
  else
    k_adjoint_combine<double><<<blocks(3 * n, 256), 256, 0, st>>>(
        n, (const double*)q, (const double*)g, (const double*)field_fwd,
        (const double*)field_t, (double*)grad_x);
  FMM_HIP(hipGetLastError());
}

}  // namespace fmm
