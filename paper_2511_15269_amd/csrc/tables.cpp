// Constant operator tables of the rotation-based translations (host).
//
// The polar rotation of App. B.2 is applied per interaction through the
// factorisation
//     rotation about y by beta = Rz(-pi/2) . Ry(-pi/2) . Rz(beta) . Ry(pi/2) . Rz(pi/2)
// so the only dense per-degree matrices are the fixed Y_n = (rotation about
// y by +pi/2) and its transpose; all angle-dependent factors are azimuthal
// 2x2 rotations (App. B.1).  Y_n is built once per order from Wigner's
// small d^n_{m'm}(pi/2), evaluated with the three-term recurrence of Jacobi
// polynomials in the degree n (the route the paper takes for its Wigner
// matrices, Sec. II.D), seeded with the closed form at n = max(|m|,|m'|).
// In the normalised real basis (see tables.h) the blocks are
//   Y(0,0)   = d_{00}
//   Y(a,0)   = sqrt2 (-1)^a d_{a0},   Y(0,b) = sqrt2 (-1)^b d_{0b}
//   Y(a,b)   = (-1)^a [(-1)^b d_{ab} + d_{a,-b}]     (cos block, a,b > 0)
//   Y(-a,-b) = (-1)^a [(-1)^b d_{ab} - d_{a,-b}]     (sin block, a,b > 0)
// and cos and sin blocks do not mix; entries vanish unless |a|+|b|+n is even
// (cos block) or odd (sin block).  Only the nonzero entries are stored, in
// the order the kernels read them (see tables.h).
//
// z-axis translations of length r (App. B.3), normalised:
//   M2M  Ct^m_n += sum_{k=|m|}^{n} N_{n|m|}/(N_{k|m|} (n-k)!) r^{n-k} Ct^m_k
//   M2L  Dt^m_n  = sgn(m) sum_{k=|m|}^{P} (-1)^{k+m} (n+k)!/(N_{n|m|} N_{k|m|})
//                  r^{-(n+k+1)} Ct^m_k
//   L2L  Dt^m_n += sum_{k=n}^{P} (-1)^{k-n} N_{k|m|}/(N_{n|m|} (k-n)!)
//                  r^{k-n} Dt^m_k
// for a translation from old centre to new centre with
// old - new = (0, 0, r).
#include <cmath>
#include <map>
#include <mutex>

#include "internal.h"
#include "tables.h"

namespace fmm {
namespace {

double fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

double Nnm(int n, int m) {
  m = m < 0 ? -m : m;
  return std::sqrt(fact(n - m) * fact(n + m));
}

// d^n_{m'm}(beta) for n <= P, stored at [(n*(2P+1) + m'+P)*(2P+1) + m+P].
std::vector<double> wigner_d(int P, double beta) {
  const int W = 2 * P + 1;
  std::vector<double> d((size_t)(P + 1) * W * W, 0.0);
  const double c = std::cos(0.5 * beta), s = std::sin(0.5 * beta);
  const double cb = std::cos(beta);
  for (int mp = -P; mp <= P; ++mp)
    for (int m = -P; m <= P; ++m) {
      const int j0 = std::max(std::abs(mp), std::abs(m));
      auto F = [&](int a) {
        return std::sqrt(fact(2 * j0) / (fact(j0 + a) * fact(j0 - a)));
      };
      double v;
      if (j0 == mp)
        v = ((j0 - m) % 2 ? -1.0 : 1.0) * F(m) * std::pow(c, j0 + m) * std::pow(s, j0 - m);
      else if (j0 == -mp)
        v = F(m) * std::pow(c, j0 - m) * std::pow(s, j0 + m);
      else if (j0 == m)
        v = F(mp) * std::pow(c, j0 + mp) * std::pow(s, j0 - mp);
      else
        v = ((mp + j0) % 2 ? -1.0 : 1.0) * F(mp) * std::pow(c, j0 - mp) * std::pow(s, j0 + mp);
      auto at = [&](int j) -> double& { return d[((size_t)j * W + mp + P) * W + m + P]; };
      at(j0) = v;
      double prev2 = 0.0, prev1 = v;
      for (int j = j0 + 1; j <= P; ++j) {
        double cur;
        if (j == 1) {
          cur = cb * prev1;
        } else {
          double a = j * (2.0 * j - 1.0) /
                     std::sqrt((double)(j * j - m * m) * (double)(j * j - mp * mp));
          double b = std::sqrt((double)((j - 1) * (j - 1) - m * m) *
                               (double)((j - 1) * (j - 1) - mp * mp)) /
                     ((j - 1.0) * (2.0 * j - 1.0));
          cur = a * ((cb - (double)(m * mp) / (j * (j - 1.0))) * prev1 - b * prev2);
        }
        at(j) = cur;
        prev2 = prev1;
        prev1 = cur;
      }
    }
  return d;
}

std::vector<double> build(int P) {
  std::vector<double> t((size_t)(tab_size(P) + tab_pad()), 0.0);
  const double s2 = std::sqrt(2.0);
  for (int n = 0; n <= P; ++n)
    for (int m = -n; m <= n; ++m) {
      double w = (m == 0 ? 1.0 : s2) * Nnm(n, m);
      t[tab_normc(P) + cidx(n, m)] = w;
      t[tab_l2p(P) + cidx(n, m)] = (m < 0 ? -w : w);
    }
  // Y_n from d(pi/2); cos(pi/2) is exactly 0
  const int W = 2 * P + 1;
  std::vector<double> d = wigner_d(P, M_PI / 2);
  for (int n = 0; n <= P; ++n) {
    auto D = [&](int a, int b) { return d[((size_t)n * W + a + P) * W + b + P]; };
    const int w = 2 * n + 1;
    std::vector<double> Y((size_t)w * w, 0.0);
    auto at = [&](int a, int b) -> double& { return Y[(a + n) * w + (b + n)]; };
    at(0, 0) = D(0, 0);
    for (int a = 1; a <= n; ++a) {
      double sa = (a % 2) ? -1.0 : 1.0;
      at(a, 0) = s2 * sa * D(a, 0);
      at(0, a) = s2 * sa * D(0, a);
      for (int b = 1; b <= n; ++b) {
        double sb = (b % 2) ? -1.0 : 1.0;
        at(a, b) = sa * (sb * D(a, b) + D(a, -b));
        at(-a, -b) = sa * (sb * D(a, b) - D(a, -b));
      }
    }
    int o = tab_y(P) + ycbase(n), ot = tab_yt(P) + ycbase(n);
    for (int a = -n; a <= n; ++a)
      for (int b = -n; b <= n; ++b)
        if (ynz(n, a, b)) {
          t[o++] = at(a, b);
          t[ot++] = at(b, a);
        }
  }
  for (int am = 0; am <= P; ++am) {
    int o = tab_tm2l(P) + zl_base(P, am);
    for (int k = am; k <= P; ++k)  // column-major: read k by k
      for (int n = am; n <= P; ++n)
        t[o++] = (((k + am) % 2) ? -1.0 : 1.0) * fact(n + k) / (Nnm(n, am) * Nnm(k, am));
    o = tab_tm2m(P) + zt_base(P, am);
    for (int n = am; n <= P; ++n)
      for (int k = am; k <= n; ++k) t[o++] = Nnm(n, am) / (Nnm(k, am) * fact(n - k));
    o = tab_tl2l(P) + zt_base(P, am);
    for (int n = am; n <= P; ++n)
      for (int k = n; k <= P; ++k)
        t[o++] = (((k - n) % 2) ? -1.0 : 1.0) * Nnm(k, am) / (Nnm(n, am) * fact(k - n));
  }
  return t;
}

std::mutex g_mu;
std::map<std::pair<int, int>, std::pair<void*, void*>> g_tabs;  // (p, dev)

}  // namespace

const void* get_tables(int p, int precision, int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(p, device);
  auto it = g_tabs.find(key);
  if (it == g_tabs.end()) {
    std::vector<double> h = build(p);
    std::vector<float> hf(h.begin(), h.end());
    void *d64 = nullptr, *d32 = nullptr;
    FMM_HIP(hipMalloc(&d64, h.size() * sizeof(double)));
    FMM_HIP(hipMalloc(&d32, hf.size() * sizeof(float)));
    FMM_HIP(hipMemcpy(d64, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
    FMM_HIP(hipMemcpy(d32, hf.data(), hf.size() * sizeof(float), hipMemcpyHostToDevice));
    it = g_tabs.emplace(key, std::make_pair(d64, d32)).first;
  }
  return precision == FMM_FP32 ? it->second.second : it->second.first;
}

}  // namespace fmm
