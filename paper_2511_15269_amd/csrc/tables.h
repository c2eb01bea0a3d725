// Layout of the constant operator tables of one expansion order P (shared by
// the host code that fills them and the kernels that read them).
//
// Coefficient vectors hold (n, m), 0 <= n <= P, -n <= m <= n, at index
// n*n + n + m.  Inside the library, multipole and local coefficients are
// kept normalised so that rotations act on them as orthogonal matrices:
//     Ct^m_n = sqrt(2 - delta_{m0}) * N_{n|m|} * C^m_n
//     Dt^m_n = sqrt(2 - delta_{m0}) / N_{n|m|} * D^m_n
// with N_{nm} = sqrt((n-m)! (n+m)!) and C, D the paper's real coefficients
// (Sec. II.C; the factor N is the N^m_{n,k} normalisation of App. B.2).
#pragma once

#define FMM_HD __host__ __device__ inline constexpr

namespace fmm {

FMM_HD int ncoef(int P) { return (P + 1) * (P + 1); }
FMM_HD int cidx(int n, int m) { return n * n + n + m; }

// Nonzero entries of the fixed rotation block Y_n (rotation about y by
// +pi/2 of normalised coefficients): rows and columns in the same
// cos (m >= 0) or sin (m < 0) block and |a| + |b| + n even (cos) or odd
// (sin).  The tables store only these, row by row, in the order the
// kernels consume them.
FMM_HD bool ynz(int n, int a, int b) {
  if ((a >= 0) != (b >= 0)) return false;
  const int par = ((a < 0 ? -a : a) + (b < 0 ? -b : b) + n) & 1;
  return a >= 0 ? par == 0 : par == 1;
}
FMM_HD int ycount(int n) { return n * n + n + 1; }
FMM_HD int ycbase(int n) {  // sum_{j<n} ycount(j)
  return (n - 1) * n * (n + 1) / 3 + n;
}
// z-axis translation coefficients per |m|, n, k (App. B.3, normalised):
// M2L has n, k in [|m|, P] (stored column by column, k outer); M2M k in
// [|m|, n] and L2L k in [n, P] (row by row, n outer).
FMM_HD int zl_base(int P, int am) {  // sum_{j<am} (P+1-j)^2
  int s = 0;
  for (int j = 0; j < am; ++j) s += (P + 1 - j) * (P + 1 - j);
  return s;
}
FMM_HD int zt_base(int P, int am) {  // sum_{j<am} (P+1-j)(P+2-j)/2
  int s = 0;
  for (int j = 0; j < am; ++j) s += (P + 1 - j) * (P + 2 - j) / 2;
  return s;
}

// [K] sqrt(2-delta) N_{n|m|}: P2M output scaling (C -> Ct)
FMM_HD int tab_normc(int) { return 0; }
// [K] sgn(m) sqrt(2-delta) N_{n|m|}: weight of Dt against R-hat in L2P
FMM_HD int tab_l2p(int P) { return ncoef(P); }
// Y_n nonzeros row by row, then Y_n^T nonzeros row by row
FMM_HD int tab_y(int P) { return 2 * ncoef(P); }
FMM_HD int tab_yt(int P) { return tab_y(P) + ycbase(P + 1); }
FMM_HD int tab_tm2l(int P) { return tab_yt(P) + ycbase(P + 1); }
FMM_HD int tab_tm2m(int P) { return tab_tm2l(P) + zl_base(P, P + 1); }
FMM_HD int tab_tl2l(int P) { return tab_tm2m(P) + zt_base(P, P + 1); }
FMM_HD int tab_size(int P) { return tab_tl2l(P) + zt_base(P, P + 1); }
// Zero entries after the last table: kernels prefetch whole 64-byte blocks
// ahead of use and may read up to this many entries past the end.
FMM_HD int tab_pad() { return 64; }

}  // namespace fmm
