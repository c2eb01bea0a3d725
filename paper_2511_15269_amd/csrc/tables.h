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

// [K] sqrt(2-delta) N_{n|m|}: P2M output scaling (C -> Ct)
FMM_HD int tab_normc(int) { return 0; }
// [K] sgn(m) sqrt(2-delta) N_{n|m|}: weight of Dt against R-hat in L2P
FMM_HD int tab_l2p(int P) { return ncoef(P); }
// dense per-degree blocks Y_n[a][b], a, b in [0, 2n+1) <-> m = a - n:
// the real rotation of normalised coefficients about the y axis by +pi/2
FMM_HD int tab_y(int P) { return 2 * ncoef(P); }
FMM_HD int ybase(int n) {  // sum_{j<n} (2j+1)^2
  return n * (4 * n * n - 1) / 3;
}
FMM_HD int tab_ysize(int P) { return ybase(P + 1); }
// [n][k][m] (m >= 0) z-axis translation coefficients (App. B.3 in the
// normalised basis); see tables.cpp
FMM_HD int tab_tm2l(int P) { return tab_y(P) + tab_ysize(P); }
FMM_HD int tab_tm2m(int P) { return tab_tm2l(P) + (P + 1) * (P + 1) * (P + 1); }
FMM_HD int tab_tl2l(int P) { return tab_tm2m(P) + (P + 1) * (P + 1) * (P + 1); }
FMM_HD int tab_size(int P) { return tab_tl2l(P) + (P + 1) * (P + 1) * (P + 1); }
FMM_HD int t3(int P, int n, int k, int m) { return (n * (P + 1) + k) * (P + 1) + m; }

}  // namespace fmm
