// Evaluation pass for up to kRB = 32 charge vectors at once on one plan
// (the paper's cached hierarchy reused for new charges, Sec. II.E), FP32.
//
// Layout: every per-point and per-box array carries the vectors innermost:
// charges qL[n][kRB] in leaf order, expansions C, D [box][(p+1)^2][kRB],
// outputs potL[n][kRB], fldL[n][3][kRB] in leaf order, scattered to the
// caller's [R][n] / [R][n][3] at the end.  Lane r of a 32-lane half-wave
// owns vector r, so every coefficient access is a contiguous 128-byte
// segment, and everything that depends only on the geometry -- rotation
// angles, scale ratios, the operator tables -- is shared by all vectors.
//
//   P2M:  block = leaf; the basis of 64 points goes to LDS, lane r then
//         forms C[k][r] = sum_i B_k(y_i) q_i[r].
//   M2M, M2L, L2L: the single-vector rotate / z-shift / rotate-back code,
//         one (box or work item, vector) per lane, two boxes or items per
//         wave (one per half-wave).
//   L2P:  block = leaf; basis and gradient of 32 points in LDS, lane r
//         forms the potential and gradient sums.
//   P2P:  a dense contraction: for a tile of 32 targets and pairs of source
//         points, the kernel entries 1/r and d/r^3 (computed per lane, one
//         entry each) are the A operand and the source charges of the 32
//         vectors the B operand of v_mfma_f32_32x32x2f32; four
//         accumulators hold the potential and the three field components
//         for 32 targets x 32 vectors.  Each source leaf is accumulated from
//         zero and added to the running sums with Neumaier compensation.
#include <cmath>

#include "internal.h"
#include "ops.h"
#include "tables.h"

namespace fmm {
namespace {

using namespace ops;
constexpr int kRB = 32;

typedef float floatx16 __attribute__((ext_vector_type(16)));

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Neumaier's compensated addition, elementwise: s + c carries the sum.
__device__ __forceinline__ void neumaier16(floatx16& s, floatx16& c, floatx16 x) {
  const floatx16 t = s + x;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const float sv = s[v], xv = x[v], tv = t[v];
    c[v] += fabsf(sv) >= fabsf(xv) ? (sv - tv) + xv : (xv - tv) + sv;
  }
  s = t;
}

// charges to leaf order, vectors innermost (zero past the last vector)
__global__ void k_bgather(int64_t n, int R, const int32_t* __restrict__ perm,
                          const float* __restrict__ q, float* __restrict__ qL) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * kRB) return;
  const int64_t j = e / kRB;
  const int r = (int)(e - j * kRB);
  qL[e] = r < R ? q[(int64_t)r * n + perm[j]] : 0.f;
}

template <int P>
__global__ __launch_bounds__(64) void k_bp2m(
    const int32_t* __restrict__ leaf_box, const int32_t* __restrict__ leaf_start,
    const double* __restrict__ xs, const double* __restrict__ ys,
    const double* __restrict__ zs, const float* __restrict__ qL,
    const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const float* __restrict__ tab, float* __restrict__ C) {
  constexpr int K = K_<P>::value;
  __shared__ float B[64][K + 1];
  const int leaf = blockIdx.x;
  const int lane = threadIdx.x;
  const int r = lane % kRB, h = lane / kRB;  // vector, half of the coefficients
  constexpr int KH = (K + 1) / 2;
  const int64_t g = leaf_box[leaf];
  const int st = leaf_start[leaf], en = leaf_start[leaf + 1];
  const double ox = cx[g], oy = cy[g], oz = cz[g], ir = 1.0 / scale[g];
  float acc[KH];
#pragma unroll
  for (int k = 0; k < KH; ++k) acc[k] = 0.f;
  for (int c0 = st; c0 < en; c0 += 64) {
    const int j = c0 + lane;
    __syncthreads();
    if (j < en) {
      regular_basis<P, float>(float((xs[j] - ox) * ir), float((ys[j] - oy) * ir),
                              float((zs[j] - oz) * ir), [&](int k, float v) { B[lane][k] = v; });
    }
    __syncthreads();
    const int cnt = min(64, en - c0);
    for (int i = 0; i < cnt; ++i) {
      const float qi = qL[(int64_t)(c0 + i) * kRB + r];
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int kk = h * KH + k;
        if (kk < K) acc[k] = fma(qi, B[i][kk], acc[k]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    const int kk = h * KH + k;
    if (kk < K) C[(g * K + kk) * kRB + r] = acc[k] * tab[tab_normc(P) + kk];
  }
}

// parent += M2M(child) over the 2^s children; one (parent, vector) per lane
template <int P>
__global__ __launch_bounds__(64) void k_bm2m(
    int64_t npar, const int32_t* __restrict__ par, const int32_t* __restrict__ child0, int s,
    const double* __restrict__ cx,
    const double* __restrict__ cy, const double* __restrict__ cz,
    const double* __restrict__ scale, const float* __restrict__ tab, float* C) {
  constexpr int K = K_<P>::value;
  const int64_t b = (int64_t)blockIdx.x * 2 + threadIdx.x / kRB;
  const int r = threadIdx.x % kRB;
  if (b >= npar) return;
  const int64_t pa = par[b];
  float acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.f;
  const int nch = 1 << s;
  for (int c = 0; c < nch; ++c) {
    const int64_t ch = child0[b] + c;
    float v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = C[(ch * K + k) * kRB + r];
    rotate_shift<P, kM2M, float>(v, cx[ch] - cx[pa], cy[ch] - cy[pa], cz[ch] - cz[pa],
                                 scale[ch], scale[pa], tab);
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += v[k];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) C[(pa * K + k) * kRB + r] = acc[k];
}

template <int P>
__global__ __launch_bounds__(64) void k_bm2l(
    int64_t nitems, const int32_t* __restrict__ item_tgt,
    const int32_t* __restrict__ item_begin, const int32_t* __restrict__ item_end,
    const int32_t* __restrict__ src, const double* __restrict__ cx,
    const double* __restrict__ cy, const double* __restrict__ cz,
    const double* __restrict__ scale, const float* __restrict__ C,
    const float* __restrict__ tab, float* __restrict__ partial) {
  constexpr int K = K_<P>::value;
  const int64_t i = (int64_t)blockIdx.x * 2 + threadIdx.x / kRB;
  const int r = threadIdx.x % kRB;
  if (i >= nitems) return;
  const int t = item_tgt[i];
  const int jb = item_begin[i], je = item_end[i];
  const double tx = cx[t], ty = cy[t], tz = cz[t], rt = scale[t];
  float acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.f;
  for (int j = jb; j < je; ++j) {
    const int sidx = src[j];
    float v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = C[((int64_t)sidx * K + k) * kRB + r];
    rotate_shift<P, kM2L, float>(v, cx[sidx] - tx, cy[sidx] - ty, cz[sidx] - tz, scale[sidx],
                                 rt, tab);
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += v[k];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) partial[(i * K + k) * kRB + r] = acc[k];
}

template <int P>
__global__ __launch_bounds__(64) void k_bl2l(
    int64_t nb, const int32_t* __restrict__ boxes, const int32_t* __restrict__ parents,
    const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const float* __restrict__ tab, float* D) {
  constexpr int K = K_<P>::value;
  const int64_t i = (int64_t)blockIdx.x * 2 + threadIdx.x / kRB;
  const int r = threadIdx.x % kRB;
  if (i >= nb) return;
  const int64_t t = boxes[i];
  const int64_t pa = parents[i];
  float v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = D[(pa * K + k) * kRB + r];
  rotate_shift<P, kL2L, float>(v, cx[pa] - cx[t], cy[pa] - cy[t], cz[pa] - cz[t], scale[pa],
                               scale[t], tab);
#pragma unroll
  for (int k = 0; k < K; ++k) D[(t * K + k) * kRB + r] = D[(t * K + k) * kRB + r] + v[k];
}

// L2P for 32 points at a time: basis and gradient in LDS, lane r sums.
template <int P>
__global__ __launch_bounds__(64) void k_bl2p(
    const int32_t* __restrict__ leaf_box, const int32_t* __restrict__ leaf_start,
    const double* __restrict__ xs, const double* __restrict__ ys,
    const double* __restrict__ zs, const double* __restrict__ cx,
    const double* __restrict__ cy, const double* __restrict__ cz,
    const double* __restrict__ scale, const float* __restrict__ D,
    const float* __restrict__ tab, float* __restrict__ potL, float* __restrict__ fldL) {
  constexpr int K = K_<P>::value;
  constexpr int NP = 32;
  __shared__ float Bv[NP][4][K];
  const int leaf = blockIdx.x;
  const int lane = threadIdx.x;
  const int r = lane % kRB, h = lane / kRB;
  const int64_t g = leaf_box[leaf];
  const int st = leaf_start[leaf], en = leaf_start[leaf + 1];
  const double ox = cx[g], oy = cy[g], oz = cz[g], ir = 1.0 / scale[g];
  const float fu = float(-kInv4Pi * ir), ff = float(kInv4Pi * ir * ir);
  float w[K];
#pragma unroll
  for (int k = 0; k < K; ++k) w[k] = D[(g * K + k) * kRB + r] * tab[tab_l2p(P) + k];
  for (int c0 = st; c0 < en; c0 += NP) {
    __syncthreads();
    if (lane < NP && c0 + lane < en) {
      const int j = c0 + lane;
      const float x = float((xs[j] - ox) * ir), y = float((ys[j] - oy) * ir),
                  z = float((zs[j] - oz) * ir);
      basis_with_gradient<P, float>(x, y, z, [&](int k, float v, float gx, float gy, float gz) {
        Bv[lane][0][k] = v;
        Bv[lane][1][k] = gx;
        Bv[lane][2][k] = gy;
        Bv[lane][3][k] = gz;
      });
    }
    __syncthreads();
    const int cnt = min(NP, en - c0);
    for (int i = h; i < cnt; i += 2) {
      float u = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        u = fma(w[k], Bv[i][0][k], u);
        gx = fma(w[k], Bv[i][1][k], gx);
        gy = fma(w[k], Bv[i][2][k], gy);
        gz = fma(w[k], Bv[i][3][k], gz);
      }
      const int64_t o = c0 + i;
      potL[o * kRB + r] = fu * u;
      fldL[(o * 3 + 0) * kRB + r] = ff * gx;
      fldL[(o * 3 + 1) * kRB + r] = ff * gy;
      fldL[(o * 3 + 2) * kRB + r] = ff * gz;
    }
  }
}

// P2P on the matrix cores.  For a tile of 32 targets (rows) and 32 vectors
// (columns), every step takes two source points: lane l computes the kernel
// entries of target (l % 32) and source (l / 32) -- the A operand -- and
// supplies the charge of source (l / 32) for vector (l % 32) -- the B
// operand.  Accumulator register v of lane l holds row
// 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32.
__global__ __launch_bounds__(64) void k_bp2p(
    const int32_t* __restrict__ leaf_start, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs,
    const float* __restrict__ qL, const int32_t* __restrict__ p2p_ptr,
    const int32_t* __restrict__ p2p_src, float* __restrict__ potL, float* __restrict__ fldL) {
  const int leaf = blockIdx.x;
  const int lane = threadIdx.x;
  const int row = lane % 32, kk = lane / 32;
  const int st = leaf_start[leaf], en = leaf_start[leaf + 1];
  const int pb = p2p_ptr[leaf], pe = p2p_ptr[leaf + 1];
  for (int i0 = st; i0 < en; i0 += 32) {
    const int i = i0 + row;
    const bool live_i = i < en;
    const int ii = live_i ? i : st;
    const double xi = xs[ii], yi = ys[ii], zi = zs[ii];
    // running sums (s*) with Neumaier compensation (c*); each source leaf is
    // accumulated on the matrix cores from zero and then added
    floatx16 su = {}, sx = {}, sy = {}, sz = {}, cu = {}, cx_ = {}, cy_ = {}, cz_ = {};
    for (int k = pb; k < pe; ++k) {
      const int sl = p2p_src[k];
      const int js = leaf_start[sl], je = leaf_start[sl + 1];
      floatx16 au = {}, ax = {}, ay = {}, az = {};
      for (int j0 = js; j0 < je; j0 += 2) {
        const int j = j0 + kk;
        const bool live_j = j < je;
        const int jj = live_j ? j : js;
        const float dx = float(xi - xs[jj]), dy = float(yi - ys[jj]), dz = float(zi - zs[jj]);
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float inv0 = __builtin_amdgcn_rsqf(r2);
        const float inv = (r2 > 0.f && live_i && live_j) ? inv0 : 0.f;
        const float inv3 = inv * inv * inv;
        const float b = live_j ? qL[(int64_t)jj * kRB + row] : 0.f;
        au = __builtin_amdgcn_mfma_f32_32x32x2f32(inv, b, au, 0, 0, 0);
        ax = __builtin_amdgcn_mfma_f32_32x32x2f32(dx * inv3, b, ax, 0, 0, 0);
        ay = __builtin_amdgcn_mfma_f32_32x32x2f32(dy * inv3, b, ay, 0, 0, 0);
        az = __builtin_amdgcn_mfma_f32_32x32x2f32(dz * inv3, b, az, 0, 0, 0);
      }
      neumaier16(su, cu, au);
      neumaier16(sx, cx_, ax);
      neumaier16(sy, cy_, ay);
      neumaier16(sz, cz_, az);
    }
    floatx16 au = su + cu, ax = sx + cx_, ay = sy + cy_, az = sz + cz_;
    const float c = float(kInv4Pi);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int ti = i0 + 8 * (v / 4) + 4 * kk + (v % 4);
      if (ti < en) {
        const int64_t o = ti;
        potL[o * kRB + row] += -c * au[v];
        // field = -grad u; grad of the near part is +(1/4pi) sum q d/r^3
        fldL[(o * 3 + 0) * kRB + row] -= c * ax[v];
        fldL[(o * 3 + 1) * kRB + row] -= c * ay[v];
        fldL[(o * 3 + 2) * kRB + row] -= c * az[v];
      }
    }
  }
}

// leaf-ordered [n][kRB] results to the caller's [R][n] and [R][n][3]
__global__ void k_bscatter(int64_t n, int R, const int32_t* __restrict__ perm,
                           const float* __restrict__ potL, const float* __restrict__ fldL,
                           float* __restrict__ pot, float* __restrict__ field) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * kRB) return;
  const int64_t j = e / kRB;
  const int r = (int)(e - j * kRB);
  if (r >= R) return;
  const int64_t o = perm[j];
  pot[(int64_t)r * n + o] = potL[e];
  if (field)
    for (int a = 0; a < 3; ++a)
      field[((int64_t)r * n + o) * 3 + a] = fldL[(j * 3 + a) * kRB + r];
}

template <int P>
void run_batch(fmm_plan* pl, const ListSet& Ls, const float* q, int R, float* pot,
               float* field, hipStream_t st) {
  const int s = pl->s;
  const float* tab = (const float*)pl->tables;
  float* qL = (float*)pl->bq;
  float* C = (float*)pl->bC;
  float* D = (float*)pl->bD;
  float* part = (float*)pl->bpart;
  float* potL = (float*)pl->bpot;
  float* fldL = (float*)pl->bfld;
  const int64_t n = pl->n;
  StageMarks mk(pl);
  mk.begin(kStSort, st);
  k_bgather<<<blocks(n * kRB, 256), 256, 0, st>>>(n, R, pl->perm, q, qL);
  mk.end(kStSort, st);
  mk.begin(kStP2M, st);
  k_bp2m<P><<<(unsigned)pl->nleaf, 64, 0, st>>>(pl->leaf_box, pl->leaf_start, pl->xs, pl->ys,
                                                pl->zs, qL, pl->cx, pl->cy, pl->cz, pl->scale,
                                                tab, C);
  mk.end(kStP2M, st);
  mk.begin(kStM2M, st);
  for (const Step& S : pl->m2m_steps)
    k_bm2m<P><<<blocks(S.n, 2), 64, 0, st>>>(S.n, S.a, S.b, s, pl->cx, pl->cy, pl->cz,
                                             pl->scale, tab, C);
  mk.end(kStM2M, st);
  mk.begin(kStM2L, st);
  if (Ls.n_items > 0)
    k_bm2l<P><<<blocks(Ls.n_items, 2), 64, 0, st>>>(Ls.n_items, Ls.item_tgt, Ls.item_begin,
                                                    Ls.item_end, Ls.m2l_src, pl->cx, pl->cy,
                                                    pl->cz, pl->scale, C, tab, part);
  mk.end(kStM2L, st);
  mk.begin(kStL2L, st);
  if (pl->l2l_sum.n > 0)
    k_psum<float><<<(unsigned)pl->l2l_sum.n, 256, 0, st>>>(
        pl->l2l_sum.n, pl->l2l_sum.a, Ls.item_ptr, part, K_<P>::value * kRB, D);
  for (const Step& S : pl->l2l_steps)
    k_bl2l<P><<<blocks(S.n, 2), 64, 0, st>>>(S.n, S.a, S.b, pl->cx, pl->cy, pl->cz, pl->scale,
                                             tab, D);
  mk.end(kStL2L, st);
  mk.begin(kStL2P, st);
  k_bl2p<P><<<(unsigned)pl->nleaf, 64, 0, st>>>(pl->leaf_box, pl->leaf_start, pl->xs, pl->ys,
                                                pl->zs, pl->cx, pl->cy, pl->cz, pl->scale, D,
                                                tab, potL, fldL);
  mk.end(kStL2P, st);
  mk.begin(kStP2P, st);
  k_bp2p<<<(unsigned)pl->nleaf, 64, 0, st>>>(pl->leaf_start, pl->xs, pl->ys, pl->zs, qL,
                                              Ls.p2p_ptr, Ls.p2p_src, potL, fldL);
  k_bscatter<<<blocks(n * kRB, 256), 256, 0, st>>>(n, R, pl->perm, potL, fldL, pot, field);
  mk.end(kStP2P, st);
  FMM_HIP(hipGetLastError());
}

}  // namespace

int batch_width() { return kRB; }

void evaluate_batch(fmm_plan* pl, int dir, const float* q, int R, float* pot, float* field,
                    hipStream_t st) {
  const ListSet& Ls = pl->lists[dir];
  switch (pl->prm.p) {
#define FMM_CASE(PP)                                   \
  case PP:                                             \
    run_batch<PP>(pl, Ls, q, R, pot, field, st); \
    break;
    FMM_CASE(1) FMM_CASE(2) FMM_CASE(3) FMM_CASE(4) FMM_CASE(5)
    FMM_CASE(6) FMM_CASE(7) FMM_CASE(8) FMM_CASE(9) FMM_CASE(10)
#undef FMM_CASE
    default:
      throw Error{FMM_ENOTSUP, "expansion order without compiled kernels"};
  }
}

}  // namespace fmm
