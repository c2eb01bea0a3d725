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
//   M2L item: thread = (target box, up to a dozen of its sources); the
//             items of one target share a block and their sums are added
//             in lane order, so results do not depend on scheduling (the
//             only atomics are adds to lane-private LDS slots).
//   M2M:      thread = child box; the 2^s children of a parent sit in
//             adjacent lanes and are summed with cross-lane shuffles.
//   L2L:      two launches for all levels: the leaves' parents get their M2L
//             sum plus the shifted M2L sums of all their ancestors, one lane
//             per ancestor (local re-centring is exact), summed across
//             lanes; each leaf then adds its parent's shifted local.
//   P2M:      block = leaf, thread = point, LDS reduction over points.
//   L2P:      block = target leaf, thread = target point; writes outputs.
//   P2P:      block = target leaf, thread = target point; adds the near
//             field; the source points of the direct list are read with
//             wave-uniform (scalar) loads.
#include <cmath>

#include <type_traits>

#include "internal.h"
#include "ops.h"
#include "tables.h"

namespace fmm {
namespace {

using namespace ops;

// ---------------------------------------------------------------- P2M
// C_leaf = normc * sum_i q_i R-hat((x_i - c) / rho)  (scaled multipole).
// G leaves per wave (LW = 64/G lanes each, lane = point).  The per-lane
// terms go to LDS in chunks of kP2MRows coefficients (row r of lane l at
// r * kRow + l); each chunk is then summed over every leaf's lanes by one
// lane per (leaf, coefficient), in a fixed order (two interleaved partial
// sums).  The kernel also does the
// sort stage: it reads each charge in input order and writes the leaf's
// 32-byte source records that P2P reads.
constexpr int kRow = 65;       // LDS row stride: a lane's rows fall in different banks
constexpr int kP2MRows = 16;   // coefficients per chunk

// Row r of buf holds coefficient rowk[r] (or k0 + r when rowk is NULL) of
// every lane; cs[leaf][coefficient] = the sum over the leaf's LW lanes.
template <int LW, int K, typename T>
__device__ __forceinline__ void leaf_sums(const T* buf, const int* rowk, int nr, int k0,
                                          T (*cs)[K], int G) {
  for (int t = threadIdx.x; t < G * nr; t += 64) {
    const int hh = t / nr, r = t - hh * nr;
    const T* row = buf + r * kRow + hh * LW;
    T s0 = T(0), s1 = T(0);
#pragma unroll
    for (int l = 0; l < LW; l += 2) {
      s0 += row[l];
      s1 += row[l + 1];
    }
    cs[hh][rowk ? rowk[r] : k0 + r] = s0 + s1;
  }
}

template <int P, typename T, int G>
__global__ __launch_bounds__(64) void k_p2m(
    int64_t nleaf, const int32_t* __restrict__ leaf_box,
    const int32_t* __restrict__ leaf_start, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs,
    const int32_t* __restrict__ perm, const T* __restrict__ q, Src<T>* __restrict__ src,
    const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const T* __restrict__ tab, T* __restrict__ C) {
  constexpr int K = K_<P>::value;
  constexpr int LW = 64 / G;
  __shared__ T cs[G][K];  // finished sums, stored coalesced at the end
  __shared__ T buf[(kP2MRows - 1) * kRow + 64];
  __shared__ int rowk[kP2MRows];  // coefficient held by each row
  const int lane = threadIdx.x;
  const int h = lane / LW, l = lane % LW;
  const int64_t leaf = (int64_t)blockIdx.x * G + h;
  const bool has = leaf < nleaf;
  const int64_t g = has ? leaf_box[leaf] : 0;
  const int st = has ? leaf_start[leaf] : 0, en = has ? leaf_start[leaf + 1] : 0;
  const double ox = cx[g], oy = cy[g], oz = cz[g], ir = 1.0 / scale[g];
  if (G > 1) {
    // at most one point per lane: every term goes to LDS as it is formed
    // (the basis comes order by order, so rows record their coefficient)
    const int j = st + l;
    const bool pt = j < en;
    const int jj = pt ? j : st;
    const T qj = pt ? q[perm[j]] : T(0);
    if (pt) src[j] = Src<T>{xs[j], ys[j], zs[j], qj};
    int e = 0;  // terms emitted so far (the same in every lane)
    regular_basis<P, T>(T((xs[jj] - ox) * ir), T((ys[jj] - oy) * ir), T((zs[jj] - oz) * ir),
                        [&](int k, T v) {
                          const int r = e % kP2MRows;
                          buf[r * kRow + lane] = qj * v;
                          if (lane == 0) rowk[r] = k;
                          ++e;
                          if (r == kP2MRows - 1 || e == K) {
                            __syncthreads();
                            leaf_sums<LW, K, T>(buf, rowk, r + 1, 0, cs, G);
                            __syncthreads();
                          }
                        });
  } else {
    T acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = T(0);
    for (int j = st + l; j < en; j += LW) {
      const T qj = q[perm[j]];
      src[j] = Src<T>{xs[j], ys[j], zs[j], qj};
      regular_basis<P, T>(T((xs[j] - ox) * ir), T((ys[j] - oy) * ir), T((zs[j] - oz) * ir),
                          [&](int k, T v) { acc[k] = fma(qj, v, acc[k]); });
    }
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += kP2MRows) {
#pragma unroll
      for (int r = 0; r < kP2MRows; ++r)
        if (k0 + r < K) buf[r * kRow + lane] = acc[k0 + r];
      __syncthreads();
      leaf_sums<LW, K, T>(buf, nullptr, (K - k0 < kP2MRows ? K - k0 : kP2MRows), k0, cs, 1);
      __syncthreads();
    }
  }
  for (int idx = lane; idx < G * K; idx += 64) {
    const int hh = idx / K, k = idx - hh * K;
    const int64_t lf = (int64_t)blockIdx.x * G + hh;
    if (lf < nleaf) C[(int64_t)leaf_box[lf] * K + k] = cs[hh][k] * tab[tab_normc(P) + k];
  }
}

// ------------------------------------------- translations shared by waves
// One translation (rotate, z-shift, rotate back) split over the NW waves of
// a block, lane l of every wave working on the same translation.  The
// rotations act degree by degree and the z-shift order by order, so wave w
// rotates the degrees of share_mask(P, NW, w, false, kind) and z-shifts the
// orders of share_mask(P, NW, w, true, kind), the coefficients passing
// between the two through a 64-lane LDS tile (three barriers).  Every
// coefficient undergoes the same operations in the same order as in
// rotate_shift, so the results are identical to the one-lane form; each
// wave holds a fraction of the coefficients and runs a fraction of the
// chain of dependent operations, which raises the occupancy where the
// one-lane form runs out of registers and cuts the latency of launches with
// few translations (the level chains).

// Multiply-adds of the two rotation phases on degree n (Y products and
// azimuth steps) and of the z-shift of orders +-am (M2L: full blocks; M2M,
// L2L: triangles).
__host__ __device__ constexpr int rot_cost(int n) { return 4 * (n * n + n + 1) + 16 * n; }
__host__ __device__ constexpr int shift_cost(int P, int am, int kind) {
  const int d = P + 1 - am;
  return (am > 0 ? 2 : 1) * (kind == kM2L ? d * d : d * (d + 1));
}

// Degrees (orders: false/true) of wave w: largest cost first, each onto the
// least loaded wave (the first of equals).
__host__ __device__ constexpr unsigned share_mask(int P, int NW, int w, bool orders, int kind) {
  int load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  unsigned mask[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  unsigned done = 0;
  for (int step = 0; step <= P; ++step) {
    int pick = -1, pc = -1;
    for (int x = 0; x <= P; ++x) {
      if ((done >> x) & 1u) continue;
      const int c = orders ? shift_cost(P, x, kind) : rot_cost(x);
      if (c > pc) {
        pc = c;
        pick = x;
      }
    }
    done |= 1u << pick;
    int best = 0;
    for (int j = 1; j < NW; ++j)
      if (load[j] < load[best]) best = j;
    load[best] += pc;
    mask[best] |= 1u << pick;
  }
  return mask[w];
}

// coefficient loops over (n, m), k = cidx(n, m): the degrees of mask DM,
// the orders of mask OM
#define FMM_DEG_LOOP(DM, stmt)                        \
  _Pragma("unroll") for (int n = 0; n <= P; ++n) {    \
    if (!(((DM) >> n) & 1u)) continue;                \
    _Pragma("unroll") for (int m = -n; m <= n; ++m) { \
      const int k = cidx(n, m);                       \
      stmt;                                           \
    }                                                 \
  }
#define FMM_ORD_LOOP(OM, stmt)                                \
  _Pragma("unroll") for (int n = 0; n <= P; ++n) {            \
    _Pragma("unroll") for (int m = -n; m <= n; ++m) {         \
      if (!(((OM) >> (m < 0 ? -m : m)) & 1u)) continue;       \
      const int k = cidx(n, m);                               \
      stmt;                                                   \
    }                                                         \
  }

// Wave W's part of one translation per lane: v holds the wave's degrees on
// entry and the translated coefficients of those degrees on return.  All
// waves of the block call it together (barriers inside; lanes with act
// false take no part but reach them).  X: LDS tile of (K - 1) kRow + 64
// entries, free again on return.
template <int P, int KIND, typename T, int NW, int W>
__device__ __forceinline__ void turn_shared(T* v, bool act, const Turn<P, KIND, T>& g,
                                            const T* __restrict__ tab, T* X, int lane) {
  constexpr int K = K_<P>::value;
  constexpr unsigned DM = share_mask(P, NW, W, false, KIND);
  constexpr unsigned OM = share_mask(P, NW, W, true, KIND);
  if (act) {
    turn_forward<P, KIND, T, DM>(v, g, tab);
    FMM_DEG_LOOP(DM, X[k * kRow + lane] = v[k])
  }
  __syncthreads();
  if (act) {
    T z[K];
    FMM_ORD_LOOP(OM, z[k] = X[k * kRow + lane])
    zshift<P, KIND, T, OM>(z, g.a, g.b, tab);
    FMM_ORD_LOOP(OM, X[k * kRow + lane] = z[k])
  }
  __syncthreads();
  if (act) FMM_DEG_LOOP(DM, v[k] = X[k * kRow + lane])
  __syncthreads();
  if (act) turn_back<P, KIND, T, DM>(v, g, tab);
}

// Waves per translation of the shared forms.
constexpr int kShareWaves = 4;

// ---------------------------------------------------------------- M2M
template <int P, typename T>
__global__ __launch_bounds__(64) void k_m2m(
    int64_t nchild, const int32_t* __restrict__ par, const int32_t* __restrict__ child0,
    int s, const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const T* __restrict__ tab, T* C) {
  constexpr int K = K_<P>::value;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < nchild;
  const int64_t ii = live ? i : 0;
  const int64_t c = child0[ii >> s] + (ii & ((1 << s) - 1));
  const int64_t pa = par[ii >> s];
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

// k_m2m with each translation shared by the kShareWaves waves of a block
// (turn_shared); the same results.
template <int P, typename T, int W>
__device__ __forceinline__ void m2m_wave(int lane, int64_t i, bool live, int64_t c, int64_t pa,
                                         int s, const Turn<P, kM2M, T>& g,
                                         const T* __restrict__ tab, T* C, T* X) {
  constexpr int K = K_<P>::value;
  constexpr unsigned DM = share_mask(P, kShareWaves, W, false, kM2M);
  T v[K];
  FMM_DEG_LOOP(DM, v[k] = live ? C[c * K + k] : T(0))
  turn_shared<P, kM2M, T, kShareWaves, W>(v, true, g, tab, X, lane);
  const int nch = 1 << s;
  for (int off = 1; off < nch; off <<= 1) FMM_DEG_LOOP(DM, v[k] += __shfl_xor(v[k], off, 64))
  if (live && (i & (nch - 1)) == 0) FMM_DEG_LOOP(DM, C[pa * K + k] = v[k])
}

template <int P, typename T>
__global__ __launch_bounds__(64 * kShareWaves) void k_m2m_shared(
    int64_t nchild, const int32_t* __restrict__ par, const int32_t* __restrict__ child0,
    int s, const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const T* __restrict__ tab, T* C) {
  constexpr int K = K_<P>::value;
  __shared__ T X[(K - 1) * kRow + 64];
  const int lane = threadIdx.x % 64;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const bool live = i < nchild;
  const int64_t ii = live ? i : 0;
  const int64_t c = child0[ii >> s] + (ii & ((1 << s) - 1));
  const int64_t pa = par[ii >> s];
  const Turn<P, kM2M, T> g(cx[c] - cx[pa], cy[c] - cy[pa], cz[c] - cz[pa], scale[c], scale[pa]);
  switch (w) {
    case 0: m2m_wave<P, T, 0>(lane, i, live, c, pa, s, g, tab, C, X); break;
    case 1: m2m_wave<P, T, 1>(lane, i, live, c, pa, s, g, tab, C, X); break;
    case 2: m2m_wave<P, T, 2>(lane, i, live, c, pa, s, g, tab, C, X); break;
    default: m2m_wave<P, T, 3>(lane, i, live, c, pa, s, g, tab, C, X); break;
  }
}

// ---------------------------------------------------------------- M2L
// Lane-private LDS rows as in P2M (row r of lane l at r * kRow + l): the
// segment sums below read different rows of the same lane without bank
// conflicts, while a wave's access to one row stays contiguous.

// For every target segment of this block (seg_tgt[g], lanes
// [seg_lanes[g] & 255, seg_lanes[g] >> 8), g in [sb, se)), adds rows
// [0, NR) of buf over the segment's lanes in lane order and stores the sums
// as coefficients k0 .. k0 + NR - 1 of the target's local.
template <int NR, typename T>
__device__ __forceinline__ void segment_sums(const T* buf, int k0, int K, int sb, int se,
                                             const int32_t* __restrict__ seg_tgt,
                                             const int32_t* __restrict__ seg_lanes, T* D) {
  const int n = (se - sb) * NR;
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
    const int g = sb + idx / NR, r = idx % NR;
    const int info = seg_lanes[g];
    T acc = T(0);
    for (int l = info & 255; l < (info >> 8); ++l) acc += buf[r * kRow + l];
    D[(int64_t)seg_tgt[g] * K + k0 + r] = acc;
  }
}

// One block = kM2LBlock lanes; lane = one work item (a run of at most a
// dozen source boxes of one target).  Every lane translates its sources and
// sums them; the items of one target share the block and their sums are
// added in lane order into the target's local, D_t = sum of its M2L
// translations, written once (no partial rows in memory).
template <int P, typename T>
__global__ __launch_bounds__(kM2LBlock) void k_m2l(
    int64_t nblocks, const int32_t* __restrict__ item_tgt,
    const int32_t* __restrict__ item_begin, const int32_t* __restrict__ item_end,
    const int32_t* __restrict__ seg_ptr, const int32_t* __restrict__ seg_tgt,
    const int32_t* __restrict__ seg_lanes, const int32_t* __restrict__ src,
    const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const T* __restrict__ C, const T* __restrict__ tab, T* __restrict__ D) {
  constexpr int K = K_<P>::value;
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x;
  const int64_t i = b * kM2LBlock + lane;
  const int t = item_tgt[i];
  const int jb = item_begin[i], je = item_end[i];  // empty for idle lanes
  const int tt = t < 0 ? 0 : t;
  const double tx = cx[tt], ty = cy[tt], tz = cz[tt], rt = scale[tt];
  // Accumulators: in FP64 with (p+1)^2 > KL the first KL coefficients live
  // in lane-private LDS rows (78 rows of 65 doubles fit 40 KiB, so four
  // 64-lane blocks fill a CU's 160 KiB, the occupancy the registers allow
  // anyway) and are updated with LDS atomic adds that need no registers; the
  // rest stay in registers.  The rows are then reused to add the items of
  // each target.
  constexpr int KL = (sizeof(T) == 8 && K > 78) ? 78 : 0;
  constexpr int KR = K - KL;                      // accumulators in registers
  constexpr int CH = KL > 0 ? (KR < KL ? KR : KL) : (KR < 16 ? KR : 16);  // rows per pass
  constexpr int NROW = KL > 0 ? KL : CH;
  __shared__ T accl[(NROW - 1) * kRow + kM2LBlock];
  T acc[KR];
#pragma unroll
  for (int k = 0; k < KL; ++k) accl[k * kRow + lane] = T(0);
#pragma unroll
  for (int k = 0; k < KR; ++k) acc[k] = T(0);
  for (int j = jb; j < je; ++j) {
    const int sidx = src[j];
    T v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = C[(int64_t)sidx * K + k];
    rotate_shift<P, kM2L, T>(v, cx[sidx] - tx, cy[sidx] - ty, cz[sidx] - tz, scale[sidx], rt,
                             tab);
#pragma unroll
    for (int k = 0; k < KL; ++k)
      __hip_atomic_fetch_add(&accl[k * kRow + lane], v[k], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
    {
      // a plain add: whether the compiler would fuse it with the last
      // product of the translation depends on the surrounding code
#pragma clang fp contract(off)
#pragma unroll
      for (int k = KL; k < K; ++k) acc[k - KL] += v[k];
    }
  }
  const int sb = seg_ptr[b], se = seg_ptr[b + 1];
  __syncthreads();
  if (KL > 0) {
    segment_sums<(KL > 0 ? KL : 1), T>(accl, 0, K, sb, se, seg_tgt, seg_lanes, D);
    __syncthreads();
  }
  // register accumulators, CH rows at a time
#pragma unroll
  for (int c0 = 0; c0 < KR; c0 += CH) {
#pragma unroll
    for (int r = 0; r < CH; ++r)
      if (c0 + r < KR) accl[r * kRow + lane] = acc[c0 + r];
    __syncthreads();
    if (c0 + CH <= KR)
      segment_sums<CH, T>(accl, KL + c0, K, sb, se, seg_tgt, seg_lanes, D);
    else
      segment_sums<(KR % CH > 0 ? KR % CH : 1), T>(accl, KL + c0, K, sb, se, seg_tgt,
                                                   seg_lanes, D);
    __syncthreads();
  }
}

template <int P, typename T, int NW, int W>
__device__ __forceinline__ void m2l_share(int lane, int jb, int je, int iters, double tx,
                                          double ty, double tz, double rt,
                                          const int32_t* __restrict__ src,
                                          const double* __restrict__ cx,
                                          const double* __restrict__ cy,
                                          const double* __restrict__ cz,
                                          const double* __restrict__ scale,
                                          const T* __restrict__ C, const T* __restrict__ tab,
                                          T* X) {
  constexpr int K = K_<P>::value;
  constexpr unsigned DM = share_mask(P, NW, W, false, kM2L);
  T acc[K];
  FMM_DEG_LOOP(DM, acc[k] = T(0))
  for (int it = 0; it < iters; ++it) {
    const int j = jb + it;
    const bool act = j < je;
    const int sidx = act ? src[j] : 0;
    const Turn<P, kM2L, T> g(cx[sidx] - tx, cy[sidx] - ty, cz[sidx] - tz, scale[sidx], rt);
    T v[K];
    if (act) FMM_DEG_LOOP(DM, v[k] = C[(int64_t)sidx * K + k])
    turn_shared<P, kM2L, T, NW, W>(v, act, g, tab, X, lane);
    if (act) {
      // a plain add, as in k_m2l
#pragma clang fp contract(off)
      FMM_DEG_LOOP(DM, acc[k] += v[k])
    }
  }
  FMM_DEG_LOOP(DM, X[k * kRow + lane] = acc[k])
}

// The same M2L items with the translation of each item shared by the NW
// waves of a block (turn_shared): lane l of every wave works on item l.
// Gives the same results as k_m2l.
template <int P, typename T, int NW>
__global__ __launch_bounds__(kM2LBlock * NW) void k_m2l_shared(
    int64_t nblocks, const int32_t* __restrict__ item_tgt,
    const int32_t* __restrict__ item_begin, const int32_t* __restrict__ item_end,
    const int32_t* __restrict__ seg_ptr, const int32_t* __restrict__ seg_tgt,
    const int32_t* __restrict__ seg_lanes, const int32_t* __restrict__ src,
    const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const T* __restrict__ C, const T* __restrict__ tab, T* __restrict__ D) {
  constexpr int K = K_<P>::value;
  __shared__ T X[(K - 1) * kRow + kM2LBlock];
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x % kM2LBlock;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kM2LBlock);
  const int64_t i = b * kM2LBlock + lane;
  const int t = item_tgt[i];
  const int jb = item_begin[i], je = item_end[i];  // empty for idle lanes
  const int tt = t < 0 ? 0 : t;
  const double tx = cx[tt], ty = cy[tt], tz = cz[tt], rt = scale[tt];
  // translations of the longest item of the block (the same in every wave)
  int iters = je - jb;
#pragma unroll
  for (int off = 1; off < kM2LBlock; off <<= 1) iters = max(iters, __shfl_xor(iters, off, 64));
  iters = __builtin_amdgcn_readfirstlane(iters);
#define FMM_M2L_WAVE(W)                                                                   \
  case W:                                                                                 \
    if constexpr (W < NW)                                                                 \
      m2l_share<P, T, NW, W>(lane, jb, je, iters, tx, ty, tz, rt, src, cx, cy, cz, scale, \
                             C, tab, X);                                                  \
    break;
  static_assert(NW <= 4, "at most four waves per translation");
  switch (w) {
    FMM_M2L_WAVE(0)
    FMM_M2L_WAVE(1)
    FMM_M2L_WAVE(2)
    FMM_M2L_WAVE(3)
    default: break;
  }
#undef FMM_M2L_WAVE
  __syncthreads();
  segment_sums<K, T>(X, 0, K, seg_ptr[b], seg_ptr[b + 1], seg_tgt, seg_lanes, D);
}

// ---------------------------------------------------------------- L2L
// Final locals of one list of boxes (FinList): GS lanes per box, lane j
// translating the expansion anc[j] of src (re-centring a truncated local
// expansion is exact, so these translations add up to the level-by-level
// chain), the lanes' results added by a butterfly in a fixed order; the
// first lane adds the box's own M2L sum (D) and writes the final local to
// out (the multipole array, free once M2L has run).
template <int P, typename T, int GS>
__global__ __launch_bounds__(64) void k_l2l_fin(
    int64_t nfin, const int32_t* __restrict__ fin_box, const int32_t* __restrict__ fin_own,
    const int32_t* __restrict__ fin_anc, const double* __restrict__ cx,
    const double* __restrict__ cy, const double* __restrict__ cz,
    const double* __restrict__ scale, const T* __restrict__ tab, const T* src,
    const T* __restrict__ D, T* out) {
  constexpr int K = K_<P>::value;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = i / GS;
  const int j = (int)(i % GS);
  const bool live = g < nfin;
  const int64_t t = live ? fin_box[g] : 0;
  const int a = live ? fin_anc[i] : -1;
  T v[K];
  if (a >= 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = src[(int64_t)a * K + k];
    rotate_shift<P, kL2L, T>(v, cx[a] - cx[t], cy[a] - cy[t], cz[a] - cz[t], scale[a], scale[t],
                             tab);
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = T(0);
  }
#pragma unroll
  for (int off = 1; off < GS; off <<= 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += __shfl_xor(v[k], off, 64);
  }
  if (live && j == 0) {
    const bool own = fin_own[g] != 0;
#pragma unroll
    for (int k = 0; k < K; ++k) out[t * K + k] = (own ? D[t * K + k] : T(0)) + v[k];
  }
}

// k_l2l_fin with each translation shared by the kShareWaves waves of a
// block (turn_shared) and the group size gs a launch argument; the same
// results.
template <int P, typename T, int W>
__device__ __forceinline__ void l2l_fin_wave(int lane, bool live, int j, int gs, int64_t t,
                                             int64_t a, bool own, const Turn<P, kL2L, T>& g,
                                             const T* __restrict__ tab, const T* src,
                                             const T* __restrict__ D, T* out, T* X) {
  constexpr int K = K_<P>::value;
  constexpr unsigned DM = share_mask(P, kShareWaves, W, false, kL2L);
  const bool act = a >= 0;
  T v[K];
  FMM_DEG_LOOP(DM, v[k] = act ? src[a * K + k] : T(0))
  turn_shared<P, kL2L, T, kShareWaves, W>(v, act, g, tab, X, lane);
  for (int off = 1; off < gs; off <<= 1) FMM_DEG_LOOP(DM, v[k] += __shfl_xor(v[k], off, 64))
  if (live && j == 0) FMM_DEG_LOOP(DM, out[t * K + k] = (own ? D[t * K + k] : T(0)) + v[k])
}

template <int P, typename T>
__global__ __launch_bounds__(64 * kShareWaves) void k_l2l_fin_shared(
    int64_t nfin, int gs, const int32_t* __restrict__ fin_box,
    const int32_t* __restrict__ fin_own, const int32_t* __restrict__ fin_anc,
    const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const T* __restrict__ tab, const T* src, const T* __restrict__ D, T* out) {
  constexpr int K = K_<P>::value;
  __shared__ T X[(K - 1) * kRow + 64];
  const int lane = threadIdx.x % 64;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const int64_t g = i / gs;
  const int j = (int)(i % gs);
  const bool live = g < nfin;
  const int64_t t = live ? fin_box[g] : 0;
  const int64_t a = live ? fin_anc[i] : -1;
  const bool own = live && fin_own[g] != 0;
  const int64_t aa = a >= 0 ? a : t;  // a valid pair for lanes without a source
  const Turn<P, kL2L, T> tr(cx[aa] - cx[t], cy[aa] - cy[t], cz[aa] - cz[t], scale[aa], scale[t]);
  switch (w) {
    case 0: l2l_fin_wave<P, T, 0>(lane, live, j, gs, t, a, own, tr, tab, src, D, out, X); break;
    case 1: l2l_fin_wave<P, T, 1>(lane, live, j, gs, t, a, own, tr, tab, src, D, out, X); break;
    case 2: l2l_fin_wave<P, T, 2>(lane, live, j, gs, t, a, own, tr, tab, src, D, out, X); break;
    default: l2l_fin_wave<P, T, 3>(lane, live, j, gs, t, a, own, tr, tab, src, D, out, X); break;
  }
}

// ---------------------------------------------------------------- L2P
// L2P: u = -1/(4 pi) (1/rho) sum w_m D R-hat(y), y = (x - c)/rho, and
// field = -grad u (an extra 1/rho from the chain rule), at every point of the
// target leaf, added to the near field P2P left in leaf order; writes the
// outputs in input order.  G leaves per wave, LW = 64/G lanes each, lane =
// point.  The gradient is evaluated from the leaf's gradient expansions
// (grad_coeff, formed once per leaf in LDS), so every point needs only the
// basis values.
template <int P, typename T, bool FIELD, int G>
__global__ __launch_bounds__(64) void k_l2p(
    int64_t nleaf, const int32_t* __restrict__ leaf_box,
    const int32_t* __restrict__ leaf_start, const int32_t* __restrict__ perm,
    const double* __restrict__ xs, const double* __restrict__ ys,
    const double* __restrict__ zs, const double* __restrict__ cx,
    const double* __restrict__ cy, const double* __restrict__ cz,
    const double* __restrict__ scale, const T* __restrict__ D, const T* __restrict__ tab,
    int64_t n, const T* __restrict__ near, T* __restrict__ pot, T* __restrict__ field) {
  constexpr int K = K_<P>::value;
  constexpr int K1 = P * P;  // coefficients of the gradient expansions
  constexpr int LW = 64 / G;
  __shared__ T w[G][K];
  __shared__ T gw[G][3][K1];
  const int lane = threadIdx.x;
  const int h = lane / LW, l = lane % LW;
  for (int idx = lane; idx < G * K; idx += 64) {
    const int hh = idx / K, k = idx - hh * K;
    const int64_t lf = (int64_t)blockIdx.x * G + hh;
    if (lf < nleaf) w[hh][k] = D[(int64_t)leaf_box[lf] * K + k] * tab[tab_l2p(P) + k];
  }
  if (FIELD) {
    __syncthreads();
    for (int idx = lane; idx < G * K1; idx += 64) {
      const int hh = idx / K1, k = idx - hh * K1;
      grad_coeff<P, T>(w[hh], k, gw[hh][0][k], gw[hh][1][k], gw[hh][2][k]);
    }
  }
  __syncthreads();
  const int64_t leaf = (int64_t)blockIdx.x * G + h;
  if (leaf >= nleaf) return;
  const int64_t g = leaf_box[leaf];
  const int st = leaf_start[leaf], en = leaf_start[leaf + 1];
  const double ox = cx[g], oy = cy[g], oz = cz[g], ir = 1.0 / scale[g];
  const T fu = T(-kInv4Pi * ir), ff = T(kInv4Pi * ir * ir);
  for (int i = st + l; i < en; i += LW) {
    T fp = T(0), fx = T(0), fy = T(0), fz = T(0);
    local_eval_grad<P, T>(T((xs[i] - ox) * ir), T((ys[i] - oy) * ir), T((zs[i] - oz) * ir),
                          w[h], gw[h][0], gw[h][1], gw[h][2], fp, fx, fy, fz);
    const int o = perm[i];
    pot[o] = near[i] + fu * fp;
    if (FIELD) {
      const T* f = near + n + 3 * (int64_t)i;
      field[3 * (int64_t)o + 0] = f[0] + ff * fx;
      field[3 * (int64_t)o + 1] = f[1] + ff * fy;
      field[3 * (int64_t)o + 2] = f[2] + ff * fz;
    }
  }
}

// One source point against the lane's target at (xi, yi, zi): the
// difference is taken in FP64 and rounded to T.  SAFE: pairs at distance 0
// contribute nothing (needed within a leaf, and between leaves when the
// point set has coincident points); otherwise the pair is known to be apart.
template <typename T, bool FIELD, bool SAFE>
__device__ __forceinline__ void p2p_pair(const Src<T>& s, double xi, double yi, double zi,
                                         T& u, T& gx, T& gy, T& gz) {
  const T dx = T(xi - s.x), dy = T(yi - s.y), dz = T(zi - s.z);
  const T r2 = dx * dx + dy * dy + dz * dz;
  const T inv0 = inv_sqrt(r2);
  const T inv = SAFE ? (r2 > T(0) ? inv0 : T(0)) : inv0;
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

// P2P: writes -1/(4 pi) sum q/r and the matching field over the direct list,
// in leaf order (near[i] and near[n + 3 i + c]); L2P adds the far field and
// writes the outputs in input order.
// Block = one near-field work item (a run of a target leaf's direct list;
// most leaves have one), lane = target point (position from the plan's
// leaf-ordered coordinates; the sources' records are this pass's, written
// by P2M).  A leaf's only item writes its near field; the items of a split
// leaf write partial rows that k_p2p_sum adds in item order.  G source groups: lanes
// [g*64/G, (g+1)*64/G) share targets with the other groups but walk every
// G-th source point starting at point g.  G = 1 keeps all source reads
// wave-uniform (scalar loads).  G = 2, 4 fill the wave when leaves hold at
// most 32 or 16 points; each source leaf is then first copied into LDS with
// one coalesced 16-byte load per lane, and the groups read their records
// from there (a per-lane global read of every record would saturate the
// texture address unit).  Per source leaf the partial sums are added to the
// running sums with Neumaier compensation (FP32 form); group sums are then
// combined with cross-lane shuffles in a fixed order.
template <typename T, bool FIELD, int G>
__global__ __launch_bounds__(64) void k_p2p(
    int64_t n, const int32_t* __restrict__ item_leaf, const int32_t* __restrict__ item_kb,
    const int32_t* __restrict__ item_ke, const int64_t* __restrict__ item_out,
    const int32_t* __restrict__ leaf_start, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs,
    const Src<T>* __restrict__ src, const int32_t* __restrict__ p2p_src, int dup,
    T* __restrict__ near, T* __restrict__ part) {
  constexpr int TL = 64 / G;  // targets per pass
  constexpr bool kComp = sizeof(T) == 4;  // FP32: compensated sums
  // G > 1: one source leaf (at most TL points) staged as 16-byte words
  __shared__ __align__(32) double2 stage[G > 1 ? 2 * TL : 1];
  // items in target-leaf order, handed to the XCDs in runs of 64:
  // neighbouring target leaves share most source leaves, so their records
  // stay in one XCD's L2, while leaves of unequal cost (several problems,
  // clustered points) spread over all XCDs
  const int item = (int)xcd_chunked<64>(blockIdx.x, gridDim.x);
  const int leaf = item_leaf[item];
  const int lane = threadIdx.x;
  const int g = G == 1 ? 0 : lane / TL;
  const int st = leaf_start[leaf], en = leaf_start[leaf + 1];
  const int pb = item_kb[item], pe = item_ke[item];
  const int64_t po = item_out[item];
  for (int i0 = st; i0 < en; i0 += TL) {
    const int i = i0 + lane % TL;
    const bool live = i < en;
    const int ia = live ? i : st;
    const Src<T> a{xs[ia], ys[ia], zs[ia], T(0)};
    T u = T(0), gx = T(0), gy = T(0), gz = T(0);
    T cu = T(0), cgx = T(0), cgy = T(0), cgz = T(0);
    for (int k = pb; k < pe; ++k) {
      const int sl = p2p_src[k];
      const int js = leaf_start[sl], cnt = leaf_start[sl + 1] - js;
      T lu = T(0), lx = T(0), ly = T(0), lz = T(0);
      const int full = cnt / G;  // points per group present in every group
      // distance-0 guard only where it can matter: the target leaf itself,
      // or every leaf when the point set has coincident points
      const bool safe = dup || sl == leaf;
      const Src<T>* rec;
      int stride;
      if (G == 1) {
        rec = src + js;
        stride = 1;
      } else {
        // cnt <= TL: the leaf's records are 2 cnt <= 64 words
        const double2* words = reinterpret_cast<const double2*>(src + js);
        __syncthreads();  // previous leaf's reads are done
        if (lane < 2 * cnt) stage[lane] = words[lane];
        __syncthreads();
        rec = reinterpret_cast<const Src<T>*>(stage) + g;
        stride = G;
      }
      auto sweep = [&](auto safe_tag) {
        constexpr bool S = decltype(safe_tag)::value;
        int c = 0;
        for (; c + kChunk <= full; c += kChunk) {
          Src<T> r[kChunk];
#pragma unroll
          for (int t = 0; t < kChunk; ++t) r[t] = rec[(c + t) * stride];
#pragma unroll
          for (int t = 0; t < kChunk; ++t)
            p2p_pair<T, FIELD, S>(r[t], a.x, a.y, a.z, lu, lx, ly, lz);
        }
        for (; c < full; ++c) p2p_pair<T, FIELD, S>(rec[c * stride], a.x, a.y, a.z, lu, lx, ly, lz);
        if (G > 1 && g < cnt - full * G)
          p2p_pair<T, FIELD, S>(rec[full * G], a.x, a.y, a.z, lu, lx, ly, lz);
      };
      if (safe)
        sweep(std::true_type{});
      else
        sweep(std::false_type{});
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
      // field = -grad u;  grad of the near part is +(1/4pi) sum q d/r^3
      if (po < 0) {  // the leaf's only item: its near field
        near[i] = -T(kInv4Pi) * u;
        if (FIELD) {
          T* f = near + n + 3 * (int64_t)i;
          f[0] = -T(kInv4Pi) * gx;
          f[1] = -T(kInv4Pi) * gy;
          f[2] = -T(kInv4Pi) * gz;
        }
      } else {  // one of several items of the leaf: rows of its partial sums
        const int nt = en - st, li = i - st;
        T* r = part + po;
        r[li] = -T(kInv4Pi) * u;
        if (FIELD) {
          r[nt + li] = -T(kInv4Pi) * gx;
          r[2 * nt + li] = -T(kInv4Pi) * gy;
          r[3 * nt + li] = -T(kInv4Pi) * gz;
        }
      }
    }
  }
}

// Near field of the leaves whose direct list was split into several items:
// the items' partial rows added in item order (Neumaier-compensated in
// FP32).  Block = split leaf, thread = target point.
template <typename T, bool FIELD>
__global__ __launch_bounds__(64) void k_p2p_sum(
    int64_t n, const int32_t* __restrict__ split_leaf, const int32_t* __restrict__ split_first,
    const int32_t* __restrict__ split_cnt, const int64_t* __restrict__ item_out,
    const int32_t* __restrict__ leaf_start, const T* __restrict__ part, T* __restrict__ near) {
  constexpr bool kComp = sizeof(T) == 4;
  const int leaf = split_leaf[blockIdx.x];
  const int f = split_first[blockIdx.x], c = split_cnt[blockIdx.x];
  const int st = leaf_start[leaf], nt = leaf_start[leaf + 1] - st;
  for (int li = threadIdx.x; li < nt; li += blockDim.x) {
#pragma unroll
    for (int comp = 0; comp < (FIELD ? 4 : 1); ++comp) {
      T acc = T(0), cc = T(0);
      for (int j = f; j < f + c; ++j) {
        const T x = part[item_out[j] + (int64_t)comp * nt + li];
        if (kComp)
          neumaier(acc, cc, x);
        else
          acc += x;
      }
      acc += cc;
      const int64_t i = st + li;
      if (comp == 0)
        near[i] = acc;
      else
        near[n + 3 * i + comp - 1] = acc;
    }
  }
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

// The near field (P2P) over the direct lists Ls into near, on stream sp:
// one launch over the work items, then the partial sums of the leaves whose
// list was split.
template <typename T>
void near_field(fmm_plan* pl, const ListSet& Ls, const Src<T>* src, int64_t n, T* near,
                bool field, hipStream_t sp, const StageMarks& mk) {
  mk.begin(kStP2P, sp);
  const int G = p2p_groups(pl);
  auto p2p = [&](auto kern) {
    kern<<<(unsigned)Ls.n_pitems, 64, 0, sp>>>(n, Ls.pitem_leaf, Ls.pitem_kb, Ls.pitem_ke,
                                               Ls.pitem_out, pl->leaf_start, pl->xs, pl->ys,
                                               pl->zs, src, Ls.p2p_src, pl->has_dup ? 1 : 0, near,
                                               (T*)Ls.p2p_part);
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
  if (Ls.n_psplit > 0) {
    auto sum = [&](auto kern) {
      kern<<<(unsigned)Ls.n_psplit, 64, 0, sp>>>(n, Ls.psplit_leaf, Ls.psplit_first,
                                                 Ls.psplit_cnt, Ls.pitem_out, pl->leaf_start,
                                                 (const T*)Ls.p2p_part, near);
    };
    if (field) sum(k_p2p_sum<T, true>);
    else sum(k_p2p_sum<T, false>);
  }
  mk.end(kStP2P, sp);
}

// One evaluation: P2P writes the near field in leaf order, L2P adds the far
// field and writes the outputs.
template <int P, typename T>
void run(fmm_plan* pl, const Workspace& ws, int dir, const T* q, T* pot, T* field,
         hipStream_t st) {
  const int s = pl->s;
  const T* tab = (const T*)pl->tables;
  Src<T>* src = (Src<T>*)ws.src;
  T* C = (T*)ws.C;
  T* D = (T*)ws.D;
  T* near = (T*)ws.near;
  const int64_t n = pl->n;
  const ListSet& Ls = pl->lists[dir];
  const Side& SS = src_side(pl, dir);  // charges: P2M, M2M
  const Side& TS = tgt_side(pl, dir);  // evaluation points: L2L, P2P, L2P
  StageMarks mk(pl);
  // the sort stage (charges into leaf-ordered source records) is folded
  // into P2M; its timing slot stays empty
  mk.begin(kStSort, st);
  mk.end(kStSort, st);
  // far field
  // leaves per wave for P2M and L2P: every lane holds at most one point
  const int GL = leaves_per_wave(pl);
  const int64_t nls = SS.nleaf, nlt = TS.nleaf;
  mk.begin(kStP2M, st);
  auto p2m = [&](auto kern) {
    kern<<<(unsigned)((nls + GL - 1) / GL), 64, 0, st>>>(
        nls, pl->leaf_box + SS.leaf0, pl->leaf_start + SS.leaf0, pl->xs, pl->ys, pl->zs,
        pl->perm, q, src, pl->cx, pl->cy, pl->cz, pl->scale, tab, C);
  };
  if (GL == 1) p2m(k_p2m<P, T, 1>);
  else if (GL == 2) p2m(k_p2m<P, T, 2>);
  else if (GL == 4) p2m(k_p2m<P, T, 4>);
  else p2m(k_p2m<P, T, 8>);
  mk.end(kStP2M, st);
  // The near field needs only the leaf-ordered source records of P2M: it
  // runs on the plan's second stream beside the far-field chain (M2M, M2L,
  // L2L), so each fills the other's idle issue slots; L2P joins the two.
  // Stage profiling keeps the stages one after another on st.
  const bool fork = pl->side_stream != nullptr && !pl->profiling && pl->near_stream != 1;
  const hipStream_t sp = fork ? pl->side_stream : st;
  if (fork) FMM_HIP(hipEventRecord(pl->ev_fork, st));
  auto near_part = [&] {
    if (fork) FMM_HIP(hipStreamWaitEvent(sp, pl->ev_fork, 0));
    near_field<T>(pl, Ls, src, n, near, field != nullptr, sp, mk);
    if (fork) FMM_HIP(hipEventRecord(pl->ev_join, sp));
  };
  // enqueued after the far-field chain when forked, so that the chain's
  // small level launches are not queued behind the near field's blocks
  if (!fork) near_part();
  mk.begin(kStM2M, st);
  const bool chain_shared = P >= kChainShareMinOrder && chain_waves(pl) > 1;
  for (const Step& S : SS.m2m_steps) {
    const int64_t nchild = S.n << s;
    if constexpr (P >= kChainShareMinOrder) {
      if (chain_shared) {
        k_m2m_shared<P, T><<<blocks(nchild, 64), 64 * kShareWaves, 0, st>>>(
            nchild, S.a, S.b, s, pl->cx, pl->cy, pl->cz, pl->scale, tab, C);
        continue;
      }
    }
    k_m2m<P, T><<<blocks(nchild, 64), 64, 0, st>>>(nchild, S.a, S.b, s, pl->cx, pl->cy, pl->cz,
                                                   pl->scale, tab, C);
  }
  mk.end(kStM2M, st);
  mk.begin(kStM2L, st);
  if (Ls.n_blocks > 0) {
    auto m2l = [&](auto kern, int nw) {
      kern<<<(unsigned)Ls.n_blocks, kM2LBlock * nw, 0, st>>>(
          Ls.n_blocks, Ls.item_tgt, Ls.item_begin, Ls.item_end, Ls.seg_ptr, Ls.seg_tgt,
          Ls.seg_lanes, Ls.m2l_src, pl->cx, pl->cy, pl->cz, pl->scale, C, tab, D);
    };
    constexpr int NW = m2l_share_waves(P, sizeof(T) == 8);
    if constexpr (NW > 1) {
      if (m2l_waves(pl) > 1)
        m2l(k_m2l_shared<P, T, NW>, NW);
      else
        m2l(k_m2l<P, T>, 1);
    } else {
      m2l(k_m2l<P, T>, 1);
    }
  }
  mk.end(kStM2L, st);
  mk.begin(kStL2L, st);
  // final locals, written over the multipoles: the leaves' parents from all
  // their ancestors, then the leaves from their parents
  T* Dfin = C;
  for (int k = 0; k < 2; ++k) {
    const FinList& F = Ls.fin[k];
    if (F.n == 0) continue;
    const T* from = k == 0 ? D : Dfin;
    if constexpr (P >= kChainShareMinOrder) {
      if (chain_shared) {
        k_l2l_fin_shared<P, T><<<blocks(F.n * F.gs, 64), 64 * kShareWaves, 0, st>>>(
            F.n, F.gs, F.box, F.own, F.anc, pl->cx, pl->cy, pl->cz, pl->scale, tab, from, D,
            Dfin);
        continue;
      }
    }
    auto l2l = [&](auto kern) {
      kern<<<blocks(F.n * F.gs, 64), 64, 0, st>>>(F.n, F.box, F.own, F.anc, pl->cx, pl->cy,
                                                 pl->cz, pl->scale, tab, from, D, Dfin);
    };
    switch (F.gs) {
      case 1: l2l(k_l2l_fin<P, T, 1>); break;
      case 2: l2l(k_l2l_fin<P, T, 2>); break;
      case 4: l2l(k_l2l_fin<P, T, 4>); break;
      case 8: l2l(k_l2l_fin<P, T, 8>); break;
      default: l2l(k_l2l_fin<P, T, 16>); break;
    }
  }
  mk.end(kStL2L, st);
  if (fork) {
    near_part();
    FMM_HIP(hipStreamWaitEvent(st, pl->ev_join, 0));
  }
  mk.begin(kStL2P, st);
  auto l2p = [&](auto kern) {
    kern<<<(unsigned)((nlt + GL - 1) / GL), 64, 0, st>>>(
        nlt, pl->leaf_box + TS.leaf0, pl->leaf_start + TS.leaf0, pl->perm, pl->xs, pl->ys,
        pl->zs, pl->cx, pl->cy, pl->cz, pl->scale, Dfin, tab, n, near, pot, field);
  };
  if (field) {
    if (GL == 1) l2p(k_l2p<P, T, true, 1>);
    else if (GL == 2) l2p(k_l2p<P, T, true, 2>);
    else if (GL == 4) l2p(k_l2p<P, T, true, 4>);
    else l2p(k_l2p<P, T, true, 8>);
  } else {
    if (GL == 1) l2p(k_l2p<P, T, false, 1>);
    else if (GL == 2) l2p(k_l2p<P, T, false, 2>);
    else if (GL == 4) l2p(k_l2p<P, T, false, 4>);
    else l2p(k_l2p<P, T, false, 8>);
  }
  mk.end(kStL2P, st);
  FMM_HIP(hipGetLastError());
}

}  // namespace

bool valid_p2p_groups(const fmm_plan* pl, int g) {
  return g == 1 || ((g == 2 || g == 4) && pl->max_leaf_count <= 64 / g);
}
bool valid_leaves_per_wave(const fmm_plan* pl, int l) {
  return l == 1 || ((l == 2 || l == 4 || l == 8) && pl->max_leaf_count <= 64 / l);
}
int p2p_groups(const fmm_plan* pl) {
  if (pl->p2p_groups && valid_p2p_groups(pl, pl->p2p_groups)) return pl->p2p_groups;
  const int m = pl->max_leaf_count;
  return m > 32 ? 1 : (m > 16 ? 2 : 4);
}
int chain_waves(const fmm_plan* pl) {
  return pl->prm.p < kChainShareMinOrder || pl->chain_waves == 1 ? 1 : kShareWaves;
}
int m2l_waves(const fmm_plan* pl) {
  const int shared = m2l_share_waves(pl->prm.p, pl->prm.precision == FMM_FP64);
  return pl->m2l_waves == 1 ? 1 : shared;
}
int leaves_per_wave(const fmm_plan* pl) {
  if (pl->leaves_per_wave && valid_leaves_per_wave(pl, pl->leaves_per_wave))
    return pl->leaves_per_wave;
  const int m = pl->max_leaf_count;
  return m > 32 ? 1 : (m > 16 ? 2 : (m > 8 ? 4 : 8));
}

namespace {

template <typename T>
void dispatch(int p, fmm_plan* pl, const Workspace& ws, int dir, const T* q, T* pot,
              T* field, hipStream_t st) {
  switch (p) {
#define FMM_CASE(PP) \
  case PP:           \
    run<PP, T>(pl, ws, dir, q, pot, field, st); \
    break;
    FMM_CASE(1) FMM_CASE(2) FMM_CASE(3) FMM_CASE(4) FMM_CASE(5)
    FMM_CASE(6) FMM_CASE(7) FMM_CASE(8) FMM_CASE(9) FMM_CASE(10)
#undef FMM_CASE
    default:
      throw Error{FMM_ENOTSUP, "expansion order without compiled kernels"};
  }
}

}  // namespace

void evaluate(fmm_plan* pl, const Workspace& ws, int dir, const void* q, int nrhs, void* pot,
              void* field, hipStream_t st) {
  // vector r of q has the source side's points, of pot/field the target side's
  const int64_t nq = src_side(pl, dir).npt, nu = tgt_side(pl, dir).npt;
  for (int r = 0; r < nrhs; ++r) {
    if (pl->prm.precision == FMM_FP32) {
      dispatch<float>(pl->prm.p, pl, ws, dir, (const float*)q + r * nq, (float*)pot + r * nu,
                      field ? (float*)field + 3 * r * nu : nullptr, st);
    } else {
      dispatch<double>(pl->prm.p, pl, ws, dir, (const double*)q + r * nq, (double*)pot + r * nu,
                       field ? (double*)field + 3 * r * nu : nullptr, st);
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
