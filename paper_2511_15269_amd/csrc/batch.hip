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
//         wave (one per half-wave); M2M translates the children of a parent
//         in parallel waves and adds them in child order.
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

#include <type_traits>

#include "internal.h"
#include "ops.h"
#include "tables.h"

namespace fmm {
namespace {

using namespace ops;
constexpr int kRB = 32;

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Neumaier's compensated addition, elementwise: s + c carries the sum.
__device__ __forceinline__ void neumaier4(floatx4& s, floatx4& c, floatx4 x) {
  const floatx4 t = s + x;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const float sv = s[v], xv = x[v], tv = t[v];
    c[v] += fabsf(sv) >= fabsf(xv) ? (sv - tv) + xv : (xv - tv) + sv;
  }
  s = t;
}

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
// The sort stage: the caller's charges (vector-major [R][n], input order)
// to leaf order with the 32 vectors innermost ([n][32], zero beyond R), for
// P2M and P2P.  Block = 64 consecutive input indices: their R rows are read
// as 256-byte runs into an LDS tile, then each point's 32 charges go out as
// one 128-byte row at its leaf position (iperm).
__global__ __launch_bounds__(256) void k_bgather(int64_t n, int R,
                                                 const int32_t* __restrict__ iperm,
                                                 const float* __restrict__ q,
                                                 float* __restrict__ qL) {
  __shared__ float T[kRB][64 + 1];
  const int64_t o0 = (int64_t)blockIdx.x * 64;
  for (int e = threadIdx.x; e < kRB * 64; e += blockDim.x) {
    const int r = e / 64, c = e % 64;
    const int64_t o = o0 + c;
    T[r][c] = (r < R && o < n) ? q[(int64_t)r * n + o] : 0.f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * kRB; e += blockDim.x) {
    const int c = e / kRB, r = e % kRB;
    const int64_t o = o0 + c;
    if (o < n) qL[(int64_t)iperm[o] * kRB + r] = T[r][c];
  }
}

// P2M as a contraction on the matrix cores: C[k][r] = normc_k sum_p
// R_k(y_p) q[p][r] for the 32 vectors r.  The basis values of up to 64
// points are formed in LDS (one lane per point); then v_mfma_f32_32x32x2f32
// takes two points per step: A = basis of 32 coefficients (rows, one tile
// of three) x 2 points, B = charges of the 2 points x 32 vectors.
// Accumulator register v of lane l holds coefficient row
// 8 (v / 4) + 4 (l / 32) + v % 4 of the tile, vector l % 32.  One wave per
// tile of 32 coefficients, the basis and charge tiles shared in LDS.  The
// charges come leaf-ordered from k_bgather.
template <int P>
__global__ __launch_bounds__(64 * ((K_<P>::value + 31) / 32)) void k_bp2m(
    const int32_t* __restrict__ leaf_box, const int32_t* __restrict__ leaf_start,
    const double* __restrict__ xs, const double* __restrict__ ys,
    const double* __restrict__ zs, const float* __restrict__ qL,
    const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const float* __restrict__ tab, float* __restrict__ C) {
  constexpr int K = K_<P>::value;
  constexpr int NT = (K + 31) / 32;  // coefficient tiles, one wave each
  __shared__ float B[64][NT * 32 + 1];
  __shared__ float Q[64][kRB];  // charges of the chunk's points
  const int leaf = blockIdx.x;
  const int lane = threadIdx.x % 64;
  const int t = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);  // this wave's tile
  const int col = lane % 32, kh = lane / 32;
  const int64_t g = leaf_box[leaf];
  const int st = leaf_start[leaf], en = leaf_start[leaf + 1];
  const double ox = cx[g], oy = cy[g], oz = cz[g], ir = 1.0 / scale[g];
  floatx16 acc = {};
  for (int c0 = st; c0 < en; c0 += 64) {
    const int cnt = min(64, en - c0);
    __syncthreads();
    if (t == 0) {
      // the first wave forms the basis (lane = point); padding rows and
      // missing points read as zero
      const int j = c0 + lane;
      const bool pt = j < en;
      const int jj = pt ? j : c0;
#pragma unroll
      for (int k = K; k < NT * 32; ++k) B[lane][k] = 0.f;
      regular_basis<P, float>(float((xs[jj] - ox) * ir), float((ys[jj] - oy) * ir),
                              float((zs[jj] - oz) * ir),
                              [&](int k, float v) { B[lane][k] = pt ? v : 0.f; });
    }
    for (int e = threadIdx.x; e < cnt * kRB; e += blockDim.x)
      Q[e / kRB][e % kRB] = qL[(int64_t)c0 * kRB + e];
    __syncthreads();
    for (int p0 = 0; p0 < cnt; p0 += 2) {
      const int pp = p0 + kh;
      const float b = pp < cnt ? Q[pp][col] : 0.f;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(B[pp < 64 ? pp : 0][t * 32 + col], b, acc, 0, 0,
                                                 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int k = t * 32 + 8 * (v / 4) + 4 * kh + v % 4;
    if (k < K) C[(g * K + k) * kRB + col] = acc[v] * tab[tab_normc(P) + k];
  }
}

// parent = sum over its 2^s children of M2M(child), 32 vectors per parent:
// wave c of a block of 2^s waves translates child c of two parents (one
// per half-wave, lane = vector), and the translated children are added in
// child order through an LDS tile (one barrier per child).
template <int P>
__global__ __launch_bounds__(512) void k_bm2m_par(
    int64_t npar, const int32_t* __restrict__ par, const int32_t* __restrict__ child0, int s,
    const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ cz, const double* __restrict__ scale,
    const float* __restrict__ tab, float* C) {
  constexpr int K = K_<P>::value;
  __shared__ float A[2][K][kRB];
  const int c = threadIdx.x / 64;  // child (wave-uniform)
  const int lane = threadIdx.x % 64;
  const int h = lane / kRB, r = lane % kRB;
  const int64_t b = (int64_t)blockIdx.x * 2 + h;
  const bool live = b < npar;
  const int64_t pa = live ? par[b] : 0;
  const int64_t ch = live ? child0[b] + c : 0;
  float v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = live ? C[(ch * K + k) * kRB + r] : 0.f;
  if (live)
    rotate_shift<P, kM2M, float>(v, cx[ch] - cx[pa], cy[ch] - cy[pa], cz[ch] - cz[pa],
                                 scale[ch], scale[pa], tab);
  const int nch = 1 << s;
  for (int step = 0; step < nch; ++step) {
    if (c == step) {
#pragma unroll
      for (int k = 0; k < K; ++k) A[h][k][r] = (step == 0 ? 0.f : A[h][k][r]) + v[k];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < 2 * K * kRB; e += blockDim.x) {
    const int hh = e / (K * kRB), kr = e % (K * kRB);
    const int64_t bb = (int64_t)blockIdx.x * 2 + hh;
    if (bb < npar) C[(int64_t)par[bb] * K * kRB + kr] = A[hh][kr / kRB][kr % kRB];
  }
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
  if (t < 0) return;  // idle lane of the packed item layout
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

// L2P as a contraction on the matrix cores: for 32 points at a time,
// u[p][r] = sum_k R_k(y_p) w_k D[k][r] and likewise the three gradient
// components.  The basis and its gradient are formed in LDS (one lane per
// point, first wave); v_mfma_f32_32x32x2f32 then takes two coefficients per
// step: A = basis values of 32 points (rows) x 2 coefficients, B = weighted
// local coefficients (2 x 32 vectors).  The block's four waves share the
// basis tile, wave c forming component c (potential, then the gradient's
// x, y, z), so that a 43 KiB tile serves four waves.  Accumulator register
// v of lane l holds point row 8 (v / 4) + 4 (l / 32) + v % 4, vector l % 32.
template <int P>
__global__ __launch_bounds__(256) void k_bl2p(
    const int32_t* __restrict__ leaf_box, const int32_t* __restrict__ leaf_start,
    const double* __restrict__ xs, const double* __restrict__ ys,
    const double* __restrict__ zs, const double* __restrict__ cx,
    const double* __restrict__ cy, const double* __restrict__ cz,
    const double* __restrict__ scale, const float* __restrict__ D,
    const float* __restrict__ tab, float* __restrict__ potL, float* __restrict__ fldL) {
  constexpr int K = K_<P>::value;
  constexpr int K2 = (K + 1) / 2 * 2;  // coefficient pairs (one zero row padded)
  constexpr int NP = 32;
  __shared__ float Bv[4][K2][NP + 1];
  const int leaf = blockIdx.x;
  const int lane = threadIdx.x % 64;
  const int comp = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);  // component of this wave
  const int col = lane % 32, kh = lane / 32;
  const int64_t g = leaf_box[leaf];
  const int st = leaf_start[leaf], en = leaf_start[leaf + 1];
  const double ox = cx[g], oy = cy[g], oz = cz[g], ir = 1.0 / scale[g];
  const float fu = float(-kInv4Pi * ir), ff = float(kInv4Pi * ir * ir);
  for (int c0 = st; c0 < en; c0 += NP) {
    const int cnt = min(NP, en - c0);
    __syncthreads();
    if (threadIdx.x < NP) {
      const bool pt = lane < cnt;
      const int j = pt ? c0 + lane : c0;
      const float x = float((xs[j] - ox) * ir), y = float((ys[j] - oy) * ir),
                  z = float((zs[j] - oz) * ir);
      basis_with_gradient<P, float>(x, y, z, [&](int k, float v, float gx, float gy, float gz) {
        Bv[0][k][lane] = pt ? v : 0.f;
        Bv[1][k][lane] = pt ? gx : 0.f;
        Bv[2][k][lane] = pt ? gy : 0.f;
        Bv[3][k][lane] = pt ? gz : 0.f;
      });
      if (K2 > K) {
#pragma unroll
        for (int c = 0; c < 4; ++c) Bv[c][K2 - 1][lane] = 0.f;
      }
    }
    __syncthreads();
    floatx16 acc = {};
    for (int k0 = 0; k0 < K2; k0 += 2) {
      const int k = k0 + kh;
      const float b = k < K ? D[(g * K + k) * kRB + col] * tab[tab_l2p(P) + k] : 0.f;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(Bv[comp][k][col], b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int pnt = 8 * (v / 4) + 4 * kh + v % 4;
      if (pnt < cnt) {
        const int64_t o = c0 + pnt;
        if (comp == 0)
          potL[o * kRB + col] = fu * acc[v];
        else
          fldL[(o * 3 + comp - 1) * kRB + col] = ff * acc[v];
      }
    }
  }
}

// P2P on the matrix cores (v_mfma_f32_16x16x4f32).  A tile is 16 targets
// (rows) x 32 vectors (columns, two 16-column halves); every step takes four
// source points: lane l computes the kernel entries of target (l % 16) and
// source (l / 16) -- the A operand -- and supplies the charges of source
// (l / 16) for vectors (l % 16) and 16 + (l % 16) -- the B operands of the
// two halves.  Accumulator register v of lane l holds row 4 (l / 16) + v,
// column l % 16 (+16 in the second half).  Source points (positions and the
// 32 charges) are staged in LDS, up to kStage points at a time, with
// coalesced loads.  A block holds TW waves, one 16-target tile each, that
// share every staged chunk.  Small tiles keep the accumulators to 32
// registers per lane; the kernel is held to three waves per SIMD (146
// registers, no spills), so that the kernel values of one wave's next step
// are computed while another wave's MFMAs run.
constexpr int kStage = 64;

template <int TW>
__global__ __launch_bounds__(64 * TW) __attribute__((amdgpu_waves_per_eu(3))) void k_bp2p(
    const int32_t* __restrict__ leaf_start, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs,
    const float* __restrict__ qL, const int32_t* __restrict__ p2p_ptr,
    const int32_t* __restrict__ p2p_src, float* __restrict__ potL, float* __restrict__ fldL) {
  __shared__ double px[kStage], py[kStage], pz[kStage];
  // charge rows padded to 48 floats: the four source rows a step reads sit
  // 16 banks apart, so a half-wave's 32 lanes hit 32 distinct banks
  constexpr int kQS = kRB + 16;
  __shared__ __align__(16) float qs[kStage][kQS];
  const int leaf = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid % 64, wv = tid / 64;
  const int row = lane % 16, kk = lane / 16;
  const int st = leaf_start[leaf], en = leaf_start[leaf + 1];
  const int pb = p2p_ptr[leaf], pe = p2p_ptr[leaf + 1];
  // every wave runs the same number of tiles (barriers inside)
  const int ntile = (en - st + 16 * TW - 1) / (16 * TW);
  for (int tl = 0; tl < ntile; ++tl) {
    const int i0 = st + 16 * (tl * TW + wv);
    const int i = i0 + row;
    const bool live_i = i < en;
    const int ii = live_i ? i : st;
    const double xi = xs[ii], yi = ys[ii], zi = zs[ii];
    // running sums (s*) with Neumaier compensation (c*) for the two column
    // halves (0, 1); each source leaf is accumulated on the matrix cores
    // from zero and then added
    floatx4 su0 = {}, sx0 = {}, sy0 = {}, sz0 = {}, su1 = {}, sx1 = {}, sy1 = {}, sz1 = {};
    floatx4 cu0 = {}, cx0 = {}, cy0 = {}, cz0 = {}, cu1 = {}, cx1 = {}, cy1 = {}, cz1 = {};
    for (int k = pb; k < pe; ++k) {
      const int sl = p2p_src[k];
      const int js = leaf_start[sl], je = leaf_start[sl + 1];
      floatx4 au0 = {}, ax0 = {}, ay0 = {}, az0 = {}, au1 = {}, ax1 = {}, ay1 = {}, az1 = {};
      for (int c0 = js; c0 < je; c0 += kStage) {
        const int cnt = min(kStage, je - c0);
        __syncthreads();  // the previous chunk's reads are done
        if (tid < cnt) {
          px[tid] = xs[c0 + tid];
          py[tid] = ys[c0 + tid];
          pz[tid] = zs[c0 + tid];
        }
        {
          const float4* from = reinterpret_cast<const float4*>(qL + (int64_t)c0 * kRB);
          for (int e = tid; e < cnt * (kRB / 4); e += 64 * TW)
            *reinterpret_cast<float4*>(&qs[e / (kRB / 4)][4 * (e % (kRB / 4))]) = from[e];
        }
        __syncthreads();
        // one step: four source points j0 .. j0+3 (lane group kk takes j0+kk)
        auto step = [&](int j0, auto check_tag) {
          constexpr bool CHECK = decltype(check_tag)::value;
          const int j = j0 + kk;
          const bool live_j = !CHECK || j < cnt;
          const int jj = CHECK ? (live_j ? j : 0) : j;
          const float dx = float(xi - px[jj]), dy = float(yi - py[jj]), dz = float(zi - pz[jj]);
          const float r2 = dx * dx + dy * dy + dz * dz;
          const float inv0 = __builtin_amdgcn_rsqf(r2);
          const float inv = (r2 > 0.f && live_i && live_j) ? inv0 : 0.f;
          const float inv3 = inv * inv * inv;
          const float q0 = qs[jj][row], q1 = qs[jj][16 + row];
          const float b0 = live_j ? q0 : 0.f;
          const float b1 = live_j ? q1 : 0.f;
          const float ex = dx * inv3, ey = dy * inv3, ez = dz * inv3;
          au0 = __builtin_amdgcn_mfma_f32_16x16x4f32(inv, b0, au0, 0, 0, 0);
          au1 = __builtin_amdgcn_mfma_f32_16x16x4f32(inv, b1, au1, 0, 0, 0);
          ax0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ex, b0, ax0, 0, 0, 0);
          ax1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ex, b1, ax1, 0, 0, 0);
          ay0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ey, b0, ay0, 0, 0, 0);
          ay1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ey, b1, ay1, 0, 0, 0);
          az0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ez, b0, az0, 0, 0, 0);
          az1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ez, b1, az1, 0, 0, 0);
        };
        int j0 = 0;
        for (; j0 + 16 <= cnt; j0 += 16) {
#pragma unroll
          for (int u = 0; u < 4; ++u) step(j0 + 4 * u, std::false_type{});
        }
        for (; j0 < cnt; j0 += 4) step(j0, std::true_type{});
      }
      neumaier4(su0, cu0, au0);
      neumaier4(sx0, cx0, ax0);
      neumaier4(sy0, cy0, ay0);
      neumaier4(sz0, cz0, az0);
      neumaier4(su1, cu1, au1);
      neumaier4(sx1, cx1, ax1);
      neumaier4(sy1, cy1, ay1);
      neumaier4(sz1, cz1, az1);
    }
    const floatx4 U[2] = {su0 + cu0, su1 + cu1}, X[2] = {sx0 + cx0, sx1 + cx1},
                  Y[2] = {sy0 + cy0, sy1 + cy1}, Z[2] = {sz0 + cz0, sz1 + cz1};
    const float c = float(kInv4Pi);
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      const int col = 16 * hf + row;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ti = i0 + 4 * kk + v;
        if (ti < en) {
          const int64_t o = ti;
          potL[o * kRB + col] += -c * U[hf][v];
          // field = -grad u; grad of the near part is +(1/4pi) sum q d/r^3
          fldL[(o * 3 + 0) * kRB + col] -= c * X[hf][v];
          fldL[(o * 3 + 1) * kRB + col] -= c * Y[hf][v];
          fldL[(o * 3 + 2) * kRB + col] -= c * Z[hf][v];
        }
      }
    }
  }
}

// Leaf-ordered [n][32] results to the caller's [R][n] and [R][n][3].
// Block = 64 consecutive output (input-order) indices: each point's
// 32-vector rows are read as 128-byte runs from its leaf position (iperm)
// into LDS tiles, then every vector's outputs for the 64 points go out as
// contiguous runs (256 bytes of potential, 768 bytes of field).
__global__ __launch_bounds__(256) void k_bscatter(int64_t n, int R,
                                                  const int32_t* __restrict__ iperm,
                                                  const float* __restrict__ potL,
                                                  const float* __restrict__ fldL,
                                                  float* __restrict__ pot,
                                                  float* __restrict__ field) {
  __shared__ float U[64][kRB + 1];
  __shared__ float F[3 * 64][kRB + 1];
  const int64_t o0 = (int64_t)blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * kRB; e += blockDim.x) {
    const int c = e / kRB, r = e % kRB;
    const int64_t o = o0 + c;
    U[c][r] = o < n ? potL[(int64_t)iperm[o] * kRB + r] : 0.f;
  }
  if (field)
    for (int e = threadIdx.x; e < 3 * 64 * kRB; e += blockDim.x) {
      const int ca = e / kRB, r = e % kRB;
      const int64_t o = o0 + ca / 3;
      F[ca][r] = o < n ? fldL[((int64_t)iperm[o] * 3 + ca % 3) * kRB + r] : 0.f;
    }
  __syncthreads();
  for (int e = threadIdx.x; e < kRB * 64; e += blockDim.x) {
    const int r = e / 64, c = e % 64;
    if (r < R && o0 + c < n) pot[(int64_t)r * n + o0 + c] = U[c][r];
  }
  if (field)
    for (int e = threadIdx.x; e < kRB * 3 * 64; e += blockDim.x) {
      const int r = e / (3 * 64), ca = e % (3 * 64);
      if (r < R && o0 + ca / 3 < n) field[((int64_t)r * n + o0) * 3 + ca] = F[ca][r];
    }
}

// iperm[perm[j]] = j: leaf position of every input index
__global__ void k_invert(int64_t n, const int32_t* __restrict__ perm, int32_t* __restrict__ iperm) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) iperm[perm[j]] = (int32_t)j;
}

template <int P>
void run_batch(fmm_plan* pl, const ListSet& Ls, const float* q, int R, float* pot,
               float* field, hipStream_t st) {
  const int s = pl->s;
  const float* tab = (const float*)pl->tables;
  float* qL = (float*)pl->ws.bq;
  float* C = (float*)pl->ws.bC;
  float* D = (float*)pl->ws.bD;
  float* part = (float*)pl->bpart;
  float* potL = (float*)pl->ws.bpot;
  float* fldL = (float*)pl->ws.bfld;
  const int64_t n = pl->n;
  StageMarks mk(pl);
  // the sort stage is folded into P2M; its timing slot stays empty
  mk.begin(kStSort, st);
  mk.end(kStSort, st);
  mk.begin(kStP2M, st);
  k_bgather<<<blocks(n, 64), 256, 0, st>>>(n, R, pl->iperm, q, qL);
  k_bp2m<P><<<(unsigned)pl->nleaf, 64 * ((K_<P>::value + 31) / 32), 0, st>>>(
      pl->leaf_box, pl->leaf_start, pl->xs, pl->ys, pl->zs, qL, pl->cx, pl->cy, pl->cz,
      pl->scale, tab, C);
  mk.end(kStP2M, st);
  mk.begin(kStM2M, st);
  for (const Step& S : pl->side[0].m2m_steps)
    k_bm2m_par<P><<<blocks(S.n, 2), 64 << s, 0, st>>>(S.n, S.a, S.b, s, pl->cx, pl->cy, pl->cz,
                                                      pl->scale, tab, C);
  mk.end(kStM2M, st);
  mk.begin(kStM2L, st);
  if (Ls.n_items > 0)
    k_bm2l<P><<<blocks(Ls.n_items, 2), 64, 0, st>>>(Ls.n_items, Ls.item_tgt, Ls.item_begin,
                                                    Ls.item_end, Ls.m2l_src, pl->cx, pl->cy,
                                                    pl->cz, pl->scale, C, tab, part);
  mk.end(kStM2L, st);
  mk.begin(kStL2L, st);
  const Step& all = pl->side[0].l2l_sum;
  if (all.n > 0)
    k_psum<float><<<(unsigned)all.n, 256, 0, st>>>(all.n, all.a, Ls.item_first, Ls.item_cnt,
                                                   part, K_<P>::value * kRB, D);
  for (const Step& S : pl->side[0].l2l_steps)
    k_bl2l<P><<<blocks(S.n, 2), 64, 0, st>>>(S.n, S.a, S.b, pl->cx, pl->cy, pl->cz, pl->scale,
                                             tab, D);
  mk.end(kStL2L, st);
  mk.begin(kStL2P, st);
  k_bl2p<P><<<(unsigned)pl->nleaf, 256, 0, st>>>(pl->leaf_box, pl->leaf_start, pl->xs, pl->ys,
                                                pl->zs, pl->cx, pl->cy, pl->cz, pl->scale, D,
                                                tab, potL, fldL);
  mk.end(kStL2P, st);
  mk.begin(kStP2P, st);
  {
    const int TW = batch_p2p_waves(pl);
    auto p2p = [&](auto kern, int tw) {
      kern<<<(unsigned)pl->nleaf, 64 * tw, 0, st>>>(pl->leaf_start, pl->xs, pl->ys, pl->zs, qL,
                                                     Ls.p2p_ptr, Ls.p2p_src, potL, fldL);
    };
    if (TW == 1) p2p(k_bp2p<1>, 1);
    else if (TW == 2) p2p(k_bp2p<2>, 2);
    else if (TW == 4) p2p(k_bp2p<4>, 4);
    else p2p(k_bp2p<8>, 8);
  }
  k_bscatter<<<blocks(n, 64), 256, 0, st>>>(n, R, pl->iperm, potL, fldL, pot, field);
  mk.end(kStP2P, st);
  FMM_HIP(hipGetLastError());
}

}  // namespace

int batch_width() { return kRB; }

int batch_p2p_waves(const fmm_plan* pl) {
  const int w = pl->batch_p2p_waves;
  if (w == 1 || w == 2 || w == 4 || w == 8) return w;
  const int mlc = pl->max_leaf_count;
  return mlc > 64 ? 8 : (mlc > 32 ? 4 : (mlc > 16 ? 2 : 1));
}

void make_iperm(fmm_plan* pl, hipStream_t st) {
  k_invert<<<blocks(pl->n, 256), 256, 0, st>>>(pl->n, pl->perm, pl->iperm);
  FMM_HIP(hipGetLastError());
}

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
