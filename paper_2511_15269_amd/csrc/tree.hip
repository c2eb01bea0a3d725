// Balanced 2^s-tree by median splits (Sec. II.A) and box geometry.
//
// Every binary split of every box of one split depth runs at once.  The
// points of each box are kept in four lists: ordered by x, by y, by z
// (each by (coordinate, input index)) and by input index.  A split then
//   1. reads the box's extent along each axis from the ends of the three
//      coordinate lists and picks the longest axis (first axis on ties);
//   2. takes as pivot the point at position ceil(n/2) of that axis's list:
//      points ranked below it form the lower child (ceil(n/2) points);
//   3. stably partitions all four lists by that test (a prefix scan of the
//      flags gives every point its slot), so each child's lists stay sorted.
// Ranks along each axis come from one stable radix sort per axis of the
// order-preserving bit pattern of the coordinate, starting from index
// order, so ties in a coordinate are broken by the input index.
// The index-ordered list of the final leaves is the leaf permutation
// (points inside a leaf by input index).
//
// Box geometry (reading, the paper leaves it open): centre = midpoint of
// the tight bounding box of the box's points, radius = half its diagonal.
// Arithmetic here must round exactly like a plain IEEE evaluation in the
// written order: no contraction into fused multiply-adds.
#pragma clang fp contract(off)

#include <algorithm>
#include <climits>
#include <cmath>

#include "internal.h"

namespace fmm {
namespace {

__global__ void k_soa_keys(const double* __restrict__ pos, int n,
                           double* __restrict__ X, uint64_t* __restrict__ keys,
                           int32_t* __restrict__ iota, int* __restrict__ bad) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  iota[i] = i;
  for (int a = 0; a < 3; ++a) {
    double v = pos[3 * (int64_t)i + a];
    if (!isfinite(v)) *bad = 1;
    X[(int64_t)a * n + i] = v;
    // order-preserving bits; -0.0 is first mapped to +0.0
    uint64_t u = __double_as_longlong(v + 0.0);
    u = (u >> 63) ? ~u : (u | 0x8000000000000000ull);
    keys[(int64_t)a * n + i] = u;
  }
}

__global__ void k_ranks(const int32_t* __restrict__ sorted, int n,
                        int32_t* __restrict__ rank) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) rank[sorted[j]] = j;
}

// Geometry of the boxes of one level (= segments of the current depth).
__global__ void k_geometry(int nseg, const int32_t* __restrict__ seg_start,
                           const int32_t* __restrict__ lx,
                           const int32_t* __restrict__ ly,
                           const int32_t* __restrict__ lz,
                           const double* __restrict__ X, int n, int64_t goff,
                           double* cx, double* cy, double* cz, double* rad) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nseg) return;
  int st = seg_start[b], en = seg_start[b + 1] - 1;
  double lo0 = X[lx[st]], hi0 = X[lx[en]];
  double lo1 = X[(int64_t)n + ly[st]], hi1 = X[(int64_t)n + ly[en]];
  double lo2 = X[2 * (int64_t)n + lz[st]], hi2 = X[2 * (int64_t)n + lz[en]];
  double e0 = hi0 - lo0, e1 = hi1 - lo1, e2 = hi2 - lo2;
  cx[goff + b] = 0.5 * (lo0 + hi0);
  cy[goff + b] = 0.5 * (lo1 + hi1);
  cz[goff + b] = 0.5 * (lo2 + hi2);
  double s2 = e0 * e0;
  s2 = s2 + e1 * e1;
  s2 = s2 + e2 * e2;
  rad[goff + b] = 0.5 * sqrt(s2);
}

// Axis and pivot rank of every segment.
__global__ void k_split_prep(int nseg, const int32_t* __restrict__ seg_start,
                             const int32_t* __restrict__ lx,
                             const int32_t* __restrict__ ly,
                             const int32_t* __restrict__ lz,
                             const double* __restrict__ X, int n,
                             const int32_t* __restrict__ rank,
                             int32_t* __restrict__ axis,
                             int32_t* __restrict__ pivot) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nseg) return;
  int st = seg_start[b], cnt = seg_start[b + 1] - st, en = st + cnt - 1;
  double e0 = X[lx[en]] - X[lx[st]];
  double e1 = X[(int64_t)n + ly[en]] - X[(int64_t)n + ly[st]];
  double e2 = X[2 * (int64_t)n + lz[en]] - X[2 * (int64_t)n + lz[st]];
  int a = 0;
  double best = e0;
  if (e1 > best) { a = 1; best = e1; }
  if (e2 > best) { a = 2; }
  int half = (cnt + 1) / 2;
  const int32_t* la = a == 0 ? lx : (a == 1 ? ly : lz);
  axis[b] = a;
  pivot[b] = half < cnt ? rank[(int64_t)a * n + la[st + half]] : INT_MAX;
}

__global__ void k_flags(int n, const int32_t* __restrict__ list,
                        const int32_t* __restrict__ seg_of,
                        const int32_t* __restrict__ axis,
                        const int32_t* __restrict__ pivot,
                        const int32_t* __restrict__ rank,
                        int32_t* __restrict__ flag) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int s = seg_of[j];
  flag[j] = rank[(int64_t)axis[s] * n + list[j]] < pivot[s] ? 1 : 0;
}

__global__ void k_scatter(int n, const int32_t* __restrict__ list,
                          const int32_t* __restrict__ seg_of,
                          const int32_t* __restrict__ seg_start,
                          const int32_t* __restrict__ flag,
                          const int32_t* __restrict__ excl,
                          int32_t* __restrict__ out) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int s = seg_of[j];
  int st = seg_start[s], cnt = seg_start[s + 1] - st, half = (cnt + 1) / 2;
  int lower_before = excl[j] - excl[st];
  int dst = flag[j] ? st + lower_before : st + half + (j - st - lower_before);
  out[dst] = list[j];
}

__global__ void k_seg_update(int n, const int32_t* __restrict__ seg_start,
                             int32_t* __restrict__ seg_of) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int s = seg_of[j];
  int st = seg_start[s], cnt = seg_start[s + 1] - st, half = (cnt + 1) / 2;
  seg_of[j] = 2 * s + (j - st >= half ? 1 : 0);
}

__global__ void k_gather_pos(int n, const int32_t* __restrict__ perm,
                             const double* __restrict__ X, double* xs,
                             double* ys, double* zs) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int i = perm[j];
  xs[j] = X[i];
  ys[j] = X[(int64_t)n + i];
  zs[j] = X[2 * (int64_t)n + i];
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Hash of a position (equal positions give equal hashes; -0 and +0 alike).
__global__ void k_pos_hash(int n, const double* __restrict__ xs, const double* __restrict__ ys,
                           const double* __restrict__ zs, uint64_t* __restrict__ h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  auto bits = [](double v) { return (uint64_t)__double_as_longlong(v + 0.0); };
  uint64_t a = bits(xs[i]) * 0x9E3779B97F4A7C15ull;
  uint64_t b = bits(ys[i]) * 0xC2B2AE3D27D4EB4Full;
  uint64_t c = bits(zs[i]) * 0x165667B19E3779F9ull;
  a ^= (b << 21) | (b >> 43);
  a ^= (c << 42) | (c >> 22);
  h[i] = a ^ (a >> 29);
}

// After sorting by hash: flag a pair of coincident points.  Within a run of
// equal hashes every element is compared with up to kWalk predecessors; a
// longer run counts as coincident (conservative).
__global__ void k_dup_check(int n, const uint64_t* __restrict__ h, const int32_t* __restrict__ idx,
                            const double* __restrict__ xs, const double* __restrict__ ys,
                            const double* __restrict__ zs, int* __restrict__ flag) {
  constexpr int kWalk = 32;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 1 || i >= n || h[i] != h[i - 1]) return;
  const int a = idx[i];
  for (int j = i - 1, w = 0; j >= 0 && h[j] == h[i]; --j, ++w) {
    const int b = idx[j];
    if (w == kWalk || (xs[a] == xs[b] && ys[a] == ys[b] && zs[a] == zs[b])) {
      *flag = 1;
      return;
    }
  }
}

}  // namespace

void build_tree(fmm_plan* pl, const double* pos, hipStream_t st) {
  const int n = (int)pl->n;
  const int L = pl->L, s = pl->s;
  const int T = 256;
  Scratch sc(pl);
  double* X = (double*)sc.get(sizeof(double) * 3 * (size_t)n);
  uint64_t* keys = (uint64_t*)sc.get(sizeof(uint64_t) * 3 * (size_t)n);
  uint64_t* keys_out = (uint64_t*)sc.get(sizeof(uint64_t) * (size_t)n);
  int32_t* iota = (int32_t*)sc.get(sizeof(int32_t) * (size_t)n);
  int32_t* rank = (int32_t*)sc.get(sizeof(int32_t) * 3 * (size_t)n);
  int32_t* lists[4];
  int32_t* lists2[4];
  for (int a = 0; a < 4; ++a) {
    lists[a] = (int32_t*)sc.get(sizeof(int32_t) * (size_t)n);
    lists2[a] = (int32_t*)sc.get(sizeof(int32_t) * (size_t)n);
  }
  int* bad = (int*)sc.get(sizeof(int));
  FMM_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));

  k_soa_keys<<<blocks(n, T), T, 0, st>>>(pos, n, X, keys, iota, bad);
  FMM_HIP(hipGetLastError());
  int hbad = 0;
  FMM_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  FMM_HIP(hipStreamSynchronize(st));
  if (hbad) throw Error{FMM_EINVAL, "positions contain NaN or Inf"};

  size_t tb = sort_pairs_u64_i32_temp(n);
  void* temp = sc.get(tb);
  for (int a = 0; a < 3; ++a) {
    sort_pairs_u64_i32(temp, tb, keys + (size_t)a * n, keys_out, iota,
                       lists[a], n, st);
    k_ranks<<<blocks(n, T), T, 0, st>>>(lists[a], n, rank + (size_t)a * n);
  }
  FMM_HIP(hipMemcpyAsync(lists[3], iota, sizeof(int32_t) * n,
                         hipMemcpyDeviceToDevice, st));

  const int64_t maxseg = (int64_t)1 << (L * s);
  int32_t* seg_start_d = (int32_t*)sc.get(sizeof(int32_t) * (maxseg + 1));
  int32_t* seg_of = (int32_t*)sc.get(sizeof(int32_t) * (size_t)n);
  int32_t* axis = (int32_t*)sc.get(sizeof(int32_t) * maxseg);
  int32_t* pivot = (int32_t*)sc.get(sizeof(int32_t) * maxseg);
  int32_t* flag = (int32_t*)sc.get(sizeof(int32_t) * (size_t)n);
  int32_t* excl = (int32_t*)sc.get(sizeof(int32_t) * (size_t)n);
  size_t sb = scan_i32_temp(n);
  void* stemp = sc.get(sb);
  FMM_HIP(hipMemsetAsync(seg_of, 0, sizeof(int32_t) * n, st));

  std::vector<int32_t> seg = {0, n};
  auto upload_segs = [&]() {
    FMM_HIP(hipMemcpyAsync(seg_start_d, seg.data(), sizeof(int32_t) * seg.size(),
                           hipMemcpyHostToDevice, st));
    // seg is rewritten on the host before the next upload
    FMM_HIP(hipStreamSynchronize(st));
  };
  upload_segs();
  for (int d = 0; d < L * s; ++d) {
    const int nseg = (int)seg.size() - 1;
    if (d % s == 0) {
      int l = d / s;
      k_geometry<<<blocks(nseg, T), T, 0, st>>>(
          nseg, seg_start_d, lists[0], lists[1], lists[2], X, n,
          pl->level_off[l], pl->cx, pl->cy, pl->cz, pl->radius);
    }
    k_split_prep<<<blocks(nseg, T), T, 0, st>>>(nseg, seg_start_d, lists[0],
                                                lists[1], lists[2], X, n, rank,
                                                axis, pivot);
    for (int a = 0; a < 4; ++a) {
      k_flags<<<blocks(n, T), T, 0, st>>>(n, lists[a], seg_of, axis, pivot,
                                          rank, flag);
      exclusive_scan_i32(stemp, sb, flag, excl, n, st);
      k_scatter<<<blocks(n, T), T, 0, st>>>(n, lists[a], seg_of, seg_start_d,
                                            flag, excl, lists2[a]);
      std::swap(lists[a], lists2[a]);
    }
    k_seg_update<<<blocks(n, T), T, 0, st>>>(n, seg_start_d, seg_of);
    FMM_HIP(hipGetLastError());
    std::vector<int32_t> nxt(2 * nseg + 1);
    for (int b = 0; b < nseg; ++b) {
      int cnt = seg[b + 1] - seg[b];
      nxt[2 * b] = seg[b];
      nxt[2 * b + 1] = seg[b] + (cnt + 1) / 2;
    }
    nxt[2 * nseg] = n;
    seg.swap(nxt);
    upload_segs();
  }
  const int nseg = (int)seg.size() - 1;
  k_geometry<<<blocks(nseg, T), T, 0, st>>>(nseg, seg_start_d, lists[0],
                                            lists[1], lists[2], X, n,
                                            pl->level_off[L], pl->cx, pl->cy,
                                            pl->cz, pl->radius);
  FMM_HIP(hipMemcpyAsync(pl->perm, lists[3], sizeof(int32_t) * n,
                         hipMemcpyDeviceToDevice, st));
  FMM_HIP(hipMemcpyAsync(pl->leaf_start, seg_start_d,
                         sizeof(int32_t) * (nseg + 1), hipMemcpyDeviceToDevice,
                         st));
  k_gather_pos<<<blocks(n, T), T, 0, st>>>(n, lists[3], X, pl->xs, pl->ys,
                                           pl->zs);
  FMM_HIP(hipGetLastError());
  int mx = 0;
  for (int b = 0; b < nseg; ++b) mx = std::max(mx, seg[b + 1] - seg[b]);
  pl->max_leaf_count = mx;
  // coincident points anywhere? (P2P then guards every pair, not only the
  // pairs inside one leaf)
  k_pos_hash<<<blocks(n, T), T, 0, st>>>(n, pl->xs, pl->ys, pl->zs, keys);
  sort_pairs_u64_i32(temp, tb, keys, keys_out, iota, lists2[0], n, st);
  FMM_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
  k_dup_check<<<blocks(n, T), T, 0, st>>>(n, keys_out, lists2[0], pl->xs, pl->ys, pl->zs, bad);
  FMM_HIP(hipGetLastError());
  FMM_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  FMM_HIP(hipStreamSynchronize(st));
  pl->has_dup = hbad != 0;
}

}  // namespace fmm
