// Interaction lists by cross-level level marching (Sec. II.B).
//
// The working set of (source box, target box) pairs starts as
// (root, root), itself tested first.  Each step refines one side -- the level with the larger
// mean box radius, the source on equal means (or the target when the plan
// asks for it), the other side once one side has reached the leaves -- by
// replacing its box with each of its 2^s children, then moves every pair
// that passes the admissibility test of eq. 4,
//     max(r_a, r_b) + theta * min(r_a, r_b) <= theta * |c_a - c_b|,  d > 0,
// to the M2L list.  When both sides are at the leaf level the pairs left
// are the direct (P2P) pairs.  Each step is one expand-test kernel, a
// prefix scan of the verdicts and one compaction kernel; the host reads one
// count per step to size the next.  Both lists are finally sorted by
// (target, source) into CSR form.  Sources and targets may be two separate
// trees of the plan (Sec. II.B, separate sources and targets): each side is
// then refined by its own level-mean radii and stops at its own depth.
// Same-level lists (the enumerated procedure at the start of Sec. II.B)
// refine both sides in every step before testing, so boxes only meet boxes
// of their own level.
// The admissibility arithmetic must round like a plain IEEE evaluation in
// the written order (no fused multiply-adds), so that the verdicts do not
// depend on the compiler.
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace fmm {
namespace {

__global__ void k_expand_test(int64_t np, int nch, int refine_src, int test,
                              const int32_t* __restrict__ ps,
                              const int32_t* __restrict__ pt, int64_t off_s,
                              int64_t off_t, const double* __restrict__ cx,
                              const double* __restrict__ cy,
                              const double* __restrict__ cz,
                              const double* __restrict__ rad, double theta,
                              int32_t* __restrict__ cs, int32_t* __restrict__ ct,
                              int32_t* __restrict__ adm) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np * nch) return;
  int64_t par = e / nch;
  int c = (int)(e - par * nch);
  int32_t s = ps[par], t = pt[par];
  if (refine_src)
    s = s * nch + c;
  else
    t = t * nch + c;
  cs[e] = s;
  ct[e] = t;
  int64_t a = off_s + s, b = off_t + t;
  double dx = cx[a] - cx[b];
  double dy = cy[a] - cy[b];
  double dz = cz[a] - cz[b];
  double d2 = dx * dx;
  d2 = d2 + dy * dy;
  d2 = d2 + dz * dz;
  double d = sqrt(d2);
  double ra = rad[a], rb = rad[b];
  double big = fmax(ra, rb), small = fmin(ra, rb);
  double lhs = big + theta * small;
  double rhs = theta * d;
  adm[e] = (test && lhs <= rhs && d > 0.0) ? 1 : 0;
}

__global__ void k_compact(int64_t ne, const int32_t* __restrict__ cs,
                          const int32_t* __restrict__ ct,
                          const int32_t* __restrict__ adm,
                          const int32_t* __restrict__ excl, int64_t off_s,
                          int64_t off_t, uint64_t* __restrict__ m2l_keys,
                          int32_t* __restrict__ ns, int32_t* __restrict__ nt) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  if (adm[e]) {
    m2l_keys[excl[e]] = ((uint64_t)(off_t + ct[e]) << 32) | (uint64_t)(off_s + cs[e]);
  } else {
    int64_t k = e - excl[e];
    ns[k] = cs[e];
    nt[k] = ct[e];
  }
}

__global__ void k_keys_from_pairs(int64_t np, const int32_t* __restrict__ ps,
                                  const int32_t* __restrict__ pt, int64_t leaf_s,
                                  int64_t leaf_t, uint64_t* __restrict__ keys) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < np) keys[e] = ((uint64_t)(leaf_t + pt[e]) << 32) | (uint64_t)(leaf_s + ps[e]);
}

// CSR from keys sorted by (target, source).
__global__ void k_csr(int64_t nk, const uint64_t* __restrict__ keys,
                      int64_t ntgt, int32_t* __restrict__ src,
                      int32_t* __restrict__ ptr) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nk) src[i] = (int32_t)(keys[i] & 0xffffffffu);
  if (i <= ntgt) {
    // first key with target >= i
    int64_t lo = 0, hi = nk;
    while (lo < hi) {
      int64_t mid = (lo + hi) / 2;
      if ((int64_t)(keys[mid] >> 32) < i)
        lo = mid + 1;
      else
        hi = mid;
    }
    ptr[i] = (int32_t)lo;
  }
}

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }


// (source << 32 | target) keys of a CSR list: the reversed pairs.
__global__ void k_transposed_keys(int64_t ntgt, const int32_t* __restrict__ ptr,
                                  const int32_t* __restrict__ src,
                                  uint64_t* __restrict__ keys) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntgt) return;
  for (int32_t k = ptr[t]; k < ptr[t + 1]; ++k)
    keys[k] = ((uint64_t)src[k] << 32) | (uint64_t)t;
}

int bits_for(int64_t v) {
  int b = 1;
  while (b < 63 && ((int64_t)1 << b) <= v) ++b;
  return b;
}

// Sort (target << 32 | source) keys and write CSR arrays owned by the plan.
void keys_to_csr(fmm_plan* pl, Scratch& sc, uint64_t* keys, int64_t nk,
                 int64_t ntgt, int32_t** src, int32_t** ptr, hipStream_t st) {
  *ptr = (int32_t*)plan_alloc(pl, sizeof(int32_t) * (ntgt + 1));
  *src = (int32_t*)plan_alloc(pl, sizeof(int32_t) * std::max<int64_t>(nk, 1));
  uint64_t* sorted = (uint64_t*)sc.get(sizeof(uint64_t) * std::max<int64_t>(nk, 1));
  if (nk > 0) {
    size_t tb = sort_keys_u64_temp(nk);
    void* tmp = sc.get(tb);
    sort_keys_u64(tmp, tb, keys, sorted, nk, 32 + bits_for(ntgt), st);
  }
  int64_t nthreads = std::max(nk, ntgt + 1);
  k_csr<<<blocks(nthreads, 256), 256, 0, st>>>(nk, sorted, ntgt, *src, *ptr);
  FMM_HIP(hipGetLastError());
}

}  // namespace

// M2L work items of a list set, packed into blocks of kM2LBlock lanes so
// that the items of one target always share a block (its partial sums are
// then added inside the block, in lane order, and written once).  Each
// target's list is split into ceil(len / kItemPairs) items of equal length
// (+-1), at most kM2LBlock of them.  Blocks are filled first-fit from a
// window of the next kPackWindow targets in box order, which keeps nearby
// targets (and so their source boxes) in neighbouring blocks while leaving
// few lanes idle; the lanes a block does not fill get target -1.
void make_items(fmm_plan* pl, ListSet& S, hipStream_t st) {
  const int kItemPairs = 12, kPackWindow = 128;
  std::vector<int32_t> mptr(pl->nbox + 1);
  FMM_HIP(hipMemcpyAsync(mptr.data(), S.m2l_ptr, sizeof(int32_t) * (pl->nbox + 1),
                         hipMemcpyDeviceToHost, st));
  FMM_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> tg, ni;  // targets with a list, in box order; their item counts
  for (int64_t t = 0; t < pl->nbox; ++t) {
    const int32_t lt = mptr[t + 1] - mptr[t];
    if (lt == 0) continue;
    tg.push_back((int32_t)t);
    ni.push_back(std::min((lt + kItemPairs - 1) / kItemPairs, kM2LBlock));
  }
  std::vector<int32_t> it_t, it_b, it_e, first(pl->nbox, 0), cnt(pl->nbox, 0);
  std::vector<int32_t> seg_ptr(1, 0), seg_tgt, seg_lanes;
  std::vector<char> placed(tg.size(), 0);
  size_t j = 0;
  while (j < tg.size()) {
    int used = 0;
    for (size_t k = j; k < tg.size() && k < j + kPackWindow && used < kM2LBlock; ++k) {
      if (placed[k] || used + ni[k] > kM2LBlock) continue;
      placed[k] = 1;
      const int32_t t = tg[k], lt = mptr[t + 1] - mptr[t];
      first[t] = (int32_t)it_t.size();
      cnt[t] = ni[k];
      seg_tgt.push_back(t);
      seg_lanes.push_back(used | ((used + ni[k]) << 8));
      for (int32_t q = 0; q < ni[k]; ++q) {
        it_t.push_back(t);
        it_b.push_back(mptr[t] + (int32_t)((int64_t)lt * q / ni[k]));
        it_e.push_back(mptr[t] + (int32_t)((int64_t)lt * (q + 1) / ni[k]));
      }
      used += ni[k];
    }
    for (; used < kM2LBlock; ++used) {
      it_t.push_back(-1);
      it_b.push_back(0);
      it_e.push_back(0);
    }
    seg_ptr.push_back((int32_t)seg_tgt.size());
    while (j < tg.size() && placed[j]) ++j;
  }
  S.n_items = (int64_t)it_t.size();
  S.n_blocks = S.n_items / kM2LBlock;
  auto up = [&](const std::vector<int32_t>& v) {
    int32_t* d = (int32_t*)plan_alloc(pl, sizeof(int32_t) * std::max<size_t>(v.size(), 1));
    if (!v.empty())
      FMM_HIP(hipMemcpyAsync(d, v.data(), sizeof(int32_t) * v.size(), hipMemcpyHostToDevice, st));
    return d;
  };
  S.item_tgt = up(it_t);
  S.item_begin = up(it_b);
  S.item_end = up(it_e);
  S.item_first = up(first);
  S.item_cnt = up(cnt);
  S.seg_ptr = up(seg_ptr);
  S.seg_tgt = up(seg_tgt);
  S.seg_lanes = up(seg_lanes);
  FMM_HIP(hipStreamSynchronize(st));
}

// Near-field work items of direction dir over the target side's leaves:
// a leaf's direct list is cut into runs of source leaves of about
// kP2PItemWork interactions (a run ends before the source leaf that would
// pass the budget; a run holds at least one leaf), so that leaves with very
// long lists (clustered points) spread over many blocks.
void make_p2p_items(fmm_plan* pl, int dir, hipStream_t st) {
  ListSet& S = pl->lists[dir];
  const Side& T = tgt_side(pl, dir);
  std::vector<int32_t> ptr(pl->nleaf + 1), src(std::max<int64_t>(S.n_p2p, 1)), ls(pl->nleaf + 1);
  FMM_HIP(hipMemcpyAsync(ptr.data(), S.p2p_ptr, sizeof(int32_t) * (pl->nleaf + 1),
                         hipMemcpyDeviceToHost, st));
  if (S.n_p2p > 0)
    FMM_HIP(hipMemcpyAsync(src.data(), S.p2p_src, sizeof(int32_t) * S.n_p2p,
                           hipMemcpyDeviceToHost, st));
  FMM_HIP(hipMemcpyAsync(ls.data(), pl->leaf_start, sizeof(int32_t) * (pl->nleaf + 1),
                         hipMemcpyDeviceToHost, st));
  FMM_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> il, kb, ke, sl, sf, sc;
  std::vector<int64_t> out;
  int64_t part = 0;
  for (int64_t t = T.leaf0; t < T.leaf0 + T.nleaf; ++t) {
    const int64_t nt = ls[t + 1] - ls[t];
    const size_t first = il.size();
    int32_t b = ptr[t];
    int64_t acc = 0;
    for (int32_t k = ptr[t]; k < ptr[t + 1]; ++k) {
      const int64_t w = nt * (int64_t)(ls[src[k] + 1] - ls[src[k]]);
      if (k > b && acc + w > kP2PItemWork) {
        il.push_back((int32_t)t);
        kb.push_back(b);
        ke.push_back(k);
        b = k;
        acc = 0;
      }
      acc += w;
    }
    il.push_back((int32_t)t);
    kb.push_back(b);
    ke.push_back(ptr[t + 1]);
    const size_t cnt = il.size() - first;
    if (cnt == 1) {
      out.push_back(-1);
      continue;
    }
    for (size_t j = 0; j < cnt; ++j) {
      out.push_back(part);
      part += 4 * nt;
    }
    sl.push_back((int32_t)t);
    sf.push_back((int32_t)first);
    sc.push_back((int32_t)cnt);
  }
  auto up32 = [&](const std::vector<int32_t>& v) {
    int32_t* d = (int32_t*)plan_alloc(pl, sizeof(int32_t) * std::max<size_t>(v.size(), 1));
    if (!v.empty())
      FMM_HIP(hipMemcpyAsync(d, v.data(), sizeof(int32_t) * v.size(), hipMemcpyHostToDevice, st));
    return d;
  };
  S.n_pitems = (int64_t)il.size();
  S.n_psplit = (int64_t)sl.size();
  S.pitem_leaf = up32(il);
  S.pitem_kb = up32(kb);
  S.pitem_ke = up32(ke);
  S.psplit_leaf = up32(sl);
  S.psplit_first = up32(sf);
  S.psplit_cnt = up32(sc);
  S.pitem_out = (int64_t*)plan_alloc(pl, sizeof(int64_t) * std::max<size_t>(out.size(), 1));
  if (!out.empty())
    FMM_HIP(hipMemcpyAsync(S.pitem_out, out.data(), sizeof(int64_t) * out.size(),
                           hipMemcpyHostToDevice, st));
  S.p2p_part_elems = part;
  const size_t es = pl->prm.precision == FMM_FP32 ? sizeof(float) : sizeof(double);
  S.p2p_part = part > 0 ? plan_alloc(pl, es * (size_t)part) : nullptr;
  FMM_HIP(hipStreamSynchronize(st));
}

void build_lists(fmm_plan* pl, const TreeDesc& ts, const TreeDesc& tt, hipStream_t st) {
  const int Ls = ts.L, Lt = tt.L, nch = pl->nch;
  const int T = 256;
  Scratch sc(pl);
  // level-mean radii, summed in box order on the host
  std::vector<double> rad(pl->nbox);
  FMM_HIP(hipMemcpyAsync(rad.data(), pl->radius, sizeof(double) * pl->nbox,
                         hipMemcpyDeviceToHost, st));
  FMM_HIP(hipStreamSynchronize(st));
  // Length scale of each box's expansions: its radius, floored at 2^-30 of
  // its tree's root radius (boxes whose points coincide have radius 0).
  {
    std::vector<double> scl(rad);
    for (const TreeDesc* t : {&ts, &tt}) {
      const double r0 = rad[t->box_base];
      const double floor_r = r0 > 0.0 ? std::ldexp(r0, -30) : 1.0;
      for (int64_t b = t->box_base; b < t->box_base + t->level_off[t->L + 1]; ++b)
        scl[b] = std::max(rad[b], floor_r);
    }
    FMM_HIP(hipMemcpyAsync(pl->scale, scl.data(), sizeof(double) * pl->nbox,
                           hipMemcpyHostToDevice, st));
    FMM_HIP(hipStreamSynchronize(st));
  }
  auto level_means = [&](const TreeDesc& t) {
    std::vector<double> avg(t.L + 1);
    for (int l = 0; l <= t.L; ++l) {
      double acc = 0.0;
      for (int64_t b = t.level_off[l]; b < t.level_off[l + 1]; ++b) acc += rad[t.box_base + b];
      avg[l] = acc / (double)(t.level_off[l + 1] - t.level_off[l]);
    }
    return avg;
  };
  const std::vector<double> avg_s = level_means(ts), avg_t = level_means(tt);

  std::vector<std::pair<uint64_t*, int64_t>> m2l_parts;
  int64_t n_m2l = 0;
  int64_t np = 1;
  // The march starts with the pair of roots; two separate hierarchies may be
  // well separated as a whole (with one tree the roots coincide, d = 0, and
  // never are).  Tested on the host in the kernel's arithmetic order.
  {
    std::vector<double> c(6);
    for (int a = 0; a < 3; ++a) {
      double* arr[3] = {pl->cx, pl->cy, pl->cz};
      FMM_HIP(hipMemcpyAsync(&c[a], arr[a] + ts.box_base, sizeof(double), hipMemcpyDeviceToHost, st));
      FMM_HIP(hipMemcpyAsync(&c[3 + a], arr[a] + tt.box_base, sizeof(double),
                             hipMemcpyDeviceToHost, st));
    }
    FMM_HIP(hipStreamSynchronize(st));
    double dx = c[0] - c[3];
    double dy = c[1] - c[4];
    double dz = c[2] - c[5];
    double d2 = dx * dx;
    d2 = d2 + dy * dy;
    d2 = d2 + dz * dz;
    const double d = std::sqrt(d2);
    const double ra = rad[ts.box_base], rb = rad[tt.box_base];
    const double big = std::fmax(ra, rb), small = std::fmin(ra, rb);
    const double lhs = big + pl->prm.theta * small;
    const double rhs = pl->prm.theta * d;
    if (lhs <= rhs && d > 0.0) {
      uint64_t* k = (uint64_t*)sc.get(sizeof(uint64_t));
      const uint64_t key = ((uint64_t)tt.box_base << 32) | (uint64_t)ts.box_base;
      FMM_HIP(hipMemcpyAsync(k, &key, sizeof(uint64_t), hipMemcpyHostToDevice, st));
      FMM_HIP(hipStreamSynchronize(st));
      m2l_parts.emplace_back(k, 1);
      n_m2l = 1;
      np = 0;
    }
  }
  int32_t* ps = (int32_t*)sc.get(sizeof(int32_t));
  int32_t* pt = (int32_t*)sc.get(sizeof(int32_t));
  FMM_HIP(hipMemsetAsync(ps, 0, sizeof(int32_t), st));
  FMM_HIP(hipMemsetAsync(pt, 0, sizeof(int32_t), st));
  int ls = 0, lt = 0;
  // One refinement of one side; with test, admissible pairs leave the
  // working set for the M2L list.
  auto step = [&](bool src_side, bool test) {
    if (src_side) ++ls; else ++lt;
    const int64_t ne = np * nch;
    int32_t* cs = (int32_t*)sc.get(sizeof(int32_t) * ne);
    int32_t* ct = (int32_t*)sc.get(sizeof(int32_t) * ne);
    int32_t* adm = (int32_t*)sc.get(sizeof(int32_t) * ne);
    int32_t* excl = (int32_t*)sc.get(sizeof(int32_t) * ne);
    const int64_t off_s = ts.box_base + ts.level_off[ls], off_t = tt.box_base + tt.level_off[lt];
    k_expand_test<<<blocks(ne, T), T, 0, st>>>(
        np, nch, src_side ? 1 : 0, test ? 1 : 0, ps, pt, off_s, off_t,
        pl->cx, pl->cy, pl->cz, pl->radius, pl->prm.theta, cs, ct, adm);
    FMM_HIP(hipGetLastError());
    size_t tb = scan_i32_temp(ne);
    void* tmp = sc.get(tb);
    exclusive_scan_i32(tmp, tb, adm, excl, ne, st);
    int32_t last_excl = 0, last_adm = 0;
    FMM_HIP(hipMemcpyAsync(&last_excl, excl + ne - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FMM_HIP(hipMemcpyAsync(&last_adm, adm + ne - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FMM_HIP(hipStreamSynchronize(st));
    const int64_t nadm = (int64_t)last_excl + last_adm;
    uint64_t* keys = (uint64_t*)sc.get(sizeof(uint64_t) * std::max<int64_t>(nadm, 1));
    int32_t* ns = (int32_t*)sc.get(sizeof(int32_t) * std::max<int64_t>(ne - nadm, 1));
    int32_t* nt = (int32_t*)sc.get(sizeof(int32_t) * std::max<int64_t>(ne - nadm, 1));
    k_compact<<<blocks(ne, T), T, 0, st>>>(ne, cs, ct, adm, excl, off_s, off_t, keys, ns, nt);
    FMM_HIP(hipGetLastError());
    if (nadm > 0) m2l_parts.emplace_back(keys, nadm);
    n_m2l += nadm;
    ps = ns;
    pt = nt;
    np = ne - nadm;
  };
  const bool same_level = pl->prm.lists == FMM_LISTS_SAME_LEVEL;
  while (np > 0 && !(ls == Ls && lt == Lt)) {
    if (same_level && ls < Ls && lt < Lt) {
      // same-level lists: both sides advance, then the pairs are tested
      step(true, false);
      step(false, true);
      continue;
    }
    bool src_side;
    if (ls == Ls)
      src_side = false;
    else if (lt == Lt)
      src_side = true;
    else if (avg_s[ls] > avg_t[lt])
      src_side = true;
    else if (avg_s[ls] < avg_t[lt])
      src_side = false;
    else
      src_side = pl->prm.tie_refine == FMM_TIE_SOURCE;
    step(src_side, true);
  }
  // M2L CSR over all target boxes
  uint64_t* all = (uint64_t*)sc.get(sizeof(uint64_t) * std::max<int64_t>(n_m2l, 1));
  int64_t o = 0;
  for (auto& pr : m2l_parts) {
    FMM_HIP(hipMemcpyAsync(all + o, pr.first, sizeof(uint64_t) * pr.second,
                           hipMemcpyDeviceToDevice, st));
    o += pr.second;
  }
  ListSet& F = pl->lists[0];
  ListSet& A = pl->lists[1];
  keys_to_csr(pl, sc, all, n_m2l, pl->nbox, &F.m2l_src, &F.m2l_ptr, st);
  F.n_m2l = A.n_m2l = n_m2l;
  // P2P CSR over leaves (what is left once both sides reached the leaves),
  // leaves numbered globally
  if (!(ls == Ls && lt == Lt)) np = 0;
  uint64_t* pk = (uint64_t*)sc.get(sizeof(uint64_t) * std::max<int64_t>(np, 1));
  if (np > 0) {
    k_keys_from_pairs<<<blocks(np, T), T, 0, st>>>(np, ps, pt, ts.leaf_base, tt.leaf_base, pk);
    FMM_HIP(hipGetLastError());
  }
  keys_to_csr(pl, sc, pk, np, pl->nleaf, &F.p2p_src, &F.p2p_ptr, st);
  F.n_p2p = A.n_p2p = np;
  // transposed lists: every (source, target) pair reversed
  uint64_t* tk = (uint64_t*)sc.get(sizeof(uint64_t) * std::max<int64_t>(std::max(n_m2l, np), 1));
  k_transposed_keys<<<blocks(pl->nbox, T), T, 0, st>>>(pl->nbox, F.m2l_ptr, F.m2l_src, tk);
  keys_to_csr(pl, sc, tk, n_m2l, pl->nbox, &A.m2l_src, &A.m2l_ptr, st);
  k_transposed_keys<<<blocks(pl->nleaf, T), T, 0, st>>>(pl->nleaf, F.p2p_ptr, F.p2p_src, tk);
  keys_to_csr(pl, sc, tk, np, pl->nleaf, &A.p2p_src, &A.p2p_ptr, st);
  FMM_HIP(hipGetLastError());

  // P2P interaction count (same in both directions)
  std::vector<int32_t> pptr(pl->nleaf + 1), psrc(std::max<int64_t>(np, 1)),
      lstart(pl->nleaf + 1);
  FMM_HIP(hipMemcpyAsync(pptr.data(), F.p2p_ptr, sizeof(int32_t) * (pl->nleaf + 1),
                         hipMemcpyDeviceToHost, st));
  FMM_HIP(hipMemcpyAsync(psrc.data(), F.p2p_src, sizeof(int32_t) * psrc.size(),
                         hipMemcpyDeviceToHost, st));
  FMM_HIP(hipMemcpyAsync(lstart.data(), pl->leaf_start, sizeof(int32_t) * (pl->nleaf + 1),
                         hipMemcpyDeviceToHost, st));
  FMM_HIP(hipStreamSynchronize(st));
  int64_t inter = 0;
  for (int64_t t = 0; t < pl->nleaf; ++t)
    for (int32_t k = pptr[t]; k < pptr[t + 1]; ++k)
      inter += (int64_t)(lstart[t + 1] - lstart[t]) * (lstart[psrc[k] + 1] - lstart[psrc[k]]);
  pl->p2p_inter = inter;
  make_items(pl, F, st);
  make_items(pl, A, st);
  make_p2p_items(pl, 0, st);
  make_p2p_items(pl, 1, st);
}

}  // namespace fmm
