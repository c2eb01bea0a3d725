// Interaction lists by cross-level level marching (Sec. II.B).
//
// The working set of (source box, target box) pairs starts as
// (root, root).  Each step refines one side -- the level with the larger
// mean box radius, the source on equal means (or the target when the plan
// asks for it), the other side once one side has reached the leaves -- by
// replacing its box with each of its 2^s children, then moves every pair
// that passes the admissibility test of eq. 4,
//     max(r_a, r_b) + theta * min(r_a, r_b) <= theta * |c_a - c_b|,  d > 0,
// to the M2L list.  When both sides are at the leaf level the pairs left
// are the direct (P2P) pairs.  Each step is one expand-test kernel, a
// prefix scan of the verdicts and one compaction kernel; the host reads one
// count per step to size the next.  Both lists are finally sorted by
// (target, source) into CSR form.
// The admissibility arithmetic must round like a plain IEEE evaluation in
// the written order (no fused multiply-adds), so that the verdicts do not
// depend on the compiler.
#pragma clang fp contract(off)

#include <algorithm>
#include <cmath>

#include "internal.h"

namespace fmm {
namespace {

__global__ void k_expand_test(int64_t np, int nch, int refine_src,
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
  adm[e] = (lhs <= rhs && d > 0.0) ? 1 : 0;
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
                                  const int32_t* __restrict__ pt,
                                  uint64_t* __restrict__ keys) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < np) keys[e] = ((uint64_t)pt[e] << 32) | (uint64_t)ps[e];
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

struct Scratch {
  std::vector<void*> ptrs;
  void* get(size_t bytes) {
    void* p = nullptr;
    FMM_HIP(hipMalloc(&p, std::max<size_t>(bytes, 16)));
    ptrs.push_back(p);
    return p;
  }
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

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

// M2L work items of a list set: consecutive per target, each target's list
// split into ceil(len / kItemPairs) items of equal length (+-1).  Shorter
// items give more, more even work units (M2L runs one wave per SIMD, so the
// last round of waves is what items of 16 leave unbalanced) at the price of
// more partial rows for the sum before L2L; 12 measured best.
void make_items(fmm_plan* pl, ListSet& S, hipStream_t st) {
  const int kItemPairs = 12;
  std::vector<int32_t> mptr(pl->nbox + 1);
  FMM_HIP(hipMemcpyAsync(mptr.data(), S.m2l_ptr, sizeof(int32_t) * (pl->nbox + 1),
                         hipMemcpyDeviceToHost, st));
  FMM_HIP(hipStreamSynchronize(st));
  std::vector<int32_t> it_t, it_b, it_e, it_ptr(pl->nbox + 1);
  for (int64_t t = 0; t < pl->nbox; ++t) {
    it_ptr[t] = (int32_t)it_t.size();
    const int32_t lt = mptr[t + 1] - mptr[t];
    const int32_t ni = (lt + kItemPairs - 1) / kItemPairs;
    for (int32_t j = 0; j < ni; ++j) {
      it_t.push_back((int32_t)t);
      it_b.push_back(mptr[t] + (int32_t)((int64_t)lt * j / ni));
      it_e.push_back(mptr[t] + (int32_t)((int64_t)lt * (j + 1) / ni));
    }
  }
  it_ptr[pl->nbox] = (int32_t)it_t.size();
  S.n_items = (int64_t)it_t.size();
  const size_t ni = std::max<size_t>(it_t.size(), 1);
  S.item_tgt = (int32_t*)plan_alloc(pl, sizeof(int32_t) * ni);
  S.item_begin = (int32_t*)plan_alloc(pl, sizeof(int32_t) * ni);
  S.item_end = (int32_t*)plan_alloc(pl, sizeof(int32_t) * ni);
  S.item_ptr = (int32_t*)plan_alloc(pl, sizeof(int32_t) * (pl->nbox + 1));
  if (!it_t.empty()) {
    FMM_HIP(hipMemcpyAsync(S.item_tgt, it_t.data(), sizeof(int32_t) * it_t.size(),
                           hipMemcpyHostToDevice, st));
    FMM_HIP(hipMemcpyAsync(S.item_begin, it_b.data(), sizeof(int32_t) * it_b.size(),
                           hipMemcpyHostToDevice, st));
    FMM_HIP(hipMemcpyAsync(S.item_end, it_e.data(), sizeof(int32_t) * it_e.size(),
                           hipMemcpyHostToDevice, st));
  }
  FMM_HIP(hipMemcpyAsync(S.item_ptr, it_ptr.data(), sizeof(int32_t) * it_ptr.size(),
                         hipMemcpyHostToDevice, st));
  FMM_HIP(hipStreamSynchronize(st));
}

}  // namespace

void build_lists(fmm_plan* pl, hipStream_t st) {
  const int L = pl->L, nch = pl->nch;
  const int T = 256;
  Scratch sc;
  // level-mean radii, summed in box order on the host
  std::vector<double> rad(pl->nbox);
  FMM_HIP(hipMemcpyAsync(rad.data(), pl->radius, sizeof(double) * pl->nbox,
                         hipMemcpyDeviceToHost, st));
  FMM_HIP(hipStreamSynchronize(st));
  // Length scale of each box's expansions: its radius, floored at 2^-30 of
  // the root radius (boxes whose points coincide have radius 0).
  {
    const double floor_r = rad[0] > 0.0 ? std::ldexp(rad[0], -30) : 1.0;
    std::vector<double> scl(pl->nbox);
    for (int64_t b = 0; b < pl->nbox; ++b) scl[b] = std::max(rad[b], floor_r);
    FMM_HIP(hipMemcpyAsync(pl->scale, scl.data(), sizeof(double) * pl->nbox,
                           hipMemcpyHostToDevice, st));
    FMM_HIP(hipStreamSynchronize(st));
  }
  std::vector<double> avg(L + 1);
  for (int l = 0; l <= L; ++l) {
    double acc = 0.0;
    for (int64_t b = pl->level_off[l]; b < pl->level_off[l + 1]; ++b) acc += rad[b];
    avg[l] = acc / (double)(pl->level_off[l + 1] - pl->level_off[l]);
  }

  int32_t* ps = (int32_t*)sc.get(sizeof(int32_t));
  int32_t* pt = (int32_t*)sc.get(sizeof(int32_t));
  FMM_HIP(hipMemsetAsync(ps, 0, sizeof(int32_t), st));
  FMM_HIP(hipMemsetAsync(pt, 0, sizeof(int32_t), st));
  int64_t np = 1;
  int ls = 0, lt = 0;
  std::vector<std::pair<uint64_t*, int64_t>> m2l_parts;
  int64_t n_m2l = 0;
  while (np > 0 && !(ls == L && lt == L)) {
    bool src_side;
    if (ls == L)
      src_side = false;
    else if (lt == L)
      src_side = true;
    else if (avg[ls] > avg[lt])
      src_side = true;
    else if (avg[ls] < avg[lt])
      src_side = false;
    else
      src_side = pl->prm.tie_refine == FMM_TIE_SOURCE;
    if (src_side) ++ls; else ++lt;
    const int64_t ne = np * nch;
    int32_t* cs = (int32_t*)sc.get(sizeof(int32_t) * ne);
    int32_t* ct = (int32_t*)sc.get(sizeof(int32_t) * ne);
    int32_t* adm = (int32_t*)sc.get(sizeof(int32_t) * ne);
    int32_t* excl = (int32_t*)sc.get(sizeof(int32_t) * ne);
    k_expand_test<<<blocks(ne, T), T, 0, st>>>(
        np, nch, src_side ? 1 : 0, ps, pt, pl->level_off[ls], pl->level_off[lt],
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
    k_compact<<<blocks(ne, T), T, 0, st>>>(ne, cs, ct, adm, excl, pl->level_off[ls],
                                           pl->level_off[lt], keys, ns, nt);
    FMM_HIP(hipGetLastError());
    if (nadm > 0) m2l_parts.emplace_back(keys, nadm);
    n_m2l += nadm;
    ps = ns;
    pt = nt;
    np = ne - nadm;
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
  // P2P CSR over leaves (what is left once both sides reached the leaves)
  if (!(ls == L && lt == L)) np = 0;
  uint64_t* pk = (uint64_t*)sc.get(sizeof(uint64_t) * std::max<int64_t>(np, 1));
  if (np > 0) {
    k_keys_from_pairs<<<blocks(np, T), T, 0, st>>>(np, ps, pt, pk);
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
}

}  // namespace fmm
