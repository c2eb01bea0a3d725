// Union of independent problems in one plan.
//
// Each problem keeps its own tree and lists (built exactly as for a single
// plan).  The union concatenates every per-point, per-box and per-leaf array
// in problem order and shifts the indices stored in them (point, box, leaf
// and list-pair ids) by the running totals, so that every evaluation stage
// runs as one launch over the work of all problems; the M2L work items are
// then packed over the union's lists.
#include <algorithm>

#include "internal.h"

namespace fmm {
namespace {

inline unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// dst[i] = src[i] + add for i < n.
__global__ void k_copy_shifted(int64_t n, const int32_t* __restrict__ src, int32_t add,
                               int32_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i] + add;
}

void copy_shifted(int32_t* dst, const int32_t* src, int64_t n, int64_t add, hipStream_t st) {
  if (n <= 0) return;
  k_copy_shifted<<<blocks(n, 256), 256, 0, st>>>(n, src, (int32_t)add, dst);
  FMM_HIP(hipGetLastError());
}

template <typename T>
void copy_plain(T* dst, const T* src, int64_t n, hipStream_t st) {
  if (n > 0) FMM_HIP(hipMemcpyAsync(dst, src, sizeof(T) * n, hipMemcpyDeviceToDevice, st));
}

}  // namespace

void build_union(fmm_plan* U, const std::vector<const fmm_plan*>& subs, hipStream_t st,
                 bool lists) {
  const fmm_plan* f = subs.front();
  U->device = f->device;
  U->prm = f->prm;
  U->s = f->s;
  U->nch = f->nch;
  U->n_problems = (int)subs.size();
  U->n = 0;
  U->nbox = 0;
  U->nleaf = 0;
  U->L = 0;
  U->p2p_inter = 0;
  U->max_leaf_count = 0;
  U->has_dup = false;
  int64_t n_m2l[2] = {0, 0}, n_p2p[2] = {0, 0};
  for (const fmm_plan* p : subs) {
    U->n += p->n;
    U->nbox += p->nbox;
    U->nleaf += p->nleaf;
    U->L = std::max(U->L, p->L);
    U->p2p_inter += p->p2p_inter;
    U->max_leaf_count = std::max(U->max_leaf_count, p->max_leaf_count);
    U->has_dup = U->has_dup || p->has_dup;
    for (int d = 0; d < 2; ++d) {
      n_m2l[d] += p->lists[d].n_m2l;
      n_p2p[d] += p->lists[d].n_p2p;
    }
  }
  if (U->n >= ((int64_t)1 << 31) || U->nbox >= ((int64_t)1 << 31))
    throw Error{FMM_EINVAL, "union too large for 32-bit indices"};
  // Level offsets have no meaning across trees; the union keeps none.
  U->level_off.clear();

  auto i32 = [&](int64_t n) { return (int32_t*)plan_alloc(U, sizeof(int32_t) * n); };
  auto f64 = [&](int64_t n) { return (double*)plan_alloc(U, sizeof(double) * n); };
  U->perm = i32(U->n);
  U->leaf_start = i32(U->nleaf + 1);
  U->xs = f64(U->n);
  U->ys = f64(U->n);
  U->zs = f64(U->n);
  U->cx = f64(U->nbox);
  U->cy = f64(U->nbox);
  U->cz = f64(U->nbox);
  U->radius = f64(U->nbox);
  U->scale = f64(U->nbox);
  for (int d = 0; d < 2 && lists; ++d) {
    ListSet& S = U->lists[d];
    S.n_m2l = n_m2l[d];
    S.n_p2p = n_p2p[d];
    S.m2l_ptr = i32(U->nbox + 1);
    S.m2l_src = i32(std::max<int64_t>(S.n_m2l, 1));
    S.p2p_ptr = i32(U->nleaf + 1);
    S.p2p_src = i32(std::max<int64_t>(S.n_p2p, 1));
  }

  int64_t pb = 0, bb = 0, lb = 0;
  int64_t mb[2] = {0, 0}, qb[2] = {0, 0};
  for (const fmm_plan* p : subs) {
    copy_shifted(U->perm + pb, p->perm, p->n, lists ? pb : 0, st);
    // n+1 entries: the last one equals the next problem's first after the
    // shift and is overwritten by it in stream order.
    copy_shifted(U->leaf_start + lb, p->leaf_start, p->nleaf + 1, pb, st);
    copy_plain(U->xs + pb, p->xs, p->n, st);
    copy_plain(U->ys + pb, p->ys, p->n, st);
    copy_plain(U->zs + pb, p->zs, p->n, st);
    copy_plain(U->cx + bb, p->cx, p->nbox, st);
    copy_plain(U->cy + bb, p->cy, p->nbox, st);
    copy_plain(U->cz + bb, p->cz, p->nbox, st);
    copy_plain(U->radius + bb, p->radius, p->nbox, st);
    copy_plain(U->scale + bb, p->scale, p->nbox, st);
    for (int d = 0; d < 2 && lists; ++d) {
      const ListSet& A = p->lists[d];
      ListSet& S = U->lists[d];
      copy_shifted(S.m2l_ptr + bb, A.m2l_ptr, p->nbox + 1, mb[d], st);
      copy_shifted(S.m2l_src + mb[d], A.m2l_src, A.n_m2l, bb, st);
      copy_shifted(S.p2p_ptr + lb, A.p2p_ptr, p->nleaf + 1, qb[d], st);
      copy_shifted(S.p2p_src + qb[d], A.p2p_src, A.n_p2p, lb, st);
      mb[d] += A.n_m2l;
      qb[d] += A.n_p2p;
    }
    pb += p->n;
    bb += p->nbox;
    lb += p->nleaf;
  }
  FMM_HIP(hipStreamSynchronize(st));
  if (!lists) return;
  // M2L and near-field work items over the union's lists: blocks may then
  // mix targets of different problems
  U->side[0].npt = U->n;
  U->side[0].nleaf = U->nleaf;
  make_items(U, U->lists[0], st);
  make_items(U, U->lists[1], st);
  make_p2p_items(U, 0, st);
  make_p2p_items(U, 1, st);
}

}  // namespace fmm
