// C ABI of the FMM library: argument checks, plan lifetime, error strings.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>

#include "internal.h"
#include "tables.h"

namespace fmm {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }
void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }

void* dev_alloc(fmm_plan* pl, size_t bytes) {
  bytes = bytes ? bytes : 16;
  void* p = nullptr;
  if (pl->allocator.alloc) {
    p = pl->allocator.alloc(pl->allocator.ctx, bytes, (void*)pl->alloc_stream);
    if (!p)
      throw Error{FMM_ENOMEM,
                  "allocator callback returned NULL for " + std::to_string(bytes) + " bytes"};
    if ((uintptr_t)p % 256 != 0) {
      pl->allocator.free(pl->allocator.ctx, p, (void*)pl->alloc_stream);
      throw Error{FMM_EINVAL, "allocator callback returned memory not aligned to 256 bytes"};
    }
    return p;
  }
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error{FMM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
  return p;
}

void dev_free(fmm_plan* pl, void* p) {
  if (!p) return;
  if (pl->allocator.free)
    pl->allocator.free(pl->allocator.ctx, p, (void*)pl->alloc_stream);
  else
    (void)hipFree(p);
}

void* plan_alloc(fmm_plan* pl, size_t bytes) {
  void* p = dev_alloc(pl, bytes);
  bytes = bytes ? bytes : 16;
  pl->bufs.push_back(DevBuf{p, bytes});
  pl->device_bytes += bytes;
  return p;
}

WorkspaceLayout workspace_layout(int64_t n, int64_t nbox, const fmm_params& prm, bool batched) {
  const size_t es = prm.precision == FMM_FP32 ? sizeof(float) : sizeof(double);
  const size_t K = (size_t)ncoef(prm.p);
  const size_t W = (size_t)batch_width() * sizeof(float);
  WorkspaceLayout L;
  const size_t sz[10] = {32 * (size_t)n,
                         es * K * (size_t)nbox,
                         es * K * (size_t)nbox,
                         es * 4 * (size_t)n,
                         es * 3 * (size_t)n,
                         batched ? W * n : 0,
                         batched ? W * K * nbox : 0,
                         batched ? W * K * nbox : 0,
                         batched ? W * n : 0,
                         batched ? W * 3 * n : 0};
  size_t o = 0;
  for (int i = 0; i < 10; ++i) {
    L.off[i] = o;
    L.size[i] = sz[i];
    o += (sz[i] + 255) / 256 * 256;
    if (i == 3) L.forward = o;
  }
  L.total = o;
  return L;
}

void bind_workspace(Workspace& ws, char* base, const WorkspaceLayout& L, int count) {
  void** slot[10] = {&ws.src, &ws.C, &ws.D, &ws.near, &ws.field_t,
                     &ws.bq,  &ws.bC, &ws.bD, &ws.bpot, &ws.bfld};
  for (int i = 0; i < 10; ++i) *slot[i] = (i < count && L.size[i] > 0) ? base + L.off[i] : nullptr;
}

hipEvent_t take_event(fmm_plan* pl) {
  if (!pl->ev_pool.empty()) {
    hipEvent_t e = pl->ev_pool.back();
    pl->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  FMM_HIP(hipEventCreate(&e));
  return e;
}

void release_profile(fmm_plan* pl) {
  for (auto& row : pl->ev_rows)
    for (hipEvent_t e : row) pl->ev_pool.push_back(e);
  pl->ev_rows.clear();
}

void plan_free_all(fmm_plan* pl) {
  for (auto& b : pl->bufs) dev_free(pl, b.ptr);
  pl->bufs.clear();
  pl->device_bytes = 0;
  if (pl->ev_fork) (void)hipEventDestroy(pl->ev_fork);
  if (pl->ev_join) (void)hipEventDestroy(pl->ev_join);
  if (pl->side_stream) (void)hipStreamDestroy(pl->side_stream);
  pl->ev_fork = pl->ev_join = nullptr;
  pl->side_stream = nullptr;
}

// The evaluation's second stream and its fork / join events (on the
// plan's device, which is current during creation).
void make_fork(fmm_plan* pl) {
  FMM_HIP(hipStreamCreateWithFlags(&pl->side_stream, hipStreamNonBlocking));
  FMM_HIP(hipEventCreateWithFlags(&pl->ev_fork, hipEventDisableTiming));
  FMM_HIP(hipEventCreateWithFlags(&pl->ev_join, hipEventDisableTiming));
}

void make_steps(fmm_plan* pl, const std::vector<std::vector<TreeDesc>>& groups,
                hipStream_t st) {
  const int s = pl->s;
  auto upload = [&](const std::vector<int32_t>& v) {
    int32_t* d = (int32_t*)plan_alloc(pl, sizeof(int32_t) * v.size());
    if (!v.empty())
      FMM_HIP(hipMemcpyAsync(d, v.data(), sizeof(int32_t) * v.size(), hipMemcpyHostToDevice, st));
    FMM_HIP(hipStreamSynchronize(st));
    return d;
  };
  std::vector<int32_t> lb;
  for (const auto& trees : groups)
    for (const TreeDesc& t : trees) {
      const int64_t nl = t.level_off[t.L + 1] - t.level_off[t.L];
      for (int64_t i = 0; i < nl; ++i) lb.push_back((int32_t)(t.box_base + t.level_off[t.L] + i));
    }
  pl->leaf_box = upload(lb);
  // Boxes whose expansions matter: those in an M2L pair (either role, so
  // both the forward and the transposed pass are covered) and all their
  // descendants.  Multipoles of other boxes are never read; locals of other
  // non-leaf boxes are zero and are not formed (children skip the
  // translation from them).
  std::vector<char> active(pl->nbox, 0);
  {
    const ListSet& F = pl->lists[0];
    std::vector<int32_t> ptr(pl->nbox + 1), src(std::max<int64_t>(F.n_m2l, 1));
    FMM_HIP(hipMemcpyAsync(ptr.data(), F.m2l_ptr, sizeof(int32_t) * (pl->nbox + 1),
                           hipMemcpyDeviceToHost, st));
    if (F.n_m2l > 0)
      FMM_HIP(hipMemcpyAsync(src.data(), F.m2l_src, sizeof(int32_t) * F.n_m2l,
                             hipMemcpyDeviceToHost, st));
    FMM_HIP(hipStreamSynchronize(st));
    for (int64_t b = 0; b < pl->nbox; ++b)
      if (ptr[b + 1] > ptr[b]) active[b] = 1;
    for (int64_t k = 0; k < F.n_m2l; ++k) active[src[k]] = 1;
    for (const auto& trees : groups)
      for (const TreeDesc& t : trees)
        for (int l = 1; l <= t.L; ++l)
          for (int64_t i = 0; i < t.level_off[l + 1] - t.level_off[l]; ++i) {
            const int64_t b = t.box_base + t.level_off[l] + i;
            if (active[t.box_base + t.level_off[l - 1] + (i >> s)]) active[b] = 1;
          }
  }
  std::vector<std::vector<int32_t>> all_of(groups.size());
  for (size_t g = 0; g < groups.size(); ++g) {
    const std::vector<TreeDesc>& trees = groups[g];
    Side& S = pl->side[g];
    S.m2m_steps.clear();
    S.l2l_steps.clear();
    int Lmax = 0;
    for (const TreeDesc& t : trees) Lmax = std::max(Lmax, t.L);
    // Upward: step h takes the parents h+1 levels above each tree's leaves.
    for (int h = 0; h < Lmax; ++h) {
      std::vector<int32_t> a, b;
      for (const TreeDesc& t : trees) {
        const int l = t.L - 1 - h;
        if (l < 0) continue;
        const int64_t np = t.level_off[l + 1] - t.level_off[l];
        for (int64_t i = 0; i < np; ++i) {
          const int64_t p = t.box_base + t.level_off[l] + i;
          if (!active[p]) continue;
          a.push_back((int32_t)p);
          b.push_back((int32_t)(t.box_base + t.level_off[l + 1] + (i << s)));
        }
      }
      if (a.empty()) continue;
      Step St;
      St.n = (int64_t)a.size();
      St.a = upload(a);
      St.b = upload(b);
      S.m2m_steps.push_back(St);
    }
    // Downward: every box whose local is formed starts from the sum of its
    // M2L translations (written by the M2L kernel, or zero); step l then
    // adds the translated parent local to the boxes of level l of every tree
    // that deep whose parent has one.
    std::vector<int32_t>& all = all_of[g];
    for (int l = 0; l <= Lmax; ++l) {
      std::vector<int32_t> a, b;
      for (const TreeDesc& t : trees) {
        if (l > t.L) continue;
        const int64_t nb = t.level_off[l + 1] - t.level_off[l];
        for (int64_t i = 0; i < nb; ++i) {
          const int64_t bx = t.box_base + t.level_off[l] + i;
          if (!active[bx] && l < t.L) continue;  // leaves are always written
          all.push_back((int32_t)bx);
          const int64_t pa = l > 0 ? t.box_base + t.level_off[l - 1] + (i >> s) : -1;
          if (pa < 0 || !active[pa]) continue;
          a.push_back((int32_t)bx);
          b.push_back((int32_t)pa);
        }
      }
      if (a.empty()) continue;
      Step St;
      St.n = (int64_t)a.size();
      St.a = upload(a);
      St.b = upload(b);
      S.l2l_steps.push_back(St);
    }
    S.l2l_sum.n = (int64_t)all.size();
    S.l2l_sum.a = upload(all);
    S.l2l_sum.b = nullptr;
  }
  // Final locals of each direction's target side.  Re-centring a truncated
  // local expansion is exact, so a box's final local is its own M2L sum plus
  // the translated M2L sums of all its ancestors; the parents of the leaves
  // get theirs that way in one launch (every translation independent), the
  // leaves then add one translation of their parent's final local.
  for (int d = 0; d < 2; ++d) {
    ListSet& L = pl->lists[d];
    const std::vector<TreeDesc>& trees = groups[pl->nsides == 1 ? 0 : 1 - d];
    std::vector<int32_t> ptr(pl->nbox + 1);
    FMM_HIP(hipMemcpyAsync(ptr.data(), L.m2l_ptr, sizeof(int32_t) * (pl->nbox + 1),
                           hipMemcpyDeviceToHost, st));
    FMM_HIP(hipStreamSynchronize(st));
    auto has = [&](int64_t b) { return ptr[b + 1] > ptr[b]; };
    std::vector<int32_t> box[2], own[2];
    std::vector<std::vector<int32_t>> src[2];
    for (const TreeDesc& t : trees) {
      std::vector<char> formed;  // parents of the leaves with a final local
      if (t.L >= 1) {
        const int lp = t.L - 1;
        const int64_t np = t.level_off[lp + 1] - t.level_off[lp];
        formed.assign(np, 0);
        for (int64_t i = 0; i < np; ++i) {
          const int64_t b = t.box_base + t.level_off[lp] + i;
          std::vector<int32_t> anc;
          for (int l = lp - 1; l >= 0; --l) {
            const int64_t a = t.box_base + t.level_off[l] + (i >> (s * (lp - l)));
            if (has(a)) anc.push_back((int32_t)a);
          }
          if (!has(b) && anc.empty()) continue;
          formed[i] = 1;
          box[0].push_back((int32_t)b);
          own[0].push_back(has(b) ? 1 : 0);
          src[0].push_back(anc);
        }
      }
      const int64_t nl = t.level_off[t.L + 1] - t.level_off[t.L];
      for (int64_t i = 0; i < nl; ++i) {
        const int64_t b = t.box_base + t.level_off[t.L] + i;
        box[1].push_back((int32_t)b);
        own[1].push_back(has(b) ? 1 : 0);
        src[1].emplace_back();
        if (t.L >= 1 && formed[i >> s])
          src[1].back().push_back((int32_t)(t.box_base + t.level_off[t.L - 1] + (i >> s)));
      }
    }
    for (int k = 0; k < 2; ++k) {
      size_t need = 1;
      for (const auto& v : src[k]) need = std::max(need, v.size());
      int gs = 1;
      while ((size_t)gs < need) gs <<= 1;
      if (gs > 16) throw Error{FMM_ENOTSUP, "more than 16 ancestors with M2L pairs"};
      std::vector<int32_t> flat((size_t)gs * box[k].size(), -1);
      for (size_t g = 0; g < box[k].size(); ++g)
        for (size_t j = 0; j < src[k][g].size(); ++j) flat[g * gs + j] = src[k][g][j];
      FinList& F = L.fin[k];
      F.gs = gs;
      F.n = (int64_t)box[k].size();
      F.box = upload(box[k]);
      F.own = upload(own[k]);
      F.anc = upload(flat);
    }
  }
}

namespace {

int depth_for(int64_t n, int leaf, int s, int max_depth) {
  int L = 0;
  while (L < max_depth) {
    const int64_t per = (n + ((int64_t)1 << (L * s)) - 1) >> (L * s);  // ceil
    if (per <= leaf) break;
    ++L;
  }
  return L;
}

void check_params(const fmm_params* prm, int64_t n) {
  if (!prm) throw Error{FMM_EINVAL, "params is NULL"};
  if (n < 1 || n >= ((int64_t)1 << 31)) throw Error{FMM_EINVAL, "n must be in [1, 2^31)"};
  if (prm->splits < 1 || prm->splits > 3) throw Error{FMM_EINVAL, "splits must be 1..3"};
  if (prm->p < 0) throw Error{FMM_EINVAL, "p must be >= 0"};
  if (prm->leaf_max < (1 << prm->splits))
    throw Error{FMM_EINVAL, "leaf_max must be >= 2^splits"};
  if (!(prm->theta > 0.0 && prm->theta < 1.0)) throw Error{FMM_EINVAL, "theta must be in (0,1)"};
  if (prm->max_depth < 0 || prm->max_depth > 16) throw Error{FMM_EINVAL, "max_depth must be 0..16"};
  if (prm->precision != FMM_FP64 && prm->precision != FMM_FP32)
    throw Error{FMM_EINVAL, "precision must be FMM_FP64 or FMM_FP32"};
  if (prm->tie_refine != FMM_TIE_SOURCE && prm->tie_refine != FMM_TIE_TARGET)
    throw Error{FMM_EINVAL, "tie_refine must be FMM_TIE_SOURCE or FMM_TIE_TARGET"};
  if (prm->max_rhs < 1) throw Error{FMM_EINVAL, "max_rhs must be >= 1"};
  if (prm->lists != FMM_LISTS_CROSS_LEVEL && prm->lists != FMM_LISTS_SAME_LEVEL)
    throw Error{FMM_EINVAL, "lists must be FMM_LISTS_CROSS_LEVEL or FMM_LISTS_SAME_LEVEL"};
  if (prm->p < FMM_MIN_ORDER || prm->p > FMM_MAX_ORDER)
    throw Error{FMM_ENOTSUP, "p outside FMM_MIN_ORDER..FMM_MAX_ORDER (no compiled kernels)"};
}

void check_allocator(const fmm_allocator* a, unsigned flags) {
  if (a && (!a->alloc || !a->free))
    throw Error{FMM_EINVAL, "allocator needs both an alloc and a free callback"};
  if ((flags & ~FMM_PLAN_NO_WORKSPACE) != 0u) throw Error{FMM_EINVAL, "unknown plan flags"};
}

void use_allocator(fmm_plan* pl, const fmm_allocator* a, hipStream_t st, unsigned flags = 0u) {
  if (a) pl->allocator = *a;
  pl->alloc_stream = st;
  pl->flags = flags;
}

void check_workspace(const fmm_plan* pl) {
  if (!pl->ws.C) throw Error{FMM_ESTATE, "the plan holds no evaluation workspace"};
}

void check_device(const fmm_plan* pl) {
  int dev = -1;
  FMM_HIP(hipGetDevice(&dev));
  if (dev != pl->device)
    throw Error{FMM_EDEVICE, "current device differs from the plan's device"};
}

// Several charge vectors: FP32 plans built for more than one vector take
// them kRB at a time through the multi-vector kernels; otherwise one pass
// per vector.
void run_vectors(fmm_plan* pl, int dir, const void* q, int nrhs, void* pot, void* field,
                 hipStream_t st) {
  if (nrhs > 1 && pl->ws.bq) {
    const int W = batch_width();
    const int64_t n = pl->n;
    for (int r0 = 0; r0 < nrhs; r0 += W) {
      const int R = std::min(W, nrhs - r0);
      evaluate_batch(pl, dir, (const float*)q + (int64_t)r0 * n, R, (float*)pot + (int64_t)r0 * n,
                     field ? (float*)field + 3 * (int64_t)r0 * n : nullptr, st);
    }
  } else {
    evaluate(pl, pl->ws, dir, q, nrhs, pot, field, st);
  }
}

// Tree and geometry (and, with lists, the interaction lists) of one point
// set: plan creation minus the level steps and the evaluation workspace.
void build_structure(fmm_plan* pl, const double* pos, int64_t n, const fmm_params* prm,
                     hipStream_t st, bool lists = true) {
  FMM_HIP(hipGetDevice(&pl->device));
  pl->prm = *prm;
  pl->n = n;
  pl->s = prm->splits;
  pl->nch = 1 << pl->s;
  pl->L = depth_for(n, prm->leaf_max, pl->s, prm->max_depth);
  pl->level_off.assign(pl->L + 2, 0);
  for (int l = 0; l <= pl->L; ++l)
    pl->level_off[l + 1] = pl->level_off[l] + ((int64_t)1 << (pl->s * l));
  pl->nbox = pl->level_off[pl->L + 1];
  pl->nleaf = (int64_t)1 << (pl->s * pl->L);
  if (pl->nbox >= ((int64_t)1 << 31)) throw Error{FMM_EINVAL, "too many boxes"};
  pl->perm = (int32_t*)plan_alloc(pl, sizeof(int32_t) * n);
  pl->leaf_start = (int32_t*)plan_alloc(pl, sizeof(int32_t) * (pl->nleaf + 1));
  pl->xs = (double*)plan_alloc(pl, sizeof(double) * n);
  pl->ys = (double*)plan_alloc(pl, sizeof(double) * n);
  pl->zs = (double*)plan_alloc(pl, sizeof(double) * n);
  pl->cx = (double*)plan_alloc(pl, sizeof(double) * pl->nbox);
  pl->cy = (double*)plan_alloc(pl, sizeof(double) * pl->nbox);
  pl->cz = (double*)plan_alloc(pl, sizeof(double) * pl->nbox);
  pl->radius = (double*)plan_alloc(pl, sizeof(double) * pl->nbox);
  pl->scale = (double*)plan_alloc(pl, sizeof(double) * pl->nbox);
  build_tree(pl, pos, st);
  pl->side[0].npt = n;
  pl->side[0].nleaf = pl->nleaf;
  if (lists) {
    const TreeDesc t{pl->L, pl->level_off, 0, 0};
    build_lists(pl, t, t, st);
  }
}

bool batched_plan(const fmm_plan* pl) {
  return pl->prm.precision == FMM_FP32 && pl->prm.max_rhs > 1 && pl->nsides == 1;
}

// Evaluation workspace (one allocation, workspace_layout) and the batched
// M2L partial rows, sized from the plan's counts.
void alloc_workspace(fmm_plan* pl, hipStream_t st) {
  const fmm_params* prm = &pl->prm;
  const bool bat = batched_plan(pl);
  const WorkspaceLayout L = workspace_layout(pl->n, pl->nbox, *prm, bat);
  if (!(pl->flags & FMM_PLAN_NO_WORKSPACE)) {
    pl->workspace_bytes = L.total;
    bind_workspace(pl->ws, (char*)plan_alloc(pl, L.total), L, 10);
  }
  if (bat) {
    const size_t K = (size_t)ncoef(prm->p);
    const size_t ni =
        (size_t)std::max<int64_t>(std::max(pl->lists[0].n_items, pl->lists[1].n_items), 1);
    pl->bpart = plan_alloc(pl, (size_t)batch_width() * sizeof(float) * K * ni);
    pl->iperm = (int32_t*)plan_alloc(pl, sizeof(int32_t) * (size_t)pl->n);
    make_iperm(pl, st);
  }
  pl->tables = get_tables(prm->p, prm->precision, pl->device);
  FMM_HIP(hipStreamSynchronize(st));
}

}  // namespace
}  // namespace fmm

using namespace fmm;

extern "C" {

int fmm_abi_version(void) { return FMM_ABI_VERSION; }

const char* fmm_last_error(void) { return fmm::last_error(); }

fmm_status fmm_plan_create_ex(const double* pos, int64_t n, const fmm_params* prm,
                              const fmm_allocator* allocator, unsigned flags, void* stream,
                              fmm_plan** out) {
  return guard([&] {
    if (!out) throw Error{FMM_EINVAL, "out is NULL"};
    if (!pos) throw Error{FMM_EINVAL, "pos is NULL"};
    check_params(prm, n);
    check_allocator(allocator, flags);
    hipStream_t st = (hipStream_t)stream;
    std::unique_ptr<fmm_plan> pl(new fmm_plan());
    use_allocator(pl.get(), allocator, st, flags);
    try {
      build_structure(pl.get(), pos, n, prm, st);
      make_steps(pl.get(), {{TreeDesc{pl->L, pl->level_off, 0, 0}}}, st);
      alloc_workspace(pl.get(), st);
      make_fork(pl.get());
    } catch (...) {
      (void)hipStreamSynchronize(st);
      plan_free_all(pl.get());
      throw;
    }
    *out = pl.release();
  });
}

fmm_status fmm_plan_create(const double* pos, int64_t n, const fmm_params* prm,
                           void* stream, fmm_plan** out) {
  return fmm_plan_create_ex(pos, n, prm, nullptr, 0u, stream, out);
}

fmm_status fmm_multi_plan_create_ex(const double* pos, const int64_t* offsets, int nprob,
                                    const fmm_params* prm, const fmm_allocator* allocator,
                                    unsigned flags, void* stream, fmm_plan** out) {
  return guard([&] {
    if (!out) throw Error{FMM_EINVAL, "out is NULL"};
    if (!pos || !offsets) throw Error{FMM_EINVAL, "pos and offsets must not be NULL"};
    if (nprob < 1) throw Error{FMM_EINVAL, "nprob must be >= 1"};
    if (offsets[0] != 0) throw Error{FMM_EINVAL, "offsets[0] must be 0"};
    for (int k = 0; k < nprob; ++k)
      if (offsets[k + 1] <= offsets[k])
        throw Error{FMM_EINVAL, "every problem needs at least one point"};
    check_params(prm, offsets[nprob]);
    check_allocator(allocator, flags);
    hipStream_t st = (hipStream_t)stream;
    std::vector<std::unique_ptr<fmm_plan>> subs;
    std::unique_ptr<fmm_plan> pl(new fmm_plan());
    use_allocator(pl.get(), allocator, st, flags);
    auto free_subs = [&] {
      for (auto& u : subs) plan_free_all(u.get());
      subs.clear();
    };
    try {
      for (int k = 0; k < nprob; ++k) {
        subs.emplace_back(new fmm_plan());
        use_allocator(subs.back().get(), allocator, st);
        build_structure(subs.back().get(), pos + 3 * offsets[k], offsets[k + 1] - offsets[k], prm,
                        st);
      }
      std::vector<const fmm_plan*> sp;
      for (auto& u : subs) sp.push_back(u.get());
      build_union(pl.get(), sp, st);
      std::vector<TreeDesc> trees;
      int64_t base = 0, lbase = 0;
      for (const fmm_plan* u : sp) {
        trees.push_back(TreeDesc{u->L, u->level_off, base, lbase});
        base += u->nbox;
        lbase += u->nleaf;
      }
      pl->side[0].npt = pl->n;
      pl->side[0].nleaf = pl->nleaf;
      make_steps(pl.get(), {trees}, st);
      (void)hipStreamSynchronize(st);
      free_subs();
      alloc_workspace(pl.get(), st);
      make_fork(pl.get());
    } catch (...) {
      (void)hipStreamSynchronize(st);
      free_subs();
      plan_free_all(pl.get());
      throw;
    }
    *out = pl.release();
  });
}

fmm_status fmm_multi_plan_create(const double* pos, const int64_t* offsets, int nprob,
                                 const fmm_params* prm, void* stream, fmm_plan** out) {
  return fmm_multi_plan_create_ex(pos, offsets, nprob, prm, nullptr, 0u, stream, out);
}

fmm_status fmm_plan_create_st(const double* src, int64_t ns, const double* tgt, int64_t nt,
                              const fmm_params* prm, const fmm_allocator* allocator,
                              unsigned flags, void* stream, fmm_plan** out) {
  return guard([&] {
    if (!out) throw Error{FMM_EINVAL, "out is NULL"};
    if (!src || !tgt) throw Error{FMM_EINVAL, "src and tgt must not be NULL"};
    check_params(prm, ns);
    check_params(prm, nt);
    if (ns + nt >= ((int64_t)1 << 31)) throw Error{FMM_EINVAL, "ns + nt must be below 2^31"};
    check_allocator(allocator, flags);
    hipStream_t st = (hipStream_t)stream;
    std::unique_ptr<fmm_plan> sub[2];
    std::unique_ptr<fmm_plan> pl(new fmm_plan());
    use_allocator(pl.get(), allocator, st, flags);
    auto free_subs = [&] {
      for (auto& u : sub)
        if (u) plan_free_all(u.get());
    };
    try {
      const double* pos[2] = {src, tgt};
      const int64_t cnt[2] = {ns, nt};
      for (int k = 0; k < 2; ++k) {
        sub[k].reset(new fmm_plan());
        use_allocator(sub[k].get(), allocator, st);
        build_structure(sub[k].get(), pos[k], cnt[k], prm, st, false);
      }
      build_union(pl.get(), {sub[0].get(), sub[1].get()}, st, false);
      pl->nsides = 2;
      pl->has_dup = true;  // a target may coincide with a source anywhere
      const TreeDesc ts{sub[0]->L, sub[0]->level_off, 0, 0};
      const TreeDesc tt{sub[1]->L, sub[1]->level_off, sub[0]->nbox, sub[0]->nleaf};
      for (int k = 0; k < 2; ++k) {
        pl->side[k].pt0 = k == 0 ? 0 : ns;
        pl->side[k].npt = cnt[k];
        pl->side[k].leaf0 = k == 0 ? 0 : sub[0]->nleaf;
        pl->side[k].nleaf = sub[k]->nleaf;
      }
      build_lists(pl.get(), ts, tt, st);
      make_steps(pl.get(), {{ts}, {tt}}, st);
      (void)hipStreamSynchronize(st);
      free_subs();
      alloc_workspace(pl.get(), st);
      make_fork(pl.get());
    } catch (...) {
      (void)hipStreamSynchronize(st);
      free_subs();
      plan_free_all(pl.get());
      throw;
    }
    *out = pl.release();
  });
}

fmm_status fmm_plan_workspace_bytes(int64_t n, const fmm_params* prm, int64_t* bytes) {
  return guard([&] {
    if (!bytes) throw Error{FMM_EINVAL, "bytes is NULL"};
    check_params(prm, n);
    const int L = depth_for(n, prm->leaf_max, prm->splits, prm->max_depth);
    int64_t nbox = 0;
    for (int l = 0; l <= L; ++l) nbox += (int64_t)1 << (prm->splits * l);
    const bool bat = prm->precision == FMM_FP32 && prm->max_rhs > 1;
    *bytes = (int64_t)workspace_layout(n, nbox, *prm, bat).total;
  });
}

fmm_status fmm_plan_get_info(const fmm_plan* pl, fmm_plan_info* info) {
  return guard([&] {
    if (!pl || !info) throw Error{FMM_EINVAL, "NULL argument"};
    fmm_plan_info r{};
    r.n = pl->n;
    r.depth = pl->L;
    r.splits = pl->s;
    r.nbox = pl->nbox;
    r.nleaf = pl->nleaf;
    r.n_m2l = pl->lists[0].n_m2l;
    r.n_p2p = pl->lists[0].n_p2p;
    r.p2p_interactions = pl->p2p_inter;
    r.device_bytes = (int64_t)pl->device_bytes;
    r.workspace_bytes = (int64_t)pl->workspace_bytes;
    r.p2p_items = pl->lists[0].n_pitems;
    *info = r;
  });
}

fmm_status fmm_evaluate(fmm_plan* pl, const void* q, int nrhs, void* pot,
                        void* field, void* stream) {
  return guard([&] {
    if (!pl) throw Error{FMM_EINVAL, "plan is NULL"};
    if (!q || !pot) throw Error{FMM_EINVAL, "q and pot must not be NULL"};
    if (nrhs < 1 || nrhs > pl->prm.max_rhs) throw Error{FMM_EINVAL, "nrhs out of range"};
    check_device(pl);
    check_workspace(pl);
    run_vectors(pl, 0, q, nrhs, pot, field, (hipStream_t)stream);
  });
}

fmm_status fmm_evaluate_transposed(fmm_plan* pl, const void* q, int nrhs, void* pot,
                                   void* field, void* stream) {
  return guard([&] {
    if (!pl) throw Error{FMM_EINVAL, "plan is NULL"};
    if (!q || !pot) throw Error{FMM_EINVAL, "q and pot must not be NULL"};
    if (nrhs < 1 || nrhs > pl->prm.max_rhs) throw Error{FMM_EINVAL, "nrhs out of range"};
    check_device(pl);
    check_workspace(pl);
    run_vectors(pl, 1, q, nrhs, pot, field, (hipStream_t)stream);
  });
}

fmm_status fmm_adjoint(fmm_plan* pl, const void* q, const void* g, int nrhs,
                       const void* field_fwd, void* grad_q, void* grad_x, void* stream) {
  return guard([&] {
    if (!pl) throw Error{FMM_EINVAL, "plan is NULL"};
    if (!g || !grad_q) throw Error{FMM_EINVAL, "g and grad_q must not be NULL"};
    if (grad_x && (!q || !field_fwd))
      throw Error{FMM_EINVAL, "grad_x needs q and field_fwd"};
    if (nrhs < 1 || nrhs > pl->prm.max_rhs) throw Error{FMM_EINVAL, "nrhs out of range"};
    if (grad_x && pl->nsides == 2)
      throw Error{FMM_ENOTSUP, "position gradients of a plan with separate targets"};
    check_device(pl);
    check_workspace(pl);
    const size_t es = pl->prm.precision == FMM_FP32 ? sizeof(float) : sizeof(double);
    const hipStream_t st = (hipStream_t)stream;
    // g lives on the target side, grad_q on the source side
    const size_t ng = (size_t)tgt_side(pl, 0).npt, nq = (size_t)src_side(pl, 0).npt;
    for (int r = 0; r < nrhs; ++r) {
      const size_t o1 = es * nq * r, o3 = 3 * o1, og = es * ng * r;
      fmm::evaluate(pl, pl->ws, 1, (const char*)g + og, 1, (char*)grad_q + o1,
                    grad_x ? pl->ws.field_t : nullptr, st);
      if (grad_x)
        fmm::adjoint_combine(pl, (const char*)q + o1, (const char*)g + o1,
                             (const char*)field_fwd + o3, pl->ws.field_t, (char*)grad_x + o3, st);
    }
  });
}

fmm_status fmm_plan_get_tree(const fmm_plan* pl, int64_t* perm, int64_t* leaf_start,
                             double* centre, double* radius) {
  return guard([&] {
    if (!pl) throw Error{FMM_EINVAL, "plan is NULL"};
    check_device(pl);
    std::vector<int32_t> p32;
    if (perm) {
      p32.resize(pl->n);
      FMM_HIP(hipMemcpy(p32.data(), pl->perm, sizeof(int32_t) * pl->n, hipMemcpyDeviceToHost));
    }
    std::vector<int32_t> l32;
    if (leaf_start) {
      l32.resize(pl->nleaf + 1);
      FMM_HIP(hipMemcpy(l32.data(), pl->leaf_start, sizeof(int32_t) * (pl->nleaf + 1),
                        hipMemcpyDeviceToHost));
    }
    std::vector<double> c[3], r;
    if (centre) {
      const double* src[3] = {pl->cx, pl->cy, pl->cz};
      for (int a = 0; a < 3; ++a) {
        c[a].resize(pl->nbox);
        FMM_HIP(hipMemcpy(c[a].data(), src[a], sizeof(double) * pl->nbox, hipMemcpyDeviceToHost));
      }
    }
    if (radius) {
      r.resize(pl->nbox);
      FMM_HIP(hipMemcpy(r.data(), pl->radius, sizeof(double) * pl->nbox, hipMemcpyDeviceToHost));
    }
    for (size_t i = 0; i < p32.size(); ++i) perm[i] = p32[i];
    for (size_t i = 0; i < l32.size(); ++i) leaf_start[i] = l32[i];
    if (centre)
      for (int64_t b = 0; b < pl->nbox; ++b)
        for (int a = 0; a < 3; ++a) centre[3 * b + a] = c[a][b];
    if (radius) std::memcpy(radius, r.data(), sizeof(double) * pl->nbox);
  });
}

fmm_status fmm_plan_get_lists(const fmm_plan* pl, int64_t* m2l_src, int64_t* m2l_tgt,
                              int64_t* p2p_src, int64_t* p2p_tgt) {
  return guard([&] {
    if (!pl) throw Error{FMM_EINVAL, "plan is NULL"};
    check_device(pl);
    auto fetch = [&](const int32_t* ptr_d, const int32_t* src_d, int64_t ntgt, int64_t nk,
                     int64_t* src, int64_t* tgt) {
      if (!src && !tgt) return;
      std::vector<int32_t> ptr(ntgt + 1), s(std::max<int64_t>(nk, 1));
      FMM_HIP(hipMemcpy(ptr.data(), ptr_d, sizeof(int32_t) * (ntgt + 1), hipMemcpyDeviceToHost));
      if (nk > 0)
        FMM_HIP(hipMemcpy(s.data(), src_d, sizeof(int32_t) * nk, hipMemcpyDeviceToHost));
      for (int64_t t = 0; t < ntgt; ++t)
        for (int32_t k = ptr[t]; k < ptr[t + 1]; ++k) {
          if (src) src[k] = s[k];
          if (tgt) tgt[k] = t;
        }
    };
    const ListSet& F = pl->lists[0];
    fetch(F.m2l_ptr, F.m2l_src, pl->nbox, F.n_m2l, m2l_src, m2l_tgt);
    fetch(F.p2p_ptr, F.p2p_src, pl->nleaf, F.n_p2p, p2p_src, p2p_tgt);
  });
}

fmm_status fmm_direct(const double* pos, int64_t n, const void* q, int precision,
                      const int64_t* targets, int64_t ntargets, void* pot, void* field,
                      void* stream) {
  return guard([&] {
    if (!pos || !q || !pot) throw Error{FMM_EINVAL, "pos, q and pot must not be NULL"};
    if (n < 1 || ntargets < 0) throw Error{FMM_EINVAL, "bad sizes"};
    if (!targets && ntargets != n) throw Error{FMM_EINVAL, "ntargets must equal n without targets"};
    if (precision != FMM_FP64 && precision != FMM_FP32) throw Error{FMM_EINVAL, "bad precision"};
    direct_sum(n, pos, q, precision, targets, ntargets, pot, field, (hipStream_t)stream);
  });
}

fmm_status fmm_plan_set_profiling(fmm_plan* pl, int enable) {
  return guard([&] {
    if (!pl) throw Error{FMM_EINVAL, "plan is NULL"};
    check_device(pl);
    pl->profiling = enable != 0;
    if (!enable) {
      for (auto& row : pl->ev_rows)
        for (hipEvent_t e : row) FMM_HIP(hipEventSynchronize(e));
      release_profile(pl);
    }
  });
}

fmm_status fmm_plan_read_profile(fmm_plan* pl, double* stage_ms, int64_t* passes) {
  return guard([&] {
    if (!pl || !stage_ms) throw Error{FMM_EINVAL, "NULL argument"};
    check_device(pl);
    double acc[FMM_NSTAGES] = {0};
    for (auto& row : pl->ev_rows) {
      for (int k = 0; k < FMM_NSTAGES; ++k) {
        FMM_HIP(hipEventSynchronize(row[2 * k + 1]));
        float ms = 0.f;
        FMM_HIP(hipEventElapsedTime(&ms, row[2 * k], row[2 * k + 1]));
        acc[k] += ms;
      }
    }
    for (int k = 0; k < FMM_NSTAGES; ++k) stage_ms[k] = acc[k];
    if (passes) *passes = (int64_t)pl->ev_rows.size();
    release_profile(pl);
  });
}

fmm_status fmm_graph_create(fmm_plan* pl, int transposed, const void* q, int nrhs, void* pot,
                            void* field, fmm_graph** out) {
  return guard([&] {
    if (!pl || !out) throw Error{FMM_EINVAL, "plan and out must not be NULL"};
    if (!q || !pot) throw Error{FMM_EINVAL, "q and pot must not be NULL"};
    if (nrhs < 1 || nrhs > pl->prm.max_rhs) throw Error{FMM_EINVAL, "nrhs out of range"};
    check_device(pl);
    check_workspace(pl);
    std::unique_ptr<fmm_graph> g(new fmm_graph());
    g->device = pl->device;
    hipStream_t cs = nullptr;
    FMM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    // the graph keeps the plan's choice of stream for the near field: on
    // the second stream it becomes a second branch of the graph, forked
    // after P2M and joined before L2P, as in eager launches
    const bool prof = pl->profiling;
    pl->profiling = false;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      try {
        run_vectors(pl, transposed ? 1 : 0, q, nrhs, pot, field, cs);
      } catch (...) {
        (void)hipStreamEndCapture(cs, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cs);
        pl->profiling = prof;
        throw;
      }
      e = hipStreamEndCapture(cs, &graph);
    }
    pl->profiling = prof;
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      throw Error{FMM_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e)};
    }
    g->graph = graph;
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      throw Error{FMM_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e)};
    }
    *out = g.release();
  });
}

fmm_status fmm_graph_launch(fmm_graph* g, void* stream) {
  return guard([&] {
    if (!g) throw Error{FMM_EINVAL, "graph is NULL"};
    int dev = -1;
    FMM_HIP(hipGetDevice(&dev));
    if (dev != g->device) throw Error{FMM_EDEVICE, "current device differs from the graph's"};
    FMM_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  });
}

fmm_status fmm_graph_destroy(fmm_graph* g) {
  return guard([&] {
    if (!g) return;
    (void)hipSetDevice(g->device);
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
  });
}

fmm_status fmm_plan_autotune(fmm_plan* pl, const void* q, void* stream, int* groups_out,
                             int* leaves_out) {
  return guard([&] {
    if (!pl || !q) throw Error{FMM_EINVAL, "plan and q must not be NULL"};
    check_device(pl);
    check_workspace(pl);
    const hipStream_t st = (hipStream_t)stream;
    const size_t es = pl->prm.precision == FMM_FP32 ? sizeof(float) : sizeof(double);
    void* pot = nullptr;
    void* fld = nullptr;
    void *qb = nullptr, *pb = nullptr, *fb = nullptr;  // 32-vector timing buffers
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool prof = pl->profiling;
    const int g0 = pl->p2p_groups, l0 = pl->leaves_per_wave, w0 = pl->m2l_waves,
              c0 = pl->chain_waves, s0 = pl->near_stream, b0 = pl->batch_p2p_waves;
    auto cleanup = [&] {
      if (pot || fld || qb || pb || fb) (void)hipStreamSynchronize(st);
      dev_free(pl, pot);
      dev_free(pl, fld);
      dev_free(pl, qb);
      dev_free(pl, pb);
      dev_free(pl, fb);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      pl->profiling = prof;
    };
    try {
      pot = dev_alloc(pl, es * (size_t)pl->n);
      fld = dev_alloc(pl, es * 3 * (size_t)pl->n);
      FMM_HIP(hipEventCreate(&e0));
      FMM_HIP(hipEventCreate(&e1));
      pl->profiling = false;
      auto time3 = [&] {
        fmm::evaluate(pl, pl->ws, 0, q, 1, pot, fld, st);
        FMM_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < 3; ++r) fmm::evaluate(pl, pl->ws, 0, q, 1, pot, fld, st);
        FMM_HIP(hipEventRecord(e1, st));
        FMM_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        FMM_HIP(hipEventElapsedTime(&ms, e0, e1));
        return ms;
      };
      if (m2l_share_waves(pl->prm.p, pl->prm.precision == FMM_FP64) > 1) {
        pl->m2l_waves = 1;
        const float one = time3();
        pl->m2l_waves = 0;
        const float shared = time3();
        pl->m2l_waves = one < shared ? 1 : 0;
      }
      if (pl->prm.p >= kChainShareMinOrder) {
        pl->chain_waves = 1;
        const float one = time3();
        pl->chain_waves = 0;
        const float shared = time3();
        pl->chain_waves = one < shared ? 1 : 0;
      }
      {
        pl->near_stream = 1;
        const float one = time3();
        pl->near_stream = 0;
        const float two = time3();
        pl->near_stream = one < two ? 1 : 0;
      }
      float best = -1.f;
      int bg = 0, bl = 0;
      for (int g : {1, 2, 4}) {
        if (!valid_p2p_groups(pl, g)) continue;
        for (int l : {1, 2, 4, 8}) {
          if (!valid_leaves_per_wave(pl, l)) continue;
          pl->p2p_groups = g;
          pl->leaves_per_wave = l;
          const float ms = time3();
          if (best < 0.f || ms < best) {
            best = ms;
            bg = g;
            bl = l;
          }
        }
      }
      pl->p2p_groups = bg;
      pl->leaves_per_wave = bl;
      if (batched_plan(pl) && pl->ws.bq) {
        // the 32-vector pass on max_rhs copies of q
        const int R = std::min(pl->prm.max_rhs, batch_width());
        const size_t row = sizeof(float) * (size_t)pl->n;
        qb = dev_alloc(pl, row * R);
        pb = dev_alloc(pl, row * R);
        fb = dev_alloc(pl, 3 * row * R);
        for (int r = 0; r < R; ++r)
          FMM_HIP(hipMemcpyAsync((char*)qb + r * row, q, row, hipMemcpyDeviceToDevice, st));
        auto timeb = [&] {
          evaluate_batch(pl, 0, (const float*)qb, R, (float*)pb, (float*)fb, st);
          FMM_HIP(hipEventRecord(e0, st));
          for (int r = 0; r < 3; ++r)
            evaluate_batch(pl, 0, (const float*)qb, R, (float*)pb, (float*)fb, st);
          FMM_HIP(hipEventRecord(e1, st));
          FMM_HIP(hipEventSynchronize(e1));
          float ms = 0.f;
          FMM_HIP(hipEventElapsedTime(&ms, e0, e1));
          return ms;
        };
        float bbest = -1.f;
        int bw = 0;
        for (int w : {1, 2, 4, 8}) {
          pl->batch_p2p_waves = w;
          const float ms = timeb();
          if (bbest < 0.f || ms < bbest) {
            bbest = ms;
            bw = w;
          }
        }
        pl->batch_p2p_waves = bw;
      }
    } catch (...) {
      pl->p2p_groups = g0;
      pl->leaves_per_wave = l0;
      pl->m2l_waves = w0;
      pl->chain_waves = c0;
      pl->near_stream = s0;
      pl->batch_p2p_waves = b0;
      cleanup();
      throw;
    }
    cleanup();
    if (groups_out) *groups_out = pl->p2p_groups;
    if (leaves_out) *leaves_out = pl->leaves_per_wave;
  });
}

fmm_status fmm_plan_set_tiles(fmm_plan* pl, const fmm_tiles* t) {
  return guard([&] {
    if (!pl || !t) throw Error{FMM_EINVAL, "plan and tiles must not be NULL"};
    if (t->p2p_groups != 0 && !valid_p2p_groups(pl, t->p2p_groups))
      throw Error{FMM_EINVAL, "p2p_groups must be 0, 1, 2 or 4 and fit the largest leaf"};
    if (t->leaves_per_wave != 0 && !valid_leaves_per_wave(pl, t->leaves_per_wave))
      throw Error{FMM_EINVAL, "leaves_per_wave must be 0, 1, 2, 4 or 8 and fit the largest leaf"};
    const int shared = m2l_share_waves(pl->prm.p, pl->prm.precision == FMM_FP64);
    if (t->m2l_waves != 0 && t->m2l_waves != 1 && t->m2l_waves != shared)
      throw Error{FMM_EINVAL, shared > 1 ? "m2l_waves must be 0, 1 or " + std::to_string(shared) +
                                               " for this order and precision"
                                         : std::string("m2l_waves must be 0 or 1 for this "
                                                       "order and precision")};
    const int chain = pl->prm.p >= kChainShareMinOrder ? 4 : 1;
    if (t->chain_waves != 0 && t->chain_waves != 1 && t->chain_waves != chain)
      throw Error{FMM_EINVAL, chain > 1 ? std::string("chain_waves must be 0, 1 or 4")
                                        : std::string("chain_waves must be 0 or 1 below p = 5")};
    pl->p2p_groups = t->p2p_groups;
    pl->leaves_per_wave = t->leaves_per_wave;
    if (t->near_stream != 0 && t->near_stream != 1 && t->near_stream != 2)
      throw Error{FMM_EINVAL, "near_stream must be 0, 1 or 2"};
    if (t->batch_p2p_waves != 0 && t->batch_p2p_waves != 1 && t->batch_p2p_waves != 2 &&
        t->batch_p2p_waves != 4 && t->batch_p2p_waves != 8)
      throw Error{FMM_EINVAL, "batch_p2p_waves must be 0, 1, 2, 4 or 8"};
    pl->m2l_waves = t->m2l_waves == 1 ? 1 : 0;
    pl->chain_waves = t->chain_waves == 1 ? 1 : 0;
    pl->near_stream = t->near_stream == 1 ? 1 : 0;
    pl->batch_p2p_waves = t->batch_p2p_waves;
  });
}

fmm_status fmm_plan_get_tiles(const fmm_plan* pl, fmm_tiles* t) {
  return guard([&] {
    if (!pl || !t) throw Error{FMM_EINVAL, "plan and tiles must not be NULL"};
    t->p2p_groups = p2p_groups(pl);
    t->leaves_per_wave = leaves_per_wave(pl);
    t->m2l_waves = m2l_waves(pl);
    t->chain_waves = chain_waves(pl);
    t->near_stream = pl->near_stream == 1 ? 1 : 2;
    t->batch_p2p_waves = batch_p2p_waves(pl);
  });
}

fmm_status fmm_plan_destroy(fmm_plan* pl) {
  return guard([&] {
    if (!pl) return;
    (void)hipSetDevice(pl->device);
    (void)hipDeviceSynchronize();
    release_profile(pl);
    for (hipEvent_t e : pl->ev_pool) (void)hipEventDestroy(e);
    plan_free_all(pl);
    delete pl;
  });
}

}  // extern "C"
