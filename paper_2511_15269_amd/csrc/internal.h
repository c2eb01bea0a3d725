// Internal declarations of the FMM library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "../../include/fmm.h"

namespace fmm {

// Status carried through host code; converted to fmm_status at the ABI.
struct Error {
  fmm_status code;
  std::string msg;
};

void set_error(const std::string& msg);
void clear_error();

#define FMM_HIP(call)                                                      \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess)                                                  \
      throw ::fmm::Error{e_ == hipErrorOutOfMemory ? FMM_ENOMEM            \
                                                   : FMM_EDEVICE,          \
                         std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// Device buffer owned by a plan.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Constant operator tables of one expansion order (values in double; the
// float path keeps a rounded copy).  Layouts are shared with the kernels in
// eval.hip through the index helpers of tables.h.
struct Tables {
  int p = -1;
  std::vector<double> host;  // all tables, concatenated
  void* dev64 = nullptr;     // device copy (double)
  void* dev32 = nullptr;     // device copy (float)
};

// Boxes whose final local one launch forms: box[g] (own[g]: add its own
// M2L sum) receives the translations of sources anc[g * gs + j] (-1: none),
// gs a power of two covering the most sources of any box.
struct FinList {
  int32_t* box = nullptr;
  int32_t* own = nullptr;
  int32_t* anc = nullptr;
  int gs = 1;
  int64_t n = 0;
};

// Lanes of one M2L block (one wave).
constexpr int kM2LBlock = 64;

// Interaction lists of one direction, CSR by target.  M2L work items: lane
// i covers pairs [item_begin[i], item_end[i]) of target item_tgt[i] (-1 for
// an idle lane); the items are packed into blocks of kM2LBlock lanes, the
// items of one target consecutive inside one block (item_first[t],
// item_cnt[t]).  Block b holds the target segments seg_ptr[b] ..
// seg_ptr[b+1]-1: segment g covers lanes [seg_lanes[g] & 255,
// seg_lanes[g] >> 8) of target seg_tgt[g].
struct ListSet {
  int32_t* m2l_ptr = nullptr;  // [nbox+1]
  int32_t* m2l_src = nullptr;  // [n_m2l]
  int32_t* p2p_ptr = nullptr;  // [nleaf+1]
  int32_t* p2p_src = nullptr;  // [n_p2p]
  int32_t* item_tgt = nullptr;    // [n_items]
  int32_t* item_begin = nullptr;  // [n_items]
  int32_t* item_end = nullptr;    // [n_items]
  int32_t* item_first = nullptr;  // [nbox]
  int32_t* item_cnt = nullptr;    // [nbox]
  int32_t* seg_ptr = nullptr;     // [n_blocks+1]
  int32_t* seg_tgt = nullptr;
  int32_t* seg_lanes = nullptr;
  // Final locals of the target side in two launches (FinList): fin[0] over
  // the leaves' parent boxes, each receiving its own M2L sum and the
  // translations of the M2L sums of all its ancestors with M2L pairs;
  // fin[1] over the leaves, each receiving its own M2L sum and the
  // translation of its parent's final local (when the parent has one).
  FinList fin[2];
  int64_t n_m2l = 0, n_p2p = 0, n_items = 0, n_blocks = 0;
  // Near-field work items: item j covers direct pairs [pitem_kb[j],
  // pitem_ke[j]) of target leaf pitem_leaf[j], about kP2PItemWork
  // interactions or one whole leaf; every target leaf has at least one.
  // pitem_out[j] < 0: the leaf's only item, written to the near field;
  // otherwise the element offset of the item's partial sums (4 rows of the
  // leaf's point count: potential, field x, y, z) in p2p_part.  The split
  // leaves psplit_leaf[i] add the partials of their psplit_cnt[i] items
  // from psplit_first[i] on, in item order.
  int32_t* pitem_leaf = nullptr;
  int32_t* pitem_kb = nullptr;
  int32_t* pitem_ke = nullptr;
  int64_t* pitem_out = nullptr;
  int32_t* psplit_leaf = nullptr;
  int32_t* psplit_first = nullptr;
  int32_t* psplit_cnt = nullptr;
  void* p2p_part = nullptr;
  int64_t n_pitems = 0, n_psplit = 0, p2p_part_elems = 0;
};

// Interactions per near-field work item before a leaf's direct list is
// split (2^16: the uniform 2^20 cube keeps one item per leaf).
constexpr int64_t kP2PItemWork = 1 << 16;

// Per-evaluation device buffers (all but the M2L partial rows of the
// batched form): leaf-ordered source records, expansions, the near field,
// the adjoint's field and the 32-vector copies.
struct Workspace {
  void* src = nullptr;      // [n] {x, y, z, q} in leaf order
  void* C = nullptr;        // [nbox][K]   multipoles (normalised)
  void* D = nullptr;        // [nbox][K]   locals (normalised)
  void* near = nullptr;     // [4n] near field in leaf order: pot [n], field [n][3]
  void* field_t = nullptr;  // [n][3] field of the transposed pass (adjoint)
  // multi-vector workspace (FP32 plans with max_rhs > 1), vectors innermost
  void* bq = nullptr;    // [n][32]
  void* bC = nullptr;    // [nbox][K][32]
  void* bD = nullptr;    // [nbox][K][32]
  void* bpot = nullptr;  // [n][32]
  void* bfld = nullptr;  // [n][3][32]
  bool stages = true;    // record stage-timing events when the plan profiles
};

// Byte offsets of the workspace buffers inside one allocation, each
// aligned to 256 bytes, in the order of Workspace; `forward` is the size of
// the leading part one single-vector evaluation uses (src, C, D, near).
struct WorkspaceLayout {
  size_t off[10] = {0};
  size_t size[10] = {0};
  size_t forward = 0;
  size_t total = 0;
};
WorkspaceLayout workspace_layout(int64_t n, int64_t nbox, const fmm_params& prm, bool batched);
// Point the buffers of ws at base + offsets (the first `count` buffers).
void bind_workspace(Workspace& ws, char* base, const WorkspaceLayout& L, int count);

// One level step of the upward (M2M) or downward (L2L) pass: n boxes a[i]
// with b[i] = first child (M2M; the 2^s children are consecutive) or parent
// (L2L; -1 for a root).
struct Step {
  int32_t* a = nullptr;
  int32_t* b = nullptr;
  int64_t n = 0;
};

// One side of a plan: the charges (sources) or the evaluation points
// (targets).  A plan over one point set has one side that plays both
// roles; a plan with separate sources and targets (Sec. II.B) has the
// sources as side 0 and the targets as side 1, each with its own tree.
// Slots [pt0, pt0 + npt) and leaves [leaf0, leaf0 + nleaf) of the plan's
// concatenated arrays are the side's; its boxes are those of its trees.
struct Side {
  int64_t pt0 = 0, npt = 0;
  int64_t leaf0 = 0, nleaf = 0;
  std::vector<Step> m2m_steps;  // bottom-up, parents of one level per step
  std::vector<Step> l2l_steps;  // top-down, boxes of one level with a parent local
  Step l2l_sum;                 // every box whose local is formed (b unused)
};

}  // namespace fmm

struct fmm_plan {
  int device = 0;
  fmm_params prm{};
  int64_t n = 0;
  int L = 0, s = 0, nch = 0;
  int64_t nbox = 0, nleaf = 0;
  std::vector<int64_t> level_off;  // host, size L+2

  // tree (device)
  int32_t* perm = nullptr;        // [n]
  int32_t* leaf_start = nullptr;  // [nleaf+1]
  double* xs = nullptr;           // leaf-ordered positions [n] x3 (SoA)
  double* ys = nullptr;
  double* zs = nullptr;
  double* cx = nullptr;  // box centres [nbox] (SoA)
  double* cy = nullptr;
  double* cz = nullptr;
  double* radius = nullptr;  // [nbox]
  double* scale = nullptr;   // [nbox] length scale of the box's expansions
  int32_t max_leaf_count = 0;
  bool has_dup = true;  // some two points coincide (set by the tree build)
  // launch tiles (0: the default rule from max_leaf_count; set by
  // fmm_plan_autotune): P2P source groups, P2M/L2P leaves per wave
  int p2p_groups = 0;
  int leaves_per_wave = 0;
  // 1: one lane per M2L translation; 0: the shared form where it is built
  // (m2l_share_waves), else one lane
  int m2l_waves = 0;
  // 1: one lane per M2M / L2L translation; 0: shared by four waves from
  // order kChainShareMinOrder on
  int chain_waves = 0;
  // waves per block of the batched near field (1, 2, 4, 8; 0: by the
  // plan's largest leaf)
  int batch_p2p_waves = 0;
  // 1: the near field on the caller's stream after the far-field chain; 0:
  // on the plan's second stream beside it
  int near_stream = 0;
  int32_t* leaf_box = nullptr;  // [nleaf] global box id of each leaf
  int nsides = 1;               // 2: separate sources (side 0) and targets (side 1)
  fmm::Side side[2];
  int n_problems = 1;           // > 1: union of independent trees

  // lists (device): [0] forward, [1] transposed (every pair reversed; the
  // adjoint operator)
  fmm::ListSet lists[2];
  int64_t p2p_inter = 0;

  // evaluation workspace: one device allocation of workspace_bytes carved
  // into the buffers below (workspace_layout); empty for plans created with
  // FMM_PLAN_NO_WORKSPACE
  fmm::Workspace ws;
  size_t workspace_bytes = 0;
  unsigned flags = 0;  // fmm_plan_create_ex flags
  // batched M2L partial rows [n_items][K][32] (FP32 plans with max_rhs > 1);
  // sized by the lists, so held with them
  void* bpart = nullptr;
  // batched plans: leaf position of every input index (inverse of perm)
  int32_t* iperm = nullptr;
  const void* tables = nullptr;  // device operator tables for (p, precision)

  std::vector<fmm::DevBuf> bufs;
  size_t device_bytes = 0;
  // device memory source of the plan (fmm_plan_create_ex), also used for
  // temporaries during the build; stream passed to the callbacks
  fmm_allocator allocator{nullptr, nullptr, nullptr};
  hipStream_t alloc_stream = nullptr;

  // second stream of the evaluation: the near field runs on it beside the
  // far-field chain (forked after P2M, joined before L2P; events without
  // timing; default priority)
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  // stage timing (fmm_plan_set_profiling)
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;               // free events
  std::vector<std::vector<hipEvent_t>> ev_rows;  // 2 FMM_NSTAGES per pass
};

// Captured evaluation (fmm_graph_create).
struct fmm_graph {
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace fmm {

// Device memory for the plan (kept until fmm_plan_destroy), through the
// plan's allocator.
void* plan_alloc(fmm_plan* pl, size_t bytes);
void plan_free_all(fmm_plan* pl);
// Temporary device memory during the build, through the plan's allocator.
void* dev_alloc(fmm_plan* pl, size_t bytes);
void dev_free(fmm_plan* pl, void* p);
// Temporaries of one build step, released when it goes out of scope.
struct Scratch {
  fmm_plan* pl;
  std::vector<void*> ptrs;
  explicit Scratch(fmm_plan* p) : pl(p) {}
  void* get(size_t bytes) {
    void* p = dev_alloc(pl, bytes);
    ptrs.push_back(p);
    return p;
  }
  ~Scratch() {
    // the build's kernels may still read them: wait for the stream first
    if (!ptrs.empty()) (void)hipStreamSynchronize(pl->alloc_stream);
    for (void* p : ptrs) dev_free(pl, p);
  }
};

// One tree inside a plan: depth, level offsets, first global box id and
// first global leaf.
struct TreeDesc {
  int L;
  std::vector<int64_t> level_off;
  int64_t box_base;
  int64_t leaf_base = 0;
};
// Leaf boxes and level steps of each side over its trees (api.cpp): side k
// takes trees[k] (a plan with one side passes one group).  M2M step h takes
// the parents h+1 levels above each tree's leaves; L2L step l takes level l
// of every tree at least that deep.  Boxes outside every M2L pair and
// without such an ancestor are left out (their expansions are never read,
// or are zero), except that every leaf gets its local.  Also, per list
// direction, the ancestors of every target-side leaf whose M2L sums reach it.
void make_steps(fmm_plan* pl, const std::vector<std::vector<TreeDesc>>& trees, hipStream_t st);
// Side whose charges a pass in direction dir (0: G-hat, 1: G-hat^T) reads,
// and side whose points it evaluates.
inline const Side& src_side(const fmm_plan* pl, int dir) {
  return pl->side[pl->nsides == 1 ? 0 : dir];
}
inline const Side& tgt_side(const fmm_plan* pl, int dir) {
  return pl->side[pl->nsides == 1 ? 0 : 1 - dir];
}
// Union of independent plans (multi.hip): every per-point, per-box and
// per-leaf array concatenated, indices shifted to global numbering.
// With lists = false the sub-plans carry trees only, and perm stays local
// to each sub-plan (input indices of its own point set).
void build_union(fmm_plan* U, const std::vector<const fmm_plan*>& subs, hipStream_t st,
                 bool lists = true);

// Tree build (tree.hip): fills perm, leaf_start, xs/ys/zs, centres, radii.
void build_tree(fmm_plan* pl, const double* pos, hipStream_t st);
// Lists (lists.hip): fills m2l_*, p2p_*, items, from the level march
// between the source tree src and the target tree tgt of the plan (the
// same tree for a plan over one point set).
void build_lists(fmm_plan* pl, const TreeDesc& src, const TreeDesc& tgt, hipStream_t st);
// M2L work items and block segments of one list set from its CSR, and the
// near-field work items of direction dir (lists.hip).
void make_items(fmm_plan* pl, ListSet& S, hipStream_t st);
void make_p2p_items(fmm_plan* pl, int dir, hipStream_t st);
// Operator tables for order p (tables.cpp), cached per process/device.
const void* get_tables(int p, int precision, int device);
// Evaluation (eval.hip): dir 0 = G-hat, dir 1 = G-hat^T.
void evaluate(fmm_plan* pl, const Workspace& ws, int dir, const void* q, int nrhs, void* pot,
              void* field, hipStream_t st);
// Up to batch_width() FP32 charge vectors in one pass (batch.hip).
int batch_width();
// waves per block of the batched near field for this plan
int batch_p2p_waves(const fmm_plan* pl);
// iperm of a batched plan from its perm (on st)
void make_iperm(fmm_plan* pl, hipStream_t st);
void evaluate_batch(fmm_plan* pl, int dir, const float* q, int R, float* pot, float* field,
                    hipStream_t st);
// Adjoint combine: grad_x = -(g * field_fwd + q * field_t) (eval.hip).
void adjoint_combine(fmm_plan* pl, const void* q, const void* g, const void* field_fwd,
                     const void* field_t, void* grad_x, hipStream_t st);

// Direct summation (direct.hip).
void direct_sum(int64_t n, const double* pos, const void* q, int precision,
                const int64_t* targets, int64_t nt, void* pot, void* field,
                hipStream_t st);
// Launch tiles in effect (eval.hip): P2P source groups G (1, 2, 4; G > 1
// needs max_leaf_count <= 64 / G) and P2M/L2P leaves per wave (1, 2, 4, 8;
// needs max_leaf_count <= 64 / leaves).
int p2p_groups(const fmm_plan* pl);
int leaves_per_wave(const fmm_plan* pl);
int m2l_waves(const fmm_plan* pl);
int chain_waves(const fmm_plan* pl);
// lowest order with the shared M2M / L2L forms
constexpr int kChainShareMinOrder = 5;
// Waves per translation of the shared M2L form for order p and precision
// (1: no shared form).  It is built where it was measured faster than one
// lane per translation: FP64 at p = 6, 7 (above, its LDS tile caps the
// occupancy; below, one lane per translation keeps two waves per SIMD
// anyway) and FP32 at p = 9, 10 (where the one-lane form runs out of
// registers).
constexpr int m2l_share_waves(int p, bool fp64) {
  return fp64 ? ((p == 6 || p == 7) ? 4 : 1) : (p >= 9 ? 4 : 1);
}
bool valid_p2p_groups(const fmm_plan* pl, int g);
bool valid_leaves_per_wave(const fmm_plan* pl, int l);

// Stage-timing helpers (api.cpp).
hipEvent_t take_event(fmm_plan* pl);
void release_profile(fmm_plan* pl);
enum { kStSort = 0, kStP2M, kStM2M, kStM2L, kStL2L, kStL2P, kStP2P };
// Begin/end events of every stage of one pass (when profiling is on), each
// pair recorded on the stream the stage runs on.
struct StageMarks {
  std::vector<hipEvent_t>* row = nullptr;
  explicit StageMarks(fmm_plan* pl, bool enabled = true) {
    if (!pl->profiling || !enabled) return;
    pl->ev_rows.emplace_back();
    row = &pl->ev_rows.back();
    for (int k = 0; k < 2 * FMM_NSTAGES; ++k) row->push_back(take_event(pl));
  }
  void begin(int k, hipStream_t s) const {
    if (row) FMM_HIP(hipEventRecord((*row)[2 * k], s));
  }
  void end(int k, hipStream_t s) const {
    if (row) FMM_HIP(hipEventRecord((*row)[2 * k + 1], s));
  }
};

// Runs f, turning exceptions into a status and the thread's error message
// (every C entry point).
template <typename F>
fmm_status guard(F&& f) {
  try {
    clear_error();
    f();
    return FMM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return FMM_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return FMM_EDEVICE;
  } catch (...) {
    set_error("unknown error");
    return FMM_EDEVICE;
  }
}

// Sorting primitives (sort.hip).
size_t sort_pairs_u64_i32_temp(int n);
void sort_pairs_u64_i32(void* temp, size_t temp_bytes, const uint64_t* kin,
                        uint64_t* kout, const int32_t* vin, int32_t* vout,
                        int n, hipStream_t st);
size_t sort_keys_u64_temp(int64_t n);
void sort_keys_u64(void* temp, size_t temp_bytes, const uint64_t* kin,
                   uint64_t* kout, int64_t n, int end_bit, hipStream_t st);
size_t scan_i32_temp(int64_t n);
void exclusive_scan_i32(void* temp, size_t temp_bytes, const int32_t* in,
                        int32_t* out, int64_t n, hipStream_t st);

}  // namespace fmm
