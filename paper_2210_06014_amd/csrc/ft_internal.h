// Internal structures shared by the host plan, the kernels and the C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fastertucker.h"

namespace ft {

// Factor-pass work item: a whole light row (kind LIGHT), the first chunk of
// a heavy row (HEAD, result written to the row's head vector) or a later
// chunk of a heavy row (COMPOSE, its affine map written to a map slot).
enum : int32_t { ITEM_LIGHT = 0, ITEM_HEAD = 1, ITEM_COMPOSE = 2 };

struct FItem {
  int64_t start;  // first CSR position
  int32_t len;    // elements (0 for padding)
  int32_t row;    // row of the updated mode
  int32_t slot;   // head-vector slot (HEAD) or map slot (COMPOSE)
  int32_t kind;
};
static_assert(sizeof(FItem) == 24, "FItem layout");

// One step of the combine reduction: fold `count` consecutive maps starting
// at in_off (in order) into one; write it to out_off, or if out_off < 0
// apply it to the head vector `heavy` and write row `row` of A(m).
struct CItem {
  int64_t in_off;
  int64_t out_off;
  int32_t count;
  int32_t row;
  int32_t heavy;
  int32_t pad;
};
static_assert(sizeof(CItem) == 32, "CItem layout");

// A piece of a row for the core, loss and gradient passes.
struct Seg {
  int64_t start;
  int32_t len;
  int32_t row;
};
static_assert(sizeof(Seg) == 16, "Seg layout");

struct ModeHost {
  std::vector<int64_t> row_ptr;   // I+1
  std::vector<int32_t> idx;       // (N-1) * nnz
  std::vector<float> val;         // nnz
  std::vector<int64_t> perm;      // nnz: CSR position -> input position
  std::vector<FItem> compose;     // COMPOSE items, padded to multiples of 4
  std::vector<FItem> apply;       // HEAD then LIGHT items, padded to multiples of 4
  std::vector<std::vector<CItem>> levels;
  std::vector<CItem> relax;       // FT_RELAXED: group items (chunk slots -> group record), then one merge item per
                                  // heavy row (its group records; out_off = elements after the head)
  std::vector<Seg> segs;
  std::vector<int64_t> seg_ptr;   // I+1: segments of row i are seg_ptr[i]..seg_ptr[i+1]-1
  std::vector<int32_t> fid;       // nnz: fiber of the element at each CSR position
  std::vector<int32_t> fib_idx;   // (N-1) x fibers: fixed indices of each fiber (modes m+1, ..., m-1)
  // FT_RELAXED with rows longer than the head: idx, val and perm with those
  // rows dealt in stride order (the order of the factor passes); empty otherwise
  std::vector<int32_t> fidx;
  std::vector<float> fval;
  std::vector<int64_t> fperm;     // host only (ft_plan_host_csr)
};

struct ModeDev {
  int64_t* row_ptr = nullptr;
  int32_t* idx = nullptr;
  float* val = nullptr;
  int32_t* perm = nullptr;  // device permutation (int32: nnz < 2^31 required with FT_WITH_PERM)
  FItem* compose = nullptr;
  FItem* apply = nullptr;
  CItem* levels = nullptr;  // all levels back to back
  CItem* relax = nullptr;
  Seg* segs = nullptr;
  int64_t* seg_ptr = nullptr;
  int32_t* fid = nullptr;
  int32_t* fib_idx = nullptr;
  int32_t* fidx = nullptr;  // factor-order copies (FT_RELAXED), or null: the factor passes read idx, val
  float* fval = nullptr;
};

// Byte offsets of a mode's arrays in the caller's plan workspace (SIZE_MAX:
// the array is empty and its device pointer stays null).
struct ModeOff {
  size_t row_ptr, idx, val, perm, compose, apply, levels, relax, segs, seg_ptr, fid, fib_idx, fidx, fval;
};

// Every array in a device workspace starts on this boundary.
constexpr size_t kAlign = 256;

// Sequential layout of arrays in one device buffer.
struct Layout {
  size_t bytes = 0;
  size_t add(size_t n) {
    if (n == 0) return SIZE_MAX;
    const size_t o = (bytes + kAlign - 1) / kAlign * kAlign;
    bytes = o + n;
    return o;
  }
};

// Scratch of one parameter set (ft_params.scratch): what the passes write
// between launches.  Byte offsets, sized for the largest mode of the plan.
struct ScratchOff {
  size_t maps = SIZE_MAX;       // float: chunk maps (J^2 + J each; FT_RELAXED: increments, then FP64 group records)
  size_t map_scale = SIZE_MAX;  // double: rho^length of each map
  size_t hvec = SIZE_MAX;       // float: head vectors of long rows (J each)
  size_t partials = SIZE_MAX;   // float: per-workgroup J x R partial sums, then their folds
  size_t dpartials = SIZE_MAX;  // double: per-workgroup FP64 loss partials, then the regulariser partials
  size_t tseg = SIZE_MAX;       // float: per-segment sums of the gradient pass (R each)
  size_t gfib = SIZE_MAX;       // float: the shared g of each fiber (J each)
};

// Device pointers of a parameter set's scratch for one call.
struct Scratch {
  float* maps = nullptr;
  double* map_scale = nullptr;
  float* hvec = nullptr;
  float* partials = nullptr;
  double* dpartials = nullptr;
  float* tseg = nullptr;
  float* gfib = nullptr;
};

struct ModeMeta {
  int64_t I = 0;
  int64_t n_compose = 0;  // padded counts
  int64_t n_apply = 0;
  int64_t n_heavy = 0;
  int64_t n_maps = 0;     // COMPOSE items (unpadded)
  std::vector<int64_t> level_off;  // offset of each level in the device array
  std::vector<int64_t> level_len;
  std::vector<int64_t> level_ncomp;  // folds at the head of each level (final items follow)
  int64_t n_level_out0 = 0;        // outputs of level 0 (ping-pong buffer size)
  int64_t n_segs = 0;
  int64_t n_relax_groups = 0;  // FT_RELAXED level-1 items
  int64_t n_relax = 0;         // FT_RELAXED level-2 items (heavy rows)
  int64_t n_fibers = 0;
  int64_t n_runs = 0;  // runs of equal column-0 index within rows
  int64_t head = 0;    // elements of a long row updated in place before its chunk maps
  bool use_fiber = false;
  ft_mode_info info{};
};

}  // namespace ft

struct ft_prof_rec {
  int kid;
  hipEvent_t start, stop;
};

struct ft_plan {
  ft_desc desc{};
  int N = 0, J = 0, R = 0;
  int64_t nnz = 0;
  int chunk = 512, head = 1024, fanin = 16;  // head 0: chosen per mode (ModeMeta::head), at most head_cap
  int64_t head_cap = 0;
  bool no_c_cache = false;  // FT_NO_C_CACHE
  bool relaxed = false;     // FT_RELAXED
  bool fused = true;        // exact factor passes launch in-place items and chunk maps together (not FT_SPLIT_FACTOR)
  bool run_reuse = false;   // segment passes reuse the column-0 C row along runs (FT_RUN_REUSE)
  int loss_mode = 0;        // the mode whose CSR the loss and forward passes walk
  std::vector<ft::ModeMeta> meta;
  std::vector<ft::ModeHost> host;
  std::vector<ft::ModeDev> dev;
  bool host_valid = false;
  bool uploaded = false;
  // device arrays of the plan: byte offsets in the caller's workspace (ft_plan_upload)
  std::vector<ft::ModeOff> off;
  size_t device_bytes = 0;
  // scratch every parameter set brings (ft_params.scratch)
  ft::ScratchOff soff;
  size_t scratch_bytes = 0;
  // kernel timing (ft_profile_enable); launches on a const plan append to it
  mutable bool prof_on = false;
  mutable std::vector<ft_prof_rec> prof;
};

namespace ft {
void set_error(const std::string& msg);
ft_status fail(ft_status s, const std::string& msg);

// kernel launchers (ft_refresh.hip, ft_factor.hip, ft_segment.hip); return hipSuccess or the launch error
constexpr int kPartials = 2048;  // max workgroups of the reduction kernels
constexpr int kSegLen = 512;     // max elements per segment
constexpr int kRelaxGroup = 256; // chunks per level-1 group of the relaxed merge

// FT_RELAXED scratch in the map region: J + 1 floats per chunk slot, then
// (8-byte aligned) J + 1 doubles per level-1 group
inline int64_t relax_incr_floats(int64_t n_maps, int J) { return (n_maps * (J + 1) + 1) / 2 * 2; }

// Launches on this thread inside an UntimedScope create no timing events
// (the entry point that must not allocate).
inline bool& untimed_flag() {
  static thread_local bool f = false;
  return f;
}
struct UntimedScope {
  bool prev;
  UntimedScope() : prev(untimed_flag()) { untimed_flag() = true; }
  ~UntimedScope() { untimed_flag() = prev; }
};

// Brackets one kernel launch with events when timing is enabled on the plan.
struct KTimer {
  const ft_plan* P;
  int kid;
  hipStream_t s;
  hipEvent_t a = nullptr;
  KTimer(const ft_plan* P_, int kid_, hipStream_t s_) : P(P_), kid(kid_), s(s_) {
    if (P && P->prof_on && !untimed_flag() && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, s);
  }
  ~KTimer() {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) == hipSuccess && hipEventRecord(b, s) == hipSuccess)
      P->prof.push_back(ft_prof_rec{kid, a, b});
    else
      (void)hipEventDestroy(a);
  }
};

inline double* relax_partials(const ft_plan* P, const Scratch& S, int m) {
  return reinterpret_cast<double*>(S.maps + relax_incr_floats(P->meta[m].n_maps, P->J));
}

// Scratch pointers of a parameter set (its buffer checked by the caller).
Scratch scratch_of(const ft_plan* P, const ft_params* p);

hipError_t launch_refresh(const ft_plan* P, int n, const ft_params* p, hipStream_t s);
hipError_t launch_factor(const ft_plan* P, int m, const ft_params* p, const Scratch& S, double lr, double lam,
                         hipStream_t s);
hipError_t launch_core_grad(const ft_plan* P, int m, const ft_params* p, const Scratch& S, float* G_out,
                            hipStream_t s);
hipError_t launch_core_update(const ft_plan* P, int m, const ft_params* p, const Scratch& S, double lr, double lam,
                              hipStream_t s);
hipError_t launch_loss(const ft_plan* P, const ft_params* p, const Scratch& S, double lam_a, double lam_b,
                       double* out4, hipStream_t s);
hipError_t launch_predict(const ft_plan* P, const ft_params* p, const int32_t* coords, int64_t q, float* out,
                          hipStream_t s);
// ft_loss_noalloc: the loss with its partials in the library's static device
// array (capacity and the bytes a plan needs, in bytes)
size_t noalloc_loss_capacity();
size_t noalloc_loss_need(const ft_plan* P);
hipError_t launch_loss_noalloc(const ft_plan* P, const ft_params* p, double lam_a, double lam_b, double* out4,
                               hipStream_t s);
hipError_t launch_forward(const ft_plan* P, const ft_params* p, const Scratch& S, float* out, hipStream_t s);
hipError_t launch_grad(const ft_plan* P, const ft_params* p, const Scratch& S, const float* upstream,
                       float* const* gA, float* const* gB, hipStream_t s);
bool supported(int N, int J, int R);
int max_fanin(int J);  // largest combine fan-in the kernels hold in LDS
}  // namespace ft
