/*
 * fastertucker.h -- C-ABI of the MI355X (gfx950) FasterTucker hot path.
 *
 * Sparse FasterTucker (Li, Duan, Yang, Li; arXiv 2210.06014) approximates an
 * N-order sparse tensor X on its observed set Omega by
 *     xhat(i_1..i_N) = sum_r prod_n C(n)[i_n, r],   C(n) = A(n) B(n)
 * (Eq. (1) evaluated through Eq. (12) and the reusable intermediate of
 * Section 3.1), with factor matrices A(n) (I_n x J) and core matrices
 * B(n) (J x R).  Training is Algorithm 2: per mode a factor pass (one SGD
 * step per observed element on the row a(m)_{i_m}, Eq. (9)-(10)), then per
 * mode a core pass (one step on B(m) with the gradient of Eq. (11) summed
 * over Omega, Algorithm 5), each followed by a refresh of C(m).
 *
 * Conventions shared by every entry point:
 *  - The library allocates no device memory.  The caller owns every device
 *    buffer: the plan's arrays live in a workspace the caller hands to
 *    ft_plan_upload (size from ft_plan_query), and each parameter set brings
 *    its own scratch buffer (ft_params.scratch, size from ft_plan_query).
 *    Both must be 256-byte aligned (torch allocations are).  The one device
 *    array of the library itself is the fixed 56 KiB static scratch of
 *    ft_loss_noalloc.
 *  - Matrices are dense row-major FP32 in device memory owned by the caller
 *    (A(n): I_n x J, B(n): J x R, C(n): I_n x R).  Eq. (1) allows a J_n per
 *    mode; the kernels are compiled for one J shared by all modes, so every
 *    J_n must be equal (FT_ERR_UNSUPPORTED otherwise).
 *  - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *    Work is enqueued on it and the call returns without synchronising,
 *    except where stated.  A plan is immutable once uploaded and may be
 *    shared by any number of parameter sets, on any streams; a parameter set
 *    (its scratch) must not be used on two streams at once.
 *  - Return value: FT_OK, or an error code with a message available from
 *    ft_last_error() (thread-local).  Argument, shape, index and workspace
 *    errors are detected on the host before anything is enqueued;
 *    FT_ERR_HIP reports a failed HIP call or kernel launch.  No exception
 *    crosses the ABI.
 *  - Floating point: FP32 arithmetic with FMA contraction, IEEE round to
 *    nearest even.  Sums over elements run in a fixed order, so results are
 *    bitwise repeatable for a given plan and input.  FP64 is used on the GPU
 *    only for the loss reduction and for powers of the weight-decay factor.
 */
#ifndef FASTERTUCKER_H
#define FASTERTUCKER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FT_OK = 0,
  FT_ERR_ARG = 1,         /* null pointer, negative size, bad mode number */
  FT_ERR_SHAPE = 2,       /* order, dims, J, R or nnz out of range */
  FT_ERR_INDEX = 3,       /* a coordinate outside its dimension */
  FT_ERR_UNSUPPORTED = 4, /* (order, J, R) combination not compiled in */
  FT_ERR_STATE = 5,       /* plan not uploaded, host copy not kept, ... */
  FT_ERR_NOMEM = 6,       /* host allocation failed */
  FT_ERR_HIP = 7,         /* a HIP call failed (copy, launch) */
  FT_ERR_WORKSPACE = 8    /* a workspace or scratch buffer is missing, too small or misaligned */
} ft_status;

#define FT_MAX_ORDER 10

/* ft_desc.flags */
#define FT_KEEP_HOST 1 /* keep the host copy of the plan after upload (ft_plan_host_csr) */
#define FT_WITH_PERM 2 /* keep element permutations on the device (ft_forward, ft_grad with upstream) */
#define FT_NO_FIBER_SHARE 4 /* compute g for every element instead of once per fiber (Section 3.2); same results */
#define FT_NO_C_CACHE 8     /* factor and core passes form every C(n) row they need from A(n) and B(n) on use
                               instead of reading the cached C (the cost structure of FastTucker, kept for the
                               comparison of Table 5; implies FT_NO_FIBER_SHARE).  Order 3, J = R = 16 and FP32
                               storage only (FT_ERR_UNSUPPORTED otherwise); loss, predict and gradient calls
                               still read C, which the refreshes keep current */
#define FT_RELAXED 16       /* relaxed factor passes, modelled on the unordered concurrent row updates of the
                               GPU factor algorithm (Algorithm 4).  The plan deals each row longer than
                               `head` in stride order (Q = ceil(L / head): positions 0, Q, 2Q, ..., then
                               1, 1 + Q, ...), so that its head and its chunks each hold a sample of the
                               whole row.  The head is updated in place (a_H); the chunks then all start
                               from a_H, as concurrent workers reading the row would; chunk k's increment
                               beyond the decay of a_H, d_k, is weighted by rho^T_k (rho = 1 - lr lam, T_k
                               the row's elements after the chunk), and the row becomes a_H + omega
                               ((rho^(L - head) - 1) a_H + sum_k rho^T_k d_k) with omega = min(1, 1 / (lr
                               sum ||g||^2)) over the chunked elements, which keeps the merged step from
                               overshooting.  Not the serial result of Algorithm 2 (it agrees to second
                               order in lr); deterministic.  Rows of at most `head` elements are updated
                               exactly as without the flag.  Not with FT_NO_C_CACHE (FT_ERR_UNSUPPORTED) */

#define FT_SPLIT_FACTOR 32   /* launch the in-place items and the chunk maps of an exact factor pass as two
                               kernels in sequence instead of one (for comparison; same results) */
#define FT_RUN_REUSE 64      /* segment passes (core, loss, forward, gradient) gather the C row of mode m + 1
                               once per run of a row's elements that share it, each slot of a wavefront
                               walking a contiguous piece of the segment, instead of gathering every row for
                               every element (same sums up to rounding order).  Fewer gathers, but measured
                               slower on MI355X, so it is off by default; kept for comparison */

/* Shape of the problem and of the plan. */
typedef struct {
  int32_t order;                /* N, 2..FT_MAX_ORDER */
  int64_t dims[FT_MAX_ORDER];   /* I_n >= 1 with I_n * R * 4 < 2^31 (C rows are gathered by 32-bit byte offsets) */
  int32_t J[FT_MAX_ORDER];      /* factor rank per mode; must all be equal */
  int32_t R;                    /* core rank */
  int64_t nnz;                  /* |Omega|, 0..2^32-1 */
  int32_t chunk;                /* elements per chunk map of a long row (0: 1024 for J >= 32, else 512;
                                   512 with FT_RELAXED) */
  int32_t head;                 /* rows of at most this many elements are updated as one serial chain; a
                                   longer row has its first `head` elements updated in place and the rest
                                   cut into chunks.  0: with FT_RELAXED, 2 chunks; otherwise each mode
                                   takes the longest of 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32 chunks,
                                   up to a cap (32 chunks for J >= 32, 24 for J = 16, 2 otherwise), that
                                   is not above the row length reached by the longest rows holding a
                                   quarter of its elements and whose serial chain a cost model of the
                                   launch (from the row lengths and whether g is shared per fiber)
                                   expects to end within the launch.  ft_plan_mode_info reports the
                                   value each mode uses */
  int32_t fanin;                /* chunk maps folded per combine step (0 or above the maximum: 16 for
                                   J <= 16, 8 above); a row with at most fanin maps has them applied in
                                   sequence to its head's result */
  int32_t flags;                /* FT_KEEP_HOST | FT_WITH_PERM | FT_NO_FIBER_SHARE | FT_NO_C_CACHE | FT_RELAXED |
                                   FT_SPLIT_FACTOR | FT_RUN_REUSE */
} ft_desc;

/* ft_params.storage */
#define FT_STORE_F32 0  /* A, B, C are read and written in FP32 */
#define FT_STORE_BF16 1 /* A16, B16, C16 are read; the FP32 masters A, B receive the updates */

/*
 * Device parameters of one model, for n < order.
 *   FT_STORE_F32:  A[n] (I_n x J), B[n] (J x R), C[n] (I_n x R), FP32.
 *   FT_STORE_BF16: the FP32 masters A[n], B[n] plus their BF16 copies
 *                  A16[n], B16[n] and C16[n] = bf16(A16[n] B16[n]) (uint16_t
 *                  arrays holding bfloat16 bits, same shapes); C[n] unused.
 *                  Every kernel reads the BF16 arrays and accumulates in FP32;
 *                  updates go to the masters, and each refresh rounds the
 *                  masters to BF16 (nearest even) before forming C16.
 */
typedef struct {
  float* A[FT_MAX_ORDER];
  float* B[FT_MAX_ORDER];
  float* C[FT_MAX_ORDER];
  void* A16[FT_MAX_ORDER];
  void* B16[FT_MAX_ORDER];
  void* C16[FT_MAX_ORDER];
  int32_t storage;
  void* scratch;        /* device buffer of at least scratch_bytes (ft_plan_query) for the plans it is used with:
                           chunk maps, partial sums and shared g that the passes write between launches */
  size_t scratch_bytes; /* its size */
} ft_params;

/* Host-side statistics of one mode of a plan (for diagnostics and tests). */
typedef struct {
  int64_t rows;          /* I_m */
  int64_t nonempty_rows; /* rows with at least one element */
  int64_t max_row;       /* largest row length */
  int64_t light_rows;    /* rows of at most `head` elements, updated in one piece */
  int64_t heavy_rows;    /* longer rows: a head plus chunks */
  int64_t chunks;        /* pieces of heavy rows, heads included */
  int64_t segments;      /* pieces of rows used by the core, loss and gradient passes */
  int32_t combine_levels;
  int32_t fiber_shared;  /* 1 if the factor pass shares g per fiber in this mode */
  int64_t fibers;        /* mode-m fibers: distinct (i_n, n != m) */
  int32_t head;          /* the plan's head length (ft_desc.head, or its default) */
  int32_t chunk;         /* the plan's chunk length (ft_desc.chunk, or its default) */
  int64_t runs;          /* runs of elements of a row sharing the index of mode m + 1 */
} ft_mode_info;

typedef struct ft_plan ft_plan;

/*
 * ft_plan_create -- host-side plan (no GPU work).
 *   coords: host int32, structure of arrays, coords[n * nnz + x] is the
 *           mode-n index of element x (0-based).  vals: host float[nnz].
 * For every mode m the elements are ordered by row i_m and, within a row,
 * by the other indices taken cyclically (i_{m+1}, ..., i_{m-1}).  This is
 * the order in which the factor pass visits a row's elements: the per-row
 * order that the fiber-major walk of Algorithm 2 produces (Section 4.5
 * describes the fiber tree whose leaves are the updated mode).
 * Errors: FT_ERR_ARG, FT_ERR_SHAPE, FT_ERR_INDEX (any coordinate out of
 * range), FT_ERR_UNSUPPORTED, FT_ERR_NOMEM.  The inputs are not retained.
 */
ft_status ft_plan_create(ft_plan** out, const ft_desc* desc, const int32_t* coords, const float* vals);

/*
 * ft_plan_query -- device bytes the plan needs (valid from ft_plan_create on):
 *   device_bytes:  its sorted arrays and work lists, the workspace of
 *                  ft_plan_upload;
 *   scratch_bytes: the scratch each parameter set used with the plan must
 *                  bring (ft_params.scratch).
 * The sizes follow from the sorted tensor (rows, long-row chunks, segments,
 * fibers), so they are known only once the host plan exists.  Either
 * output may be NULL.
 */
ft_status ft_plan_query(const ft_plan* plan, size_t* device_bytes, size_t* scratch_bytes);

/*
 * ft_plan_upload -- copies the plan's arrays into the caller's device buffer
 * d_workspace (at least device_bytes, 256-byte aligned), with
 * hipMemcpyAsync on `stream`, and waits for the copies; then frees the host
 * copy unless FT_KEEP_HOST was given.  The workspace must stay allocated and
 * unmodified while the plan is used.  With FT_KEEP_HOST the plan can be
 * uploaded again (to another workspace); otherwise a second upload is
 * FT_ERR_STATE.  Errors: FT_ERR_ARG, FT_ERR_STATE, FT_ERR_WORKSPACE, FT_ERR_HIP.
 */
ft_status ft_plan_upload(ft_plan* plan, void* d_workspace, size_t workspace_bytes, void* stream);

/* Frees the host side of the plan (device memory belongs to the caller). */
void ft_plan_destroy(ft_plan* plan);

ft_status ft_plan_mode_info(const ft_plan* plan, int32_t mode, ft_mode_info* info);

/*
 * ft_plan_host_csr -- copy of the host CSR of one mode (needs FT_KEEP_HOST).
 *   row_ptr int64[I_m + 1]; idx int32[(N-1) * nnz] where column k holds the
 *   indices of mode (m + 1 + k) mod N; vals float[nnz]; perm int64[nnz]
 *   maps a CSR position to the element's input position.  Any may be NULL.
 *   Rows are sorted by (i_m, i_{m+1}, ..., i_{m-1}).  factor_order != 0
 *   returns the order the factor passes read instead: with FT_RELAXED, rows
 *   longer than the head hold their elements in the dealt (stride) order
 *   there; otherwise it is the sorted order.
 */
ft_status ft_plan_host_csr(const ft_plan* plan, int32_t mode, int32_t factor_order, int64_t* row_ptr, int32_t* idx,
                           float* vals, int64_t* perm);

/*
 * ft_refresh -- C(n) = A(n) B(n) for n = mode, or for every mode if mode < 0
 * (the reusable intermediate of Section 3.1; Algorithm 3).  MFMA FP32.
 */
ft_status ft_refresh(const ft_plan* plan, const ft_params* p, int32_t mode, void* stream);

/*
 * ft_predict -- xhat for q query coordinates (device int32, structure of
 * arrays [N][q]) into d_out float[q]: prediction of missing elements once A
 * and B are found (Section 2.4).  Uses the C(n) in p, which must be current.
 * Indices are not checked on the device; they must be in range.
 */
ft_status ft_predict(const ft_plan* plan, const ft_params* p, const int32_t* d_coords, int64_t q, float* d_out,
                     void* stream);

/*
 * ft_factor_pass -- factor module of Algorithm 2 for one mode m: for every
 * element x of Omega, in the plan's per-row order, with
 *     w_x = prod_{n != m} C(n)[i_n, :]   (Eq. (12)),   g_x = B(m) w_x,
 *     e = x - a.g_x,   a <- a + lr (e g_x - lam a)     (Eq. (9), (10))
 * on a = A(m)[i_m, :].  Rows are independent within the pass; a row longer
 * than the head length is updated in place for its first `head` elements,
 * the rest is cut into chunks, and the exact sequential result is recovered
 * by applying the chunks' affine maps in order.  C(m) is NOT
 * refreshed (call ft_refresh, or use ft_factor_epoch).
 */
ft_status ft_factor_pass(const ft_plan* plan, const ft_params* p, int32_t mode, double lr, double lam,
                         void* stream);

/* ft_factor_epoch -- ft_factor_pass then ft_refresh for m = 0..N-1. */
ft_status ft_factor_epoch(const ft_plan* plan, const ft_params* p, double lr, double lam, void* stream);

/*
 * ft_core_grad -- G = sum_{x in Omega} e_x A(m)[i_m, :]^T w_x  (J x R, FP32,
 * row-major into d_G) at the current parameters: the accumulated gradient of
 * Algorithm 5 (Eq. (11) without the regulariser, negated).
 */
ft_status ft_core_grad(const ft_plan* plan, const ft_params* p, int32_t mode, float* d_G, void* stream);

/*
 * ft_core_pass -- core module for mode m: B(m) <- B(m) + lr (G / |Omega| -
 * lam B(m)) with G as in ft_core_grad (Algorithm 5).  C(m) is not refreshed.
 */
ft_status ft_core_pass(const ft_plan* plan, const ft_params* p, int32_t mode, double lr, double lam,
                       void* stream);

/* ft_core_epoch -- ft_core_pass then ft_refresh for m = 0..N-1. */
ft_status ft_core_epoch(const ft_plan* plan, const ft_params* p, double lr, double lam, void* stream);

/* ft_epoch -- one iteration of Algorithm 2: ft_factor_epoch, ft_core_epoch.
 * C must be current on entry and is current on return. */
ft_status ft_epoch(const ft_plan* plan, const ft_params* p, double lr_a, double lam_a, double lr_b, double lam_b,
                   void* stream);

/*
 * ft_loss -- the objective of Eq. (6) in four FP64 numbers written to device
 * memory d_out4: [sum_x (x - xhat)^2, sqrt(that / |Omega|),
 * lam_a sum_n ||A(n)||^2, lam_b sum_n ||B(n)||^2].  Uses the current C.
 */
ft_status ft_loss(const ft_plan* plan, const ft_params* p, double lam_a, double lam_b, double* d_out4,
                  void* stream);

/*
 * ft_loss_noalloc -- ft_loss for callers that cannot allocate device memory
 * or bring a scratch buffer: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  Same kernels, launch grid and
 * result as ft_loss (bit for bit); ft_params.scratch may be NULL.  The FP64
 * partial sums live in a static device array of the library (56 KiB:
 * 2048 loss partials plus 2 FT_MAX_ORDER x 256 regulariser partials), held on
 * every GPU the library runs on until the process ends and located on the
 * first call on each device (make that first call outside graph capture).
 * Nothing is allocated, freed or memset; kernel timing (ft_profile_enable) is
 * skipped for this call.  Every call on a GPU shares that GPU's array, so
 * calls that overlap on one GPU (two streams, two threads) race and give
 * wrong sums; serialise them.  A plan needing more partials than the array
 * holds gets FT_ERR_WORKSPACE (no plan of order <= FT_MAX_ORDER does).
 */
ft_status ft_loss_noalloc(const ft_plan* plan, const ft_params* p, double lam_a, double lam_b, double* d_out4,
                          void* stream);

/* ft_forward -- xhat of every element of the plan, in input order, into
 * d_out float[nnz].  Needs FT_WITH_PERM. */
ft_status ft_forward(const ft_plan* plan, const ft_params* p, float* d_out, void* stream);

/*
 * ft_grad -- gradient of a loss L at fixed parameters given dL/dxhat_x:
 *     dA(n)[i] = sum_{x: i_n = i} delta_x B(n) w(n)_x,
 *     dB(n)    = sum_x delta_x A(n)[i_n, :]^T w(n)_x          (Eq. (10), (11))
 * d_upstream: float[nnz] in input order (needs FT_WITH_PERM), or NULL for
 * delta_x = -(x - xhat_x), the gradient of 1/2 sum e^2.  d_gA[n] (I_n x J)
 * and d_gB[n] (J x R) are overwritten.  Uses the current C.
 */
ft_status ft_grad(const ft_plan* plan, const ft_params* p, const float* d_upstream, float* const* d_gA,
                  float* const* d_gB, void* stream);

/*
 * Kernel timing.  While enabled on a plan, every launch of the kernels
 * listed in ft_kernel_id is bracketed by two hipEvents recorded on the
 * call's stream.  ft_profile_read waits for the recorded events, returns the
 * accumulated milliseconds and launch counts per kernel (arrays of
 * FT_K_COUNT entries, either may be NULL) and clears them.  Enabling or
 * disabling also clears them.  Not for use while another thread launches
 * work with the same plan.
 */
typedef enum {
  FT_K_FACTOR_COMPOSE = 0, /* chunk maps of long rows (FT_RELAXED: chunk increments) */
  FT_K_FACTOR_APPLY = 1,   /* short rows and heads of long rows, applied in place */
  FT_K_COMBINE = 2,        /* folds of chunk maps (FT_RELAXED: the merge of the increments) */
  FT_K_REFRESH = 3,        /* C = A B */
  FT_K_SEGSUM = 4,         /* core and gradient segment sums */
  FT_K_REDUCE = 5,         /* partial-sum reduction and B step */
  FT_K_LOSS = 6,           /* loss and forward gather */
  FT_K_FIBER_G = 7,        /* shared g per fiber */
  FT_K_FACTOR_FUSED = 8,   /* in-place items and chunk maps of an exact factor pass in one launch */
  FT_K_COUNT = 9
} ft_kernel_id;
ft_status ft_profile_enable(ft_plan* plan, int32_t enable);
ft_status ft_profile_read(ft_plan* plan, double* ms, int64_t* launches);

/* Name of a status code, and the message of the last error on this thread. */
const char* ft_status_str(ft_status s);
const char* ft_last_error(void);

/* Whether (order, J, R) has compiled kernels. */
int32_t ft_supported(int32_t order, int32_t J, int32_t R);

#ifdef __cplusplus
}
#endif
#endif
