/*
 * fgt.h -- C ABI of the MI355X (gfx950) one-dimensional fast Gauss transform.
 *
 * The transform (paper: S. Jiang, "A fast Gauss transform in one dimension
 * using sum-of-exponentials approximations", arXiv 1909.09825):
 *
 *     u_i = sum_{j=1..N} exp(-(x_i - y_j)^2 / (4 delta)) alpha_j,   i = 1..M     (1.1)-(1.2)
 *
 * evaluated through a sum-of-exponentials (SOE) approximation of the kernel,
 *
 *     exp(-x^2/(4 delta)) ~ S(x) = Re sum_{k=1..n_e} omega_k exp(-tau0_k |x| / sqrt(delta))     (1.3)
 *
 * (one node per conjugate pair, weight doubled), by sorting targets and sources
 * together and running, per mode, the forward recurrence (4.5) and the
 * backward recurrence (4.6) as parallel affine scans, then accumulating
 * Re(omega_k (h+ + h-)) at the targets (4.1).
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers (hipMalloc'd or equivalent) holding
 *     contiguous arrays of the plan's element type (double for FGT_F64, float
 *     for FGT_F32); the caller owns them.  Inputs are only read.
 *   - Work is enqueued on `stream` and the call returns without synchronising;
 *     nothing is allocated on the device by fgt_eval.
 *   - Return value: FGT_OK or one of the positive error codes below.  A call that
 *     returns an error has enqueued nothing.
 *   - Sizes are element counts.  M + N must be below 2^32.
 */
#ifndef FGT_H_
#define FGT_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define FGT_OK 0
#define FGT_EINVAL 1        /* bad argument: sizes, null pointers, delta, digits, workspace */
#define FGT_EUNSUPPORTED 2  /* valid request the library does not serve (e.g. FP32 beyond 6 digits) */
#define FGT_ENONFINITE 3    /* a coordinate was NaN or infinite (reported by fgt_last_device_status) */
#define FGT_EDEVICE 4       /* a HIP runtime call failed */
#define FGT_EUNSORTED 5     /* FGT_PRESORTED given for points that are not in ascending order */
#define FGT_ENOSPACE 6      /* problem larger than the fixed workspace of fgt_eval_noalloc */

/* Element types. */
#define FGT_F64 0
#define FGT_F32 1

/* Largest number of modes a plan may hold. */
#define FGT_MAX_MODES 8

typedef struct fgt_plan_s* fgt_plan_t;

/*
 * fgt_plan -- choose an SOE table and scale it to delta.
 *
 * Picks the smallest shipped table whose measured max error E_n (the
 * measurement of (3.1): delta = 1, x = 0 and 1e5 log-spaced points on
 * [1e-5, 1e2], plus a denser check grid) is at most 10^-digits, and scales
 * the nodes to tau_k = tau0_k / sqrt(delta) (E_n does not depend on delta).
 *   delta  > 0 and finite.
 *   digits in [1, fgt_max_digits(dtype)].
 *   dtype  FGT_F64 or FGT_F32 (FP32 serves at most 6 digits).
 *   out    receives the plan; the caller releases it with fgt_plan_destroy.
 * A plan is immutable host data and may be shared by concurrent calls.
 * Errors: FGT_EINVAL (delta, digits, dtype, null out), FGT_EUNSUPPORTED.
 */
int fgt_plan(double delta, int digits, int dtype, fgt_plan_t* out);

/* Largest `digits` fgt_plan accepts for `dtype` (0 for an unknown dtype). */
int fgt_max_digits(int dtype);

/*
 * fgt_plan_info -- the plan's table and stated bounds (host pointers; any may be null).
 *   n_modes          number of modes n_e.
 *   err_bound        E_n: |S(x) - exp(-x^2/(4 delta))| <= E_n for all x, so
 *                    |u_SOE - u| <= E_n sum_j |alpha_j| (triangle inequality).
 *   deriv_err_bound  E'_n: bound on |S'(x) - G'(x)| in units of 1/sqrt(delta).
 *   tau, omega       2*n_modes doubles each, (re, im) interleaved; tau is the
 *                    node already divided by sqrt(delta).
 *   delta            the plan's delta.
 * Errors: FGT_EINVAL for a null plan.
 */
int fgt_plan_info(fgt_plan_t plan, int* n_modes, double* err_bound, double* deriv_err_bound,
                  double* tau, double* omega, double* delta);

/* Release a plan.  Accepts null. */
void fgt_plan_destroy(fgt_plan_t plan);

/*
 * fgt_workspace_size -- bytes of device workspace fgt_eval needs for M targets
 * and N sources with this plan (0 for a null plan or negative sizes).
 * The workspace holds the sort keys and permutation (double-buffered), the
 * radix histograms and look-back state, per-tile scan carries and a status word.
 */
size_t fgt_workspace_size(fgt_plan_t plan, int64_t M, int64_t N);

/*
 * fgt_eval -- u = SOE approximation of (1.1) for targets x[M], sources y[N],
 * strengths alpha[N]; writes u[M] in the order of x.
 *   ws/ws_bytes  device workspace of at least fgt_workspace_size(plan, M, N)
 *                bytes, 256-byte aligned; its contents need not be cleared and
 *                are clobbered.  One workspace may not be used by two calls at
 *                once.
 *   u            may not alias x, y, alpha or ws.
 * M == 0 enqueues nothing; N == 0 writes zeros.  Problems with M + N <= 4096
 * run in two launches, one workgroup per mode and a sum over the modes (the
 * sort then orders every key bit); larger ones as the sequence of sort and
 * scan kernels.  Either way the
 * workspace afterwards holds the sorted state fgt_eval_sorted and fgt_backward
 * (FGT_SORTED) start from.
 * Non-finite coordinates are detected on the device and reported by
 * fgt_last_device_status; u is then unspecified.
 * Errors: FGT_EINVAL (negative sizes, M + N >= 2^32, null pointer with a
 * non-zero size, workspace too small or misaligned), FGT_EDEVICE.
 */
int fgt_eval(fgt_plan_t plan, const void* x, int64_t M, const void* y, const void* alpha,
             int64_t N, void* u, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * fgt_eval_noalloc -- fgt_eval for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and result as fgt_eval, without the workspace:
 * the call uses a fixed array of FGT_NOALLOC_BYTES bytes in device memory,
 * built into the library, one per device, held until the process ends.  It
 * calls no allocator (neither hipMalloc nor any library routine that
 * allocates).  The address of a device's array is looked up once, at the
 * first call on that device (then a mutex serialises the look-up).
 *   stream  must belong to the current device (FGT_EINVAL otherwise).
 * Limit: fgt_workspace_size(plan, M, N) <= FGT_NOALLOC_BYTES, which holds for
 * M + N up to 1,500,000 points (FP64 or FP32, any digits); larger problems
 * return FGT_ENOSPACE and enqueue nothing.
 * Every call on one device shares that device's array: the call clears what
 * must start at zero, and two calls that overlap in time on one device (other
 * streams, other host threads) race and give wrong results.  Calls on one
 * stream are ordered and safe.  The array's device status word is not
 * readable (fgt_last_device_status needs a caller's workspace): with
 * non-finite coordinates u is unspecified.
 * Errors: as fgt_eval, plus FGT_ENOSPACE.
 */
#define FGT_NOALLOC_BYTES (64u << 20)
int fgt_eval_noalloc(fgt_plan_t plan, const void* x, int64_t M, const void* y, const void* alpha,
                     int64_t N, void* u, hipStream_t stream);

/* Flag for fgt_backward: the workspace already holds the sort of (x, y). */
#define FGT_SORTED 1
/* Flag for fgt_eval_self: the points are already in ascending order. */
#define FGT_PRESORTED 2

/*
 * fgt_eval_self -- the transform with targets identical to the sources
 * (Section 5's first test case):  u_i = sum_j S(x_i - x_j) alpha_j,  i, j = 1..N,
 * the self term included.  Every sorted point is then both a source and a
 * target, so half as many points are sorted and scanned as with fgt_eval(x, x).
 *   flags  0, or FGT_PRESORTED when x is already ascending (e.g. Chebyshev
 *          points in order): the radix sort is skipped.  The order is checked on
 *          the device; a violation is reported by fgt_last_device_status as
 *          FGT_EUNSORTED (u is then unspecified).
 *   ws     fgt_workspace_size(plan, 0, N) bytes, as for fgt_eval.
 * N == 0 enqueues nothing.  Errors: as fgt_eval, plus FGT_EINVAL for unknown flags.
 */
int fgt_eval_self(fgt_plan_t plan, const void* x, int64_t N, const void* alpha, void* u, int flags,
                  void* ws, size_t ws_bytes, hipStream_t stream);

/* Flag for fgt_sort: sort every key bit, and code FP64 keys only where exact. */
#define FGT_SORT_EXACT 4

/*
 * fgt_sort -- the sort step of Section 4 alone, exactly as fgt_eval runs it
 * for M + N > 4096 (fgt_eval sorts smaller problems with every key bit, as
 * FGT_SORT_EXACT does here):
 * the merged points [y_1..y_N, x_1..x_M] in ascending order (the paper sorts
 * sources and targets before the recurrences and times that step on its
 * own, Section 5).  Writes, per sorted position p, the merged index perm[p]
 * (perm[p] < N: source perm[p]; otherwise target perm[p] - N) and the
 * coordinate z[p] that the scans use; either may be null.  alpha (may be
 * null) is gathered into sorted order as fgt_eval does, so with alpha given
 * the workspace afterwards holds the state fgt_eval_sorted and fgt_backward
 * (FGT_SORTED) start from.
 *   flags 0: the plan's resolution.  Points whose coordinates differ by less
 *          than the key width resolution[0] may be left in either order (the
 *          change this makes to any transform value is at most 1e-6 E_n
 *          sum|alpha|), and an FP64 coordinate may be moved by less than
 *          resolution[1] when it is finer than the key grid fitted to the
 *          range (0 when every point lies on that grid).
 *   FGT_SORT_EXACT: every key bit is sorted and the FP64 grid code is used
 *          only where it is exact: perm is then the stable ascending order of
 *          [y; x] (equal coordinates keep their merged order, -0 equals +0)
 *          and z[p] is the input coordinate bit for bit (-0 stored as +0).
 *   perm       [M + N] uint32 device array, z [M + N] of the plan's type.
 *   resolution host double[2] (may be null): the key width and the FP64
 *              code tolerance of this call (both 0 with FGT_SORT_EXACT).
 *   ws         as for fgt_eval.
 * Non-finite coordinates are reported by fgt_last_device_status.
 * Errors: as fgt_eval, plus FGT_EINVAL for unknown flags.
 */
int fgt_sort(fgt_plan_t plan, const void* x, int64_t M, const void* y, const void* alpha, int64_t N,
             int flags, uint32_t* perm, void* z, double* resolution, void* ws, size_t ws_bytes,
             hipStream_t stream);

/*
 * fgt_eval_sorted -- fgt_eval for new strengths alpha[N] on points already
 * sorted: `ws` must hold the sorted state that the last fgt_eval (or
 * fgt_backward without FGT_SORTED) wrote for the same plan, M, N and point
 * coordinates.  Only the strengths are gathered again, so repeated transforms
 * with fixed points skip the radix sort (the sort of Section 4 depends on the
 * coordinates alone).  A workspace that does not hold such a state gives
 * unspecified values but no access outside u, alpha and ws.
 * Errors: as fgt_eval.
 */
int fgt_eval_sorted(fgt_plan_t plan, int64_t M, int64_t N, const void* alpha, void* u, void* ws,
                    size_t ws_bytes, hipStream_t stream);

/*
 * fgt_backward -- gradients of L = sum_i g_i u_i, u the transform of fgt_eval.
 * With S the plan's SOE kernel and S' its x-derivative
 * (S'(r) = Re sum_k (-tau_k omega_k) sign(r) exp(-tau_k |r|), sign(0) taken as the
 * side the sort puts the pair on):
 *   dalpha[j] = sum_i g_i S(y_j - x_i)                  transposed transform (sources
 *                                                       and targets swapped),
 *   dx[i]     = g_i sum_j alpha_j S'(x_i - y_j),
 *   dy[j]     = alpha_j sum_i g_i S'(y_j - x_i),
 *   ddelta[0] = -(sum_i x_i dx[i] + sum_j y_j dy[j]) / (2 delta)
 * (the last from u(c x, c y; c^2 delta) = u(x, y; delta), which S obeys exactly
 * because its nodes scale as 1/sqrt(delta)).  All are device arrays of the plan's
 * type: g[M], dalpha[N], dx[M], dy[N], ddelta a single element.  Any output may
 * be null to skip it.  The gradients come from one adjoint pass over the sorted
 * points in which the strengths alpha (for dL/dx) and g (for dL/dalpha, dL/dy)
 * share every mode exponential.
 *   flags  0 or FGT_SORTED.  With FGT_SORTED, `ws` must hold the state left by
 *          the last fgt_eval or fgt_eval_sorted with this plan and these
 *          points: its sort and its strengths, which are used in place of
 *          `alpha` (x, y and alpha are then not read and may be null).
 *          Without it the points are sorted first and alpha is read.
 *   ws     as for fgt_eval; the call leaves the sorted state in it.
 * M == 0 or N == 0 writes zeros to every requested output.
 * Errors: as fgt_eval, plus FGT_EINVAL for unknown flags.
 */
int fgt_backward(fgt_plan_t plan, const void* x, int64_t M, const void* y, const void* alpha,
                 int64_t N, const void* g, void* dalpha, void* dx, void* dy, void* ddelta,
                 int flags, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Batched transforms.  B independent transforms in CSR layout: transform b has
 * targets x[x_off[b] .. x_off[b+1]), sources y[y_off[b] .. y_off[b+1]), its own
 * delta[b] > 0, and R strength columns: alpha is [y_off[B]][R] row-major and
 * u is [x_off[B]][R] row-major, u[i][r] = sum_j S_b(x_i - y_j) alpha[j][r] over
 * the sources of the transform that target i belongs to.  All transforms share
 * the SOE table chosen for `digits`; since its nodes scale as 1/sqrt(delta)
 * (1.3), transform b runs on coordinates scaled by 1/sqrt(delta_b).  Only FP64
 * is served (FGT_EUNSUPPORTED for FGT_F32).
 *
 * fgt_batch_plan -- validate the layout and build the per-transform tables.
 *   delta, x_off, y_off  HOST arrays ([B], [B+1], [B+1]); offsets start at 0 and
 *                        do not decrease.  1 <= R <= 64.  x_off[B] + y_off[B]
 *                        must be below 2^31 - 1.
 *   out                  receives the plan (device tables allocated here, with
 *                        hipMalloc and synchronous copies; release with
 *                        fgt_batch_destroy once no fgt_batch_eval using it is pending).
 * Errors: FGT_EINVAL (null pointers, offsets, deltas, R, digits), FGT_EUNSUPPORTED,
 * FGT_EDEVICE.
 */
typedef struct fgt_batch_s* fgt_batch_t;
int fgt_batch_plan(int64_t B, const double* delta, int digits, int dtype, const int64_t* x_off,
                   const int64_t* y_off, int R, fgt_batch_t* out);

/* Device workspace bytes for fgt_batch_eval (0 for a null plan). */
size_t fgt_batch_workspace_size(fgt_batch_t plan);

/* Modes, stated bound E_n and total merged points of a batch plan (host pointers, any null). */
int fgt_batch_info(fgt_batch_t plan, int* n_modes, double* err_bound, int64_t* total_points);

/*
 * fgt_batch_eval -- all B transforms, enqueued on `stream` as a fixed sequence
 * of kernels: no allocation, no host synchronisation and no memset, so the
 * call may be captured into a HIP graph and replayed.  x, y, alpha, u, ws are
 * device pointers (ws 256-byte aligned, fgt_batch_workspace_size bytes, not
 * shared with a concurrent call).  Non-finite scaled coordinates are reported by
 * fgt_last_device_status(ws, stream).
 * Errors: FGT_EINVAL (null pointers, workspace), FGT_EDEVICE.
 */
int fgt_batch_eval(fgt_batch_t plan, const void* x, const void* y, const void* alpha, void* u,
                   void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * fgt_batch_sorted -- the sort step of a batch (Section 4's ascending order of
 * each transform's merged sources and targets) as the last fgt_batch_eval on
 * `ws` left it, copied out on `stream`.
 *   codes [P] uint32 device array (may be null), P = sum_b (M_b + N_b): at
 *         sorted position p, the point's code: j for source row j (y[j],
 *         alpha rows), SN + i for target row i (x[i]), SN = sum_b N_b.
 *         Transform b holds positions [base_b, base_b + M_b + N_b), base_b
 *         the sum of M + N over the transforms before it.
 *   z     [P] double device array (may be null): the point's coordinate as
 *         given (unscaled), bit for bit.
 *   resolution  host double (may be null): the sort resolution s in scaled
 *         units (coordinate / sqrt(delta_b)).
 * Order within transform b: ascending in the key
 *   q = trunc(clamp((z / sqrt(delta_b) - lo_b) * 2^62 / (hi_b - lo_b), 0, 2^62)),
 * lo_b, hi_b the smallest and largest scaled coordinate (each product and
 * difference rounded in FP64 as written), with the key bits below
 * 8 floor(L / 8) ignored, L = floor(log2(s 2^62 / (hi_b - lo_b))) clamped to
 * [0, 62]; equal (truncated) keys keep the merged order [sources; targets].
 * The key never decreases as the coordinate grows, so two points out of
 * coordinate order have equal keys above those bits: they lie closer than
 * s sqrt(delta_b) plus the rounding of the key's arithmetic (at most 2^11 + 1
 * key units, a key unit being (hi_b - lo_b) sqrt(delta_b) / 2^62, plus two
 * units in the last place of the larger coordinate).
 * ws must hold a completed fgt_batch_eval of this plan: otherwise the values
 * are unspecified (no access outside ws, codes and z).
 * Errors: FGT_EINVAL (null plan or ws, short or misaligned workspace), FGT_EDEVICE.
 */
int fgt_batch_sorted(fgt_batch_t plan, const void* ws, size_t ws_bytes, uint32_t* codes, void* z,
                     double* resolution, hipStream_t stream);

/*
 * Autotuning.  Two choices shape the batched kernels: the points each lane
 * runs per column in the scan (`chunk`: 8 or 16) and the size the sort aims
 * for when it splits a transform into LDS-sorted buckets (`bucket_points`:
 * 1024 or 2048).  fgt_batch_tune times the four combinations on the given
 * data (one warm-up and three timed fgt_batch_eval calls each, HIP events on
 * `stream`, which it synchronises), keeps the fastest in the plan and, if
 * `cache_path` is not null, records it in that JSON file under a key made of
 * the architecture, log2 of B and of the total points, R and the mode count;
 * a later call with a matching key takes the recorded choice without timing.
 * u and ws are overwritten.  fgt_batch_config / fgt_batch_set_config read and
 * set the choice directly (default: chunk 16, buckets of 2048).
 * Errors: FGT_EINVAL (null plan, values outside the choices), as fgt_batch_eval.
 */
int fgt_batch_tune(fgt_batch_t plan, const void* x, const void* y, const void* alpha, void* u,
                   void* ws, size_t ws_bytes, hipStream_t stream, const char* cache_path);
int fgt_batch_config(fgt_batch_t plan, int* chunk, int* bucket_points);
int fgt_batch_set_config(fgt_batch_t plan, int chunk, int bucket_points);

/* Release a batch plan.  Accepts null. */
void fgt_batch_destroy(fgt_batch_t plan);

/*
 * fgt_eval_batched -- one-shot form: plan, evaluate, wait for `stream`, release.
 * Arguments as for fgt_batch_plan and fgt_batch_eval; the workspace size comes
 * from fgt_eval_batched_workspace_size (0 on invalid arguments).  Unlike the
 * other entry points it allocates (the plan's tables) and synchronises.
 */
size_t fgt_eval_batched_workspace_size(int64_t B, const int64_t* x_off, const int64_t* y_off,
                                       int R, int digits);
int fgt_eval_batched(int64_t B, const double* delta, int digits, int dtype, const int64_t* x_off,
                     const int64_t* y_off, const void* x, const void* y, const void* alpha, int R,
                     void* u, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * fgt_last_device_status -- synchronise `stream`, then read and clear the
 * status word that the last call on workspace `ws` left there.
 * Returns FGT_OK, FGT_ENONFINITE, FGT_EUNSORTED, or FGT_EINVAL / FGT_EDEVICE.
 */
int fgt_last_device_status(void* ws, hipStream_t stream);

/*
 * Phase timing for benchmarks.  Between fgt_profile_begin and fgt_profile_end
 * every fgt_eval records HIP events on its own stream around each kernel
 * group (phase names: fgt_profile_phase_name).  fgt_profile_end waits for the
 * recorded events and returns, per phase, the milliseconds summed over the
 * calls (ms[max_phases], host memory), the number of phases and of calls.
 * A number of phases above the number of phase names means that some call
 * marked more phase boundaries than the profiler records (a library defect).
 * Not thread-safe; meant for single-threaded benchmark drivers.
 */
int fgt_profile_begin(void);
int fgt_profile_end(double* ms, int max_phases, int* n_phases, int* n_calls);
const char* fgt_profile_phase_name(int phase);

/* Human-readable text for a status code (static storage). */
const char* fgt_strerror(int status);

/* Library version string (static storage). */
const char* fgt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FGT_H_ */
