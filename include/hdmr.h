/*
 * hdmr.h -- C ABI of the MI355X (gfx950) library for anchored cut-HDMR
 * expansions whose component functions are hierarchical sparse grids.
 *
 * Method: Eftekhari & Scheidegger, "High-Dimensional Dynamic Stochastic Model
 * Representation" (arXiv 2202.06555).  A model represents
 *
 *     F(x) = c0 + sum_S w_S u_S(x_S),   u_S(x_S) = sum_j alpha_{S,j} prod_{q in S} phi_{l_jq,i_jq}(x_q)
 *
 * with the 1-D hat basis of eq (3.1), the odd index sets of eq (3.3) (zero
 * boundary), the tensor basis of eq (3.2) and the interpolant of eq (3.6).
 * With w_S = 1 and c0 = f(xbar) this is the cut-HDMR expansion of eq (3.16)
 * grouped per component; with w_S = b_S of eq (4.2) it is the vectorised form
 * a(x)^T b of Sec. 4.1.  Every alpha row carries m outputs (f : [0,1]^d -> R^m,
 * Sec. 3.1).
 *
 * Conventions shared by every entry point:
 *   - Return value: HDMR_OK (0) or a negative HDMR_E* code; the message of the
 *     last failure on the calling thread is available from hdmr_last_error().
 *     No C++ exception crosses this boundary.
 *   - Pointers named "host" are CPU memory; "dev" pointers are device memory
 *     of the model's device (e.g. from hipMalloc or a torch CUDA tensor).  The
 *     caller owns every buffer it passes and the library never frees them.
 *     The library owns every hdmr_model until hdmr_free.
 *   - Arrays are dense and row-major: points n x d, values n x m, gradients
 *     n x d x m, all float64.  Device pointers must be 8-byte aligned.
 *   - stream is a hipStream_t (NULL = the legacy default stream).  Evaluation
 *     calls enqueue work on it and return without waiting; a fault inside a
 *     kernel surfaces as HDMR_EDEVICE at the next call that synchronises.
 *   - Points outside [0,1]^d evaluate with the zero extension eq (3.1) gives;
 *     a NaN coordinate makes every output (and gradient entry) of that point NaN.
 *   - Limits: |S| <= 4 per component, d <= 32767, 1 <= level <= 30, and
 *     sum_q (l_q - 1) <= 31 for each stored level multi-index.
 *   - Environment variables (diagnostics and tests; only HDMR_MIXED_SPLIT
 *     changes a result, within the mixed path's error):
 *     HDMR_EVAL_PATH=gather|sorted forces hdmr_eval's kernel;
 *     HDMR_SORTED_VARIANT=<bits> selects another tile shape of the cell-sorted
 *     kernel; HDMR_BATCH_PATH=gather|sorted replaces hdmr_eval_batched's
 *     measured choice; HDMR_MIXED_SPLIT=2 keeps two BF16 terms instead of
 *     three; HDMR_BUILD_PROFILE=1 prints the build's phase times to stderr;
 *     HDMR_REFINE=host admits a build's children on the host instead of on
 *     the device (the same grids and surpluses, bit for bit);
 *     HDMR_FAIL_ALLOC=k makes the library's device allocation number k
 *     (counted from when the variable takes that value) fail, so that the
 *     HDMR_ENOMEM paths can be tested from the host.
 */
#ifndef HDMR_H
#define HDMR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HDMR_OK 0
#define HDMR_EINVAL (-1)       /* bad argument: null pointer, shape, m mismatch, misalignment */
#define HDMR_ENOMEM (-2)       /* host or device allocation failed                            */
#define HDMR_EDEVICE (-3)      /* HIP runtime error (message has the HIP error string)        */
#define HDMR_ECALLBACK (-4)    /* the user function returned non-zero                         */
#define HDMR_EUNSUPPORTED (-5) /* outside the documented limits or not implemented            */

#define HDMR_PLAIN_FP64 0      /* FP64 basis, FP64 contraction, FP64 sum                       */
#define HDMR_MIXED 1           /* FP32 basis, split-BF16 MFMA contraction, FP64 anchor sum     */

typedef struct hdmr_model hdmr_model;
typedef void *hdmr_stream_t;   /* a hipStream_t */

/* User function f : [0,1]^d -> R^m evaluated on the host: X is n x d (host),
 * Y is n x m (host, written by f).  Returns 0 on success.  Must give identical
 * outputs for identical rows. */
typedef int (*hdmr_fn)(const double *X, int64_t n, int32_t d, double *Y, int32_t m, void *user);

/* Library set-up on a device.  Optional: every entry point initialises the
 * current device on first use.  Returns HDMR_EDEVICE if no device is usable. */
int hdmr_init(int32_t device);

/* ---------------------------------------------------------------------------
 * Building a model from a function (Alg. 2).
 *
 * For every index set S (explicit list, or all 1 <= |S| <= max_order), an
 * adaptive sparse grid is grown by ascending level sums from the root
 * (l = 1, i = 1).  Grid nodes get nodal values of the cut function
 * g_S = f(xbar \ x_S) (Alg. 2 step 6) and of the cut-HDMR component
 * u_S = sum_{v subset S} (-1)^{|S|-|v|} f(xbar \ x_v) (eq (2.2.6)); both are
 * hierarchised on the device in FP64 (alpha = y - interpolant of the coarser
 * level sums, the defining equations of eq (3.6)).  A node is accepted when
 * max_o |alpha^g_o| > eps_gamma (eq (3.8)); the children of accepted nodes
 * (l + e_q, 2 i_q -+ 1) are admitted when every parent (refine_rule 0) or any
 * parent (refine_rule 1) is accepted (the exclusion rule of Sec. 3.1).
 * eps_gamma < 0 accepts every node, which yields the regular grid of the
 * level rule: eq (3.5) (level_rule 1: |l|_1 <= max_level + |S| - 1) or the
 * full grid of eq (3.4) (level_rule 0: every l_q <= max_level).
 * form 0 stores u_S with w_S = 1 and c0 = f(xbar); form 1 stores g_S with the
 * eq (4.2) coefficients b_S and c0 = b_empty f(xbar).
 * f is called on the host, once per level sum with every new node of every
 * component (rows are deduplicated).  The result lives on the current device.
 *
 * With eps_eta > 0 or eps_rho > 0 the build follows Alg. 2: the expansion
 * orders k = 1, 2, ... are built in turn; the candidates of order k are the
 * index sets of size k (of the explicit list, or all of them up to
 * max_order) that contain no rejected set.  With Q f_u the quadrature
 * (eq (3.7)) of the interpolant of the component function u_S (computed on
 * the device) and Q f_empty = f(xbar), D_k = ||sum of Q f_v over the kept v
 * with |v| < k||_2 (2-norm over the m outputs).  A candidate of order >= 2 is
 * kept when eta_u = ||Q f_u||_2 / D_k > eps_eta (eq (3.19)), else it joins
 * the reject set Z and no superset of it is built (eps_eta <= 0: all kept).
 * After order k, rho_k = ||sum of Q f_u over the kept order-k u||_2 / D_k
 * (eq (3.18)); order k+1 follows only if rho_k > eps_rho (eps_rho <= 0:
 * always).  The model holds the kept components (form 1: b_S over the kept
 * family); hdmr_build_report returns the candidates, eta, kept flags and rho.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t d, m;                 /* input dimension, number of outputs                     */
  int32_t max_order;            /* used when n_components == 0: all 1 <= |S| <= max_order */
  int32_t max_level;            /* L                                                      */
  int32_t level_rule;           /* 0: every l_q <= L;  1: |l|_1 <= L + |S| - 1            */
  int32_t refine_rule;          /* 0: all parents accepted;  1: any parent accepted       */
  double eps_gamma;             /* eq (3.8) threshold; < 0 = accept all                   */
  const double *anchor;         /* host, d: the anchor point xbar (eq (2.2.5))            */
  int32_t n_components;         /* 0 = all index sets up to max_order                     */
  const int32_t *comp_offsets;  /* host, n_components+1 offsets into comp_dims            */
  const int32_t *comp_dims;     /* host, the index sets, each strictly increasing         */
  int32_t form;                 /* 0: component form; 1: eq (4.2) form                    */
  double eps_eta, eps_rho;      /* eq (3.19)/(3.18) thresholds of Alg. 2 (<= 0: off)      */
} asg_build_params;

int asg_build_components(const asg_build_params *params, hdmr_fn f, void *user, hdmr_model **out);

/* Report of an adaptive build (Alg. 2).  *n_candidates and *n_orders receive
 * the counts; the arrays (host, may be NULL; query the counts first) receive
 * per candidate in build order: cand_k = |S|, cand_dims (n_candidates x 4,
 * -1 padded), eta (eq (3.19); NaN where not tested: order 1, or eps_eta <= 0),
 * kept (1/0); rho (n_orders values, eq (3.18)).  Models not built with the
 * criteria report zero candidates. */
int hdmr_build_report(const hdmr_model *model, int32_t *n_candidates, int32_t *n_orders, int32_t *cand_k,
                      int32_t *cand_dims, double *eta, uint8_t *kept, double *rho);

/* Quadrature of eq (3.7) over [0,1]^d on the device: q (host, n_components x
 * m, may be NULL) receives Q u_S = sum_j alpha_j 2^-|l_j|_1 per component (the
 * integral of a zero-boundary hat of level l is 2^-l); total (host, m, may be
 * NULL) receives c0 + sum_S w_S Q u_S, the integral of F.  Synchronous. */
int hdmr_quadrature(const hdmr_model *model, double *q, double *total);

/* Model from given grids and surpluses (host arrays, copied to the current
 * device).  Component s has index set comp_dims[comp_offsets[s] ..
 * comp_offsets[s+1]) and comp_npts[s] rows; levels/indices hold
 * sum_s comp_npts[s]*|S_s| entries (row-major per component, components
 * concatenated), surpluses hold sum_s comp_npts[s]*m values, weights[s] is
 * w_S, c0 has m values.  Levels must be >= 1, indices odd with
 * 0 < i < 2^level (eq (3.3)), rows unique within a component. */
int hdmr_model_from_surpluses(int32_t d, int32_t m, const double *c0, int32_t n_components,
                              const int32_t *comp_offsets, const int32_t *comp_dims,
                              const int64_t *comp_npts, const uint8_t *levels,
                              const uint32_t *indices, const double *surpluses,
                              const double *weights, hdmr_model **out);

/* The naive evaluation of eq (3.16) (Sec. 4.1, Sec. 5.1): a new model whose
 * evaluation sums, for every retained index set u (the components of src)
 * and every nonempty v subset u, (-1)^(|u|-|v|) times the interpolant of the
 * cut function g_v as its own term, recomputing the interpolants that several
 * u share, plus c0 = f(xbar) sum_{u in U + {empty}} (-1)^|u|.  src must hold
 * the cut-function surpluses g_v of a family closed under subsets (a form 1
 * build); its weights and c0 are not used.  f_anchor (host, m values) is
 * f(xbar).  Evaluated with hdmr_eval it gives the same values as src (the
 * eq (4.2) regrouping a(x)^T b) up to rounding, with the work of eq (3.16)
 * term by term.  A family that is not closed under subsets gives HDMR_EINVAL.
 * The new model lives on the current device and is freed with hdmr_free. */
int hdmr_model_naive(const hdmr_model *src, const double *f_anchor, hdmr_model **out);

/* F at n points: points (dev, n x d), values (dev, n x m).  m must equal the
 * model's m.  precision is HDMR_PLAIN_FP64 or HDMR_MIXED.  n = 0 is a no-op. */
int hdmr_eval(const hdmr_model *model, const double *points, int64_t n, double *values, int32_t m,
              int32_t precision, hdmr_stream_t stream);

/* hdmr_eval without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and precisions as hdmr_eval, and the
 * same kernels.  The cell-sorted path (HDMR_MIXED, or n >= 16384 points in
 * plain precision) takes its workspace from a static device array of 256 MiB
 * that the library holds on every device it runs on until the process ends;
 * it also uses a second stream and events created once per device at set-up
 * (hdmr_init, else the first call on that device).  A call whose workspace
 * would exceed 256 MiB (about n (8 d + 8 AS + 4 AS [mixed] + 90) bytes plus
 * the model's cell lists, AS = m rounded up to 16) is rejected with
 * HDMR_EINVAL before any work is enqueued.  Every call on one device shares
 * that device's array and set-up: calls that overlap on one device (other
 * streams or threads) race and must be serialised by the caller; the array
 * keeps the last call's contents, and every call initialises what it reads. */
int hdmr_eval_noalloc(const hdmr_model *model, const double *points, int64_t n, double *values, int32_t m,
                      int32_t precision, hdmr_stream_t stream);

/* F and its gradient: grad (dev, n x d x m) receives dF_o/dx_q as the right
 * partial derivative (the left one at x_q = 1; zero outside [0,1] and for
 * dimensions no component uses).  values may be NULL. */
int hdmr_eval_grad(const hdmr_model *model, const double *points, int64_t n, double *values,
                   double *grad, int32_t m, hdmr_stream_t stream);

/* Many models in one call: model i is evaluated at n[i] points
 * points[i] (dev, n[i] x d_i) into values[i] (dev, n[i] x m_i), as hdmr_eval
 * does.  Models of uneven size, dimension and output width are batched: every
 * model routed to the gather kernel runs in one persistent launch (work
 * units of a few points taken from a device queue, heaviest models first),
 * replayed from a hipGraph cached per batch signature (models, points,
 * values, n, precision); models with n >= 16384 are first timed on the call's
 * data on each candidate path (persistent gather in plain precision, and the
 * cell-sorted path with five contraction tile shapes: row batch, work-item
 * size, grid) and the fastest is kept per (model, size bucket floor(log2 n),
 * precision) -- the call that measures leaves correct values.  With
 * HDMR_MIXED every model with grid points takes the cell-sorted path (the
 * gather kernel is FP64 only).  paths (host, count entries, may be NULL)
 * receives the path used per model: -1 none (n = 0), 0 persistent gather,
 * 1 + v the cell-sorted path with tile shape v (bit 0: the smaller row batch,
 * bit 1: work items of 128 points instead of 256, bit 2: a persistent grid of
 * three workgroups per CU).  All models must live on one device (max d 1900).  The
 * caller must not free or overwrite a model while a batched call using it
 * may still run on a stream.  The cached graphs are released when their
 * models are freed. */
int hdmr_eval_batched(const hdmr_model *const *models, const double *const *points, const int64_t *n,
                      double *const *values, int32_t count, int32_t precision, int32_t *paths,
                      hdmr_stream_t stream);

/* Work counts of an evaluation (diagnostic, synchronous on stream): *hits
 * receives the number of (point, stored row) pairs with a nonzero basis
 * product -- the nonzeros of the sparse basis matrix of eq (3.6) summed over
 * components -- and *probes the number of (point, level multi-index) lookups
 * the kernels perform.  Used to price a launch in flops (2 * hits * m). */
int hdmr_eval_stats(const hdmr_model *model, const double *points, int64_t n, int64_t *hits, int64_t *probes,
                    hdmr_stream_t stream);

/* Sizes of a model (host). */
typedef struct {
  int32_t d, m, n_components, n_tuples;
  int64_t n_rows;               /* stored grid points over all components          */
  int64_t device_bytes;         /* device memory the model holds                   */
  int32_t max_level;            /* largest level in any dimension                   */
  int32_t max_k;                /* largest |S|                                      */
  int32_t n_passes;             /* passes of the cell-sorted evaluation             */
  int32_t pass_key_dims;        /* key dimensions summed over the passes            */
} hdmr_model_info;

int hdmr_get_info(const hdmr_model *model, hdmr_model_info *info);

/* Copy one component's grid back to the host, in the model's internal row
 * order: *npts rows, *k = |S|, dims (k entries, host), levels/indices
 * (npts x k, host), surpluses (npts x m, host), *weight = w_S.  Every output
 * pointer except npts may be NULL; query npts and k first, then allocate. */
int hdmr_export_component(const hdmr_model *model, int32_t comp, int64_t *npts, int32_t *k, int32_t *dims,
                          uint8_t *levels, uint32_t *indices, double *surpluses, double *weight);

/* Model files.  hdmr_model_save writes d, m, c0 and every component's
 * index set, weight, grid (levels, odd indices) and surpluses (the model's
 * internal row order) to a versioned binary file at path; hdmr_model_load
 * reads one and builds the model on the current device, validating the grids
 * as hdmr_model_from_surpluses does.  A missing, foreign, truncated or
 * corrupt file gives HDMR_EINVAL (an unknown version HDMR_EUNSUPPORTED).
 * Files use the host's byte order. */
int hdmr_model_save(const hdmr_model *model, const char *path);
int hdmr_model_load(const char *path, hdmr_model **out);

void hdmr_free(hdmr_model *model);

/* Per-kernel device timing (diagnostic; not part of the method).  While
 * enabled, the evaluation brackets each stage of every pass with device
 * events recorded on the launch stream.  The stages are:
 *   "sort"     -- keys and key coordinates, radix sort, cell bounds;
 *   "rows"     -- per-cell row discovery and the work items of the cells;
 *   "contract" -- the matrix-core contraction of the tiles.
 * hdmr_timing_enable(on): on != 0 enables timing and discards earlier
 * records; on == 0 disables it and discards them.
 * hdmr_timing_read(stage, total_ms, launches) waits for the recorded events
 * and returns the summed device time (ms) and the number of bracketed launches
 * of that stage since enabling.  Unknown stage names give HDMR_EINVAL.
 * Calls from several threads are serialised. */
int hdmr_timing_enable(int32_t on);
int hdmr_timing_read(const char *stage, double *total_ms, int64_t *launches);

/* Message of the last failure on the calling thread ("" if none). */
const char *hdmr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HDMR_H */
