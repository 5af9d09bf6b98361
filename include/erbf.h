/*
 * erbf.h -- C ABI of the MI355X ERBF-fit library.
 *
 * The library evaluates a sparse network of ellipsoidal radial basis
 * functions (ERBFs) at precomputed signed-distance grid points and returns
 * the sparse-fit loss and its gradient with respect to every kernel's
 * weight, centre, per-axis scale and orientation -- the optimisation step of
 * SE-RBFNet (Lian et al., "Approximating Signed Distance Fields With Sparse
 * Ellipsoidal Radial Basis Function Networks", arXiv 2505.02350).
 *
 * Model (paper Section 3.2, eq. 3-7 and eq. 3-26; cull of eq. 3-15-1):
 *     f(x) = sum_j a_j [ |x - c_j|^2 < r_j^2 ] exp(-| D_j R_j (x - c_j) |^2)
 *     a_j  = w_j |w_j|  (ERBF_WEIGHT_SIGNED_SQUARE)   or   w_j (ERBF_WEIGHT_LINEAR)
 *     D_j  = diag(exp(s_j)),  R_j = R(q_j / |q_j|),  r_j = cull_k / min_k exp(s_jk)
 * Orientation is a quaternion (w, x, y, z) by default (ERBF_ORIENT_QUATERNION);
 * the paper's Euler angles (eq. 3-6, read as R = Rz(tz) Ry(ty) Rx(tx) with the
 * standard right-handed axis rotations) are ERBF_ORIENT_EULER, with the
 * angles (tx, ty, tz) in the first three orientation slots and the fourth
 * unused (its gradient is 0).  Scales are optimised as logarithms s = ln d.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All pointers named *_dev or documented as "device" point to device
 *    memory of the context's device, owned by the caller.  The library never
 *    allocates device memory: every scratch buffer lives in the caller's
 *    workspace (erbf_workspace_size / erbf_ctx_create) or, for the
 *    context-free surface calls, in scratch arguments.
 *  - Calls that take a hipStream_t only enqueue work on that stream; they do
 *    not synchronise and are safe to capture into a hipGraph, except the
 *    calls documented as "synchronous" (erbf_ctx_create,
 *    erbf_refine_level, erbf_seed_from_error, erbf_init_inscribed,
 *    erbf_surface_extract, erbf_autotune).
 *  - A context holds one or more independent shapes (the batched extension);
 *    a plain fit is a context with one shape.  Kernels of all shapes share
 *    one global index space: shape b owns slots [kbase_b, kbase_b + cap_b),
 *    kbase_b = sum of the capacities of the shapes before it.
 *  - Parameters, gradients and Adam moments share the packed layout
 *        float p[11 * cap_total]:  w | cx cy cz | sx sy sz | qw qx qy qz
 *    each segment cap_total floats long; the live kernels of shape b are
 *    slots kbase_b .. kbase_b + m_b - 1, m_b = m_dev[b].  Slots past m_b are
 *    ignored and their gradients written as 0.
 *  - Grid points: every grid level of every shape is a uniform cell-centred
 *    grid of n^3 points (axis table given by the caller, x fastest:
 *    idx = (k n + j) n + i).  A sample level instead holds up to
 *    level_samples surface samples P (label 1; the training set of Section
 *    3.4.2 is V = {G, P}) in that many index slots, in the caller's order.
 *    Per-point arrays of a call (targets, f, G) are the concatenation over
 *    shapes (outer) and their declared levels (inner), n^3 or level_samples
 *    entries each.
 *  - Every call returns ERBF_OK or a negative error code; erbf_last_error()
 *    returns a thread-local message for the last failure.  No exception
 *    crosses the ABI.  Device-side conditions that cannot be returned
 *    (bucket overflow) are reported in erbf_stats.flags and never overrun a
 *    buffer.
 */
#ifndef ERBF_H
#define ERBF_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ERBF_ABI_VERSION 7
#define ERBF_MAX_LEVELS 8
#define ERBF_MAX_SHAPES 1024

enum {
  ERBF_OK = 0,
  ERBF_ERR_INVALID_ARG = -1,  /* bad pointer, size or configuration */
  ERBF_ERR_HIP = -2,          /* a HIP runtime call failed; message has the hipError_t */
  ERBF_ERR_WORKSPACE = -3,    /* workspace too small for the configuration */
  ERBF_ERR_CAPACITY = -4,     /* seeding would exceed a shape's kernel capacity */
  ERBF_ERR_UNSUPPORTED = -5,  /* valid request this build does not implement */
  ERBF_ERR_STATE = -6         /* call out of order (e.g. no level registered) */
};

/* erbf_stats.flags bits */
#define ERBF_FLAG_BUCKET_OVERFLOW 1  /* bucket list exceeded pair_cap: f, loss, grads invalid */

enum { ERBF_WEIGHT_SIGNED_SQUARE = 0, ERBF_WEIGHT_LINEAR = 1 };

/* Orientation parameterisations (Section 3.2). */
enum { ERBF_ORIENT_QUATERNION = 0, ERBF_ORIENT_EULER = 1 };

/* Loss-weight modes (Section 3.3, eq. 3-14 and eq. 3-21; Algorithm 3). */
enum {
  ERBF_MODE_FIXED = 0,    /* alpha = 1, beta = lambda                              */
  ERBF_MODE_DYNAMIC = 1,  /* eq. 3-21 when l1_active and max|E| < tau_m, else (1, 0) */
  ERBF_MODE_L2 = 2        /* alpha = 1, beta = 0                                    */
};

typedef struct erbf_ctx erbf_ctx;

/* One shape: its levels (appended by erbf_refine_level in this order) and
 * its kernel capacity.  A level is a grid level (level_samples 0) or a
 * surface-sample level (level_samples > 0: up to that many samples, binned
 * for the kernel lists into the 8^3-cell tiles of a grid of level_n cells
 * per axis; about 256 samples per occupied tile suits the kernels). */
typedef struct {
  int32_t n_levels;                  /* 1 .. ERBF_MAX_LEVELS */
  int32_t level_n[ERBF_MAX_LEVELS];  /* points (or binning cells) per axis of each level, 1 .. 2048 */
  int32_t m_cap;                     /* kernel slots of this shape, >= 1 */
  int32_t level_samples[ERBF_MAX_LEVELS]; /* 0: grid level; > 0: sample capacity, <= 2^26 */
} erbf_shape_desc;

typedef struct {
  int32_t n_shapes;               /* 1 .. ERBF_MAX_SHAPES */
  const erbf_shape_desc* shapes;  /* host array [n_shapes] */
  int64_t pair_cap;   /* capacity of the tile->kernel bucket lists (entries over all
                         shapes); exceeded => ERBF_FLAG_BUCKET_OVERFLOW */
  float cull_k;       /* cull radius factor: r = cull_k / min d (eq. 3-15 with
                         eps = exp(-cull_k^2)); > 0 */
  int32_t weight_map; /* ERBF_WEIGHT_SIGNED_SQUARE (eq. 3-26) or ERBF_WEIGHT_LINEAR */
  int32_t orientation; /* ERBF_ORIENT_QUATERNION or ERBF_ORIENT_EULER (eq. 3-6); also
                          decides the identity rotation that seeding writes */
  int32_t batch_cap;   /* largest point count of an erbf_loss_grad_minibatch call, >= 0 */
} erbf_config;

/* A level (eq. 3-16: the training set is the union of the levels
 * registered so far).  All arrays are device memory owned by the caller and
 * must stay valid for the context's lifetime.  A grid level gives axis,
 * target, sdf and active_bits; a sample level gives only samples and
 * n_samples (its targets are 1, eq. 3-10 on the surface; the other fields
 * are ignored). */
typedef struct {
  int32_t n;                    /* points per axis; must equal the declared level_n */
  const float* axis;            /* [n] increasing cell-centred coordinates in [-1, 1] */
  const float* target;          /* [n^3] normalised targets (eq. 3-10) or NULL (eval/vjp only) */
  const float* sdf;             /* [n^3] raw signed distance, or NULL; required for seeding */
  const uint32_t* active_bits;  /* [ceil(n^3/32)] training-point mask (bit i%32 of word i/32),
                                   or NULL for all points */
  const float* samples;         /* sample level: [n_samples * 3] x, y, z in [-1, 1] */
  int64_t n_samples;            /* sample level: 0 .. its declared capacity */
} erbf_level;

typedef struct {
  float* p;         /* device [11 * cap_total], packed layout above */
  int32_t* m_dev;   /* device [n_shapes]: live kernel count of each shape */
} erbf_params;

typedef struct {
  int32_t mode;            /* ERBF_MODE_* */
  float lambda;            /* fixed-mode L1 weight, used when lambda_dev is NULL */
  const float* lambda_dev; /* device [n_shapes] per-shape fixed-mode weight, or NULL */
  int32_t l1_active;       /* dynamic mode: L1 term scheduled on (eq. l1_activate) */
  float tau1, tau2;        /* id_all thresholds of eq. 3-18 (paper: 0.9, 1.1) */
  float tau_m;             /* max-error gate of eq. l1_activate2 (paper: 0.02) */
  const int32_t* l1_active_dev; /* device [n_shapes] per-shape L1 flags (the
                                   control state's l1_active), or NULL to use
                                   l1_active for every shape */
} erbf_loss_cfg;

/* Per-shape step statistics, written to device memory by erbf_loss_grad. */
typedef struct {
  double L2;          /* sum over id_all of E^2 (eq. 3-14_2) */
  double L1;          /* sum of |w| over live kernels */
  double loss;        /* alpha * L2 + beta * L1 */
  double alpha, beta; /* loss weights used for the gradient (eq. 3-21) */
  int64_t n_idall;    /* points in id_all (eq. 3-18) */
  int64_t P_fwd;      /* in-ball point-kernel pairs over active points */
  int64_t P_bwd;      /* in-ball pairs whose upstream G is non-zero */
  int64_t n_bucket_pairs; /* bucket entries needed by this call (all shapes) */
  float max_abs_E;    /* max |E| over id_all, 0 if empty */
  int32_t m;          /* live kernels */
  int32_t flags;      /* ERBF_FLAG_* */
  int32_t reserved;
  /* running totals: each call adds its P_fwd, P_bwd and 1 to the values
   * already in stats_dev (zero the buffer to reset them) */
  int64_t P_fwd_total, P_bwd_total, calls;
} erbf_stats;

typedef struct {
  float lr;            /* used when lr_dev is NULL */
  const float* lr_dev; /* device [n_shapes] per-shape learning rate, or NULL */
  float beta1, beta2, eps;  /* Adam hyper-parameters (0.9, 0.999, 1e-8) */
  /* device [1] or NULL: while the word is non-zero the call leaves the
   * parameters, the moments and the step counters as they are (the hold
   * word of erbf_sched_state) */
  const int32_t* hold_dev;
} erbf_adam_cfg;

typedef struct {
  float top_frac;      /* candidates: ceil(top_frac * n_idall) largest |E| (<= 0.05) */
  int32_t k_new;       /* kernels appended per call, 1 .. 4096 */
  float r_nms;         /* extreme-point radius; <= 0 selects twice the finest spacing */
  float eps;           /* eq. 3-24 epsilon (paper: 1e-7) */
  float min_abs_err;   /* candidates also need |E| > min_abs_err (Algorithm 2: tau_m / 2) */
  int32_t w_rule;      /* 0: w = -sign(E)|E| (eq. 3-24 literally); 1: w = -sign(E) sqrt|E| */
} erbf_seed_cfg;

/* ---- context ----------------------------------------------------------- */

int32_t erbf_abi_version(void);
const char* erbf_last_error(void);

/* Bytes of device workspace a context with this configuration needs. */
int erbf_workspace_size(const erbf_config* cfg, size_t* bytes);

/* Create a context on `device` using the caller's workspace (device memory
 * of at least erbf_workspace_size bytes, 256-byte aligned).  Synchronous.
 * Returns ERBF_ERR_WORKSPACE if `bytes` is too small. */
int erbf_ctx_create(int device, const erbf_config* cfg, void* workspace, size_t bytes,
                    erbf_ctx** out);
void erbf_ctx_destroy(erbf_ctx* ctx);

/* Total kernel slots (sum of the shapes' m_cap) and points of the active
 * levels (length of the per-point arrays of the next call). */
int erbf_ctx_info(const erbf_ctx* ctx, int32_t* cap_total, int64_t* n_points,
                  int32_t* n_active_levels_shape0);

/* ---- data preparation (eq. 3-10) --------------------------------------- */

/* out_dev[0] = min(out_dev[0], min_i S[i]) if accumulate, else min_i S[i].
 * Device result; the minimum over every level is eq. 3-10's m. */
int erbf_sdf_min(const float* S, int64_t n, float* out_dev, int accumulate, hipStream_t stream);

/* t[i] = 2 exp(-h (S[i] - m)^2), h = ln 2 / m^2 (eq. 3-10), evaluated in
 * double and rounded once.  m must be < 0. */
int erbf_targets_from_sdf(const float* S, int64_t n, float m, float* t, hipStream_t stream);

/* bits of |S| < band (a banded level's training points).  `bits` holds
 * ceil(n/32) words; trailing bits are 0. */
int erbf_band_bits(const float* S, int64_t n, float band, uint32_t* bits, hipStream_t stream);

/* The octree layer below a level (eq. 3-16 on an octree, Section 3.4.2):
 * the training points of the level with 2 n_parent points per axis that are
 * the children of subdivided cells of the level with n_parent points per
 * axis.  A parent cell (width 2/n_parent, centred on its grid point) is
 * subdivided when it is present (its bit in parent_bits; every cell when
 * parent_bits is NULL) and |S_parent| <= sqrt(3)/n_parent, its
 * half-diagonal, compared in double.  S_parent: device [n_parent^3] raw
 * signed distance, x fastest; child_bits: device [ceil((2 n_parent)^3/32)]
 * words in erbf_level.active_bits form (trailing bits 0).  n_parent in
 * 1 .. 1024. */
int erbf_octree_bits(const float* S_parent, const uint32_t* parent_bits, int32_t n_parent,
                     uint32_t* child_bits, hipStream_t stream);

/* ---- the step ------------------------------------------------------------ */

/* Append the next level of `shape` (eq. 3-16 / Algorithm 3: training starts
 * on a coarse level and finer levels are appended).  Builds the level's
 * tile occupancy in the workspace.  Synchronous. */
int erbf_refine_level(erbf_ctx* ctx, int32_t shape, const erbf_level* level, hipStream_t stream);

/* f at every point of every active level (eq. 3-9 with eq. 3-15-1), 0 at
 * points outside a level's active mask.  f_out: device [n_points]. */
int erbf_eval(erbf_ctx* ctx, const erbf_params* params, float* f_out, erbf_stats* stats_dev,
              hipStream_t stream);

/* One loss + gradient evaluation (eq. 3-9, 3-18, 3-19, 3-21 and Appendix
 * A).  grad_out: device [11 * cap_total], the combined gradient
 * alpha dL2 + beta dL1 in the packed layout.  stats_dev: device
 * [n_shapes].  f_out, G_out: optional device [n_points]; G = 2 E on id_all,
 * 0 elsewhere.  Every active level needs a target. */
int erbf_loss_grad(erbf_ctx* ctx, const erbf_params* params, const erbf_loss_cfg* cfg,
                   float* grad_out, erbf_stats* stats_dev, float* f_out, float* G_out,
                   hipStream_t stream);

/* Batched fitting (many independent shapes in one context): the loss and
 * gradient of every shape of the context, each stage one launch over all
 * shapes' tiles and kernels, with per-shape statistics and loss weights
 * (per-shape lambda through cfg->lambda_dev, per-shape L1 flags through
 * cfg->l1_active_dev).  The same call as erbf_loss_grad, which treats a
 * multi-shape context this way; results of each shape equal those of a
 * one-shape context holding that shape alone.  stats_dev: device
 * [n_shapes]. */
int erbf_loss_grad_batched(erbf_ctx* ctx, const erbf_params* params, const erbf_loss_cfg* cfg,
                           float* grad_out, erbf_stats* stats_dev, float* f_out, float* G_out,
                           hipStream_t stream);

/* One mini-batch step's loss and gradient (Algorithm 3, the inner loop over
 * batches of B_s shuffled points): as erbf_loss_grad, but f, the id_all mask,
 * E, L2, max|E| (hence the gate of eq. 3-21), the pair counts and the
 * gradient cover only the batch.  pts: device [n_pts] distinct indices into
 * the context's per-point arrays (shape-major over the declared levels, x
 * fastest), 0 <= n_pts <= batch_cap; indices outside the registered
 * levels' active points contribute nothing.  f_out: optional device
 * [n_pts], f at the batch points in batch order.  The bucket lists are
 * rebuilt from the current parameters as in erbf_loss_grad. */
int erbf_loss_grad_minibatch(erbf_ctx* ctx, const erbf_params* params, const erbf_loss_cfg* cfg,
                         const int64_t* pts, int32_t n_pts, float* grad_out, erbf_stats* stats_dev,
                         float* f_out, hipStream_t stream);

/* Vector-Jacobian product of erbf_eval: grad_out = (df/dtheta)^T grad_f,
 * grad_f: device [n_points] (entries at inactive points are ignored).
 * stats_dev optional (P_fwd, P_bwd). */
int erbf_vjp(erbf_ctx* ctx, const erbf_params* params, const float* grad_f, float* grad_out,
             erbf_stats* stats_dev, hipStream_t stream);

/* One Adam step (Kingma & Ba, bias-corrected; Algorithm 3) on the live
 * kernels of every shape.  m1, m2: device moments in the packed layout;
 * step_dev: device [n_shapes] step counters, incremented by this call. */
int erbf_adam_step(erbf_ctx* ctx, const erbf_params* params, const float* grad, float* m1,
                   float* m2, int32_t* step_dev, const erbf_adam_cfg* cfg, hipStream_t stream);

/* Append new kernels at local maxima of the residual (Algorithm 2, eq. 3-22,
 * 3-24, 3-25) to `shape`.  resid: device [n_points] residual E (or G with
 * resid_scale = 0.5), 0 outside id_all; n_idall: its id_all count.
 * Candidates are the ceil(top_frac * n_idall) grid points of largest |E|
 * (ties to the lower index) with |E| > max(min_abs_err, eps); surface
 * samples are never candidates.  A candidate is kept when no point of the
 * training set V within r_nms -- grid points of the shape's active levels
 * and its registered surface samples -- has a larger |E|; the first k_new
 * kept by the same order become kernels: centre at the point, weight
 * -sign(E)|E| (w_rule 0) or -sign(E) sqrt|E| (w_rule 1), the three scales
 * d = sqrt(ln(|E| / eps)) / dbar, identity rotation.  dbar is the distance
 * to the nearest registered surface sample of the shape (eq. 3-24), or,
 * when the shape has none, |S| at the point; in both cases at least the
 * finest grid spacing.  New kernels get zero Adam moments in m1/m2 (either
 * may be NULL).  Every active grid level of the shape needs `sdf`.
 * Synchronous; *n_added receives the number appended.  ERBF_ERR_CAPACITY
 * (nothing appended) if the shape cannot hold them. */
int erbf_seed_from_error(erbf_ctx* ctx, const erbf_params* params, int32_t shape,
                         const float* resid, float resid_scale, int64_t n_idall,
                         const erbf_seed_cfg* cfg, float* m1, float* m2, int32_t* n_added,
                         hipStream_t stream);

/* Initial kernels of `shape` from maximal inscribed spheres (Algorithm 1,
 * eq. 3-11, eq. 3-12), replacing its live kernels.  Candidates are the
 * training points of the shape's registered levels with 1 < target < 2
 * (eq. 3-10, interior points) and a finite raw SDF.  Each round takes the
 * candidate of largest |S| (its distance to the surface; ties to the lower
 * point index, levels in registration order, x fastest) as a centre c with
 * weight w = its target, and drops every candidate within distance |S| of
 * it (squared distances in double precision, each product and sum rounded
 * separately); rounds end when no candidate is left or after
 * min(max_centres, m_cap) centres (max_centres <= 0: m_cap).  Each centre
 * then gets d1 = d2 = d3 = 2 sqrt(-ln(gamma / w^2)) / dhat, dhat the distance
 * to the nearest other centre (2 for a single centre), stored as s = ln d,
 * and the identity rotation.  The shape's Adam moments in m1/m2 (either may
 * be NULL) are cleared.  Every registered level needs `target` and `sdf`;
 * gamma in (0, 1) (paper: 1e-3).  Synchronous; *n_centres receives the
 * number of kernels (also written to m_dev[shape]) and *n_left the
 * candidates no sphere covers (non-zero only when the limit stopped the
 * rounds). */
int erbf_init_inscribed(erbf_ctx* ctx, const erbf_params* params, int32_t shape, float gamma,
                        int32_t max_centres, float* m1, float* m2, int32_t* n_centres,
                        int64_t* n_left, hipStream_t stream);

/* ---- surface evaluation (Section 4, Evaluation Metric) -------------------- */

/* S[i] = m + sqrt(ln(2 / t[i]) / h), h = ln 2 / m^2: eq. 3-10 inverted on
 * its branch S >= m (t >= 2 gives m; t <= 0 gives +inf), in double, rounded
 * once.  Takes the network's normalised output back to a signed distance
 * before its zero-level surface is extracted.  m < 0. */
int erbf_sdf_from_targets(const float* t, int64_t n, float m, float* S, hipStream_t stream);

/* Device scratch bytes of erbf_surface_extract for a grid of n points per
 * axis, 2 <= n <= 1024. */
int erbf_surface_scratch_size(int32_t n, size_t* bytes);

/* The iso-surface of the grid field F (device [n^3], x fastest, on the
 * cell-centred axis, device [n]) by marching tetrahedra: each cube of eight
 * neighbouring points is split into six tetrahedra around its main diagonal;
 * a tetrahedron whose corners straddle iso (inside: F < iso) gives one or two
 * triangles with vertices interpolated linearly along its straddling edges
 * (on the finite corner when the other corner's value is infinite).
 * Triangles come out in cube order (x fastest), then tetrahedron and case
 * order: tris device [tri_cap * 9] (x, y, z of three vertices each).
 * Synchronous; *n_tris receives the count.  ERBF_ERR_CAPACITY (nothing
 * written, *n_tris the count needed) when it exceeds tri_cap. */
int erbf_surface_extract(const float* F, int32_t n, const float* axis, float iso, void* scratch,
                         size_t scratch_bytes, float* tris, int64_t tri_cap, int64_t* n_tris,
                         hipStream_t stream);

/* Points uniform by area on the triangles (the paper samples 10^5 per
 * surface): u device [n_samples * 3] uniforms in [0, 1) chosen by the
 * caller; sample s takes the first triangle whose running area sum (double,
 * a blocked scan in a fixed order) exceeds u0 times the total, and the point
 * (1 - sqrt(u1)) A + sqrt(u1) (1 - u2) B + sqrt(u1) u2 C.  area_scratch:
 * device [n_tris + ceil(n_tris / 1024)] doubles; pts, normals: device
 * [n_samples * 3] (unit triangle normals);
 * tri_index: device [n_samples] or NULL. */
int erbf_surface_sample(const float* tris, int64_t n_tris, const float* u, int64_t n_samples,
                        double* area_scratch, float* pts, float* normals, int32_t* tri_index,
                        hipStream_t stream);

/* HD, CD and CS between the point set Pt (normals Nt) of the ground-truth
 * surface and Pr (Nr) of the reconstructed one, each point's closest point
 * in the other set by Euclidean distance (ties to the lower index):
 * out[0] = HD, the largest closest distance either way; out[1] = CD, half
 * the mean closest distance each way; out[2] = CS, half the mean |n . n'|
 * each way.  scratch: device [2 (nt + nr)] doubles; out: device [3]. */
int erbf_surface_metrics(const float* Pt, const float* Nt, int64_t nt, const float* Pr, const float* Nr,
                         int64_t nr, double* scratch, double* out, hipStream_t stream);

/* erbf_surface_metrics for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same computation and result, with the per-point scratch
 * taken from a buffer built into the library (16 MiB per GPU, held until the
 * process ends) instead of a scratch argument.  nt + nr <= 2^20, else
 * ERBF_ERR_INVALID_ARG.  Allocates nothing.  Every call on one GPU shares
 * that buffer: calls that overlap on one GPU (different streams or threads)
 * race and must be serialised by the caller. */
int erbf_surface_metrics_noalloc(const float* Pt, const float* Nt, int64_t nt, const float* Pr,
                                 const float* Nr, int64_t nr, double* out, hipStream_t stream);

/* ---- training control (Algorithm 3) -------------------------------------- */

/* Constants of Algorithm 3 (paper values in parentheses). */
typedef struct {
  int32_t k_l2;      /* window of eq. l1_activate, 1 .. 32 (10) */
  float tau_l2;      /* threshold on the standard deviation of L2 over the window (0.5) */
  int32_t k_l1;      /* window of eq. add_activate, 1 .. 64 (50) */
  float tau_l1;      /* threshold on max - min of the effective basis count (5) */
  float tau_d;       /* eq. 3-27 / b_f threshold on |w| (0.01) */
  int32_t T_e, M_e;  /* the final L2 phase runs from epoch T_e to M_e (1600, 2000); T_e < M_e */
  float lr0;         /* learning rate before the final phase (0.01) */
  float lr_final;    /* learning rate at T_e, annealed by cosine (1e-3) ... */
  float lr_min;      /* ... down to lr_min at M_e (1e-5) */
  int32_t refine_epochs[4]; /* epochs after which the next grid level is requested,
                               0 = unused (400, 800) */
} erbf_sched_cfg;

/* Per-shape control state: caller-owned device arrays.  The scalar fields
 * hold n_shapes entries, l2_ring n_shapes * k_l2 and bf_ring n_shapes * k_l1.
 * After erbf_sched_step for epoch e: epoch = e; l1_active feeds the next
 * erbf_loss_cfg.l1_active_dev; lr feeds the next erbf_adam_cfg.lr_dev;
 * add_request asks the caller to add kernels (erbf_seed_from_error,
 * Algorithm 2); refine_request asks for the next grid level
 * (erbf_refine_level); b_f is the effective basis count and n_pruned the
 * kernels removed by eq. 3-27 in this call.
 *
 * hold (device [1], or NULL for none) lets a caller enqueue the next step
 * before it has read this call's requests: a call that leaves a request to
 * act on -- add_request for a shape with fewer live kernels than its m_cap
 * (after this call's pruning) and a non-empty id_all in stats_dev, or
 * refine_request -- sets the word to 1, and a call that finds it non-zero
 * changes no field (n_pruned aside, which it sets to 0).  Passed as
 * the next step's erbf_adam_cfg.hold_dev, the word makes that step leave the
 * parameters, moments and step counters unchanged too, so the caller can
 * handle the requests, clear the word (to 0) and repeat the step, on exactly
 * the trajectory of a caller that waits for every call. */
typedef struct {
  int32_t* epoch;
  int32_t* l1_active;
  int32_t* final_phase;
  int32_t* add_request;
  int32_t* refine_request;
  int32_t* b_f;
  int32_t* n_pruned;
  float* lr;
  double* l2_ring;
  int32_t* bf_ring;
  int32_t* hold;
} erbf_sched_state;

/* Reset the control state (epoch 0, L1 off, lr = lr0).  INVALID_ARG for a
 * bad configuration or a NULL array. */
int erbf_sched_init(erbf_ctx* ctx, const erbf_sched_cfg* cfg, const erbf_sched_state* state,
                    hipStream_t stream);

/* Algorithm 3's control after one step (erbf_loss_grad, then erbf_adam_step)
 * of every shape, on the device and in its order: record L2 (from
 * stats_dev, written by the step's erbf_loss_grad) and the effective basis
 * count b_f = #{|w| >= tau_d} after the update; outside the final phase,
 * prune by eq. 3-27 when epoch % k_l2 == 0, L1 is on and epoch < T_e
 * (kernels with |w| < tau_d leave; the others, their Adam moments m1/m2
 * (optional) and their order are kept, m_dev shrinks); turn L1 on when the
 * population standard deviation of the last k_l2 L2 values is below tau_l2
 * (eq. l1_activate); request new kernels and turn L1 off when L1 is on and
 * the last k_l1 counts vary by less than tau_l1 (eq. add_activate); at
 * epoch T_e enter the final phase (L1 off, no pruning or adding, cosine
 * learning rate).  No host synchronisation; capturable. */
int erbf_sched_step(erbf_ctx* ctx, const erbf_params* params, const erbf_sched_cfg* cfg,
                    const erbf_sched_state* state, const erbf_stats* stats_dev, float* m1, float* m2,
                    hipStream_t stream);

/* One optimisation step (Algorithm 3's inner step): erbf_loss_grad followed
 * by erbf_adam_step on its gradient, with the same arguments and results
 * (grad_out receives the combined gradient alpha dL2 + beta dL1, step_dev is
 * incremented, stats_dev, f_out and G_out as for erbf_loss_grad), in fewer
 * launches: the combination of eq. 3-21 is applied inside the Adam pass. */
int erbf_train_step(erbf_ctx* ctx, const erbf_params* params, const erbf_loss_cfg* cfg,
                    const erbf_adam_cfg* adam, float* grad_out, float* m1, float* m2, int32_t* step_dev,
                    erbf_stats* stats_dev, float* f_out, float* G_out, hipStream_t stream);

/* ---- measurement --------------------------------------------------------- */

/* Time the hot kernels of the next `max_calls` erbf_loss_grad / erbf_vjp
 * calls (0 disables): the forward kernel and the two backward kernels are
 * launched with start/stop events taken at the kernels' own start and end
 * (hipExtLaunchKernel), on the call's stream.  Not for use while a stream
 * is being captured. */
int erbf_timing_enable(erbf_ctx* ctx, int32_t max_calls);

/* Synchronise on the recorded events; ms[0..2] receive the summed times
 * (milliseconds) of the forward, backward-tile and backward-reduce kernels
 * and *n_calls the number of calls recorded.  Clears the records.  A kernel
 * launched right after another timed kernel (nothing in between) is timed
 * from that kernel's stop event, so its interval includes the gap between
 * the two launches. */
int erbf_timing_read(erbf_ctx* ctx, double* ms, int32_t* n_calls);

/* ---- launch variants and the autotuner ------------------------------------ */

/* Launch variants of the per-tile kernels (bit flags; results do not depend
 * on the variant, only the time does):
 *   1  forward tiles (with 4: forward + backward tiles) walked round-robin by
 *      a persistent grid
 *   2  backward tiles walked round-robin by a persistent grid (without 4)
 *   4  the loss call takes each tile through the forward, the loss and the
 *      backward moments in one kernel, instead of a forward kernel and a
 *      backward kernel
 * 0 (the default) launches one workgroup per tile for both kernels. */
#define ERBF_VARIANT_FWD_PERSISTENT 1
#define ERBF_VARIANT_BWD_PERSISTENT 2
#define ERBF_VARIANT_FUSED 4
#define ERBF_N_VARIANTS 8

int erbf_set_variant(erbf_ctx* ctx, int32_t variant);
int erbf_get_variant(const erbf_ctx* ctx, int32_t* variant);

/* The launch choices of a context (results do not depend on them, except
 * that samp_split regroups the sums of f at surface samples, within float32
 * rounding; every other choice gives bit-identical results):
 *   variant      ERBF_VARIANT_* bits above (default 0)
 *   slot_chunk   0: workgroup b of a one-workgroup-per-tile launch takes
 *                active tile b; C in 1 .. 256: runs of C consecutive tiles
 *                are dealt to the GPU's eight XCDs round-robin (neighbouring
 *                tiles share kernel records in one XCD's L2) (default 8)
 *   samp_split   workgroups per active surface-sample tile, 1 .. 32 (default 16)
 *   bucket_rank  how the tile -> kernel lists are ordered (ascending kernel
 *                slot either way): 0 (default) runs a stable radix sort of the
 *                kernel-major entries; 1 places each entry in its tile with an
 *                atomic counter and then ranks it within the tile from a bitmap
 *                of the tile's kernels (shape capacities <= 32768)
 *   fwd_chunk    kernel records a forward tile workgroup stages in LDS at a
 *                time: 64, 128 or 256 (default 256; the fused variant always
 *                uses 256)
 *   bwd_waves    waves of a backward tile workgroup, each taking its own
 *                groups of 64 kernels of the tile's list: 2, 4 or 8 (default
 *                4; the fused variant always uses 4)
 *   tile_order   1 (default): the tile kernels take the active tiles longest
 *                list first (64 classes of list length, 16 entries wide; a
 *                one-workgroup pass orders them after every list build, and
 *                slot_chunk deals runs of that order to the XCDs), so that
 *                the long tiles do not finish last; 0: in slot order */
typedef struct {
  int32_t variant;
  int32_t slot_chunk;
  int32_t samp_split;
  int32_t bucket_rank;
  int32_t fwd_chunk;
  int32_t bwd_waves;
  int32_t tile_order;
} erbf_launch_cfg;

/* ERBF_ERR_UNSUPPORTED for bucket_rank 1 with a shape capacity above 32768. */
int erbf_set_launch(erbf_ctx* ctx, const erbf_launch_cfg* cfg);
int erbf_get_launch(const erbf_ctx* ctx, erbf_launch_cfg* cfg);

/* Tune the context's launch choices for erbf_loss_grad by timing it (one
 * warm-up and `reps` timed calls per candidate, HIP events on `stream`), one
 * choice after the other: the variant (every ERBF_N_VARIANTS entry), then
 * slot_chunk (0, 2, 8, 32), tile_order (0, 1), bwd_waves (2, 4, 8) and
 * fwd_chunk (64, 128, 256) (both unless the fused variant won), samp_split
 * (8, 16, 32; only when a
 * surface sample level is registered) and
 * bucket_rank (when the shapes allow the ranked lists), each with the best
 * of the choices before it.  The choice is kept per context, so contexts
 * holding shapes of different size classes are tuned apart.
 * The fastest set stays in the context (erbf_get_launch); *chosen receives
 * its variant and times_ms (optional) the mean time of each variant
 * [ERBF_N_VARIANTS] (a negative entry for a variant that is the same launch
 * as a lower one and is not timed).  grad_scratch: device [11 * cap_total].
 * The parameters are read, not modified.  Synchronous. */
int erbf_autotune(erbf_ctx* ctx, const erbf_params* params, const erbf_loss_cfg* cfg, float* grad_scratch,
                  int32_t reps, int32_t* chosen, float* times_ms, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* ERBF_H */
