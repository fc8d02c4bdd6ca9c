/*
 * neupig.h -- C ABI of the MI355X (gfx950) Neu-PiG optimization-step library.
 *
 * The library runs one full optimization step of Neu-PiG (Kaltheuner et al.,
 * "Neu-PiG: Neural Preconditioned Grids for Fast Dynamic Surface
 * Reconstruction on Long Sequences", arXiv 2602.22212) over all frames at
 * once, on one GPU:
 *   encode   multi-resolution latent-grid lookup at the reference vertices
 *            (Sec. 3.2, level-averaged position grid + normal-direction grid)
 *   decode   time-modulated MLP to a per-frame 6-DoF deformation, applied to
 *            every vertex (Sec. 3.3, 3.4; exponential-map rotation head of the
 *            supplementary rotation study, Table 11)
 *   chamfer  bidirectional nearest-neighbour Chamfer distance per frame and
 *            the confidence-weighted deformation loss (Sec. 3.5)
 *   backward hand-written gradients of all of the above
 *   precond  Sobolev preconditioning (I + lambda L)^-2 of the grid gradients
 *            (Sec. 3.5, "Preconditioning")
 *   adam     Adam update (Sec. 3.5, "Implementation Details")
 *
 * Problem statement (Sec. 3): a reference mesh (vertex positions and vertex
 * normals at a key frame) and T unstructured point clouds go in; per-frame
 * deformed vertices come out.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every pointer named *_dev is device memory on the plan's GPU; the caller
 *    owns it and must keep it alive until the work enqueued on the plan's
 *    stream has finished. Pointers named *_host are host memory.
 *  - Calls enqueue work on the stream given at plan creation and return
 *    without waiting, unless documented as synchronizing.
 *  - Floating-point inputs and outputs are float32 unless stated; per-frame
 *    loss values are float64. Indices are int32 (V, N_t < 2^31), frame
 *    offsets int64.
 *  - A non-OK status leaves outputs untouched when the failure is found by
 *    host-side validation (done before any launch). npg_last_error() returns
 *    a message for the calling thread's last failure.
 *  - Frames are 0-based: t = 0..T-1.
 *
 * Flat parameter vector (float32, length npg_param_count):
 *   [ G_p level 0 | ... | G_p level L-1 | G_n | W_1 b_1 | ... | W_H+1 b_H+1 ]
 *   level l:  R_l^3 nodes x F_p features, node (ix,iy,iz) at row
 *             (iz*R_l + iy)*R_l + ix, features innermost; the grid spans
 *             [-1,1]^3 with corner nodes on +-1; ix follows the first
 *             coordinate.
 *   G_n:      R_n^3 x F_n, same node order, looked up at the unit normal.
 *   W_k:      [out][in] row-major, then b_k [out]. Layer 1 maps the decoder
 *             input y = (z_n, z_p, gamma(t)) (Sec. 3.3, in this order) of
 *             width F_n + F_p + (2M or 1) to the hidden width; H hidden
 *             layers; the last layer maps to 6 outputs (omega, d) with the
 *             exp-map head or 7 (q, d) with the quaternion head.
 * The same layout is used for gradients and the two Adam moment vectors.
 */
#ifndef NEUPIG_H
#define NEUPIG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NPG_MAX_LEVELS 16

typedef enum {
  NPG_OK = 0,
  NPG_EINVAL = 1,      /* invalid argument (null pointer, bad size, non-finite input) */
  NPG_ENOMEM = 2,      /* device allocation failed */
  NPG_EHIP = 3,        /* a HIP runtime call failed */
  NPG_ENOTCONV = 4,    /* warning: a preconditioner solve hit cg_maxit */
  NPG_ENONFINITE = 5   /* a non-finite value was produced during a step */
} npg_status;

enum { NPG_ACT_RELU = 0, NPG_ACT_LEAKY = 1 };
enum { NPG_PRECOND_CG = 0, NPG_PRECOND_DCT = 1 };
/* Rotation head (Sec. 3.4): the exponential map of the supplementary rotation
 * study (6 network outputs: omega, d) or the unit quaternion
 * (1 + q_w, q_x, q_y, q_z)/norm of the main text (7 outputs: q, d). */
enum { NPG_ROT_EXPMAP = 0, NPG_ROT_QUAT = 1 };
/* Arithmetic of the decoder MLP: float32 throughout, or the mixed form with
 * every MLP matrix operand (decoder input incl. the gathered grid features,
 * weights, hidden activations, back-propagated gradients) rounded to
 * bfloat16 on the matrix cores with float32 accumulation; biases, the
 * transform, the loss, the preconditioner and the float32 master parameters
 * and Adam state are unchanged. */
enum { NPG_PREC_FP32 = 0, NPG_PREC_BF16 = 1 };
/* Nearest-neighbour search of the Chamfer distance (Sec. 3.5): both give the
 * same indices and distances bit for bit. PRUNED (the default) visits the
 * points of a frame in Morton-ordered tiles and skips a tile whose bounding
 * box is provably farther than every current minimum of a wave of queries;
 * EXHAUSTIVE evaluates every vertex-point pair in one pass for both
 * directions. A plan with more than 131072 vertices, or a frame with more
 * than 131072 points, takes the exhaustive search under either setting. */
enum { NPG_NN_PRUNED = 0, NPG_NN_EXHAUSTIVE = 1 };

/* Hyper-parameters. Every reading the paper leaves open is a field here. */
typedef struct npg_config {
  int32_t n_levels;               /* L, position-grid levels, 1..16 (Sec. 3.2)     */
  int32_t res[NPG_MAX_LEVELS];    /* nodes per axis of each level, >= 2            */
  int32_t feat_p;                 /* F_p, features per position-grid node, 1..4    */
  int32_t res_n;                  /* R_n, normal grid nodes per axis (paper: 4)    */
  int32_t feat_n;                 /* F_n, normal grid features (paper: 2), 1..4    */
  int32_t time_freqs;             /* M Fourier frequencies (Sec. 3.3; paper: 4);   */
                                  /* 0 selects the scalar code t/(T-1)             */
  int32_t mlp_hidden;             /* H hidden layers, 1..3                          */
  int32_t mlp_width;              /* hidden width: 32, 64 or 128                    */
  int32_t act;                    /* NPG_ACT_RELU or NPG_ACT_LEAKY                  */
  float leaky_slope;              /* negative slope of LeakyReLU, in (0, 1] (0.01)  */
  float alpha_t;                  /* displacement squashing tanh(alpha d), 0.1      */
  float lr_mlp;                   /* Adam learning rate of the MLP (1e-3)           */
  float lr_grid[NPG_MAX_LEVELS];  /* per-level grid learning rates                  */
  float lr_n;                     /* normal-grid learning rate                      */
  float lam[NPG_MAX_LEVELS];      /* per-level smoothness lambda of (I+lambda L)^-2 */
  float lam_n;                    /* normal-grid smoothness lambda                  */
  float beta1, beta2, eps;        /* Adam constants (0.9, 0.999, 1e-8)              */
  int32_t conf_weight;            /* 1: confidence weight of Sec. 3.5, 0: w = 1     */
  int32_t t_key;                  /* key frame, 0-based; -1 selects (T-1)/2         */
  double cg_rtol;                 /* relative residual stop of each CG solve        */
  int32_t cg_maxit;               /* iteration cap of each CG solve                 */
  int32_t precond;                /* NPG_PRECOND_CG (iterative) or _DCT (exact)     */
  int32_t rot_head;               /* NPG_ROT_EXPMAP or NPG_ROT_QUAT                 */
  float w_iso;                    /* isometry-loss weight of Sec. 3.5 (paper: 100); */
                                  /* 0 disables the term, > 0 needs the mesh edges  */
  int32_t precision;              /* NPG_PREC_FP32 or NPG_PREC_BF16                 */
  int32_t cg_mg;                  /* CG form: 1 preconditions every solve with a     */
                                  /* multigrid V-cycle, 0 runs plain CG             */
  int32_t nn_search;              /* NPG_NN_PRUNED (default) or NPG_NN_EXHAUSTIVE   */
  int32_t cg_one_stream;          /* CG form: 0 (default) iterates the grids before */
                                  /* the largest on a second stream beside it when  */
                                  /* the largest is a z-column-tiled grid; 1 keeps  */
                                  /* every launch on the plan's stream (the same    */
                                  /* launches, one group after the other); the      */
                                  /* results are the same bit for bit               */
} npg_config;

typedef struct npg_plan npg_plan;

typedef struct npg_batch npg_batch;

/* Message describing the calling thread's last non-OK status. */
const char* npg_last_error(void);

/* Number of floats in the flat parameter vector of a config (host only). */
npg_status npg_param_count(const npg_config* cfg, int64_t* count_host);

/*
 * Create a plan for one sequence (Sec. 3 problem statement).
 *   ref_xyz_dev  [V][3]  reference-mesh vertex positions, inside [-1,1]^3
 *                        (coordinates outside are clamped by the grid lookup)
 *   ref_nrm_dev  [V][3]  unit vertex normals
 *   pts_dev      [sum N_t][3] all frames' points, frame after frame
 *   frame_off_host [T+1] int64 offsets of each frame into pts, off[0] = 0,
 *                        strictly increasing (every frame has >= 1 point)
 *   stream       hipStream_t (as void*) all work of this plan is ordered on:
 *                        enqueued on it, except that the CG solves run the
 *                        grids before the largest on a second stream of the
 *                        plan's own (cg_one_stream = 0), forked from this one
 *                        by an event and joined back into it before the solve
 *                        returns, so this stream still orders every result
 * Copies the inputs (they may be freed after return), validates them (finite
 * values, sizes), builds the static interpolation and scatter tables, and
 * allocates all workspace. Parameters start at zero and Adam at step 0.
 * Synchronizes the stream. Errors: NPG_EINVAL, NPG_ENOMEM, NPG_EHIP.
 */
npg_status npg_plan_create(const npg_config* cfg, int64_t V, const float* ref_xyz_dev,
                           const float* ref_nrm_dev, int32_t T, const float* pts_dev,
                           const int64_t* frame_off_host, void* stream, npg_plan** out);

/* Free every allocation of the plan. Synchronizes the stream. */
npg_status npg_plan_destroy(npg_plan* plan);

/*
 * Load the optimizer state: params [P], Adam first/second moments m, v [P]
 * (either may be NULL: zero) and the count of Adam steps already taken.
 * Synchronizes.
 */
npg_status npg_set_state(npg_plan* plan, const float* params_dev, const float* m_dev,
                         const float* v_dev, int64_t adam_steps);

/* Copy the optimizer state out (any pointer may be NULL). Synchronizes. */
npg_status npg_get_state(npg_plan* plan, float* params_dev, float* m_dev, float* v_dev,
                         int64_t* adam_steps_host);

/*
 * Parameters by block (Sec. 3.2 grids and the Sec. 3.3 network), one device
 * buffer each, in this order: the L position grids [R_l^3][F_p] (node
 * (z, y, x) at (z*R + y)*R + x), the normal grid [R_n^3][F_n], then for the
 * network's H + 1 layers W_k [out][in] and b_k [out] (first layer
 * in = F_n + F_p + 2M, or 1 without time frequencies; hidden out = W; last
 * out = 6, or 7 with the quaternion head). bufs_host holds
 * L + 1 + 2(H + 1) pointers owned by the caller. Import replaces the plan's
 * parameters (Adam moments and step count untouched); export copies them
 * out. Synchronize. NPG_EINVAL for a NULL array or buffer.
 */
npg_status npg_params_import(npg_plan* plan, const float* const* bufs_host);
npg_status npg_params_export(npg_plan* plan, float* const* bufs_host);

/* Checkpoint of the whole optimizer state (flat parameters, Adam moments,
 * step count): the same as npg_set_state / npg_get_state. */
npg_status npg_state_import(npg_plan* plan, const float* params_dev, const float* m_dev,
                            const float* v_dev, int64_t adam_steps);
npg_status npg_state_export(npg_plan* plan, float* params_dev, float* m_dev, float* v_dev,
                            int64_t* adam_steps_host);

/*
 * One full optimization step on the plan's own state (all stages below in
 * order, then the Adam update with step count adam_steps + 1).
 *   epoch, n_epochs  0-based epoch e and e_max of the confidence catch-up
 *                    delta = 1 - sqrt(e / e_max) (Sec. 3.5)
 *   loss_dev   [1] float64 (may be NULL): L_def + w_iso L_iso of this step's
 *              forward pass
 *   cd_dev     [T] float64 (may be NULL): per-frame Chamfer distances
 * Returns NPG_ENOTCONV (after completing the step) if a CG solve hit its cap.
 * In the FP32 form the step's decoder forward keeps the hidden activations
 * of layers 2..H for its backward (a plan buffer of T V (H-1) W floats,
 * allocated at plan creation when it takes at most 8 GiB and the device has
 * the memory; other plans recompute them): the same results, bitwise.
 * With the CG preconditioner the call synchronizes between batches of
 * iterations to test convergence (the first batch as long as the previous
 * call's same solve, at most 128, and 16 after a solve that reached the cap;
 * then 2 at a time).
 */
npg_status npg_step(npg_plan* plan, int32_t epoch, int32_t n_epochs, double* loss_dev,
                    double* cd_dev);

/*
 * The same step as npg_step, replayed as one HIP graph: the first call
 * records every stage's launches into a graph (on a stream of the plan's
 * own; nothing runs while recording) and each call replays it on the plan's
 * stream after a one-thread kernel has written the step's scalars (the
 * confidence exponent of `epoch`, the Adam bias corrections) to device
 * memory. Results are bitwise those of npg_step, for both preconditioners.
 * The CG form records a fixed number of iterations per solve (what the same
 * solve took last time plus 2; 16 before any solve) and a device-side test of
 * the convergence flags after each solve: a solve that has not converged
 * within them leaves the optimizer state untouched (Adam is skipped on the
 * device), and the call records twice the iterations (at most cg_maxit) and
 * runs the step again; iterations recorded past convergence change nothing.
 * The recording is renewed when the counts leave more than 6 idle iterations.
 * Returns NPG_ENOTCONV (after completing the step) if a solve recorded with
 * cg_maxit iterations did not converge. npg_tune_nn and npg_plan_set_edges
 * drop the recorded graph (the next call records it again). Synchronizes at
 * the end, like npg_step; per-stage times (npg_stage_times) and CG iteration
 * profiling (npg_profile) are not recorded.
 */
npg_status npg_step_graph(npg_plan* plan, int32_t epoch, int32_t n_epochs, double* loss_dev,
                          double* cd_dev);

/*
 * Mesh edges of the reference surface for the isometry loss (Sec. 3.5):
 * edges_host [n_edges][2] int32 vertex pairs (host memory, read during the
 * call; 1 <= n_edges < 2^30, endpoints in [0, V), i != j; a repeated edge
 * counts twice). Replaces earlier edges. Synchronizes. NPG_EINVAL on a bad
 * edge, leaving the previous edges in place.
 */
npg_status npg_plan_set_edges(npg_plan* plan, int64_t n_edges, const int32_t* edges_host);

/* Deformed vertices of every frame with the plan's parameters, [T][V][3]. */
npg_status npg_deform(npg_plan* plan, float* xhat_dev);

/*
 * Inference export (Sec. 3.4 applied with the plan's parameters): deformed
 * vertices xhat_dev [T][V][4] and, if nhat_dev is not NULL, deformed unit
 * normals nhat_dev [T][V][4] (reference normal turned by the vertex's
 * predicted rotation); the 4th component is 0.
 */
npg_status npg_predict(npg_plan* plan, float* xhat_dev, float* nhat_dev);

/*
 * Sec. 4 "Evaluation Metrics" against ground truth. The paper names CD, NC,
 * F-score and correspondence error only; per frame t these readings are
 * computed, with nearest neighbours a (prediction -> truth) and b (truth ->
 * prediction) between the predicted vertices x^_t and the true vertices g_t:
 *   out[t][0] CD   = mean_i |x^_i - g_a(i)|^2 + mean_j |g_j - x^_b(j)|^2
 *   out[t][1] NC   = (mean_i |n^_i . m_a(i)| + mean_j |m_j . n^_b(j)|) / 2
 *   out[t][2] F    = 2PR/(P+R); P, R: shares of squared NN distances < tau^2
 *                    in each direction (0 when P + R = 0)
 *   out[t][3] Corr = mean_i |x^_i - g_i| (vertex i against its own truth)
 * xhat_dev, nhat_dev: predicted vertices/normals [T][V][4] (npg_predict);
 * gt_dev, gtn_dev: true vertices and unit normals [T][V][4] (4th component
 * ignored), same vertex order; tau > 0 (the paper's F-0.5% is 0.5% of the
 * object's scale, chosen by the caller); out_dev [T][4] float64.
 * Allocates temporary device memory (about T * V * 8 * ceil(V / 2048) bytes)
 * and synchronizes.
 */
npg_status npg_metrics(npg_plan* plan, const float* xhat_dev, const float* nhat_dev, const float* gt_dev,
                       const float* gtn_dev, float tau, double* out_dev);

/*
 * npg_metrics for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * arguments, layouts and results (bitwise), with the workspace taken from a
 * fixed array of the library (64 MiB per GPU, created when the library is
 * loaded on that GPU and held until the process ends) instead of temporary
 * allocations. Frames are processed in chunks that fit the array. Enqueues on
 * the plan's stream and returns without synchronizing; calls no allocating
 * routine. Every call on one GPU uses that GPU's one array: calls that can
 * overlap in time on one GPU (other streams, other host threads) race;
 * calls enqueued on one stream are ordered. NPG_EINVAL (nothing enqueued) if
 * one frame's workspace, about V * (20 + 8 * ceil(V / (16 * nn_threads)))
 * bytes with the plan's nearest-neighbour work-group size, exceeds 64 MiB.
 */
npg_status npg_metrics_noalloc(npg_plan* plan, const float* xhat_dev, const float* nhat_dev, const float* gt_dev,
                               const float* gtn_dev, float tau, double* out_dev);

/*
 * Batched sequences (survey config 5: many independent sequences at once).
 * n_seq sequences, each described exactly as for npg_plan_create by the
 * k-th entry of every array (its own config, so its own grids and MLP; host
 * arrays of device pointers for xyz/nrm/pts, host frame offsets). The batch
 * owns one plan and one default-priority HIP stream per sequence; reach a
 * sequence's plan (state import/export, npg_deform, stages) through
 * npg_batch_plan. NPG_EINVAL names the first invalid sequence; nothing is
 * left allocated on failure. Synchronizes.
 */
npg_status npg_plan_create_batched(const npg_config* cfg, int32_t n_seq, const int64_t* V, const float* const* xyz_dev,
                                   const float* const* nrm_dev, const int32_t* T, const float* const* pts_dev,
                                   const int64_t* const* frame_off_host, npg_batch** out);

/* The plan of sequence k (owned by the batch; do not destroy it). */
npg_status npg_batch_plan(npg_batch* batch, int32_t k, npg_plan** out);

/*
 * One optimization step of every sequence (npg_step on each plan), the
 * sequences running concurrently from host worker threads on their own
 * streams. loss_dev: NULL or n_seq float64 device pointers (each may be
 * NULL). Returns the most severe status over the sequences (EHIP/EINVAL >
 * ENONFINITE > ENOTCONV > OK) with the sequence index in npg_last_error();
 * every sequence has completed its step when the call returns.
 */
npg_status npg_batch_step(npg_batch* batch, int32_t epoch, int32_t n_epochs, double* const* loss_dev);

/*
 * The same batch step with every sequence's step replayed from recorded HIP
 * graphs (each plan's npg_step_graph recording, made on first use and again
 * when that recording changes). Mode NPG_BATCH_ONE_GRAPH (default): one batch
 * graph holds the recordings as independent branches (child graphs) and is
 * launched on a stream of the batch's own after the work already enqueued on
 * the sequences' streams. Mode NPG_BATCH_GRAPH_PER_STREAM: each recording is
 * launched on its sequence's own stream, all before the first wait. A
 * sequence whose recorded CG solve stops short runs its step again alone, as
 * npg_step_graph does. Results are bitwise those of npg_batch_step (either
 * mode); status and loss_dev as there. Synchronizes.
 */
enum { NPG_BATCH_ONE_GRAPH = 0, NPG_BATCH_GRAPH_PER_STREAM = 1 };
npg_status npg_batch_step_graph(npg_batch* batch, int32_t epoch, int32_t n_epochs, double* const* loss_dev);
npg_status npg_batch_graph_mode(npg_batch* batch, int32_t mode);

npg_status npg_batch_destroy(npg_batch* batch);

/* ---- stage entry points (stateless with respect to parameters) ---------- */

/* Sec. 3.2. z_dev [V][F_n+F_p] = (z_n(n_i), (1/L) sum_l z_p^l(x_i)). */
npg_status npg_encode_fwd(npg_plan* plan, const float* params_dev, float* z_dev);

/*
 * Sec. 3.3-3.4. For every frame t and vertex i: y = (z_i, gamma(t)),
 * o = MLP(y), x^ = Exp(o[0:3]) x_i + tanh(alpha o[3:6]).
 *   xhat_dev [T][V][4] (fourth component written as 0).
 */
npg_status npg_decode_fwd(npg_plan* plan, const float* params_dev, const float* z_dev,
                          float* xhat_dev);

/*
 * Sec. 3.5. Per frame: a_i = argmin_j |x^_i - p_j|^2 and b_j = argmin_i, with
 * the lowest index on exact ties (distances in float32, direct form
 * (x-p).(x-p) with a fixed operation order; the config's nn_search picks the
 * pruned or the exhaustive search, with identical results), and
 * cd_t = mean_i da_i + mean_j db_j summed in float64.
 *   a_dev [T][V] int32 (index within frame t), da_dev [T][V] float32,
 *   b_dev [sum N_t] int32 (vertex index), db_dev [sum N_t] float32,
 *   cd_dev [T] float64.
 */
npg_status npg_chamfer_fwd(npg_plan* plan, const float* xhat_dev, int32_t* a_dev,
                           float* da_dev, int32_t* b_dev, float* db_dev, double* cd_dev);

/*
 * Sec. 3.5. Confidence weights w_t (product of omega(tau)^delta between the
 * key frame and t) and L_def = (1/T) sum_t w_t cd_t, all float64 on device.
 *   w_dev [T], loss_dev [1].
 */
npg_status npg_loss(npg_plan* plan, const double* cd_dev, int32_t epoch, int32_t n_epochs,
                    double* w_dev, double* loss_dev);

/*
 * Gradient of L_def w.r.t. x^ with assignments and weights held fixed:
 * gx_i,t = (w_t/T)[(2/V)(x^_i - p_a_i) + (2/N_t) sum_{j: b_j = i}(x^_i - p_j)].
 *   gxhat_dev [T][V][4] (fourth component 0).
 */
npg_status npg_chamfer_bwd(npg_plan* plan, const float* xhat_dev, const int32_t* a_dev,
                           const int32_t* b_dev, const double* w_dev, float* gxhat_dev);

/*
 * Sec. 3.5 objective on deformed vertices xhat_dev [T][V][4]: the Chamfer
 * outputs of npg_chamfer_fwd (a_dev, da_dev, b_dev, db_dev, cd_dev), the
 * confidence weights of npg_loss (w_dev [T]) and
 *   loss_dev [1] = L_def + w_iso L_iso
 * (the isometry term with the plan's w_iso and mesh edges, only when
 * w_iso > 0; iso_dev [1] (may be NULL) then receives L_iso). Everything in
 * float64 on the device. NPG_EINVAL when w_iso > 0 and no edges are set.
 */
npg_status npg_objective_fwd(npg_plan* plan, const float* xhat_dev, int32_t epoch, int32_t n_epochs,
                             int32_t* a_dev, float* da_dev, int32_t* b_dev, float* db_dev, double* cd_dev,
                             double* w_dev, double* iso_dev, double* loss_dev);

/*
 * Gradient of that objective w.r.t. x^ with the assignments a, b and the
 * weights w of npg_objective_fwd held fixed (the weights and the key-frame
 * edge lengths are stop-gradients of Sec. 3.5), times an upstream factor g:
 *   gxhat_dev [T][V][4] = g (dL_def/dx^ + w_iso dL_iso/dx^)
 * g_dev: one float64 on the device (a reverse-mode caller's upstream
 * gradient), or NULL for g = 1 (then bitwise the gradient npg_step forms).
 * The factor multiplies the float64 frame weights and the isometry term's
 * float64 scale before any float32 rounding.
 */
npg_status npg_objective_bwd(npg_plan* plan, const float* xhat_dev, const int32_t* a_dev, const int32_t* b_dev,
                             const double* w_dev, const double* g_dev, float* gxhat_dev);

/*
 * Backward of decode: recomputes the MLP forward per tile (this entry point
 * never reads stored activations), back-propagates gxhat through the
 * transform and the MLP.
 *   grad_dev [P]: the MLP block of the flat gradient is overwritten (grid
 *                 blocks untouched); gz_dev [V][F_n+F_p] = sum over frames of
 *                 the decoder-input gradient's z part.
 */
npg_status npg_decode_bwd(npg_plan* plan, const float* params_dev, const float* z_dev,
                          const float* gxhat_dev, float* grad_dev, float* gz_dev);

/*
 * Backward of encode: grid blocks of grad_dev [P] are overwritten with the
 * dense gradient (zero at nodes no vertex touches); deterministic segmented
 * reduction over a node-sorted table, no atomics.
 */
npg_status npg_encode_bwd(npg_plan* plan, const float* gz_dev, float* grad_dev);

/*
 * Sec. 3.5 "Preconditioning": every grid block of grad_dev [P] is replaced
 * in place by (I + lambda L)^-2 g per feature channel, L the 6-neighbour
 * lattice Laplacian with free boundary (degree minus adjacency). MLP block
 * untouched. With NPG_PRECOND_CG: two conjugate-gradient solves from zero
 * with float64 inner products, synchronizing between batches of iterations, each
 * stopped at ||r|| <= cg_rtol ||b||; with cg_mg = 1 the solves are
 * preconditioned by a symmetric multigrid V-cycle (2x2x2 aggregates, Galerkin
 * coarse operators, damped Jacobi smoothing), which cuts the iteration count
 * several-fold. iters_host [2*(L+1)] (may be NULL) receives the iteration
 * counts.
 */
npg_status npg_precond(npg_plan* plan, float* grad_dev, int32_t* iters_host);

/*
 * Final relative residuals ||r||_2 / ||b||_2 of the CG recurrence (r updated
 * as r - alpha A p; float64, the largest over a grid's feature channels) of
 * the last preconditioning (by
 * npg_precond or inside npg_step) of the CG form: relres_host
 * [2*(L+1)], the first solve of every grid (position levels, then the
 * normal grid), then the second. 0 before any preconditioning, for a zero
 * right-hand side, and for the DCT form (exact). Host only; no GPU work.
 */
npg_status npg_precond_residuals(npg_plan* plan, double* relres_host);

/*
 * Sec. 3.5 "Isometry Loss" on deformed vertices xhat_dev [T][V][4] (as from
 * npg_decode_fwd): iso_dev [1] float64 receives
 *   L_iso = (1/(T E)) sum_t sum_(i,j) | |x^_i,t - x^_j,t| - |x^_i,key - x^_j,key| |
 * (key frame t_key of the config; its lengths are a stop-gradient);
 * gxhat_dev [T][V][4] (may be NULL) is incremented by w_iso dL_iso/dx^
 * (w column untouched); sign_dev [T][E] int8 (may be NULL) receives the
 * subgradient decision sign(|e_t| - |e_key|) of every frame and edge, in
 * the order of npg_plan_set_edges. Lengths and decisions are evaluated in
 * float64 from the float32 vertices; sign(0) = 0. NPG_EINVAL without edges.
 */
npg_status npg_iso(npg_plan* plan, const float* xhat_dev, float* gxhat_dev, double* iso_dev,
                   int8_t* sign_dev);

/*
 * Autotuner of the nearest-neighbour search (npg_chamfer_fwd, the metrics
 * and every step): its work-group size, 64, 128 (the default) or 256 threads
 * (the exhaustive pass: threads of 16 vertices; the pruned search: 1, 2 or 4
 * independent waves). threads = 0 times the three candidates of the plan's
 * search (nn_search) on its current deformed vertices and point sets (one
 * warm-up and two timed calls each, HIP events on the plan's stream) and keeps
 * the fastest; the metrics always use the exhaustive pass;
 * threads = 64, 128 or 256 sets it without timing. chosen_host [1] (may be
 * NULL) receives the work-group size in use; ms_host [3] (may be NULL) the
 * measured milliseconds per call for 64, 128, 256 (0 when not timed). Indices,
 * distances and sums do not depend on the choice (bitwise). Synchronizes the
 * plan's stream. NPG_EINVAL for other values of threads.
 */
npg_status npg_tune_nn(npg_plan* plan, int32_t threads, int32_t* chosen_host, float* ms_host);

/*
 * Autotuner of the decode backward's schedule: its work items are 64-vertex
 * blocks times nch frame chunks, dealt to min(items, CUs) persistent
 * work-groups. nch = 0 times up to 4 candidates (the load-balancing default
 * h, h/2, 2h and 4h within [n_min, T]; n_min = ceil(T/16) in the BF16 form,
 * else 1) on the plan's current parameters (one warm-up and two timed calls
 * each) and keeps the fastest; nch > 0 sets it without timing. cand_host [4]
 * and ms_host [4] (may be NULL) receive the candidates (0: unused slot) and
 * their milliseconds per call; chosen_host [1] (may be NULL) the count in use.
 * The chunk count fixes the grouping of the float32 per-chunk sums of the
 * first-layer gradient: results are deterministic for a given count and agree
 * within float32 rounding between counts (not bitwise). Grows workspace when
 * needed; synchronizes. NPG_EINVAL for a count outside [n_min, T].
 */
npg_status npg_tune_mlp(npg_plan* plan, int32_t nch, int32_t* chosen_host, int32_t* cand_host, float* ms_host);

/*
 * Autotuner of the CG preconditioner's work-group tiles on grids with
 * R >= 100 (F = 4): z planes per 64 x 4-column tile, 32, 64 (the default) or
 * 128. zs = 0 times four iterations of both solves per candidate on a fixed
 * non-zero right-hand side in the plan's gradient buffer (workspace between
 * steps; parameters and Adam state untouched) and keeps the fastest; zs > 0
 * sets it without timing. ms_host [3] (may be NULL): milliseconds per timed
 * call for 32, 64, 128 (0 when not timed). The tiles fix the grouping of the
 * float64 inner-product partial sums: results are deterministic for a given
 * choice and agree within the solver tolerance between choices (not bitwise).
 * Rebuilds the CG workspace; synchronizes. NPG_EINVAL for other values or the
 * DCT form.
 */
npg_status npg_tune_cg(npg_plan* plan, int32_t zs, int32_t* chosen_host, float* ms_host);

/*
 * Chain rule for reverse-mode callers (torch.autograd Functions built on the
 * stage entry points above): x_dev[k] *= c * s_dev[0] for 0 <= k < n, the
 * factor formed in float64 on the device (s_dev: one float64, typically the
 * upstream gradient of a scalar loss; c: a host constant). x_dev is float64
 * with is_f64 != 0, else float32; in place, on the plan's stream.
 * NPG_EINVAL for NULL pointers or n < 0; n = 0 does nothing.
 */
npg_status npg_scale(npg_plan* plan, const double* s_dev, double c, void* x_dev, int32_t is_f64,
                     int64_t n);

/*
 * Adam (bias-corrected, step count adam_step >= 1) over the flat vector with
 * per-block learning rates (levels, normal grid, MLP).
 */
npg_status npg_adam(npg_plan* plan, float* params_dev, const float* grad_dev, float* m_dev,
                    float* v_dev, int64_t adam_step);

/* Kernel time of the last npg_step per stage in milliseconds (host, [9]):
 * encode, decode, chamfer+loss, chamfer_bwd, iso (0 without the isometry
 * term), decode_bwd, encode_bwd, precond, adam. Valid after the stream has
 * finished the step. */
npg_status npg_stage_times(npg_plan* plan, float* ms_host);

/*
 * Profiling of the preconditioner's CG iterations: with enable != 0,
 * npg_step records HIP events around every iteration on the plan's stream and
 * resolves them after the step (one extra stream synchronisation per step).
 * Enabling resets the accumulators.
 */
npg_status npg_profile(npg_plan* plan, int32_t enable);

/* Accumulated since npg_profile(plan, 1) over the eager steps: summed time
 * of the CG iterations (ms; HIP events on the plan's stream bracket each whole
 * iteration: both streaming kernels, the V-cycle and both reductions), the
 * number of iterations launched, and their algorithmic bytes: cg_bytes_host
 * counts 6 float32 vector passes (x, r, p each read and written) over the R^3 F
 * unknowns of every grid for each iteration that grid took; cg_bytes_mg_host
 * (may be NULL) counts, for the V-cycle form, also z (written and read) and
 * every coarse level's right-hand side and correction (written and read). */
npg_status npg_profile_read(npg_plan* plan, double* cg_ms_host, int64_t* cg_iters_host,
                            double* cg_bytes_host, double* cg_bytes_mg_host);

#ifdef __cplusplus
}
#endif
#endif /* NEUPIG_H */
