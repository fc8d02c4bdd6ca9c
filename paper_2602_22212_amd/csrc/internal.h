// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/neupig.h"

#define NPG_MAX_SYS (NPG_MAX_LEVELS + 1)
// Largest buffer of stored hidden activations (npg_plan::act); a step whose
// activations take more recomputes them in the backward.
constexpr int64_t kActMaxBytes = int64_t(8) << 30;

// One grid "system": a position level or the normal grid.
struct NpgGrid {
  int R;            // nodes per axis
  int F;            // features per node
  int64_t nodes;    // R^3
  int64_t poff;     // offset (floats) into the flat parameter vector
  int64_t noff;     // offset (nodes) into the concatenated node space
  float lam;        // smoothness of the preconditioner
  float lr;         // Adam learning rate
  float scale;      // 1/L for position levels, 1 for the normal grid
};

// Directions kept per CG solve: iteration k writes its direction into ring
// slot k mod kCgDirs, and x takes the terms of kCgDirs iterations in one pass.
constexpr int kCgDirs = 8;

struct NpgCG {  // conjugate-gradient workspace
  float *x, *r;                // [n_grid_params] each, grid layout
  float* pd[kCgDirs] = {};     // [n_grid_params] each: the ring of directions
  double* ahist;               // [2 solves][n_sys][4][kCgDirs] alpha of each ring slot
  int last_iters[2] = {0, 0};  // iterations the last first / second solve took (its first batch)
  int last_grp[2][2] = {{0, 0}, {0, 0}};  // the same per solve and group of grids
  int* act_host = nullptr;     // [n_sys] pinned host copy of the active flags (eager solves)
  hipEvent_t ev_grp[2] = {nullptr, nullptr};  // per group: its last batch's flags are on the host
  double* part;                // [n_blocks][4 waves][4 channels] partial dots
  double* st;                  // [n_sys][4][8] per-system/channel scalars
  int* active;                 // [n_sys] any channel still iterating
  int* any_active;             // [1]
  int* blk_sys;                // [n_blocks] system of each block
  int64_t* blk_start;          // [n_blocks] first node of each block
  int* sys_blk0;               // [n_sys+1]
  int n_blocks;
  // multigrid V-cycle preconditioner of the solves (cfg.cg_mg)
  int mg;                      // 1: preconditioned CG
  float* z;                    // [n_grid_params] preconditioned residual
  float *mgB, *mgX;            // coarse levels of every system: right-hand sides, corrections
  double* part2;               // [n_blocks][4] partial r.z (the CG work-group table)
  double* part3;               // level-1 r.z partials of the large grids (their launches' blocks)
  int2* r3;                    // [n_sys] range of part3 of each system (empty: none)
  int* sys_split;              // [n_sys] 1: r.z split over the finest restriction and level 1
  int n_split;                 // systems with the split (large grids)
  std::vector<int> mg_l_p3;    // per launch: first part3 block of its level-1 tasks, -1 if none
  void* mg_tasks;              // device table of the V-cycle launches (struct MgTask)
  std::vector<std::vector<int>> mg_l_blk0;  // per launch: first block of each task, padded with INT_MAX
  std::vector<int> mg_l_task0, mg_l_ntask, mg_l_nblk;  // per launch: first task, tasks, blocks
  int mg_nlev;                 // levels of the deepest hierarchy
  double mg_elems[NPG_MAX_SYS];  // per system: coarse-level floats summed over the levels
  // Iterations in two groups of grids on two streams (n_grp = 2): group g
  // holds systems [grp_sys[g], grp_sys[g+1]) and work-groups [grp_blk[g],
  // grp_blk[g+1]) of the table; group 1 (the largest grid and the systems
  // after it) runs on the plan's stream, group 0 on stream2; per V-cycle
  // launch, group 0's blocks are [0, mg_split[l]), group 1's the rest
  int n_grp = 1;
  int grp_sys[3] = {0, 0, 0}, grp_blk[3] = {0, 0, 0};
  std::vector<int> mg_split;
  hipStream_t stream2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

struct NpgDct;
struct NpgNn;

// Per-step scalars the loss and Adam kernels of a graph-captured step read
// from device memory (the eager step passes them as kernel arguments).
struct NpgStepScal {
  double delta;                // confidence catch-up exponent 1 - sqrt(e / e_max)
  float inv_bc1, inv_sqrt_bc2;  // Adam bias corrections 1 / (1 - b1^k), 1 / sqrt(1 - b2^k)
  int cg_state;                 // recorded CG solves: bit w set if solve w had not converged within its
                                // recorded iterations (Adam then leaves the state untouched); bit 2: a
                                // solve recorded with cg_maxit iterations did not converge
};

struct npg_plan {
  npg_config cfg;
  hipStream_t stream;
  int device;
  int n_cu;
  int64_t V;
  int T;
  int64_t Ntot;
  std::vector<int64_t> off_h;
  int n_sys;           // L + 1
  int L;
  NpgGrid g[NPG_MAX_SYS];
  int64_t n_grid_params, n_nodes, mlp_off, n_params;
  int Fz, Din, W, H, M;
  int n_out;  // network outputs: 6 (exp map) or 7 (quaternion)
  int t_key;
  // static device data
  float4 *xyz, *nrm, *pts;
  int32_t* vperm;      // [V] vertices in Morton order of their rest positions (encode, pruned search)
  int64_t* d_off;
  int* pt_frame;
  NpgGrid* d_g;
  // encode-backward table (node-sorted)
  int64_t n_entries;
  int32_t* e_vert;     // [E] vertex of each entry
  float* e_w;          // [E] trilinear weight
  int64_t n_seg;
  int32_t* seg_key;    // [U] global node of each segment
  int32_t* seg_chunk0; // [U+1] first chunk of each segment
  int64_t n_chunk;
  int32_t* chunk_start;  // [C+1] first entry of each chunk
  float* chunk_sum;      // [C][4]
  int8_t* chunk_sys;     // [C] grid system of each chunk
  // owned optimizer state
  float *params, *m, *v, *grad;
  int64_t adam_k;
  // intermediates
  float *z, *gz;
  float4 *xhat, *gxhat;
  int32_t *a, *b;
  float *da, *db;
  double *cd, *w, *loss;
  double* w_g;             // [T] confidence weights times an upstream factor (npg_objective_bwd)
  // chamfer workspace
  int nvb;                 // vertex blocks per frame of the NN main pass
  int nn_threads;          // its work-group size and that of the pruned search (64, 128, 256; npg_tune_nn)
  int nvb_max;             // vertex blocks at 64 threads (colpart sizing)
  float* colpart;          // [T][nvb][Nmax] 64-bit column records (2 floats each)
  int64_t Nmax;
  long long* acc;          // [T][V][3] fixed-point accumulators
  // MLP workspace
  float *mlpA, *mlpB;      // [V][W], [T][W]
  float* wpack;            // repacked / transposed hidden and output weights
  uint16_t* wpack16;       // bfloat16 copy of wpack (BF16 form only)
  float* gam;              // [T][Din-Fz] time code
  float *Gv, *Gt, *Gt_part, *gW_part;
  float* act;              // [T][V][H-1][W] hidden activations of layers 2..H, written by the step's forward
                           // for its backward (FP32 form, when at most kActMaxBytes), else NULL
  int n_vblk_mlp;
  int64_t gw_part_len;
  // MLP backward schedule (both precisions): n_vblk_mlp 64-vertex blocks x
  // mlp_nch frame chunks, items dealt round-robin to mlp_grid persistent
  // work-groups; per-chunk vertex sums in Gv_part
  int mlp_nch, mlp_grid;
  int mlp_nch_alloc = 0, mlp_grid_alloc = 0;  // capacity of Gv_part (chunks) and gW_part (work-groups)
  int cg_zs = 64;          // z planes per work-group tile of the CG kernels on large grids (npg_tune_cg)
  double cg_relres[2 * NPG_MAX_SYS];  // last preconditioning: final ||r||/||b|| per grid, both solves
  float* Gv_part;          // [mlp_nch][V][W] (NULL when mlp_nch == 1)
  float* fl_part;          // [ceil(V/64)][W][8] first-layer partial sums
  // preconditioner workspaces
  NpgCG cg;
  NpgDct* dct;
  NpgNn* nn;               // pruned nearest-neighbour search tables (nn.hip)
  // isometry term: vertex -> incident-edge table (row [V+1]; per entry the
  // other endpoint and the edge id with the ownership bit 31), loss partials
  int64_t n_edges;
  int* iso_row;
  int* iso_nbr;
  uint32_t* iso_eid;
  double* iso_part;
  double* iso_val;
  int n_iso_blk;
  int* d_flag;             // non-finite flag
  hipEvent_t ev[10];
  float stage_ms[8];
  // optional timing of the CG iterations (profiling only)
  int prof_cg;
  std::vector<hipEvent_t> prof_ev;
  // graph-captured step (npg_step_graph): its scalars, graph and capture stream
  NpgStepScal* d_scal = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t cap_stream = nullptr;
  unsigned char* scratch = nullptr;  // this device's copy of the library's fixed scratch array
  int graph_iters[2] = {0, 0};       // CG form: iterations recorded for each solve
  int64_t graph_gen = 0;             // incremented by every recording (batch graphs compare it)
  int prof_n;                       // events recorded in the current step (one pair per batch of iterations)
  int prof_it;                      // iterations those pairs bracket
  double prof_cg_ms;                // accumulated time of resolved steps' iteration batches
  int64_t prof_cg_launches;         // accumulated CG iterations
  double prof_cg_bytes;             // accumulated algorithmic bytes
  double cg_alg_bytes;              // algorithmic bytes of the last preconditioner call (6 passes)
  double cg_alg_bytes_mg;           // the same counting z and the V-cycle's coarse levels
  double prof_cg_bytes_mg;          // accumulated cg_alg_bytes_mg
  int64_t cg_iters_sum;             // sum over grids and solves of the iteration counts
};

// error helpers (plan.hip)
npg_status npg_fail(npg_status s, const std::string& msg);
#define NPG_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return npg_fail(NPG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---- launchers --------------------------------------------------------------
// setup.hip
hipError_t npg_launch_pack(const float* src, float4* dst, int64_t n, hipStream_t s);
hipError_t npg_launch_point_frames(const int64_t* off, int T, int* pt_frame, int64_t N, hipStream_t s);
hipError_t npg_launch_check_finite(const float* p, int64_t n, int* flag, hipStream_t s);
npg_status npg_build_scatter_table(npg_plan* P);
// encode.hip
hipError_t npg_launch_encode_fwd(const npg_plan* P, const float* params, float* z);
hipError_t npg_launch_encode_bwd(const npg_plan* P, const float* gz, float* grad);
// mlp.hip
// act (FP32 form, H > 1; NULL: none): the forward also writes the hidden
// activations of layers 2..H there, and the backward reads them instead of
// recomputing (only for the parameters and z of the forward that wrote them)
hipError_t npg_launch_decode_fwd(const npg_plan* P, const float* params, const float* z, float4* xhat,
                                 float4* nhat = nullptr, float* act = nullptr);
hipError_t npg_launch_decode_bwd(const npg_plan* P, const float* params, const float* z,
                                 const float4* gxhat, float* grad, float* gz, const float* act = nullptr);
// chamfer.hip
hipError_t npg_launch_chamfer_fwd(const npg_plan* P, const float4* xhat, int32_t* a, float* da,
                                  int32_t* b, float* db, double* cd);
// sc: NULL, or the step scalars in device memory (then delta is read there)
double npg_loss_delta(int epoch, int n_epochs);
hipError_t npg_launch_loss(const npg_plan* P, const double* cd, int epoch, int n_epochs, double* w,
                           double* loss, const NpgStepScal* sc = nullptr);
hipError_t npg_launch_chamfer_bwd(const npg_plan* P, const float4* xhat, const int32_t* a,
                                  const int32_t* b, const double* w, float4* gxhat);
// precond.hip
npg_status npg_run_precond_cg(npg_plan* P, float* grad, int32_t* iters);
// graph-recordable CG preconditioning: n_iter[w] iterations of solve w, then
// a device-side convergence check into *state_dev (bits as NpgStepScal::cg_state)
npg_status npg_run_precond_cg_fixed(npg_plan* P, float* grad, const int n_iter[2], int* state_dev);
// host bookkeeping of the last CG preconditioning (iteration counts, residuals,
// algorithmic bytes); synchronizes
npg_status npg_cg_report(npg_plan* P, int32_t* iters);
// dct.hip
npg_status npg_dct_setup(npg_plan* P);
void npg_dct_free(npg_plan* P);
npg_status npg_iso_set_edges(npg_plan* P, int64_t E, const int32_t* edges_host);
void npg_iso_free(npg_plan* P);
npg_status npg_run_metrics(npg_plan* P, const float4* xhat, const float4* nhat, const float4* gt, const float4* gtn,
                           float tau, double* out);
// the same metrics in a fixed device array of the library (no allocation,
// no synchronisation); the array's address on the plan's device is found at
// plan creation by npg_scratch_setup
npg_status npg_scratch_setup(npg_plan* P);
npg_status npg_run_metrics_noalloc(npg_plan* P, const float4* xhat, const float4* nhat, const float4* gt,
                                   const float4* gtn, float tau, double* out);
// nT: frames in this launch (xhat, a, da hold nT frames of V vertices; off
// [nT+1] and pt_frame index the nT frames' points); 0 means all T frames
// nn.hip: the plan's vertex order; the pruned search (both directions, the plan's own points)
npg_status npg_vertex_order(npg_plan* P);
npg_status npg_nn_setup(npg_plan* P);
void npg_nn_free(npg_plan* P);
hipError_t npg_launch_nn_pruned(const npg_plan* P, const float4* xhat, int32_t* a, float* da, int32_t* b,
                                float* db);
// the plan's own points, by the search cfg.nn_search names (chamfer.hip)
hipError_t npg_launch_nn_step(const npg_plan* P, const float4* xhat, int32_t* a, float* da, int32_t* b, float* db);
hipError_t npg_launch_nn(const npg_plan* P, const float4* xhat, const float4* pts, const int64_t* off,
                         const int* pt_frame, int64_t Ntot, int64_t Nmax, void* colpart, int32_t* a, float* da,
                         int32_t* b, float* db, int nT = 0);
// gs: NULL, or an upstream factor in device memory multiplying the gradient
hipError_t npg_launch_iso(const npg_plan* P, const float4* xhat, float4* gxhat, double* iso, int8_t* sign,
                          double* loss, const double* gs = nullptr);
// chain.hip: out[t] = w[t] * g[0] (float64), t < n
hipError_t npg_launch_scaled_copy(const npg_plan* P, const double* w, const double* g, double* out, int n);
npg_status npg_run_precond_dct(npg_plan* P, float* grad);
// plan.hip: drop the captured step (after a change that alters its launches)
void npg_graph_reset(npg_plan* P);
// plan.hip: pieces of the graph-replayed step (npg_step_graph, batch graph)
npg_status npg_graph_prepare(npg_plan* P);
npg_status npg_graph_set_scalars(npg_plan* P, int epoch, int n_epochs, hipStream_t s);
npg_status npg_graph_read(npg_plan* P, hipStream_t s, NpgStepScal* sc, int* flag);
bool npg_graph_redo(npg_plan* P, const NpgStepScal& sc);
npg_status npg_graph_finish(npg_plan* P, const NpgStepScal& sc, int flag, double* loss_out, double* cd_out,
                            hipStream_t s);
// adam.hip
// sc: NULL, or the step scalars in device memory (then the bias corrections
// are read there and k is not used)
void npg_adam_scalars(const npg_plan* P, int64_t k, float* inv_bc1, float* inv_sqrt_bc2);
hipError_t npg_launch_adam(const npg_plan* P, float* params, const float* grad, float* m, float* v,
                           int64_t k, int* flag, const NpgStepScal* sc = nullptr);

// ---- device helpers shared by the kernels ----------------------------------
// Cell of a coordinate in a grid of R nodes per axis spanning [-1,1] (corner
// nodes on +-1): clamp to the box, u = (x+1)/2 (R-1), i0 = min(floor(u), R-2),
// fraction u - i0. NaN maps to the first cell.
__device__ __forceinline__ void npg_cell(float x, int R, int& i0, float& f) {
  float c = fminf(fmaxf(x, -1.0f), 1.0f);
  float u = (c + 1.0f) * 0.5f * (float)(R - 1);
  int i = (int)floorf(u);
  i = i < 0 ? 0 : (i > R - 2 ? R - 2 : i);
  i0 = i;
  f = u - (float)i;
}

// bfloat16 (round to nearest, ties to even) of a float32, as its 16 bits and
// widened back to float32.
__device__ __forceinline__ uint16_t npg_bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float npg_bf16_round(float x) { return __uint_as_float((uint32_t)npg_bf16_bits(x) << 16); }

__device__ __forceinline__ float npg_corner_w(int c, float fx, float fy, float fz) {
  float wx = (c & 1) ? fx : 1.0f - fx;
  float wy = (c & 2) ? fy : 1.0f - fy;
  float wz = (c & 4) ? fz : 1.0f - fz;
  return wx * wy * wz;
}
