// C ABI of the library: plan creation (validation, packing, static tables,
// workspace), state import/export, the full step and the stage entry points.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"

// launchers defined in the other translation units
int64_t npg_wpack_len(int W, int H);
int64_t npg_gw_part_len(int W, int H, int n_out);
void npg_mlp_schedule(int64_t V, int T, int n_cu, int tc_max, int* nvb, int* nch, int* grid);
int npg_mlp_bf16_frames();
int64_t npg_first_layer_blocks(int64_t V);
int npg_chamfer_vblock(int threads);
npg_status npg_cg_setup(npg_plan* P);
void npg_cg_free(npg_plan* P);

namespace {
thread_local std::string g_err;

__global__ void k_gamma(int T, int M, float* __restrict__ gam) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const double tt = T > 1 ? (double)t / (double)(T - 1) : 0.0;
  if (M == 0) {
    gam[t] = (float)tt;
    return;
  }
  double nu = 1.0;
  for (int j = 0; j < M; ++j) {
    gam[(int64_t)t * 2 * M + 2 * j] = (float)sin(M_PI * nu * tt);
    gam[(int64_t)t * 2 * M + 2 * j + 1] = (float)cos(M_PI * nu * tt);
    nu *= 2.0;
  }
}

__global__ void k_unpack_xyz(const float4* __restrict__ src, float* __restrict__ dst, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) {
    float4 v = src[i];
    dst[3 * i] = v.x;
    dst[3 * i + 1] = v.y;
    dst[3 * i + 2] = v.z;
  }
}

template <typename T>
npg_status dalloc(T** p, int64_t count) {
  if (count <= 0) count = 1;
  hipError_t e = hipMalloc((void**)p, (size_t)count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return npg_fail(NPG_ENOMEM, std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  return NPG_OK;
}

#define TRY(x)                      \
  do {                              \
    npg_status s_ = (x);            \
    if (s_ != NPG_OK) return s_;    \
  } while (0)

#define CHECK_ARG(cond, msg) \
  do {                       \
    if (!(cond)) return npg_fail(NPG_EINVAL, msg); \
  } while (0)

npg_status validate_cfg(const npg_config* c) {
  CHECK_ARG(c, "config is NULL");
  CHECK_ARG(c->n_levels >= 1 && c->n_levels <= NPG_MAX_LEVELS, "n_levels must be in 1..16");
  for (int l = 0; l < c->n_levels; ++l) {
    CHECK_ARG(c->res[l] >= 2 && c->res[l] <= 1024, "every level needs 2..1024 nodes per axis");
    CHECK_ARG(isfinite(c->lam[l]) && c->lam[l] >= 0.f, "lambda must be finite and >= 0");
    CHECK_ARG(isfinite(c->lr_grid[l]), "grid learning rates must be finite");
  }
  CHECK_ARG(c->feat_p >= 1 && c->feat_p <= 4, "feat_p must be in 1..4");
  CHECK_ARG(c->feat_n >= 1 && c->feat_n <= 4, "feat_n must be in 1..4");
  CHECK_ARG(c->res_n >= 2 && c->res_n <= 1024, "res_n must be in 2..1024");
  CHECK_ARG(c->time_freqs >= 0 && c->time_freqs <= 8, "time_freqs must be in 0..8");
  CHECK_ARG(c->mlp_hidden >= 1 && c->mlp_hidden <= 3, "mlp_hidden must be in 1..3");
  CHECK_ARG(c->mlp_width == 32 || c->mlp_width == 64 || c->mlp_width == 128, "mlp_width must be 32, 64 or 128");
  CHECK_ARG(c->act == NPG_ACT_RELU || c->act == NPG_ACT_LEAKY, "act must be NPG_ACT_RELU or NPG_ACT_LEAKY");
  CHECK_ARG(isfinite(c->leaky_slope) && c->leaky_slope > 0.f && c->leaky_slope <= 1.f, "leaky_slope must be in (0, 1]");
  CHECK_ARG(isfinite(c->alpha_t), "alpha_t must be finite");
  CHECK_ARG(c->beta1 >= 0.f && c->beta1 < 1.f && c->beta2 >= 0.f && c->beta2 < 1.f, "Adam betas must be in [0,1)");
  CHECK_ARG(c->eps > 0.f, "eps must be > 0");
  CHECK_ARG(c->cg_maxit >= 1 && c->cg_rtol > 0.0, "cg_maxit >= 1 and cg_rtol > 0 are required");
  CHECK_ARG(c->precond == NPG_PRECOND_CG || c->precond == NPG_PRECOND_DCT, "precond must be CG or DCT");
  CHECK_ARG(c->cg_mg == 0 || c->cg_mg == 1, "cg_mg must be 0 or 1");
  CHECK_ARG(c->cg_one_stream == 0 || c->cg_one_stream == 1, "cg_one_stream must be 0 or 1");
  CHECK_ARG(c->nn_search == NPG_NN_PRUNED || c->nn_search == NPG_NN_EXHAUSTIVE,
            "nn_search must be NPG_NN_PRUNED or NPG_NN_EXHAUSTIVE");
  CHECK_ARG(c->rot_head == NPG_ROT_EXPMAP || c->rot_head == NPG_ROT_QUAT, "rot_head must be EXPMAP or QUAT");
  CHECK_ARG(c->w_iso >= 0.f && std::isfinite(c->w_iso), "w_iso must be finite and >= 0");
  CHECK_ARG(c->precision == NPG_PREC_FP32 || c->precision == NPG_PREC_BF16, "precision must be FP32 or BF16");
  if (c->precond == NPG_PRECOND_DCT) {
    for (int l = 0; l < c->n_levels; ++l)
      CHECK_ARG(c->res[l] <= 256, "the DCT preconditioner supports up to 256 nodes per axis");
    CHECK_ARG(c->res_n <= 256, "the DCT preconditioner supports up to 256 nodes per axis");
  }
  return NPG_OK;
}

}  // namespace

npg_status npg_fail(npg_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

void npg_graph_reset(npg_plan* P) {
  if (P->graph_exec) hipGraphExecDestroy(P->graph_exec);
  if (P->graph) hipGraphDestroy(P->graph);
  P->graph_exec = nullptr;
  P->graph = nullptr;
}

namespace {
// a deterministic non-zero vector (autotuner input)
__global__ void k_fill_pattern(float* __restrict__ x, int64_t n) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < n) x[e] = (float)((e * 2654435761u) % 2048u) * (1.0f / 1024.0f) - 1.0f;
}

__global__ void k_set_step_scal(NpgStepScal* __restrict__ sc, double delta, float inv_bc1, float inv_sqrt_bc2) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc->delta = delta;
    sc->inv_bc1 = inv_bc1;
    sc->inv_sqrt_bc2 = inv_sqrt_bc2;
    sc->cg_state = 0;
  }
}

// Records the stages of npg_step into P->graph on a stream of its own; the
// loss and Adam kernels take their per-step scalars from P->d_scal. The CG
// form records P->graph_iters[w] iterations of solve w and a device-side
// convergence check (NpgStepScal::cg_state). Nothing is executed.
npg_status capture_step(npg_plan* P) {
  if (!P->d_scal) NPG_HIP(hipMalloc(&P->d_scal, sizeof(NpgStepScal)));
  if (!P->cap_stream) NPG_HIP(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
  hipStream_t keep = P->stream;
  const int keep_prof = P->prof_cg;
  P->prof_cg = 0;  // no profiling events inside the recording
  P->stream = P->cap_stream;
  NPG_HIP(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeRelaxed));
  auto enqueue = [&]() -> npg_status {
    NPG_HIP(npg_launch_encode_fwd(P, P->params, P->z));
    NPG_HIP(npg_launch_decode_fwd(P, P->params, P->z, P->xhat, nullptr, P->act));
    NPG_HIP(npg_launch_chamfer_fwd(P, P->xhat, P->a, P->da, P->b, P->db, P->cd));
    NPG_HIP(npg_launch_loss(P, P->cd, 0, 1, P->w, P->loss, P->d_scal));
    NPG_HIP(npg_launch_chamfer_bwd(P, P->xhat, P->a, P->b, P->w, P->gxhat));
    if (P->cfg.w_iso > 0.f) NPG_HIP(npg_launch_iso(P, P->xhat, P->gxhat, P->iso_val, nullptr, P->loss));
    NPG_HIP(npg_launch_decode_bwd(P, P->params, P->z, P->gxhat, P->grad, P->gz, P->act));
    NPG_HIP(npg_launch_encode_bwd(P, P->gz, P->grad));
    npg_status st = P->cfg.precond == NPG_PRECOND_DCT
                        ? npg_run_precond_dct(P, P->grad)
                        : npg_run_precond_cg_fixed(P, P->grad, P->graph_iters, &P->d_scal->cg_state);
    if (st != NPG_OK) return st;
    NPG_HIP(npg_launch_adam(P, P->params, P->grad, P->m, P->v, 1, P->d_flag, P->d_scal));
    return NPG_OK;
  };
  const npg_status st = enqueue();
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(P->cap_stream, &g);  // always ends the capture
  P->stream = keep;
  P->prof_cg = keep_prof;
  if (st != NPG_OK) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  NPG_HIP(e);
  P->graph = g;
  P->graph_gen += 1;
  NPG_HIP(hipGraphInstantiate(&P->graph_exec, P->graph, nullptr, nullptr, 0));
  return NPG_OK;
}
}  // namespace

// ---- the graph-replayed step (npg_step_graph, npg_batch_step_graph) -------
// Iteration counts of the CG form's recorded solves: what the last
// preconditioning took plus 2 (16 without one), recorded again when that
// leaves more than 6 idle; then the graph is recorded if there is none.
npg_status npg_graph_prepare(npg_plan* P) {
  if (P->cfg.precond == NPG_PRECOND_CG) {
    const int maxit = P->cfg.cg_maxit;
    for (int w = 0; w < 2; ++w) {
      const int last = P->cg.last_iters[w];
      const int want = std::min(maxit, last > 0 ? last + 2 : 16);
      if (P->graph_iters[w] == 0 || (last > 0 && P->graph_iters[w] > last + 6)) {
        if (P->graph_iters[w] != want) npg_graph_reset(P);
        P->graph_iters[w] = want;
      }
    }
  }
  if (!P->graph_exec) {
    const npg_status st = capture_step(P);
    if (st != NPG_OK) {
      npg_graph_reset(P);
      return st;
    }
  }
  return NPG_OK;
}

// The scalars of the next step (Adam step adam_k + 1) on stream s.
npg_status npg_graph_set_scalars(npg_plan* P, int epoch, int n_epochs, hipStream_t s) {
  float ib1 = 1.f, ib2 = 1.f;
  npg_adam_scalars(P, P->adam_k + 1, &ib1, &ib2);
  hipLaunchKernelGGL(k_set_step_scal, dim3(1), dim3(64), 0, s, P->d_scal, npg_loss_delta(epoch, n_epochs), ib1, ib2);
  NPG_HIP(hipGetLastError());
  return NPG_OK;
}

// Enqueue the reads of the replay's outcome (step scalars, non-finite flag).
npg_status npg_graph_read(npg_plan* P, hipStream_t s, NpgStepScal* sc, int* flag) {
  NPG_HIP(hipMemcpyAsync(sc, P->d_scal, sizeof(NpgStepScal), hipMemcpyDeviceToHost, s));
  NPG_HIP(hipMemcpyAsync(flag, P->d_flag, 4, hipMemcpyDeviceToHost, s));
  return NPG_OK;
}

// After a replay: true when a recorded solve stopped short (Adam left the
// state untouched); the next npg_graph_prepare records twice the iterations
// of that solve (at most cg_maxit) and the step is to be run again.
bool npg_graph_redo(npg_plan* P, const NpgStepScal& sc) {
  if (!(sc.cg_state & 3)) return false;
  for (int w = 0; w < 2; ++w)
    if (sc.cg_state & (1 << w)) P->graph_iters[w] = std::min(P->cfg.cg_maxit, 2 * P->graph_iters[w]);
  npg_graph_reset(P);
  return true;
}

// After a completed replay: the step count, the CG bookkeeping, the outputs
// and the status (synchronizes s).
npg_status npg_graph_finish(npg_plan* P, const NpgStepScal& sc, int flag, double* loss_out, double* cd_out,
                            hipStream_t s) {
  P->adam_k += 1;  // the update has been applied
  if (P->cfg.precond == NPG_PRECOND_CG) {
    const npg_status st = npg_cg_report(P, nullptr);
    if (st != NPG_OK) return st;
  }
  if (loss_out) NPG_HIP(hipMemcpyAsync(loss_out, P->loss, 8, hipMemcpyDeviceToDevice, s));
  if (cd_out) NPG_HIP(hipMemcpyAsync(cd_out, P->cd, 8 * (size_t)P->T, hipMemcpyDeviceToDevice, s));
  NPG_HIP(hipStreamSynchronize(s));
  if (flag) {
    NPG_HIP(hipMemsetAsync(P->d_flag, 0, 4, s));
    NPG_HIP(hipStreamSynchronize(s));
    return npg_fail(NPG_ENONFINITE, "a non-finite value was produced during the step");
  }
  if (sc.cg_state & 4) return npg_fail(NPG_ENOTCONV, "a CG solve reached cg_maxit");
  return NPG_OK;
}

// Frame chunks of the MLP backward: the decode backward's work items are
// 64-vertex blocks x nch frame chunks on min(items, n_cu) persistent
// work-groups; grows the per-chunk and per-work-group partial buffers when
// needed (synchronizes).
static npg_status set_mlp_chunks(npg_plan* P, int nch) {
  const int64_t nb = (P->V + 63) / 64;
  const int grid = (int)std::min<int64_t>(nb * nch, P->n_cu);
  NPG_HIP(hipStreamSynchronize(P->stream));
  if (nch > 1 && nch > P->mlp_nch_alloc) {
    if (P->Gv_part) NPG_HIP(hipFree(P->Gv_part));
    P->Gv_part = nullptr;
    P->mlp_nch_alloc = 0;
    NPG_HIP(hipMalloc(&P->Gv_part, (size_t)nch * P->V * P->W * 4));
    P->mlp_nch_alloc = nch;
  }
  if (grid > P->mlp_grid_alloc) {
    NPG_HIP(hipFree(P->gW_part));
    P->gW_part = nullptr;
    P->mlp_grid_alloc = 0;
    NPG_HIP(hipMalloc(&P->gW_part, (size_t)grid * P->gw_part_len * 4));
    P->mlp_grid_alloc = grid;
  }
  P->mlp_nch = nch;
  P->mlp_grid = grid;
  return NPG_OK;
}

// Milliseconds per call of `run` (one warm-up, two timed calls, HIP events
// on the plan's stream).
template <typename F>
static npg_status time_calls(npg_plan* P, F run, float* ms) {
  TRY(run());
  NPG_HIP(hipEventRecord(P->ev[0], P->stream));
  for (int r = 0; r < 2; ++r) TRY(run());
  NPG_HIP(hipEventRecord(P->ev[1], P->stream));
  NPG_HIP(hipEventSynchronize(P->ev[1]));
  NPG_HIP(hipEventElapsedTime(ms, P->ev[0], P->ev[1]));
  *ms *= 0.5f;
  return NPG_OK;
}

extern "C" {

const char* npg_last_error(void) { return g_err.c_str(); }

npg_status npg_param_count(const npg_config* cfg, int64_t* count) {
  TRY(validate_cfg(cfg));
  CHECK_ARG(count, "count_host is NULL");
  int64_t n = 0;
  for (int l = 0; l < cfg->n_levels; ++l) n += (int64_t)cfg->res[l] * cfg->res[l] * cfg->res[l] * cfg->feat_p;
  n += (int64_t)cfg->res_n * cfg->res_n * cfg->res_n * cfg->feat_n;
  const int W = cfg->mlp_width, H = cfg->mlp_hidden;
  const int Din = cfg->feat_n + cfg->feat_p + (cfg->time_freqs > 0 ? 2 * cfg->time_freqs : 1);
  const int n_out = cfg->rot_head == NPG_ROT_QUAT ? 7 : 6;
  n += (int64_t)W * Din + W + (int64_t)(H - 1) * ((int64_t)W * W + W) + n_out * (int64_t)W + n_out;
  *count = n;
  return NPG_OK;
}

npg_status npg_plan_destroy(npg_plan* P) {
  if (!P) return NPG_OK;
  hipStreamSynchronize(P->stream);
  void* bufs[] = {P->xyz, P->nrm, P->pts, P->vperm, P->d_off, P->pt_frame, P->d_g, P->e_vert, P->e_w, P->seg_key,
                  P->seg_chunk0, P->chunk_start, P->chunk_sum, P->chunk_sys, P->params, P->m, P->v, P->grad,
                  P->z, P->gz, P->xhat, P->gxhat, P->a, P->b, P->da, P->db, P->cd, P->w, P->loss, P->colpart,
                  P->w_g, P->acc, P->mlpA, P->mlpB, P->wpack, P->wpack16, P->Gv, P->Gt, P->Gt_part, P->gW_part, P->Gv_part, P->fl_part, P->gam, P->d_flag, P->act};
  for (void* b : bufs)
    if (b) hipFree(b);
  npg_graph_reset(P);
  if (P->cap_stream) hipStreamDestroy(P->cap_stream);
  if (P->d_scal) hipFree(P->d_scal);
  npg_cg_free(P);
  npg_dct_free(P);
  npg_nn_free(P);
  npg_iso_free(P);
  for (auto& e : P->ev)
    if (e) hipEventDestroy(e);
  for (auto& e : P->prof_ev)
    if (e) hipEventDestroy(e);
  delete P;
  return NPG_OK;
}

npg_status npg_plan_create(const npg_config* cfg, int64_t V, const float* xyz, const float* nrm, int32_t T,
                           const float* pts, const int64_t* off, void* stream, npg_plan** out) {
  CHECK_ARG(out, "out is NULL");
  *out = nullptr;
  TRY(validate_cfg(cfg));
  CHECK_ARG(V >= 1 && V < ((int64_t)1 << 31) / 16, "V must be in 1..2^27");
  CHECK_ARG(T >= 1, "T must be >= 1");
  CHECK_ARG(xyz && nrm && pts && off, "input pointers must be non-NULL");
  CHECK_ARG(off[0] == 0, "frame_off[0] must be 0");
  int64_t Nmax = 0;
  for (int t = 0; t < T; ++t) {
    CHECK_ARG(off[t + 1] > off[t], "every frame needs at least one point (frame_off strictly increasing)");
    Nmax = std::max(Nmax, off[t + 1] - off[t]);
  }
  CHECK_ARG(off[T] < ((int64_t)1 << 31), "total point count must be < 2^31");
  CHECK_ARG(cfg->t_key >= -1 && cfg->t_key < T, "t_key must be -1 or a frame index");

  npg_plan* P = new npg_plan();  // value-initialised: every pointer starts NULL
  P->off_h.assign(off, off + T + 1);
  P->cfg = *cfg;
  P->stream = (hipStream_t)stream;
  P->V = V;
  P->T = T;
  P->Ntot = off[T];
  P->Nmax = Nmax;
  P->L = cfg->n_levels;
  P->n_sys = P->L + 1;
  P->t_key = cfg->t_key >= 0 ? cfg->t_key : (T - 1) / 2;
  auto fail = [&](npg_status s) {
    std::string keep = g_err;
    npg_plan_destroy(P);
    g_err = keep;
    return s;
  };
#define TRYP(x)                        \
  do {                                 \
    npg_status s_ = (x);               \
    if (s_ != NPG_OK) return fail(s_); \
  } while (0)
#define HIPP(x)                                                                                  \
  do {                                                                                           \
    hipError_t e_ = (x);                                                                         \
    if (e_ != hipSuccess) return fail(npg_fail(NPG_EHIP, std::string(#x) + ": " + hipGetErrorString(e_))); \
  } while (0)

  HIPP(hipGetDevice(&P->device));
  TRYP(npg_scratch_setup(P));  // this device's address of the fixed scratch array
  int ncu = 0;
  HIPP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, P->device));
  P->n_cu = ncu > 0 ? ncu : 256;

  // grid systems: position levels then the normal grid
  int64_t poff = 0, noff = 0;
  for (int s = 0; s < P->n_sys; ++s) {
    NpgGrid& g = P->g[s];
    const bool pos = s < P->L;
    g.R = pos ? cfg->res[s] : cfg->res_n;
    g.F = pos ? cfg->feat_p : cfg->feat_n;
    g.nodes = (int64_t)g.R * g.R * g.R;
    g.poff = poff;
    g.noff = noff;
    g.lam = pos ? cfg->lam[s] : cfg->lam_n;
    g.lr = pos ? cfg->lr_grid[s] : cfg->lr_n;
    g.scale = pos ? 1.0f / (float)P->L : 1.0f;
    poff += g.nodes * g.F;
    noff += g.nodes;
  }
  P->n_grid_params = poff;
  P->n_nodes = noff;
  P->mlp_off = poff;
  TRYP(npg_param_count(cfg, &P->n_params));
  if (noff >= ((int64_t)1 << 31)) return fail(npg_fail(NPG_EINVAL, "grids too large (2^31 nodes)"));
  P->W = cfg->mlp_width;
  P->H = cfg->mlp_hidden;
  P->M = cfg->time_freqs;
  P->Fz = cfg->feat_n + cfg->feat_p;
  P->Din = P->Fz + (P->M > 0 ? 2 * P->M : 1);
  P->n_out = cfg->rot_head == NPG_ROT_QUAT ? 7 : 6;

  // inputs
  TRYP(dalloc(&P->xyz, V));
  TRYP(dalloc(&P->nrm, V));
  TRYP(dalloc(&P->pts, P->Ntot));
  TRYP(dalloc(&P->d_off, T + 1));
  TRYP(dalloc(&P->pt_frame, P->Ntot));
  TRYP(dalloc(&P->d_g, P->n_sys));
  TRYP(dalloc(&P->d_flag, 4));
  HIPP(hipMemcpy(P->d_off, off, (T + 1) * 8, hipMemcpyHostToDevice));
  HIPP(hipMemcpy(P->d_g, P->g, sizeof(NpgGrid) * P->n_sys, hipMemcpyHostToDevice));
  HIPP(hipMemsetAsync(P->d_flag, 0, 16, P->stream));
  HIPP(npg_launch_check_finite(xyz, 3 * V, P->d_flag, P->stream));
  HIPP(npg_launch_check_finite(nrm, 3 * V, P->d_flag, P->stream));
  HIPP(npg_launch_check_finite(pts, 3 * P->Ntot, P->d_flag, P->stream));
  int bad = 0;
  HIPP(hipMemcpyAsync(&bad, P->d_flag, 4, hipMemcpyDeviceToHost, P->stream));
  HIPP(hipStreamSynchronize(P->stream));
  if (bad) return fail(npg_fail(NPG_EINVAL, "non-finite value in ref_xyz, ref_nrm or pts"));
  HIPP(npg_launch_pack(xyz, P->xyz, V, P->stream));
  HIPP(npg_launch_pack(nrm, P->nrm, V, P->stream));
  HIPP(npg_launch_pack(pts, P->pts, P->Ntot, P->stream));
  HIPP(npg_launch_point_frames(P->d_off, T, P->pt_frame, P->Ntot, P->stream));
  const int Dt = P->Din - P->Fz;
  TRYP(dalloc(&P->gam, (int64_t)T * Dt));
  hipLaunchKernelGGL(k_gamma, dim3((T + 127) / 128), dim3(128), 0, P->stream, T, P->M, P->gam);
  HIPP(hipGetLastError());

  TRYP(npg_build_scatter_table(P));
  TRYP(npg_vertex_order(P));

  // optimizer state and intermediates
  const int64_t NP = P->n_params;
  TRYP(dalloc(&P->params, NP));
  TRYP(dalloc(&P->m, NP));
  TRYP(dalloc(&P->v, NP));
  TRYP(dalloc(&P->grad, NP));
  HIPP(hipMemsetAsync(P->params, 0, NP * 4, P->stream));
  HIPP(hipMemsetAsync(P->m, 0, NP * 4, P->stream));
  HIPP(hipMemsetAsync(P->v, 0, NP * 4, P->stream));
  TRYP(dalloc(&P->z, V * P->Fz));
  TRYP(dalloc(&P->gz, V * P->Fz));
  const int64_t TV = (int64_t)T * V;
  TRYP(dalloc(&P->xhat, TV));
  TRYP(dalloc(&P->gxhat, TV));
  TRYP(dalloc(&P->a, TV));
  TRYP(dalloc(&P->da, TV));
  TRYP(dalloc(&P->b, P->Ntot));
  TRYP(dalloc(&P->db, P->Ntot));
  TRYP(dalloc(&P->cd, T));
  TRYP(dalloc(&P->w, T));
  TRYP(dalloc(&P->loss, 1));
  TRYP(dalloc(&P->w_g, T));
  P->nn_threads = 128;
  P->nvb = (int)((V + npg_chamfer_vblock(128) - 1) / npg_chamfer_vblock(128));
  P->nvb_max = (int)((V + npg_chamfer_vblock(64) - 1) / npg_chamfer_vblock(64));
  TRYP(dalloc(&P->colpart, 2 * (int64_t)T * P->nvb_max * Nmax));
  if (cfg->nn_search == NPG_NN_PRUNED) TRYP(npg_nn_setup(P));
  TRYP(dalloc(&P->acc, 3 * TV));
  TRYP(dalloc(&P->mlpA, V * P->W));
  TRYP(dalloc(&P->mlpB, (int64_t)T * P->W));
  TRYP(dalloc(&P->wpack, npg_wpack_len(P->W, P->H)));
  if (cfg->precision == NPG_PREC_BF16)
    HIPP(hipMalloc(&P->wpack16, npg_wpack_len(P->W, P->H) * sizeof(uint16_t)));
  P->n_vblk_mlp = (int)((V + 63) / 64);
  P->gw_part_len = npg_gw_part_len(P->W, P->H, P->n_out);
  TRYP(dalloc(&P->Gv, V * P->W));
  TRYP(dalloc(&P->Gt, (int64_t)T * P->W));
  TRYP(dalloc(&P->Gt_part, (int64_t)T * P->n_vblk_mlp * P->W));
  {
    int nvb = 0;
    npg_mlp_schedule(V, T, P->n_cu, cfg->precision == NPG_PREC_BF16 ? npg_mlp_bf16_frames() : 0, &nvb,
                     &P->mlp_nch, &P->mlp_grid);
  }
  if (P->mlp_nch > 1) TRYP(dalloc(&P->Gv_part, (int64_t)P->mlp_nch * V * P->W));
  TRYP(dalloc(&P->gW_part, (int64_t)P->mlp_grid * P->gw_part_len));
  P->mlp_nch_alloc = P->mlp_nch > 1 ? P->mlp_nch : 0;
  P->mlp_grid_alloc = P->mlp_grid;
  TRYP(dalloc(&P->fl_part, npg_first_layer_blocks(V) * P->W * 8));
  {
    // the step's forward keeps the hidden activations of layers 2..H for its
    // backward (FP32 form) when they fit kActMaxBytes and device memory;
    // otherwise (act stays NULL) the backward recomputes them
    const int64_t n_act = TV * (P->H - 1) * P->W;
    if (cfg->precision != NPG_PREC_BF16 && P->H > 1 && n_act * 4 <= kActMaxBytes &&
        hipMalloc(&P->act, n_act * sizeof(float)) != hipSuccess) {
      P->act = nullptr;
      (void)hipGetLastError();  // clear the failed allocation's error
    }
  }
  if (cfg->precond == NPG_PRECOND_DCT) TRYP(npg_dct_setup(P));
  else TRYP(npg_cg_setup(P));
  for (auto& e : P->ev) HIPP(hipEventCreate(&e));
  P->adam_k = 0;
  HIPP(hipStreamSynchronize(P->stream));
  *out = P;
  return NPG_OK;
#undef TRYP
#undef HIPP
}

npg_status npg_set_state(npg_plan* P, const float* params, const float* m, const float* v, int64_t k) {
  CHECK_ARG(P && params, "plan and params_dev must be non-NULL");
  CHECK_ARG(k >= 0, "adam_steps must be >= 0");
  const size_t nb = (size_t)P->n_params * 4;
  NPG_HIP(hipMemcpyAsync(P->params, params, nb, hipMemcpyDeviceToDevice, P->stream));
  if (m) NPG_HIP(hipMemcpyAsync(P->m, m, nb, hipMemcpyDeviceToDevice, P->stream));
  else NPG_HIP(hipMemsetAsync(P->m, 0, nb, P->stream));
  if (v) NPG_HIP(hipMemcpyAsync(P->v, v, nb, hipMemcpyDeviceToDevice, P->stream));
  else NPG_HIP(hipMemsetAsync(P->v, 0, nb, P->stream));
  P->adam_k = k;
  NPG_HIP(hipStreamSynchronize(P->stream));
  return NPG_OK;
}

npg_status npg_get_state(npg_plan* P, float* params, float* m, float* v, int64_t* k) {
  CHECK_ARG(P, "plan is NULL");
  const size_t nb = (size_t)P->n_params * 4;
  if (params) NPG_HIP(hipMemcpyAsync(params, P->params, nb, hipMemcpyDeviceToDevice, P->stream));
  if (m) NPG_HIP(hipMemcpyAsync(m, P->m, nb, hipMemcpyDeviceToDevice, P->stream));
  if (v) NPG_HIP(hipMemcpyAsync(v, P->v, nb, hipMemcpyDeviceToDevice, P->stream));
  if (k) *k = P->adam_k;
  NPG_HIP(hipStreamSynchronize(P->stream));
  return NPG_OK;
}

npg_status npg_encode_fwd(npg_plan* P, const float* params, float* z) {
  CHECK_ARG(P && params && z, "NULL argument");
  NPG_HIP(npg_launch_encode_fwd(P, params, z));
  return NPG_OK;
}

npg_status npg_decode_fwd(npg_plan* P, const float* params, const float* z, float* xhat) {
  CHECK_ARG(P && params && z && xhat, "NULL argument");
  NPG_HIP(npg_launch_decode_fwd(P, params, z, reinterpret_cast<float4*>(xhat)));
  return NPG_OK;
}

npg_status npg_chamfer_fwd(npg_plan* P, const float* xhat, int32_t* a, float* da, int32_t* b, float* db,
                           double* cd) {
  CHECK_ARG(P && xhat && a && da && b && db && cd, "NULL argument");
  NPG_HIP(npg_launch_chamfer_fwd(P, reinterpret_cast<const float4*>(xhat), a, da, b, db, cd));
  return NPG_OK;
}

npg_status npg_loss(npg_plan* P, const double* cd, int32_t epoch, int32_t n_epochs, double* w, double* loss) {
  CHECK_ARG(P && cd && w && loss, "NULL argument");
  CHECK_ARG(n_epochs >= 1 && epoch >= 0 && epoch <= n_epochs, "need 0 <= epoch <= n_epochs, n_epochs >= 1");
  NPG_HIP(npg_launch_loss(P, cd, epoch, n_epochs, w, loss));
  return NPG_OK;
}

npg_status npg_objective_fwd(npg_plan* P, const float* xhat, int32_t epoch, int32_t n_epochs, int32_t* a, float* da,
                             int32_t* b, float* db, double* cd, double* w, double* iso, double* loss) {
  CHECK_ARG(P && xhat && a && da && b && db && cd && w && loss, "NULL argument");
  CHECK_ARG(n_epochs >= 1 && epoch >= 0 && epoch <= n_epochs, "need 0 <= epoch <= n_epochs, n_epochs >= 1");
  CHECK_ARG(P->cfg.w_iso == 0.f || P->n_edges > 0, "w_iso > 0 needs the mesh edges (npg_plan_set_edges)");
  const float4* x = reinterpret_cast<const float4*>(xhat);
  NPG_HIP(npg_launch_chamfer_fwd(P, x, a, da, b, db, cd));
  NPG_HIP(npg_launch_loss(P, cd, epoch, n_epochs, w, loss));
  if (P->cfg.w_iso > 0.f) NPG_HIP(npg_launch_iso(P, x, nullptr, iso ? iso : P->iso_val, nullptr, loss));
  return NPG_OK;
}

npg_status npg_objective_bwd(npg_plan* P, const float* xhat, const int32_t* a, const int32_t* b, const double* w,
                             const double* g, float* gxhat) {
  CHECK_ARG(P && xhat && a && b && w && gxhat, "NULL argument");
  CHECK_ARG(P->cfg.w_iso == 0.f || P->n_edges > 0, "w_iso > 0 needs the mesh edges (npg_plan_set_edges)");
  const float4* x = reinterpret_cast<const float4*>(xhat);
  float4* gx = reinterpret_cast<float4*>(gxhat);
  const double* wg = w;
  if (g) {  // the upstream factor enters the float64 frame weights
    NPG_HIP(npg_launch_scaled_copy(P, w, g, P->w_g, P->T));
    wg = P->w_g;
  }
  NPG_HIP(npg_launch_chamfer_bwd(P, x, a, b, wg, gx));
  if (P->cfg.w_iso > 0.f) NPG_HIP(npg_launch_iso(P, x, gx, P->iso_val, nullptr, nullptr, g));
  return NPG_OK;
}

npg_status npg_chamfer_bwd(npg_plan* P, const float* xhat, const int32_t* a, const int32_t* b, const double* w,
                           float* gxhat) {
  CHECK_ARG(P && xhat && a && b && w && gxhat, "NULL argument");
  NPG_HIP(npg_launch_chamfer_bwd(P, reinterpret_cast<const float4*>(xhat), a, b, w,
                                 reinterpret_cast<float4*>(gxhat)));
  return NPG_OK;
}

npg_status npg_decode_bwd(npg_plan* P, const float* params, const float* z, const float* gxhat, float* grad,
                          float* gz) {
  CHECK_ARG(P && params && z && gxhat && grad && gz, "NULL argument");
  NPG_HIP(npg_launch_decode_bwd(P, params, z, reinterpret_cast<const float4*>(gxhat), grad, gz));
  return NPG_OK;
}

npg_status npg_encode_bwd(npg_plan* P, const float* gz, float* grad) {
  CHECK_ARG(P && gz && grad, "NULL argument");
  NPG_HIP(npg_launch_encode_bwd(P, gz, grad));
  return NPG_OK;
}

npg_status npg_precond(npg_plan* P, float* grad, int32_t* iters) {
  CHECK_ARG(P && grad, "NULL argument");
  if (P->cfg.precond == NPG_PRECOND_DCT) {
    if (iters)
      for (int s = 0; s < 2 * P->n_sys; ++s) iters[s] = 0;
    return npg_run_precond_dct(P, grad);
  }
  return npg_run_precond_cg(P, grad, iters);
}

npg_status npg_adam(npg_plan* P, float* params, const float* grad, float* m, float* v, int64_t k) {
  CHECK_ARG(P && params && grad && m && v, "NULL argument");
  CHECK_ARG(k >= 1, "adam_step must be >= 1");
  NPG_HIP(npg_launch_adam(P, params, grad, m, v, k, P->d_flag));
  return NPG_OK;
}

npg_status npg_step(npg_plan* P, int32_t epoch, int32_t n_epochs, double* loss_out, double* cd_out) {
  CHECK_ARG(P, "plan is NULL");
  CHECK_ARG(n_epochs >= 1 && epoch >= 0 && epoch <= n_epochs, "need 0 <= epoch <= n_epochs, n_epochs >= 1");
  CHECK_ARG(P->cfg.w_iso == 0.f || P->n_edges > 0, "w_iso > 0 needs the mesh edges (npg_plan_set_edges)");
  hipStream_t s = P->stream;
  NPG_HIP(hipEventRecord(P->ev[0], s));
  NPG_HIP(npg_launch_encode_fwd(P, P->params, P->z));
  NPG_HIP(hipEventRecord(P->ev[1], s));
  NPG_HIP(npg_launch_decode_fwd(P, P->params, P->z, P->xhat, nullptr, P->act));
  NPG_HIP(hipEventRecord(P->ev[2], s));
  NPG_HIP(npg_launch_chamfer_fwd(P, P->xhat, P->a, P->da, P->b, P->db, P->cd));
  NPG_HIP(npg_launch_loss(P, P->cd, epoch, n_epochs, P->w, P->loss));
  NPG_HIP(hipEventRecord(P->ev[3], s));
  NPG_HIP(npg_launch_chamfer_bwd(P, P->xhat, P->a, P->b, P->w, P->gxhat));
  NPG_HIP(hipEventRecord(P->ev[4], s));
  if (P->cfg.w_iso > 0.f) NPG_HIP(npg_launch_iso(P, P->xhat, P->gxhat, P->iso_val, nullptr, P->loss));
  NPG_HIP(hipEventRecord(P->ev[5], s));
  NPG_HIP(npg_launch_decode_bwd(P, P->params, P->z, P->gxhat, P->grad, P->gz, P->act));
  NPG_HIP(hipEventRecord(P->ev[6], s));
  NPG_HIP(npg_launch_encode_bwd(P, P->gz, P->grad));
  NPG_HIP(hipEventRecord(P->ev[7], s));
  npg_status pst = P->cfg.precond == NPG_PRECOND_DCT ? npg_run_precond_dct(P, P->grad)
                                                     : npg_run_precond_cg(P, P->grad, nullptr);
  if (pst != NPG_OK && pst != NPG_ENOTCONV) return pst;
  NPG_HIP(hipEventRecord(P->ev[8], s));
  P->adam_k += 1;
  NPG_HIP(npg_launch_adam(P, P->params, P->grad, P->m, P->v, P->adam_k, P->d_flag));
  NPG_HIP(hipEventRecord(P->ev[9], s));
  if (P->prof_cg) {
    // resolve this step's CG iteration timings (the stream is drained below)
    NPG_HIP(hipStreamSynchronize(s));
    for (int k = 0; k + 1 < P->prof_n; k += 2) {
      float a = 0.f;
      NPG_HIP(hipEventElapsedTime(&a, P->prof_ev[k], P->prof_ev[k + 1]));
      P->prof_cg_ms += (double)a;
    }
    P->prof_cg_launches += P->prof_it;
    if (P->cfg.precond == NPG_PRECOND_CG) {
      P->prof_cg_bytes += P->cg_alg_bytes;
      P->prof_cg_bytes_mg += P->cg_alg_bytes_mg;
    }
    P->prof_n = 0;
    P->prof_it = 0;
  }
  if (loss_out) NPG_HIP(hipMemcpyAsync(loss_out, P->loss, 8, hipMemcpyDeviceToDevice, s));
  if (cd_out) NPG_HIP(hipMemcpyAsync(cd_out, P->cd, 8 * (size_t)P->T, hipMemcpyDeviceToDevice, s));
  int flag = 0;
  NPG_HIP(hipMemcpyAsync(&flag, P->d_flag, 4, hipMemcpyDeviceToHost, s));
  NPG_HIP(hipStreamSynchronize(s));
  if (flag) {
    NPG_HIP(hipMemsetAsync(P->d_flag, 0, 4, s));
    return npg_fail(NPG_ENONFINITE, "a non-finite value was produced during the step");
  }
  if (pst == NPG_ENOTCONV) return npg_fail(NPG_ENOTCONV, "a CG solve reached cg_maxit");
  return NPG_OK;
}

npg_status npg_step_graph(npg_plan* P, int32_t epoch, int32_t n_epochs, double* loss_out, double* cd_out) {
  CHECK_ARG(P, "plan is NULL");
  CHECK_ARG(n_epochs >= 1 && epoch >= 0 && epoch <= n_epochs, "need 0 <= epoch <= n_epochs, n_epochs >= 1");
  CHECK_ARG(P->cfg.w_iso == 0.f || P->n_edges > 0, "w_iso > 0 needs the mesh edges (npg_plan_set_edges)");
  hipStream_t s = P->stream;
  NpgStepScal sc_h{};
  int flag = 0;
  for (;;) {
    TRY(npg_graph_prepare(P));
    TRY(npg_graph_set_scalars(P, epoch, n_epochs, s));
    NPG_HIP(hipGraphLaunch(P->graph_exec, s));
    TRY(npg_graph_read(P, s, &sc_h, &flag));
    NPG_HIP(hipStreamSynchronize(s));
    if (!npg_graph_redo(P, sc_h)) break;
    if (flag) NPG_HIP(hipMemsetAsync(P->d_flag, 0, 4, s));
  }
  return npg_graph_finish(P, sc_h, flag, loss_out, cd_out, s);
}

npg_status npg_profile(npg_plan* P, int32_t enable) {
  CHECK_ARG(P, "plan is NULL");
  if (enable && P->prof_ev.empty()) {
    P->prof_ev.resize(2 * 2 * (size_t)P->cfg.cg_maxit + 8, nullptr);
    for (auto& e : P->prof_ev) NPG_HIP(hipEventCreate(&e));
  }
  P->prof_cg = enable ? 1 : 0;
  P->prof_n = 0;
  P->prof_it = 0;
  P->prof_cg_ms = 0.0;
  P->prof_cg_launches = 0;
  P->prof_cg_bytes = 0.0;
  P->prof_cg_bytes_mg = 0.0;
  return NPG_OK;
}

npg_status npg_profile_read(npg_plan* P, double* cg_ms, int64_t* cg_iters, double* cg_bytes, double* cg_bytes_mg) {
  CHECK_ARG(P && cg_ms && cg_iters && cg_bytes, "NULL argument");
  *cg_ms = P->prof_cg_ms;
  *cg_iters = P->prof_cg_launches;
  *cg_bytes = P->prof_cg_bytes;
  if (cg_bytes_mg) *cg_bytes_mg = P->prof_cg_bytes_mg;
  return NPG_OK;
}

npg_status npg_stage_times(npg_plan* P, float* ms) {
  CHECK_ARG(P && ms, "NULL argument");
  for (int k = 0; k < 9; ++k) NPG_HIP(hipEventElapsedTime(ms + k, P->ev[k], P->ev[k + 1]));
  return NPG_OK;
}

npg_status npg_plan_set_edges(npg_plan* P, int64_t n_edges, const int32_t* edges_host) {
  CHECK_ARG(P && edges_host, "plan and edges_host must be non-NULL");
  CHECK_ARG(n_edges >= 1 && n_edges < (int64_t)1 << 30, "need 1 <= n_edges < 2^30");
  npg_graph_reset(P);  // a captured step holds the old edge buffers
  return npg_iso_set_edges(P, n_edges, edges_host);
}

npg_status npg_iso(npg_plan* P, const float* xhat_dev, float* gxhat_dev, double* iso_dev, int8_t* sign_dev) {
  CHECK_ARG(P && xhat_dev && iso_dev, "plan, xhat_dev and iso_dev must be non-NULL");
  CHECK_ARG(P->n_edges > 0, "no mesh edges (npg_plan_set_edges)");
  NPG_HIP(npg_launch_iso(P, reinterpret_cast<const float4*>(xhat_dev), reinterpret_cast<float4*>(gxhat_dev),
                         iso_dev, sign_dev, nullptr));
  return NPG_OK;
}

npg_status npg_predict(npg_plan* P, float* xhat_dev, float* nhat_dev) {
  CHECK_ARG(P && xhat_dev, "plan and xhat_dev must be non-NULL");
  NPG_HIP(npg_launch_encode_fwd(P, P->params, P->z));
  NPG_HIP(npg_launch_decode_fwd(P, P->params, P->z, reinterpret_cast<float4*>(xhat_dev),
                                reinterpret_cast<float4*>(nhat_dev)));
  return NPG_OK;
}

npg_status npg_metrics(npg_plan* P, const float* xhat_dev, const float* nhat_dev, const float* gt_dev,
                       const float* gtn_dev, float tau, double* out_dev) {
  CHECK_ARG(P && xhat_dev && nhat_dev && gt_dev && gtn_dev && out_dev, "NULL argument");
  CHECK_ARG(tau > 0.f && std::isfinite(tau), "tau must be finite and > 0");
  return npg_run_metrics(P, reinterpret_cast<const float4*>(xhat_dev), reinterpret_cast<const float4*>(nhat_dev),
                         reinterpret_cast<const float4*>(gt_dev), reinterpret_cast<const float4*>(gtn_dev), tau,
                         out_dev);
}

npg_status npg_metrics_noalloc(npg_plan* P, const float* xhat_dev, const float* nhat_dev, const float* gt_dev,
                               const float* gtn_dev, float tau, double* out_dev) {
  CHECK_ARG(P && xhat_dev && nhat_dev && gt_dev && gtn_dev && out_dev, "NULL argument");
  CHECK_ARG(tau > 0.f && std::isfinite(tau), "tau must be finite and > 0");
  return npg_run_metrics_noalloc(P, reinterpret_cast<const float4*>(xhat_dev),
                                 reinterpret_cast<const float4*>(nhat_dev), reinterpret_cast<const float4*>(gt_dev),
                                 reinterpret_cast<const float4*>(gtn_dev), tau, out_dev);
}

npg_status npg_deform(npg_plan* P, float* out) {
  CHECK_ARG(P && out, "NULL argument");
  NPG_HIP(npg_launch_encode_fwd(P, P->params, P->z));
  NPG_HIP(npg_launch_decode_fwd(P, P->params, P->z, P->xhat));
  const int64_t n = (int64_t)P->T * P->V;
  hipLaunchKernelGGL(k_unpack_xyz, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, P->stream, P->xhat, out, n);
  NPG_HIP(hipGetLastError());
  return NPG_OK;
}

// Blocks of the flat parameter vector in order: the L position grids
// [R_l^3][F], the normal grid [R_n^3][F_n], then W_k [out][in] and b_k [out]
// of the H + 1 MLP layers. (offset, count) in floats.
static std::vector<std::pair<int64_t, int64_t>> param_blocks(const npg_plan* P) {
  std::vector<std::pair<int64_t, int64_t>> b;
  for (int s = 0; s < P->n_sys; ++s) b.emplace_back(P->g[s].poff, P->g[s].nodes * P->g[s].F);
  int64_t off = P->mlp_off;
  int din = P->Din;
  for (int k = 0; k <= P->H; ++k) {
    const int dout = k < P->H ? P->W : P->n_out;
    b.emplace_back(off, (int64_t)dout * din);
    off += (int64_t)dout * din;
    b.emplace_back(off, dout);
    off += dout;
    din = dout;
  }
  return b;
}

static npg_status copy_blocks(npg_plan* P, float* const* dst, const float* const* src, bool import) {
  const auto blocks = param_blocks(P);
  for (size_t k = 0; k < blocks.size(); ++k)
    CHECK_ARG(import ? src[k] != nullptr : dst[k] != nullptr, "block buffer " + std::to_string(k) + " is NULL");
  for (size_t k = 0; k < blocks.size(); ++k) {
    const size_t nb = (size_t)blocks[k].second * 4;
    if (import) NPG_HIP(hipMemcpyAsync(P->params + blocks[k].first, src[k], nb, hipMemcpyDeviceToDevice, P->stream));
    else NPG_HIP(hipMemcpyAsync(dst[k], P->params + blocks[k].first, nb, hipMemcpyDeviceToDevice, P->stream));
  }
  NPG_HIP(hipStreamSynchronize(P->stream));
  return NPG_OK;
}

npg_status npg_params_import(npg_plan* P, const float* const* bufs) {
  CHECK_ARG(P && bufs, "NULL argument");
  return copy_blocks(P, nullptr, bufs, true);
}

npg_status npg_params_export(npg_plan* P, float* const* bufs) {
  CHECK_ARG(P && bufs, "NULL argument");
  return copy_blocks(P, bufs, nullptr, false);
}

npg_status npg_state_import(npg_plan* P, const float* params, const float* m, const float* v, int64_t adam_steps) {
  return npg_set_state(P, params, m, v, adam_steps);
}

npg_status npg_state_export(npg_plan* P, float* params, float* m, float* v, int64_t* adam_steps) {
  return npg_get_state(P, params, m, v, adam_steps);
}

npg_status npg_precond_residuals(npg_plan* P, double* relres) {
  CHECK_ARG(P && relres, "NULL argument");
  for (int k = 0; k < 2 * P->n_sys; ++k) relres[k] = P->cfg.precond == NPG_PRECOND_CG ? P->cg_relres[k] : 0.0;
  return NPG_OK;
}

npg_status npg_tune_nn(npg_plan* P, int32_t threads, int32_t* chosen, float* ms) {
  CHECK_ARG(P, "plan is NULL");
  CHECK_ARG(threads == 0 || threads == 64 || threads == 128 || threads == 256, "threads must be 0, 64, 128 or 256");
  npg_graph_reset(P);  // a captured step holds the old launch shape
  auto set = [&](int kt) {
    P->nn_threads = kt;
    const int vb = npg_chamfer_vblock(kt);
    P->nvb = (int)((P->V + vb - 1) / vb);
  };
  if (ms)
    for (int k = 0; k < 3; ++k) ms[k] = 0.f;
  if (threads != 0) {
    set(threads);
  } else {
    // the current deformed vertices of the plan's parameters
    NPG_HIP(npg_launch_encode_fwd(P, P->params, P->z));
    NPG_HIP(npg_launch_decode_fwd(P, P->params, P->z, P->xhat));
    const int cand[3] = {64, 128, 256};
    float best = 0.f;
    int best_kt = 128;
    for (int k = 0; k < 3; ++k) {
      set(cand[k]);
      NPG_HIP(npg_launch_nn_step(P, P->xhat, P->a, P->da, P->b, P->db));  // warm-up
      NPG_HIP(hipEventRecord(P->ev[0], P->stream));
      for (int r = 0; r < 2; ++r)
        NPG_HIP(npg_launch_nn_step(P, P->xhat, P->a, P->da, P->b, P->db));
      NPG_HIP(hipEventRecord(P->ev[1], P->stream));
      NPG_HIP(hipEventSynchronize(P->ev[1]));
      float t = 0.f;
      NPG_HIP(hipEventElapsedTime(&t, P->ev[0], P->ev[1]));
      t *= 0.5f;
      if (ms) ms[k] = t;
      if (k == 0 || t < best) {
        best = t;
        best_kt = cand[k];
      }
    }
    set(best_kt);
  }
  if (chosen) *chosen = P->nn_threads;
  NPG_HIP(hipStreamSynchronize(P->stream));
  return NPG_OK;
}

npg_status npg_tune_mlp(npg_plan* P, int32_t nch, int32_t* chosen, int32_t* cand, float* ms) {
  CHECK_ARG(P, "plan is NULL");
  const int tc = P->cfg.precision == NPG_PREC_BF16 ? npg_mlp_bf16_frames() : 0;
  const int n_min = tc > 0 ? (P->T + tc - 1) / tc : 1;
  CHECK_ARG(nch == 0 || (nch >= n_min && nch <= P->T),
            "nch must be 0 or a chunk count in [" + std::to_string(n_min) + ", T]");
  npg_graph_reset(P);  // a captured step holds the old launch shape
  for (int k = 0; k < 4; ++k) {
    if (cand) cand[k] = 0;
    if (ms) ms[k] = 0.f;
  }
  if (nch != 0) {
    TRY(set_mlp_chunks(P, nch));
  } else {
    int nvb = 0, h = 1, g = 0;
    npg_mlp_schedule(P->V, P->T, P->n_cu, tc, &nvb, &h, &g);
    std::vector<int> c = {h};
    for (int n : {std::max(n_min, h / 2), std::min(P->T, 2 * h), std::min(P->T, 4 * h)})
      if (std::find(c.begin(), c.end(), n) == c.end()) c.push_back(n);
    // the plan's current decoder input and deformed vertices (the latter as
    // the upstream gradient: finite values of the right shape)
    NPG_HIP(npg_launch_encode_fwd(P, P->params, P->z));
    NPG_HIP(npg_launch_decode_fwd(P, P->params, P->z, P->xhat, nullptr, P->act));
    float best = 0.f;
    int best_n = h;
    for (size_t k = 0; k < c.size(); ++k) {
      TRY(set_mlp_chunks(P, c[k]));
      float t = 0.f;
      TRY(time_calls(
          P,
          [&]() -> npg_status {
            NPG_HIP(npg_launch_decode_bwd(P, P->params, P->z, P->xhat, P->grad, P->gz, P->act));
            return NPG_OK;
          },
          &t));
      if (cand) cand[k] = c[k];
      if (ms) ms[k] = t;
      if (k == 0 || t < best) {
        best = t;
        best_n = c[k];
      }
    }
    TRY(set_mlp_chunks(P, best_n));
  }
  if (chosen) *chosen = P->mlp_nch;
  NPG_HIP(hipStreamSynchronize(P->stream));
  return NPG_OK;
}

npg_status npg_tune_cg(npg_plan* P, int32_t zs, int32_t* chosen, float* ms) {
  CHECK_ARG(P, "plan is NULL");
  CHECK_ARG(zs == 0 || zs == 32 || zs == 64 || zs == 128, "zs must be 0, 32, 64 or 128");
  CHECK_ARG(P->cfg.precond == NPG_PRECOND_CG, "npg_tune_cg needs the CG preconditioner");
  npg_graph_reset(P);  // a captured step holds the old work-group table
  if (ms)
    for (int k = 0; k < 3; ++k) ms[k] = 0.f;
  auto set = [&](int z) -> npg_status {
    NPG_HIP(hipStreamSynchronize(P->stream));
    npg_cg_free(P);
    P->cg_zs = z;
    return npg_cg_setup(P);
  };
  if (zs != 0) {
    TRY(set(zs));
  } else {
    if (!P->d_scal) NPG_HIP(hipMalloc(&P->d_scal, sizeof(NpgStepScal)));
    const int cand[3] = {32, 64, 128};
    const int iters[2] = {4, 4};
    float best = 0.f;
    int best_z = 64;
    for (int k = 0; k < 3; ++k) {
      TRY(set(cand[k]));
      // a fixed number of iterations of both solves on a non-zero right-hand
      // side (the gradient buffer is workspace between steps)
      hipLaunchKernelGGL(k_fill_pattern, dim3((unsigned)((P->n_grid_params + 255) / 256)), dim3(256), 0,
                         P->stream, P->grad, P->n_grid_params);
      NPG_HIP(hipGetLastError());
      float t = 0.f;
      TRY(time_calls(P, [&] { return npg_run_precond_cg_fixed(P, P->grad, iters, &P->d_scal->cg_state); }, &t));
      if (ms) ms[k] = t;
      if (k == 0 || t < best) {
        best = t;
        best_z = cand[k];
      }
    }
    TRY(set(best_z));
  }
  if (chosen) *chosen = P->cg_zs;
  NPG_HIP(hipStreamSynchronize(P->stream));
  return NPG_OK;
}

}  // extern "C"
