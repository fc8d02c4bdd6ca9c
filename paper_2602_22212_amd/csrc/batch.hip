// Batched sequences (many independent reconstructions at once): one plan per
// sequence, each with its own grids, MLP, optimizer state and HIP stream
// (default priority). The eager batch step runs every sequence's step from
// its own host thread, so the sequences' kernels overlap on the GPU; each
// sequence's step synchronizes only its own stream (CG convergence tests,
// the non-finite flag). The graph batch step replays one HIP graph whose
// independent branches are the sequences' recorded steps (each a child graph
// of its plan's npg_step_graph recording). Results are those of the
// sequence's own npg_step.
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

struct npg_batch {
  std::vector<npg_plan*> plans;
  std::vector<hipStream_t> streams;
  int device = 0;
  // graph batch step: the batch graph, the recordings it was built from
  // (plan graph generations), its launch stream and per-plan events
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int64_t> built_gen;
  hipStream_t bstream = nullptr;
  std::vector<hipEvent_t> ev;
  int graph_mode = 0;  // NPG_BATCH_ONE_GRAPH or NPG_BATCH_GRAPH_PER_STREAM
};

namespace {

int severity(npg_status s) {
  switch (s) {
    case NPG_OK: return 0;
    case NPG_ENOTCONV: return 1;
    case NPG_ENONFINITE: return 2;
    default: return 3;
  }
}

void drop_graph(npg_batch* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
  B->built_gen.clear();
}

void destroy(npg_batch* B) {
  drop_graph(B);
  if (B->bstream) {
    (void)hipStreamSynchronize(B->bstream);
    (void)hipStreamDestroy(B->bstream);
  }
  for (hipEvent_t e : B->ev)
    if (e) (void)hipEventDestroy(e);
  for (npg_plan* P : B->plans)
    if (P) npg_plan_destroy(P);
  for (hipStream_t s : B->streams)
    if (s) hipStreamDestroy(s);
  delete B;
}

npg_status finish_batch(npg_batch* B, int epoch, int n_epochs, double* const* loss_dev,
                        const std::vector<NpgStepScal>& sc, const std::vector<int>& flag);

}  // namespace

extern "C" {

npg_status npg_plan_create_batched(const npg_config* cfg, int32_t n_seq, const int64_t* V, const float* const* xyz,
                                   const float* const* nrm, const int32_t* T, const float* const* pts,
                                   const int64_t* const* frame_off, npg_batch** out) {
  if (!out) return npg_fail(NPG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfg || n_seq < 1 || !V || !xyz || !nrm || !T || !pts || !frame_off)
    return npg_fail(NPG_EINVAL, "need n_seq >= 1 and non-NULL per-sequence arrays");
  npg_batch* B = new npg_batch();
  if (hipGetDevice(&B->device) != hipSuccess) {
    delete B;
    return npg_fail(NPG_EHIP, "hipGetDevice failed");
  }
  for (int k = 0; k < n_seq; ++k) {
    hipStream_t s = nullptr;
    if (hipStreamCreate(&s) != hipSuccess) {
      destroy(B);
      return npg_fail(NPG_EHIP, "stream creation failed for sequence " + std::to_string(k));
    }
    B->streams.push_back(s);
    npg_plan* P = nullptr;
    npg_status st = npg_plan_create(&cfg[k], V[k], xyz[k], nrm[k], T[k], pts[k], frame_off[k], s, &P);
    if (st != NPG_OK) {
      std::string msg = "sequence " + std::to_string(k) + ": " + npg_last_error();
      destroy(B);
      return npg_fail(st, msg);
    }
    B->plans.push_back(P);
  }
  *out = B;
  return NPG_OK;
}

npg_status npg_batch_plan(npg_batch* B, int32_t k, npg_plan** out) {
  if (!B || !out || k < 0 || k >= (int)B->plans.size()) return npg_fail(NPG_EINVAL, "bad batch, index or out");
  *out = B->plans[k];
  return NPG_OK;
}

npg_status npg_batch_step(npg_batch* B, int32_t epoch, int32_t n_epochs, double* const* loss_dev) {
  if (!B) return npg_fail(NPG_EINVAL, "batch is NULL");
  const int n = (int)B->plans.size();
  std::vector<npg_status> st(n, NPG_OK);
  std::vector<std::string> msg(n);
  std::vector<std::thread> workers;
  workers.reserve(n);
  for (int k = 0; k < n; ++k)
    workers.emplace_back([&, k] {
      hipSetDevice(B->device);
      st[k] = npg_step(B->plans[k], epoch, n_epochs, loss_dev ? loss_dev[k] : nullptr, nullptr);
      if (st[k] != NPG_OK) msg[k] = npg_last_error();
    });
  for (auto& w : workers) w.join();
  int worst = 0;
  for (int k = 1; k < n; ++k)
    if (severity(st[k]) > severity(st[worst])) worst = k;
  if (st[worst] != NPG_OK) return npg_fail(st[worst], "sequence " + std::to_string(worst) + ": " + msg[worst]);
  return NPG_OK;
}

npg_status npg_batch_step_graph(npg_batch* B, int32_t epoch, int32_t n_epochs, double* const* loss_dev) {
  if (!B) return npg_fail(NPG_EINVAL, "batch is NULL");
  if (n_epochs < 1 || epoch < 0 || epoch > n_epochs)
    return npg_fail(NPG_EINVAL, "need 0 <= epoch <= n_epochs, n_epochs >= 1");
  const int n = (int)B->plans.size();
  for (int k = 0; k < n; ++k) {
    npg_plan* P = B->plans[k];
    if (P->cfg.w_iso != 0.f && P->n_edges == 0)
      return npg_fail(NPG_EINVAL, "sequence " + std::to_string(k) + ": w_iso > 0 needs the mesh edges");
    const npg_status st = npg_graph_prepare(P);
    if (st != NPG_OK) return npg_fail(st, "sequence " + std::to_string(k) + ": " + npg_last_error());
  }
  std::vector<NpgStepScal> sc(n);
  std::vector<int> flag(n, 0);
  if (B->graph_mode == NPG_BATCH_GRAPH_PER_STREAM) {
    // every sequence's recording replayed on its own stream, all enqueued
    // before the first wait
    for (int k = 0; k < n; ++k) {
      npg_plan* P = B->plans[k];
      npg_status st = npg_graph_set_scalars(P, epoch, n_epochs, P->stream);
      if (st != NPG_OK) return st;
      NPG_HIP(hipGraphLaunch(P->graph_exec, P->stream));
      st = npg_graph_read(P, P->stream, &sc[k], &flag[k]);
      if (st != NPG_OK) return st;
    }
    for (int k = 0; k < n; ++k) NPG_HIP(hipStreamSynchronize(B->plans[k]->stream));
    return finish_batch(B, epoch, n_epochs, loss_dev, sc, flag);
  }
  bool stale = !B->exec || (int)B->built_gen.size() != n;
  for (int k = 0; !stale && k < n; ++k) stale = B->built_gen[k] != B->plans[k]->graph_gen;
  if (stale) {
    drop_graph(B);
    NPG_HIP(hipGraphCreate(&B->graph, 0));
    for (int k = 0; k < n; ++k) {
      hipGraphNode_t node;
      NPG_HIP(hipGraphAddChildGraphNode(&node, B->graph, nullptr, 0, B->plans[k]->graph));
      B->built_gen.push_back(B->plans[k]->graph_gen);
    }
    NPG_HIP(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
  }
  if (!B->bstream) NPG_HIP(hipStreamCreate(&B->bstream));
  if (B->ev.empty()) {
    B->ev.resize(n, nullptr);
    for (auto& e : B->ev) NPG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  hipStream_t s = B->bstream;
  // earlier work enqueued on the sequences' own streams comes first
  for (int k = 0; k < n; ++k) {
    NPG_HIP(hipEventRecord(B->ev[k], B->plans[k]->stream));
    NPG_HIP(hipStreamWaitEvent(s, B->ev[k], 0));
  }
  for (int k = 0; k < n; ++k) {
    const npg_status st = npg_graph_set_scalars(B->plans[k], epoch, n_epochs, s);
    if (st != NPG_OK) return st;
  }
  NPG_HIP(hipGraphLaunch(B->exec, s));
  for (int k = 0; k < n; ++k) {
    const npg_status st = npg_graph_read(B->plans[k], s, &sc[k], &flag[k]);
    if (st != NPG_OK) return st;
  }
  NPG_HIP(hipStreamSynchronize(s));
  return finish_batch(B, epoch, n_epochs, loss_dev, sc, flag);
}

npg_status npg_batch_graph_mode(npg_batch* B, int32_t mode) {
  if (!B) return npg_fail(NPG_EINVAL, "batch is NULL");
  if (mode != NPG_BATCH_ONE_GRAPH && mode != NPG_BATCH_GRAPH_PER_STREAM)
    return npg_fail(NPG_EINVAL, "mode must be NPG_BATCH_ONE_GRAPH or NPG_BATCH_GRAPH_PER_STREAM");
  B->graph_mode = mode;
  return NPG_OK;
}

}  // extern "C"

namespace {
// After the replays have finished: each sequence's step count, outputs and
// status; a sequence whose recorded CG solve stopped short (Adam skipped)
// records more iterations and runs its step again alone.
npg_status finish_batch(npg_batch* B, int epoch, int n_epochs, double* const* loss_dev,
                        const std::vector<NpgStepScal>& sc, const std::vector<int>& flag) {
  const int n = (int)B->plans.size();
  std::vector<npg_status> st(n, NPG_OK);
  std::vector<std::string> msg(n);
  for (int k = 0; k < n; ++k) {
    npg_plan* P = B->plans[k];
    double* loss = loss_dev ? loss_dev[k] : nullptr;
    if (npg_graph_redo(P, sc[k])) {
      if (flag[k]) NPG_HIP(hipMemsetAsync(P->d_flag, 0, 4, P->stream));
      st[k] = npg_step_graph(P, epoch, n_epochs, loss, nullptr);
    } else {
      st[k] = npg_graph_finish(P, sc[k], flag[k], loss, nullptr, P->stream);
    }
    if (st[k] != NPG_OK) msg[k] = npg_last_error();
  }
  int worst = 0;
  for (int k = 1; k < n; ++k)
    if (severity(st[k]) > severity(st[worst])) worst = k;
  if (st[worst] != NPG_OK) return npg_fail(st[worst], "sequence " + std::to_string(worst) + ": " + msg[worst]);
  return NPG_OK;
}
}  // namespace

extern "C" {

npg_status npg_batch_destroy(npg_batch* B) {
  if (!B) return NPG_OK;
  destroy(B);
  return NPG_OK;
}

}  // extern "C"
