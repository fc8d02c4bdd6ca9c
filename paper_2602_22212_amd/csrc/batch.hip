// Batched sequences (many independent reconstructions at once): one plan per
// sequence, each with its own grids, MLP, optimizer state and HIP stream
// (default priority). A batch step runs every sequence's step from its own
// host thread, so the sequences' kernels overlap on the GPU; each sequence's
// step synchronizes only its own stream (CG convergence tests, the
// non-finite flag). Results are those of the sequence's own npg_step.
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

struct npg_batch {
  std::vector<npg_plan*> plans;
  std::vector<hipStream_t> streams;
  int device = 0;
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

void destroy(npg_batch* B) {
  for (npg_plan* P : B->plans)
    if (P) npg_plan_destroy(P);
  for (hipStream_t s : B->streams)
    if (s) hipStreamDestroy(s);
  delete B;
}

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

npg_status npg_batch_destroy(npg_batch* B) {
  if (!B) return NPG_OK;
  destroy(B);
  return NPG_OK;
}

}  // extern "C"
