// ms_batch.hip -- uneven batches: environments of several models stepped
// together.
//
// Each model keeps its own step kernels (its own tables, LDS block and
// register budget), all on the stream the batch gives the model (a split
// step's second stream is not used here: the batch's own streams provide
// the concurrency). The kernels are issued either concurrently, each on an
// internal stream of its own forked from the caller's stream and joined
// back, so the GPU runs the models' envs side by side, or serially on the
// caller's stream (a model whose envs fill the GPU runs no slower alone, and
// kernels with different LDS blocks sharing a CU can leave part of its LDS
// idle). The launches are captured once as a HIP graph per argument set and
// replayed, one graph launch per rollout. The autotuner times, per model,
// each envs-per-workgroup choice, and for the whole batch the three issue
// modes, and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ms.h"
#include "ms_step_types.h"

struct ms_batch {
  std::vector<ms_model *> models;
  std::vector<int> n_env;
  std::vector<int> wpg;        // envs per workgroup per model (0: most resident envs)
  int issue = MS_ISSUE_CONCURRENT;  // an MS_ISSUE_* mode
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done;
  hipEvent_t fork = nullptr;
  hipStream_t cap = nullptr;  // graphs are recorded here (any caller stream, even the null one)
  // cached graph of the last argument set
  std::vector<unsigned char> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

thread_local std::string b_err;

ms_status bfail(ms_status s, const std::string &m) {
  b_err = m;
  return s;
}

ms_status bhip(hipError_t e, const char *what) {
  if (e != hipSuccess) return bfail(MS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return MS_OK;
}

void drop_graph(ms_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->key.clear();
}

// issue order of the models
std::vector<int> order(const ms_batch *b) {
  std::vector<int> o(b->models.size());
  for (size_t i = 0; i < o.size(); ++i) o[i] = (int)i;
  if (b->issue != MS_ISSUE_CONCURRENT) {
    auto work = [&](int i) {
      const ms::Tables &t = b->models[i]->t;
      return (double)b->n_env[i] * (double)(t.nv * t.nv + 20 * t.n_mus);
    };
    std::stable_sort(o.begin(), o.end(), [&](int a, int c) { return work(a) > work(c); });
  }
  return o;
}

// one rollout per model: serially on st, or forked onto the model's own
// stream and joined back
ms_status issue(ms_batch *b, const ms_batch_state *s, const ms_excitation *exc, int n_steps,
                const ms_step_opts *opts, hipStream_t st) {
  if (b->issue == MS_ISSUE_SERIAL) {
    for (int i : order(b)) {
      ms_status r = rollout_impl(b->models[i], b->n_env[i], s[i].q, s[i].qd, s[i].act,
                                 s[i].status, &exc[i], n_steps, opts, b->wpg[i], st, nullptr,
                                 true);
      if (r != MS_OK)
        return bfail(r, std::string("model ") + std::to_string(i) + ": " + ms_last_error());
    }
    return MS_OK;
  }
  ms_status r = bhip(hipEventRecord(b->fork, st), "event record");
  if (r != MS_OK) return r;
  for (int i : order(b)) {
    r = bhip(hipStreamWaitEvent(b->streams[i], b->fork, 0), "stream wait");
    if (r != MS_OK) return r;
    r = rollout_impl(b->models[i], b->n_env[i], s[i].q, s[i].qd, s[i].act, s[i].status, &exc[i],
                     n_steps, opts, b->wpg[i], b->streams[i], nullptr, true);
    if (r != MS_OK) return bfail(r, std::string("model ") + std::to_string(i) + ": " + ms_last_error());
    r = bhip(hipEventRecord(b->done[i], b->streams[i]), "event record");
    if (r != MS_OK) return r;
    r = bhip(hipStreamWaitEvent(st, b->done[i], 0), "stream wait");
    if (r != MS_OK) return r;
  }
  return MS_OK;
}

std::vector<unsigned char> make_key(const ms_batch *b, const ms_batch_state *s,
                                    const ms_excitation *exc, int n_steps,
                                    const ms_step_opts *opts) {
  std::vector<unsigned char> k;
  auto put = [&](const void *p, size_t n) {
    const unsigned char *c = (const unsigned char *)p;
    k.insert(k.end(), c, c + n);
  };
  const size_t nm = b->models.size();
  put(s, nm * sizeof(ms_batch_state));
  put(exc, nm * sizeof(ms_excitation));
  put(&n_steps, sizeof n_steps);
  put(opts, sizeof *opts);
  put(b->wpg.data(), nm * sizeof(int));
  put(&b->issue, sizeof(int));
  return k;
}

// record the batch's launches for these arguments as the batch's graph
// (replacing any), on the internal capture stream
ms_status capture(ms_batch *b, const ms_batch_state *s, const ms_excitation *exc, int n_steps,
                  const ms_step_opts *opts) {
  drop_graph(b);
  // split-schedule workspaces are allocated before the capture, never in it
  for (size_t i = 0; i < b->models.size(); ++i) {
    if (effective_schedule(b->models[i]) != MS_SCHED_SPLIT) continue;
    const ms_status rs = reserve_split(b->models[i], b->n_env[i], nullptr);
    if (rs != MS_OK) return bfail(rs, std::string("model ") + std::to_string(i) + ": " + ms_last_error());
  }
  ms_status r = bhip(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal),
                     "begin capture");
  if (r != MS_OK) return r;
  ms_status ri = issue(b, s, exc, n_steps, opts, b->cap);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap, &g);
  if (ri != MS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return ri;
  }
  r = bhip(e, "end capture");
  if (r != MS_OK) return r;
  b->graph = g;
  r = bhip(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "graph instantiate");
  if (r != MS_OK) drop_graph(b);
  return r;
}

}  // namespace

extern "C" {

const char *ms_batch_last_error(void) { return b_err.c_str(); }

ms_status ms_batch_create(ms_model *const *models, const int32_t *n_env, int32_t n_models,
                          ms_batch **out) {
  b_err.clear();
  if (!models || !n_env || !out || n_models <= 0) return bfail(MS_E_ARG, "bad arguments");
  *out = nullptr;
  ms_batch *b = new ms_batch();
  for (int i = 0; i < n_models; ++i) {
    if (!models[i] || n_env[i] <= 0) {
      delete b;
      return bfail(MS_E_ARG, "NULL model or n_env <= 0");
    }
    b->models.push_back(models[i]);
    b->n_env.push_back(n_env[i]);
    b->wpg.push_back(0);
  }
  hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  for (int i = 0; i < n_models && e == hipSuccess; ++i) {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) b->streams.push_back(s);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->done.push_back(ev);
  }
  if (e != hipSuccess) {
    ms_batch_destroy(b);
    return bhip(e, "batch streams");
  }
  *out = b;
  return MS_OK;
}

void ms_batch_destroy(ms_batch *b) {
  if (!b) return;
  drop_graph(b);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->done) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

ms_status ms_batch_rollout(ms_batch *b, const ms_batch_state *states, const ms_excitation *exc,
                           int32_t n_steps, const ms_step_opts *opts, void *stream) {
  b_err.clear();
  if (!b || !states || !exc || !opts) return bfail(MS_E_ARG, "NULL argument");
  if (n_steps < 0) return bfail(MS_E_ARG, "n_steps must be >= 0");
  if (n_steps == 0) return MS_OK;
  hipStream_t st = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  ms_status r = bhip(hipStreamIsCapturing(st, &cs), "capture status");
  if (r != MS_OK) return r;
  if (cs != hipStreamCaptureStatusNone) return issue(b, states, exc, n_steps, opts, st);
  std::vector<unsigned char> key = make_key(b, states, exc, n_steps, opts);
  if (!b->exec || key != b->key) {
    r = capture(b, states, exc, n_steps, opts);
    if (r != MS_OK) return r;
    b->key = key;
  }
  return bhip(hipGraphLaunch(b->exec, st), "graph launch");
}

ms_status ms_batch_autotune(ms_batch *b, const ms_batch_state *states, const ms_excitation *exc,
                            int32_t n_probe, const ms_step_opts *opts, void *stream) {
  b_err.clear();
  if (!b || !states || !exc || !opts || n_probe <= 0) return bfail(MS_E_ARG, "bad arguments");
  hipStream_t st = (hipStream_t)stream;
  const int nm = (int)b->models.size();
  // scratch copies of the states (and AR(1) noise states), refreshed before
  // every probe so each probe starts from the caller's state
  std::vector<void *> owned;
  auto dup = [&](const void *src, size_t bytes, void **dst) -> ms_status {
    *dst = nullptr;
    if (!src || bytes == 0) return MS_OK;
    if (hipMalloc(dst, bytes) != hipSuccess) return bfail(MS_E_ALLOC, "autotune scratch");
    owned.push_back(*dst);
    return MS_OK;
  };
  std::vector<ms_batch_state> sc(nm);
  std::vector<ms_excitation> ec(exc, exc + nm);
  std::vector<size_t> bq(nm), bqd(nm), ba(nm), bs(nm), bx(nm);
  ms_status r = MS_OK;
  for (int i = 0; i < nm && r == MS_OK; ++i) {
    const ms::Tables &t = b->models[i]->t;
    const size_t E = (size_t)b->n_env[i];
    bq[i] = 4 * E * t.nq; bqd[i] = 4 * E * t.nv; ba[i] = 4 * E * t.n_mus; bs[i] = 4 * E;
    bx[i] = exc[i].kind == MS_EXC_AR1 ? 4 * E * t.n_mus : 0;
    void *p = nullptr;
    if ((r = dup(states[i].q, bq[i], &p)) == MS_OK) sc[i].q = (float *)p;
    if (r == MS_OK && (r = dup(states[i].qd, bqd[i], &p)) == MS_OK) sc[i].qd = (float *)p;
    if (r == MS_OK && (r = dup(states[i].act, ba[i], &p)) == MS_OK) sc[i].act = (float *)p;
    if (r == MS_OK && (r = dup(states[i].status, bs[i], &p)) == MS_OK) sc[i].status = (uint32_t *)p;
    if (r == MS_OK && (r = dup(exc[i].x, bx[i], &p)) == MS_OK) ec[i].x = (float *)p;
  }
  auto refresh = [&](int i) -> ms_status {
    hipError_t e = hipSuccess;
    const std::pair<const void *, void *> cp[5] = {{states[i].q, sc[i].q}, {states[i].qd, sc[i].qd},
                                                   {states[i].act, sc[i].act},
                                                   {states[i].status, sc[i].status},
                                                   {exc[i].x, ec[i].x}};
    const size_t by[5] = {bq[i], bqd[i], ba[i], bs[i], bx[i]};
    for (int k = 0; k < 5 && e == hipSuccess; ++k)
      if (cp[k].first && cp[k].second && by[k])
        e = hipMemcpyAsync(cp[k].second, cp[k].first, by[k], hipMemcpyDeviceToDevice, st);
    return bhip(e, "autotune refresh");
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (r == MS_OK) r = bhip(hipEventCreate(&e0), "event");
  if (r == MS_OK) r = bhip(hipEventCreate(&e1), "event");
  auto timed = [&](auto &&fn, float *ms) -> ms_status {
    ms_status q = bhip(hipEventRecord(e0, st), "event record");
    if (q == MS_OK) q = fn();
    if (q == MS_OK) q = bhip(hipEventRecord(e1, st), "event record");
    if (q == MS_OK) q = bhip(hipEventSynchronize(e1), "event sync");
    if (q == MS_OK) q = bhip(hipEventElapsedTime(ms, e0, e1), "elapsed");
    return q;
  };
  // 1. per model, alone: envs per workgroup
  constexpr int kReps = 3;
  const int choices[3] = {1, 2, 4};
  for (int i = 0; i < nm && r == MS_OK; ++i) {
    float best = 1e30f;
    int wbest = 1;
    for (int w : choices) {
      if (b->models[i]->t.lt.size() * 4 + (size_t)w * b->models[i]->t.lds_bytes > 160 * 1024)
        continue;
      for (int rep = 0; rep < kReps && r == MS_OK; ++rep) {  // fastest of kReps probes
        float t_ms = 0.f;
        r = refresh(i);
        if (r == MS_OK)
          r = timed([&] {
            return rollout_impl(b->models[i], b->n_env[i], sc[i].q, sc[i].qd, sc[i].act,
                                sc[i].status, &ec[i], n_probe, opts, w, st, nullptr, true);
          }, &t_ms);
        if (r == MS_OK && t_ms < best) {
          best = t_ms;
          wbest = w;
        }
      }
    }
    b->wpg[i] = wbest;
  }
  // 2. the whole batch, replayed as the graph a rollout launches: issue mode
  // by the mean of kReps replays after one warm-up (concurrent kernels vary
  // from one replay to the next)
  float t_mode[3] = {1e30f, 1e30f, 1e30f};
  for (int o = 0; o < 3 && r == MS_OK; ++o) {
    b->issue = o;
    r = capture(b, sc.data(), ec.data(), n_probe, opts);
    float sum = 0.f;
    for (int rep = 0; rep <= kReps && r == MS_OK; ++rep) {
      float t_ms = 0.f;
      for (int i = 0; i < nm && r == MS_OK; ++i) r = refresh(i);
      if (r == MS_OK)
        r = timed([&] { return bhip(hipGraphLaunch(b->exec, st), "graph launch"); }, &t_ms);
      if (rep > 0) sum += t_ms;
    }
    if (r == MS_OK) t_mode[o] = sum / kReps;
  }
  // concurrent replays vary by a few percent from one to the next (the
  // dispatcher's interleaving of workgroups of different kernels): a
  // concurrent mode is kept only if it beats serial by more than 2 %
  const int fast = t_mode[0] <= t_mode[1] ? 0 : 1;
  b->issue = t_mode[fast] < 0.98f * t_mode[MS_ISSUE_SERIAL] ? fast : MS_ISSUE_SERIAL;
  (void)hipStreamSynchronize(st);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (void *p : owned) (void)hipFree(p);
  drop_graph(b);
  return r;
}

ms_status ms_batch_config(const ms_batch *b, int32_t *env_per_wg, int32_t *issue_mode) {
  if (!b || !env_per_wg || !issue_mode) return bfail(MS_E_ARG, "NULL argument");
  for (size_t i = 0; i < b->wpg.size(); ++i) env_per_wg[i] = b->wpg[i];
  *issue_mode = b->issue;
  return MS_OK;
}

ms_status ms_batch_set_config(ms_batch *b, const int32_t *env_per_wg, int32_t issue_mode) {
  if (!b || !env_per_wg) return bfail(MS_E_ARG, "NULL argument");
  if (issue_mode < MS_ISSUE_CONCURRENT || issue_mode > MS_ISSUE_SERIAL)
    return bfail(MS_E_ARG, "unknown issue mode");
  for (size_t i = 0; i < b->wpg.size(); ++i) {
    const int w = env_per_wg[i];
    if (w != 0 && w != 1 && w != 2 && w != 4)
      return bfail(MS_E_ARG, "envs per workgroup must be 0 (most resident envs), 1, 2 or 4");
    if (b->models[i]->t.lt.size() * 4 + (size_t)w * b->models[i]->t.lds_bytes > 160 * 1024)
      return bfail(MS_E_UNSUPPORTED, "workgroup LDS would exceed 160 KiB");
  }
  for (size_t i = 0; i < b->wpg.size(); ++i) b->wpg[i] = env_per_wg[i];
  b->issue = issue_mode;
  drop_graph(b);
  return MS_OK;
}

}  // extern "C"
