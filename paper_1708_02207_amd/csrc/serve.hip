// Continuous-batching likelihood server (C ABI in include/hdd.h).
//
// One HDD handle, one HIP stream and one worker thread per served mesh size.
// Requests (a parameter sample's kappa, its observation sites and
// observations) queue per mesh; whenever a mesh's handle is free its worker
// takes every waiting request up to the mesh's slot count as one batch:
// Leaves to Root for all of them, then the sample-specific point values and
// Gaussian log-likelihoods (Section 1.2).  Batches of different meshes run
// concurrently on their own streams, so requests that arrive while others
// are on the GPU are admitted as soon as a slot frees up.
//
// HBM admission: a mesh's device workspace (all factors of a full batch) is
// allocated when its first batch is admitted and counted against the
// server's budget.  When a batch needs a workspace that does not fit, idle
// meshes' workspaces are released, least recently used first; if that is
// not enough the batch waits until running batches finish.  A mesh whose
// single-sample workspace exceeds the budget is refused at creation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hdd.h"
#include "trace.hpp"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  int64_t id = 0;
  int mesh = 0;
  std::vector<double> kappa, xy, y;
  double sigma = 1.0;
  std::vector<double> values;
  double loglik = 0.0;
  int status = HDD_OK;
  bool done = false;
  double t_submit = 0.0, t_start = 0.0, t_done = 0.0;
  int batch = 0;
};

struct Mesh {
  int n = 0, nc = 0, slots = 0;
  hdd_opts opts{};
  hdd_handle h = nullptr;    // resident handle (null while evicted)
  void* ws = nullptr;        // its device workspace
  size_t ws_bytes = 0;       // workspace of a full batch
  bool busy = false;         // a batch is running on the handle
  double last_used = 0.0;
  hipStream_t st = nullptr;
  double* pinned = nullptr;  // kappa of one batch, [slots][nc][nc][2]
  std::vector<double> f;     // nodal right-hand side, [(nc+1)^2]
  std::deque<std::shared_ptr<Request>> queue;
  std::thread worker;
  int64_t batches = 0;
};

}  // namespace

struct hdd_server {
  int device = 0;
  std::vector<std::unique_ptr<Mesh>> meshes;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_mem;
  double budget = 0.0;         // bytes for all workspaces (0: no limit)
  size_t used = 0;             // bytes of resident workspaces
  int64_t evictions = 0, creations = 0;
  std::unordered_map<int64_t, std::shared_ptr<Request>> reqs;
  int64_t next_id = 1, submitted = 0, completed = 0;
  bool stop = false;
};

namespace {

// Releases a mesh's handle and workspace (the mesh is idle).
void release_workspace(Mesh* m) {
  if (m->h) hdd_destroy(m->h);
  if (m->ws) (void)hipFree(m->ws);
  m->h = nullptr;
  m->ws = nullptr;
}

// Makes mesh m's handle resident within the budget (lk holds S->mu):
// evicts idle meshes, least recently used first, or waits for running
// batches.  Returns an HDD code; on success m->h is valid and m->busy set.
int admit(hdd_server* S, Mesh* m, std::unique_lock<std::mutex>& lk) {
  for (;;) {
    if (S->stop) return HDD_ESTATE;
    if (m->h) {
      m->busy = true;
      return HDD_OK;
    }
    if (S->budget <= 0.0 || double(S->used + m->ws_bytes) <= S->budget) break;
    Mesh* victim = nullptr;
    for (auto& o : S->meshes)
      if (o.get() != m && o->h && !o->busy && (!victim || o->last_used < victim->last_used)) victim = o.get();
    if (victim) {
      // free it outside the lock; nobody else touches an idle mesh's handle
      // while its worker sleeps (the worker re-admits it first)
      hdd_handle vh = victim->h;
      void* vws = victim->ws;
      victim->h = nullptr;
      victim->ws = nullptr;
      lk.unlock();
      hdd_destroy(vh);
      (void)hipFree(vws);
      lk.lock();
      S->used -= victim->ws_bytes;
      S->evictions += 1;
      continue;
    }
    S->cv_mem.wait(lk);  // every resident mesh is running a batch
  }
  S->used += m->ws_bytes;
  m->busy = true;
  lk.unlock();
  int st = HDD_OK;
  if (hipMalloc(&m->ws, m->ws_bytes) != hipSuccess) {
    m->ws = nullptr;
    st = HDD_ENOMEM;
  }
  if (st == HDD_OK) st = hdd_create(&m->opts, m->slots, m->st, m->ws, m->ws_bytes, &m->h);
  lk.lock();
  if (st != HDD_OK) {
    if (m->ws) (void)hipFree(m->ws);
    m->ws = nullptr;
    m->h = nullptr;
    m->busy = false;
    S->used -= m->ws_bytes;
    S->cv_mem.notify_all();
    return st;
  }
  S->creations += 1;
  return HDD_OK;
}

void run_mesh(hdd_server* S, Mesh* m) {
  if (hipSetDevice(S->device) != hipSuccess) return;
  const size_t kn = size_t(m->nc) * m->nc * 2;
  std::vector<std::shared_ptr<Request>> batch;
  std::vector<int32_t> off;
  std::vector<double> xy, y, sig, vals, ll;
  std::vector<int32_t> sstat;
  for (;;) {
    batch.clear();
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !m->queue.empty(); });
      if (S->stop) return;
      // the handle must be resident within the HBM budget
      const int adm = admit(S, m, lk);
      if (adm != HDD_OK) {
        if (S->stop) return;
        // the batch's requests fail with the admission code
        while (!m->queue.empty()) {
          auto r = m->queue.front();
          m->queue.pop_front();
          r->status = adm;
          r->done = true;
          S->completed += 1;
        }
        S->cv_done.notify_all();
        continue;
      }
      // up to the slot count, and up to the handle's limit on the sites of
      // one ragged query (a request never exceeds it alone)
      int pts = 0;
      while (!m->queue.empty() && int(batch.size()) < m->slots) {
        const int np = int(m->queue.front()->xy.size() / 2);
        if (!batch.empty() && pts + np > HDD_MAX_QUERY_POINTS) break;
        pts += np;
        batch.push_back(m->queue.front());
        m->queue.pop_front();
      }
    }
    const int B = int(batch.size());
    const double t0 = now_s();
    off.assign(B + 1, 0);
    xy.clear();
    y.clear();
    sig.assign(B, 1.0);
    for (int b = 0; b < B; ++b) {
      const Request& r = *batch[b];
      std::memcpy(m->pinned + b * kn, r.kappa.data(), kn * sizeof(double));
      off[b + 1] = off[b] + int32_t(r.xy.size() / 2);
      xy.insert(xy.end(), r.xy.begin(), r.xy.end());
      if (r.y.empty()) y.insert(y.end(), r.xy.size() / 2, 0.0);
      else y.insert(y.end(), r.y.begin(), r.y.end());
      sig[b] = r.sigma;
    }
    vals.assign(off[B], 0.0);
    ll.assign(B, 0.0);
    sstat.assign(B, HDD_OK);
    // Codes that concern single samples (a failed pivot, a refinement that
    // did not converge) still deliver every sample's values; each request
    // then gets its own sample's status.  Any other code fails the batch.
    auto per_sample = [](int c) { return c == HDD_OK || c == HDD_ENOTSPD || c == HDD_ENOTCONVERGED; };
    hdd::Range rg("served batch n=%d requests=%d", m->n, B);
    int st = hdd_build(m->h, B, m->pinned, m->f.data(), nullptr, HDD_MEM_HOST);
    if (per_sample(st)) st = hdd_query_points_ragged(m->h, off.data(), xy.data(), vals.data(), HDD_MEM_HOST);
    if (per_sample(st)) st = hdd_loglik_ragged(m->h, off.data(), xy.data(), y.data(), sig.data(), 0, ll.data(), HDD_MEM_HOST);
    if (per_sample(st)) {
      const int st2 = hdd_sample_status(m->h, sstat.data());
      if (st2 != HDD_OK) st = st2;
    }
    if (!per_sample(st)) sstat.assign(B, st);
    const double t1 = now_s();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (int b = 0; b < B; ++b) {
        Request& r = *batch[b];
        r.values.assign(vals.begin() + off[b], vals.begin() + off[b + 1]);
        r.loglik = r.y.empty() ? 0.0 : ll[b];
        r.status = sstat[b];
        r.t_start = t0;
        r.t_done = t1;
        r.batch = B;
        r.done = true;
      }
      S->completed += B;
      m->batches += 1;
      m->busy = false;
      m->last_used = now_s();
    }
    S->cv_done.notify_all();
    S->cv_mem.notify_all();
  }
}

void destroy_server(hdd_server* S) {
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  S->cv_mem.notify_all();
  for (auto& m : S->meshes)
    if (m->worker.joinable()) m->worker.join();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    for (auto& kv : S->reqs)
      if (!kv.second->done) {
        kv.second->status = HDD_ESTATE;
        kv.second->done = true;
      }
  }
  S->cv_done.notify_all();
  for (auto& m : S->meshes) {
    release_workspace(m.get());
    if (m->pinned) (void)hipHostFree(m->pinned);
    if (m->st) (void)hipStreamDestroy(m->st);
  }
  delete S;
}

}  // namespace

extern "C" {

int hdd_server_create(const hdd_server_opts* o, const double* const* f, hdd_server_t* out) {
  if (!o || !out || o->n_meshes < 1 || o->n_meshes > HDD_SERVER_MAX_MESHES || o->slots < 0 || o->hbm_budget < 0.0)
    return HDD_EINVAL;
  for (int i = 0; i < 7; ++i)
    if (o->reserved[i] != 0) return HDD_EINVAL;
  if (o->max_refine < 0) return HDD_EINVAL;
  *out = nullptr;
  hdd_server* S = new (std::nothrow) hdd_server;
  if (!S) return HDD_ENOMEM;
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return HDD_EDEVICE;
  }
  std::vector<hdd_opts> opts(o->n_meshes);
  for (int i = 0; i < o->n_meshes; ++i) {
    int st = hdd_default_opts(o->n[i], o->precision, &opts[i]);
    if (st == HDD_OK && o->leaf[i] > 0) opts[i].leaf = o->leaf[i];
    if (st == HDD_OK && o->max_refine > 0) opts[i].max_refine = o->max_refine;
    // with a finite budget workspaces are released while other meshes run:
    // a release may synchronize the device, which must not meet another
    // mesh's graph capture, so those handles issue their launches eagerly
    if (st == HDD_OK && o->hbm_budget > 0.0) opts[i].flags |= HDD_FLAG_NO_GRAPH;
    if (st != HDD_OK) {
      delete S;
      return st;
    }
  }
  // slots per mesh: as requested (default 32), halved while a mesh's
  // full-batch workspace alone exceeds the budget; a mesh whose single-sample
  // workspace exceeds it is refused
  const int slots0 = o->slots > 0 ? o->slots : 32;
  std::vector<int> mslots(o->n_meshes, slots0);
  std::vector<size_t> wbytes(o->n_meshes, 0);
  for (int i = 0; i < o->n_meshes; ++i) {
    for (;;) {
      size_t b = 0;
      const int st = hdd_workspace_size(&opts[i], mslots[i], &b);
      if (st != HDD_OK) {
        delete S;
        return st;
      }
      wbytes[i] = b;
      if (o->hbm_budget <= 0.0 || double(b) <= o->hbm_budget) break;
      if (mslots[i] == 1) {
        delete S;
        return HDD_ENOMEM;
      }
      mslots[i] /= 2;
    }
  }
  S->budget = o->hbm_budget;
  for (int i = 0; i < o->n_meshes; ++i) {
    auto m = std::make_unique<Mesh>();
    m->n = o->n[i];
    m->nc = o->n[i] + 1;
    m->slots = mslots[i];
    m->opts = opts[i];
    m->ws_bytes = wbytes[i];
    const size_t nf = size_t(m->nc + 1) * (m->nc + 1);
    if (f && f[i]) m->f.assign(f[i], f[i] + nf);
    else m->f.assign(nf, 1.0);
    int st = HDD_OK;
    if (hipStreamCreateWithFlags(&m->st, hipStreamNonBlocking) != hipSuccess) st = HDD_EDEVICE;
    if (st == HDD_OK && hipHostMalloc(reinterpret_cast<void**>(&m->pinned),
                                      size_t(m->slots) * m->nc * m->nc * 2 * sizeof(double)) != hipSuccess)
      st = HDD_ENOMEM;
    S->meshes.push_back(std::move(m));
    if (st != HDD_OK) {
      destroy_server(S);
      return st;
    }
  }
  for (auto& m : S->meshes) m->worker = std::thread(run_mesh, S, m.get());
  *out = S;
  return HDD_OK;
}

int hdd_server_slots(hdd_server_t S, int32_t* slots) {
  if (!S || !slots || S->meshes.empty()) return HDD_EINVAL;
  *slots = S->meshes[0]->slots;
  for (auto& m : S->meshes) *slots = std::min(*slots, m->slots);
  return HDD_OK;
}

int hdd_server_memory(hdd_server_t S, int64_t* out) {
  if (!S || !out) return HDD_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  int64_t resident = 0;
  for (auto& m : S->meshes) resident += m->h ? 1 : 0;
  out[0] = int64_t(S->used);
  out[1] = resident;
  out[2] = S->evictions;
  out[3] = S->creations;
  return HDD_OK;
}

int hdd_server_submit(hdd_server_t S, int32_t mesh, const double* kappa, int32_t n_pts, const double* xy,
                      const double* y, double sigma, int64_t* id) {
  if (!S || !kappa || !xy || !id || mesh < 0 || mesh >= int(S->meshes.size()) || n_pts < 1 ||
      n_pts > HDD_SERVER_MAX_POINTS || !(sigma > 0.0))
    return HDD_EINVAL;
  Mesh* m = S->meshes[mesh].get();
  const size_t kn = size_t(m->nc) * m->nc * 2;
  for (size_t i = 0; i < kn; ++i)
    if (!(kappa[i] > 0.0) || !(kappa[i] < 1e300)) return HDD_EINVAL;
  for (int p = 0; p < 2 * n_pts; ++p)
    if (!(xy[p] >= 0.0 && xy[p] <= 1.0)) return HDD_EINVAL;
  auto r = std::make_shared<Request>();
  r->mesh = mesh;
  r->kappa.assign(kappa, kappa + kn);
  r->xy.assign(xy, xy + 2 * n_pts);
  if (y) r->y.assign(y, y + n_pts);
  r->sigma = sigma;
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return HDD_ESTATE;
    r->id = S->next_id++;
    S->reqs[r->id] = r;
    m->queue.push_back(r);
    S->submitted += 1;
  }
  S->cv_work.notify_all();
  *id = r->id;
  return HDD_OK;
}

int hdd_server_poll(hdd_server_t S, int64_t id, int32_t* done) {
  if (!S || !done) return HDD_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return HDD_EINVAL;
  *done = it->second->done ? 1 : 0;
  return HDD_OK;
}

int hdd_server_result(hdd_server_t S, int64_t id, double* values, double* loglik, double* times) {
  if (!S) return HDD_EINVAL;
  std::shared_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return HDD_EINVAL;
    r = it->second;
    S->cv_done.wait(lk, [&] { return r->done; });
    S->reqs.erase(it);
  }
  if (values) std::memcpy(values, r->values.data(), r->values.size() * sizeof(double));
  if (loglik) *loglik = r->loglik;
  if (times) {
    times[0] = r->t_start - r->t_submit;
    times[1] = r->t_done - r->t_start;
    times[2] = r->t_done - r->t_submit;
    times[3] = double(r->batch);
  }
  return r->status;
}

int hdd_server_stats(hdd_server_t S, int64_t* out) {
  if (!S || !out) return HDD_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  int64_t queued = 0, batches = 0;
  for (auto& m : S->meshes) {
    queued += int64_t(m->queue.size());
    batches += m->batches;
  }
  out[0] = S->submitted;
  out[1] = S->completed;
  out[2] = batches;
  out[3] = queued;
  return HDD_OK;
}

int hdd_server_destroy(hdd_server_t S) {
  if (!S) return HDD_EINVAL;
  destroy_server(S);
  return HDD_OK;
}

}  // extern "C"
