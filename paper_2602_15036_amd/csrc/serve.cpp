// Serving: the HIP executor behind the continuous-batching scheduler and the
// litho_serve_* C ABI.
//
// Each slot owns a non-blocking HIP stream (default priority), a completion
// event and one device arena (request I/O buffers plus the imaging workspace),
// grown to the largest request the slot has run; the scheduler counts every
// arena against the HBM budget and releases idle ones when a request would
// not fit otherwise.  Host requests are staged in pinned buffers from a
// server-wide pool: the submitting thread copies the mask (and target) in,
// the slot's stream moves them to the arena and the results back into pinned
// memory, and the polling thread copies them out, so the scheduler thread
// does no bulk host copy.  When the pool reaches its cap
// (LITHO_SERVE_PINNED_MB, default 4096) a request falls back to pageable
// copies through the slot's own staging.  A device-resident request reads and
// writes the caller's device buffers directly.
// Slots run concurrently, so requests of different clip sizes and banks
// overlap on the device; every request keeps the bank's resident kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "litho_internal.hpp"
#include "serve_core.hpp"

namespace litho {
namespace {

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Pinned host buffers, reused across requests (power-of-two size classes).
class PinnedPool {
 public:
  explicit PinnedPool(size_t cap) : cap_(cap) {}
  ~PinnedPool() {
    for (auto &kv : free_) (void)hipHostFree(kv.second);
  }
  // nullptr when the cap would be exceeded or the allocation fails
  void *get(size_t bytes, size_t *cls) {
    size_t c = 4096;
    while (c < bytes) c <<= 1;
    *cls = c;
    std::lock_guard<std::mutex> lk(mu_);
    auto it = free_.find(c);
    if (it != free_.end()) {
      void *p = it->second;
      free_.erase(it);
      return p;
    }
    if (total_ + c > cap_) return nullptr;
    void *p = nullptr;
    if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    total_ += c;
    return p;
  }
  void put(void *p, size_t cls) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    free_.emplace(cls, p);
  }

 private:
  std::mutex mu_;
  std::multimap<size_t, void *> free_;
  size_t total_ = 0, cap_;
};

size_t pinned_cap() {
  const char *e = std::getenv("LITHO_SERVE_PINNED_MB");
  size_t mb = 4096;
  if (e && *e) mb = size_t(std::strtoull(e, nullptr, 10));
  return mb << 20;
}

struct ServeReq {
  litho_bank *bank = nullptr;
  int K_use = 0, mode = 0, n = 0, P = 1, prec = LITHO_PREC_FP32;
  double slope = 0, thr = 0;
  size_t ws_bytes = 0;       // imaging workspace of one clip
  // host I/O through pinned staging (in: mask, target; out: image, grad, loss)
  PinnedPool *pool = nullptr;
  float *p_in = nullptr, *p_out = nullptr;
  size_t in_cls = 0, out_cls = 0;
  // host I/O fallback (pool at its cap): pageable copies
  std::vector<float> mask, target;
  std::vector<float> image, grad;
  double loss = 0;
  // device-resident I/O (d_mask != nullptr)
  const float *d_mask = nullptr, *d_target = nullptr;
  float *d_image = nullptr, *d_grad = nullptr;
  double *d_loss = nullptr;
  bool on_device() const { return d_mask != nullptr; }
  size_t px() const { return size_t(n) * n; }
  // pinned output: image [P][px], grad [px], loss (double, 8-byte aligned)
  size_t out_loss_offset() const { return (px() * (P + 1) + 1) & ~size_t(1); }
  ~ServeReq() {
    if (pool) {
      pool->put(p_in, in_cls);
      pool->put(p_out, out_cls);
    }
  }
};

class HipExecutor final : public serve::Executor {
 public:
  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    char *arena = nullptr;            // device: workspace, then mask, target, image, grad, loss
    size_t arena_bytes = 0;
    size_t host_px = 0;               // pageable-fallback staging capacity (pixels, per plane for image)
    int host_planes = 0;
    float *h_in = nullptr, *h_image = nullptr, *h_grad = nullptr;
    double *h_loss = nullptr;
    std::string error;
  };

  HipExecutor(int nslots, int device) : slots_(size_t(nslots)), device_(device) {}

  ~HipExecutor() override {
    (void)hipSetDevice(device_);
    for (auto &s : slots_) {
      if (s.stream) (void)hipStreamSynchronize(s.stream);
      if (s.arena) (void)hipFree(s.arena);
      free_host(s);
      if (s.done) (void)hipEventDestroy(s.done);
      if (s.stream) (void)hipStreamDestroy(s.stream);
    }
  }

  int init() {
    LITHO_HIP_TRY(hipSetDevice(device_));
    for (auto &s : slots_) {
      LITHO_HIP_TRY(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
      LITHO_HIP_TRY(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
    }
    return LITHO_OK;
  }

  // Device bytes a request needs on its slot: the imaging workspace of one
  // clip, plus its I/O buffers unless they are device-resident.
  static size_t arena_need(size_t ws_bytes, size_t px, int P, bool on_device) {
    if (on_device) return ws_bytes;
    return ws_bytes + align_up(2 * px * sizeof(float)) + align_up(px * P * sizeof(float)) +
           align_up(px * sizeof(float)) + 256;
  }

  int slots() const override { return int(slots_.size()); }
  void thread_init() override { (void)hipSetDevice(device_); }
  size_t held(int si) const override { return slots_[size_t(si)].arena_bytes; }
  void trim(int si) override {
    Slot &s = slots_[size_t(si)];
    if (!s.arena) return;
    (void)hipStreamSynchronize(s.stream);
    (void)hipFree(s.arena);
    s.arena = nullptr;
    s.arena_bytes = 0;
  }

  int launch(serve::Job &job, int si) override {
    auto *r = static_cast<ServeReq *>(job.payload.get());
    Slot &s = slots_[size_t(si)];
    const size_t px = r->px();
    int rc = grow(s, job.footprint);
    if (rc != LITHO_OK) {
      job.error = last_error();
      return rc;
    }
    char *ws = s.arena;
    if (r->on_device()) return run(job, *r, s, ws, r->d_mask, r->d_target, r->d_image, r->d_grad, r->d_loss);
    char *io = s.arena + r->ws_bytes;
    float *d_mask = reinterpret_cast<float *>(io);
    float *d_target = d_mask + px;
    float *d_image = reinterpret_cast<float *>(io + align_up(2 * px * sizeof(float)));
    float *d_grad = reinterpret_cast<float *>(reinterpret_cast<char *>(d_image) + align_up(px * r->P * sizeof(float)));
    double *d_loss = reinterpret_cast<double *>(reinterpret_cast<char *>(d_grad) + align_up(px * sizeof(float)));
    const size_t in_bytes = px * sizeof(float) * (r->mode == 1 ? 2 : 1);
    const float *src = r->p_in;
    if (!src) {
      rc = ensure_host(s, px, r->P);
      if (rc != LITHO_OK) {
        job.error = last_error();
        return rc;
      }
      std::memcpy(s.h_in, r->mask.data(), px * sizeof(float));
      if (r->mode == 1) std::memcpy(s.h_in + px, r->target.data(), px * sizeof(float));
      src = s.h_in;
    }
    if (hipMemcpyAsync(d_mask, src, in_bytes, hipMemcpyHostToDevice, s.stream) != hipSuccess) {
      job.error = "litho_serve: H2D copy failed";
      return LITHO_E_HIP;
    }
    rc = image_call(*r, s, ws, d_mask, d_target, d_image, d_grad, d_loss);
    if (rc != LITHO_OK) {
      job.error = last_error();
      return rc;
    }
    float *o_image = r->p_out ? r->p_out : s.h_image;
    float *o_grad = r->p_out ? r->p_out + px * r->P : s.h_grad;
    double *o_loss = r->p_out ? reinterpret_cast<double *>(r->p_out + r->out_loss_offset()) : s.h_loss;
    bool ok = hipMemcpyAsync(o_image, d_image, px * r->P * sizeof(float), hipMemcpyDeviceToHost, s.stream) ==
              hipSuccess;
    if (r->mode == 1) {
      ok = ok && hipMemcpyAsync(o_grad, d_grad, px * sizeof(float), hipMemcpyDeviceToHost, s.stream) == hipSuccess;
      ok = ok && hipMemcpyAsync(o_loss, d_loss, sizeof(double), hipMemcpyDeviceToHost, s.stream) == hipSuccess;
    }
    ok = ok && hipEventRecord(s.done, s.stream) == hipSuccess;
    if (!ok) {
      job.error = "litho_serve: D2H copy or event record failed";
      return LITHO_E_HIP;
    }
    return LITHO_OK;
  }

  bool ready(int si) override {
    Slot &s = slots_[size_t(si)];
    const hipError_t e = hipEventQuery(s.done);
    if (e == hipErrorNotReady) return false;
    s.error = e == hipSuccess ? "" : hipGetErrorString(e);
    return true;
  }

  int collect(serve::Job &job, int si) override {
    Slot &s = slots_[size_t(si)];
    if (!s.error.empty()) {
      job.error = s.error;
      return LITHO_E_HIP;
    }
    auto *r = static_cast<ServeReq *>(job.payload.get());
    if (r->on_device()) {
      r->loss = std::numeric_limits<double>::quiet_NaN();
      return LITHO_OK;
    }
    if (r->p_out) {
      // results wait in the request's pinned buffer for the polling thread
      if (r->mode == 1) r->loss = *reinterpret_cast<const double *>(r->p_out + r->out_loss_offset());
      return LITHO_OK;
    }
    const size_t px = r->px();
    r->image.assign(s.h_image, s.h_image + px * r->P);
    if (r->mode == 1) {
      r->grad.assign(s.h_grad, s.h_grad + px);
      r->loss = *s.h_loss;
    }
    return LITHO_OK;
  }

 private:
  int run(serve::Job &job, ServeReq &r, Slot &s, char *ws, const float *d_mask, const float *d_target,
          float *d_image, float *d_grad, double *d_loss) {
    int rc = image_call(r, s, ws, d_mask, d_target, d_image, d_grad, d_loss);
    if (rc != LITHO_OK) {
      job.error = last_error();
      return rc;
    }
    if (hipEventRecord(s.done, s.stream) != hipSuccess) {
      job.error = "litho_serve: event record failed";
      return LITHO_E_HIP;
    }
    return LITHO_OK;
  }

  static int image_call(ServeReq &r, Slot &s, char *ws, const float *d_mask, const float *d_target,
                        float *d_image, float *d_grad, double *d_loss) {
    if (r.mode == 1) {
      litho_resist_t res{r.slope, r.thr};
      return image_grad_impl(r.bank, d_mask, 1, r.K_use, d_target, &res, nullptr, d_image, d_loss, d_grad, true,
                             r.prec, s.stream, 0, -1, ws, r.ws_bytes);
    }
    return image_grad_impl(r.bank, d_mask, 1, r.K_use, nullptr, nullptr, nullptr, d_image, nullptr, nullptr, false,
                           r.prec, s.stream, 0, -1, ws, r.ws_bytes);
  }

  // Grows the slot's arena to `bytes` (scheduler thread, slot idle; the
  // scheduler has already counted the growth against the budget).
  int grow(Slot &s, size_t bytes) {
    if (s.arena_bytes >= bytes) return LITHO_OK;
    if (s.arena) {
      (void)hipStreamSynchronize(s.stream);
      (void)hipFree(s.arena);
      s.arena = nullptr;
      s.arena_bytes = 0;
    }
    if (hipMalloc(&s.arena, bytes) != hipSuccess) {
      (void)hipGetLastError();
      s.arena = nullptr;
      set_error("litho_serve: cannot allocate a %zu byte slot arena", bytes);
      return LITHO_E_NOMEM;
    }
    s.arena_bytes = bytes;
    return LITHO_OK;
  }

  static void free_host(Slot &s) {
    for (float *p : {s.h_in, s.h_image, s.h_grad})
      if (p) (void)hipHostFree(p);
    if (s.h_loss) (void)hipHostFree(s.h_loss);
    s.h_in = s.h_image = s.h_grad = nullptr;
    s.h_loss = nullptr;
    s.host_px = 0;
    s.host_planes = 0;
  }

  // Pinned staging of the pageable fallback, grown to px pixels and P planes.
  int ensure_host(Slot &s, size_t px, int P) {
    if (s.host_px >= px && s.host_planes >= P) return LITHO_OK;
    free_host(s);
    if (hipHostMalloc(&s.h_in, 2 * px * sizeof(float), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&s.h_image, px * P * sizeof(float), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&s.h_grad, px * sizeof(float), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&s.h_loss, sizeof(double), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      free_host(s);
      set_error("litho_serve: cannot allocate pinned staging for %zu pixels", px);
      return LITHO_E_NOMEM;
    }
    s.host_px = px;
    s.host_planes = P;
    return LITHO_OK;
  }

  std::vector<Slot> slots_;
  int device_;
};

}  // namespace
}  // namespace litho

struct litho_server {
  std::vector<litho_bank *> banks;
  std::unique_ptr<litho::PinnedPool> pool;
  std::unique_ptr<litho::HipExecutor> ex;
  std::unique_ptr<litho::serve::Scheduler> sched;
};

using namespace litho;

// Imaging workspace of one clip of a request (its slot arena adds the I/O buffers).
static size_t request_workspace(litho_bank *bk, int K_use, int mode, int prec) {
  return plan_call(bk, 1, K_use, mode == 1, mode == 1, prec).per_clip;
}

extern "C" int litho_serve_create(litho_bank_t *const *banks, int n_banks, const litho_serve_cfg_t *cfg,
                                  litho_server_t **out) {
  clear_error();
  if (!out || !banks || n_banks < 1 || !cfg || cfg->max_slots < 1 || cfg->max_slots > 64 || cfg->max_queue < 1 ||
      cfg->hbm_budget == 0) {
    set_error("litho_serve_create: invalid argument");
    return LITHO_E_INVALID;
  }
  *out = nullptr;
  for (int i = 0; i < n_banks; ++i)
    if (!banks[i]) {
      set_error("litho_serve_create: bank %d is NULL", i);
      return LITHO_E_INVALID;
    }
  auto srv = std::make_unique<litho_server>();
  srv->banks.assign(banks, banks + n_banks);
  srv->pool = std::make_unique<PinnedPool>(pinned_cap());
  srv->ex = std::make_unique<HipExecutor>(cfg->max_slots, banks[0]->device);
  LITHO_TRY(srv->ex->init());
  srv->sched = std::make_unique<serve::Scheduler>(srv->ex.get(), cfg->hbm_budget, cfg->max_queue);
  *out = srv.release();
  return LITHO_OK;
}

extern "C" int litho_serve_submit(litho_server_t *srv, const litho_request_t *req, uint64_t *ticket) {
  clear_error();
  if (!srv || !req || !ticket || (!req->h_mask && !req->d_mask)) {
    set_error("litho_serve_submit: NULL argument");
    return LITHO_E_INVALID;
  }
  const bool dev = req->d_mask != nullptr;
  if (dev && (!req->d_image || (req->mode == 1 && (!req->d_target || !req->d_grad)))) {
    set_error("litho_serve_submit: a device-resident request needs d_image (and d_target, d_grad in mode 1)");
    return LITHO_E_INVALID;
  }
  if (req->bank < 0 || req->bank >= int(srv->banks.size())) {
    set_error("litho_serve_submit: bank index %d out of range", req->bank);
    return LITHO_E_INVALID;
  }
  litho_bank *bk = srv->banks[size_t(req->bank)];
  if (req->K_use < 1 || req->K_use > bk->host.K || (req->mode != 0 && req->mode != 1) ||
      (req->mode == 1 && !dev && !req->h_target)) {
    set_error("litho_serve_submit: invalid request (K_use=%d mode=%d)", req->K_use, req->mode);
    return LITHO_E_INVALID;
  }
  LITHO_TRY(check_prec(req->prec, "litho_serve_submit"));
  auto r = std::make_shared<ServeReq>();
  r->bank = bk;
  r->K_use = req->K_use;
  r->mode = req->mode;
  r->prec = req->prec;
  r->n = bk->host.n;
  r->P = bk->host.n_focus;
  r->slope = req->slope;
  r->thr = req->threshold;
  const size_t px = size_t(r->n) * r->n;
  r->ws_bytes = request_workspace(bk, req->K_use, req->mode, req->prec);
  if (dev) {
    r->d_mask = req->d_mask;
    r->d_target = req->mode == 1 ? req->d_target : nullptr;
    r->d_image = req->d_image;
    r->d_grad = req->mode == 1 ? req->d_grad : nullptr;
    r->d_loss = req->mode == 1 ? req->d_loss : nullptr;
  } else {
    // copy the inputs on this (the caller's) thread, into pinned staging when
    // the pool has room, else into pageable memory
    r->pool = srv->pool.get();
    const size_t in_bytes = px * sizeof(float) * (req->mode == 1 ? 2 : 1);
    const size_t out_bytes = (px * size_t(r->P + 1) + 4) * sizeof(float);
    r->p_in = static_cast<float *>(r->pool->get(in_bytes, &r->in_cls));
    r->p_out = r->p_in ? static_cast<float *>(r->pool->get(out_bytes, &r->out_cls)) : nullptr;
    if (r->p_in && r->p_out) {
      std::memcpy(r->p_in, req->h_mask, px * sizeof(float));
      if (req->mode == 1) std::memcpy(r->p_in + px, req->h_target, px * sizeof(float));
    } else {
      r->pool->put(r->p_in, r->in_cls);
      r->p_in = nullptr;
      r->mask.assign(req->h_mask, req->h_mask + px);
      if (req->mode == 1) r->target.assign(req->h_target, req->h_target + px);
    }
  }
  auto job = std::make_shared<serve::Job>();
  job->footprint = HipExecutor::arena_need(r->ws_bytes, px, r->P, dev);
  job->payload = r;
  const int rc = srv->sched->submit(job, ticket);
  if (rc == LITHO_E_NOMEM)
    set_error("litho_serve_submit: request needs %zu bytes, more than the budget", job->footprint);
  else if (rc == LITHO_E_BUSY)
    set_error("litho_serve_submit: queue full");
  else if (rc != LITHO_OK)
    set_error("litho_serve_submit: server is stopping");
  return rc;
}

extern "C" int litho_serve_poll(litho_server_t *srv, uint64_t ticket, float *h_image, float *h_grad,
                                litho_result_info_t *info, int64_t timeout_us) {
  clear_error();
  if (!srv) {
    set_error("litho_serve_poll: NULL server");
    return LITHO_E_INVALID;
  }
  std::shared_ptr<serve::Job> job;
  const int rc = srv->sched->wait(ticket, timeout_us, &job);
  if (rc == LITHO_E_NOTFOUND) {
    set_error("litho_serve_poll: unknown ticket %llu", (unsigned long long)ticket);
    return rc;
  }
  if (rc == LITHO_PENDING) return rc;
  auto *r = static_cast<ServeReq *>(job->payload.get());
  if (info) {
    info->status = job->status;
    info->n = r->n;
    info->n_focus = r->P;
    info->loss = r->loss;
    info->t_submit_us = job->t_submit;
    info->t_start_us = job->t_start;
    info->t_done_us = job->t_done;
  }
  if (job->status != LITHO_OK) {
    set_error("litho_serve: request failed: %s", job->error.c_str());
    return job->status;
  }
  if (r->on_device()) return LITHO_OK;
  const size_t px = r->px();
  if (r->p_out) {
    // out of the request's pinned buffer on this (the polling) thread; the
    // buffers go back to the pool with the request
    if (h_image) std::memcpy(h_image, r->p_out, px * r->P * sizeof(float));
    if (h_grad && r->mode == 1) std::memcpy(h_grad, r->p_out + px * r->P, px * sizeof(float));
    return LITHO_OK;
  }
  if (h_image) std::memcpy(h_image, r->image.data(), r->image.size() * sizeof(float));
  if (h_grad && r->mode == 1) std::memcpy(h_grad, r->grad.data(), r->grad.size() * sizeof(float));
  return LITHO_OK;
}

extern "C" void litho_serve_destroy(litho_server_t *srv) {
  if (!srv) return;
  srv->sched.reset();  // drains queued and running requests
  srv->ex.reset();
  delete srv;
}
