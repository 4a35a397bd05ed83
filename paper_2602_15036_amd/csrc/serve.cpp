// Serving: the HIP executor behind the continuous-batching scheduler and the
// litho_serve_* C ABI.
//
// Each slot owns a non-blocking HIP stream (default priority), a completion
// event, device buffers for one request and pinned host staging.  A request
// on a slot is: pinned copy of its mask (and target) -> H2D -> SOCS image (and
// loss + gradient) on the slot's stream -> D2H into pinned memory -> event.
// A device-resident request skips the copies: it reads and writes the
// caller's device buffers directly.
// Slots run concurrently, so requests of different clip sizes and banks
// overlap on the device; every request keeps the bank's resident kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <limits>
#include <memory>
#include <vector>

#include "common.hpp"
#include "litho_internal.hpp"
#include "serve_core.hpp"

namespace litho {
namespace {

struct ServeReq {
  litho_bank *bank = nullptr;
  int K_use = 0, mode = 0, n = 0, P = 1, prec = LITHO_PREC_FP32;
  double slope = 0, thr = 0;
  std::vector<float> mask, target;
  std::vector<float> image, grad;
  double loss = 0;
  // device-resident I/O (d_mask != nullptr)
  const float *d_mask = nullptr, *d_target = nullptr;
  float *d_image = nullptr, *d_grad = nullptr;
  double *d_loss = nullptr;
  bool on_device() const { return d_mask != nullptr; }
};

class HipExecutor final : public serve::Executor {
 public:
  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    size_t dev_px = 0, host_px = 0;  // capacity in pixels (per plane for image)
    int dev_planes = 0, host_planes = 0;
    float *d_mask = nullptr, *d_target = nullptr, *d_image = nullptr, *d_grad = nullptr;
    double *d_loss = nullptr;
    float *h_in = nullptr, *h_image = nullptr, *h_grad = nullptr;
    double *h_loss = nullptr;
    std::string error;
  };

  HipExecutor(int nslots, int device) : slots_(size_t(nslots)), device_(device) {}

  ~HipExecutor() override {
    (void)hipSetDevice(device_);
    for (auto &s : slots_) {
      if (s.stream) (void)hipStreamSynchronize(s.stream);
      free_dev(s);
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

  int slots() const override { return int(slots_.size()); }
  void thread_init() override { (void)hipSetDevice(device_); }

  int launch(serve::Job &job, int si) override {
    auto *r = static_cast<ServeReq *>(job.payload.get());
    Slot &s = slots_[size_t(si)];
    if (r->on_device()) return launch_device(job, *r, s);
    const size_t px = size_t(r->n) * r->n;
    int rc = ensure(s, px, r->P);
    if (rc != LITHO_OK) {
      job.error = last_error();
      return rc;
    }
    std::memcpy(s.h_in, r->mask.data(), px * sizeof(float));
    if (r->mode == 1) std::memcpy(s.h_in + px, r->target.data(), px * sizeof(float));
    const size_t in_bytes = px * sizeof(float) * (r->mode == 1 ? 2 : 1);
    if (hipMemcpyAsync(s.d_mask, s.h_in, in_bytes, hipMemcpyHostToDevice, s.stream) != hipSuccess) {
      job.error = "litho_serve: H2D copy failed";
      return LITHO_E_HIP;
    }
    if (r->mode == 1) {
      litho_resist_t res{r->slope, r->thr};
      rc = image_grad_impl(r->bank, s.d_mask, 1, r->K_use, s.d_target, &res, nullptr, s.d_image, s.d_loss,
                           s.d_grad, true, r->prec, s.stream);
    } else {
      rc = image_grad_impl(r->bank, s.d_mask, 1, r->K_use, nullptr, nullptr, nullptr, s.d_image, nullptr, nullptr,
                           false, r->prec, s.stream);
    }
    if (rc != LITHO_OK) {
      job.error = last_error();
      return rc;
    }
    bool ok = hipMemcpyAsync(s.h_image, s.d_image, px * r->P * sizeof(float), hipMemcpyDeviceToHost, s.stream) ==
              hipSuccess;
    if (r->mode == 1) {
      ok = ok && hipMemcpyAsync(s.h_grad, s.d_grad, px * sizeof(float), hipMemcpyDeviceToHost, s.stream) ==
                     hipSuccess;
      ok = ok && hipMemcpyAsync(s.h_loss, s.d_loss, sizeof(double), hipMemcpyDeviceToHost, s.stream) == hipSuccess;
    }
    ok = ok && hipEventRecord(s.done, s.stream) == hipSuccess;
    if (!ok) {
      job.error = "litho_serve: D2H copy or event record failed";
      return LITHO_E_HIP;
    }
    return LITHO_OK;
  }

  int launch_device(serve::Job &job, ServeReq &r, Slot &s) {
    int rc;
    if (r.mode == 1) {
      litho_resist_t res{r.slope, r.thr};
      rc = image_grad_impl(r.bank, r.d_mask, 1, r.K_use, r.d_target, &res, nullptr, r.d_image, r.d_loss, r.d_grad,
                           true, r.prec, s.stream);
    } else {
      rc = image_grad_impl(r.bank, r.d_mask, 1, r.K_use, nullptr, nullptr, nullptr, r.d_image, nullptr, nullptr,
                           false, r.prec, s.stream);
    }
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
    const size_t px = size_t(r->n) * r->n;
    r->image.assign(s.h_image, s.h_image + px * r->P);
    if (r->mode == 1) {
      r->grad.assign(s.h_grad, s.h_grad + px);
      r->loss = *s.h_loss;
    }
    return LITHO_OK;
  }

 private:
  static void free_dev(Slot &s) {
    for (float *p : {s.d_mask, s.d_image, s.d_grad})
      if (p) (void)hipFree(p);
    if (s.d_loss) (void)hipFree(s.d_loss);
    s.d_mask = s.d_target = s.d_image = s.d_grad = nullptr;
    s.d_loss = nullptr;
    s.dev_px = 0;
    s.dev_planes = 0;
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

  // Grows the slot's buffers to px pixels and P planes (only on the scheduler
  // thread, while the slot is idle).
  int ensure(Slot &s, size_t px, int P) {
    if (s.dev_px < px || s.dev_planes < P) {
      free_dev(s);
      const size_t mask_bytes = 2 * px * sizeof(float);  // mask + target, contiguous
      if (hipMalloc(&s.d_mask, mask_bytes) != hipSuccess || hipMalloc(&s.d_image, px * P * sizeof(float)) !=
              hipSuccess || hipMalloc(&s.d_grad, px * sizeof(float)) != hipSuccess ||
          hipMalloc(&s.d_loss, sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        free_dev(s);
        set_error("litho_serve: cannot allocate slot buffers for %zu pixels", px);
        return LITHO_E_NOMEM;
      }
      s.d_target = s.d_mask + px;
      s.dev_px = px;
      s.dev_planes = P;
    }
    s.d_target = s.d_mask + px;
    if (s.host_px < px || s.host_planes < P) {
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
    }
    return LITHO_OK;
  }

  std::vector<Slot> slots_;
  int device_;
};

}  // namespace
}  // namespace litho

struct litho_server {
  std::vector<litho_bank *> banks;
  std::unique_ptr<litho::HipExecutor> ex;
  std::unique_ptr<litho::serve::Scheduler> sched;
};

using namespace litho;

// Device bytes a request holds while it runs: the workspace of one clip of
// its bank, plus the slot's I/O buffers unless its I/O is device-resident.
static size_t request_footprint(litho_bank *bk, int K_use, int mode, int prec, bool on_device) {
  const size_t px = size_t(bk->host.n) * bk->host.n;
  const CallLayout L = plan_call(bk, 1, K_use, mode == 1, mode == 1, prec);
  return (on_device ? 0 : px * sizeof(float) * (3 + size_t(bk->host.n_focus))) + L.per_clip;
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
  if (dev) {
    r->d_mask = req->d_mask;
    r->d_target = req->mode == 1 ? req->d_target : nullptr;
    r->d_image = req->d_image;
    r->d_grad = req->mode == 1 ? req->d_grad : nullptr;
    r->d_loss = req->mode == 1 ? req->d_loss : nullptr;
  } else {
    r->mask.assign(req->h_mask, req->h_mask + px);
    if (req->mode == 1) r->target.assign(req->h_target, req->h_target + px);
  }
  auto job = std::make_shared<serve::Job>();
  job->footprint = request_footprint(bk, req->K_use, req->mode, req->prec, dev);
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
