// Serving form of the local-energy path (C ABI in include/nqs.h): requests of
// any resident instance/ansatz pair arrive while others run; each slot owns a
// device stream, so the kernels of admitted requests overlap on the GPU.  A
// request is admitted by its exact device-memory footprint
// (nqs_eloc_workspace_bytes with a bounded rows-per-pass), never beyond the
// budget, which also caps the context's workspace pool.
//
// Results do not depend on what else runs: draws are keyed by the request's
// seed and request-local sample index, each sample's reduction order is fixed
// by its own rows, and the kernel configuration depends only on (K, chi,
// precision).
#include "nqs.h"
#include "internal.h"
#include "admission.h"

#include <cstring>
#include <memory>
#include <string>

namespace {

struct ServeJob {
  nqs_request req{};
  nqs_eloc_stats stats{};
  std::string err;
};

}  // namespace

struct nqs_server {
  nqs_ctx* ctx = nullptr;
  int device = 0;
  int32_t max_rows = 0;
  std::vector<hipStream_t> streams;
  std::unique_ptr<nqs::Scheduler<ServeJob>> sched;
};

extern "C" {

double nqs_monotonic_seconds(void) { return nqs::mono_seconds(); }

nqs_status nqs_serve_create(nqs_ctx* ctx, int n_slots, size_t budget_bytes, int32_t max_rows_per_pass,
                            nqs_server** out) {
  if (!ctx || !out || n_slots < 1 || n_slots > 64 || budget_bytes == 0 || max_rows_per_pass <= 0)
    return NQS_EINVAL;
  const int device = nqs_ctx_device(ctx);
  nqs_status st = nqs_ctx_set_pool_limit(ctx, budget_bytes);
  if (st != NQS_OK) return st;
  std::unique_ptr<nqs_server> s(new nqs_server());
  s->ctx = ctx;
  s->device = device;
  s->max_rows = max_rows_per_pass;
  if (hipSetDevice(device) != hipSuccess) return NQS_EDEVICE;
  for (int k = 0; k < n_slots; ++k) {
    hipStream_t h;
    if (hipStreamCreateWithFlags(&h, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      return NQS_EDEVICE;
    }
    s->streams.push_back(h);
  }
  nqs_server* raw = s.get();
  s->sched.reset(new nqs::Scheduler<ServeJob>(
      n_slots, budget_bytes, [raw](ServeJob& j, int slot) -> int {
        (void)hipSetDevice(raw->device);
        const nqs_request& r = j.req;
        const nqs_status rc = nqs_eloc(raw->ctx, r.inst, r.ans, r.samples, nullptr, r.N, &r.opts, r.eloc,
                                       r.etnum, r.logabs, r.sign, r.fsq, &j.stats, raw->streams[slot]);
        if (rc != NQS_OK) j.err = nqs_last_error();
        return rc;
      }));
  *out = s.release();
  return NQS_OK;
}

nqs_status nqs_serve_destroy(nqs_server* s) {
  if (!s) return NQS_OK;
  s->sched.reset();   // drains the queue and joins the slots
  for (auto h : s->streams) (void)hipStreamDestroy(h);
  (void)nqs_ctx_set_pool_limit(s->ctx, 0);
  delete s;
  return NQS_OK;
}

nqs_status nqs_serve_footprint(nqs_server* s, const nqs_request* req, size_t* bytes) {
  if (!s || !req || !bytes) return NQS_EINVAL;
  nqs_eloc_opts o = req->opts;
  if (o.max_rows_per_pass == 0) o.max_rows_per_pass = s->max_rows;
  if (o.max_rows_per_pass == 0) return NQS_EINVAL;
  return nqs_eloc_workspace_bytes(req->inst, req->ans, req->N, &o, 0, bytes);
}

nqs_status nqs_serve_submit(nqs_server* s, const nqs_request* req, int64_t* ticket) {
  if (!s || !req || !req->inst || !req->ans || req->N < 0 || (!req->samples && req->N > 0)) return NQS_EINVAL;
  ServeJob j;
  j.req = *req;
  if (j.req.opts.max_rows_per_pass == 0) j.req.opts.max_rows_per_pass = s->max_rows;
  size_t bytes = 0;
  nqs_status st = nqs_eloc_workspace_bytes(req->inst, req->ans, req->N, &j.req.opts, 0, &bytes);
  if (st != NQS_OK) return st;
  const double t = req->t_arrival > 0 ? req->t_arrival : nqs::mono_seconds();
  if (s->sched->submit(std::move(j), bytes, t, ticket) != 0) return NQS_ENOMEM;
  return NQS_OK;
}

static void fill_completion(const nqs::Scheduler<ServeJob>::Done& d, nqs_completion* out) {
  std::memset(out, 0, sizeof *out);
  out->ticket = d.ticket;
  out->user_tag = d.job.req.user_tag;
  out->status = d.status;
  out->t_submit = d.t_submit;
  out->t_start = d.t_start;
  out->t_end = d.t_end;
  out->footprint = d.bytes;
  out->stats = d.job.stats;
  std::strncpy(out->message, d.job.err.c_str(), sizeof(out->message) - 1);
}

nqs_status nqs_serve_poll(nqs_server* s, nqs_completion* out) {
  if (!s || !out) return NQS_EINVAL;
  nqs::Scheduler<ServeJob>::Done d;
  if (!s->sched->try_pop_done(&d)) return NQS_EBUSY;
  fill_completion(d, out);
  return NQS_OK;
}

nqs_status nqs_serve_wait(nqs_server* s, double timeout_s, nqs_completion* out) {
  if (!s || !out) return NQS_EINVAL;
  nqs::Scheduler<ServeJob>::Done d;
  if (!s->sched->wait_done(&d, timeout_s)) return NQS_EBUSY;
  fill_completion(d, out);
  return NQS_OK;
}

nqs_status nqs_serve_info(nqs_server* s, nqs_serve_status* out) {
  if (!s || !out) return NQS_EINVAL;
  out->budget = s->sched->budget();
  out->reserved = s->sched->reserved();
  out->peak_reserved = s->sched->peak_reserved();
  out->in_flight = s->sched->in_flight();
  out->peak_in_flight = s->sched->peak_in_flight();
  out->queued = int64_t(s->sched->queued());
  out->skips = s->sched->skips();
  return NQS_OK;
}

}  // extern "C"
