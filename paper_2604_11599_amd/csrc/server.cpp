// Serving engine: admission by HBM footprint and continuous batching of
// shots requests (one persistent launch per tick over a slice of every
// admitted request) and energy+gradient requests.
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "qsv.h"

namespace {

struct Req {
  uint64_t ticket = 0;
  bool vqe = false;
  const qsv_program* prog = nullptr;
  uint32_t n = 0, n_params = 0, n_clbits = 0, max_events = 0;
  std::vector<double> theta;
  uint64_t shots = 0, done_shots = 0, seed = 0;
  size_t footprint = 0;
  bool finished = false;
  // shots results
  std::vector<uint64_t> creg;
  std::vector<uint8_t> record;
  std::vector<uint32_t> n_events;
  std::vector<double> record_prob;
  std::vector<int32_t> status;
  // energy + gradient
  std::vector<double> coeff;
  std::vector<uint8_t> pauli;
  double energy = 0.0;
  std::vector<double> grad;
};

}  // namespace

struct qsv_server {
  qsv_context* ctx = nullptr;
  size_t budget = 0, used = 0;
  uint32_t slice = 256;
  uint64_t next_ticket = 1;
  std::deque<uint64_t> waiting;
  std::vector<uint64_t> running;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
};

namespace {

qsv_status info_of(const qsv_program* p, qsv_program_info* info) {
  return qsv_program_info_get(p, info);
}

// state buffers a request of more than 2^16 amplitudes is charged for
// (distinct histories are few)
constexpr uint64_t kWideSlots = 16;

// shots of a request per tick: states of more than 2^16 amplitudes all at once
// (with many shots they run on the tile-pass path, where shots with equal
// histories share one state); narrower ones a slice per tick
uint64_t shots_per_tick(uint32_t n, uint64_t shots, uint32_t slice) {
  return n > 16 ? shots : slice;
}

}  // namespace

extern "C" {

qsv_status qsv_server_create(qsv_context* ctx, size_t hbm_budget, uint32_t shots_per_tick, qsv_server** out) {
  if (!ctx || !out || hbm_budget == 0) return QSV_ERR_ARG;
  std::unique_ptr<qsv_server> s(new qsv_server());
  s->ctx = ctx;
  s->budget = hbm_budget;
  s->slice = shots_per_tick ? shots_per_tick : 256;
  *out = s.release();
  return QSV_OK;
}

void qsv_server_destroy(qsv_server* srv) { delete srv; }

qsv_status qsv_submit(qsv_server* srv, const qsv_program* prog, const double* theta, uint64_t n_shots, uint64_t seed,
                      uint64_t* ticket) {
  if (!srv || !prog || !ticket) return QSV_ERR_ARG;
  qsv_program_info info;
  if (info_of(prog, &info) != QSV_OK) return QSV_ERR_ARG;
  if (info.n_params && !theta) return QSV_ERR_ARG;
  std::unique_ptr<Req> r(new Req());
  r->ticket = srv->next_ticket++;
  r->prog = prog;
  r->n = info.n_qubits;
  r->n_params = info.n_params;
  r->n_clbits = info.n_clbits;
  r->max_events = info.max_events;
  if (info.n_params) r->theta.assign(theta, theta + info.n_params);
  r->shots = n_shots;
  r->seed = seed;
  const uint64_t cw = std::max<uint32_t>(1, (info.n_clbits + 63) / 64);
  r->creg.assign(n_shots * cw, 0);
  r->record.assign(n_shots * std::max<uint32_t>(1, info.max_events), 0);
  r->n_events.assign(n_shots, 0);
  r->record_prob.assign(n_shots, 0.0);
  r->status.assign(n_shots, 0);
  const uint64_t per = shots_per_tick(r->n, n_shots, srv->slice);
  r->footprint = (size_t)std::min<uint64_t>(std::min<uint64_t>(n_shots, per), r->n > 16 ? kWideSlots : per) *
                 (16ull << r->n);
  *ticket = r->ticket;
  if (n_shots == 0) r->finished = true;
  else srv->waiting.push_back(r->ticket);
  srv->reqs[r->ticket] = std::move(r);
  return QSV_OK;
}

qsv_status qsv_submit_expval_grad(qsv_server* srv, const qsv_program* prog, const double* theta,
                                  const qsv_pauli_sum* h, uint64_t* ticket) {
  if (!srv || !prog || !h || !ticket) return QSV_ERR_ARG;
  qsv_program_info info;
  if (info_of(prog, &info) != QSV_OK) return QSV_ERR_ARG;
  if (!info.is_unitary) return QSV_ERR_UNSUPPORTED;
  if ((info.n_params && !theta) || (h->n_terms && (!h->coeff || !h->pauli))) return QSV_ERR_ARG;
  std::unique_ptr<Req> r(new Req());
  r->ticket = srv->next_ticket++;
  r->vqe = true;
  r->prog = prog;
  r->n = info.n_qubits;
  r->n_params = info.n_params;
  if (info.n_params) r->theta.assign(theta, theta + info.n_params);
  r->coeff.assign(h->coeff, h->coeff + h->n_terms);
  r->pauli.assign(h->pauli, h->pauli + (size_t)h->n_terms * info.n_qubits);
  r->grad.assign(std::max<uint32_t>(1, info.n_params), 0.0);
  r->footprint = 2 * (16ull << r->n);
  *ticket = r->ticket;
  srv->waiting.push_back(r->ticket);
  srv->reqs[r->ticket] = std::move(r);
  return QSV_OK;
}

qsv_status qsv_server_step(qsv_server* srv, uint32_t* n_running, uint32_t* n_waiting) {
  if (!srv) return QSV_ERR_ARG;
  // admission in arrival order while the footprint fits (a request larger than
  // the whole budget is admitted alone)
  while (!srv->waiting.empty()) {
    Req& r = *srv->reqs[srv->waiting.front()];
    if (srv->used + r.footprint > srv->budget && !srv->running.empty()) break;
    srv->used += r.footprint;
    srv->running.push_back(r.ticket);
    srv->waiting.pop_front();
  }
  // one slice of every admitted shots request in one persistent launch
  std::vector<qsv_request> batch;
  std::vector<Req*> owners;
  std::vector<uint64_t> slice_shots;
  for (uint64_t t : srv->running) {
    Req& r = *srv->reqs[t];
    if (r.vqe || r.finished) continue;
    const uint64_t k = std::min<uint64_t>(shots_per_tick(r.n, r.shots, srv->slice), r.shots - r.done_shots);
    const uint64_t cw = std::max<uint32_t>(1, (r.n_clbits + 63) / 64);
    const uint64_t mr = std::max<uint32_t>(1, r.max_events);
    qsv_request q;
    std::memset(&q, 0, sizeof(q));
    q.prog = r.prog;
    q.theta = r.theta.empty() ? nullptr : r.theta.data();
    q.n_shots = k;
    q.opts.seed = r.seed;
    q.opts.shot_offset = r.done_shots;
    q.out.creg = r.creg.data() + r.done_shots * cw;
    q.out.record = r.max_events ? r.record.data() + r.done_shots * mr : nullptr;
    q.out.n_events = r.n_events.data() + r.done_shots;
    q.out.record_prob = r.record_prob.data() + r.done_shots;
    q.out.shot_status = r.status.data() + r.done_shots;
    batch.push_back(q);
    owners.push_back(&r);
    slice_shots.push_back(k);
  }
  if (!batch.empty()) {
    qsv_status rc = qsv_run_batch(srv->ctx, batch.data(), (uint32_t)batch.size());
    if (rc != QSV_OK) return rc;
    for (size_t i = 0; i < owners.size(); ++i) {
      owners[i]->done_shots += slice_shots[i];
      if (owners[i]->done_shots == owners[i]->shots) owners[i]->finished = true;
    }
  }
  // energy + gradient requests (one parameter vector each)
  for (uint64_t t : srv->running) {
    Req& r = *srv->reqs[t];
    if (!r.vqe || r.finished) continue;
    qsv_pauli_sum h;
    std::memset(&h, 0, sizeof(h));
    h.n_terms = (uint32_t)r.coeff.size();
    h.coeff = r.coeff.data();
    h.pauli = r.pauli.data();
    qsv_status rc = qsv_expval_grad(srv->ctx, r.prog, r.theta.empty() ? nullptr : r.theta.data(), 1, &h,
                                    &r.energy, r.grad.data());
    if (rc != QSV_OK) return rc;
    r.finished = true;
  }
  // retire
  std::vector<uint64_t> still;
  for (uint64_t t : srv->running) {
    Req& r = *srv->reqs[t];
    if (r.finished) srv->used -= r.footprint;
    else still.push_back(t);
  }
  srv->running.swap(still);
  if (n_running) *n_running = (uint32_t)srv->running.size();
  if (n_waiting) *n_waiting = (uint32_t)srv->waiting.size();
  return QSV_OK;
}

qsv_status qsv_poll(qsv_server* srv, uint64_t ticket, int32_t* done) {
  if (!srv || !done) return QSV_ERR_ARG;
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return QSV_ERR_ARG;
  *done = it->second->finished ? 1 : 0;
  return QSV_OK;
}

qsv_status qsv_fetch_shots(qsv_server* srv, uint64_t ticket, qsv_shot_results* out) {
  if (!srv || !out || !out->creg) return QSV_ERR_ARG;
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end() || it->second->vqe || !it->second->finished) return QSV_ERR_ARG;
  Req& r = *it->second;
  const uint64_t cw = std::max<uint32_t>(1, (r.n_clbits + 63) / 64);
  std::memcpy(out->creg, r.creg.data(), r.shots * cw * 8);
  if (out->record && r.max_events) std::memcpy(out->record, r.record.data(), r.shots * r.max_events);
  if (out->n_events) std::memcpy(out->n_events, r.n_events.data(), r.shots * 4);
  if (out->record_prob) std::memcpy(out->record_prob, r.record_prob.data(), r.shots * 8);
  if (out->shot_status) std::memcpy(out->shot_status, r.status.data(), r.shots * 4);
  srv->reqs.erase(it);
  return QSV_OK;
}

qsv_status qsv_fetch_expval_grad(qsv_server* srv, uint64_t ticket, double* energy, double* grad) {
  if (!srv || !energy) return QSV_ERR_ARG;
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end() || !it->second->vqe || !it->second->finished) return QSV_ERR_ARG;
  Req& r = *it->second;
  *energy = r.energy;
  if (grad && r.n_params) std::memcpy(grad, r.grad.data(), r.n_params * 8);
  srv->reqs.erase(it);
  return QSV_OK;
}

}  // extern "C"
