// Serving engine: continuous batching of shots and energy+gradient requests.
//
// Work runs in three lanes, each a host thread that drives a context forked
// from the caller's (its own stream and scratch), so the lanes' device work
// overlaps on the GPU:
//   persistent lane  shots requests that run as work items of the persistent
//                    launch (states of up to 20 qubits and fewer than 64
//                    shots, or up to 12 qubits): every round runs one slice
//                    of shots of every request the lane holds in one launch;
//                    requests handed over meanwhile join the next round;
//   wide lane        the other shots requests (wider states, or 13..20 qubits
//                    with at least 64 shots) on the tile passes with shared
//                    trajectories, one request per call, in arrival order;
//   energy lane      energy+gradient requests, one sweep per program over all
//                    vectors it holds, each vector with its own Hamiltonian.
// Admission happens on the caller's thread in qsv_server_step, in arrival
// order while the admitted set's HBM footprint fits the budget; the call never
// waits for device work, so requests that arrive while the lanes compute are
// admitted at the next step and join the lanes' next rounds. A request's
// results depend only on (program, theta, seed, shot index) or (program,
// theta, Hamiltonian), never on what else is in flight.
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "qsv.h"

namespace {

enum LaneKind { L_PERSISTENT = 0, L_WIDE = 1, L_ENERGY = 2, L_COUNT = 3 };

struct Req {
  uint64_t ticket = 0;
  bool vqe = false;
  const qsv_program* prog = nullptr;
  uint32_t n = 0, n_params = 0, n_clbits = 0, max_events = 0;
  std::vector<double> theta;
  uint64_t shots = 0, done_shots = 0, seed = 0;
  size_t footprint = 0;
  int lane = L_PERSISTENT;
  std::atomic<int> finished{0};  // set last by the lane that ran the request
  qsv_status error = QSV_OK;
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

struct Lane {
  int kind = L_PERSISTENT;
  qsv_context* ctx = nullptr;
  uint32_t slice = 256;
  std::thread th;
  std::mutex mu;                 // guards queue and stop
  std::condition_variable cv;
  std::vector<Req*> queue;       // handed over by admission, taken by the lane
  bool stop = false;
  std::mutex run_mu;             // held while the lane's context works
};

// streamed (HBM-slot) states of the persistent launch and the shot count
// from which such requests run on the tile passes instead (as qsv_run_batch
// routes them)
constexpr uint32_t kPersistentMaxBits = 20;
constexpr uint32_t kResidentBits = 12;
constexpr uint64_t kWideMinShots = 64;
// state buffers a wide request is charged for (distinct histories are few)
constexpr uint64_t kWideSlots = 16;

int lane_of(const Req& r) {
  if (r.vqe) return L_ENERGY;
  if (r.n > kPersistentMaxBits || (r.n > kResidentBits && r.shots >= kWideMinShots)) return L_WIDE;
  return L_PERSISTENT;
}

void finish(Req* r, qsv_status st) {
  r->error = st;
  r->finished.store(1, std::memory_order_release);
}

void run_persistent(Lane& L, std::vector<Req*>& held) {
  std::vector<qsv_request> batch;
  std::vector<uint64_t> slice_shots;
  for (Req* rp : held) {
    Req& r = *rp;
    const uint64_t k = std::min<uint64_t>(r.n > 16 ? r.shots : L.slice, r.shots - r.done_shots);
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
    slice_shots.push_back(k);
  }
  qsv_status rc;
  {
    std::lock_guard<std::mutex> lk(L.run_mu);
    rc = qsv_run_batch(L.ctx, batch.data(), (uint32_t)batch.size());
  }
  std::vector<Req*> still;
  for (size_t i = 0; i < held.size(); ++i) {
    Req* r = held[i];
    if (rc != QSV_OK) {
      finish(r, rc);
      continue;
    }
    r->done_shots += slice_shots[i];
    if (r->done_shots == r->shots) finish(r, QSV_OK);
    else still.push_back(r);
  }
  held.swap(still);
}

void run_wide(Lane& L, Req* r) {
  qsv_run_opts o;
  std::memset(&o, 0, sizeof(o));
  o.seed = r->seed;
  o.flags = QSV_RUN_SHARE_TRAJ;
  qsv_shot_results out;
  std::memset(&out, 0, sizeof(out));
  out.creg = r->creg.data();
  out.record = r->max_events ? r->record.data() : nullptr;
  out.n_events = r->n_events.data();
  out.record_prob = r->record_prob.data();
  out.shot_status = r->status.data();
  qsv_status rc;
  {
    std::lock_guard<std::mutex> lk(L.run_mu);
    rc = qsv_run_shots(L.ctx, r->prog, r->theta.empty() ? nullptr : r->theta.data(), r->shots, &o, &out);
  }
  r->done_shots = r->shots;
  finish(r, rc);
}

void run_energy(Lane& L, std::vector<Req*>& held) {
  // one sweep per program over all its vectors, each with its own Hamiltonian
  std::map<const qsv_program*, std::vector<Req*>> by_prog;
  for (Req* r : held) by_prog[r->prog].push_back(r);
  held.clear();
  for (auto& kv : by_prog) {
    std::vector<Req*>& rs = kv.second;
    const uint32_t P = rs[0]->n_params, B = (uint32_t)rs.size();
    std::vector<double> theta((size_t)B * std::max<uint32_t>(P, 1), 0.0), energy(B), grad((size_t)B * std::max<uint32_t>(P, 1));
    std::vector<qsv_pauli_sum> hs(B);
    for (uint32_t b = 0; b < B; ++b) {
      if (P) std::memcpy(&theta[(size_t)b * P], rs[b]->theta.data(), P * 8);
      std::memset(&hs[b], 0, sizeof(hs[b]));
      hs[b].n_terms = (uint32_t)rs[b]->coeff.size();
      hs[b].coeff = rs[b]->coeff.data();
      hs[b].pauli = rs[b]->pauli.data();
    }
    qsv_status rc;
    {
      std::lock_guard<std::mutex> lk(L.run_mu);
      rc = qsv_expval_grad_each(L.ctx, kv.first, theta.data(), B, hs.data(), energy.data(), grad.data());
    }
    for (uint32_t b = 0; b < B; ++b) {
      if (rc == QSV_OK) {
        rs[b]->energy = energy[b];
        if (P) std::memcpy(rs[b]->grad.data(), &grad[(size_t)b * P], P * 8);
      }
      finish(rs[b], rc);
    }
  }
}

void lane_main(Lane* Lp) {
  Lane& L = *Lp;
  std::vector<Req*> held;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(L.mu);
      L.cv.wait(lk, [&] { return L.stop || !L.queue.empty() || !held.empty(); });
      if (L.stop) return;
      if (L.kind == L_WIDE) {
        if (held.empty() && !L.queue.empty()) {
          held.push_back(L.queue.front());
          L.queue.erase(L.queue.begin());
        }
      } else {
        held.insert(held.end(), L.queue.begin(), L.queue.end());
        L.queue.clear();
      }
    }
    if (L.kind == L_PERSISTENT) {
      run_persistent(L, held);
    } else if (L.kind == L_WIDE) {
      run_wide(L, held[0]);
      held.clear();
    } else {
      run_energy(L, held);
    }
  }
}

}  // namespace

struct qsv_server {
  qsv_context* ctx = nullptr;
  size_t budget = 0, used = 0;
  uint32_t slice = 256;
  uint64_t next_ticket = 1;
  std::deque<Req*> waiting;
  std::vector<Req*> running;  // admitted, not yet retired
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  Lane lanes[L_COUNT];
};

namespace {

void stop_lanes(qsv_server* s) {
  for (Lane& L : s->lanes) {
    if (L.th.joinable()) {
      {
        std::lock_guard<std::mutex> lk(L.mu);
        L.stop = true;
      }
      L.cv.notify_all();
      L.th.join();
    }
    if (L.ctx) qsv_destroy(L.ctx);
    L.ctx = nullptr;
  }
}

}  // namespace

extern "C" {

qsv_status qsv_server_create(qsv_context* ctx, size_t hbm_budget, uint32_t shots_per_tick, qsv_server** out) {
  if (!ctx || !out || hbm_budget == 0) return QSV_ERR_ARG;
  *out = nullptr;
  std::unique_ptr<qsv_server> s(new qsv_server());
  s->ctx = ctx;
  s->budget = hbm_budget;
  s->slice = shots_per_tick ? shots_per_tick : 256;
  for (int k = 0; k < L_COUNT; ++k) {
    Lane& L = s->lanes[k];
    L.kind = k;
    L.slice = s->slice;
    const qsv_status st = qsv_context_fork(ctx, &L.ctx);
    if (st != QSV_OK) {
      stop_lanes(s.get());
      return st;
    }
  }
  for (Lane& L : s->lanes) L.th = std::thread(lane_main, &L);
  *out = s.release();
  return QSV_OK;
}

void qsv_server_destroy(qsv_server* srv) {
  if (!srv) return;
  stop_lanes(srv);
  delete srv;
}

qsv_status qsv_submit(qsv_server* srv, const qsv_program* prog, const double* theta, uint64_t n_shots, uint64_t seed,
                      uint64_t* ticket) {
  if (!srv || !prog || !ticket) return QSV_ERR_ARG;
  qsv_program_info info;
  if (qsv_program_info_get(prog, &info) != QSV_OK) return QSV_ERR_ARG;
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
  r->lane = lane_of(*r);
  // states resident at once: a slice of shots in the persistent launch, a
  // handful of shared histories on the tile passes
  const uint64_t resident = r->lane == L_WIDE ? std::min<uint64_t>(n_shots, kWideSlots)
                                              : std::min<uint64_t>(n_shots, r->n > 16 ? n_shots : srv->slice);
  r->footprint = (size_t)std::max<uint64_t>(resident, 1) * (16ull << r->n);
  *ticket = r->ticket;
  if (n_shots == 0) finish(r.get(), QSV_OK);
  else srv->waiting.push_back(r.get());
  srv->reqs[r->ticket] = std::move(r);
  return QSV_OK;
}

qsv_status qsv_submit_expval_grad(qsv_server* srv, const qsv_program* prog, const double* theta,
                                  const qsv_pauli_sum* h, uint64_t* ticket) {
  if (!srv || !prog || !h || !ticket) return QSV_ERR_ARG;
  qsv_program_info info;
  if (qsv_program_info_get(prog, &info) != QSV_OK) return QSV_ERR_ARG;
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
  r->lane = L_ENERGY;
  r->footprint = 2 * (16ull << r->n);
  *ticket = r->ticket;
  srv->waiting.push_back(r.get());
  srv->reqs[r->ticket] = std::move(r);
  return QSV_OK;
}

qsv_status qsv_server_step(qsv_server* srv, uint32_t* n_running, uint32_t* n_waiting) {
  if (!srv) return QSV_ERR_ARG;
  // retire what the lanes finished: its memory goes back to the budget
  std::vector<Req*> still;
  for (Req* r : srv->running) {
    if (r->finished.load(std::memory_order_acquire)) srv->used -= r->footprint;
    else still.push_back(r);
  }
  srv->running.swap(still);
  // admission in arrival order while the footprint fits (a request larger than
  // the whole budget is admitted alone); each goes to its lane
  std::vector<Req*> handed[L_COUNT];
  while (!srv->waiting.empty()) {
    Req* r = srv->waiting.front();
    if (srv->used + r->footprint > srv->budget && !srv->running.empty()) break;
    srv->used += r->footprint;
    srv->running.push_back(r);
    srv->waiting.pop_front();
    handed[r->lane].push_back(r);
  }
  for (int k = 0; k < L_COUNT; ++k) {
    if (handed[k].empty()) continue;
    Lane& L = srv->lanes[k];
    {
      std::lock_guard<std::mutex> lk(L.mu);
      L.queue.insert(L.queue.end(), handed[k].begin(), handed[k].end());
    }
    L.cv.notify_one();
  }
  if (n_running) *n_running = (uint32_t)srv->running.size();
  if (n_waiting) *n_waiting = (uint32_t)srv->waiting.size();
  return QSV_OK;
}

qsv_status qsv_poll(qsv_server* srv, uint64_t ticket, int32_t* done) {
  if (!srv || !done) return QSV_ERR_ARG;
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return QSV_ERR_ARG;
  *done = it->second->finished.load(std::memory_order_acquire) ? 1 : 0;
  return QSV_OK;
}

qsv_status qsv_fetch_shots(qsv_server* srv, uint64_t ticket, qsv_shot_results* out) {
  if (!srv || !out || !out->creg) return QSV_ERR_ARG;
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end() || it->second->vqe || !it->second->finished.load(std::memory_order_acquire))
    return QSV_ERR_ARG;
  Req& r = *it->second;
  if (std::find(srv->running.begin(), srv->running.end(), &r) != srv->running.end()) {
    srv->used -= r.footprint;  // finished since the last step: retire it now
    srv->running.erase(std::find(srv->running.begin(), srv->running.end(), &r));
  }
  const qsv_status err = r.error;
  if (err == QSV_OK) {
    const uint64_t cw = std::max<uint32_t>(1, (r.n_clbits + 63) / 64);
    std::memcpy(out->creg, r.creg.data(), r.shots * cw * 8);
    if (out->record && r.max_events) std::memcpy(out->record, r.record.data(), r.shots * r.max_events);
    if (out->n_events) std::memcpy(out->n_events, r.n_events.data(), r.shots * 4);
    if (out->record_prob) std::memcpy(out->record_prob, r.record_prob.data(), r.shots * 8);
    if (out->shot_status) std::memcpy(out->shot_status, r.status.data(), r.shots * 4);
  }
  srv->reqs.erase(it);
  return err;
}

qsv_status qsv_fetch_expval_grad(qsv_server* srv, uint64_t ticket, double* energy, double* grad) {
  if (!srv || !energy) return QSV_ERR_ARG;
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end() || !it->second->vqe || !it->second->finished.load(std::memory_order_acquire))
    return QSV_ERR_ARG;
  Req& r = *it->second;
  if (std::find(srv->running.begin(), srv->running.end(), &r) != srv->running.end()) {
    srv->used -= r.footprint;
    srv->running.erase(std::find(srv->running.begin(), srv->running.end(), &r));
  }
  const qsv_status err = r.error;
  if (err == QSV_OK) {
    *energy = r.energy;
    if (grad && r.n_params) std::memcpy(grad, r.grad.data(), r.n_params * 8);
  }
  srv->reqs.erase(it);
  return err;
}

qsv_status qsv_server_profile(qsv_server* srv, qsv_profile* out) {
  if (!srv || !out) return QSV_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  for (Lane& L : srv->lanes) {
    std::lock_guard<std::mutex> lk(L.run_mu);
    qsv_profile p;
    if (qsv_profile_read(L.ctx, &p) != QSV_OK) return QSV_ERR_ARG;
    out->pass_launches += p.pass_launches;
    out->pass_ms += p.pass_ms;
    out->pass_uncond_launches += p.pass_uncond_launches;
    out->pass_uncond_ms += p.pass_uncond_ms;
    out->pass_uncond_bytes += p.pass_uncond_bytes;
    out->pass_uncond_flops += p.pass_uncond_flops;
    out->site_launches += p.site_launches;
    out->site_ms += p.site_ms;
    out->other_launches += p.other_launches;
    out->other_ms += p.other_ms;
    out->ham_launches += p.ham_launches;
    out->ham_ms += p.ham_ms;
    out->ham_bytes += p.ham_bytes;
    out->sweep_launches += p.sweep_launches;
    out->sweep_ms += p.sweep_ms;
    out->sweep_bytes += p.sweep_bytes;
    out->persistent_launches += p.persistent_launches;
    out->persistent_ms += p.persistent_ms;
    out->persistent_bytes += p.persistent_bytes;
  }
  return QSV_OK;
}

}  // extern "C"
