// C ABI of libqsv (see include/qsv.h): contexts, program loading, shot
// execution, expectation values and adjoint gradients on one GPU.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <functional>
#include <chrono>
#include <cstdio>
#include <map>
#include <mutex>
#include <sstream>
#include <unordered_map>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "kernels.h"
#include "planner.h"
#include "qsv.h"
#include "qsv_diag.h"
#include "qsv_plan.h"

using namespace qsv;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct qsv_context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  uint32_t flags = 0;
  uint8_t* arena = nullptr;
  size_t arena_bytes = 0;
  size_t arena_top = 0;
  std::string err;
  std::vector<DevBuf> cache;  // grow-only scratch slots (used when no arena is given)
  size_t slot = 0;
  // profiling (QSV_FLAG_PROFILE): events around every launch, harvested after each sync
  struct Rec {
    hipEvent_t a, b;
    int kind;  // Kind
    bool uncond;
    double bytes, flops;
  };
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<Rec> recs;
  qsv_profile prof{};
  // set for the duration of a qsv_run_shots_noalloc call: scratch comes from
  // the device's fixed array and no events are created or recorded
  bool noalloc = false;
  bool capturing = false;  // launches are being recorded into a HIP graph
  std::string arch;        // the device's architecture name (autotuning cache key)
  qsv_context* parent = nullptr;  // a forked context runs its parent's programs
  // qsv_run_batch's extra lanes: forks that run the tile-pass requests, each
  // from a host thread of its own, while this context runs the persistent
  // launches (created on first use, destroyed with this context)
  std::vector<qsv_context*> batch_forks;
  hipEvent_t batch_ev = nullptr;  // orders the forks' work after this context's queued work
  bool profiling() const { return (flags & QSV_FLAG_PROFILE) != 0 && !noalloc && !capturing; }
  // the arena scratch is carved from in the current call, if any
  uint8_t* call_arena() const { return noalloc ? static_cast<uint8_t*>(noalloc_scratch(device)) : arena; }
  size_t call_arena_bytes() const { return noalloc ? kNoAllocScratchBytes : arena_bytes; }
};

struct qsv_program {
  qsv_context* ctx = nullptr;
  qsv_program_desc desc{};
  std::vector<qsv_instr> instr;
  std::vector<qsv_pred> pred;
  std::vector<qsv_cop> code;
  std::vector<qsv_lin> lin;
  std::vector<qsv_noise> noise;
  Plan plan;
  // device copies of the static plan
  DGate* d_gates = nullptr;
  Phase* d_phases = nullptr;
  DStep* d_steps = nullptr;
  PassArgs* d_passes = nullptr;
  SiteArgs* d_sites = nullptr;
  GateSrc* d_src = nullptr;
  uint32_t* d_dense = nullptr;  // indices of the dense phases
  SiteEvent* d_events = nullptr;
  DPred* d_preds = nullptr;
  qsv_cop* d_code = nullptr;
  // derived parameters by index: entries [lin_off[k], lin_off[k + 1]) of (in, coef)
  uint32_t* d_lin_off = nullptr;
  uint32_t* d_lin_in = nullptr;
  double* d_lin_coef = nullptr;
  // depolarizing slots: counters, and the plan's (matrix slot, counter) lists
  qsv_noise* d_noise = nullptr;
  uint32_t* d_noise_slot = nullptr;
  uint32_t* d_noise_ctr = nullptr;
  uint32_t* d_noise_dense = nullptr;  // per noise slot: the dense phase holding it, or kNoDense
  // a program without parameters: its matrix slots bound and its dense phases
  // composed once, when the plan is installed (every call reads them)
  double* d_const_mats = nullptr;
  uint32_t* d_csr_off = nullptr;
  uint32_t* d_csr_sj = nullptr;
  double* d_csr_scale = nullptr;
  uint32_t pblocks = 1;
  // matrix-core adjoint sweep: angle entries of the dense phases of eligible
  // passes, and per phase the first entry (ang_off[phase + 1] ends it)
  AngEnt* d_ang_ent = nullptr;
  uint32_t* d_ang_off = nullptr;
  uint32_t n_ang_ent = 0;
  std::vector<uint8_t> bw_mfma;  // per pass: swept on the matrix cores
  PlanOptions opts;              // the options the current plan was built with
  // the captured launch sequence of the last QSV_RUN_GRAPH call and what it
  // was captured for (call shape and the scratch pointers it refers to)
  mutable hipGraphExec_t graph = nullptr;
  mutable std::vector<uint64_t> graph_key;
};

namespace {

#define HIP_TRY(call)                                                             \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);               \
      return e_ == hipErrorOutOfMemory ? QSV_ERR_NOMEM : QSV_ERR_DEVICE;          \
    }                                                                             \
  } while (0)

qsv_status set_err(qsv_context* ctx, qsv_status st, const std::string& m) {
  if (ctx) ctx->err = m;
  return st;
}

// Whether ctx may run prog: programs of the same context family (a context,
// its forks, and the programs any of them loaded).
bool owns(const qsv_context* ctx, const qsv_program* prog) {
  const qsv_context* a = ctx->parent ? ctx->parent : ctx;
  const qsv_context* b = prog->ctx->parent ? prog->ctx->parent : prog->ctx;
  return a == b;
}

// HIP keeps the most recent failed call's status per host thread until
// hipGetLastError reads it, and every kernel launcher reads it right after its
// launch. So a call whose status is not checked here, or a failed call made
// by other code on the thread between two library calls, would otherwise be
// reported as a failure of the next launch. Statuses that are deliberately
// ignored go through ignore(), which clears that state again, and every entry
// point clears it after selecting the device (enter()).
inline void clear_error() { (void)hipGetLastError(); }
inline void ignore(hipError_t) { clear_error(); }

hipError_t enter_device(int device) {
  clear_error();
  const hipError_t e = hipSetDevice(device);
  clear_error();
  return e;
}

// Scratch allocation for one call: from the caller's arena (bump pointer,
// reset per call) or from grow-only cached hipMalloc slots.
struct Scratch {
  qsv_context* ctx;
  explicit Scratch(qsv_context* c) : ctx(c) {
    ctx->arena_top = 0;
    ctx->slot = 0;
  }
  hipError_t get(size_t bytes, void** out) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    if (uint8_t* base = ctx->call_arena()) {
      if (ctx->arena_top + bytes > ctx->call_arena_bytes()) return hipErrorOutOfMemory;
      *out = base + ctx->arena_top;
      ctx->arena_top += bytes;
      return hipSuccess;
    }
    if (ctx->noalloc) return hipErrorOutOfMemory;  // never allocate on that path
    if (ctx->slot == ctx->cache.size()) ctx->cache.push_back(DevBuf{});
    DevBuf& b = ctx->cache[ctx->slot++];
    if (b.bytes < bytes) {
      if (b.p) ignore(hipFree(b.p));
      b.p = nullptr;
      b.bytes = 0;
      hipError_t e = hipMalloc(&b.p, bytes);
      if (e != hipSuccess) return e;
      b.bytes = bytes;
    }
    *out = b.p;
    return hipSuccess;
  }
  template <class T>
  hipError_t get(size_t count, T** out) {
    return get(count * sizeof(T), reinterpret_cast<void**>(out));
  }
};

template <class T>
hipError_t upload(const std::vector<T>& v, T** out) {
  *out = nullptr;
  if (v.empty()) return hipSuccess;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(out), v.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

// Launch classes of the profile.
enum Kind { K_PASS = 0, K_SITE = 1, K_OTHER = 2, K_HAM = 3, K_SWEEP = 4, K_PERSISTENT = 5 };

// Brackets one launch with profiling events when the context profiles.
// a += b, field by field (the batch fork's launches counted in its parent)
void add_profile(qsv_profile* a, const qsv_profile& b) {
  a->pass_launches += b.pass_launches;
  a->pass_ms += b.pass_ms;
  a->pass_uncond_launches += b.pass_uncond_launches;
  a->pass_uncond_ms += b.pass_uncond_ms;
  a->pass_uncond_bytes += b.pass_uncond_bytes;
  a->pass_uncond_flops += b.pass_uncond_flops;
  a->site_launches += b.site_launches;
  a->site_ms += b.site_ms;
  a->other_launches += b.other_launches;
  a->other_ms += b.other_ms;
  a->ham_launches += b.ham_launches;
  a->ham_ms += b.ham_ms;
  a->ham_bytes += b.ham_bytes;
  a->sweep_launches += b.sweep_launches;
  a->sweep_ms += b.sweep_ms;
  a->sweep_bytes += b.sweep_bytes;
  a->persistent_launches += b.persistent_launches;
  a->persistent_ms += b.persistent_ms;
  a->persistent_bytes += b.persistent_bytes;
}

struct Prof {
  qsv_context* ctx;
  hipStream_t st;
  hipEvent_t a = nullptr;
  Prof(qsv_context* c, hipStream_t s) : ctx(c), st(s) {
    if (!ctx->profiling()) return;
    a = next();
    if (hipEventRecord(a, st) != hipSuccess) {
      clear_error();
      a = nullptr;
    }
  }
  hipEvent_t next() {
    if (ctx->ev_used == ctx->ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        clear_error();
        return nullptr;
      }
      ctx->ev_pool.push_back(e);
    }
    return ctx->ev_pool[ctx->ev_used++];
  }
  void done(int kind, bool uncond = false, double bytes = 0, double flops = 0) {
    if (!ctx->profiling() || !a) return;
    hipEvent_t b = next();
    if (!b) return;
    if (hipEventRecord(b, st) != hipSuccess) {
      clear_error();
      return;
    }
    ctx->recs.push_back({a, b, kind, uncond, bytes, flops});
  }
};

// After a stream sync: fold the recorded launch times into the counters.
void harvest(qsv_context* ctx) {
  if (!ctx->profiling()) return;
  for (const auto& r : ctx->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
      clear_error();
      continue;
    }
    qsv_profile& p = ctx->prof;
    if (r.kind == 0) {
      p.pass_launches++;
      p.pass_ms += ms;
      if (r.uncond) {
        p.pass_uncond_launches++;
        p.pass_uncond_ms += ms;
        p.pass_uncond_bytes += r.bytes;
        p.pass_uncond_flops += r.flops;
      }
    } else if (r.kind == K_SITE) {
      p.site_launches++;
      p.site_ms += ms;
    } else if (r.kind == K_HAM) {
      p.ham_launches++;
      p.ham_ms += ms;
      p.ham_bytes += r.bytes;
    } else if (r.kind == K_SWEEP) {
      p.sweep_launches++;
      p.sweep_ms += ms;
      p.sweep_bytes += r.bytes;
    } else if (r.kind == K_PERSISTENT) {
      p.persistent_launches++;
      p.persistent_ms += ms;
    } else {
      p.other_launches++;
      p.other_ms += ms;
    }
  }
  ctx->recs.clear();
  ctx->ev_used = 0;
}

// algorithmic HBM bytes per amplitude of a tile pass: read and write of one
// complex128, or the write alone for the pass that also initialises |0...0>
double pass_bytes_per_amp(const PassArgs& a) { return a.init ? 16.0 : 32.0; }

size_t free_device_bytes() {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    clear_error();
    return 0;
  }
  return fr;
}

// ---------------------------------------------------------------------------
// Autotuning cache: the plan options measured fastest, per device
// architecture, qubit count and precision, shared by the contexts of the
// process.
// ---------------------------------------------------------------------------
struct TuneEntry {
  PlanOptions best;
  double best_ms = 0.0, default_ms = 0.0;
};
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;

std::string tune_key(const std::string& arch, uint32_t n, bool c64) {
  return arch + " " + std::to_string(n) + " " + (c64 ? "c64" : "c128");
}

bool tuned_options(const qsv_context* ctx, uint32_t n, bool c64, PlanOptions* o) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(tune_key(ctx->arch, n, c64));
  if (it == g_tune.end()) return false;
  *o = it->second.best;
  return true;
}

void to_public(const PlanOptions& o, qsv_plan_options* out) {
  out->tile_bits = o.tile_bits;
  out->low_bits = o.low_bits;
  out->dense_min_cost = o.dense_min_cost;
}

// The theta rows gate matrices are bound from: theta itself, or theta
// extended by the program's derived parameters into ext ([batch][P + D]).
hipError_t bind_theta(const qsv_program* prog, const double* theta, uint32_t batch, double* ext, hipStream_t st,
                      const double** rows, uint32_t* stride) {
  const uint32_t P = prog->desc.n_params, D = prog->desc.n_derived;
  if (!D) {
    *rows = theta;
    *stride = P;
    return hipSuccess;
  }
  *rows = ext;
  *stride = P + D;
  return launch_derive_params(theta, P, D, prog->d_lin_off, prog->d_lin_in, prog->d_lin_coef, batch, ext, st);
}

// Frees the device copies of a program's plan.
void free_plan_buffers(qsv_program* p) {
  if (p->graph) ignore(hipGraphExecDestroy(p->graph));
  p->graph = nullptr;
  p->graph_key.clear();
  void* ptrs[] = {p->d_gates, p->d_phases, p->d_steps, p->d_passes, p->d_sites, p->d_src, p->d_dense,
                  p->d_events, p->d_preds, p->d_csr_off, p->d_csr_sj, p->d_csr_scale, p->d_ang_ent, p->d_ang_off,
                  p->d_code, p->d_lin_off, p->d_lin_in, p->d_lin_coef, p->d_noise, p->d_noise_slot,
                  p->d_noise_ctr, p->d_noise_dense, p->d_const_mats};
  for (void* q : ptrs)
    if (q) ignore(hipFree(q));
  p->d_gates = nullptr;
  p->d_phases = nullptr;
  p->d_steps = nullptr;
  p->d_passes = nullptr;
  p->d_sites = nullptr;
  p->d_src = nullptr;
  p->d_dense = nullptr;
  p->d_events = nullptr;
  p->d_preds = nullptr;
  p->d_csr_off = nullptr;
  p->d_csr_sj = nullptr;
  p->d_csr_scale = nullptr;
  p->d_ang_ent = nullptr;
  p->d_ang_off = nullptr;
  p->d_code = nullptr;
  p->d_lin_off = nullptr;
  p->d_lin_in = nullptr;
  p->d_lin_coef = nullptr;
  p->d_noise = nullptr;
  p->d_noise_slot = nullptr;
  p->d_noise_ctr = nullptr;
  p->d_noise_dense = nullptr;
  p->d_const_mats = nullptr;
}

// Plans the program's stream with options o and uploads the plan (replacing a
// previous one). The device must be current.
qsv_status install_plan(qsv_context* ctx, qsv_program* p, const PlanOptions& o) {
  free_plan_buffers(p);
  const qsv_program_desc* desc = &p->desc;
  p->opts = o;
  p->pblocks = 1;
  p->plan = build_plan(p->desc, o);
  const Plan& pl = p->plan;
  for (const SiteArgs& s : pl.sites) p->pblocks = std::max(p->pblocks, s.blocks);
  std::vector<DPred> dp;
  for (const qsv_pred& q : p->pred) {
    DPred d{};
    d.lo = q.lo;
    d.width = q.width;
    d.value = q.value;
    d.cmp = q.cmp;
    dp.push_back(d);
  }
  // parameter -> (slot*3 + angle, scale) lists for the gradient chain rule
  std::vector<uint32_t> off(desc->n_params + 1, 0), sj;
  std::vector<double> sc;
  // (an angle on a derived parameter contributes to each of its inputs)
  std::vector<std::vector<std::pair<uint32_t, double>>> derived(desc->n_derived);
  for (const qsv_lin& l : p->lin) derived[l.out].push_back({l.in, l.coef});
  {
    std::vector<std::vector<std::pair<uint32_t, double>>> lists(desc->n_params);
    for (uint32_t s = 0; s < pl.gate_src.size(); ++s)
      for (int j = 0; j < 3; ++j) {
        const uint32_t par = pl.gate_src[s].param[j];
        if (par == QSV_NONE) continue;
        if (par < desc->n_params) {
          lists[par].push_back({s * 3 + j, pl.gate_src[s].scale[j]});
        } else {
          for (const auto& t : derived[par - desc->n_params])
            lists[t.first].push_back({s * 3 + j, pl.gate_src[s].scale[j] * t.second});
        }
      }
    for (uint32_t k = 0; k < desc->n_params; ++k) {
      off[k + 1] = off[k] + (uint32_t)lists[k].size();
      for (auto& e : lists[k]) {
        sj.push_back(e.first);
        sc.push_back(e.second);
      }
    }
  }
  // angle entries for the matrix-core adjoint sweep (all-dense passes of
  // 2^10..2^12-amplitude tiles whose phases have at most kMaxPhaseAngles angles)
  std::vector<AngEnt> ang;
  std::vector<uint32_t> ang_off(pl.phases.size() + 1, 0);
  p->bw_mfma.assign(pl.passes.size(), 0);
  {
    std::vector<uint32_t> cnt(pl.phases.size(), 0);
    for (size_t k = 0; k < pl.passes.size(); ++k) {
      if (!mfma_sweep_pass(pl, k)) continue;
      p->bw_mfma[k] = 1;
      const PassArgs& a = pl.passes[k];
      for (uint32_t q = 0; q < a.phase_count; ++q) {
        const uint32_t pg = a.phase_begin + q;
        const Phase& ph = pl.phases[pg];
        for (uint32_t i = 0; i < ph.gate_count; ++i) cnt[pg] += pl.gates[ph.gate_begin + i].nang;
      }
    }
    for (size_t pg = 0; pg < pl.phases.size(); ++pg) {
      ang_off[pg + 1] = ang_off[pg] + cnt[pg];
      const Phase& ph = pl.phases[pg];
      if (!cnt[pg]) continue;
      for (uint32_t i = 0; i < ph.gate_count; ++i)
        for (uint32_t j = 0; j < pl.gates[ph.gate_begin + i].nang; ++j)
          ang.push_back(AngEnt{ph.gate_begin + i, (uint16_t)i, (uint8_t)j, 0});
    }
  }
  p->n_ang_ent = (uint32_t)ang.size();
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = upload(ang, &p->d_ang_ent);
  if (e == hipSuccess && std::count(p->bw_mfma.begin(), p->bw_mfma.end(), 1)) e = upload(ang_off, &p->d_ang_off);
  if (e == hipSuccess) e = upload(pl.gates, &p->d_gates);
  if (e == hipSuccess) e = upload(pl.phases, &p->d_phases);
  {
    std::vector<DStep> ds;
    for (const Step& st : pl.steps) ds.push_back(DStep{(uint32_t)st.kind, st.index});
    if (e == hipSuccess) e = upload(ds, &p->d_steps);
  }
  if (e == hipSuccess) e = upload(pl.passes, &p->d_passes);
  if (e == hipSuccess) e = upload(pl.sites, &p->d_sites);
  if (e == hipSuccess) e = upload(pl.gate_src, &p->d_src);
  if (e == hipSuccess) e = upload(pl.dense_phases, &p->d_dense);
  if (e == hipSuccess) e = upload(pl.events, &p->d_events);
  if (e == hipSuccess) e = upload(dp, &p->d_preds);
  if (e == hipSuccess) e = upload(p->code, &p->d_code);
  if (e == hipSuccess) e = upload(p->noise, &p->d_noise);
  if (e == hipSuccess) e = upload(pl.noise_slot, &p->d_noise_slot);
  if (e == hipSuccess) e = upload(pl.noise_ctr, &p->d_noise_ctr);
  if (e == hipSuccess && !pl.noise_slot.empty()) {
    // the dense phase (index into dense_phases) whose composed matrix holds each noise slot
    std::vector<uint32_t> slot_dense(pl.gate_src.size(), kNoDense), nd(pl.noise_slot.size(), kNoDense);
    for (size_t d = 0; d < pl.dense_phases.size(); ++d) {
      const Phase& ph = pl.phases[pl.dense_phases[d]];
      for (uint32_t g = ph.gate_begin; g < ph.gate_begin + ph.gate_count; ++g)
        if (pl.gates[g].mat < slot_dense.size()) slot_dense[pl.gates[g].mat] = (uint32_t)d;
    }
    for (size_t k = 0; k < pl.noise_slot.size(); ++k)
      if (pl.noise_slot[k] < slot_dense.size()) nd[k] = slot_dense[pl.noise_slot[k]];
    e = upload(nd, &p->d_noise_dense);
  }
  if (desc->n_derived) {
    std::vector<uint32_t> loff(desc->n_derived + 1, 0), lin_in;
    std::vector<double> lin_coef;
    for (uint32_t k = 0; k < desc->n_derived; ++k) {
      for (const auto& t : derived[k]) {
        lin_in.push_back(t.first);
        lin_coef.push_back(t.second);
      }
      loff[k + 1] = (uint32_t)lin_in.size();
    }
    if (e == hipSuccess) e = upload(loff, &p->d_lin_off);
    if (e == hipSuccess) e = upload(lin_in, &p->d_lin_in);
    if (e == hipSuccess) e = upload(lin_coef, &p->d_lin_coef);
  }
  if (e == hipSuccess) e = upload(off, &p->d_csr_off);
  if (e == hipSuccess) e = upload(sj, &p->d_csr_sj);
  if (e == hipSuccess) e = upload(sc, &p->d_csr_scale);
  if (e == hipSuccess && desc->n_params == 0 && !pl.gate_src.empty()) {
    // no parameter: the same matrices at every call, bound and composed here
    // (noise slots as the identity: also the noise-free set of noisy calls)
    const uint32_t n_slots = (uint32_t)pl.gate_src.size();
    e = hipMalloc(reinterpret_cast<void**>(&p->d_const_mats), (size_t)n_slots * kMatStride * sizeof(double));
    // (no slot reads theta; the pointer passed for it is only a valid address)
    if (e == hipSuccess)
      e = launch_bind_matrices(p->d_src, n_slots, p->d_const_mats, 0u, 1u, p->d_const_mats, nullptr, ctx->stream);
    if (e == hipSuccess)
      e = launch_compose_dense(p->d_phases, p->d_dense, (uint32_t)pl.dense_phases.size(), p->d_gates, 1u, 0u,
                               p->d_const_mats, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  }
  if (e != hipSuccess) {
    free_plan_buffers(p);
    return set_err(ctx, e == hipErrorOutOfMemory ? QSV_ERR_NOMEM : QSV_ERR_DEVICE,
                   std::string("program upload: ") + hipGetErrorString(e));
  }
  return QSV_OK;
}


}  // namespace

extern "C" {

qsv_status qsv_create(const qsv_config* cfg, qsv_context** out) {
  if (!out) return QSV_ERR_ARG;
  *out = nullptr;
  std::unique_ptr<qsv_context> ctx(new qsv_context());
  qsv_config def{};
  if (!cfg) cfg = &def;
  ctx->device = cfg->device;
  ctx->flags = cfg->flags;
  ctx->arena = static_cast<uint8_t*>(cfg->arena);
  ctx->arena_bytes = cfg->arena ? cfg->arena_bytes : 0;
  int count = 0;
  clear_error();
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
    clear_error();
    return QSV_ERR_DEVICE;
  }
  if (cfg->device < 0 || cfg->device >= count) return QSV_ERR_ARG;
  if (enter_device(cfg->device) != hipSuccess) return QSV_ERR_DEVICE;
  // this device's address of the fixed scratch array (no-allocation entry point)
  if (noalloc_scratch_init(cfg->device) != hipSuccess) {
    clear_error();
    return QSV_ERR_DEVICE;
  }
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, cfg->device) != hipSuccess) {
      clear_error();
      return QSV_ERR_DEVICE;
    }
    ctx->arch = prop.gcnArchName;
    const size_t colon = ctx->arch.find(':');  // feature suffixes (sramecc, xnack) are not part of the key
    if (colon != std::string::npos) ctx->arch.resize(colon);
  }
  if (cfg->stream) {
    ctx->stream = static_cast<hipStream_t>(cfg->stream);
  } else if (cfg->flags & QSV_FLAG_NULL_STREAM) {
    ctx->stream = nullptr;  // the device's null stream
  } else {
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
      clear_error();
      return QSV_ERR_DEVICE;
    }
    ctx->own_stream = true;
  }
  *out = ctx.release();
  return QSV_OK;
}

qsv_status qsv_context_fork(qsv_context* parent, qsv_context** out) {
  if (!parent || !out) return QSV_ERR_ARG;
  *out = nullptr;
  if (parent->parent) return set_err(parent, QSV_ERR_ARG, "a forked context cannot be forked");
  qsv_config cfg{};
  cfg.device = parent->device;
  cfg.flags = parent->flags & ~(uint32_t)QSV_FLAG_NULL_STREAM;  // always a stream of its own
  qsv_context* c = nullptr;
  const qsv_status st = qsv_create(&cfg, &c);
  if (st != QSV_OK) return set_err(parent, st, "qsv_context_fork: context creation failed");
  c->parent = parent;
  *out = c;
  return QSV_OK;
}

void qsv_destroy(qsv_context* ctx) {
  if (!ctx) return;
  for (qsv_context* f : ctx->batch_forks) qsv_destroy(f);
  ignore(enter_device(ctx->device));
  if (ctx->batch_ev) ignore(hipEventDestroy(ctx->batch_ev));
  ignore(hipStreamSynchronize(ctx->stream));
  for (hipEvent_t e : ctx->ev_pool) ignore(hipEventDestroy(e));
  for (auto& b : ctx->cache)
    if (b.p) ignore(hipFree(b.p));
  if (ctx->own_stream) ignore(hipStreamDestroy(ctx->stream));
  delete ctx;
}

const char* qsv_last_error(const qsv_context* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

qsv_status qsv_load_program(qsv_context* ctx, const qsv_program_desc* desc, qsv_program** out) {
  if (!ctx || !desc || !out) return set_err(ctx, QSV_ERR_ARG, "null argument");
  *out = nullptr;
  if (desc->n_qubits > (uint32_t)kMaxQubits)
    return set_err(ctx, QSV_ERR_LIMIT, "more than 34 qubits do not fit one GPU's HBM");
  std::string err;
  if (!validate_program(*desc, &err)) return set_err(ctx, QSV_ERR_ARG, err);
  if (enter_device(ctx->device) != hipSuccess) return set_err(ctx, QSV_ERR_DEVICE, "hipSetDevice failed");
  std::unique_ptr<qsv_program> p(new qsv_program());
  p->ctx = ctx;
  p->instr.assign(desc->instr, desc->instr + desc->n_instr);
  p->pred.assign(desc->pred, desc->pred + desc->n_pred);
  if (desc->n_code) p->code.assign(desc->code, desc->code + desc->n_code);
  if (desc->n_lin) p->lin.assign(desc->lin, desc->lin + desc->n_lin);
  if (desc->n_noise) p->noise.assign(desc->noise, desc->noise + desc->n_noise);
  p->desc = *desc;
  p->desc.instr = p->instr.data();
  p->desc.pred = p->pred.data();
  p->desc.code = p->code.data();
  p->desc.lin = p->lin.data();
  p->desc.noise = p->noise.data();
  PlanOptions o;
  if (ctx->flags & QSV_FLAG_TUNED_PLANS) tuned_options(ctx, desc->n_qubits, false, &o);
  const qsv_status st = install_plan(ctx, p.get(), o);
  if (st != QSV_OK) return st;
  *out = p.release();
  return QSV_OK;
}

qsv_status qsv_program_info_get(const qsv_program* prog, qsv_program_info* out) {
  if (!prog || !out) return QSV_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  out->n_qubits = prog->desc.n_qubits;
  out->n_clbits = prog->desc.n_clbits;
  out->n_params = prog->desc.n_params;
  out->max_events = prog->plan.max_record;
  out->n_passes = (uint32_t)prog->plan.passes.size();
  out->n_sites = (uint32_t)prog->plan.sites.size();
  out->is_unitary = prog->plan.unitary ? 1 : 0;
  return QSV_OK;
}

void qsv_program_free(qsv_program* p) {
  if (!p) return;
  ignore(enter_device(p->ctx->device));
  free_plan_buffers(p);
  delete p;
}

qsv_status qsv_run_shots(qsv_context* ctx, const qsv_program* prog, const double* theta, uint64_t n_shots,
                         const qsv_run_opts* opts, qsv_shot_results* out) {
  if (!ctx || !prog || !out) return set_err(ctx, QSV_ERR_ARG, "null argument");
  if (!owns(ctx, prog)) return set_err(ctx, QSV_ERR_ARG, "program belongs to another context");
  if (!out->creg) return set_err(ctx, QSV_ERR_ARG, "creg output is required");
  const qsv_run_opts def{};
  if (!opts) opts = &def;
  if (opts->forced_len && !opts->forced) return set_err(ctx, QSV_ERR_ARG, "forced_len without forced");
  if (prog->desc.n_params && !theta) return set_err(ctx, QSV_ERR_ARG, "theta is required");
  if (!(opts->readout_error >= 0.0 && opts->readout_error < 1.0) ||
      !(opts->reset_error >= 0.0 && opts->reset_error < 1.0))
    return set_err(ctx, QSV_ERR_ARG, "error rates must lie in [0, 1)");
  if (!(opts->depolarizing >= 0.0 && opts->depolarizing <= 1.0))
    return set_err(ctx, QSV_ERR_ARG, "the depolarizing rate must lie in [0, 1]");
  if (opts->depolarizing > 0.0 && prog->plan.noise_slot.empty())
    return set_err(ctx, QSV_ERR_ARG, "a depolarizing rate needs a program with noise slots (QSV_OP_NOISE)");
  if (n_shots == 0) return QSV_OK;
  HIP_TRY(enter_device(ctx->device));
  const Plan& pl = prog->plan;
  // noisy calls: every shot binds its own matrices (its Paulis in the slots)
  const bool noisy = opts->depolarizing > 0.0;
  const uint32_t n = prog->desc.n_qubits;
  const uint32_t cw = std::max<uint32_t>(1, (prog->desc.n_clbits + 63) / 64);
  const uint32_t maxrec = std::max<uint32_t>(1, pl.max_record);
  const uint64_t dim = 1ull << n;
  const bool c64 = (opts->flags & QSV_RUN_COMPLEX64) != 0;
  const size_t state_bytes = dim * (c64 ? sizeof(float2) : sizeof(double2));
  // state buffers are allocated in 16-byte units (two complex64 amplitudes)
  auto state_units = [&](uint64_t bufs) -> size_t { return c64 ? (size_t)((bufs * dim + 1) / 2) : (size_t)(bufs * dim); };
  // shots per batch: what fits in the arena / free memory after the per-shot scratch
  size_t per_shot = state_bytes + sizeof(ShotCtl) + cw * 8 + maxrec + opts->forced_len +
                    (size_t)prog->pblocks * kSiteBins * 8 + 4 * 256 +
                    (noisy ? pl.gate_src.size() * kMatStride * 8 + pl.dense_phases.size() : 0);
  const bool in_arena = ctx->call_arena() != nullptr;
  size_t budget = in_arena ? ctx->call_arena_bytes() : (free_device_bytes() / 10) * 8;
  size_t fixed = pl.gate_src.size() * kMatStride * 8 + prog->desc.n_params * 8 + (1u << 20) +
                 (opts->state_out ? dim * sizeof(double2) : 0);
  if (budget <= fixed + per_shot) {
    if (ctx->noalloc)
      return set_err(ctx, QSV_ERR_LIMIT,
                     "one shot of this program needs " + std::to_string(fixed + per_shot) +
                         " bytes of scratch; the no-allocation entry point has " +
                         std::to_string(kNoAllocScratchBytes));
    if (in_arena) return set_err(ctx, QSV_ERR_NOMEM, "arena too small for one shot");
    budget = fixed + per_shot;  // try anyway; hipMalloc reports the failure
  }
  uint64_t batch = std::min<uint64_t>(n_shots, (budget - fixed) / per_shot);
  batch = std::max<uint64_t>(1, std::min<uint64_t>(batch, 65535));
  Scratch scr(ctx);
  hipStream_t st = ctx->stream;
  double* d_theta = nullptr;
  double* d_mats = nullptr;
  const uint32_t n_slots = (uint32_t)pl.gate_src.size();
  HIP_TRY(scr.get(std::max<uint32_t>(1, prog->desc.n_params), &d_theta));
  // matrices: one set for the call, or one per shot of a batch when noisy
  const uint64_t ms = noisy ? (uint64_t)std::max<uint32_t>(1, n_slots) * kMatStride : 0;
  // (noisy: one more set after the shots' sets, bound without Paulis: the
  // composed matrices of every phase in which a shot draws none)
  // (a program without parameters reads the matrices composed at load; its
  // noisy calls take them as the set without Paulis)
  double* const cmats = prog->d_const_mats;
  if (noisy || !cmats)
    HIP_TRY(scr.get((size_t)std::max<uint32_t>(1, n_slots) * kMatStride * (noisy ? batch + (cmats ? 0 : 1) : 1),
                    &d_mats));
  else
    d_mats = cmats;
  const uint32_t n_dense = (uint32_t)pl.dense_phases.size();
  uint8_t* d_dirty = nullptr;
  if (noisy && n_dense) HIP_TRY(scr.get((size_t)((batch * n_dense + 3) & ~3ull), &d_dirty));
  double* d_ext = nullptr;
  if (prog->desc.n_derived) HIP_TRY(scr.get(prog->desc.n_params + prog->desc.n_derived, &d_ext));
  if (prog->desc.n_params)
    HIP_TRY(hipMemcpyAsync(d_theta, theta, prog->desc.n_params * 8, hipMemcpyHostToDevice, st));
  RunBuffers rb{};
  // state buffers: one per shot, or with trajectory sharing one per slot that
  // owns its state, grown on demand (doubling) up to one per shot
  const bool share_req = (opts->flags & QSV_RUN_SHARE_TRAJ) != 0 && !noisy;
  // a captured launch sequence: one batch, no host decisions between launches
  const bool use_graph = (opts->flags & QSV_RUN_GRAPH) != 0 && !share_req && n_shots <= batch &&
                         ctx->stream != nullptr && !ctx->noalloc;
  // binds the call's matrices (noisy: the shots of the batch, each with its
  // Paulis drawn under the batch's key, already in d_key)
  auto bind = [&](uint32_t bs) -> qsv_status {
    const double* rows = nullptr;
    uint32_t stride = 0;
    const uint32_t sets = noisy ? bs : 1u;
    if (!noisy && cmats) return QSV_OK;  // bound and composed at load
    HIP_TRY(bind_theta(prog, d_theta, 1, d_ext, st, &rows, &stride));
    HIP_TRY(launch_bind_matrices(prog->d_src, n_slots, rows, noisy ? 0u : stride,
                                 noisy ? bs + (cmats ? 0u : 1u) : 1u, d_mats, nullptr, st));
    if (noisy) {
      // the shots' Paulis, marking the phases they fall in; the set without
      // Paulis (composed at load, else after the shots' sets and composed
      // here) is copied into every phase no Pauli touched
      double* clean = cmats ? cmats : d_mats + (uint64_t)bs * ms;
      HIP_TRY(launch_noise_matrices(prog->d_noise_slot, prog->d_noise_ctr, (uint32_t)pl.noise_slot.size(),
                                    prog->d_noise, rb.key, opts->depolarizing, bs, ms, d_mats, prog->d_noise_dense,
                                    n_dense, d_dirty, st));
      if (!cmats)
        HIP_TRY(launch_compose_dense(prog->d_phases, prog->d_dense, n_dense, prog->d_gates, 1u, ms, clean, st));
      HIP_TRY(launch_compose_dense(prog->d_phases, prog->d_dense, n_dense, prog->d_gates, bs, ms, d_mats, st,
                                   d_dirty, clean));
      return QSV_OK;
    }
    HIP_TRY(launch_compose_dense(prog->d_phases, prog->d_dense, n_dense, prog->d_gates, sets, ms, d_mats, st));
    return QSV_OK;
  };
  if (!use_graph && !noisy) {
    const qsv_status bs = bind(1);
    if (bs != QSV_OK) return bs;
  }
  // (in an arena every shot's buffer is reserved up front: a bump allocator
  // cannot reuse the buffers a doubling leaves behind)
  uint64_t cap = (share_req && batch > 1 && !in_arena) ? std::min<uint64_t>(batch, 8) : batch;
  HIP_TRY(scr.get(state_units(cap), &rb.state));
  HIP_TRY(scr.get(batch, &rb.ctl));
  HIP_TRY(scr.get(batch * cw, &rb.creg));
  HIP_TRY(scr.get(batch * maxrec, &rb.record));
  HIP_TRY(scr.get(batch * prog->pblocks * kSiteBins, &rb.partials));
  uint8_t* d_forced = nullptr;
  if (opts->forced_len) HIP_TRY(scr.get(batch * opts->forced_len, &d_forced));
  double2* d_out = nullptr;
  if (opts->state_out) HIP_TRY(scr.get(dim, &d_out));
  uint64_t* d_key = nullptr;
  HIP_TRY(scr.get(2, &d_key));
  rb.key = d_key;
  rb.stride = dim;
  rb.c64 = c64 ? 1u : 0u;
  rb.cw = cw;
  rb.max_record = maxrec;
  rb.pblocks = prog->pblocks;
  rb.forced = d_forced;
  rb.forced_len = opts->forced_len;
  rb.seed = opts->seed;
  rb.readout_err = opts->readout_error;
  rb.reset_err = opts->reset_error;
  std::vector<ShotCtl> hctl(batch);
  // trajectory sharing: slot g holds one state (buffer buf_of[g]) and control
  // block for every shot s with slot_of[s] == g, i.e. the same history so far
  ShotCtl* d_slot_ctl = nullptr;
  uint32_t *d_slot_of = nullptr, *d_buf_of = nullptr, *d_rep = nullptr, *d_pairs = nullptr;
  if (share_req && batch > 1) {
    HIP_TRY(scr.get(batch, &d_slot_ctl));
    HIP_TRY(scr.get(batch, &d_slot_of));
    HIP_TRY(scr.get(batch, &d_buf_of));
    HIP_TRY(scr.get(batch, &d_rep));
    HIP_TRY(scr.get(2 * batch, &d_pairs));
  }
  std::vector<uint32_t> slot_of, buf_of, rep, pairs;
  std::vector<uint64_t> hcreg;
  std::vector<uint8_t> hrec;
  // room for `need` state buffers; a larger allocation takes over the current ones
  auto ensure_capacity = [&](uint64_t need) -> qsv_status {
    if (need <= cap) return QSV_OK;
    const uint64_t ncap = std::min<uint64_t>(batch, std::max<uint64_t>(2 * cap, need));
    double2* ns = nullptr;
    HIP_TRY(scr.get(state_units(ncap), &ns));
    HIP_TRY(hipMemcpyAsync(ns, rb.state, cap * state_bytes, hipMemcpyDeviceToDevice, st));
    rb.state = ns;
    cap = ncap;
    return QSV_OK;
  };
  uint64_t hkey[2];  // (seed, shot_base) of the current batch; stays alive until its sync
  for (uint64_t s0 = 0; s0 < n_shots; s0 += batch) {
    const uint32_t bs = (uint32_t)std::min<uint64_t>(batch, n_shots - s0);
    const bool share = share_req && bs > 1;
    rb.shots = bs;
    rb.shot_base = opts->shot_offset + s0;
    if (opts->forced_len)
      HIP_TRY(hipMemcpyAsync(d_forced, opts->forced + s0 * opts->forced_len, (size_t)bs * opts->forced_len,
                             hipMemcpyHostToDevice, st));
    hkey[0] = opts->seed;
    hkey[1] = rb.shot_base;
    HIP_TRY(hipMemcpyAsync(d_key, hkey, sizeof(hkey), hipMemcpyHostToDevice, st));
    if (use_graph) {
      // the whole launch sequence of the call, captured once and replayed
      auto issue = [&]() -> qsv_status {
        const qsv_status b = bind(bs);
        if (b != QSV_OK) return b;
        HIP_TRY(launch_init_ctl(rb.ctl, rb.creg, cw, rb.record, maxrec, bs, st));
        for (const Step& step : pl.steps) {
          if (step.kind == Step::INIT)
            HIP_TRY(launch_init_state(rb.state, rb.stride, n, bs, st, c64));
          else if (step.kind == Step::PASS)
            HIP_TRY(launch_tile_pass(rb, prog->d_gates, prog->d_phases, d_mats, ms, pl.passes[step.index], st));
          else
            HIP_TRY(launch_site(rb, pl.sites[step.index], prog->d_events, prog->d_preds, prog->d_code, st));
        }
        if (opts->state_out) HIP_TRY(launch_materialize(rb, n, 0, d_out, st));
        return QSV_OK;
      };
      auto bits = [](double x) {
        uint64_t u;
        std::memcpy(&u, &x, 8);
        return u;
      };
      const std::vector<uint64_t> gkey = {
          n_shots, opts->flags, opts->forced_len, bits(opts->readout_error), bits(opts->reset_error),
          bits(opts->depolarizing),
          opts->state_out ? 1ull : 0ull, (uint64_t)(uintptr_t)d_theta, (uint64_t)(uintptr_t)d_mats,
          (uint64_t)(uintptr_t)rb.state, (uint64_t)(uintptr_t)rb.ctl, (uint64_t)(uintptr_t)rb.creg,
          (uint64_t)(uintptr_t)rb.record, (uint64_t)(uintptr_t)rb.partials, (uint64_t)(uintptr_t)d_forced,
          (uint64_t)(uintptr_t)d_out, (uint64_t)(uintptr_t)d_key, (uint64_t)(uintptr_t)st};
      if (!prog->graph || prog->graph_key != gkey) {
        if (prog->graph) ignore(hipGraphExecDestroy(prog->graph));
        prog->graph = nullptr;
        prog->graph_key.clear();
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
        ctx->capturing = true;
        const qsv_status is = issue();
        ctx->capturing = false;
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(st, &g);
        if (is != QSV_OK || ee != hipSuccess) {
          if (g) ignore(hipGraphDestroy(g));
          clear_error();
          return is != QSV_OK ? is : set_err(ctx, QSV_ERR_DEVICE, std::string("hipStreamEndCapture: ") +
                                                                    hipGetErrorString(ee));
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        ignore(hipGraphDestroy(g));
        if (ie != hipSuccess)
          return set_err(ctx, QSV_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
        prog->graph = ex;
        prog->graph_key = gkey;
      }
      {
        Prof pr(ctx, st);
        HIP_TRY(hipGraphLaunch(prog->graph, st));
        pr.done(K_OTHER);
      }
      if (opts->state_out)
        HIP_TRY(hipMemcpyAsync(opts->state_out, d_out, dim * sizeof(double2), hipMemcpyDeviceToHost, st));
    } else {
    if (noisy) {
      const qsv_status b = bind(bs);
      if (b != QSV_OK) return b;
    }
    HIP_TRY(launch_init_ctl(rb.ctl, rb.creg, cw, rb.record, maxrec, bs, st));
    // the view the passes run on: one state per slot with the slot's control block
    RunBuffers rp = rb;
    uint32_t n_slot = bs;
    if (share) {
      n_slot = 1;
      slot_of.assign(bs, 0);
      buf_of.assign(1, 0);
      rep.assign(1, 0);
      HIP_TRY(hipMemcpyAsync(d_slot_of, slot_of.data(), bs * 4, hipMemcpyHostToDevice, st));
      HIP_TRY(hipMemcpyAsync(d_buf_of, buf_of.data(), 4, hipMemcpyHostToDevice, st));
      HIP_TRY(hipMemcpyAsync(d_rep, rep.data(), 4, hipMemcpyHostToDevice, st));
      HIP_TRY(launch_ctl_gather(d_slot_ctl, rb.ctl, d_rep, 1, st));
      rp.ctl = d_slot_ctl;
    }
    for (size_t k = 0; k < pl.steps.size(); ++k) {
      const Step& step = pl.steps[k];
      rp.shots = n_slot;
      Prof pr(ctx, st);
      if (step.kind == Step::INIT) {
        HIP_TRY(launch_init_state(rp.state, rp.stride, n, n_slot, st, c64));
        pr.done(2);
      } else if (step.kind == Step::PASS) {
        if (share) {
          // copy on write: slots that still read a parent's buffer get their own
          pairs.clear();
          for (uint32_t g = 0; g < n_slot; ++g)
            if (buf_of[g] != g) {
              pairs.push_back(g);
              pairs.push_back(buf_of[g]);
              buf_of[g] = g;
            }
          if (!pairs.empty()) {
            const qsv_status cs = ensure_capacity(n_slot);
            if (cs != QSV_OK) return cs;
            rp.state = rb.state;
            HIP_TRY(hipMemcpyAsync(d_pairs, pairs.data(), pairs.size() * 4, hipMemcpyHostToDevice, st));
            HIP_TRY(launch_buf_copy(rb.state, rb.stride, n, d_pairs, (uint32_t)pairs.size() / 2, st, c64));
            HIP_TRY(hipMemcpyAsync(d_buf_of, buf_of.data(), n_slot * 4, hipMemcpyHostToDevice, st));
            HIP_TRY(hipStreamSynchronize(st));  // the host tables change again after the uploads
          }
        }
        HIP_TRY(launch_tile_pass(rp, prog->d_gates, prog->d_phases, d_mats, ms, pl.passes[step.index], st));
        const double amps = (double)dim * n_slot;
        pr.done(0, pl.pass_uncond[step.index] != 0,
                pass_bytes_per_amp(pl.passes[step.index]) * (c64 ? 0.5 : 1.0) * amps,
                pl.pass_flops_per_amp[step.index] * amps);
      } else if (!share) {
        HIP_TRY(launch_site(rb, pl.sites[step.index], prog->d_events, prog->d_preds, prog->d_code, st));
        pr.done(1);
      } else {
        const SiteArgs& sa = pl.sites[step.index];
        // every shot takes its slot's control block (passes change only its
        // pending collapse), histograms per slot, outcomes per shot
        HIP_TRY(launch_ctl_gather(rb.ctl, d_slot_ctl, d_slot_of, bs, st));
        RunBuffers rs = rb;
        rs.slot_of = d_slot_of;
        rs.buf_of = d_buf_of;
        rs.site_ctl = d_slot_ctl;
        rs.site_slots = n_slot;
        HIP_TRY(launch_site(rs, sa, prog->d_events, prog->d_preds, prog->d_code, st));
        pr.done(1);
        if (sa.nq) {
          // split the slots by the new histories
          hcreg.resize((size_t)bs * cw);
          hrec.resize((size_t)bs * maxrec);
          HIP_TRY(hipMemcpyAsync(hctl.data(), rb.ctl, (size_t)bs * sizeof(ShotCtl), hipMemcpyDeviceToHost, st));
          HIP_TRY(hipMemcpyAsync(hcreg.data(), rb.creg, hcreg.size() * 8, hipMemcpyDeviceToHost, st));
          HIP_TRY(hipMemcpyAsync(hrec.data(), rb.record, hrec.size(), hipMemcpyDeviceToHost, st));
          HIP_TRY(hipStreamSynchronize(st));
          std::unordered_map<std::string, uint32_t> seen;
          std::vector<uint8_t> kept(n_slot, 0);
          std::string key;
          for (uint32_t sh = 0; sh < bs; ++sh) {
            const uint32_t g = slot_of[sh];
            ShotCtl c = hctl[sh];
            c.wg_done = 0;
            key.assign(reinterpret_cast<const char*>(&g), 4);
            key.append(reinterpret_cast<const char*>(&c), sizeof(c));
            key.append(reinterpret_cast<const char*>(&hcreg[(size_t)sh * cw]), (size_t)cw * 8);
            key.append(reinterpret_cast<const char*>(&hrec[(size_t)sh * maxrec]),
                       std::min<uint32_t>(c.n_record, maxrec));
            auto it = seen.find(key);
            if (it != seen.end()) {
              slot_of[sh] = it->second;
              continue;
            }
            uint32_t ng = g;
            if (kept[g]) {
              ng = n_slot++;
              buf_of.push_back(buf_of[g]);
              rep.push_back(sh);
            } else {
              kept[g] = 1;
              rep[g] = sh;
            }
            seen.emplace(key, ng);
            slot_of[sh] = ng;
          }
          HIP_TRY(hipMemcpyAsync(d_slot_of, slot_of.data(), bs * 4, hipMemcpyHostToDevice, st));
          HIP_TRY(hipMemcpyAsync(d_buf_of, buf_of.data(), n_slot * 4, hipMemcpyHostToDevice, st));
          HIP_TRY(hipMemcpyAsync(d_rep, rep.data(), n_slot * 4, hipMemcpyHostToDevice, st));
          HIP_TRY(hipStreamSynchronize(st));
        }
        HIP_TRY(launch_ctl_gather(d_slot_ctl, rb.ctl, d_rep, n_slot, st));
      }
    }
    if (share && s0 == 0 && opts->state_out) {
      // shot 0's slot reads its own buffer for the materialization
      const uint32_t g = slot_of[0];
      if (buf_of[g] != g) {
        const qsv_status cs = ensure_capacity((uint64_t)g + 1);
        if (cs != QSV_OK) return cs;
        rp.state = rb.state;
        pairs.assign({g, buf_of[g]});
        buf_of[g] = g;
        HIP_TRY(hipMemcpyAsync(d_pairs, pairs.data(), 8, hipMemcpyHostToDevice, st));
        HIP_TRY(launch_buf_copy(rb.state, rb.stride, n, d_pairs, 1, st, c64));
      }
      HIP_TRY(launch_materialize(rp, n, g, d_out, st));
      HIP_TRY(hipMemcpyAsync(opts->state_out, d_out, dim * sizeof(double2), hipMemcpyDeviceToHost, st));
    }
    if (!share && s0 == 0 && opts->state_out) {
      HIP_TRY(launch_materialize(rb, n, 0, d_out, st));
      HIP_TRY(hipMemcpyAsync(opts->state_out, d_out, dim * sizeof(double2), hipMemcpyDeviceToHost, st));
    }
    }  // eager launches
    HIP_TRY(hipMemcpyAsync(out->creg + s0 * cw, rb.creg, (size_t)bs * cw * 8, hipMemcpyDeviceToHost, st));
    if (out->record && pl.max_record) {
      if (maxrec == pl.max_record) {
        HIP_TRY(hipMemcpyAsync(out->record + s0 * pl.max_record, rb.record, (size_t)bs * maxrec,
                               hipMemcpyDeviceToHost, st));
      }
    }
    HIP_TRY(hipMemcpyAsync(hctl.data(), rb.ctl, (size_t)bs * sizeof(ShotCtl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    harvest(ctx);
    for (uint32_t s = 0; s < bs; ++s) {
      if (out->n_events) out->n_events[s0 + s] = hctl[s].n_events;
      if (out->record_prob) out->record_prob[s0 + s] = hctl[s].record_prob;
      if (out->shot_status) out->shot_status[s0 + s] = hctl[s].status;
    }
  }
  return QSV_OK;
}

qsv_status qsv_run_shots_noalloc(qsv_context* ctx, const qsv_program* prog, const double* theta,
                                 uint64_t n_shots, const qsv_run_opts* opts, qsv_shot_results* out) {
  if (!ctx) return QSV_ERR_ARG;
  if (!noalloc_scratch(ctx->device))
    return set_err(ctx, QSV_ERR_DEVICE, "no fixed scratch address for this device");
  ctx->noalloc = true;
  const qsv_status st = qsv_run_shots(ctx, prog, theta, n_shots, opts, out);
  ctx->noalloc = false;
  return st;
}

// Streamed-state requests at least this wide take the tile passes whatever
// their shot count: one workgroup per state would make their long
// trajectories the tail of the persistent launch.
constexpr uint32_t kTilePathMinWidth = 18;
// Forks (each with a host thread) that run a batch's tile-pass requests.
constexpr size_t kBatchLanes = 12;

qsv_status qsv_run_batch(qsv_context* ctx, const qsv_request* reqs, uint32_t n_reqs) {
  if (!ctx || (n_reqs && !reqs)) return set_err(ctx, QSV_ERR_ARG, "null argument");
  HIP_TRY(enter_device(ctx->device));
  std::vector<uint32_t> pers, big;
  uint32_t max_stream = 0, cw = 1, rec_max = 1;
  uint64_t items = 0;
  for (uint32_t r = 0; r < n_reqs; ++r) {
    const qsv_request& q = reqs[r];
    if (!q.prog || !owns(ctx, q.prog)) return set_err(ctx, QSV_ERR_ARG, "request " + std::to_string(r) + ": bad program");
    if (!q.out.creg) return set_err(ctx, QSV_ERR_ARG, "request " + std::to_string(r) + ": creg output is required");
    if (q.prog->desc.n_params && !q.theta) return set_err(ctx, QSV_ERR_ARG, "request " + std::to_string(r) + ": theta is required");
    if (q.opts.forced_len && !q.opts.forced) return set_err(ctx, QSV_ERR_ARG, "forced_len without forced");
    if (!(q.opts.readout_error >= 0.0 && q.opts.readout_error < 1.0) ||
        !(q.opts.reset_error >= 0.0 && q.opts.reset_error < 1.0))
      return set_err(ctx, QSV_ERR_ARG, "request " + std::to_string(r) + ": error rates must lie in [0, 1)");
    if (!q.prog->plan.noise_slot.empty() || q.opts.depolarizing != 0.0)
      return set_err(ctx, QSV_ERR_UNSUPPORTED, "request " + std::to_string(r) +
                                                   ": programs with noise slots run through qsv_run_shots");
    const uint32_t n = q.prog->desc.n_qubits;
    if (q.n_shots == 0) continue;
    // wide states, and streamed states with many shots, run on the tile-pass
    // path (decided from the request alone, so its results do not depend on
    // the rest of the batch)
    if (n > (uint32_t)kStreamMaxBits ||
        (n > (uint32_t)kResidentMaxBits && (q.n_shots >= kTilePathMinShots || n >= kTilePathMinWidth))) {
      big.push_back(r);
      continue;
    }
    pers.push_back(r);
    items += q.n_shots;
    if (n > (uint32_t)kResidentMaxBits) max_stream = std::max(max_stream, n);
    cw = std::max<uint32_t>(cw, (q.prog->desc.n_clbits + 63) / 64);
    rec_max = std::max<uint32_t>(rec_max, q.prog->plan.max_record);
  }
  if (items > 0xFFFFFFFFull) return set_err(ctx, QSV_ERR_LIMIT, "too many work items in one batch");
  hipStream_t st = ctx->stream;
  // The tile-pass requests, with shared trajectories (bit-identical to running
  // every shot from |0...0>), each as one qsv_run_shots call.
  auto run_big = [&](qsv_context* c, uint32_t lane, uint32_t stride) -> qsv_status {
    for (size_t k = lane; k < big.size(); k += stride) {
      const uint32_t r = big[k];
      qsv_run_opts o = reqs[r].opts;
      o.state_out = nullptr;
      o.flags = QSV_RUN_SHARE_TRAJ;
      qsv_shot_results out = reqs[r].out;
      const qsv_status rc = qsv_run_shots(c, reqs[r].prog, reqs[r].theta, reqs[r].n_shots, &o, &out);
      if (rc != QSV_OK) return rc;
    }
    return QSV_OK;
  };
  // With persistent work too, they run on the batch forks, each from a host
  // thread of its own (request k on lane k mod lanes), so their launches
  // overlap each other and the persistent launches. Not for a fork (forks are
  // not forked), a caller's arena (a fork would allocate), or capture.
  const uint32_t lanes = (uint32_t)std::min<size_t>(kBatchLanes, big.size());
  std::vector<qsv_status> big_rc(lanes, QSV_OK);
  std::vector<std::thread> big_th;
  struct Join {
    std::vector<std::thread>& t;
    ~Join() {
      for (std::thread& x : t)
        if (x.joinable()) x.join();
    }
  } join{big_th};
  if (lanes && !pers.empty() && !ctx->parent && !ctx->arena && !ctx->noalloc && !ctx->capturing) {
    while (ctx->batch_forks.size() < lanes) {
      qsv_context* f = nullptr;
      if (qsv_context_fork(ctx, &f) != QSV_OK) break;
      ctx->batch_forks.push_back(f);
    }
    if (!ctx->batch_ev && hipEventCreateWithFlags(&ctx->batch_ev, hipEventDisableTiming) != hipSuccess) {
      clear_error();
      ctx->batch_ev = nullptr;
    }
    if (ctx->batch_forks.size() >= lanes && ctx->batch_ev) {
      HIP_TRY(hipEventRecord(ctx->batch_ev, st));
      for (uint32_t l = 0; l < lanes; ++l) HIP_TRY(hipStreamWaitEvent(ctx->batch_forks[l]->stream, ctx->batch_ev, 0));
      for (uint32_t l = 0; l < lanes; ++l)
        big_th.emplace_back([&big_rc, &run_big, &ctx, l, lanes] {
          big_rc[l] = run_big(ctx->batch_forks[l], l, lanes);
        });
    }
  }
  if (!pers.empty()) {
    // widest circuits first: long items start early and short ones fill in
    std::stable_sort(pers.begin(), pers.end(), [&](uint32_t a, uint32_t b) {
      return reqs[a].prog->desc.n_qubits > reqs[b].prog->desc.n_qubits;
    });
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess) {
      clear_error();
      cus = 0;
    }
    if (cus <= 0) cus = 256;
    const uint32_t wgs = (uint32_t)std::min<uint64_t>(items, (uint64_t)cus * 2);
    uint64_t pers_bytes[2] = {0, 0};  // streamed-state HBM bytes of the two launches (profile)
    const uint64_t slot_amps = max_stream ? (1ull << max_stream) : 1;
    Scratch scr(ctx);
    size_t mat_total = 0, theta_total = 0, forced_total = 0;
    for (uint32_t r : pers) {
      mat_total += std::max<size_t>(1, reqs[r].prog->plan.gate_src.size()) * kMatStride;
      theta_total += std::max<uint32_t>(1, reqs[r].prog->desc.n_params);
      forced_total += reqs[r].opts.forced_len ? reqs[r].n_shots * reqs[r].opts.forced_len : 0;
    }
    double *d_mats, *d_theta;
    uint8_t* d_forced = nullptr;
    ReqDev* d_reqs;
    uint32_t *d_item_req, *d_queue;
    double2* d_scratch;
    ShotCtl* d_ctl;
    uint64_t* d_creg;
    uint8_t* d_rec;
    HIP_TRY(scr.get(mat_total, &d_mats));
    HIP_TRY(scr.get(theta_total, &d_theta));
    if (forced_total) HIP_TRY(scr.get(forced_total, &d_forced));
    HIP_TRY(scr.get(pers.size(), &d_reqs));
    HIP_TRY(scr.get(items, &d_item_req));
    HIP_TRY(scr.get(64, &d_queue));
    HIP_TRY(scr.get((size_t)wgs * slot_amps, &d_scratch));
    HIP_TRY(scr.get(items, &d_ctl));
    HIP_TRY(scr.get(items * cw, &d_creg));
    HIP_TRY(scr.get(items * rec_max, &d_rec));
    std::vector<ReqDev> rd(pers.size());
    std::vector<uint32_t> item_req(items);
    std::vector<ComposeUnit> units;  // the dense phases of every request, composed in one launch
    std::vector<BindUnit> binds;     // the matrix slots of every request, bound in one launch
    uint64_t bind_total = 0;
    size_t mo = 0, to = 0, fo = 0;
    uint32_t ib = 0;
    for (size_t i = 0; i < pers.size(); ++i) {
      const qsv_request& q = reqs[pers[i]];
      const qsv_program* p = q.prog;
      const uint32_t P = p->desc.n_params, slots = (uint32_t)p->plan.gate_src.size();
      if (P) HIP_TRY(hipMemcpyAsync(d_theta + to, q.theta, P * 8, hipMemcpyHostToDevice, st));
      double* ext = nullptr;
      if (p->desc.n_derived) HIP_TRY(scr.get(P + p->desc.n_derived, &ext));
      const double* rows = nullptr;
      uint32_t stride = 0;
      HIP_TRY(bind_theta(p, d_theta + to, 1, ext, st, &rows, &stride));
      (void)stride;  // one theta row per request
      // a program without parameters reads the matrices composed at load
      double* const rmats = p->d_const_mats ? p->d_const_mats : d_mats + mo;
      if (!p->d_const_mats) {
        binds.push_back({p->d_src, rows, rmats, bind_total});
        bind_total += slots;
        for (uint32_t ph : p->plan.dense_phases) units.push_back({p->d_phases, p->d_gates, rmats, ph, 0u});
      }
      ReqDev& R = rd[i];
      std::memset(&R, 0, sizeof(R));
      R.steps = p->d_steps;
      R.passes = p->d_passes;
      R.phases = p->d_phases;
      R.gates = p->d_gates;
      R.sites = p->d_sites;
      R.events = p->d_events;
      R.preds = p->d_preds;
      R.code = p->d_code;
      R.mats = rmats;
      if (q.opts.forced_len) {
        HIP_TRY(hipMemcpyAsync(d_forced + fo, q.opts.forced, q.n_shots * q.opts.forced_len, hipMemcpyHostToDevice, st));
        R.forced = d_forced + fo;
        fo += q.n_shots * q.opts.forced_len;
      }
      R.forced_len = q.opts.forced_len;
      R.seed = q.opts.seed;
      R.shot_offset = q.opts.shot_offset;
      R.readout_err = q.opts.readout_error;
      R.reset_err = q.opts.reset_error;
      R.n = p->desc.n_qubits;
      R.n_steps = (uint32_t)p->plan.steps.size();
      R.item_begin = ib;
      for (uint64_t k = 0; k < q.n_shots; ++k) item_req[ib + k] = (uint32_t)i;
      ib += (uint32_t)q.n_shots;
      mo += std::max<size_t>(1, slots) * kMatStride;
      to += std::max<uint32_t>(1, P);
    }
    // every request's gate matrices, then the composed 16x16 matrices of
    // their dense phases, one launch each
    if (!binds.empty()) {
      BindUnit* d_binds = nullptr;
      HIP_TRY(scr.get(binds.size(), &d_binds));
      HIP_TRY(hipMemcpyAsync(d_binds, binds.data(), binds.size() * sizeof(BindUnit), hipMemcpyHostToDevice, st));
      HIP_TRY(launch_bind_units(d_binds, (uint32_t)binds.size(), bind_total, st));
    }
    if (!units.empty()) {
      ComposeUnit* d_units = nullptr;
      HIP_TRY(scr.get(units.size(), &d_units));
      HIP_TRY(hipMemcpyAsync(d_units, units.data(), units.size() * sizeof(ComposeUnit), hipMemcpyHostToDevice, st));
      HIP_TRY(launch_compose_units(d_units, (uint32_t)units.size(), st));
    }
    // Shot branching for streamed states: the deterministic prefix (every step
    // before the first measurement) of a request with several shots runs once,
    // as one item of a first launch, into a buffer of its own; the request's
    // shots then start from that state and control block.
    {
      std::vector<ReqDev> pre;
      std::vector<uint32_t> pre_of;  // index into rd
      size_t pre_amps = 0;
      for (size_t i = 0; i < pers.size(); ++i) {
        const qsv_request& q = reqs[pers[i]];
        const Plan& pl = q.prog->plan;
        if (q.prog->desc.n_qubits <= (uint32_t)kResidentMaxBits || q.n_shots < 2) continue;
        uint32_t prefix_end = 0;
        for (const Step& s : pl.steps) {
          if (s.kind == Step::SITE && pl.sites[s.index].nq > 0) break;
          ++prefix_end;
        }
        if (prefix_end == 0) continue;
        ReqDev P = rd[i];
        P.n_steps = prefix_end;
        P.item_begin = (uint32_t)pre.size();
        P.forced = nullptr;
        P.forced_len = 0;
        pre.push_back(P);
        pre_of.push_back((uint32_t)i);
        rd[i].step_begin = prefix_end;
        pre_amps += 1ull << q.prog->desc.n_qubits;
      }
      if (!pre.empty()) {
        double2* d_pstate;
        ShotCtl* d_pctl;
        uint64_t* d_pcreg;
        uint8_t* d_prec;
        ReqDev* d_pre;
        uint32_t* d_pitem;
        HIP_TRY(scr.get(pre_amps, &d_pstate));
        HIP_TRY(scr.get(pre.size(), &d_pctl));
        HIP_TRY(scr.get(pre.size() * cw, &d_pcreg));
        HIP_TRY(scr.get(pre.size() * rec_max, &d_prec));
        HIP_TRY(scr.get(pre.size(), &d_pre));
        HIP_TRY(scr.get(pre.size(), &d_pitem));
        size_t off = 0;
        std::vector<uint32_t> pitem(pre.size());
        for (size_t k = 0; k < pre.size(); ++k) {
          pre[k].state_out = reinterpret_cast<double*>(d_pstate + off);
          rd[pre_of[k]].init_state = reinterpret_cast<const double*>(d_pstate + off);
          rd[pre_of[k]].init_ctl = d_pctl + k;
          rd[pre_of[k]].init_creg = d_pcreg + k * cw;
          off += 1ull << pre[k].n;
          pitem[k] = (uint32_t)k;
        }
        HIP_TRY(hipMemcpyAsync(d_pre, pre.data(), pre.size() * sizeof(ReqDev), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_pitem, pitem.data(), pitem.size() * 4, hipMemcpyHostToDevice, st));
        Prof pr(ctx, st);
        HIP_TRY(launch_persistent(d_pre, d_pitem, (uint32_t)pre.size(), d_queue, d_scratch, slot_amps,
                                  std::min<uint32_t>(wgs, (uint32_t)pre.size()), d_pctl, d_pcreg, cw, d_prec, rec_max,
                                  st));
        pr.done(K_PERSISTENT);
        if (ctx->profiling())
          HIP_TRY(hipMemcpyAsync(&pers_bytes[0], d_queue + 2, 8, hipMemcpyDeviceToHost, st));
      }
    }
    HIP_TRY(hipMemcpyAsync(d_reqs, rd.data(), rd.size() * sizeof(ReqDev), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(d_item_req, item_req.data(), items * 4, hipMemcpyHostToDevice, st));
    {
      Prof pr(ctx, st);
      HIP_TRY(launch_persistent(d_reqs, d_item_req, (uint32_t)items, d_queue, d_scratch, slot_amps, wgs, d_ctl,
                                d_creg, cw, d_rec, rec_max, st));
      pr.done(K_PERSISTENT);
      if (ctx->profiling())
        HIP_TRY(hipMemcpyAsync(&pers_bytes[1], d_queue + 2, 8, hipMemcpyDeviceToHost, st));
    }
    std::vector<ShotCtl> hctl(items);
    std::vector<uint64_t> hcreg(items * cw);
    std::vector<uint8_t> hrec(items * rec_max);
    HIP_TRY(hipMemcpyAsync(hctl.data(), d_ctl, items * sizeof(ShotCtl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hcreg.data(), d_creg, items * cw * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hrec.data(), d_rec, items * rec_max, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    harvest(ctx);
    ctx->prof.persistent_bytes += (double)pers_bytes[0] + (double)pers_bytes[1];
    for (size_t i = 0; i < pers.size(); ++i) {
      const qsv_request& q = reqs[pers[i]];
      const uint32_t qcw = std::max<uint32_t>(1, (q.prog->desc.n_clbits + 63) / 64);
      const uint32_t mr = q.prog->plan.max_record;
      for (uint64_t k = 0; k < q.n_shots; ++k) {
        const uint64_t it = rd[i].item_begin + k;
        std::memcpy(q.out.creg + k * qcw, &hcreg[it * cw], qcw * 8);
        if (q.out.record && mr) std::memcpy(q.out.record + k * mr, &hrec[it * rec_max], mr);
        if (q.out.n_events) q.out.n_events[k] = hctl[it].n_events;
        if (q.out.record_prob) q.out.record_prob[k] = hctl[it].record_prob;
        if (q.out.shot_status) q.out.shot_status[k] = hctl[it].status;
      }
    }
  }
  if (!big_th.empty()) {
    for (std::thread& t : big_th) t.join();
    for (uint32_t l = 0; l < lanes; ++l) {
      qsv_context* f = ctx->batch_forks[l];
      if (ctx->profiling()) {
        add_profile(&ctx->prof, f->prof);
        std::memset(&f->prof, 0, sizeof(f->prof));
      }
    }
    for (uint32_t l = 0; l < lanes; ++l)
      if (big_rc[l] != QSV_OK) return set_err(ctx, big_rc[l], ctx->batch_forks[l]->err);
    return QSV_OK;
  }
  return run_big(ctx, 0, 1);
}

}  // extern "C"

namespace {

// The Hamiltonian sweep's tile for one Hamiltonian with X masks gx: all
// qubits when the state fits a tile, else qubits 0..3 (16-amplitude runs) and
// the t - 4 others that put the most distinct X masks inside the tile (every
// choice tried while there are at most 200000, else greedily).
HamTile ham_tile(uint32_t n, const std::vector<uint64_t>& gx) {
  HamTile T{};
  const uint32_t t = std::min<uint32_t>(kTileMaxBits, n);
  T.t = t;
  uint64_t mask = (t == 64) ? ~0ull : ((1ull << t) - 1ull);
  if (n > t) {
    const uint32_t low = 4, free = n - low, k = t - low;
    auto local = [&](uint64_t m) {
      uint32_t c = 0;
      for (uint64_t x : gx) c += (x & ~m) == 0;
      return c;
    };
    double combos = 1.0;
    for (uint32_t i = 0; i < k; ++i) combos = combos * (free - i) / (i + 1);
    const uint64_t lowm = (1ull << low) - 1ull;
    if (combos <= 200000.0) {
      uint32_t best = 0;
      uint64_t bm = 0;
      for (uint64_t s = (1ull << k) - 1ull; s < (1ull << free);) {  // subsets of size k in increasing order
        const uint32_t c = local(lowm | (s << low));
        if (c > best || bm == 0) {
          best = c;
          bm = s;
        }
        const uint64_t u = s & (0ull - s), v = s + u;
        s = v + (((v ^ s) / u) >> 2);
      }
      mask = lowm | (bm << low);
    } else {
      mask = lowm;
      for (uint32_t i = 0; i < k; ++i) {
        uint32_t best = 0, bq = n;
        for (uint32_t q = low; q < n; ++q)
          if (!((mask >> q) & 1ull)) {
            const uint32_t c = local(mask | (1ull << q));
            if (bq == n || c > best) {
              best = c;
              bq = q;
            }
          }
        mask |= 1ull << bq;
      }
    }
  }
  uint32_t j = 0;
  for (uint32_t q = 0; q < n && j < t; ++q)
    if ((mask >> q) & 1ull) T.tq[j++] = (uint8_t)q;
  // the tile-index bits that pick the XCD: the outside qubits in the fewest
  // remote X masks (every choice of kXcdBits of them; ties to the lowest)
  std::vector<uint32_t> out;
  for (uint32_t q = 0; q < n; ++q)
    if (!((mask >> q) & 1ull)) out.push_back(q);
  T.nx = (uint8_t)std::min<size_t>(kXcdBits, out.size());
  auto cost = [&](uint64_t sel) {
    uint32_t c = 0;
    for (uint64_t x : gx) c += (x & sel) != 0;
    return c;
  };
  std::vector<uint32_t> best(T.nx), cur(T.nx);
  uint32_t best_c = UINT32_MAX;
  std::function<void(uint32_t, uint32_t)> pick = [&](uint32_t from, uint32_t k) {
    if (k == T.nx) {
      uint64_t sel = 0;
      for (uint32_t q : cur) sel |= 1ull << q;
      const uint32_t c = cost(sel);
      if (c < best_c) {
        best_c = c;
        best = cur;
      }
      return;
    }
    for (uint32_t i = from; i < out.size(); ++i) {
      cur[k] = out[i];
      pick(i + 1, k + 1);
    }
  };
  pick(0, 0);
  for (uint32_t k = 0; k < T.nx; ++k) T.xq[k] = (uint8_t)best[k];
  return T;
}

// h: one Hamiltonian shared by every vector (per_vector false) or h[b] for
// vector b (per_vector true).
qsv_status expval_impl(qsv_context* ctx, const qsv_program* prog, const double* theta, uint32_t batch,
                       const qsv_pauli_sum* h, double* energy, double* grad, bool per_vector = false) {
  if (!ctx || !prog || !h || !energy) return set_err(ctx, QSV_ERR_ARG, "null argument");
  if (!owns(ctx, prog)) return set_err(ctx, QSV_ERR_ARG, "program belongs to another context");
  if (!prog->plan.unitary)
    return set_err(ctx, QSV_ERR_UNSUPPORTED, "expectation values need a program without measurement or control flow");
  const uint32_t n_ham = per_vector ? batch : 1;
  for (uint32_t k = 0; k < n_ham; ++k)
    if (h[k].n_terms && (!h[k].coeff || !h[k].pauli)) return set_err(ctx, QSV_ERR_ARG, "null Hamiltonian arrays");
  if (prog->desc.n_params && !theta) return set_err(ctx, QSV_ERR_ARG, "theta is required");
  if (batch == 0) return QSV_OK;
  HIP_TRY(enter_device(ctx->device));
  const Plan& pl = prog->plan;
  const uint32_t n = prog->desc.n_qubits, P = prog->desc.n_params;
  const uint64_t dim = 1ull << n;
  const uint32_t n_slots = (uint32_t)pl.gate_src.size();
  const bool dev = (ctx->flags & QSV_FLAG_DEVICE_PTRS) != 0;
  hipStream_t st = ctx->stream;
  // Pauli strings as (x mask, z mask, #Y), every Hamiltonian's terms in a row;
  // vector b uses terms [toff[b], toff[b + 1]) (per-vector Hamiltonians only)
  std::vector<uint64_t> xm, zm;
  std::vector<uint32_t> ny, toff(1, 0);
  std::vector<double> cf;
  for (uint32_t k = 0; k < n_ham; ++k) {
    for (uint32_t t = 0; t < h[k].n_terms; ++t) {
      uint64_t x = 0, z = 0;
      uint32_t y = 0;
      for (uint32_t q = 0; q < n; ++q) {
        uint8_t c = h[k].pauli[(size_t)t * n + q];
        if (c > 3) return set_err(ctx, QSV_ERR_ARG, "Pauli code must be 0..3");
        if (c == 1 || c == 2) x |= 1ull << q;
        if (c == 3 || c == 2) z |= 1ull << q;
        if (c == 2) ++y;
      }
      xm.push_back(x);
      zm.push_back(z);
      ny.push_back(y & 3u);
      cf.push_back(h[k].coeff[t]);
    }
    toff.push_back((uint32_t)xm.size());
  }
  const uint32_t T = (uint32_t)xm.size();
  // energy partials: one per amplitude tile of the Hamiltonian sweep
  const uint32_t blocks = 1u << (n - std::min<uint32_t>(kTileMaxBits, n));
  // vectors per chunk: states (x2 with a gradient) must fit
  size_t per = dim * 16 * (grad ? 2 : 1) + (size_t)n_slots * kMatStride * 8 * (grad ? 4 : 1) +
               (size_t)blocks * 8 + P * 16 + 4096;
  // the matrix-core sweep needs its LDS on this device
  bool lds_ok = false;
  if (grad) {
    int l1 = 0, l2 = 0;
    HIP_TRY(hipDeviceGetAttribute(&l1, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    HIP_TRY(hipDeviceGetAttribute(&l2, hipDeviceAttributeSharedMemPerBlockOptin, ctx->device));
    lds_ok = (size_t)std::max(l1, l2) >= backward_mfma_lds(kTileMaxBits);
  }
  auto on_mfma = [&](size_t k) { return lds_ok && prog->bw_mfma[k] != 0; };
  auto parts_of = [&](size_t k) { return on_mfma(k) ? pl.passes[k].tiles : backward_parts(pl.passes[k]); };
  const uint32_t n_ent = lds_ok ? prog->n_ang_ent : 0;
  size_t maxg = 1;
  if (grad) {
    for (size_t k = 0; k < pl.passes.size(); ++k)
      maxg = std::max<size_t>(maxg, (size_t)parts_of(k) * pl.passes[k].gate_count * 3);
    per += maxg * 8 + (size_t)n_slots * 3 * 8 + (size_t)n_ent * 256 * 16;
  }
  size_t budget = ctx->arena ? ctx->arena_bytes : (free_device_bytes() / 10) * 8;
  uint64_t chunk = std::max<uint64_t>(1, std::min<uint64_t>(batch, (budget > 65536 ? budget - 65536 : 0) / per));
  chunk = std::min<uint64_t>(chunk, 65535);
  Scratch scr(ctx);
  // per Hamiltonian: its tile, and its terms grouped by X mask (groups in
  // ascending mask, terms in their order within a group)
  std::vector<HamTile> htiles(n_ham);
  std::vector<HamGroup> hgroups;
  std::vector<uint32_t> goff(1, 0);
  std::vector<HamTerm> gterms;
  for (uint32_t k = 0; k < n_ham; ++k) {
    std::vector<uint32_t> order;
    for (uint32_t t = toff[k]; t < toff[k + 1]; ++t) order.push_back(t);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return xm[a] < xm[b]; });
    std::vector<uint64_t> gx;
    for (uint32_t t : order)
      if (gx.empty() || gx.back() != xm[t]) gx.push_back(xm[t]);
    htiles[k] = ham_tile(n, gx);
    const HamTile& TQ = htiles[k];
    uint64_t tmask = 0;
    for (uint32_t j = 0; j < TQ.t; ++j) tmask |= 1ull << TQ.tq[j];
    for (size_t i = 0; i < order.size();) {
      HamGroup G{};
      G.x = xm[order[i]];
      G.local = (G.x & ~tmask) == 0 ? 1u : 0u;
      for (uint32_t j = 0; j < TQ.t; ++j)
        if ((G.x >> TQ.tq[j]) & 1ull) G.xl |= 1u << j;
      G.t0 = (uint32_t)gterms.size();
      size_t i1 = i;
      while (i1 < order.size() && xm[order[i1]] == G.x) ++i1;
      // real phases (#Y even) first, then imaginary, each in term order
      std::stable_sort(order.begin() + i, order.begin() + i1,
                       [&](uint32_t a, uint32_t b) { return (ny[a] & 1u) < (ny[b] & 1u); });
      G.ti = G.t0;
      for (size_t i2 = i; i2 < i1; ++i2) G.ti += (ny[order[i2]] & 1u) ? 0u : 1u;
      for (; i < i1; ++i) {
        const uint32_t k = order[i];
        HamTerm M{};
        M.zo = zm[k] & ~tmask;
        for (uint32_t j = 0; j < TQ.t; ++j)
          if ((zm[k] >> TQ.tq[j]) & 1ull) M.zl |= 1u << j;
        // i^ny = (+-1) or (+-i); (-1)^popcount((i ^ x) & z) = (-1)^popcount(x & z) (-1)^popcount(i & z)
        M.imag = ny[k] & 1u;
        const bool neg = ((ny[k] >> 1) & 1u) ^ (uint32_t)(__builtin_popcountll(G.x & zm[k]) & 1);
        M.r = neg ? -cf[k] : cf[k];
        gterms.push_back(M);
      }
      G.t1 = (uint32_t)gterms.size();
      hgroups.push_back(G);
    }
    goff.push_back((uint32_t)hgroups.size());
  }
  const uint32_t ht = htiles[0].t;  // the same for every Hamiltonian (min(12, n))
  HamTile* d_htiles = nullptr;
  HamGroup* d_hgroups = nullptr;
  uint32_t* d_goff = nullptr;
  HamTerm* d_gterms = nullptr;
  HIP_TRY(scr.get(n_ham, &d_htiles));
  HIP_TRY(scr.get(std::max<size_t>(1, hgroups.size()), &d_hgroups));
  HIP_TRY(scr.get(n_ham + 1, &d_goff));
  HIP_TRY(scr.get(std::max<uint32_t>(T, 1), &d_gterms));
  HIP_TRY(hipMemcpyAsync(d_htiles, htiles.data(), n_ham * sizeof(HamTile), hipMemcpyHostToDevice, st));
  if (!hgroups.empty())
    HIP_TRY(hipMemcpyAsync(d_hgroups, hgroups.data(), hgroups.size() * sizeof(HamGroup), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d_goff, goff.data(), goff.size() * 4, hipMemcpyHostToDevice, st));
  if (T) HIP_TRY(hipMemcpyAsync(d_gterms, gterms.data(), T * sizeof(HamTerm), hipMemcpyHostToDevice, st));
  double *d_theta, *d_mats, *d_dmats = nullptr, *d_tp, *d_energy, *d_dEda = nullptr, *d_gpart = nullptr,
                            *d_grad = nullptr;
  RunBuffers rb{};
  double2* d_lam = nullptr;
  HIP_TRY(scr.get(chunk * std::max<uint32_t>(P, 1), &d_theta));
  double* d_ext = nullptr;
  if (prog->desc.n_derived) HIP_TRY(scr.get(chunk * (P + prog->desc.n_derived), &d_ext));
  HIP_TRY(scr.get(chunk * std::max<uint32_t>(n_slots, 1) * kMatStride, &d_mats));
  HIP_TRY(scr.get(chunk * blocks, &d_tp));
  HIP_TRY(scr.get(chunk, &d_energy));
  HIP_TRY(scr.get(chunk * dim, &rb.state));
  HIP_TRY(scr.get(chunk, &rb.ctl));
  HIP_TRY(scr.get(chunk, &rb.creg));
  double* d_smats = nullptr;
  if (grad) {
    HIP_TRY(scr.get(chunk * std::max<uint32_t>(n_slots, 1) * 3 * kMatStride, &d_dmats));
    if (n_ent) HIP_TRY(scr.get(chunk * n_ent * 512, &d_smats));
    HIP_TRY(scr.get(chunk * std::max<uint32_t>(n_slots, 1) * 3, &d_dEda));
    HIP_TRY(scr.get(chunk * maxg, &d_gpart));
    HIP_TRY(scr.get(chunk * std::max<uint32_t>(P, 1), &d_grad));
    HIP_TRY(scr.get(chunk * dim, &d_lam));
  }
  rb.stride = dim;
  rb.cw = 1;
  const uint64_t ms = (uint64_t)n_slots * kMatStride;
  for (uint64_t b0 = 0; b0 < batch; b0 += chunk) {
    const uint32_t bs = (uint32_t)std::min<uint64_t>(chunk, batch - b0);
    rb.shots = bs;
    if (P)
      HIP_TRY(hipMemcpyAsync(d_theta, theta + b0 * P, (size_t)bs * P * 8,
                             dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    const double* rows = nullptr;
    uint32_t stride = 0;
    HIP_TRY(bind_theta(prog, d_theta, bs, d_ext, st, &rows, &stride));
    HIP_TRY(launch_bind_matrices(prog->d_src, n_slots, rows, stride, bs, d_mats, d_dmats, st));
    HIP_TRY(launch_compose_dense(prog->d_phases, prog->d_dense, (uint32_t)pl.dense_phases.size(), prog->d_gates, bs,
                                 ms, d_mats, st));
    if (grad && n_ent)
      HIP_TRY(launch_compose_grad(prog->d_gates, prog->d_ang_ent, n_ent, bs, ms, d_mats, d_dmats, d_smats, st));
    HIP_TRY(launch_init_ctl(rb.ctl, rb.creg, 1, nullptr, 0, bs, st));
    for (const Step& step : pl.steps) {
      Prof pr(ctx, st);
      if (step.kind == Step::INIT) {
        HIP_TRY(launch_init_state(rb.state, rb.stride, n, bs, st));
        pr.done(2);
      } else if (step.kind == Step::PASS) {
        HIP_TRY(launch_tile_pass(rb, prog->d_gates, prog->d_phases, d_mats, ms, pl.passes[step.index], st));
        const double amps = (double)dim * bs;
        pr.done(0, pl.pass_uncond[step.index] != 0, pass_bytes_per_amp(pl.passes[step.index]) * amps,
                pl.pass_flops_per_amp[step.index] * amps);
      }
    }
    // lambda = H psi (kept for the gradient) and the energy Re <psi|lambda> in one sweep
    if (T) {
      Prof pr(ctx, st);
      HIP_TRY(launch_hamiltonian(rb.state, grad ? d_lam : nullptr, dim, n, bs, d_htiles + (per_vector ? b0 : 0),
                                 per_vector ? 1u : 0u, d_hgroups, d_goff + (per_vector ? b0 : 0), d_gterms, ht,
                                 d_tp, st));
      pr.done(K_HAM, false, (grad ? 32.0 : 16.0) * (double)dim * bs);
      HIP_TRY(launch_energy_sum(d_tp, blocks, bs, d_energy, st));
    } else {
      HIP_TRY(hipMemsetAsync(d_energy, 0, bs * 8, st));
      if (grad) HIP_TRY(hipMemsetAsync(d_lam, 0, (size_t)bs * dim * sizeof(double2), st));
    }
    if (grad) {
      HIP_TRY(hipMemsetAsync(d_dEda, 0, (size_t)bs * std::max<uint32_t>(n_slots, 1) * 3 * 8, st));
      for (size_t k = pl.steps.size(); k-- > 0;) {
        const Step& step = pl.steps[k];
        if (step.kind != Step::PASS) continue;
        const PassArgs& a = pl.passes[step.index];
        Prof pr(ctx, st);
        if (on_mfma(step.index))
          HIP_TRY(launch_backward_mfma(rb.state, d_lam, dim, bs, prog->d_phases, prog->d_ang_off, prog->d_ang_ent,
                                       d_mats, ms, d_smats, n_ent, a, d_gpart, st));
        else
          HIP_TRY(launch_backward_pass(rb.state, d_lam, dim, bs, prog->d_gates, prog->d_phases, d_mats, d_dmats, ms,
                                       a, d_gpart, st));
        pr.done(K_SWEEP, false, 64.0 * (double)dim * bs);
        Prof pr2(ctx, st);
        HIP_TRY(launch_grad_reduce(d_gpart, parts_of(step.index), a.gate_count, 0, prog->d_gates + a.gate_begin, bs,
                                   std::max<uint32_t>(n_slots, 1), d_dEda, st));
        pr2.done(K_OTHER);
      }
      HIP_TRY(launch_grad_chain(d_dEda, std::max<uint32_t>(n_slots, 1), prog->d_csr_off, prog->d_csr_sj,
                                prog->d_csr_scale, P, bs, d_grad, st));
      if (P)
        HIP_TRY(hipMemcpyAsync(grad + b0 * P, d_grad, (size_t)bs * P * 8,
                               dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipMemcpyAsync(energy + b0, d_energy, (size_t)bs * 8,
                           dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    if (!dev) {
      HIP_TRY(hipStreamSynchronize(st));
      harvest(ctx);
    }
  }
  if (dev) {
    HIP_TRY(hipStreamSynchronize(st));
    harvest(ctx);
  }
  return QSV_OK;
}

}  // namespace

extern "C" {

qsv_status qsv_expval(qsv_context* ctx, const qsv_program* prog, const double* theta, uint32_t batch,
                      const qsv_pauli_sum* h, double* energy) {
  return expval_impl(ctx, prog, theta, batch, h, energy, nullptr);
}

qsv_status qsv_expval_grad(qsv_context* ctx, const qsv_program* prog, const double* theta, uint32_t batch,
                           const qsv_pauli_sum* h, double* energy, double* grad) {
  if (!grad) return set_err(ctx, QSV_ERR_ARG, "grad is required");
  return expval_impl(ctx, prog, theta, batch, h, energy, grad);
}

qsv_status qsv_expval_grad_each(qsv_context* ctx, const qsv_program* prog, const double* theta, uint32_t batch,
                                const qsv_pauli_sum* h, double* energy, double* grad) {
  if (!grad) return set_err(ctx, QSV_ERR_ARG, "grad is required");
  return expval_impl(ctx, prog, theta, batch, h, energy, grad, true);
}

qsv_status qsv_diag_copy(qsv_context* ctx, void* dst, const void* src, size_t bytes) {
  if (!ctx || !dst || !src || bytes % 16) return set_err(ctx, QSV_ERR_ARG, "bad copy arguments");
  HIP_TRY(enter_device(ctx->device));
  HIP_TRY(launch_copy(dst, src, bytes, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return QSV_OK;
}

qsv_status qsv_profile_read(qsv_context* ctx, qsv_profile* out) {
  if (!ctx || !out) return QSV_ERR_ARG;
  if (!ctx->profiling()) return set_err(ctx, QSV_ERR_ARG, "context was created without QSV_FLAG_PROFILE");
  *out = ctx->prof;
  return QSV_OK;
}

qsv_status qsv_profile_reset(qsv_context* ctx) {
  if (!ctx) return QSV_ERR_ARG;
  std::memset(&ctx->prof, 0, sizeof(ctx->prof));
  return QSV_OK;
}

// Host-only planner inspection (no device calls).
qsv_status qsv_plan_inspect(const qsv_program_desc* desc, uint32_t tile_bits, qsv_plan_stats* out) {
  if (!desc || !out) return QSV_ERR_ARG;
  if (desc->n_qubits > (uint32_t)kMaxQubits) return QSV_ERR_LIMIT;
  std::string err;
  if (!validate_program(*desc, &err)) return QSV_ERR_ARG;
  PlanOptions o;
  if (tile_bits) o.tile_bits = std::min<uint32_t>(tile_bits, kTileMaxBits);
  Plan pl = build_plan(*desc, o);
  std::memset(out, 0, sizeof(*out));
  out->n_steps = (uint32_t)pl.steps.size();
  out->n_passes = (uint32_t)pl.passes.size();
  out->n_sites = (uint32_t)pl.sites.size();
  out->n_gates = (uint32_t)pl.gates.size();
  out->n_events = (uint32_t)pl.events.size();
  out->max_record = pl.max_record;
  out->is_unitary = pl.unitary ? 1 : 0;
  out->init_step = (!pl.steps.empty() && pl.steps[0].kind == Step::INIT) ? 1 : 0;
  uint32_t k = 0;
  for (const Step& s : pl.steps) {
    if (k >= QSV_PLAN_MAX_STEPS) break;
    out->step_kind[k] = s.kind;
    if (s.kind == Step::PASS) {
      const PassArgs& a = pl.passes[s.index];
      out->step_mask[k] = a.tile_mask;
      out->step_count[k] = a.gate_count;
    } else if (s.kind == Step::SITE) {
      const SiteArgs& a = pl.sites[s.index];
      uint64_t m = 0;
      for (uint32_t j = 0; j < a.nq; ++j) m |= 1ull << a.q[j];
      out->step_mask[k] = m;
      out->step_count[k] = a.ev_count;
    }
    ++k;
  }
  // instruction index of every planned gate, in execution order, with its phase's register qubits
  uint32_t g = 0;
  out->n_phases = (uint32_t)pl.phases.size();
  out->n_dense_phases = (uint32_t)pl.dense_phases.size();
  for (size_t k = 0; k < pl.passes.size(); ++k) out->n_mfma_sweep_passes += mfma_sweep_pass(pl, k) ? 1u : 0u;
  for (const Step& s : pl.steps) {
    if (s.kind != Step::PASS) continue;
    const PassArgs& a = pl.passes[s.index];
    for (uint32_t i = 0; i < a.gate_count && g < QSV_PLAN_MAX_GATES; ++i, ++g) {
      const uint32_t gi = a.gate_begin + i;
      out->gate_instr[g] = pl.slot_instr[pl.gates[gi].mat];
      uint64_t regs = 0;
      for (uint32_t p = a.phase_begin; p < a.phase_begin + a.phase_count; ++p) {
        const Phase& ph = pl.phases[p];
        if (gi >= ph.gate_begin && gi < ph.gate_begin + ph.gate_count)
          for (int k = 0; k < kRegBits; ++k) regs |= 1ull << a.tq[ph.r[k]];
      }
      out->gate_regs[g] = regs;
    }
  }
  return QSV_OK;
}

// ---------------------------------------------------------------------------
// Plan autotuning
// ---------------------------------------------------------------------------
qsv_status qsv_program_plan_get(const qsv_program* prog, qsv_plan_options* out) {
  if (!prog || !out) return QSV_ERR_ARG;
  to_public(prog->opts, out);
  return QSV_OK;
}

qsv_status qsv_program_replan(qsv_context* ctx, qsv_program* prog, const qsv_plan_options* o) {
  if (!ctx || !prog || !o) return set_err(ctx, QSV_ERR_ARG, "null argument");
  if (prog->ctx != ctx) return set_err(ctx, QSV_ERR_ARG, "program belongs to another context");
  if (o->tile_bits < 1 || o->tile_bits > (uint32_t)kTileMaxBits || o->low_bits < 1 || o->low_bits > o->tile_bits ||
      !(o->dense_min_cost >= 0.0))
    return set_err(ctx, QSV_ERR_ARG, "plan options out of range");
  HIP_TRY(enter_device(ctx->device));
  HIP_TRY(hipStreamSynchronize(ctx->stream));  // no launch of the old plan is still running
  PlanOptions po;
  po.tile_bits = o->tile_bits;
  po.low_bits = o->low_bits;
  po.dense_min_cost = o->dense_min_cost;
  return install_plan(ctx, prog, po);
}

qsv_status qsv_autotune(qsv_context* ctx, qsv_program* prog, const double* theta, uint64_t n_shots,
                        uint32_t run_flags, qsv_tune_report* out) {
  if (!ctx || !prog || !out) return set_err(ctx, QSV_ERR_ARG, "null argument");
  if (prog->ctx != ctx) return set_err(ctx, QSV_ERR_ARG, "program belongs to another context");
  if (prog->desc.n_params && !theta) return set_err(ctx, QSV_ERR_ARG, "theta is required");
  if (n_shots == 0) return set_err(ctx, QSV_ERR_ARG, "n_shots must be positive");
  HIP_TRY(enter_device(ctx->device));
  const uint32_t n = prog->desc.n_qubits;
  const bool c64 = (run_flags & QSV_RUN_COMPLEX64) != 0;
  // candidates: the default plan first, then tile widths, the always-held low
  // qubits and the dense-phase threshold
  std::vector<PlanOptions> cand;
  auto add = [&](uint32_t t, uint32_t low, double dense) {
    PlanOptions o;
    o.tile_bits = std::min<uint32_t>(t, std::max<uint32_t>(1, n));
    o.low_bits = std::min<uint32_t>(low, o.tile_bits);
    o.dense_min_cost = dense;
    for (const PlanOptions& c : cand)
      if (c.tile_bits == o.tile_bits && c.low_bits == o.low_bits && c.dense_min_cost == o.dense_min_cost) return;
    cand.push_back(o);
  };
  const PlanOptions def;
  add(def.tile_bits, def.low_bits, def.dense_min_cost);
  for (uint32_t t : {12u, 11u, 10u})
    for (uint32_t low : {4u, 5u})
      for (double dense : {QSV_DENSE_MIN_COST, 0.0, 3.0}) add(t, low, dense);
  const uint32_t cw = std::max<uint32_t>(1, (prog->desc.n_clbits + 63) / 64);
  std::vector<uint64_t> creg((size_t)n_shots * cw);
  qsv_shot_results res{};
  res.creg = creg.data();
  qsv_run_opts ro{};
  ro.seed = 0x5eed;
  ro.flags = run_flags & (QSV_RUN_SHARE_TRAJ | QSV_RUN_COMPLEX64);
  std::vector<double> ms(cand.size(), 0.0);
  for (size_t k = 0; k < cand.size(); ++k) {
    qsv_status st = install_plan(ctx, prog, cand[k]);
    if (st != QSV_OK) return st;
    st = qsv_run_shots(ctx, prog, theta, n_shots, &ro, &res);  // first run: warm-up
    if (st != QSV_OK) return st;
    double best = 1e300;
    for (int r = 0; r < 2; ++r) {
      const auto t0 = std::chrono::steady_clock::now();
      st = qsv_run_shots(ctx, prog, theta, n_shots, &ro, &res);
      if (st != QSV_OK) return st;
      best = std::min(best, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
    }
    ms[k] = best;
  }
  const size_t b = (size_t)(std::min_element(ms.begin(), ms.end()) - ms.begin());
  const qsv_status st = install_plan(ctx, prog, cand[b]);
  if (st != QSV_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    TuneEntry& e = g_tune[tune_key(ctx->arch, n, c64)];
    e.best = cand[b];
    e.best_ms = ms[b];
    e.default_ms = ms[0];
  }
  std::memset(out, 0, sizeof(*out));
  to_public(cand[b], &out->best);
  to_public(cand[0], &out->deflt);
  out->best_ms = ms[b];
  out->default_ms = ms[0];
  out->n_candidates = (uint32_t)cand.size();
  std::snprintf(out->arch, sizeof(out->arch), "%s", ctx->arch.c_str());
  return QSV_OK;
}

qsv_status qsv_tune_lookup(qsv_context* ctx, uint32_t n_qubits, uint32_t run_flags, qsv_plan_options* out,
                           int32_t* found) {
  if (!ctx || !out || !found) return set_err(ctx, QSV_ERR_ARG, "null argument");
  PlanOptions o;
  *found = tuned_options(ctx, n_qubits, (run_flags & QSV_RUN_COMPLEX64) != 0, &o) ? 1 : 0;
  to_public(o, out);
  return QSV_OK;
}

qsv_status qsv_tune_export(char* buf, size_t cap, size_t* len) {
  if (!len) return QSV_ERR_ARG;
  std::ostringstream os;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : g_tune) {
      char line[256];
      std::snprintf(line, sizeof(line), "%s %u %u %.17g %.6g %.6g\n", kv.first.c_str(), kv.second.best.tile_bits,
                    kv.second.best.low_bits, kv.second.best.dense_min_cost, kv.second.best_ms, kv.second.default_ms);
      os << line;
    }
  }
  const std::string s = os.str();
  *len = s.size() + 1;
  if (!buf) return QSV_OK;
  if (cap < s.size() + 1) return QSV_ERR_LIMIT;
  std::memcpy(buf, s.c_str(), s.size() + 1);
  return QSV_OK;
}

qsv_status qsv_tune_import(const char* text) {
  if (!text) return QSV_ERR_ARG;
  std::istringstream is(text);
  std::string line;
  std::map<std::string, TuneEntry> add;
  while (std::getline(is, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream ls(line);
    std::string arch, prec;
    uint32_t n = 0;
    TuneEntry e;
    if (!(ls >> arch >> n >> prec >> e.best.tile_bits >> e.best.low_bits >> e.best.dense_min_cost >> e.best_ms >>
          e.default_ms))
      return QSV_ERR_ARG;
    if ((prec != "c64" && prec != "c128") || n < 1 || n > (uint32_t)kMaxQubits || e.best.tile_bits < 1 ||
        e.best.tile_bits > (uint32_t)kTileMaxBits || e.best.low_bits < 1 || e.best.low_bits > e.best.tile_bits ||
        !(e.best.dense_min_cost >= 0.0))
      return QSV_ERR_ARG;
    add[tune_key(arch, n, prec == "c64")] = e;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : add) g_tune[kv.first] = kv.second;
  return QSV_OK;
}

}  // extern "C"
