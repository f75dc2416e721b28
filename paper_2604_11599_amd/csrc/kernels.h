// Launchers of the gfx950 kernels (host-callable, C++ linkage, internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qsv_types.h"

namespace qsv {

struct RunBuffers {
  double2* state;          // [shots][2^n]
  uint64_t stride;         // amplitudes between consecutive shots
  ShotCtl* ctl;            // [shots]
  uint64_t* creg;          // [shots][cw]
  uint32_t cw;
  uint8_t* record;         // [shots][max_record]
  uint32_t max_record;
  double* partials;        // [shots][pblocks][kSiteBins]
  uint32_t pblocks;        // reduction workgroups per shot in the partials layout
  const uint8_t* forced;   // [shots][forced_len] or null
  uint32_t forced_len;
  uint64_t seed, shot_base;   // Philox key (seed, shot_base + shot)
  uint32_t shots;
  uint32_t c64;            // 1: complex64 amplitudes (state holds float2 values, same stride in amplitudes)
  double readout_err, reset_err;  // error rates of measurements (recorded bit) and resets
  // trajectory sharing (null: one state per shot): a site's histogram of
  // slot g reads state buffer buf_of[g]; shot s finalises from slot slot_of[s]
  const uint32_t* buf_of;
  const uint32_t* slot_of;
  const ShotCtl* site_ctl;  // slot control blocks the histograms follow
  uint32_t site_slots;      // slots the site reduces over
  // device copy of (seed, shot_base), read by the site finaliser instead of
  // the two fields above when set (a captured launch sequence keeps its
  // kernel arguments; the key of each call is written here before it runs)
  const uint64_t* key;
};

// Workgroups of `kernel` (threads per workgroup, bytes of dynamic LDS) that the
// current device holds at once; the first query for a kernel also raises its
// LDS limit to max_lds. Cached per device, kernel, size and LDS.
hipError_t resident_grid(const void* kernel, uint32_t threads, size_t lds, size_t max_lds, uint32_t* out);

// theta [batch][P] -> [batch][P + D] with the derived parameters appended
hipError_t launch_derive_params(const double* theta, uint32_t P, uint32_t D, const uint32_t* off, const uint32_t* in,
                                const double* coef, uint32_t batch, double* out, hipStream_t st);
// Per-shot Paulis of the depolarizing slots (rate p; key = (seed, first shot)
// in device memory, shot s uses key word 1 + s) into the shots' matrices.
// nd, n_dense, dirty: see k_noise_matrices (dirty may be null; else it is
// cleared here first, shots * n_dense bytes, rounded up to whole words).
hipError_t launch_noise_matrices(const uint32_t* slot, const uint32_t* ctr, uint32_t n, const qsv_noise* noise,
                                 const uint64_t* key, double p, uint32_t shots, uint64_t mat_stride, double* mats,
                                 const uint32_t* nd, uint32_t n_dense, uint8_t* dirty, hipStream_t st);
// One dense phase of one program to compose: phase `phase` of `phases`, its
// gates in `gates`, its matrix slots (gate matrices bound) at `mats`.
struct ComposeUnit {
  const Phase* phases;
  const DGate* gates;
  double* mats;
  uint32_t phase;
  uint32_t pad;
};
hipError_t launch_compose_units(const ComposeUnit* units, uint32_t n_units, hipStream_t st);
// The matrix slots of one program to bind: slots [slot_begin, next unit's
// slot_begin) of the flat range are slots 0.. of `src`, bound from the theta
// row `theta` into `mats`.
struct BindUnit {
  const GateSrc* src;
  const double* theta;
  double* mats;
  uint64_t slot_begin;
};
hipError_t launch_bind_units(const BindUnit* units, uint32_t n_units, uint64_t n_total, hipStream_t st);
hipError_t launch_bind_matrices(const GateSrc* src, uint32_t n_slots, const double* theta,
                                uint32_t n_params, uint32_t batch, double* mats, double* dmats,
                                hipStream_t st);
// dirty, clean: see k_compose_dense (both null: compose every phase of every batch element).
hipError_t launch_compose_dense(const Phase* phases, const uint32_t* dense, uint32_t n_dense, const DGate* gates,
                                uint32_t batch, uint64_t mat_stride, double* mats, hipStream_t st,
                                const uint8_t* dirty = nullptr, const double* clean = nullptr);
hipError_t launch_init_ctl(ShotCtl* ctl, uint64_t* creg, uint32_t cw, uint8_t* record, uint32_t max_record,
                           uint32_t shots, hipStream_t st);
hipError_t launch_init_state(double2* state, uint64_t stride, uint32_t n, uint32_t shots, hipStream_t st,
                             bool c64 = false);
hipError_t launch_tile_pass(const RunBuffers& rb, const DGate* gates, const Phase* phases, const double* mats,
                            uint64_t mat_stride, const PassArgs& a, hipStream_t st);
hipError_t launch_site(const RunBuffers& rb, const SiteArgs& a, const SiteEvent* ev,
                       const DPred* preds, const qsv_cop* code, hipStream_t st);
hipError_t launch_copy(void* dst, const void* src, uint64_t bytes, hipStream_t st);
// dst[i] = src[idx[i]] for i < count (control blocks of trajectory slots and shots)
hipError_t launch_ctl_gather(ShotCtl* dst, const ShotCtl* src, const uint32_t* idx, uint32_t count, hipStream_t st);
// state buffer pairs[2k] <- state buffer pairs[2k + 1] (2^n amplitudes each, k < n_pairs)
hipError_t launch_buf_copy(double2* state, uint64_t stride, uint32_t n, const uint32_t* pairs, uint32_t n_pairs,
                           hipStream_t st, bool c64 = false);
hipError_t launch_materialize(const RunBuffers& rb, uint32_t n, uint32_t shot, double2* out,
                              hipStream_t st);

// Persistent interpreter over (request, shot) work items.
hipError_t launch_persistent(const ReqDev* reqs, const uint32_t* item_req, uint32_t n_items, uint32_t* queue,
                             double2* scratch, uint64_t slot_amps, uint32_t workgroups, ShotCtl* out_ctl,
                             uint64_t* out_creg, uint32_t cw, uint8_t* out_rec, uint32_t rec_max, hipStream_t st);

// Expectation values and adjoint gradients over a batch of parameter vectors.
// lambda = H psi (lam may be null) and per-slice partials of Re <psi|H psi>
// (epart[batch][blocks]); launch_energy_sum reduces them to energy[batch].
// Tiles of 2^t amplitudes (t <= 12; 2^(n - t) per vector); tiles_of[h] and
// groups [goff[h], goff[h + 1]) belong to Hamiltonian h = per_vector ? b : 0;
// epart is [batch][2^(n - t)].
hipError_t launch_hamiltonian(const double2* psi, double2* lam, uint64_t stride, uint32_t n, uint32_t batch,
                              const HamTile* tiles_of, uint32_t per_vector, const HamGroup* groups,
                              const uint32_t* goff, const HamTerm* terms, uint32_t t, double* epart,
                              hipStream_t st);
hipError_t launch_energy_sum(const double* epart, uint32_t blocks, uint32_t batch, double* energy, hipStream_t st);
hipError_t launch_backward_pass(double2* psi, double2* lam, uint64_t stride, uint32_t batch,
                                const DGate* gates, const Phase* phases, const double* mats, const double* dmats,
                                uint64_t mat_stride, const PassArgs& a, double* gpart, hipStream_t st);
uint32_t backward_parts(const PassArgs& a);
// Matrix-core adjoint sweep of all-dense passes with 10 <= t <= 12: S matrices
// of the angle entries (per vector, 256 complex each), then the sweep, which
// writes per-tile partials (backward_parts = tiles).
hipError_t launch_compose_grad(const DGate* gates, const AngEnt* ent, uint32_t n_ent, uint32_t batch,
                               uint64_t mat_stride, const double* mats, const double* dmats, double* smats,
                               hipStream_t st);
size_t backward_mfma_lds(uint32_t t);
hipError_t launch_backward_mfma(double2* psi, double2* lam, uint64_t stride, uint32_t batch, const Phase* phases,
                                const uint32_t* ang_off, const AngEnt* ent, const double* mats, uint64_t mat_stride,
                                const double* smats, uint32_t n_ent, const PassArgs& a, double* gpart,
                                hipStream_t st);
hipError_t launch_grad_reduce(const double* gpart, uint32_t parts, uint32_t gate_count,
                              uint32_t slot_begin_of_pass, const DGate* gates, uint32_t batch,
                              uint32_t n_slots, double* dEda, hipStream_t st);
hipError_t launch_grad_chain(const double* dEda, uint32_t n_slots, const uint32_t* csr_off,
                             const uint32_t* csr_slot, const double* csr_scale, uint32_t n_params,
                             uint32_t batch, double* grad, hipStream_t st);

// Fixed device scratch of qsv_run_shots_noalloc: a file-scope device array of
// kNoAllocScratchBytes per device. noalloc_scratch_init(device) must run with
// `device` current (context creation does this); it looks up that device's
// address of the array once. noalloc_scratch(device) returns it (null before
// the init succeeded).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr int kNoAllocMaxDevices = 64;
hipError_t noalloc_scratch_init(int device);
void* noalloc_scratch(int device);

}  // namespace qsv
