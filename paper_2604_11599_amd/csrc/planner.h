// Host-side planner: turns a validated instruction stream into the sequence of
// GPU steps (state init, tile passes, measurement sub-sites).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "qsv.h"
#include "qsv_types.h"

namespace qsv {

struct Step {
  enum Kind : uint8_t { INIT = 0, PASS = 1, SITE = 2 } kind;
  uint32_t index;  // into Plan::passes or Plan::sites
};

struct Plan {
  uint32_t n = 0;
  std::vector<Step> steps;
  std::vector<PassArgs> passes;
  std::vector<uint8_t> pass_uncond;        // 1: no gate of the pass is guarded
  std::vector<double> pass_flops_per_amp;  // algorithmic flops per amplitude of each pass
  std::vector<DGate> gates;       // gates of all passes, pass by pass (phase order)
  std::vector<Phase> phases;      // register phases of all passes
  std::vector<SiteArgs> sites;
  std::vector<SiteEvent> events;  // events of all sites, site by site
  std::vector<GateSrc> gate_src;  // one matrix slot per planned gate
  std::vector<uint32_t> slot_instr;  // instruction index of each matrix slot
  std::vector<uint32_t> dense_phases;  // phases applied as one composed 16x16 matrix
  // depolarizing slots: (matrix slot, index into the program's noise counters);
  // a slot's matrix is the identity unless a call with a positive rate binds
  // its shot's Pauli there
  std::vector<uint32_t> noise_slot, noise_ctr;
  uint32_t max_record = 0;        // measure instructions in the stream
  uint32_t max_events = 0;        // measure + reset instructions
  bool unitary = true;
  double pass_bytes_per_amp = 32.0;  // HBM bytes per amplitude per pass (read + write)
};

#ifndef QSV_DENSE_MIN_COST
#define QSV_DENSE_MIN_COST 0.5
#endif

struct PlanOptions {
  uint32_t tile_bits = kTileMaxBits;  // t_max
  uint32_t low_bits = 4;              // tile always holds qubits 0..low_bits-1 (256 B runs)
  uint32_t candidates = 8;            // seeds tried per pass by the greedy tile chooser
  bool window_seeds = true;           // also try windows of consecutive qubits as tiles
  bool register_phases = true;        // split passes into 4-qubit register phases
  double dense_min_cost = QSV_DENSE_MIN_COST;        // compose a phase into a 16x16 matrix from this gate cost on (0: never)
};

// Checks ranges and structure; on failure returns false and sets *err.
bool validate_program(const qsv_program_desc& d, std::string* err);

// Builds the plan. The stream must have passed validate_program.
Plan build_plan(const qsv_program_desc& d, const PlanOptions& opt);

// Whether the adjoint sweep of pass k can run on the matrix cores: a unitary
// program, every phase of the pass dense, 2^10..2^12 amplitudes per tile and
// at most kMaxPhaseAngles differentiated angles per phase.
bool mfma_sweep_pass(const Plan& pl, size_t k);

}  // namespace qsv
