// Internal plan and control-block types shared by the host planner and the
// gfx950 kernels. Plain-old-data only: these structs are copied to the device
// verbatim.
#pragma once
#include <stdint.h>

#include "qsv.h"

namespace qsv {

constexpr int kMaxQubits = 34;      // 2^34 complex128 = 256 GiB, the HBM ceiling of one MI355X
constexpr int kTileMaxBits = 12;    // tile = 2^12 complex128 = 64 KiB of LDS per workgroup
constexpr int kTileThreads = 256;   // workgroup size of the LDS-only tile pass
constexpr int kRegBits = 4;         // register-blocked pass: 2^4 amplitudes per thread
constexpr int kPhaseMaxGates = 32;  // gates per register phase (staged in LDS)
constexpr int kSiteQubits = 4;      // qubits histogrammed per measurement sub-site (16 bins)
constexpr int kSiteBins = 1 << kSiteQubits;
constexpr int kMatStride = 8;       // doubles per gate matrix slot (2x2 complex, row-major re, im)
constexpr int kRedThreads = 256;    // workgroup size of the probability reduction
constexpr int kRedMaxBlocks = 1024; // reduction workgroups per shot (upper bound)

// How a gate is applied inside a tile. Local bit positions refer to the tile's
// qubit list (bit k of the tile-local index <-> tile qubit k).
enum GateType : uint8_t {
  GT_DENSE1 = 0,  // 2x2 matrix on b0
  GT_DIAG1 = 1,   // diag(d0, d1) on b0 (matrix slot holds d0, d1)
  GT_X1 = 2,      // swap the b0 halves
  GT_CX = 3,      // swap the b1 halves where b0 is set
  GT_CTRL1 = 4,   // 2x2 matrix on b1 where b0 is set
  GT_CPHASE = 5,  // multiply by phase where b0 and b1 are both set (slot holds the phase)
  GT_SWAP = 6,    // exchange bits b0 and b1
};

struct DGate {      // 32 bytes (one scalar 8-dword load)
  uint8_t type, b0, b1;  // GateType; tile-local bits of the operands
  uint8_t nang;          // angles the adjoint differentiates (0 for parameter-free gates)
  uint8_t j0, j1;        // positions of b0, b1 among the register bits of the gate's phase
  uint8_t q0, q1;        // global qubits of the operands
  uint32_t mat;          // matrix slot (= index of the gate in the plan's gate array)
  uint32_t pad;
  uint64_t guard;        // active iff (flags & guard) == guard
  uint64_t pad2;
};

// Source of a gate matrix: rebuilt on the device from theta at every call.
// GateSrc kind of a depolarizing slot (QSV_OP_NOISE): bound as the identity,
// its Pauli written per shot by the noise kernel.
constexpr uint32_t kNoiseSlotKind = QSV_G_COUNT;

struct GateSrc {    // 64 bytes
  uint32_t kind;    // QSV_G_*
  uint32_t param[3];
  double scale[3];
  double offset[3];
};

// A phase of a register-blocked pass: the gates of the phase act only on the
// 4 tile-local bits r[0..3]; every thread holds the 16 amplitudes that differ
// in those bits (register k <-> local index with bit j of k on bit r[j]).
// A dense phase also has its gates' product M (16x16 complex) in kDenseSlots
// consecutive matrix slots from slot `dense`, as 256 complex values with
// M[i][c] at position (c / 4) * 64 + i + 16 (c % 4): the order in which the
// 64 lanes of a wave take their matrix-core operands. The forward pass applies
// it on the matrix cores instead of the gate list.
constexpr uint32_t kNoDense = 0xFFFFFFFFu;
constexpr int kDenseDoubles = 16 * 16 * 2;
constexpr int kDenseSlots = kDenseDoubles / kMatStride;
constexpr uint32_t kDenseMinTileBits = 10;  // full 64-lane waves of amplitude groups
constexpr uint32_t kLdsDensePhases = 4;     // dense phases a pass keeps in LDS (4 KiB each)
// One differentiated angle of a gate inside a dense phase. For the phase's
// gates G_1..G_m (applied in that order) and angle j of gate G_i, the adjoint
// sweep uses S = (G_{i-1}..G_1)^dag G_i^dag (dG_i/d angle_j) (G_{i-1}..G_1),
// composed per parameter vector and stored like a dense phase matrix.
struct AngEnt {     // 8 bytes
  uint32_t gate;    // index of G_i in the plan's gate array
  uint16_t off;     // number of gates of the phase before G_i (they start at gate - off)
  uint8_t j;        // angle of G_i
  uint8_t pad;
};
constexpr uint32_t kMaxPhaseAngles = 3 * kPhaseMaxGates;  // angles of one phase (at most 3 per gate)
constexpr uint32_t kBwWaves = 8;          // waves of that sweep's workgroup at 2^12 amplitudes

struct Phase {      // 16 bytes
  uint8_t r[kRegBits];
  uint32_t gate_begin, gate_count;
  uint32_t dense;   // first matrix slot of the composed matrix, or kNoDense
};

// A tile pass: every workgroup loads the 2^t amplitudes that share the values
// of the non-tile qubits, applies the pass's gates and stores them back.
struct PassArgs {
  uint32_t t;                    // tile bits (tile = 2^t amplitudes)
  uint32_t n;                    // qubits of the state
  uint32_t gate_begin, gate_count;
  uint32_t init;                 // 1: the state is |0...0>; generate instead of loading
  uint32_t tiles;                // workgroups per shot = 2^(n - t)
  uint64_t tile_mask;            // global bits covered by the tile
  uint8_t tq[kTileMaxBits];      // global qubit of local bit k (ascending)
  uint32_t phase_begin, phase_count;  // register-blocked phases (phase_count = 0: LDS-only pass)
  uint32_t uncond;               // 1: no gate of the pass is guarded
  uint32_t all_dense;            // 1: every phase has a composed dense matrix
};

// Sequential events of a measurement site, replayed per shot by one thread.
enum SiteOp : uint8_t {
  SE_MEASURE = 1, SE_RESET = 2, SE_SETF = 3, SE_CLRF = 4, SE_X = 5, SE_SETB = 6, SE_CLRB = 7,
  SE_CSTORE = 8  // classical bits [cbit, cbit + flag) <- expression at code[pred]
};
constexpr int kCStack = 16;  // stack depth of classical expressions

struct SiteEvent {  // 24 bytes
  uint8_t op;       // SE_*
  uint8_t k;        // index of the qubit in the site's qubit list (MEASURE/RESET)
  uint8_t flag;     // SETF/CLRF flag bit
  uint8_t pad;
  uint32_t q;       // global qubit (MEASURE/RESET/X)
  uint32_t cbit;    // MEASURE target bit or 0xFFFFFFFF; SETB/CLRB bit
  uint32_t pred;    // SETF predicate index
  uint64_t guard;
};

struct SiteArgs {
  uint32_t nq;                   // qubits histogrammed (0 = control-only site)
  uint32_t n;
  uint32_t ev_begin, ev_count;
  uint32_t blocks;               // reduction workgroups per shot
  uint32_t pad;
  uint8_t q[kSiteQubits];        // global qubits of the histogram bins
};

struct DPred {      // device copy of qsv_pred
  uint32_t lo, width;
  uint64_t value;
  uint32_t cmp, pad;
};

// Per-shot control block. The stored amplitudes `mem` relate to the logical
// state by a qubit-flip frame and a pending collapse:
//   psi[i] = ((i & pend_mask) == pend_val) ? mem[i ^ frame] * pend_scale : 0.
// X gates next to measurements and the flip of a reset only update `frame`
// (no data moves); the next tile pass that runs for the shot applies and
// clears the pending collapse.
struct ShotCtl {
  uint64_t flags;
  uint64_t pend_mask, pend_val, frame;
  double pend_scale;
  double record_prob;
  uint32_t n_events;     // measure + reset events consumed (Philox word index)
  uint32_t n_record;     // measure events recorded
  int32_t status;
  uint32_t wg_done;      // workgroups of the current pass finished for this shot
};

// Tiles of the Hamiltonian sweep: tile-local bit j <-> qubit tq[j] (ascending).
// Bits 0..nx-1 of the tile index select outside qubits xq[0..nx-1], the rest
// the other outside qubits in ascending order. Workgroups go to the XCDs
// round-robin, so those bits pick the XCD (and its L2) of a tile: chosen among
// the qubits the fewest X masks flip, they keep most partner tiles on the XCD
// that reads them.
constexpr uint32_t kXcdBits = 3;  // 8 XCDs
struct HamTile {
  uint8_t tq[kTileMaxBits];
  uint8_t xq[kXcdBits];
  uint8_t nx;
  uint32_t t;
};

// The terms of one Hamiltonian with one X mask (the qubits its Pauli string
// flips), grouped so that each amplitude reads its partner once per group.
struct HamGroup {   // 32 bytes
  uint64_t x;       // X/Y support over the global qubits
  uint32_t xl;      // the same over the tile-local bits (when local)
  uint32_t local;   // 1: x lies within the tile
  uint32_t t0, t1;  // terms [t0, t1): those with a real phase in [t0, ti), imaginary in [ti, t1)
  uint32_t ti;
  uint32_t pad;
};

// One term of a group, with its phase folded in: the term adds
//   r * (-1)^popcount(i & z) * (imag ? i : 1) * psi[i ^ x]
// to lambda[i], where r = c * (+-1) carries i^ny and (-1)^popcount(x & z), and
// the parity of i & z splits into the tile-local bits (zl, over local index
// bits) and the bits outside the tile (zo, over global qubits).
struct HamTerm {    // 24 bytes
  uint64_t zo;
  uint32_t zl;
  uint32_t imag;
  double r;
};

// Device copy of a plan step (Step in planner.h).
struct DStep {
  uint32_t kind, index;   // 0 init, 1 pass, 2 site
};

constexpr int kResidentMaxBits = 12;  // persistent kernel keeps states up to 2^12 amplitudes in LDS
constexpr int kStreamMaxBits = 20;    // larger states (up to 2^20) live in a per-workgroup HBM slot
constexpr uint64_t kTilePathMinShots = 64;  // streamed-state requests with this many shots use tile passes

// One request of a persistent batch: a loaded program, its bound matrices and
// where its shots' results go. Work item i belongs to the request whose
// [item_begin, item_begin + shots) range contains it.
struct ReqDev {
  const DStep* steps;
  const PassArgs* passes;
  const Phase* phases;
  const DGate* gates;
  const SiteArgs* sites;
  const SiteEvent* events;
  const DPred* preds;
  const qsv_cop* code;    // classical expression code
  const double* mats;
  const uint8_t* forced;  // [shots][forced_len] or null
  uint64_t seed, shot_offset;
  uint32_t n, n_steps, forced_len, item_begin;
  // Shot branching in a persistent launch: an item runs steps [step_begin,
  // n_steps). With init_state set it starts from that state, control block and
  // classical bits (the deterministic prefix, computed once per request: it
  // may assign bits before the first measurement) instead of |0...0>; with
  // state_out set (prefix items) it works in, and leaves its state in, that
  // buffer instead of the workgroup's slot.
  uint32_t step_begin, pad;
  double readout_err, reset_err;  // error rates of measurements (recorded bit) and resets
  const double* init_state;  // complex128 amplitudes (re, im)
  const ShotCtl* init_ctl;
  const uint64_t* init_creg;  // [cw] classical bits at the end of the prefix
  double* state_out;         // complex128 amplitudes (re, im)
};

}  // namespace qsv
