// Planner: validated instruction stream -> GPU steps.
//
// The stream is cut into maximal runs of gates and runs of non-unitary events
// (measure, reset, flag updates; X gates adjacent to them are folded in as
// relabelings of the index space). Gate runs become tile passes, each covering
// at most 2^t amplitudes per workgroup: the tile's qubit set T always holds
// the lowest qubits (contiguous 256-byte runs in HBM) and is grown greedily
// along the gate list, taking every gate whose qubits fit in T and whose
// earlier dependencies were taken too. Event runs become measurement
// sub-sites of at most kSiteQubits histogrammed qubits each.
#include "planner.h"

#include <algorithm>
#include <functional>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <unordered_map>

namespace qsv {

namespace {

int angle_count(uint32_t kind) {
  switch (kind) {
    case QSV_G_RX: case QSV_G_RY: case QSV_G_RZ: case QSV_G_P:
    case QSV_G_CP: case QSV_G_CRX: case QSV_G_CRY: case QSV_G_CRZ:
      return 1;
    case QSV_G_U:
      return 3;
    default:
      return 0;
  }
}

bool two_qubit(uint32_t kind) { return kind >= QSV_G_CX && kind < QSV_G_COUNT; }

// Algorithmic flops per amplitude of a gate as applied in a tile: a dense 2x2
// complex matrix-vector product costs 2 complex multiplies (6 flops each) and
// one complex add (2) per output amplitude.
// Relative cost of applying a gate from the gate list of a register phase, in
// units of one dense 2x2 gate (8 FMA per amplitude plus dispatch). A dense
// 16x16 phase product (48 matrix-core products per wave) costs about as much
// as 5 of them, but passes made only of dense phases run the eight-wave tile
// pass, which more than pays for the few light phases it makes dense, so by
// default every unguarded phase is made dense.
double gate_dispatch_cost(GateType t) {
  switch (t) {
    case GT_DENSE1: case GT_CTRL1: return 1.0;
    case GT_DIAG1: return 0.8;
    default: return 0.65;
  }
}

double gate_flops_per_amp(GateType t) {
  switch (t) {
    case GT_DENSE1: return 14.0;
    case GT_DIAG1: return 6.0;
    case GT_CTRL1: return 7.0;
    case GT_CPHASE: return 1.5;
    default: return 0.0;
  }
}

GateType gate_type(uint32_t kind) {
  switch (kind) {
    case QSV_G_X: return GT_X1;
    case QSV_G_Z: case QSV_G_S: case QSV_G_SDG: case QSV_G_T: case QSV_G_TDG:
    case QSV_G_RZ: case QSV_G_P:
      return GT_DIAG1;
    case QSV_G_CX: return GT_CX;
    case QSV_G_CY: case QSV_G_CH: case QSV_G_CRX: case QSV_G_CRY: case QSV_G_CRZ:
      return GT_CTRL1;
    case QSV_G_CZ: case QSV_G_CP: return GT_CPHASE;
    case QSV_G_SWAP: return GT_SWAP;
    default: return GT_DENSE1;
  }
}

struct GateRef {
  uint32_t instr;
  uint64_t qmask;
};

// Greedy growth of a tile qubit set from `start` along the gate list.
uint64_t grow(const std::vector<GateRef>& rem, uint64_t start, uint32_t tmax,
              std::vector<uint8_t>* taken, uint32_t* count) {
  uint64_t T = start, blocked = 0;
  uint32_t c = 0;
  taken->assign(rem.size(), 0);
  for (size_t i = 0; i < rem.size(); ++i) {
    uint64_t m = rem[i].qmask;
    if (m & blocked) {
      blocked |= m;
      continue;
    }
    uint64_t u = T | m;
    if ((uint32_t)__builtin_popcountll(u) <= tmax) {
      T = u;
      (*taken)[i] = 1;
      ++c;
    } else {
      blocked |= m;
    }
  }
  *count = c;
  return T;
}

// Reorders the gates of pass *pa into phases whose gates touch at most
// kRegBits tile-local bits, greedily (same growth rule as the tile chooser,
// on local bit masks), and records the phases.
constexpr int kLook = 2;  // further choices the phase planner looks ahead

void split_phases(Plan* plan, PassArgs* pa, uint32_t candidates) {
  std::vector<GateRef> rem;
  std::vector<DGate> src(plan->gates.begin() + pa->gate_begin,
                         plan->gates.begin() + pa->gate_begin + pa->gate_count);
  for (uint32_t i = 0; i < src.size(); ++i) {
    uint64_t m = 1ull << src[i].b0;
    if (src[i].type >= GT_CX) m |= 1ull << src[i].b1;
    rem.push_back({i, m});
  }
  std::vector<DGate> out;
  pa->phase_begin = (uint32_t)plan->phases.size();
  std::vector<uint8_t> taken, best_taken;
  while (!rem.empty()) {
    uint32_t best = 0;
    uint64_t bestR = 0;
    std::vector<uint64_t> seeds{0};
    for (size_t i = 0; i < rem.size() && seeds.size() <= candidates; ++i)
      if (std::find(seeds.begin(), seeds.end(), rem[i].qmask) == seeds.end()) seeds.push_back(rem[i].qmask);
    // windows of kRegBits consecutive local bits (consecutive qubits of the tile)
    for (uint32_t a = 0; a + kRegBits <= pa->t; ++a) {
      const uint64_t w = ((1ull << kRegBits) - 1ull) << a;
      if (std::find(seeds.begin(), seeds.end(), w) == seeds.end()) seeds.push_back(w);
    }
    // the lookahead below estimates the rest with these seeds; the choice
    // itself also tries every set of kRegBits local bits
    const std::vector<uint64_t> base_seeds = seeds;
    if (pa->t >= (uint32_t)kRegBits && pa->t <= 12u)
      for (uint64_t w = (1ull << kRegBits) - 1ull; w < (1ull << pa->t);) {
        if (std::find(seeds.begin(), seeds.end(), w) == seeds.end()) seeds.push_back(w);
        const uint64_t u = w & (0ull - w), v = w + u;
        w = v + (((v ^ w) / u) >> 2);
      }
    // phases the plain greedy choice needs for a gate list
    std::function<uint32_t(const std::vector<GateRef>&)> greedy_phases = [&](const std::vector<GateRef>& r0) {
      std::vector<GateRef> r = r0, nx;
      std::vector<uint8_t> tk;
      uint32_t np = 0;
      while (!r.empty()) {
        uint32_t bc = 0;
        std::vector<uint8_t> bt;
        for (uint64_t s : base_seeds) {
          uint32_t c = 0;
          grow(r, s, kRegBits, &tk, &c);
          if (c > bc) {
            bc = c;
            bt = tk;
          }
        }
        nx.clear();
        for (size_t i = 0; i < r.size(); ++i)
          if (!bt[i]) nx.push_back(r[i]);
        r.swap(nx);
        ++np;
      }
      return np;
    };
    struct Cand {
      uint32_t c;
      uint64_t R;
      std::vector<uint8_t> taken;
    };
    std::vector<Cand> cands;
    for (uint64_t s : seeds) {
      uint32_t c = 0;
      uint64_t R = grow(rem, s, kRegBits, &taken, &c);
      if (c) cands.push_back({c, R, taken});
    }
    std::stable_sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.c > y.c; });
    // the fewest phases for a gate list when the next kLook choices each try
    // their best few candidates and the rest is planned greedily
    // results by (depth, remaining gates): different orders of the same
    // choices leave the same rest, which is planned once per decision
    std::unordered_map<std::string, uint32_t> memo;
    const size_t words = (src.size() + 63) / 64;
    std::function<uint32_t(const std::vector<GateRef>&, int)> look = [&](const std::vector<GateRef>& r, int depth) {
      if (r.empty()) return 0u;
      std::string key(1 + 8 * words, '\0');
      key[0] = (char)depth;
      for (const GateRef& g : r) key[1 + g.instr / 8] |= (char)(1u << (g.instr % 8));
      const auto hit = memo.find(key);
      if (hit != memo.end()) return hit->second;
      if (depth == 0) return memo[key] = greedy_phases(r);
      std::vector<Cand> cs;
      std::vector<uint8_t> tk;
      for (uint64_t s : base_seeds) {
        uint32_t c = 0;
        const uint64_t R = grow(r, s, kRegBits, &tk, &c);
        if (c) cs.push_back({c, R, tk});
      }
      std::stable_sort(cs.begin(), cs.end(), [](const Cand& x, const Cand& y) { return x.c > y.c; });
      uint32_t bt = UINT32_MAX;
      for (size_t k = 0; k < cs.size() && k < 4; ++k) {
        std::vector<GateRef> rest;
        for (size_t i = 0; i < r.size(); ++i)
          if (!cs[k].taken[i]) rest.push_back(r[i]);
        bt = std::min(bt, 1 + look(rest, depth - 1));
      }
      return memo[key] = bt;
    };
    // lookahead over the best candidates: the fewest phases in total (this
    // one plus the best plan of the rest), then the most gates
    uint32_t best_total = UINT32_MAX;
    for (size_t k = 0; k < cands.size() && k < 16; ++k) {
      std::vector<GateRef> rest;
      for (size_t i = 0; i < rem.size(); ++i)
        if (!cands[k].taken[i]) rest.push_back(rem[i]);
      const uint32_t total = 1 + look(rest, kLook);
      if (total < best_total || (total == best_total && cands[k].c > best)) {
        best_total = total;
        best = cands[k].c;
        bestR = cands[k].R;
        best_taken = cands[k].taken;
      }
    }
    // pad with the highest unused local bits (keeps the low bits on lanes)
    for (int b = (int)pa->t - 1; b >= 0 && __builtin_popcountll(bestR) < kRegBits; --b) bestR |= 1ull << b;
    Phase ph;
    std::memset(&ph, 0, sizeof(ph));
    uint32_t k = 0;
    for (uint32_t b = 0; b < pa->t; ++b)
      if (bestR >> b & 1) ph.r[k++] = (uint8_t)b;
    auto pos = [&](uint8_t b) {
      for (int j = 0; j < kRegBits; ++j)
        if (ph.r[j] == b) return (uint8_t)j;
      return (uint8_t)0;
    };
    std::vector<GateRef> next;
    std::vector<DGate> chunk;
    for (size_t i = 0; i < rem.size(); ++i) {
      if (!best_taken[i]) {
        next.push_back(rem[i]);
        continue;
      }
      DGate g = src[rem[i].instr];
      g.j0 = pos(g.b0);
      g.j1 = g.type >= GT_CX ? pos(g.b1) : g.j0;
      chunk.push_back(g);
    }
    // phases longer than kPhaseMaxGates are split into consecutive phases on the same bits
    for (size_t c0 = 0; c0 < chunk.size(); c0 += kPhaseMaxGates) {
      ph.gate_begin = pa->gate_begin + (uint32_t)out.size();
      for (size_t c = c0; c < chunk.size() && c < c0 + kPhaseMaxGates; ++c) out.push_back(chunk[c]);
      ph.gate_count = pa->gate_begin + (uint32_t)out.size() - ph.gate_begin;
      plan->phases.push_back(ph);
    }
    rem.swap(next);
  }
  std::copy(out.begin(), out.end(), plan->gates.begin() + pa->gate_begin);
  pa->phase_count = (uint32_t)plan->phases.size() - pa->phase_begin;
}

}  // namespace

bool validate_program(const qsv_program_desc& d, std::string* err) {
  auto fail = [&](const std::string& m) {
    *err = m;
    return false;
  };
  if (d.n_qubits < 1) return fail("program has no qubits");
  if (d.n_instr && !d.instr) return fail("instr is NULL");
  if (d.n_pred && !d.pred) return fail("pred is NULL");
  if (d.n_clbits > (1u << 20)) return fail("too many classical bits");
  if (d.n_code && !d.code) return fail("code is NULL");
  if (d.n_lin && !d.lin) return fail("lin is NULL");
  if (d.n_derived > (1u << 20)) return fail("too many derived parameters");
  for (uint32_t i = 0; i < d.n_lin; ++i)
    if (d.lin[i].out >= d.n_derived || d.lin[i].in >= d.n_params)
      return fail("derived parameter entry " + std::to_string(i) + " out of range");
  // classical expressions: every one that a predicate or store names must end
  // within the code, read bits in range and leave exactly one value on a
  // stack of at most kCStack values
  auto expr_ok = [&](uint64_t begin, std::string* why) {
    if (begin >= d.n_code) return (*why = "expression start out of range", false);
    int depth = 0;
    for (uint64_t pc = begin; pc < d.n_code; ++pc) {
      const qsv_cop& c = d.code[pc];
      int pops = 0, pushes = 1;
      if (c.op == QSV_C_END) return depth == 1 ? true : (*why = "expression leaves a bad stack", false);
      if (c.op >= QSV_C_COUNT) return (*why = "unknown expression op", false);
      if (c.op == QSV_C_BITS) {
        if (c.width < 1 || c.width > 64 || (uint64_t)c.lo + c.width > d.n_clbits)
          return (*why = "expression bits out of range", false);
      } else if (c.op == QSV_C_NEG || c.op == QSV_C_NOT || c.op == QSV_C_LNOT) {
        pops = 1;
      } else if (c.op != QSV_C_IMM) {
        pops = 2;
      }
      if (depth < pops) return (*why = "expression stack underflow", false);
      depth += pushes - pops;
      if (depth > kCStack) return (*why = "expression stack deeper than 16", false);
    }
    return (*why = "expression does not end", false);
  };
  std::string why;
  for (uint32_t i = 0; i < d.n_pred; ++i) {
    const qsv_pred& p = d.pred[i];
    if (p.cmp > QSV_CMP_EXPR) return fail("predicate " + std::to_string(i) + ": bad comparison");
    if (p.cmp == QSV_CMP_EXPR) {
      if (!expr_ok(p.value, &why)) return fail("predicate " + std::to_string(i) + ": " + why);
    } else if (p.cmp != QSV_CMP_TRUE) {
      if (p.width < 1 || p.width > 64) return fail("predicate " + std::to_string(i) + ": width must be 1..64");
      if ((uint64_t)p.lo + p.width > d.n_clbits)
        return fail("predicate " + std::to_string(i) + ": bits out of range");
    }
  }
  for (uint32_t i = 0; i < d.n_instr; ++i) {
    const qsv_instr& in = d.instr[i];
    std::string at = "instruction " + std::to_string(i) + ": ";
    switch (in.op) {
      case QSV_OP_GATE: {
        if (in.kind >= QSV_G_COUNT) return fail(at + "unknown gate kind");
        if (in.q0 >= d.n_qubits) return fail(at + "qubit out of range");
        if (two_qubit(in.kind) && (in.q1 >= d.n_qubits || in.q1 == in.q0))
          return fail(at + "second qubit out of range or repeated");
        for (int k = 0; k < angle_count(in.kind); ++k)
          if (in.param[k] != QSV_NONE && in.param[k] >= d.n_params + d.n_derived)
            return fail(at + "parameter index out of range");
        break;
      }
      case QSV_OP_MEASURE:
        if (in.q0 >= d.n_qubits) return fail(at + "qubit out of range");
        if (in.cbit != QSV_NONE && in.cbit >= d.n_clbits) return fail(at + "classical bit out of range");
        break;
      case QSV_OP_RESET:
        if (in.q0 >= d.n_qubits) return fail(at + "qubit out of range");
        break;
      case QSV_OP_SETF:
        if (in.pred >= d.n_pred) return fail(at + "predicate out of range");
        if (in.flag >= 64) return fail(at + "flag out of range");
        break;
      case QSV_OP_CLRF:
        if (in.flag >= 64) return fail(at + "flag out of range");
        break;
      case QSV_OP_SETB: case QSV_OP_CLRB:
        if (in.cbit >= d.n_clbits) return fail(at + "classical bit out of range");
        break;
      case QSV_OP_CSTORE:
        if (in.flag < 1 || in.flag > 64 || (uint64_t)in.cbit + in.flag > d.n_clbits)
          return fail(at + "stored bits out of range");
        if (!expr_ok(in.pred, &why)) return fail(at + why);
        break;
      case QSV_OP_NOISE:
        if (in.q0 >= d.n_qubits) return fail(at + "qubit out of range");
        if (in.kind != QSV_G_ID) return fail(at + "a noise slot carries gate kind 0");
        if (in.pred >= d.n_noise || !d.noise) return fail(at + "noise counter out of range");
        break;
      default:
        return fail(at + "unknown op");
    }
  }
  return true;
}

Plan build_plan(const qsv_program_desc& d, const PlanOptions& opt) {
  Plan plan;
  const uint32_t n = d.n_qubits;
  plan.n = n;
  const uint32_t tmax = std::min<uint32_t>(opt.tile_bits, n);
  const uint32_t low = std::min<uint32_t>(opt.low_bits, tmax);
  const uint64_t low_mask = (low >= 64) ? ~0ull : ((1ull << low) - 1);

  for (uint32_t i = 0; i < d.n_instr; ++i) {
    const qsv_instr& in = d.instr[i];
    if (in.op == QSV_OP_MEASURE) ++plan.max_record, ++plan.max_events;
    if (in.op == QSV_OP_RESET) ++plan.max_events;
    if (in.op != QSV_OP_GATE) plan.unitary = false;
  }

  auto add_slot = [&](uint32_t i) {
    const qsv_instr& in = d.instr[i];
    GateSrc s;
    std::memset(&s, 0, sizeof(s));
    s.kind = in.op == QSV_OP_NOISE ? kNoiseSlotKind : in.kind;
    for (int k = 0; k < 3; ++k) {
      s.param[k] = in.op == QSV_OP_NOISE ? QSV_NONE : in.param[k];
      s.scale[k] = in.op == QSV_OP_NOISE ? 0.0 : in.scale[k];
      s.offset[k] = in.op == QSV_OP_NOISE ? 0.0 : in.offset[k];
    }
    plan.gate_src.push_back(s);
    plan.slot_instr.push_back(i);
    return (uint32_t)(plan.gate_src.size() - 1);
  };

  auto emit_gate_run = [&](const std::vector<uint32_t>& run) {
    std::vector<GateRef> rem;
    for (uint32_t i : run) {
      const qsv_instr& in = d.instr[i];
      if (in.op == QSV_OP_GATE && in.kind == QSV_G_ID) continue;
      uint64_t m = 1ull << in.q0;
      if (two_qubit(in.kind)) m |= 1ull << in.q1;
      rem.push_back({i, m});
    }
    std::vector<uint8_t> taken, best_taken;
    while (!rem.empty()) {
      uint32_t best = 0;
      uint64_t bestT = 0;
      // candidate seeds: the low qubits alone, then low qubits + each early
      // gate, then the low qubits + every window of consecutive other qubits
      // that fills the tile (nearest-neighbour circuits advance in such blocks)
      std::vector<uint64_t> seeds{low_mask};
      for (size_t i = 0; i < rem.size() && seeds.size() <= opt.candidates; ++i) {
        uint64_t s = low_mask | rem[i].qmask;
        if (std::find(seeds.begin(), seeds.end(), s) == seeds.end()) seeds.push_back(s);
      }
      if (opt.window_seeds && n > tmax) {
        const uint32_t free_bits = tmax - (uint32_t)__builtin_popcountll(low_mask);
        for (uint32_t a = low; a + free_bits <= n; ++a) {
          const uint64_t s = low_mask | (((1ull << free_bits) - 1ull) << a);
          if (std::find(seeds.begin(), seeds.end(), s) == seeds.end()) seeds.push_back(s);
        }
      }
      // greedy register-phase count of the gates a candidate tile takes, by
      // (tile, gates taken): several seeds often grow into the same tile
      std::map<std::pair<uint64_t, std::vector<uint8_t>>, uint32_t> est_memo;
      auto est_phases_raw = [&](uint64_t T, const std::vector<uint8_t>& tk) {
        std::vector<GateRef> g, nx;
        for (size_t i = 0; i < rem.size(); ++i)
          if (tk[i]) g.push_back(rem[i]);
        std::vector<uint64_t> subs;
        std::vector<uint32_t> bits;
        for (uint32_t q = 0; q < n; ++q)
          if ((T >> q) & 1ull) bits.push_back(q);
        const uint32_t nb = (uint32_t)bits.size();
        if (nb < (uint32_t)kRegBits) return 1u;
        for (uint32_t m = (1u << kRegBits) - 1u; m < (1u << nb);) {
          uint64_t sm = 0;
          for (uint32_t j = 0; j < nb; ++j)
            if ((m >> j) & 1u) sm |= 1ull << bits[j];
          subs.push_back(sm);
          const uint32_t u = m & (0u - m), v = m + u;
          m = v + (((v ^ m) / u) >> 2);
        }
        std::vector<uint8_t> t2, bt;
        uint32_t np = 0;
        while (!g.empty()) {
          uint32_t bc = 0;
          for (uint64_t sm : subs) {
            uint32_t c2 = 0;
            grow(g, sm, kRegBits, &t2, &c2);
            if (c2 > bc) {
              bc = c2;
              bt = t2;
            }
          }
          if (!bc) break;
          nx.clear();
          for (size_t i = 0; i < g.size(); ++i)
            if (!bt[i]) nx.push_back(g[i]);
          g.swap(nx);
          ++np;
        }
        return np;
      };
      auto est_phases = [&](uint64_t T, const std::vector<uint8_t>& tk) {
        const auto key = std::make_pair(T, tk);
        const auto hit = est_memo.find(key);
        if (hit != est_memo.end()) return hit->second;
        return est_memo[key] = est_phases_raw(T, tk);
      };
      // among the tiles that take at least 90 % of the most gates any seed
      // takes, the lowest estimated cost per gate: the tile's phases plus the
      // pass's own HBM read and write, which costs about 0.6 of a phase
      uint32_t cmax = 0;
      std::vector<std::pair<uint64_t, uint32_t>> grown;
      for (uint64_t s : seeds) {
        if ((uint32_t)__builtin_popcountll(s) > tmax) continue;
        uint32_t c = 0;
        grow(rem, s, tmax, &taken, &c);
        grown.push_back({s, c});
        cmax = std::max(cmax, c);
      }
      double best_score = 1e300;
      for (const auto& sc : grown) {
        if (!sc.second || sc.second * 10u < cmax * 9u) continue;
        uint32_t c = 0;
        const uint64_t T = grow(rem, sc.first, tmax, &taken, &c);
        const double score = opt.register_phases ? (0.6 + est_phases(T, taken)) / c : 1.0 / c;
        if (score < best_score) {
          best_score = score;
          best = c;
          bestT = T;
          best_taken = taken;
        }
      }
      if (best == 0) {  // cannot happen for validated streams: every gate fits a fresh tile
        bestT = low_mask | rem[0].qmask;
        best_taken.assign(rem.size(), 0);
        best_taken[0] = 1;
      }
      // pad the tile with the lowest unused qubits up to tmax bits
      for (uint32_t q = 0; q < n && (uint32_t)__builtin_popcountll(bestT) < tmax; ++q)
        bestT |= 1ull << q;
      PassArgs pa;
      std::memset(&pa, 0, sizeof(pa));
      pa.t = tmax;
      pa.n = n;
      pa.tile_mask = bestT;
      pa.tiles = 1u << (n - tmax);
      int pos[64];
      uint32_t k = 0;
      for (uint32_t q = 0; q < n; ++q)
        if (bestT >> q & 1) {
          pa.tq[k] = (uint8_t)q;
          pos[q] = (int)k++;
        }
      pa.gate_begin = (uint32_t)plan.gates.size();
      std::vector<GateRef> next;
      for (size_t i = 0; i < rem.size(); ++i) {
        if (!best_taken[i]) {
          next.push_back(rem[i]);
          continue;
        }
        const qsv_instr& in = d.instr[rem[i].instr];
        DGate g;
        std::memset(&g, 0, sizeof(g));
        // a depolarizing slot is a one-qubit gate whose matrix each shot binds
        g.type = in.op == QSV_OP_NOISE ? GT_DENSE1 : gate_type(in.kind);
        g.b0 = (uint8_t)pos[in.q0];
        g.b1 = two_qubit(in.kind) ? (uint8_t)pos[in.q1] : 0;
        g.guard = in.guard;
        g.mat = add_slot(rem[i].instr);
        bool has_param = false;
        for (int k = 0; k < angle_count(in.kind); ++k) has_param |= in.param[k] != QSV_NONE;
        g.nang = has_param ? (uint8_t)angle_count(in.kind) : 0;
        g.q0 = (uint8_t)in.q0;
        g.q1 = two_qubit(in.kind) ? (uint8_t)in.q1 : (uint8_t)in.q0;
        plan.gates.push_back(g);
      }
      pa.gate_count = (uint32_t)plan.gates.size() - pa.gate_begin;
      uint8_t uncond = 1;
      double fl = 0.0;
      for (uint32_t g = pa.gate_begin; g < pa.gate_begin + pa.gate_count; ++g) {
        if (plan.gates[g].guard) uncond = 0;
        fl += gate_flops_per_amp((GateType)plan.gates[g].type);
      }
      if (opt.register_phases && pa.t >= (uint32_t)kRegBits) split_phases(&plan, &pa, opt.candidates);
      plan.steps.push_back({Step::PASS, (uint32_t)plan.passes.size()});
      plan.passes.push_back(pa);
      plan.pass_uncond.push_back(uncond);
      plan.passes.back().uncond = uncond;
      plan.pass_flops_per_amp.push_back(fl);
      rem.swap(next);
    }
  };

  auto emit_site_run = [&](const std::vector<uint32_t>& run) {
    SiteArgs cur;
    std::memset(&cur, 0, sizeof(cur));
    cur.n = n;
    cur.ev_begin = (uint32_t)plan.events.size();
    auto close = [&]() {
      cur.ev_count = (uint32_t)plan.events.size() - cur.ev_begin;
      if (cur.ev_count == 0) return;
      uint64_t free_elems = 1ull << n;
      uint64_t blocks = free_elems / (kRedThreads * 64ull);
      cur.blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(blocks, kRedMaxBlocks));
      if (cur.nq == 0) cur.blocks = 0;
      plan.steps.push_back({Step::SITE, (uint32_t)plan.sites.size()});
      plan.sites.push_back(cur);
      std::memset(&cur, 0, sizeof(cur));
      cur.n = n;
      cur.ev_begin = (uint32_t)plan.events.size();
    };
    for (uint32_t i : run) {
      const qsv_instr& in = d.instr[i];
      SiteEvent e;
      std::memset(&e, 0, sizeof(e));
      e.guard = in.guard;
      e.cbit = 0xFFFFFFFFu;
      if (in.op == QSV_OP_MEASURE || in.op == QSV_OP_RESET) {
        int k = -1;
        for (uint32_t j = 0; j < cur.nq; ++j)
          if (cur.q[j] == in.q0) k = (int)j;
        if (k < 0) {
          if (cur.nq == (uint32_t)kSiteQubits) close();
          k = (int)cur.nq;
          cur.q[cur.nq++] = (uint8_t)in.q0;
        }
        e.op = in.op == QSV_OP_MEASURE ? SE_MEASURE : SE_RESET;
        e.k = (uint8_t)k;
        e.q = in.q0;
        if (in.op == QSV_OP_MEASURE) e.cbit = in.cbit;
      } else if (in.op == QSV_OP_SETF) {
        e.op = SE_SETF;
        e.flag = (uint8_t)in.flag;
        e.pred = in.pred;
      } else if (in.op == QSV_OP_CLRF) {
        e.op = SE_CLRF;
        e.flag = (uint8_t)in.flag;
      } else if (in.op == QSV_OP_SETB || in.op == QSV_OP_CLRB) {
        e.op = in.op == QSV_OP_SETB ? SE_SETB : SE_CLRB;
        e.cbit = in.cbit;
      } else if (in.op == QSV_OP_CSTORE) {
        e.op = SE_CSTORE;
        e.cbit = in.cbit;
        e.flag = (uint8_t)in.flag;
        e.pred = in.pred;
      } else {  // an X gate folded into the site
        e.op = SE_X;
        e.q = in.q0;
      }
      plan.events.push_back(e);
    }
    close();
  };

  // Flag updates move back over the gates before them whose guards do not
  // read the flag they write: a gate changes no classical bit or flag, and a
  // flag update reads none of the amplitudes, so the two commute. The flags of
  // an if/else that follows another if then join the site before the first
  // if's gates, and the guarded gates of both share a pass.
  std::vector<uint32_t> order(d.n_instr);
  for (uint32_t i = 0; i < d.n_instr; ++i) order[i] = i;
  for (size_t k = 0; k < order.size(); ++k) {
    const qsv_instr& in = d.instr[order[k]];
    if (in.op != QSV_OP_SETF && in.op != QSV_OP_CLRF) continue;
    const uint64_t fb = 1ull << in.flag;
    for (size_t j = k; j > 0; --j) {
      const qsv_instr& g = d.instr[order[j - 1]];
      if ((g.op != QSV_OP_GATE && g.op != QSV_OP_NOISE) || (g.guard & fb)) break;
      std::swap(order[j - 1], order[j]);
    }
  }
  // Cut the stream into gate runs and event runs.
  std::vector<uint32_t> run;
  bool in_site = false;
  for (uint32_t i : order) {
    const qsv_instr& in = d.instr[i];
    bool event = in.op != QSV_OP_GATE && in.op != QSV_OP_NOISE;
    bool foldable_x = in.op == QSV_OP_GATE && in.kind == QSV_G_X && in_site;
    if (event || foldable_x) {
      if (!in_site && !run.empty()) {
        emit_gate_run(run);
        run.clear();
      }
      in_site = true;
      run.push_back(i);
    } else {
      if (in_site && !run.empty()) {
        emit_site_run(run);
        run.clear();
      }
      in_site = false;
      run.push_back(i);
    }
  }
  if (!run.empty()) {
    if (in_site) emit_site_run(run);
    else emit_gate_run(run);
  }
  // Matrix slots in plan order: gate i of the plan reads slot i, so a pass's
  // matrices are contiguous and can be staged without an indirection.
  {
    std::vector<GateSrc> src(plan.gates.size());
    std::vector<uint32_t> instr(plan.gates.size());
    for (size_t i = 0; i < plan.gates.size(); ++i) {
      src[i] = plan.gate_src[plan.gates[i].mat];
      instr[i] = plan.slot_instr[plan.gates[i].mat];
      plan.gates[i].mat = (uint32_t)i;
      if (d.instr[instr[i]].op == QSV_OP_NOISE) {
        plan.noise_slot.push_back((uint32_t)i);
        plan.noise_ctr.push_back(d.instr[instr[i]].pred);
      }
    }
    plan.gate_src.swap(src);
    plan.slot_instr.swap(instr);
  }
  // Dense phases: an unguarded phase (of a pass with full-wave tiles) whose
  // gates would cost more than one dense 16x16 product gets its composed
  // matrix in kDenseSlots consecutive slots after the gate slots (composed on
  // the device after the gate matrices are bound); the forward pass applies it
  // instead of the gate list.
  for (Phase& ph : plan.phases) ph.dense = kNoDense;
  std::vector<uint8_t> dense_ok(plan.phases.size(), 0);
  for (const PassArgs& pa : plan.passes)
    if (pa.t >= kDenseMinTileBits)
      for (uint32_t p = pa.phase_begin; p < pa.phase_begin + pa.phase_count; ++p) dense_ok[p] = 1;
  for (uint32_t p = 0; p < plan.phases.size(); ++p) {
    Phase& ph = plan.phases[p];
    if (opt.dense_min_cost <= 0.0 || !dense_ok[p]) continue;
    double cost = 0.0;
    bool guarded = false;
    for (uint32_t g = ph.gate_begin; g < ph.gate_begin + ph.gate_count; ++g) {
      guarded |= plan.gates[g].guard != 0;
      cost += gate_dispatch_cost((GateType)plan.gates[g].type);
    }
    if (guarded || cost < opt.dense_min_cost) continue;
    ph.dense = (uint32_t)plan.gate_src.size();
    GateSrc id;
    std::memset(&id, 0, sizeof(id));
    id.kind = QSV_G_ID;
    for (int k = 0; k < 3; ++k) id.param[k] = QSV_NONE;
    for (int k = 0; k < kDenseSlots; ++k) {
      plan.gate_src.push_back(id);
      plan.slot_instr.push_back(UINT32_MAX);
    }
    plan.dense_phases.push_back(p);
  }
  for (PassArgs& pa : plan.passes) {
    pa.all_dense = pa.phase_count > 0 ? 1u : 0u;
    for (uint32_t p = pa.phase_begin; p < pa.phase_begin + pa.phase_count; ++p)
      if (plan.phases[p].dense == kNoDense) pa.all_dense = 0;
  }
  // State initialisation: folded into the first pass when the program starts with gates.
  if (!plan.steps.empty() && plan.steps[0].kind == Step::PASS) {
    plan.passes[plan.steps[0].index].init = 1;
  } else {
    plan.steps.insert(plan.steps.begin(), Step{Step::INIT, 0});
  }
  return plan;
}

bool mfma_sweep_pass(const Plan& pl, size_t k) {
  const PassArgs& a = pl.passes[k];
  if (!pl.unitary || !a.phase_count || !a.all_dense || a.t < kDenseMinTileBits || a.t > (uint32_t)kTileMaxBits)
    return false;
  for (uint32_t q = 0; q < a.phase_count; ++q) {
    const Phase& ph = pl.phases[a.phase_begin + q];
    if (ph.gate_count > 65535u) return false;
    uint32_t na = 0;
    for (uint32_t i = 0; i < ph.gate_count; ++i) na += pl.gates[ph.gate_begin + i].nang;
    if (na > kMaxPhaseAngles) return false;
  }
  return true;
}

}  // namespace qsv
