// gfx950 kernels of expectation values and adjoint gradients (complex128).
//
// A batch of parameter vectors b holds its states at psi + b * stride.
//   k_hamiltonian / k_energy_sum   H psi and <psi|H|psi> in one sweep
//   k_backward_pass   adjoint sweep of one pass on (psi, lambda) with gradient partials
//   k_backward_r      the same on register phases
//   k_compose_grad / k_backward_mfma   the sweep of all-dense passes on the matrix cores
//   k_grad_reduce / k_grad_chain   fixed-order gradient reductions
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "device_common.h"
#include "kernels.h"

namespace qsv {

// ---------------------------------------------------------------------------
// Expectation values: H = sum_t c_t P_t with P_t = i^ny X^x Z^z (Y = i X Z).
// (P psi)[i] = i^ny (-1)^popcount((i ^ x) & z) psi[i ^ x]; lambda = H psi and
// E = Re <psi|lambda> in one sweep over the state.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 ipow(uint32_t k) {
  switch (k & 3u) {
    case 0: return make_double2(1, 0);
    case 1: return make_double2(0, 1);
    case 2: return make_double2(-1, 0);
    default: return make_double2(0, -1);
  }
}

// lambda = H psi over amplitude tiles. A workgroup stages the 2^t amplitudes
// of one tile of vector b in LDS (the tile holds qubits 0..3, so every
// global access is a run of 16 amplitudes, and the qubits that put the most
// distinct X masks of its Hamiltonian inside the tile), then sums the
// Hamiltonian's groups of terms with equal X mask x for each of them:
//   lambda[i] += psi[i ^ x] * sum_t r_t (-1)^popcount(i & z_t) (i or 1)
// reading psi[i ^ x] from LDS when x lies within the tile, else from memory
// (a run of the partner tile), groups in ascending x; within a group the
// terms with a real phase first, then those with an imaginary one, each part
// one real sum f and two multiply-adds per amplitude. Thread tid holds local indices l_j = tid | (j << 9): the
// sign's parity over the bits outside the tile is the same for the whole
// workgroup, over local bits 9..11 the same for every thread, so only
// popcount(tid & zl) is per thread. The energy partial of the tile,
// Re sum conj(psi) lambda, goes to epart[b][tile] (fixed-order tree).
constexpr uint32_t kHamThreads = 512;
constexpr uint32_t kHamPerThread = (1u << kTileMaxBits) / kHamThreads;  // 8

__global__ __launch_bounds__(kHamThreads, 4) void k_hamiltonian(
    const double2* __restrict__ psi, double2* __restrict__ lam, uint64_t stride, uint32_t n,
    const HamTile* __restrict__ tiles_of, uint32_t per_vector, const HamGroup* __restrict__ groups,
    const uint32_t* __restrict__ goff, const HamTerm* __restrict__ terms, uint32_t n_tiles,
    double* __restrict__ epart) {
  extern __shared__ double2 tl[];
  __shared__ uint64_t lut[128];
  __shared__ double red[kHamThreads];
  const uint32_t tid = threadIdx.x, tile = blockIdx.x, b = blockIdx.y, h = per_vector ? b : 0u;
  const HamTile* TQ = tiles_of + h;
  const uint32_t t = TQ->t, T = 1u << t;
  // local index -> global bits: low six local bits through lut[0..63], the rest through lut[64..127]
  if (tid < 128) {
    const uint32_t k = tid & 63u, hi = tid >> 6;
    uint64_t m = 0;
    for (uint32_t j = 0; j < 6; ++j)
      if (hi * 6 + j < t && ((k >> j) & 1u)) m |= 1ull << TQ->tq[hi * 6 + j];
    lut[tid] = m;
  }
  uint64_t tmask = 0;
  for (uint32_t j = 0; j < t; ++j) tmask |= 1ull << TQ->tq[j];
  uint64_t base = 0;  // the tile index scattered over the qubits outside the tile
  {
    uint64_t xm = 0;
    for (uint32_t j = 0; j < TQ->nx; ++j) {
      base |= (uint64_t)((tile >> j) & 1u) << TQ->xq[j];
      xm |= 1ull << TQ->xq[j];
    }
    uint32_t k = TQ->nx;
    for (uint32_t q = 0; q < n; ++q)
      if (!(((tmask | xm) >> q) & 1ull)) base |= (uint64_t)((tile >> k++) & 1u) << q;
  }
  __syncthreads();
  const double2* st = psi + (uint64_t)b * stride;
  for (uint32_t l = tid; l < T; l += kHamThreads) tl[l] = st[base | lut[l & 63u] | lut[64 + (l >> 6)]];
  __syncthreads();
  // this thread's amplitudes: j < cnt (cnt = 0 when the tile is smaller than tid)
  const uint32_t cnt = T >= kHamThreads ? T / kHamThreads : (tid < T ? 1u : 0u);
  uint64_t gi[kHamPerThread];
#pragma unroll
  for (uint32_t j = 0; j < kHamPerThread; ++j) gi[j] = base | lut[tid & 63u] | lut[64 + (((tid >> 6) | (j << 3)) & 63u)];
  double2 acc[kHamPerThread];
#pragma unroll
  for (uint32_t j = 0; j < kHamPerThread; ++j) acc[j] = make_double2(0.0, 0.0);
  // f[j] = sum over terms [k0, k1) of r (-1)^popcount(i_j & z): the sign's
  // parity over the workgroup's bits outside the tile and over local bits
  // 9..11 (j) is uniform, only tid & zl is per thread
  auto add_term = [&](uint32_t k, bool first, double* f) {
    const HamTerm M = terms[k];
    const double sl = (__popc(tid & M.zl) & 1) ? -1.0 : 1.0;
    const uint32_t pw = (uint32_t)__popcll(base & M.zo);
#pragma unroll
    for (uint32_t j = 0; j < kHamPerThread; ++j) {
      const double c = ((pw + (uint32_t)__popc((j << 9) & M.zl)) & 1u) ? -M.r : M.r;
      f[j] = first ? sl * c : fma(sl, c, f[j]);
    }
  };
  auto sum_terms = [&](uint32_t k0, uint32_t k1, double* f) {  // k0 < k1
    add_term(k0, true, f);
    for (uint32_t k = k0 + 1; k < k1; ++k) add_term(k, false, f);
  };
  const uint32_t g0 = goff[h], g1 = goff[h + 1];
  if (cnt) {
    for (uint32_t g = g0; g < g1; ++g) {
      const HamGroup G = groups[g];
      double2 v[kHamPerThread];
      if (G.local) {
#pragma unroll
        for (uint32_t j = 0; j < kHamPerThread; ++j) v[j] = tl[((tid | (j << 9)) ^ G.xl) & (T - 1u)];
      } else {
#pragma unroll
        for (uint32_t j = 0; j < kHamPerThread; ++j) v[j] = j < cnt ? st[gi[j] ^ G.x] : make_double2(0.0, 0.0);
      }
      double f[kHamPerThread];
      if (G.t0 < G.ti) {  // terms with a real phase: lambda += f psi
        sum_terms(G.t0, G.ti, f);
#pragma unroll
        for (uint32_t j = 0; j < kHamPerThread; ++j) {
          acc[j].x = fma(f[j], v[j].x, acc[j].x);
          acc[j].y = fma(f[j], v[j].y, acc[j].y);
        }
      }
      if (G.ti < G.t1) {  // terms with an imaginary phase: lambda += i f psi
        sum_terms(G.ti, G.t1, f);
#pragma unroll
        for (uint32_t j = 0; j < kHamPerThread; ++j) {
          acc[j].x = fma(-f[j], v[j].y, acc[j].x);
          acc[j].y = fma(f[j], v[j].x, acc[j].y);
        }
      }
    }
  }
  double e = 0.0;
#pragma unroll
  for (uint32_t j = 0; j < kHamPerThread; ++j)
    if (j < cnt) {
      if (lam) lam[(uint64_t)b * stride + gi[j]] = acc[j];
      const double2 p = tl[tid | (j << 9)];
      e += p.x * acc[j].x + p.y * acc[j].y;
    }
  red[tid] = e;
  __syncthreads();
  for (uint32_t s = kHamThreads / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) epart[(uint64_t)b * n_tiles + tile] = red[0];
}

hipError_t launch_hamiltonian(const double2* psi, double2* lam, uint64_t stride, uint32_t n, uint32_t batch,
                              const HamTile* tiles_of, uint32_t per_vector, const HamGroup* groups,
                              const uint32_t* goff, const HamTerm* terms, uint32_t t, double* epart,
                              hipStream_t st) {
  if (t > kTileMaxBits || t > n) return hipErrorInvalidValue;
  const uint32_t n_tiles = 1u << (n - t);
  hipLaunchKernelGGL(k_hamiltonian, dim3(n_tiles, batch), dim3(kHamThreads), sizeof(double2) << t, st, psi, lam,
                     stride, n, tiles_of, per_vector, groups, goff, terms, n_tiles, epart);
  return hipGetLastError();
}

// energy[b] = sum over blk of epart[b][blk]: one workgroup per vector, strided
// partial sums then a tree, both in a fixed order
__global__ __launch_bounds__(256) void k_energy_sum(const double* __restrict__ epart, uint32_t blocks,
                                                   double* __restrict__ energy) {
  __shared__ double red[256];
  const uint32_t tid = threadIdx.x, b = blockIdx.x;
  double v = 0.0;
  for (uint32_t k = tid; k < blocks; k += 256) v += epart[(uint64_t)b * blocks + k];
  red[tid] = v;
  __syncthreads();
  for (uint32_t s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) energy[b] = red[0];
}

hipError_t launch_energy_sum(const double* epart, uint32_t blocks, uint32_t batch, double* energy, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_sum, dim3(batch), dim3(256), 0, st, epart, blocks, energy);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint sweep of one pass: for the pass's gates in reverse order,
//   psi <- U^dag psi ; g_j = 2 Re <lam| dU/da_j |psi> ; lam <- U^dag lam
// Partial gradient sums per workgroup: gpart[b][tile][gate][angle].
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cdot_conj(double2 l, double2 v) {  // conj(l) * v
  return make_double2(l.x * v.x + l.y * v.y, l.x * v.y - l.y * v.x);
}

__device__ double block_sum(double v, double* red) {
  const uint32_t tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (uint32_t s = kTileThreads / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kTileThreads) void k_backward_pass(
    double2* __restrict__ psi, double2* __restrict__ lam, uint64_t stride, const DGate* __restrict__ gates,
    const double* __restrict__ mats, const double* __restrict__ dmats, uint64_t mat_stride, PassArgs a,
    double* __restrict__ gpart) {
  extern __shared__ double2 sm[];
  __shared__ double red[kTileThreads];
  const uint32_t T = 1u << a.t;
  double2* tp = sm;
  double2* tl = sm + T;
  const uint32_t b = blockIdx.y, w = blockIdx.x, tid = threadIdx.x;
  uint64_t base = 0;
  {
    uint32_t k = 0;
    for (uint32_t q = 0; q < a.n; ++q)
      if (!((a.tile_mask >> q) & 1ull)) base |= (uint64_t)((w >> k++) & 1u) << q;
  }
  double2* sp = psi + (uint64_t)b * stride;
  double2* sl = lam + (uint64_t)b * stride;
  for (uint32_t l = tid; l < T; l += kTileThreads) {
    uint64_t gi = base | local_to_global(l, a);
    tp[l] = sp[gi];
    tl[l] = sl[gi];
  }
  __syncthreads();
  const double* mb = mats + (uint64_t)b * mat_stride;
  const double* db = dmats + (uint64_t)b * mat_stride * 3;
  for (int32_t gi = (int32_t)a.gate_count - 1; gi >= 0; --gi) {
    const DGate g = gates[a.gate_begin + gi];
    const double* m = mb + (uint64_t)g.mat * kMatStride;
    const double* dm = db + (uint64_t)g.mat * 3 * kMatStride;
    // U^dag on psi
    M2 u = load_m2(m, 0);
    M2 ud;
    ud.a = cconj(u.a);
    ud.b = cconj(u.c);
    ud.c = cconj(u.b);
    ud.d = cconj(u.d);
    const bool one = (g.type == GT_DENSE1 || g.type == GT_DIAG1 || g.type == GT_X1);
    const uint32_t B0 = 1u << g.b0, B1 = 1u << g.b1;
    const uint32_t lo = g.b0 < g.b1 ? g.b0 : g.b1, hi = g.b0 < g.b1 ? g.b1 : g.b0;
    const uint32_t cnt = one ? (T >> 1) : (T >> 2);
    // indices of the 2-vector the gate acts on
    auto pair = [&](uint32_t p, uint32_t* i0, uint32_t* i1) {
      if (one) {
        *i0 = ins0(p, g.b0);
        *i1 = *i0 | B0;
      } else {
        uint32_t i = ins0(ins0(p, lo), hi) | B0;
        *i0 = i;
        *i1 = i | B1;
      }
    };
    if (g.type == GT_SWAP) {
      for (uint32_t p = tid; p < cnt; p += kTileThreads) {
        uint32_t i = ins0(ins0(p, lo), hi);
        double2 x = tp[i | B0];
        tp[i | B0] = tp[i | B1];
        tp[i | B1] = x;
        x = tl[i | B0];
        tl[i | B0] = tl[i | B1];
        tl[i | B1] = x;
      }
      __syncthreads();
      continue;
    }
    // psi <- U^dag psi
    for (uint32_t p = tid; p < cnt; p += kTileThreads) {
      uint32_t i0, i1;
      pair(p, &i0, &i1);
      double2 x0 = tp[i0], x1 = tp[i1];
      tp[i0] = cmac2(ud.a, x0, ud.b, x1);
      tp[i1] = cmac2(ud.c, x0, ud.d, x1);
    }
    __syncthreads();
    // gradient partials for each angle the gate depends on (at most 3)
    const uint32_t nang = g.nang;
    for (uint32_t j = 0; j < nang; ++j) {
      M2 d = load_m2(dm + j * kMatStride, 0);
      double acc = 0.0;
      for (uint32_t p = tid; p < cnt; p += kTileThreads) {
        uint32_t i0, i1;
        pair(p, &i0, &i1);
        double2 x0 = tp[i0], x1 = tp[i1];
        double2 y0 = cmac2(d.a, x0, d.b, x1), y1 = cmac2(d.c, x0, d.d, x1);
        acc += cdot_conj(tl[i0], y0).x + cdot_conj(tl[i1], y1).x;
      }
      double tot = block_sum(acc, red);
      if (tid == 0)
        gpart[(((uint64_t)b * a.tiles + w) * a.gate_count + gi) * 3 + j] = 2.0 * tot;
    }
    // lam <- U^dag lam
    for (uint32_t p = tid; p < cnt; p += kTileThreads) {
      uint32_t i0, i1;
      pair(p, &i0, &i1);
      double2 x0 = tl[i0], x1 = tl[i1];
      tl[i0] = cmac2(ud.a, x0, ud.b, x1);
      tl[i1] = cmac2(ud.c, x0, ud.d, x1);
    }
    __syncthreads();
  }
  for (uint32_t l = tid; l < T; l += kTileThreads) {
    uint64_t gi = base | local_to_global(l, a);
    sp[gi] = tp[l];
    sl[gi] = tl[l];
  }
}


// ---------------------------------------------------------------------------
// Register-blocked adjoint sweep of one pass (psi and lambda together).
//
// Both tiles live in registers, 16 + 16 amplitudes per thread, in the mapping
// of the current phase; LDS (one 2^t buffer) only re-maps one state at a time
// between phases. Phases and the gates inside them run in reverse order:
//   psi <- U^dag psi ; g_j = 2 Re <lambda| dU/da_j |psi> ; lambda <- U^dag lambda
// Per-gate partial gradients are reduced over each wave with shuffles and
// stored per (tile, wave); k_grad_reduce sums them in a fixed order.
// ---------------------------------------------------------------------------
template <int J>
__device__ __forceinline__ double r_gdot1(const double2 (&x)[kR], const double2 (&l)[kR], const M2& d) {
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    if (k & (1 << J)) continue;
    const int k1 = k | (1 << J);
    const double2 y0 = cmac2(d.a, x[k], d.b, x[k1]), y1 = cmac2(d.c, x[k], d.d, x[k1]);
    acc += l[k].x * y0.x + l[k].y * y0.y + l[k1].x * y1.x + l[k1].y * y1.y;
  }
  return acc;
}

template <int C, int T>
__device__ __forceinline__ double r_gdot2(const double2 (&x)[kR], const double2 (&l)[kR], const M2& d) {
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    if (!((k >> C) & 1) || (k & (1 << T))) continue;
    const int k1 = k | (1 << T);
    const double2 y0 = cmac2(d.a, x[k], d.b, x[k1]), y1 = cmac2(d.c, x[k], d.d, x[k1]);
    acc += l[k].x * y0.x + l[k].y * y0.y + l[k1].x * y1.x + l[k1].y * y1.y;
  }
  return acc;
}

// Re sum conj(lambda) * (D psi) over this thread's pairs of the gate.
__device__ __forceinline__ double r_gdot(const double2 (&x)[kR], const double2 (&l)[kR], uint8_t type, int j0,
                                         int j1, const M2& d) {
  if (type <= GT_X1) {
    switch (j0) {
      case 0: return r_gdot1<0>(x, l, d);
      case 1: return r_gdot1<1>(x, l, d);
      case 2: return r_gdot1<2>(x, l, d);
      default: return r_gdot1<3>(x, l, d);
    }
  }
#define QSV_G2(C, T) \
  case (C * 4 + T): return r_gdot2<C, T>(x, l, d);
  switch (j0 * 4 + j1) {
    QSV_G2(0, 1) QSV_G2(0, 2) QSV_G2(0, 3)
    QSV_G2(1, 0) QSV_G2(1, 2) QSV_G2(1, 3)
    QSV_G2(2, 0) QSV_G2(2, 1) QSV_G2(2, 3)
    QSV_G2(3, 0) QSV_G2(3, 1) QSV_G2(3, 2)
    default: return 0.0;
  }
#undef QSV_G2
}

// A register mapping: thread element k sits at tile-local index
// lb | (bit 0 of k ? o[0]) | ... | (bit 3 of k ? o[3]).
struct RMap {
  uint32_t lb, o[4];
};

__device__ __forceinline__ uint32_t rmap_l(const RMap& m, int k) {
  return m.lb | ((k & 1) ? m.o[0] : 0u) | ((k & 2) ? m.o[1] : 0u) | ((k & 4) ? m.o[2] : 0u) |
         ((k & 8) ? m.o[3] : 0u);
}

// moves one state's registers from mapping A to mapping B through LDS
__device__ __forceinline__ void remap(double2 (&x)[kR], double2* __restrict__ buf, const RMap& ma, const RMap& mb) {
#pragma unroll
  for (int k = 0; k < kR; ++k) buf[swz(rmap_l(ma, k))] = x[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kR; ++k) x[k] = buf[swz(rmap_l(mb, k))];
  __syncthreads();
}

__device__ __forceinline__ RMap phase_map(const Phase& ph, uint32_t T, uint32_t tid) {
  RMap m;
  m.o[0] = 1u << ph.r[0];
  m.o[1] = 1u << ph.r[1];
  m.o[2] = 1u << ph.r[2];
  m.o[3] = 1u << ph.r[3];
  m.lb = pdep32(tid, (T - 1u) & ~(m.o[0] | m.o[1] | m.o[2] | m.o[3]));
  return m;
}

// the load layout l = tid + k * nthr (nthr = T / 16)
__device__ __forceinline__ RMap load_map(uint32_t nthr, uint32_t tid) {
  RMap m;
  m.lb = tid;
  m.o[0] = nthr;
  m.o[1] = nthr << 1;
  m.o[2] = nthr << 2;
  m.o[3] = nthr << 3;
  return m;
}

__global__ __launch_bounds__(kTileThreads) void k_backward_r(
    double2* __restrict__ psi, double2* __restrict__ lam, uint64_t stride, const DGate* __restrict__ gates,
    const Phase* __restrict__ phases, const double* __restrict__ mats, const double* __restrict__ dmats,
    uint64_t mat_stride, PassArgs a, double* __restrict__ gpart) {
  extern __shared__ double2 buf[];
  const uint32_t b = blockIdx.y, w = blockIdx.x, tid = threadIdx.x;
  const uint32_t T = 1u << a.t, nthr = T >> kRegBits, nwaves = (nthr + 63u) / 64u, wave = tid >> 6;
  uint64_t base = 0;
  {
    uint32_t k = 0;
    for (uint32_t q = 0; q < a.n; ++q)
      if (!((a.tile_mask >> q) & 1ull)) base |= (uint64_t)((w >> k++) & 1u) << q;
  }
  double2* sp = psi + (uint64_t)b * stride;
  double2* sl = lam + (uint64_t)b * stride;
  uint64_t gthr = base;
  for (uint32_t bb = 0; bb + kRegBits < a.t; ++bb) gthr |= (uint64_t)((tid >> bb) & 1u) << a.tq[bb];
  const uint64_t h0 = 1ull << a.tq[a.t - 4], h1 = 1ull << a.tq[a.t - 3], h2 = 1ull << a.tq[a.t - 2],
                 h3 = 1ull << a.tq[a.t - 1];
  RMap cur = load_map(nthr, tid);
  double2 x[kR], l[kR];
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    const uint64_t gi = gthr | ((k & 1) ? h0 : 0ull) | ((k & 2) ? h1 : 0ull) | ((k & 4) ? h2 : 0ull) |
                        ((k & 8) ? h3 : 0ull);
    x[k] = sp[gi];
    l[k] = sl[gi];
  }
  const double* mb = mats + (uint64_t)b * mat_stride;
  const double* db = dmats + (uint64_t)b * mat_stride * 3;
  double* gp = gpart + (((uint64_t)b * a.tiles + w) * nwaves + wave) * a.gate_count * 3;
  for (int32_t p = (int32_t)a.phase_count - 1; p >= 0; --p) {
    const Phase ph = phases[a.phase_begin + p];
    const RMap nxt = phase_map(ph, T, tid);
    remap(x, buf, cur, nxt);
    remap(l, buf, cur, nxt);
    cur = nxt;
    for (int32_t i = (int32_t)ph.gate_count - 1; i >= 0; --i) {
      const uint32_t gi = ph.gate_begin + (uint32_t)i;
      const DGate g = gates[gi];
      const double* m = mb + (uint64_t)g.mat * kMatStride;
      // U^dag: conjugate transpose of the 2x2 (the phase of a controlled phase is conjugated)
      double md[8] = {m[0], -m[1], m[4], -m[5], m[2], -m[3], m[6], -m[7]};
      r_apply(x, g.type, g.j0, g.j1, md);
      for (uint32_t j = 0; j < g.nang; ++j) {
        const M2 d = load_m2(db + (uint64_t)g.mat * 3 * kMatStride + j * kMatStride, 0);
        double v = r_gdot(x, l, g.type, g.j0, g.j1, d);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((tid & 63u) == 0) gp[(uint64_t)(gi - a.gate_begin) * 3 + j] = 2.0 * v;
      }
      r_apply(l, g.type, g.j0, g.j1, md);
    }
  }
  // back to the load mapping and out
  const RMap out = load_map(nthr, tid);
  remap(x, buf, cur, out);
  remap(l, buf, cur, out);
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    const uint64_t gi = gthr | ((k & 1) ? h0 : 0ull) | ((k & 2) ? h1 : 0ull) | ((k & 4) ? h2 : 0ull) |
                        ((k & 8) ? h3 : 0ull);
    sp[gi] = x[k];
    sl[gi] = l[k];
  }
}

hipError_t launch_backward_pass(double2* psi, double2* lam, uint64_t stride, uint32_t batch, const DGate* gates,
                                const Phase* phases, const double* mats, const double* dmats, uint64_t mat_stride,
                                const PassArgs& a, double* gpart, hipStream_t st) {
  dim3 grid(a.tiles, batch);
  if (a.phase_count) {
    const size_t lds = sizeof(double2) << a.t;
    hipLaunchKernelGGL(k_backward_r, grid, dim3(1u << (a.t - kRegBits)), lds, st, psi, lam, stride, gates, phases,
                       mats, dmats, mat_stride, a, gpart);
    return hipGetLastError();
  }
  size_t lds = (size_t)2 * sizeof(double2) << a.t;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_backward_pass),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_backward_pass, grid, dim3(kTileThreads), lds, st, psi, lam, stride, gates, mats, dmats,
                     mat_stride, a, gpart);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint sweep of an all-dense pass on the matrix cores.
//
// A phase with gates G_1..G_m has the composed matrix W = G_m..G_1. With psi_a
// and lambda_a the states after the phase, the sweep forms psi_b = W^dag psi_a
// and lambda_b = W^dag lambda_a, and the derivative along angle j of G_i is
//   2 Re <lambda_a| G_m..G_{i+1} G_i' G_{i-1}..G_1 |psi_b>
//     = 2 Re <lambda_b| S |psi_b> = 2 Re tr(S C),
// with S = W^dag G_m..G_i'..G_1 = (G_{i-1}..G_1)^dag G_i^dag G_i' (G_{i-1}..G_1)
// (composed once per call) and C[r][c] = sum over amplitude groups g of
// psi_b[r][g] conj(lambda_b[c][g]), a 16 x 16 product over the groups.
// ---------------------------------------------------------------------------

// derivative of a controlled gate: zero where the control C is clear, the
// 2x2 derivative on target T where it is set
template <int C, int T>
__device__ __forceinline__ void r_dctrl(double2 (&a)[kR], const M2& u) {
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    if (!((k >> C) & 1)) {
      a[k] = make_double2(0.0, 0.0);
      continue;
    }
    if (k & (1 << T)) continue;
    const int k1 = k | (1 << T);
    const double2 x0 = a[k], x1 = a[k1];
    a[k] = cmac2(u.a, x0, u.b, x1);
    a[k1] = cmac2(u.c, x0, u.d, x1);
  }
}

// the derivative matrix dm of a gate (one angle) on a thread's 16 amplitudes
__device__ __forceinline__ void r_apply_deriv(double2 (&a)[kR], uint8_t type, int j0, int j1, const double* dm) {
  const M2 u = load_m2(dm, 0);
  if (type <= GT_X1) {
    switch (j0) {
      case 0: r_dense<0>(a, u); break;
      case 1: r_dense<1>(a, u); break;
      case 2: r_dense<2>(a, u); break;
      default: r_dense<3>(a, u); break;
    }
    return;
  }
#define QSV_D2(C, T) \
  case (C * 4 + T): r_dctrl<C, T>(a, u); break;
  switch (j0 * 4 + j1) {
    QSV_D2(0, 1) QSV_D2(0, 2) QSV_D2(0, 3)
    QSV_D2(1, 0) QSV_D2(1, 2) QSV_D2(1, 3)
    QSV_D2(2, 0) QSV_D2(2, 1) QSV_D2(2, 3)
    QSV_D2(3, 0) QSV_D2(3, 1) QSV_D2(3, 2)
    default: break;
  }
#undef QSV_D2
}

// a gate's inverse: the conjugate transpose of its 2x2 (a controlled phase's phase is conjugated)
__device__ __forceinline__ void r_apply_dag(double2 (&a)[kR], const DGate& g, const double* m) {
  const double md[8] = {m[0], -m[1], m[4], -m[5], m[2], -m[3], m[6], -m[7]};
  r_apply(a, g.type, g.j0, g.j1, md);
}

// Column c of S for every angle entry and parameter vector (one thread each),
// stored in matrix-core operand order like a composed phase matrix.
__global__ __launch_bounds__(128) void k_compose_grad(const DGate* __restrict__ gates, const AngEnt* __restrict__ ent, uint32_t n_ent,
                               uint32_t batch, uint64_t mat_stride, const double* __restrict__ mats,
                               const double* __restrict__ dmats, double* __restrict__ smats) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)n_ent * kR * batch) return;
  const uint32_t c = (uint32_t)(idx % kR);
  const uint64_t rest = idx / kR;
  const uint32_t e = (uint32_t)(rest % n_ent), b = (uint32_t)(rest / n_ent);
  const AngEnt en = ent[e];
  const double* mb = mats + (uint64_t)b * mat_stride;
  const double* db = dmats + (uint64_t)b * mat_stride * 3;
  const uint32_t g0 = en.gate - en.off;
  double2 v[kR];
#pragma unroll
  for (int k = 0; k < kR; ++k) v[k] = make_double2(k == (int)c ? 1.0 : 0.0, 0.0);
  for (uint32_t i = 0; i < en.off; ++i) {
    const DGate g = gates[g0 + i];
    r_apply(v, g.type, g.j0, g.j1, mb + (uint64_t)g.mat * kMatStride);
  }
  const DGate gi = gates[en.gate];
  r_apply_deriv(v, gi.type, gi.j0, gi.j1, db + (uint64_t)gi.mat * 3 * kMatStride + (uint64_t)en.j * kMatStride);
  r_apply_dag(v, gi, mb + (uint64_t)gi.mat * kMatStride);
  for (uint32_t i = en.off; i-- > 0;) {
    const DGate g = gates[g0 + i];
    r_apply_dag(v, g, mb + (uint64_t)g.mat * kMatStride);
  }
  double2* S = reinterpret_cast<double2*>(smats) + ((uint64_t)b * n_ent + e) * 256u;
#pragma unroll
  for (uint32_t r = 0; r < (uint32_t)kR; ++r) S[dense_pos(r, c)] = v[r];
}

hipError_t launch_compose_grad(const DGate* gates, const AngEnt* ent, uint32_t n_ent, uint32_t batch,
                               uint64_t mat_stride, const double* mats, const double* dmats, double* smats,
                               hipStream_t st) {
  const uint64_t total = (uint64_t)n_ent * kR * batch;
  if (!total) return hipSuccess;
  hipLaunchKernelGGL(k_compose_grad, dim3((uint32_t)((total + 127) / 128)), dim3(128), 0, st, gates, ent, n_ent,
                     batch, mat_stride, mats, dmats, smats);
  return hipGetLastError();
}

// lane l's matrix-core B operand of conj(W) over the 4 K chunks: conj(W[4 kb + l / 16][l % 16])
__device__ __forceinline__ void load_wfrag(double2 (&wf)[4], const double2* __restrict__ Wc, uint32_t lane) {
  const uint32_t q = lane >> 4, j = lane & 15u;
#pragma unroll
  for (uint32_t kb = 0; kb < 4; ++kb) wf[kb] = Wc[dense_pos(4u * kb + q, j)];
}

// One phase of the sweep for the 32 amplitude groups (2 blocks of 16) of this
// thread's wave, on the matrix cores. psi_b^T = psi_a^T conj(W): as the A
// operand, lane l supplies psi_a[component 4 kb + l / 16][group l % 16] (kb =
// 0..3), the amplitudes the forward phase reads; as the B operand it supplies
// conj(W[4 kb + l / 16][l % 16]) (wf). Result element v of lane l is then
// psi_b[component l % 16][group 4 v + l / 16], which is both the A operand
// (psi_b) and, conjugated for lambda, the B operand of C over the K chunk of
// groups 4 v..4 v + 3; results are written back from that layout. Complex
// products use three real ones (as in the forward phase). The reads of block
// 1 are issued before the writes of block 0; waves own disjoint groups.
__device__ __forceinline__ void adjoint_phase_mfma(double2* __restrict__ tp, double2* __restrict__ tl, uint32_t T,
                                                   uint32_t lane, uint32_t wave, const Phase& ph,
                                                   const double2 (&wf)[4], qsv_d4& c1, qsv_d4& c2, qsv_d4& c3) {
  constexpr uint32_t kBlocks = 2;
  const uint32_t q = lane >> 4, j = lane & 15u;
  const uint32_t o0 = 1u << ph.r[0], o1 = 1u << ph.r[1], o2 = 1u << ph.r[2], o3 = 1u << ph.r[3];
  const UBits u = ubits((T - 1u) & ~(o0 | o1 | o2 | o3));
  // group of block cb, K chunk v, lane: 32 wave + 16 cb + 4 v + q (writes) or 32 wave + 16 cb + j (reads)
  const uint32_t pw = (((wave >> 0) & 1u) ? u.b[5] : 0u) | (((wave >> 1) & 1u) ? u.b[6] : 0u) |
                      (((wave >> 2) & 1u) ? u.b[7] : 0u);
  const uint32_t cqq = ((q & 1u) ? o0 : 0u) | ((q & 2u) ? o1 : 0u);
  const uint32_t cj = ((j & 1u) ? o0 : 0u) | ((j & 2u) ? o1 : 0u) | ((j & 4u) ? o2 : 0u) | ((j & 8u) ? o3 : 0u);
  const uint32_t rl = swz(udep<4>(u, j) | cqq);  // per-lane part of the read slots
  const uint32_t wl = swz(udep<2>(u, q) | cj);   // per-lane part of the write slots
  double wa[4], wb[4], ws[4];  // conj(W) = wa + i wb, and wa + wb
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    wa[kb] = wf[kb].x;
    wb[kb] = -wf[kb].y;
    ws[kb] = wf[kb].x - wf[kb].y;
  }
  double2 x[2][4], y[2][4];
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    const uint32_t sl = rl ^ swz(pw | ((k & 1u) ? o2 : 0u) | ((k & 2u) ? o3 : 0u));
    x[0][k] = tp[sl];
    y[0][k] = tl[sl];
  }
#pragma unroll
  for (uint32_t cb = 0; cb < kBlocks; ++cb) {
    const uint32_t s = cb & 1u;
    qsv_d4 p1 = {0.0, 0.0, 0.0, 0.0}, p2 = p1, p3 = p1, l1 = p1, l2 = p1, l3 = p1;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      p1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[s][kb].x, wa[kb], p1, 0, 0, 0);
      p2 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[s][kb].y, wb[kb], p2, 0, 0, 0);
      p3 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[s][kb].x + x[s][kb].y, ws[kb], p3, 0, 0, 0);
      l1 = __builtin_amdgcn_mfma_f64_16x16x4f64(y[s][kb].x, wa[kb], l1, 0, 0, 0);
      l2 = __builtin_amdgcn_mfma_f64_16x16x4f64(y[s][kb].y, wb[kb], l2, 0, 0, 0);
      l3 = __builtin_amdgcn_mfma_f64_16x16x4f64(y[s][kb].x + y[s][kb].y, ws[kb], l3, 0, 0, 0);
    }
    if (cb + 1 < kBlocks) {
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t sl = rl ^ swz(pw | u.b[4] | ((k & 1u) ? o2 : 0u) | ((k & 2u) ? o3 : 0u));
        x[s ^ 1u][k] = tp[sl];
        y[s ^ 1u][k] = tl[sl];
      }
    }
#pragma unroll
    for (uint32_t v = 0; v < 4; ++v) {
      const double pr = p1[v] - p2[v], pi = p3[v] - p1[v] - p2[v];
      const double lr = l1[v] - l2[v], li = l3[v] - l1[v] - l2[v];
      // C += psi_b conj(lambda_b) over groups 4 v..4 v + 3 of the block
      c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(pr, lr, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(pi, -li, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(pr + pi, lr - li, c3, 0, 0, 0);
      const uint32_t sl =
          wl ^ swz(pw | (cb ? u.b[4] : 0u) | ((v & 1u) ? u.b[2] : 0u) | ((v & 2u) ? u.b[3] : 0u));
      tp[sl] = make_double2(pr, pi);
      tl[sl] = make_double2(lr, li);
    }
  }
}

// Sums a[0..7] over the 64 lanes of the wave; lane l returns the sum of
// a[l >> 3]. Three exchange steps each hand half of the remaining values to
// the partner lane (xor 32, 16, 8), then a butterfly over the last 3 bits:
// 10 shuffles instead of 48.
__device__ __forceinline__ double wave_sum8(const double (&a)[8], uint32_t lane) {
  const bool h5 = (lane >> 5) & 1u, h4 = (lane >> 4) & 1u, h3 = (lane >> 3) & 1u;
  double b[4], c[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double keep = h5 ? a[4 + i] : a[i], send = h5 ? a[i] : a[4 + i];
    b[i] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double keep = h4 ? b[2 + i] : b[i], send = h4 ? b[i] : b[2 + i];
    c[i] = keep + __shfl_xor(send, 16, 64);
  }
  double d = (h3 ? c[1] : c[0]) + __shfl_xor(h3 ? c[0] : c[1], 8, 64);
  d += __shfl_xor(d, 4, 64);
  d += __shfl_xor(d, 2, 64);
  d += __shfl_xor(d, 1, 64);
  return d;
}

// Persistent workgroups of 2^(t-3) threads (8 amplitudes of psi and of lambda
// per thread) over the items (vector, tile) of an all-dense pass with
// 10 <= t <= 12. Phases run in reverse order. After each, the waves' partial
// C are summed in LDS in a fixed order; angle e of the phase is then taken by
// wave e mod (waves), which reduces 2 Re tr(S C) over its lanes and writes
// gpart[vector][tile][gate][angle]. Those traces overlap the next phase's
// products (no barrier until that phase ends).
__global__ __launch_bounds__(kBwWaves * 64) void k_backward_mfma(
    double2* __restrict__ psi, double2* __restrict__ lam, uint64_t stride, const Phase* __restrict__ phases,
    const uint32_t* __restrict__ ang_off, const AngEnt* __restrict__ ent, const double* __restrict__ mats,
    uint64_t mat_stride, const double* __restrict__ smats, uint32_t n_ent, PassArgs a, uint32_t batch,
    double* __restrict__ gpart) {
  extern __shared__ double2 lds[];
  const uint32_t tid = threadIdx.x, T = 1u << a.t, nthr = T >> 3, nwaves = nthr >> 6;
  const uint32_t lane = tid & 63u, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double2* const tp = lds;
  double2* const tl = lds + T;
  double2* const cbuf = lds + 2 * T;  // [waves][256]: partial C per wave, then the sum in slot 0
  const uint64_t total = (uint64_t)a.tiles * batch, G = gridDim.x;
  const uint64_t free_mask = ~a.tile_mask & ((a.n >= 64) ? ~0ull : ((1ull << a.n) - 1ull));
  uint64_t tb = 0;  // this thread's bits over tile qubits tq[0..t-4]
  for (uint32_t bb = 0; bb + 3 < a.t; ++bb) tb |= (uint64_t)((tid >> bb) & 1u) << a.tq[bb];
  const uint64_t h0 = 1ull << a.tq[a.t - 3], h1 = 1ull << a.tq[a.t - 2], h2 = 1ull << a.tq[a.t - 1];
  for (uint64_t it = blockIdx.x; it < total; it += G) {
    const uint32_t b = (uint32_t)(it / a.tiles), w = (uint32_t)(it % a.tiles);
    const uint64_t gthr = tile_base(w, free_mask) | tb;
    double2* sp = psi + (uint64_t)b * stride;
    double2* sl = lam + (uint64_t)b * stride;
    double2 rp[8], rl[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t gi = gthr | ((k & 1) ? h0 : 0ull) | ((k & 2) ? h1 : 0ull) | ((k & 4) ? h2 : 0ull);
      rp[k] = sp[gi];
      rl[k] = sl[gi];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      tp[swz(tid + (uint32_t)k * nthr)] = rp[k];
      tl[swz(tid + (uint32_t)k * nthr)] = rl[k];
    }
    const double* mb = mats + (uint64_t)b * mat_stride;
    const double2* sb = reinterpret_cast<const double2*>(smats) + (uint64_t)b * n_ent * 256u;
    double* gp = gpart + ((uint64_t)b * a.tiles + w) * a.gate_count * 3;
    double2 wf[4];
    load_wfrag(wf, reinterpret_cast<const double2*>(
                       mb + (uint64_t)load_phase(phases + a.phase_begin + a.phase_count - 1).dense * kMatStride),
               lane);
    __syncthreads();
    for (uint32_t p = a.phase_count; p-- > 0;) {
      const uint32_t pg = a.phase_begin + p;
      const Phase ph = load_phase(phases + pg);
      double2 wn[4];  // the next phase's operand, requested before this phase's products
      if (p > 0)
        load_wfrag(wn, reinterpret_cast<const double2*>(mb + (uint64_t)load_phase(phases + pg - 1).dense * kMatStride),
                   lane);
      const uint32_t e0 = cst(ang_off)[pg], ne = cst(ang_off)[pg + 1] - e0;
      // this wave's angles: e = wave + k * waves; lane k holds the gradient slot of the k-th
      const uint32_t my_n = ne > wave ? (ne - wave + nwaves - 1) / nwaves : 0u;
      uint32_t gslot = 0;
      if (lane < my_n) {
        const AngEnt en = ent[e0 + wave + lane * nwaves];
        gslot = (en.gate - a.gate_begin) * 3u + en.j;
      }
      qsv_d4 c1 = {0.0, 0.0, 0.0, 0.0}, c2 = c1, c3 = c1;
      adjoint_phase_mfma(tp, tl, T, lane, wave, ph, wf, c1, c2, c3);
      // this wave's first S, requested before the partials are summed (its
      // load then overlaps the barriers below)
      double2 s0[4];
      if (my_n) {
        const double2* S = sb + (uint64_t)(e0 + wave) * 256u;
#pragma unroll
        for (int v = 0; v < 4; ++v) s0[v] = S[v * 64 + (int)lane];
      }
#pragma unroll
      for (int v = 0; v < 4; ++v)
        cbuf[wave * 256u + (uint32_t)v * 64u + lane] = make_double2(c1[v] - c2[v], c3[v] - c1[v] - c2[v]);
      __syncthreads();
      // C of the tile: the waves' partials summed in wave order
      for (uint32_t e = tid; e < 256u; e += nthr) {
        double2 acc = cbuf[e];
        for (uint32_t ww = 1; ww < nwaves; ++ww) {
          const double2 v = cbuf[ww * 256u + e];
          acc.x += v.x;
          acc.y += v.y;
        }
        cbuf[e] = acc;
      }
      __syncthreads();
      double cr[4] = {0.0, 0.0, 0.0, 0.0}, ci[4] = {0.0, 0.0, 0.0, 0.0};
      if (my_n) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double2 c = cbuf[(uint32_t)v * 64u + lane];
          cr[v] = c.x;
          ci[v] = c.y;
        }
      }
      __syncthreads();  // every wave holds the sum before the next phase writes its partials
      for (uint32_t k0 = 0; k0 < my_n; k0 += 8) {
        double part[8];
#pragma unroll
        for (uint32_t uu = 0; uu < 8; ++uu) {
          part[uu] = 0.0;
          if (k0 + uu < my_n) {
            const double2* S = sb + (uint64_t)(e0 + wave + (k0 + uu) * nwaves) * 256u;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const double2 sv = (k0 + uu == 0) ? s0[v] : S[v * 64 + (int)lane];
              part[uu] += sv.x * cr[v] - sv.y * ci[v];
            }
          }
        }
        const double tot = wave_sum8(part, lane);
        const uint32_t k = k0 + (lane >> 3);
        const uint32_t slot = __shfl(gslot, (int)(k & 63u), 64);
        if ((lane & 7u) == 0 && k < my_n) gp[slot] = 2.0 * tot;
      }
      if (p > 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) wf[k] = wn[k];
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      rp[k] = tp[swz(tid + (uint32_t)k * nthr)];
      rl[k] = tl[swz(tid + (uint32_t)k * nthr)];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t gi = gthr | ((k & 1) ? h0 : 0ull) | ((k & 2) ? h1 : 0ull) | ((k & 4) ? h2 : 0ull);
      sp[gi] = rp[k];
      sl[gi] = rl[k];
    }
    __syncthreads();
  }
}

// Dynamic LDS of k_backward_mfma for tiles of 2^t amplitudes: the psi and
// lambda tiles and one 16x16 complex C per wave (2^12 amplitudes: 160 KiB).
size_t backward_mfma_lds(uint32_t t) {
  return (size_t)2 * sizeof(double2) * (1u << t) + (size_t)((1u << t) / 512u) * 256u * sizeof(double2);
}

hipError_t launch_backward_mfma(double2* psi, double2* lam, uint64_t stride, uint32_t batch, const Phase* phases,
                                const uint32_t* ang_off, const AngEnt* ent, const double* mats, uint64_t mat_stride,
                                const double* smats, uint32_t n_ent, const PassArgs& a, double* gpart,
                                hipStream_t st) {
  const uint64_t total = (uint64_t)a.tiles * batch;
  if (!total) return hipSuccess;
  const size_t lds = backward_mfma_lds(a.t);
  uint32_t g = 0;
  hipError_t e = resident_grid((const void*)k_backward_mfma, 1u << (a.t - 3), lds,
                               backward_mfma_lds(kTileMaxBits), &g);
  if (e != hipSuccess) return e;
  if ((uint64_t)g > total) g = (uint32_t)total;
  hipLaunchKernelGGL(k_backward_mfma, dim3(g), dim3(1u << (a.t - 3)), lds, st, psi, lam, stride, phases, ang_off,
                     ent, mats, mat_stride, smats, n_ent, a, batch, gpart);
  return hipGetLastError();
}

// Number of partial-gradient slots per (vector, gate, angle) written by the backward sweep of a pass.
uint32_t backward_parts(const PassArgs& a) {
  if (!a.phase_count) return a.tiles;
  const uint32_t nthr = 1u << (a.t - kRegBits);
  return a.tiles * ((nthr + 63u) / 64u);
}

// dEda[b][slot][j] = sum over tiles (fixed order) of the pass's partials.
__global__ void k_grad_reduce(const double* __restrict__ gpart, uint32_t parts, uint32_t gate_count,
                              const DGate* __restrict__ gates, uint32_t batch, uint32_t n_slots,
                              double* __restrict__ dEda) {
  uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)batch * gate_count * 3) return;
  uint32_t j = idx % 3, gi = (idx / 3) % gate_count, b = (uint32_t)(idx / 3 / gate_count);
  if (j >= gates[gi].nang) return;
  // the partials of tile w at src[w * step], added in tile order; each group
  // of 16 is loaded before it is added, so the loads are in flight together
  const double* src = gpart + ((uint64_t)b * parts * gate_count + gi) * 3 + j;
  const uint64_t step = (uint64_t)gate_count * 3;
  double acc = 0.0;
  uint32_t w = 0;
  for (; w + 16 <= parts; w += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = src[(uint64_t)(w + u) * step];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc += v[u];
  }
  for (; w < parts; ++w) acc += src[(uint64_t)w * step];
  dEda[((uint64_t)b * n_slots + gates[gi].mat) * 3 + j] = acc;
}

hipError_t launch_grad_reduce(const double* gpart, uint32_t parts, uint32_t gate_count, uint32_t slot_begin_of_pass,
                              const DGate* gates, uint32_t batch, uint32_t n_slots, double* dEda, hipStream_t st) {
  (void)slot_begin_of_pass;
  uint64_t total = (uint64_t)batch * gate_count * 3;
  if (!total) return hipSuccess;
  hipLaunchKernelGGL(k_grad_reduce, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, st, gpart, parts,
                     gate_count, gates, batch, n_slots, dEda);
  return hipGetLastError();
}

// grad[b][p] = sum over (slot, j) feeding parameter p of scale * dEda[b][slot][j], in CSR order.
__global__ void k_grad_chain(const double* __restrict__ dEda, uint32_t n_slots, const uint32_t* __restrict__ off,
                             const uint32_t* __restrict__ sj, const double* __restrict__ scale, uint32_t n_params,
                             uint32_t batch, double* __restrict__ grad) {
  uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)batch * n_params) return;
  uint32_t p = idx % n_params, b = (uint32_t)(idx / n_params);
  double acc = 0.0;
  for (uint32_t k = off[p]; k < off[p + 1]; ++k)
    acc += scale[k] * dEda[(uint64_t)b * n_slots * 3 + sj[k]];
  grad[idx] = acc;
}

hipError_t launch_grad_chain(const double* dEda, uint32_t n_slots, const uint32_t* csr_off, const uint32_t* csr_slot,
                             const double* csr_scale, uint32_t n_params, uint32_t batch, double* grad, hipStream_t st) {
  uint64_t total = (uint64_t)batch * n_params;
  if (!total) return hipSuccess;
  hipLaunchKernelGGL(k_grad_chain, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, st, dEda, n_slots, csr_off,
                     csr_slot, csr_scale, n_params, batch, grad);
  return hipGetLastError();
}

}  // namespace qsv
