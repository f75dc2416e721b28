// gfx950 kernels of expectation values and adjoint gradients (complex128).
//
// A batch of parameter vectors b holds its states at psi + b * stride.
//   k_pauli_terms / k_energy_reduce / k_apply_hamiltonian   <psi|H|psi>, H psi
//   k_backward_pass   adjoint sweep of one pass on (psi, lambda) with gradient partials
//   k_backward_r      the same on register phases
//   k_grad_reduce / k_grad_chain   fixed-order gradient reductions
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "device_common.h"
#include "kernels.h"

namespace qsv {

// ---------------------------------------------------------------------------
// Expectation values: <psi|P|psi> for P = i^ny X^x Z^z (Y = i X Z)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 ipow(uint32_t k) {
  switch (k & 3u) {
    case 0: return make_double2(1, 0);
    case 1: return make_double2(0, 1);
    case 2: return make_double2(-1, 0);
    default: return make_double2(0, -1);
  }
}

// Block partials of Re sum_i conj(psi[i ^ x]) * phase(i) * psi[i] per term.
__global__ __launch_bounds__(256) void k_pauli_terms(const double2* __restrict__ psi, uint64_t stride, uint32_t n,
                                                    const uint64_t* __restrict__ xmask,
                                                    const uint64_t* __restrict__ zmask,
                                                    const uint32_t* __restrict__ ny, uint32_t n_terms,
                                                    double* __restrict__ out, uint32_t blocks) {
  __shared__ double red[256];
  const uint32_t blk = blockIdx.x % blocks, tb = blockIdx.x / blocks, tid = threadIdx.x;
  const uint32_t term = tb % n_terms, b = tb / n_terms;
  const double2* st = psi + (uint64_t)b * stride;
  const uint64_t dim = 1ull << n, per = (dim + blocks - 1) / blocks;
  const uint64_t j0 = per * blk, j1 = (j0 + per < dim) ? j0 + per : dim;
  const uint64_t x = xmask[term], z = zmask[term];
  const double2 ph = ipow(ny[term]);
  double acc = 0.0;
  for (uint64_t i = j0 + tid; i < j1; i += 256) {
    double2 a = st[i], bb = st[i ^ x];
    double sgn = (__popcll(i & z) & 1) ? -1.0 : 1.0;
    double2 pa = cmul(ph, cscale(a, sgn));
    acc += bb.x * pa.x + bb.y * pa.y;  // Re(conj(bb) * pa)
  }
  red[tid] = acc;
  __syncthreads();
  for (uint32_t s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) out[((uint64_t)b * n_terms + term) * blocks + blk] = red[0];
}

hipError_t launch_pauli_terms(const double2* psi, uint64_t stride, uint32_t n, uint32_t batch,
                              const uint64_t* xmask, const uint64_t* zmask, const uint32_t* ny,
                              const double* coeff, uint32_t n_terms, double* term_partials, uint32_t blocks,
                              hipStream_t st) {
  (void)coeff;
  hipLaunchKernelGGL(k_pauli_terms, dim3(blocks * batch * n_terms), dim3(256), 0, st, psi, stride, n, xmask,
                     zmask, ny, n_terms, term_partials, blocks);
  return hipGetLastError();
}

__global__ void k_energy_reduce(const double* __restrict__ tp, uint32_t n_terms, uint32_t blocks,
                                const double* __restrict__ coeff, uint32_t batch, double* __restrict__ energy) {
  uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  double e = 0.0;
  for (uint32_t t = 0; t < n_terms; ++t) {
    double v = 0.0;
    for (uint32_t k = 0; k < blocks; ++k) v += tp[((uint64_t)b * n_terms + t) * blocks + k];
    e += coeff[t] * v;
  }
  energy[b] = e;
}

hipError_t launch_energy_reduce(const double* term_partials, uint32_t n_terms, uint32_t blocks,
                                const double* coeff, uint32_t batch, double* energy, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_reduce, dim3((batch + 63) / 64), dim3(64), 0, st, term_partials, n_terms, blocks,
                     coeff, batch, energy);
  return hipGetLastError();
}

// lam = sum_j c_j P_j psi, terms accumulated in a fixed order per element:
// (P psi)[i] = phase(i ^ x) * psi[i ^ x].
__global__ void k_apply_hamiltonian(const double2* __restrict__ psi, double2* __restrict__ lam, uint64_t stride,
                                    uint32_t n, const uint64_t* __restrict__ xmask,
                                    const uint64_t* __restrict__ zmask, const uint32_t* __restrict__ ny,
                                    const double* __restrict__ coeff, uint32_t n_terms, uint32_t batch) {
  const uint64_t dim = 1ull << n, total = dim * batch;
  for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t b = idx / dim, i = idx % dim;
    const double2* st = psi + b * stride;
    double2 acc = make_double2(0.0, 0.0);
    for (uint32_t t = 0; t < n_terms; ++t) {
      uint64_t src = i ^ xmask[t];
      double2 v = st[src];
      double sgn = (__popcll(src & zmask[t]) & 1) ? -1.0 : 1.0;
      acc = cadd(acc, cscale(cmul(ipow(ny[t]), v), coeff[t] * sgn));
    }
    lam[b * stride + i] = acc;
  }
}

hipError_t launch_apply_hamiltonian(const double2* psi, double2* lam, uint64_t stride, uint32_t n, uint32_t batch,
                                    const uint64_t* xmask, const uint64_t* zmask, const uint32_t* ny,
                                    const double* coeff, uint32_t n_terms, hipStream_t st) {
  uint64_t total = (1ull << n) * batch;
  uint64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_apply_hamiltonian, dim3((uint32_t)blocks), dim3(256), 0, st, psi, lam, stride, n, xmask,
                     zmask, ny, coeff, n_terms, batch);
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
  double acc = 0.0;
  for (uint32_t w = 0; w < parts; ++w) acc += gpart[(((uint64_t)b * parts + w) * gate_count + gi) * 3 + j];
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
