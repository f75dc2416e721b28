// gfx950 kernels of the dynamic-circuit state-vector path (complex128).
//
// State layout: shot s holds its 2^n amplitudes contiguously at
// state + s * stride (double2 = re, im; index i = sum_q b_q 2^q).
//
// Kernels:
//   k_bind_matrices   2x2 gate matrices (and their angle derivatives) from theta
//   k_init_state      |0...0> for every shot
//   k_tile_pass       one fused gate pass: each workgroup stages a 2^t tile in
//                     LDS, applies the pending collapse, the pass's guarded
//                     gates (in the shot's qubit-flip frame) and stores it back
//   k_site_reduce     per-workgroup probability histogram over <= 4 qubits
//   k_site_finalize   per shot: fixed-order sum of the histograms, Philox draws,
//                     outcomes, classical bits, flags, record, new pending collapse
//   k_materialize     the logical state of one shot (collapse + frame applied)
// The expectation-value and adjoint-gradient kernels are in adjoint.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "device_common.h"
#include "kernels.h"
#include "qsv.h"

namespace qsv {

// Philox4x64-10 (Salmon et al., SC'11): multipliers and Weyl increments of
// Philox4x64. One block for key (k0, k1) and counter (c0, c1, c2, c3), in place.
__device__ __forceinline__ void philox_block(uint64_t& c0, uint64_t& c1, uint64_t& c2, uint64_t& c3, uint64_t k0,
                                             uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
}

// The shot's word of measure/reset event `event`: counter (event / 4 + 1, 0, 0, 0), word event % 4.
__device__ __forceinline__ uint64_t philox_word(uint64_t seed, uint64_t shot, uint64_t event) {
  uint64_t c0 = event / 4 + 1, c1 = 0, c2 = 0, c3 = 0;
  philox_block(c0, c1, c2, c3, seed, shot);
  switch (event & 3) {
    case 0: return c0;
    case 1: return c1;
    case 2: return c2;
    default: return c3;
  }
}

// ---------------------------------------------------------------------------
// Matrix binding (compile once, run many: angles are affine in theta)
// ---------------------------------------------------------------------------
__device__ void set2(double* m, double2 a, double2 b, double2 c, double2 d) {
  m[0] = a.x; m[1] = a.y; m[2] = b.x; m[3] = b.y; m[4] = c.x; m[5] = c.y; m[6] = d.x; m[7] = d.y;
}
__device__ __forceinline__ double2 cexpi(double t) {
  double s, c;
  sincos(t, &s, &c);
  return make_double2(c, s);
}

// theta extended by the derived parameters: out[b] = theta[b] (P values)
// followed by D values, derived k = sum of coef[e] * theta[b][in[e]] over
// e in [off[k], off[k + 1]) in that order.
__global__ void k_derive_params(const double* __restrict__ theta, uint32_t P, uint32_t D,
                                const uint32_t* __restrict__ off, const uint32_t* __restrict__ in,
                                const double* __restrict__ coef, uint32_t batch, double* __restrict__ out) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t W = P + D;
  if (idx >= (uint64_t)batch * W) return;
  const uint32_t b = (uint32_t)(idx / W), j = (uint32_t)(idx % W);
  const double* t = theta + (uint64_t)b * P;
  double v = 0.0;
  if (j < P) {
    v = t[j];
  } else {
    for (uint32_t e = off[j - P]; e < off[j - P + 1]; ++e) v += coef[e] * t[in[e]];
  }
  out[idx] = v;
}

hipError_t launch_derive_params(const double* theta, uint32_t P, uint32_t D, const uint32_t* off, const uint32_t* in,
                                const double* coef, uint32_t batch, double* out, hipStream_t st) {
  const uint64_t total = (uint64_t)batch * (P + D);
  if (!total) return hipSuccess;
  hipLaunchKernelGGL(k_derive_params, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, st, theta, P, D, off, in,
                     coef, batch, out);
  return hipGetLastError();
}

// One matrix slot from its source and a theta row: the 2x2 matrix at m and,
// when dm is set, its derivatives by each angle.
__device__ __forceinline__ void bind_slot(const GateSrc& g, const double* __restrict__ th, double* m, double* dm) {
  double a[3];
  for (int k = 0; k < 3; ++k) {
    a[k] = g.offset[k];
    if (g.param[k] != QSV_NONE) a[k] += g.scale[k] * th[g.param[k]];
  }
  const double2 Z0 = make_double2(0, 0), O1 = make_double2(1, 0), I1 = make_double2(0, 1);
  const double r2 = 0.70710678118654752440;
  if (dm)
    for (int k = 0; k < 3 * kMatStride; ++k) dm[k] = 0.0;
  switch (g.kind) {
    case QSV_G_X: case QSV_G_CX: set2(m, Z0, O1, O1, Z0); break;
    case QSV_G_Y: case QSV_G_CY: set2(m, Z0, make_double2(0, -1), I1, Z0); break;
    case QSV_G_Z: case QSV_G_CZ: set2(m, O1, Z0, Z0, make_double2(-1, 0)); break;
    case QSV_G_H: case QSV_G_CH:
      set2(m, make_double2(r2, 0), make_double2(r2, 0), make_double2(r2, 0), make_double2(-r2, 0));
      break;
    case QSV_G_S: set2(m, O1, Z0, Z0, I1); break;
    case QSV_G_SDG: set2(m, O1, Z0, Z0, make_double2(0, -1)); break;
    case QSV_G_T: set2(m, O1, Z0, Z0, make_double2(r2, r2)); break;
    case QSV_G_TDG: set2(m, O1, Z0, Z0, make_double2(r2, -r2)); break;
    case QSV_G_SX:
      set2(m, make_double2(0.5, 0.5), make_double2(0.5, -0.5), make_double2(0.5, -0.5), make_double2(0.5, 0.5));
      break;
    case QSV_G_SXDG:
      set2(m, make_double2(0.5, -0.5), make_double2(0.5, 0.5), make_double2(0.5, 0.5), make_double2(0.5, -0.5));
      break;
    case QSV_G_RX: case QSV_G_CRX: {
      double s, c;
      sincos(0.5 * a[0], &s, &c);
      set2(m, make_double2(c, 0), make_double2(0, -s), make_double2(0, -s), make_double2(c, 0));
      if (dm) set2(dm, make_double2(-0.5 * s, 0), make_double2(0, -0.5 * c), make_double2(0, -0.5 * c),
                   make_double2(-0.5 * s, 0));
      break;
    }
    case QSV_G_RY: case QSV_G_CRY: {
      double s, c;
      sincos(0.5 * a[0], &s, &c);
      set2(m, make_double2(c, 0), make_double2(-s, 0), make_double2(s, 0), make_double2(c, 0));
      if (dm) set2(dm, make_double2(-0.5 * s, 0), make_double2(-0.5 * c, 0), make_double2(0.5 * c, 0),
                   make_double2(-0.5 * s, 0));
      break;
    }
    case QSV_G_RZ: case QSV_G_CRZ: {
      double2 e0 = cexpi(-0.5 * a[0]), e1 = cexpi(0.5 * a[0]);
      set2(m, e0, Z0, Z0, e1);
      if (dm) set2(dm, make_double2(0.5 * e0.y, -0.5 * e0.x), Z0, Z0, make_double2(-0.5 * e1.y, 0.5 * e1.x));
      break;
    }
    case QSV_G_P: case QSV_G_CP: {
      double2 e = cexpi(a[0]);
      set2(m, O1, Z0, Z0, e);
      if (dm) set2(dm, Z0, Z0, Z0, make_double2(-e.y, e.x));
      break;
    }
    case QSV_G_U: {
      double s, c;
      sincos(0.5 * a[0], &s, &c);
      double2 ep = cexpi(a[1]), el = cexpi(a[2]), epl = cexpi(a[1] + a[2]);
      set2(m, make_double2(c, 0), cscale(el, -s), cscale(ep, s), cscale(epl, c));
      if (dm) {
        // d/dtheta, d/dphi, d/dlambda of U(theta, phi, lambda)
        set2(dm, make_double2(-0.5 * s, 0), cscale(el, -0.5 * c), cscale(ep, 0.5 * c), cscale(epl, -0.5 * s));
        set2(dm + kMatStride, Z0, Z0, cmul(I1, cscale(ep, s)), cmul(I1, cscale(epl, c)));
        set2(dm + 2 * kMatStride, Z0, cmul(I1, cscale(el, -s)), Z0, cmul(I1, cscale(epl, c)));
      }
      break;
    }
    default: set2(m, O1, Z0, Z0, O1); break;  // ID, SWAP (unused)
  }
}


__global__ void k_bind_matrices(const GateSrc* __restrict__ src, uint32_t n_slots,
                                const double* __restrict__ theta, uint32_t n_params, uint32_t batch,
                                double* __restrict__ mats, double* __restrict__ dmats) {
  uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)n_slots * batch) return;
  uint32_t b = (uint32_t)(idx / n_slots), slot = (uint32_t)(idx % n_slots);
  bind_slot(src[slot], theta + (uint64_t)b * n_params, mats + idx * kMatStride,
            dmats ? dmats + idx * 3 * kMatStride : nullptr);
}

// The matrix slots of many programs at once (a batch of requests, each with its
// own theta row and matrices): one thread per slot; unit k covers slots
// [units[k].slot_begin, units[k + 1].slot_begin) of the flat range.
__global__ void k_bind_units(const BindUnit* __restrict__ units, uint32_t n_units, uint64_t n_total) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_total) return;
  uint32_t lo = 0, hi = n_units;  // the last unit whose slot_begin <= idx
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (units[mid].slot_begin <= idx) lo = mid;
    else hi = mid;
  }
  const BindUnit u = units[lo];
  const uint64_t slot = idx - u.slot_begin;
  bind_slot(u.src[slot], u.theta, u.mats + slot * kMatStride, nullptr);
}

hipError_t launch_bind_units(const BindUnit* units, uint32_t n_units, uint64_t n_total, hipStream_t st) {
  if (!n_total || !n_units) return hipSuccess;
  hipLaunchKernelGGL(k_bind_units, dim3((uint32_t)((n_total + 255) / 256)), dim3(256), 0, st, units, n_units,
                     n_total);
  return hipGetLastError();
}

hipError_t launch_bind_matrices(const GateSrc* src, uint32_t n_slots, const double* theta,
                                uint32_t n_params, uint32_t batch, double* mats, double* dmats,
                                hipStream_t st) {
  uint64_t total = (uint64_t)n_slots * batch;
  if (total == 0) return hipSuccess;
  uint32_t blocks = (uint32_t)((total + 255) / 256);
  hipLaunchKernelGGL(k_bind_matrices, dim3(blocks), dim3(256), 0, st, src, n_slots, theta, n_params,
                     batch, mats, dmats);
  return hipGetLastError();
}

// Depolarizing slots of a call with rate p (one thread per shot and slot): the
// word of counter (noise[ctr[e]].ctr[0..2], 1) under key (key[0], key[1] + s),
// as u = (w >> 11) 2^-53, puts X (u < p/3), Y (u < 2p/3), Z (u < p) or the
// identity into matrix slot slot[e] of shot s. The fourth counter word is 0 in
// every measure/reset event's counter, so the two kinds of draws never meet.
// With dirty: a slot that draws a Pauli marks dirty[s * n_dense + nd[e]]
// (nd[e]: the dense phase holding slot e, or kNoDense), so that only those
// phases of the shot are composed again.
__global__ void k_noise_matrices(const uint32_t* __restrict__ slot, const uint32_t* __restrict__ ctr, uint32_t n,
                                 const qsv_noise* __restrict__ noise, const uint64_t* __restrict__ key, double p,
                                 uint32_t shots, uint64_t mat_stride, double* __restrict__ mats,
                                 const uint32_t* __restrict__ nd, uint32_t n_dense, uint8_t* __restrict__ dirty) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)n * shots) return;
  const uint32_t s = (uint32_t)(idx / n), e = (uint32_t)(idx % n);
  const qsv_noise c = noise[ctr[e]];
  uint64_t c0 = c.ctr[0], c1 = c.ctr[1], c2 = c.ctr[2], c3 = 1;
  philox_block(c0, c1, c2, c3, key[0], key[1] + s);
  const double u = (double)(c0 >> 11) * 0x1p-53;
  const double2 Z0 = make_double2(0, 0), O1 = make_double2(1, 0);
  double* m = mats + (uint64_t)s * mat_stride + (uint64_t)slot[e] * kMatStride;
  if (u < p && dirty && nd[e] != kNoDense) dirty[(uint64_t)s * n_dense + nd[e]] = 1;
  if (u >= p) set2(m, O1, Z0, Z0, O1);
  else if (u < p / 3.0) set2(m, Z0, O1, O1, Z0);
  else if (u < 2.0 * p / 3.0) set2(m, Z0, make_double2(0, -1), make_double2(0, 1), Z0);
  else set2(m, O1, Z0, Z0, make_double2(-1, 0));
}

// one workgroup clears n words (a fill kernel: safe to capture in a graph)
__global__ void k_zero_u32(uint32_t* p, uint32_t n);

hipError_t launch_noise_matrices(const uint32_t* slot, const uint32_t* ctr, uint32_t n, const qsv_noise* noise,
                                 const uint64_t* key, double p, uint32_t shots, uint64_t mat_stride, double* mats,
                                 const uint32_t* nd, uint32_t n_dense, uint8_t* dirty, hipStream_t st) {
  if (dirty && n_dense && shots) {
    const uint64_t words = ((uint64_t)shots * n_dense + 3) / 4;
    if (words > 0xFFFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, st, reinterpret_cast<uint32_t*>(dirty), (uint32_t)words);
  }
  const uint64_t total = (uint64_t)n * shots;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_noise_matrices, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, st, slot, ctr, n, noise,
                     key, p, shots, mat_stride, mats, nd, n_dense, dirty);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Control blocks and state initialisation
// ---------------------------------------------------------------------------
__global__ void k_init_ctl(ShotCtl* ctl, uint64_t* creg, uint32_t cw, uint8_t* record, uint32_t max_record,
                           uint32_t shots) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= shots) return;
  ShotCtl c;
  c.flags = 0;
  c.pend_mask = 0;
  c.pend_val = 0;
  c.frame = 0;
  c.pend_scale = 1.0;
  c.record_prob = 1.0;
  c.n_events = 0;
  c.n_record = 0;
  c.status = 0;
  c.wg_done = 0;
  ctl[s] = c;
  for (uint32_t w = 0; w < cw; ++w) creg[(uint64_t)s * cw + w] = 0;
  if (record)
    for (uint32_t w = 0; w < max_record; ++w) record[(uint64_t)s * max_record + w] = 0;
}

hipError_t launch_init_ctl(ShotCtl* ctl, uint64_t* creg, uint32_t cw, uint8_t* record, uint32_t max_record,
                           uint32_t shots, hipStream_t st) {
  if (!shots) return hipSuccess;
  hipLaunchKernelGGL(k_init_ctl, dim3((shots + 255) / 256), dim3(256), 0, st, ctl, creg, cw, record, max_record,
                     shots);
  return hipGetLastError();
}

template <typename CT>
__global__ void k_init_state(CT* __restrict__ state, uint64_t stride, uint64_t dim, uint32_t shots) {
  uint64_t total = dim * shots;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t s = i / dim, j = i % dim;
    state[s * stride + j] = cmake<CT>(j == 0 ? 1.0 : 0.0, 0.0);
  }
}

hipError_t launch_init_state(double2* state, uint64_t stride, uint32_t n, uint32_t shots, hipStream_t st, bool c64) {
  uint64_t total = (1ull << n) * shots;
  uint64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (c64)
    hipLaunchKernelGGL(k_init_state<float2>, dim3((uint32_t)blocks), dim3(256), 0, st,
                       reinterpret_cast<float2*>(state), stride, 1ull << n, shots);
  else
    hipLaunchKernelGGL(k_init_state<double2>, dim3((uint32_t)blocks), dim3(256), 0, st, state, stride, 1ull << n,
                       shots);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tile pass
// ---------------------------------------------------------------------------
// Applies one gate to the LDS tile (tile-local logical indices).
template <typename CT>
__device__ __forceinline__ void tile_apply(CT* __restrict__ tile, uint32_t t, const DGate& g,
                                           const double* __restrict__ m) {
  const uint32_t tid = threadIdx.x;
  switch (g.type) {
    case GT_DENSE1: case GT_DIAG1: {
      const M2x<CT> u = load_m2x<CT>(m, 0);
      const uint32_t np = 1u << (t - 1), bit = 1u << g.b0;
      if (g.type == GT_DIAG1) {
        for (uint32_t p = tid; p < np; p += kTileThreads) {
          uint32_t i0 = ins0(p, g.b0), i1 = i0 | bit;
          tile[i0] = cmul(u.a, tile[i0]);
          tile[i1] = cmul(u.d, tile[i1]);
        }
      } else {
        for (uint32_t p = tid; p < np; p += kTileThreads) {
          uint32_t i0 = ins0(p, g.b0), i1 = i0 | bit;
          CT x0 = tile[i0], x1 = tile[i1];
          tile[i0] = cmac2(u.a, x0, u.b, x1);
          tile[i1] = cmac2(u.c, x0, u.d, x1);
        }
      }
      break;
    }
    case GT_X1: {
      const uint32_t np = 1u << (t - 1), bit = 1u << g.b0;
      for (uint32_t p = tid; p < np; p += kTileThreads) {
        uint32_t i0 = ins0(p, g.b0), i1 = i0 | bit;
        CT x0 = tile[i0];
        tile[i0] = tile[i1];
        tile[i1] = x0;
      }
      break;
    }
    default: {  // two-qubit gates
      const uint32_t lo = g.b0 < g.b1 ? g.b0 : g.b1, hi = g.b0 < g.b1 ? g.b1 : g.b0;
      const uint32_t nq = 1u << (t - 2);
      const uint32_t B0 = 1u << g.b0, B1 = 1u << g.b1;
      if (g.type == GT_CX) {
        for (uint32_t p = tid; p < nq; p += kTileThreads) {
          uint32_t i = ins0(ins0(p, lo), hi) | B0;
          CT x = tile[i];
          tile[i] = tile[i | B1];
          tile[i | B1] = x;
        }
      } else if (g.type == GT_CTRL1) {
        const M2x<CT> u = load_m2x<CT>(m, 0);
        for (uint32_t p = tid; p < nq; p += kTileThreads) {
          uint32_t i = ins0(ins0(p, lo), hi) | B0;
          CT x0 = tile[i], x1 = tile[i | B1];
          tile[i] = cmac2(u.a, x0, u.b, x1);
          tile[i | B1] = cmac2(u.c, x0, u.d, x1);
        }
      } else if (g.type == GT_CPHASE) {
        const CT ph = cmake<CT>(m[6], m[7]);
        for (uint32_t p = tid; p < nq; p += kTileThreads) {
          uint32_t i = ins0(ins0(p, lo), hi) | B0 | B1;
          tile[i] = cmul(ph, tile[i]);
        }
      } else {  // GT_SWAP
        for (uint32_t p = tid; p < nq; p += kTileThreads) {
          uint32_t i = ins0(ins0(p, lo), hi);
          CT x = tile[i | B0];
          tile[i | B0] = tile[i | B1];
          tile[i | B1] = x;
        }
      }
      break;
    }
  }
}

template <typename CT>
__global__ __launch_bounds__(kTileThreads) void k_tile_pass(
    CT* __restrict__ state, uint64_t stride, ShotCtl* __restrict__ ctl,
    const DGate* __restrict__ gates, const double* __restrict__ mats, uint64_t mat_stride, PassArgs a) {
  extern __shared__ double2 qsv_lds[];
  CT* const tile = reinterpret_cast<CT*>(qsv_lds);
  const uint32_t shot = blockIdx.y, w = blockIdx.x, tid = threadIdx.x;
  ShotCtl* c = ctl + shot;
  if (c->status != 0) return;
  const uint64_t flags = c->flags, M = c->pend_mask, F = c->frame;
  const double s = c->pend_scale;
  const bool pending = M != 0 || s != 1.0;
  bool any = false;
  for (uint32_t i = 0; i < a.gate_count && !any; ++i) any = guard_ok(flags, gates[a.gate_begin + i].guard);
  if (!a.init && !any) return;  // the pending collapse stays owed to a later pass
  const uint64_t V = c->pend_val;
  // Tile w holds the logical indices whose non-tile bits spell w; amplitude i is
  // stored at memory index i ^ F (the shot's flip frame), so a workgroup reads
  // and writes one memory tile and gates act on logical indices.
  uint64_t base = 0;
  {
    uint32_t k = 0;
    for (uint32_t q = 0; q < a.n; ++q)
      if (!((a.tile_mask >> q) & 1ull)) base |= (uint64_t)((w >> k++) & 1u) << q;
  }
  CT* st = state + (uint64_t)shot * stride;
  const uint32_t T = 1u << a.t;
  for (uint32_t l = tid; l < T; l += kTileThreads) {
    uint64_t gi = base | local_to_global(l, a);
    CT v;
    if (a.init) {
      v = cmake<CT>(gi == 0 ? 1.0 : 0.0, 0.0);
    } else if ((gi & M) != V) {
      v = cmake<CT>(0.0, 0.0);
    } else {
      v = st[gi ^ F];
      if (pending) v = cscale(v, s);
    }
    tile[l] = v;
  }
  __syncthreads();
  const double* mb = mats + (uint64_t)shot * mat_stride;
  for (uint32_t i = 0; i < a.gate_count; ++i) {
    DGate g = gates[a.gate_begin + i];
    if (!guard_ok(flags, g.guard)) continue;
    tile_apply(tile, a.t, g, mb + (uint64_t)g.mat * kMatStride);
    __syncthreads();
  }
  for (uint32_t l = tid; l < T; l += kTileThreads) st[(base | local_to_global(l, a)) ^ F] = tile[l];
  if (pending) {
    // the last workgroup of this shot to finish clears the pending collapse
    __syncthreads();
    if (tid == 0) {
      __threadfence();
      uint32_t done = atomicAdd(&c->wg_done, 1u);
      if (done == a.tiles - 1) {
        c->pend_mask = 0;
        c->pend_val = 0;
        c->pend_scale = 1.0;
        c->wg_done = 0;
      }
    }
  }
}

template <bool kDenseOnly, typename CT>
__global__ __launch_bounds__(kTileThreads) void k_tile_pass_r(CT* __restrict__ state, uint64_t stride, ShotCtl* __restrict__ ctl,
                              const DGate* __restrict__ gates, const Phase* __restrict__ phases,
                              const double* __restrict__ mats, uint64_t mat_stride, PassArgs a, uint32_t shots);

hipError_t resident_grid(const void* kernel, uint32_t threads, size_t lds, size_t max_lds, uint32_t* out) {
  struct Entry {
    int dev;
    const void* kernel;
    uint32_t threads;
    size_t lds;
    uint32_t grid;
  };
  static Entry cache[64];
  static int used = 0;
  static std::mutex mu;  // forked contexts launch from several host threads
  std::lock_guard<std::mutex> lk(mu);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  for (int i = 0; i < used; ++i)
    if (cache[i].dev == dev && cache[i].kernel == kernel && cache[i].threads == threads && cache[i].lds == lds) {
      *out = cache[i].grid;
      return hipSuccess;
    }
  e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)max_lds);
  if (e != hipSuccess) return e;
  int cus = 0, per = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, (int)threads, lds);
  if (e != hipSuccess) return e;
  const uint32_t grid = (uint32_t)std::max(1, cus) * (uint32_t)std::max(1, per);
  if (used < 64) cache[used++] = Entry{dev, kernel, threads, lds, grid};
  *out = grid;
  return hipSuccess;
}

// Waves per SIMD the eight-wave dense pass is compiled for: two workgroups per
// CU with complex128 tiles (64 KiB of LDS each), three with complex64 tiles
// (32 KiB), so that the HBM, LDS and matrix-core work of different workgroups
// overlap.
// kPreload: the staged phases' descriptors are read once per workgroup into
// scalar registers (complex128; the complex64 build, held to 80 VGPRs for its
// third workgroup, spills more with them and runs slower).
template <typename CT> struct D8Waves;
template <> struct D8Waves<double2> { static constexpr int kMin = 4; static constexpr bool kPreload = true; };
template <> struct D8Waves<float2> { static constexpr int kMin = 6; static constexpr bool kPreload = false; };
template <typename CT>
__global__ __launch_bounds__(2 * kTileThreads, D8Waves<CT>::kMin) void k_tile_pass_d8(
    CT* __restrict__ state, uint64_t stride, ShotCtl* __restrict__ ctl, const Phase* __restrict__ phases,
    const double* __restrict__ mats, uint64_t mat_stride, PassArgs a, uint32_t shots, uint32_t lds_mats);

template <typename CT>
static hipError_t tile_pass_t(const RunBuffers& rb, CT* state, const DGate* gates, const Phase* phases,
                              const double* mats, uint64_t mat_stride, const PassArgs& a, hipStream_t st) {
  dim3 grid(a.tiles, rb.shots);
  size_t lds = (size_t)sizeof(CT) << a.t;
  if (a.phase_count) {
    const uint64_t total = (uint64_t)a.tiles * rb.shots;
    const size_t mat_lds = (size_t)a.phase_count * 256u * sizeof(CT);
    const size_t max_lds = (sizeof(CT) << kTileMaxBits) + kLdsDensePhases * 256u * sizeof(CT);
    const uint32_t nthr = 1u << (a.t - kRegBits);
    uint32_t g = 0;
    hipError_t e = hipSuccess;
    // the dense-only variant stages the pass's matrices once per workgroup,
    // so it runs where every shot of the launch shares them
    const bool dense_only = a.all_dense && a.t >= kDenseMinTileBits && a.phase_count <= kLdsDensePhases &&
                            mat_stride == 0;
    // all-dense passes: eight amplitudes per thread, 2^(t - 9) waves per tile
    if (a.all_dense && a.t >= kDenseMinTileBits) {
      const uint32_t staged = (a.phase_count <= kLdsDensePhases && mat_stride == 0) ? 1u : 0u;
      const size_t l8 = lds + (staged ? mat_lds : 0);
      e = resident_grid((const void*)k_tile_pass_d8<CT>, 2 * nthr, l8, max_lds, &g);
      if (e != hipSuccess) return e;
      if ((uint64_t)g > total) g = (uint32_t)total;
      if (!g) return hipSuccess;
      hipLaunchKernelGGL(k_tile_pass_d8<CT>, dim3(g), dim3(2 * nthr), l8, st, state, rb.stride, rb.ctl, phases, mats,
                         mat_stride, a, rb.shots, staged);
      return hipGetLastError();
    }
    if (dense_only) lds += mat_lds;
    e = dense_only ? resident_grid((const void*)k_tile_pass_r<true, CT>, nthr, lds, max_lds, &g)
                   : resident_grid((const void*)k_tile_pass_r<false, CT>, nthr, lds, max_lds, &g);
    if (e != hipSuccess) return e;
    if ((uint64_t)g > total) g = (uint32_t)total;
    if (!g) return hipSuccess;
    if (dense_only)
      k_tile_pass_r<true, CT><<<dim3(g), dim3(nthr), lds, st>>>(state, rb.stride, rb.ctl, gates, phases, mats,
                                                                 mat_stride, a, rb.shots);
    else
      k_tile_pass_r<false, CT><<<dim3(g), dim3(nthr), lds, st>>>(state, rb.stride, rb.ctl, gates, phases, mats,
                                                                  mat_stride, a, rb.shots);
  } else {
    hipLaunchKernelGGL(k_tile_pass<CT>, grid, dim3(kTileThreads), lds, st, state, rb.stride, rb.ctl, gates,
                       mats, mat_stride, a);
  }
  return hipGetLastError();
}

hipError_t launch_tile_pass(const RunBuffers& rb, const DGate* gates, const Phase* phases, const double* mats,
                            uint64_t mat_stride, const PassArgs& a, hipStream_t st) {
  if (rb.c64)
    return tile_pass_t(rb, reinterpret_cast<float2*>(rb.state), gates, phases, mats, mat_stride, a, st);
  return tile_pass_t(rb, rb.state, gates, phases, mats, mat_stride, a, st);
}

// ---------------------------------------------------------------------------
// Register-blocked tile pass
//
// Each thread owns the 16 amplitudes of the tile that differ only in the
// phase's 4 register bits, applies the phase's gates to them in registers and
// hands them back through LDS, where the next phase picks up a different set
// of 4 bits. One LDS round trip per phase instead of one per gate.
// ---------------------------------------------------------------------------

// Composes every dense phase: column c of the phase's complex matrix M is the
// phase's gate list applied, in order, to the basis vector e_c (one thread per
// batch element, phase and column), stored in matrix-core operand order.

__device__ __forceinline__ void compose_column(const Phase& ph, const DGate* __restrict__ gates, double* mb,
                                               uint32_t c) {
  double2 a[kR];
#pragma unroll
  for (int k = 0; k < kR; ++k) a[k] = make_double2(k == (int)c ? 1.0 : 0.0, 0.0);
  for (uint32_t i = 0; i < ph.gate_count; ++i) {
    const DGate g = gates[ph.gate_begin + i];
    r_apply(a, g.type, g.j0, g.j1, mb + (uint64_t)g.mat * kMatStride);
  }
  double2* A = reinterpret_cast<double2*>(mb + (uint64_t)ph.dense * kMatStride);
#pragma unroll
  for (uint32_t r = 0; r < (uint32_t)kR; ++r) A[dense_pos(r, c)] = a[r];
}

// With dirty: a phase whose slots all hold what they hold in the matrix set
// `clean` (dirty[b * n_dense + d] == 0) takes its column from clean's composed
// matrix, the same gate list applied to the same matrices.
__global__ void k_compose_dense(const Phase* __restrict__ phases, const uint32_t* __restrict__ dense,
                                uint32_t n_dense, const DGate* __restrict__ gates, uint32_t batch,
                                uint64_t mat_stride, double* __restrict__ mats, const uint8_t* __restrict__ dirty,
                                const double* __restrict__ clean) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)n_dense * kR * batch) return;
  // column fastest, then batch element, then phase: the lanes of a wave
  // compose one phase (one gate list, no divergence) for four batch elements
  const uint32_t c = (uint32_t)(idx % kR);
  const uint64_t rest = idx / kR;
  const uint32_t b = (uint32_t)(rest % batch), d = (uint32_t)(rest / batch);
  const Phase ph = phases[dense[d]];
  double* mb = mats + (uint64_t)b * mat_stride;
  if (dirty && !dirty[(uint64_t)b * n_dense + d]) {
    const double2* src = reinterpret_cast<const double2*>(clean + (uint64_t)ph.dense * kMatStride);
    double2* dst = reinterpret_cast<double2*>(mb + (uint64_t)ph.dense * kMatStride);
#pragma unroll
    for (uint32_t r = 0; r < (uint32_t)kR; ++r) dst[dense_pos(r, c)] = src[dense_pos(r, c)];
    return;
  }
  compose_column(ph, gates, mb, c);
}

// The same over the dense phases of many programs at once (a batch of
// requests, each with its own matrices): one thread per unit and column.
__global__ void k_compose_units(const ComposeUnit* __restrict__ units, uint32_t n_units) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)n_units * kR) return;
  const ComposeUnit u = units[idx / kR];
  compose_column(u.phases[u.phase], u.gates, u.mats, (uint32_t)(idx % kR));
}

hipError_t launch_compose_units(const ComposeUnit* units, uint32_t n_units, hipStream_t st) {
  const uint64_t total = (uint64_t)n_units * kR;
  if (!total) return hipSuccess;
  hipLaunchKernelGGL(k_compose_units, dim3((uint32_t)((total + 127) / 128)), dim3(128), 0, st, units, n_units);
  return hipGetLastError();
}

hipError_t launch_compose_dense(const Phase* phases, const uint32_t* dense, uint32_t n_dense, const DGate* gates,
                                uint32_t batch, uint64_t mat_stride, double* mats, hipStream_t st,
                                const uint8_t* dirty, const double* clean) {
  const uint64_t total = (uint64_t)n_dense * kR * batch;
  if (!total) return hipSuccess;
  hipLaunchKernelGGL(k_compose_dense, dim3((uint32_t)((total + 127) / 128)), dim3(128), 0, st, phases, dense,
                     n_dense, gates, batch, mat_stride, mats, dirty, clean);
  return hipGetLastError();
}

// group bits 4..7 of a wave-uniform group index, scattered over the mask bits
__device__ __forceinline__ uint32_t udep_hi(const UBits& u, uint32_t g) {
  return (((g >> 4) & 1u) ? u.b[4] : 0u) | (((g >> 5) & 1u) ? u.b[5] : 0u) | (((g >> 6) & 1u) ? u.b[6] : 0u) |
         (((g >> 7) & 1u) ? u.b[7] : 0u);
}

// One dense phase on the matrix cores, for the 64 amplitude groups of this
// thread's wave (group g = tile-local indices with the non-register bits set
// to the bits of g). With M = A + iB and a block of 16 groups as X + iY (16
// components x 16 groups), the product is formed from three real 16x16
// products, P1 = A X, P2 = B Y, P3 = (A + B)(X + Y): real part P1 - P2,
// imaginary part P3 - P1 - P2 (three real multiplications per complex one
// instead of four). Each real product is 4 v_mfma_f64_16x16x4f64; that
// instruction takes A[l % 16][l / 16] and B[l / 16][l % 16] from lane l and
// returns D[4 v + l / 16][l % 16] in its result element v (the
// double-precision form interleaves the rows). So lane l needs M[l % 16][4 kb +
// l / 16] (kb = 0..3: the complex values at Mc[kb * 64 + l]), reads the
// components q + 4 kb (q = l / 16) of its group in each block and writes back
// the same components. The wave reads a block before it writes it, and the
// blocks of different waves are disjoint.
// lane l's matrix-core operand of a phase matrix: Mc[kb * 64 + l], kb = 0..3;
// from LDS when the pass's matrices are staged there (in the amplitude type),
// else from HBM, rounded to it (two loops, so the compiler keeps the LDS reads
// as LDS reads)
template <typename CT>
__device__ __forceinline__ void load_mfrag(CT (&mf)[4], bool staged, const CT* __restrict__ lds_mats,
                                           const double2* __restrict__ gmat, uint32_t lane) {
  typedef typename CxT<CT>::R R;
  typedef __attribute__((address_space(3))) const R lds_r;
  typedef __attribute__((address_space(1))) const double glb_d;
  if (staged) {
    const lds_r* l = (const lds_r*)lds_mats;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      mf[kb].x = l[2 * (kb * 64 + (int)lane)];
      mf[kb].y = l[2 * (kb * 64 + (int)lane) + 1];
    }
  } else {
    const glb_d* g = (const glb_d*)gmat;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) mf[kb] = cmake<CT>(g[2 * (kb * 64 + (int)lane)], g[2 * (kb * 64 + (int)lane) + 1]);
  }
}

// One 16x16x4 product step on the matrix cores in the amplitude precision.
// kRowsInterleaved: result element v of lane l is row 4 v + l / 16 (the
// double-precision instruction) rather than row 4 (l / 16) + v (single).
template <typename CT> struct MfmaT;
template <> struct MfmaT<double2> {
  typedef double R;
  typedef qsv_d4 V4;
  static constexpr bool kRowsInterleaved = true;
  __device__ static V4 step(double a, double b, V4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
template <> struct MfmaT<float2> {
  typedef float R;
  typedef qsv_f4 V4;
  static constexpr bool kRowsInterleaved = false;
  __device__ static V4 step(float a, float b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

template <int kBlocks, typename CT>
__device__ __forceinline__ void dense_phase_mfma(CT* __restrict__ tile, uint32_t T, uint32_t tid,
                                                 const Phase& ph, const CT (&mf)[4]) {
  typedef MfmaT<CT> Mf;
  typedef typename Mf::R R;
  // this wave's groups: gbase + 16 cb + j, cb < kBlocks
  const uint32_t lane = tid & 63u, q = lane >> 4, j = lane & 15u;
  const uint32_t wbase = __builtin_amdgcn_readfirstlane(tid >> 6) * (16u * kBlocks);
  const uint32_t o0 = 1u << ph.r[0], o1 = 1u << ph.r[1], o2 = 1u << ph.r[2], o3 = 1u << ph.r[3];
  const UBits u = ubits((T - 1u) & ~(o0 | o1 | o2 | o3));
  R fa[4], fb[4], fs[4];  // fragments of A, B and A + B
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    fa[kb] = mf[kb].x;
    fb[kb] = mf[kb].y;
    fs[kb] = mf[kb].x + mf[kb].y;
  }
  // slot of component q + 4 k of group gbase + 16 cb + j: a per-lane part (group
  // bits 0..3, component bits of q) XOR a wave-uniform part (higher group bits,
  // component bits of k)
  const uint32_t rl = swz(udep<4>(u, j) | ((q & 1u) ? o0 : 0u) | ((q & 2u) ? o1 : 0u));
  // where results go when the result rows are grouped: element v of lane l is
  // component 4 q + v (component bits 0..1 from v, bits 2..3 from q)
  const uint32_t rw = swz(udep<4>(u, j) | ((q & 1u) ? o2 : 0u) | ((q & 2u) ? o3 : 0u));
  // software-pipelined over the blocks: the reads of block b + 1 are issued
  // before the writes of block b, so the LDS round trip of the next block
  // overlaps the tail of the current block's products
  uint32_t slot[2][4];
  CT x[2][4];
  {
    const uint32_t ug = udep_hi(u, wbase);
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
      slot[0][k] = rl ^ swz(ug | ((k & 1u) ? o2 : 0u) | ((k & 2u) ? o3 : 0u));
      x[0][k] = tile[slot[0][k]];
    }
  }
#pragma unroll
  for (uint32_t cb = 0; cb < (uint32_t)kBlocks; ++cb) {
    const uint32_t c = cb & 1u;
    typename Mf::V4 p1 = {0, 0, 0, 0}, p2 = {0, 0, 0, 0}, p3 = {0, 0, 0, 0};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      p1 = Mf::step(fa[kb], x[c][kb].x, p1);
      p2 = Mf::step(fb[kb], x[c][kb].y, p2);
      p3 = Mf::step(fs[kb], x[c][kb].x + x[c][kb].y, p3);
    }
    // the block's results go to the slots it read (every read of the block
    // is complete: its values entered the products above)
    uint32_t wslot[4];
    if (Mf::kRowsInterleaved) {
#pragma unroll
      for (int v = 0; v < 4; ++v) wslot[v] = slot[c][v];
    } else {
      const uint32_t ug = udep_hi(u, wbase + 16u * cb);
#pragma unroll
      for (uint32_t v = 0; v < 4; ++v) wslot[v] = rw ^ swz(ug | ((v & 1u) ? o0 : 0u) | ((v & 2u) ? o1 : 0u));
    }
    if (cb + 1 < (uint32_t)kBlocks) {
      const uint32_t ug = udep_hi(u, wbase + 16u * (cb + 1));
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k) {
        slot[c ^ 1u][k] = rl ^ swz(ug | ((k & 1u) ? o2 : 0u) | ((k & 2u) ? o3 : 0u));
        x[c ^ 1u][k] = tile[slot[c ^ 1u][k]];
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      CT o;
      o.x = p1[v] - p2[v];
      o.y = p3[v] - p1[v] - p2[v];
      tile[wslot[v]] = o;
    }
  }
}

// Runs the register phases of a pass on a tile of T amplitudes staged in LDS
// (slot swz(l) holds tile-local index l). Threads tid < nthr own 16 amplitudes
// per phase; every thread of the workgroup reaches the barriers.
// kDense: apply the composed matrix of dense phases on the matrix cores;
// kGates: apply gate lists (of every phase when !kDense, else of the phases
// that are not dense). A kernel built without kGates runs only passes whose
// phases are all dense (unguarded, on tiles of at least 64 threads).
// lds_mats: the pass's dense matrices staged in LDS (phase p at lds_mats + 256 p),
// or null to read them from the matrix slots.
template <bool kDense, bool kGates, typename CT>
__device__ __forceinline__ void run_phases(CT* __restrict__ tile, uint32_t T, uint32_t tid, uint32_t nthr, uint64_t flags,
                           const Phase* __restrict__ phases, uint32_t pb, uint32_t pc,
                           const DGate* __restrict__ gates, const double* __restrict__ mb,
                           const CT* __restrict__ lds_mats = nullptr) {
  CT r[kR];
  for (uint32_t p = 0; p < pc; ++p) {
    const Phase ph = load_phase(phases + pb + p);
    if (kGates) {
      bool act = false;
      for (uint32_t i = 0; i < ph.gate_count && !act; ++i) act = guard_ok(flags, gates[ph.gate_begin + i].guard);
      if (!act) continue;
    }
    if (kDense && ph.dense != kNoDense && nthr >= 64u) {
      if (tid < nthr) {
        CT mf[4];
        load_mfrag(mf, lds_mats != nullptr, lds_mats + (size_t)p * 256u,
                   reinterpret_cast<const double2*>(mb + (uint64_t)ph.dense * kMatStride), tid & 63u);
        dense_phase_mfma<4>(tile, T, tid, ph, mf);
      }
    } else if (kGates && tid < nthr) {
      const uint32_t o0 = 1u << ph.r[0], o1 = 1u << ph.r[1], o2 = 1u << ph.r[2], o3 = 1u << ph.r[3];
      const uint32_t lb = pdep32(tid, (T - 1u) & ~(o0 | o1 | o2 | o3));
#pragma unroll
      for (int k = 0; k < kR; ++k) {
        const uint32_t l = lb | ((k & 1) ? o0 : 0u) | ((k & 2) ? o1 : 0u) | ((k & 4) ? o2 : 0u) | ((k & 8) ? o3 : 0u);
        r[k] = tile[swz(l)];
      }
      {
      // DGate words: [0] type | b0 | b1 | nang | j0 | j1 | q0 | q1, [1] mat | pad, [2] guard;
      // gate words and matrices are wave-uniform scalar loads, the next gate's
      // are requested before the current gate is applied
      const uint64_t* gw = reinterpret_cast<const uint64_t*>(gates + ph.gate_begin);
      const double* mp = mb + (uint64_t)ph.gate_begin * kMatStride;
      uint64_t w0n = gw[0], gdn = gw[2];
      double mn[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) mn[e] = mp[e];
      for (uint32_t i = 0; i < ph.gate_count; ++i) {
        const uint64_t w0 = w0n, gd = gdn;
        double m[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) m[e] = mn[e];
        if (i + 1 < ph.gate_count) {
          w0n = gw[(uint64_t)(i + 1) * 4];
          gdn = gw[(uint64_t)(i + 1) * 4 + 2];
#pragma unroll
          for (int e = 0; e < 8; ++e) mn[e] = mp[(uint64_t)(i + 1) * kMatStride + e];
        }
        if (!guard_ok(flags, gd)) continue;
        r_apply(r, (uint8_t)(w0 & 0xFFu), (int)((w0 >> 32) & 0xFFu), (int)((w0 >> 40) & 0xFFu), m);
      }
      }
#pragma unroll
      for (int k = 0; k < kR; ++k) {
        const uint32_t l = lb | ((k & 1) ? o0 : 0u) | ((k & 2) ? o1 : 0u) | ((k & 4) ? o2 : 0u) | ((k & 8) ? o3 : 0u);
        tile[swz(l)] = r[k];
      }
    }
    __syncthreads();
  }
}

// Tile-local index l = tid + k * 2^(t-4) (k = 0..15) of thread tid < 2^(t-4):
// its global index is base | (tid's bits over tq[0..t-5]) | (k's bits over
// tq[t-4..t-1]). Logical amplitude i is stored at memory index i ^ F (the
// shot's flip frame), so a workgroup reads and writes one memory tile while
// gates see logical indices.
__device__ __forceinline__ void store_tile16(const double2* __restrict__ tile, double2* __restrict__ st,
                                             const PassArgs& a, uint64_t base, uint32_t tid, uint64_t F) {
  const uint32_t nthr = 1u << (a.t - kRegBits);
  uint64_t gthr = base;
  for (uint32_t b = 0; b + kRegBits < a.t; ++b) gthr |= (uint64_t)((tid >> b) & 1u) << a.tq[b];
  const uint64_t h0 = 1ull << a.tq[a.t - 4], h1 = 1ull << a.tq[a.t - 3], h2 = 1ull << a.tq[a.t - 2],
                 h3 = 1ull << a.tq[a.t - 1];
  double2 r[kR];
#pragma unroll
  for (int k = 0; k < kR; ++k) r[k] = tile[swz(tid + (uint32_t)k * nthr)];
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    const uint64_t gi = gthr | ((k & 1) ? h0 : 0ull) | ((k & 2) ? h1 : 0ull) | ((k & 4) ? h2 : 0ull) |
                        ((k & 8) ? h3 : 0ull);
    st[gi ^ F] = r[k];
  }
}

// Whether the pass has work for a shot: the shot is alive and (the pass
// initialises the state, or some gate of the pass is enabled by its flags).
__device__ __forceinline__ bool pass_active(const ShotCtl* __restrict__ c, const PassArgs& a,
                                            const DGate* __restrict__ gates) {
  const QSV_CONST ShotCtl* cc = cst(c);
  if (cc->status != 0) return false;
  if (a.init || a.uncond) return true;
  const uint64_t flags = cc->flags;
  for (uint32_t i = 0; i < a.gate_count; ++i)
    if (guard_ok(flags, cst(gates + a.gate_begin + i)->guard)) return true;
  return false;
}

__device__ __forceinline__ uint64_t next_pass_item(uint64_t it, uint64_t total, uint64_t G, const ShotCtl* ctl,
                                                   const PassArgs& a, const DGate* __restrict__ gates,
                                                   uint32_t& last_shot, bool& last_active) {
  for (; it < total; it += G) {
    const uint32_t shot = (uint32_t)(it / a.tiles);
    if (shot != last_shot) {
      last_shot = shot;
      last_active = pass_active(ctl + shot, a, gates);
    }
    if (last_active) break;
  }
  return it;
}

// The 16 amplitudes of a thread (address bits gthr | subsets of h0..h3) in the
// load layout: logical amplitude i is stored at memory index i ^ F. Every
// amplitude is read (one straight run of loads); those outside a pending
// collapse are zeroed when staged.
template <typename CT>
__device__ __forceinline__ void fetch16(CT (&r)[kR], const CT* __restrict__ st, uint64_t gthr, uint64_t h0,
                                        uint64_t h1, uint64_t h2, uint64_t h3, bool init, uint64_t F) {
  if (init) {
#pragma unroll
    for (int k = 0; k < kR; ++k) {
      const uint64_t gi = gthr | ((k & 1) ? h0 : 0ull) | ((k & 2) ? h1 : 0ull) | ((k & 4) ? h2 : 0ull) |
                          ((k & 8) ? h3 : 0ull);
      r[k] = cmake<CT>(gi == 0 ? 1.0 : 0.0, 0.0);
    }
  } else {
#pragma unroll
    for (int k = 0; k < kR; ++k) {
      const uint64_t gi = gthr | ((k & 1) ? h0 : 0ull) | ((k & 2) ? h1 : 0ull) | ((k & 4) ? h2 : 0ull) |
                          ((k & 8) ? h3 : 0ull);
      r[k] = st[gi ^ F];
    }
  }
}

// the 16 amplitudes of a thread into LDS (load layout l = tid + k nthr), with
// the pending collapse's scale applied
template <typename CT>
__device__ __forceinline__ void stage16(CT* __restrict__ tile, const CT (&r)[kR], uint32_t tid,
                                        uint32_t nthr, uint64_t gthr, uint64_t h0, uint64_t h1, uint64_t h2,
                                        uint64_t h3, uint64_t M, uint64_t V, double s) {
  if (M == 0 && s == 1.0) {
#pragma unroll
    for (int k = 0; k < kR; ++k) tile[swz(tid + (uint32_t)k * nthr)] = r[k];
  } else {
#pragma unroll
    for (int k = 0; k < kR; ++k) {
      const uint64_t gi = gthr | ((k & 1) ? h0 : 0ull) | ((k & 2) ? h1 : 0ull) | ((k & 4) ? h2 : 0ull) |
                          ((k & 8) ? h3 : 0ull);
      tile[swz(tid + (uint32_t)k * nthr)] = ((gi & M) == V) ? cscale(r[k], s) : cmake<CT>(0.0, 0.0);
    }
  }
}

// Persistent register-blocked pass. The grid holds as many workgroups as fit
// on the device at once; workgroup b takes the work items (shot, tile)
// b, b + G, b + 2G, ... (item = shot * tiles + tile) of shots the pass has work
// for. While it runs the phases of one tile, the 16 loads per thread of its
// next tile are already in flight (held in registers), so HBM reads overlap
// the gate arithmetic of the same workgroup. kDenseOnly: the variant for
// passes whose phases are all dense (matrix cores only, fewer live registers).
template <bool kDenseOnly, typename CT>
__global__ __launch_bounds__(kTileThreads) void k_tile_pass_r(
    CT* __restrict__ state, uint64_t stride, ShotCtl* __restrict__ ctl, const DGate* __restrict__ gates,
    const Phase* __restrict__ phases, const double* __restrict__ mats, uint64_t mat_stride, PassArgs a,
    uint32_t shots) {
  extern __shared__ double2 qsv_lds[];
  CT* const tile = reinterpret_cast<CT*>(qsv_lds);
  const uint32_t tid = threadIdx.x;
  const uint32_t nthr = 1u << (a.t - kRegBits), T = 1u << a.t;
  const uint64_t total = (uint64_t)a.tiles * shots, G = gridDim.x;
  const uint64_t free_mask = ~a.tile_mask & ((a.n >= 64) ? ~0ull : ((1ull << a.n) - 1ull));
  uint64_t tb = 0;  // this thread's bits over tile qubits tq[0..t-5]
  for (uint32_t b = 0; b + kRegBits < a.t; ++b) tb |= (uint64_t)((tid >> b) & 1u) << a.tq[b];
  const uint64_t h0 = 1ull << a.tq[a.t - 4], h1 = 1ull << a.tq[a.t - 3], h2 = 1ull << a.tq[a.t - 2],
                 h3 = 1ull << a.tq[a.t - 1];
  // next item at or after `it` (in steps of G) whose shot the pass has work for;
  // the answer for the last shot looked at is kept
  uint32_t last_shot = 0xFFFFFFFFu;
  bool last_active = false;
  CT nx[kR];
  // the dense-only variant prefetches the next tile and keeps the pass's
  // dense matrices in LDS after the tile (no vector loads but the prefetch
  // while it computes); the gate-list variant (more live registers) loads each
  // tile when it starts on it
  constexpr bool kPrefetch = kDenseOnly;
  CT* lds_mats = nullptr;
  if (kDenseOnly) {
    lds_mats = tile + T;
    const double* mb0 = mats;  // dense matrices are per call (mat_stride 0 on this path)
    for (uint32_t p = 0; p < a.phase_count; ++p) {
      const double2* src = reinterpret_cast<const double2*>(mb0 + (uint64_t)cst(phases + a.phase_begin + p)->dense *
                                                                      kMatStride);
      for (uint32_t e = tid; e < 256u; e += nthr) lds_mats[p * 256u + e] = cmake<CT>(src[e].x, src[e].y);
    }
    __syncthreads();
  }
  // Loop order: prefetch the next tile, run the phases and store this tile,
  // then stage the next tile in LDS. Staging comes after the stores are issued,
  // so it waits for the prefetched loads only (the stores may still be in
  // flight: the vector-memory counter completes in issue order).
  uint64_t it = next_pass_item(blockIdx.x, total, G, ctl, a, gates, last_shot, last_active);
  if (it < total) {
    const uint32_t sh = (uint32_t)(it / a.tiles);
    const QSV_CONST ShotCtl* cc = cst(ctl + sh);
    const uint64_t g0 = tile_base(it % a.tiles, free_mask) | tb;
    fetch16(nx, state + (uint64_t)sh * stride, g0, h0, h1, h2, h3, a.init, cc->frame);
    stage16(tile, nx, tid, nthr, g0, h0, h1, h2, h3, cc->pend_mask, cc->pend_val, cc->pend_scale);
    __syncthreads();
  }
  while (it < total) {
    const uint32_t shot = (uint32_t)(it / a.tiles);
    ShotCtl* c = ctl + shot;
    const uint64_t flags = cst(c)->flags, F = cst(c)->frame;
    const bool pending = cst(c)->pend_mask != 0 || cst(c)->pend_scale != 1.0;
    const uint64_t base = tile_base(it % a.tiles, free_mask);
    const uint64_t nit = next_pass_item(it + G, total, G, ctl, a, gates, last_shot, last_active);
    const uint32_t nshot = (uint32_t)(nit / a.tiles);
    const uint64_t ngthr = nit < total ? tile_base(nit % a.tiles, free_mask) | tb : 0ull;
    if (kPrefetch && nit < total)
      fetch16(nx, state + (uint64_t)nshot * stride, ngthr, h0, h1, h2, h3, a.init, cst(ctl + nshot)->frame);
    run_phases<true, !kDenseOnly>(tile, T, tid, nthr, flags, phases, a.phase_begin, a.phase_count, gates,
                                  mats + (uint64_t)shot * mat_stride, lds_mats);
    {
      // back to HBM in the load layout (address bits computed once, above)
      CT* st = state + (uint64_t)shot * stride;
      const uint64_t gthr = base | tb;
      CT r[kR];
#pragma unroll
      for (int k = 0; k < kR; ++k) r[k] = tile[swz(tid + (uint32_t)k * nthr)];
#pragma unroll
      for (int k = 0; k < kR; ++k) {
        const uint64_t gi = gthr | ((k & 1) ? h0 : 0ull) | ((k & 2) ? h1 : 0ull) | ((k & 4) ? h2 : 0ull) |
                            ((k & 8) ? h3 : 0ull);
        st[gi ^ F] = r[k];
      }
    }
    if (pending) {
      __syncthreads();
      if (tid == 0) {
        __threadfence();
        const uint32_t done = atomicAdd(&c->wg_done, 1u);
        if (done == a.tiles - 1) {
          c->pend_mask = 0;
          c->pend_val = 0;
          c->pend_scale = 1.0;
          c->wg_done = 0;
        }
      }
    }
    __syncthreads();
    if (nit < total) {
      // nit is a tile its shot has not finished, so that shot's pending
      // collapse is still in place
      const QSV_CONST ShotCtl* cn = cst(ctl + nshot);
      if (!kPrefetch) fetch16(nx, state + (uint64_t)nshot * stride, ngthr, h0, h1, h2, h3, a.init, cn->frame);
      stage16(tile, nx, tid, nthr, ngthr, h0, h1, h2, h3, cn->pend_mask, cn->pend_val, cn->pend_scale);
      __syncthreads();
    }
    it = nit;
  }
}

// Tile pass for passes made only of dense phases, on tiles of 2^t amplitudes
// (10 <= t <= 12), with 2^(t - 9) waves per tile: each thread stages and
// stores 8 amplitudes (load layout l = tid + k * 2^(t - 3)), each wave applies
// the phases to 2 blocks of 16 amplitude groups on the matrix cores, and at
// most 128 registers per thread let several workgroups share a CU (two of
// 2^12, three of 2^11, five of 2^10 amplitudes with their staged matrices),
// so that the waits of one workgroup (LDS, barriers, HBM) are covered by the
// others' matrix-core work. With
// lds_mats the pass's matrices (shared by every shot: mat_stride 0, at most
// kLdsDensePhases of them) are staged in LDS once; otherwise each phase reads
// its matrix from the shot's matrix slots.
template <typename CT>
__global__ __launch_bounds__(2 * kTileThreads, D8Waves<CT>::kMin) void k_tile_pass_d8(
    CT* __restrict__ state, uint64_t stride, ShotCtl* __restrict__ ctl, const Phase* __restrict__ phases,
    const double* __restrict__ mats, uint64_t mat_stride, PassArgs a, uint32_t shots, uint32_t lds_mats) {
  extern __shared__ double2 qsv_lds[];
  CT* const tile = reinterpret_cast<CT*>(qsv_lds);
  constexpr uint32_t kA = 8;
  const uint32_t tid = threadIdx.x, T = 1u << a.t, lane = tid & 63u, nth = T / kA;  // nth = blockDim.x
  const uint64_t total = (uint64_t)a.tiles * shots, G = gridDim.x;
  const uint64_t free_mask = ~a.tile_mask & ((a.n >= 64) ? ~0ull : ((1ull << a.n) - 1ull));
  uint64_t tb = 0;  // this thread's bits over tile qubits tq[0..t-4]
  for (uint32_t b = 0; b + 3 < a.t; ++b) tb |= (uint64_t)((tid >> b) & 1u) << a.tq[b];
  const uint64_t h0 = 1ull << a.tq[a.t - 3], h1 = 1ull << a.tq[a.t - 2], h2 = 1ull << a.tq[a.t - 1];
  CT* const lmats = tile + T;
  if (lds_mats)
    for (uint32_t p = 0; p < a.phase_count; ++p) {
      const double2* src =
          reinterpret_cast<const double2*>(mats + (uint64_t)cst(phases + a.phase_begin + p)->dense * kMatStride);
      for (uint32_t e = tid; e < 256u; e += nth) lmats[p * 256u + e] = cmake<CT>(src[e].x, src[e].y);
    }
  // the first phases' descriptors, read once (wave-uniform, scalar registers):
  // every tile runs the same phases, and a descriptor read inside the tile
  // loop would make each phase wait for it, and for the matrix operand reads
  // issued with it, before any of its address work
  Phase pre[kLdsDensePhases];
  if constexpr (D8Waves<CT>::kPreload) {
#pragma unroll
    for (uint32_t p = 0; p < kLdsDensePhases; ++p)
      pre[p] = load_phase(phases + a.phase_begin + (p < a.phase_count ? p : 0u));
  }
  uint32_t last_shot = 0xFFFFFFFFu;
  bool last_active = false;
  uint64_t it = next_pass_item(blockIdx.x, total, G, ctl, a, nullptr, last_shot, last_active);
  while (it < total) {
    const uint32_t shot = (uint32_t)(it / a.tiles);
    ShotCtl* c = ctl + shot;
    const uint64_t F = cst(c)->frame, M = cst(c)->pend_mask, V = cst(c)->pend_val;
    const double sc = cst(c)->pend_scale;
    const bool pending = M != 0 || sc != 1.0;
    const uint64_t gthr = tile_base(it % a.tiles, free_mask) | tb;
    // amplitude k of this thread is at physical index (gthr | h_k) ^ F = lb + off(k):
    // flipping tile bit h moves by +h, or by -h where the frame holds that bit
    // (gthr never does), so the offsets are wave-uniform and only lb is per lane
    const int64_t d0 = (F & h0) ? -(int64_t)h0 : (int64_t)h0, d1 = (F & h1) ? -(int64_t)h1 : (int64_t)h1,
                  d2 = (F & h2) ? -(int64_t)h2 : (int64_t)h2;
    auto off = [&](int k) { return ((k & 1) ? d0 : 0) + ((k & 2) ? d1 : 0) + ((k & 4) ? d2 : 0); };
    CT* sp = state + (uint64_t)shot * stride + (gthr ^ F);
    CT r[kA];
#pragma unroll
    for (int k = 0; k < (int)kA; ++k) r[k] = a.init ? cmake<CT>(k == 0 && gthr == 0 ? 1.0 : 0.0, 0.0) : sp[off(k)];
#pragma unroll
    for (int k = 0; k < (int)kA; ++k) {
      const uint64_t gi = gthr | ((k & 1) ? h0 : 0ull) | ((k & 2) ? h1 : 0ull) | ((k & 4) ? h2 : 0ull);
      tile[swz(tid + (uint32_t)k * nth)] =
          !pending ? r[k] : (((gi & M) == V) ? cscale(r[k], sc) : cmake<CT>(0.0, 0.0));
    }
    __syncthreads();
    if (D8Waves<CT>::kPreload && lds_mats) {
      // staged matrices (at most kLdsDensePhases phases): descriptors and
      // operands from registers and LDS only
#pragma unroll
      for (uint32_t p = 0; p < kLdsDensePhases; ++p) {
        if (p >= a.phase_count) break;
        CT mf[4];
        load_mfrag(mf, true, lmats + (size_t)p * 256u, nullptr, lane);
        dense_phase_mfma<2>(tile, T, tid, pre[p], mf);
        __syncthreads();
      }
    } else {
      const double* ms = mats + (uint64_t)shot * mat_stride;
      for (uint32_t p = 0; p < a.phase_count; ++p) {
        const Phase ph = load_phase(phases + a.phase_begin + p);
        CT mf[4];
        load_mfrag(mf, lds_mats != 0u, lmats + (size_t)p * 256u,
                   reinterpret_cast<const double2*>(ms + (uint64_t)ph.dense * kMatStride), lane);
        dense_phase_mfma<2>(tile, T, tid, ph, mf);
        __syncthreads();
      }
    }
#pragma unroll
    for (int k = 0; k < (int)kA; ++k) r[k] = tile[swz(tid + (uint32_t)k * nth)];
#pragma unroll
    for (int k = 0; k < (int)kA; ++k) sp[off(k)] = r[k];
    if (pending) {
      __syncthreads();
      if (tid == 0) {
        __threadfence();
        const uint32_t done = atomicAdd(&c->wg_done, 1u);
        if (done == a.tiles - 1) {
          c->pend_mask = 0;
          c->pend_val = 0;
          c->pend_scale = 1.0;
          c->wg_done = 0;
        }
      }
    }
    // no barrier before the next tile: its staging writes go to the slots
    // swz(tid + k * nth) that this thread has just read for the stores
    // (one wave's LDS accesses complete in order), and the staging barrier
    // orders them before any other thread's reads
    it = next_pass_item(it + G, total, G, ctl, a, nullptr, last_shot, last_active);
  }
}

// ---------------------------------------------------------------------------
// Measurement sites
// ---------------------------------------------------------------------------
// Histogram of |psi|^2 over the site's qubits (logical values), restricted to
// the pending collapse. Each workgroup covers a contiguous slice of the free
// (unrestricted) index space; every thread keeps its own 16 bins in LDS and
// the bins are summed in a fixed order, so the result does not depend on how
// many shots share the launch.
// The histogram of one block of one shot's state over the site's qubits (see
// k_site_reduce), summed in a fixed order; threads tid < kSiteBins return bin
// tid, the others 0. Every thread of the workgroup calls it (two barriers).
template <typename CT>
__device__ __forceinline__ double site_bins(const CT* __restrict__ state, uint64_t stride,
                                            const ShotCtl* __restrict__ c, const SiteArgs& a, uint32_t blk,
                                            uint64_t buf, uint32_t tid, double (*bins)[kRedThreads],
                                            double (*red)[kSiteBins]) {
  for (int b = 0; b < kSiteBins; ++b) bins[b][tid] = 0.0;
  if (c->status == 0) {
    const uint64_t M = c->pend_mask, F = c->frame, Vm = c->pend_val ^ (F & M);
    const double s2 = c->pend_scale * c->pend_scale;
    const uint32_t r = (uint32_t)__popcll(M);
    const uint64_t nfree = 1ull << (a.n - r);
    const uint64_t per = (nfree + a.blocks - 1) / a.blocks;
    const uint64_t j0 = per * blk, j1 = (j0 + per < nfree) ? j0 + per : nfree;
    const CT* st = state + buf * stride;
    uint32_t qbit[kSiteQubits];
    uint32_t fq = 0;
    for (uint32_t k = 0; k < a.nq; ++k) {
      qbit[k] = a.q[k];
      fq |= (uint32_t)((F >> a.q[k]) & 1ull) << k;
    }
    for (uint64_t j = j0 + tid; j < j1; j += kRedThreads) {
      uint64_t gi = j;
      if (M) {
        uint64_t mm = M;
        while (mm) {
          uint32_t b = __ffsll((long long)mm) - 1;
          mm &= mm - 1;
          gi = ins0_64(gi, b);
        }
        gi |= Vm;
      }
      const CT v = st[gi];
      const double vx = v.x, vy = v.y;
      double p = (vx * vx + vy * vy) * s2;
      uint32_t bin = 0;
      for (uint32_t k = 0; k < a.nq; ++k) bin |= (uint32_t)((gi >> qbit[k]) & 1ull) << k;
      bin ^= fq;
      bins[bin][tid] += p;
    }
  }
  __syncthreads();
  {
    const uint32_t b = tid & (kSiteBins - 1), part = tid / kSiteBins;
    double acc = 0.0;
    for (uint32_t k = 0; k < kSiteBins; ++k) acc += bins[b][part * kSiteBins + k];
    red[part][b] = acc;
  }
  __syncthreads();
  double acc = 0.0;
  if (tid < kSiteBins)
    for (uint32_t part = 0; part < kRedThreads / kSiteBins; ++part) acc += red[part][tid];
  return acc;
}

template <typename CT>
__global__ __launch_bounds__(kRedThreads) void k_site_reduce(
    const CT* __restrict__ state, uint64_t stride, const ShotCtl* __restrict__ ctl, SiteArgs a,
    double* __restrict__ partials, uint32_t pblocks, const uint32_t* __restrict__ buf_of) {
  __shared__ double bins[kSiteBins][kRedThreads];
  __shared__ double red[kRedThreads / kSiteBins][kSiteBins];
  const uint32_t shot = blockIdx.y, blk = blockIdx.x, tid = threadIdx.x;
  const double v = site_bins(state, stride, ctl + shot, a, blk, buf_of ? buf_of[shot] : shot, tid, bins, red);
  if (tid < kSiteBins) partials[((uint64_t)shot * pblocks + blk) * kSiteBins + tid] = v;
}

// A classical expression (postfix code from code[pc] to its QSV_C_END) on one
// shot's classical bits, in 64-bit two's complement (include/qsv.h).
__device__ int64_t cexec(const qsv_cop* __restrict__ code, uint64_t pc, const uint64_t* creg) {
  int64_t s[kCStack];
  int sp = 0;
  for (;; ++pc) {
    const qsv_cop c = code[pc];
    if (c.op == QSV_C_END) return s[sp - 1];
    if (c.op == QSV_C_IMM) {
      s[sp++] = c.imm;
      continue;
    }
    if (c.op == QSV_C_BITS) {
      uint64_t v = 0;
      for (uint32_t i = 0; i < c.width; ++i) {
        const uint32_t bit = c.lo + i;
        v |= ((creg[bit >> 6] >> (bit & 63)) & 1ull) << i;
      }
      if (c.sgn && c.width < 64 && ((v >> (c.width - 1)) & 1ull)) v |= ~0ull << c.width;
      s[sp++] = (int64_t)v;
      continue;
    }
    if (c.op == QSV_C_NEG || c.op == QSV_C_NOT || c.op == QSV_C_LNOT) {
      const uint64_t a = (uint64_t)s[sp - 1];
      s[sp - 1] = c.op == QSV_C_NEG ? (int64_t)(0ull - a) : c.op == QSV_C_NOT ? (int64_t)~a : (int64_t)(a == 0);
      continue;
    }
    const int64_t b = s[--sp], a = s[sp - 1];
    const uint64_t ua = (uint64_t)a, ub = (uint64_t)b;
    int64_t r;
    switch (c.op) {
      case QSV_C_ADD: r = (int64_t)(ua + ub); break;
      case QSV_C_SUB: r = (int64_t)(ua - ub); break;
      case QSV_C_MUL: r = (int64_t)(ua * ub); break;
      case QSV_C_DIV:  // truncation toward zero; INT64_MIN / -1 wraps to INT64_MIN
        r = b == 0 ? 0 : (b == -1 ? (int64_t)(0ull - ua) : a / b);
        break;
      case QSV_C_MOD: r = (b == 0 || b == -1) ? 0 : a % b; break;
      case QSV_C_AND: r = a & b; break;
      case QSV_C_OR: r = a | b; break;
      case QSV_C_XOR: r = a ^ b; break;
      case QSV_C_SHL: r = (b < 0 || b >= 64) ? 0 : (int64_t)(ua << b); break;
      case QSV_C_SHR: r = (b < 0 || b >= 64) ? (a < 0 ? -1 : 0) : (a >> b); break;
      case QSV_C_EQ: r = a == b; break;
      case QSV_C_NE: r = a != b; break;
      case QSV_C_LT: r = a < b; break;
      case QSV_C_GT: r = a > b; break;
      case QSV_C_LE: r = a <= b; break;
      case QSV_C_GE: r = a >= b; break;
      case QSV_C_LAND: r = (a != 0) && (b != 0); break;
      default: r = (a != 0) || (b != 0); break;
    }
    s[sp - 1] = r;
  }
}

__device__ bool eval_pred(const DPred& p, const uint64_t* creg, const qsv_cop* code) {
  if (p.cmp == QSV_CMP_TRUE) return true;
  if (p.cmp == QSV_CMP_EXPR) return cexec(code, p.value, creg) != 0;
  uint64_t v = 0;
  for (uint32_t i = 0; i < p.width; ++i) {
    uint32_t bit = p.lo + i;
    v |= ((creg[bit >> 6] >> (bit & 63)) & 1ull) << i;
  }
  switch (p.cmp) {
    case QSV_CMP_EQ: return v == p.value;
    case QSV_CMP_NE: return v != p.value;
    case QSV_CMP_LT: return v < p.value;
    case QSV_CMP_GT: return v > p.value;
    case QSV_CMP_LE: return v <= p.value;
    default: return v >= p.value;
  }
}

// The sequential events of a measurement site for one shot, given the
// histogram of |psi|^2 over the site's qubits (logical values, pending collapse
// applied): Philox draws, outcomes (or forced ones), classical bits, flags,
// record, trajectory probability; then the site's collapse and flips are
// composed into the shot's pending collapse and flip frame.
__device__ __forceinline__ void site_events(ShotCtl& cc, const double* bins, const SiteArgs& a, const SiteEvent* __restrict__ ev,
                            const DPred* __restrict__ preds, const qsv_cop* __restrict__ code, uint64_t* cr,
                            uint8_t* rec, uint32_t max_record,
                            const uint8_t* frow, uint32_t forced_len, uint64_t seed, uint64_t key1,
                            double readout_err, double reset_err) {
  uint32_t rm = 0, rv = 0;  // restriction on the bins (pre-site logical values)
  uint64_t xf = 0;          // flips applied during this site
  const double kZero = 0x1p-60;
  for (uint32_t e = 0; e < a.ev_count; ++e) {
    const SiteEvent E = ev[a.ev_begin + e];
    const bool active = guard_ok(cc.flags, E.guard);
    if (E.op == SE_SETF) {
      bool v = active && eval_pred(preds[E.pred], cr, code);
      cc.flags = (cc.flags & ~(1ull << E.flag)) | ((uint64_t)v << E.flag);
      continue;
    }
    if (!active) continue;
    if (E.op == SE_CLRF) {
      cc.flags &= ~(1ull << E.flag);
    } else if (E.op == SE_SETB || E.op == SE_CLRB) {  // classical assignment of one bit
      const uint64_t m = 1ull << (E.cbit & 63u);
      cr[E.cbit >> 6] = (E.op == SE_SETB) ? (cr[E.cbit >> 6] | m) : (cr[E.cbit >> 6] & ~m);
    } else if (E.op == SE_CSTORE) {  // classical assignment of a computed value
      const uint64_t v = (uint64_t)cexec(code, E.pred, cr);
      for (uint32_t i = 0; i < E.flag; ++i) {
        const uint32_t bit = E.cbit + i;
        const uint64_t m = 1ull << (bit & 63u);
        cr[bit >> 6] = ((v >> i) & 1ull) ? (cr[bit >> 6] | m) : (cr[bit >> 6] & ~m);
      }
    } else if (E.op == SE_X) {
      xf ^= 1ull << E.q;
    } else {  // measure or reset
      const uint32_t k = E.k, fq = (uint32_t)((xf >> E.q) & 1ull);
      double p[2] = {0.0, 0.0};
      for (uint32_t b = 0; b < (uint32_t)kSiteBins; ++b)
        if ((b & rm) == rv) p[((b >> k) & 1u) ^ fq] += bins[b];
      const double norm = p[0] + p[1];
      const uint64_t word = philox_word(seed, key1, cc.n_events);
      const double u = (double)(word >> 11) * 0x1p-53;
      cc.n_events++;
      uint32_t o;
      if (E.op == SE_MEASURE && frow && cc.n_record < forced_len) {
        o = frow[cc.n_record] ? 1u : 0u;
        if (p[o] / norm < kZero) {
          cc.status = QSV_ERR_FORCED_ZERO_PROB;
          return;
        }
      } else {
        o = (u < p[0] / norm) ? 0u : 1u;
      }
      cc.record_prob *= p[o] / norm;
      rm |= 1u << k;
      rv |= (o ^ fq) << k;
      if (E.op == SE_MEASURE) {
        // readout error: the next word flips the recorded bit (the state keeps o)
        uint32_t r = o;
        if (readout_err > 0.0) {
          const uint64_t w2 = philox_word(seed, key1, cc.n_events);
          cc.n_events++;
          if ((double)(w2 >> 11) * 0x1p-53 < readout_err) r ^= 1u;
        }
        if (cc.n_record < max_record) rec[cc.n_record] = (uint8_t)r;
        cc.n_record++;
        if (E.cbit != 0xFFFFFFFFu) {
          uint64_t bitm = 1ull << (E.cbit & 63);
          cr[E.cbit >> 6] = r ? (cr[E.cbit >> 6] | bitm) : (cr[E.cbit >> 6] & ~bitm);
        }
      } else {
        if (o) xf ^= 1ull << E.q;  // reset: flip the qubit back to |0>
        // reset error: the next word leaves the qubit flipped
        if (reset_err > 0.0) {
          const uint64_t w2 = philox_word(seed, key1, cc.n_events);
          cc.n_events++;
          if ((double)(w2 >> 11) * 0x1p-53 < reset_err) xf ^= 1ull << E.q;
        }
      }
    }
  }
  // compose the site's collapse with the incoming one (all in logical frames)
  uint64_t R = 0, RV = 0;
  double mass = 0.0;
  for (uint32_t k = 0; k < a.nq; ++k)
    if (rm >> k & 1u) {
      R |= 1ull << a.q[k];
      RV |= (uint64_t)((rv >> k) & 1u) << a.q[k];
    }
  if (rm) {
    for (uint32_t b = 0; b < (uint32_t)kSiteBins; ++b)
      if ((b & rm) == rv) mass += bins[b];
    cc.pend_scale = cc.pend_scale / sqrt(mass);
  }
  const uint64_t M = cc.pend_mask;
  cc.pend_val = ((cc.pend_val ^ (xf & M)) & M) | ((RV ^ (xf & R)) & R);
  cc.pend_mask = M | R;
  cc.frame ^= xf;
}

// The site's events for one shot from its 16 bins, by one thread.
__device__ __forceinline__ void finalize_shot(ShotCtl* __restrict__ c, const double (&bins)[kSiteBins],
                                              const SiteArgs& a, const SiteEvent* __restrict__ ev,
                                              const DPred* __restrict__ preds, const qsv_cop* __restrict__ code,
                                              uint64_t* __restrict__ creg, uint32_t cw, uint8_t* __restrict__ record,
                                              uint32_t max_record, const uint8_t* __restrict__ forced,
                                              uint32_t forced_len, uint64_t seed, uint64_t shot_base, uint32_t shot,
                                              double readout_err, double reset_err,
                                              const uint64_t* __restrict__ key) {
  ShotCtl cc = *c;
  if (key) {
    seed = key[0];
    shot_base = key[1];
  }
  site_events(cc, bins, a, ev, preds, code, creg + (uint64_t)shot * cw, record + (uint64_t)shot * max_record,
              max_record, forced ? forced + (uint64_t)shot * forced_len : nullptr, forced_len, seed,
              shot_base + shot, readout_err, reset_err);
  *c = cc;
}

__global__ __launch_bounds__(64) void k_site_finalize(
    ShotCtl* __restrict__ ctl, SiteArgs a, const SiteEvent* __restrict__ ev,
    const DPred* __restrict__ preds, const qsv_cop* __restrict__ code, const double* __restrict__ partials,
    uint32_t pblocks,
    uint64_t* __restrict__ creg,
    uint32_t cw, uint8_t* __restrict__ record, uint32_t max_record, const uint8_t* __restrict__ forced,
    uint32_t forced_len, uint64_t seed, uint64_t shot_base, const uint32_t* __restrict__ slot_of, double readout_err,
    double reset_err, const uint64_t* __restrict__ key) {
  __shared__ double part[4][kSiteBins];
  const uint32_t shot = blockIdx.x, tid = threadIdx.x;
  ShotCtl* c = ctl + shot;
  if (a.nq) {
    const double* pp = partials + (uint64_t)(slot_of ? slot_of[shot] : shot) * pblocks * kSiteBins;
    const uint32_t b = tid & (kSiteBins - 1), q = tid / kSiteBins;
    double acc = 0.0;
    for (uint32_t k = q; k < a.blocks; k += 4) acc += pp[(uint64_t)k * kSiteBins + b];
    part[q][b] = acc;
  }
  __syncthreads();
  if (tid != 0 || c->status != 0) return;
  double bins[kSiteBins];
  for (int b = 0; b < kSiteBins; ++b) bins[b] = a.nq ? ((part[0][b] + part[1][b]) + part[2][b]) + part[3][b] : 0.0;
  finalize_shot(c, bins, a, ev, preds, code, creg, cw, record, max_record, forced, forced_len, seed, shot_base, shot,
                readout_err, reset_err, key);
}

// Both steps of a site whose histogram takes one block (states of up to 14
// qubits) and whose shots own their states: one workgroup per shot builds the
// bins as k_site_reduce does and its first thread runs the events. The bins
// equal those of the two launches (there each is the one block's sum plus
// three zeros).
template <typename CT>
__global__ __launch_bounds__(kRedThreads) void k_site_fused(
    const CT* __restrict__ state, uint64_t stride, ShotCtl* __restrict__ ctl, SiteArgs a,
    const SiteEvent* __restrict__ ev, const DPred* __restrict__ preds, const qsv_cop* __restrict__ code,
    uint64_t* __restrict__ creg, uint32_t cw, uint8_t* __restrict__ record, uint32_t max_record,
    const uint8_t* __restrict__ forced, uint32_t forced_len, uint64_t seed, uint64_t shot_base,
    const uint32_t* __restrict__ buf_of, double readout_err, double reset_err, const uint64_t* __restrict__ key) {
  __shared__ double bins[kSiteBins][kRedThreads];
  __shared__ double red[kRedThreads / kSiteBins][kSiteBins];
  __shared__ double fin[kSiteBins];
  const uint32_t shot = blockIdx.x, tid = threadIdx.x;
  ShotCtl* c = ctl + shot;
  const double v = site_bins(state, stride, c, a, 0u, buf_of ? buf_of[shot] : shot, tid, bins, red);
  if (tid < kSiteBins) fin[tid] = v;
  __syncthreads();
  if (tid != 0 || c->status != 0) return;
  double b16[kSiteBins];
  for (int b = 0; b < kSiteBins; ++b) b16[b] = fin[b];
  finalize_shot(c, b16, a, ev, preds, code, creg, cw, record, max_record, forced, forced_len, seed, shot_base, shot,
                readout_err, reset_err, key);
}

hipError_t launch_site(const RunBuffers& rb, const SiteArgs& a, const SiteEvent* ev, const DPred* preds,
                       const qsv_cop* code, hipStream_t st) {
  if (a.nq && a.blocks == 1 && !rb.slot_of) {
    if (rb.c64)
      hipLaunchKernelGGL(k_site_fused<float2>, dim3(rb.shots), dim3(kRedThreads), 0, st,
                         reinterpret_cast<const float2*>(rb.state), rb.stride, rb.ctl, a, ev, preds, code, rb.creg,
                         rb.cw, rb.record, rb.max_record, rb.forced, rb.forced_len, rb.seed, rb.shot_base, rb.buf_of,
                         rb.readout_err, rb.reset_err, rb.key);
    else
      hipLaunchKernelGGL(k_site_fused<double2>, dim3(rb.shots), dim3(kRedThreads), 0, st, rb.state, rb.stride, rb.ctl,
                         a, ev, preds, code, rb.creg, rb.cw, rb.record, rb.max_record, rb.forced, rb.forced_len,
                         rb.seed, rb.shot_base, rb.buf_of, rb.readout_err, rb.reset_err, rb.key);
    return hipGetLastError();
  }
  if (a.nq) {
    // with trajectory sharing the histograms are taken per slot (slot control
    // blocks in site_ctl), the outcomes per shot
    const dim3 grid(a.blocks, rb.slot_of ? rb.site_slots : rb.shots);
    const ShotCtl* hc = rb.slot_of ? rb.site_ctl : rb.ctl;
    if (rb.c64)
      hipLaunchKernelGGL(k_site_reduce<float2>, grid, dim3(kRedThreads), 0, st,
                         reinterpret_cast<const float2*>(rb.state), rb.stride, hc, a, rb.partials, rb.pblocks,
                         rb.buf_of);
    else
      hipLaunchKernelGGL(k_site_reduce<double2>, grid, dim3(kRedThreads), 0, st, rb.state, rb.stride, hc, a,
                         rb.partials, rb.pblocks, rb.buf_of);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_site_finalize, dim3(rb.shots), dim3(64), 0, st, rb.ctl, a, ev, preds, code, rb.partials,
                     rb.pblocks, rb.creg, rb.cw, rb.record, rb.max_record, rb.forced, rb.forced_len, rb.seed,
                     rb.shot_base, rb.slot_of, rb.readout_err, rb.reset_err, rb.key);
  return hipGetLastError();
}

__global__ void k_ctl_gather(ShotCtl* __restrict__ dst, const ShotCtl* __restrict__ src,
                             const uint32_t* __restrict__ idx, uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[idx[i]];
}

hipError_t launch_ctl_gather(ShotCtl* dst, const ShotCtl* src, const uint32_t* idx, uint32_t count, hipStream_t st) {
  if (!count) return hipSuccess;
  hipLaunchKernelGGL(k_ctl_gather, dim3((count + 255) / 256), dim3(256), 0, st, dst, src, idx, count);
  return hipGetLastError();
}

// Copy-on-write of trajectory slots: buffer pairs[2k] takes the amplitudes of
// buffer pairs[2k + 1]. Sources are never destinations in one launch.
template <typename CT>
__global__ void k_buf_copy(CT* __restrict__ state, uint64_t stride, uint64_t dim,
                           const uint32_t* __restrict__ pairs, uint32_t n_pairs) {
  const uint64_t total = dim * n_pairs;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = i / dim, j = i % dim;
    state[(uint64_t)pairs[2 * k] * stride + j] = state[(uint64_t)pairs[2 * k + 1] * stride + j];
  }
}

hipError_t launch_buf_copy(double2* state, uint64_t stride, uint32_t n, const uint32_t* pairs, uint32_t n_pairs,
                           hipStream_t st, bool c64) {
  if (!n_pairs) return hipSuccess;
  const uint64_t total = (1ull << n) * n_pairs;
  uint64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (c64)
    hipLaunchKernelGGL(k_buf_copy<float2>, dim3((uint32_t)blocks), dim3(256), 0, st, reinterpret_cast<float2*>(state),
                       stride, 1ull << n, pairs, n_pairs);
  else
    hipLaunchKernelGGL(k_buf_copy<double2>, dim3((uint32_t)blocks), dim3(256), 0, st, state, stride, 1ull << n, pairs,
                       n_pairs);
  return hipGetLastError();
}

// Plain streaming copy (calibration of hardware byte counters).
__global__ void k_copy(double2* __restrict__ dst, const double2* __restrict__ src, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

hipError_t launch_copy(void* dst, const void* src, uint64_t bytes, hipStream_t st) {
  const uint64_t n = bytes / 16;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (!blocks) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3((uint32_t)blocks), dim3(256), 0, st, static_cast<double2*>(dst),
                     static_cast<const double2*>(src), n);
  return hipGetLastError();
}

// The logical state of one shot: psi[i] = cond(i) ? mem[i ^ frame] * scale : 0,
// as complex128 whatever the amplitude type.
template <typename CT>
__global__ void k_materialize(const CT* __restrict__ state, uint64_t stride, const ShotCtl* ctl,
                              uint32_t shot, uint64_t dim, double2* __restrict__ out) {
  const ShotCtl c = ctl[shot];
  const CT* st = state + (uint64_t)shot * stride;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
       i += (uint64_t)gridDim.x * blockDim.x) {
    double2 v = make_double2(0.0, 0.0);
    if ((i & c.pend_mask) == c.pend_val) {
      const CT x = st[i ^ c.frame];
      v = cscale(make_double2(x.x, x.y), c.pend_scale);
    }
    out[i] = v;
  }
}

hipError_t launch_materialize(const RunBuffers& rb, uint32_t n, uint32_t shot, double2* out, hipStream_t st) {
  uint64_t dim = 1ull << n;
  uint64_t blocks = (dim + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (rb.c64)
    hipLaunchKernelGGL(k_materialize<float2>, dim3((uint32_t)blocks), dim3(256), 0, st,
                       reinterpret_cast<const float2*>(rb.state), rb.stride, rb.ctl, shot, dim, out);
  else
    hipLaunchKernelGGL(k_materialize<double2>, dim3((uint32_t)blocks), dim3(256), 0, st, rb.state, rb.stride, rb.ctl,
                       shot, dim, out);
  return hipGetLastError();
}


__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Persistent interpreter: one launch runs every shot of every request.
//
// Workgroups pop work items (request, shot) from an atomic counter until the
// queue is empty, so trajectories of uneven length (loop exits, taken
// branches) and circuits of different widths share one launch. A state of
// n <= 12 qubits stays in LDS from the first gate to the last measurement; a
// larger one lives in the workgroup's HBM slot and every pass streams it tile
// by tile. Each item is processed by one workgroup in a fixed order, so its
// results do not depend on what else is in the batch.
// ---------------------------------------------------------------------------
// Deterministic workgroup sum of 16 per-thread bins (wave shuffles, then waves in order).
__device__ void wg_bins(double (&acc)[kSiteBins], double* red /* [4][16] in LDS */, double* out /* [16] */) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
#pragma unroll
  for (int b = 0; b < kSiteBins; ++b) {
    double v = acc[b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave * kSiteBins + b] = v;
  }
  __syncthreads();
  if (tid < (uint32_t)kSiteBins) {
    double v = 0.0;
    for (uint32_t w = 0; w < blockDim.x / 64u; ++w) v += red[w * kSiteBins + tid];
    out[tid] = v;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kTileThreads) void k_persistent(
    const ReqDev* __restrict__ reqs, const uint32_t* __restrict__ item_req, uint32_t n_items,
    uint32_t* __restrict__ queue, double2* __restrict__ scratch, uint64_t slot_amps, ShotCtl* __restrict__ out_ctl,
    uint64_t* __restrict__ out_creg, uint32_t cw, uint8_t* __restrict__ out_rec, uint32_t rec_max) {
  extern __shared__ double2 tile[];
  __shared__ ShotCtl cs;
  // algorithmic HBM bytes of the streamed (HBM-slot) states, summed over the
  // launch for the profile: queue[2..3] as one 64-bit counter
  unsigned long long* const hbm_bytes = reinterpret_cast<unsigned long long*>(queue + 2);
  __shared__ uint32_t item_s;
  __shared__ double red[4 * kSiteBins];
  __shared__ double bins[kSiteBins];
  const uint32_t tid = threadIdx.x;
  double2* const wg_slot = scratch + (uint64_t)blockIdx.x * slot_amps;
  for (;;) {
    if (tid == 0) item_s = atomicAdd(queue, 1u);
    __syncthreads();
    const uint32_t item = item_s;
    if (item >= n_items) break;  // every workgroup reaches this once the queue is drained
    const ReqDev R = reqs[item_req[item]];
    const uint32_t shot = item - R.item_begin, n = R.n;
    const bool resident = n <= (uint32_t)kResidentMaxBits;
    double2* const slot = R.state_out ? reinterpret_cast<double2*>(R.state_out) : wg_slot;
    const double2* const init_state = reinterpret_cast<const double2*>(R.init_state);
    uint64_t* cr = out_creg + (uint64_t)item * cw;
    uint8_t* rec = out_rec + (uint64_t)item * rec_max;
    for (uint32_t w = tid; w < cw; w += blockDim.x) cr[w] = R.init_creg ? R.init_creg[w] : 0ull;
    for (uint32_t w = tid; w < rec_max; w += blockDim.x) rec[w] = 0;
    if (tid == 0) {
      ShotCtl c;
      if (R.init_ctl) {
        c = *R.init_ctl;
      } else {
        c.flags = 0;
        c.pend_mask = 0;
        c.pend_val = 0;
        c.frame = 0;
        c.pend_scale = 1.0;
        c.record_prob = 1.0;
        c.n_events = 0;
        c.n_record = 0;
        c.status = 0;
      }
      c.wg_done = 0;
      cs = c;
    }
    const uint64_t dim = 1ull << n;
    if (init_state) {  // the request's shared prefix, computed once
      if (resident) {
        for (uint32_t l = tid; l < (uint32_t)dim; l += blockDim.x) tile[swz(l)] = init_state[l];
      } else {
        for (uint64_t j = tid; j < dim; j += blockDim.x) slot[j] = init_state[j];
        if (tid == 0) atomicAdd(hbm_bytes, 32ull * dim);
      }
    }
    __syncthreads();
    for (uint32_t k = R.step_begin; k < R.n_steps; ++k) {
      if (cs.status != 0) break;
      const DStep stp = R.steps[k];
      const uint64_t flags = cs.flags;
      if (stp.kind == 0) {  // |0...0>
        if (resident) {
          for (uint32_t l = tid; l < (uint32_t)dim; l += blockDim.x) tile[swz(l)] = make_double2(l == 0 ? 1.0 : 0.0, 0.0);
        } else {
          for (uint64_t j = tid; j < dim; j += blockDim.x) slot[j] = make_double2(j == 0 ? 1.0 : 0.0, 0.0);
          if (tid == 0) atomicAdd(hbm_bytes, 16ull * dim);
        }
        __syncthreads();
      } else if (stp.kind == 1) {  // gate pass
        const PassArgs a = R.passes[stp.index];
        bool any = a.init != 0;
        for (uint32_t i = 0; i < a.gate_count && !any; ++i) any = guard_ok(flags, R.gates[a.gate_begin + i].guard);
        if (!any) continue;
        if (resident) {
          if (a.init) {
            for (uint32_t l = tid; l < (uint32_t)dim; l += blockDim.x) tile[swz(l)] = make_double2(l == 0 ? 1.0 : 0.0, 0.0);
            __syncthreads();
          }
          if (a.phase_count) {
            run_phases<true, true>(tile, (uint32_t)dim, tid, (uint32_t)dim >> kRegBits, flags, R.phases, a.phase_begin,
                       a.phase_count, R.gates, R.mats);
          } else {
            // fewer than 4 qubits: one LDS sweep per gate (slots are unswizzled for T < 16)
            for (uint32_t i = 0; i < a.gate_count; ++i) {
              const DGate g = R.gates[a.gate_begin + i];
              if (!guard_ok(flags, g.guard)) continue;
              tile_apply(tile, a.t, g, R.mats + (uint64_t)g.mat * kMatStride);
              __syncthreads();
            }
          }
        } else {
          // stream the HBM slot tile by tile; the pending collapse and frame
          // apply on staging. The 16 loads per thread of the next tile are
          // issued before the current tile's phases run (tiles of one pass
          // are disjoint), so they overlap its gate arithmetic.
          const uint64_t M = cs.pend_mask, V = cs.pend_val, F = cs.frame;
          const double sc = cs.pend_scale;
          const uint32_t T = 1u << a.t, nthr = T >> kRegBits;
          uint64_t tb = 0;  // this thread's bits over tile qubits tq[0..t-5]
          for (uint32_t b = 0; b + kRegBits < a.t; ++b) tb |= (uint64_t)((tid >> b) & 1u) << a.tq[b];
          const uint64_t h0 = 1ull << a.tq[a.t - 4], h1 = 1ull << a.tq[a.t - 3], h2 = 1ull << a.tq[a.t - 2],
                         h3 = 1ull << a.tq[a.t - 1];
          const uint64_t free_mask = ~a.tile_mask & ((n >= 64) ? ~0ull : ((1ull << n) - 1ull));
          double2 nx[kR];
          if (tid < nthr) fetch16(nx, slot, tile_base(0, free_mask) | tb, h0, h1, h2, h3, a.init != 0, F);
          for (uint32_t w = 0; w < a.tiles; ++w) {
            const uint64_t gthr = tile_base(w, free_mask) | tb;
            if (tid < nthr) stage16(tile, nx, tid, nthr, gthr, h0, h1, h2, h3, M, V, sc);
            __syncthreads();
            if (w + 1 < a.tiles && tid < nthr)
              fetch16(nx, slot, tile_base(w + 1, free_mask) | tb, h0, h1, h2, h3, a.init != 0, F);
            run_phases<true, true>(tile, T, tid, nthr, flags, R.phases, a.phase_begin, a.phase_count, R.gates, R.mats);
            if (tid < nthr) store_tile16(tile, slot, a, tile_base(w, free_mask), tid, F);
            __syncthreads();
          }
          if (tid == 0) {
            cs.pend_mask = 0;
            cs.pend_val = 0;
            cs.pend_scale = 1.0;
            atomicAdd(hbm_bytes, 32ull * dim);
          }
          __syncthreads();
        }
      } else {  // measurement site
        const SiteArgs sa = R.sites[stp.index];
        if (sa.nq) {
          double acc[kSiteBins];
#pragma unroll
          for (int b = 0; b < kSiteBins; ++b) acc[b] = 0.0;
          const uint64_t M = cs.pend_mask, V = cs.pend_val, F = cs.frame;
          const double s2 = cs.pend_scale * cs.pend_scale;
          const uint32_t r = (uint32_t)__popcll(M);
          const uint64_t nfree = 1ull << (n - r);
          for (uint64_t j = tid; j < nfree; j += blockDim.x) {
            uint64_t gi = j;
            if (M) {
              uint64_t mm = M;
              while (mm) {
                const uint32_t b = __ffsll((long long)mm) - 1;
                mm &= mm - 1;
                gi = ins0_64(gi, b);
              }
              gi |= V;
            }
            const double2 v = resident ? tile[swz((uint32_t)(gi ^ F))] : slot[gi ^ F];
            const double p = (v.x * v.x + v.y * v.y) * s2;
            uint32_t bin = 0;
            for (uint32_t q = 0; q < sa.nq; ++q) bin |= (uint32_t)((gi >> sa.q[q]) & 1ull) << q;
#pragma unroll
            for (int b = 0; b < kSiteBins; ++b) acc[b] += (bin == (uint32_t)b) ? p : 0.0;
          }
          wg_bins(acc, red, bins);
          if (!resident && tid == 0) atomicAdd(hbm_bytes, 16ull * nfree);
        }
        if (tid == 0) {
          double hb[kSiteBins];
          for (int b = 0; b < kSiteBins; ++b) hb[b] = sa.nq ? bins[b] : 0.0;
          ShotCtl c = cs;
          site_events(c, hb, sa, R.events, R.preds, R.code, cr, rec, rec_max,
                      R.forced ? R.forced + (uint64_t)shot * R.forced_len : nullptr, R.forced_len, R.seed,
                      R.shot_offset + shot, R.readout_err, R.reset_err);
          cs = c;
        }
        __syncthreads();
        if (resident && (cs.pend_mask != 0 || cs.pend_scale != 1.0 || cs.frame != 0)) {
          // materialise the collapse and the flips in LDS: psi[i] = cond(i) ? mem[i ^ F] * s : 0
          const uint64_t M = cs.pend_mask, V = cs.pend_val, F = cs.frame;
          const double sc = cs.pend_scale;
          for (uint32_t l = tid; l < (uint32_t)dim; l += blockDim.x) {
            const uint32_t m = l ^ (uint32_t)F;
            if (m < l) continue;  // each pair (l, l ^ F) is handled by its smaller index
            const double2 a0 = tile[swz(l)], a1 = tile[swz(m)];
            tile[swz(l)] = ((l & M) == V) ? cscale(a1, sc) : make_double2(0.0, 0.0);
            if (m != l) tile[swz(m)] = ((m & M) == V) ? cscale(a0, sc) : make_double2(0.0, 0.0);
          }
          __syncthreads();
          if (tid == 0) {
            cs.pend_mask = 0;
            cs.pend_val = 0;
            cs.pend_scale = 1.0;
            cs.frame = 0;
          }
          __syncthreads();
        }
      }
    }
    if (R.state_out && resident)
      for (uint32_t l = tid; l < (uint32_t)dim; l += blockDim.x) slot[l] = tile[swz(l)];
    if (tid == 0) out_ctl[item] = cs;
    __syncthreads();
  }
}

hipError_t launch_persistent(const ReqDev* reqs, const uint32_t* item_req, uint32_t n_items, uint32_t* queue,
                             double2* scratch, uint64_t slot_amps, uint32_t workgroups, ShotCtl* out_ctl,
                             uint64_t* out_creg, uint32_t cw, uint8_t* out_rec, uint32_t rec_max, hipStream_t st) {
  if (!n_items) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, queue, 4u);  // queue head and byte counter
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = sizeof(double2) << kResidentMaxBits;
  hipLaunchKernelGGL(k_persistent, dim3(workgroups), dim3(kTileThreads), lds, st, reqs, item_req, n_items, queue,
                     scratch, slot_amps, out_ctl, out_creg, cw, out_rec, rec_max);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed device scratch of the no-allocation entry point
// ---------------------------------------------------------------------------
// Every device the library runs on holds one copy of this array from the
// moment the code object is loaded there until the process ends. In host code
// the array's name is not a device address: each device's copy is reached only
// through the address hipGetSymbolAddress returns with that device current,
// taken once per device by noalloc_scratch_init (called when a context is
// created) and handed to the kernels as an ordinary buffer argument.
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current first
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace qsv
