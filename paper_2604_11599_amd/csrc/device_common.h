// Device helpers shared by the gate-pass kernels and the adjoint kernels:
// complex arithmetic, 2x2 gate matrices, constant-address-space reads, register
// phases (gate application on 16 amplitudes held by one thread), the operand
// order of the matrix cores, and index scatter.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qsv_types.h"

namespace qsv {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// u * a + v * b
__device__ __forceinline__ double2 cmac2(double2 u, double2 a, double2 v, double2 b) {
  double re = u.x * a.x - u.y * a.y + v.x * b.x - v.y * b.y;
  double im = u.x * a.y + u.y * a.x + v.x * b.y + v.y * b.x;
  return make_double2(re, im);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
// complex64 amplitudes: the same operations in single precision
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, double s) {
  const float f = (float)s;
  return make_float2(a.x * f, a.y * f);
}
__device__ __forceinline__ float2 cmac2(float2 u, float2 a, float2 v, float2 b) {
  float re = u.x * a.x - u.y * a.y + v.x * b.x - v.y * b.y;
  float im = u.x * a.y + u.y * a.x + v.x * b.y + v.y * b.x;
  return make_float2(re, im);
}

// Amplitude types of the state: complex128 (double2) or complex64 (float2).
// Gate matrices are always bound in double precision and rounded to the
// amplitude type where they are applied.
template <typename CT> struct CxT;
template <> struct CxT<double2> {
  typedef double R;
  __device__ static double2 make(double re, double im) { return make_double2(re, im); }
};
template <> struct CxT<float2> {
  typedef float R;
  __device__ static float2 make(double re, double im) { return make_float2((float)re, (float)im); }
};
template <typename CT>
__device__ __forceinline__ CT cmake(double re, double im) {
  return CxT<CT>::make(re, im);
}

__device__ __forceinline__ uint32_t ins0(uint32_t x, uint32_t b) {
  return ((x >> b) << (b + 1)) | (x & ((1u << b) - 1u));
}
__device__ __forceinline__ uint64_t ins0_64(uint64_t x, uint32_t b) {
  return ((x >> b) << (b + 1)) | (x & ((1ull << b) - 1ull));
}

// 2x2 matrix of a slot, conjugated by X when the frame flips its qubit.
template <typename CT>
struct M2x {
  CT a, b, c, d;
};
typedef M2x<double2> M2;
template <typename CT>
__device__ __forceinline__ M2x<CT> load_m2x(const double* m, uint32_t flip) {
  M2x<CT> r;
  r.a = cmake<CT>(m[0], m[1]);
  r.b = cmake<CT>(m[2], m[3]);
  r.c = cmake<CT>(m[4], m[5]);
  r.d = cmake<CT>(m[6], m[7]);
  if (flip) {
    CT t = r.a;
    r.a = r.d;
    r.d = t;
    t = r.b;
    r.b = r.c;
    r.c = t;
  }
  return r;
}
__device__ __forceinline__ M2 load_m2(const double* m, uint32_t flip) { return load_m2x<double2>(m, flip); }

__device__ __forceinline__ bool guard_ok(uint64_t flags, uint64_t guard) { return (flags & guard) == guard; }

// Reads through the constant address space: wave-uniform values that the
// kernel reading them does not write become scalar loads, which keep the
// vector-memory counter free for the loads that overlap the arithmetic.
#define QSV_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const QSV_CONST T* cst(const T* p) {
  return (const QSV_CONST T*)p;
}

__device__ __forceinline__ Phase load_phase(const Phase* p) {
  static_assert(sizeof(Phase) == 16, "Phase is two 8-byte words");
  const QSV_CONST uint64_t* w = (const QSV_CONST uint64_t*)p;
  const uint64_t w0 = w[0], w1 = w[1];
  Phase ph;
  __builtin_memcpy(&ph, &w0, 8);
  __builtin_memcpy(reinterpret_cast<char*>(&ph) + 8, &w1, 8);
  return ph;
}

// Global index of tile-local element l.
__device__ __forceinline__ uint64_t local_to_global(uint32_t l, const PassArgs& a) {
  uint64_t g = 0;
  for (uint32_t k = 0; k < a.t; ++k) g |= (uint64_t)((l >> k) & 1u) << a.tq[k];
  return g;
}

// ---------------------------------------------------------------------------
// Register phases: a thread holds the 16 amplitudes of a tile that differ only
// in the phase's 4 register bits (element k: bit j of k is register bit j).
// LDS slots are XOR-swizzled (bits 4..11 folded onto bits 0..3) so that the
// lanes of a wave spread over the banks for any choice of register bits.
// ---------------------------------------------------------------------------
constexpr int kR = 1 << kRegBits;

__device__ __forceinline__ uint32_t swz(uint32_t l) { return l ^ ((l >> 4) & 15u) ^ ((l >> 8) & 15u); }

template <int J, typename CT>
__device__ __forceinline__ void r_dense(CT (&a)[kR], const M2x<CT>& u) {
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    if (k & (1 << J)) continue;
    const int k1 = k | (1 << J);
    const CT x0 = a[k], x1 = a[k1];
    a[k] = cmac2(u.a, x0, u.b, x1);
    a[k1] = cmac2(u.c, x0, u.d, x1);
  }
}

template <int J, typename CT>
__device__ __forceinline__ void r_diag(CT (&a)[kR], const M2x<CT>& u) {
#pragma unroll
  for (int k = 0; k < kR; ++k) a[k] = cmul((k & (1 << J)) ? u.d : u.a, a[k]);
}

template <int J, typename CT>
__device__ __forceinline__ void r_x(CT (&a)[kR]) {
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    if (k & (1 << J)) continue;
    const CT x = a[k];
    a[k] = a[k | (1 << J)];
    a[k | (1 << J)] = x;
  }
}

// memory value CV of the control bit C selects the pairs along T
template <int C, int T, int CV, typename CT>
__device__ __forceinline__ void r_cx(CT (&a)[kR]) {
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    if (((k >> C) & 1) != CV || (k & (1 << T))) continue;
    const CT x = a[k];
    a[k] = a[k | (1 << T)];
    a[k | (1 << T)] = x;
  }
}

template <int C, int T, int CV, typename CT>
__device__ __forceinline__ void r_ctrl(CT (&a)[kR], const M2x<CT>& u) {
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    if (((k >> C) & 1) != CV || (k & (1 << T))) continue;
    const int k1 = k | (1 << T);
    const CT x0 = a[k], x1 = a[k1];
    a[k] = cmac2(u.a, x0, u.b, x1);
    a[k1] = cmac2(u.c, x0, u.d, x1);
  }
}

template <int C, int T, int SC, int ST, typename CT>
__device__ __forceinline__ void r_cphase(CT (&a)[kR], CT ph) {
#pragma unroll
  for (int k = 0; k < kR; ++k)
    if (((k >> C) & 1) == SC && ((k >> T) & 1) == ST) a[k] = cmul(ph, a[k]);
}

// SWAP in the flip frame: exchange 01<->10, or 00<->11 when one operand is flipped
template <int A, int B, int ANTI, typename CT>
__device__ __forceinline__ void r_swap(CT (&a)[kR]) {
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    if (ANTI) {
      if ((k & (1 << A)) || (k & (1 << B))) continue;
      const int k2 = k | (1 << A) | (1 << B);
      const CT x = a[k];
      a[k] = a[k2];
      a[k2] = x;
    } else {
      if (!(k & (1 << A)) || (k & (1 << B))) continue;
      const int k2 = (k ^ (1 << A)) | (1 << B);
      const CT x = a[k];
      a[k] = a[k2];
      a[k2] = x;
    }
  }
}

template <int C, int T, typename CT>
__device__ __forceinline__ void r_two(CT (&a)[kR], uint8_t type, const double* m) {
  switch (type) {
    case GT_CX: r_cx<C, T, 1>(a); break;
    case GT_CTRL1: r_ctrl<C, T, 1>(a, load_m2x<CT>(m, 0)); break;
    case GT_CPHASE: r_cphase<C, T, 1, 1>(a, cmake<CT>(m[6], m[7])); break;
    default: r_swap<C, T, 0>(a); break;
  }
}

template <int J, typename CT>
__device__ __forceinline__ void r_one(CT (&a)[kR], uint8_t type, const double* m) {
  if (type == GT_X1) {
    r_x<J>(a);
    return;
  }
  const M2x<CT> u = load_m2x<CT>(m, 0);
  if (type == GT_DIAG1) r_diag<J>(a, u);
  else r_dense<J>(a, u);
}

template <typename CT>
__device__ __forceinline__ void r_apply(CT (&a)[kR], uint8_t type, int j0, int j1, const double* m) {
  if (type <= GT_X1) {
    switch (j0) {
      case 0: r_one<0>(a, type, m); break;
      case 1: r_one<1>(a, type, m); break;
      case 2: r_one<2>(a, type, m); break;
      default: r_one<3>(a, type, m); break;
    }
    return;
  }
#define QSV_R2(C, T) \
  case (C * 4 + T): r_two<C, T>(a, type, m); break;
  switch (j0 * 4 + j1) {
    QSV_R2(0, 1) QSV_R2(0, 2) QSV_R2(0, 3)
    QSV_R2(1, 0) QSV_R2(1, 2) QSV_R2(1, 3)
    QSV_R2(2, 0) QSV_R2(2, 1) QSV_R2(2, 3)
    QSV_R2(3, 0) QSV_R2(3, 1) QSV_R2(3, 2)
    default: break;
  }
#undef QSV_R2
}
// position of element (row i, column c) of a 16x16 complex matrix in matrix-core
// operand order: lane l of a wave reads M[l % 16][4 kb + l / 16] at kb * 64 + l
__device__ __forceinline__ uint32_t dense_pos(uint32_t i, uint32_t c) { return (c >> 2) * 64u + i + 16u * (c & 3u); }

// scatter the low bits of x over the set bits of mask (ascending)
__device__ __forceinline__ uint32_t pdep32(uint32_t x, uint32_t mask) {
  uint32_t r = 0;
  while (mask) {
    const uint32_t b = mask & (0u - mask);
    if (x & 1u) r |= b;
    x >>= 1;
    mask ^= b;
  }
  return r;
}

typedef double qsv_d4 __attribute__((ext_vector_type(4)));
typedef float qsv_f4 __attribute__((ext_vector_type(4)));

// global index bits of tile w: the bits of w scattered over the non-tile qubits
__device__ __forceinline__ uint64_t tile_base(uint64_t w, uint64_t free_mask) {
  uint64_t base = 0, m = free_mask;
  while (m) {
    const uint64_t bit = m & (0ull - m);
    if (w & 1ull) base |= bit;
    w >>= 1;
    m ^= bit;
  }
  return base;
}

// LDS slots: the slot of tile-local index l is swz(l); swz and the scatter of
// bits over a mask are both linear over GF(2) (swz(a ^ b) = swz(a) ^ swz(b)),
// so every slot a lane touches in a phase is a per-lane part, formed once per
// phase, XOR a wave-uniform part (scalar registers).

// the set bits of a wave-uniform mask, lowest first, one bit each (0 past the last)
struct UBits {
  uint32_t b[8];
};
__device__ __forceinline__ UBits ubits(uint32_t m) {
  UBits u;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    u.b[k] = m & (0u - m);
    m &= m - 1u;
  }
  return u;
}

// bits 0..kBits-1 of x scattered over the first kBits set bits of the mask
template <int kBits>
__device__ __forceinline__ uint32_t udep(const UBits& u, uint32_t x) {
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < kBits; ++k) r |= ((x >> k) & 1u) ? u.b[k] : 0u;
  return r;
}

}  // namespace qsv
