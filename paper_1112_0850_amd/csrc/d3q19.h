// d3q19.h -- D3Q19 lattice constants and population storage formats for the
// gfx950 kernels (device side of the library; interface order of lbm.h).
//
// Lattice: 19 velocities in 3-D (Sec. 2; Qian et al. 1992), weights
// 1/3, 1/18, 1/36 by |c|^2 = 0, 1, 2.  Directions 2k-1 and 2k (k = 1..9) are
// opposite pairs, which the collision code exploits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 19;

struct D3Q19 {
  static constexpr int cx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr int opp[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  // weight numerators over 36: 12/36 = 1/3, 2/36 = 1/18, 1/36
  static constexpr int w36[Q] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
};

template <typename C>
__host__ __device__ constexpr C weight(int i) {
  return C(D3Q19::w36[i]) / C(36);
}

// Coefficients of the offset-form equilibrium and Guo term in precision C:
//   g^eq_i = W_i (drho - 3/2 j.u) + c_i (c_i.j)(c_i.u) +- a_i (c_i.j),
//   S_i    = (1 - omega/2) [ q_i (c_i.u)(c_i.F) - 3 W_i u.F +- a_i (c_i.F) ],
// with exact values W = w, c = 9w/2, a = 3w, q = 9w.  c and q are exact
// binary fractions (1/4, 1/8; 1/2, 1/4).  W and a cannot be exact, so they
// are chosen next to w and 3w such that, in exact arithmetic on the rounded
// constants, sum W_i = 1 and 2 a_axis + 8 a_diag = 1: the collision then
// conserves mass and momentum without a systematic bias from the rounding of
// the weights (which would otherwise accumulate coherently over many steps).
template <typename C>
struct Coef;

template <>
struct Coef<float> {
  static constexpr float W0 = 0x1.555558p-2f, W1 = 0x1.c71c7p-5f, W2 = 0x1.c71c7p-6f;
  static constexpr float A1 = 0x1.555554p-3f, A2 = 0x1.555556p-4f;
};

template <>
struct Coef<double> {
  static constexpr double W0 = 0x1.5555555555556p-2, W1 = 0x1.c71c71c71c71cp-5,
                          W2 = 0x1.c71c71c71c71cp-6;
  static constexpr double A1 = 0x1.5555555555554p-3, A2 = 0x1.5555555555556p-4;
};

// Per-direction coefficient by speed class: 0 rest, 1 axis (|c|^2 = 1), 2 diagonal.
__host__ __device__ constexpr int speed_class(int i) { return i == 0 ? 0 : (i <= 6 ? 1 : 2); }

template <typename C>
__host__ __device__ constexpr C coef_W(int i) {
  return speed_class(i) == 0 ? Coef<C>::W0 : (speed_class(i) == 1 ? Coef<C>::W1 : Coef<C>::W2);
}
template <typename C>
__host__ __device__ constexpr C coef_a(int i) {
  return speed_class(i) == 1 ? Coef<C>::A1 : Coef<C>::A2;
}
template <typename C>
__host__ __device__ constexpr C coef_c(int i) {
  return speed_class(i) == 1 ? C(0.25) : C(0.125);
}
template <typename C>
__host__ __device__ constexpr C coef_q(int i) {
  return speed_class(i) == 1 ? C(0.5) : C(0.25);
}

constexpr uint8_t FLAG_SOLID = 1;
constexpr uint8_t FLAG_NOFORCE = 2;
constexpr uint8_t FLAG_MOVING = 4;  // with FLAG_SOLID: a wall cell moving with the wall velocity

// Storage formats of the population offset g = f - w.  `load` widens a stored
// element to the compute type, `store` rounds to nearest-even.  U is the raw
// bit type of a stored element; kRest and kMoving are the two solid-cell
// markers of the format: quiet NaNs with the sign bit set and a fixed
// payload, which neither arithmetic (its NaNs are the default positive NaN
// or a propagated input) nor overflow (infinity) produces.  The kernels
// compare raw bits against them, so a NaN or infinity that arises in a fluid
// cell is not mistaken for a wall and propagates.  kMoving = kRest | 1.
enum StorageKind { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2, ST_F64 = 3, ST_F32X = 4 };

template <int K>
struct Storage;

template <>
struct Storage<ST_F32> {
  using T = float;
  using C = float;
  using U = uint32_t;
  static constexpr U kRest = 0xFFD0D0D0u, kMoving = 0xFFD0D0D1u;
  __device__ static C load(T v, C) { return v; }
  __device__ static T store(C v, C) { return v; }
};

// FP32 storage with FP64 collision arithmetic (opt-in accuracy mode).
template <>
struct Storage<ST_F32X> {
  using T = float;
  using C = double;
  using U = uint32_t;
  static constexpr U kRest = 0xFFD0D0D0u, kMoving = 0xFFD0D0D1u;
  __device__ static C load(T v, C) { return v; }
  __device__ static T store(C v, C) { return T(v); }
};

template <>
struct Storage<ST_F64> {
  using T = double;
  using C = double;
  using U = uint64_t;
  static constexpr U kRest = 0xFFFD0D0D0D0D0D0Cull, kMoving = 0xFFFD0D0D0D0D0D0Dull;
  __device__ static C load(T v, C) { return v; }
  __device__ static T store(C v, C) { return v; }
};

// binary16 holding 2^s g: the exact power-of-two scale keeps small offsets
// out of the subnormal range.  Conversions use the hardware's round-to-
// nearest-even mode.
template <>
struct Storage<ST_F16> {
  using T = _Float16;
  using C = float;
  using U = uint16_t;
  static constexpr U kRest = 0xFED4u, kMoving = 0xFED5u;
  __device__ static C load(T v, C inv_scale) { return float(v) * inv_scale; }
  __device__ static T store(C v, C scale) { return T(v * scale); }
};

// bfloat16: the top 16 bits of the binary32 pattern; the conversion is the
// hardware's round-to-nearest-even.
template <>
struct Storage<ST_BF16> {
  using T = __bf16;
  using C = float;
  using U = uint16_t;
  static constexpr U kRest = 0xFFD4u, kMoving = 0xFFD5u;
  __device__ static C load(T v, C) { return float(v); }
  __device__ static T store(C v, C) { return T(v); }
};

// Raw bits of a stored element and back.
template <int K>
__device__ __forceinline__ typename Storage<K>::U raw_bits(typename Storage<K>::T v) {
  return __builtin_bit_cast(typename Storage<K>::U, v);
}
template <int K>
__device__ __forceinline__ typename Storage<K>::T from_bits(typename Storage<K>::U u) {
  return __builtin_bit_cast(typename Storage<K>::T, u);
}

}  // namespace lbm
