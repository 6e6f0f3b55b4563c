// Storage precision of the populations. The arithmetic type R is double for FP64 storage and
// float otherwise. The *_DEV storages hold each population as its deviation from the lattice
// weight (scaled by 2^k for FP16 so that deviations of order 1e-6 stay out of the subnormal
// range); a uniform fluid at rest therefore stores exact zeros.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

namespace lbm {

template <int P>
struct Prec;

template <>
struct Prec<0> {
  using S = double;
  using R = double;
  __device__ static inline R ld(S s, R, R) { return s; }
  __device__ static inline S st(R v, R, R) { return v; }
};

template <>
struct Prec<1> {
  using S = float;
  using R = float;
  __device__ static inline R ld(S s, R, R) { return s; }
  __device__ static inline S st(R v, R, R) { return v; }
};

template <>
struct Prec<2> {
  using S = __half;
  using R = float;
  __device__ static inline R ld(S s, R w, R inv_scale) { return w + __half2float(s) * inv_scale; }
  __device__ static inline S st(R v, R w, R scale) { return __float2half_rn((v - w) * scale); }
};

template <>
struct Prec<3> {
  using S = __hip_bfloat16;
  using R = float;
  __device__ static inline R ld(S s, R w, R inv_scale) { return w + __bfloat162float(s) * inv_scale; }
  __device__ static inline S st(R v, R w, R scale) { return __float2bfloat16((v - w) * scale); }
};

}  // namespace lbm
