// Device helpers shared by the 2D and 3D sweep kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

namespace lmdg {
namespace {

// Value of lane l - 1 within each row of 16 lanes (lane 0 of a row gets 0).
__device__ __forceinline__ float shr1(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, false));
}
__device__ __forceinline__ double shr1(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x111, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x111, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum of the four lanes r, r+16, r+32, r+48 (same row, four direction slots),
// returned to all four; the pairing order is fixed, so results are reproducible.
__device__ __forceinline__ float quad_sum(float v) {
  unsigned u = __float_as_uint(v);
  auto a = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  float s = __uint_as_float(a[0]) + __uint_as_float(a[1]);
  unsigned us = __float_as_uint(s);
  auto b = __builtin_amdgcn_permlane32_swap(us, us, false, false);
  return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}
__device__ __forceinline__ double quad_sum(double v) {
  unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  auto al = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  auto ah = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  double s = __hiloint2double((int)ah[0], (int)al[0]) + __hiloint2double((int)ah[1], (int)al[1]);
  lo = (unsigned)__double2loint(s);
  hi = (unsigned)__double2hiint(s);
  auto bl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  auto bh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double((int)bh[0], (int)bl[0]) + __hiloint2double((int)bh[1], (int)bl[1]);
}

template <typename T>
__device__ __forceinline__ T load_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr long long kSpinLimit = 1ll << 25;

// Immediate of s_waitcnt vmcnt(0) in the gfx9 encoding (expcnt and lgkmcnt at their
// maxima, so they are not waited for): the wave's vector memory operations have
// completed.  Agent-scope atomic stores are written through to the agent's coherence
// point, so after this wait they are visible to every workgroup.
constexpr int kWaitVmem = 0x0F70;
// Reciprocal from a hardware estimate refined by Newton steps r <- r + r (1 - d r);
// the denominators of the low-memory sweeps do not depend on the upwind values, so
// this runs off the step's dependency chain.  FP64: the single-precision estimate
// (about 23 correct bits) doubles its correct bits with each of two FP64 steps.
__device__ __forceinline__ double recip(double d) {
  double r = (double)__builtin_amdgcn_rcpf((float)d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float recip(float d) {
  float r = __builtin_amdgcn_rcpf(d);
  const float e = fmaf(-d, r, 1.0f);
  return fmaf(r, e, r);
}

}  // namespace
}  // namespace lmdg
