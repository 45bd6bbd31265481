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
// Value of lane l - 1 within each row of 16 lanes; lane 0 of a row gets its own `first`.
__device__ __forceinline__ float shr1_or(float v, float first) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(first), __float_as_int(v), 0x111, 0xf, 0xf, false));
}
__device__ __forceinline__ double shr1_or(double v, double first) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(__double2loint(first), lo, 0x111, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(__double2hiint(first), hi, 0x111, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sums over the four 16-lane groups (direction slots) of four values at once: lane
// group g receives the sum of its g-th argument over the four groups.  A row swap of two
// different values pairs rows 0,1 and 2,3 of both (no operand copies), a half-wave swap
// then pairs the two halves; each sum is (r0 + r1) + (r2 + r3) over the row groups r.
__device__ __forceinline__ float quad_sum4(float a, float b, float c, float d) {
  auto ab = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  auto cd = __builtin_amdgcn_permlane16_swap(__float_as_uint(c), __float_as_uint(d), false, false);
  const float sab = __uint_as_float(ab[0]) + __uint_as_float(ab[1]);  // rows: a01 b01 a23 b23
  const float scd = __uint_as_float(cd[0]) + __uint_as_float(cd[1]);  // rows: c01 d01 c23 d23
  auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(sab), __float_as_uint(scd), false, false);
  return __uint_as_float(h[0]) + __uint_as_float(h[1]);
}
__device__ __forceinline__ double pair_rows(double a, double b) {
  // rows of the result: a0+a1, b0+b1, a2+a3, b2+b3
  auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false, false);
  auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ double quad_sum4(double a, double b, double c, double d) {
  const double sab = pair_rows(a, b), scd = pair_rows(c, d);
  auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(sab), (unsigned)__double2loint(scd), false, false);
  auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(sab), (unsigned)__double2hiint(scd), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

// Workgroup barrier that orders LDS accesses only: it waits for the wave's own LDS
// operations, not for its global loads in flight (a plain __syncthreads waits for
// those too, which would expose the latency of every prefetch issued before it).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T>
__device__ __forceinline__ T load_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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
