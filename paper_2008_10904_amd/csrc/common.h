// Shared device/host definitions of the resolvent library (internal, not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace res {

// Interleaved complex of real type R; 16-byte (double) or 8-byte (float) aligned so one vector load moves it.
template <typename R> struct alignas(2 * sizeof(R)) cx {
  R re, im;
};

template <typename R> __host__ __device__ __forceinline__ cx<R> mk(R re, R im) {
  cx<R> z;
  z.re = re;
  z.im = im;
  return z;
}
template <typename R> __host__ __device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) {
  return mk<R>(a.re + b.re, a.im + b.im);
}
template <typename R> __host__ __device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return mk<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// a * b + c
template <typename R> __host__ __device__ __forceinline__ cx<R> cfma(cx<R> a, cx<R> b, cx<R> c) {
  c.re = fma(a.re, b.re, c.re);
  c.re = fma(-a.im, b.im, c.re);
  c.im = fma(a.re, b.im, c.im);
  c.im = fma(a.im, b.re, c.im);
  return c;
}
// conj(a) * b + c
template <typename R> __host__ __device__ __forceinline__ cx<R> cfma_conj(cx<R> a, cx<R> b, cx<R> c) {
  c.re = fma(a.re, b.re, c.re);
  c.re = fma(a.im, b.im, c.re);
  c.im = fma(a.re, b.im, c.im);
  c.im = fma(-a.im, b.re, c.im);
  return c;
}
template <typename R> __host__ __device__ __forceinline__ cx<R> cconj(cx<R> a) { return mk<R>(a.re, -a.im); }

// Component-wise select (a ternary on the whole struct can be lowered through a stack slot).
template <typename R> __host__ __device__ __forceinline__ cx<R> csel(bool c, cx<R> a, cx<R> b) {
  return mk<R>(c ? a.re : b.re, c ? a.im : b.im);
}

template <typename To, typename From> __host__ __device__ __forceinline__ cx<To> ccast(cx<From> a) {
  return mk<To>((To)a.re, (To)a.im);
}

// Streaming (non-temporal) load of one complex value: used for data read once per step (forcing rows).
template <typename R> __device__ __forceinline__ cx<R> load_nt(const cx<R>* p);
template <> __device__ __forceinline__ cx<double> load_nt<double>(const cx<double>* p) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 t = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return mk<double>(t.x, t.y);
}
template <> __device__ __forceinline__ cx<float> load_nt<float>(const cx<float>* p) {
  typedef float v2 __attribute__((ext_vector_type(2)));
  const v2 t = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return mk<float>(t.x, t.y);
}

// s_waitcnt immediate (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8) that waits for
// every outstanding vector-memory operation and leaves the other counters alone.
constexpr int kWaitVmcnt0 = 0x0F70;

// Workgroup barrier that orders LDS only: unlike __syncthreads() it does not wait for outstanding global
// loads, so loads issued ahead of time (prefetched forcing rows) stay in flight across the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Work of one workgroup of the 1-D stepper: column `col`, a region [dof0, dof0 + ndof) of that column that it
// marches, and inside it the owned unknowns [dof0 + own0, dof0 + own0 + nown) whose values it publishes.  Outside
// an instance the step stencil has no couplings, so regions may span instances; when the region is cut inside
// an instance, the cut must lie at least 4 unknowns per step away from the owned range (the step stencil has
// radius 4), so that the owned values are exact after the launch's steps.
struct Seg1D {
  int32_t col;
  int32_t own0;
  int64_t dof0;
  int32_t ndof;
  int32_t nown;
  int32_t left, right;  // workgroups owning the halo on either side (-1: none); used by the persistent stepper
};

// Radius of the one-step propagator stencil of a three-point operator: P(Z) = sum_{m<=4} Z^m/m! couples
// unknowns up to four apart.
constexpr int kBandRadius = 4;
constexpr int kBandWidth = 2 * kBandRadius + 1;

}  // namespace res
