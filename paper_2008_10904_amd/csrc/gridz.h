// Structured-grid stencil application shared by the stepping and adjoint kernels (internal).
#pragma once

#include "common.h"

namespace res {

template <typename R> struct GridCoef {
  const R* cxm; const R* cxp; const R* cym; const R* cyp; const R* czm; const R* czp;
  const R* d;  // [nodes]
  const R* K;  // [lines][3][3] or null
};

// (Z x)_c at node p of column block b; x laid out [block][ncomp][nodes], stored as X and converted to R (the
// coefficient and arithmetic type).
template <typename R, int NC, typename X = R>
__device__ __forceinline__ void apply_z(const GridCoef<R>& Cf, const cx<X>* __restrict__ x, int64_t nodes, int64_t nx,
                                        int64_t ny, int64_t nz, int64_t ix, int64_t iy, int64_t iz, int64_t p, int64_t l,
                                        cx<R> out[NC]) {
  const R cxm = Cf.cxm[l], cxp = Cf.cxp[l], cym = Cf.cym[l], cyp = Cf.cyp[l];
  const R czm = nz > 1 ? Cf.czm[l] : R(0), czp = nz > 1 ? Cf.czp[l] : R(0);
  const R dd = Cf.d[p];
  const int64_t sy = nx, sz = nx * ny;
  cx<R> self[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const cx<X>* xc = x + c * nodes + p;
    cx<R> s = ccast<R>(xc[0]);
    self[c] = s;
    cx<R> acc = mk<R>(dd * s.re, dd * s.im);
    if (ix > 0) { const cx<R> t = ccast<R>(xc[-1]); acc.re += cxm * t.re; acc.im += cxm * t.im; }
    if (ix + 1 < nx) { const cx<R> t = ccast<R>(xc[1]); acc.re += cxp * t.re; acc.im += cxp * t.im; }
    if (iy > 0) { const cx<R> t = ccast<R>(xc[-sy]); acc.re += cym * t.re; acc.im += cym * t.im; }
    if (iy + 1 < ny) { const cx<R> t = ccast<R>(xc[sy]); acc.re += cyp * t.re; acc.im += cyp * t.im; }
    if (iz > 0) { const cx<R> t = ccast<R>(xc[-sz]); acc.re += czm * t.re; acc.im += czm * t.im; }
    if (iz + 1 < nz) { const cx<R> t = ccast<R>(xc[sz]); acc.re += czp * t.re; acc.im += czp * t.im; }
    out[c] = acc;
  }
  if (NC == 3 && Cf.K != nullptr) {
    const R* Kl = Cf.K + l * 9;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int cp = 0; cp < NC; ++cp) {
        const R kk = Kl[c * 3 + cp];
        out[c].re += kk * self[cp].re;
        out[c].im += kk * self[cp].im;
      }
  }
}

}  // namespace res
