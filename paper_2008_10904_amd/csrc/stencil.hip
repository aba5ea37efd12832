// 2-D and 3-D structured-grid operators: five-point (one complex unknown per node) and seven-point with three
// coupled components per node, real coefficients.
//
//   (Z q)_c(x,y,z) = cxm[l] q_c(x-1) + cxp[l] q_c(x+1) + cym[l] q_c(y-1) + cyp[l] q_c(y+1)
//                  + czm[l] q_c(z-1) + czp[l] q_c(z+1) + d[node] q_c + sum_c' K[l][c][c'] q_c'
//
// with l = z*ny + y the x-line index and every coefficient already multiplied by h (Z = h L).  Homogeneous
// Dirichlet values outside the grid.  The RK4 step of du/dt = L u + f is marched in the nested (Horner) form
//
//   v <- u + Z u / 4,  v <- u + Z v / 3,  v <- u + Z v / 2,  u <- u + Z v + sum_j G_j e^{i w_j t_s}
//
// which equals P(Z) u_s + forcing of the classical four-stage scheme (the forcing enters through
// G_j = h Q_j(Z) F_j, built by three Horner passes of the same stencil; see step1d.hip).  One launch per stage:
// a thread owns one node and all k columns and components there, so the line coefficients are loaded once and
// reused; x is the fastest index across threads (coalesced rows), y/z neighbours come through the caches.
#include "common.h"
#include "kernels.h"
#include "gridz.h"

namespace res {

// One Horner stage for all k columns:  out = u + s * Z vin   (stage 4,3,2: s = 1/4, 1/3, 1/2)
// or, last stage (s = 1):  u = u + Z vin + phi * frc   (in place; frc may be null), and before that, if snap is
// given, the snapshot row receives u (the state before this step's update).
template <typename R, int NC, bool LAST>
__global__ __launch_bounds__(256) void grid_stage_kernel(GridCoef<R> Cf, int64_t nx, int64_t ny, int64_t nz, int k,
                                                         cx<R>* u, const cx<R>* __restrict__ vin, cx<R>* vout,
                                                         R s, const cx<R>* __restrict__ frc, R phr, R phi,
                                                         cx<R>* __restrict__ snap) {
  const int64_t nodes = nx * ny * nz;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= nodes) return;
  const int64_t ix = p % nx;
  const int64_t l = p / nx;
  const int64_t iy = l % ny, iz = l / ny;
  const int64_t blk = (int64_t)NC * nodes;
  for (int b = 0; b < k; ++b) {
    cx<R> zv[NC];
    apply_z<R, NC>(Cf, vin + b * blk, nodes, nx, ny, nz, ix, iy, iz, p, l, zv);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int64_t e = b * blk + c * nodes + p;
      const cx<R> uu = u[e];
      if (LAST) {
        if (snap != nullptr) snap[e] = uu;
        cx<R> r = mk<R>(uu.re + zv[c].re, uu.im + zv[c].im);
        if (frc != nullptr) {
          const cx<R> f = frc[e];
          r.re += phr * f.re - phi * f.im;
          r.im += phr * f.im + phi * f.re;
        }
        u[e] = r;
      } else {
        vout[e] = mk<R>(uu.re + s * zv[c].re, uu.im + s * zv[c].im);
      }
    }
  }
}

// Whole RK4 step of the 2-D five-point operator in one launch (temporal blocking).  A workgroup of 4 x 64
// threads owns a 56 x 32 tile of one column and works on the 64 x 40 window around it (halo 4 = the radius of
// P(Z)).  Lane l of strip w holds window column l, rows 10w .. 10w+9, in registers (the state u, the diagonal,
// the current stage values); each stage publishes the stage input to one of two LDS windows, so x-neighbours
// and the strip-end y-neighbours come from LDS and the other y-neighbours from the thread's own registers.  The
// valid region shrinks by one node per stage; values outside the grid are zero (homogeneous Dirichlet).  The
// new state goes to uout (a different buffer: neighbouring tiles read this step's u as their halo).  HBM
// traffic per step: the state once (plus halo rows, mostly from L2), the forcing row once, the new state once.
template <typename R>
__global__ __launch_bounds__(256) void grid_step2d_kernel(GridCoef<R> Cf, int64_t nx, int64_t ny,
                                                          const cx<R>* __restrict__ uin, cx<R>* __restrict__ uout,
                                                          const cx<R>* __restrict__ frc, R phr, R phi,
                                                          cx<R>* __restrict__ snap) {
  constexpr int H = 4, WX = 64, WY = 40, TX = WX - 2 * H, TY = WY - 2 * H, RS = WY / 4;
  __shared__ cx<R> Lw[2][WY][WX];
  __shared__ R cxm[WY], cxp[WY], cym[WY], cyp[WY];
  const int tid = threadIdx.x;
  const int lx = tid & 63, ly0 = (tid >> 6) * RS;
  const int64_t x0 = (int64_t)blockIdx.x * TX - H, y0 = (int64_t)blockIdx.y * TY - H;
  const int64_t cb = (int64_t)blockIdx.z * nx * ny;  // column offset
  const int64_t ix = x0 + lx;
  const bool xin = ix >= 0 && ix < nx;
  if (tid < WY) {
    const int64_t iy = y0 + tid;
    const bool in = iy >= 0 && iy < ny;
    cxm[tid] = in ? Cf.cxm[iy] : R(0);
    cxp[tid] = in ? Cf.cxp[iy] : R(0);
    cym[tid] = in ? Cf.cym[iy] : R(0);
    cyp[tid] = in ? Cf.cyp[iy] : R(0);
  }
  cx<R> u[RS], x[RS];
  R d[RS];
  bool in[RS];
#pragma unroll
  for (int r = 0; r < RS; ++r) {
    const int64_t iy = y0 + ly0 + r;
    in[r] = xin && iy >= 0 && iy < ny;
    const int64_t p = iy * nx + ix;
    u[r] = in[r] ? uin[cb + p] : mk<R>(R(0), R(0));
    d[r] = in[r] ? Cf.d[p] : R(0);
    x[r] = u[r];
  }
  // stage m = 1..4: y = u + s (Z x) on the valid region (m <= lx < WX - m, m <= ly < WY - m), zero elsewhere;
  // the last stage has s = 1 and adds the forcing.  Operation order as apply_z: diagonal, -x, +x, -y, +y.
#pragma unroll
  for (int m = 1; m <= 4; ++m) {
    cx<R>(*Lm)[WX] = Lw[m & 1];
#pragma unroll
    for (int r = 0; r < RS; ++r) Lm[ly0 + r][lx] = x[r];
    __syncthreads();
    const R s = m == 1 ? R(0.25) : m == 2 ? R(1) / R(3) : m == 3 ? R(0.5) : R(1);
    const bool xok = lx >= m && lx < WX - m;
    cx<R> y[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int ly = ly0 + r;
      y[r] = mk<R>(R(0), R(0));
      if (!(xok && ly >= m && ly < WY - m && in[r])) continue;
      const cx<R> lf = Lm[ly][lx - 1], rt = Lm[ly][lx + 1];
      const cx<R> dn = r > 0 ? x[r - 1] : Lm[ly - 1][lx];
      const cx<R> up = r < RS - 1 ? x[r + 1] : Lm[ly + 1][lx];
      cx<R> z = mk<R>(d[r] * x[r].re, d[r] * x[r].im);
      z.re += cxm[ly] * lf.re; z.im += cxm[ly] * lf.im;
      z.re += cxp[ly] * rt.re; z.im += cxp[ly] * rt.im;
      z.re += cym[ly] * dn.re; z.im += cym[ly] * dn.im;
      z.re += cyp[ly] * up.re; z.im += cyp[ly] * up.im;
      y[r] = mk<R>(u[r].re + s * z.re, u[r].im + s * z.im);
    }
#pragma unroll
    for (int r = 0; r < RS; ++r) x[r] = y[r];
  }
  // interior of the tile: forcing, snapshot of u (the state before the step) and the new state
  if (lx < H || lx >= WX - H) return;
#pragma unroll
  for (int r = 0; r < RS; ++r) {
    const int ly = ly0 + r;
    if (ly < H || ly >= WY - H || !in[r]) continue;
    const int64_t e = cb + (y0 + ly) * nx + ix;
    if (snap != nullptr) snap[e] = u[r];
    cx<R> v = x[r];
    if (frc != nullptr) {
      const cx<R> f = frc[e];
      v.re += phr * f.re - phi * f.im;
      v.im += phr * f.im + phi * f.re;
    }
    uout[e] = v;
  }
}

// One Horner pass of G = h Q_j(Z) F over [n_w][k] blocks (see tri_horner_kernel for the coefficients).
template <typename TF, typename TO, int NC>
__global__ __launch_bounds__(256) void grid_horner_kernel(GridCoef<double> Cf, int64_t nx, int64_t ny, int64_t nz,
                                                          const cx<double>* __restrict__ yin,
                                                          const cx<TF>* __restrict__ F, cx<TO>* __restrict__ yout,
                                                          int k, int nw, double sw0h, double sdwh, double h, int pass) {
  const int64_t nodes = nx * ny * nz;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= nodes) return;
  const int64_t ix = p % nx;
  const int64_t l = p / nx;
  const int64_t iy = l % ny, iz = l / ny;
  const int64_t blk = (int64_t)NC * nodes;
  const int b = blockIdx.y;  // block = j * k + column
  const int j = b / k;
  double sa, ca;
  sincos(0.5 * (sw0h + (double)j * sdwh), &sa, &ca);
  const cx<double> a = mk<double>(ca, sa);
  const cx<double> bb = cmul(a, a);
  cx<double> zx[NC];
  if (pass == 0) {
    // Z applied to F (converted on the fly)
    cx<double> xs[NC];
    (void)xs;
    const cx<TF>* Fb = F + (int64_t)b * blk;
    const double cxm = Cf.cxm[l], cxp = Cf.cxp[l], cym = Cf.cym[l], cyp = Cf.cyp[l];
    const double czm = nz > 1 ? Cf.czm[l] : 0.0, czp = nz > 1 ? Cf.czp[l] : 0.0, dd = Cf.d[p];
    const int64_t sy = nx, sz = nx * ny;
    cx<double> self[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const cx<TF>* xc = Fb + c * nodes + p;
      const cx<double> sv = ccast<double>(xc[0]);
      self[c] = sv;
      cx<double> acc = mk<double>(dd * sv.re, dd * sv.im);
      auto add = [&](double coef, cx<TF> t) { acc.re += coef * (double)t.re; acc.im += coef * (double)t.im; };
      if (ix > 0) add(cxm, xc[-1]);
      if (ix + 1 < nx) add(cxp, xc[1]);
      if (iy > 0) add(cym, xc[-sy]);
      if (iy + 1 < ny) add(cyp, xc[sy]);
      if (iz > 0) add(czm, xc[-sz]);
      if (iz + 1 < nz) add(czp, xc[sz]);
      zx[c] = acc;
    }
    if (NC == 3 && Cf.K != nullptr) {
      const double* Kl = Cf.K + l * 9;
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int cp = 0; cp < NC; ++cp) {
          zx[c].re += Kl[c * 3 + cp] * self[cp].re;
          zx[c].im += Kl[c * 3 + cp] * self[cp].im;
        }
    }
  } else {
    apply_z<double, NC>(Cf, yin + (int64_t)b * blk, nodes, nx, ny, nz, ix, iy, iz, p, l, zx);
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int64_t e = (int64_t)b * blk + c * nodes + p;
    const cx<double> fz = ccast<double>(F[e]);
    cx<double> y;
    if (pass == 0) {
      const cx<double> c2 = mk<double>((1.0 + a.re) / 12.0, a.im / 12.0);
      y = cfma(c2, fz, mk<double>(zx[c].re / 24.0, zx[c].im / 24.0));
    } else if (pass == 1) {
      const cx<double> c1 = mk<double>((1.0 + 2.0 * a.re) / 6.0, 2.0 * a.im / 6.0);
      y = cfma(c1, fz, zx[c]);
    } else {
      const cx<double> c0 = mk<double>((1.0 + 4.0 * a.re + bb.re) / 6.0, (4.0 * a.im + bb.im) / 6.0);
      y = cfma(c0, fz, zx[c]);
      y = mk<double>(h * y.re, h * y.im);
    }
    yout[e] = ccast<TO>(y);
  }
}

// ---------------------------------------------------------------------------------------------------------
template <typename R> static GridCoef<R> coef_of(const GridOpDev& g, int fp64) {
  (void)fp64;
  GridCoef<R> c;
  c.cxm = (const R*)g.cxm; c.cxp = (const R*)g.cxp; c.cym = (const R*)g.cym; c.cyp = (const R*)g.cyp;
  c.czm = (const R*)g.czm; c.czp = (const R*)g.czp; c.d = (const R*)g.d; c.K = (const R*)g.K;
  return c;
}

int launch_grid_stage(const GridOpDev& g, int fp64, int k, void* u, const void* vin, void* vout, double s, int last,
                      const void* frc, double phr, double phi, void* snap, hipStream_t st) {
  const int64_t nodes = g.nx * g.ny * g.nz;
  const dim3 grid((unsigned)((nodes + 255) / 256));
#define RES_GS(R, NC, L)                                                                                          \
  hipLaunchKernelGGL((grid_stage_kernel<R, NC, L>), grid, dim3(256), 0, st, coef_of<R>(g, fp64), g.nx, g.ny, g.nz, \
                     k, (cx<R>*)u, (const cx<R>*)vin, (cx<R>*)vout, (R)s, (const cx<R>*)frc, (R)phr, (R)phi,      \
                     (cx<R>*)snap)
#define RES_GS2(R, NC) \
  if (last) RES_GS(R, NC, true); else RES_GS(R, NC, false)
  if (fp64) {
    if (g.ncomp == 3) { RES_GS2(double, 3); } else { RES_GS2(double, 1); }
  } else {
    if (g.ncomp == 3) { RES_GS2(float, 3); } else { RES_GS2(float, 1); }
  }
#undef RES_GS2
#undef RES_GS
  return 0;
}

int launch_grid_step2d(const GridOpDev& g, int fp64, int k, const void* uin, void* uout, const void* frc, double phr,
                       double phi, void* snap, hipStream_t st) {
  constexpr int TX = 56, TY = 32;  // interior of the 64 x 40 window
  if (g.ncomp != 1 || g.nz != 1 || k < 1 || k > 65535) return -1;
  const dim3 grid((unsigned)((g.nx + TX - 1) / TX), (unsigned)((g.ny + TY - 1) / TY), (unsigned)k);
  if (fp64)
    hipLaunchKernelGGL((grid_step2d_kernel<double>), grid, dim3(256), 0, st, coef_of<double>(g, 1), g.nx,
                       g.ny, (const cx<double>*)uin, (cx<double>*)uout, (const cx<double>*)frc, phr, phi,
                       (cx<double>*)snap);
  else
    hipLaunchKernelGGL((grid_step2d_kernel<float>), grid, dim3(256), 0, st, coef_of<float>(g, 0), g.nx,
                       g.ny, (const cx<float>*)uin, (cx<float>*)uout, (const cx<float>*)frc, (float)phr, (float)phi,
                       (cx<float>*)snap);
  return 0;
}

int launch_grid_horner(const GridOpDev& g64, const cx<double>* yin, const void* F, int f_fp64, void* yout,
                       int out_fp64, int k, int nw, double sw0h, double sdwh, double h, int pass, hipStream_t st) {
  const int64_t nodes = g64.nx * g64.ny * g64.nz;
  if ((int64_t)nw * k > 65535) return -1;
  const dim3 grid((unsigned)((nodes + 255) / 256), (unsigned)(nw * k));
  GridCoef<double> c = coef_of<double>(g64, 1);
#define RES_GH(TF, TO, NC)                                                                                        \
  hipLaunchKernelGGL((grid_horner_kernel<TF, TO, NC>), grid, dim3(256), 0, st, c, g64.nx, g64.ny, g64.nz, yin,    \
                     (const cx<TF>*)F, (cx<TO>*)yout, k, nw, sw0h, sdwh, h, pass)
#define RES_GH2(TF, TO) \
  if (g64.ncomp == 3) RES_GH(TF, TO, 3); else RES_GH(TF, TO, 1)
  if (f_fp64 && out_fp64) { RES_GH2(double, double); }
  else if (f_fp64) { RES_GH2(double, float); }
  else if (out_fp64) { RES_GH2(float, double); }
  else { RES_GH2(float, float); }
#undef RES_GH2
#undef RES_GH
  return 0;
}

}  // namespace res
