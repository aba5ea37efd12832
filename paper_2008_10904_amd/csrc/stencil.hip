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
// G_j = h Q_j(Z) F_j, built by three Horner passes of the same stencil; see step1d.hip).  2-D one-component
// operators run the whole step in one launch (grid_step2d_kernel); 3-D three-component operators run one launch
// per stage, marching along z (grid_stage3d_kernel).
#include "common.h"
#include "kernels.h"
#include "gridz.h"

namespace res {

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

// One Horner stage of a 3-D three-component operator, marching along z.  A workgroup of 64 x 4 threads owns a
// 64 x 4 column of nodes in x and y and a chunk of ZC planes of one state column b.  Each thread keeps the three
// components of vin at planes z-1, z, z+1 of its own (x, y) in registers; plane z is also published to LDS with
// a one-node ring around the tile (loaded by the edge threads), which supplies the x and y neighbours.  Every
// value of vin is therefore read once from HBM per stage (plus the ring, mostly from L2), u once and vout
// written once, against several reads of vin's neighbour planes when every node reads its own stencil.
//   out = u + s (Z vin)   (stages 1-3),      u <- u + Z vin + phi frc   (LAST, in place; snapshot of u first)
// Operation order per component as apply_z: diagonal, -x, +x, -y, +y, -z, +z, then the coupling.
template <typename R, bool LAST, int ZC>
__global__ __launch_bounds__(256) void grid_stage3d_kernel(GridCoef<R> Cf, int64_t nx, int64_t ny, int64_t nz,
                                                           cx<R>* u, const cx<R>* __restrict__ vin,
                                                           cx<R>* __restrict__ vout, R s,
                                                           const cx<R>* __restrict__ frc, R phr, R phi,
                                                           cx<R>* __restrict__ snap) {
  constexpr int TX = 64, TY = 4, NC = 3;
  __shared__ cx<R> Lp[2][NC][TY + 2][TX + 2];
  const int tid = threadIdx.x;
  const int lx = tid & 63, ly = tid >> 6;
  const int64_t nodes = nx * ny * nz;
  const int64_t ix = (int64_t)blockIdx.x * TX + lx, iy = (int64_t)blockIdx.y * TY + ly;
  const int64_t nzc = (nz + ZC - 1) / ZC;
  const int64_t b = blockIdx.z / nzc, z0 = (blockIdx.z % nzc) * ZC;
  const int64_t z1 = z0 + ZC < nz ? z0 + ZC : nz;
  const bool own = ix < nx && iy < ny;
  const int64_t cb = b * NC * nodes;
  const int64_t sy = nx, sz = nx * ny;
  // ring cells of the tile for the x/y neighbours: (ry, rx) in the (TY+2) x (TX+2) window, ry or rx on the edge
  // (4*66 + ... = 140 cells); thread t < 140 loads ring cell t of every plane.
  int ring_ry = -1, ring_rx = -1;
  if (tid < 2 * (TX + 2)) {
    ring_ry = tid < TX + 2 ? 0 : TY + 1;
    ring_rx = tid < TX + 2 ? tid : tid - (TX + 2);
  } else if (tid < 2 * (TX + 2) + 2 * TY) {
    const int t = tid - 2 * (TX + 2);
    ring_ry = 1 + (t >> 1);
    ring_rx = (t & 1) ? TX + 1 : 0;
  }
  const int64_t rgx = (int64_t)blockIdx.x * TX + ring_rx - 1, rgy = (int64_t)blockIdx.y * TY + ring_ry - 1;
  const bool ring_in = ring_ry >= 0 && rgx >= 0 && rgx < nx && rgy >= 0 && rgy < ny;
  auto ld = [&](int64_t z, int c) -> cx<R> {  // vin at this thread's (x, y), plane z, component c (0 outside)
    return (own && z >= 0 && z < nz) ? vin[cb + c * nodes + z * sz + iy * sy + ix] : mk<R>(R(0), R(0));
  };
  // Per-plane operands of this thread's node: line coefficients, diagonal, coupling row block, u (and the
  // forcing in the last stage).  They are loaded one plane ahead, with vin two planes ahead, so that every global
  // load of an iteration is in flight while the previous plane is computed.
  struct PlaneOps {
    R cxm, cxp, cym, cyp, czm, czp, dd;
    R K[9];
    cx<R> uu[NC], ff[NC];
  };
  auto load_ops = [&](int64_t z) -> PlaneOps {
    PlaneOps o;
    const bool ok = own && z < nz;
    const int64_t l = ok ? z * ny + iy : 0;
    const int64_t p = ok ? z * sz + iy * sy + ix : 0;
    o.cxm = ok ? Cf.cxm[l] : R(0); o.cxp = ok ? Cf.cxp[l] : R(0);
    o.cym = ok ? Cf.cym[l] : R(0); o.cyp = ok ? Cf.cyp[l] : R(0);
    o.czm = ok ? Cf.czm[l] : R(0); o.czp = ok ? Cf.czp[l] : R(0);
    o.dd = ok ? Cf.d[p] : R(0);
#pragma unroll
    for (int q = 0; q < 9; ++q) o.K[q] = (ok && Cf.K != nullptr) ? Cf.K[l * 9 + q] : R(0);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      o.uu[c] = ok ? u[cb + c * nodes + p] : mk<R>(R(0), R(0));
      o.ff[c] = (LAST && ok && frc != nullptr) ? frc[cb + c * nodes + p] : mk<R>(R(0), R(0));
    }
    return o;
  };
  cx<R> xm[NC], x0[NC], xp[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    xm[c] = ld(z0 - 1, c);
    x0[c] = ld(z0, c);
    xp[c] = ld(z0 + 1, c);
  }
  PlaneOps cur = load_ops(z0);
  for (int64_t z = z0; z < z1; ++z) {
    cx<R>(*L)[TY + 2][TX + 2] = Lp[z & 1];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      L[c][ly + 1][lx + 1] = x0[c];
      if (ring_ry >= 0)
        L[c][ring_ry][ring_rx] = ring_in ? vin[cb + c * nodes + z * sz + rgy * sy + rgx] : mk<R>(R(0), R(0));
    }
    __syncthreads();
    // next planes' operands, in flight while this plane is computed
    cx<R> xn[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) xn[c] = ld(z + 2, c);
    const PlaneOps nxt = load_ops(z + 1);
    if (own) {
      const int64_t p = z * sz + iy * sy + ix;
      cx<R> zv[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        cx<R> acc = mk<R>(cur.dd * x0[c].re, cur.dd * x0[c].im);
        const cx<R> w = L[c][ly + 1][lx], e = L[c][ly + 1][lx + 2], sn = L[c][ly][lx + 1], nn = L[c][ly + 2][lx + 1];
        acc.re += cur.cxm * w.re; acc.im += cur.cxm * w.im;
        acc.re += cur.cxp * e.re; acc.im += cur.cxp * e.im;
        acc.re += cur.cym * sn.re; acc.im += cur.cym * sn.im;
        acc.re += cur.cyp * nn.re; acc.im += cur.cyp * nn.im;
        acc.re += cur.czm * xm[c].re; acc.im += cur.czm * xm[c].im;
        acc.re += cur.czp * xp[c].re; acc.im += cur.czp * xp[c].im;
        zv[c] = acc;
      }
      if (Cf.K != nullptr) {
        cx<R> add[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          add[c] = zv[c];
#pragma unroll
          for (int cp = 0; cp < NC; ++cp) {
            add[c].re += cur.K[c * 3 + cp] * x0[cp].re;
            add[c].im += cur.K[c * 3 + cp] * x0[cp].im;
          }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) zv[c] = add[c];
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int64_t e = cb + c * nodes + p;
        const cx<R> uu = cur.uu[c];
        if (LAST) {
          if (snap != nullptr) snap[e] = uu;
          const cx<R> f = cur.ff[c];
          cx<R> r = mk<R>(uu.re + zv[c].re, uu.im + zv[c].im);
          r.re += phr * f.re - phi * f.im;
          r.im += phr * f.im + phi * f.re;
          u[e] = r;
        } else {
          vout[e] = mk<R>(uu.re + s * zv[c].re, uu.im + s * zv[c].im);
        }
      }
    }
    cur = nxt;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      xm[c] = x0[c];
      x0[c] = xp[c];
      xp[c] = xn[c];
    }
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

int launch_grid_stage3d(const GridOpDev& g, int fp64, int k, void* u, const void* vin, void* vout, double s, int last,
                        const void* frc, double phr, double phi, void* snap, hipStream_t st) {
  constexpr int ZC = 16;  // planes per workgroup: enough workgroups for whole rounds of the chip
  if (g.ncomp != 3 || k < 1) return -1;
  const int64_t nzc = (g.nz + ZC - 1) / ZC;
  if ((int64_t)k * nzc > 65535) return -1;
  const dim3 grid((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + 3) / 4), (unsigned)(k * nzc));
#define RES_G3(R, L)                                                                                              \
  hipLaunchKernelGGL((grid_stage3d_kernel<R, L, ZC>), grid, dim3(256), 0, st, coef_of<R>(g, fp64), g.nx, g.ny,     \
                     g.nz, (cx<R>*)u, (const cx<R>*)vin, (cx<R>*)vout, (R)s, (const cx<R>*)frc, (R)phr, (R)phi,    \
                     (cx<R>*)snap)
  if (fp64) {
    if (last) RES_G3(double, true); else RES_G3(double, false);
  } else {
    if (last) RES_G3(float, true); else RES_G3(float, false);
  }
#undef RES_G3
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
