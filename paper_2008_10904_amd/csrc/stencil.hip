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
// operators run the whole step in one launch (grid_step2d_kernel); 3-D three-component operators run two launches
// of two stages each, marching along z (grid_pair3d_kernel).
#include <algorithm>
#include <cstdlib>

#include "common.h"
#include "kernels.h"
#include "gridz.h"

namespace res {

// Whole RK4 step of the 2-D five-point operator in one launch (temporal blocking).  A workgroup of NWAVE x 64
// threads owns a 56 x (WY - 8) tile of one column and works on the 64 x WY window around it (halo 4 = the radius
// of P(Z)).  Lane l of strip w holds window column l, rows RS w .. RS w + RS - 1 (RS = WY / NWAVE), in registers
// (the state u, the diagonal, the current stage values); each stage publishes the stage input to one of two LDS
// windows, so x-neighbours and the strip-end y-neighbours come from LDS and the other y-neighbours from the
// thread's own registers.  The valid region shrinks by one node per stage; values outside the grid are zero
// (homogeneous Dirichlet).  The new state goes to uout (a different buffer: neighbouring tiles read this step's u
// as their halo).  HBM traffic per step: the state once (plus halo rows, mostly from L2), the forcing row once,
// the new state once.
//
// NSTEP = 2 takes two steps per launch on a window with a halo of 8: after the first step's four stages the new
// state (with the first step's forcing row frc, and the snapshot of u into snap) replaces u on the region the
// second step still reads, and the second step ends with frc2 and snap2.  Every node gets the arithmetic of two
// one-step launches in the same order, so the results are the same bits; the state between the steps never
// leaves the registers, and the launches and the state's round trip through memory are halved.
template <typename R, int NWAVE, int WY, int NSTEP = 1>
__global__ __launch_bounds__(64 * NWAVE) void grid_step2d_kernel(GridCoef<R> Cf, int64_t nx, int64_t ny,
                                                          const cx<R>* __restrict__ uin, cx<R>* __restrict__ uout,
                                                          const cx<R>* __restrict__ frc, R phr, R phi,
                                                          cx<R>* __restrict__ snap,
                                                          const cx<R>* __restrict__ frc2,
                                                          cx<R>* __restrict__ snap2) {
  constexpr int H = 4 * NSTEP, WX = 64, TX = WX - 2 * H, TY = WY - 2 * H, RS = WY / NWAVE;
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
  for (int m = 1; m <= 4 * NSTEP; ++m) {
    cx<R>(*Lm)[WX] = Lw[m & 1];
#pragma unroll
    for (int r = 0; r < RS; ++r) Lm[ly0 + r][lx] = x[r];
    __syncthreads();
    const int mm = (m - 1) % 4 + 1;  // stage within its step
    const R s = mm == 1 ? R(0.25) : mm == 2 ? R(1) / R(3) : mm == 3 ? R(0.5) : R(1);
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
    if (NSTEP == 2 && m == 4) {
      // end of the first step on the region the second one reads (the window less a ring of 4): forcing, the
      // snapshot of u at the tile interior, and the new state as the second step's u and stage input
      const bool xok1 = lx >= 4 && lx < WX - 4;
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        const int ly = ly0 + r;
        cx<R> v = mk<R>(R(0), R(0));
        if (xok1 && ly >= 4 && ly < WY - 4 && in[r]) {
          const int64_t e = cb + (y0 + ly) * nx + ix;
          if (snap != nullptr && lx >= H && lx < WX - H && ly >= H && ly < WY - H) snap[e] = u[r];
          v = x[r];
          if (frc != nullptr) {
            const cx<R> f = frc[e];
            v.re += phr * f.re - phi * f.im;
            v.im += phr * f.im + phi * f.re;
          }
        }
        u[r] = v;
        x[r] = v;
      }
    }
  }
  // interior of the tile: forcing, snapshot of u (the state before the last step) and the new state
  const cx<R>* fl = NSTEP == 2 ? frc2 : frc;
  cx<R>* sl = NSTEP == 2 ? snap2 : snap;
  if (lx < H || lx >= WX - H) return;
#pragma unroll
  for (int r = 0; r < RS; ++r) {
    const int ly = ly0 + r;
    if (ly < H || ly >= WY - H || !in[r]) continue;
    const int64_t e = cb + (y0 + ly) * nx + ix;
    if (sl != nullptr) sl[e] = u[r];
    cx<R> v = x[r];
    if (fl != nullptr) {
      const cx<R> f = fl[e];
      v.re += phr * f.re - phi * f.im;
      v.im += phr * f.im + phi * f.re;
    }
    uout[e] = v;
  }
}

// Two Horner stages of a 3-D three-component operator in one pass, marching along z; a step is two passes.  A
// workgroup of TX x TY threads covers a TX x TY window of (x, y) nodes of one state column; the window's interior
// (halo 2 = the reach of two stages) is its output tile.  At plane a of the march it evaluates
//   stage A at plane a:      y = u + sa Z x    on the window (its outer ring is not needed later),
//   stage B at plane a - 1:  out = u + sb Z y  on the interior (plus phi frc in the second pass),
// with x and y published to double-buffered LDS planes for the x/y neighbours and kept in per-thread register
// rings for the z neighbours; the line coefficients of the window rows sit in four LDS plane slots.  One barrier
// per plane orders every LDS access.  Every global load of a plane is issued one plane ahead of its use, with
// clamped addresses, and masked when it is used.  Values outside the grid are zero (homogeneous Dirichlet).
//   pass 1 (SECOND = false): x = u,  sa = 1/4, sb = 1/3: out = the third stage's input,
//   pass 2 (SECOND = true):  x = vin, sa = 1/2, sb = 1:  out = the new state, in a buffer other than u (windows
//                            read u at halo nodes that neighbouring tiles update); snapshot of u first.
// Operation order per component as apply_z: diagonal, -x, +x, -y, +y, -z, +z, then the coupling.
template <typename R, bool SECOND, int TX, int TY, int ZC>
__global__ __launch_bounds__(TX * TY) void grid_pair3d_kernel(GridCoef<R> Cf, int64_t nx, int64_t ny, int64_t nz,
                                                              int64_t ncol,
                                                              const cx<R>* __restrict__ u,
                                                              const cx<R>* __restrict__ vin,
                                                              cx<R>* __restrict__ out,
                                                              const cx<R>* __restrict__ frc, R phr, R phi,
                                                              cx<R>* __restrict__ snap) {
  constexpr int H = 2, NC = 3, OX = TX - 2 * H, OY = TY - 2 * H, NQ = 15;
  __shared__ cx<R> Xs[2][NC][TY][TX];
  __shared__ cx<R> Ys[2][NC][TY][TX];
  __shared__ R Cs[4][TY][NQ];  // plane slot, window row: cxm cxp cym cyp czm czp K[9]
  const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
  const int64_t nodes = nx * ny * nz, sz = nx * ny;
  const int64_t nzc = (nz + ZC - 1) / ZC;
  // Tile order: workgroups are dealt to the eight XCDs in turn (id mod 8); each XCD takes a contiguous run of
  // tiles (x fastest, then y, then z chunk and column), so the tiles whose halos overlap run side by side and
  // share that XCD's L2.
  const int64_t gx = (nx + OX - 1) / OX, gy = (ny + OY - 1) / OY, ntile = gx * gy * nzc * ncol;
  const int64_t tile = (int64_t)(blockIdx.x & 7) * ((ntile + 7) / 8) + (blockIdx.x >> 3);
  if (tile >= ntile) return;  // padding of the grid to a multiple of 8 (whole workgroup)
  const int64_t tx = tile % gx, ty = (tile / gx) % gy, tzb = tile / (gx * gy);
  const int64_t b = tzb / nzc, z0 = (tzb % nzc) * ZC;
  const int64_t z1 = z0 + ZC < nz ? z0 + ZC : nz;
  const int64_t ix = tx * OX - H + lx, iy = ty * OY - H + ly;
  const bool inxy = ix >= 0 && ix < nx && iy >= 0 && iy < ny;
  const bool interior = inxy && lx >= H && lx < TX - H && ly >= H && ly < TY - H;
  const int64_t cb = b * NC * nodes;
  const int64_t pxy = inxy ? iy * nx + ix : 0;
  const cx<R>* __restrict__ X = SECOND ? vin : u;
  const R sa = SECOND ? R(0.5) : R(0.25), sb = SECOND ? R(1) : R(1) / R(3);
  const cx<R> zero = mk<R>(R(0), R(0));
  const bool coupled = Cf.K != nullptr;
  // LDS neighbours, clamped at the window edge (edge threads compute values that are never used)
  const int xl = lx > 0 ? lx - 1 : 0, xr = lx < TX - 1 ? lx + 1 : TX - 1;
  const int yl = ly > 0 ? ly - 1 : 0, yr = ly < TY - 1 ? ly + 1 : TY - 1;
  auto zin = [&](int64_t z) { return z >= 0 && z < nz; };
  auto zc = [&](int64_t z) -> int64_t { return z < 0 ? 0 : (z >= nz ? nz - 1 : z); };

  struct V3 {
    cx<R> c[NC];
  };
  // raw loads (clamped, unconditional); masking happens at use
  auto ld3 = [&](const cx<R>* __restrict__ A, int64_t z) -> V3 {
    V3 r;
    const int64_t e = cb + zc(z) * sz + pxy;
#pragma unroll
    for (int c = 0; c < NC; ++c) r.c[c] = A[e + c * nodes];
    return r;
  };
  auto mask3 = [&](const V3& v, bool ok) -> V3 {
    V3 r;
#pragma unroll
    for (int c = 0; c < NC; ++c) r.c[c] = ok ? v.c[c] : zero;
    return r;
  };
  auto ldd = [&](int64_t z) -> R { return Cf.d[zc(z) * sz + pxy]; };
  // line coefficient q of window row r at plane z (staging threads tid < TY * NQ)
  const int cr = tid / NQ, cq = tid % NQ;
  const bool stager = tid < TY * NQ;
  const int64_t ciy = ty * OY - H + cr;
  const bool crow_in = stager && ciy >= 0 && ciy < ny;
  auto ldc = [&](int64_t z) -> R {
    const int64_t l = zc(z) * ny + (crow_in ? ciy : 0);
    const R* src = cq == 0 ? Cf.cxm : cq == 1 ? Cf.cxp : cq == 2 ? Cf.cym : cq == 3 ? Cf.cyp
                 : cq == 4 ? Cf.czm : cq == 5 ? Cf.czp : Cf.K;
    if (!stager || src == nullptr) return R(0);
    return cq < 6 ? src[l] : src[l * 9 + (cq - 6)];
  };
  auto put_coef = [&](int64_t z, R v) {
    if (stager) Cs[z & 3][cr][cq] = (crow_in && zin(z)) ? v : R(0);
  };
  // (Z x) at this thread's node of plane z: centre x0, z neighbours xm/xp (masked), x/y neighbours from plane L
  auto apply = [&](const cx<R> (*L)[TY][TX], const V3& xm, const V3& x0, const V3& xp, R dd, int slot) -> V3 {
    const R* cf = Cs[slot][ly];
    const R cxm = cf[0], cxp = cf[1], cym = cf[2], cyp = cf[3], czm = cf[4], czp = cf[5];
    V3 zv;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      cx<R> acc = mk<R>(dd * x0.c[c].re, dd * x0.c[c].im);
      const cx<R> w = L[c][ly][xl], e = L[c][ly][xr], sn = L[c][yl][lx], nn = L[c][yr][lx];
      acc.re += cxm * w.re; acc.im += cxm * w.im;
      acc.re += cxp * e.re; acc.im += cxp * e.im;
      acc.re += cym * sn.re; acc.im += cym * sn.im;
      acc.re += cyp * nn.re; acc.im += cyp * nn.im;
      acc.re += czm * xm.c[c].re; acc.im += czm * xm.c[c].im;
      acc.re += czp * xp.c[c].re; acc.im += czp * xp.c[c].im;
      zv.c[c] = acc;
    }
    if (coupled) {
      V3 add;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        add.c[c] = zv.c[c];
#pragma unroll
        for (int cp = 0; cp < NC; ++cp) {
          const R kk = cf[6 + c * 3 + cp];
          add.c[c].re += kk * x0.c[cp].re;
          add.c[c].im += kk * x0.c[cp].im;
        }
      }
      zv = add;
    }
    return zv;
  };

  // rings at the start of iteration a: x(a-1), x(a), x(a+1); u(a-1), u(a); d(a-1), d(a); y(a-2), y(a-1); f(a-1);
  // the coefficients of plane a+1 in a register (staged to LDS in iteration a).  The forcing is loaded after the
  // stage that uses it, which keeps the second pass within the register budget of 1,024-thread workgroups.
  int64_t a = z0 - 1;
  V3 xm = mask3(ld3(X, a - 1), inxy && zin(a - 1)), x0 = mask3(ld3(X, a), inxy && zin(a)), xp = ld3(X, a + 1);
  V3 um, u0;
  if (SECOND) {
    um = ld3(u, a - 1);
    u0 = ld3(u, a);
  }
  R dm = ldd(a - 1), d0 = ldd(a);
  V3 ym, y0;
#pragma unroll
  for (int c = 0; c < NC; ++c) ym.c[c] = y0.c[c] = zero;
  const bool forced = SECOND && frc != nullptr && interior;  // only the output nodes read the forcing
  V3 fm;
  if (forced) fm = ld3(frc, a - 1);
  put_coef(a, ldc(a));
  R creg = ldc(a + 1);
  for (; a <= z1; ++a) {
    const bool ain = inxy && zin(a);
    xp = mask3(xp, inxy && zin(a + 1));  // x(a-1) and x(a) were masked when they arrived at this position
#pragma unroll
    for (int c = 0; c < NC; ++c) Xs[a & 1][c][ly][lx] = x0.c[c];
    put_coef(a + 1, creg);
    __syncthreads();
    // next plane's operands, in flight while this plane is computed
    const V3 xn = ld3(X, a + 2);
    V3 un;
    if (SECOND) un = ld3(u, a + 1);
    const R dn = ldd(a + 1);
    creg = ldc(a + 2);
    // stage A at plane a
    V3 y;
    {
      const V3 uu = SECOND ? u0 : x0;
      const V3 zv = apply(Xs[a & 1], xm, x0, xp, d0, (int)(a & 3));
#pragma unroll
      for (int c = 0; c < NC; ++c)
        y.c[c] = ain ? mk<R>(uu.c[c].re + sa * zv.c[c].re, uu.c[c].im + sa * zv.c[c].im) : zero;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) Ys[a & 1][c][ly][lx] = y.c[c];
    // stage B at plane a - 1 (its y plane was published in the previous iteration)
    const int64_t zb = a - 1;
    if (zb >= z0 && zb < z1) {
      const V3 zv = apply(Ys[zb & 1], ym, y0, y, dm, (int)(zb & 3));
      if (interior) {
        const int64_t e = cb + zb * sz + pxy;
        const V3 ub = SECOND ? um : xm;  // u at plane zb (pass 1: x = u)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          cx<R> r = mk<R>(ub.c[c].re + sb * zv.c[c].re, ub.c[c].im + sb * zv.c[c].im);
          if (SECOND) {
            if (snap != nullptr) snap[e + c * nodes] = ub.c[c];
            if (forced) {
              const cx<R> f = fm.c[c];
              r.re += phr * f.re - phi * f.im;
              r.im += phr * f.im + phi * f.re;
            }
          }
          out[e + c * nodes] = r;
        }
      }
    }
    xm = x0;
    x0 = xp;
    xp = xn;
    if (SECOND) {
      um = u0;
      u0 = un;
    }
    if (forced) fm = ld3(frc, a);  // for the next stage B (loaded after this one has used fm)
    dm = d0;
    d0 = dn;
    ym = y0;
    y0 = y;
  }
}

// Whole RK4 step of the 3-D three-component operator in one launch, marching along z (FP32 state).
//
// The four Horner stages v1 = u + Z u/4, v2 = u + Z v1/3, v3 = u + Z v2/2, u' = u + Z v3 + phi frc are pipelined
// over the planes: at plane step a the workgroup evaluates v1 at plane a-1, v2 at a-2, v3 at a-3 and the new
// state at a-4, each from the previous stage's planes just above and below it, so the state is read once and
// written once per step and no stage value leaves the chip (a stage has radius 1 in z, hence the lag of one plane
// per stage).  A workgroup of 64 x TY threads covers a 64 x TY window of (x, y) nodes of one state column; wave w
// holds window row w, lane l window column l.  Stage m is valid on the window shrunk by m nodes per side (halo 4 =
// the reach of four stages), so the output tile is the 56 x (TY - 8) interior, and the waves of rows outside stage
// m's rows skip it (the skipped work balances over the four SIMDs: row w runs on SIMD w mod 4); so do the waves of
// rows outside the grid, whose values stay zero.
//
// Where the operands come from: the x neighbours are the lanes next door, moved by DPP wave shifts (no LDS); the y
// neighbours are other waves' rows, read from that stage's plane in LDS (one buffer per stage, published once per
// plane step); the z neighbours and the centre are per-thread registers.  The three register roles of each stage
// (plane below, centre, plane just computed) rotate with period three, so the plane loop is unrolled three times
// and the rotation is a renaming, not a copy; the Horner bases u(a-3) and u(a-4) sit in a two-plane LDS ring that
// each thread reads for its own node only.  A row's line coefficients are wave-uniform: one packed scalar load per
// stage (GridOpDev::lc).  Two LDS-only barriers per plane step (before the stage planes are read and before they
// are overwritten) leave the global loads and stores in flight; the next step's state plane and diagonal and the
// forcing of the output nodes are loaded at the top of a step and consumed at its end.  Values outside the grid are zero (homogeneous
// Dirichlet): only the first and last tile in x hold lanes outside it, and only they mask.  Operation order per
// component as apply_z: diagonal, -x, +x, -y, +y, -z, +z, then the coupling; KV selects its pattern (0: none; 1:
// the shear terms K01, K02 of the first component; 2: their transpose K10, K20 in Z^H; 3: all nine, read from K).
// u' goes to a buffer other than u (windows read u at halo nodes that neighbouring tiles update); the snapshot (if
// any) takes u.
struct alignas(32) LineCoef8 {
  float v[8];  // cxm cxp cym cyp czm czp kA kB
};

// Value of lane l - 1 (dir = 0) or l + 1 (dir = 1) of the wave, 0 beyond its ends.
template <int DIR> __device__ __forceinline__ float lane_shift(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), DIR == 0 ? 0x138 : 0x130, 0xf, 0xf, true));
}

template <int TY, int KV, bool ZS>
__global__ __launch_bounds__(64 * TY) void grid_step3d_kernel(GridCoef<float> Cf, const LineCoef8* __restrict__ lc,
                                                              int64_t nx, int64_t ny, int64_t nz, int64_t ncol,
                                                              const cx<float>* __restrict__ u,
                                                              cx<float>* __restrict__ out,
                                                              const cx<float>* __restrict__ frc, float phr, float phi,
                                                              cx<float>* __restrict__ snap, int nzc) {
  constexpr int H = 4, TX = 64, OX = TX - 2 * H, OY = TY - 2 * H, NC = 3;
  __shared__ cx<float> Ls[4][NC][TY][TX];
  __shared__ cx<float> Us[2][NC][TY][TX];
  const int lx = threadIdx.x & 63;
  const int wy = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // window row: uniform across the wave
  // 32-bit offsets inside one column (the launcher checks 3 * nodes < 2^31); 64-bit only for the column base
  const int nodes = (int)(nx * ny * nz), sz = (int)(nx * ny), nx32 = (int)nx, ny32 = (int)ny, nz32 = (int)nz;
  // Tile order: workgroups are dealt to the eight XCDs in turn (id mod 8); each XCD takes a contiguous run of
  // tiles (z chunk fastest, then x, then y, then column), so tiles whose halos overlap march side by side and
  // share its L2.
  // (ZS: the planes are split into nzc chunks; without it nzc is 1 and the chunk logic compiles away)
  if (!ZS) nzc = 1;
  const int64_t gx = (nx + OX - 1) / OX, gy = (ny + OY - 1) / OY, ntile = gx * gy * ncol * nzc;
  const int64_t tile = (int64_t)(blockIdx.x & 7) * ((ntile + 7) / 8) + (blockIdx.x >> 3);
  if (tile >= ntile) return;  // padding of the grid to a multiple of 8 (whole workgroup)
  const int zcix = ZS ? (int)(tile % nzc) : 0;
  const int64_t xyb = ZS ? tile / nzc : tile;
  const int tx = (int)(xyb % gx), ty = (int)((xyb / gx) % gy);
  const int64_t b = xyb / (gx * gy);
  // z chunk [z0, z1) of the output planes; a chunk after the first starts its march two planes early and
  // discards the outputs below z0 (stage 4 at plane z0 needs stage 1 from plane z0 - 3 on, which needs u from
  // plane z0 - 4); every output node gets the same arithmetic as in a single chunk
  const int zlen = ZS ? (int)((nz + nzc - 1) / nzc) : (int)nz;
  const int z0 = ZS ? zcix * zlen : 0, z1 = ZS ? min((int)nz, z0 + zlen) : (int)nz;
  if (ZS && z0 >= (int)nz) return;  // whole workgroup
  const int a_start = (!ZS || zcix == 0) ? 0 : z0 - 2, a_end = z1 + 4;
  const int x0w = tx * OX - H;                      // first window column (uniform)
  const int ix = x0w + lx, iy = ty * OY - H + wy;   // iy uniform
  const bool yin = iy >= 0 && iy < ny32;            // uniform
  const bool xin = ix >= 0 && ix < nx32;
  const bool xedge = x0w < 0 || x0w + TX > nx32;    // uniform: this tile has lanes outside the grid
  const int iyc = yin ? iy : 0;
  const uint32_t pxy = (uint32_t)(iyc * nx32 + (xin ? ix : 0));  // this lane's node in a plane (clamped)
  const int64_t cb = b * NC * (int64_t)nodes;
  const cx<float>* __restrict__ ucol = u + cb;
  const cx<float>* __restrict__ fcol = frc != nullptr ? frc + cb : nullptr;
  cx<float>* __restrict__ ocol = out + cb;
  cx<float>* __restrict__ scol = snap != nullptr ? snap + cb : nullptr;
  const cx<float> zero = mk<float>(0.f, 0.f);
  const int yl = wy > 0 ? wy - 1 : 0, yr = wy < TY - 1 ? wy + 1 : TY - 1;
  // window rows on which stage m (1..4) is evaluated (none for rows outside the grid)
  auto row_ok = [&](int m) { return yin && wy >= m && wy < TY - m; };
  auto zc = [&](int z) -> int { return z < 0 ? 0 : (z >= nz32 ? nz32 - 1 : z); };
  auto zin = [&](int z) { return z >= 0 && z < nz32; };

  struct V3 {
    cx<float> c[NC];
  };
  auto ld3 = [&](const cx<float>* __restrict__ col, int z) -> V3 {  // clamped plane, unconditional
    V3 r;
    const int o = zc(z) * sz;
#pragma unroll
    for (int c = 0; c < NC; ++c) r.c[c] = (col + (int64_t)(c * nodes + o))[pxy];
    return r;
  };
  auto mask_x = [&](V3& v) {  // zero at lanes outside the grid (first and last tile in x only)
    if (xedge) {
#pragma unroll
      for (int c = 0; c < NC; ++c) v.c[c] = csel(xin, v.c[c], zero);
    }
  };
  auto zero3 = [&](V3& v) {
#pragma unroll
    for (int c = 0; c < NC; ++c) v.c[c] = zero;
  };
  // base + s * (Z x) at this thread's node of plane z: centre x0 and z neighbours xm, xp from registers, x
  // neighbours by lane shifts of x0, y neighbours from LDS stage buffer S
  auto stage = [&](int S, int z, const V3& xm, const V3& x0, const V3& xp, const V3& base, float dd, float s) -> V3 {
    const int l = z * ny32 + iyc;
    const LineCoef8 q = lc[l];
    const float cxm = q.v[0], cxp = q.v[1], cym = q.v[2], cyp = q.v[3], czm = q.v[4], czp = q.v[5];
    V3 zv;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      cx<float> acc = mk<float>(dd * x0.c[c].re, dd * x0.c[c].im);
      const cx<float> sn = Ls[S][c][yl][lx], nn = Ls[S][c][yr][lx];
      acc.re += cxm * lane_shift<0>(x0.c[c].re); acc.im += cxm * lane_shift<0>(x0.c[c].im);
      acc.re += cxp * lane_shift<1>(x0.c[c].re); acc.im += cxp * lane_shift<1>(x0.c[c].im);
      acc.re += cym * sn.re; acc.im += cym * sn.im;
      acc.re += cyp * nn.re; acc.im += cyp * nn.im;
      acc.re += czm * xm.c[c].re; acc.im += czm * xm.c[c].im;
      acc.re += czp * xp.c[c].re; acc.im += czp * xp.c[c].im;
      zv.c[c] = acc;
    }
    if (KV == 1) {  // first component: + K01 x_1 + K02 x_2
      zv.c[0].re += q.v[6] * x0.c[1].re; zv.c[0].im += q.v[6] * x0.c[1].im;
      zv.c[0].re += q.v[7] * x0.c[2].re; zv.c[0].im += q.v[7] * x0.c[2].im;
    } else if (KV == 2) {  // second and third components: + K10 x_0, + K20 x_0
      zv.c[1].re += q.v[6] * x0.c[0].re; zv.c[1].im += q.v[6] * x0.c[0].im;
      zv.c[2].re += q.v[7] * x0.c[0].re; zv.c[2].im += q.v[7] * x0.c[0].im;
    } else if (KV == 3) {
      const float* Kl = Cf.K + (int64_t)l * 9;
      V3 add;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        add.c[c] = zv.c[c];
#pragma unroll
        for (int cp = 0; cp < NC; ++cp) {
          add.c[c].re += Kl[c * 3 + cp] * x0.c[cp].re;
          add.c[c].im += Kl[c * 3 + cp] * x0.c[cp].im;
        }
      }
      zv = add;
    }
    V3 r;
#pragma unroll
    for (int c = 0; c < NC; ++c) r.c[c] = mk<float>(base.c[c].re + s * zv.c[c].re, base.c[c].im + s * zv.c[c].im);
    mask_x(r);
    return r;
  };

  const bool interior = yin && xin && lx >= H && lx < TX - H && wy >= H && wy < TY - H;
  const bool forced = fcol != nullptr && interior;  // only the output nodes read the forcing
  float d4 = 0.f, d3 = 0.f, d2 = 0.f, d1 = 0.f;
  // One plane step.  On entry: LDS stage buffers 0..3 hold u(a-1), v1(a-2), v2(a-3), v3(a-4) and registers
  // uZp = u(a), uC = u(a-1), uZm = u(a-2), vmZm = vm at the plane below the stage's centre, vmC = vm at the centre;
  // vmN receives the stage's new plane.  On exit uZm holds u(a+1) and the roles have moved by one: the next step
  // takes (uZm, uZp, uC) as (uZp, uC, uZm) and (vmC, vmN, vmZm) as (vmZm, vmC, vmN).  A stage that is skipped
  // (plane outside the grid) leaves a zero plane behind.
  auto step = [&](int a, V3& uZp, V3& uC, V3& uZm, V3& v1Zm, V3& v1C, V3& v1N, V3& v2Zm, V3& v2C, V3& v2N,
                  V3& v3Zm, V3& v3C, V3& v3N) {
    lds_barrier();  // the stage planes of this step are published
    // operands of the next step: the state plane a+1, the diagonal of plane a; the forcing of plane a-4
    const V3 un = ld3(ucol, a + 1);
    const float dn = Cf.d[(int64_t)zc(a) * sz + pxy];
    V3 f4;
    if (forced) f4 = ld3(fcol, a - 4);
    if (row_ok(1) && zin(a - 1)) v1N = stage(0, a - 1, uZm, uC, uZp, uC, d1, 0.25f);
    else zero3(v1N);
    if (row_ok(2) && zin(a - 2)) v2N = stage(1, a - 2, v1Zm, v1C, v1N, uZm, d2, 1.f / 3.f);
    else zero3(v2N);
    V3 u3, u4;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      u3.c[c] = Us[(a - 1) & 1][c][wy][lx];
      u4.c[c] = Us[a & 1][c][wy][lx];
    }
    if (row_ok(3) && zin(a - 3)) v3N = stage(2, a - 3, v2Zm, v2C, v2N, u3, d3, 0.5f);
    else zero3(v3N);
    if (row_ok(4) && zin(a - 4)) {
      V3 r = stage(3, a - 4, v3Zm, v3C, v3N, u4, d4, 1.f);
      if (interior && (!ZS || a - 4 >= z0)) {
        const int e = (a - 4) * sz;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          if (forced) {
            const cx<float> f = f4.c[c];
            r.c[c].re += phr * f.re - phi * f.im;
            r.c[c].im += phr * f.im + phi * f.re;
          }
          if (scol != nullptr) (scol + (int64_t)(c * nodes + e))[pxy] = u4.c[c];
          (ocol + (int64_t)(c * nodes + e))[pxy] = r.c[c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) Us[a & 1][c][wy][lx] = uZm.c[c];  // u(a-2): read as u(a-3), then u(a-4)
    lds_barrier();  // every read of the stage planes is done before they are overwritten
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      Ls[0][c][wy][lx] = uZp.c[c];
      Ls[1][c][wy][lx] = v1N.c[c];
      Ls[2][c][wy][lx] = v2N.c[c];
      Ls[3][c][wy][lx] = v3N.c[c];
    }
    if (yin && zin(a + 1)) {
      uZm = un;
      mask_x(uZm);
    } else {
      zero3(uZm);
    }
    d4 = d3; d3 = d2; d2 = d1; d1 = dn;
  };

  V3 A, B, C, P1, Q1, R1, P2, Q2, R2, P3, Q3, R3;
  zero3(A); zero3(B); zero3(C);
  zero3(P1); zero3(Q1); zero3(R1); zero3(P2); zero3(Q2); zero3(R2); zero3(P3); zero3(Q3); zero3(R3);
  // entry state of step a_start: u(a_start), u(a_start - 1), u(a_start - 2) (zero outside the grid), stage buffer 0
  // = u(a_start - 1), the diagonal of plane a_start - 1
  if (yin) {
    if (zin(a_start)) A = ld3(ucol, a_start);
    if (zin(a_start - 1)) B = ld3(ucol, a_start - 1);
    if (zin(a_start - 2)) C = ld3(ucol, a_start - 2);
    mask_x(A);
    mask_x(B);
    mask_x(C);
  }
  if (zin(a_start - 1)) d1 = Cf.d[(int64_t)(a_start - 1) * sz + pxy];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    Ls[0][c][wy][lx] = B.c[c];
#pragma unroll
    for (int S = 1; S < 4; ++S) Ls[S][c][wy][lx] = zero;
  }
  const int steps = a_end;
  int a = a_start;
  for (; a + 2 < steps; a += 3) {
    step(a, A, B, C, P1, Q1, R1, P2, Q2, R2, P3, Q3, R3);
    step(a + 1, C, A, B, Q1, R1, P1, Q2, R2, P2, Q3, R3, P3);
    step(a + 2, B, C, A, R1, P1, Q1, R2, P2, Q2, R3, P3, Q3);
  }
  if (a < steps) step(a, A, B, C, P1, Q1, R1, P2, Q2, R2, P3, Q3, R3);
  if (a + 1 < steps) step(a + 1, C, A, B, Q1, R1, P1, Q2, R2, P2, Q3, R3, P3);
}

// One Horner pass of G = h Q_j(Z) F over [n_w][k] blocks (see tri_horner_kernel for the coefficients).
template <typename TF, typename TO, int NC>
__global__ __launch_bounds__(256) void grid_horner_kernel(GridCoef<double> Cf, int64_t nx, int64_t ny, int64_t nz,
                                                          const cx<double>* __restrict__ yin,
                                                          const cx<TF>* __restrict__ F, cx<TO>* __restrict__ yout,
                                                          int k, int nw, double sw0h, double sdwh, double h, int pass,
                                                          int j0) {
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
  sincos(0.5 * (sw0h + (double)(j0 + j) * sdwh), &sa, &ca);
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
  if (g.ncomp != 1 || g.nz != 1 || k < 1 || k > 65535) return -1;
  // FP32: 16 waves of 3 rows on a 64 x 48 window (measured on 1024 x 512 x 2: 12.1 us per step, against 13.2 for
  // 10 waves of 4 rows on 64 x 40, 15.5 for 4 waves of 10 rows and 14.2 for 16 waves of 4 rows on 64 x 64: more
  // waves hide the latency of the stage chain); FP64 keeps 4 waves of 10 rows (twice the registers per row).
  constexpr int WY = 48;
  const dim3 grid((unsigned)((g.nx + 55) / 56), (unsigned)((g.ny + WY - 9) / (WY - 8)), (unsigned)k);
  if (fp64)
    hipLaunchKernelGGL((grid_step2d_kernel<double, 4, 40>), dim3((unsigned)((g.nx + 55) / 56),
                       (unsigned)((g.ny + 31) / 32), (unsigned)k), dim3(256), 0, st, coef_of<double>(g, 1), g.nx,
                       g.ny, (const cx<double>*)uin, (cx<double>*)uout, (const cx<double>*)frc, phr, phi,
                       (cx<double>*)snap, nullptr, nullptr);
  else
    hipLaunchKernelGGL((grid_step2d_kernel<float, 16, WY>), grid, dim3(1024), 0, st, coef_of<float>(g, 0), g.nx,
                       g.ny, (const cx<float>*)uin, (cx<float>*)uout, (const cx<float>*)frc, (float)phr, (float)phi,
                       (cx<float>*)snap, nullptr, nullptr);
  return 0;
}

int launch_grid_step2d_pair(const GridOpDev& g, int k, const void* uin, void* uout, const void* frc,
                            const void* frc2, double phr, double phi, void* snap, void* snap2, int wy,
                            hipStream_t st) {
  if (g.ncomp != 1 || g.nz != 1 || k < 1 || k > 65535 || (wy != 48 && wy != 64)) return -1;
  // 16 waves on a 64 x wy window, halo 8: output tiles of 48 x (wy - 16)
  const dim3 grid((unsigned)((g.nx + 47) / 48), (unsigned)((g.ny + wy - 17) / (wy - 16)), (unsigned)k);
#define RES_S2P(W)                                                                                                 \
  hipLaunchKernelGGL((grid_step2d_kernel<float, 16, W, 2>), grid, dim3(1024), 0, st, coef_of<float>(g, 0), g.nx,   \
                     g.ny, (const cx<float>*)uin, (cx<float>*)uout, (const cx<float>*)frc, (float)phr, (float)phi, \
                     (cx<float>*)snap, (const cx<float>*)frc2, (cx<float>*)snap2)
  if (wy == 48) RES_S2P(48); else RES_S2P(64);
#undef RES_S2P
  return 0;
}

int launch_grid_pair3d(const GridOpDev& g, int fp64, int k, const void* u, const void* vin, void* out, int second,
                       const void* frc, double phr, double phi, void* snap, hipStream_t st) {
  constexpr int ZC = 32;  // planes per workgroup
  if (g.ncomp != 3 || k < 1) return -1;
  const int64_t nzc = (g.nz + ZC - 1) / ZC;
#define RES_P3(R, S, TX, TY)                                                                                       \
  do {                                                                                                            \
    const int64_t tiles = ((g.nx + TX - 5) / (TX - 4)) * ((g.ny + TY - 5) / (TY - 4)) * nzc * k;                 \
    if (tiles > 0x7ffffff0) return -1;                                                                            \
    hipLaunchKernelGGL((grid_pair3d_kernel<R, S, TX, TY, ZC>), dim3((unsigned)((tiles + 7) / 8 * 8)),            \
                       dim3(TX * TY), 0, st, coef_of<R>(g, fp64), g.nx, g.ny, g.nz, (int64_t)k, (const cx<R>*)u,  \
                       (const cx<R>*)vin, (cx<R>*)out, (const cx<R>*)frc, (R)phr, (R)phi, (cx<R>*)snap);         \
  } while (0)
  // LDS: two double-buffered window planes of three components: 64 x 16 windows in FP32, 64 x 8 in FP64 (rows
  // of 64 keep every wave's loads on whole cache lines; 32 x 32 windows measured 12 % slower)
  if (fp64) {
    if (second) RES_P3(double, true, 64, 8); else RES_P3(double, false, 64, 8);
  } else {
    if (second) RES_P3(float, true, 64, 16); else RES_P3(float, false, 64, 16);
  }
#undef RES_P3
  return 0;
}

int launch_grid_step3d(const GridOpDev& g, int k, const void* uin, void* uout, const void* frc, double phr,
                       double phi, void* snap, hipStream_t st) {
  constexpr int TY = 16;  // 16 waves: a 64 x 16 window, 56 x 8 output nodes per plane
  if (g.ncomp != 3 || k < 1 || 3 * g.nx * g.ny * g.nz >= ((int64_t)1 << 31)) return -1;
  const int64_t xy_tiles = ((g.nx + 55) / 56) * ((g.ny + TY - 9) / (TY - 8)) * k;
  // A workgroup marches all the planes of its tile, one workgroup per CU: when the tiles do not fill the CUs (one
  // column of the full 3-D grid: 80 tiles), the planes are split into chunks of at least 16 so that they do.
  // RESOLVENT_STEP3D_ZCHUNKS fixes the number of chunks.
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cus = n;
    else
      cus = 256;
  }
  int nzc = (int)std::max<int64_t>(1, std::min<int64_t>(cus / std::max<int64_t>(1, xy_tiles), g.nz / 16));
  if (const char* e = std::getenv("RESOLVENT_STEP3D_ZCHUNKS")) nzc = std::max(1, std::atoi(e));
  nzc = (int)std::min<int64_t>(nzc, g.nz);
  const int64_t tiles = xy_tiles * nzc;
  if (tiles > 0x7ffffff0) return -1;
  if (g.lc == nullptr) return -1;
  const dim3 grid((unsigned)((tiles + 7) / 8 * 8));
#define RES_S3(KV)                                                                                                \
  if (nzc > 1) RES_S3Z(KV, true); else RES_S3Z(KV, false)
#define RES_S3Z(KV, ZS)                                                                                           \
  hipLaunchKernelGGL((grid_step3d_kernel<TY, KV, ZS>), grid, dim3(64 * TY), 0, st, coef_of<float>(g, 0),         \
                     (const LineCoef8*)g.lc, g.nx, g.ny, g.nz, (int64_t)k, (const cx<float>*)uin, (cx<float>*)uout, \
                     (const cx<float>*)frc, (float)phr, (float)phi, (cx<float>*)snap, nzc)
  // coupling pattern: the shear terms of the first component (Z), their transpose (Z^H), none, or general
  switch (g.kv) {
    case 0: RES_S3(0); break;
    case 1: RES_S3(1); break;
    case 2: RES_S3(2); break;
    default: RES_S3(3); break;
  }
#undef RES_S3
#undef RES_S3Z
  return 0;
}

int launch_grid_horner(const GridOpDev& g64, const cx<double>* yin, const void* F, int f_fp64, void* yout,
                       int out_fp64, int k, int nw, double sw0h, double sdwh, double h, int pass, hipStream_t st,
                       int j0) {
  const int64_t nodes = g64.nx * g64.ny * g64.nz;
  if ((int64_t)nw * k > 65535) return -1;
  const dim3 grid((unsigned)((nodes + 255) / 256), (unsigned)(nw * k));
  GridCoef<double> c = coef_of<double>(g64, 1);
#define RES_GH(TF, TO, NC)                                                                                        \
  hipLaunchKernelGGL((grid_horner_kernel<TF, TO, NC>), grid, dim3(256), 0, st, c, g64.nx, g64.ny, g64.nz, yin,    \
                     (const cx<TF>*)F, (cx<TO>*)yout, k, nw, sw0h, sdwh, h, pass, j0)
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
