// Discrete adjoint of the RK4 march (reverse-mode differentiation of a time-stepped run).  The arithmetic and the
// reaction-field gradient are FP64; the rows (states, stage values, lambda, forcing and seed rows) are stored as T:
// FP64, or FP32 for mixed-precision operators (half the memory and traffic; every value is rounded to FP32 when
// it is stored, as in the forward march).
//
// With Z = h L, K_i = Z y_i + h f_i and the classical stages y_1 = u, y_2 = u + K_1/2, y_3 = u + K_2/2,
// y_4 = u + K_3, u' = u + (K_1 + 2 K_2 + 2 K_3 + K_4)/6, the gradient lambda' = dJ/du' (convention dJ/dRe + i dJ/dIm)
// propagates back as
//
//   Kb_4 = lambda'/6,                 yb_4 = Z^H Kb_4,
//   Kb_3 = lambda'/3 + yb_4,          yb_3 = Z^H Kb_3,
//   Kb_2 = lambda'/3 + yb_3/2,        yb_2 = Z^H Kb_2,
//   Kb_1 = lambda'/6 + yb_2/2,        yb_1 = Z^H Kb_1,
//   lambda = lambda' + yb_4 + yb_3 + yb_2 + yb_1   (+ the projection's injection at sampled steps),
//
// and a real perturbation d mu of L's diagonal (dZ = h diag(d mu)) contributes h Re(conj(Kb_i) y_i) per node and
// stage.  The forward stages y_i are recomputed from the state u_s (from checkpoints).  One launch per stage; a
// thread owns one site (unknown of the three-point operator, or grid node with all its components) and all k
// columns, so the reaction-field gradient of a node is accumulated without atomics.
#include "common.h"
#include "gridz.h"
#include "kernels.h"

namespace res {

// (Z x)[site] for column base x.  KIND 0: three-point complex operator (tri = [N][3]); KIND 1: structured grid.
template <int KIND, int NC, typename T>
__device__ __forceinline__ void zsite(const AdjOpDev& op, const cx<T>* __restrict__ x, int64_t p,
                                      cx<double> out[NC]) {
  if (KIND == 0) {
    const cx<double>* tri = (const cx<double>*)op.tri;
    cx<double> acc = cmul(tri[3 * p + 1], ccast<double>(x[p]));
    if (p > 0) acc = cfma(tri[3 * p], ccast<double>(x[p - 1]), acc);
    if (p + 1 < op.nsite) acc = cfma(tri[3 * p + 2], ccast<double>(x[p + 1]), acc);
    out[0] = acc;
  } else {
    GridCoef<double> c;
    c.cxm = (const double*)op.g.cxm; c.cxp = (const double*)op.g.cxp; c.cym = (const double*)op.g.cym;
    c.cyp = (const double*)op.g.cyp; c.czm = (const double*)op.g.czm; c.czp = (const double*)op.g.czp;
    c.d = (const double*)op.g.d; c.K = (const double*)op.g.K;
    const int64_t nx = op.g.nx, ny = op.g.ny, nz = op.g.nz;
    const int64_t ix = p % nx, l = p / nx, iy = l % ny, iz = l / ny;
    apply_z<double, NC, T>(c, x, op.nsite, nx, ny, nz, ix, iy, iz, p, l, out);
  }
}

// Forward stage m (1..4):  K_m = Z yin + h f;  m=1: yout = u + K_1/2;  m=2: yout = u + K_2/2, acc = K_1 + 2 K_2;
// m=3: yout = u + K_3;  m=4: uout = u + (acc + 2 K_3 + K_4)/6 (uout may equal u).  The earlier stage increments
// are recovered from the stage values, K_1 = 2 (y_2 - u) at m = 2 (yin = y_2) and K_3 = y_4 - u at m = 4
// (yin = y_4), so only stages 2 and 4 touch acc (four fewer rows moved per step).  acc may be null when only the
// stage values are wanted (m < 4); f null means no forcing.  gadd (m = 4, null: none) is added to uout: with f null
// at every stage the step is u' = P(Z) u + gadd, the march with pre-filtered forcing rows.
template <int KIND, int NC, typename T>
__global__ __launch_bounds__(256) void fwd_stage_kernel(AdjOpDev op, int k, int m, const cx<T>* u,
                                                        cx<T>* uout, const cx<T>* __restrict__ yin,
                                                        cx<T>* yout,
                                                        cx<T>* acc, const cx<T>* __restrict__ f, double h,
                                                        const cx<T>* __restrict__ gadd) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= op.nsite) return;
  const int64_t blk = (int64_t)NC * op.nsite;
  for (int b = blockIdx.y; b < k; b += gridDim.y) {  // one column per grid row
    cx<double> z[NC];
    zsite<KIND, NC, T>(op, yin + b * blk, p, z);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int64_t e = b * blk + c * op.nsite + p;
      cx<double> K = z[c];
      if (f != nullptr) {
        const cx<double> fv = ccast<double>(f[e]);
        K.re += h * fv.re;
        K.im += h * fv.im;
      }
      const cx<double> uu = ccast<double>(u[e]);
      if (m == 4) {
        const cx<double> a = ccast<double>(acc[e]), y4 = ccast<double>(yin[e]);
        const double k3r = y4.re - uu.re, k3i = y4.im - uu.im;
        cx<double> un = mk<double>(uu.re + (a.re + 2.0 * k3r + K.re) / 6.0, uu.im + (a.im + 2.0 * k3i + K.im) / 6.0);
        if (gadd != nullptr) {
          const cx<double> g = ccast<double>(gadd[e]);
          un.re += g.re;
          un.im += g.im;
        }
        uout[e] = ccast<T>(un);
      } else {
        const double w = m == 3 ? 1.0 : 0.5;
        yout[e] = ccast<T>(mk<double>(uu.re + w * K.re, uu.im + w * K.im));
        if (acc != nullptr && m == 2) {
          const cx<double> y2 = ccast<double>(yin[e]);
          acc[e] = ccast<T>(mk<double>(2.0 * (y2.re - uu.re) + 2.0 * K.re, 2.0 * (y2.im - uu.im) + 2.0 * K.im));
        }
      }
    }
  }
}

// Reverse stage m (4..1) with opH = Z^H; see the header comment.  lam holds lambda' (read at every stage);
// kin = Kb_m (m < 4), kout = Kb_{m-1} (m > 1); mu row r += h Re(conj(Kb_m) y_m) summed over the columns of grid
// row r (mu [rev_stage_rows(k)][nsite], null: skipped; a node's columns go to separate rows, summed afterwards).  No running sum is
// kept: with yb_4 = Kb_3 - lambda'/3, yb_3 = 2 Kb_2 - 2 lambda'/3 and yb_2 = 2 Kb_1 - lambda'/3, stage 1 forms
// lambda = -lambda'/3 + Kb_3 + 2 Kb_2 + 2 Kb_1 + yb_1 (+ inj, null: none) from k3 = Kb_3 and k2 = Kb_2 into
// lam_out (which must not alias lam, kin, k3 or k2).
template <int KIND, int NC, typename T>
__global__ __launch_bounds__(256) void rev_stage_kernel(AdjOpDev opH, int k, int m,
                                                        const cx<T>* __restrict__ lam,
                                                        cx<T>* __restrict__ lam_out,
                                                        const cx<T>* __restrict__ kin,
                                                        const cx<T>* __restrict__ y, cx<T>* kout,
                                                        const cx<T>* __restrict__ k3,
                                                        const cx<T>* __restrict__ k2, double* __restrict__ mu,
                                                        const cx<T>* __restrict__ inj, double h) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= opH.nsite) return;
  const int64_t blk = (int64_t)NC * opH.nsite;
  double musum = 0.0;
  for (int b = blockIdx.y; b < k; b += gridDim.y) {  // one column per grid row
    cx<double> z[NC];
    zsite<KIND, NC, T>(opH, (m == 4 ? lam : kin) + b * blk, p, z);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int64_t e = b * blk + c * opH.nsite + p;
      const cx<double> lp = ccast<double>(lam[e]);
      cx<double> kb;  // Kb_m at this point
      if (m == 4) {
        kb = mk<double>(lp.re / 6.0, lp.im / 6.0);
        kout[e] = ccast<T>(mk<double>(lp.re / 3.0 + z[c].re / 6.0, lp.im / 3.0 + z[c].im / 6.0));  // Z^H (lambda'/6)
      } else {
        kb = ccast<double>(kin[e]);
        if (m == 1) {
          const cx<double> a3 = ccast<double>(k3[e]), a2 = ccast<double>(k2[e]);
          cx<double> l = mk<double>(a3.re + 2.0 * (a2.re + kb.re) - lp.re / 3.0 + z[c].re,
                                    a3.im + 2.0 * (a2.im + kb.im) - lp.im / 3.0 + z[c].im);
          if (inj != nullptr) {
            const cx<double> q = ccast<double>(inj[e]);
            l.re += q.re;
            l.im += q.im;
          }
          lam_out[e] = ccast<T>(l);
        } else {
          const double w = m == 3 ? 1.0 / 3.0 : 1.0 / 6.0;
          kout[e] = ccast<T>(mk<double>(w * lp.re + 0.5 * z[c].re, w * lp.im + 0.5 * z[c].im));
        }
      }
      if (mu != nullptr) {
        const cx<double> yy = ccast<double>(y[e]);
        musum += kb.re * yy.re + kb.im * yy.im;  // Re(conj(kb) y)
      }
    }
  }
  if (mu != nullptr) mu[blockIdx.y * opH.nsite + p] += h * musum;
}

// ---------------------------------------------------------------------------------------------------------
int launch_fwd_stage(const AdjOpDev& op, int k, int m, const void* u, void* uout, const void* yin, void* yout,
                     void* acc, const void* f, double h, hipStream_t st, const void* gadd, int rows64) {
  const dim3 grid((unsigned)((op.nsite + 255) / 256), (unsigned)std::min(k, 65535));
#define RES_F(KIND, NC, T)                                                                                       \
  hipLaunchKernelGGL((fwd_stage_kernel<KIND, NC, T>), grid, dim3(256), 0, st, op, k, m, (const cx<T>*)u,        \
                     (cx<T>*)uout, (const cx<T>*)yin, (cx<T>*)yout, (cx<T>*)acc, (const cx<T>*)f, h,             \
                     (const cx<T>*)gadd)
#define RES_F2(T)                      \
  if (op.kind == 0) RES_F(0, 1, T);    \
  else if (op.ncomp == 3) RES_F(1, 3, T); \
  else RES_F(1, 1, T)
  if (rows64) { RES_F2(double); }
  else { RES_F2(float); }
#undef RES_F2
#undef RES_F
  return 0;
}

// The four forward stages of one step in one launch, for a 2-D one-component grid operator: a 64 x 16 tile of the
// state with a halo of four sites (the reach of four stencil applications) sits in LDS; stage m computes the
// padded-tile sites [m, P - m) from the previous stage's values, so the last stage covers the tile.  Writes the
// stage inputs y2, y3, y4 and the new state uout on the tile (each may be null; uout null: the three stages only),
// adding the row gadd to uout when given.
// The stage values are those of fwd_stage_kernel (same operand order); the RK4 accumulator keeps the increments
// K_m themselves instead of recovering K_1 and K_3 from stage values.  Out-of-domain sites hold zero.  uout must not alias u (neighbouring tiles read u's halo).
//
// Each of the 1,024 threads owns one tile site (its RK4 accumulator stays in a register) and at most one site of
// the halo ring of the current stage (516 sites at most).  The stage values live in one LDS buffer updated in
// place: every thread computes its sites from the buffer, then all write after a barrier.  With the state tile,
// 55 KB of LDS: two workgroups per CU.
constexpr int kFsTX = 64, kFsTY = 16, kFsH = 4, kFsPX = kFsTX + 2 * kFsH, kFsPY = kFsTY + 2 * kFsH;

// Ring site i (< ring count) of stage m: the region [m, P - m) minus the tile, as a top band, a bottom band and the
// left and right bands of the tile rows.
__device__ __forceinline__ void ring_site(int m, int i, int* py, int* px) {
  const int band = kFsH - m, wx = kFsPX - 2 * m, ntop = band * wx;
  if (i < ntop) {
    *py = m + i / wx;
    *px = m + i % wx;
  } else if (i < 2 * ntop) {
    const int j = i - ntop;
    *py = kFsH + kFsTY + j / wx;
    *px = m + j % wx;
  } else {
    const int j = i - 2 * ntop, row = j / (2 * band), c = j % (2 * band);
    *py = kFsH + row;
    *px = c < band ? m + c : kFsH + kFsTX + (c - band);
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void fwd_step2d_kernel(GridCoef<double> Cf, int64_t nx, int64_t ny,
                                                          const cx<T>* __restrict__ u, cx<T>* uout,
                                                          cx<T>* y2o, cx<T>* y3o, cx<T>* y4o,
                                                          const cx<T>* __restrict__ fa,
                                                          const cx<T>* __restrict__ fb,
                                                          const cx<T>* __restrict__ fc, double h,
                                                          const cx<T>* __restrict__ gadd) {
  __shared__ cx<double> U[kFsPY][kFsPX], Y[kFsPY][kFsPX];
  const int64_t nodes = nx * ny;
  const int64_t col = blockIdx.z;
  const int64_t gx0 = (int64_t)blockIdx.x * kFsTX - kFsH, gy0 = (int64_t)blockIdx.y * kFsTY - kFsH;
  const cx<double> zero = mk<double>(0.0, 0.0);
  for (int i = threadIdx.x; i < kFsPX * kFsPY; i += blockDim.x) {
    const int py = i / kFsPX, px = i - py * kFsPX;
    const int64_t gx = gx0 + px, gy = gy0 + py;
    const cx<double> v =
        (gx >= 0 && gx < nx && gy >= 0 && gy < ny) ? ccast<double>(u[col * nodes + gy * nx + gx]) : zero;
    U[py][px] = v;
    Y[py][px] = v;
  }
  __syncthreads();
  const int t = threadIdx.x;
  const int tpy = kFsH + t / kFsTX, tpx = kFsH + t % kFsTX;  // the thread's tile site
  cx<double> acc = zero;
  // K = Z x + h f at padded site (py, px) of the LDS buffer x (apply_z order: diagonal, x-, x+, y-, y+)
  auto stage_k = [&](cx<double>(*X)[kFsPX], const cx<T>* f, int py, int px, int64_t gx, int64_t gy) {
    const int64_t p = gy * nx + gx;
    const double dd = Cf.d[p], cxm = Cf.cxm[gy], cxp = Cf.cxp[gy], cym = Cf.cym[gy], cyp = Cf.cyp[gy];
    const cx<double> sv = X[py][px];
    cx<double> K = mk<double>(dd * sv.re, dd * sv.im);
    if (gx > 0) { const cx<double> q = X[py][px - 1]; K.re += cxm * q.re; K.im += cxm * q.im; }
    if (gx + 1 < nx) { const cx<double> q = X[py][px + 1]; K.re += cxp * q.re; K.im += cxp * q.im; }
    if (gy > 0) { const cx<double> q = X[py - 1][px]; K.re += cym * q.re; K.im += cym * q.im; }
    if (gy + 1 < ny) { const cx<double> q = X[py + 1][px]; K.re += cyp * q.re; K.im += cyp * q.im; }
    if (f != nullptr) {
      const cx<double> fv = ccast<double>(f[col * nodes + p]);
      K.re += h * fv.re;
      K.im += h * fv.im;
    }
    return K;
  };
  const int mlast = uout != nullptr ? 4 : 3;
  for (int m = 1; m <= mlast; ++m) {
    const cx<T>* f = m == 1 ? fa : (m == 4 ? fc : fb);
    cx<T>* go = m == 1 ? y2o : (m == 2 ? y3o : (m == 3 ? y4o : uout));
    const double w = m == 3 ? 1.0 : 0.5;
    // the tile site
    const int64_t gx = gx0 + tpx, gy = gy0 + tpy;
    const bool tin = gx < nx && gy < ny;  // tile sites are never left of or above the domain
    cx<double> tv = zero;
    if (tin) {
      const cx<double> K = stage_k(Y, f, tpy, tpx, gx, gy);
      const cx<double> uu = U[tpy][tpx];
      if (m < 4) {
        tv = mk<double>(uu.re + w * K.re, uu.im + w * K.im);
        acc = m == 1 ? K : mk<double>(acc.re + 2.0 * K.re, acc.im + 2.0 * K.im);
      } else {
        tv = mk<double>(uu.re + (acc.re + K.re) / 6.0, uu.im + (acc.im + K.im) / 6.0);
        if (gadd != nullptr) {
          const cx<double> g = ccast<double>(gadd[col * nodes + gy * nx + gx]);
          tv.re += g.re;
          tv.im += g.im;
        }
      }
    }
    // one ring site (stages 1..3)
    const int band = kFsH - m;
    const int nring = 2 * band * (kFsPX - 2 * m) + 2 * band * kFsTY;
    int rpy = 0, rpx = 0;
    const bool has_ring = m < 4 && t < nring;
    cx<double> rv = zero;
    if (has_ring) {
      ring_site(m, t, &rpy, &rpx);
      const int64_t rgx = gx0 + rpx, rgy = gy0 + rpy;
      if (rgx >= 0 && rgx < nx && rgy >= 0 && rgy < ny) {
        const cx<double> K = stage_k(Y, f, rpy, rpx, rgx, rgy);
        const cx<double> uu = U[rpy][rpx];
        rv = mk<double>(uu.re + w * K.re, uu.im + w * K.im);
      }
    }
    __syncthreads();  // every read of the stage's operand is done
    if (m < 4) {
      Y[tpy][tpx] = tv;
      if (has_ring) Y[rpy][rpx] = rv;
    }
    if (tin && go != nullptr) go[col * nodes + gy * nx + gx] = ccast<T>(tv);
    __syncthreads();
  }
}

// The four reverse stages of one step in one launch, for a 2-D one-component grid operator (the recursion of the
// header comment, with opH's coefficients of Z^H): a 64 x 16 tile of lambda' with a halo of four sites in LDS;
// step s = 1..4 (stage m = 5 - s) applies Z^H on the padded sites [s, P - s), from lambda'/6 (s = 1) or the
// previous Kb (updated in place in one LDS buffer, as in fwd_step2d_kernel); the running sum lambda' + sum yb and
// the mu contributions h Re(conj(Kb_m) y_m) stay in registers on the tile.  One workgroup per tile and column; a
// node's mu contributions of the step are summed over the stages and added to the column's own partial row
// mu_cols[column][node] (summed over the columns once at the end, without atomics).  lam_out must not alias lam.
template <typename T>
__global__ __launch_bounds__(1024) void rev_step2d_kernel(GridCoef<double> Cf, int64_t nx, int64_t ny,
                                                          const cx<T>* __restrict__ lam, cx<T>* lam_out,
                                                          const cx<T>* __restrict__ y2,
                                                          const cx<T>* __restrict__ y3,
                                                          const cx<T>* __restrict__ y4,
                                                          const cx<T>* __restrict__ u, double* mu_cols,
                                                          const cx<T>* __restrict__ inj, double h) {
  __shared__ cx<double> L[kFsPY][kFsPX], KB[kFsPY][kFsPX];
  double* mu = mu_cols != nullptr ? mu_cols + (int64_t)blockIdx.z * nx * ny : nullptr;
  const int64_t nodes = nx * ny;
  const int64_t gx0 = (int64_t)blockIdx.x * kFsTX - kFsH, gy0 = (int64_t)blockIdx.y * kFsTY - kFsH;
  const cx<double> zero = mk<double>(0.0, 0.0);
  const int t = threadIdx.x;
  const int tpy = kFsH + t / kFsTX, tpx = kFsH + t % kFsTX;
  const int64_t tgx = gx0 + tpx, tgy = gy0 + tpy;
  const bool tin = tgx < nx && tgy < ny;  // tile sites are never left of or above the domain
  const int64_t tp = tgy * nx + tgx;
  // (Z^H x)(site) from an LDS buffer (apply_z order: diagonal, x-, x+, y-, y+)
  auto zh = [&](cx<double>(*X)[kFsPX], int py, int px, int64_t gx, int64_t gy) {
    const int64_t p = gy * nx + gx;
    const double dd = Cf.d[p], cxm = Cf.cxm[gy], cxp = Cf.cxp[gy], cym = Cf.cym[gy], cyp = Cf.cyp[gy];
    const cx<double> sv = X[py][px];
    cx<double> z = mk<double>(dd * sv.re, dd * sv.im);
    if (gx > 0) { const cx<double> q = X[py][px - 1]; z.re += cxm * q.re; z.im += cxm * q.im; }
    if (gx + 1 < nx) { const cx<double> q = X[py][px + 1]; z.re += cxp * q.re; z.im += cxp * q.im; }
    if (gy > 0) { const cx<double> q = X[py - 1][px]; z.re += cym * q.re; z.im += cym * q.im; }
    if (gy + 1 < ny) { const cx<double> q = X[py + 1][px]; z.re += cyp * q.re; z.im += cyp * q.im; }
    return z;
  };
  // Kb_{m-1} at a site from y_bar_m = z and lambda' (step s = 5 - m; s = 4 produces lambda instead)
  auto next_kb = [&](int s, cx<double> lp, cx<double> z) {
    const double wl = s == 1 ? 1.0 / 3.0 : (s == 2 ? 1.0 / 3.0 : 1.0 / 6.0);
    const double wz = s == 1 ? 1.0 : 0.5;
    return mk<double>(wl * lp.re + wz * z.re, wl * lp.im + wz * z.im);
  };
  double musum = 0.0;
  {
    const int64_t cb = (int64_t)blockIdx.z * nodes;
    for (int i = t; i < kFsPX * kFsPY; i += blockDim.x) {
      const int py = i / kFsPX, px = i - py * kFsPX;
      const int64_t gx = gx0 + px, gy = gy0 + py;
      L[py][px] = (gx >= 0 && gx < nx && gy >= 0 && gy < ny) ? ccast<double>(lam[cb + gy * nx + gx]) : zero;
    }
    __syncthreads();
    cx<double> ub = zero;
    for (int s = 1; s <= 4; ++s) {
      cx<double>(*X)[kFsPX] = s == 1 ? L : KB;
      const double xs = s == 1 ? 1.0 / 6.0 : 1.0;  // Kb_4 = lambda'/6
      const cx<T>* ys = s == 1 ? y4 : (s == 2 ? y3 : (s == 3 ? y2 : u));
      cx<double> tv = zero;
      if (tin) {
        const cx<double> lp = L[tpy][tpx];
        cx<double> z = zh(X, tpy, tpx, tgx, tgy);
        z = mk<double>(xs * z.re, xs * z.im);
        const cx<double> kx = X[tpy][tpx];
        const cx<double> kb = mk<double>(xs * kx.re, xs * kx.im);  // Kb_m at the tile site
        if (mu != nullptr) {
          const cx<double> yy = ccast<double>(ys[cb + tp]);
          musum += kb.re * yy.re + kb.im * yy.im;
        }
        if (s == 1) ub = mk<double>(lp.re + z.re, lp.im + z.im);
        else ub = mk<double>(ub.re + z.re, ub.im + z.im);
        tv = s < 4 ? next_kb(s, lp, z) : ub;
      }
      const int band = kFsH - s;
      const int nring = s < 4 ? 2 * band * (kFsPX - 2 * s) + 2 * band * kFsTY : 0;
      int rpy = 0, rpx = 0;
      const bool has_ring = t < nring;
      cx<double> rv = zero;
      if (has_ring) {
        ring_site(s, t, &rpy, &rpx);
        const int64_t rgx = gx0 + rpx, rgy = gy0 + rpy;
        if (rgx >= 0 && rgx < nx && rgy >= 0 && rgy < ny) {
          cx<double> z = zh(X, rpy, rpx, rgx, rgy);
          z = mk<double>(xs * z.re, xs * z.im);
          rv = next_kb(s, L[rpy][rpx], z);
        }
      }
      __syncthreads();  // every read of the step's operand is done
      if (s < 4) {
        KB[tpy][tpx] = tv;
        if (has_ring) KB[rpy][rpx] = rv;
      } else if (tin) {
        cx<double> l = tv;
        if (inj != nullptr) {
          const cx<double> q = ccast<double>(inj[cb + tp]);
          l.re += q.re;
          l.im += q.im;
        }
        lam_out[cb + tp] = ccast<T>(l);
      }
      __syncthreads();
    }
  }
  if (mu != nullptr && tin) mu[tp] += h * musum;
}

int launch_rev_step2d(const AdjOpDev& opH, int k, const void* lam, void* lam_out, const void* y2, const void* y3,
                      const void* y4, const void* u, double* mu_cols, const void* inj, double h, hipStream_t st,
                      int rows64) {
  if (opH.kind != 1 || opH.ncomp != 1 || opH.g.nz != 1 || k < 1 || k > 65535 || lam_out == lam) return -1;
  GridCoef<double> c;
  c.cxm = (const double*)opH.g.cxm; c.cxp = (const double*)opH.g.cxp; c.cym = (const double*)opH.g.cym;
  c.cyp = (const double*)opH.g.cyp; c.czm = (const double*)opH.g.czm; c.czp = (const double*)opH.g.czp;
  c.d = (const double*)opH.g.d; c.K = (const double*)opH.g.K;
  const dim3 grid((unsigned)((opH.g.nx + kFsTX - 1) / kFsTX), (unsigned)((opH.g.ny + kFsTY - 1) / kFsTY),
                  (unsigned)k);
#define RES_RS(T)                                                                                                \
  hipLaunchKernelGGL(rev_step2d_kernel<T>, grid, dim3(1024), 0, st, c, opH.g.nx, opH.g.ny, (const cx<T>*)lam,     \
                     (cx<T>*)lam_out, (const cx<T>*)y2, (const cx<T>*)y3, (const cx<T>*)y4, (const cx<T>*)u,      \
                     mu_cols, (const cx<T>*)inj, h)
  if (rows64) RES_RS(double);
  else RES_RS(float);
#undef RES_RS
  return 0;
}

// mu[p] += sum_b cols[b][p] (b < k, in order).
__global__ __launch_bounds__(256) void sum_columns_kernel(const double* __restrict__ cols, int k, int64_t n,
                                                          double* __restrict__ mu) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < k; ++b) s += cols[(int64_t)b * n + p];
    mu[p] += s;
  }
}

int launch_sum_columns(const double* cols, int k, int64_t n, double* mu, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) return 0;
  hipLaunchKernelGGL(sum_columns_kernel, dim3((unsigned)blocks), dim3(256), 0, st, cols, k, n, mu);
  return 0;
}

int launch_fwd_step2d(const AdjOpDev& op, int k, const void* u, void* uout, void* y2, void* y3, void* y4,
                      const void* fa, const void* fb, const void* fc, double h, hipStream_t st, const void* gadd,
                      int rows64) {
  if (op.kind != 1 || op.ncomp != 1 || op.g.nz != 1 || k < 1 || k > 65535 || (uout != nullptr && uout == u))
    return -1;
  GridCoef<double> c;
  c.cxm = (const double*)op.g.cxm; c.cxp = (const double*)op.g.cxp; c.cym = (const double*)op.g.cym;
  c.cyp = (const double*)op.g.cyp; c.czm = (const double*)op.g.czm; c.czp = (const double*)op.g.czp;
  c.d = (const double*)op.g.d; c.K = (const double*)op.g.K;
  const dim3 grid((unsigned)((op.g.nx + kFsTX - 1) / kFsTX), (unsigned)((op.g.ny + kFsTY - 1) / kFsTY), (unsigned)k);
#define RES_FS(T)                                                                                                \
  hipLaunchKernelGGL(fwd_step2d_kernel<T>, grid, dim3(1024), 0, st, c, op.g.nx, op.g.ny, (const cx<T>*)u,         \
                     (cx<T>*)uout, (cx<T>*)y2, (cx<T>*)y3, (cx<T>*)y4, (const cx<T>*)fa, (const cx<T>*)fb,          \
                     (const cx<T>*)fc, h, (const cx<T>*)gadd)
  if (rows64) RES_FS(double);
  else RES_FS(float);
#undef RES_FS
  return 0;
}

int rev_stage_rows(int k) { return std::min(k, 65535); }

int launch_rev_stage(const AdjOpDev& opH, int k, int m, const void* lam, void* lam_out, const void* kin,
                     const void* y, void* kout, const void* k3, const void* k2, double* mu, const void* inj, double h,
                     hipStream_t st, int rows64) {
  const dim3 grid((unsigned)((opH.nsite + 255) / 256), (unsigned)rev_stage_rows(k));
#define RES_R(KIND, NC, T)                                                                                         \
  hipLaunchKernelGGL((rev_stage_kernel<KIND, NC, T>), grid, dim3(256), 0, st, opH, k, m, (const cx<T>*)lam,     \
                     (cx<T>*)lam_out, (const cx<T>*)kin, (const cx<T>*)y, (cx<T>*)kout, (const cx<T>*)k3,         \
                     (const cx<T>*)k2, mu, (const cx<T>*)inj, h)
#define RES_R2(T)                      \
  if (opH.kind == 0) RES_R(0, 1, T);   \
  else if (opH.ncomp == 3) RES_R(1, 3, T); \
  else RES_R(1, 1, T)
  if (rows64) { RES_R2(double); }
  else { RES_R2(float); }
#undef RES_R2
#undef RES_R
  return 0;
}

}  // namespace res
