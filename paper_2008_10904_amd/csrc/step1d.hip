// 1-D time-marching kernels: fused RK4 step of a three-point operator and the forcing pre-filter.
//
// Method (Sec. 2.1 last paragraphs, Sec. 2.2, Sec. 2.3): the response to f(t) = sum_j F_j e^{i w_j t} is
// obtained by marching du/dt = L u + f from u = 0.  For a linear autonomous L the classical RK4 step with
// the forcing evaluated at the stage times t, t+h/2, t+h/2, t+h is exactly
//
//     u_{s+1} = P(Z) u_s + sum_j G_j e^{i w_j t_s},   Z = h L,   P(Z) = I + Z + Z^2/2 + Z^3/6 + Z^4/24,
//     G_j     = h Q_j(Z) F_j,  Q_j(Z) = [(1+4a+b) I + (1+2a) Z + (1+a) Z^2/2 + Z^3/4] / 6,
//
// with a = e^{i w_j h/2}, b = e^{i w_j h} (expand the four stages).  For a three-point L, P(Z) is a
// nine-point stencil (radius 4); the host builds it once per operator.  The stepper therefore does ONE
// neighbour exchange and nine complex multiply-adds per unknown and step instead of four exchanges and
// twelve; the forcing sum is a precomputed row of the synthesis GEMM.
//
// Multi-step form: m consecutive steps compose to
//
//     u_{s+m} = P(Z)^m u_s + sum_j e^{i w_j t_s} G_j^(m),   G_j^(m) = sum_{r<m} e^{i w_j r h} P(Z)^(m-1-r) G_j,
//
// so a kernel step of m RK4 steps is one band product with P(Z)^m (radius 4m, built on the host in FP64) plus one
// forcing row synthesised from G^(m) at every m-th step.  G^(m) comes from m-1 Horner passes of P(Z) over G:
// y_0 = G, y_i = P(Z) y_{i-1} + e^{i w_j i h} G.  The dependent chain per m steps is one LDS exchange and one
// band product instead of m of each.
#include "step1d_kernel.h"

namespace res {

template <typename R> __global__ void fill_empty_kernel(typename EmptyMark<R>::U* p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = EmptyMark<R>::bits;
}

// One Horner pass of G = h Q_j(Z) F over [n_w][k][N] (three passes build G):
//   pass 0: y = c3 (Z F) + c2 F      pass 1: y = Z y_in + c1 F      pass 2: G = h (Z y_in + c0 F)
// with c3 = 1/24, c2 = (1+a)/12, c1 = (1+2a)/6, c0 = (1+4a+b)/6, a = e^{i sw_j h/2}, b = a^2, and
// sw_j = sigma w_j (sigma = -1 for the adjoint run).  tri = [N][3] complex (Z's sub, main, super diagonals,
// zero across instance boundaries).
template <typename TF, typename TO>
__global__ __launch_bounds__(256) void tri_horner_kernel(const cx<double>* __restrict__ tri,
                                                         const cx<double>* __restrict__ yin,
                                                         const cx<TF>* __restrict__ F, cx<TO>* __restrict__ yout,
                                                         int64_t N, int32_t k, int32_t nw, double sw0h, double sdwh,
                                                         double h, int pass, int32_t j0) {
  const int64_t total = (int64_t)nw * k * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = e % N;
    const int64_t j = e / ((int64_t)k * N);
    double sa, ca;
    sincos(0.5 * (sw0h + (double)(j0 + j) * sdwh), &sa, &ca);
    const cx<double> a = mk<double>(ca, sa);
    const cx<double> b = cmul(a, a);
    const cx<double> one = mk<double>(1.0, 0.0);
    const cx<double> fz = ccast<double>(F[e]);
    // neighbours of the operand (F on pass 0, y_in afterwards)
    cx<double> xm, x0, xp;
    if (pass == 0) {
      x0 = fz;
      xm = n > 0 ? ccast<double>(F[e - 1]) : mk<double>(0, 0);
      xp = n + 1 < N ? ccast<double>(F[e + 1]) : mk<double>(0, 0);
    } else {
      x0 = yin[e];
      xm = n > 0 ? yin[e - 1] : mk<double>(0, 0);
      xp = n + 1 < N ? yin[e + 1] : mk<double>(0, 0);
    }
    const cx<double> zl = tri[3 * n + 0], zd = tri[3 * n + 1], zu = tri[3 * n + 2];
    cx<double> zx = cmul(zd, x0);
    zx = cfma(zl, xm, zx);
    zx = cfma(zu, xp, zx);
    cx<double> y;
    if (pass == 0) {
      const cx<double> c2 = mk<double>((1.0 + a.re) / 12.0, a.im / 12.0);
      y = cfma(c2, fz, mk<double>(zx.re / 24.0, zx.im / 24.0));
    } else if (pass == 1) {
      const cx<double> c1 = mk<double>((1.0 + 2.0 * a.re) / 6.0, 2.0 * a.im / 6.0);
      y = cfma(c1, fz, zx);
    } else {
      const cx<double> c0 = mk<double>((one.re + 4.0 * a.re + b.re) / 6.0, (4.0 * a.im + b.im) / 6.0);
      y = cfma(c0, fz, zx);
      y = mk<double>(h * y.re, h * y.im);
    }
    yout[e] = ccast<TO>(y);
  }
}

// One pass of the multi-step forcing combination over [n_w][k][N] FP64 blocks:
//   y = P x + e^{i sw_j h i} G,   sw_j = sigma w_j,
// with P = FP64 [N][9] band of P(Z) (or P(Z^H) for the adjoint), zero across instance boundaries.
template <typename TO>
__global__ __launch_bounds__(256) void band_horner_kernel(const cx<double>* __restrict__ band,
                                                          const cx<double>* __restrict__ x,
                                                          const cx<double>* __restrict__ G, cx<TO>* __restrict__ y,
                                                          int64_t N, int32_t k, int32_t nw, double sw0h, double sdwh,
                                                          int i, int32_t j0) {
  const int64_t total = (int64_t)nw * k * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = e % N;
    const int64_t j = e / ((int64_t)k * N);
    cx<double> acc = mk<double>(0, 0);
#pragma unroll
    for (int d = -kBandRadius; d <= kBandRadius; ++d)
      if (n + d >= 0 && n + d < N) acc = cfma(band[n * kBandWidth + d + kBandRadius], x[e + d], acc);
    double sn, cs;
    sincos((double)i * (sw0h + (double)(j0 + j) * sdwh), &sn, &cs);
    acc = cfma(mk<double>(cs, sn), G[e], acc);
    y[e] = ccast<TO>(acc);
  }
}

// ---------------------------------------------------------------------------------------------------------
// launchers (the stepper's own are in step1d_kernel.h)
// ---------------------------------------------------------------------------------------------------------
int launch_fill_empty(void* xbuf, int fp64, int64_t count, hipStream_t st) {
  const int64_t words = 2 * count;  // re and im of `count` complex slots
  const unsigned grid = (unsigned)std::min<int64_t>(1024, (words + 255) / 256);
  if (fp64) hipLaunchKernelGGL(fill_empty_kernel<double>, dim3(grid), dim3(256), 0, st, (EmptyMark<double>::U*)xbuf, words);
  else hipLaunchKernelGGL(fill_empty_kernel<float>, dim3(grid), dim3(256), 0, st, (EmptyMark<float>::U*)xbuf, words);
  return 0;
}

int launch_step1d(const Step1DArgs& a, hipStream_t st) {
  if (a.persist && (a.block <= 0 || a.block % step1d_prefetch(a.cfg) != 0)) return -3;
  switch (a.mstep) {
    case 1: return launch_step1d_ms<1>(a, st);
    case 2: return launch_step1d_m2(a, st);
    case 4: return launch_step1d_m4(a, st);
    default: return -5;
  }
}

int step1d_coresident(int fp64, int cfg, int device, int mstep) {
  switch (mstep) {
    case 1: return step1d_coresident_ms<1>(fp64, cfg, device);
    case 2: return step1d_coresident_m2(fp64, cfg, device);
    case 4: return step1d_coresident_m4(fp64, cfg, device);
    default: return 0;
  }
}

int step1d_prefetch(int cfg) {
  static const int pd[] = {4, 4, 4, 4, 2, 2, 2, 2, 4, 4, 4, 4, 8, 8, 8, 8};
  return (cfg >= 0 && cfg < kStep1DConfigs) ? pd[cfg] : 0;
}

int step1d_capacity(int cfg) {
  static const int cap[] = {64, 128, 256, 512, 1024, 2048, 2048, 2048, 1024, 1024, 512, 256, 256, 512, 128, 512};
  return (cfg >= 0 && cfg < kStep1DConfigs) ? cap[cfg] : 0;
}

int launch_tri_horner(const cx<double>* tri, const cx<double>* yin, const void* F, int f_fp64, void* yout,
                      int out_fp64, int64_t N, int k, int nw, double sw0h, double sdwh, double h, int pass,
                      hipStream_t st, int j0) {
  const int64_t total = (int64_t)nw * k * N;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
#define RES_TH(TF, TO)                                                                                         \
  hipLaunchKernelGGL((tri_horner_kernel<TF, TO>), dim3((unsigned)blocks), dim3(256), 0, st, tri, yin,         \
                     (const cx<TF>*)F, (cx<TO>*)yout, N, k, nw, sw0h, sdwh, h, pass, j0)
  if (f_fp64 && out_fp64) RES_TH(double, double);
  else if (f_fp64 && !out_fp64) RES_TH(double, float);
  else if (!f_fp64 && out_fp64) RES_TH(float, double);
  else RES_TH(float, float);
#undef RES_TH
  return 0;
}


int launch_band_horner(const cx<double>* band, const cx<double>* x, const cx<double>* G, void* y, int out_fp64,
                       int64_t N, int k, int nw, double sw0h, double sdwh, int i, hipStream_t st, int j0) {
  const int64_t total = (int64_t)nw * k * N;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (out_fp64)
    hipLaunchKernelGGL((band_horner_kernel<double>), dim3((unsigned)blocks), dim3(256), 0, st, band, x, G,
                       (cx<double>*)y, N, k, nw, sw0h, sdwh, i, j0);
  else
    hipLaunchKernelGGL((band_horner_kernel<float>), dim3((unsigned)blocks), dim3(256), 0, st, band, x, G,
                       (cx<float>*)y, N, k, nw, sw0h, sdwh, i, j0);
  return 0;
}

}  // namespace res
