// Kernels of the transient-response method with time-domain hand-off (Sec. 2.2, App. B, App. C).
//
// A signal is a series of samples [n][ncols] (working precision, ncols = k N): sample i is the signal at
// t_i = i * every * h.  The run forced by it is the ordinary 1-D stepper fed with one forcing row per RK4 step;
// the rows come from the stage-forcing pre-filter below, which interpolates the samples at the stage times.
#include "common.h"
#include "gridz.h"
#include "kernels.h"

namespace res {

// Sample j of a series read forward or in reversed order (the adjoint run marches the reversed signal).
template <typename TS>
__device__ __forceinline__ cx<double> sample(const cx<TS>* __restrict__ S, int64_t n, int64_t ncols, int64_t col,
                                             int64_t j, int rev) {
  const int64_t r = rev ? n - 1 - j : j;
  return ccast<double>(S[r * ncols + col]);
}

// First and second derivatives per sample interval at sample j (App. C): second-order central differences for
// the cubic scheme; five-point central differences for the quintic scheme, second-order central ones at the
// samples next to the ends; at the two end samples a first-order one-sided first derivative and (quintic) a zero
// second derivative.
template <typename TS>
__device__ __forceinline__ void sample_slopes(const cx<TS>* __restrict__ S, int64_t n, int64_t ncols, int64_t col,
                                              int64_t j, int rev, int scheme, cx<double>* d, cx<double>* dd) {
  *dd = mk<double>(0.0, 0.0);
  if (j == 0) {
    const cx<double> a = sample(S, n, ncols, col, 0, rev), b = sample(S, n, ncols, col, 1, rev);
    *d = mk<double>(b.re - a.re, b.im - a.im);
    return;
  }
  if (j == n - 1) {
    const cx<double> a = sample(S, n, ncols, col, n - 2, rev), b = sample(S, n, ncols, col, n - 1, rev);
    *d = mk<double>(b.re - a.re, b.im - a.im);
    return;
  }
  const cx<double> m1 = sample(S, n, ncols, col, j - 1, rev), p1 = sample(S, n, ncols, col, j + 1, rev);
  if (scheme == 1 || j == 1 || j == n - 2) {
    *d = mk<double>(0.5 * (p1.re - m1.re), 0.5 * (p1.im - m1.im));
    if (scheme == 2) {
      const cx<double> c = sample(S, n, ncols, col, j, rev);
      *dd = mk<double>(p1.re - 2.0 * c.re + m1.re, p1.im - 2.0 * c.im + m1.im);
    }
    return;
  }
  const cx<double> m2 = sample(S, n, ncols, col, j - 2, rev), p2 = sample(S, n, ncols, col, j + 2, rev);
  const cx<double> c = sample(S, n, ncols, col, j, rev);
  *d = mk<double>((m2.re - 8.0 * m1.re + 8.0 * p1.re - p2.re) / 12.0, (m2.im - 8.0 * m1.im + 8.0 * p1.im - p2.im) / 12.0);
  *dd = mk<double>((-m2.re + 16.0 * m1.re - 30.0 * c.re + 16.0 * p1.re - p2.re) / 12.0,
                   (-m2.im + 16.0 * m1.im - 30.0 * c.im + 16.0 * p1.im - p2.im) / 12.0);
}

// The signal at half step q2 (time q2 h / 2) by linear (scheme 0), cubic Hermite (1) or quintic Hermite (2)
// interpolation between samples.
template <typename TS>
__device__ cx<double> signal_at(const cx<TS>* __restrict__ S, int64_t n, int64_t ncols, int64_t col, int64_t q2,
                                int every, int scheme, int rev) {
  const int64_t per = 2 * (int64_t)every;  // half steps per sample interval
  int64_t i = q2 / per;
  double u = (double)(q2 - i * per) / (double)per;
  if (i >= n - 1) {
    i = n - 2;
    u = 1.0;
  }
  const cx<double> p0 = sample(S, n, ncols, col, i, rev), p1 = sample(S, n, ncols, col, i + 1, rev);
  if (scheme == 0) return mk<double>((1.0 - u) * p0.re + u * p1.re, (1.0 - u) * p0.im + u * p1.im);
  cx<double> d0, d1, dd0, dd1;
  sample_slopes(S, n, ncols, col, i, rev, scheme, &d0, &dd0);
  sample_slopes(S, n, ncols, col, i + 1, rev, scheme, &d1, &dd1);
  const double u2 = u * u, u3 = u2 * u;
  double a0, a1, a2 = 0.0, b0, b1, b2 = 0.0;  // weights of p0, d0, dd0, p1, d1, dd1
  if (scheme == 1) {
    a0 = 2.0 * u3 - 3.0 * u2 + 1.0;
    a1 = u3 - 2.0 * u2 + u;
    b0 = 3.0 * u2 - 2.0 * u3;
    b1 = u3 - u2;
  } else {
    const double u4 = u3 * u, u5 = u4 * u;
    a0 = 1.0 - 10.0 * u3 + 15.0 * u4 - 6.0 * u5;
    a1 = u - 6.0 * u3 + 8.0 * u4 - 3.0 * u5;
    a2 = 0.5 * (u2 - 3.0 * u3 + 3.0 * u4 - u5);
    b0 = 10.0 * u3 - 15.0 * u4 + 6.0 * u5;
    b1 = -4.0 * u3 + 7.0 * u4 - 3.0 * u5;
    b2 = 0.5 * (u3 - 2.0 * u4 + u5);
  }
  return mk<double>(a0 * p0.re + a1 * d0.re + a2 * dd0.re + b0 * p1.re + b1 * d1.re + b2 * dd1.re,
                    a0 * p0.im + a1 * d0.im + a2 * dd0.im + b0 * p1.im + b1 * d1.im + b2 * dd1.im);
}

// One pass of the stage-forcing pre-filter.  Classical RK4 on du/dt = L u + f with stage forcing f_a = f(t),
// f_b = f(t + h/2), f_c = f(t + h) adds, with Z = h L,
//     g = (h/6) [ f_a + 4 f_b + f_c + Z (f_a + 2 f_b + Z ((f_a + f_b)/2 + Z f_a / 4)) ],
// evaluated from the inside out: pass 0 writes x2 = (f_a + f_b)/2 + Z f_a / 4, pass 1 x1 = f_a + 2 f_b + Z x2
// (both FP64), pass 2 the forcing row g (working precision).  Rows r < rows are steps s0 + r.
template <typename TS, typename TO>
__global__ __launch_bounds__(256) void signal_prefilter_kernel(const cx<TS>* __restrict__ S, int64_t n, int every,
                                                               int scheme, int rev, const cx<double>* __restrict__ tri,
                                                               const cx<double>* __restrict__ xin,
                                                               cx<double>* __restrict__ xout, cx<TO>* __restrict__ g,
                                                               int64_t s0, int64_t rows, int64_t N, int64_t ncols,
                                                               double h, int pass) {
  const int64_t total = rows * ncols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ncols, col = e - r * ncols;
    const int64_t node = col % N;
    const int64_t q2 = 2 * (s0 + r);  // half step of the stage time t
    const cx<double> zl = tri[3 * node + 0], zd = tri[3 * node + 1], zu = tri[3 * node + 2];
    const bool has_m = node > 0, has_p = node + 1 < N;
    const cx<double> fa = signal_at(S, n, ncols, col, q2, every, scheme, rev);
    const cx<double> fb = signal_at(S, n, ncols, col, q2 + 1, every, scheme, rev);
    cx<double> xm, x0, xp;  // operand of Z at node - 1, node, node + 1
    if (pass == 0) {
      x0 = fa;
      xm = has_m ? signal_at(S, n, ncols, col - 1, q2, every, scheme, rev) : mk<double>(0.0, 0.0);
      xp = has_p ? signal_at(S, n, ncols, col + 1, q2, every, scheme, rev) : mk<double>(0.0, 0.0);
    } else {
      x0 = xin[e];
      xm = has_m ? xin[e - 1] : mk<double>(0.0, 0.0);
      xp = has_p ? xin[e + 1] : mk<double>(0.0, 0.0);
    }
    cx<double> zx = cmul(zd, x0);
    zx = cfma(zl, xm, zx);
    zx = cfma(zu, xp, zx);
    if (pass == 0) {
      xout[e] = mk<double>(0.5 * (fa.re + fb.re) + 0.25 * zx.re, 0.5 * (fa.im + fb.im) + 0.25 * zx.im);
    } else if (pass == 1) {
      xout[e] = mk<double>(fa.re + 2.0 * fb.re + zx.re, fa.im + 2.0 * fb.im + zx.im);
    } else {
      const cx<double> fc = signal_at(S, n, ncols, col, q2 + 2, every, scheme, rev);
      const double c = h / 6.0;
      g[e] = ccast<TO>(mk<double>(c * (fa.re + 4.0 * fb.re + fc.re + zx.re), c * (fa.im + 4.0 * fb.im + fc.im + zx.im)));
    }
  }
}

int launch_signal_prefilter(const void* S, int64_t n, int every, int scheme, int rev, const cx<double>* tri,
                            const void* xin, void* xout, void* g, int fp64, int g_fp64, int64_t s0, int64_t rows,
                            int64_t N, int64_t ncols, double h, int pass, hipStream_t st) {
  int64_t blocks = (rows * ncols + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) return 0;
#define RES_SP(TS, TO)                                                                                           \
  hipLaunchKernelGGL((signal_prefilter_kernel<TS, TO>), dim3((unsigned)blocks), dim3(256), 0, st,                \
                     (const cx<TS>*)S, n, every, scheme, rev, tri, (const cx<double>*)xin, (cx<double>*)xout,     \
                     (cx<TO>*)g, s0, rows, N, ncols, h, pass)
  if (fp64) RES_SP(double, double);
  else if (g_fp64) RES_SP(float, double);
  else RES_SP(float, float);
#undef RES_SP
  return 0;
}

// One pass of the combined forcing of M steps (the multi-step march of a signal run): with the per-step rows g_s
// (FP64) and the band of P(Z) (FP64 [N][9], zero across instance boundaries), kernel step R needs
//     g^(M)_R = sum_{r<M} P^{M-1-r} g_{RM + r},
// built by Horner passes y_0 = g_{RM}, y_i = P y_{i-1} + g_{RM+i}.  Pass i reads y_{i-1} from rows R * xstride of
// xin (xstride = M with xin = g for i = 1, else 1) and writes y_i to out (working precision on the last pass).
template <typename TO>
__global__ __launch_bounds__(256) void row_horner_kernel(const cx<double>* __restrict__ band,
                                                         const cx<double>* __restrict__ xin, int64_t xstride,
                                                         const cx<double>* __restrict__ g, int M, int i,
                                                         cx<TO>* __restrict__ out, int64_t rows, int64_t N,
                                                         int64_t ncols) {
  const int64_t total = rows * ncols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t R = e / ncols, c = e - R * ncols;
    const int64_t n = c % N;
    const cx<double>* xr = xin + R * xstride * ncols;
    cx<double> acc = g[(R * M + i) * ncols + c];
#pragma unroll
    for (int d = -kBandRadius; d <= kBandRadius; ++d)
      if (n + d >= 0 && n + d < N) acc = cfma(band[n * kBandWidth + d + kBandRadius], xr[c + d], acc);
    out[e] = ccast<TO>(acc);
  }
}

int launch_row_horner(const cx<double>* band, const void* xin, int64_t xstride, const void* g, int M, int i,
                      void* out, int out_fp64, int64_t rows, int64_t N, int64_t ncols, hipStream_t st) {
  int64_t blocks = (rows * ncols + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) return 0;
  if (out_fp64)
    hipLaunchKernelGGL((row_horner_kernel<double>), dim3((unsigned)blocks), dim3(256), 0, st, band,
                       (const cx<double>*)xin, xstride, (const cx<double>*)g, M, i, (cx<double>*)out, rows, N, ncols);
  else
    hipLaunchKernelGGL((row_horner_kernel<float>), dim3((unsigned)blocks), dim3(256), 0, st, band,
                       (const cx<double>*)xin, xstride, (const cx<double>*)g, M, i, (cx<float>*)out, rows, N, ncols);
  return 0;
}

// ---- grid operators ------------------------------------------------------------------------------------------
// The signal at the half steps of a tile, H[q][c] = f((2 s0 + q) h / 2) for q < nhalf (FP64).
template <typename TS>
__global__ __launch_bounds__(256) void signal_half_rows_kernel(const cx<TS>* __restrict__ S, int64_t n, int every,
                                                               int scheme, int rev, cx<double>* __restrict__ H,
                                                               int64_t s0, int64_t nhalf, int64_t ncols) {
  const int64_t total = nhalf * ncols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = e / ncols, c = e - q * ncols;
    H[e] = signal_at(S, n, ncols, c, 2 * s0 + q, every, scheme, rev);
  }
}

int launch_signal_half_rows(const void* S, int64_t n, int every, int scheme, int rev, int fp64, void* H, int64_t s0,
                            int64_t nhalf, int64_t ncols, hipStream_t st) {
  int64_t blocks = (nhalf * ncols + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) return 0;
  if (fp64)
    hipLaunchKernelGGL((signal_half_rows_kernel<double>), dim3((unsigned)blocks), dim3(256), 0, st,
                       (const cx<double>*)S, n, every, scheme, rev, (cx<double>*)H, s0, nhalf, ncols);
  else
    hipLaunchKernelGGL((signal_half_rows_kernel<float>), dim3((unsigned)blocks), dim3(256), 0, st,
                       (const cx<float>*)S, n, every, scheme, rev, (cx<double>*)H, s0, nhalf, ncols);
  return 0;
}

// One pass of the stage-forcing pre-filter (the same three passes as signal_prefilter_kernel) for a grid operator:
// f_a, f_b, f_c of row r are the half-step rows 2r, 2r + 1, 2r + 2 of H, and Z is the grid stencil (FP64
// coefficients).  Workgroup (x, y, z) = (node block, column, row).
template <typename TO, int NC>
__global__ __launch_bounds__(256) void grid_signal_pass_kernel(GridCoef<double> Cf, int64_t nx, int64_t ny, int64_t nz,
                                                               const cx<double>* __restrict__ H,
                                                               const cx<double>* __restrict__ xin,
                                                               cx<double>* __restrict__ xout, cx<TO>* __restrict__ g,
                                                               int k, double h, int pass) {
  const int64_t nodes = nx * ny * nz;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= nodes) return;
  const int64_t ix = p % nx, l = p / nx, iy = l % ny, iz = l / ny;
  const int64_t blk = (int64_t)NC * nodes, ncols = (int64_t)k * blk;
  const int64_t b = blockIdx.y, r = blockIdx.z;
  const cx<double>* fa = H + (2 * r) * ncols + b * blk;
  const cx<double>* fb = fa + ncols;
  const cx<double>* x = pass == 0 ? fa : xin + r * ncols + b * blk;
  cx<double> zx[NC];
  apply_z<double, NC>(Cf, x, nodes, nx, ny, nz, ix, iy, iz, p, l, zx);
  const int64_t base = r * ncols + b * blk + p;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const cx<double> a = fa[c * nodes + p], bb = fb[c * nodes + p];
    if (pass == 0) {
      xout[base + c * nodes] = mk<double>(0.5 * (a.re + bb.re) + 0.25 * zx[c].re, 0.5 * (a.im + bb.im) + 0.25 * zx[c].im);
    } else if (pass == 1) {
      xout[base + c * nodes] = mk<double>(a.re + 2.0 * bb.re + zx[c].re, a.im + 2.0 * bb.im + zx[c].im);
    } else {
      const cx<double> fc = fb[ncols + c * nodes + p];
      const double cc = h / 6.0;
      g[base + c * nodes] = ccast<TO>(mk<double>(cc * (a.re + 4.0 * bb.re + fc.re + zx[c].re),
                                                 cc * (a.im + 4.0 * bb.im + fc.im + zx[c].im)));
    }
  }
}

// rows <= 65535 and k <= 65535 (grid dimensions).
int launch_grid_signal_pass(const GridOpDev& g64, const void* H, const void* xin, void* xout, void* g, int out_fp64,
                            int k, int64_t rows, double h, int pass, hipStream_t st) {
  if (rows < 1 || rows > 65535 || k < 1 || k > 65535) return -1;
  const int64_t nodes = g64.nx * g64.ny * g64.nz;
  GridCoef<double> c;
  c.cxm = (const double*)g64.cxm; c.cxp = (const double*)g64.cxp; c.cym = (const double*)g64.cym;
  c.cyp = (const double*)g64.cyp; c.czm = (const double*)g64.czm; c.czp = (const double*)g64.czp;
  c.d = (const double*)g64.d; c.K = (const double*)g64.K;
  const dim3 grid((unsigned)((nodes + 255) / 256), (unsigned)k, (unsigned)rows);
#define RES_GS(TO, NC)                                                                                          \
  hipLaunchKernelGGL((grid_signal_pass_kernel<TO, NC>), grid, dim3(256), 0, st, c, g64.nx, g64.ny, g64.nz,       \
                     (const cx<double>*)H, (const cx<double>*)xin, (cx<double>*)xout, (cx<TO>*)g, k, h, pass)
  if (g64.ncomp == 3) {
    if (out_fp64) RES_GS(double, 3);
    else RES_GS(float, 3);
  } else {
    if (out_fp64) RES_GS(double, 1);
    else RES_GS(float, 1);
  }
#undef RES_GS
  return 0;
}

// dst[(row0 + dir * r) * ncols + c] = src[r * src_ld + c] for r < rows (dir = +1 or -1).
template <typename T>
__global__ __launch_bounds__(256) void copy_rows_kernel(const cx<T>* __restrict__ src, int64_t src_ld,
                                                        cx<T>* __restrict__ dst, int64_t row0, int dir, int64_t rows,
                                                        int64_t ncols) {
  const int64_t total = rows * ncols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ncols, c = e - r * ncols;
    dst[(row0 + dir * r) * ncols + c] = src[r * src_ld + c];
  }
}

int launch_copy_rows(const void* src, int64_t src_ld, void* dst, int64_t row0, int dir, int64_t rows, int64_t ncols,
                     int fp64, hipStream_t st) {
  int64_t blocks = (rows * ncols + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) return 0;
  if (fp64)
    hipLaunchKernelGGL((copy_rows_kernel<double>), dim3((unsigned)blocks), dim3(256), 0, st, (const cx<double>*)src,
                       src_ld, (cx<double>*)dst, row0, dir, rows, ncols);
  else
    hipLaunchKernelGGL((copy_rows_kernel<float>), dim3((unsigned)blocks), dim3(256), 0, st, (const cx<float>*)src,
                       src_ld, (cx<float>*)dst, row0, dir, rows, ncols);
  return 0;
}

// FIR filtering along time with the n/2-sample delay removed (App. B):
//     y[t][c] = wt(t) * sum_{m=0}^{n} b[m] x[t + n/2 - m][c],   x = 0 outside [0, T),
// with the optional taper wt (zero on the first and last `pad` samples, raised-cosine ramps of `ramp` samples, one
// between; pad < 0: no taper).  Each lane owns one column and kFirRT consecutive output times t0 .. t0 + kFirRT - 1
// and walks the taps: for tap m it needs x[t0 + j + n/2 - m], j < kFirRT, a window that slides down by one sample
// per tap.  The window lives in registers as a ring (slot (j - u) mod kFirRT at step u of an unrolled group of
// kFirRT taps), so each tap costs one new sample load, one broadcast read of the tap from LDS (zero-padded to a
// whole group) and kFirRT complex multiply-adds.  FP64 accumulation in both precisions.  Two instantiations:
// kFirRT = 16 (one load per 64 FMAs), and 8 for grids that would otherwise give the chip fewer than two waves per
// SIMD.
constexpr int kFirRT = 16, kFirRTSmall = 8;

__device__ __forceinline__ double taper_at(int64_t t, int64_t T, int64_t pad, int64_t ramp) {
  if (pad < 0) return 1.0;
  const int64_t a = (t < T - 1 - t ? t : T - 1 - t) - pad;
  if (a < 0) return 0.0;
  if (a < ramp) return 0.5 - 0.5 * cos(M_PI * ((double)a + 0.5) / (double)ramp);
  return 1.0;
}

template <typename T>
__device__ __forceinline__ cx<double> load_or_zero(const cx<T>* __restrict__ x, int64_t q, int64_t Tn, int64_t ncols,
                                                   int64_t c, bool live) {
  return (live && q >= 0 && q < Tn) ? ccast<double>(x[q * ncols + c]) : mk<double>(0.0, 0.0);
}

template <typename T, int RT>
__global__ __launch_bounds__(256) void fir_kernel(const cx<double>* __restrict__ taps, int order,
                                                  const cx<T>* __restrict__ x, cx<T>* __restrict__ y, int64_t Tn,
                                                  int64_t ncols, int64_t pad, int64_t ramp) {
  extern __shared__ cx<double> sb[];
  const int ntap = (order + RT) / RT * RT;  // order + 1 rounded up to whole groups
  for (int m = threadIdx.x; m < ntap; m += blockDim.x) sb[m] = m <= order ? taps[m] : mk<double>(0.0, 0.0);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t c = (int64_t)blockIdx.x * 64 + lane;
  const int64_t t0 = ((int64_t)blockIdx.y * (blockDim.x >> 6) + wave) * RT;
  if (t0 >= Tn) return;
  const bool live = c < ncols;
  const int64_t base = t0 + order / 2;  // x index of output j at tap m: base + j - m
  cx<double> acc[RT], ring[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) {
    acc[j] = mk<double>(0.0, 0.0);
    ring[j] = load_or_zero(x, base + j, Tn, ncols, c, live);
  }
  for (int m0 = 0; m0 < ntap; m0 += RT) {
#pragma unroll
    for (int u = 0; u < RT; ++u) {
      const cx<double> b = sb[m0 + u];
#pragma unroll
      for (int j = 0; j < RT; ++j) acc[j] = cfma(b, ring[(j - u + RT) % RT], acc[j]);
      // the slot of offset j - u = RT - 1 - u is not needed again: it takes the sample of offset -(u + 1)
      ring[(RT - 1 - u) % RT] = load_or_zero(x, base - (m0 + u) - 1, Tn, ncols, c, live);
    }
  }
  if (!live) return;
#pragma unroll
  for (int j = 0; j < RT; ++j) {
    const int64_t t = t0 + j;
    if (t < Tn) {
      const double w = taper_at(t, Tn, pad, ramp);
      y[t * ncols + c] = ccast<T>(mk<double>(w * acc[j].re, w * acc[j].im));
    }
  }
}

int fir_max_order() { return 65536 / (int)sizeof(cx<double>) - kFirRT; }

int launch_fir(const cx<double>* taps, int order, const void* x, void* y, int64_t Tn, int64_t ncols, int64_t pad,
               int64_t ramp, int fp64, hipStream_t st) {
  if (order < 0 || order > fir_max_order() || Tn < 1 || ncols < 1) return -1;
  const int64_t cblocks = (ncols + 63) / 64;
  const bool small = cblocks * ((Tn + kFirRT - 1) / kFirRT) < 2 * 1024;  // waves at 16 outputs per lane
  const int rt = small ? kFirRTSmall : kFirRT;
  const dim3 grid((unsigned)cblocks, (unsigned)((Tn + 4 * rt - 1) / (4 * rt)));
  const size_t lds = (size_t)((order + rt) / rt * rt) * sizeof(cx<double>);
#define RES_FIR(T, R)                                                                                           \
  hipLaunchKernelGGL((fir_kernel<T, R>), grid, dim3(256), lds, st, taps, order, (const cx<T>*)x, (cx<T>*)y, Tn,  \
                     ncols, pad, ramp)
  if (fp64) {
    if (small) RES_FIR(double, kFirRTSmall);
    else RES_FIR(double, kFirRT);
  } else {
    if (small) RES_FIR(float, kFirRTSmall);
    else RES_FIR(float, kFirRT);
  }
#undef RES_FIR
  return 0;
}

// Fourier transform of a series at arbitrary frequencies, out[j][c] = dt sum_i x[i][c] e^{-i w_j i dt} (FP64), in
// two deterministic stages: workgroup row blockIdx.y sums its chunk of kDftChunk samples into part[chunk][j][c]
// (the phase advances by a complex rotation per sample and is recomputed exactly every 64 samples), then the
// chunks are added in order.
constexpr int kDftChunk = 256;

template <typename T>
__global__ __launch_bounds__(256) void series_dft_kernel(const cx<T>* __restrict__ x, int64_t Tn, int64_t ncols,
                                                         const double* __restrict__ omegas, int nw, double dt,
                                                         cx<double>* __restrict__ part) {
  const int64_t total = (int64_t)nw * ncols;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int64_t j = e / ncols, c = e - j * ncols;
  const int64_t i0 = (int64_t)blockIdx.y * kDftChunk;
  const int64_t i1 = i0 + kDftChunk < Tn ? i0 + kDftChunk : Tn;
  const double w = omegas[j];
  double sr, cr;
  sincos(-w * dt, &sr, &cr);
  const cx<double> rot = mk<double>(cr, sr);
  cx<double> acc = mk<double>(0.0, 0.0), ph = mk<double>(1.0, 0.0);
  for (int64_t i = i0; i < i1; ++i) {
    if (((i - i0) & 63) == 0) {
      double s, co;
      sincos(-w * dt * (double)i, &s, &co);
      ph = mk<double>(co, s);
    }
    acc = cfma(ph, ccast<double>(x[i * ncols + c]), acc);
    ph = cmul(ph, rot);
  }
  part[(int64_t)blockIdx.y * total + e] = mk<double>(dt * acc.re, dt * acc.im);
}

__global__ __launch_bounds__(256) void sum_chunks_kernel(const cx<double>* __restrict__ part, int64_t total,
                                                         int nchunk, cx<double>* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    cx<double> s = mk<double>(0.0, 0.0);
    for (int q = 0; q < nchunk; ++q) s = cadd(s, part[(int64_t)q * total + e]);
    out[e] = s;
  }
}

int64_t series_dft_part_elems(int64_t Tn, int64_t ncols, int nw) {
  return ((Tn + kDftChunk - 1) / kDftChunk) * (int64_t)nw * ncols;
}

// part: series_dft_part_elems(Tn, ncols, nw) FP64 complex values of scratch.
int launch_series_dft(const void* x, int fp64, int64_t Tn, int64_t ncols, const double* omegas, int nw, double dt,
                      void* part, void* out, hipStream_t st) {
  const int64_t total = (int64_t)nw * ncols;
  const int64_t nchunk = (Tn + kDftChunk - 1) / kDftChunk;
  if (total < 1 || Tn < 1 || nchunk > 65535) return -1;
  const dim3 grid((unsigned)((total + 255) / 256), (unsigned)nchunk);
  if (fp64)
    hipLaunchKernelGGL((series_dft_kernel<double>), grid, dim3(256), 0, st, (const cx<double>*)x, Tn, ncols, omegas,
                       nw, dt, (cx<double>*)part);
  else
    hipLaunchKernelGGL((series_dft_kernel<float>), grid, dim3(256), 0, st, (const cx<float>*)x, Tn, ncols, omegas,
                       nw, dt, (cx<double>*)part);
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(sum_chunks_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (const cx<double>*)part, total,
                     (int)nchunk, (cx<double>*)out);
  return 0;
}

// Taps of the frequency-sampling FIR design (App. B) from the sampled response D[q] at nu_q = -1 + 2q/M:
//     taps[m] = w_m (1/M) sum_q D[q] e^{i pi nu_q (m - n/2)},  e^{i pi nu_q r} = (-1)^r E[(q r) mod M],
// E[p] = e^{2 pi i p / M} (a table), w_m the Hamming window.  One workgroup per tap; lanes stride over q and the
// partial sums are added in a fixed order.
__global__ __launch_bounds__(256) void fir_taps_kernel(const double* __restrict__ D, const cx<double>* __restrict__ E,
                                                       int64_t M, int order, cx<double>* __restrict__ taps) {
  __shared__ cx<double> red[256];
  const int m = blockIdx.x;
  const int64_t r = (int64_t)m - order / 2;
  const int64_t rm = ((r % M) + M) % M;
  cx<double> acc = mk<double>(0.0, 0.0);
  for (int64_t q = threadIdx.x; q < M; q += blockDim.x) {
    const cx<double> e = E[(q * rm) % M];
    acc = mk<double>(fma(D[q], e.re, acc.re), fma(D[q], e.im, acc.im));
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    cx<double> t = red[0];
    if (r & 1) t = mk<double>(-t.re, -t.im);
    const double wm = (0.54 - 0.46 * cos(2.0 * M_PI * (double)m / (double)order)) / (double)M;
    taps[m] = mk<double>(wm * t.re, wm * t.im);
  }
}

int launch_fir_taps(const double* D, const void* E, int64_t M, int order, void* taps, hipStream_t st) {
  if (order < 2 || M < 1) return -1;
  hipLaunchKernelGGL(fir_taps_kernel, dim3((unsigned)(order + 1)), dim3(256), 0, st, D, (const cx<double>*)E, M, order,
                     (cx<double>*)taps);
  return 0;
}

// out[j][c] = X[j][c] / norms[j] (X FP64 [nw][ncols], out in the working precision; a zero norm gives zeros).
template <typename TO>
__global__ __launch_bounds__(256) void scale_rows_kernel(const cx<double>* __restrict__ X, const double* __restrict__ norms,
                                                         int64_t nrows, int64_t ncols, cx<TO>* __restrict__ out) {
  const int64_t total = nrows * ncols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double nv = norms[e / ncols];
    const double s = nv > 0.0 ? 1.0 / nv : 0.0;
    out[e] = ccast<TO>(mk<double>(s * X[e].re, s * X[e].im));
  }
}

int launch_scale_rows(const void* X, const double* norms, int64_t nrows, int64_t ncols, void* out, int out_fp64,
                      hipStream_t st) {
  int64_t blocks = (nrows * ncols + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) return 0;
  if (out_fp64)
    hipLaunchKernelGGL((scale_rows_kernel<double>), dim3((unsigned)blocks), dim3(256), 0, st, (const cx<double>*)X,
                       norms, nrows, ncols, (cx<double>*)out);
  else
    hipLaunchKernelGGL((scale_rows_kernel<float>), dim3((unsigned)blocks), dim3(256), 0, st, (const cx<double>*)X,
                       norms, nrows, ncols, (cx<float>*)out);
  return 0;
}

// norms[j] = sqrt(sum_c |X[j][c]|^2) for X FP64 [nw][ncols]: one workgroup per row.
__global__ __launch_bounds__(256) void row_norms_kernel(const cx<double>* __restrict__ X, int64_t ncols,
                                                        double* __restrict__ norms) {
  __shared__ double red[4];
  const int64_t j = blockIdx.x;
  double s = 0.0;
  for (int64_t c = threadIdx.x; c < ncols; c += blockDim.x) {
    const cx<double> z = X[j * ncols + c];
    s = fma(z.re, z.re, fma(z.im, z.im, s));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) norms[j] = sqrt(red[0] + red[1] + red[2] + red[3]);
}

int launch_row_norms(const void* X, int64_t nrows, int64_t ncols, double* norms, hipStream_t st) {
  if (nrows < 1) return 0;
  hipLaunchKernelGGL(row_norms_kernel, dim3((unsigned)nrows), dim3(256), 0, st, (const cx<double>*)X, ncols, norms);
  return 0;
}

// x *= 1 / ||x|| over count complex values: partial sums of squares per workgroup, then one workgroup turns them
// into the scale, then the scaling pass reads it.
template <typename T>
__global__ __launch_bounds__(256) void sumsq_kernel(const cx<T>* __restrict__ x, int64_t count,
                                                    double* __restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    const cx<double> z = ccast<double>(x[e]);
    s = fma(z.re, z.re, fma(z.im, z.im, s));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void inv_norm_kernel(const double* __restrict__ part, int nparts,
                                                       double* __restrict__ scale) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += part[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = red[0] + red[1] + red[2] + red[3];
    scale[0] = t > 0.0 ? 1.0 / sqrt(t) : 0.0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void scale_by_kernel(cx<T>* __restrict__ x, int64_t count,
                                                       const double* __restrict__ scale) {
  const double s = scale[0];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    const cx<double> z = ccast<double>(x[e]);
    x[e] = ccast<T>(mk<double>(s * z.re, s * z.im));
  }
}

constexpr int kNormParts = 1024;
int normalise_parts() { return kNormParts; }

// part: kNormParts doubles, scale: one double (device scratch).
int launch_normalise(void* x, int fp64, int64_t count, double* part, double* scale, hipStream_t st) {
  if (count < 1) return 0;
  int64_t blocks = (count + 255) / 256;
  if (blocks > kNormParts) blocks = kNormParts;
  if (fp64) {
    hipLaunchKernelGGL((sumsq_kernel<double>), dim3((unsigned)blocks), dim3(256), 0, st, (const cx<double>*)x, count,
                       part);
  } else {
    hipLaunchKernelGGL((sumsq_kernel<float>), dim3((unsigned)blocks), dim3(256), 0, st, (const cx<float>*)x, count,
                       part);
  }
  hipLaunchKernelGGL(inv_norm_kernel, dim3(1), dim3(256), 0, st, part, (int)blocks, scale);
  int64_t sb = (count + 255) / 256;
  if (sb > 65536) sb = 65536;
  if (fp64)
    hipLaunchKernelGGL((scale_by_kernel<double>), dim3((unsigned)sb), dim3(256), 0, st, (cx<double>*)x, count, scale);
  else
    hipLaunchKernelGGL((scale_by_kernel<float>), dim3((unsigned)sb), dim3(256), 0, st, (cx<float>*)x, count, scale);
  return 0;
}

}  // namespace res
