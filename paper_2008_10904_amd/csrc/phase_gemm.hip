// Forcing synthesis and Fourier projection as complex GEMMs on MFMA (FP64 16x16x4 or FP32 16x16x4).
//
//   synthesis  (Sec. 2.3, eq. forceFseries, complex branch):  out[r][n] = sum_j e^{i sw_j t_s} G[j][n],
//              s = s0 + r*stride, t_s = s h  -- the rows are forcing samples of (usually consecutive) steps;
//   projection (eq. fourier, evaluated as a finite sum):     acc[j][n] += scale * sum_m e^{-i sw_j t_m} X[m][n],
//              t_m = (s0 + m*stride) h  -- the rows of X are state snapshots.
//
// sw_j = sigma (w0 + j dw) with dw = 2 pi / (P h).  Phases are index-exact:
//   e^{i sw_j t_s} = e^{i sigma w0 h s} * btab[(j * (s mod P)) mod P]^sigma,   btab[m] = e^{2 pi i m / P},
// so no phase is ever accumulated in working precision; the w0 factor is one FP64 sincos per row (synthesis) or
// an FP64 rotation per sample, re-evaluated exactly every 64 K chunks (projection).  The table index advances
// incrementally (no division in the inner loop).
//
// Tiling: one 256-thread workgroup computes a 64 x 64 tile of the (complex) output; each wave owns a 32 x 32
// quarter = 2 x 2 MFMA tiles, each complex tile being four real MFMAs (re*re - im*im, re*im + im*re).
// The generated phase operand and the data operand are staged through LDS 16 deep in K, loaded into registers
// one chunk ahead of the matrix-core work.  Workgroups walk the M tiles of one column tile on one XCD.  The
// projection can split K over gridDim.y, writing FP64 partial tiles that a reduction adds into the FP64
// accumulator.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace res {

template <typename R> struct Mfma;
// Operand layouts (both shapes): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].  Result element v of
// lane l is D[row(l, v)][l % 16] with row = l/16 + 4v for the FP64 shape and 4(l/16) + v for the FP32 shape
// (checked on gfx950 with a one-wave probe).
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mac(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int GBM = 64, GBN = 64, GKC = 16;

template <typename R, int MODE>
__global__ __launch_bounds__(256) void phase_gemm_kernel(PhaseGemmArgs a) {
  typedef typename Mfma<R>::v4 v4;
  __shared__ R As[2][GBM][GKC + 1];
  __shared__ R Bs[2][GKC][GBN + 1];
  __shared__ double ph_re[GBM], ph_im[GBM];  // MODE 0: per-row factors e^{i sigma w0 h s}

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // Tile order: workgroups are dealt to the eight XCDs in turn (id mod 8), and each XCD has its own L2.  All M
  // tiles of one column tile go to the same XCD, one after the other, so that its data operand (the column tile's
  // K rows) is read from HBM once and then hit in that XCD's L2.
  const int64_t gyt = (a.M + GBM - 1) / GBM;
  const int64_t slot = (int64_t)(blockIdx.x >> 3);
  const int64_t mt = slot % gyt;
  const int64_t nt = (slot / gyt) * 8 + (blockIdx.x & 7);
  if (nt * GBN >= a.Ncols) return;  // padding of the column tiles to a multiple of 8 (whole workgroup)
  const int64_t n0 = nt * GBN;
  const int64_t m0 = mt * GBM;
  const int64_t P = a.P;
  const cx<R>* __restrict__ btab = (const cx<R>*)a.btab;
  const cx<R>* __restrict__ B = (const cx<R>*)a.bmat;
  const double sig = (double)a.sigma;
  const int64_t ldb = a.ldb > 0 ? a.ldb : a.Ncols;

  // K range of this split
  const int64_t kb = (int64_t)blockIdx.y * a.k_per_split;
  int64_t ke = kb + a.k_per_split;
  if (ke > a.K) ke = a.K;

  // Phase-operand generation: thread owns A-row ar = tid / 4 and four consecutive K entries (tid % 4) * 4 + q.
  const int ar = tid >> 2;
  const int ak = (tid & 3) * 4;
  // idx(kk) = table index of A[ar][kk]; it advances by `step` per kk and by `step16` per K chunk.
  int64_t idx = 0, step = 0, step16 = 0;
  bool arow_ok;
  if (MODE == 0) {
    // row = time sample s = s0 + (m0 + ar) * stride; column kk = frequency j: index (j * smod) mod P
    const int64_t s = a.s0 + (m0 + ar) * (a.stride > 0 ? a.stride : 1);
    arow_ok = (m0 + ar) < a.M;
    const int64_t smod = s % P;
    step = smod;
    step16 = (smod * (int64_t)GKC) % P;
    idx = ((kb + ak) % P) * smod % P;
  } else {
    // row = frequency j = m0 + ar; column kk = sample m: s = s0 + m*stride, index (j * s) mod P
    const int64_t j = m0 + ar;
    arow_ok = j < a.M;
    const int64_t jstr = (j % P) * (a.stride % P) % P;
    step = jstr;
    step16 = (jstr * (int64_t)GKC) % P;
    const int64_t s = a.s0 + (kb + ak) * a.stride;
    idx = (j % P) * (s % P) % P;
  }

  if (MODE == 0 && tid < GBM) {
    const int64_t s = a.s0 + (m0 + tid) * (a.stride > 0 ? a.stride : 1);
    double sn, cs;
    sincos(sig * a.w0h * (double)s, &sn, &cs);
    ph_re[tid] = cs;
    ph_im[tid] = sn;
  }

  v4 cre[2][2], cim[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cre[i][j] = v4{0, 0, 0, 0};
      cim[i][j] = v4{0, 0, 0, 0};
    }

  // Operands of one K chunk are loaded into registers one chunk ahead, so that the table gathers and data loads
  // of chunk c+1 are in flight while chunk c runs on the matrix cores.  The loads are unconditional (addresses
  // clamped into range) and carry no arithmetic, so nothing waits for them before the next chunk is staged; the
  // staging step masks the out-of-range entries, conjugates the table values (adjoint sign, and the projection's
  // e^{-i...}) and multiplies the projection rows by the per-sample factor conj(e^{i sigma w0 h s_m}) (the
  // projection phase factorises over j and m).  That factor advances by one FP64 complex product per chunk and is
  // re-evaluated with sincos every 64 chunks, so its drift stays at the FP64 rounding level.
  const int kr = tid >> 4;
  const int nc = (tid & 15) * 4;
  const bool conj_a = (a.sigma < 0) != (MODE == 1);
  cx<R> ra[4], rb[4];
  auto load = [&](int64_t k0) {
    int64_t id = idx;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ra[q] = btab[id];
      id += step;
      if (id >= P) id -= P;
    }
    idx += step16;
    if (idx >= P) idx -= P;
    const int64_t kk = k0 + kr < ke ? k0 + kr : ke - 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t n = n0 + nc + q < a.Ncols ? n0 + nc + q : a.Ncols - 1;
      rb[q] = B[kk * ldb + n];
    }
  };
  double zr = 1.0, zi = 0.0, wr = 1.0, wi = 0.0;  // MODE 1: sample factor of row kr, and its per-chunk step
  if (MODE == 1) {
    double sn, cs;
    sincos(sig * a.w0h * (double)(GKC * a.stride), &sn, &cs);
    wr = cs;
    wi = -sn;
  }
  auto stage = [&](int64_t k0, int64_t c) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool ok = arow_ok && k0 + ak + q < ke;
      As[0][ar][ak + q] = ok ? ra[q].re : R(0);
      As[1][ar][ak + q] = ok ? (conj_a ? -ra[q].im : ra[q].im) : R(0);
    }
    const bool rok = k0 + kr < ke;
    R pr = R(1), pi = R(0);
    if (MODE == 1) {
      if ((c & 63) == 0) {
        double sn, cs;
        sincos(sig * a.w0h * (double)(a.s0 + (k0 + kr) * a.stride), &sn, &cs);
        zr = cs;
        zi = -sn;
      } else {
        const double t = zr * wr - zi * wi;
        zi = zr * wi + zi * wr;
        zr = t;
      }
      pr = (R)zr;
      pi = (R)zi;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool ok = rok && n0 + nc + q < a.Ncols;
      cx<R> v = rb[q];
      if (MODE == 1) v = mk<R>(v.re * pr - v.im * pi, v.re * pi + v.im * pr);
      Bs[0][kr][nc + q] = ok ? v.re : R(0);
      Bs[1][kr][nc + q] = ok ? v.im : R(0);
    }
  };

  if (kb < ke) load(kb);
  int64_t c = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += GKC, ++c) {
    stage(k0, c);
    __syncthreads();
    load(k0 + GKC);
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of this chunk's matrix-core work
#pragma unroll
    for (int k4 = 0; k4 < GKC; k4 += 4) {
      R are[2], aim[2], nai[2], bre[2], bim[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int r = wm * 32 + t * 16 + (lane & 15);
        are[t] = As[0][r][k4 + (lane >> 4)];
        aim[t] = As[1][r][k4 + (lane >> 4)];
        nai[t] = -aim[t];
        const int c = wn * 32 + t * 16 + (lane & 15);
        bre[t] = Bs[0][k4 + (lane >> 4)][c];
        bim[t] = Bs[1][k4 + (lane >> 4)][c];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cre[i][j] = Mfma<R>::mac(are[i], bre[j], cre[i][j]);
          cre[i][j] = Mfma<R>::mac(nai[i], bim[j], cre[i][j]);
          cim[i][j] = Mfma<R>::mac(are[i], bim[j], cim[i][j]);
          cim[i][j] = Mfma<R>::mac(aim[i], bre[j], cim[i][j]);
        }
    }
    __syncthreads();
  }

  // ---- epilogue: lane holds rows Mfma<R>::row(lane, v), column lane%16 of each 16x16 tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rl = wm * 32 + i * 16 + Mfma<R>::row(lane, v);
        const int cl = wn * 32 + j * 16 + (lane & 15);
        const int64_t row = m0 + rl, col = n0 + cl;
        if (row >= a.M || col >= a.Ncols) continue;
        const double xr = (double)cre[i][j][v], xi = (double)cim[i][j][v];
        if (MODE == 0) {
          const double pr = ph_re[rl], pi = ph_im[rl];
          cx<R>* out = (cx<R>*)a.out;
          out[row * a.Ncols + col] = mk<R>((R)(xr * pr - xi * pi), (R)(xr * pi + xi * pr));
        } else if (a.partial != nullptr) {
          cx<double>* part = (cx<double>*)a.partial;
          part[((int64_t)blockIdx.y * a.M + row) * a.Ncols + col] = mk<double>(xr, xi);
        } else {
          cx<double>* acc = (cx<double>*)a.out;
          cx<double> o = acc[row * a.Ncols + col];
          o.re += a.scale * xr;
          o.im += a.scale * xi;
          acc[row * a.Ncols + col] = o;
        }
      }
}

// acc[e] += scale * sum_z partial[z][e]
__global__ __launch_bounds__(256) void reduce_partials_kernel(const cx<double>* __restrict__ part,
                                                              cx<double>* __restrict__ acc, int64_t count,
                                                              int nsplit, double scale) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    double re = 0, im = 0;
    for (int z = 0; z < nsplit; ++z) {
      const cx<double> p = part[(int64_t)z * count + e];
      re += p.re;
      im += p.im;
    }
    cx<double> o = acc[e];
    o.re += scale * re;
    o.im += scale * im;
    acc[e] = o;
  }
}

int launch_phase_gemm(const PhaseGemmArgs& a, int fp64, hipStream_t st) {
  if (a.M <= 0 || a.Ncols <= 0 || a.K <= 0) return 0;
  const int64_t gx = (a.Ncols + GBN - 1) / GBN;
  const int64_t gy = (a.M + GBM - 1) / GBM;
  const int64_t gz = (a.K + a.k_per_split - 1) / a.k_per_split;
  const int64_t blocks = (gx + 7) / 8 * 8 * gy;  // column tiles padded to a multiple of 8 (see the tile order)
  if (blocks > 0x7fffffff || gz > 65535) return -1;
  dim3 grid((unsigned)blocks, (unsigned)gz);
  if (a.mode == 0) {
    if (fp64) hipLaunchKernelGGL((phase_gemm_kernel<double, 0>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((phase_gemm_kernel<float, 0>), grid, dim3(256), 0, st, a);
  } else {
    if (fp64) hipLaunchKernelGGL((phase_gemm_kernel<double, 1>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((phase_gemm_kernel<float, 1>), grid, dim3(256), 0, st, a);
  }
  return 0;
}

// t[m] = e^{2 pi i m / P} for m < P in the working precision, evaluated in FP64 on the device.
template <typename R>
__global__ __launch_bounds__(256) void phase_table_kernel(cx<R>* __restrict__ t, int64_t P) {
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < P; m += (int64_t)gridDim.x * blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)P, &sn, &cs);
    t[m] = ccast<R>(mk<double>(cs, sn));
  }
}

int launch_phase_table(void* t, int fp64, int64_t P, hipStream_t st) {
  if (P <= 0) return -1;
  const unsigned grid = (unsigned)std::min<int64_t>(4096, (P + 255) / 256);
  if (fp64) hipLaunchKernelGGL(phase_table_kernel<double>, dim3(grid), dim3(256), 0, st, (cx<double>*)t, P);
  else hipLaunchKernelGGL(phase_table_kernel<float>, dim3(grid), dim3(256), 0, st, (cx<float>*)t, P);
  return 0;
}

int launch_reduce_partials(const void* part, void* acc, int64_t count, int nsplit, double scale, hipStream_t st) {
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (const cx<double>*)part,
                     (cx<double>*)acc, count, nsplit, scale);
  return 0;
}

}  // namespace res
