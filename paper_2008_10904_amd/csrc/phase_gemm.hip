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
// quarter = 2 x 2 MFMA tiles.  In FP32 a complex tile is three real MFMAs (Gauss: P1 = Ar Br, P2 = Ai Bi,
// P3 = (Ar + Ai)(Br + Bi); re = P1 - P2, im = P3 - P1 - P2, formed in FP64 in the epilogue); in FP64 four
// (re*re - im*im, re*im + im*re), since a third FP64 accumulator set would halve the waves per SIMD.
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

  constexpr bool kGauss = sizeof(R) == 4;
  v4 c1[2][2], c2[2][2], c3[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      c1[i][j] = v4{0, 0, 0, 0};
      c2[i][j] = v4{0, 0, 0, 0};
      c3[i][j] = v4{0, 0, 0, 0};
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
      R are[2], aim[2], bre[2], bim[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int r = wm * 32 + t * 16 + (lane & 15);
        are[t] = As[0][r][k4 + (lane >> 4)];
        aim[t] = As[1][r][k4 + (lane >> 4)];
        const int c = wn * 32 + t * 16 + (lane & 15);
        bre[t] = Bs[0][k4 + (lane >> 4)][c];
        bim[t] = Bs[1][k4 + (lane >> 4)][c];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (kGauss) {  // c1 = ArBr, c2 = AiBi, c3 = (Ar + Ai)(Br + Bi)
            c1[i][j] = Mfma<R>::mac(are[i], bre[j], c1[i][j]);
            c2[i][j] = Mfma<R>::mac(aim[i], bim[j], c2[i][j]);
            c3[i][j] = Mfma<R>::mac(are[i] + aim[i], bre[j] + bim[j], c3[i][j]);
          } else {  // c1 = re, c2 = im
            c1[i][j] = Mfma<R>::mac(are[i], bre[j], c1[i][j]);
            c1[i][j] = Mfma<R>::mac(-aim[i], bim[j], c1[i][j]);
            c2[i][j] = Mfma<R>::mac(are[i], bim[j], c2[i][j]);
            c2[i][j] = Mfma<R>::mac(aim[i], bre[j], c2[i][j]);
          }
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
        const double p1 = (double)c1[i][j][v], p2 = (double)c2[i][j][v];
        const double xr = kGauss ? p1 - p2 : p1, xi = kGauss ? (double)c3[i][j][v] - p1 - p2 : p2;
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

// ---- synthesis of a few rows from a short frequency block, FP32 ------------------------------------------------
// out[r][n] = e^{i sigma w0 h s_r} sum_j A[r][j] G[j][n] for at most 256 rows (forcing tiles, the reverse mode's
// segment and seed rows) and at most 192 frequencies.  There the GEMM is short in M and K and long in N (the 3-D
// workload's tile: 64 rows, 96 frequencies, 37.7 M columns), and the tiled kernel above spends its time
// regenerating the phase operand and staging both operands through LDS for every 64-column tile.  Here a
// workgroup generates the phase operand of its 64-row tile once, into LDS, and each of its eight waves streams
// 32-column tiles of G straight from HBM into MFMA operand registers, one 32-frequency chunk ahead of the matrix
// cores, with the 64 x 32 output tile in accumulators.  A complex product takes three real MFMAs (Gauss):
// P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi); re = P1 - P2, im = P3 - P1 - P2.
constexpr int SY_ROWS = 64, SY_KMAX = 192, SY_LDA = 80, SY_KC = 8;  // SY_KC: K-steps of 4 per register chunk

__global__ __launch_bounds__(512) void synth_rows_kernel(PhaseGemmArgs a) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  // A planes [k][row] with a row stride of 80 floats (16 mod 32 banks): the 16 rows x 4 k of an operand read
  // fall in distinct banks for each half-wave
  __shared__ float Ar[SY_KMAX * SY_LDA], Ai[SY_KMAX * SY_LDA];
  __shared__ double ph_re[SY_ROWS], ph_im[SY_ROWS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kq = lane >> 4, cl = lane & 15;  // operand lane layout: A[cl][kq], B[kq][cl]
  const int64_t m0 = (int64_t)blockIdx.y * SY_ROWS;
  const int K = (int)a.K;
  const int nkc = (K + 4 * SY_KC - 1) / (4 * SY_KC);  // register chunks per column tile
  const int Kp = nkc * 4 * SY_KC;
  const int64_t P = a.P;
  const int64_t str = a.stride > 0 ? a.stride : 1;
  const cx<float>* __restrict__ btab = (const cx<float>*)a.btab;
  const bool conj_a = a.sigma < 0;
  for (int e = tid; e < Kp * SY_ROWS; e += blockDim.x) {
    const int k = e / SY_ROWS, r = e - k * SY_ROWS;
    float re = 0.f, im = 0.f;
    if (k < K && m0 + r < a.M) {
      const int64_t smod = (a.s0 + (m0 + r) * str) % P;
      const cx<float> t = btab[((int64_t)k * smod) % P];  // k < 192 and smod < P: no overflow
      re = t.re;
      im = conj_a ? -t.im : t.im;
    }
    Ar[k * SY_LDA + r] = re;
    Ai[k * SY_LDA + r] = im;
  }
  if (tid < SY_ROWS) {
    double sn, cs;
    sincos((double)a.sigma * a.w0h * (double)(a.s0 + (m0 + tid) * str), &sn, &cs);
    ph_re[tid] = cs;
    ph_im[tid] = sn;
  }
  __syncthreads();  // the only barrier: from here on the waves are independent

  const cx<float>* __restrict__ B = (const cx<float>*)a.bmat;
  cx<float>* __restrict__ out = (cx<float>*)a.out;
  const int64_t ldb = a.ldb > 0 ? a.ldb : a.Ncols;
  const int64_t ncols = a.Ncols;
  const int64_t ntiles = (ncols + 31) / 32;
  const int64_t wstride = (int64_t)gridDim.x * 8;
  const int64_t t0 = (int64_t)blockIdx.x * 8 + wave;
  if (t0 >= ntiles) return;
  const int64_t nq = ((ntiles - 1 - t0) / wstride + 1) * nkc;  // chunks of this wave, in order

  v4 p1[4][2], p2[4][2], p3[4][2];
  auto zero = [&]() {
#pragma unroll
    for (int tr = 0; tr < 4; ++tr)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        p1[tr][c] = v4{0.f, 0.f, 0.f, 0.f};
        p2[tr][c] = v4{0.f, 0.f, 0.f, 0.f};
        p3[tr][c] = v4{0.f, 0.f, 0.f, 0.f};
      }
  };
  // chunk q: column tile t0 + (q / nkc) * wstride, frequencies (q % nkc) * 32 ..; rows past K read row K - 1
  // (finite data against zero phases), columns past the end read the last column (results not stored)
  auto load = [&](int64_t q, float (&xr)[SY_KC][2], float (&xi)[SY_KC][2]) {
    const int64_t n0 = (t0 + (q / nkc) * wstride) * 32;
    const int kc = (int)(q % nkc);
#pragma unroll
    for (int s = 0; s < SY_KC; ++s) {
      const int k = min(kc * 4 * SY_KC + 4 * s + kq, K - 1);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int64_t n = min(n0 + 16 * c + cl, ncols - 1);
        const cx<float> v = B[(int64_t)k * ldb + n];
        xr[s][c] = v.re;
        xi[s][c] = v.im;
      }
    }
  };
  auto compute = [&](int64_t q, float (&xr)[SY_KC][2], float (&xi)[SY_KC][2]) {
    const int kc = (int)(q % nkc);
#pragma unroll
    for (int s = 0; s < SY_KC; ++s) {
      const int kr = kc * 4 * SY_KC + 4 * s + kq;
      float ar[4], ai[4];
#pragma unroll
      for (int tr = 0; tr < 4; ++tr) {
        ar[tr] = Ar[kr * SY_LDA + 16 * tr + cl];
        ai[tr] = Ai[kr * SY_LDA + 16 * tr + cl];
      }
#pragma unroll
      for (int tr = 0; tr < 4; ++tr)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          p1[tr][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[tr], xr[s][c], p1[tr][c], 0, 0, 0);
          p2[tr][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[tr], xi[s][c], p2[tr][c], 0, 0, 0);
          p3[tr][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[tr] + ai[tr], xr[s][c] + xi[s][c], p3[tr][c], 0,
                                                           0, 0);
        }
    }
    if (kc != nkc - 1) return;
    // the tile is complete: rows 4 kq + v of each 16 x 16 block, column cl
    const int64_t n0 = (t0 + (q / nkc) * wstride) * 32;
#pragma unroll
    for (int tr = 0; tr < 4; ++tr)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rl = 16 * tr + 4 * kq + v;
          const int64_t row = m0 + rl, col = n0 + 16 * c + cl;
          const double x1 = p1[tr][c][v], x2 = p2[tr][c][v], x3 = p3[tr][c][v];
          const double xr0 = x1 - x2, xi0 = x3 - x1 - x2;
          const double pr = ph_re[rl], pi = ph_im[rl];
          if (row < a.M && col < ncols)
            out[row * ncols + col] = mk<float>((float)(xr0 * pr - xi0 * pi), (float)(xr0 * pi + xi0 * pr));
        }
    zero();
  };

  zero();
  float xa[SY_KC][2], ya[SY_KC][2], xb[SY_KC][2], yb[SY_KC][2];
  load(0, xa, ya);
  int64_t q = 0;
  for (; q + 1 < nq; q += 2) {
    load(q + 1, xb, yb);
    compute(q, xa, ya);
    if (q + 2 < nq) load(q + 2, xa, ya);
    compute(q + 1, xb, yb);
  }
  if (q < nq) compute(q, xa, ya);
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
  if (a.mode == 0 && !fp64 && a.K <= SY_KMAX && a.M <= 4 * SY_ROWS && a.k_per_split >= a.K) {
    // one 512-thread workgroup per CU (123 KB of LDS at most): 256 over the M tiles, a multiple of 8 per M tile so
    // that the workgroups of one column range sit on one XCD
    const int64_t mt = (a.M + SY_ROWS - 1) / SY_ROWS;
    const int64_t per = ((256 / mt) + 7) / 8 * 8;
    const int64_t gxs = std::max<int64_t>(1, std::min<int64_t>(per, (((a.Ncols + 31) / 32) + 7) / 8));
    hipLaunchKernelGGL(synth_rows_kernel, dim3((unsigned)gxs, (unsigned)mt), dim3(512), 0, st, a);
    return 0;
  }
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
