// Per-frequency normalisation, orthogonalisation and small SVDs of the block power iteration (Appendix A with
// the frequency-domain normalisation of Sec. 2.3), all in FP64.
//
// The iterates are stored [n_w][k][N]: for frequency j and instance m the n_m x k matrix X_{j,m} has columns
// X[j][a][off_m .. off_{m+1}).  QR uses CholeskyQR2: G = X^H X reduced over the unknowns (many workgroups per
// matrix, FP64 partial sums), G = R^H R on one thread, X <- X R^{-1}, repeated once; the second pass makes
// Q orthonormal to working precision while the iterates stay far from rank deficiency (condition number well
// below 1e8).  The k x k SVD of R_Y is a complex one-sided Jacobi iteration.
#include "common.h"
#include "kernels.h"

namespace res {

constexpr int kMaxK = 8;
constexpr int kMaxPairs = kMaxK * (kMaxK + 1) / 2;

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Partial Gram matrices: part[((j*ninst + m)*nsplit + sp)*NP + pair] = sum over this block's unknowns of
// conj(X_a) X_b for a <= b (pairs in row-major upper-triangle order).  Sets *flag if a sum is not finite.
template <typename T, int KM>
__global__ __launch_bounds__(256) void gram_kernel(const cx<T>* __restrict__ X, int64_t N, int32_t k,
                                                   const int64_t* __restrict__ off, int32_t ninst,
                                                   int32_t nsplit, cx<double>* __restrict__ part,
                                                   int* __restrict__ flag) {
  constexpr int NP = KM * (KM + 1) / 2;
  __shared__ double red[4][2 * NP];
  const int sp = blockIdx.x, m = blockIdx.y, j = blockIdx.z;
  const int64_t lo = off[m], hi = off[m + 1];
  const int64_t chunk = (hi - lo + nsplit - 1) / nsplit;
  const int64_t a0 = lo + sp * chunk;
  const int64_t a1 = (a0 + chunk < hi) ? a0 + chunk : hi;
  double acc_re[NP], acc_im[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) acc_re[p] = acc_im[p] = 0.0;
  for (int64_t n = a0 + threadIdx.x; n < a1; n += 256) {
    cx<double> x[KM];
#pragma unroll
    for (int a = 0; a < KM; ++a) x[a] = a < k ? ccast<double>(X[((int64_t)j * k + a) * N + n]) : mk<double>(0, 0);
    int p = 0;
#pragma unroll
    for (int a = 0; a < KM; ++a)
#pragma unroll
      for (int b = a; b < KM; ++b, ++p) {
        acc_re[p] += x[a].re * x[b].re + x[a].im * x[b].im;
        acc_im[p] += x[a].re * x[b].im - x[a].im * x[b].re;
      }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const double r = wave_sum(acc_re[p]);
    const double i = wave_sum(acc_im[p]);
    if (lane == 0) {
      red[w][2 * p] = r;
      red[w][2 * p + 1] = i;
    }
  }
  __syncthreads();
  if (threadIdx.x < NP) {
    const int p = threadIdx.x;
    const double r = red[0][2 * p] + red[1][2 * p] + red[2][2 * p] + red[3][2 * p];
    const double i = red[0][2 * p + 1] + red[1][2 * p + 1] + red[2][2 * p + 1] + red[3][2 * p + 1];
    if (!isfinite(r) || !isfinite(i)) atomicOr(flag, 1);
    part[(((int64_t)j * ninst + m) * nsplit + sp) * NP + p] = mk<double>(r, i);
  }
}

__device__ __forceinline__ int pair_index(int a, int b, int k) {
  // index of (a, b), a <= b, in row-major upper-triangle order for a k x k matrix padded to KM = k
  return a * k - a * (a - 1) / 2 + (b - a);
}

// One thread per (j, m): sum the partial Grams, Cholesky G = R^H R (R upper, positive diagonal), R^{-1}.
// If rprev != null, rtot = R * rprev (the R factor of the two CholeskyQR passes combined).
// If norm_hist != null, norm_hist[(j*ninst+m)... ] receives sqrt(||x_a||) (eq. tildeSig with unit inputs),
// written to hist[((m*nw + j)*k + a)*2 + 1].
__global__ void chol_kernel(const cx<double>* __restrict__ part, int32_t nsplit, int32_t np_stride, int32_t k,
                            int32_t nw, int32_t ninst, cx<double>* __restrict__ rout, cx<double>* __restrict__ rinv,
                            const cx<double>* __restrict__ rprev, cx<double>* __restrict__ rtot,
                            double* __restrict__ hist, int* __restrict__ flag) {
  const int pidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (pidx >= nw * ninst) return;
  const int j = pidx / ninst, m = pidx % ninst;
  cx<double> G[kMaxK][kMaxK];
  for (int a = 0; a < k; ++a)
    for (int b = a; b < k; ++b) {
      double re = 0, im = 0;
      const int p = pair_index(a, b, np_stride == 0 ? k : np_stride);
      for (int s = 0; s < nsplit; ++s) {
        const cx<double> v = part[((int64_t)pidx * nsplit + s) * (np_stride * (np_stride + 1) / 2) + p];
        re += v.re;
        im += v.im;
      }
      G[a][b] = mk<double>(re, im);
      G[b][a] = mk<double>(re, -im);
    }
  if (hist != nullptr)
    for (int a = 0; a < k; ++a) hist[(((int64_t)m * nw + j) * k + a) * 2 + 1] = sqrt(sqrt(G[a][a].re));
  // Cholesky of the diagonally scaled Gram D^-1 G D^-1 (D = column norms), then R = R_s D.  The power
  // iterates are graded (column norms follow the gains, squared after an adjoint run), and the scaling keeps
  // the factorisation as accurate as that of column-normalised data.
  double dsc[kMaxK];
  bool bad = false;
  for (int a = 0; a < k; ++a) {
    dsc[a] = sqrt(G[a][a].re);
    if (!(dsc[a] > 0.0) || !isfinite(dsc[a])) {
      bad = true;
      dsc[a] = 1.0;
    }
  }
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) G[a][b] = mk<double>(G[a][b].re / (dsc[a] * dsc[b]), G[a][b].im / (dsc[a] * dsc[b]));
  cx<double> R[kMaxK][kMaxK];
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) R[a][b] = mk<double>(0, 0);
  for (int i = 0; i < k; ++i) {
    double d = G[i][i].re;
    for (int p = 0; p < i; ++p) d -= R[p][i].re * R[p][i].re + R[p][i].im * R[p][i].im;
    if (!(d > 0.0) || !isfinite(d)) {
      bad = true;
      d = 1e-300;
    }
    const double rii = sqrt(d);
    R[i][i] = mk<double>(rii, 0.0);
    for (int jj = i + 1; jj < k; ++jj) {
      cx<double> s = G[i][jj];
      for (int p = 0; p < i; ++p) s = cfma_conj(mk<double>(-R[p][i].re, -R[p][i].im), R[p][jj], s);
      R[i][jj] = mk<double>(s.re / rii, s.im / rii);
    }
  }
  for (int a = 0; a < k; ++a)
    for (int b = a; b < k; ++b) R[a][b] = mk<double>(R[a][b].re * dsc[b], R[a][b].im * dsc[b]);
  if (bad) atomicOr(flag, 2);
  // inverse of the upper triangular R
  cx<double> Ri[kMaxK][kMaxK];
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) Ri[a][b] = mk<double>(0, 0);
  for (int c = 0; c < k; ++c) {
    // solve R x = e_c, x upper part
    for (int i = c; i >= 0; --i) {
      cx<double> s = mk<double>(i == c ? 1.0 : 0.0, 0.0);
      for (int p = i + 1; p <= c; ++p) s = cfma(mk<double>(-R[i][p].re, -R[i][p].im), Ri[p][c], s);
      Ri[i][c] = mk<double>(s.re / R[i][i].re, s.im / R[i][i].re);
    }
  }
  const int64_t base = (int64_t)pidx * kMaxK * kMaxK;
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) {
      if (rout) rout[base + a * kMaxK + b] = R[a][b];
      rinv[base + a * kMaxK + b] = Ri[a][b];
    }
  if (rprev != nullptr && rtot != nullptr) {
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) {
        cx<double> s = mk<double>(0, 0);
        for (int p = 0; p < k; ++p) s = cfma(R[a][p], rprev[base + p * kMaxK + b], s);
        rtot[base + a * kMaxK + b] = s;
      }
  }
}

// Xout[j][b][n] = sum_a Xin[j][a][n] * M[j][m][a][b] for n in instance m (in place allowed).
template <typename TI, typename TO, int KM>
__global__ __launch_bounds__(256) void rmul_kernel(const cx<TI>* Xin, cx<TO>* Xout, int64_t N, int32_t k,
                                                   const int64_t* __restrict__ off, int32_t ninst, int32_t nsplit,
                                                   const cx<double>* __restrict__ M) {
  __shared__ cx<double> Ms[kMaxK * kMaxK];
  const int sp = blockIdx.x, m = blockIdx.y, j = blockIdx.z;
  const int64_t base = ((int64_t)j * ninst + m) * kMaxK * kMaxK;
  if (threadIdx.x < kMaxK * kMaxK) Ms[threadIdx.x] = M[base + threadIdx.x];
  __syncthreads();
  const int64_t lo = off[m], hi = off[m + 1];
  const int64_t chunk = (hi - lo + nsplit - 1) / nsplit;
  const int64_t a0 = lo + sp * chunk;
  const int64_t a1 = (a0 + chunk < hi) ? a0 + chunk : hi;
  for (int64_t n = a0 + threadIdx.x; n < a1; n += 256) {
    cx<double> x[KM];
#pragma unroll
    for (int a = 0; a < KM; ++a) x[a] = a < k ? ccast<double>(Xin[((int64_t)j * k + a) * N + n]) : mk<double>(0, 0);
#pragma unroll
    for (int b = 0; b < KM; ++b) {
      if (b >= k) break;
      cx<double> y = mk<double>(0, 0);
#pragma unroll
      for (int a = 0; a < KM; ++a)
        if (a < k) y = cfma(x[a], Ms[a * kMaxK + b], y);
      Xout[((int64_t)j * k + b) * N + n] = ccast<TO>(y);
    }
  }
}

// Complex one-sided Jacobi SVD of the k x k matrix A = R_Y (one thread per (j, m)).
// Outputs (all [nw][ninst][kMaxK][kMaxK] unless noted): phi = left singular vectors, psi = right singular
// vectors, apsi = A psi (= phi Sigma); gains[(m*nw + j)*k + i] descending; hist[...][0] = gains.
__global__ void svd_kernel(const cx<double>* __restrict__ A_in, int32_t k, int32_t nw, int32_t ninst,
                           cx<double>* __restrict__ phi, cx<double>* __restrict__ psi,
                           cx<double>* __restrict__ apsi, double* __restrict__ gains, double* __restrict__ hist) {
  const int pidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (pidx >= nw * ninst) return;
  const int j = pidx / ninst, m = pidx % ninst;
  const int64_t base = (int64_t)pidx * kMaxK * kMaxK;
  cx<double> A[kMaxK][kMaxK], V[kMaxK][kMaxK];
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) {
      A[a][b] = A_in[base + a * kMaxK + b];
      V[a][b] = mk<double>(a == b ? 1.0 : 0.0, 0.0);
    }
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        double al = 0, be = 0;
        cx<double> ga = mk<double>(0, 0);
        for (int r = 0; r < k; ++r) {
          al += A[r][p].re * A[r][p].re + A[r][p].im * A[r][p].im;
          be += A[r][q].re * A[r][q].re + A[r][q].im * A[r][q].im;
          ga = cfma_conj(A[r][p], A[r][q], ga);
        }
        const double g = sqrt(ga.re * ga.re + ga.im * ga.im);
        if (!(g > 1e-15 * sqrt(al * be)) || g == 0.0) continue;
        rotated = true;
        // make a_p^H a_q real by scaling column q with e^{-i phase(ga)}
        const cx<double> e = mk<double>(ga.re / g, -ga.im / g);
        const double zeta = (be - al) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int r = 0; r < k; ++r) {
          const cx<double> ap = A[r][p], aq = cmul(A[r][q], e);
          A[r][p] = mk<double>(c * ap.re - s * aq.re, c * ap.im - s * aq.im);
          A[r][q] = mk<double>(s * ap.re + c * aq.re, s * ap.im + c * aq.im);
          const cx<double> vp = V[r][p], vq = cmul(V[r][q], e);
          V[r][p] = mk<double>(c * vp.re - s * vq.re, c * vp.im - s * vq.im);
          V[r][q] = mk<double>(s * vp.re + c * vq.re, s * vp.im + c * vq.im);
        }
      }
    if (!rotated) break;
  }
  double sig[kMaxK];
  int ord[kMaxK];
  for (int i = 0; i < k; ++i) {
    double s2 = 0;
    for (int r = 0; r < k; ++r) s2 += A[r][i].re * A[r][i].re + A[r][i].im * A[r][i].im;
    sig[i] = sqrt(s2);
    ord[i] = i;
  }
  for (int i = 0; i < k; ++i)  // selection sort, descending
    for (int jj = i + 1; jj < k; ++jj)
      if (sig[ord[jj]] > sig[ord[i]]) {
        const int t = ord[i];
        ord[i] = ord[jj];
        ord[jj] = t;
      }
  for (int i = 0; i < k; ++i) {
    const int o = ord[i];
    const double s = sig[o];
    gains[((int64_t)m * nw + j) * k + i] = s;
    if (hist) hist[(((int64_t)m * nw + j) * k + i) * 2 + 0] = s;
    for (int r = 0; r < k; ++r) {
      psi[base + r * kMaxK + i] = V[r][o];
      apsi[base + r * kMaxK + i] = A[r][o];
      phi[base + r * kMaxK + i] = s > 0 ? mk<double>(A[r][o].re / s, A[r][o].im / s) : mk<double>(0, 0);
    }
  }
}

// dst (FP64) = 0 or x, with conversion; and non-finite detection over any complex array.
template <typename T>
__global__ __launch_bounds__(256) void finite_kernel(const cx<T>* __restrict__ x, int64_t count, int* flag) {
  bool bad = false;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    const cx<T> v = x[e];
    if (!isfinite((double)v.re) || !isfinite((double)v.im)) bad = true;
  }
  if (bad) atomicOr(flag, 4);
}

template <typename TI, typename TO>
__global__ __launch_bounds__(256) void convert_kernel(const cx<TI>* __restrict__ x, cx<TO>* __restrict__ y,
                                                      int64_t count, double scale) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    const cx<TI> v = x[e];
    y[e] = mk<TO>((TO)(scale * (double)v.re), (TO)(scale * (double)v.im));
  }
}

// Zero fill of 4-byte words (a kernel, so that it can sit in a captured graph where memset nodes are avoided).
__global__ __launch_bounds__(256) void zero_kernel(uint32_t* __restrict__ p, int64_t words) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < words; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = 0u;
}

// ------------------------------------------------------------------------------------------------------
static inline unsigned grid1d(int64_t count) {
  int64_t b = (count + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

int launch_gram(const void* X, int x_fp64, int64_t N, int k, const int64_t* off, int ninst, int nw, int nsplit,
                void* part, int* flag, hipStream_t st) {
  dim3 grid(nsplit, ninst, nw);
#define RES_G(T, KM) hipLaunchKernelGGL((gram_kernel<T, KM>), grid, dim3(256), 0, st, (const cx<T>*)X, N, k, off, \
                                        ninst, nsplit, (cx<double>*)part, flag)
  const int km = gram_km(k);
  if (x_fp64) {
    if (km == 1) RES_G(double, 1); else if (km == 2) RES_G(double, 2); else if (km == 4) RES_G(double, 4); else RES_G(double, 8);
  } else {
    if (km == 1) RES_G(float, 1); else if (km == 2) RES_G(float, 2); else if (km == 4) RES_G(float, 4); else RES_G(float, 8);
  }
#undef RES_G
  return 0;
}

int gram_km(int k) { return k <= 1 ? 1 : k <= 2 ? 2 : k <= 4 ? 4 : 8; }

int launch_chol(const void* part, int nsplit, int k, int nw, int ninst, void* rout, void* rinv, const void* rprev,
                void* rtot, double* hist, int* flag, hipStream_t st) {
  const int n = nw * ninst;
  hipLaunchKernelGGL(chol_kernel, dim3((n + 63) / 64), dim3(64), 0, st, (const cx<double>*)part, nsplit,
                     gram_km(k), k, nw, ninst, (cx<double>*)rout, (cx<double>*)rinv, (const cx<double>*)rprev,
                     (cx<double>*)rtot, hist, flag);
  return 0;
}

int launch_rmul(const void* Xin, int in_fp64, void* Xout, int out_fp64, int64_t N, int k, const int64_t* off,
                int ninst, int nw, int nsplit, const void* M, hipStream_t st) {
  dim3 grid(nsplit, ninst, nw);
  const int km = gram_km(k);
#define RES_R(TI, TO, KM) hipLaunchKernelGGL((rmul_kernel<TI, TO, KM>), grid, dim3(256), 0, st, (const cx<TI>*)Xin, \
                                             (cx<TO>*)Xout, N, k, off, ninst, nsplit, (const cx<double>*)M)
#define RES_RK(TI, TO) \
  if (km == 1) RES_R(TI, TO, 1); else if (km == 2) RES_R(TI, TO, 2); else if (km == 4) RES_R(TI, TO, 4); else RES_R(TI, TO, 8)
  if (in_fp64 && out_fp64) { RES_RK(double, double); }
  else if (in_fp64) { RES_RK(double, float); }
  else if (out_fp64) { RES_RK(float, double); }
  else { RES_RK(float, float); }
#undef RES_RK
#undef RES_R
  return 0;
}

int launch_svd(const void* A, int k, int nw, int ninst, void* phi, void* psi, void* apsi, double* gains,
               double* hist, hipStream_t st) {
  const int n = nw * ninst;
  hipLaunchKernelGGL(svd_kernel, dim3((n + 63) / 64), dim3(64), 0, st, (const cx<double>*)A, k, nw, ninst,
                     (cx<double>*)phi, (cx<double>*)psi, (cx<double>*)apsi, gains, hist);
  return 0;
}

int launch_finite(const void* x, int fp64, int64_t count, int* flag, hipStream_t st) {
  if (fp64) hipLaunchKernelGGL((finite_kernel<double>), dim3(grid1d(count)), dim3(256), 0, st, (const cx<double>*)x, count, flag);
  else hipLaunchKernelGGL((finite_kernel<float>), dim3(grid1d(count)), dim3(256), 0, st, (const cx<float>*)x, count, flag);
  return 0;
}

// Per-(instance, frequency) amplitude weights: fac = sigma_1^(-power) from the leading gain estimates (1 where a
// gain is not a positive finite number).
__global__ void freq_weight_kernel(const double* __restrict__ gains, double* __restrict__ fac, int ninst, int nw,
                                   int k, double power) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst * nw) return;
  const double g = gains[(int64_t)i * k];
  fac[i] = (g > 0.0 && isfinite(g)) ? pow(g, -power) : 1.0;
}

// out[j][c][n] = in[j][c][n] * fac[m(n)][j] (invert: divided by it), m(n) the instance of unknown n; FP64.
__global__ __launch_bounds__(256) void freq_scale_kernel(const cx<double>* __restrict__ in, cx<double>* __restrict__ out,
                                                         int64_t N, int k, int nw, const int64_t* __restrict__ off,
                                                         int ninst, const double* __restrict__ fac, int invert) {
  const int64_t total = (int64_t)nw * k * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = e % N;
    const int64_t j = e / ((int64_t)k * N);
    int lo = 0, hi = ninst - 1;  // instance m with off[m] <= n < off[m+1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off[mid] <= n) lo = mid;
      else hi = mid - 1;
    }
    const double f = fac[(int64_t)lo * nw + j];
    const double w = invert ? 1.0 / f : f;
    const cx<double> v = in[e];
    out[e] = mk<double>(v.re * w, v.im * w);
  }
}

int launch_freq_weights(const double* gains, double* fac, int ninst, int nw, int k, hipStream_t st, double power) {
  const int n = ninst * nw;
  hipLaunchKernelGGL(freq_weight_kernel, dim3((n + 255) / 256), dim3(256), 0, st, gains, fac, ninst, nw, k, power);
  return 0;
}

int launch_freq_scale(const void* in, void* out, int64_t N, int k, int nw, const int64_t* off, int ninst,
                      const double* fac, int invert, hipStream_t st) {
  const int64_t count = (int64_t)nw * k * N;
  hipLaunchKernelGGL(freq_scale_kernel, dim3(grid1d(count)), dim3(256), 0, st, (const cx<double>*)in,
                     (cx<double>*)out, N, k, nw, off, ninst, fac, invert);
  return 0;
}

// out[b][n] = in[b][n] * s[n] for `blocks` consecutive blocks of N values (diagonal B, C and metric scalings).
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void node_scale_kernel(const cx<TI>* in, cx<TO>* out, const double* __restrict__ s,
                                                         int64_t count, int64_t N) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    const double w = s[e % N];
    const cx<TI> v = in[e];
    out[e] = mk<TO>((TO)(w * (double)v.re), (TO)(w * (double)v.im));
  }
}

int launch_node_scale(const void* in, int in_fp64, void* out, int out_fp64, const double* s, int64_t blocks,
                      int64_t N, hipStream_t st) {
  const int64_t count = blocks * N;
#define RES_NS(TI, TO) hipLaunchKernelGGL((node_scale_kernel<TI, TO>), dim3(grid1d(count)), dim3(256), 0, st, \
                                          (const cx<TI>*)in, (cx<TO>*)out, s, count, N)
  if (in_fp64 && out_fp64) RES_NS(double, double);
  else if (in_fp64) RES_NS(double, float);
  else if (out_fp64) RES_NS(float, double);
  else RES_NS(float, float);
#undef RES_NS
  return 0;
}

int launch_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes % 4 != 0) return -1;
  const int64_t words = (int64_t)(bytes / 4);
  if (words > 0) hipLaunchKernelGGL(zero_kernel, dim3(grid1d(words)), dim3(256), 0, st, (uint32_t*)p, words);
  return 0;
}

int launch_convert(const void* x, int in_fp64, void* y, int out_fp64, int64_t count, double scale, hipStream_t st) {
#define RES_C(TI, TO) hipLaunchKernelGGL((convert_kernel<TI, TO>), dim3(grid1d(count)), dim3(256), 0, st, \
                                         (const cx<TI>*)x, (cx<TO>*)y, count, scale)
  if (in_fp64 && out_fp64) RES_C(double, double);
  else if (in_fp64) RES_C(double, float);
  else if (out_fp64) RES_C(float, double);
  else RES_C(float, float);
#undef RES_C
  return 0;
}

}  // namespace res
