// Block Arnoldi (Krylov-subspace) estimates of resolvent gains and modes (Appendix A), FP64.
//
// The basis is stored block by block, [block][n_w][k][N]; for frequency j and instance m the n_m x k matrix of
// block b has columns B_b[j][a][off_m .. off_{m+1}), as the iterates of the power iteration.  The kernels:
//   - xgram: the cross products C_b = B_b^H W of every basis block with a new block W (split over the unknowns,
//     FP64 partial sums, reduced by xgram_reduce into C and, on the first pass, into the projected matrix H);
//   - combine: W -= sum_b B_b C_b (Gram-Schmidt update) or out = (sum_b X_b M_b) diag(s) (Ritz vectors);
//   - heig: cyclic Jacobi eigen-decomposition of the small Hermitian H (one workgroup per frequency and
//     instance), completed from its upper triangle, returning the top k eigenvalues as gains sqrt(lambda) and
//     their eigenvectors.
#include "common.h"
#include "kernels.h"

namespace res {

constexpr int kMaxKrylov = 40;  // basis columns per frequency (blocks * k)

namespace {

__device__ __forceinline__ double kwave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// part[((((bi * nw + j) * ninst + m) * nsplit + sp) * KM + a) * KM + b] = sum over the split's unknowns of
// instance m of conj(B_bi[j][a][n]) W[j][b][n], a, b < k.
template <int KM>
__global__ __launch_bounds__(256) void xgram_kernel(const cx<double>* __restrict__ basis, int64_t bstride,
                                                    const cx<double>* __restrict__ W, int64_t N, int32_t k,
                                                    const int64_t* __restrict__ off, int32_t ninst, int32_t nsplit,
                                                    int32_t nw, cx<double>* __restrict__ part) {
  __shared__ double red[4][2 * KM * KM];
  const int sp = blockIdx.x, m = blockIdx.y;
  const int j = blockIdx.z % nw, bi = blockIdx.z / nw;
  const cx<double>* A = basis + (int64_t)bi * bstride + (int64_t)j * k * N;
  const cx<double>* Wj = W + (int64_t)j * k * N;
  const int64_t lo = off[m], hi = off[m + 1];
  const int64_t chunk = (hi - lo + nsplit - 1) / nsplit;
  const int64_t a0 = lo + sp * chunk;
  const int64_t a1 = (a0 + chunk < hi) ? a0 + chunk : hi;
  double acc_re[KM * KM], acc_im[KM * KM];
#pragma unroll
  for (int p = 0; p < KM * KM; ++p) acc_re[p] = acc_im[p] = 0.0;
  for (int64_t n = a0 + threadIdx.x; n < a1; n += 256) {
    cx<double> x[KM], w[KM];
#pragma unroll
    for (int a = 0; a < KM; ++a) {
      x[a] = a < k ? A[(int64_t)a * N + n] : mk<double>(0, 0);
      w[a] = a < k ? Wj[(int64_t)a * N + n] : mk<double>(0, 0);
    }
#pragma unroll
    for (int a = 0; a < KM; ++a)
#pragma unroll
      for (int b = 0; b < KM; ++b) {
        acc_re[a * KM + b] += x[a].re * w[b].re + x[a].im * w[b].im;
        acc_im[a * KM + b] += x[a].re * w[b].im - x[a].im * w[b].re;
      }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int p = 0; p < KM * KM; ++p) {
    const double r = kwave_sum(acc_re[p]);
    const double i = kwave_sum(acc_im[p]);
    if (lane == 0) {
      red[wv][2 * p] = r;
      red[wv][2 * p + 1] = i;
    }
  }
  __syncthreads();
  if (threadIdx.x < KM * KM) {
    const int p = threadIdx.x;
    const double r = red[0][2 * p] + red[1][2 * p] + red[2][2 * p] + red[3][2 * p];
    const double i = red[0][2 * p + 1] + red[1][2 * p + 1] + red[2][2 * p + 1] + red[3][2 * p + 1];
    part[((((int64_t)bi * nw + j) * ninst + m) * nsplit + sp) * KM * KM + p] = mk<double>(r, i);
  }
}

// C[((j * ninst + m) * nb * k + bi * k + a) * k + b] = sum of the split partials; on the first pass also
// H[((j * ninst + m) * hld + bi * k + a) * hld + col0 + b] (column block col0 / k of the projected matrix).
__global__ void xgram_reduce_kernel(const cx<double>* __restrict__ part, int32_t nsplit, int32_t km, int32_t k,
                                    int32_t nb, int32_t nw, int32_t ninst, cx<double>* __restrict__ C,
                                    cx<double>* __restrict__ H, int32_t hld, int32_t col0) {
  const int64_t total = (int64_t)nb * nw * ninst * k * k;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int b = (int)(e % k);
  const int a = (int)((e / k) % k);
  const int64_t rest = e / ((int64_t)k * k);
  const int m = (int)(rest % ninst);
  const int j = (int)((rest / ninst) % nw);
  const int bi = (int)(rest / ((int64_t)ninst * nw));
  const cx<double>* src = part + (((int64_t)bi * nw + j) * ninst + m) * nsplit * km * km + a * km + b;
  double re = 0, im = 0;
  for (int sp = 0; sp < nsplit; ++sp) {
    re += src[(int64_t)sp * km * km].re;
    im += src[(int64_t)sp * km * km].im;
  }
  const int row = bi * k + a;
  C[(((int64_t)j * ninst + m) * nb * k + row) * k + b] = mk<double>(re, im);
  if (H != nullptr) H[(((int64_t)j * ninst + m) * hld + row) * hld + col0 + b] = mk<double>(re, im);
}

// For n in instance m and columns c < kout:
//   SUBTRACT:  out[j][c][n] -= sum_{bi < nb, a < k} X_bi[j][a][n] M[j][m][bi * k + a][c]
//   otherwise: out[j][c][n]  = s[j][m][c] * sum_{bi < nb, a < k} X_bi[j][a][n] M[j][m][bi * k + a][c]
// M is [n_w][ninst][mld][kout] (rows bi * k + a), s is [n_w][ninst][kout]; the coefficients of one (j, m) are
// staged in LDS (nb * k * kout <= 512).
template <typename RO, int KO, bool SUBTRACT>
__global__ __launch_bounds__(256) void combine_kernel(cx<RO>* out, const cx<double>* __restrict__ X, int64_t xstride,
                                                      int32_t nb, int64_t N, int32_t k, int32_t kout,
                                                      const int64_t* __restrict__ off, int32_t ninst, int32_t nsplit,
                                                      const cx<double>* __restrict__ M, int32_t mld,
                                                      const double* __restrict__ s) {
  __shared__ cx<double> Ms[512];
  const int sp = blockIdx.x, m = blockIdx.y, j = blockIdx.z;
  const int rows = nb * k;
  const cx<double>* Mj = M + ((int64_t)j * ninst + m) * mld * kout;
  for (int t = threadIdx.x; t < rows * kout; t += 256) Ms[t] = Mj[t];
  __syncthreads();
  double sc[KO];
#pragma unroll
  for (int c = 0; c < KO; ++c) sc[c] = (!SUBTRACT && c < kout) ? s[((int64_t)j * ninst + m) * kout + c] : 1.0;
  const int64_t lo = off[m], hi = off[m + 1];
  const int64_t chunk = (hi - lo + nsplit - 1) / nsplit;
  const int64_t a0 = lo + sp * chunk;
  const int64_t a1 = (a0 + chunk < hi) ? a0 + chunk : hi;
  for (int64_t n = a0 + threadIdx.x; n < a1; n += 256) {
    cx<double> y[KO];
#pragma unroll
    for (int c = 0; c < KO; ++c) y[c] = mk<double>(0, 0);
    for (int r = 0; r < rows; ++r) {
      const int bi = r / k, a = r % k;
      const cx<double> x = X[(int64_t)bi * xstride + ((int64_t)j * k + a) * N + n];
#pragma unroll
      for (int c = 0; c < KO; ++c)
        if (c < kout) y[c] = cfma(x, Ms[r * kout + c], y[c]);
    }
#pragma unroll
    for (int c = 0; c < KO; ++c) {
      if (c >= kout) break;
      const int64_t e = ((int64_t)j * kout + c) * N + n;
      if (SUBTRACT) {
        cx<double> o = ccast<double>(out[e]);
        o.re -= y[c].re;
        o.im -= y[c].im;
        out[e] = ccast<RO>(o);
      } else {
        out[e] = ccast<RO>(mk<double>(sc[c] * y[c].re, sc[c] * y[c].im));
      }
    }
  }
}

// Cyclic Jacobi eigen-decomposition of the n x n Hermitian completion of the upper triangle of H[j][m] (leading
// dimension hld), one 64-thread workgroup per (j, m), the matrix and the eigenvectors in LDS.  Each rotation
// zeroes A_pq with G = diag(1, e^{-i phi}) R(theta) on (p, q), A <- G^H A G, V <- V G; sweeps stop when no
// off-diagonal element exceeds 1e-17 sqrt(|A_pp A_qq|) (at most 40 sweeps).  Outputs: gains[(m * nw + j) * k + i]
// = sqrt(max(lambda_i, 0)) for the k largest eigenvalues (descending); if psi != null, psi[j][m][r][i] (leading
// dimension pld rows) = their eigenvectors.
__global__ __launch_bounds__(64) void heig_kernel(const cx<double>* __restrict__ H, int32_t hld, int32_t n,
                                                  int32_t k, int32_t nw, int32_t ninst, double* __restrict__ gains,
                                                  cx<double>* __restrict__ psi, int32_t pld) {
  extern __shared__ cx<double> sm[];
  cx<double>* A = sm;          // [n][n]
  cx<double>* V = sm + n * n;  // [n][n]
  __shared__ int sel[8];
  __shared__ int rotated;
  const int j = blockIdx.x % nw, m = blockIdx.x / nw;
  const int t = threadIdx.x;
  const cx<double>* Hj = H + ((int64_t)j * ninst + m) * hld * hld;
  for (int e = t; e < n * n; e += 64) {
    const int r = e / n, c = e % n;
    cx<double> v = r <= c ? Hj[(int64_t)r * hld + c] : Hj[(int64_t)c * hld + r];
    if (r > c) v.im = -v.im;
    if (r == c) v.im = 0.0;
    A[e] = v;
    V[e] = mk<double>(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (t == 0) rotated = 0;
    __syncthreads();
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cx<double> z = A[p * n + q];
        const double app = A[p * n + p].re, aqq = A[q * n + q].re;
        const double r = sqrt(z.re * z.re + z.im * z.im);
        if (!(r > 1e-17 * sqrt(fabs(app * aqq))) || r < 1e-300) continue;  // uniform: every lane reads the same
        const double er = z.re / r, ei = z.im / r;   // e^{i phi}
        const double zeta = (aqq - app) / (2.0 * r);
        const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + tt * tt), s = tt * c;
        // G = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] on (p, q)
        const cx<double> gpp = mk<double>(c, 0), gpq = mk<double>(s, 0);
        const cx<double> gqp = mk<double>(-s * er, s * ei), gqq = mk<double>(c * er, -c * ei);
        __syncthreads();
        if (t < n) {  // columns p, q of A and V
          const cx<double> ap = A[t * n + p], aq = A[t * n + q];
          A[t * n + p] = cadd(cmul(ap, gpp), cmul(aq, gqp));
          A[t * n + q] = cadd(cmul(ap, gpq), cmul(aq, gqq));
          const cx<double> vp = V[t * n + p], vq = V[t * n + q];
          V[t * n + p] = cadd(cmul(vp, gpp), cmul(vq, gqp));
          V[t * n + q] = cadd(cmul(vp, gpq), cmul(vq, gqq));
        }
        __syncthreads();
        if (t < n) {  // rows p, q of A: A <- G^H A
          const cx<double> ap = A[p * n + t], aq = A[q * n + t];
          A[p * n + t] = cadd(cmul(cconj(gpp), ap), cmul(cconj(gqp), aq));
          A[q * n + t] = cadd(cmul(cconj(gpq), ap), cmul(cconj(gqq), aq));
        }
        __syncthreads();
        if (t == 0) {
          A[p * n + q] = mk<double>(0, 0);
          A[q * n + p] = mk<double>(0, 0);
          A[p * n + p].im = 0.0;
          A[q * n + q].im = 0.0;
          rotated = 1;
        }
        __syncthreads();
      }
    __syncthreads();
    if (!rotated) break;
  }
  if (t == 0) {
    // the k largest eigenvalues, descending
    for (int i = 0; i < k; ++i) {
      int best = -1;
      for (int r = 0; r < n; ++r) {
        bool used = false;
        for (int u = 0; u < i; ++u) used |= sel[u] == r;
        if (!used && (best < 0 || A[r * n + r].re > A[best * n + best].re)) best = r;
      }
      sel[i] = best;
      const double lam = A[best * n + best].re;
      gains[((int64_t)m * nw + j) * k + i] = sqrt(lam > 0 ? lam : 0.0);
    }
  }
  __syncthreads();
  if (psi != nullptr)
    for (int e = t; e < n * k; e += 64) {
      const int r = e / k, i = e % k;
      psi[(((int64_t)j * ninst + m) * pld + r) * k + i] = V[r * n + sel[i]];
    }
}

// inv[(j * ninst + m) * k + i] = 1 / gains[(m * nw + j) * k + i] (0 for a zero gain): the scale of the response
// modes, in the [n_w][ninst][k] order of combine_kernel.
__global__ void recip_gains_kernel(const double* __restrict__ gains, double* __restrict__ inv, int32_t ninst,
                                   int32_t nw, int32_t k) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)ninst * nw * k) return;
  const int i = (int)(e % k);
  const int m = (int)((e / k) % ninst);
  const int j = (int)(e / ((int64_t)k * ninst));
  const double g = gains[((int64_t)m * nw + j) * k + i];
  inv[e] = g > 0 ? 1.0 / g : 0.0;
}

}  // namespace

int launch_recip_gains(const double* gains, double* inv, int ninst, int nw, int k, hipStream_t st) {
  const int64_t n = (int64_t)ninst * nw * k;
  hipLaunchKernelGGL(recip_gains_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, gains, inv, ninst, nw,
                     k);
  return 0;
}

int launch_xgram(const void* basis, int64_t bstride, int nb, const void* W, int64_t N, int k, const int64_t* off,
                 int ninst, int nw, int nsplit, void* part, hipStream_t st) {
  if ((int64_t)nw * nb > 65535 || ninst > 65535) return -1;
  dim3 grid(nsplit, ninst, nw * nb);
  const int km = gram_km(k);
#define RES_X(KM) hipLaunchKernelGGL((xgram_kernel<KM>), grid, dim3(256), 0, st, (const cx<double>*)basis, bstride, \
                                     (const cx<double>*)W, N, k, off, ninst, nsplit, nw, (cx<double>*)part)
  if (km == 1) RES_X(1); else if (km == 2) RES_X(2); else if (km == 4) RES_X(4); else RES_X(8);
#undef RES_X
  return 0;
}

int launch_xgram_reduce(const void* part, int nsplit, int k, int nb, int nw, int ninst, void* C, void* H, int hld,
                        int col0, hipStream_t st) {
  const int64_t total = (int64_t)nb * nw * ninst * k * k;
  hipLaunchKernelGGL(xgram_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     (const cx<double>*)part, nsplit, gram_km(k), k, nb, nw, ninst, (cx<double>*)C, (cx<double>*)H,
                     hld, col0);
  return 0;
}

int launch_combine(void* out, int out_fp64, int subtract, const void* X, int64_t xstride, int nb, int64_t N, int k,
                   int kout, const int64_t* off, int ninst, int nw, int nsplit, const void* M, int mld,
                   const double* s, hipStream_t st) {
  if (nb * k * kout > 512 || kout > 8) return -1;
  dim3 grid(nsplit, ninst, nw);
#define RES_C(RO, KO, SUB) hipLaunchKernelGGL((combine_kernel<RO, KO, SUB>), grid, dim3(256), 0, st, (cx<RO>*)out, \
                                              (const cx<double>*)X, xstride, nb, N, k, kout, off, ninst, nsplit, \
                                              (const cx<double>*)M, mld, s)
  const int ko = gram_km(kout);
  if (subtract) {
    if (ko == 1) RES_C(double, 1, true); else if (ko == 2) RES_C(double, 2, true);
    else if (ko == 4) RES_C(double, 4, true); else RES_C(double, 8, true);
  } else if (out_fp64) {
    if (ko == 1) RES_C(double, 1, false); else if (ko == 2) RES_C(double, 2, false);
    else if (ko == 4) RES_C(double, 4, false); else RES_C(double, 8, false);
  } else {
    if (ko == 1) RES_C(float, 1, false); else if (ko == 2) RES_C(float, 2, false);
    else if (ko == 4) RES_C(float, 4, false); else RES_C(float, 8, false);
  }
#undef RES_C
  return 0;
}

int launch_heig(const void* H, int hld, int n, int k, int nw, int ninst, double* gains, void* psi, int pld,
                hipStream_t st) {
  if (n < 1 || n > kMaxKrylov || k > n || k > 8) return -1;  // 2 n^2 complex in LDS, within 64 KiB
  const size_t lds = (size_t)2 * n * n * sizeof(cx<double>);
  hipLaunchKernelGGL(heig_kernel, dim3((unsigned)(nw * ninst)), dim3(64), lds, st, (const cx<double>*)H, hld, n, k,
                     nw, ninst, gains, (cx<double>*)psi, pld);
  return 0;
}

}  // namespace res
