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
#include "common.h"
#include "kernels.h"

namespace res {

// One workgroup marches one segment (a column's run of whole instances) for n_steps steps.  Thread t owns V
// consecutive unknowns held in registers together with their nine stencil coefficients; the state is
// exchanged through a double-buffered LDS row once per step (one barrier per step).  Forcing rows are
// prefetched PD steps ahead into a register ring.
//
// Forcing of local step t: phi * frc[row][col*N + i] with row = frc_row0 + t (mod frc_period if > 0).
// Snapshot rows: u_t (the state BEFORE step t's update) is written to snap[snap_row0 + m] for
// t = snap_first + m*snap_stride, m < snap_count.
template <typename R, int NT, int V, int PD>
__global__ __launch_bounds__(NT) void step1d_kernel(const Seg1D* __restrict__ segs, const cx<R>* __restrict__ band,
                                                    cx<R>* __restrict__ state, int64_t N, int64_t row_len,
                                                    int64_t n_steps, const cx<R>* __restrict__ frc,
                                                    int64_t frc_row0, int64_t frc_period, R phi_re, R phi_im,
                                                    cx<R>* __restrict__ snap, int64_t snap_first,
                                                    int64_t snap_stride, int64_t snap_count, int64_t snap_row0) {
  constexpr int W = NT * V + 2 * kBandRadius;
  __shared__ cx<R> buf[2][W];
  const Seg1D sg = segs[blockIdx.x];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)sg.col * N + sg.dof0;
  const cx<R> zero = mk<R>(0, 0);
  const cx<R> phi = mk<R>(phi_re, phi_im);

  cx<R> p[V][kBandWidth];
  cx<R> u[V];
  bool valid[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int64_t l = (int64_t)tid * V + v;
    valid[v] = l < sg.ndof;
    u[v] = valid[v] ? state[base + l] : zero;
#pragma unroll
    for (int d = 0; d < kBandWidth; ++d) p[v][d] = valid[v] ? band[(sg.dof0 + l) * kBandWidth + d] : zero;
  }
  if (tid < kBandRadius) {
    buf[0][tid] = zero;
    buf[1][tid] = zero;
    buf[0][W - 1 - tid] = zero;
    buf[1][W - 1 - tid] = zero;
  }

  cx<R> f[PD][V];
  // Forcing rows are loaded strictly in step order, so the (wrapping) row index advances by one per load.
  int64_t lrow = frc_period > 0 ? frc_row0 % frc_period : frc_row0;
  auto load_forcing = [&](int64_t t, cx<R>* dst) {
    if (frc == nullptr || t >= n_steps) {
#pragma unroll
      for (int v = 0; v < V; ++v) dst[v] = zero;
      return;
    }
    const cx<R>* src = frc + lrow * row_len + base + (int64_t)tid * V;
    if (++lrow == frc_period) lrow = 0;
#pragma unroll
    for (int v = 0; v < V; ++v) dst[v] = valid[v] ? load_nt<R>(src + v) : zero;
  };
#pragma unroll
  for (int q = 0; q < PD; ++q) load_forcing(q, f[q]);

  int64_t next_snap = (snap != nullptr && snap_count > 0) ? snap_first : -1;
  int64_t snap_m = 0;

  for (int64_t t0 = 0; t0 < n_steps; t0 += PD) {
#pragma unroll
    for (int q = 0; q < PD; ++q) {
      const int64_t t = t0 + q;
      if (t < n_steps) {
        cx<R>* row = buf[t & 1];
#pragma unroll
        for (int v = 0; v < V; ++v) row[kBandRadius + tid * V + v] = u[v];
        __syncthreads();
        if (t == next_snap) {
          cx<R>* dst = snap + (snap_row0 + snap_m) * row_len + base + (int64_t)tid * V;
#pragma unroll
          for (int v = 0; v < V; ++v)
            if (valid[v]) dst[v] = u[v];
          ++snap_m;
          next_snap = (snap_m < snap_count) ? next_snap + snap_stride : -1;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
          cx<R> acc = cmul(phi, f[q][v]);
#pragma unroll
          for (int d = 0; d < kBandWidth; ++d) acc = cfma(p[v][d], row[tid * V + v + d], acc);
          u[v] = acc;
        }
        load_forcing(t + PD, f[q]);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v)
    if (valid[v]) state[base + (int64_t)tid * V + v] = u[v];
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
                                                         double h, int pass) {
  const int64_t total = (int64_t)nw * k * N;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = e % N;
    const int64_t j = e / ((int64_t)k * N);
    double sa, ca;
    sincos(0.5 * (sw0h + (double)j * sdwh), &sa, &ca);
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

// ---------------------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------------------
template <typename R, int NT, int V, int PD>
static void launch_step1d_cfg(const Step1DArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((step1d_kernel<R, NT, V, PD>), dim3(a.nseg), dim3(NT), 0, st, a.segs,
                     (const cx<R>*)a.band, (cx<R>*)a.state, a.N, a.row_len, a.n_steps, (const cx<R>*)a.frc,
                     a.frc_row0, a.frc_period, (R)a.phi_re, (R)a.phi_im, (cx<R>*)a.snap, a.snap_first,
                     a.snap_stride, a.snap_count, a.snap_row0);
}

template <typename R> static int launch_step1d_t(const Step1DArgs& a, hipStream_t st) {
  switch (a.cfg) {
    case 0: launch_step1d_cfg<R, 64, 1, 4>(a, st); break;
    case 1: launch_step1d_cfg<R, 128, 1, 4>(a, st); break;
    case 2: launch_step1d_cfg<R, 256, 1, 4>(a, st); break;
    case 3: launch_step1d_cfg<R, 256, 2, 4>(a, st); break;
    case 4: launch_step1d_cfg<R, 256, 4, 2>(a, st); break;
    case 5: launch_step1d_cfg<R, 256, 8, 2>(a, st); break;
    case 6: launch_step1d_cfg<R, 512, 4, 2>(a, st); break;
    case 7: launch_step1d_cfg<R, 1024, 2, 2>(a, st); break;
    case 8: launch_step1d_cfg<R, 512, 2, 4>(a, st); break;
    case 9: launch_step1d_cfg<R, 1024, 1, 4>(a, st); break;
    default: return -1;
  }
  return 0;
}

int step1d_capacity(int cfg) {
  static const int cap[] = {64, 128, 256, 512, 1024, 2048, 2048, 2048, 1024, 1024};
  return (cfg >= 0 && cfg < kStep1DConfigs) ? cap[cfg] : 0;
}

int launch_step1d(const Step1DArgs& a, hipStream_t st) {
  return a.fp64 ? launch_step1d_t<double>(a, st) : launch_step1d_t<float>(a, st);
}

int launch_tri_horner(const cx<double>* tri, const cx<double>* yin, const void* F, int f_fp64, void* yout,
                      int out_fp64, int64_t N, int k, int nw, double sw0h, double sdwh, double h, int pass,
                      hipStream_t st) {
  const int64_t total = (int64_t)nw * k * N;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
#define RES_TH(TF, TO)                                                                                         \
  hipLaunchKernelGGL((tri_horner_kernel<TF, TO>), dim3((unsigned)blocks), dim3(256), 0, st, tri, yin,         \
                     (const cx<TF>*)F, (cx<TO>*)yout, N, k, nw, sw0h, sdwh, h, pass)
  if (f_fp64 && out_fp64) RES_TH(double, double);
  else if (f_fp64 && !out_fp64) RES_TH(double, float);
  else if (!f_fp64 && out_fp64) RES_TH(float, double);
  else RES_TH(float, float);
#undef RES_TH
  return 0;
}

}  // namespace res
