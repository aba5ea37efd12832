// Kernel launchers of the resolvent library (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace res {

// ---- 1-D stepper --------------------------------------------------------------------------------------
constexpr int kStep1DConfigs = 16;
struct Step1DArgs {
  int fp64;
  int cfg;                 // index into the (threads, unknowns per thread, prefetch depth) table
  const Seg1D* segs;
  int64_t nseg;
  int mstep;               // RK4 steps per kernel step: 1, 2 or 4
  const void* band;        // [N][8*mstep+1] complex (working precision): P(Z)^mstep
  const void* state_in;    // [ncol][N]
  void* state_out;         // [ncol][N] (may equal state_in when every region is owned entirely)
  int64_t N, row_len;      // row_len = ncol * N
  int64_t n_steps;
  const void* frc;         // forcing rows or null
  int64_t frc_row0, frc_period;
  double phi_re, phi_im;
  void* snap;              // snapshot rows (length snap_ld >= row_len + 1) or null
  int64_t snap_ld, snap_first, snap_stride, snap_count, snap_row0;
  // persistent variant: blocks of `block` steps with neighbour exchange through xbuf ([2][2][row_len] complex
  // slots in uncached memory, every slot empty at launch: launch_fill_empty)
  int persist;
  void* xbuf;
  int64_t block;
  uint64_t spin_ns;
  int* err;
};
int step1d_coresident(int fp64, int cfg, int device, int mstep);
int launch_step1d_m2(const Step1DArgs& a, hipStream_t st);
int launch_step1d_m4(const Step1DArgs& a, hipStream_t st);
int step1d_coresident_m2(int fp64, int cfg, int device);
int step1d_coresident_m4(int fp64, int cfg, int device);
int step1d_prefetch(int cfg);
int step1d_capacity(int cfg);
int launch_step1d(const Step1DArgs& a, hipStream_t st);
int launch_fill_empty(void* xbuf, int fp64, int64_t count, hipStream_t st);
int launch_tri_horner(const cx<double>* tri, const cx<double>* yin, const void* F, int f_fp64, void* yout,
                      int out_fp64, int64_t N, int k, int nw, double sw0h, double sdwh, double h, int pass,
                      hipStream_t st, int j0 = 0);
// y = P x + e^{i sw_j h i} G over [n_w][k][N] FP64 blocks (multi-step forcing combination; band FP64 [N][9])
// The Horner launchers take blocks of frequencies j0 .. j0 + nw - 1 (w_j = w0 + j dw): the pointers address
// block j0, the phases use the global index.
int launch_band_horner(const cx<double>* band, const cx<double>* x, const cx<double>* G, void* y, int out_fp64,
                       int64_t N, int k, int nw, double sw0h, double sdwh, int i, hipStream_t st, int j0 = 0);

// ---- 2-D / 3-D stencils -------------------------------------------------------------------------------
// Device coefficients of Z = h L on an nx*ny*nz grid (real, working precision or FP64): per x-line
// neighbour coefficients [ny*nz], diagonal [nodes], 3x3 component coupling per line [ny*nz][3][3] or null.
struct GridOpDev {
  int ncomp;
  int64_t nx, ny, nz;
  const void* cxm; const void* cxp; const void* cym; const void* cyp; const void* czm; const void* czp;
  const void* d;
  const void* K;
  int kmask;  // bit c*3+c' set when K[.][c][c'] is nonzero on some line (0 without coupling)
  // FP32 three-component sets: the line coefficients packed per line, [lines][8] = cxm cxp cym cyp czm czp kA kB,
  // with (kA, kB) = (K01, K02) when kv = 1 (the shear terms of the first component), (K10, K20) when kv = 2 (their
  // transpose), unused otherwise (kv = 0: no coupling, 3: general, read from K); null for other sets
  const void* lc;
  int kv;
};
// Two Horner stages of a 3-D three-component operator in one launch, marching along z (see stencil.hip): pass 1
// (second = 0) writes the third stage's input from u, pass 2 the new state from vin and u (out != u).
int launch_grid_pair3d(const GridOpDev& g, int fp64, int k, const void* u, const void* vin, void* out, int second,
                       const void* frc, double phr, double phi, void* snap, hipStream_t st);
// Whole RK4 step of a 3-D three-component operator in one launch (four stages pipelined along z), FP32 state;
// uout != uin.  Returns -1 for other operators.
int launch_grid_step3d(const GridOpDev& g, int k, const void* uin, void* uout, const void* frc, double phr,
                       double phi, void* snap, hipStream_t st);
// Whole RK4 step of a 2-D one-component operator in one launch (LDS temporal blocking); uout != uin.
int launch_grid_step2d(const GridOpDev& g, int fp64, int k, const void* uin, void* uout, const void* frc, double phr,
                       double phi, void* snap, hipStream_t st);
// Two RK4 steps of a 2-D one-component operator (FP32) in one launch: frc/snap belong to the first step,
// frc2/snap2 to the second (each may be NULL); wy = 48 or 64 (window rows).  The same bits as two launches of
// launch_grid_step2d.
int launch_grid_step2d_pair(const GridOpDev& g, int k, const void* uin, void* uout, const void* frc,
                            const void* frc2, double phr, double phi, void* snap, void* snap2, int wy,
                            hipStream_t st);
int launch_grid_horner(const GridOpDev& g64, const cx<double>* yin, const void* F, int f_fp64, void* yout,
                       int out_fp64, int k, int nw, double sw0h, double sdwh, double h, int pass, hipStream_t st,
                       int j0 = 0);

// ---- discrete adjoint (reverse-mode) stage kernels ------------------------------------------------------
// kind 0: three-point complex operator, tri = [nsite][3] (lower, diag, upper) of Z (or Z^H); kind 1: grid
// operator g (FP64 coefficients), nsite = nodes, ncomp components per node.  Columns are [k][ncomp][nsite].
// FP64 arithmetic and mu accumulation; the rows are complex FP64 if rows64, else complex FP32.
struct AdjOpDev {
  int kind;
  int ncomp;
  int64_t nsite;
  const void* tri;
  GridOpDev g;
};
int launch_fwd_stage(const AdjOpDev& op, int k, int m, const void* u, void* uout, const void* yin, void* yout,
                     void* acc, const void* f, double h, hipStream_t st, const void* gadd, int rows64);
// The four forward stages of one step in one launch for a 2-D one-component grid operator (stage inputs y2, y3, y4
// and uout may each be null; uout must not alias u).  gadd (null: none) is added to uout: with fa = fb = fc = null
// the step is u' = P(Z) u + gadd, the march with pre-filtered forcing rows.  Returns -1 for other operators.
int launch_fwd_step2d(const AdjOpDev& op, int k, const void* u, void* uout, void* y2, void* y3, void* y4,
                      const void* fa, const void* fb, const void* fc, double h, hipStream_t st, const void* gadd,
                      int rows64);
// The four reverse stages of one step in one launch for a 2-D one-component grid operator (one workgroup per tile
// and column; the mu contributions go to the per-column rows mu_cols [k][nodes]; lam_out must not alias lam).
// Returns -1 for other operators.
int launch_rev_step2d(const AdjOpDev& opH, int k, const void* lam, void* lam_out, const void* y2, const void* y3,
                      const void* y4, const void* u, double* mu_cols, const void* inj, double h, hipStream_t st,
                      int rows64);
// mu[p] += sum over the k rows of cols [k][n].
int launch_sum_columns(const double* cols, int k, int64_t n, double* mu, hipStream_t st);
// Grid rows (and mu rows) of the reverse stage launches for k columns.
int rev_stage_rows(int k);
int launch_rev_stage(const AdjOpDev& opH, int k, int m, const void* lam, void* lam_out, const void* kin,
                     const void* y, void* kout, const void* k3, const void* k2, double* mu, const void* inj, double h,
                     hipStream_t st, int rows64);

// ---- block Arnoldi (krylov.hip) ---------------------------------------------------------------------------
int launch_xgram(const void* basis, int64_t bstride, int nb, const void* W, int64_t N, int k, const int64_t* off,
                 int ninst, int nw, int nsplit, void* part, hipStream_t st);
int launch_xgram_reduce(const void* part, int nsplit, int k, int nb, int nw, int ninst, void* C, void* H, int hld,
                        int col0, hipStream_t st);
int launch_combine(void* out, int out_fp64, int subtract, const void* X, int64_t xstride, int nb, int64_t N, int k,
                   int kout, const int64_t* off, int ninst, int nw, int nsplit, const void* M, int mld,
                   const double* s, hipStream_t st);
int launch_heig(const void* H, int hld, int n, int k, int nw, int ninst, double* gains, void* psi, int pld,
                hipStream_t st);
int launch_recip_gains(const double* gains, double* inv, int ninst, int nw, int k, hipStream_t st);

// ---- phase GEMMs --------------------------------------------------------------------------------------
struct PhaseGemmArgs {
  int mode;                // 0 synthesis, 1 projection
  int64_t M, Ncols, K;
  const void* btab;        // [P] complex (working precision): e^{2 pi i m / P}
  int64_t P;
  int sigma;               // +1 direct, -1 adjoint
  double w0h;              // omega0 * h
  int64_t s0, stride;      // synthesis: first step; projection: step of sample 0 and sample spacing
  const void* bmat;        // [K][ldb] (ldb >= Ncols; 0 means Ncols)
  int64_t ldb;
  void* out;               // synthesis: [M][Ncols] working precision; projection: FP64 accumulator [M][Ncols]
  double scale;            // projection scale
  int64_t k_per_split;     // K entries per split (projection), >= K for no split
  void* partial;           // projection split partials (FP64) or null
};
int launch_phase_gemm(const PhaseGemmArgs& a, int fp64, hipStream_t st);
int launch_reduce_partials(const void* part, void* acc, int64_t count, int nsplit, double scale, hipStream_t st);
// Phase table t[m] = e^{2 pi i m / P}, m < P (working precision), computed on the device.
int launch_phase_table(void* t, int fp64, int64_t P, hipStream_t st);

// ---- per-frequency QR / SVD ----------------------------------------------------------------------------
int gram_km(int k);
int launch_gram(const void* X, int x_fp64, int64_t N, int k, const int64_t* off, int ninst, int nw, int nsplit,
                void* part, int* flag, hipStream_t st);
int launch_chol(const void* part, int nsplit, int k, int nw, int ninst, void* rout, void* rinv, const void* rprev,
                void* rtot, double* hist, int* flag, hipStream_t st);
int launch_rmul(const void* Xin, int in_fp64, void* Xout, int out_fp64, int64_t N, int k, const int64_t* off,
                int ninst, int nw, int nsplit, const void* M, hipStream_t st);
int launch_svd(const void* A, int k, int nw, int ninst, void* phi, void* psi, void* apsi, double* gains,
               double* hist, hipStream_t st);
int launch_finite(const void* x, int fp64, int64_t count, int* flag, hipStream_t st);
int launch_convert(const void* x, int in_fp64, void* y, int out_fp64, int64_t count, double scale, hipStream_t st);
// out[b][n] = in[b][n] * s[n] over `blocks` blocks of N values (in place allowed when the types match).
int launch_node_scale(const void* in, int in_fp64, void* out, int out_fp64, const double* s, int64_t blocks,
                      int64_t N, hipStream_t st);
int launch_zero(void* p, size_t bytes, hipStream_t st);  // bytes: a multiple of 4

// ---- transient-response method with time-domain hand-off (trm.hip) ------------------------------------------
// Stage-forcing pre-filter of a run forced by a sampled signal S [n][ncols] (working precision, sample i at step
// i*every, read reversed if rev): pass 0 and 1 write FP64 xout, pass 2 the forcing rows g (working precision) of
// steps s0 .. s0 + rows - 1.  scheme: 0 linear, 1 cubic Hermite, 2 quintic Hermite.
int launch_signal_prefilter(const void* S, int64_t n, int every, int scheme, int rev, const cx<double>* tri,
                            const void* xin, void* xout, void* g, int fp64, int g_fp64, int64_t s0, int64_t rows,
                            int64_t N, int64_t ncols, double h, int pass, hipStream_t st);
// Horner pass i (1 <= i < M) of the combined forcing of M steps over per-step FP64 rows g: out = P xin + g_{RM+i}.
int launch_row_horner(const cx<double>* band, const void* xin, int64_t xstride, const void* g, int M, int i,
                      void* out, int out_fp64, int64_t rows, int64_t N, int64_t ncols, hipStream_t st);
int launch_copy_rows(const void* src, int64_t src_ld, void* dst, int64_t row0, int dir, int64_t rows, int64_t ncols,
                     int fp64, hipStream_t st);
// Grid operators: the signal at the half steps of a tile (FP64 [nhalf][ncols]), and one pre-filter pass over `rows`
// steps with the FP64 coefficient set g64 (passes 0, 1 write FP64 xout; pass 2 the rows g, working precision).
int launch_signal_half_rows(const void* S, int64_t n, int every, int scheme, int rev, int fp64, void* H, int64_t s0,
                            int64_t nhalf, int64_t ncols, hipStream_t st);
int launch_grid_signal_pass(const GridOpDev& g64, const void* H, const void* xin, void* xout, void* g, int out_fp64,
                            int k, int64_t rows, double h, int pass, hipStream_t st);
int fir_max_order();
// y = delay-compensated FIR of x along time (taps FP64 complex [order+1] on the device), times the taper of
// `pad`/`ramp` samples (pad < 0: none).  Returns -1 for an order beyond fir_max_order().
int launch_fir(const cx<double>* taps, int order, const void* x, void* y, int64_t Tn, int64_t ncols, int64_t pad,
               int64_t ramp, int fp64, hipStream_t st);
// out [nw][ncols] FP64 = dt sum_i x_i e^{-i w_j t_i}; part: series_dft_part_elems(...) FP64 complex scratch.
int64_t series_dft_part_elems(int64_t Tn, int64_t ncols, int nw);
int launch_series_dft(const void* x, int fp64, int64_t Tn, int64_t ncols, const double* omegas, int nw, double dt,
                      void* part, void* out, hipStream_t st);
// FIR taps [order + 1] (FP64 complex) from the response sampled at M frequencies and the table E[p] = e^{2 pi i p/M}.
int launch_fir_taps(const double* D, const void* E, int64_t M, int order, void* taps, hipStream_t st);
int launch_row_norms(const void* X, int64_t nrows, int64_t ncols, double* norms, hipStream_t st);
// out[j][c] = X[j][c] / norms[j], X FP64 [nrows][ncols], out working precision.
int launch_scale_rows(const void* X, const double* norms, int64_t nrows, int64_t ncols, void* out, int out_fp64,
                      hipStream_t st);
int normalise_parts();
int launch_normalise(void* x, int fp64, int64_t count, double* part, double* scale, hipStream_t st);
// Amplitude weights of the block power iteration (fac[ninst][nw] = 1/sqrt(leading gain)) and their application
// to FP64 blocks [nw][k][N] (invert: divide).
int launch_freq_weights(const double* gains, double* fac, int ninst, int nw, int k, hipStream_t st,
                        double power = 0.5);
int launch_freq_scale(const void* in, void* out, int64_t N, int k, int nw, const int64_t* off, int ninst,
                      const double* fac, int invert, hipStream_t st);

}  // namespace res
