// Reverse mode of the host runtime: the gradient of a real objective of u_hat = resolvent_apply(f_hat) with respect
// to f_hat and to a real perturbation of L's diagonal (checkpointed forward march, segment recomputation, the
// reverse stages and the forcing gradient's projection), and its C ABI entry points.
#include "runtime_state.h"

namespace rt {

// ---------------------------------------------------------------------------------------------------------
// Reverse mode: gradient of a real objective of u_hat = resolvent_apply(f_hat) with respect to f_hat and to a real
// perturbation of L's diagonal, by the exact discrete adjoint of the classical four-stage march (see adjoint.hip).
//
// The forward trajectory is marched once in stage form (FP64, raw forcing sampled at the stage times t_s,
// t_s + h/2, t_s + h, synthesised on the half-step grid) keeping the state every C steps; the segments are then
// visited in reverse: the states of the segment are recomputed from its checkpoint, and each step runs three
// stage recomputations and four reverse stages.  The adjoint state lambda_s = dJ/du_s receives the projection's
// seed scale * sum_j e^{+i w_j t_s} g_j at the sampled steps.  The forcing gradient uses the single-step form
// u_{s+1} = P(Z) u_s + sum_j e^{i w_j t_s} h Q_j(Z) F_j:  F_grad_j = (h Q_j(Z))^H sum_{forced s} e^{-i w_j t_s}
// lambda_{s+1}, i.e. a Fourier projection of the lambda rows followed by the forcing pre-filter of Z^H at the
// negated frequencies ((h Q_w(Z))^H = h Q_{-w}(Z^H)).
AdjOpDev adj_op(const resolvent_op* op, int s) {
  AdjOpDev a{};
  if (is_grid(op)) {
    a.kind = 1;
    a.ncomp = op->ncomp;
    a.nsite = op->nx * op->ny * op->nz;
    a.g = op->g64[s];
  } else {
    a.kind = 0;
    a.ncomp = 1;
    a.nsite = op->N;
    a.tri = op->d_tri[s];
  }
  return a;
}

// One chunk of kc columns.  F: raw forcing rows [nw][kc][N] in the row precision (null without mu_grad); G: the
// scaled seed in the row precision; f_out: forcing gradient [nw][kc][N] in the working precision, or null; mu_grad
// (FP64 [nsite]) receives += this chunk's contribution.  Every row buffer holds the row precision: FP64 (r64), or
// FP32 with FP64 arithmetic in the kernels and FP64 accumulation of both gradients.
int backward_chunk(resolvent_op* op, const Plan& pl, int k, int r64, const void* F, const void* G, void* f_out,
                   double* mu_grad, int64_t C, hipStream_t st) {
  const int64_t N = op->N, ncols = (int64_t)k * N, S = pl.S;
  const int nw = pl.nw;
  const size_t rowb = (size_t)ncols * (r64 ? sizeof(cd) : sizeof(std::complex<float>));
  const double h = op->h;
  const int64_t ncp = (S + C - 1) / C;
  const AdjOpDev fwd = adj_op(op, 0), rev = adj_op(op, 1);
  const int64_t nsite = fwd.nsite;
  const bool need_states = mu_grad != nullptr;

  void *frow, *cps, *seg, *u, *acc, *y2, *y3, *y4, *ka, *kb, *ub, *lrows, *carry, *inj, *facc = nullptr;
  void *btab_half = nullptr, *btab;
  frow = cps = seg = nullptr;
  if (need_states) {
    RES_TRY(ws_get(op, "bw_frow", (size_t)(2 * C + 1) * rowb, &frow));
    RES_TRY(ws_get(op, "bw_ckpt", (size_t)ncp * rowb, &cps));
    RES_TRY(ws_get(op, "bw_seg", (size_t)C * rowb, &seg));
  }
  RES_TRY(ws_get(op, "bw_u", rowb, &u));
  RES_TRY(ws_get(op, "bw_acc", rowb, &acc));
  RES_TRY(ws_get(op, "bw_y2", rowb, &y2));
  RES_TRY(ws_get(op, "bw_y3", rowb, &y3));
  RES_TRY(ws_get(op, "bw_y4", rowb, &y4));
  RES_TRY(ws_get(op, "bw_ka", rowb, &ka));
  RES_TRY(ws_get(op, "bw_kb", rowb, &kb));
  RES_TRY(ws_get(op, "bw_ub", rowb, &ub));
  RES_TRY(ws_get(op, "bw_carry", rowb, &carry));
  RES_TRY(ws_get(op, "bw_inj", (size_t)C * rowb, &inj));
  if (f_out) {
    RES_TRY(ws_get(op, "bw_facc", (size_t)nw * ncols * sizeof(cd), &facc));
    RES_TRY(zero_device(facc, (size_t)nw * ncols * sizeof(cd), st));
  }
  if (r64) {
    if (need_states) RES_TRY(phase_table64(op, 2 * pl.P, &btab_half));
    RES_TRY(phase_table64(op, pl.P, &btab));
  } else {
    if (need_states) RES_TRY(phase_table(op, 2 * pl.P, &btab_half));
    RES_TRY(phase_table(op, pl.P, &btab));
  }
  auto row = [&](void* base, int64_t r) { return (void*)((char*)base + (size_t)r * rowb); };
  // raw forcing of steps [sa, sb) for the segment recomputation: half-step samples 2 sa .. 2 sb.  The GEMM works
  // on 64-row tiles, so the 2 C + 1 samples of a whole segment would take a third tile for a single row: with
  // `shared`, the last sample is the first one (row 0) of the segment synthesised just before (the next one in
  // time: segments are visited in reverse) and is copied instead.
  auto synth_segment = [&](int64_t sa, int64_t sb, bool shared) -> int {
    if (sa >= pl.forced_end) return RES_OK;
    const int64_t len = sb - sa;
    int64_t n = 2 * len + 1;
    if (shared) {
      HIP_TRY(hipMemcpyAsync(row(frow, 2 * len), row(frow, 0), rowb, hipMemcpyDeviceToDevice, st));
      --n;
    }
    return synth_rows(r64, nw, 2 * pl.P, pl.w0 * h * 0.5, +1, btab_half, F, ncols, 2 * sa, 1, n, frow, st);
  };
  auto frc = [&](int64_t s, int64_t r, int half) -> const void* {
    return s < pl.forced_end ? row(frow, 2 * r + half) : nullptr;
  };
  auto first_m_at_or_after = [&](int64_t t) -> int64_t {
    if (t <= pl.pfirst) return 0;
    return std::min(pl.pcount, (t - pl.pfirst + pl.pstride - 1) / pl.pstride);
  };

  // 2-D one-component grids take the four forward stages of a step in one LDS-tiled launch (launch_fwd_step2d);
  // other operators one launch per stage.  The fused step cannot update the state in place, so the checkpoint
  // march ping-pongs between u and a second row.
  const bool fused = fwd.kind == 1 && fwd.ncomp == 1 && fwd.g.nz == 1;
  // Mixed-precision three-component grids with FP32 rows march the checkpoint states, and the adjoint recursion
  // when no mu gradient is asked for, with the forward march's fused one-launch step (launch_grid_step3d, FP32
  // arithmetic): u' = P(Z) u + G_s and lambda_s = P(Z^H) lambda_{s+1} + seed_s, since P(Z)^H = P(Z^H).  Both
  // need only the states; the stage values of the recomputed segments and the reverse stages of the mu gradient
  // keep the stage kernels.
  const bool fused3 = fwd.kind == 1 && fwd.ncomp == 3 && !r64 && !op->fp64();
  void* u2 = nullptr;
  // per-column mu rows of the reverse steps (one row per column, or per grid row of the stage launches), summed at
  // the end: the columns of a node run in different threads, and the sum stays deterministic
  double* mu_cols = nullptr;
  const int mu_rows = fused ? k : rev_stage_rows(k);
  if (fused || fused3) RES_TRY(ws_get(op, "bw_u2", rowb, &u2));
  if (mu_grad) {
    void* p;
    RES_TRY(ws_get(op, "bw_mu_cols", (size_t)mu_rows * nsite * sizeof(double), &p));
    mu_cols = (double*)p;
    RES_TRY(zero_device(mu_cols, (size_t)mu_rows * nsite * sizeof(double), st));
  }

  // 1. forward march with checkpoints.  It only needs the states, so it steps u' = P(Z) u + sum_j e^{i w_j t_s} G_j
  // with the pre-filtered forcing G_j = h Q_j(Z) F_j (FP64 Horner passes, stored in the row precision): one
  // synthesised row per step instead of two half-step rows, read once per step instead of at every stage.
  void* Gpre = nullptr;
  if (need_states && pl.forced_end > 0) {
    RES_TRY(ws_get(op, "bw_Gpre", (size_t)nw * rowb, &Gpre));
    RES_TRY(prefilter(op, pl, k, F, r64, Gpre, +1, 1, st, r64));
  }
  RES_TRY(zero_device(u, rowb, st));
  void* ucur = u;
  for (int64_t c = 0; c < (need_states ? ncp : 0); ++c) {
    const int64_t sa = c * C, sb = std::min(S, sa + C);
    HIP_TRY(hipMemcpyAsync(row(cps, c), ucur, rowb, hipMemcpyDeviceToDevice, st));
    if (c == ncp - 1) break;  // the state after the last step is not needed
    const int64_t nf = std::min(sb, pl.forced_end) - sa;
    if (nf > 0) RES_TRY(synth_rows(r64, nw, pl.P, pl.w0 * h, +1, btab, Gpre, ncols, sa, 1, nf, frow, st));
    for (int64_t s = sa; s < sb; ++s) {
      const void* g = s < pl.forced_end ? row(frow, s - sa) : nullptr;
      if (fused) {
        void* unext = ucur == u ? u2 : u;
        if (launch_fwd_step2d(fwd, k, ucur, unext, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, h, st, g,
                              r64))
          return fail(RES_EINVAL, "fused forward step launch");
        ucur = unext;
        continue;
      }
      if (fused3) {
        void* unext = ucur == u ? u2 : u;
        if (launch_grid_step3d(op->gw[0], k, ucur, unext, g, 1.0, 0.0, nullptr, st))
          return fail(RES_EINVAL, "3-D step launch");
        ucur = unext;
        continue;
      }
      launch_fwd_stage(fwd, k, 1, u, nullptr, u, y2, acc, nullptr, h, st, nullptr, r64);
      launch_fwd_stage(fwd, k, 2, u, nullptr, y2, y3, acc, nullptr, h, st, nullptr, r64);
      launch_fwd_stage(fwd, k, 3, u, nullptr, y3, y2, acc, nullptr, h, st, nullptr, r64);
      launch_fwd_stage(fwd, k, 4, u, u, y2, nullptr, acc, nullptr, h, st, g, r64);
    }
  }
  HIP_TRY(hipGetLastError());

  // 2. reverse sweep over the segments.  The segment's forward recomputation keeps the three stage inputs of every
  // step but its last when they fit in half of the free device memory, so the reverse steps do not march them
  // again (the values are the same: the stages of a step depend only on its state and forcing).
  void* stg = nullptr;
  {
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    const auto held = op->ws.find("bw_stages");
    const double avail = (double)free_b + (held != op->ws.end() ? (double)held->second.bytes : 0.0);
    const size_t need = (size_t)3 * C * rowb;
    if (need_states && (double)need <= 0.5 * avail && ws_get(op, "bw_stages", need, &stg) != RES_OK) {
      g_last_error.clear();
      stg = nullptr;
    }
  }
  // The lambda rows of G consecutive segments are kept together, so that the forcing gradient's projection runs on
  // up to 256 rows at a time (64-row projections spend most of their time reading and writing the accumulator).
  // G shrinks to what a quarter of the device memory left after the stage rows holds.
  int64_t G_seg = std::max<int64_t>(1, std::min<int64_t>(ncp, 256 / C));
  if (G_seg > 1) {
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    const auto held = op->ws.find("bw_lrows");
    const double avail = (double)free_b + (held != op->ws.end() ? (double)held->second.bytes : 0.0);
    G_seg = std::max<int64_t>(1, std::min<int64_t>(G_seg, (int64_t)(0.25 * avail / ((double)C * rowb))));
  }
  RES_TRY(ws_get(op, "bw_lrows", (size_t)(G_seg * C) * rowb, &lrows));
  auto srow = [&](int64_t r, int i) { return row(stg, 3 * r + i); };
  RES_TRY(zero_device(carry, rowb, st));  // lambda_S = 0: u_S is not sampled
  for (int64_t c = ncp - 1; c >= 0; --c) {
    const int64_t sa = c * C, sb = std::min(S, sa + C), len = sb - sa;
    if (need_states) {
      RES_TRY(synth_segment(sa, sb, c + 1 < ncp && sb < pl.forced_end));
      // states u_sa .. u_{sb-1}
      HIP_TRY(hipMemcpyAsync(row(seg, 0), row(cps, c), rowb, hipMemcpyDeviceToDevice, st));
    }
    for (int64_t s = sa; need_states && s + 1 < sb; ++s) {
      const int64_t r = s - sa;
      void* us = row(seg, r);
      void* a2 = stg ? srow(r, 0) : y2;
      void* a3 = stg ? srow(r, 1) : y3;
      void* a4 = stg ? srow(r, 2) : y2;
      if (fused) {
        if (launch_fwd_step2d(fwd, k, us, row(seg, r + 1), stg ? a2 : nullptr, stg ? a3 : nullptr,
                              stg ? a4 : nullptr, frc(s, r, 0), frc(s, r, 1), frc(s, r, 2), h, st, nullptr, r64))
          return fail(RES_EINVAL, "fused forward step launch");
        continue;
      }
      launch_fwd_stage(fwd, k, 1, us, nullptr, us, a2, acc, frc(s, r, 0), h, st, nullptr, r64);
      launch_fwd_stage(fwd, k, 2, us, nullptr, a2, a3, acc, frc(s, r, 1), h, st, nullptr, r64);
      launch_fwd_stage(fwd, k, 3, us, nullptr, a3, a4, acc, frc(s, r, 1), h, st, nullptr, r64);
      launch_fwd_stage(fwd, k, 4, us, row(seg, r + 1), a4, nullptr, acc, frc(s, r, 2), h, st, nullptr, r64);
    }
    // projection seeds of the sampled steps in [sa, sb)
    const int64_t ma = first_m_at_or_after(sa), mb = first_m_at_or_after(sb);
    if (mb > ma)
      RES_TRY(synth_rows(r64, nw, pl.P, pl.w0 * h, +1, btab, G, ncols, pl.pfirst + ma * pl.pstride, pl.pstride,
                         mb - ma, inj, st));
    // lambda rows: lseg[r] = lambda_{sa + r + 1}, segment c at row (c - cg) C of its group's rows
    const int64_t cg = c / G_seg * G_seg;
    void* lseg = row(lrows, (c - cg) * C);
    HIP_TRY(hipMemcpyAsync(row(lseg, len - 1), carry, rowb, hipMemcpyDeviceToDevice, st));
    for (int64_t s = sb - 1; s >= sa; --s) {
      const int64_t r = s - sa;
      void* us = need_states ? row(seg, r) : nullptr;
      const void *s2 = y2, *s3 = y3, *s4 = y4;  // stage inputs of step s
      if (!need_states) {
        s2 = s3 = s4 = nullptr;
      } else if (stg && s + 1 < sb) {
        s2 = srow(r, 0);
        s3 = srow(r, 1);
        s4 = srow(r, 2);
      } else if (fused) {
        if (launch_fwd_step2d(fwd, k, us, nullptr, y2, y3, y4, frc(s, r, 0), frc(s, r, 1), nullptr, h, st, nullptr,
                              r64))
          return fail(RES_EINVAL, "fused forward step launch");
      } else {
        launch_fwd_stage(fwd, k, 1, us, nullptr, us, y2, nullptr, frc(s, r, 0), h, st, nullptr, r64);
        launch_fwd_stage(fwd, k, 2, us, nullptr, y2, y3, nullptr, frc(s, r, 1), h, st, nullptr, r64);
        launch_fwd_stage(fwd, k, 3, us, nullptr, y3, y4, nullptr, frc(s, r, 1), h, st, nullptr, r64);
      }
      const void* lp = row(lseg, r);
      const void* seed = nullptr;
      if (s >= pl.pfirst && (s - pl.pfirst) % pl.pstride == 0) {
        const int64_t m = (s - pl.pfirst) / pl.pstride;
        if (m < pl.pcount) seed = row(inj, m - ma);
      }
      if (fused) {
        if (launch_rev_step2d(rev, k, lp, r > 0 ? row(lseg, r - 1) : carry, s2, s3, s4, us, mu_cols, seed, h, st,
                              r64))
          return fail(RES_EINVAL, "fused reverse step launch");
        continue;
      }
      if (fused3 && !need_states) {
        if (launch_grid_step3d(op->gw[1], k, lp, r > 0 ? row(lseg, r - 1) : carry, seed, 1.0, 0.0, nullptr, st))
          return fail(RES_EINVAL, "3-D step launch");
        continue;
      }
      // Kb_3 in ka, Kb_2 in kb, Kb_1 in ub; stage 1 combines the three into lambda
      launch_rev_stage(rev, k, 4, lp, nullptr, nullptr, s4, ka, nullptr, nullptr, mu_cols, nullptr, h, st, r64);
      launch_rev_stage(rev, k, 3, lp, nullptr, ka, s3, kb, nullptr, nullptr, mu_cols, nullptr, h, st, r64);
      launch_rev_stage(rev, k, 2, lp, nullptr, kb, s2, ub, nullptr, nullptr, mu_cols, nullptr, h, st, r64);
      launch_rev_stage(rev, k, 1, lp, r > 0 ? row(lseg, r - 1) : carry, ub, us, nullptr, ka, kb, mu_cols, seed, h,
                       st, r64);
    }
    HIP_TRY(hipGetLastError());
    // forcing gradient: Fourier sums of lambda_{s+1} over the forced steps of the group, once its first segment
    // is done
    if (c == cg) {
      const int64_t ga = cg * C, gb = std::min(S, (cg + G_seg) * C);
      const int64_t nf = std::min(gb, pl.forced_end) - ga;
      if (f_out && nf > 0)
        RES_TRY(project_rows(op, r64, nw, pl.P, pl.w0 * h, +1, btab, lrows, ncols, ncols, ga, 1, nf, 1.0,
                             (double*)facc, st));
    }
  }
  if (mu_cols) launch_sum_columns(mu_cols, mu_rows, nsite, mu_grad, st);
  // 3. F_grad_j = h Q_{-w_j}(Z^H) facc_j (FP64 Horner passes, written in the working precision)
  if (f_out) {
    RES_TRY(prefilter(op, pl, k, facc, 1, f_out, -1, 1, st, op->fp64()));
    launch_finite(facc, 1, (int64_t)nw * ncols, op->d_flag, st);
  }
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

// Frees the handle's workspace (the forward drivers' state, forcing, snapshot and accumulator blocks and the reverse
// mode's own rows), so that the reverse mode can size its rows to the device memory; every driver sizes its
// workspace again on its next call.  Kept: the device copy of the stepper regions and the weighted reverse mode's
// scaled inputs (in use).
int release_workspace(resolvent_op* op) {
  if (op->capturing || op->arena) return RES_OK;
  HIP_TRY(hipDeviceSynchronize());
  for (auto& kv : op->ws) {
    const std::string& name = kv.first;
    if (name.compare(0, 6, "bw_wsc") == 0 || name == "segs") continue;
    if (kv.second.p) HIP_TRY(hipFree(kv.second.p));
    kv.second.p = nullptr;
    kv.second.bytes = 0;
  }
  return RES_OK;
}

// Copies columns [c0, c0 + kc) of a [nw][k][N] block (precision in_fp64) into a [nw][kc][N] block (precision
// out_fp64), times scale.
void gather_columns(const void* x, int in_fp64, int64_t k, int64_t c0, int64_t kc, int64_t N, int nw, void* y,
                    int out_fp64, double scale, hipStream_t st) {
  const size_t ies = in_fp64 ? sizeof(cd) : sizeof(std::complex<float>);
  const size_t oes = out_fp64 ? sizeof(cd) : sizeof(std::complex<float>);
  if (kc == k) {
    launch_convert(x, in_fp64, y, out_fp64, (int64_t)nw * k * N, scale, st);
    return;
  }
  for (int j = 0; j < nw; ++j)
    launch_convert((const char*)x + (size_t)((int64_t)j * k + c0) * N * ies, in_fp64,
                   (char*)y + (size_t)((int64_t)j * kc) * N * oes, out_fp64, kc * N, scale, st);
}

int backward(resolvent_op* op, const Plan& pl, int k, const void* f_hat, const void* g_hat, void* f_grad,
             double* mu_grad, int64_t C, hipStream_t st) {
  const int64_t N = op->N, S = pl.S;
  const int nw = pl.nw;
  const int r64 = op->fp64() || op->rev_rows64;
  const size_t res = r64 ? sizeof(cd) : sizeof(std::complex<float>);
  if (C <= 0) C = std::max<int64_t>(1, (int64_t)std::ceil(std::sqrt((double)S)));
  C = std::min<int64_t>(C, S);
  const int64_t ncp = (S + C - 1) / C;
  // The adjoint recursion for lambda is linear and does not involve the forward trajectory: only the mu gradient
  // needs the states and stage values, so without it the forcing, the forward march, its checkpoints and the
  // segment recomputation are skipped (the forcing gradient then costs one adjoint march).
  const bool need_states = mu_grad != nullptr;
  const bool f_direct = (op->fp64() ? 1 : 0) == r64;  // the caller's forcing is already in the row precision

  // Columns evolve independently under the march and the mu gradient is a sum over columns, so the columns are
  // processed in chunks of kc when the rows of all k do not fit: the bytes a chunk holds (the stage rows and the
  // extra lambda rows are sized later from what is left) against the free device memory, after the handle's
  // workspace is released when all k columns do not fit beside it.
  const double horner_budget = env_double("RESOLVENT_HORNER_BUDGET_GB", 8.0) * 1073741824.0;
  auto need = [&](int64_t kc) {
    const double row = (double)kc * N * res, blk = nw * row;
    double b = blk + (double)(2 * C + 12) * row;  // seed, lambda rows, injections, work rows
    if (f_grad) b += (double)nw * kc * N * sizeof(cd) + std::min(horner_budget, 2.0 * nw * kc * N * sizeof(cd));
    if (need_states) {
      b += blk + (kc < k || !f_direct ? blk : 0.0) + (double)(ncp + 3 * C + 1) * row;
      b += std::min(horner_budget, 2.0 * nw * kc * N * sizeof(cd)) + (double)(k + 1) * adj_op(op, 0).nsite * 8.0;
    }
    return b;
  };
  auto available = [&](double* out) -> int {
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    *out = 0.92 * (double)free_b - 2.0 * 1073741824.0;
    return RES_OK;
  };
  int64_t kc = k;
  const long forced = env_long("RESOLVENT_BACKWARD_COLUMNS", 0);
  if (forced > 0) {
    kc = std::min<int64_t>(k, forced);
  } else {
    double avail = 0;
    RES_TRY(available(&avail));
    if (need(k) > avail) {
      RES_TRY(release_workspace(op));
      RES_TRY(available(&avail));
    }
    while (kc > 1 && need(kc) > avail) --kc;
  }

  if (mu_grad) RES_TRY(zero_device(mu_grad, (size_t)adj_op(op, 0).nsite * sizeof(double), st));
  for (int64_t c0 = 0; c0 < k; c0 += kc) {
    const int64_t kcc = std::min<int64_t>(kc, k - c0);
    const size_t blk = (size_t)nw * kcc * N * res;
    void* G;
    RES_TRY(ws_get(op, "bw_G", blk, &G));
    gather_columns(g_hat, op->fp64(), k, c0, kcc, N, nw, G, r64, pl.scale, st);
    const void* F = nullptr;
    if (need_states) {
      if (kcc == k && f_direct) {
        F = f_hat;
      } else {
        void* p;
        RES_TRY(ws_get(op, "bw_F", blk, &p));
        gather_columns(f_hat, op->fp64(), k, c0, kcc, N, nw, p, r64, 1.0, st);
        F = p;
      }
    }
    // the chunk's forcing gradient goes straight to f_grad when the chunk is every column, else into the seed
    // block (no longer read by then) and is scattered from there
    void* fo = f_grad ? (kcc == k ? f_grad : G) : nullptr;
    RES_TRY(backward_chunk(op, pl, (int)kcc, r64, F, G, fo, mu_grad, C, st));
    if (f_grad && kcc < k) {
      const size_t es = op->wsize();
      for (int j = 0; j < nw; ++j)
        HIP_TRY(hipMemcpyAsync((char*)f_grad + (size_t)((int64_t)j * k + c0) * N * es,
                               (const char*)G + (size_t)((int64_t)j * kcc) * N * es, (size_t)kcc * N * es,
                               hipMemcpyDeviceToDevice, st));
    }
  }
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

}  // namespace rt

extern "C" {

int resolvent_apply_backward(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                             const void* f_hat, const void* g_hat, void* f_grad, double* mu_grad,
                             int32_t checkpoint_every, void* stream) {
  g_last_error.clear();
  if (!op || !f_hat || !g_hat) return fail(RES_EINVAL, "NULL argument");
  if (k < 1) return fail(RES_EINVAL, "k must be >= 1");
  if (checkpoint_every < 0) return fail(RES_EINVAL, "checkpoint_every must be >= 0");
  Plan pl;
  RES_TRY(make_plan(op, grid, run, &pl));
  if (!f_grad && !mu_grad) return RES_OK;
  hipStream_t st = (hipStream_t)stream;
  CaptureScope cap(op, st);
  if (!op->weighted) return backward(op, pl, k, f_hat, g_hat, f_grad, mu_grad, checkpoint_every, st);
  // y = C R B f with real diagonal B, C: the reverse mode of R at the input B f with the cotangent C g; the forcing
  // gradient is B R^H C g (the metrics do not enter a Euclidean vector-Jacobian product)
  const double* w = (const double*)op->d_wsc;
  const int64_t blocks = (int64_t)pl.nw * k;
  const int fp = op->fp64();
  void *fb, *gc;
  RES_TRY(ws_get(op, "bw_wsc_f", (size_t)blocks * op->N * op->wsize(), &fb));
  RES_TRY(ws_get(op, "bw_wsc_g", (size_t)blocks * op->N * op->wsize(), &gc));
  launch_node_scale(f_hat, fp, fb, fp, w + (size_t)kWscB * op->N, blocks, op->N, st);
  launch_node_scale(g_hat, fp, gc, fp, w + (size_t)kWscC * op->N, blocks, op->N, st);
  RES_TRY(backward(op, pl, k, fb, gc, f_grad, mu_grad, checkpoint_every, st));
  if (f_grad) launch_node_scale(f_grad, fp, f_grad, fp, w + (size_t)kWscB * op->N, blocks, op->N, st);
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

int resolvent_op_set_backward_rows(resolvent_op* op, int32_t fp64) {
  if (!op) return fail(RES_EINVAL, "NULL op");
  op->rev_rows64 = fp64 != 0;
  return RES_OK;
}

}  // extern "C"
