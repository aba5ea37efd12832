// The 1-D stepper kernel and its launch helpers (internal), instantiated per steps-per-kernel-step MS by
// step1d.hip (MS = 1), step1d_m2.hip and step1d_m4.hip so that the three compile in parallel.
#pragma once

#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace res {

// Empty mark of an exchange slot: a signalling-NaN bit pattern that no arithmetic produces (computed NaNs are
// quiet), compared as raw bits.
template <typename R> struct EmptyMark;
template <> struct EmptyMark<double> {
  typedef unsigned long long U;
  static constexpr U bits = 0x7FF4DEAD5EA1ED00ull;
};
template <> struct EmptyMark<float> {
  typedef unsigned int U;
  static constexpr U bits = 0x7FA5EA1Du;
};

// DS read instructions of the band product kept in flight per lane (one unknown per thread, four RK4 steps per
// kernel step, at most 512 threads), FP64 and FP32; 0 leaves the schedule to the compiler.
#ifndef RES_LDS_AHEAD64
#define RES_LDS_AHEAD64 4
#endif
#ifndef RES_LDS_AHEAD32
#define RES_LDS_AHEAD32 0
#endif
constexpr int kLdsAhead64 = RES_LDS_AHEAD64;
constexpr int kLdsAhead32 = RES_LDS_AHEAD32;

// One workgroup marches its region for n_steps kernel steps of MS RK4 steps each: the band is P(Z)^MS (radius
// 4*MS) and each forcing row is the combined forcing of the MS steps it covers (see the pre-filter in
// step1d.hip), so a kernel step is one exchange through LDS and one band product whatever MS is.  Thread t holds V consecutive unknowns of the region in
// registers together with their nine stencil coefficients; the state is exchanged through a double-buffered LDS
// row once per step (one LDS-only barrier per step).  Forcing rows are prefetched PD steps ahead into a register
// ring.  Threads past the region end work on a clamped copy of its last unknown with zero coefficients, so every
// load is in bounds and no branch depends on the lane.
//
// Forcing of local step t: phi * frc[row][col*N + i] with row = frc_row0 + t (mod frc_period if > 0).
// Snapshots (u_t, the state BEFORE step t's update) of the owned unknowns go to rows of length snap_ld whose last
// element is a scratch slot that non-owned lanes overwrite, keeping every snapshot store unconditional.
// SNAP: 0 = none, 1 = every step into row snap_row0 + t, 2 = steps snap_first + m*snap_stride into row
// snap_row0 + m.  Keeping the store pattern a compile-time property lets the compiler count outstanding memory
// operations exactly, so the prefetched loads are waited for with partial counts.
//
// PERSIST: the launch marches all n_steps in blocks of `block` steps (a multiple of PD).  Between blocks each
// workgroup publishes the owned values its neighbours need (the 4*block nearest each end of its owned range, in
// one row per direction) into rows (b - 1) & 1 of xbuf and takes its halo from the neighbours' rows.  Every slot
// has one writer and one reader and holds either a value or the empty mark (a NaN bit pattern no arithmetic
// produces): a halo lane polls its own slot until the neighbour's value has replaced the mark, takes it and
// re-arms the slot, so the data itself carries the ready signal and no flag round trip is needed.  A
// workgroup rewrites a row only after it has seen the neighbours' values of the following block, which they
// publish only after their re-arming stores have completed (the vmcnt(0) wait that opens every exchange), so a
// value is never overwritten by a late re-arm.  All slot accesses are agent-scope atomics (device-coherent) to
// uncached memory; rows start empty (launch_fill_empty before each persistent launch).  Every wait is bounded
// by `spin_ns` of wall-clock time: on expiry the workgroup sets *err and returns, and its neighbours then time
// out in turn, so every wave of the grid terminates.  The grid must be co-resident (cooperative launch).
template <typename R, int NT, int V, int PD, bool FORCED, int SNAP, bool PERSIST, int MS>
__global__ __launch_bounds__(NT) void step1d_kernel(const Seg1D* __restrict__ segs, const cx<R>* __restrict__ band,
                                                    const cx<R>* __restrict__ state_in, cx<R>* __restrict__ state_out,
                                                    int64_t N, int64_t row_len, int64_t n_steps,
                                                    const cx<R>* __restrict__ frc, int64_t frc_row0,
                                                    int64_t frc_period, R phi_re, R phi_im, cx<R>* __restrict__ snap,
                                                    int64_t snap_ld, int64_t snap_first, int64_t snap_stride,
                                                    int64_t snap_count, int64_t snap_row0, cx<R>* xbuf,
                                                    int64_t block, uint64_t spin_ns, int* err) {
  constexpr int RAD = kBandRadius * MS, BW = 2 * RAD + 1;  // band of P(Z)^MS
  constexpr int NACC = MS > 1 ? 4 : 2;                       // partial sums of the band product
  constexpr int W = NT * V + 2 * RAD;
  __shared__ cx<R> buf[2][W];
  const Seg1D sg = segs[blockIdx.x];
  const int tid = threadIdx.x;
  const int64_t cbase = (int64_t)sg.col * N + sg.dof0;
  const cx<R> zero = mk<R>(0, 0);
  const cx<R> phi = mk<R>(phi_re, phi_im);

  cx<R> p[V][BW];
  cx<R> u[V];
  int lc[V];
  bool valid[V], own[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int l = tid * V + v;
    valid[v] = l < sg.ndof;
    own[v] = valid[v] && l >= sg.own0 && l < sg.own0 + sg.nown;
    lc[v] = valid[v] ? l : sg.ndof - 1;
    const cx<R> s0 = state_in[cbase + lc[v]];
    u[v] = csel(valid[v], s0, zero);
#pragma unroll
    for (int d = 0; d < BW; ++d) {
      const cx<R> c = band[(sg.dof0 + lc[v]) * BW + d];
      p[v][d] = csel(valid[v], c, zero);
    }
  }
  if (tid < RAD) {
    buf[0][tid] = zero;
    buf[1][tid] = zero;
    buf[0][W - 1 - tid] = zero;
    buf[1][W - 1 - tid] = zero;
  }

  // Forcing rows are consumed strictly in step order; `lrow` is the (wrapping) row of the next load.  Rows travel
  // by value (a pointer to the ring would force it into scratch memory).
  struct FRow {
    cx<R> v[V];
  };
  int64_t lrow = frc_period > 0 ? frc_row0 % frc_period : frc_row0;
  const cx<R>* fbase = FORCED ? frc + cbase : nullptr;
  auto load_row = [&]() -> FRow {
    FRow r;
    const cx<R>* src = fbase + lrow * row_len;
#pragma unroll
    for (int v = 0; v < V; ++v) r.v[v] = load_nt<R>(src + lc[v]);
    if (++lrow == frc_period) lrow = 0;
    return r;
  };

  int64_t next_snap = (SNAP == 2 && snap_count > 0) ? snap_first : -1;
  int64_t snap_m = 0;
  int64_t sidx[V];  // snapshot column of each lane: owned unknown or the row's scratch slot
#pragma unroll
  for (int v = 0; v < V; ++v) sidx[v] = own[v] ? cbase + lc[v] : snap_ld - 1;

  // one step: exchange through LDS, snapshot of u_t, u <- P(Z) u + phi f
  auto step = [&](int64_t t, const FRow f) {
    cx<R>* row = buf[t & 1];
#pragma unroll
    for (int v = 0; v < V; ++v) row[RAD + tid * V + v] = u[v];
    lds_barrier();
    if (SNAP == 1) {
      cx<R>* dst = snap + (snap_row0 + t) * snap_ld;
#pragma unroll
      for (int v = 0; v < V; ++v) dst[sidx[v]] = u[v];
    } else if (SNAP == 2 && t == next_snap) {
      cx<R>* dst = snap + (snap_row0 + snap_m) * snap_ld;
#pragma unroll
      for (int v = 0; v < V; ++v) dst[sidx[v]] = u[v];
      ++snap_m;
      next_snap = (snap_m < snap_count) ? next_snap + snap_stride : -1;
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      // interleaved partial sums shorten the dependent FMA chain
      cx<R> a[NACC];
      a[0] = FORCED ? cmul(phi, f.v[v]) : zero;
#pragma unroll
      for (int q = 1; q < NACC; ++q) a[q] = zero;
#pragma unroll
      for (int d = 0; d < BW; ++d) a[d % NACC] = cfma(p[v][d], row[tid * V + v + d], a[d % NACC]);
      cx<R> acc = cadd(a[0], a[1]);
      if (NACC == 4) acc = cadd(acc, cadd(a[2], a[3]));
      u[v] = csel(valid[v], acc, zero);
    }
    constexpr int want = sizeof(R) == 8 ? kLdsAhead64 : kLdsAhead32;
    if constexpr (V == 1 && MS == 4 && NT <= 512 && want > 0) {
      // Keep the next neighbour reads in flight: the first `ahead` DS reads go out together and each one after
      // them follows the complex FMAs of one read's values (four VALU instructions per value).  Left to itself
      // the scheduler keeps one read ahead, and every read's LDS latency then stalls the band product.  FP32
      // pairs two values in one read (ds_read2_b64).  Only the 33-diagonal band of four steps, with at least
      // 256 VGPRs per lane: the shorter bands and the 1,024-thread workgroups (128 VGPRs, which already spill)
      // ran slower with it.
      constexpr int per = sizeof(R) == 8 ? 1 : 2;
      constexpr int nds = (BW + per - 1) / per;
      constexpr int ahead = want < nds ? want : nds;
      __builtin_amdgcn_sched_group_barrier(0x100, ahead, 0);  // DS reads
#pragma unroll
      for (int d = 0; d < nds - ahead; ++d) {
        __builtin_amdgcn_sched_group_barrier(0x002, 4 * per, 0);  // VALU
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);        // DS read
      }
    }
  };

  if (PERSIST) {
    // Blocks of `block` steps (a multiple of PD) with a neighbour exchange before every block but the first.
    // exchange(b) publishes the owned values of the state after block b-1, waits for both neighbours to have
    // published theirs and reloads the halo; it returns false when the wait was abandoned (the grid drains).
    __shared__ int abort_flag;
    if (tid == 0) abort_flag = 0;  // ordered before any exchange by the first step's barrier
    typedef typename EmptyMark<R>::U U;
    const int halo = RAD * (int)block;  // halo width of a region = owned values a neighbour reads
    auto exchange = [&](int64_t b) -> bool {
      // rows: [(b - 1) & 1][side], side 0 = values near the owner's left end (read by its left neighbour),
      // side 1 = values near its right end (read by its right neighbour); every slot has one writer, one reader
      U* rows = reinterpret_cast<U*>(xbuf + (int64_t)((b - 1) & 1) * 2 * row_len + cbase);
      U* to_left = rows;
      U* to_right = rows + 2 * row_len;
      // The slots this workgroup re-armed at the previous exchange must be empty again before a neighbour can
      // see this block's values: it rewrites them only after it has seen these.
      __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (own[v]) {
          const int pos = lc[v] - sg.own0;
          const U re = __builtin_bit_cast(U, u[v].re), im = __builtin_bit_cast(U, u[v].im);
          if (pos < halo) {
            __hip_atomic_store(to_left + 2 * lc[v], re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(to_left + 2 * lc[v] + 1, im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          if (sg.nown - 1 - pos < halo) {
            __hip_atomic_store(to_right + 2 * lc[v], re, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(to_right + 2 * lc[v] + 1, im, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      const uint64_t t0 = wall_clock64();
      const uint64_t limit = spin_ns / 10;  // wall_clock64 ticks at 100 MHz
      bool late = false;
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (valid[v] && !own[v]) {
          // a halo value left of the owned range is the left neighbour's right-end value, and vice versa
          U* slot = (lc[v] < sg.own0 ? to_right : to_left) + 2 * lc[v];
          U re, im;
          while (true) {
            re = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            im = __hip_atomic_load(slot + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (re != EmptyMark<R>::bits && im != EmptyMark<R>::bits) break;
            if (wall_clock64() - t0 > limit) { late = true; break; }
            __builtin_amdgcn_s_sleep(1);
          }
          __hip_atomic_store(slot, EmptyMark<R>::bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(slot + 1, EmptyMark<R>::bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          u[v] = mk<R>(__builtin_bit_cast(R, re), __builtin_bit_cast(R, im));
        }
      if (late) abort_flag = 1;
      __syncthreads();
      if (abort_flag) {
        if (tid == 0) atomicOr(err, 8);
        return false;
      }
      return true;
    };
    if (FORCED) {
      // One flat loop over rounds of PD steps (the ring's period); the exchange is a uniform branch inside it.
      FRow f[PD];
#pragma unroll
      for (int q = 0; q < PD; ++q) f[q] = load_row();
      const int64_t n_main = (n_steps / PD) * PD;
      const int64_t rounds_per_block = block / PD;
      int64_t t = 0, b = 0, until_exchange = rounds_per_block;
      for (; t < n_main; t += PD) {
        if (until_exchange == 0) {
          if (!exchange(++b)) return;
          until_exchange = rounds_per_block;
        }
        --until_exchange;
#pragma unroll
        for (int q = 0; q < PD; ++q) {
          step(t + q, f[q]);
          __builtin_amdgcn_sched_barrier(0);
          f[q] = load_row();  // refills past the last step read padding rows
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      if (t < n_steps) {
        if (until_exchange == 0 && !exchange(++b)) return;
#pragma unroll
        for (int q = 0; q < PD; ++q)
          if (t + q < n_steps) step(t + q, f[q]);
      }
    } else {
      FRow none;
#pragma unroll
      for (int v = 0; v < V; ++v) none.v[v] = zero;
      for (int64_t t = 0; t < n_steps; ++t) {
        if (t > 0 && t % block == 0 && !exchange(t / block)) return;
        step(t, none);
      }
    }
  } else {
  const int64_t n_main = FORCED ? (n_steps / PD) * PD : n_steps;
  int64_t t = 0;
  if (FORCED) {
    // prefetch ring: f[q] holds the row of step t0 + q; it is refilled with step t0 + q + PD right after use
    FRow f[PD];
#pragma unroll
    for (int q = 0; q < PD; ++q) f[q] = load_row();
    for (; t < n_main; t += PD) {
#pragma unroll
      for (int q = 0; q < PD; ++q) {
        step(t + q, f[q]);
        // keep the refill of slot q after the step that consumes it (hoisting it would force a copy of the
        // slot and a full wait on the loads in flight).  Refills past the last step read padding rows.
        __builtin_amdgcn_sched_barrier(0);
        f[q] = load_row();
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int q = 0; q < PD; ++q)
      if (t + q < n_steps) step(t + q, f[q]);
  } else {
    FRow none;
#pragma unroll
    for (int v = 0; v < V; ++v) none.v[v] = zero;
    for (; t < n_steps; ++t) step(t, none);
  }
  }
#pragma unroll
  for (int v = 0; v < V; ++v)
    if (own[v]) state_out[cbase + lc[v]] = u[v];
}

template <typename R, int NT, int V, int PD, bool F, int S, bool PERSIST, int MS>
int launch_step1d_one(const Step1DArgs& a, hipStream_t st) {
  const cx<R>* band = (const cx<R>*)a.band;
  const cx<R>* sin = (const cx<R>*)a.state_in;
  cx<R>* sout = (cx<R>*)a.state_out;
  const cx<R>* frc = (const cx<R>*)a.frc;
  R phr = (R)a.phi_re, phi = (R)a.phi_im;
  cx<R>* snap = (cx<R>*)a.snap;
  cx<R>* xbuf = (cx<R>*)a.xbuf;
  auto kern = step1d_kernel<R, NT, V, PD, F, S, PERSIST, MS>;
  if (!PERSIST) {
    hipLaunchKernelGGL(kern, dim3(a.nseg), dim3(NT), 0, st, a.segs, band, sin, sout, a.N, a.row_len, a.n_steps, frc,
                       a.frc_row0, a.frc_period, phr, phi, snap, a.snap_ld, a.snap_first, a.snap_stride,
                       a.snap_count, a.snap_row0, xbuf, a.block, a.spin_ns, a.err);
    return 0;
  }
  void* args[] = {(void*)&a.segs, (void*)&band, (void*)&sin, (void*)&sout, (void*)&a.N, (void*)&a.row_len,
                  (void*)&a.n_steps, (void*)&frc, (void*)&a.frc_row0, (void*)&a.frc_period, (void*)&phr,
                  (void*)&phi, (void*)&snap, (void*)&a.snap_ld, (void*)&a.snap_first, (void*)&a.snap_stride,
                  (void*)&a.snap_count, (void*)&a.snap_row0, (void*)&xbuf, (void*)&a.block, (void*)&a.spin_ns,
                  (void*)&a.err};
  return hipLaunchCooperativeKernel((const void*)kern, dim3(a.nseg), dim3(NT), args, 0, st) == hipSuccess ? 0 : -2;
}

template <typename R, int NT, int V, int PD, int MS>
int launch_step1d_cfg(const Step1DArgs& a, hipStream_t st) {
  // snapshot mode: every step when the launch projects each of its steps from row snap_row0 on
  const int mode = (a.snap == nullptr || a.snap_count <= 0) ? 0
                   : (a.snap_first == 0 && a.snap_stride == 1 && a.snap_count == a.n_steps) ? 1 : 2;
#define RES_STEP(F, S)                                                            \
  return a.persist ? launch_step1d_one<R, NT, V, PD, F, S, true, MS>(a, st)      \
                   : launch_step1d_one<R, NT, V, PD, F, S, false, MS>(a, st)
  if constexpr (MS > 1) {
    // multi-step marches are always forced; a sample at every kernel step takes the general strided form
    if (a.frc == nullptr) return -4;
    if (mode == 0) RES_STEP(true, 0); else RES_STEP(true, 2);
  } else {
    if (a.frc != nullptr) {
      if (mode == 0) RES_STEP(true, 0); else if (mode == 1) RES_STEP(true, 1); else RES_STEP(true, 2);
    } else {
      if (mode == 0) RES_STEP(false, 0); else if (mode == 1) RES_STEP(false, 1); else RES_STEP(false, 2);
    }
  }
#undef RES_STEP
}

// Largest grid of this configuration that is co-resident on the device (for the persistent variant).
template <typename R, int NT, int V, int PD, int MS>
int coresident_cfg(int device) {
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, step1d_kernel<R, NT, V, PD, true, 2, true, MS>, NT, 0) !=
      hipSuccess)
    return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  return per_cu * cus;
}

#define RES_CFGS(X)               \
  X(0, 64, 1, 4)                  \
  X(1, 128, 1, 4)                 \
  X(2, 256, 1, 4)                 \
  X(3, 256, 2, 4)                 \
  X(4, 256, 4, 2)                 \
  X(5, 256, 8, 2)                 \
  X(6, 512, 4, 2)                 \
  X(7, 1024, 2, 2)                \
  X(8, 512, 2, 4)                 \
  X(9, 1024, 1, 4)                \
  X(10, 512, 1, 4)                \
  X(11, 128, 2, 4)                \
  X(12, 256, 1, 8)                \
  X(13, 512, 1, 8)                \
  X(14, 128, 1, 8)                \
  X(15, 256, 2, 8)

template <int MS> int launch_step1d_ms(const Step1DArgs& a, hipStream_t st) {
  switch (a.cfg) {
#define RES_CASE(I, NT, V, PD) \
  case I: return a.fp64 ? launch_step1d_cfg<double, NT, V, PD, MS>(a, st) : launch_step1d_cfg<float, NT, V, PD, MS>(a, st);
    RES_CFGS(RES_CASE)
#undef RES_CASE
    default: return -1;
  }
}

template <int MS> int step1d_coresident_ms(int fp64, int cfg, int device) {
  switch (cfg) {
#define RES_CASE(I, NT, V, PD) \
  case I: return fp64 ? coresident_cfg<double, NT, V, PD, MS>(device) : coresident_cfg<float, NT, V, PD, MS>(device);
    RES_CFGS(RES_CASE)
#undef RES_CASE
    default: return 0;
  }
}

}  // namespace res
