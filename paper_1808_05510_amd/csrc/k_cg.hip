// Persistent (cooperative) conjugate-gradient kernels:
//  * k_pcg      Jacobi-PCG on the ALS half-step systems (eqs. ALS_linsys and
//               ALS_linsys_v), one launch per solve, three grid barriers per
//               iteration;
//  * k_galerkin matrix-valued CG on the projected equation (eq. Proj_Sylv)
//               in FP64, four grid barriers per iteration.
// Control flow is uniform over the grid: every workgroup reduces the same
// partial sums in the same order, so all take identical branch decisions and
// every grid barrier is reached by all workgroups; loops are bounded by maxit.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "cr_internal.hpp"

namespace cgrp = cooperative_groups;

namespace cr {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Sum of v over a workgroup of BS threads; result returned to every thread.
// LEAD: the leading workgroup barrier, which keeps red from being rewritten
// while a slower wave still reads a previous sum; a sum that is the first use
// of red after a grid barrier (which starts and ends with one) drops it.
template <int BS = NT, bool LEAD = true>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wsum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (LEAD) __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < BS / WAVE; ++k) s += red[k];
  return s;
}

// Two workgroup sums in one pass (the wave sums interleave, one LDS round);
// red holds 2 BS / WAVE doubles.
template <int BS = NT, bool LEAD = true>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
  a = wsum(a);
  b = wsum(b);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (LEAD) __syncthreads();
  if (lane == 0) {
    red[wv] = a;
    red[BS / WAVE + wv] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int k = 0; k < BS / WAVE; ++k) {
    sa += red[k];
    sb += red[BS / WAVE + k];
  }
  a = sa;
  b = sb;
}

// Grid totals of slots sa and sb, both loads issued before the reduction.
template <int BS = NT, bool LEAD = true>
__device__ __forceinline__ void grid_total2(const double* part, int sa, int sb, int nwg,
                                            double* red, double& ta, double& tb) {
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nwg; k += BS) {
    a += part[(int64_t)sa * nwg + k];
    b += part[(int64_t)sb * nwg + k];
  }
  block_sum2<BS, LEAD>(a, b, red);
  ta = a;
  tb = b;
}

// Grid total of slot `slot` of the partial array (part[slot*nwg + b]),
// summed in the same order by every workgroup.
template <int BS = NT, bool LEAD = true>
__device__ __forceinline__ double grid_total(const double* part, int slot, int nwg, double* red) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nwg; b += BS) s += part[(int64_t)slot * nwg + b];
  return block_sum<BS, LEAD>(s, red);
}

// ------------------------------------------------------------ grid barrier
// Two implementations, chosen per launch: the cooperative-groups grid sync,
// or a barrier on device words (bar[0] generation, bar[64] timeout flag,
// bar[128] arrival counter: separate 256-byte lines).  Thread 0 of each
// workgroup arrives with a release add (its workgroup's stores were ordered
// before it by __syncthreads); the last arrival takes an acquire fence,
// resets the counter and publishes the next generation with a release store;
// the others poll the generation with relaxed loads and take one acquire
// fence when it changes.  Polling with acquire loads instead would
// invalidate the caches on every poll, which made the barrier several times
// slower.  The poll is bounded: after 2^22 sleeps (a fraction of a second,
// far above any legitimate wait between phases) it sets the timeout flag;
// once set, every later barrier is skipped, so a faulty launch ends quickly
// instead of hanging the device, and the host reports the flag as an error.
__device__ __forceinline__ void grid_barrier(const BarrierArg& b, cgrp::grid_group& grid) {
  if (b.mode == 0) {
    grid.sync();
    return;
  }
  __syncthreads();
  if (threadIdx.x == 0 &&
      __hip_atomic_load(b.bar + BAR_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
    const unsigned nwg = gridDim.x;
    const unsigned gen = __hip_atomic_load(b.bar + BAR_GEN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned prev =
        __hip_atomic_fetch_add(b.bar + BAR_COUNT, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == nwg - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(b.bar + BAR_COUNT, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(b.bar + BAR_GEN, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(b.bar + BAR_GEN, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > b.spin_max) {
          __hip_atomic_store(b.bar + BAR_TIMEOUT, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  __syncthreads();
}

// Wave sums of WAVE per-lane values at once, lane l receiving the sum over
// the wave of value l: a butterfly that halves the values held at each step
// (lanes with bit o set keep the upper half and send the lower), 63
// exchanges per lane instead of 6 for each of the 64 values.  val(j) gives
// this lane's value j.
template <typename F>
__device__ __forceinline__ double wave_transpose_sum(F val) {
  const int lane = threadIdx.x & (WAVE - 1);
  double v[WAVE / 2];
  {
    const bool up = (lane & 32) != 0;
#pragma unroll
    for (int j = 0; j < WAVE / 2; ++j) {
      const double lo = val(j), hi = val(j + WAVE / 2);
      v[j] = (up ? hi : lo) + __shfl_xor(up ? lo : hi, 32, WAVE);
    }
  }
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) {
    const bool up = (lane & o) != 0;
#pragma unroll
    for (int j = 0; j < o; ++j) {
      const double send = up ? v[j] : v[j + o];
      const double keep = up ? v[j + o] : v[j];
      v[j] = keep + __shfl_xor(send, o, WAVE);
    }
  }
  return v[0];
}

constexpr int PCG_MAX_VPT = 8;
constexpr int PCG_MAX_NINJ = 1024;
// Partial-sum slots.  Every slot has one writer phase per use and is never
// rewritten before a grid barrier separates the write from all reads: the
// final phase, which may start while slower workgroups still read the slots
// of the exit test, has a slot of its own.
constexpr int PCG_SLOTS = 5;  // 0: p.q, 1: r.z, 2: r.r, 3: b.b, 4: x.x

template <typename T, int K>
__device__ __forceinline__ double lap(const T* __restrict__ w, const int32_t* __restrict__ nbr,
                                      int64_t n, int64_t i) {
  double s = (double)K * (double)w[i];
#pragma unroll
  for (int k = 0; k < K; ++k) s -= (double)w[nbr[(int64_t)k * n + i]];
  return s;
}

// partial X^T z over this workgroup's voxels, z staged in LDS
template <typename T, int BS, bool CO = false>
__device__ void lr_partial(const PcgArgs<T>& a, const double* zs, int64_t lo, int64_t n, int nwg,
                           double* lrpart, int al0 = 0) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int per = a.vpt * (BS / WAVE);  // rows per lane
  for (int al = al0 + wv; al < a.ninj; al += BS / WAVE) {
    const T* xc = a.Xm + (int64_t)al * a.ldx;
    double acc = 0.0;
    for (int k = 0; k < per; ++k) {
      const int loc = lane + WAVE * k;
      // two-level launches: the slot's voxel (-1 for an idle slot)
      const int64_t i = CO ? (int64_t)a.co.slot_vox[lo + loc] : lo + loc;
      if (i >= 0 && i < n) acc += (double)xc[i] * zs[loc];
    }
    acc = wsum(acc);
    if (lane == 0) lrpart[(int64_t)al * nwg + blockIdx.x] = acc;
  }
}

// Register-resident Jacobi-PCG.  Workgroup b owns voxels b*NT*VPT + tid + NT*m
// (m < VPT); each thread keeps, for its voxels, the neighbour indices and the
// CG vectors x, r, z, p, t = L p, q = A p in registers for the whole solve.
// Only z and t are also written to global memory, because the stencil needs
// their values at neighbouring voxels owned by other workgroups.  Per
// iteration: phase B (q = A p, needs t at neighbours), phase C (x, r, z
// updates), phase D (p = z + beta p, t = L z + beta t, needs z at
// neighbours), each ended by a grid barrier.
// NXR > 0 (low-rank term, one voxel per thread, n_inj <= NXR): each thread
// keeps its voxel's row of X in registers, so the X^T z partials and the
// X (g o s) products read no memory.  NXR is 64 (rows held in FP64), or 128
// for FP32 data (rows held in FP32, 128 registers).  XTAIL: more injections than NXR; the
// first NXR rows are in registers and the rest are streamed (z staged in LDS
// for their partials), which halves the X traffic at 128 injections.
// CO (two-level, one voxel per thread): thread slots hold the voxels of whole
// aggregates (CoarseArg); z = D^-1 r + P Ainv P^T r needs the restricted
// residual of every workgroup, so each z update takes one more grid barrier
// (four per iteration).
template <typename T, int K, bool LR, int VPT, int BS, int NXR, bool XTAIL = false,
          bool CO = false>
__global__ __launch_bounds__(BS) void k_pcg(PcgArgs<T> a) {
  static_assert(!XTAIL || NXR > 0, "a streamed tail follows register rows");
  static_assert(NXR == 0 || (LR && VPT == 1), "register-resident X needs LR and VPT 1");
  static_assert(!CO || VPT == 1, "two-level launches hold one voxel per thread");
  cgrp::grid_group grid = cgrp::this_grid();
  __shared__ double red[2 * BS / WAVE];
  __shared__ double redc[2 * BS / WAVE];  // phase C's own reduction slots (no leading barrier)
  __shared__ double zs[BS * VPT];
  __shared__ double slr[LR ? PCG_MAX_NINJ : 1];
  __shared__ double lred[NXR > 0 ? BS / WAVE : 1][NXR > 0 ? NXR : 1];
  __shared__ double crs[CO ? BS : 1];         // w r of the workgroup's slots
  __shared__ double cys[CO ? CO_MAXLOC : 1];  // Ainv rc of the workgroup's aggregates
  const int64_t n = a.g.n;
  const int nwg = gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * BS * VPT;
  // voxel of this thread's slot m (two-level: from the slot map)
  const int64_t co_vox = CO ? (int64_t)a.co.slot_vox[lo + threadIdx.x] : 0;
  const double co_w = CO ? a.co.slot_w[lo + threadIdx.x] : 0.0;
  const int co_a0 = CO ? a.co.wg_agg[blockIdx.x] : 0;
  const int co_nla = CO ? a.co.wg_agg[blockIdx.x + 1] - co_a0 : 0;
  const int co_la = CO ? (co_vox >= 0 ? a.co.slot_agg[lo + threadIdx.x] - co_a0 : -1) : -1;
  auto vox = [&](int m) -> int64_t { return CO ? co_vox : lo + threadIdx.x + BS * m; };
  // restriction: rc[a] = sum over the aggregate's slots of w r (the
  // workgroup's own aggregates); starts and ends with a workgroup barrier
  auto co_restrict = [&](double rv) {
    if constexpr (CO) {
      __syncthreads();
      crs[threadIdx.x] = co_w * rv;
      __syncthreads();
      for (int la = threadIdx.x; la < co_nla; la += BS) {
        const int ag = co_a0 + la;
        double s = 0.0;
        for (int q = a.co.agg_lo[ag]; q < a.co.agg_hi[ag]; ++q) s += crs[q];
        a.co.rc[ag] = s;
      }
    }
  };
  // after a grid barrier: y = Ainv rc for the workgroup's aggregates (one
  // wave per aggregate row), returns w y of this thread's aggregate
  auto co_apply = [&]() -> double {
    if constexpr (CO) {
      const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
      const int m = a.co.m;
      for (int la = wv; la < co_nla; la += BS / WAVE) {
        const double* row = a.co.Ainv + (int64_t)(co_a0 + la) * m;
        double s = 0.0;
        for (int b = lane; b < m; b += WAVE) s += row[b] * a.co.rc[b];
        s = wsum(s);
        if (lane == 0) cys[la] = s;
      }
      __syncthreads();
      return co_la >= 0 ? co_w * cys[co_la] : 0.0;
    }
    return 0.0;
  };
  double* part = a.part;
  double* lrpart = a.part + PCG_SLOTS * nwg;
  const double lam = a.lam;
  const double c1 = a.coef[0], c0 = a.coef[1];
  T* __restrict__ zg = a.z;
  T* __restrict__ tg = a.t;
  const T* __restrict__ Xm = a.Xm;
  const int64_t ldx = a.ldx;
  const int ninj = a.ninj;

  // 64 rows are held in FP64; 128 rows (FP32 data) stay FP32 and their
  // products are formed in FP32, so the compiler cannot hoist 128 converted
  // values into registers
  using XR = typename std::conditional<(NXR > PCG_NXR), T, double>::type;
  XR xr[NXR > 0 ? NXR : 1];
  auto xz = [&](int al, double zv) -> double {
    if constexpr (std::is_same<XR, double>::value)
      return xr[al] * zv;
    else
      return (double)(xr[al] * (XR)zv);
  };
  if (NXR > 0) {
    const int64_t i0 = vox(0);
#pragma unroll
    for (int al = 0; al < NXR; ++al)
      xr[al] = (i0 >= 0 && i0 < n && al < ninj) ? (XR)Xm[(int64_t)al * ldx + i0] : (XR)0;
    for (int al = threadIdx.x; al < NXR; al += BS) slr[al] = 0.0;
  }
  // per-workgroup partials of X^T z into lrpart (z of this thread's voxels)
  auto lr_part = [&](const double* zv) {
    if (NXR > 0) {
      static_assert(NXR % WAVE == 0, "the transposed wave sums cover WAVE injections each");
      const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
      const double zv0 = zv[0];
      if constexpr (BS == NT) {
        // one butterfly per 64 injections (256-thread groups)
        lred[wv][lane] = wave_transpose_sum([&](int al) { return xz(al, zv0); });
        if constexpr (NXR > WAVE)
          lred[wv][WAVE + lane] = wave_transpose_sum([&](int al) { return xz(WAVE + al, zv0); });
      } else {
        // 512-thread groups have 256 registers: a wave sum per injection
#pragma unroll
        for (int al = 0; al < (NXR > 0 ? NXR : 1); ++al) {
          const double v = wsum(xz(al, zv0));
          if (lane == 0) lred[wv][al] = v;
        }
      }
      __syncthreads();
      for (int al = threadIdx.x; al < (XTAIL ? NXR : ninj); al += BS) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < BS / WAVE; ++w) t += lred[w][al];
        lrpart[(int64_t)al * nwg + blockIdx.x] = t;
      }
      if constexpr (XTAIL) lr_partial<T, BS, CO>(a, zs, lo, n, nwg, lrpart, NXR);
    } else {
      lr_partial<T, BS, CO>(a, zs, lo, n, nwg, lrpart);
    }
  };

  int32_t nb[VPT][K];
  double x[VPT], r[VPT], z[VPT], p[VPT], t[VPT], mi[VPT], dd[VPT];
  bool ok[VPT];
  double rz = 0.0, bb = 0.0;
#pragma unroll
  for (int m = 0; m < VPT; ++m) {
    const int64_t i = vox(m);
    ok[m] = i >= 0 && i < n;
    double bi = 0.0;
    mi[m] = 0.0;
    dd[m] = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) nb[m][k] = 0;
    if (ok[m]) {
#pragma unroll
      for (int k = 0; k < K; ++k) nb[m][k] = a.g.nbr[(int64_t)k * n + i];
      bi = (double)a.b[i];
      mi[m] = (double)a.minv[i];
      if (a.dvec) dd[m] = (double)a.dvec[i];
    }
    x[m] = (a.x0 && ok[m]) ? (double)a.x0[i] : 0.0;
    r[m] = (double)(T)bi;
    double zc = 0.0;
    if constexpr (CO) {
      co_restrict(r[m]);
      grid_barrier(a.bar, grid);
      zc = co_apply();
    }
    z[m] = (double)(T)(mi[m] * r[m] + zc);
    p[m] = 0.0;
    t[m] = 0.0;
    if (ok[m]) zg[i] = (T)z[m];
    zs[threadIdx.x + BS * m] = z[m];
    rz += r[m] * z[m];
    bb += r[m] * r[m];
  }
  __syncthreads();
  if (LR) lr_part(z);
  block_sum2<BS>(rz, bb, red);
  if (threadIdx.x == 0) {
    part[1 * nwg + blockIdx.x] = rz;
    part[3 * nwg + blockIdx.x] = bb;
  }
  grid_barrier(a.bar, grid);
  double rz_cur, rr;
  grid_total2<BS, false>(part, 1, 3, nwg, red, rz_cur, rr);
  int status = 0, it = 0;
  // from a warm start x0 the kernel's b is the residual b - A x0: the
  // tolerance stays relative to the original right-hand side
  const double bnorm2 = a.bref ? *a.bref : rr;
  const double tol2 = a.rtol * a.rtol * bnorm2;
  if (!(bnorm2 > 0.0)) status = 2;  // zero or non-finite right-hand side

  if (status == 0 && !(rr <= tol2)) {
    // ---- p = z, t = L z, s = X^T z
#pragma unroll
    for (int m = 0; m < VPT; ++m) {
      if (ok[m]) {
        double s = (double)K * z[m];
#pragma unroll
        for (int k = 0; k < K; ++k) s -= (double)zg[nb[m][k]];
        p[m] = z[m];
        t[m] = (double)(T)s;
        tg[vox(m)] = (T)t[m];
      }
    }
    if (LR) {
      for (int al = blockIdx.x; al < ninj; al += nwg) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nwg; b += BS) s += lrpart[(int64_t)al * nwg + b];
        s = block_sum<BS>(s, red);
        if (threadIdx.x == 0) a.sbuf[al] = s;
      }
    }
    grid_barrier(a.bar, grid);

    for (it = 0; it < a.maxit; ++it) {
      // ---- phase B: q = A p, partial p.q
      // (the neighbour t values are loaded before the low-rank set-up's
      // workgroup barrier, so the two latencies overlap)
      constexpr int KP = VPT <= 2 ? K : 1;
      double tn[VPT <= 2 ? VPT : 1][KP];
      if constexpr (VPT <= 2) {
#pragma unroll
        for (int m = 0; m < VPT; ++m)
#pragma unroll
          for (int k = 0; k < K; ++k) tn[m][k] = ok[m] ? (double)tg[nb[m][k]] : 0.0;
      }
      if (LR) {
        for (int al = threadIdx.x; al < ninj; al += BS) slr[al] = a.gw[al] * a.sbuf[al];
        __syncthreads();
      }
      double q[VPT];
      double pq = 0.0;
#pragma unroll
      for (int m = 0; m < VPT; ++m) {
        q[m] = 0.0;
        if (ok[m]) {
          const int64_t i = vox(m);
          double lt = (double)K * t[m];
          if constexpr (VPT <= 2) {
#pragma unroll
            for (int k = 0; k < K; ++k) lt -= tn[m][k];
          } else {
#pragma unroll
            for (int k = 0; k < K; ++k) lt -= (double)tg[nb[m][k]];
          }
          double qi = lam * (lt + c1 * t[m] + c0 * p[m]) + dd[m] * p[m];
          if (LR) {
            double s = 0.0;
            if (NXR > 0) {
#pragma unroll
              for (int al = 0; al < (NXR > 0 ? NXR : 1); ++al) s += xz(al, slr[al]);
              if constexpr (XTAIL)
                for (int al = NXR; al < ninj; ++al)
                  s += (double)Xm[(int64_t)al * ldx + i] * slr[al];
            } else {
              for (int al = 0; al < ninj; ++al) s += (double)Xm[(int64_t)al * ldx + i] * slr[al];
            }
            qi += s;
          }
          q[m] = (double)(T)qi;
          pq += p[m] * q[m];
        }
      }
      pq = block_sum<BS, false>(pq, red);
      if (threadIdx.x == 0) part[0 * nwg + blockIdx.x] = pq;
      grid_barrier(a.bar, grid);

      // ---- phase C: x += alpha p, r -= alpha q, z = M^-1 r
      const double pq_tot = grid_total<BS, false>(part, 0, nwg, red);
      if (!(pq_tot > 0.0)) {
        status = 2;
        break;
      }
      const double alpha = rz_cur / pq_tot;
      double rzn = 0.0, rrn = 0.0;
      if constexpr (CO) {
        // two-level: r first, its restriction to every workgroup, then z
        if (ok[0]) {
          x[0] = (double)(T)(x[0] + alpha * p[0]);
          r[0] = (double)(T)(r[0] - alpha * q[0]);
        }
        co_restrict(r[0]);
        grid_barrier(a.bar, grid);
        const double zc = co_apply();
        if (ok[0]) {
          z[0] = (double)(T)(mi[0] * r[0] + zc);
          zg[vox(0)] = (T)z[0];
          rzn += r[0] * z[0];
          rrn += r[0] * r[0];
        }
        if (LR && (NXR == 0 || XTAIL)) zs[threadIdx.x] = z[0];
      } else {
#pragma unroll
      for (int m = 0; m < VPT; ++m) {
        if (ok[m]) {
          x[m] = (double)(T)(x[m] + alpha * p[m]);
          r[m] = (double)(T)(r[m] - alpha * q[m]);
          z[m] = (double)(T)(mi[m] * r[m]);
          zg[lo + threadIdx.x + BS * m] = (T)z[m];
          rzn += r[m] * z[m];
          rrn += r[m] * r[m];
        }
        if (LR && (NXR == 0 || XTAIL)) zs[threadIdx.x + BS * m] = z[m];
      }
      }
      if constexpr (LR && (NXR == 0 || XTAIL)) {
        __syncthreads();
        lr_part(z);
        block_sum2<BS>(rzn, rrn, red);
      } else {
        // the wave sums of r.z, r.r (and the X^T z partials) meet at one
        // workgroup barrier; redc and lred are written in this phase only
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const double wa = wsum(rzn), wb = wsum(rrn);
        if constexpr (LR) {
          const double zv0 = z[0];
          if constexpr (BS == NT) {
            lred[wv][lane] = wave_transpose_sum([&](int al) { return xz(al, zv0); });
            if constexpr (NXR > WAVE)
              lred[wv][WAVE + lane] =
                  wave_transpose_sum([&](int al) { return xz(WAVE + al, zv0); });
          } else {
#pragma unroll
            for (int al = 0; al < (NXR > 0 ? NXR : 1); ++al) {
              const double v = wsum(xz(al, zv0));
              if (lane == 0) lred[wv][al] = v;
            }
          }
        }
        if (lane == 0) {
          redc[wv] = wa;
          redc[BS / WAVE + wv] = wb;
        }
        __syncthreads();
        rzn = 0.0;
        rrn = 0.0;
#pragma unroll
        for (int k = 0; k < BS / WAVE; ++k) {
          rzn += redc[k];
          rrn += redc[BS / WAVE + k];
        }
        if constexpr (LR) {
          for (int al = threadIdx.x; al < ninj; al += BS) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < BS / WAVE; ++w) t += lred[w][al];
            lrpart[(int64_t)al * nwg + blockIdx.x] = t;
          }
        }
      }
      if (threadIdx.x == 0) {
        part[1 * nwg + blockIdx.x] = rzn;
        part[2 * nwg + blockIdx.x] = rrn;
      }
      grid_barrier(a.bar, grid);

      // ---- phase D: beta, convergence, p = z + beta p, t = L z + beta t
      // (the neighbour z values and this workgroup's first low-rank partial
      // sum are loaded before the reduction, so their latency overlaps it)
      double zn[VPT <= 2 ? VPT : 1][KP];
      if constexpr (VPT <= 2) {
#pragma unroll
        for (int m = 0; m < VPT; ++m)
#pragma unroll
          for (int k = 0; k < K; ++k) zn[m][k] = ok[m] ? (double)zg[nb[m][k]] : 0.0;
      }
      double ls0 = 0.0;
      if (LR && (int)blockIdx.x < ninj)
        for (int b = threadIdx.x; b < nwg; b += BS) ls0 += lrpart[(int64_t)blockIdx.x * nwg + b];
      double rz_new;
      grid_total2<BS, false>(part, 1, 2, nwg, red, rz_new, rr);
      if (rr <= tol2) {
        ++it;
        break;
      }
      const double beta = rz_new / rz_cur;
      rz_cur = rz_new;
#pragma unroll
      for (int m = 0; m < VPT; ++m) {
        if (ok[m]) {
          double lz = (double)K * z[m];
          if constexpr (VPT <= 2) {
#pragma unroll
            for (int k = 0; k < K; ++k) lz -= zn[m][k];
          } else {
#pragma unroll
            for (int k = 0; k < K; ++k) lz -= (double)zg[nb[m][k]];
          }
          p[m] = (double)(T)(z[m] + beta * p[m]);
          t[m] = (double)(T)(lz + beta * t[m]);
          tg[vox(m)] = (T)t[m];
        }
      }
      if (LR) {
        for (int al = blockIdx.x; al < ninj; al += nwg) {
          double s = 0.0;
          if (al == (int)blockIdx.x) {
            s = ls0;
          } else {
            for (int b = threadIdx.x; b < nwg; b += BS) s += lrpart[(int64_t)al * nwg + b];
          }
          s = block_sum<BS>(s, red);
          if (threadIdx.x == 0) a.sbuf[al] = s + beta * a.sbuf[al];
        }
      }
      grid_barrier(a.bar, grid);
    }
    if (status == 0 && !(rr <= tol2)) status = 1;
  }

  // ---- final: x to global, xout = x / ||x||
  double xx = 0.0;
#pragma unroll
  for (int m = 0; m < VPT; ++m) xx += x[m] * x[m];
  xx = block_sum<BS>(xx, red);
  if (threadIdx.x == 0) part[4 * nwg + blockIdx.x] = xx;
  grid_barrier(a.bar, grid);
  const double xnorm2 = grid_total<BS, false>(part, 4, nwg, red);
  const double xn = sqrt(xnorm2);
  const double inv = xn > 0.0 ? 1.0 / xn : 0.0;
#pragma unroll
  for (int m = 0; m < VPT; ++m) {
    const int64_t i = vox(m);
    if (ok[m]) {
      a.x[i] = (T)x[m];
      a.xout[i] = (T)(x[m] * inv);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.scal[0] = xn;
    a.scal[1] = bnorm2 > 0.0 ? sqrt(rr / bnorm2) : 0.0;
    a.scal[2] = (double)it;
    const bool timed_out =
        a.bar.mode == 1 &&
        __hip_atomic_load(a.bar.bar + BAR_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    a.scal[3] = timed_out ? PERSIST_TIMEOUT : (double)status;
  }
}

template <typename T, int K, bool LR, int BS>
static void* pcg_fn_vb(int vpt) {
  switch (vpt) {
    case 1: return (void*)&k_pcg<T, K, LR, 1, BS, 0>;
    case 2: return (void*)&k_pcg<T, K, LR, 2, BS, 0>;
    case 4: return (void*)&k_pcg<T, K, LR, 4, BS, 0>;
    case 8: return (void*)&k_pcg<T, K, LR, 8, BS, 0>;
    default: return nullptr;
  }
}

// two-level launches (v-systems: low-rank term, one voxel per thread)
template <typename T, int K>
static void* pcg_fn_co(int bs, int nxr, int xtail) {
  if (nxr == 0)
    return bs == 512 ? (void*)&k_pcg<T, K, true, 1, 512, 0, false, true>
                     : bs == NT ? (void*)&k_pcg<T, K, true, 1, NT, 0, false, true> : nullptr;
  if (xtail)
    return (nxr == PCG_NXR && bs == 512) ? (void*)&k_pcg<T, K, true, 1, 512, PCG_NXR, true, true>
                                          : nullptr;
  if (nxr == PCG_NXR2) {
    if constexpr (std::is_same<T, float>::value)
      return bs == 512 ? (void*)&k_pcg<T, K, true, 1, 512, PCG_NXR2, false, true>
                       : bs == NT ? (void*)&k_pcg<T, K, true, 1, NT, PCG_NXR2, false, true>
                                  : nullptr;
    return nullptr;
  }
  if (nxr != PCG_NXR) return nullptr;
  return bs == 512 ? (void*)&k_pcg<T, K, true, 1, 512, PCG_NXR, false, true>
                   : bs == NT ? (void*)&k_pcg<T, K, true, 1, NT, PCG_NXR, false, true> : nullptr;
}

template <typename T, int K, bool LR>
static void* pcg_fn_v(int vpt, int bs, int nxr, int xtail, bool co) {
  if (co) {
    if (!LR || vpt != 1) return nullptr;
    return pcg_fn_co<T, K>(bs, nxr, xtail);
  }
  if (nxr > 0) {  // register-resident X: one voxel per thread, 256- or 512-thread groups
    if (!LR || vpt != 1) return nullptr;
    if (xtail) {  // 64 register rows and a streamed tail, 512-thread groups
      if (nxr != PCG_NXR) return nullptr;
      return bs == 512 ? (void*)&k_pcg<T, K, true, 1, 512, PCG_NXR, true> : nullptr;
    }
    if (nxr == PCG_NXR2) {  // 128 rows: FP32 data only
      if constexpr (std::is_same<T, float>::value)
        return bs == 512 ? (void*)&k_pcg<T, K, true, 1, 512, PCG_NXR2>
                         : bs == NT ? (void*)&k_pcg<T, K, true, 1, NT, PCG_NXR2> : nullptr;
      return nullptr;
    }
    if (nxr != PCG_NXR) return nullptr;
    return bs == 512 ? (void*)&k_pcg<T, K, true, 1, 512, PCG_NXR>
                     : bs == NT ? (void*)&k_pcg<T, K, true, 1, NT, PCG_NXR> : nullptr;
  }
  return bs == 1024 ? pcg_fn_vb<T, K, LR, 1024>(vpt)
                    : bs == NT ? pcg_fn_vb<T, K, LR, NT>(vpt) : nullptr;
}

template <typename T>
static void* pcg_select(int K, bool lr, int vpt, int bs, int nxr, int xtail, bool co) {
  switch (K) {
#define CASE(KK)                                                                     \
  case KK:                                                                           \
    return lr ? pcg_fn_v<T, KK, true>(vpt, bs, nxr, xtail, co)                       \
              : pcg_fn_v<T, KK, false>(vpt, bs, nxr, xtail, co);
    CASE(2) CASE(4) CASE(6) CASE(8)
#undef CASE
    default:
      return nullptr;
  }
}

template <typename T>
int pcg_max_wg(const PcgArgs<T>& a) {
  void* fn = pcg_select<T>(a.g.K, a.Xm != nullptr, a.vpt, a.bs, a.nxr, a.xtail,
                           a.co.slot_vox != nullptr);
  if (!fn) return 0;
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, a.bs, 0) != hipSuccess) return 0;
  return per * ncu;
}

template <typename T>
cr_status pcg_solve(const PcgArgs<T>& a, int nwg, hipStream_t st) {
  if (a.vpt < 1 || a.vpt > PCG_MAX_VPT) {
    set_error("pcg: voxels per thread out of range");
    return CR_EINVAL;
  }
  if (a.Xm && a.ninj > PCG_MAX_NINJ) {
    set_error("pcg: n_inj above the low-rank limit");
    return CR_EINVAL;
  }
  if (!a.co.slot_vox && (int64_t)nwg * a.bs * a.vpt < a.g.n) {
    set_error("pcg: grid does not cover the voxels");
    return CR_EINVAL;
  }
  void* fn = pcg_select<T>(a.g.K, a.Xm != nullptr, a.vpt, a.bs, a.nxr, a.xtail,
                           a.co.slot_vox != nullptr);
  if (!fn) {
    set_error("pcg: unsupported stencil width or voxels per thread");
    return CR_EINVAL;
  }
  PcgArgs<T> arg = a;
  if (arg.bar.mode == 1) CR_HIP(hipMemsetAsync(arg.bar.bar, 0, BAR_WORDS * sizeof(unsigned), st));
  void* params[] = {&arg};
  if (arg.bar.coop || arg.bar.mode == 0)
    CR_HIP(hipLaunchCooperativeKernel(fn, dim3(nwg), dim3(arg.bs), params, 0, st));
  else
    CR_HIP(hipLaunchKernel(fn, dim3(nwg), dim3(arg.bs), params, 0, st));
  return CR_OK;
}

// Jacobi inverse diagonal.  (L^2)_ii = deg_i^2 + deg_i for a unit-weight
// graph Laplacian, (L)_ii = deg_i.
template <typename T>
__global__ __launch_bounds__(NT) void k_pcg_diag(int64_t n, const uint8_t* __restrict__ deg,
                                                 double lam, const double* __restrict__ coef,
                                                 const T* __restrict__ dvec,
                                                 const T* __restrict__ Xm, int64_t ldx, int ninj,
                                                 const double* __restrict__ gw,
                                                 T* __restrict__ minv) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const double dg = (double)deg[i];
  double v = lam * (dg * dg + dg + coef[0] * dg + coef[1]);
  if (dvec) v += (double)dvec[i];
  if (Xm)
    for (int al = 0; al < ninj; ++al) {
      const double x = (double)Xm[(int64_t)al * ldx + i];
      v += gw[al] * x * x;
    }
  minv[i] = (T)(v > 0.0 ? 1.0 / v : 1.0);
}

template <typename T>
cr_status pcg_diag(const Geom& g, double lam, const double* coef, const T* dvec, const T* Xm,
                   int64_t ldx, int ninj, const double* gw, T* minv, hipStream_t st) {
  if (g.n == 0) return CR_OK;
  hipLaunchKernelGGL((k_pcg_diag<T>), dim3((unsigned)((g.n + NT - 1) / NT)), dim3(NT), 0, st, g.n,
                     g.deg, lam, coef, dvec, Xm, ldx, ninj, gw, minv);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// ================================================================ Galerkin CG
// Partial-sum slots: 0 <P,Q>, 1 initial ||R||^2, 2 ||R||^2, 3 ||B||^2,
// 4 <Z,B>, 5 <Z,R> (6 * nwg doubles).
// A_p(P) = lam (P Bx2 + 2 By1 P Bx1 + By2 P) + sum_a G_a (P h_a) h_a^T, with
// h_a = H[:,a] (H(k,a) stored as Ht[a + k*ninj]).  Column c of every r x r
// matrix is owned by workgroup c mod nwg for element-wise updates.
__device__ __forceinline__ double Hk(const GalerkinArgs& a, int k, int al) {
  return a.H[(int64_t)k * a.ninj + al];
}
__device__ __forceinline__ double Sk(const GalerkinArgs& a, int k, int al) {
  return a.S[(int64_t)k * a.ninj + al];
}

// phase 1: SG[:,a] = G_a (P h_a) for the workgroup's injections; Y2 = By1 P
// for its columns.
__device__ void gal_phase1(const GalerkinArgs& a, const double* Pm, double* tsh) {
  const int r = a.r, ld = a.ldr;
  for (int al = blockIdx.x; al < a.ninj; al += gridDim.x) {
    __syncthreads();
    for (int i = threadIdx.x; i < r; i += NT) {
      double s = 0.0;
      for (int k = 0; k < r; ++k) s += Pm[(int64_t)k * ld + i] * Hk(a, k, al);
      tsh[i] = s;
    }
    __syncthreads();
    const double* Ga = a.G + (int64_t)al * ld * ld;
    for (int i = threadIdx.x; i < r; i += NT) {
      double s = 0.0;
      for (int k = 0; k < r; ++k) s += Ga[(int64_t)k * ld + i] * tsh[k];
      a.SG[(int64_t)al * ld + i] = s;
    }
  }
  for (int c = blockIdx.x; c < r; c += gridDim.x) {
    for (int i = threadIdx.x; i < r; i += NT) {
      double s = 0.0;
      for (int k = 0; k < r; ++k) s += a.By1[(int64_t)k * ld + i] * Pm[(int64_t)c * ld + k];
      a.Y2[(int64_t)c * ld + i] = s;
    }
  }
}

// phase 2: Q[:,c] for the workgroup's columns; returns partial <Pm, Q>.
__device__ double gal_phase2(const GalerkinArgs& a, const double* Pm) {
  const int r = a.r, ld = a.ldr;
  double dot = 0.0;
  for (int c = blockIdx.x; c < r; c += gridDim.x) {
    for (int i = threadIdx.x; i < r; i += NT) {
      double s = 0.0;
      for (int al = 0; al < a.ninj; ++al) s += a.SG[(int64_t)al * ld + i] * Hk(a, c, al);
      double t = 0.0;
      for (int k = 0; k < r; ++k)
        t += Pm[(int64_t)k * ld + i] * a.Bx2[(int64_t)c * ld + k] +
             a.By2[(int64_t)k * ld + i] * Pm[(int64_t)c * ld + k] +
             2.0 * a.Y2[(int64_t)k * ld + i] * a.Bx1[(int64_t)c * ld + k];
      const double q = s + a.lam * t;
      a.Q[(int64_t)c * ld + i] = q;
      dot += Pm[(int64_t)c * ld + i] * q;
    }
  }
  return dot;
}

__global__ __launch_bounds__(NT) void k_galerkin(GalerkinArgs a) {
  cgrp::grid_group grid = cgrp::this_grid();
  __shared__ double red[NT / WAVE];
  extern __shared__ double tsh[];
  const int r = a.r, ld = a.ldr, nwg = gridDim.x;
  double* part = a.part;

  // ---- B = S H^T ; Q = A_p(Z)
  gal_phase1(a, a.Z, tsh);
  for (int c = blockIdx.x; c < r; c += nwg)
    for (int i = threadIdx.x; i < r; i += NT) {
      double s = 0.0;
      for (int al = 0; al < a.ninj; ++al) s += Sk(a, i, al) * Hk(a, c, al);
      a.Bm[(int64_t)c * ld + i] = s;
    }
  grid_barrier(a.bar, grid);
  gal_phase2(a, a.Z);
  // R = B - Q, P = R (own columns); partial ||R||^2, ||B||^2
  double rr = 0.0, bb = 0.0;
  for (int c = blockIdx.x; c < r; c += nwg)
    for (int i = threadIdx.x; i < r; i += NT) {
      const int64_t e = (int64_t)c * ld + i;
      const double b = a.Bm[e];
      const double rv = b - a.Q[e];
      a.R[e] = rv;
      a.P[e] = rv;
      rr += rv * rv;
      bb += b * b;
    }
  rr = block_sum(rr, red);
  bb = block_sum(bb, red);
  if (threadIdx.x == 0) {
    part[1 * nwg + blockIdx.x] = rr;
    part[3 * nwg + blockIdx.x] = bb;
  }
  grid_barrier(a.bar, grid);
  rr = grid_total(part, 1, nwg, red);
  bb = grid_total(part, 3, nwg, red);
  const double tol2 = a.rtol * a.rtol * bb;
  int it = 0, status = 0;
  for (; it < a.maxit && rr > tol2; ++it) {
    gal_phase1(a, a.P, tsh);
    grid_barrier(a.bar, grid);
    double pq = gal_phase2(a, a.P);
    pq = block_sum(pq, red);
    if (threadIdx.x == 0) part[0 * nwg + blockIdx.x] = pq;
    grid_barrier(a.bar, grid);
    const double pq_tot = grid_total(part, 0, nwg, red);
    if (!(pq_tot > 0.0)) {
      status = 2;
      break;
    }
    const double alpha = rr / pq_tot;
    double rrn = 0.0;
    for (int c = blockIdx.x; c < r; c += nwg)
      for (int i = threadIdx.x; i < r; i += NT) {
        const int64_t e = (int64_t)c * ld + i;
        a.Z[e] += alpha * a.P[e];
        const double rv = a.R[e] - alpha * a.Q[e];
        a.R[e] = rv;
        rrn += rv * rv;
      }
    rrn = block_sum(rrn, red);
    if (threadIdx.x == 0) part[2 * nwg + blockIdx.x] = rrn;
    grid_barrier(a.bar, grid);
    const double rr_new = grid_total(part, 2, nwg, red);
    const double beta = rr_new / rr;
    rr = rr_new;
    if (rr <= tol2) {
      ++it;
      break;
    }
    for (int c = blockIdx.x; c < r; c += nwg)
      for (int i = threadIdx.x; i < r; i += NT) {
        const int64_t e = (int64_t)c * ld + i;
        a.P[e] = a.R[e] + beta * a.P[e];
      }
    grid_barrier(a.bar, grid);
  }
  if (status == 0 && rr > tol2) status = 1;
  // energy pieces: <Z, B>, <Z, R>
  double zb = 0.0, zr = 0.0;
  for (int c = blockIdx.x; c < r; c += nwg)
    for (int i = threadIdx.x; i < r; i += NT) {
      const int64_t e = (int64_t)c * ld + i;
      zb += a.Z[e] * a.Bm[e];
      zr += a.Z[e] * a.R[e];
    }
  zb = block_sum(zb, red);
  zr = block_sum(zr, red);
  // slots 4, 5 are written only here (slower workgroups may still be reading
  // slots 0..3 of the exit test)
  if (threadIdx.x == 0) {
    part[4 * nwg + blockIdx.x] = zb;
    part[5 * nwg + blockIdx.x] = zr;
  }
  grid_barrier(a.bar, grid);
  zb = grid_total(part, 4, nwg, red);
  zr = grid_total(part, 5, nwg, red);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.scal[0] = (double)it;
    a.scal[1] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    const bool timed_out =
        a.bar.mode == 1 &&
        __hip_atomic_load(a.bar.bar + BAR_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
    a.scal[2] = timed_out ? PERSIST_TIMEOUT : (double)status;
    a.scal[3] = -0.5 * zb - 0.5 * zr;  // 1/2 <Z, A_p Z> - <Z, B> with A_p Z = B - R
  }
}

int galerkin_max_wg(int r) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (void*)k_galerkin, NT,
                                                   sizeof(double) * std::max(r, 1)) != hipSuccess)
    return 0;
  return per * ncu;
}

cr_status galerkin_cg(const GalerkinArgs& a, int nwg, hipStream_t st) {
  if (a.r <= 0) return CR_OK;
  GalerkinArgs arg = a;
  if (arg.bar.mode == 1) CR_HIP(hipMemsetAsync(arg.bar.bar, 0, BAR_WORDS * sizeof(unsigned), st));
  void* params[] = {&arg};
  if (!arg.bar.coop && arg.bar.mode == 1)
    CR_HIP(hipLaunchKernel((void*)k_galerkin, dim3(nwg), dim3(NT), params, sizeof(double) * a.r, st));
  else
    CR_HIP(hipLaunchCooperativeKernel((void*)k_galerkin, dim3(nwg), dim3(NT), params,
                                    sizeof(double) * a.r, st));
  return CR_OK;
}

// ------------------------------------------------------------ refinement helpers
template <typename T, int K, bool LR>
__global__ __launch_bounds__(NT) void k_als_resid(int64_t n, const int32_t* __restrict__ nbr,
                                                  double lam, const double* __restrict__ coef,
                                                  const T* __restrict__ dvec,
                                                  const T* __restrict__ Xm, int64_t ldx, int ninj,
                                                  const double* __restrict__ gw,
                                                  const double* __restrict__ s,
                                                  const T* __restrict__ b,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ t,
                                                  double* __restrict__ r) {
  __shared__ double gs[LR ? PCG_MAX_NINJ : 1];
  if (LR) {
    for (int al = threadIdx.x; al < ninj; al += NT) gs[al] = gw[al] * s[al];
    __syncthreads();
  }
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i], ti = t[i];
  double q = lam * (lap<double, K>(t, nbr, n, i) + coef[0] * ti + coef[1] * xi);
  if (dvec) q += (double)dvec[i] * xi;
  if (LR) {
    double acc = 0.0;
    for (int al = 0; al < ninj; ++al) acc += (double)Xm[(int64_t)al * ldx + i] * gs[al];
    q += acc;
  }
  r[i] = (double)b[i] - q;
}

template <typename T>
cr_status als_residual(const Geom& g, double lam, const double* coef, const T* dvec, const T* Xm,
                       int64_t ldx, int ninj, const double* gw, const double* s, const T* b,
                       const double* x, double* t, double* r, hipStream_t st) {
  if (g.n == 0) return CR_OK;
  CR_TRY(stencil<double>(g, 1, x, g.n, t, g.n, st));
  const dim3 grid((unsigned)((g.n + NT - 1) / NT));
  switch (g.K) {
#define CASE(KK)                                                                                \
  case KK:                                                                                      \
    if (Xm)                                                                                     \
      hipLaunchKernelGGL((k_als_resid<T, KK, true>), grid, dim3(NT), 0, st, g.n, g.nbr, lam,   \
                         coef, dvec, Xm, ldx, ninj, gw, s, b, x, t, r);                        \
    else                                                                                        \
      hipLaunchKernelGGL((k_als_resid<T, KK, false>), grid, dim3(NT), 0, st, g.n, g.nbr, lam,  \
                         coef, dvec, Xm, ldx, ninj, gw, s, b, x, t, r);                        \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default:
      set_error("unsupported stencil width");
      return CR_EINVAL;
  }
  CR_HIP(hipGetLastError());
  return CR_OK;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_accumulate(int64_t n, const T* __restrict__ e,
                                                   double* __restrict__ x, int init) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  x[i] = init ? (double)e[i] : x[i] + (double)e[i];
}

template <typename T>
cr_status accumulate(int64_t n, const T* e, double* x, bool init, hipStream_t st) {
  if (n == 0) return CR_OK;
  hipLaunchKernelGGL((k_accumulate<T>), dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, n, e,
                     x, init ? 1 : 0);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_normalize_out(int64_t n, const double* __restrict__ x,
                                                      const double* __restrict__ nrm2,
                                                      T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const double s = nrm2[0] > 0.0 ? 1.0 / sqrt(nrm2[0]) : 0.0;
  out[i] = (T)(x[i] * s);
}

template <typename T>
cr_status normalize_out(int64_t n, const double* x, const double* nrm2, T* out, hipStream_t st) {
  if (n == 0) return CR_OK;
  hipLaunchKernelGGL((k_normalize_out<T>), dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, n,
                     x, nrm2, out);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

#define INST(T)                                                                              \
  template cr_status als_residual<T>(const Geom&, double, const double*, const T*, const T*, \
                                     int64_t, int, const double*, const double*, const T*,  \
                                     const double*, double*, double*, hipStream_t);          \
  template cr_status accumulate<T>(int64_t, const T*, double*, bool, hipStream_t);          \
  template cr_status normalize_out<T>(int64_t, const double*, const double*, T*, hipStream_t); \
  template cr_status pcg_solve<T>(const PcgArgs<T>&, int, hipStream_t);                     \
  template int pcg_max_wg<T>(const PcgArgs<T>&);                                            \
  template cr_status pcg_diag<T>(const Geom&, double, const double*, const T*, const T*,    \
                                 int64_t, int, const double*, T*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace cr
