// Persistent (cooperative) conjugate-gradient kernels:
//  * k_pcg      Jacobi-PCG on the ALS half-step systems (eqs. ALS_linsys and
//               ALS_linsys_v), one launch per solve, three grid barriers per
//               iteration;
//  * k_galerkin matrix-valued CG on the projected equation (eq. Proj_Sylv)
//               in FP64 (FP64 MFMA tiles), four grid barriers per iteration.
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
    const bool last = prev == nwg - 1;
    if (last) {
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
// XLDS (with XTAIL): the first a.xlds tail rows are loaded once into LDS
// (dynamic shared memory, a.xlds * BS values of type T) and read from there every
// iteration; the rows after them, if any, are streamed (512-thread groups
// only: 256-thread groups hold the whole tail).
// CO (two-level, one voxel per thread): thread slots hold the voxels of whole
// aggregates (CoarseArg); z = D^-1 r + P Ainv P^T r needs the restricted
// residual of every workgroup, so each z update takes one more grid barrier
// (four per iteration).
// R2 (one voxel per thread, no tail, no coarse level): phase B is folded into
// phase D, which also carries u = L^2 p by its own recurrence u = L^2 z +
// beta u from z at the voxels of the thread's row of L^2 (tables in LDS), and
// every workgroup sums all X^T z partials itself; two grid barriers per
// iteration.
template <typename T, int K, bool LR, int VPT, int BS, int NXR, bool XTAIL = false,
          bool CO = false, bool XLDS = false, bool R2 = false>
__global__ __launch_bounds__(BS) void k_pcg(PcgArgs<T> a) {
  static_assert(!R2 || (VPT == 1 && !XTAIL && !CO && !XLDS && (!LR || NXR > 0)),
                "the two-barrier form: one voxel per thread, no tail of X, no coarse level");
  static_assert(!XTAIL || NXR > 0, "a streamed tail follows register rows");
  static_assert(!XLDS || (XTAIL && !CO), "the LDS-resident rows are part of the tail");
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
  extern __shared__ double xtl_raw[];
  T* const xtl = reinterpret_cast<T*>(xtl_raw);  // XLDS: tail rows (type T), xtl[(al - NXR) * BS + thread]
  // R2: this thread's row of L^2 (ring-2 voxels and all coefficients), and
  // the workgroup's own copy of s = X^T p with its reduction slots
  __shared__ int32_t r2x[R2 ? R2_NX : 1][R2 ? BS : 1];
  __shared__ int8_t r2k[R2 ? R2_NC : 1][R2 ? BS : 1];
  __shared__ double s2[R2 && LR ? NXR : 1];
  __shared__ double s2n[R2 && LR ? NXR : 1];
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
    if constexpr (XLDS) {
      for (int al = NXR; al < NXR + a.xlds; ++al)
        xtl[(al - NXR) * BS + threadIdx.x] = (i0 >= 0 && i0 < n) ? Xm[(int64_t)al * ldx + i0] : (T)0;
    }
  }
  if constexpr (R2) {
    const int64_t i0 = vox(0);
    const bool in = i0 >= 0 && i0 < n;
#pragma unroll
    for (int e = 0; e < R2_NX; ++e) r2x[e][threadIdx.x] = in ? a.g.r2idx[(int64_t)e * n + i0] : 0;
#pragma unroll
    for (int e = 0; e < R2_NC; ++e)
      r2k[e][threadIdx.x] = in ? a.g.r2cf[(int64_t)e * n + i0] : (int8_t)0;
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
      if constexpr (XLDS) {
        // tail partials from the LDS rows: one wave per injection; the
        // rows after them streamed
        for (int al = NXR + wv; al < NXR + a.xlds; al += BS / WAVE) {
          const T* xt = xtl + (al - NXR) * BS;
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < BS / WAVE; ++k)
            acc += (double)xt[lane + WAVE * k] * zs[lane + WAVE * k];
          acc = wsum(acc);
          if (lane == 0) lrpart[(int64_t)al * nwg + blockIdx.x] = acc;
        }
        // (256-thread groups hold the whole tail: no streamed rows)
        if constexpr (BS != NT)
          if (NXR + a.xlds < ninj) lr_partial<T, BS, CO>(a, zs, lo, n, nwg, lrpart, NXR + a.xlds);
      } else if constexpr (XTAIL) {
        lr_partial<T, BS, CO>(a, zs, lo, n, nwg, lrpart, NXR);
      }
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

  constexpr int KP = VPT <= 2 ? K : 1;
  double q[VPT];
#pragma unroll
  for (int m = 0; m < VPT; ++m) q[m] = 0.0;
  // R2 (one voxel per thread): u = L^2 p kept by its own recurrence from
  // L^2 z, formed from z at the ring-2 voxels of the thread's row of L^2,
  // so that q = A p needs no neighbour values of t and no third barrier.
  // Every workgroup also sums all workgroups' X^T z partials itself (in the
  // same order, so the copies of s = X^T p agree bit for bit).
  double u2 = 0.0;
  // gathered in the storage type (FP32 data: half the registers), widened
  // where they are used
  T zn1[R2 ? K : 1], z2[R2 ? R2_NX : 1];
  auto r2_load = [&]() {
    if constexpr (R2) {
#pragma unroll
      for (int k = 0; k < K; ++k) zn1[k] = ok[0] ? zg[nb[0][k]] : (T)0;
#pragma unroll
      for (int e = 0; e < R2_NX; ++e) z2[e] = ok[0] ? zg[r2x[e][threadIdx.x]] : (T)0;
      if constexpr (LR) {
        // wave w sums injections w, w + BS/WAVE, ...: every partial load of
        // a lane is issued before the first wave sum
        constexpr int NJ = (NXR > 0 ? NXR : 1) / (BS / WAVE);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        double acc[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[j] = 0.0;
        for (int b = lane; b < nwg; b += WAVE) {
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            const int al = wv + (BS / WAVE) * j;
            if (al < ninj) acc[j] += lrpart[(int64_t)al * nwg + b];
          }
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int al = wv + (BS / WAVE) * j;
          const double v = wsum(acc[j]);
          if (lane == 0 && al < ninj) s2n[al] = v;
        }
      }
    }
  };
  auto r2_update = [&](double beta, bool first) {
    if constexpr (R2) {
      if (ok[0]) {
        double lz = (double)K * z[0];
        double l2 = (double)r2k[0][threadIdx.x] * z[0];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          lz -= (double)zn1[k];
          l2 += (double)r2k[1 + k][threadIdx.x] * (double)zn1[k];
        }
#pragma unroll
        for (int e = 0; e < R2_NX; ++e)
          l2 += (double)r2k[R2_C0 + e][threadIdx.x] * (double)z2[e];
        p[0] = (double)(T)(z[0] + beta * p[0]);
        t[0] = (double)(T)(lz + beta * t[0]);
        u2 = (double)(T)(l2 + beta * u2);
      }
      if constexpr (LR) {
        __syncthreads();
        for (int al = threadIdx.x; al < ninj; al += BS) {
          s2[al] = first ? s2n[al] : s2n[al] + beta * s2[al];
          slr[al] = a.gw[al] * s2[al];
        }
        __syncthreads();
      }
      double pq = 0.0;
      q[0] = 0.0;
      if (ok[0]) {
        double qi = lam * (u2 + c1 * t[0] + c0 * p[0]) + dd[0] * p[0];
        if constexpr (LR) {
          double sacc = 0.0;
#pragma unroll
          for (int al = 0; al < (NXR > 0 ? NXR : 1); ++al) sacc += xz(al, slr[al]);
          qi += sacc;
        }
        q[0] = (double)(T)qi;
        pq = p[0] * q[0];
      }
      // (with the low-rank term the workgroup barriers above already
      // separate this write of red from the grid total's reads of it)
      pq = block_sum<BS, !LR>(pq, red);
      if (threadIdx.x == 0) part[0 * nwg + blockIdx.x] = pq;
    }
  };

  if (status == 0 && !(rr <= tol2)) {
    if constexpr (R2) {
      // ---- p = z, t = L z, u = L^2 z, s = X^T z (reduced in every
      // workgroup), q = A p and its partial p.q: the loop then starts with
      // phase C and ends with phase D, two grid barriers per iteration
      r2_load();
      r2_update(0.0, true);
      grid_barrier(a.bar, grid);
    } else {
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
    }

    for (it = 0; it < a.maxit; ++it) {
      if constexpr (!R2) {
      // ---- phase B: q = A p, partial p.q
      // (the neighbour t values are loaded before the low-rank set-up's
      // workgroup barrier, so the two latencies overlap)
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
              if constexpr (XLDS) {
                const int al1 = BS == NT ? ninj : NXR + a.xlds;
                for (int al = NXR; al < al1; ++al)
                  s += (double)xtl[(al - NXR) * BS + threadIdx.x] * slr[al];
                if constexpr (BS != NT)
                  for (int al = al1; al < ninj; ++al)
                    s += (double)Xm[(int64_t)al * ldx + i] * slr[al];
              } else if constexpr (XTAIL) {
                for (int al = NXR; al < ninj; ++al)
                  s += (double)Xm[(int64_t)al * ldx + i] * slr[al];
              }
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
      }

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
      if constexpr (R2) {
        // two-barrier form: also u = L^2 z + beta u and s = X^T z + beta s,
        // then q = A p and its partial p.q (phase B folded in)
        r2_load();
        double rz_new;
        grid_total2<BS, false>(part, 1, 2, nwg, red, rz_new, rr);
        if (rr <= tol2) {
          ++it;
          break;
        }
        const double beta = rz_new / rz_cur;
        rz_cur = rz_new;
        r2_update(beta, false);
      } else {
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
    return (xtail == 1 && nxr == PCG_NXR && bs == 512)
               ? (void*)&k_pcg<T, K, true, 1, 512, PCG_NXR, true, true>
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
    if (xtail == 2) {  // 64 register rows and the tail (or its first rows) in LDS
      if (nxr != PCG_NXR) return nullptr;
      return bs == NT ? (void*)&k_pcg<T, K, true, 1, NT, PCG_NXR, true, false, true>
                      : bs == 512 ? (void*)&k_pcg<T, K, true, 1, 512, PCG_NXR, true, false, true>
                                  : nullptr;
    }
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

// The two-barrier form (R2) where the geometry has its rows of L^2 and the
// launch holds one voxel per thread with no tail of X and no coarse level.
template <typename T>
static void* pcg_select_r2(const PcgArgs<T>& a, bool co) {
  if (!a.g.r2idx || !a.g.r2cf || co || a.vpt != 1 || a.xtail != 0) return nullptr;
  const bool lr = a.Xm != nullptr;
  switch (a.g.K) {
#define R2CASE(KK)                                                                          \
  case KK:                                                                                  \
    if (!lr)                                                                                \
      return a.bs == 1024 ? (void*)&k_pcg<T, KK, false, 1, 1024, 0, false, false, false, true> \
             : a.bs == NT ? (void*)&k_pcg<T, KK, false, 1, NT, 0, false, false, false, true>   \
                          : nullptr;                                                        \
    if (a.nxr == PCG_NXR)                                                                   \
      return a.bs == NT ? (void*)&k_pcg<T, KK, true, 1, NT, PCG_NXR, false, false, false, true> \
             : a.bs == 512                                                                  \
                 ? (void*)&k_pcg<T, KK, true, 1, 512, PCG_NXR, false, false, false, true>   \
                 : nullptr;                                                                 \
    if constexpr (std::is_same<T, float>::value) {                                         \
      if (a.nxr == PCG_NXR2)                                                                \
        return a.bs == NT                                                                   \
                   ? (void*)&k_pcg<T, KK, true, 1, NT, PCG_NXR2, false, false, false, true> \
                   : a.bs == 512                                                            \
                         ? (void*)&k_pcg<T, KK, true, 1, 512, PCG_NXR2, false, false, false, true> \
                         : nullptr;                                                         \
    }                                                                                       \
    return nullptr;
    R2CASE(4) R2CASE(6)
#undef R2CASE
    default:
      return nullptr;
  }
}

// dynamic LDS of a launch: the tail rows of the LDS-resident form
template <typename T>
static size_t pcg_dyn_lds(const PcgArgs<T>& a) {
  return a.xtail == 2 ? sizeof(T) * (size_t)std::max(0, a.xlds) * (size_t)a.bs : 0;
}

template <typename T>
int pcg_max_wg(const PcgArgs<T>& a) {
  void* fn = pcg_select_r2<T>(a, a.co.slot_vox != nullptr);
  if (!fn)
    fn = pcg_select<T>(a.g.K, a.Xm != nullptr, a.vpt, a.bs, a.nxr, a.xtail,
                       a.co.slot_vox != nullptr);
  if (!fn) return 0;
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, a.bs, pcg_dyn_lds(a)) != hipSuccess)
    return 0;
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
  void* fn = pcg_select_r2<T>(a, a.co.slot_vox != nullptr);
  if (!fn)
    fn = pcg_select<T>(a.g.K, a.Xm != nullptr, a.vpt, a.bs, a.nxr, a.xtail,
                       a.co.slot_vox != nullptr);
  if (!fn) {
    set_error("pcg: unsupported stencil width or voxels per thread");
    return CR_EINVAL;
  }
  PcgArgs<T> arg = a;
  if (arg.bar.mode == 1) CR_HIP(hipMemsetAsync(arg.bar.bar, 0, BAR_WORDS * sizeof(unsigned), st));
  void* params[] = {&arg};
  const size_t dyn = pcg_dyn_lds(arg);
  if (arg.bar.coop || arg.bar.mode == 0)
    CR_HIP(hipLaunchCooperativeKernel(fn, dim3(nwg), dim3(arg.bs), params, dyn, st));
  else
    CR_HIP(hipLaunchKernel(fn, dim3(nwg), dim3(arg.bs), params, dyn, st));
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
// A_p(P) = lam (P Bx2 + 2 By1 P Bx1 + By2 P) + sum_a G_a (P h_a) h_a^T with
// h_a = H[:, a] (H(k, a) stored at H[a + k ninj]), all r x r column-major
// with leading dimension ldr.  One operator application is three phases
// separated by grid barriers:
//   A: T = P H (r x ninj) and Y2 = By1 P (and, before the loop, B = S H^T);
//   B: SG[:, a] = G_a T[:, a] for every injection (the Gram tensor, streamed
//      once; optionally from a BF16 copy);
//   C: Q = lam (P Bx2 + By2 P + 2 Y2 Bx1) + SG H^T, with the partial dot
//      products CG needs.
// The products of A and C are FP64 MFMA tiles (16 x 16 x 4): one output tile
// per task, the four waves of a workgroup taking interleaved k-steps and
// summing through LDS.  Phase C also sums <P,Q>, <R,Q>, <Q,Q> and <R,R> of
// the current vectors, so ||R - alpha Q||^2 = <R,R> - 2 alpha <R,Q> +
// alpha^2 <Q,Q> gives beta without a separate reduction, and the update
// Z += alpha P, R -= alpha Q, P = R + beta P is one elementwise phase: four
// grid barriers per iteration.  (<R,R> is summed afresh each step: carried
// over from the previous expansion, its rounding error would stay at
// eps ||R_0||^2 and swamp the later steps.)  Partial-sum slots (9 nwg
// doubles): 0 <P,Q>, 1 <R,Q>, 2 <Q,Q>, 3 <R,R>, 4 initial ||R||^2,
// 5 ||B||^2, 6 <Z,B>, 7 <Z,R>, 8 final ||R||^2.
namespace galk {

constexpr int NW = NT / WAVE;  // waves per workgroup
typedef double dbl4 __attribute__((ext_vector_type(4)));
// v_mfma_f64_16x16x4f64: lane l supplies A(row l % 16, k l / 16) and
// B(k l / 16, col l % 16); result element e of lane l is
// D(row l / 16 + 4 e, col l % 16).
__device__ __forceinline__ dbl4 mfma64(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Wave wv's share (k-steps wv, wv + 4, ...) of C(tile) += s A B over k < K.
// AROW: A(i, k) = A[i lda + k], else A[k lda + i]; BROW: B(k, j) = B[k ldb + j],
// else B[j ldb + k].  Tile rows i0 .. i0 + 16 NB - 1 (< m), columns j0 ..
// (< n); lane l supplies A(row l % 16, k l / 16) and B(k l / 16, col l % 16).
template <int NB, bool AROW, bool BROW>
__device__ __forceinline__ void tile_acc(dbl4 (&acc)[NB][NB], const double* __restrict__ A,
                                         int64_t lda, const double* __restrict__ B, int64_t ldb,
                                         int K, double s, int i0, int j0, int m, int n) {
  constexpr int UNR = 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int fr = lane & 15, fk = lane >> 4;
  const int nst = (K + 3) >> 2;
  bool aok[NB], bok[NB];
  int ia[NB], jb[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    ia[t] = i0 + 16 * t + fr;
    jb[t] = j0 + 16 * t + fr;
    aok[t] = ia[t] < m;
    bok[t] = jb[t] < n;
  }
  for (int st0 = wv; st0 < nst; st0 += NW * UNR) {
    double av[UNR][NB], bv[UNR][NB];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int k = 4 * (st0 + NW * u) + fk;
      const bool kok = k < K;
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        const int64_t ea = AROW ? (int64_t)ia[t] * lda + k : (int64_t)k * lda + ia[t];
        const int64_t eb = BROW ? (int64_t)k * ldb + jb[t] : (int64_t)jb[t] * ldb + k;
        av[u][t] = (kok && aok[t]) ? A[ea] * s : 0.0;
        bv[u][t] = (kok && bok[t]) ? B[eb] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = mfma64(av[u][a], bv[u][b], acc[a][b]);
  }
}

template <int NB>
__device__ __forceinline__ void acc_zero(dbl4 (&acc)[NB][NB]) {
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
}

// Sums the four waves' tiles through LDS and calls f(row, col, value) once per
// tile entry inside the m x n bounds (entries spread over the workgroup).
template <int NB, typename F>
__device__ __forceinline__ void tile_reduce(const dbl4 (&acc)[NB][NB], double* lds, int i0,
                                            int j0, int m, int n, F&& f) {
  constexpr int Q = NB * NB * 4;  // doubles per lane
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) lds[((wv * Q) + (a * NB + b) * 4 + e) * WAVE + lane] = acc[a][b][e];
  __syncthreads();
#pragma unroll
  for (int q0 = 0; q0 < Q * WAVE; q0 += NT) {
    const int idx = q0 + threadIdx.x;
    const int ln = idx & 63, q = idx >> 6;
    const int blk = q >> 2, e = q & 3;
    const int a = blk / NB, b = blk % NB;
    const int row = i0 + 16 * a + (ln >> 4) + 4 * e;
    const int col = j0 + 16 * b + (ln & 15);
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) v += lds[(w * Q + q) * WAVE + ln];
    if (row < m && col < n) f(row, col, v);
  }
  __syncthreads();
}

// Phase A.  INIT additionally forms B = S H^T into Bm.
template <int NB, bool INIT>
__device__ void phase_a(const GalerkinArgs& a, const double* Xm, double* lds) {
  constexpr int TS = 16 * NB;
  const int r = a.r, ld = a.ldr, ni = a.ninj;
  const int nt = (r + TS - 1) / TS, nti = (ni + TS - 1) / TS;
  const int ny2 = nt * nt, nT = nt * nti;
  const int ntask = ny2 + nT + (INIT ? ny2 : 0);
  for (int t = blockIdx.x; t < ntask; t += gridDim.x) {
    dbl4 acc[NB][NB];
    acc_zero(acc);
    if (t < ny2) {  // Y2 = By1 X
      const int i0 = (t % nt) * TS, j0 = (t / nt) * TS;
      tile_acc<NB, false, false>(acc, a.By1, ld, Xm, ld, r, 1.0, i0, j0, r, r);
      tile_reduce(acc, lds, i0, j0, r, r,
                  [&](int i, int j, double v) { a.Y2[(int64_t)j * ld + i] = v; });
    } else if (t < ny2 + nT) {  // T = X H
      const int u = t - ny2;
      const int i0 = (u % nt) * TS, j0 = (u / nt) * TS;
      tile_acc<NB, false, true>(acc, Xm, ld, a.H, ni, r, 1.0, i0, j0, r, ni);
      tile_reduce(acc, lds, i0, j0, r, ni,
                  [&](int i, int j, double v) { a.T[(int64_t)j * ld + i] = v; });
    } else {  // B = S H^T: S(i, c) = S[i ninj + c], H^T(c, j) = H[j ninj + c]
      const int u = t - ny2 - nT;
      const int i0 = (u % nt) * TS, j0 = (u / nt) * TS;
      tile_acc<NB, true, false>(acc, a.S, ni, a.H, ni, ni, 1.0, i0, j0, r, r);
      tile_reduce(acc, lds, i0, j0, r, r,
                  [&](int i, int j, double v) { a.Bm[(int64_t)j * ld + i] = v; });
    }
  }
}

// Phase B: SG[:, al] = G_al T[:, al].  FP64 Grams: task (injection, block of
// 128 rows), lane l owns rows l and l + 64, wave wv the k-steps wv, wv + 4, ...
// (so each load instruction reads 512 contiguous bytes of one Gram column).
// BF16 Grams (Gb, rows padded to ldh, block al at al r ldh): blocks of 256
// rows, lane l owns rows 4l .. 4l + 3 (one 8-byte load).
template <bool LOW>
__device__ void phase_b(const GalerkinArgs& a, double* lds) {
  const int r = a.r, ld = a.ldr;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int ROWS = LOW ? 256 : 128;
  constexpr int PER = ROWS / WAVE;
  const int nrb = (r + ROWS - 1) / ROWS;
  const int ntask = a.ninj * nrb;
  for (int t = blockIdx.x; t < ntask; t += gridDim.x) {
    const int al = t / nrb, rb = t % nrb;
    const int row0 = rb * ROWS;
    const double* tv = a.T + (int64_t)al * ld;
    double acc[PER];
#pragma unroll
    for (int p = 0; p < PER; ++p) acc[p] = 0.0;
    if constexpr (LOW) {
      const int ldh = a.ldh;
      const int rowq = row0 + 4 * lane;  // < ldh when row0 + 4 lane < r (ldh >= r, ldh % 4 == 0)
      const bool ok = rowq < r;
      const __bf16* g = a.Gb + (int64_t)al * r * ldh + rowq;
      constexpr int UNR = 8;
      for (int k0 = wv; k0 < r; k0 += NW * UNR) {
        uint2 w[UNR];
        double tk[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int k = k0 + NW * u;
          const bool kk = k < r;
          w[u] = (kk && ok) ? *reinterpret_cast<const uint2*>(g + (int64_t)k * ldh) : uint2{0u, 0u};
          tk[u] = kk ? tv[k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          // a BF16 value is the high half of the FP32 with the same bits
          acc[0] += (double)__uint_as_float(w[u].x << 16) * tk[u];
          acc[1] += (double)__uint_as_float(w[u].x & 0xffff0000u) * tk[u];
          acc[2] += (double)__uint_as_float(w[u].y << 16) * tk[u];
          acc[3] += (double)__uint_as_float(w[u].y & 0xffff0000u) * tk[u];
        }
      }
    } else {
      const double* g = a.G + (int64_t)al * ld * ld;
      bool ok[PER];
#pragma unroll
      for (int p = 0; p < PER; ++p) ok[p] = row0 + lane + WAVE * p < r;
      constexpr int UNR = 8;
      for (int k0 = wv; k0 < r; k0 += NW * UNR) {
        double gv[UNR][PER], tk[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const int k = k0 + NW * u;
          const bool kk = k < r;
          tk[u] = kk ? tv[k] : 0.0;
#pragma unroll
          for (int p = 0; p < PER; ++p)
            gv[u][p] = (kk && ok[p]) ? g[(int64_t)k * ld + row0 + lane + WAVE * p] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
          for (int p = 0; p < PER; ++p) acc[p] += gv[u][p] * tk[u];
      }
    }
    // sum the four waves (row index = the lane's rows)
#pragma unroll
    for (int p = 0; p < PER; ++p) lds[(wv * PER + p) * WAVE + lane] = acc[p];
    __syncthreads();
    for (int q = threadIdx.x; q < ROWS; q += NT) {
      // q enumerates (p, lane) as stored: row of entry (p, ln)
      const int p = q / WAVE, ln = q % WAVE;
      const int row = LOW ? row0 + 4 * ln + p : row0 + ln + WAVE * p;
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) v += lds[(w * PER + p) * WAVE + ln];
      if (row < r) a.SG[(int64_t)al * ld + row] = v;
    }
    __syncthreads();
  }
}

// Phase C: Q tiles.  INIT: R = B - Q, P = R, partial ||R||^2 and ||B||^2
// (slots 4, 5); else Q stored with partial <P,Q>, <R,Q>, <Q,Q>, <R,R>
// (slots 0-3).
template <int NB, bool INIT>
__device__ void phase_c(const GalerkinArgs& a, const double* Xm, double* lds, double* red) {
  constexpr int TS = 16 * NB;
  const int r = a.r, ld = a.ldr, ni = a.ninj;
  const int nt = (r + TS - 1) / TS;
  const double lam = a.lam;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int t = blockIdx.x; t < nt * nt; t += gridDim.x) {
    const int i0 = (t % nt) * TS, j0 = (t / nt) * TS;
    dbl4 acc[NB][NB];
    acc_zero(acc);
    tile_acc<NB, false, false>(acc, Xm, ld, a.Bx2, ld, r, lam, i0, j0, r, r);
    tile_acc<NB, false, false>(acc, a.By2, ld, Xm, ld, r, lam, i0, j0, r, r);
    tile_acc<NB, false, false>(acc, a.Y2, ld, a.Bx1, ld, r, 2.0 * lam, i0, j0, r, r);
    // SG H^T: SG(i, c) = SG[c ld + i], H^T(c, j) = H[j ninj + c]
    tile_acc<NB, false, false>(acc, a.SG, ld, a.H, ni, ni, 1.0, i0, j0, r, r);
    tile_reduce(acc, lds, i0, j0, r, r, [&](int i, int j, double q) {
      const int64_t e = (int64_t)j * ld + i;
      if (INIT) {
        const double b = a.Bm[e];
        const double rv = b - q;
        a.R[e] = rv;
        a.P[e] = rv;
        s0 += rv * rv;
        s1 += b * b;
      } else {
        const double rv = a.R[e];
        a.Q[e] = q;
        s0 += a.P[e] * q;
        s1 += rv * q;
        s2 += q * q;
        s3 += rv * rv;
      }
    });
  }
  const int nwg = gridDim.x;
  if (INIT) {
    block_sum2(s0, s1, red);
    if (threadIdx.x == 0) {
      a.part[4 * nwg + blockIdx.x] = s0;
      a.part[5 * nwg + blockIdx.x] = s1;
    }
  } else {
    block_sum2(s0, s1, red);
    block_sum2(s2, s3, red + 2 * NW);
    if (threadIdx.x == 0) {
      a.part[0 * nwg + blockIdx.x] = s0;
      a.part[1 * nwg + blockIdx.x] = s1;
      a.part[2 * nwg + blockIdx.x] = s2;
      a.part[3 * nwg + blockIdx.x] = s3;
    }
  }
}

// Q = A_p(X) in three phases (INIT: from X = Z, also B and R = B - Q).
template <int NB, bool INIT>
__device__ __forceinline__ void apply(const GalerkinArgs& a, const double* Xm, bool low,
                                      double* lds, double* red, cgrp::grid_group& grid) {
  phase_a<NB, INIT>(a, Xm, lds);
  grid_barrier(a.bar, grid);
  if (low)
    phase_b<true>(a, lds);
  else
    phase_b<false>(a, lds);
  grid_barrier(a.bar, grid);
  phase_c<NB, INIT>(a, Xm, lds, red);
  grid_barrier(a.bar, grid);
}

}  // namespace galk

template <int NB>
__global__ __launch_bounds__(NT) void k_galerkin(GalerkinArgs a) {
  using namespace galk;
  cgrp::grid_group grid = cgrp::this_grid();
  __shared__ double lds[NW * NB * NB * 4 * WAVE > NW * 4 * WAVE ? NW * NB * NB * 4 * WAVE
                                                               : NW * 4 * WAVE];
  __shared__ double red[4 * NW];
  const int r = a.r, ld = a.ldr, nwg = gridDim.x;
  const int64_t nel = (int64_t)r * r;
  const int64_t gtid = (int64_t)blockIdx.x * NT + threadIdx.x, gstride = (int64_t)nwg * NT;
  double* part = a.part;

  // ---- B = S H^T, R = B - A_p(Z) with the FP64 Grams, P = R
  apply<NB, true>(a, a.Z, false, lds, red, grid);
  double rr, bb;
  grid_total2<NT, false>(part, 4, 5, nwg, red, rr, bb);
  const double rr0 = rr;
  const double tol2 = fmax(a.rtol * a.rtol * bb, a.inner_rel * a.inner_rel * rr0);
  const bool low = a.Gb != nullptr;
  int it = 0, status = 0;
  for (; it < a.maxit && rr > tol2; ++it) {
    apply<NB, false>(a, a.P, low, lds, red, grid);
    double pq, rq, qq;
    grid_total2<NT, false>(part, 0, 1, nwg, red, pq, rq);
    grid_total2(part, 2, 3, nwg, red, qq, rr);
    if (!(pq > 0.0)) {
      status = 2;
      break;
    }
    const double alpha = rr / pq;
    const double rr_new = fmax(rr - 2.0 * alpha * rq + alpha * alpha * qq, 0.0);
    const double beta = rr_new / rr;
    for (int64_t q = gtid; q < nel; q += gstride) {
      const int64_t e = (q / r) * ld + q % r;
      const double p = a.P[e];
      a.Z[e] += alpha * p;
      const double rv = a.R[e] - alpha * a.Q[e];
      a.R[e] = rv;
      a.P[e] = rv + beta * p;
    }
    rr = rr_new;
    grid_barrier(a.bar, grid);
  }
  if (status == 0 && rr > tol2) status = 1;
  // energy pieces <Z,B>, <Z,R> and the final ||R||^2 (slots 6-8)
  double zb = 0.0, zr = 0.0, rf = 0.0;
  for (int64_t q = gtid; q < nel; q += gstride) {
    const int64_t e = (q / r) * ld + q % r;
    const double z = a.Z[e], rv = a.R[e];
    zb += z * a.Bm[e];
    zr += z * rv;
    rf += rv * rv;
  }
  block_sum2(zb, zr, red);
  rf = block_sum(rf, red + 2 * NW);
  if (threadIdx.x == 0) {
    part[6 * nwg + blockIdx.x] = zb;
    part[7 * nwg + blockIdx.x] = zr;
    part[8 * nwg + blockIdx.x] = rf;
  }
  grid_barrier(a.bar, grid);
  if (blockIdx.x == 0) {
    grid_total2<NT, false>(part, 6, 7, nwg, red, zb, zr);
    rf = grid_total(part, 8, nwg, red);
    if (threadIdx.x == 0) {
      a.scal[0] = (double)it;
      a.scal[1] = bb > 0.0 ? sqrt(rf / bb) : 0.0;
      const bool timed_out =
          a.bar.mode == 1 &&
          __hip_atomic_load(a.bar.bar + BAR_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
      a.scal[2] = timed_out ? PERSIST_TIMEOUT : (double)status;
      a.scal[3] = -0.5 * zb - 0.5 * zr;  // 1/2 <Z, A_p Z> - <Z, B> with A_p Z = B - R
      a.scal[4] = bb > 0.0 ? sqrt(rr0 / bb) : 0.0;
    }
  }
}

// Output tiles of 32 x 32 once there are enough of them to give every
// workgroup one; 16 x 16 below.
static int gal_nb(int r, int nwg) {
  const int nt32 = (r + 31) / 32;
  return nt32 * nt32 >= nwg ? 2 : 1;
}

int galerkin_max_wg(int r) {
  int dev = 0, ncu = 0, p1 = 0, p2 = 0;
  (void)r;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&p1, (void*)k_galerkin<1>, NT, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&p2, (void*)k_galerkin<2>, NT, 0) != hipSuccess)
    return 0;
  return std::min(p1, p2) * ncu;
}

__global__ __launch_bounds__(NT) void k_gram_bf16(int r, int ld, int ldh, int ninj,
                                                  const double* __restrict__ G,
                                                  __bf16* __restrict__ Gb) {
  const int64_t n = (int64_t)ninj * r * ldh;
  for (int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x; q < n; q += (int64_t)gridDim.x * NT) {
    const int row = (int)(q % ldh);
    const int64_t ak = q / ldh;  // al r + k
    const int k = (int)(ak % r), al = (int)(ak / r);
    const double v = row < r ? G[((int64_t)al * ld + k) * ld + row] : 0.0;
    Gb[q] = (__bf16)(float)v;
  }
}

cr_status gram_to_bf16(int r, int ld, int ldh, int ninj, const double* G, __bf16* Gb,
                       hipStream_t st) {
  const int64_t n = (int64_t)ninj * r * ldh;
  if (n == 0) return CR_OK;
  const unsigned nb = (unsigned)std::min<int64_t>((n + NT - 1) / NT, 8192);
  hipLaunchKernelGGL(k_gram_bf16, dim3(nb), dim3(NT), 0, st, r, ld, ldh, ninj, G, Gb);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

cr_status galerkin_cg(const GalerkinArgs& a, int nwg, int nb, hipStream_t st) {
  if (a.r <= 0) return CR_OK;
  GalerkinArgs arg = a;
  if (arg.bar.mode == 1) CR_HIP(hipMemsetAsync(arg.bar.bar, 0, BAR_WORDS * sizeof(unsigned), st));
  void* params[] = {&arg};
  if (nb != 1 && nb != 2) nb = gal_nb(a.r, nwg);
  const void* fn = nb == 2 ? (const void*)k_galerkin<2> : (const void*)k_galerkin<1>;
  if (!arg.bar.coop && arg.bar.mode == 1)
    CR_HIP(hipLaunchKernel(fn, dim3(nwg), dim3(NT), params, 0, st));
  else
    CR_HIP(hipLaunchCooperativeKernel(fn, dim3(nwg), dim3(NT), params, 0, st));
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
