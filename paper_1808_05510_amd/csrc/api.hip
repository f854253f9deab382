// libconnreg host side: problem handle, workspace, the C ABI entry points and
// the greedy driver (Algorithm 1 of the paper) on top of the kernels in
// k_blas.hip and k_cg.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "cr_internal.hpp"

namespace cr {
static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }
}  // namespace cr

using namespace cr;

// ===================================================================== handle
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

static bool poison_workspace() {
  static const bool v = [] {
    const char* e = std::getenv("CONNREG_POISON");
    return e && std::atoi(e) != 0;
  }();
  return v;
}

// Two-level preconditioner of the v-systems (cr_problem_set_coarse): the
// aggregate packing for 256- and 512-thread workgroups and the coarse
// operator's geometry (C1 = P^T L_x P, C2 = P^T L_x^2 P) and data (Y = P^T X).
struct CoarsePack {
  int bs = 0, nwg = 0;
  int32_t *slot_vox = nullptr, *slot_agg = nullptr, *wg_agg = nullptr;
  int32_t *agg_lo = nullptr, *agg_hi = nullptr;
  double* slot_w = nullptr;
};
struct CoarseLevel {
  bool valid = false;
  int m = 0, block = 0;
  CoarsePack pack[2];  // 256- and 512-thread workgroups
  double *C1 = nullptr, *C2 = nullptr, *Y = nullptr;
};

struct cr_problem {
  int dev = -1;               // device the handle was created on
  hipStream_t st = nullptr;
  hipStream_t aux = nullptr;  // library-owned second stream (default priority) for fork/join
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool op_fork = true;  // op_apply's data term on the auxiliary stream (CONNREG_OP_FORK=0: serial)
  // op_apply in fused ring-2 window sweeps where the geometry has the tables
  // (CONNREG_OP_FUSED: 0 off, 1 FP64 only, 2 FP64 and FP32).  Off by default:
  // on the cortex shells at r = 100 the fused call measured 912 against
  // 770 us (FP64) and 703 against 500 us (FP32); its window loop is latency
  // bound at two workgroups per CU, and each ring-2 window is 11 times its tile
  int op_fused = 0;
  cr_precision prec = CR_PREC_FP64;
  int64_t ny = 0, nx = 0;
  int ninj = 0;
  double lam = 0.0;
  Geom gy, gx;
  double* X64 = nullptr;
  double* OY64 = nullptr;
  float* X32 = nullptr;
  float* OY32 = nullptr;
  uint32_t* bits = nullptr;
  int32_t* hptr = nullptr;
  int32_t* hidx = nullptr;
  int64_t nholes = 0;
  bool use_holes = false;
  double dnorm = 0.0;
  double half_oy2 = 0.0;      // 1/2 ||Omega o Y||_F^2 (J = energy + this)
  int resid_qr = 1;           // residual norm from CholQR2 factors: 0 never, 1 below
                              // RESID_QR_SWITCH (Gram form above), 2 always
                              // (CONNREG_RESID_QR)
  double* hscal = nullptr;  // pinned host scratch
  unsigned* bar = nullptr;  // grid-barrier words (BAR_WORDS)
  cr_pc* pc = nullptr;      // learned preconditioner for the u-systems (not owned)
  int fcg_mode = 0;         // u-systems: 0 Jacobi-PCG, 1 FCG + base step, 2 FCG + base step + network
  BoxBasis boxy;            // spectral basis of the target grid when it is a full box
  BoxBasis boxx;            // spectral basis of the source grid when it is a full box
  CoarseLevel cv;           // two-level preconditioner of the v-systems
  bool kr_omega_ready = false;
  bool smw_xh_ready = false;    // workspace "smw_Xh" holds Q^T X of the source box  // workspace "kraux" holds the BF16 copy of Omega
  int64_t pc_fallbacks = 0;
  int cu_share = 0;         // > 0: persistent grids limited to this many CUs' worth of slots
  int coop = 1;             // persistent kernels launched cooperatively
  int tuned_vpt_u = 0, tuned_vpt_v = 0;  // autotuned PCG voxels per thread (0 = heuristic)
  // threads per PCG workgroup: 1024 (a quarter of the workgroups, so a quarter
  // of the arrivals at every grid barrier; measured 5% faster FP64 and 16%
  // faster mixed solves on the 40^3 / 30^3 problem than 256); CONNREG_PCG_BS=256
  // restores 256.  Batched solves use 256 (their CU shares are sized for it).
  int pcg_bs = 1024;
  int pcg_xbs = 0;           // v-system group size with register-resident X (0: 256;
                             // CONNREG_PCG_XBS=256 or 512)
  bool no_xreg = false;     // CONNREG_PCG_XREG=0: v-system PCG streams X (no register-resident rows)
  bool pcg_xlds = true;     // rows of X beyond the register rows held in LDS (CONNREG_PCG_XLDS=0: streamed)
  int pcg_xlds_f32 = 1;     // FP32 data: 64 register rows and an LDS tail where 128 register
                            // rows would need 512-thread groups (CONNREG_PCG_XLDS_F32=0: off,
                            // 2: also where they fit 256-thread groups)
  bool batch_xreg = true;   // batches keep the register form of the v-system PCG
                            // (CONNREG_BATCH_XREG=0: any form that fits a share)
  bool pcg_warm = true;     // FP64 ALS half-steps warm-started (CONNREG_PCG_WARM=0: from zero)
  int bar_mode = 1;
  unsigned bar_spin = 1u << 22;  // grid-barrier poll bound (CONNREG_BAR_SPIN, for tests)
  int gal_low = -1;  // projected CG on BF16 Grams with FP64 correction steps: -1 for mixed
                     // problems, 0 never, 1 always (CONNREG_GAL_LOW)
  int gal_tile = 0;  // projected CG output tiles: 0 by size, 16 or 32 (CONNREG_GAL_TILE)
  std::map<std::string, DevBuf> ws;
  std::vector<void*> owned;

  template <typename T>
  T* buf(const std::string& name, int64_t count) {
    size_t need = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    DevBuf& b = ws[name];
    if (b.bytes >= need) return (T*)b.p;
    if (b.p) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(b.p);
      b.p = nullptr;
      b.bytes = 0;
    }
    if (hipMalloc(&b.p, need) != hipSuccess) {
      b.p = nullptr;
      set_error("device allocation of workspace '" + name + "' (" + std::to_string(need) +
                " bytes) failed");
      return nullptr;
    }
    b.bytes = need;
    // CONNREG_POISON=1: fill new workspace with NaN bytes, so that a read of
    // workspace the library never wrote shows up in results (checking aid)
    if (poison_workspace()) (void)hipMemsetAsync(b.p, 0xFF, need, st);
    return (T*)b.p;
  }
  template <typename T>
  const T* X() const;
  template <typename T>
  const T* OY() const;
};
template <>
const double* cr_problem::X<double>() const { return X64; }
template <>
const float* cr_problem::X<float>() const { return X32; }
template <>
const double* cr_problem::OY<double>() const { return OY64; }
template <>
const float* cr_problem::OY<float>() const { return OY32; }

#define WS(T, name, count)                                   \
  ({                                                         \
    T* p_ = P->buf<T>(name, (count));                        \
    if (!p_) return CR_ENOMEM;                               \
    p_;                                                      \
  })

// the residual norm switches from the Gram form to CholQR2 factors below
// this relative residual; CholQR2 needs factor widths k = n_inj + 3r <= KMAX
constexpr double RESID_QR_SWITCH = 1e-6;
constexpr int RESID_QR_KMAX = 1024;
constexpr int PCG_U_VPT2_WG = 96;
// with neither factor (both have more columns than rows, or dependent ones)
// the residual's entries are formed when n_y n_x k is at most this
constexpr double RESID_DENSE_MAX = 2e11;

static int64_t gemm_part_cap(const cr_problem* P) {
  (void)P;
  return (int64_t)1 << 24;  // doubles (128 MB) of split-K partials
}

// ===================================================================== small kernels
// coef for the factored residual products (see apply_R / apply_RT): one wave
// per coefficient, its lanes splitting the r-long dot product with Z
__global__ __launch_bounds__(256) void k_rcoef(int ninj, int r, const double* __restrict__ y0,
                                               const double* __restrict__ Z, int64_t ldz,
                                               int trans, double lam,
                                               double* __restrict__ coef) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t < ninj) {
    if (lane == 0) coef[t] = y0[t];
    return;
  }
  const int e = t - ninj;
  if (e >= 3 * r) return;
  const int blk = e / r, i = e % r;
  // R   : coef blocks [-lam Z q3 | -2lam Z q2 | -lam Z q1] over [U | LU | L2U],
  //       q = y0 blocks [V^T v | LV^T v | L2V^T v]  -> source block 2,1,0
  // R^T : coef blocks [-lam Z^T e1 | -2lam Z^T e2 | -lam Z^T e3] over [L2V | LV | V],
  //       e = y0 blocks [U^T u | LU^T u | L2U^T u] -> source block 0,1,2
  const int src = trans ? blk : 2 - blk;
  const double sc = (blk == 1 ? -2.0 : -1.0) * lam;
  const double* q = y0 + ninj + (int64_t)src * r;
  double s = 0.0;
  if (trans)
    for (int k = lane; k < r; k += 64) s += Z[(int64_t)i * ldz + k] * q[k];
  else
    for (int k = lane; k < r; k += 64) s += Z[(int64_t)k * ldz + i] * q[k];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) coef[t] = sc * s;
}

__global__ void k_set2(double* dst, const double* s0, double f0, const double* s1, double f1) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dst[0] = f0 * s0[0];
    dst[1] = f1 * s1[0];
  }
}

// mirror column j of a symmetric matrix into row j
__global__ void k_mirror(double* B, int64_t ld, int j) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k <= j) B[(int64_t)k * ld + j] = B[(int64_t)j * ld + k];
}

// G[a](k, j) = G[a](j, k) = C[k + a*ldc] for k <= j
__global__ void k_scatter_gram(int ninj, int j, const double* __restrict__ C, int64_t ldc,
                               double* __restrict__ G, int64_t ldr) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)ninj * (j + 1)) return;
  const int a = (int)(e / (j + 1)), k = (int)(e % (j + 1));
  const double v = C[(int64_t)a * ldc + k];
  double* Ga = G + (int64_t)a * ldr * ldr;
  Ga[(int64_t)j * ldr + k] = v;
  Ga[(int64_t)k * ldr + j] = v;
}

// C[k + a*ldc] = c0[k] for all a (k < m)
__global__ void k_bcast_cols(int m, int ninj, const double* __restrict__ c0, double* C,
                             int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * ninj) return;
  C[(e / m) * ldc + e % m] = c0[e % m];
}

// Cm = blockdiag(I_ninj, s1 Z^T, s2 Z^T, s3 Z^T), k x k
__global__ void k_build_cm(int ninj, int r, const double* __restrict__ Z, int64_t ldz, double lam,
                           double* __restrict__ Cm) {
  const int k = ninj + 3 * r;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)k * k) return;
  const int i = (int)(e % k), j = (int)(e / k);
  double v = 0.0;
  if (i < ninj || j < ninj) {
    v = (i == j) ? 1.0 : 0.0;
  } else {
    const int bi = (i - ninj) / r, bj = (j - ninj) / r;
    if (bi == bj) {
      const int ii = (i - ninj) % r, jj = (j - ninj) % r;
      const double s = (bi == 1 ? -2.0 : -1.0) * lam;
      v = s * Z[(int64_t)ii * ldz + jj];  // (Z^T)(ii, jj) = Z(jj, ii)
    }
  }
  Cm[e] = v;
}

// out = {||Z - Zold||_F^2, ||Z||_F^2} over the leading r x r block (ld ldr)
// ||Z - Zold||_F^2 and ||Z||_F^2 over the r x r core: per-workgroup partials
// (part[2 b], part[2 b + 1]), then k_dw_final sums them in a fixed order
constexpr int DW_MAXWG = 256;
__global__ __launch_bounds__(256) void k_dw(int r, int64_t ldr, const double* __restrict__ Z,
                                            const double* __restrict__ Zold,
                                            double* __restrict__ part) {
  __shared__ double red[2][4];
  double dd = 0.0, zz = 0.0;
  const int64_t n = (int64_t)r * r;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e % r, j = e / r;
    const double a = Z[j * ldr + i], b = Zold[j * ldr + i];
    dd += (a - b) * (a - b);
    zz += a * a;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    dd += __shfl_xor(dd, o, 64);
    zz += __shfl_xor(zz, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = dd;
    red[1][threadIdx.x >> 6] = zz;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    part[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

__global__ __launch_bounds__(64) void k_dw_final(int nb, const double* __restrict__ part,
                                                 double* __restrict__ out) {
  double dd = 0.0, zz = 0.0;
  for (int b = threadIdx.x; b < nb; b += 64) {
    dd += part[2 * b];
    zz += part[2 * b + 1];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    dd += __shfl_xor(dd, o, 64);
    zz += __shfl_xor(zz, o, 64);
  }
  if (threadIdx.x == 0) {
    out[0] = dd;
    out[1] = zz;
  }
}

__global__ void k_neg(int n, const double* __restrict__ a, double* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = -a[i];
}

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

static int device_cus() {
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return ncu;
}

// workgroups of a kernel whose whole-device resident capacity is maxwg that
// fit in `share` CUs
static int share_cap(int maxwg, int share) {
  const int ncu = std::max(1, device_cus());
  return std::max(1, (int)((int64_t)maxwg * share / ncu));
}

// q = lam*(L t + c1 t + c0 p) + d o p with t = L p (runtime stencil width)
__global__ void k_uapply(int64_t n, int K, const int32_t* __restrict__ nbr, double lam,
                         const double* __restrict__ coef, const double* __restrict__ d,
                         const double* __restrict__ p, const double* __restrict__ t,
                         double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double lt = (double)K * t[i];
  for (int k = 0; k < K; ++k) lt -= t[nbr[(int64_t)k * n + i]];
  q[i] = lam * (lt + coef[0] * t[i] + coef[1] * p[i]) + d[i] * p[i];
}
// p = z + beta * pp
__global__ void k_axpby(int64_t n, const double* __restrict__ z, double beta,
                        const double* __restrict__ pp, double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = z[i] + beta * pp[i];
}
// x += t
__global__ void k_add_to(int64_t n, const double* __restrict__ t, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += t[i];
}
// x += alpha p ; r -= alpha q
__global__ void k_xr_update(int64_t n, double alpha, const double* __restrict__ p,
                            const double* __restrict__ q, double* __restrict__ x,
                            double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] += alpha * p[i];
  r[i] -= alpha * q[i];
}
// z = minv o r
__global__ void k_jacobi(int64_t n, const double* __restrict__ minv, const double* __restrict__ r,
                         double* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = minv[i] * r[i];
}

// ===================================================================== solver context
// ----------------------------------------------------------- device-scalar FCG
// Scalars of the flexible CG live in device memory, so an iteration is a
// fixed launch sequence with no host synchronisation:
//   S[0] b.b   S[1] r.r   S[2] p.q of the previous step   S[5] alpha   S[6] beta
//   S[7] state (0 running, 1 converged, 2 breakdown)   S[8] iterations
//   S[10] 1 when the base step replaces the network output   S[11] fallbacks
//   S[12] w.w   S[13] mean of d   S[16..19] [r.z, qq.z, r.w, qq.w]   S[20..21] [q.p, r.p]
enum { FS_BB = 0, FS_RR = 1, FS_PQP = 2, FS_ALPHA = 5, FS_BETA = 6, FS_STATE = 7, FS_IT = 8,
       FS_USEW = 10, FS_FB = 11, FS_WW = 12, FS_DBAR = 13, FS_DZ = 16, FS_DP = 20, FS_N = 24 };

__global__ void k_fcg_beta(double* S, int first, int net) {
  if (S[FS_STATE] != 0.0) return;
  double zr = S[FS_DZ + 0], zq = S[FS_DZ + 1];
  const bool ok = net == 0 || (zr > 0.0 && isfinite(zr) && (first || isfinite(zq)));
  if (!ok) {  // the network output is not a descent direction: use the base step
    zr = S[FS_DZ + 2];
    zq = S[FS_DZ + 3];
    S[FS_FB] += 1.0;
  }
  S[FS_USEW] = (net == 0 || !ok) ? 1.0 : 0.0;
  S[FS_BETA] = first ? 0.0 : -zq / S[FS_PQP];
}

__global__ void k_fcg_dir(int64_t n, const double* __restrict__ z, const double* __restrict__ w,
                          const double* __restrict__ S, const double* __restrict__ pp,
                          double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || S[FS_STATE] != 0.0) return;
  const double beta = S[FS_BETA];
  const double zi = S[FS_USEW] != 0.0 ? w[i] : z[i];
  p[i] = beta != 0.0 ? zi + beta * pp[i] : zi;
}

__global__ void k_fcg_alpha(double* S) {
  if (S[FS_STATE] != 0.0) {
    S[FS_ALPHA] = 0.0;
    return;
  }
  const double pq = S[FS_DP + 0], pr = S[FS_DP + 1];
  if (!(pq > 0.0) || !isfinite(pr)) {
    S[FS_STATE] = 2.0;
    S[FS_ALPHA] = 0.0;
    return;
  }
  S[FS_ALPHA] = pr / pq;
  S[FS_PQP] = pq;
}

__global__ void k_fcg_update(int64_t n, const double* __restrict__ S, const double* __restrict__ p,
                             const double* __restrict__ q, double* __restrict__ x,
                             double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double a = S[FS_ALPHA];
  if (i >= n || a == 0.0) return;
  x[i] += a * p[i];
  r[i] -= a * q[i];
}

// a zero or non-finite right-hand side ends the flexible CG as a breakdown
// (every later scalar kernel of the iteration is then a no-op)
__global__ void k_fcg_init(double* S) {
  if (!(S[FS_BB] > 0.0)) S[FS_STATE] = 2.0;
}

__global__ void k_fcg_check(double* S, double tol2) {
  if (S[FS_STATE] != 0.0) return;
  S[FS_IT] += 1.0;
  if (S[FS_RR] <= tol2 * S[FS_BB]) S[FS_STATE] = 1.0;
}

__global__ void k_scale1(double* x, double s) { x[0] *= s; }

__global__ void k_fill(int64_t n, double v, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

template <typename T>
struct Ctx {
  cr_problem* P;
  hipStream_t st;
  int64_t ny, nx;
  int ninj;
  double lam;
  int rmax;  // capacity of the rank dimension (leading dimension of Grams)
  // current iterate (bases in T, core in double)
  T* U = nullptr;
  int64_t ldu = 0;
  T* V = nullptr;
  int64_t ldv = 0;
  T *LU = nullptr, *L2U = nullptr, *LV = nullptr, *L2V = nullptr;
  double* Z = nullptr;
  int64_t ldz = 0;
  T* N = nullptr;
  double *Ht = nullptr, *St = nullptr, *G = nullptr;
  double *By1 = nullptr, *By2 = nullptr, *Bx1 = nullptr, *Bx2 = nullptr;
  double* Tm = nullptr;
  // vectors
  T *vu = nullptr, *vv = nullptr, *rhs_u = nullptr, *rhs_v = nullptr, *dvec = nullptr;
  T *minv_u = nullptr, *minv_v = nullptr, *Lv = nullptr, *Lu = nullptr;
  T* pw_u[6];
  T* pw_v[6];
  double *y0 = nullptr, *coef = nullptr, *cu = nullptr, *cv = nullptr, *gw = nullptr;
  double *sc = nullptr, *part = nullptr, *pcgpart = nullptr, *sbuf = nullptr, *gpart = nullptr;
  double* tmp = nullptr;
  int pcg_vpt_u = 1, pcg_vpt_v = 1, pcg_nwg_u = 1, pcg_nwg_v = 1, pcg_bs = NT;
  int64_t pcgpart_size = 0;
  int pcg_xtail_v = 0;  // v-system: register rows plus a tail of X (1 streamed, 2 LDS first)
  int pcg_xlds_v = 0;   // v-system tail rows held in LDS (pcg_xtail_v 2)
  int pcg_bs_v = NT, pcg_nxr_v = 0;  // v-system: X rows in registers when n_inj <= PCG_NXR
  // stats of the last ALS
  int it_u = 0, it_v = 0, notconv = 0;

  explicit Ctx(cr_problem* p)
      : P(p), st(p->st), ny(p->ny), nx(p->nx), ninj(p->ninj), lam(p->lam), rmax(0) {}

  const T* X() const { return P->X<T>(); }
  const T* OY() const { return P->OY<T>(); }

  // ------------------------------------------------------------ allocation
  cr_status alloc_vectors(int vpt_opt) {
    const int64_t nmax = std::max(ny, nx);
    vu = WS(T, "vu", ny);
    vv = WS(T, "vv", nx);
    rhs_u = WS(T, "rhs_u", ny);
    rhs_v = WS(T, "rhs_v", nx);
    dvec = WS(T, "dvec", ny);
    minv_u = WS(T, "minv_u", ny);
    minv_v = WS(T, "minv_v", nx);
    Lv = WS(T, "Lv", nx);
    Lu = WS(T, "Lu", ny);
    T* pw = WS(T, "pcgwork", 6 * nmax);
    for (int k = 0; k < 6; ++k) {
      pw_u[k] = pw + k * nmax;
      pw_v[k] = pw + k * nmax;
    }
    const int kmax = ninj + 3 * std::max(rmax, 1) + 8;
    y0 = WS(double, "y0", kmax);
    coef = WS(double, "coef", kmax);
    cu = WS(double, "cu", 4);
    cv = WS(double, "cv", 4);
    gw = WS(double, "gw", ninj);
    sc = WS(double, "sc", 32);
    tmp = WS(double, "tmp", 16);
    sbuf = WS(double, "sbuf", ninj);
    const int64_t pt = std::max(gemv_t_part_size(nmax, kmax), gemv_t_part_size(nmax, 1));
    part = WS(double, "part", pt);
    // PCG grid sizes: the fewest voxels per thread (1, 2, 4, 8) whose grid
    // fits co-resident on the device and stays at or below 512 workgroups.
    // Measured on the 40^3 / 30^3 problem: one voxel per thread beats more
    // voxels per thread, whose per-phase latency grows faster than the grid
    // barrier (3 us at 64, 8 us at 256 groups) shrinks; wider workgroups
    // (pcg_bs) cut the group count without adding work per thread.
    // u-systems without the two-barrier form (no rows of L^2 for it) whose
    // one-voxel grid exceeds PCG_U_VPT2_WG workgroups take two voxels per
    // thread, halving the arrivals at the grid barrier (1024-thread groups,
    // three barriers: the cortex shells 5.77 -> 5.55 s and the flatmap-sized
    // map 11.86 -> 11.35 s, both FP64).  The two-barrier form holds one voxel
    // per thread and beats both on the shells (FP64 5.38 s, mixed 2.45
    // against 2.80 s).
    pcg_bs = P->cu_share > 0 ? NT : P->pcg_bs;
    auto pick = [&](const Geom& g, const T* Xm, int& vpt, int& nwg) -> bool {
      const int tuned = Xm ? P->tuned_vpt_v : P->tuned_vpt_u;
      int want = vpt_opt > 0 ? vpt_opt : tuned;
      if (want <= 0 && !Xm && P->cu_share <= 0 && !g.r2idx &&
          (g.n + (int64_t)pcg_bs - 1) / pcg_bs > PCG_U_VPT2_WG)
        want = 2;
      for (int v = 1; v <= 8; v *= 2) {
        if (want > 0 && v < want) continue;
        PcgArgs<T> probe{};
        probe.g = g;
        probe.Xm = Xm;
        probe.vpt = v;
        const int bs = Xm ? pcg_bs_v : pcg_bs;
        probe.bs = bs;
        int maxwg = pcg_max_wg<T>(probe);
        if (P->cu_share > 0) maxwg = share_cap(maxwg, P->cu_share);
        const int64_t w = std::max<int64_t>(1, (g.n + (int64_t)bs * v - 1) / ((int64_t)bs * v));
        if (maxwg > 0 && w <= maxwg && (w <= 512 || want > 0 || v == 8)) {
          vpt = v;
          nwg = (int)w;
          return true;
        }
      }
      return false;
    };
    if (vpt_opt != 0 && vpt_opt != 1 && vpt_opt != 2 && vpt_opt != 4 && vpt_opt != 8) {
      set_error("pcg_vpt must be 0 (auto), 1, 2, 4 or 8");
      return CR_EINVAL;
    }
    // v-system: X rows in registers (256-thread groups, one voxel per thread)
    // when n_inj fits and the grid fits, else the general kernel with the
    // default group size (measured on the shells: 256-thread groups there cost
    // more in barrier arrivals than the 1024-thread kernel's register spills)
    pcg_bs_v = pcg_bs;
    pcg_nxr_v = 0;
    pcg_xtail_v = 0;
    pcg_xlds_v = 0;
    {
      const int tuned = P->tuned_vpt_v;
      const int want = vpt_opt > 0 ? vpt_opt : tuned;
      // rows of X in registers: 64 for either type, 128 for FP32 data
      const int nxr_sel = ninj <= PCG_NXR ? PCG_NXR
                          : (std::is_same<T, float>::value && ninj <= PCG_NXR2) ? PCG_NXR2 : 0;
      // FP32 data with more than 64 injections: when 128 register rows need
      // 512-thread groups (their 256-thread form does not fit one group per
      // CU), 64 rows in registers and the rest in LDS instead (below)
      const bool f32_lds = std::is_same<T, float>::value && ninj > PCG_NXR && P->pcg_xlds &&
                           P->pcg_xlds_f32 > 0;
      if (nxr_sel > 0 && want <= 1 && !P->no_xreg) {
        // 256-thread groups, whose kernel sums the X^T z partials with one
        // butterfly per wave (512-thread groups have no registers for it and
        // take a wave sum per injection: mixed 40^3/30^3 solve 2.22 s against
        // 1.61 s at 256; CONNREG_PCG_XBS=512 selects them)
        // (128 FP32 rows need 288 registers at 256 threads, one wave per SIMD;
        // at 512 threads they fit in 255, two waves per SIMD, with a wave sum
        // per injection, so a grid that does not fit at 256 tries 512)
        const int xbs = P->pcg_xbs > 0 ? P->pcg_xbs : NT;
        for (int bs : {xbs, NT, 512}) {
          if (f32_lds && nxr_sel == PCG_NXR2 && (bs == 512 || P->pcg_xlds_f32 == 2)) break;
          PcgArgs<T> probe{};
          probe.g = P->gx;
          probe.Xm = X();
          probe.vpt = 1;
          probe.bs = bs;
          probe.nxr = nxr_sel;
          int maxwg = pcg_max_wg<T>(probe);
          if (P->cu_share > 0) maxwg = share_cap(maxwg, P->cu_share);
          const int64_t w = std::max<int64_t>(1, (nx + bs - 1) / bs);
          if (maxwg > 0 && w <= maxwg) {
            pcg_vpt_v = 1;
            pcg_nwg_v = (int)w;
            pcg_bs_v = bs;
            pcg_nxr_v = nxr_sel;
            break;
          }
        }
      }
      // more injections than register rows: 64 rows in registers and the
      // rest in LDS, loaded once per solve: all of them in 256-thread groups
      // (one per CU; at most PCG_XLDS_MAX rows), else the first
      // PCG_XLDS_MAX512 in 512-thread groups with the rest streamed, when
      // the grid fits
      if (pcg_nxr_v == 0 && ninj > PCG_NXR && want <= 1 && !P->no_xreg && P->pcg_xlds) {
        const int tail = ninj - PCG_NXR;
        for (int bs : {NT, 512}) {
          const int cap = pcg_xlds_cap(bs, (int)sizeof(T));
          const int rows = bs == NT ? tail : std::min(tail, cap);
          if (bs == NT && tail > cap) continue;
          PcgArgs<T> probe{};
          probe.g = P->gx;
          probe.Xm = X();
          probe.ninj = ninj;
          probe.vpt = 1;
          probe.bs = bs;
          probe.nxr = PCG_NXR;
          probe.xtail = 2;
          probe.xlds = rows;
          int maxwg = pcg_max_wg<T>(probe);
          if (P->cu_share > 0) maxwg = share_cap(maxwg, P->cu_share);
          const int64_t w = std::max<int64_t>(1, (nx + bs - 1) / bs);
          if (maxwg > 0 && w <= maxwg) {
            pcg_vpt_v = 1;
            pcg_nwg_v = (int)w;
            pcg_bs_v = bs;
            pcg_nxr_v = PCG_NXR;
            pcg_xtail_v = 2;
            pcg_xlds_v = rows;
            break;
          }
        }
      }
      // FP32 data whose LDS form did not fit: back to 128 register rows in
      // 512-thread groups
      if (pcg_nxr_v == 0 && f32_lds && nxr_sel == PCG_NXR2 && want <= 1 && !P->no_xreg) {
        PcgArgs<T> probe{};
        probe.g = P->gx;
        probe.Xm = X();
        probe.vpt = 1;
        probe.bs = 512;
        probe.nxr = PCG_NXR2;
        int maxwg = pcg_max_wg<T>(probe);
        if (P->cu_share > 0) maxwg = share_cap(maxwg, P->cu_share);
        const int64_t w = std::max<int64_t>(1, (nx + 511) / 512);
        if (maxwg > 0 && w <= maxwg) {
          pcg_vpt_v = 1;
          pcg_nwg_v = (int)w;
          pcg_bs_v = 512;
          pcg_nxr_v = PCG_NXR2;
        }
      }
      // else the rest streamed, in 512-thread groups (253 VGPRs, two waves per SIMD)
      if (pcg_nxr_v == 0 && ninj > PCG_NXR && want <= 1 && !P->no_xreg) {
        PcgArgs<T> probe{};
        probe.g = P->gx;
        probe.Xm = X();
        probe.vpt = 1;
        probe.bs = 512;
        probe.nxr = PCG_NXR;
        probe.xtail = 1;
        int maxwg = pcg_max_wg<T>(probe);
        if (P->cu_share > 0) maxwg = share_cap(maxwg, P->cu_share);
        const int64_t w = std::max<int64_t>(1, (nx + 511) / 512);
        if (maxwg > 0 && w <= maxwg) {
          pcg_vpt_v = 1;
          pcg_nwg_v = (int)w;
          pcg_bs_v = 512;
          pcg_nxr_v = PCG_NXR;
          pcg_xtail_v = 1;
        }
      }
    }
    if (!pick(P->gy, nullptr, pcg_vpt_u, pcg_nwg_u) ||
        (pcg_nxr_v == 0 && !pick(P->gx, X(), pcg_vpt_v, pcg_nwg_v))) {
      set_error("problem too large for one cooperative PCG grid");
      return CR_EINVAL;
    }
    const int nwg = std::max(pcg_nwg_u, pcg_nwg_v);
    // partial sums for the widest grid (the two-level packing may use more
    // workgroups than the plain v-system grid)
    int nwg_all = nwg;
    if (P->cv.valid) nwg_all = std::max({nwg_all, P->cv.pack[0].nwg, P->cv.pack[1].nwg});
    pcgpart_size = (int64_t)(6 + ninj) * nwg_all;
    pcgpart = WS(double, "pcgpart", pcgpart_size);
    return CR_OK;
  }

  cr_status alloc_rank(int rcap) {
    rmax = std::max(rcap, 1);
    const int64_t r2 = (int64_t)rmax * rmax;
    LU = WS(T, "LU", ny * rmax);
    L2U = WS(T, "L2U", ny * rmax);
    LV = WS(T, "LV", nx * rmax);
    L2V = WS(T, "L2V", nx * rmax);
    N = WS(T, "N", ny * ninj);
    Ht = WS(double, "Ht", (int64_t)ninj * rmax);
    St = WS(double, "St", (int64_t)ninj * rmax);
    G = WS(double, "G", (int64_t)ninj * r2);
    By1 = WS(double, "By1", r2);
    By2 = WS(double, "By2", r2);
    Bx1 = WS(double, "Bx1", r2);
    Bx2 = WS(double, "Bx2", r2);
    Tm = WS(double, "Tm", (int64_t)rmax * ninj);
    gpart = WS(double, "gpart", gemm_part_cap(P));
    return CR_OK;
  }

  // Host copy of device scalars; fails when a persistent kernel's grid
  // barrier timed out (the live flag, for reads right after the launch; the
  // kernels also record PERSIST_TIMEOUT in their status scalars for reads
  // deferred past later launches, checked where those are read).
  cr_status read_scalars(const double* dev, int count, double* host) {
    unsigned* flag = (unsigned*)(P->hscal + 60);
    CR_HIP(hipMemcpyAsync(P->hscal, dev, sizeof(double) * count, hipMemcpyDeviceToHost, st));
    CR_HIP(hipMemcpyAsync(flag, P->bar + BAR_TIMEOUT, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    CR_HIP(hipStreamSynchronize(st));
    if (*flag) {
      set_error("grid barrier timed out in a persistent kernel");
      return CR_EHIP;
    }
    std::memcpy(host, P->hscal, sizeof(double) * count);
    return CR_OK;
  }

  // ------------------------------------------------------------ derived data
  // stencil columns [c0, c0+nc) of U, V into LU, L2U, LV, L2V
  cr_status stencil_cols(int c0, int nc) {
    CR_TRY(stencil<T>(P->gy, nc, U + c0 * ldu, ldu, LU + c0 * ny, ny, st));
    CR_TRY(stencil<T>(P->gy, nc, LU + c0 * ny, ny, L2U + c0 * ny, ny, st));
    CR_TRY(stencil<T>(P->gx, nc, V + c0 * ldv, ldv, LV + c0 * nx, nx, st));
    CR_TRY(stencil<T>(P->gx, nc, LV + c0 * nx, nx, L2V + c0 * nx, nx, st));
    return CR_OK;
  }

  // H^T = X^T V (ninj x r, ld ninj)
  cr_status compute_Ht(int r) {
    if (r == 0) return CR_OK;
    Blocks<T> A, B;
    A.clear();
    B.clear();
    A.add(X(), nx, ninj);
    B.add(V, ldv, r);
    return gemm_tn<T>(nx, A, B, nullptr, nullptr, 0, Ht, ninj, gpart, gemm_part_cap(P), st);
  }

  // N = OY - Omega o (U Z H)
  cr_status build_N(int r) {
    if (r > 0)
      CR_TRY(small_gemm(r, ninj, r, Z, ldz, false, Ht, ninj, true, 1.0, Tm, r, st));
    return masked_tall_gemm<T>(ny, r, ninj, U, ldu, Tm, r, P->bits, OY(), ny, N, ny, st);
  }

  // out = R v  (R = N X^T - lam (U Z L2V^T + 2 LU Z LV^T + L2U Z V^T)); y0 keeps
  // [X^T v | V^T v | LV^T v | L2V^T v]
  cr_status apply_R(int r, const T* v, T* out) {
    Blocks<T> A;
    A.clear();
    A.add(X(), nx, ninj);
    A.add(V, ldv, r);
    A.add(LV, nx, r);
    A.add(L2V, nx, r);
    CR_TRY(gemv_t<T>(nx, A, v, y0, part, st));
    const int k = ninj + 3 * r;
    hipLaunchKernelGGL(k_rcoef, dim3((unsigned)((k + 3) / 4)), dim3(256), 0, st, ninj, r, y0, Z, ldz, 0,
                       lam, coef);
    CR_HIP(hipGetLastError());
    Blocks<T> B;
    B.clear();
    B.add(N, ny, ninj);
    B.add(U, ldu, r);
    B.add(LU, ny, r);
    B.add(L2U, ny, r);
    return gemv_n<T>(ny, B, coef, 0.0, out, st);
  }

  // out = R^T u; y0 keeps [N^T u | U^T u | LU^T u | L2U^T u]
  cr_status apply_RT(int r, const T* u, T* out) {
    Blocks<T> A;
    A.clear();
    A.add(N, ny, ninj);
    A.add(U, ldu, r);
    A.add(LU, ny, r);
    A.add(L2U, ny, r);
    CR_TRY(gemv_t<T>(ny, A, u, y0, part, st));
    const int k = ninj + 3 * r;
    hipLaunchKernelGGL(k_rcoef, dim3((unsigned)((k + 3) / 4)), dim3(256), 0, st, ninj, r, y0, Z, ldz, 1,
                       lam, coef);
    CR_HIP(hipGetLastError());
    Blocks<T> B;
    B.clear();
    B.add(X(), nx, ninj);
    B.add(L2V, nx, r);
    B.add(LV, nx, r);
    B.add(V, ldv, r);
    return gemv_n<T>(nx, B, coef, 0.0, out, st);
  }

  cr_status dot(int64_t n, const T* a, const T* b, double* out) {
    Blocks<T> A;
    A.clear();
    A.add(a, n, 1);
    return gemv_t<T>(n, A, b, out, part, st);
  }

  // ------------------------------------------------------------ ALS
  // x0 / xbuf / bref: warm start (xbuf receives the unnormalised solution,
  // default the work vector), see pcg_warm
  // Coarse operator of the current v-system, A_c = P^T B_hat P =
  // lam (C2 + 2c C1 + e I) + Y diag(g) Y^T, and its inverse by Cholesky (one
  // workgroup), a row-parallel triangular inverse and Ainv = L^-T L^-1
  // (matrix cores); Ainv stays zero if the factorisation fails (Jacobi).
  double *co_Ainv = nullptr, *co_rc = nullptr;
  cr_status coarse_factor() {
    const CoarseLevel& cl = P->cv;
    const int m = cl.m;
    const int64_t mm = (int64_t)m * m;
    double* A = WS(double, "co_A", mm);
    double* Li = WS(double, "co_Li", mm);
    co_Ainv = WS(double, "co_Ainv", mm);
    co_rc = WS(double, "co_rc", m);
    double* info = WS(double, "co_info", 2);
    CR_TRY(coarse_assemble(m, lam, cv, cl.C1, cl.C2, cl.Y, ninj, gw, A, st));
    CR_TRY(chol_lower(m, A, m, info, st));
    CR_TRY(trinv_rows(m, A, m, Li, m, info, st));
    Blocks<double> B;
    B.clear();
    B.add(Li, m, m);
    return gemm_tn<double>(m, B, B, nullptr, nullptr, 0, co_Ainv, m, gpart, gemm_part_cap(P), st);
  }

  cr_status pcg(bool usys, const T* b, T* xout, double rtol, int maxit, double* scal,
                const T* x0 = nullptr, T* xbuf = nullptr, const double* bref = nullptr) {
    PcgArgs<T> a{};
    a.g = usys ? P->gy : P->gx;
    a.lam = lam;
    a.coef = usys ? cu : cv;
    a.dvec = usys ? dvec : nullptr;
    a.Xm = usys ? nullptr : X();
    a.ldx = nx;
    a.ninj = ninj;
    a.gw = gw;
    a.minv = usys ? minv_u : minv_v;
    a.b = b;
    T** w = usys ? pw_u : pw_v;
    a.x = w[0];
    a.r = w[1];
    a.z = w[2];
    a.p = w[3];
    a.t = w[4];
    a.q = w[5];
    a.xout = xout;
    a.x0 = x0;
    a.bref = bref;
    if (xbuf) a.x = xbuf;
    a.part = pcgpart;
    a.sbuf = sbuf;
    a.scal = scal;
    a.rtol = rtol;
    a.maxit = maxit;
    a.vpt = usys ? pcg_vpt_u : pcg_vpt_v;
    a.bs = usys ? pcg_bs : pcg_bs_v;
    a.nxr = usys ? 0 : pcg_nxr_v;
    a.xtail = usys ? 0 : pcg_xtail_v;
    a.xlds = usys ? 0 : pcg_xlds_v;
    a.bar.bar = P->bar;
    a.bar.mode = P->bar_mode;
    a.bar.coop = P->coop;
    a.bar.spin_max = P->bar_spin;
    int nwg = usys ? pcg_nwg_u : pcg_nwg_v;
    if (!usys && P->cv.valid && co_Ainv && a.vpt == 1 && (a.bs == NT || a.bs == 512)) {
      PcgArgs<T> c = a;
      if (c.xtail == 2) {  // the two-level form streams the tail (512-thread groups)
        c.xtail = 1;
        c.xlds = 0;
        c.bs = 512;
      }
      const CoarsePack& pk = P->cv.pack[c.bs == NT ? 0 : 1];
      c.co.slot_vox = pk.slot_vox;
      c.co.slot_agg = pk.slot_agg;
      c.co.slot_w = pk.slot_w;
      c.co.wg_agg = pk.wg_agg;
      c.co.agg_lo = pk.agg_lo;
      c.co.agg_hi = pk.agg_hi;
      c.co.m = P->cv.m;
      c.co.Ainv = co_Ainv;
      c.co.rc = co_rc;
      int maxwg = pcg_max_wg<T>(c);
      if (P->cu_share > 0) maxwg = share_cap(maxwg, P->cu_share);
      // the two-level grid must be co-resident; else plain Jacobi-PCG
      if (maxwg >= pk.nwg && pk.nwg * 6 + (int64_t)ninj * pk.nwg <= pcgpart_size) {
        return pcg_solve<T>(c, pk.nwg, st);
      }
    }
    return pcg_solve<T>(a, nwg, st);
  }

  // FP64 Jacobi-PCG of an ALS half-step, warm-started from the previous
  // sweep's unnormalised solution of the same system (the system changes
  // with the other factor, its solution little once the sweeps settle): the
  // kernel starts at x0 with the residual b - A x0 and stops at
  // ||b - A x|| <= rtol ||b||.  The first solve of each system in an ALS
  // starts from zero.
  bool warm_u_ok = false, warm_v_ok = false;
  cr_status pcg_warm(bool usys, const T* b, T* xout, double rtol, int maxit, double* scal) {
    const int64_t n = usys ? ny : nx;
    T* xw = WS(T, usys ? "warm_u" : "warm_v", n);
    bool& valid = usys ? warm_u_ok : warm_v_ok;
    if constexpr (std::is_same<T, double>::value) {
      if (valid && P->pcg_warm) {
        double* r0 = WS(double, "warm_r", n);
        double* t0 = WS(double, "warm_t", n);
        double* bref = tmp + 12;
        CR_TRY(dot(n, b, b, bref));
        if (!usys) {
          Blocks<T> A;
          A.clear();
          A.add(X(), nx, ninj);
          CR_TRY((gemv_tx<T, double>(nx, A, xw, y0, part, st)));
        }
        CR_TRY(als_residual<T>(usys ? P->gy : P->gx, lam, usys ? cu : cv, usys ? dvec : nullptr,
                               usys ? nullptr : X(), nx, ninj, gw, y0, b, xw, t0, r0, st));
        return pcg(usys, r0, xout, rtol, maxit, scal, xw, xw, bref);
      }
    }
    valid = true;
    return pcg(usys, b, xout, rtol, maxit, scal, nullptr, xw, nullptr);
  }

  struct SolveOut {
    double norm = 0.0, relres = 0.0;
    int iters = 0, status = 0;
  };

  cr_status dot64(int64_t n, const double* a, const double* b, double* out) {
    Blocks<double> A;
    A.clear();
    A.add(a, n, 1);
    return gemv_t<double>(n, A, b, out, part, st);
  }

  // Direct solve of the v-system (eq. ALS_linsys_v) on a full source box by
  // the Sherman-Morrison-Woodbury identity with spectral solves (k_spec.hip),
  // in FP64, followed by up to two refinement steps with the same factors
  // until the FP64 residual meets rtol.  done = false (nothing written) when
  // it does not, and the caller falls back to PCG.
  cr_status smw_v(const T* b, T* xout, double rtol, SolveOut* out, bool& done) {
    done = false;
    const int64_t n = nx;
    double* Xh = WS(double, "smw_Xh", n * ninj);  // Q^T X of the source box, per handle
    double* Yh = WS(double, "smw_Yh", n * ninj);  // Xh scaled by 1/s, per solve
    double* Km = WS(double, "smw_K", (int64_t)ninj * ninj);
    double* h = WS(double, "smw_h", ninj);
    double* kv = WS(double, "smw_k", ninj);
    double* b64 = WS(double, "smw_b", n);
    double* x64 = WS(double, "smw_x", n);
    double* t64 = WS(double, "smw_t", n);
    double* r64 = WS(double, "smw_r", n);
    double* w64 = WS(double, "smw_w", n);
    const double* X64 = P->X64;
    CR_TRY((convert2d<double, T>(n, 1, b, n, b64, n, st)));
    if (!P->smw_xh_ready) {
      CR_TRY(box_transform_cols(P->boxx, false, ninj, X64, n, Xh, n, Yh, n, st));
      P->smw_xh_ready = true;
    }
    // K = chol(I + G^1/2 Xh^T diag(1/s) Xh G^1/2)
    CR_HIP(hipMemcpyAsync(Yh, Xh, sizeof(double) * n * ninj, hipMemcpyDeviceToDevice, st));
    CR_TRY(box_scale_cols(P->boxx, cv, lam, nullptr, ninj, Yh, n, st));
    Blocks<double> A, B, H;
    A.clear();
    A.add(X64, n, ninj);
    H.clear();
    H.add(Xh, n, ninj);
    B.clear();
    B.add(Yh, n, ninj);
    CR_TRY(gemm_tn<double>(n, H, B, nullptr, nullptr, 0, Km, ninj, gpart, gemm_part_cap(P), st));
    CR_TRY(smw_factor(ninj, gw, Km, st));
    // x = 0, r = b; then x += SMW(r), r = b - A x, up to three times
    CR_HIP(hipMemsetAsync(x64, 0, sizeof(double) * n, st));
    CR_HIP(hipMemcpyAsync(r64, b64, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    CR_TRY(dot64(n, b64, b64, tmp + 9));
    double q[2] = {0.0, 0.0};
    for (int pass = 0; pass < 3; ++pass) {
      // rh = Q^T r (in w64); th = rh / s (in t64); h = Xh^T th
      CR_TRY(box_transform_cols(P->boxx, false, 1, r64, n, w64, n, t64, n, st));
      CR_HIP(hipMemcpyAsync(t64, w64, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      CR_TRY(box_scale_cols(P->boxx, cv, lam, nullptr, 1, t64, n, st));
      CR_TRY((gemv_tx<double, double>(n, H, t64, h, part, st)));
      CR_TRY(smw_apply(ninj, gw, Km, h, kv, st));
      // xh = (rh + Xh k) / s, increment = Q xh
      CR_TRY(gemv_n<double>(n, H, kv, 1.0, w64, st));
      CR_TRY(box_scale_cols(P->boxx, cv, lam, nullptr, 1, w64, n, st));
      CR_TRY(box_transform_cols(P->boxx, true, 1, w64, n, t64, n, r64, n, st));
      hipLaunchKernelGGL(k_add_to, dim3(nblk(n)), dim3(256), 0, st, n, t64, x64);
      CR_HIP(hipGetLastError());
      // r = b - A x in FP64 with FP64 operator data
      CR_TRY((gemv_tx<double, double>(n, A, x64, y0, part, st)));
      CR_TRY(als_residual<double>(P->gx, lam, cv, nullptr, X64, n, ninj, gw, y0, b64, x64, w64,
                                  r64, st));
      CR_TRY(dot64(n, r64, r64, tmp + 10));
      CR_TRY(read_scalars(tmp + 9, 2, q));
      if (!std::isfinite(q[1])) return CR_OK;
      if (q[1] <= rtol * rtol * q[0]) break;
    }
    if (!(q[1] <= rtol * rtol * q[0])) return CR_OK;
    done = true;
    *out = SolveOut{};
    out->iters = 1;
    out->relres = q[0] > 0.0 ? std::sqrt(q[1] / q[0]) : 0.0;
    CR_TRY(dot64(n, x64, x64, tmp + 11));
    CR_TRY(normalize_out<T>(n, x64, tmp + 11, xout, st));
    double hn[1];
    CR_TRY(read_scalars(tmp + 11, 1, hn));
    out->norm = std::sqrt(std::max(hn[0], 0.0));
    return CR_OK;
  }

  // Solve the u-system (usys) or the v-system for b; xout = unit solution.
  // FP64: one PCG launch; its scalars stay in dsc[0..3] for a later read.
  // Mixed: FP32 PCG corrections inside an FP64 residual-and-refinement loop
  // (x accumulated in FP64, r = b - A x evaluated in FP64 arithmetic).
  cr_status solve_sys(bool usys, const T* b, T* xout, double rtol, int maxit, double* dsc,
                      SolveOut* out, bool& deferred) {
    if (usys && P->fcg_mode > 0) {
      deferred = false;
      double* xs = WS(double, "fcg_x", ny);
      int fb = 0;
      const double *b64 = (const double*)b, *d64 = (const double*)dvec, *m64 = (const double*)minv_u;
      if (!std::is_same<T, double>::value) {
        // mixed handle: the flexible CG runs in FP64 on FP64 copies
        double* cb = WS(double, "fcg_b", ny);
        double* cd = WS(double, "fcg_d", ny);
        double* cm = WS(double, "fcg_m", ny);
        CR_TRY((convert2d<double, T>(ny, 1, b, ny, cb, ny, st)));
        CR_TRY((convert2d<double, T>(ny, 1, dvec, ny, cd, ny, st)));
        CR_TRY((convert2d<double, T>(ny, 1, minv_u, ny, cm, ny, st)));
        b64 = cb;
        d64 = cd;
        m64 = cm;
      }
      CR_TRY(fcg_u(b64, xs, rtol, maxit, out, &fb, d64, m64, P->fcg_mode == 2));
      P->pc_fallbacks += fb;
      if (out->status != 0) {
        // the flexible CG failed: Jacobi-PCG decides
        ++P->pc_fallbacks;
        CR_TRY(pcg(true, b, xout, rtol, maxit, dsc));
        double h[4];
        CR_TRY(read_scalars(dsc, 4, h));
        *out = SolveOut{h[0], h[1], out->iters + (int)h[2], (int)h[3]};
        return CR_OK;
      }
      CR_TRY(dot64(ny, xs, xs, tmp + 11));
      CR_TRY(normalize_out<T>(ny, xs, tmp + 11, xout, st));
      return CR_OK;
    }
    if (!usys && P->fcg_mode > 0 && P->boxx.valid && ninj <= SMW_MAX) {
      bool done = false;
      CR_TRY(smw_v(b, xout, rtol, out, done));
      if (done) {
        deferred = false;
        return CR_OK;
      }
    }
    if (std::is_same<T, double>::value) {
      deferred = true;
      return pcg_warm(usys, b, xout, rtol, maxit, dsc);
    }
    deferred = false;
    const int64_t n = usys ? ny : nx;
    const Geom& g = usys ? P->gy : P->gx;
    double* x64 = WS(double, "ref_x", n);
    double* r64 = WS(double, "ref_r", n);
    double* t64 = WS(double, "ref_t", n);
    T* rb = WS(T, "ref_b", n);
    T** w = usys ? pw_u : pw_v;
    const double in_rtol = std::max(rtol, 1e-5);
    *out = SolveOut{};
    double h[4], q[2];
    CR_TRY(dot(n, b, b, tmp + 9));
    // warm start: from the second sweep of an ALS on, the FP64 iterate starts
    // at the previous sweep's solution of this system and the loop below
    // begins with its residual; else a first FP32 solve from zero
    double* xw64 = WS(double, usys ? "mwarm_u" : "mwarm_v", n);
    bool& warm = usys ? warm_u_ok : warm_v_ok;
    if (warm && P->pcg_warm) {
      CR_HIP(hipMemcpyAsync(x64, xw64, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    } else {
      CR_TRY(pcg(usys, b, xout, in_rtol, maxit, dsc));
      CR_TRY(read_scalars(dsc, 4, h));
      out->iters += (int)h[2];
      if (h[3] == 2.0) {
        out->status = 2;
        return CR_OK;
      }
      CR_TRY(accumulate<T>(n, w[0], x64, true, st));
    }
    double rr = 0.0, bb = 0.0, rr_prev = -1.0;
    for (int k = 0; k < 12; ++k) {
      if (!usys) {
        Blocks<T> A;
        A.clear();
        A.add(X(), nx, ninj);
        CR_TRY((gemv_tx<T, double>(nx, A, x64, y0, part, st)));
      }
      CR_TRY(als_residual<T>(g, lam, usys ? cu : cv, usys ? dvec : nullptr,
                             usys ? nullptr : X(), nx, ninj, gw, y0, b, x64, t64, r64, st));
      CR_TRY(dot64(n, r64, r64, tmp + 10));
      CR_TRY(read_scalars(tmp + 9, 2, q));
      bb = q[0];
      rr = q[1];
      if (!(rr > rtol * rtol * bb)) break;
      // stagnation at the FP64 floor of the residual: stop refining
      if (rr_prev >= 0.0 && rr > 0.25 * rr_prev) break;
      rr_prev = rr;
      CR_TRY((convert2d<T, double>(n, 1, r64, n, rb, n, st)));
      // the correction only has to take the residual from sqrt(rr) to
      // rtol ||b|| (with a factor 2 of margin), not by a full in_rtol again
      const double need = 0.5 * rtol * std::sqrt(bb / rr);
      CR_TRY(pcg(usys, rb, xout, std::max(in_rtol, need), maxit, dsc));
      CR_TRY(read_scalars(dsc, 4, h));
      out->iters += (int)h[2];
      if (h[3] == 2.0) break;
      CR_TRY(accumulate<T>(n, w[0], x64, false, st));
    }
    out->relres = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    out->status = (rr <= rtol * rtol * bb) ? 0 : 1;
    CR_HIP(hipMemcpyAsync(xw64, x64, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    warm = true;
    CR_TRY(dot64(n, x64, x64, tmp + 11));
    CR_TRY(normalize_out<T>(n, x64, tmp + 11, xout, st));
    CR_TRY(read_scalars(tmp + 11, 1, h));
    out->norm = std::sqrt(std::max(h[0], 0.0));
    return CR_OK;
  }

  // Flexible CG (one previous direction kept, Notay's FCG(1)) on the u-system
  // of eq. ALS_linsys.  The preconditioner is a base step w = M^-1 r, the
  // spectral solve of the box when the target grid is a full box, else
  // Jacobi, optionally refined by the learned network (z = network(w));
  // whenever the network's z is not a descent direction (r.z <= 0 or not
  // finite) the iteration uses w instead and counts a fallback.  All scalars
  // stay on the device; the host checks convergence after 1, 2, 4, 8, 16
  // iterations and every 16 after that.
  cr_status fcg_u(const double* b, double* xsol, double rtol, int maxit, SolveOut* out,
                  int* fallbacks, const double* dv, const double* mi, bool use_net) {
    cr_pc* pc = P->pc;
    const bool net = use_net && pc;
    const int64_t n = ny;
    double* W = WS(double, "fcg_work", 9 * n);
    double *r = W, *z = W + n, *p = W + 2 * n, *q = W + 3 * n, *pp = W + 4 * n, *qq = W + 5 * n,
           *t = W + 6 * n, *w = W + 7 * n, *t2 = W + 8 * n;
    double* S = WS(double, "fcg_S", FS_N);
    CR_HIP(hipMemsetAsync(S, 0, sizeof(double) * FS_N, st));
    CR_HIP(hipMemsetAsync(xsol, 0, sizeof(double) * n, st));
    CR_HIP(hipMemsetAsync(pp, 0, sizeof(double) * n, st));
    CR_HIP(hipMemsetAsync(qq, 0, sizeof(double) * n, st));
    CR_HIP(hipMemcpyAsync(r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    CR_TRY(dot64(n, b, b, S + FS_BB));
    const bool spectral = P->boxy.valid;
    if (spectral) {
      double* ones = WS(double, "fcg_ones", n);
      hipLaunchKernelGGL(k_fill, dim3(nblk(n)), dim3(256), 0, st, n, 1.0, ones);
      CR_HIP(hipGetLastError());
      CR_TRY(dot64(n, dv, ones, S + FS_DBAR));
      hipLaunchKernelGGL(k_scale1, dim3(1), dim3(1), 0, st, S + FS_DBAR, 1.0 / (double)n);
      CR_HIP(hipGetLastError());
    }
    // (the zero right-hand side is detected on the device: no host read here)
    hipLaunchKernelGGL(k_fcg_init, dim3(1), dim3(1), 0, st, S);
    CR_HIP(hipGetLastError());
    double h[FS_N];
    *out = SolveOut{};
    const double tol2 = rtol * rtol;
    int it = 0;
    for (; it < maxit; ++it) {
      // base step w, then z (network refinement or w itself)
      if (spectral) {
        CR_TRY(box_spectral_solve(P->boxy, cu, lam, S + FS_DBAR, r, w, t2, st));
      } else {
        hipLaunchKernelGGL(k_jacobi, dim3(nblk(n)), dim3(256), 0, st, n, mi, r, w);
        CR_HIP(hipGetLastError());
      }
      const double* zz = w;
      if (net) {
        CR_TRY(dot64(n, w, w, S + FS_WW));
        CR_TRY(lpc_input(pc->net, w, S + FS_WW, mi, dv, P->gy.deg, cu, lam, pc->acts.in, st));
        CR_TRY(lpc_forward(pc->net, pc->acts.in, pc->acts, st));
        CR_TRY(lpc_output(pc->net, pc->acts.in, pc->acts.y, z, st));
        zz = z;
      }
      // [r.z, qq.z, r.w, qq.w] (without the network z is w and only the
      // first pair is read)
      Blocks<double> A;
      A.clear();
      A.add(r, n, 1);
      A.add(qq, n, 1);
      CR_TRY(gemv_t<double>(n, A, zz, S + FS_DZ, part, st));
      if (net) CR_TRY(gemv_t<double>(n, A, w, S + FS_DZ + 2, part, st));
      hipLaunchKernelGGL(k_fcg_beta, dim3(1), dim3(1), 0, st, S, it == 0 ? 1 : 0, net ? 1 : 0);
      hipLaunchKernelGGL(k_fcg_dir, dim3(nblk(n)), dim3(256), 0, st, n, zz, w, S, pp, p);
      CR_HIP(hipGetLastError());
      CR_TRY(stencil<double>(P->gy, 1, p, n, t, n, st));
      hipLaunchKernelGGL(k_uapply, dim3(nblk(n)), dim3(256), 0, st, n, P->gy.K, P->gy.nbr, lam,
                         cu, dv, p, t, q);
      CR_HIP(hipGetLastError());
      A.clear();
      A.add(q, n, 1);
      A.add(r, n, 1);
      CR_TRY(gemv_t<double>(n, A, p, S + FS_DP, part, st));
      hipLaunchKernelGGL(k_fcg_alpha, dim3(1), dim3(1), 0, st, S);
      hipLaunchKernelGGL(k_fcg_update, dim3(nblk(n)), dim3(256), 0, st, n, S, p, q, xsol, r);
      CR_HIP(hipGetLastError());
      CR_TRY(dot64(n, r, r, S + FS_RR));
      hipLaunchKernelGGL(k_fcg_check, dim3(1), dim3(1), 0, st, S, tol2);
      CR_HIP(hipGetLastError());
      std::swap(p, pp);
      std::swap(q, qq);
      // host checks after 1, 2, 4, 8, 16 iterations, then every 16: a solve
      // that converges in a few steps runs at most as many again
      const int done_its = it + 1;
      if ((done_its & (done_its - 1)) == 0 || (done_its & 15) == 0 || done_its == maxit) {
        CR_TRY(read_scalars(S, FS_N, h));
        if (h[FS_STATE] != 0.0) break;
      }
    }
    // ||x||^2 goes into the slot of ||w||^2 (free after the loop), so one
    // read brings every final scalar
    CR_TRY(dot64(n, xsol, xsol, S + FS_WW));
    CR_TRY(read_scalars(S, FS_N, h));
    const double bb = h[FS_BB];
    out->iters = (int)h[FS_IT];
    out->relres = bb > 0.0 ? std::sqrt(std::max(h[FS_RR], 0.0) / bb) : 0.0;
    out->status = h[FS_STATE] == 2.0 ? 2 : h[FS_STATE] == 1.0 ? 0 : 1;
    *fallbacks = (int)h[FS_FB];
    out->norm = std::sqrt(std::max(h[FS_WW], 0.0));
    return CR_OK;
  }

  // One ALS sweep: u from v (eq. ALS_linsys), then v from u (eq. ALS_linsys_v).
  cr_status sweep(int r, T* v, T* u, double rtol, int maxit, SolveOut* ou, SolveOut* ov) {
    bool du = false, dv = false;
    // u-half
    CR_TRY(stencil<T>(P->gx, 1, v, nx, Lv, nx, st));
    CR_TRY(apply_R(r, v, rhs_u));  // y0[0:ninj] = h = X^T v
    CR_TRY(masked_quad_ws<T>(ny, ninj, P->bits, y0, dvec, tmp + 8, st));
    CR_TRY(dot(nx, Lv, v, tmp + 0));   // b = v^T L_x v
    CR_TRY(dot(nx, Lv, Lv, tmp + 1));  // a = ||L_x v||^2
    hipLaunchKernelGGL(k_set2, dim3(1), dim3(1), 0, st, cu, tmp + 0, 2.0, tmp + 1, 1.0);
    CR_HIP(hipGetLastError());
    CR_TRY(pcg_diag<T>(P->gy, lam, cu, dvec, nullptr, 0, 0, nullptr, minv_u, st));
    CR_TRY(solve_sys(true, rhs_u, u, rtol, maxit, sc + 0, ou, du));
    // v-half
    CR_TRY(stencil<T>(P->gy, 1, u, ny, Lu, ny, st));
    CR_TRY(apply_RT(r, u, rhs_v));
    CR_TRY(masked_colsq<T>(ny, ninj, P->bits, u, gw, part, st));
    CR_TRY(dot(ny, Lu, u, tmp + 2));   // c = u^T L_y u
    CR_TRY(dot(ny, Lu, Lu, tmp + 3));  // e = ||L_y u||^2
    hipLaunchKernelGGL(k_set2, dim3(1), dim3(1), 0, st, cv, tmp + 2, 2.0, tmp + 3, 1.0);
    CR_HIP(hipGetLastError());
    CR_TRY(pcg_diag<T>(P->gx, lam, cv, nullptr, X(), nx, ninj, gw, minv_v, st));
    if (P->cv.valid) CR_TRY(coarse_factor());
    CR_TRY(solve_sys(false, rhs_v, v, rtol, maxit, sc + 4, ov, dv));
    if (du || dv) {
      double hs[8];
      CR_TRY(read_scalars(sc, 8, hs));
      if ((du && hs[3] == PERSIST_TIMEOUT) || (dv && hs[7] == PERSIST_TIMEOUT)) {
        set_error("grid barrier timed out in a persistent PCG kernel");
        return CR_EHIP;
      }
      if (du) *ou = SolveOut{hs[0], hs[1], (int)hs[2], (int)hs[3]};
      if (dv) *ov = SolveOut{hs[4], hs[5], (int)hs[6], (int)hs[7]};
    }
    return CR_OK;
  }

  cr_status als(int r, T* v, T* u, const cr_solve_opts& o, cr_als_stats* stats, bool& zero_rhs) {
    zero_rhs = false;
    warm_u_ok = warm_v_ok = false;
    int sweeps = 0;
    double delta = 0.0;
    SolveOut su, sv;
    it_u = it_v = notconv = 0;
    const int fixed = o.als_fixed_sweeps;
    while (true) {
      CR_TRY(sweep(r, v, u, o.pcg_rtol, o.pcg_maxit, &su, &sv));
      ++sweeps;
      it_u += su.iters;
      it_v += sv.iters;
      notconv += (su.status == 1) + (sv.status == 1);
      if (su.status == 2 || sv.status == 2 || !(su.norm > 0.0) || !(sv.norm > 0.0)) {
        zero_rhs = true;
        break;
      }
      delta = std::fabs(su.norm / sv.norm - 1.0);
      if (fixed > 0) {
        if (sweeps >= fixed) break;
      } else if (delta <= o.als_delta || sweeps >= o.als_max_sweeps) {
        break;
      }
    }
    if (stats) {
      stats->sweeps = sweeps;
      stats->delta = delta;
      stats->unorm = su.norm;
      stats->vnorm = sv.norm;
      stats->pcg_iters_u = it_u;
      stats->pcg_iters_v = it_v;
      stats->pcg_notconv = notconv;
    }
    return CR_OK;
  }

  // x <- x - B (B^T x) twice, then normalise; breakdown when ||x_perp|| <= tol ||x||.
  cr_status cgs2(int64_t n, const T* B, int64_t ldb, int j, T* x, double tol, bool& breakdown) {
    double h[2];
    CR_TRY(dot(n, x, x, tmp + 4));
    if (j > 0) {
      Blocks<T> A;
      A.clear();
      A.add(B, ldb, j);
      for (int pass = 0; pass < 2; ++pass) {
        CR_TRY(gemv_t<T>(n, A, x, y0, part, st));
        hipLaunchKernelGGL(k_neg, dim3(nblk(j)), dim3(256), 0, st, j, y0, coef);
        CR_HIP(hipGetLastError());
        CR_TRY(gemv_n<T>(n, A, coef, 1.0, x, st));
      }
    }
    CR_TRY(dot(n, x, x, tmp + 5));
    CR_TRY(read_scalars(tmp + 4, 2, h));
    breakdown = !(h[1] > tol * tol * h[0]) || !std::isfinite(h[1]);
    if (breakdown) return CR_OK;
    return scale_inv_sqrt<T>(n, x, tmp + 5, st);
  }

  // ------------------------------------------------------------ Grams
  // masked Gram column j: G_a(k, j) = sum_i U_ik omega_ia U_ij, k <= j
  cr_status gram_column(int j, int64_t ldr) {
    double* C = WS(double, "gramcol", (int64_t)(j + 1) * ninj);
    const T* uj = U + (int64_t)j * ldu;
    Blocks<T> A;
    A.clear();
    A.add(U, ldu, j + 1);
    if (P->use_holes) {
      CR_TRY(gemv_t<T>(ny, A, uj, y0, part, st));
      const int64_t m = (int64_t)(j + 1) * ninj;
      hipLaunchKernelGGL(k_bcast_cols, dim3(nblk(m)), dim3(256), 0, st, j + 1, ninj, y0, C,
                         (int64_t)(j + 1));
      CR_HIP(hipGetLastError());
      CR_TRY(hole_gram_col<T>(ninj, P->hptr, P->hidx, j + 1, U, ldu, uj, C, j + 1, st));
    } else {
      Blocks<T> Bd;
      Bd.clear();
      CR_TRY(gemm_tn<T>(ny, A, Bd, P->bits, uj, ninj, C, j + 1, gpart, gemm_part_cap(P), st));
    }
    const int64_t m = (int64_t)(j + 1) * ninj;
    hipLaunchKernelGGL(k_scatter_gram, dim3(nblk(m)), dim3(256), 0, st, ninj, j, C,
                       (int64_t)(j + 1), G, ldr);
    CR_HIP(hipGetLastError());
    return CR_OK;
  }

  // all projected quantities for new column j (columns < j already present)
  cr_status project_column(int j, int64_t ldr) {
    const T* uj = U + (int64_t)j * ldu;
    const T* vj = V + (int64_t)j * ldv;
    const T* luj = LU + (int64_t)j * ny;
    const T* lvj = LV + (int64_t)j * nx;
    Blocks<T> A;
    A.clear();
    A.add(U, ldu, j + 1);
    CR_TRY(gemv_t<T>(ny, A, luj, By1 + j * ldr, part, st));
    A.clear();
    A.add(LU, ny, j + 1);
    CR_TRY(gemv_t<T>(ny, A, luj, By2 + j * ldr, part, st));
    A.clear();
    A.add(V, ldv, j + 1);
    CR_TRY(gemv_t<T>(nx, A, lvj, Bx1 + j * ldr, part, st));
    A.clear();
    A.add(LV, nx, j + 1);
    CR_TRY(gemv_t<T>(nx, A, lvj, Bx2 + j * ldr, part, st));
    for (double* B : {By1, By2, Bx1, Bx2}) {
      hipLaunchKernelGGL(k_mirror, dim3(nblk(j + 1)), dim3(256), 0, st, B, ldr, j);
      CR_HIP(hipGetLastError());
    }
    A.clear();
    A.add(X(), nx, ninj);
    CR_TRY(gemv_t<T>(nx, A, vj, Ht + (int64_t)j * ninj, part, st));
    A.clear();
    A.add(OY(), ny, ninj);
    CR_TRY(gemv_t<T>(ny, A, uj, St + (int64_t)j * ninj, part, st));
    return gram_column(j, ldr);
  }

  // ------------------------------------------------------------ Galerkin
  // Projected CG (eq. Proj_Sylv) from the current Z.  FP64 form: one launch.
  // Low form (BF16 copy of the Gram tensor): iterative refinement, each launch
  // forms the residual with the FP64 operator and runs CG on the BF16 operator
  // until that residual has dropped by GAL_LOW_INNER (or to rtol ||B||); the
  // loop ends when a launch starts from a residual already at rtol ||B||.
  // scal4: total iterations, relative residual (FP64 operator in the low
  // form), status, energy.
  static constexpr double GAL_LOW_INNER = 1e-3;
  static constexpr int GAL_LOW_MAXOUTER = 40;
  int last_gal_outer = 0;

  cr_status galerkin(int r, int64_t ldr, double rtol, int maxit, double* scal4) {
    const int64_t r2 = ldr * ldr;
    GalerkinArgs a{};
    a.r = r;
    a.ldr = (int)ldr;
    a.ninj = ninj;
    a.lam = lam;
    a.G = G;
    a.H = Ht;
    a.S = St;
    a.By1 = By1;
    a.By2 = By2;
    a.Bx1 = Bx1;
    a.Bx2 = Bx2;
    a.Z = Z;
    a.R = WS(double, "gR", r2);
    a.P = WS(double, "gP", r2);
    a.Q = WS(double, "gQ", r2);
    a.Y2 = WS(double, "gY2", r2);
    a.Bm = WS(double, "gB", r2);
    a.T = WS(double, "gT", ldr * ninj);
    a.SG = WS(double, "gSG", ldr * ninj);
    const int maxwg = galerkin_max_wg(r);
    if (maxwg <= 0) {
      set_error("cooperative launch not available for the Galerkin kernel");
      return CR_EHIP;
    }
    // one workgroup per 16 x 16 output tile or per Gram block of 128 rows,
    // at most two per CU
    int ncu = 0;
    CR_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, P->dev));
    const int64_t nt16 = (r + 15) / 16, nrb = (r + 127) / 128;
    const int64_t want = std::max<int64_t>(nt16 * nt16, (int64_t)ninj * nrb);
    int nwg = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)maxwg, 2 * (int64_t)ncu, want}));
    if (P->cu_share > 0) nwg = std::max(1, std::min(nwg, share_cap(maxwg, P->cu_share)));
    a.part = WS(double, "galpart", 9 * nwg);
    a.scal = sc + 8;
    a.rtol = rtol;
    a.maxit = maxit;
    a.bar.bar = P->bar;
    a.bar.mode = P->bar_mode;
    a.bar.coop = P->coop;
    a.bar.spin_max = P->bar_spin;
    const bool low = P->gal_low == 1 || (P->gal_low == -1 && !std::is_same<T, double>::value);
    last_gal_outer = 1;
    if (!low) {
      CR_TRY(galerkin_cg(a, nwg, P->gal_tile / 16, st));
      return read_scalars(sc + 8, 4, scal4);
    }
    const int ldh = (r + 3) / 4 * 4;
    __bf16* gb = WS(__bf16, "gGb", (int64_t)ninj * r * ldh);
    CR_TRY(gram_to_bf16(r, (int)ldr, ldh, ninj, G, gb, st));
    a.ldh = ldh;
    a.Gb = gb;
    a.inner_rel = GAL_LOW_INNER;
    double tot = 0.0, s5[5] = {0, 0, 0, 0, 0};
    int outer = 0;
    for (; outer < GAL_LOW_MAXOUTER; ++outer) {
      a.maxit = std::max(1, maxit - (int)tot);
      CR_TRY(galerkin_cg(a, nwg, P->gal_tile / 16, st));
      CR_TRY(read_scalars(sc + 8, 5, s5));
      tot += s5[0];
      if (s5[2] == PERSIST_TIMEOUT || s5[2] == 2.0) break;
      // the launch started at the tolerance: Z is unchanged and s5[4] is its
      // FP64 relative residual
      if (s5[4] <= rtol || s5[0] == 0.0) {
        s5[1] = s5[4];
        s5[2] = s5[4] <= rtol ? 0.0 : 1.0;
        break;
      }
      if (tot >= maxit) {
        s5[2] = 1.0;
        break;
      }
    }
    last_gal_outer = outer + 1;
    scal4[0] = tot;
    scal4[1] = s5[1];
    scal4[2] = s5[2];
    scal4[3] = s5[3];
    return CR_OK;
  }

  // ------------------------------------------------------------ residual norm
  // Grams of the residual factors F = [N | U | L_y U | L_y^2 U] and
  // G = [X | L_x^2 V | L_x V | V] (R = F Cm G^T), kept in the capacity layout
  // (block b >= 1 at ninj + (b - 1) rmax).  In the greedy loop, where every
  // rank appends one basis column, only the new rows and columns and the
  // N-rows (N changes with Z) are computed: n_y (n_inj k + 9r) + 3 n_x k
  // multiply-adds per rank instead of n_y k^2 + n_x k^2.
  double *GFcap = nullptr, *GXcap = nullptr;
  int gram_r = -1;        // rank the capacity Grams hold (-1: none)
  bool gram_inc = false;  // incremental updates allowed (the greedy loop)

  cr_status residual_grams(int r, double* GF, double* GX) {
    const int k = ninj + 3 * r;
    const int rc = std::max(rmax, 1);
    const int64_t K = ninj + 3 * (int64_t)rc;
    GFcap = WS(double, "resGFcap", K * K);
    GXcap = WS(double, "resGXcap", K * K);
    double* C = WS(double, "resC", (int64_t)k * std::max(k, 3));
    Blocks<T> Fall, Gall;
    Fall.clear();
    Fall.add(N, ny, ninj);
    Fall.add(U, ldu, r);
    Fall.add(LU, ny, r);
    Fall.add(L2U, ny, r);
    Gall.clear();
    Gall.add(X(), nx, ninj);
    Gall.add(L2V, nx, r);
    Gall.add(LV, nx, r);
    Gall.add(V, ldv, r);
    const int64_t cap = gemm_part_cap(P);
    if (!(gram_inc && r >= 1 && gram_r == r - 1)) {
      CR_TRY(gemm_tn<T>(ny, Fall, Fall, nullptr, nullptr, 0, C, k, gpart, cap, st));
      CR_TRY(gram_scatter(k, k, C, k, 0, 0, -1, ninj, r, rc, GFcap, K, st));
      CR_TRY(gemm_tn<T>(nx, Gall, Gall, nullptr, nullptr, 0, C, k, gpart, cap, st));
      CR_TRY(gram_scatter(k, k, C, k, 0, 0, -1, ninj, r, rc, GXcap, K, st));
    } else {
      const int j = r - 1;
      Blocks<T> Fu, Fn, Nb, Gn;
      Fu.clear();
      Fu.add(U, ldu, r);
      Fu.add(LU, ny, r);
      Fu.add(L2U, ny, r);
      Fn.clear();
      Fn.add(U + (int64_t)j * ldu, ldu, 1);
      Fn.add(LU + (int64_t)j * ny, ny, 1);
      Fn.add(L2U + (int64_t)j * ny, ny, 1);
      CR_TRY(gemm_tn<T>(ny, Fu, Fn, nullptr, nullptr, 0, C, 3 * r, gpart, cap, st));
      CR_TRY(gram_scatter(3 * r, 3, C, 3 * r, ninj, 0, j, ninj, r, rc, GFcap, K, st));
      Nb.clear();
      Nb.add(N, ny, ninj);
      CR_TRY(gemm_tn<T>(ny, Nb, Fall, nullptr, nullptr, 0, C, ninj, gpart, cap, st));
      CR_TRY(gram_scatter(ninj, k, C, ninj, 0, 0, -1, ninj, r, rc, GFcap, K, st));
      Gn.clear();
      Gn.add(L2V + (int64_t)j * nx, nx, 1);
      Gn.add(LV + (int64_t)j * nx, nx, 1);
      Gn.add(V + (int64_t)j * ldv, ldv, 1);
      CR_TRY(gemm_tn<T>(nx, Gall, Gn, nullptr, nullptr, 0, C, k, gpart, cap, st));
      CR_TRY(gram_scatter(k, 3, C, k, 0, 0, j, ninj, r, rc, GXcap, K, st));
    }
    gram_r = r;
    CR_TRY(gram_gather(k, ninj, r, rc, GFcap, K, GF, st));
    CR_TRY(gram_gather(k, ninj, r, rc, GXcap, K, GX, st));
    return CR_OK;
  }

  // Upper factor R of a tall factor Fb (columns in blocks) from its Gram Gr
  // (k x k, preserved) by CholQR2 with column scaling: Gr = S^-1 A1 S^-1,
  // A1 = L1 L1^T, Q1 = Fb S L1^-T, Q1^T Q1 = L2 L2^T, R = L2^T L1^T S^-1.
  // ok = false when a Cholesky pivot fails (columns too close to dependent,
  // or more columns than rows).  *Fc_out: the factor in FP64 (n x k, kept
  // under the tag), also on failure.
  cr_status cholqr2_r(int64_t n, const Blocks<T>& Fb, const double* Gr, int k, const char* tag,
                      double* R, bool& ok, double** Fc_out) {
    ok = false;
    const int64_t kk = (int64_t)k * k;
    const std::string t(tag);
    double* A1 = WS(double, "qrA1" + t, kk);
    double* A2 = WS(double, "qrA2" + t, kk);
    double* W1 = WS(double, "qrW1" + t, kk);
    double* W2 = WS(double, "qrW2" + t, kk);
    double* sv = WS(double, "qrs" + t, 2 * k + 8);
    double* info = sv + 2 * k;
    double* ones = sv + k;
    double* Fc = WS(double, "qrFc" + t, n * k);
    double* Q = WS(double, "qrQ", n * k);
    int off = 0;
    for (int b = 0; b < Fb.nb; ++b) {
      const int nc = Fb.col0[b + 1] - Fb.col0[b];
      CR_TRY((convert2d<double, T>(n, nc, Fb.p[b], Fb.ld[b], Fc + (int64_t)off * n, n, st)));
      off += nc;
    }
    *Fc_out = Fc;
    if (k > n) return CR_OK;
    CR_TRY((convert2d<double, double>(k, k, Gr, k, A1, k, st)));
    CR_TRY(diag_scale(k, A1, k, sv, st));
    CR_TRY(chol_lower(k, A1, k, info, st));
    double h;
    CR_TRY(read_scalars(info, 1, &h));
    if (h != 0.0) return CR_OK;
    // Q = Fc (L1^-1 diag(s))^T
    CR_TRY(trinv_lower(k, A1, k, W1, k, st));
    CR_TRY(tri_scale(k, 0, W1, k, sv, W2, k, st));
    CR_TRY(tall_small(n, k, k, Fc, n, W2, k, true, 1.0, Q, n, st));
    Blocks<double> Qb;
    Qb.clear();
    Qb.add(Q, n, k);
    CR_TRY(gemm_tn<double>(n, Qb, Qb, nullptr, nullptr, 0, A2, k, gpart, gemm_part_cap(P), st));
    CR_TRY(chol_lower(k, A2, k, info, st));
    CR_TRY(read_scalars(info, 1, &h));
    if (h != 0.0) return CR_OK;
    hipLaunchKernelGGL(k_fill, dim3(nblk(k)), dim3(256), 0, st, (int64_t)k, 1.0, ones);
    CR_HIP(hipGetLastError());
    CR_TRY(tri_scale(k, 1, A2, k, ones, W1, k, st));  // L2^T
    CR_TRY(tri_scale(k, 1, A1, k, sv, W2, k, st));    // L1^T S^-1
    CR_TRY(small_gemm(k, k, k, W1, k, false, W2, k, false, 1.0, R, k, st));
    ok = true;
    return CR_OK;
  }

  cr_status residual(int r, double* abs_out, double* rel_out) {
    const int k = ninj + 3 * r;
    const int64_t k2 = (int64_t)k * k;
    double* GF = WS(double, "resGF", k2);
    double* GX = WS(double, "resGX", k2);
    double* Cm = WS(double, "resCm", k2);
    double* M1 = WS(double, "resM1", k2);
    double* M2 = WS(double, "resM2", k2);
    CR_TRY(residual_grams(r, GF, GX));
    hipLaunchKernelGGL(k_build_cm, dim3(nblk(k2)), dim3(256), 0, st, ninj, r, Z, ldz, lam, Cm);
    CR_HIP(hipGetLastError());
    // ||R||^2 = trace(GF Cm^T GX Cm) = sum_ij GF_ij (Cm^T GX Cm)_ij
    CR_TRY(small_gemm(k, k, k, GX, k, false, Cm, k, false, 1.0, M1, k, st));
    CR_TRY(small_gemm(k, k, k, Cm, k, true, M1, k, false, 1.0, M2, k, st));
    Blocks<double> A;
    A.clear();
    A.add(GF, k2, 1);
    double* part64 = (double*)part;
    CR_TRY(gemv_t<double>(k2, A, M2, tmp + 6, part64, st));
    double h;
    CR_TRY(read_scalars(tmp + 6, 1, &h));
    double nr = std::sqrt(std::max(h, 0.0));
    // Below a relative residual of about 1e-6 the Gram form's cancellation
    // (absolute error near sqrt(eps) ||F|| ||G||) dominates: recompute from
    // the CholQR2 factors, ||R||_F = ||R_F Cm^T R_G^T||_F (error near
    // eps ||F|| ||G||)
    const double rel = P->dnorm > 0 ? nr / P->dnorm : nr;
    last_resid_qr = false;
    if (P->resid_qr == 2 || (P->resid_qr == 1 && rel < RESID_QR_SWITCH)) {
      if (k <= RESID_QR_KMAX) {
        Blocks<T> Fall, Gall;
        Fall.clear();
        Fall.add(N, ny, ninj);
        Fall.add(U, ldu, r);
        Fall.add(LU, ny, r);
        Fall.add(L2U, ny, r);
        Gall.clear();
        Gall.add(X(), nx, ninj);
        Gall.add(L2V, nx, r);
        Gall.add(LV, nx, r);
        Gall.add(V, ldv, r);
        double* RF = WS(double, "qrRF", k2);
        double* RG = WS(double, "qrRG", k2);
        bool okf = false, okg = false;
        double *Fc = nullptr, *Gc = nullptr;
        CR_TRY(cholqr2_r(ny, Fall, GF, k, "F", RF, okf, &Fc));
        CR_TRY(cholqr2_r(nx, Gall, GX, k, "G", RG, okg, &Gc));
        // R = F Cm^T G^T (G_R = G Cm).  Both factors: ||R||_F =
        // ||R_F Cm^T R_G^T||_F.  One: ||F (Cm^T R_G^T)||_F or
        // ||G (Cm R_F^T)||_F, an n x k product.  Neither (more columns than
        // rows on both sides, e.g. at full rank): the entries of R itself,
        // when n_y n_x k is moderate; else the Gram value stands.
        bool done = false;
        const double* hsrc = tmp + 7;
        if (okf && okg) {
          CR_TRY(small_gemm(k, k, k, Cm, k, true, RG, k, true, 1.0, M1, k, st));
          CR_TRY(small_gemm(k, k, k, RF, k, false, M1, k, false, 1.0, M2, k, st));
          CR_TRY(sumsq(k, k, M2, k, 1.0, part64, tmp + 7, st));
          done = true;
        } else if (okf || okg) {
          const int64_t n = okg ? ny : nx;
          double* W = WS(double, "qrQ", n * k);
          if (okg)
            CR_TRY(small_gemm(k, k, k, Cm, k, true, RG, k, true, 1.0, M1, k, st));
          else
            CR_TRY(small_gemm(k, k, k, Cm, k, false, RF, k, true, 1.0, M1, k, st));
          CR_TRY(tall_small(n, k, k, okg ? Fc : Gc, n, M1, k, false, 1.0, W, n, st));
          CR_TRY(sumsq(n, k, W, n, 1.0, part64, tmp + 7, st));
          done = true;
        } else if ((double)ny * (double)nx * (double)k <= RESID_DENSE_MAX) {
          double* W = WS(double, "qrQ", ny * k);
          double* ep = WS(double, "qrEP", entry_stats_part_size(ny, nx) + 8);
          CR_TRY(tall_small(ny, k, k, Fc, ny, Cm, k, true, 1.0, W, ny, st));  // F Cm^T
          CR_TRY(entry_stats(ny, nx, k, W, ny, Gc, nx, ep + 8, ep, st));
          hsrc = ep + 4;  // sum of the squared entries
          done = true;
        }
        if (done) {
          CR_TRY(read_scalars(hsrc, 1, &h));
          nr = std::sqrt(std::max(h, 0.0));
          last_resid_qr = true;
        }
      }
    }
    if (abs_out) *abs_out = nr;
    if (rel_out) *rel_out = P->dnorm > 0 ? nr / P->dnorm : nr;
    return CR_OK;
  }
  bool last_resid_qr = false;
};

// ===================================================================== create / destroy
// Rows of L^2 for the two-barrier PCG and the fused operator sweep
// (ring2_tables); each set is uploaded only when every row or tile fits.
static cr_status build_win2(Geom& g, const std::vector<int32_t>& nbr, bool target,
                            hipStream_t st) {
  const int K = g.K;
  // the two-barrier PCG's tables, by default for the target geometry (the
  // u-systems) only.  The v-systems' low-rank term needs the sums of all
  // workgroups' X^T z partials in every workgroup, which read more than the
  // third barrier costs (40^3 / 30^3 FP64 solve: 2.39 s with three barriers,
  // 2.34 s with the two-barrier u-systems, 3.01 s with both).
  // CONNREG_PCG_R2: 0 none, u (default) target, v source, 1 both
  const char* r2env = std::getenv("CONNREG_PCG_R2");
  const char* r2sel = r2env ? r2env : "u";
  const bool r2want = std::strcmp(r2sel, "1") == 0 ||
                      (std::strcmp(r2sel, "u") == 0 && target) ||
                      (std::strcmp(r2sel, "v") == 0 && !target);
  const Ring2Host h = ring2_tables(g.n, K, nbr.data(), r2want);
  if (!h.rows) return CR_OK;
  if (r2want) {
    if (hipMalloc(&g.r2idx, sizeof(int32_t) * h.r2idx.size()) != hipSuccess ||
        hipMalloc(&g.r2cf, h.r2cf.size()) != hipSuccess) {
      set_error("device allocation of the L^2 row tables failed");
      return CR_ENOMEM;
    }
    CR_HIP(stage_to_device(g.r2idx, h.r2idx.data(), sizeof(int32_t) * h.r2idx.size(), st));
    CR_HIP(stage_to_device(g.r2cf, h.r2cf.data(), h.r2cf.size(), st));
  }
  if (h.windows) {
    if (hipMalloc(&g.w2tab, sizeof(int32_t) * h.w2tab.size()) != hipSuccess ||
        hipMalloc(&g.w2ent, sizeof(uint32_t) * h.w2ent.size()) != hipSuccess) {
      set_error("device allocation of the ring-2 window tables failed");
      return CR_ENOMEM;
    }
    CR_HIP(stage_to_device(g.w2tab, h.w2tab.data(), sizeof(int32_t) * h.w2tab.size(), st));
    CR_HIP(stage_to_device(g.w2ent, h.w2ent.data(), sizeof(uint32_t) * h.w2ent.size(), st));
  }
  return CR_OK;
}

static cr_status build_geom(const cr_csr& L, Geom& g, const char* which, hipStream_t st) {
  const int64_t n = L.n;
  if (n <= 0 || !L.rowptr || !L.colidx || !L.val) {
    set_error(std::string(which) + ": empty or null CSR");
    return CR_EINVAL;
  }
  if (n > INT32_MAX) {
    set_error(std::string(which) + ": too many voxels");
    return CR_EINVAL;
  }
  int K = 1;
  std::vector<uint8_t> deg(n);
  for (int64_t i = 0; i < n; ++i) {
    const int b = L.rowptr[i], e = L.rowptr[i + 1];
    if (e < b) {
      set_error(std::string(which) + ": rowptr not monotone");
      return CR_EINVAL;
    }
    int off = 0;
    double diag = 0.0;
    bool has_diag = false;
    for (int k = b; k < e; ++k) {
      const int j = L.colidx[k];
      if (j < 0 || j >= n) {
        set_error(std::string(which) + ": column index out of range");
        return CR_EINVAL;
      }
      if (j == i) {
        diag = L.val[k];
        has_diag = true;
      } else {
        if (L.val[k] != -1.0) {
          set_error(std::string(which) + ": off-diagonal entries must be -1 (graph Laplacian)");
          return CR_EINVAL;
        }
        ++off;
      }
    }
    if (off > 8) {
      set_error(std::string(which) + ": more than 8 neighbours per voxel");
      return CR_EINVAL;
    }
    if ((off > 0 || has_diag) && diag != (double)off) {
      set_error(std::string(which) + ": diagonal must equal the neighbour count");
      return CR_EINVAL;
    }
    deg[i] = (uint8_t)off;
    K = std::max(K, off);
  }
  // pad the width to an even K in {2, 4, 6, 8}: extra self entries keep every
  // row exact and bound the number of kernel variants
  K = std::min(8, std::max(2, (K + 1) / 2 * 2));
  std::vector<int32_t> nbr((size_t)K * n);
  for (int64_t i = 0; i < n; ++i) {
    int c = 0;
    for (int k = L.rowptr[i]; k < L.rowptr[i + 1]; ++k) {
      const int j = L.colidx[k];
      if (j == i) continue;
      // symmetry: row j must contain i
      const int* rb = L.colidx + L.rowptr[j];
      const int* re = L.colidx + L.rowptr[j + 1];
      bool found = false;
      for (const int* q = rb; q < re; ++q)
        if (*q == i) {
          found = true;
          break;
        }
      if (!found) {
        set_error(std::string(which) + ": Laplacian not symmetric");
        return CR_EINVAL;
      }
      nbr[(size_t)c * n + i] = j;
      ++c;
    }
    for (; c < K; ++c) nbr[(size_t)c * n + i] = (int32_t)i;
  }
  g.n = n;
  g.K = K;
  if (hipMalloc(&g.nbr, sizeof(int32_t) * nbr.size()) != hipSuccess ||
      hipMalloc(&g.deg, n) != hipSuccess) {
    set_error("device allocation of the neighbour table failed");
    return CR_ENOMEM;
  }
  CR_HIP(stage_to_device(g.nbr, nbr.data(), sizeof(int32_t) * nbr.size(), st));
  CR_HIP(stage_to_device(g.deg, deg.data(), n, st));
  // window tables for the multi-column stencil (optional: left null when a
  // tile reads more than WIN_NI intervals or WIN_MAX voxels)
  const int64_t ntile = (n + NT - 1) / NT;
  std::vector<int32_t> itab((size_t)ntile * WIN_TAB, 0);
  std::vector<uint16_t> wpos((size_t)(K + 1) * n);
  std::vector<int32_t> idx;
  bool fits = true;
  for (int64_t t = 0; t < ntile && fits; ++t) {
    const int64_t t0 = t * NT, t1 = std::min(n, t0 + NT);
    idx.clear();
    for (int64_t i = t0; i < t1; ++i) {
      idx.push_back((int32_t)i);
      for (int k = 0; k < K; ++k) idx.push_back(nbr[(size_t)k * n + i]);
    }
    std::sort(idx.begin(), idx.end());
    idx.erase(std::unique(idx.begin(), idx.end()), idx.end());
    int32_t* it = itab.data() + t * WIN_TAB;
    int nint = 0, tot = 0;
    size_t a = 0;
    while (a < idx.size()) {
      size_t b = a;
      while (b + 1 < idx.size() && idx[b + 1] - idx[b] <= WIN_GAP) ++b;
      if (nint == WIN_NI) {
        fits = false;
        break;
      }
      it[2 + nint] = idx[a];
      it[2 + WIN_NI + nint] = tot;
      tot += idx[b] - idx[a] + 1;
      ++nint;
      a = b + 1;
    }
    if (!fits || tot > WIN_MAX) {
      fits = false;
      break;
    }
    it[0] = nint;
    it[1] = tot;
    auto pos = [&](int32_t j) {
      int q = 0;
      while (q + 1 < nint && it[2 + q + 1] <= j) ++q;
      return (uint16_t)(it[2 + WIN_NI + q] + (j - it[2 + q]));
    };
    for (int64_t i = t0; i < t1; ++i) {
      wpos[(size_t)i] = pos((int32_t)i);
      for (int k = 0; k < K; ++k) wpos[(size_t)(k + 1) * n + i] = pos(nbr[(size_t)k * n + i]);
    }
  }
  if (fits) {
    if (hipMalloc(&g.witab, sizeof(int32_t) * itab.size()) != hipSuccess ||
        hipMalloc(&g.wpos, sizeof(uint16_t) * wpos.size()) != hipSuccess) {
      set_error("device allocation of the window tables failed");
      return CR_ENOMEM;
    }
    CR_HIP(stage_to_device(g.witab, itab.data(), sizeof(int32_t) * itab.size(), st));
    CR_HIP(stage_to_device(g.wpos, wpos.data(), sizeof(uint16_t) * wpos.size(), st));
  }
  return build_win2(g, nbr, which[2] == 'y', st);
}

template <typename T>
static cr_status dev_alloc(cr_problem* P, T** p, int64_t count) {
  if (hipMalloc((void**)p, sizeof(T) * (size_t)std::max<int64_t>(count, 1)) != hipSuccess) {
    set_error("device allocation failed");
    return CR_ENOMEM;
  }
  P->owned.push_back(*p);
  return CR_OK;
}

static cr_status scratch_setup(int dev);

static cr_status create_impl(const cr_problem_desc* d, cr_precision prec, void* stream,
                             cr_problem* P) {
  P->st = (hipStream_t)stream;
  P->prec = prec;
  CR_HIP(hipGetDevice(&P->dev));
  CR_TRY(scratch_setup(P->dev));
  CR_HIP(hipStreamCreateWithFlags(&P->aux, hipStreamNonBlocking));
  CR_HIP(hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming));
  CR_HIP(hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming));
  if (const char* e = std::getenv("CONNREG_OP_FORK")) P->op_fork = std::atoi(e) != 0;
  if (const char* e = std::getenv("CONNREG_OP_FUSED")) P->op_fused = std::atoi(e);
  if (const char* e = std::getenv("CONNREG_PCG_BS")) P->pcg_bs = std::atoi(e) == NT ? NT : 1024;
  if (const char* e = std::getenv("CONNREG_PCG_XREG")) P->no_xreg = std::atoi(e) == 0;
  if (const char* e = std::getenv("CONNREG_PCG_XBS")) P->pcg_xbs = std::atoi(e) == NT ? NT : 512;
  if (const char* e = std::getenv("CONNREG_PCG_XLDS")) P->pcg_xlds = std::atoi(e) != 0;
  if (const char* e = std::getenv("CONNREG_PCG_XLDS_F32"))
    P->pcg_xlds_f32 = std::max(0, std::min(2, std::atoi(e)));
  if (const char* e = std::getenv("CONNREG_BATCH_XREG")) P->batch_xreg = std::atoi(e) != 0;
  if (const char* e = std::getenv("CONNREG_PCG_WARM")) P->pcg_warm = std::atoi(e) != 0;
  if (const char* e = std::getenv("CONNREG_RESID_QR")) P->resid_qr = std::max(0, std::min(2, std::atoi(e)));
  if (const char* e = std::getenv("CONNREG_GAL_LOW")) P->gal_low = std::max(-1, std::min(1, std::atoi(e)));
  if (const char* e = std::getenv("CONNREG_GAL_TILE")) P->gal_tile = std::atoi(e);
  if (const char* e = std::getenv("CONNREG_BAR_SPIN"))
    P->bar_spin = (unsigned)std::max(1L, std::min(1L << 22, std::atol(e)));
  P->ny = d->Ly.n;
  P->nx = d->Lx.n;
  P->ninj = (int)d->n_inj;
  P->lam = d->lambda;
  if (d->n_inj <= 0 || d->n_inj > 1024) {
    set_error("n_inj must be in [1, 1024]");
    return CR_EINVAL;
  }
  if (!d->X || !d->Y || !d->Omega || d->ldx < P->nx || d->ldy < P->ny || d->ldo < P->ny) {
    set_error("X, Y, Omega must be non-null with ld >= rows");
    return CR_EINVAL;
  }
  if (!(d->lambda >= 0.0) || !std::isfinite(d->lambda)) {
    set_error("lambda must be finite and >= 0");
    return CR_EINVAL;
  }
  CR_TRY(build_geom(d->Ly, P->gy, "L_y", P->st));
  CR_TRY(build_geom(d->Lx, P->gx, "L_x", P->st));
  const int64_t ny = P->ny, nx = P->nx, ni = P->ninj;
  std::vector<double> X((size_t)nx * ni), Y((size_t)ny * ni);
  std::vector<uint8_t> Om((size_t)ny * ni);
  CR_HIP(hipStreamSynchronize(P->st));
  CR_HIP(stage_to_host(X.data(), d->X, nx * sizeof(double), ni, d->ldx * sizeof(double), P->st));
  CR_HIP(stage_to_host(Y.data(), d->Y, ny * sizeof(double), ni, d->ldy * sizeof(double), P->st));
  CR_HIP(stage_to_host(Om.data(), d->Omega, ny, ni, d->ldo, P->st));
  for (double x : X)
    if (!std::isfinite(x)) {
      set_error("X has non-finite entries");
      return CR_ENONFINITE;
    }
  std::vector<double> OY((size_t)ny * ni);
  std::vector<float> OYf((size_t)ny * ni), Xf((size_t)nx * ni);
  const int nw = (int)((ni + 31) / 32);
  std::vector<uint32_t> bits((size_t)nw * ny, 0u);
  std::vector<int32_t> hptr(ni + 1, 0), hidx;
  for (int64_t a = 0; a < ni; ++a) {
    hptr[a] = (int32_t)hidx.size();
    for (int64_t i = 0; i < ny; ++i) {
      const size_t e = (size_t)a * ny + i;
      const bool obs = Om[e] != 0;
      if (obs && !std::isfinite(Y[e])) {
        set_error("Y has non-finite observed entries");
        return CR_ENONFINITE;
      }
      OY[e] = obs ? Y[e] : 0.0;
      OYf[e] = (float)OY[e];
      if (obs)
        bits[(size_t)(a / 32) * ny + i] |= 1u << (a % 32);
      else
        hidx.push_back((int32_t)i);
    }
  }
  hptr[ni] = (int32_t)hidx.size();
  for (size_t e = 0; e < X.size(); ++e) Xf[e] = (float)X[e];
  P->nholes = (int64_t)hidx.size();
  P->use_holes = P->nholes * 8 <= ny * ni;
  CR_TRY(dev_alloc(P, &P->X64, nx * ni));
  CR_TRY(dev_alloc(P, &P->X32, nx * ni));
  CR_TRY(dev_alloc(P, &P->OY64, ny * ni));
  CR_TRY(dev_alloc(P, &P->OY32, ny * ni));
  CR_TRY(dev_alloc(P, &P->bits, (int64_t)nw * ny));
  CR_TRY(dev_alloc(P, &P->hptr, ni + 1));
  CR_TRY(dev_alloc(P, &P->hidx, std::max<int64_t>(P->nholes, 1)));
  CR_HIP(stage_to_device(P->X64, X.data(), sizeof(double) * X.size(), P->st));
  CR_HIP(stage_to_device(P->X32, Xf.data(), sizeof(float) * Xf.size(), P->st));
  CR_HIP(stage_to_device(P->OY64, OY.data(), sizeof(double) * OY.size(), P->st));
  CR_HIP(stage_to_device(P->OY32, OYf.data(), sizeof(float) * OYf.size(), P->st));
  CR_HIP(stage_to_device(P->bits, bits.data(), sizeof(uint32_t) * bits.size(), P->st));
  CR_HIP(stage_to_device(P->hptr, hptr.data(), sizeof(int32_t) * hptr.size(), P->st));
  if (P->nholes)
    CR_HIP(stage_to_device(P->hidx, hidx.data(), sizeof(int32_t) * hidx.size(), P->st));
  CR_TRY(dev_alloc(P, &P->bar, BAR_WORDS));
  CR_HIP(hipMemset(P->bar, 0, BAR_WORDS * sizeof(unsigned)));
  if (const char* e = std::getenv("CONNREG_GRID_BARRIER"))
    P->bar_mode = (std::strcmp(e, "cg") == 0) ? 0 : 1;
  if (hipHostMalloc((void**)&P->hscal, 64 * sizeof(double)) != hipSuccess) {
    set_error("pinned host allocation failed");
    return CR_ENOMEM;
  }
  // ||D||_F^2 = trace((OY^T OY)(X^T X))
  double* gpart = P->buf<double>("gpart", gemm_part_cap(P));
  double* g1 = P->buf<double>("dn1", ni * ni);
  double* g2 = P->buf<double>("dn2", ni * ni);
  double* s = P->buf<double>("dns", 1);
  double* pp = P->buf<double>("part", gemv_t_part_size(ni * ni, 1) + 1);
  if (!gpart || !g1 || !g2 || !s || !pp) return CR_ENOMEM;
  Blocks<double> A, B;
  A.clear();
  A.add(P->OY64, ny, (int)ni);
  CR_TRY(gemm_tn<double>(ny, A, A, nullptr, nullptr, 0, g1, ni, gpart, gemm_part_cap(P), P->st));
  B.clear();
  B.add(P->X64, nx, (int)ni);
  CR_TRY(gemm_tn<double>(nx, B, B, nullptr, nullptr, 0, g2, ni, gpart, gemm_part_cap(P), P->st));
  Blocks<double> C;
  C.clear();
  C.add(g1, ni * ni, 1);
  CR_TRY(gemv_t<double>(ni * ni, C, g2, s, pp, P->st));
  CR_HIP(hipMemcpyAsync(P->hscal, s, sizeof(double), hipMemcpyDeviceToHost, P->st));
  CR_HIP(hipStreamSynchronize(P->st));
  P->dnorm = std::sqrt(std::max(P->hscal[0], 0.0));
  {
    double* ps = P->buf<double>("oy2part", 520);
    if (!ps) return CR_ENOMEM;
    CR_TRY(sumsq(ny, ni, P->OY64, ny, 0.5, ps, ps + 512, P->st));
    CR_HIP(hipMemcpyAsync(P->hscal, ps + 512, sizeof(double), hipMemcpyDeviceToHost, P->st));
    CR_HIP(hipStreamSynchronize(P->st));
    P->half_oy2 = P->hscal[0];
  }
  return CR_OK;
}

extern "C" cr_status cr_problem_create(const cr_problem_desc* desc, cr_precision prec,
                                       void* hip_stream, cr_problem** out) {
  if (!desc || !out) {
    set_error("null argument");
    return CR_EINVAL;
  }
  if (prec != CR_PREC_FP64 && prec != CR_PREC_MIXED) {
    set_error("unknown precision");
    return CR_EINVAL;
  }
  *out = nullptr;
  cr_problem* P = new cr_problem();
  cr_status s = create_impl(desc, prec, hip_stream, P);
  if (s != CR_OK) {
    cr_problem_destroy(P);
    return s;
  }
  *out = P;
  return CR_OK;
}

extern "C" void cr_problem_destroy(cr_problem* P) {
  if (!P) return;
  (void)hipStreamSynchronize(P->st);
  for (auto& kv : P->ws)
    if (kv.second.p) (void)hipFree(kv.second.p);
  for (void* p : P->owned) (void)hipFree(p);
  for (Geom* g : {&P->gy, &P->gx}) {
    if (g->nbr) (void)hipFree(g->nbr);
    if (g->deg) (void)hipFree(g->deg);
    if (g->witab) (void)hipFree(g->witab);
    if (g->wpos) (void)hipFree(g->wpos);
    if (g->w2tab) (void)hipFree(g->w2tab);
    if (g->w2ent) (void)hipFree(g->w2ent);
    if (g->r2idx) (void)hipFree(g->r2idx);
    if (g->r2cf) (void)hipFree(g->r2cf);
  }
  if (P->hscal) (void)hipHostFree(P->hscal);
  if (P->aux) {
    (void)hipStreamSynchronize(P->aux);
    (void)hipStreamDestroy(P->aux);
  }
  if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
  if (P->ev_join) (void)hipEventDestroy(P->ev_join);
  delete P;
}

extern "C" cr_status cr_rhs_norm(cr_problem* P, double* out) {
  if (!P || !out) {
    set_error("null argument");
    return CR_EINVAL;
  }
  *out = P->dnorm;
  return CR_OK;
}

extern "C" const char* cr_last_error(void) { return g_err.c_str(); }
extern "C" const char* cr_version(void) { return "libconnreg 0.1 (gfx950)"; }

extern "C" void cr_solve_opts_default(cr_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_rank = 20;
  o->tau_dW = 0.0;
  o->tau_res = 0.0;
  o->als_delta = 0.1;
  o->als_max_sweeps = 10;
  o->als_fixed_sweeps = 0;
  o->pcg_rtol = 1e-8;
  o->pcg_maxit = 5000;
  o->galerkin_rtol = 0.0;
  o->galerkin_maxit = 0;
  o->seed = 0;
  o->orth_tol = 1e-10;
  o->pcg_vpt = 0;
  o->verbose = 0;
}

// ===================================================================== op_apply
template <typename T>
static cr_status op_apply_check(cr_problem* P, int64_t r, const T* U, int64_t ldu, const T* Z,
                                int64_t ldz, const T* V, int64_t ldv, T* F, int64_t ldf, T* G,
                                int64_t ldg) {
  if (!P || r < 0 || (r > 0 && (!U || !Z || !V)) || !F || (r > 0 && !G)) {
    set_error("null argument or negative rank");
    return CR_EINVAL;
  }
  if ((r > 0 && (ldu < P->ny || ldv < P->nx || ldz < r || ldg < P->nx)) || ldf < P->ny) {
    set_error("leading dimension too small");
    return CR_EINVAL;
  }
  return CR_OK;
}

// The operator application on given workspace: Tm (r x n_inj, T = Z H), and
// for r > ZH_RMAX also Ht (n_inj x r) and Zd (r x r); gpart holds up to cap
// doubles of split-K partials of H = V^T X.
template <typename T>
static cr_status op_apply_run(cr_problem* P, int64_t r, const T* U, int64_t ldu, const T* Z,
                              int64_t ldz, const T* V, int64_t ldv, T* F, int64_t ldf, T* G,
                              int64_t ldg, double* Tm, double* Ht, double* Zd, double* gpart,
                              int64_t cap) {
  const int64_t ny = P->ny, nx = P->nx;
  const int ninj = P->ninj;
  hipStream_t st = P->st;
  const int rr = (int)r;
  // fork: the data term (H^T = X^T V, T = Z H, the masked product,
  // MFMA-heavy) runs on the auxiliary stream while the four stencil sweeps
  // (gather-heavy) run on the caller's stream; the caller's stream then waits
  // for both.
  CR_HIP(hipEventRecord(P->ev_fork, st));
  CR_HIP(hipStreamWaitEvent(P->aux, P->ev_fork, 0));
  // fused form: T = Z H on the auxiliary stream while the source-side sweep
  // (L_x V, L_x^2 V in one pass) runs on the caller's stream; then one
  // target-side pass writes L_y U, L_y^2 U and Omega o (U T)
  const bool fused = rr >= 1 && P->op_fused >= (sizeof(T) == 8 ? 1 : 2) &&
                     op_win2_ok<T>(P->gy, rr, ninj) && op_win2_ok<T>(P->gx, rr, 0);
  auto data_term = [&]() -> cr_status {
    hipStream_t as = P->op_fork ? P->aux : st;
    if (r > 0) {
      Blocks<T> A, B;
      A.clear();
      B.clear();
      A.add(P->X<T>(), nx, ninj);
      B.add(V, ldv, rr);
      if (rr <= ZH_RMAX) {
        // H = V^T X (V as the left operand: each column of H contiguous in
        // the partials), then T = Z H in one kernel
        int ks = 0;
        CR_TRY(gemm_tn<T>(nx, B, A, nullptr, nullptr, 0, Ht, rr, gpart, cap, as, &ks));
        CR_TRY(zh_from_partials<T>(ninj, rr, ks, gpart, Z, ldz, Tm, r, as));
      } else {
        CR_TRY(gemm_tn<T>(nx, A, B, nullptr, nullptr, 0, Ht, ninj, gpart, cap, as));
        CR_TRY((convert2d<double, T>(r, r, Z, ldz, Zd, r, as)));
        CR_TRY(small_gemm(rr, ninj, rr, Zd, r, false, Ht, ninj, true, 1.0, Tm, r, as));
      }
    }
    if (fused) return CR_OK;
    return masked_tall_gemm<T>(ny, rr, ninj, U, ldu, Tm, std::max<int64_t>(r, 1), P->bits,
                               (const T*)nullptr, 0, F + 2 * r * ldf, ldf, as);
  };
  const cr_status sd = data_term();
  cr_status ss = CR_OK;
  if (sd == CR_OK && fused) {
    ss = op_win2<T>(P->gx, rr, V, ldv, G, G + r * ldg, ldg, 0, nullptr, 0, nullptr, nullptr, 0,
                    st);
    CR_HIP(hipEventRecord(P->ev_join, P->aux));
    CR_HIP(hipStreamWaitEvent(st, P->ev_join, 0));
    if (ss == CR_OK)
      ss = op_win2<T>(P->gy, rr, U, ldu, F, F + r * ldf, ldf, ninj, Tm, r, P->bits,
                      F + 2 * r * ldf, ldf, st);
    return ss;
  }
  if (sd == CR_OK) {
    ss = stencil<T>(P->gy, rr, U, ldu, F, ldf, st);
    if (ss == CR_OK) ss = stencil<T>(P->gy, rr, F, ldf, F + r * ldf, ldf, st);
    if (ss == CR_OK) ss = stencil<T>(P->gx, rr, V, ldv, G, ldg, st);
    if (ss == CR_OK) ss = stencil<T>(P->gx, rr, G, ldg, G + r * ldg, ldg, st);
  }
  // always join, so that nothing the caller's stream owns is left in flight
  CR_HIP(hipEventRecord(P->ev_join, P->aux));
  CR_HIP(hipStreamWaitEvent(st, P->ev_join, 0));
  return sd != CR_OK ? sd : ss;
}

template <typename T>
static cr_status op_apply_impl(cr_problem* P, int64_t r, const T* U, int64_t ldu, const T* Z,
                               int64_t ldz, const T* V, int64_t ldv, T* F, int64_t ldf, T* G,
                               int64_t ldg) {
  CR_TRY(op_apply_check<T>(P, r, U, ldu, Z, ldz, V, ldv, F, ldf, G, ldg));
  const int ninj = P->ninj;
  // workspace first (allocation may synchronise)
  double* Tm = WS(double, "Tm_op", std::max<int64_t>(r, 1) * ninj);
  double* Ht = WS(double, "Ht_op", (int64_t)ninj * std::max<int64_t>(r, 1));
  double* Zd = WS(double, "Zd_op", std::max<int64_t>(r * r, 1));
  double* gpart = WS(double, "gpart", gemm_part_cap(P));
  return op_apply_run<T>(P, r, U, ldu, Z, ldz, V, ldv, F, ldf, G, ldg, Tm, Ht, Zd, gpart,
                         gemm_part_cap(P));
}

// ------------------------------------------------- allocation-free operator application
// cr_op_apply_noalloc keeps its workspace (T = Z H and the split-K partials
// of H = V^T X) in this device array instead of handle workspace.  Each
// device holds its own copy for the life of the process; its address on the
// device is looked up once per device when a handle is created there
// (hipGetSymbolAddress: the array's name in host code is not a device
// address).  Calls that overlap on one device share it and race.
constexpr int64_t NA_MAX_R = 256, NA_MAX_INJ = 256;
constexpr int64_t NA_T_DOUBLES = NA_MAX_R * NA_MAX_INJ;  // T = Z H: 512 KiB
constexpr int64_t NA_SCRATCH_DOUBLES = (int64_t)2 << 20;  // 16 MiB in all
constexpr int NA_MAX_DEV = 64;
static __device__ __align__(256) double scratch[NA_SCRATCH_DOUBLES];
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[NA_MAX_DEV] = {};

// device address of `scratch` on the current device (looked up once per device)
static cr_status scratch_setup(int dev) {
  if (dev < 0 || dev >= NA_MAX_DEV) {
    set_error("device ordinal out of range for the scratch table");
    return CR_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return CR_OK;
  double* p = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    set_error(std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    return CR_EHIP;
  }
  g_scratch_ptr[dev] = p;
  return CR_OK;
}

extern "C" cr_status cr_op_apply_noalloc(cr_problem* P, int64_t r, const double* U, int64_t ldu,
                                         const double* Z, int64_t ldz, const double* V,
                                         int64_t ldv, double* F, int64_t ldf, double* G,
                                         int64_t ldg) {
  CR_TRY(op_apply_check<double>(P, r, U, ldu, Z, ldz, V, ldv, F, ldf, G, ldg));
  if (r > NA_MAX_R || P->ninj > NA_MAX_INJ) {
    set_error("cr_op_apply_noalloc: r = " + std::to_string(r) + ", n_inj = " +
              std::to_string(P->ninj) + " beyond the static scratch limits (r <= " +
              std::to_string(NA_MAX_R) + ", n_inj <= " + std::to_string(NA_MAX_INJ) + ")");
    return CR_EINVAL;
  }
  double* base = (P->dev >= 0 && P->dev < NA_MAX_DEV) ? g_scratch_ptr[P->dev] : nullptr;
  if (!base) {
    set_error("cr_op_apply_noalloc: scratch address of the handle's device not set up");
    return CR_EHIP;
  }
  return op_apply_run<double>(P, r, U, ldu, Z, ldz, V, ldv, F, ldf, G, ldg, base, nullptr, nullptr,
                              base + NA_T_DOUBLES, NA_SCRATCH_DOUBLES - NA_T_DOUBLES);
}

extern "C" cr_status cr_op_apply(cr_problem* P, int64_t r, const double* U, int64_t ldu,
                                 const double* Z, int64_t ldz, const double* V, int64_t ldv,
                                 double* F, int64_t ldf, double* G, int64_t ldg) {
  return op_apply_impl<double>(P, r, U, ldu, Z, ldz, V, ldv, F, ldf, G, ldg);
}

extern "C" cr_status cr_op_apply_f32(cr_problem* P, int64_t r, const float* U, int64_t ldu,
                                     const float* Z, int64_t ldz, const float* V, int64_t ldv,
                                     float* F, int64_t ldf, float* G, int64_t ldg) {
  return op_apply_impl<float>(P, r, U, ldu, Z, ldz, V, ldv, F, ldf, G, ldg);
}

// A(U Z V^T) = F G^T with k = 3r + n_inj columns (eq. multitermSylv, each
// term kept in factored form):
//   F = [lam U | 2 lam L_y U | lam L_y^2 U | Omega o (U Z H)],
//   G = [L_x^2 V Z^T | L_x V Z^T | V Z^T | X].
// The operator's products come from op_apply_impl (written straight into F's
// middle blocks); G's stencil blocks pass through workspace.
extern "C" cr_status cr_op_apply_factors(cr_problem* P, int64_t r, const double* U, int64_t ldu,
                                         const double* Z, int64_t ldz, const double* V,
                                         int64_t ldv, double* F, int64_t ldf, double* G,
                                         int64_t ldg) {
  if (!P || r < 0 || (r > 0 && (!U || !Z || !V)) || !F || !G) {
    set_error("null argument or negative rank");
    return CR_EINVAL;
  }
  const int64_t ny = P->ny, nx = P->nx;
  if (ldf < ny || ldg < nx || (r > 0 && (ldu < ny || ldv < nx || ldz < r))) {
    set_error("leading dimension too small");
    return CR_EINVAL;
  }
  hipStream_t st = P->st;
  const int rr = (int)r;
  double* Gs = WS(double, "G_fac", nx * std::max<int64_t>(2 * r, 1));
  CR_TRY(op_apply_impl<double>(P, r, U, ldu, Z, ldz, V, ldv, F + r * ldf, ldf, Gs, nx));
  const double lam = P->lam;
  if (r > 0) {
    // F's blocks scaled in place; G's blocks are (.) Z^T
    CR_TRY(tall_small(ny, rr, rr, U, ldu, nullptr, 0, false, lam, F, ldf, st));
    CR_TRY(tall_small(ny, rr, rr, F + r * ldf, ldf, nullptr, 0, false, 2.0 * lam, F + r * ldf, ldf,
                      st));
    CR_TRY(tall_small(ny, rr, rr, F + 2 * r * ldf, ldf, nullptr, 0, false, lam, F + 2 * r * ldf,
                      ldf, st));
    CR_TRY(tall_small(nx, rr, rr, Gs + r * nx, nx, Z, ldz, true, 1.0, G, ldg, st));
    CR_TRY(tall_small(nx, rr, rr, Gs, nx, Z, ldz, true, 1.0, G + r * ldg, ldg, st));
    CR_TRY(tall_small(nx, rr, rr, V, ldv, Z, ldz, true, 1.0, G + 2 * r * ldg, ldg, st));
  }
  CR_TRY((convert2d<double, double>(nx, P->ninj, P->X64, nx, G + 3 * r * ldg, ldg, st)));
  return CR_OK;
}

// ===================================================================== post-processing
// Host copy of `count` device doubles through the handle's pinned scratch.
static cr_status read_scalars(cr_problem* P, const double* dev, double* host, int count) {
  CR_HIP(hipMemcpyAsync(P->hscal, dev, sizeof(double) * count, hipMemcpyDeviceToHost, P->st));
  CR_HIP(hipStreamSynchronize(P->st));
  std::memcpy(host, P->hscal, sizeof(double) * count);
  return CR_OK;
}

static bool post_args_ok(cr_problem* P, int64_t r, const double* U, int64_t ldu, const double* Z,
                         int64_t ldz, const double* V, int64_t ldv) {
  if (!P || r < 1 || !U || !Z || !V || ldu < P->ny || ldv < P->nx || ldz < r) {
    set_error("null argument, r < 1 or leading dimension too small");
    return false;
  }
  return true;
}

// SVD of W = U Z V^T from the SVD of its core (section on the top-view
// results): Z = Zu diag(s) Zv^T by one-sided Jacobi, then Uh = U Zu, Vh = V Zv.
extern "C" cr_status cr_core_svd(cr_problem* P, int64_t r, const double* U, int64_t ldu,
                                 const double* Z, int64_t ldz, const double* V, int64_t ldv,
                                 double* Uh, int64_t lduh, double* s, double* Vh, int64_t ldvh,
                                 int32_t* sweeps_out) {
  if (!post_args_ok(P, r, U, ldu, Z, ldz, V, ldv)) return CR_EINVAL;
  if (!Uh || !s || !Vh || lduh < P->ny || ldvh < P->nx) {
    set_error("cr_core_svd: null output or leading dimension too small");
    return CR_EINVAL;
  }
  hipStream_t st = P->st;
  const int rr = (int)r;
  double* A = WS(double, "svd_A", r * r);
  double* Zu = WS(double, "svd_Zu", r * r);
  double* Zv = WS(double, "svd_Zv", r * r);
  double* work = WS(double, "svd_work", r * r + r + 8);
  CR_TRY((convert2d<double, double>(r, r, Z, ldz, A, r, st)));
  double* info = work + r * r + r;
  CR_TRY(small_svd(rr, A, r, Zu, r, s, Zv, r, work, info, st));
  CR_TRY(tall_small(P->ny, rr, rr, U, ldu, Zu, r, false, 1.0, Uh, lduh, st));
  CR_TRY(tall_small(P->nx, rr, rr, V, ldv, Zv, r, false, 1.0, Vh, ldvh, st));
  double h[2];
  CR_TRY(read_scalars(P, info, h, 2));
  if (sweeps_out) *sweeps_out = (int32_t)h[0];
  if (h[1] != 1.0) {
    set_error("one-sided Jacobi SVD of the core did not converge");
    return CR_NOTCONV;
  }
  return CR_OK;
}

// J(W) of eq. obj_fun for W = U Z V^T, FP64: misfit 1/2 ||Omega o Y -
// Omega o (U Z H)||_F^2 (H = V^T X) and regulariser lambda/2 ||F G^T||_F^2 with
// F = [L_y U | U], G = [V Z^T | L_x V Z^T] (L_y W + W L_x^T in factored form),
// the latter through the Grams F^T F and G^T G.
extern "C" cr_status cr_objective(cr_problem* P, int64_t r, const double* U, int64_t ldu,
                                  const double* Z, int64_t ldz, const double* V, int64_t ldv,
                                  double* out3) {
  if (!post_args_ok(P, r, U, ldu, Z, ldz, V, ldv)) return CR_EINVAL;
  if (!out3) {
    set_error("cr_objective: null output");
    return CR_EINVAL;
  }
  hipStream_t st = P->st;
  const int rr = (int)r, ninj = P->ninj;
  const int64_t ny = P->ny, nx = P->nx;
  if (rr > ZH_RMAX) {
    set_error("cr_objective: r beyond the supported range");
    return CR_EINVAL;
  }
  double* Tm = WS(double, "obj_T", r * ninj);
  double* gpart = WS(double, "gpart", gemm_part_cap(P));
  double* N = WS(double, "obj_N", ny * ninj);
  double* LyU = WS(double, "obj_LyU", ny * r);
  double* LxV = WS(double, "obj_LxV", nx * r);
  double* Gm = WS(double, "obj_G", nx * 2 * r);
  double* FtF = WS(double, "obj_FtF", 4 * r * r);
  double* GtG = WS(double, "obj_GtG", 4 * r * r);
  double* sc = WS(double, "obj_sc", 512 + 8);
  // misfit
  {
    Blocks<double> A, B;
    A.clear();
    B.clear();
    A.add(P->X64, nx, ninj);
    B.add(V, ldv, rr);
    int ks = 0;
    CR_TRY(gemm_tn<double>(nx, B, A, nullptr, nullptr, 0, nullptr, rr, gpart, gemm_part_cap(P), st,
                           &ks));
    CR_TRY(zh_from_partials<double>(ninj, rr, ks, gpart, Z, ldz, Tm, r, st));
    CR_TRY(masked_tall_gemm<double>(ny, rr, ninj, U, ldu, Tm, r, P->bits, P->OY64, ny, N, ny, st));
    CR_TRY(sumsq(ny, ninj, N, ny, 0.5, sc, sc + 512, st));
  }
  // regulariser
  CR_TRY(stencil<double>(P->gy, rr, U, ldu, LyU, ny, st));
  CR_TRY(stencil<double>(P->gx, rr, V, ldv, LxV, nx, st));
  CR_TRY(tall_small(nx, rr, rr, V, ldv, Z, ldz, true, 1.0, Gm, nx, st));
  CR_TRY(tall_small(nx, rr, rr, LxV, nx, Z, ldz, true, 1.0, Gm + r * nx, nx, st));
  {
    Blocks<double> F, G;
    F.clear();
    F.add(LyU, ny, rr);
    F.add(U, ldu, rr);
    G.clear();
    G.add(Gm, nx, 2 * rr);
    CR_TRY(gemm_tn<double>(ny, F, F, nullptr, nullptr, 0, FtF, 2 * r, gpart, gemm_part_cap(P), st));
    CR_TRY(gemm_tn<double>(nx, G, G, nullptr, nullptr, 0, GtG, 2 * r, gpart, gemm_part_cap(P), st));
  }
  CR_TRY(trace_prod(2 * rr, FtF, 2 * r, GtG, 2 * r, 0.5 * P->lam, sc + 513, st));
  double h[2];
  CR_TRY(read_scalars(P, sc + 512, h, 2));
  out3[0] = h[0] + h[1];
  out3[1] = h[0];
  out3[2] = h[1];
  return CR_OK;
}

// Statistics over every entry of W = U Z V^T (section on dropping the
// nonnegativity constraint), without forming W: A = U Z, then W = A V^T
// tile by tile on the FP64 matrix cores.
extern "C" cr_status cr_entry_stats(cr_problem* P, int64_t r, const double* U, int64_t ldu,
                                    const double* Z, int64_t ldz, const double* V, int64_t ldv,
                                    cr_entry_stats_t* out) {
  if (!post_args_ok(P, r, U, ldu, Z, ldz, V, ldv)) return CR_EINVAL;
  if (!out) {
    set_error("cr_entry_stats: null output");
    return CR_EINVAL;
  }
  hipStream_t st = P->st;
  const int rr = (int)r;
  const int64_t ny = P->ny, nx = P->nx;
  double* A = WS(double, "es_A", ny * r);
  double* part = WS(double, "es_part", entry_stats_part_size(ny, nx) + 8);
  double* res = WS(double, "es_res", 8);
  CR_TRY(tall_small(ny, rr, rr, U, ldu, Z, ldz, false, 1.0, A, ny, st));
  CR_TRY(entry_stats(ny, nx, rr, A, ny, V, ldv, part, res, st));
  double h[6];
  CR_TRY(read_scalars(P, res, h, 6));
  out->count_neg = h[0];
  out->min = h[1];
  out->max = h[2];
  out->max_abs = h[3];
  out->sum_sq = h[4];
  out->sum_sq_neg = h[5];
  out->entries = (double)ny * (double)nx;
  return CR_OK;
}

// ===================================================================== iterate setup
// Bring an external iterate (double U, Z, V) into ctx: bases in T (copied when
// T is float or the leading dimensions differ), core copied to ld r, derived
// stencils, H^T and N.
template <typename T>
static cr_status load_iterate(Ctx<T>& c, int r, const double* U, int64_t ldu, const double* Z,
                              int64_t ldz, const double* V, int64_t ldv, bool need_N) {
  cr_problem* P = c.P;
  const int64_t ny = c.ny, nx = c.nx;
  c.U = WS(T, "U_in", ny * std::max(r, 1));
  c.V = WS(T, "V_in", nx * std::max(r, 1));
  c.ldu = ny;
  c.ldv = nx;
  if (r > 0) {
    CR_TRY((convert2d<T, double>(ny, r, U, ldu, c.U, ny, c.st)));
    CR_TRY((convert2d<T, double>(nx, r, V, ldv, c.V, nx, c.st)));
  }
  c.Z = WS(double, "Z_in", (int64_t)std::max(r, 1) * std::max(r, 1));
  c.ldz = std::max(r, 1);
  if (r > 0 && Z) CR_TRY((convert2d<double, double>(r, r, Z, ldz, c.Z, r, c.st)));
  CR_TRY(c.alloc_rank(std::max(r, 1)));
  if (r > 0) CR_TRY(c.stencil_cols(0, r));
  if (need_N) {
    CR_TRY(c.compute_Ht(r));
    CR_TRY(c.build_N(r));
  }
  return CR_OK;
}

template <typename T>
static cr_status als_step_impl(cr_problem* P, int64_t r, const double* U, int64_t ldu,
                               const double* Z, int64_t ldz, const double* V, int64_t ldv,
                               double* v_io, double* u_out, const cr_solve_opts* opts,
                               cr_als_stats* stats) {
  cr_solve_opts o;
  if (opts)
    o = *opts;
  else
    cr_solve_opts_default(&o);
  Ctx<T> c(P);
  CR_TRY(load_iterate<T>(c, (int)r, U, ldu, Z, ldz, V, ldv, true));
  CR_TRY(c.alloc_vectors(o.pcg_vpt));
  CR_TRY((convert2d<T, double>(c.nx, 1, v_io, c.nx, c.vv, c.nx, c.st)));
  // normalise the initial vector
  CR_TRY(c.dot(c.nx, c.vv, c.vv, c.tmp + 7));
  CR_TRY(scale_inv_sqrt<T>(c.nx, c.vv, c.tmp + 7, c.st));
  bool zero = false;
  CR_TRY(c.als((int)r, c.vv, c.vu, o, stats, zero));
  CR_TRY((convert2d<double, T>(c.nx, 1, c.vv, c.nx, v_io, c.nx, c.st)));
  CR_TRY((convert2d<double, T>(c.ny, 1, c.vu, c.ny, u_out, c.ny, c.st)));
  CR_HIP(hipStreamSynchronize(c.st));
  if (zero) {
    set_error("ALS right-hand side vanished");
    return CR_BREAKDOWN;
  }
  return c.notconv ? CR_NOTCONV : CR_OK;
}

extern "C" cr_status cr_als_step(cr_problem* P, int64_t r, const double* U, int64_t ldu,
                                 const double* Z, int64_t ldz, const double* V, int64_t ldv,
                                 double* v_io, double* u_out, const cr_solve_opts* opts,
                                 cr_als_stats* stats) {
  if (!P || r < 0 || !v_io || !u_out || (r > 0 && (!U || !Z || !V))) {
    set_error("null argument or negative rank");
    return CR_EINVAL;
  }
  return P->prec == CR_PREC_MIXED
             ? als_step_impl<float>(P, r, U, ldu, Z, ldz, V, ldv, v_io, u_out, opts, stats)
             : als_step_impl<double>(P, r, U, ldu, Z, ldz, V, ldv, v_io, u_out, opts, stats);
}

template <typename T>
static cr_status galerkin_impl(cr_problem* P, int64_t r, const double* U, int64_t ldu,
                               const double* V, int64_t ldv, double* Z_io, int64_t ldz,
                               double rtol, int32_t maxit, int32_t* iters_out) {
  Ctx<T> c(P);
  CR_TRY(load_iterate<T>(c, (int)r, U, ldu, Z_io, ldz, V, ldv, false));
  const int rr = (int)r;
  const int64_t ldr = rr;
  // projected data in ld r
  for (double* B : {c.By1, c.By2, c.Bx1, c.Bx2}) CR_HIP(hipMemsetAsync(B, 0, sizeof(double) * ldr * ldr, c.st));
  CR_TRY(c.alloc_vectors(0));
  for (int j = 0; j < rr; ++j) CR_TRY(c.project_column(j, ldr));
  double s[4];
  CR_TRY(c.galerkin(rr, ldr, rtol, maxit > 0 ? maxit : 50 * rr + 200, s));
  CR_TRY((convert2d<double, double>(r, r, c.Z, r, Z_io, ldz, c.st)));
  CR_HIP(hipStreamSynchronize(c.st));
  if (iters_out) *iters_out = (int32_t)s[0];
  if (s[2] == PERSIST_TIMEOUT) {
    set_error("grid barrier timed out in the projected CG kernel");
    return CR_EHIP;
  }
  if (s[2] == 2.0) {
    set_error("projected operator not positive definite on a CG direction");
    return CR_ENONFINITE;
  }
  return s[2] == 1.0 ? CR_NOTCONV : CR_OK;
}

extern "C" cr_status cr_galerkin_project(cr_problem* P, int64_t r, const double* U, int64_t ldu,
                                         const double* V, int64_t ldv, double* Z_io, int64_t ldz,
                                         double rtol, int32_t maxit, int32_t* iters_out) {
  if (!P || r <= 0 || !U || !V || !Z_io || ldu < P->ny || ldv < P->nx || ldz < r) {
    set_error("invalid arguments to cr_galerkin_project");
    return CR_EINVAL;
  }
  return P->prec == CR_PREC_MIXED
             ? galerkin_impl<float>(P, r, U, ldu, V, ldv, Z_io, ldz, rtol, maxit, iters_out)
             : galerkin_impl<double>(P, r, U, ldu, V, ldv, Z_io, ldz, rtol, maxit, iters_out);
}

template <typename T>
static cr_status residual_impl(cr_problem* P, int64_t r, const double* U, int64_t ldu,
                               const double* Z, int64_t ldz, const double* V, int64_t ldv,
                               double* abs_out, double* rel_out) {
  Ctx<T> c(P);
  CR_TRY(load_iterate<T>(c, (int)r, U, ldu, Z, ldz, V, ldv, true));
  CR_TRY(c.alloc_vectors(0));
  return c.residual((int)r, abs_out, rel_out);
}

extern "C" cr_status cr_residual_norm(cr_problem* P, int64_t r, const double* U, int64_t ldu,
                                      const double* Z, int64_t ldz, const double* V, int64_t ldv,
                                      double* abs_out, double* rel_out) {
  if (!P || r < 0 || (r > 0 && (!U || !Z || !V || ldu < P->ny || ldv < P->nx || ldz < r))) {
    set_error("invalid arguments to cr_residual_norm");
    return CR_EINVAL;
  }
  return P->prec == CR_PREC_MIXED
             ? residual_impl<float>(P, r, U, ldu, Z, ldz, V, ldv, abs_out, rel_out)
             : residual_impl<double>(P, r, U, ldu, Z, ldz, V, ldv, abs_out, rel_out);
}

// ===================================================================== greedy solve
template <typename T>
static cr_status greedy_impl(cr_problem* P, const cr_solve_opts& o, double* Uo, double* Vo,
                             double* Zo, int64_t* rank_io, cr_solve_stats* stats, cr_rank_cb cb,
                             void* user) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  const int rmax = o.max_rank;
  const int64_t ny = P->ny, nx = P->nx;
  Ctx<T> c(P);
  c.gram_inc = true;  // one basis column per rank: residual Grams updated incrementally
  CR_TRY(c.alloc_rank(rmax));
  CR_TRY(c.alloc_vectors(o.pcg_vpt));
  // bases: the caller's buffers directly in FP64, internal copies otherwise
  if (std::is_same<T, double>::value) {
    c.U = (T*)Uo;
    c.V = (T*)Vo;
  } else {
    c.U = WS(T, "Ug", ny * rmax);
    c.V = WS(T, "Vg", nx * rmax);
  }
  c.ldu = ny;
  c.ldv = nx;
  c.Z = Zo;
  c.ldz = rmax;
  const int64_t ldr = rmax;
  double* Zold = WS(double, "Zold", (int64_t)rmax * rmax);
  double* dws = WS(double, "dws", 2 + 2 * DW_MAXWG);
  int r0 = (int)*rank_io;
  if (r0 < 0 || r0 > rmax) {
    set_error("rank_io out of range");
    return CR_EINVAL;
  }
  // clear everything beyond the resumed core
  std::vector<double> hz((size_t)rmax * rmax, 0.0);
  if (r0 > 0) {
    CR_HIP(hipMemcpy2DAsync(hz.data(), rmax * sizeof(double), Zo, rmax * sizeof(double),
                            r0 * sizeof(double), r0, hipMemcpyDeviceToHost, c.st));
    CR_HIP(hipStreamSynchronize(c.st));
  }
  CR_HIP(hipMemcpyAsync(Zo, hz.data(), sizeof(double) * hz.size(), hipMemcpyHostToDevice, c.st));
  for (double* B : {c.By1, c.By2, c.Bx1, c.Bx2})
    CR_HIP(hipMemsetAsync(B, 0, sizeof(double) * ldr * ldr, c.st));
  CR_HIP(hipMemsetAsync(c.G, 0, sizeof(double) * ldr * ldr * c.ninj, c.st));
  if (r0 > 0) {
    if (!std::is_same<T, double>::value) {
      CR_TRY((convert2d<T, double>(ny, r0, Uo, ny, c.U, ny, c.st)));
      CR_TRY((convert2d<T, double>(nx, r0, Vo, nx, c.V, nx, c.st)));
    }
    CR_TRY(c.stencil_cols(0, r0));
    for (int j = 0; j < r0; ++j) CR_TRY(c.project_column(j, ldr));
  }
  CR_TRY(c.build_N(r0));
  const double tau = o.tau_res > 0 ? o.tau_res : o.tau_dW;
  const double g_rtol = o.galerkin_rtol > 0 ? o.galerkin_rtol : std::max(tau, 1e-14) / 2;
  cr_status final_status = CR_OK;
  int r = r0;
  double relres = 1.0, dW = 1.0;
  int64_t tot_pcg = 0, tot_gal = 0;
  int tot_notconv = 0;
  if (r0 > 0) CR_TRY(c.residual(r0, nullptr, &relres));
  bool stop = (o.tau_res > 0 && r0 > 0 && relres <= o.tau_res);
  while (!stop && r < rmax) {
    const int j = r;
    // initial ALS vector: v = R^T q / ||R^T q||, q from SplitMix64 stream j
    CR_TRY(splitmix_fill<T>(ny, o.seed, (uint64_t)j, c.vu, c.st));
    CR_TRY(c.apply_RT(j, c.vu, c.vv));
    CR_TRY(c.dot(nx, c.vv, c.vv, c.tmp + 7));
    CR_TRY(scale_inv_sqrt<T>(nx, c.vv, c.tmp + 7, c.st));
    cr_als_stats as{};
    bool zero = false;
    CR_TRY(c.als(j, c.vv, c.vu, o, &as, zero));
    tot_pcg += as.pcg_iters_u + as.pcg_iters_v;
    tot_notconv += as.pcg_notconv;
    if (zero) {
      final_status = CR_BREAKDOWN;
      break;
    }
    // U_{j+1} = orth([U_j, u]), V_{j+1} = orth([V_j, v]) by CGS2 into column j
    T* uj = c.U + (int64_t)j * ny;
    T* vj = c.V + (int64_t)j * nx;
    CR_HIP(hipMemcpyAsync(uj, c.vu, sizeof(T) * ny, hipMemcpyDeviceToDevice, c.st));
    CR_HIP(hipMemcpyAsync(vj, c.vv, sizeof(T) * nx, hipMemcpyDeviceToDevice, c.st));
    bool bu = false, bv = false;
    CR_TRY(c.cgs2(ny, c.U, ny, j, uj, o.orth_tol, bu));
    CR_TRY(c.cgs2(nx, c.V, nx, j, vj, o.orth_tol, bv));
    if (bu || bv) {
      final_status = CR_BREAKDOWN;
      break;
    }
    CR_TRY(c.stencil_cols(j, 1));
    CR_TRY(c.project_column(j, ldr));
    // Galerkin update from the padded previous core (row/column j are zero)
    CR_HIP(hipMemcpyAsync(Zold, Zo, sizeof(double) * ldr * ldr, hipMemcpyDeviceToDevice, c.st));
    double gs[4];
    const int gmax = o.galerkin_maxit > 0 ? o.galerkin_maxit : 50 * (j + 1) + 200;
    CR_TRY(c.galerkin(j + 1, ldr, g_rtol, gmax, gs));
    if (gs[2] == PERSIST_TIMEOUT) {
      set_error("grid barrier timed out in the projected CG kernel");
      return CR_EHIP;
    }
    if (gs[2] == 2.0) {
      set_error("projected operator not positive definite on a CG direction");
      return CR_ENONFINITE;
    }
    tot_gal += (int64_t)gs[0];
    r = j + 1;
    CR_TRY(c.build_N(r));
    CR_TRY(c.residual(r, nullptr, &relres));
    // delta W = ||Z_j - pad(Z_{j-1})||_F / ||Z_j||_F (orthonormal bases)
    {
      const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(DW_MAXWG, ((int64_t)r * r + 2047) / 2048));
      hipLaunchKernelGGL(k_dw, dim3(nb), dim3(NT), 0, c.st, r, ldr, Zo, Zold, dws + 2);
      CR_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_dw_final, dim3(1), dim3(64), 0, c.st, nb, dws + 2, dws);
      CR_HIP(hipGetLastError());
    }
    CR_HIP(hipMemcpyAsync(P->hscal, dws, 2 * sizeof(double), hipMemcpyDeviceToHost, c.st));
    CR_HIP(hipStreamSynchronize(c.st));
    const double dd = P->hscal[0], zz = P->hscal[1];
    dW = zz > 0 ? std::sqrt(dd / zz) : 0.0;
    const double secs = std::chrono::duration<double>(clk::now() - t0).count();
    if (!std::isfinite(relres)) {
      set_error("non-finite residual");
      return CR_ENONFINITE;
    }
    if (o.verbose)
      std::fprintf(stderr,
                   "[connreg] rank %3d relres %.3e dW %.3e E %.6e sweeps %d pcg %d/%d gal %d  %.3fs\n",
                   r, relres, dW, gs[3], as.sweeps, as.pcg_iters_u, as.pcg_iters_v, (int)gs[0],
                   secs);
    if (cb) {
      cr_rank_info info{};
      info.rank = r;
      info.relres = relres;
      info.dW = dW;
      info.energy = gs[3];
      info.J = gs[3] + P->half_oy2;
      info.sweeps = as.sweeps;
      info.pcg_iters = as.pcg_iters_u + as.pcg_iters_v;
      info.galerkin_iters = (int)gs[0];
      info.seconds = secs;
      cb(&info, user);
    }
    if ((o.tau_res > 0 && relres <= o.tau_res) || (o.tau_dW > 0 && dW <= o.tau_dW)) stop = true;
  }
  if (!stop && final_status == CR_OK && (o.tau_res > 0 || o.tau_dW > 0)) final_status = CR_NOTCONV;
  if (!std::is_same<T, double>::value && r > 0) {
    CR_TRY((convert2d<double, T>(ny, r, c.U, ny, Uo, ny, c.st)));
    CR_TRY((convert2d<double, T>(nx, r, c.V, nx, Vo, nx, c.st)));
  }
  CR_HIP(hipStreamSynchronize(c.st));
  *rank_io = r;
  if (stats) {
    stats->rank = r;
    stats->relres = relres;
    stats->dW = dW;
    stats->pcg_iters = tot_pcg;
    stats->galerkin_iters = tot_gal;
    stats->pcg_notconv = tot_notconv;
    stats->seconds = std::chrono::duration<double>(clk::now() - t0).count();
  }
  return final_status;
}

extern "C" cr_status cr_greedy_solve(cr_problem* P, const cr_solve_opts* opts, double* U,
                                     double* V, double* Z, int64_t* rank_io,
                                     cr_solve_stats* stats, cr_rank_cb cb, void* user) {
  if (!P || !opts || !U || !V || !Z || !rank_io) {
    set_error("null argument");
    return CR_EINVAL;
  }
  if (opts->max_rank <= 0 || opts->max_rank > std::min<int64_t>(std::min(P->nx, P->ny), 2000)) {
    set_error("max_rank must be in [1, min(n_x, n_y, 2000)]");
    return CR_EINVAL;
  }
  if (opts->pcg_maxit <= 0 || !(opts->pcg_rtol > 0)) {
    set_error("pcg_maxit and pcg_rtol must be positive");
    return CR_EINVAL;
  }
  return P->prec == CR_PREC_MIXED
             ? greedy_impl<float>(P, *opts, U, V, Z, rank_io, stats, cb, user)
             : greedy_impl<double>(P, *opts, U, V, Z, rank_io, stats, cb, user);
}

// ===================================================================== u-systems and the network
extern "C" cr_status cr_problem_set_pc(cr_problem* P, cr_pc* pc) {
  if (!P) {
    set_error("null handle");
    return CR_EINVAL;
  }
  if (pc) {
    const int64_t N = (int64_t)pc->net.nx * pc->net.ny * pc->net.nz;
    if (N != P->ny) {
      set_error("the network's box must match the target grid");
      return CR_EINVAL;
    }
  }
  P->pc = pc;
  P->fcg_mode = pc ? 2 : 0;
  P->pc_fallbacks = 0;
  return CR_OK;
}

extern "C" cr_status cr_problem_set_precond(cr_problem* P, int32_t kind) {
  if (!P || kind < 0 || kind > 2 || (kind == 2 && !P->pc)) {
    set_error("precond must be 0 (Jacobi-PCG), 1 (flexible CG with the base step) or 2 "
              "(flexible CG with the learned network, after cr_problem_set_pc)");
    return CR_EINVAL;
  }
  P->fcg_mode = kind;
  return CR_OK;
}

// Target (which 0) or source (which 1) grid as a full d0 x d1 x d2 box
// (first axis fastest): checks that the Laplacian is the box's free-face
// 7-point Laplacian, then builds the per-axis DCT-II bases used by the
// spectral base step (target) and the SMW v-solve (source).
extern "C" cr_status cr_problem_set_box(cr_problem* P, int32_t which, const int32_t* dims) {
  if (!P || (which != 0 && which != 1)) {
    set_error("which must be 0 (target) or 1 (source)");
    return CR_EINVAL;
  }
  const Geom& geo = which == 0 ? P->gy : P->gx;
  if (!dims || dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0 ||
      (int64_t)dims[0] * dims[1] * dims[2] != geo.n) {
    set_error("box dimensions must be positive and multiply to the number of voxels");
    return CR_EINVAL;
  }
  const int64_t n = geo.n;
  const int K = geo.K;
  std::vector<int32_t> nbr((size_t)K * n);
  CR_HIP(stage_to_host(nbr.data(), geo.nbr, sizeof(int32_t) * nbr.size(), 1, 0, P->st));
  const int d0 = dims[0], d1 = dims[1], d2 = dims[2];
  for (int64_t i = 0; i < n; ++i) {
    const int i0 = (int)(i % d0), i1 = (int)((i / d0) % d1), i2 = (int)(i / ((int64_t)d0 * d1));
    int64_t want[6];
    int nw = 0;
    if (i0 > 0) want[nw++] = i - 1;
    if (i0 + 1 < d0) want[nw++] = i + 1;
    if (i1 > 0) want[nw++] = i - d0;
    if (i1 + 1 < d1) want[nw++] = i + d0;
    if (i2 > 0) want[nw++] = i - (int64_t)d0 * d1;
    if (i2 + 1 < d2) want[nw++] = i + (int64_t)d0 * d1;
    int have = 0;
    for (int k = 0; k < K; ++k) {
      const int64_t j = nbr[(size_t)k * n + i];
      if (j == i) continue;
      bool found = false;
      for (int m = 0; m < nw; ++m) found = found || want[m] == j;
      if (!found) {
        set_error("the Laplacian is not the box's 7-point Laplacian");
        return CR_EINVAL;
      }
      ++have;
    }
    if (have != nw) {
      set_error("the Laplacian is not the box's 7-point Laplacian");
      return CR_EINVAL;
    }
  }
  BoxBasis bx;
  bx.valid = true;
  for (int a = 0; a < 3; ++a) {
    const int m = dims[a];
    bx.dims[a] = m;
    std::vector<double> Q((size_t)m * m), mu(m);
    for (int k = 0; k < m; ++k) {
      const double c = k == 0 ? std::sqrt(1.0 / m) : std::sqrt(2.0 / m);
      for (int j = 0; j < m; ++j) Q[(size_t)j * m + k] = c * std::cos(M_PI * k * (j + 0.5) / m);
      mu[k] = 2.0 - 2.0 * std::cos(M_PI * k / m);
    }
    CR_TRY(dev_alloc(P, &bx.Q[a], (int64_t)m * m));
    CR_TRY(dev_alloc(P, &bx.mu[a], m));
    CR_HIP(stage_to_device(bx.Q[a], Q.data(), sizeof(double) * Q.size(), P->st));
    CR_HIP(stage_to_device(bx.mu[a], mu.data(), sizeof(double) * m, P->st));
  }
  (which == 0 ? P->boxy : P->boxx) = bx;
  if (which != 0) P->smw_xh_ready = false;
  return CR_OK;
}

// ===================================================================== two-level set-up
// Aggregates = the source voxels grouped by cubes of `block` voxels per axis
// of their coordinates; packed whole into workgroups (in cube order) for
// 256- and 512-thread launches; coarse geometry C1 = P^T L P and C2 =
// (L P)^T (L P) from the neighbour table, and Y = P^T X, all in FP64 on the
// host at set-up (P the normalised aggregate indicator matrix).
static constexpr int CO_MMAX = 2048;

static cr_status coarse_pack(cr_problem* P, int bs, const std::vector<int32_t>& order,
                             const std::vector<int32_t>& agg_first,
                             const std::vector<double>& agg_w, CoarsePack& pk) {
  const int m = (int)agg_first.size() - 1;
  std::vector<int32_t> wg_agg{0}, agg_lo(m), agg_hi(m);
  int fill = 0, nloc = 0;
  for (int a = 0; a < m; ++a) {
    const int sz = agg_first[a + 1] - agg_first[a];
    if (fill + sz > bs || nloc == CO_MAXLOC) {
      wg_agg.push_back(a);
      fill = 0;
      nloc = 0;
    }
    agg_lo[a] = fill;
    agg_hi[a] = fill + sz;
    fill += sz;
    ++nloc;
  }
  wg_agg.push_back(m);
  const int nwg = (int)wg_agg.size() - 1;
  std::vector<int32_t> svox((size_t)nwg * bs, -1), sagg((size_t)nwg * bs, -1);
  std::vector<double> sw((size_t)nwg * bs, 0.0);
  for (int w = 0; w < nwg; ++w)
    for (int a = wg_agg[w]; a < wg_agg[w + 1]; ++a)
      for (int q = 0; q < agg_hi[a] - agg_lo[a]; ++q) {
        const size_t slot = (size_t)w * bs + agg_lo[a] + q;
        svox[slot] = order[agg_first[a] + q];
        sagg[slot] = a;
        sw[slot] = agg_w[a];
      }
  pk.bs = bs;
  pk.nwg = nwg;
  CR_TRY(dev_alloc(P, &pk.slot_vox, (int64_t)svox.size()));
  CR_TRY(dev_alloc(P, &pk.slot_agg, (int64_t)sagg.size()));
  CR_TRY(dev_alloc(P, &pk.slot_w, (int64_t)sw.size()));
  CR_TRY(dev_alloc(P, &pk.wg_agg, (int64_t)wg_agg.size()));
  CR_TRY(dev_alloc(P, &pk.agg_lo, (int64_t)m));
  CR_TRY(dev_alloc(P, &pk.agg_hi, (int64_t)m));
  CR_HIP(stage_to_device(pk.slot_vox, svox.data(), sizeof(int32_t) * svox.size(), P->st));
  CR_HIP(stage_to_device(pk.slot_agg, sagg.data(), sizeof(int32_t) * sagg.size(), P->st));
  CR_HIP(stage_to_device(pk.slot_w, sw.data(), sizeof(double) * sw.size(), P->st));
  CR_HIP(stage_to_device(pk.wg_agg, wg_agg.data(), sizeof(int32_t) * wg_agg.size(), P->st));
  CR_HIP(stage_to_device(pk.agg_lo, agg_lo.data(), sizeof(int32_t) * m, P->st));
  CR_HIP(stage_to_device(pk.agg_hi, agg_hi.data(), sizeof(int32_t) * m, P->st));
  return CR_OK;
}

extern "C" cr_status cr_problem_set_coarse(cr_problem* P, int32_t which, const int32_t* coords,
                                           int32_t dim, int32_t block) {
  if (!P) {
    set_error("null handle");
    return CR_EINVAL;
  }
  if (which != 1) {
    set_error("cr_problem_set_coarse: only the source grid (which = 1, the v-systems)");
    return CR_EINVAL;
  }
  if (block <= 0) {
    P->cv.valid = false;
    return CR_OK;
  }
  if (!coords || dim < 1 || dim > 3) {
    set_error("cr_problem_set_coarse: coordinates required, dim in 1..3");
    return CR_EINVAL;
  }
  const int64_t n = P->nx;
  // aggregate key of every voxel: its cube of block^dim voxels
  int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < dim; ++d) {
      lo[d] = std::min(lo[d], coords[i * dim + d]);
      hi[d] = std::max(hi[d], coords[i * dim + d]);
    }
  int64_t ext[3] = {1, 1, 1};
  for (int d = 0; d < dim; ++d) ext[d] = (int64_t)(hi[d] - lo[d]) / block + 1;
  std::vector<int64_t> key(n);
  for (int64_t i = 0; i < n; ++i) {
    int64_t k = 0;
    for (int d = dim - 1; d >= 0; --d) k = k * ext[d] + (coords[i * dim + d] - lo[d]) / block;
    key[i] = k;
  }
  std::vector<int32_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  std::vector<int32_t> agg_of(n), agg_first;
  for (int64_t q = 0; q < n; ++q) {
    if (q == 0 || key[order[q]] != key[order[q - 1]]) agg_first.push_back((int32_t)q);
    agg_of[order[q]] = (int32_t)agg_first.size() - 1;
  }
  agg_first.push_back((int32_t)n);
  const int m = (int)agg_first.size() - 1;
  int maxsz = 0;
  for (int a = 0; a < m; ++a) maxsz = std::max(maxsz, agg_first[a + 1] - agg_first[a]);
  if (maxsz > NT) {
    set_error("cr_problem_set_coarse: an aggregate has more than 256 voxels (smaller block)");
    return CR_EINVAL;
  }
  if (m > CO_MMAX) {
    set_error("cr_problem_set_coarse: " + std::to_string(m) + " aggregates, at most " +
              std::to_string(CO_MMAX) + " (larger block)");
    return CR_EINVAL;
  }
  std::vector<double> aw(m);
  for (int a = 0; a < m; ++a) aw[a] = 1.0 / std::sqrt((double)(agg_first[a + 1] - agg_first[a]));
  // neighbour table of the source Laplacian (absent neighbours point to the voxel)
  const int K = P->gx.K;
  std::vector<int32_t> nbr((size_t)K * n);
  CR_HIP(stage_to_host(nbr.data(), P->gx.nbr, sizeof(int32_t) * nbr.size(), 1, 0, P->st));
  // row i of L P: K w_i P_i,. - sum_k P_nbr_k(i),.  (sparse over aggregates)
  std::vector<double> C1((size_t)m * m, 0.0), C2((size_t)m * m, 0.0);
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t i = 0; i < n; ++i) {
    row.clear();
    auto add = [&](int32_t a, double v) {
      for (auto& e : row)
        if (e.first == a) {
          e.second += v;
          return;
        }
      row.emplace_back(a, v);
    };
    add(agg_of[i], (double)K * aw[agg_of[i]]);
    for (int k = 0; k < K; ++k) {
      const int32_t j = nbr[(size_t)k * n + i];
      add(agg_of[j], -aw[agg_of[j]]);
    }
    const int32_t ai = agg_of[i];
    for (auto& e : row) {
      if (e.second == 0.0) continue;
      C1[(size_t)e.first * m + ai] += aw[ai] * e.second;  // (P^T L P)[a(i), b]
      for (auto& f : row) C2[(size_t)f.first * m + e.first] += e.second * f.second;
    }
  }
  // Y = P^T X (FP64)
  const int ni = P->ninj;
  std::vector<double> X((size_t)n * ni), Y((size_t)m * ni, 0.0);
  CR_HIP(stage_to_host(X.data(), P->X64, sizeof(double) * X.size(), 1, 0, P->st));
  for (int al = 0; al < ni; ++al)
    for (int64_t i = 0; i < n; ++i)
      Y[(size_t)al * m + agg_of[i]] += aw[agg_of[i]] * X[(size_t)al * n + i];
  CoarseLevel cl;
  cl.m = m;
  cl.block = block;
  CR_TRY(coarse_pack(P, NT, order, agg_first, aw, cl.pack[0]));
  CR_TRY(coarse_pack(P, 512, order, agg_first, aw, cl.pack[1]));
  CR_TRY(dev_alloc(P, &cl.C1, (int64_t)m * m));
  CR_TRY(dev_alloc(P, &cl.C2, (int64_t)m * m));
  CR_TRY(dev_alloc(P, &cl.Y, (int64_t)m * ni));
  CR_HIP(stage_to_device(cl.C1, C1.data(), sizeof(double) * C1.size(), P->st));
  CR_HIP(stage_to_device(cl.C2, C2.data(), sizeof(double) * C2.size(), P->st));
  CR_HIP(stage_to_device(cl.Y, Y.data(), sizeof(double) * Y.size(), P->st));
  cl.valid = true;
  P->cv = cl;
  return CR_OK;
}

extern "C" cr_status cr_u_system(cr_problem* P, int64_t r, const double* U, int64_t ldu,
                                 const double* Z, int64_t ldz, const double* V, int64_t ldv,
                                 const double* v, double* rhs_out, double* d_out,
                                 double* coef_out) {
  if (!P || r < 0 || !v || !rhs_out || !d_out || !coef_out || (r > 0 && (!U || !Z || !V))) {
    set_error("invalid arguments to cr_u_system");
    return CR_EINVAL;
  }
  if (P->prec != CR_PREC_FP64) {
    set_error("cr_u_system needs an FP64 handle");
    return CR_EINVAL;
  }
  Ctx<double> c(P);
  CR_TRY(load_iterate<double>(c, (int)r, U, ldu, Z, ldz, V, ldv, true));
  CR_TRY(c.alloc_vectors(0));
  CR_HIP(hipMemcpyAsync(c.vv, v, sizeof(double) * c.nx, hipMemcpyDeviceToDevice, c.st));
  CR_TRY(stencil<double>(P->gx, 1, c.vv, c.nx, c.Lv, c.nx, c.st));
  CR_TRY(c.apply_R((int)r, c.vv, rhs_out));
  CR_TRY(masked_quad_ws<double>(c.ny, c.ninj, P->bits, c.y0, d_out, c.tmp + 8, c.st));
  CR_TRY(c.dot(c.nx, c.Lv, c.vv, c.tmp + 0));
  CR_TRY(c.dot(c.nx, c.Lv, c.Lv, c.tmp + 1));
  double h[2];
  CR_TRY(c.read_scalars(c.tmp, 2, h));
  coef_out[0] = 2.0 * h[0];
  coef_out[1] = h[1];
  return CR_OK;
}

extern "C" cr_status cr_u_solve(cr_problem* P, const double* d, const double* coef,
                                const double* rhs, double* x_out, double rtol, int32_t maxit,
                                int32_t precond, cr_pc* pc, int32_t* iters_out,
                                double* relres_out, int32_t* fallbacks_out) {
  if (!P || !d || !coef || !rhs || !x_out || !(rtol > 0) || maxit <= 0 || precond < 0 ||
      precond > 2 || (precond == 2 && !pc)) {
    set_error("invalid arguments to cr_u_solve");
    return CR_EINVAL;
  }
  if (P->prec != CR_PREC_FP64) {
    set_error("cr_u_solve needs an FP64 handle");
    return CR_EINVAL;
  }
  if (pc && (int64_t)pc->net.nx * pc->net.ny * pc->net.nz != P->ny) {
    set_error("the network's box does not match the target grid");
    return CR_EINVAL;
  }
  Ctx<double> c(P);
  CR_TRY(c.alloc_rank(1));
  CR_TRY(c.alloc_vectors(0));
  CR_HIP(hipMemcpyAsync(c.cu, coef, 2 * sizeof(double), hipMemcpyHostToDevice, c.st));
  CR_HIP(hipMemcpyAsync(c.dvec, d, sizeof(double) * c.ny, hipMemcpyDeviceToDevice, c.st));
  CR_TRY(pcg_diag<double>(P->gy, c.lam, c.cu, c.dvec, nullptr, 0, 0, nullptr, c.minv_u, c.st));
  Ctx<double>::SolveOut so;
  int fb = 0;
  if (precond > 0) {
    cr_pc* saved = P->pc;
    P->pc = pc;
    cr_status s = c.fcg_u(rhs, x_out, rtol, maxit, &so, &fb, c.dvec, c.minv_u, precond == 2);
    P->pc = saved;
    CR_TRY(s);
  } else {
    CR_TRY(c.pcg(true, rhs, c.vu, rtol, maxit, c.sc));
    double h[4];
    CR_TRY(c.read_scalars(c.sc, 4, h));
    so = Ctx<double>::SolveOut{h[0], h[1], (int)h[2], (int)h[3]};
    CR_HIP(hipMemcpyAsync(x_out, c.pw_u[0], sizeof(double) * c.ny, hipMemcpyDeviceToDevice, c.st));
  }
  CR_HIP(hipStreamSynchronize(c.st));
  if (iters_out) *iters_out = so.iters;
  if (relres_out) *relres_out = so.relres;
  if (fallbacks_out) *fallbacks_out = fb;
  if (so.status == 2) {
    set_error("u-system solve broke down (zero right-hand side or indefinite step)");
    return CR_ENONFINITE;
  }
  return so.status == 1 ? CR_NOTCONV : (fb ? CR_PC_FALLBACK : CR_OK);
}

extern "C" cr_status cr_pc_train_step(cr_pc* pc, cr_problem* P, int32_t batch, const double* b,
                                      const double* x, const double* d, const double* coef,
                                      float lr, double* loss_out) {
  if (!pc || !P || batch <= 0 || !b || !x || !d || !coef) {
    set_error("invalid arguments to cr_pc_train_step");
    return CR_EINVAL;
  }
  const int64_t n = P->ny;
  if ((int64_t)pc->net.nx * pc->net.ny * pc->net.nz != n) {
    set_error("the network's box does not match the target grid");
    return CR_EINVAL;
  }
  hipStream_t st = pc->st;
  const int64_t lsz = lpc_loss_scratch(pc->net);
  const int64_t need = 8 + lsz + gemv_t_part_size(n, 1) + 6 * n;
  if (pc->dwork_n < need) {
    if (pc->dwork) (void)hipFree(pc->dwork);
    pc->dwork = nullptr;
    pc->dwork_n = 0;
    if (hipMalloc(&pc->dwork, sizeof(double) * need) != hipSuccess) {
      set_error("allocation of training scratch failed");
      return CR_ENOMEM;
    }
    pc->dwork_n = need;
  }
  double* sc = pc->dwork;           // [0] ||w||^2, [2..3] coefficients
  double* lscr = sc + 8;            // loss scratch (tot[3] = loss)
  double* gpart = lscr + lsz;       // gemv partials
  double* minv = gpart + gemv_t_part_size(n, 1);
  double* w = minv + n;
  double* wt = w + n;      // spectral scratch
  double* ones = wt + n;
  hipLaunchKernelGGL(k_fill, dim3(nblk(n)), dim3(256), 0, st, n, 1.0, ones);
  CR_HIP(hipGetLastError());
  double total = 0.0;
  for (int s = 0; s < batch; ++s) {
    const double* bs = b + (int64_t)s * n;
    const double* xs = x + (int64_t)s * n;
    const double* ds = d + (int64_t)s * n;
    CR_HIP(hipMemcpyAsync(sc + 2, coef + 2 * s, 2 * sizeof(double), hipMemcpyHostToDevice, st));
    CR_TRY(pcg_diag<double>(P->gy, P->lam, sc + 2, ds, nullptr, 0, 0, nullptr, minv, st));
    if (P->boxy.valid) {
      // the base step of the flexible CG: spectral solve with the mean of d
      Blocks<double> Dm;
      Dm.clear();
      Dm.add(ds, n, 1);
      CR_TRY(gemv_t<double>(n, Dm, ones, sc + 4, gpart, st));
      hipLaunchKernelGGL(k_scale1, dim3(1), dim3(1), 0, st, sc + 4, 1.0 / (double)n);
      CR_TRY(box_spectral_solve(P->boxy, sc + 2, P->lam, sc + 4, bs, w, wt, st));
    } else {
      hipLaunchKernelGGL(k_jacobi, dim3(nblk(n)), dim3(256), 0, st, n, minv, bs, w);
    }
    CR_HIP(hipGetLastError());
    Blocks<double> A;
    A.clear();
    A.add(w, n, 1);
    CR_TRY(gemv_t<double>(n, A, w, sc + 0, gpart, st));
    CR_TRY(lpc_input(pc->net, w, sc + 0, minv, ds, P->gy.deg, sc + 2, P->lam, pc->acts.in, st));
    CR_TRY(lpc_forward(pc->net, pc->acts.in, pc->acts, st));
    CR_TRY(lpc_loss(pc->net, pc->acts.in, pc->acts.y, xs, pc->acts.dy, lscr, st));
    CR_TRY(lpc_backward(pc->net, pc->acts.in, pc->acts, st));
    double l = 0.0;
    CR_HIP(hipMemcpyAsync(&pc->hloss, lscr + lsz - 1, sizeof(double), hipMemcpyDeviceToHost, st));
    CR_HIP(hipStreamSynchronize(st));
    l = pc->hloss;
    total += l;
  }
  CR_TRY(lpc_adam(pc->net, lr, 1.0f / (float)batch, st));
  CR_HIP(hipStreamSynchronize(st));
  if (loss_out) *loss_out = total / batch;
  return std::isfinite(total) ? CR_OK : CR_ENONFINITE;
}

// ===================================================================== masked Grams
extern "C" cr_status cr_masked_gram(cr_problem* P, int64_t r, const double* U, int64_t ldu,
                                    int32_t mode, double* G, int64_t ldg) {
  if (!P || r <= 0 || !U || !G || ldu < P->ny || ldg < r || (mode != 0 && mode != 1)) {
    set_error("invalid arguments to cr_masked_gram");
    return CR_EINVAL;
  }
  if (mode == 1) {
    float* part = P->buf<float>("krpart", kr_gram_part_size(P->ny, (int)r, P->ninj));
    if (!part) return CR_ENOMEM;
    // the BF16 copy of Omega survives between calls (the block list behind it
    // is rewritten every call); a reallocation (larger r) rebuilds it
    const int64_t aux_bytes = kr_gram_aux_size(P->ny, (int)r, P->ninj);
    const bool ready = P->ws.count("kraux") && P->ws["kraux"].bytes >= (size_t)aux_bytes &&
                       P->kr_omega_ready;
    char* aux = P->buf<char>("kraux", aux_bytes);
    if (!aux) return CR_ENOMEM;
    const cr_status s = kr_gram_bf16<double>(P->ny, (int)r, P->ninj, U, ldu, P->bits, G, ldg,
                                             part, aux, ready, P->st);
    P->kr_omega_ready = s == CR_OK;
    return s;
  }
  Ctx<double> c(P);
  CR_TRY(c.alloc_rank((int)r));
  CR_TRY(c.alloc_vectors(0));
  c.U = const_cast<double*>(U);
  c.ldu = ldu;
  c.G = G;
  for (int j = 0; j < (int)r; ++j) CR_TRY(c.gram_column(j, ldg));
  return CR_OK;
}

// ===================================================================== batched solves, autotuning
// The v-system counts as fitting only in the form it takes alone: with its
// rows of X in registers when n_inj allows (64 rows, 128 FP32 rows, or 64 and
// a streamed tail), since losing them to a share cost more than concurrency
// gained (16-problem batch: 15.4 s one at a time against 16.8 s batched).
template <typename T>
static bool xreg_fits_share(cr_problem* P, int share) {
  const int ninj = P->ninj;
  const int nxr = ninj <= PCG_NXR ? PCG_NXR
                  : (std::is_same<T, float>::value && ninj <= PCG_NXR2) ? PCG_NXR2 : PCG_NXR;
  const int xtail = (ninj > nxr) ? 1 : 0;
  for (int bs : {NT, 512}) {
    PcgArgs<T> probe{};
    probe.g = P->gx;
    probe.Xm = P->X<T>();
    probe.vpt = 1;
    probe.bs = bs;
    probe.nxr = nxr;
    probe.xtail = xtail;
    const int m = pcg_max_wg<T>(probe);
    const int64_t w = (P->gx.n + bs - 1) / bs;
    if (m > 0 && w <= (share > 0 ? share_cap(m, share) : m)) return true;
  }
  return false;
}

// does every persistent PCG grid of problem P fit in `share` CUs?
template <typename T>
static bool fits_share_t(cr_problem* P, int share) {
  // v-systems solved directly (SMW on a full source box) use their PCG only
  // as a fallback, in whatever form fits: no register-form requirement
  const bool v_direct = P->fcg_mode > 0 && P->boxx.valid && P->ninj <= SMW_MAX;
  if (v_direct || !P->batch_xreg) {
    // (the fallback grids are checked below)
  } else if (!P->no_xreg && !xreg_fits_share<T>(P, 0)) {
    // (no register form even alone: the streamed form decides below)
  } else if (!P->no_xreg && !xreg_fits_share<T>(P, share)) {
    return false;
  }
  for (int sys = 0; sys < 2; ++sys) {
    const Geom& g = sys ? P->gx : P->gy;
    bool ok = false;
    for (int v = 1; v <= 8 && !ok; v *= 2) {
      PcgArgs<T> probe{};
      probe.g = g;
      probe.Xm = sys ? P->X<T>() : nullptr;
      probe.vpt = v;
      const int m = pcg_max_wg<T>(probe);
      const int64_t w = (g.n + (int64_t)NT * v - 1) / ((int64_t)NT * v);
      ok = m > 0 && w <= share_cap(m, share);
    }
    if (!ok) return false;
  }
  return true;
}

static bool fits_share(cr_problem* P, int share) {
  return P->prec == CR_PREC_MIXED ? fits_share_t<float>(P, share)
                                  : fits_share_t<double>(P, share);
}

extern "C" cr_status cr_greedy_solve_batch(int32_t count, cr_problem** probs,
                                           const cr_solve_opts* opts, double** U, double** V,
                                           double** Z, int64_t* ranks, cr_solve_stats* stats,
                                           int32_t* statuses) {
  if (count <= 0 || !probs || !opts || !U || !V || !Z || !ranks || !statuses) {
    set_error("invalid arguments to cr_greedy_solve_batch");
    return CR_EINVAL;
  }
  for (int k = 0; k < count; ++k)
    for (int l = 0; l < k; ++l)
      if (!probs[k] || probs[k] == probs[l] || probs[k]->st == probs[l]->st) {
        set_error("batched problems need distinct handles on distinct streams");
        return CR_EINVAL;
      }
  int dev = 0;
  CR_HIP(hipGetDevice(&dev));
  const int ncu = device_cus();
  // the most problems that can run at once: each of K workers owns 3/4 of
  // 1/K of the CUs (a margin for packing losses) and every grid must fit
  int K = std::min(count, 16);
  for (; K > 1; --K) {
    const int share = std::max(1, 3 * ncu / (4 * K));
    bool all = true;
    for (int k = 0; k < count && all; ++k) all = fits_share(probs[k], share);
    if (all) break;
  }
  const int share = K > 1 ? std::max(1, 3 * ncu / (4 * K)) : 0;
  // largest problems first
  std::vector<int> order(count);
  for (int k = 0; k < count; ++k) order[k] = k;
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return probs[a]->ny > probs[b]->ny; });
  // Each worker runs its problems on a pair of streams created here, one
  // after another, so the K workers' streams spread over the device's
  // hardware queues; the problems' own streams, created whenever their
  // handles were, could share queues and serialise concurrent problems.
  // The problems' pending work is finished first; their streams are restored
  // after each solve (which ends with a wait on the stream it ran on).
  std::vector<hipStream_t> wst(2 * K, nullptr);
  for (int k = 0; k < count; ++k) CR_HIP(hipStreamSynchronize(probs[k]->st));
  for (int w = 0; w < 2 * K && K > 1; ++w) {
    if (hipStreamCreateWithFlags(&wst[w], hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t sw : wst)
        if (sw) (void)hipStreamDestroy(sw);
      set_error("stream creation for the batch workers failed");
      return CR_EHIP;
    }
  }
  std::vector<int> saved_cap(count), saved_coop(count), saved_mode(count);
  for (int k = 0; k < count; ++k) {
    saved_cap[k] = probs[k]->cu_share;
    saved_coop[k] = probs[k]->coop;
    saved_mode[k] = probs[k]->bar_mode;
    probs[k]->cu_share = share;
    probs[k]->coop = K > 1 ? 0 : 1;
    probs[k]->bar_mode = 1;
  }
  std::vector<std::string> errs(count);
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  for (int w = 0; w < K; ++w)
    th.emplace_back([&, w]() {
      (void)hipSetDevice(dev);
      for (int q = next++; q < count; q = next++) {
        const int k = order[q];
        cr_problem* P = probs[k];
        hipStream_t own = P->st, own_aux = P->aux;
        if (K > 1) {
          P->st = wst[2 * w];
          P->aux = wst[2 * w + 1];
        }
        cr_status s = P->prec == CR_PREC_MIXED
                          ? greedy_impl<float>(P, opts[k], U[k], V[k], Z[k], &ranks[k],
                                               stats ? &stats[k] : nullptr, nullptr, nullptr)
                          : greedy_impl<double>(P, opts[k], U[k], V[k], Z[k], &ranks[k],
                                                stats ? &stats[k] : nullptr, nullptr, nullptr);
        if (K > 1) {
          (void)hipStreamSynchronize(P->st);
          (void)hipStreamSynchronize(P->aux);
          P->st = own;
          P->aux = own_aux;
        }
        statuses[k] = s;
        if (s < 0) errs[k] = cr_last_error();
      }
    });
  for (auto& t : th) t.join();
  for (hipStream_t sw : wst)
    if (sw) (void)hipStreamDestroy(sw);
  cr_status worst = CR_OK;
  for (int k = 0; k < count; ++k) {
    probs[k]->cu_share = saved_cap[k];
    probs[k]->coop = saved_coop[k];
    probs[k]->bar_mode = saved_mode[k];
    if (statuses[k] < 0 && worst == CR_OK) {
      worst = (cr_status)statuses[k];
      set_error("problem " + std::to_string(k) + ": " + errs[k]);
    }
  }
  return worst;
}

// Autotuner: times 60 Jacobi-PCG iterations of a representative u- and
// v-system for each admissible voxels-per-thread (1, 2, 4, 8) within the
// handle's current workgroup cap and keeps the fastest for later solves.
template <typename T>
static cr_status autotune_impl(cr_problem* P, int32_t cu_share, int32_t* vpt_u, int32_t* vpt_v,
                               double* us_u, double* us_v) {
  const int saved = P->cu_share;
  P->cu_share = cu_share > 0 ? cu_share : saved;
  cr_status status = CR_OK;
  double best[2] = {1e300, 1e300};
  int bestv[2] = {0, 0};
  hipEvent_t e0, e1;
  CR_HIP(hipEventCreate(&e0));
  CR_HIP(hipEventCreate(&e1));
  for (int v = 1; v <= 8 && status == CR_OK; v *= 2) {
    Ctx<T> c(P);
    status = c.alloc_rank(1);
    if (status != CR_OK) break;
    status = c.alloc_vectors(v);
    if (status != CR_OK) {  // this grid shape does not fit the cap
      status = CR_OK;
      continue;
    }
    // representative systems: d = 1 + |q|, unit coefficients, rhs = q
    double hc[2] = {1.0, 0.5};
    CR_HIP(hipMemcpyAsync(c.cu, hc, sizeof(hc), hipMemcpyHostToDevice, c.st));
    CR_HIP(hipMemcpyAsync(c.cv, hc, sizeof(hc), hipMemcpyHostToDevice, c.st));
    CR_TRY(splitmix_fill<T>(c.ny, 7, 1, c.rhs_u, c.st));
    CR_TRY(splitmix_fill<T>(c.nx, 7, 2, c.rhs_v, c.st));
    CR_TRY(splitmix_fill<T>(c.ny, 7, 3, c.dvec, c.st));
    std::vector<double> ones(c.ninj, 1.0);
    CR_HIP(hipMemcpyAsync(c.gw, ones.data(), sizeof(double) * c.ninj, hipMemcpyHostToDevice, c.st));
    CR_TRY(pcg_diag<T>(P->gy, c.lam, c.cu, c.dvec, nullptr, 0, 0, nullptr, c.minv_u, c.st));
    CR_TRY(pcg_diag<T>(P->gx, c.lam, c.cv, nullptr, c.X(), c.nx, c.ninj, c.gw, c.minv_v, c.st));
    for (int sys = 0; sys < 2; ++sys) {
      const bool us = sys == 0;
      double t = 0.0;
      for (int rep = 0; rep < 3; ++rep) {
        CR_HIP(hipEventRecord(e0, c.st));
        CR_TRY(c.pcg(us, us ? c.rhs_u : c.rhs_v, us ? c.vu : c.vv, 1e-300, 60, c.sc));
        CR_HIP(hipEventRecord(e1, c.st));
        CR_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        CR_HIP(hipEventElapsedTime(&ms, e0, e1));
        double h[4];
        CR_TRY(c.read_scalars(c.sc, 4, h));
        const double per = 1e3 * ms / std::max(1.0, h[2]);
        if (rep > 0) t = rep == 1 ? per : std::min(t, per);
      }
      if (t < best[sys]) {
        best[sys] = t;
        bestv[sys] = v;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->cu_share = saved;
  if (status != CR_OK) return status;
  P->tuned_vpt_u = bestv[0];
  P->tuned_vpt_v = bestv[1];
  if (vpt_u) *vpt_u = bestv[0];
  if (vpt_v) *vpt_v = bestv[1];
  if (us_u) *us_u = best[0];
  if (us_v) *us_v = best[1];
  return CR_OK;
}

extern "C" cr_status cr_autotune_pcg(cr_problem* P, int32_t cu_share, int32_t* vpt_u,
                                     int32_t* vpt_v, double* us_u, double* us_v) {
  if (!P) {
    set_error("null handle");
    return CR_EINVAL;
  }
  return P->prec == CR_PREC_FP64 ? autotune_impl<double>(P, cu_share, vpt_u, vpt_v, us_u, us_v)
                                 : autotune_impl<float>(P, cu_share, vpt_u, vpt_v, us_u, us_v);
}

extern "C" cr_status cr_problem_set_tuning(cr_problem* P, int32_t vpt_u, int32_t vpt_v) {
  if (!P) {
    set_error("null handle");
    return CR_EINVAL;
  }
  for (int v : {vpt_u, vpt_v})
    if (v != 0 && v != 1 && v != 2 && v != 4 && v != 8) {
      set_error("voxels per thread must be 0, 1, 2, 4 or 8");
      return CR_EINVAL;
    }
  P->tuned_vpt_u = vpt_u;
  P->tuned_vpt_v = vpt_v;
  return CR_OK;
}
