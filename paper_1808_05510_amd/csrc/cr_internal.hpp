// Internal declarations of libconnreg (not installed; the public C ABI is
// include/connreg.h).  Kernels are written for gfx950 (CDNA4, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>
#include <string>
#include <vector>

#include "../../include/connreg.h"
#include "ring2.hpp"

namespace cr {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);

#define CR_HIP(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      ::cr::set_error(std::string("HIP error ") + hipGetErrorString(e_) +   \
                      " at " __FILE__ ":" + std::to_string(__LINE__));      \
      return CR_EHIP;                                                       \
    }                                                                       \
  } while (0)

#define CR_TRY(call)                 \
  do {                               \
    cr_status s_ = (call);           \
    if (s_ < 0) return s_;           \
  } while (0)

// ---------------------------------------------------------------- set-up transfers
// Host <-> device copies of set-up data (problem arrays, geometry tables,
// spectral bases, network parameters) go through pinned staging memory, as
// copies ordered on the handle's stream followed by a wait on that stream:
// the pattern of every scalar read of the solvers.  Synchronous copies to or
// from pageable memory came back with zeros in the copied arrays under a
// kernel-tracing profiler, right after another handle was destroyed.
// stage_to_host copies rows x width bytes, source rows spitch bytes apart
// (0: contiguous), into dst packed
inline hipError_t stage_to_host(void* dst, const void* src, size_t width, size_t rows,
                                size_t spitch, hipStream_t st) {
  if (width == 0 || rows == 0) return hipSuccess;
  if (spitch == 0) spitch = width;
  void* pin = nullptr;
  hipError_t e = hipHostMalloc(&pin, width * rows);
  if (e != hipSuccess) return e;
  e = hipMemcpy2DAsync(pin, width, src, spitch, width, rows, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) std::memcpy(dst, pin, width * rows);
  (void)hipHostFree(pin);
  return e;
}

inline hipError_t stage_to_device(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  void* pin = nullptr;
  hipError_t e = hipHostMalloc(&pin, bytes);
  if (e != hipSuccess) return e;
  std::memcpy(pin, src, bytes);
  e = hipMemcpyAsync(dst, pin, bytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipHostFree(pin);
  return e;
}

constexpr int WAVE = 64;
constexpr int NT = 256;  // threads per workgroup for streaming kernels

// ---------------------------------------------------------------- geometry
// A voxel graph Laplacian L = Deg - Adj stored as an ELL neighbour table of
// width K, structure-of-arrays (nbr[k*n + i]); an absent neighbour points to
// the voxel itself, so (L w)_i = K w_i - sum_k w[nbr[k*n+i]] for every row.
// LDS-window form of the stencil: per tile of NT consecutive voxels, the set
// of voxels its rows read (the tile and its neighbours) as at most WIN_NI
// index intervals (gaps of up to WIN_GAP voxels bridged) of total length at
// most WIN_MAX, so that a workgroup stages them with coalesced loads.
constexpr int WIN_NI = 16, WIN_MAX = 2048, WIN_GAP = 32;
constexpr int WIN_TAB = 2 + 2 * WIN_NI;  // count, total, starts, LDS prefixes

// (the ring-2 forms of L^2, W2_* and R2_*, are defined in ring2.hpp)

struct Geom {
  int64_t n = 0;
  int K = 0;
  int32_t* nbr = nullptr;  // device, K*n
  uint8_t* deg = nullptr;  // device, n
  // window tables (null when some tile's window does not fit):
  int32_t* witab = nullptr;  // device, ntile * WIN_TAB
  uint16_t* wpos = nullptr;  // device, (K + 1) * n: window position of i, then of nbr_k(i)
  // ring-2 window tables (null when some tile's window or row does not fit):
  int32_t* w2tab = nullptr;   // device, ceil(n / W2_TILE) * W2_TAB
  uint32_t* w2ent = nullptr;  // device, W2_NE * n (entry e of voxel i at e * n + i)
  // rows of L^2 for the two-barrier PCG (null when not built or some row
  // does not fit)
  int32_t* r2idx = nullptr;  // device, R2_NX * n
  int8_t* r2cf = nullptr;    // device, R2_NC * n
};

// A column-block list: columns [col0, col0+ncols) of the logical matrix live
// at p + (c-col0)*ld.  Up to 6 blocks, passed by value to kernels.
template <typename T>
struct Blocks {
  static constexpr int MAXB = 6;
  const T* p[MAXB];
  int64_t ld[MAXB];
  int col0[MAXB + 1];
  int nb = 0;
  void clear() { nb = 0; col0[0] = 0; }
  void add(const T* ptr, int64_t ldp, int ncols) {
    if (ncols <= 0) return;
    p[nb] = ptr; ld[nb] = ldp; col0[nb + 1] = col0[nb] + ncols; ++nb;
  }
  __host__ __device__ int ncols() const { return nb ? col0[nb] : 0; }
  __device__ __forceinline__ const T* col(int c) const {
    int b = 0;
#pragma unroll
    for (int k = 1; k < MAXB; ++k)
      if (k < nb && c >= col0[k]) b = k;
    return p[b] + (int64_t)(c - col0[b]) * ld[b];
  }
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return CR_OK or CR_EHIP.
// Stencil: out[:,c] = L w[:,c] for c < ncols (w, out column-major).
template <typename T>
cr_status stencil(const Geom& g, int ncols, const T* w, int64_t ldw, T* out, int64_t ldo,
                  hipStream_t st);

// y[c] = sum_i A[i,c] * x[i] for the block list A (n rows), accumulated in
// double; y written as double.  part: workspace of >= ncols * nrb doubles.
template <typename T>
cr_status gemv_t(int64_t n, const Blocks<T>& A, const T* x, double* y, double* part,
                 hipStream_t st);
int64_t gemv_t_part_size(int64_t n, int ncols);
// the same with an x vector of another type (FP32 matrix, FP64 vector)
template <typename T, typename TX>
cr_status gemv_tx(int64_t n, const Blocks<T>& A, const TX* x, double* y, double* part,
                  hipStream_t st);

// y = beta*y + sum_c A[:,c] * coef[c]; coef is a device double array.
template <typename T>
cr_status gemv_n(int64_t n, const Blocks<T>& A, const double* coef, double beta, T* y,
                 hipStream_t st);

// C (p x q, ldc, double) = A^T B for block lists A, B over n rows.  When
// mask_bits is non-null B is implicit: B[i,a] = omega_{i,a} * w[i] with
// omega bit a of word bits[(a/32)*n + i].  part: >= ksplit*p*q doubles.
// With ks_out non-null the split-K partials are left unreduced in part
// (part[z p q + i + j p], z < *ks_out) and C is not written.
template <typename T>
cr_status gemm_tn(int64_t n, const Blocks<T>& A, const Blocks<T>& B, const uint32_t* mask_bits,
                  const T* w, int q_mask, double* C, int64_t ldc, double* part,
                  int64_t part_cap, hipStream_t st, int* ks_out = nullptr);

// T (r x p, double, ldt) = Z H with H = V^T X (r x p) given as the ks split-K
// partials of gemm_tn(V, X) (ks_out form: part[z r p + j + a r]); Z: r x r
// (ldz).  One workgroup per column of T; the partials are summed in a fixed
// order.  r <= ZH_RMAX.
constexpr int ZH_RMAX = 2048;
template <typename T>
cr_status zh_from_partials(int p, int r, int ks, const double* part, const T* Z, int64_t ldz,
                           double* Tm, int64_t ldt, hipStream_t st);

// N = OY - Omega o (U T)  (n x ninj), or, with OY == nullptr, N = Omega o (U T).
// U: n x r (ldu), T: r x ninj (double, ldt).
template <typename T>
cr_status masked_tall_gemm(int64_t n, int r, int ninj, const T* U, int64_t ldu,
                           const double* Tm, int64_t ldt, const uint32_t* bits,
                           const T* OY, int64_t ldoy, T* N, int64_t ldn, hipStream_t st);

// Fused operator sweep (ring-2 window form): out1 = L w, out2 = L^2 w for the
// r columns of w (ldw; outputs ldo), and with N != nullptr also
// N = Omega o (w T) (n x ninj, ldn; T: r x ninj double, ldt).  Needs the
// geometry's ring-2 tables and ninj <= 128 (op_win2_ok).
template <typename T>
bool op_win2_ok(const Geom& g, int r, int ninj);
template <typename T>
cr_status op_win2(const Geom& g, int r, const T* w, int64_t ldw, T* out1, T* out2, int64_t ldo,
                  int ninj, const double* Tm, int64_t ldt, const uint32_t* bits, T* N,
                  int64_t ldn, hipStream_t st);

// d_i = sum_a omega_ia h_a^2 (h: device double, ninj); tmp: 1 device double
template <typename T>
cr_status masked_quad_ws(int64_t n, int ninj, const uint32_t* bits, const double* h, T* d,
                         double* tmp, hipStream_t st);

// g_a = sum_i omega_ia w_i^2 (double out), part >= ninj*nrb doubles
template <typename T>
cr_status masked_colsq(int64_t n, int ninj, const uint32_t* bits, const T* w, double* g,
                       double* part, hipStream_t st);

// elementwise helpers
template <typename Td, typename Ts>
cr_status convert(int64_t n, const Ts* src, Td* dst, hipStream_t st);
template <typename Td, typename Ts>
cr_status convert2d(int64_t rows, int64_t cols, const Ts* src, int64_t lds, Td* dst,
                    int64_t ldd, hipStream_t st);

// ---------------------------------------------------------------- PCG
// SPD system on one voxel graph:
//   A x = lam*(L^2 x + c1 L x + c0 x) + dvec o x + Xm diag(gw) Xm^T x
// Jacobi preconditioned CG from x0 = 0 in one cooperative launch; on exit
// xout = x / ||x|| and scal[0] = ||x||, scal[1] = final ||r||/||b||,
// scal[2] = iterations, scal[3] = status (0 ok, 1 not converged, 2 breakdown).
// grid barrier selection for the persistent kernels (see k_cg.hip)
// barrier words: [0] generation, [64] timeout flag, [128] arrivals (separate
// 256-byte lines)
constexpr int BAR_GEN = 0, BAR_TIMEOUT = 64, BAR_COUNT = 128, BAR_WORDS = 192;
struct BarrierArg {
  unsigned* bar = nullptr;  // BAR_WORDS device words, zeroed before each launch
  int mode = 1;             // 0: cooperative-groups grid sync, 1: atomic barrier
  int coop = 1;             // 1: cooperative launch; 0: ordinary launch (mode 1 only, for
                            // concurrent persistent kernels that together fit on the device)
  unsigned spin_max = 1u << 22;  // polls before a waiting workgroup gives up (timeout flag)
};
// Status a persistent kernel writes when its grid barrier timed out: the
// kernel records it in its own scalars, so a read deferred past a later
// launch (which clears the barrier words) still sees it.
constexpr double PERSIST_TIMEOUT = 3.0;

// Two-level preconditioner of the v-system PCG: aggregates of source voxels
// (a partition into spatial blocks), packed whole into workgroups; thread
// slot s of the launch holds voxel slot_vox[s] (-1: idle) of aggregate
// slot_agg[s], weight slot_w[s] = 1 / sqrt(|aggregate|).  Workgroup b owns
// aggregates [wg_agg[b], wg_agg[b+1]), aggregate a the slots
// [agg_lo[a], agg_hi[a]) of its workgroup.  M^-1 r = D^-1 r + P Ainv P^T r
// with P the normalised indicator matrix and Ainv = (P^T A P)^-1 (m x m,
// rebuilt for every solve; all zero when its Cholesky factorisation fails,
// which leaves plain Jacobi).  rc: m doubles, the restricted residual.
struct CoarseArg {
  const int32_t* slot_vox = nullptr;
  const int32_t* slot_agg = nullptr;
  const double* slot_w = nullptr;
  const int32_t* wg_agg = nullptr;
  const int32_t* agg_lo = nullptr;
  const int32_t* agg_hi = nullptr;
  int m = 0;
  const double* Ainv = nullptr;
  double* rc = nullptr;
};
constexpr int CO_MAXLOC = 64;  // aggregates per workgroup

template <typename T>
struct PcgArgs {
  CoarseArg co;         // two-level (CO kernels only)
  Geom g;
  double lam;
  const double* coef;   // device: coef[0] = c1, coef[1] = c0
  const T* dvec;        // may be null
  const T* Xm;          // may be null (no low-rank term)
  int64_t ldx;
  int ninj;
  const double* gw;     // ninj weights (device)
  const T* minv;        // Jacobi inverse diagonal
  const T* b;
  T* x; T* r; T* z; T* p; T* t; T* q;
  T* xout;
  const T* x0 = nullptr;        // initial iterate (null: zero); b is then b - A x0
  const double* bref = nullptr;  // device ||b||^2 of the original system (null: ||b||^2 of b)
  double* part;         // >= nwg*5 + ninj*nwg
  double* sbuf;         // >= ninj
  double* scal;         // >= 4
  double rtol;
  int maxit;
  int vpt;              // voxels per thread
  int bs = NT;          // threads per workgroup (NT or 1024)
  int nxr = 0;          // PCG_NXR or PCG_NXR2: X rows in registers (low-rank term, vpt 1)
  int xtail = 0;        // 1: more injections than nxr, the rest streamed; 2: the first xlds
                        // of the rest in LDS, any after them streamed
  int xlds = 0;         // xtail 2: tail rows held in LDS
  BarrierArg bar;
};
constexpr int PCG_NXR = 64;  // injections held in registers by the X-resident PCG
constexpr int PCG_NXR2 = 128;  // the same for FP32 data up to 128 injections
// rows of X beyond the register rows that the LDS-resident form can hold
// beside the kernel's static LDS (12 KB at 256 threads, 16.5 KB at 512)
// within 160 KB: 72 / 35 FP64 rows, 147 / 71 FP32 rows at 256 / 512 threads
inline int pcg_xlds_cap(int bs, int bytes) {
  const int stat = bs == 256 ? 12352 : 16512;
  return (160 * 1024 - stat) / (bs * bytes);
}
template <typename T>
cr_status pcg_solve(const PcgArgs<T>& a, int nwg, hipStream_t st);
template <typename T>
int pcg_max_wg(const PcgArgs<T>& a);

// Jacobi inverse diagonal: minv_i = 1 / (lam*(deg^2 + deg + c1*deg + c0) + d_i
//                                        + sum_a gw_a Xm_ia^2)
template <typename T>
cr_status pcg_diag(const Geom& g, double lam, const double* coef, const T* dvec, const T* Xm,
                   int64_t ldx, int ninj, const double* gw, T* minv, hipStream_t st);

// FP64 residual of the same operator for iterative refinement:
//   r = b - (lam*(L^2 x + c1 L x + c0 x) + dvec o x + Xm (gw o s)),  s = Xm^T x given,
// x, r, t (= L x, written here) in FP64; operator data in T.
template <typename T>
cr_status als_residual(const Geom& g, double lam, const double* coef, const T* dvec, const T* Xm,
                       int64_t ldx, int ninj, const double* gw, const double* s, const T* b,
                       const double* x, double* t, double* r, hipStream_t st);
// x += e (e in T, x in FP64); x = e when init
template <typename T>
cr_status accumulate(int64_t n, const T* e, double* x, bool init, hipStream_t st);
// out = (T)(x / sqrt(nrm2[0]))
template <typename T>
cr_status normalize_out(int64_t n, const double* x, const double* nrm2, T* out, hipStream_t st);

// ---------------------------------------------------------------- Galerkin
struct GalerkinArgs {
  int r, ldr, ninj;
  double lam;
  const double* G;    // ninj blocks of ldr*ldr (col-major r x r each)
  const __bf16* Gb;   // optional BF16 copy (block al at al*r*ldh, rows padded to ldh, ldh % 4 == 0):
                      // when set, the CG iterations use it; the initial residual always uses G
  int ldh;
  const double* H;    // H = V^T X stored transposed: H(k,a) = H[a + k*ninj]
  const double* S;    // S = U^T (Omega o Y) stored the same way
  const double* By1; const double* By2; const double* Bx1; const double* Bx2;  // ld ldr
  double* Z;          // in/out, ld ldr
  double* R; double* P; double* Q; double* Y2; double* Bm;  // work, r x r (ld ldr)
  double* T;          // work, r x ninj (ld ldr): P H
  double* SG;         // work, r x ninj (ld ldr)
  double* part;       // >= 9*nwg
  double* scal;       // out: [0] iters, [1] relres, [2] status, [3] energy,
                      //      [4] relres of the initial residual (FP64 operator)
  double rtol;
  double inner_rel;   // also stop once ||R|| <= inner_rel ||R_0|| (0: off)
  int maxit;
  BarrierArg bar;
};
// nb: output tiles of 16 nb x 16 nb (1 or 2; 0 chooses by r and nwg)
cr_status galerkin_cg(const GalerkinArgs& a, int nwg, int nb, hipStream_t st);
// Gb (ninj blocks of r x ldh BF16) = the r x r leading blocks of G, rounded
cr_status gram_to_bf16(int r, int ld, int ldh, int ninj, const double* G, __bf16* Gb,
                       hipStream_t st);
int galerkin_max_wg(int r);

// ---------------------------------------------------------------- learned preconditioner
constexpr int LPC_MAXC = 8;
constexpr int LPC_LAYERS = 5;
// Per-axis DCT-II bases of a full box (first axis fastest): Q[a] row-major
// d_a x d_a (row = position, column = mode), mu[a] the path-graph eigenvalues.
struct BoxBasis {
  bool valid = false;
  int dims[3] = {0, 0, 0};
  double* Q[3] = {nullptr, nullptr, nullptr};
  double* mu[3] = {nullptr, nullptr, nullptr};
};
// out = Q diag(1 / (lam (mu^2 + c[0] mu + c[1]) + dbar[0])) Q^T r; tmp: n doubles;
// dbar may be null (0).  The _cols form solves ncols columns at once.
cr_status box_spectral_solve(const BoxBasis& bx, const double* c, double lam, const double* dbar,
                             const double* r, double* out, double* tmp, hipStream_t st);
cr_status box_spectral_solve_cols(const BoxBasis& bx, const double* c, double lam,
                                  const double* dbar, int ncols, const double* R, int64_t ldr,
                                  double* OUT, int64_t ldo, double* TMP, int64_t ldt,
                                  hipStream_t st);
// The three passes of Q^T (forward) or Q (inverse) alone, on ncols columns;
// OUT receives the result, TMP is scratch of the same shape (ldt).
cr_status box_transform_cols(const BoxBasis& bx, bool inverse, int ncols, const double* R,
                             int64_t ldr, double* OUT, int64_t ldo, double* TMP, int64_t ldt,
                             hipStream_t st);
// XH[:, j] /= lam (mu^2 + c[0] mu + c[1]) + dbar[0] in the spectral domain
// (dbar may be null: 0), ncols columns of leading dimension ld
cr_status box_scale_cols(const BoxBasis& bx, const double* c, double lam, const double* dbar,
                         int ncols, double* XH, int64_t ld, hipStream_t st);
// SMW solve of the v-system on a full source box (n_inj <= SMW_MAX)
constexpr int SMW_MAX = 128;
cr_status smw_factor(int n, const double* g, double* K, hipStream_t st);
cr_status smw_apply(int n, const double* g, const double* L, const double* h, double* kvec,
                    hipStream_t st);

struct LpcNet {
  int nx = 0, ny = 0, nz = 0, C = 0;
  int ci[LPC_LAYERS], co[LPC_LAYERS];
  float *W[LPC_LAYERS], *B[LPC_LAYERS], *gW[LPC_LAYERS], *gB[LPC_LAYERS];
  float *mW[LPC_LAYERS], *vW[LPC_LAYERS], *mB[LPC_LAYERS], *vB[LPC_LAYERS];
  int step = 0;
  int64_t nparam = 0;
  float* mem = nullptr;  // one allocation: params, grads, Adam moments
};
struct LpcActs {
  float *in = nullptr, *a0, *a1, *p, *a2, *a3, *s, *y, *dy, *ds, *da3, *da2, *dp, *da0, *partial;
  float* mem = nullptr;
};
cr_status lpc_forward(const LpcNet& net, const float* in, LpcActs& a, hipStream_t st);
cr_status lpc_backward(LpcNet& net, const float* in, LpcActs& a, hipStream_t st);
// network input from w = minv o r (w2 = ||w||^2 on the device)
cr_status lpc_input(const LpcNet& net, const double* w, const double* w2, const double* minv,
                    const double* dvec, const uint8_t* deg, const double* coef, double lam,
                    float* in, hipStream_t st);
// z = in0 + y
cr_status lpc_output(const LpcNet& net, const float* in0, const float* y, double* z,
                     hipStream_t st);
// loss 1 - cos^2(in0 + y, xs) into scratch[3 * nblocks + 3] and dy = dL/dy
int64_t lpc_loss_scratch(const LpcNet& net);
cr_status lpc_loss(const LpcNet& net, const float* in0, const float* y, const double* xs,
                   float* dy, double* scratch, hipStream_t st);
cr_status lpc_adam(LpcNet& net, float lr, float scale, hipStream_t st);

// ---------------------------------------------------------------- BF16 Khatri-Rao Grams
// part: kr_gram_part_size floats; aux: kr_gram_aux_size bytes holding the BF16
// copy of Omega (built when omega_ready is false, reusable afterwards) and the
// block list
int64_t kr_gram_part_size(int64_t n, int r, int ninj);
int64_t kr_gram_aux_size(int64_t n, int r, int ninj);
template <typename TU>
cr_status kr_gram_bf16(int64_t n, int r, int ninj, const TU* U, int64_t ldu, const uint32_t* bits,
                       double* G, int64_t ldr, float* part, void* aux, bool omega_ready,
                       hipStream_t st);

// ---------------------------------------------------------------- post-processing (k_post.hip)
// out[:, c] = s * sum_k M[:, k] op(B)[k, c] (c < ncols, k < kd; op(B) = B^T
// when transB); B == nullptr: out = s * M (in place allowed)
cr_status tall_small(int64_t n, int kd, int ncols, const double* M, int64_t ldm, const double* B,
                     int64_t ldb, bool transB, double s, double* out, int64_t ldo, hipStream_t st);
// SVD of the r x r matrix A (overwritten): A = Uo diag(s) Vo^T, s descending;
// work: r*r + r doubles; info[2] = {sweeps, converged}
cr_status small_svd(int r, double* A, int64_t lda, double* Uo, int64_t ldu, double* s, double* Vo,
                    int64_t ldvo, double* work, double* info, hipStream_t st);
// out[0] = scale * ||X||_F^2 (X rows x cols); part: 512 doubles
cr_status sumsq(int64_t rows, int64_t cols, const double* x, int64_t ld, double scale,
                double* part, double* out, hipStream_t st);
// out[0] = scale * trace(P Q), P, Q m x m
cr_status trace_prod(int m, const double* P, int64_t ldp, const double* Q, int64_t ldq,
                     double scale, double* out, hipStream_t st);
// statistics over every entry of W = A B^T (A na x k, B nb x k) into out[6] =
// {negative count, min, max, max |w|, sum w^2, sum of w^2 over w < 0}
int64_t entry_stats_part_size(int64_t na, int64_t nb);
cr_status entry_stats(int64_t na, int64_t nb, int k, const double* A, int64_t lda,
                      const double* B, int64_t ldb, double* part, double* out, hipStream_t st);

// residual Grams in the capacity layout (block b >= 1 at ninj + (b-1) rmax)
cr_status gram_scatter(int m, int n, const double* C, int64_t ldc, int row0, int col0, int newcol,
                       int ninj, int r, int rmax, double* Gc, int64_t ldg, hipStream_t st);
cr_status gram_gather(int k, int ninj, int r, int rmax, const double* Gc, int64_t ldg, double* out,
                      hipStream_t st);
// CholQR2 pieces: symmetric diagonal scaling to unit diagonal (s = 1/sqrt(diag));
// in-place lower Cholesky (info[0] = 0 or failing pivot + 1); lower inverse;
// tri_scale mode 0: out = X diag(s), mode 1: out = L^T diag(1/s)
cr_status diag_scale(int k, double* A, int64_t lda, double* s, hipStream_t st);
cr_status chol_lower(int k, double* A, int64_t lda, double* info, hipStream_t st);
cr_status trinv_lower(int k, const double* L, int64_t ldl, double* X, int64_t ldx, hipStream_t st);
cr_status tri_scale(int k, int mode, const double* X, int64_t ldx, const double* s, double* out,
                    int64_t ldo, hipStream_t st);

// two-level coarse operator: A = lam (C2 + coef[0] C1 + coef[1] I) + Y diag(gw) Y^T
// (Y may be null), and the lower-triangular inverse of a Cholesky factor
// (X zero when info[0] != 0)
cr_status coarse_assemble(int m, double lam, const double* coef, const double* C1,
                          const double* C2, const double* Y, int ninj, const double* gw, double* A,
                          hipStream_t st);
cr_status trinv_rows(int k, const double* L, int64_t ldl, double* X, int64_t ldx,
                     const double* info, hipStream_t st);

// ---------------------------------------------------------------- small ops
// out[i] = sum_k M[i + k*ldm] * v[k] * alpha  (i < m, k < kk), single block
cr_status small_gemv(int m, int kk, const double* M, int64_t ldm, bool trans, const double* v,
                     double alpha, double* out, hipStream_t st);
// C (m x n, ldc) = alpha * op(A) op(B), op = transpose when ta/tb, all double, small
cr_status small_gemm(int m, int n, int k, const double* A, int64_t lda, bool ta, const double* B,
                     int64_t ldb, bool tb, double alpha, double* C, int64_t ldc, hipStream_t st);

// x[i] *= 1/sqrt(nrm2[0]) with nrm2 a device double
template <typename T>
cr_status scale_inv_sqrt(int64_t n, T* x, const double* nrm2, hipStream_t st);
// q[i] = SplitMix64 uniform in [-1,1) (stream `stream` of `seed`)
template <typename T>
cr_status splitmix_fill(int64_t n, uint64_t seed, uint64_t stream, T* q, hipStream_t st);
// hole-list Gram update: Gcol[a][c] -= sum_{i in hole_a} U[i,c] w[i] (c < r)
template <typename T>
cr_status hole_gram_col(int ninj, const int32_t* hptr, const int32_t* hidx, int r,
                        const T* U, int64_t ldu, const T* w, double* out, int64_t ldo,
                        hipStream_t st);

}  // namespace cr

// preconditioner object of the C ABI
struct cr_pc {
  cr::LpcNet net;
  cr::LpcActs acts;
  hipStream_t st = nullptr;
  double* dwork = nullptr;  // FCG / training scratch (grown on demand)
  int64_t dwork_n = 0;
  double hloss = 0.0;
};
