// Spectral solves on a full box.  With voxels numbered first axis fastest,
// the graph Laplacian of a d0 x d1 x d2 box with free (Neumann) faces is
// Q diag(mu) Q^T, Q = Q2 (x) Q1 (x) Q0, where Q_a holds the eigenvectors of
// the path-graph Laplacian of length m = d_a: column k is
// cos(pi k (j + 1/2) / m) normalised, eigenvalue 2 - 2 cos(pi k / m), and
// mu(k0, k1, k2) = mu0[k0] + mu1[k1] + mu2[k2].
//
// The u-system matrix of eq. ALS_linsys is lam (L^2 + 2 b L + a I) + diag(d)
// (b = v^T L_x v, a = ||L_x v||^2, d the masked quadratic forms).  With d
// replaced by its mean dbar it is diagonal in Q, so
//     M^-1 r = Q diag(1 / (lam (mu^2 + 2 b mu + a) + dbar)) Q^T r
// is an SPD approximate inverse, exact where d is constant; it serves as the
// base step of the flexible CG (alone, or refined by the learned network).
// On the source box the same transforms solve the v-system exactly through
// the Sherman-Morrison-Woodbury identity (below).
#include <hip/hip_runtime.h>

#include "cr_internal.hpp"

namespace cr {

// one 1-D transform along `axis` for every pencil of the box:
//   forward (Q^T):  out[.., k, ..] = sum_j Q[j m + k] in[.., j, ..]
//   inverse (Q):    out[.., j, ..] = sum_k Q[j m + k] in[.., k, ..]
// Q is row-major m x m (row = position j, column = mode k).
// blockIdx.y selects the column of an n x ncols block (leading dimensions
// ldi, ldo).  Index arithmetic is 32-bit (the box has fewer than 2^31
// voxels, checked when the basis is built) and the m-term sum runs four
// independent partial sums, so the loads of several terms are in flight at
// once: the transform is latency-bound at these sizes.
__global__ __launch_bounds__(NT) void k_box_axis(int d0, int d1, int d2, int axis,
                                                 const double* __restrict__ Q, int inverse,
                                                 const double* __restrict__ in, int64_t ldi,
                                                 double* __restrict__ out, int64_t ldo) {
  const int n = d0 * d1 * d2;
  const int o = blockIdx.x * NT + threadIdx.x;
  if (o >= n) return;
  in += (int64_t)blockIdx.y * ldi;
  out += (int64_t)blockIdx.y * ldo;
  int t, s, m;
  if (axis == 0) {
    t = o % d0;
    s = 1;
    m = d0;
  } else if (axis == 1) {
    t = (o / d0) % d1;
    s = d0;
    m = d1;
  } else {
    s = d0 * d1;
    t = o / s;
    m = d2;
  }
  const double* ib = in + (o - t * s);
  // inverse: coefficients Q[t m + k] (stride 1); forward: Q[k m + t] (stride m)
  const double* q = inverse ? Q + t * m : Q + t;
  const int qs = inverse ? 1 : m;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int k = 0;
  for (; k + 4 <= m; k += 4) {
    a0 += q[k * qs] * ib[k * s];
    a1 += q[(k + 1) * qs] * ib[(k + 1) * s];
    a2 += q[(k + 2) * qs] * ib[(k + 2) * s];
    a3 += q[(k + 3) * qs] * ib[(k + 3) * s];
  }
  for (; k < m; ++k) a0 += q[k * qs] * ib[k * s];
  out[o] = (a0 + a1) + (a2 + a3);
}

// xhat /= lam (mu^2 + c[0] mu + c[1]) + dbar   (c = [2 b, a]; dbar may be null: 0)
__global__ __launch_bounds__(NT) void k_box_scale(int d0, int d1, int d2,
                                                  const double* __restrict__ mu0,
                                                  const double* __restrict__ mu1,
                                                  const double* __restrict__ mu2,
                                                  const double* __restrict__ c, double lam,
                                                  const double* __restrict__ dbar,
                                                  double* __restrict__ xh, int64_t ld) {
  const int64_t n = (int64_t)d0 * d1 * d2;
  const int64_t o = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (o >= n) return;
  xh += (int64_t)blockIdx.y * ld;
  const int i0 = (int)(o % d0);
  const int64_t rest = o / d0;
  const int i1 = (int)(rest % d1);
  const int i2 = (int)(rest / d1);
  const double mu = mu0[i0] + mu1[i1] + mu2[i2];
  const double den = lam * (mu * mu + c[0] * mu + c[1]) + (dbar ? dbar[0] : 0.0);
  xh[o] = xh[o] / den;
}

cr_status box_spectral_solve(const BoxBasis& bx, const double* c, double lam, const double* dbar,
                             const double* r, double* out, double* tmp, hipStream_t st) {
  const int64_t n = (int64_t)bx.dims[0] * bx.dims[1] * bx.dims[2];
  return box_spectral_solve_cols(bx, c, lam, dbar, 1, r, n, out, n, tmp, n, st);
}

cr_status box_spectral_solve_cols(const BoxBasis& bx, const double* c, double lam,
                                  const double* dbar, int ncols, const double* R, int64_t ldr,
                                  double* OUT, int64_t ldo, double* TMP, int64_t ldt,
                                  hipStream_t st) {
  if (ncols <= 0) return CR_OK;
  const int64_t n = (int64_t)bx.dims[0] * bx.dims[1] * bx.dims[2];
  const dim3 g((unsigned)((n + NT - 1) / NT), (unsigned)ncols);
  const int d0 = bx.dims[0], d1 = bx.dims[1], d2 = bx.dims[2];
  // forward: R -> TMP -> OUT -> TMP
  hipLaunchKernelGGL(k_box_axis, g, dim3(NT), 0, st, d0, d1, d2, 0, bx.Q[0], 0, R, ldr, TMP, ldt);
  hipLaunchKernelGGL(k_box_axis, g, dim3(NT), 0, st, d0, d1, d2, 1, bx.Q[1], 0, TMP, ldt, OUT, ldo);
  hipLaunchKernelGGL(k_box_axis, g, dim3(NT), 0, st, d0, d1, d2, 2, bx.Q[2], 0, OUT, ldo, TMP, ldt);
  hipLaunchKernelGGL(k_box_scale, g, dim3(NT), 0, st, d0, d1, d2, bx.mu[0], bx.mu[1], bx.mu[2], c,
                     lam, dbar, TMP, ldt);
  // inverse: TMP -> OUT -> TMP -> OUT
  hipLaunchKernelGGL(k_box_axis, g, dim3(NT), 0, st, d0, d1, d2, 2, bx.Q[2], 1, TMP, ldt, OUT, ldo);
  hipLaunchKernelGGL(k_box_axis, g, dim3(NT), 0, st, d0, d1, d2, 1, bx.Q[1], 1, OUT, ldo, TMP, ldt);
  hipLaunchKernelGGL(k_box_axis, g, dim3(NT), 0, st, d0, d1, d2, 0, bx.Q[0], 1, TMP, ldt, OUT, ldo);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

cr_status box_transform_cols(const BoxBasis& bx, bool inverse, int ncols, const double* R,
                             int64_t ldr, double* OUT, int64_t ldo, double* TMP, int64_t ldt,
                             hipStream_t st) {
  if (ncols <= 0) return CR_OK;
  const int64_t n = (int64_t)bx.dims[0] * bx.dims[1] * bx.dims[2];
  const dim3 g((unsigned)((n + NT - 1) / NT), (unsigned)ncols);
  const int d0 = bx.dims[0], d1 = bx.dims[1], d2 = bx.dims[2];
  const int inv = inverse ? 1 : 0;
  // forward: axes 0, 1, 2; inverse: axes 2, 1, 0 (R -> OUT -> TMP -> OUT)
  const int a0 = inverse ? 2 : 0, a2 = inverse ? 0 : 2;
  hipLaunchKernelGGL(k_box_axis, g, dim3(NT), 0, st, d0, d1, d2, a0, bx.Q[a0], inv, R, ldr, OUT, ldo);
  hipLaunchKernelGGL(k_box_axis, g, dim3(NT), 0, st, d0, d1, d2, 1, bx.Q[1], inv, OUT, ldo, TMP, ldt);
  hipLaunchKernelGGL(k_box_axis, g, dim3(NT), 0, st, d0, d1, d2, a2, bx.Q[a2], inv, TMP, ldt, OUT, ldo);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

cr_status box_scale_cols(const BoxBasis& bx, const double* c, double lam, const double* dbar,
                         int ncols, double* XH, int64_t ld, hipStream_t st) {
  if (ncols <= 0) return CR_OK;
  const int64_t n = (int64_t)bx.dims[0] * bx.dims[1] * bx.dims[2];
  const dim3 g((unsigned)((n + NT - 1) / NT), (unsigned)ncols);
  hipLaunchKernelGGL(k_box_scale, g, dim3(NT), 0, st, bx.dims[0], bx.dims[1], bx.dims[2],
                     bx.mu[0], bx.mu[1], bx.mu[2], c, lam, dbar, XH, ld);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// ---------------------------------------------------------------- v-system by SMW
// The v-system of eq. ALS_linsys_v is S + X G X^T with S = lam (L_x^2 + 2 c L_x
// + e I), diagonal in the source box's basis, and G = diag(g), g >= 0.  With
// W = X G^1/2, the Sherman-Morrison-Woodbury identity gives
//   (S + W W^T)^-1 b = S^-1 (b + X k),  k = -G^1/2 K^-1 G^1/2 X^T S^-1 b,
//   K = I + G^1/2 X^T S^-1 X G^1/2  (SPD, n_inj x n_inj),
// the paper's SMW route for this system with the spectral solve in place of
// a sparse factorisation.  With S = Q diag(s) Q^T and Xh = Q^T X (fixed per
// handle), X^T S^-1 X = Xh^T diag(1/s) Xh and X^T S^-1 b = Xh^T (bh / s), so
// one solve needs single-column transforms only.  K is factored (Cholesky)
// by one workgroup in LDS.

// K (n x n, column-major, holds the Gram X^T S^-1 X on entry) <- lower
// Cholesky factor of I + G^1/2 sym(K) G^1/2; a non-positive pivot leaves NaN
// in the factor (the caller's residual check then rejects the solve).
// Right-looking, one barrier per column: step k updates the trailing lower
// triangle with A_ik A_jk / A_kk (no square root needed there) and writes the
// scaled column L_ik = A_ik / sqrt(A_kk) into the upper triangle, which no
// thread reads; the diagonal goes to its own array.
constexpr int SMW_NT = 1024;

__global__ __launch_bounds__(SMW_NT) void k_smw_factor(int n, const double* __restrict__ g,
                                                       double* __restrict__ K) {
  __shared__ double A[SMW_MAX][SMW_MAX + 1];
  __shared__ double dg[SMW_MAX];
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += SMW_NT) {
    const int i = e % n, j = e / n;
    const double v = 0.5 * (K[(int64_t)j * n + i] + K[(int64_t)i * n + j]);
    A[i][j] = sqrt(g[i] * g[j]) * v + (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const double akk = A[k][k];
    const double inv = 1.0 / akk;
    const double rs = akk > 0.0 ? 1.0 / sqrt(akk) : __builtin_nan("");
    const int m = n - k - 1;
    // trailing lower triangle (k < j <= i < n) over the m x m square
    for (int e = tid; e < m * m; e += SMW_NT) {
      const int a = e / m, b = e - a * m;
      if (b <= a) {
        const int i = k + 1 + a, j = k + 1 + b;
        A[i][j] -= A[i][k] * A[j][k] * inv;
      }
    }
    for (int i = k + 1 + tid; i < n; i += SMW_NT) A[k][i] = A[i][k] * rs;
    if (tid == 0) dg[k] = akk > 0.0 ? sqrt(akk) : __builtin_nan("");
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += SMW_NT) {
    const int i = e % n, j = e / n;
    K[(int64_t)j * n + i] = j < i ? A[j][i] : (j == i ? dg[i] : 0.0);
  }
}

// kvec = -G^1/2 K^-1 G^1/2 h with K = L L^T (L from k_smw_factor): the
// workgroup stages L in LDS, then one wave solves L y = z and L^T w = y with
// rows i and i + 64 in lane i % 64 and the pivot broadcast by a shuffle.
__global__ __launch_bounds__(NT) void k_smw_apply(int n, const double* __restrict__ g,
                                                  const double* __restrict__ L,
                                                  const double* __restrict__ h,
                                                  double* __restrict__ kvec) {
  __shared__ double Ls[SMW_MAX * SMW_MAX];
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += NT) Ls[e] = L[e];
  __syncthreads();
  if (tid >= WAVE) return;
  const int lane = tid;
  const int i0 = lane, i1 = lane + WAVE;
  double z0 = i0 < n ? sqrt(g[i0]) * h[i0] : 0.0;
  double z1 = i1 < n ? sqrt(g[i1]) * h[i1] : 0.0;
  for (int j = 0; j < n; ++j) {  // L y = z (column j: L(i, j) = Ls[j n + i])
    const int src = j & (WAVE - 1);
    const double zj = __shfl(j < WAVE ? z0 : z1, src, WAVE) / Ls[j * n + j];
    if (i0 == j) z0 = zj;
    if (i1 == j) z1 = zj;
    if (i0 > j && i0 < n) z0 -= Ls[j * n + i0] * zj;
    if (i1 > j && i1 < n) z1 -= Ls[j * n + i1] * zj;
  }
  for (int j = n - 1; j >= 0; --j) {  // L^T w = y (row j of L^T: L(j, i) = Ls[i n + j])
    const int src = j & (WAVE - 1);
    const double zj = __shfl(j < WAVE ? z0 : z1, src, WAVE) / Ls[j * n + j];
    if (i0 == j) z0 = zj;
    if (i1 == j) z1 = zj;
    if (i0 < j) z0 -= Ls[i0 * n + j] * zj;
    if (i1 < j) z1 -= Ls[i1 * n + j] * zj;
  }
  if (i0 < n) kvec[i0] = -sqrt(g[i0]) * z0;
  if (i1 < n) kvec[i1] = -sqrt(g[i1]) * z1;
}

cr_status smw_factor(int n, const double* g, double* K, hipStream_t st) {
  if (n < 1 || n > SMW_MAX) {
    set_error("SMW factor: n_inj out of range");
    return CR_EINVAL;
  }
  hipLaunchKernelGGL(k_smw_factor, dim3(1), dim3(SMW_NT), 0, st, n, g, K);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

cr_status smw_apply(int n, const double* g, const double* L, const double* h, double* kvec,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_smw_apply, dim3(1), dim3(NT), 0, st, n, g, L, h, kvec);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

}  // namespace cr
