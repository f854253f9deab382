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
#include <hip/hip_runtime.h>

#include "cr_internal.hpp"

namespace cr {

// one 1-D transform along `axis` for every pencil of the box:
//   forward (Q^T):  out[.., k, ..] = sum_j Q[j m + k] in[.., j, ..]
//   inverse (Q):    out[.., j, ..] = sum_k Q[j m + k] in[.., k, ..]
// Q is row-major m x m (row = position j, column = mode k).
__global__ __launch_bounds__(NT) void k_box_axis(int d0, int d1, int d2, int axis,
                                                 const double* __restrict__ Q, int inverse,
                                                 const double* __restrict__ in,
                                                 double* __restrict__ out) {
  const int64_t n = (int64_t)d0 * d1 * d2;
  const int64_t o = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (o >= n) return;
  const int i0 = (int)(o % d0);
  const int64_t rest = o / d0;
  const int i1 = (int)(rest % d1);
  const int i2 = (int)(rest / d1);
  const int m = axis == 0 ? d0 : axis == 1 ? d1 : d2;
  const int t = axis == 0 ? i0 : axis == 1 ? i1 : i2;
  const int64_t s = axis == 0 ? 1 : axis == 1 ? (int64_t)d0 : (int64_t)d0 * d1;
  const int64_t base = o - (int64_t)t * s;
  double acc = 0.0;
  if (inverse) {
    const double* qrow = Q + (int64_t)t * m;
    for (int k = 0; k < m; ++k) acc += qrow[k] * in[base + k * s];
  } else {
    for (int j = 0; j < m; ++j) acc += Q[(int64_t)j * m + t] * in[base + j * s];
  }
  out[o] = acc;
}

// xhat /= lam (mu^2 + c[0] mu + c[1]) + dbar   (c = [2 b, a])
__global__ __launch_bounds__(NT) void k_box_scale(int d0, int d1, int d2,
                                                  const double* __restrict__ mu0,
                                                  const double* __restrict__ mu1,
                                                  const double* __restrict__ mu2,
                                                  const double* __restrict__ c, double lam,
                                                  const double* __restrict__ dbar,
                                                  double* __restrict__ xh) {
  const int64_t n = (int64_t)d0 * d1 * d2;
  const int64_t o = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (o >= n) return;
  const int i0 = (int)(o % d0);
  const int64_t rest = o / d0;
  const int i1 = (int)(rest % d1);
  const int i2 = (int)(rest / d1);
  const double mu = mu0[i0] + mu1[i1] + mu2[i2];
  const double den = lam * (mu * mu + c[0] * mu + c[1]) + dbar[0];
  xh[o] = xh[o] / den;
}

cr_status box_spectral_solve(const BoxBasis& bx, const double* c, double lam, const double* dbar,
                             const double* r, double* out, double* tmp, hipStream_t st) {
  const int64_t n = (int64_t)bx.dims[0] * bx.dims[1] * bx.dims[2];
  const unsigned g = (unsigned)((n + NT - 1) / NT);
  const int d0 = bx.dims[0], d1 = bx.dims[1], d2 = bx.dims[2];
  // forward: r -> tmp -> out -> tmp
  hipLaunchKernelGGL(k_box_axis, dim3(g), dim3(NT), 0, st, d0, d1, d2, 0, bx.Q[0], 0, r, tmp);
  hipLaunchKernelGGL(k_box_axis, dim3(g), dim3(NT), 0, st, d0, d1, d2, 1, bx.Q[1], 0, tmp, out);
  hipLaunchKernelGGL(k_box_axis, dim3(g), dim3(NT), 0, st, d0, d1, d2, 2, bx.Q[2], 0, out, tmp);
  hipLaunchKernelGGL(k_box_scale, dim3(g), dim3(NT), 0, st, d0, d1, d2, bx.mu[0], bx.mu[1],
                     bx.mu[2], c, lam, dbar, tmp);
  // inverse: tmp -> out -> tmp -> out
  hipLaunchKernelGGL(k_box_axis, dim3(g), dim3(NT), 0, st, d0, d1, d2, 2, bx.Q[2], 1, tmp, out);
  hipLaunchKernelGGL(k_box_axis, dim3(g), dim3(NT), 0, st, d0, d1, d2, 1, bx.Q[1], 1, out, tmp);
  hipLaunchKernelGGL(k_box_axis, dim3(g), dim3(NT), 0, st, d0, d1, d2, 0, bx.Q[0], 1, tmp, out);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

}  // namespace cr
