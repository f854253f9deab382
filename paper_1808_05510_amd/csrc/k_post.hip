// Post-processing of a greedy solution W = U Z V^T (the steps after
// Algorithm 1 in the paper's real-data sections), FP64:
//  - the SVD of the small core by one-sided Jacobi rotations, giving the SVD
//    of W as (U Zu) diag(s) (V Zv)^T (section on the top-view results);
//  - products of tall voxel-length blocks with small r x r matrices;
//  - statistics over every entry of a low-rank W = A B^T on the FP64 matrix
//    cores (count and size of negative entries: section on dropping the
//    nonnegativity constraint), never storing W;
//  - deterministic sums of squares and the trace of a product of Grams.
#include <hip/hip_runtime.h>

#include "cr_internal.hpp"

#include <algorithm>

namespace cr {

// ============================================================== small-matrix products
// out[:, c] = s * sum_k M[:, k] op(B)[k, c], c < ncols, k < kd, with
// op(B)[k, c] = B[c, k] (transB) or B[k, c].  One thread per row, 32 output
// columns per workgroup column; B staged in LDS in chunks of 128 k.  With
// B == nullptr, out = s * M (kd = ncols; in place allowed).
__global__ __launch_bounds__(256) void k_tall_small(int64_t n, int kd, int ncols,
                                                    const double* __restrict__ M, int64_t ldm,
                                                    const double* __restrict__ B, int64_t ldb,
                                                    int transB, double s, double* out,
                                                    int64_t ldo) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c0 = blockIdx.y * 32;
  const int nc = min(32, ncols - c0);
  if (!B) {
    if (i < n)
      for (int c = 0; c < nc; ++c)
        out[(int64_t)(c0 + c) * ldo + i] = s * M[(int64_t)(c0 + c) * ldm + i];
    return;
  }
  __shared__ double bs[128][33];
  double acc[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) acc[c] = 0.0;
  for (int k0 = 0; k0 < kd; k0 += 128) {
    const int nk = min(128, kd - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * 128; e += 256) {
      const int c = e % 32, k = e / 32;
      double v = 0.0;
      if (c < nc && k < nk)
        v = transB ? B[(int64_t)(k0 + k) * ldb + c0 + c] : B[(int64_t)(c0 + c) * ldb + k0 + k];
      bs[k][c] = v;
    }
    __syncthreads();
    if (i < n)
      for (int k = 0; k < nk; ++k) {
        const double m = M[(int64_t)(k0 + k) * ldm + i];
#pragma unroll
        for (int c = 0; c < 32; ++c) acc[c] += m * bs[k][c];
      }
  }
  if (i < n)
#pragma unroll
    for (int c = 0; c < 32; ++c)
      if (c < nc) out[(int64_t)(c0 + c) * ldo + i] = s * acc[c];
}

cr_status tall_small(int64_t n, int kd, int ncols, const double* M, int64_t ldm, const double* B,
                     int64_t ldb, bool transB, double s, double* out, int64_t ldo,
                     hipStream_t st) {
  if (n == 0 || ncols == 0) return CR_OK;
  hipLaunchKernelGGL(k_tall_small, dim3((unsigned)((n + 255) / 256), (unsigned)((ncols + 31) / 32)),
                     dim3(256), 0, st, n, kd, ncols, M, ldm, B, ldb, transB ? 1 : 0, s, out, ldo);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// ============================================================== one-sided Jacobi SVD
// A (r x r, lda) is replaced column by column by rotations J_pq that make
// columns p and q orthogonal (Hestenes' one-sided Jacobi method); the same
// rotations accumulate in Vr (r x r, starts at I), so A_in Vr = A_out with
// orthogonal columns: A_in = (A_out / s) diag(s) Vr^T, s = column norms.
// Pairs are taken in round-robin tournament order (m - 1 rounds of m/2
// disjoint pairs per sweep, m = r rounded up to even): the pairs of a round
// are independent and are spread over the workgroup's waves.  Sweeps repeat
// until no pair has |a_p . a_q| > tol ||a_p|| ||a_q||, at most max_sweeps.
// info[0] = sweeps, info[1] = 1 when converged.
__device__ __forceinline__ double wsum64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

constexpr int SVD_NT = 1024;

__device__ __forceinline__ void tour_pair(int m, int round, int k, int& p, int& q) {
  // circle method: player m-1 fixed, the others rotate
  if (k == 0) {
    p = m - 1;
    q = round % (m - 1);
  } else {
    p = (round + k) % (m - 1);
    q = (round + m - 1 - k) % (m - 1);
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

__global__ __launch_bounds__(SVD_NT) void k_jacobi_svd(int r, double* __restrict__ A, int64_t lda,
                                                       double* __restrict__ Vr, int64_t ldv,
                                                       int max_sweeps, double tol,
                                                       double* __restrict__ info) {
  __shared__ int rotated;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = SVD_NT / 64;
  for (int64_t e = threadIdx.x; e < (int64_t)r * r; e += SVD_NT) {
    const int i = (int)(e % r), j = (int)(e / r);
    Vr[(int64_t)j * ldv + i] = i == j ? 1.0 : 0.0;
  }
  const int m = r + (r & 1);
  int sweep = 0, conv = 0;
  __syncthreads();
  while (sweep < max_sweeps && r > 1) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < m - 1; ++round) {
      for (int k = wv; k < m / 2; k += nw) {
        int p, q;
        tour_pair(m, round, k, p, q);
        if (q >= r) continue;  // the dummy player of an odd r
        double* ap = A + (int64_t)p * lda;
        double* aq = A + (int64_t)q * lda;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = lane; i < r; i += 64) {
          const double x = ap[i], y = aq[i];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
        al = wsum64(al);
        be = wsum64(be);
        ga = wsum64(ga);
        if (!(fabs(ga) > tol * sqrt(al * be))) continue;
        // rotation angle that zeroes the off-diagonal of [al ga; ga be]
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int i = lane; i < r; i += 64) {
          const double x = ap[i], y = aq[i];
          ap[i] = c * x - s * y;
          aq[i] = s * x + c * y;
        }
        double* vp = Vr + (int64_t)p * ldv;
        double* vq = Vr + (int64_t)q * ldv;
        for (int i = lane; i < r; i += 64) {
          const double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
        if (lane == 0) atomicAdd(&rotated, 1);
      }
      __threadfence_block();
      __syncthreads();
    }
    ++sweep;
    const int any = rotated;
    __syncthreads();
    if (!any) {
      conv = 1;
      break;
    }
  }
  if (r <= 1) conv = 1;
  if (threadIdx.x == 0) {
    info[0] = (double)sweep;
    info[1] = (double)conv;
  }
}

// s_j = ||A[:, j]||; column j goes to position rank(j) (descending s, ties by
// index): Uo[:, rank] = A[:, j] / s_j (0 when s_j = 0), Vo[:, rank] = Vr[:, j]
__global__ __launch_bounds__(NT) void k_svd_finish(int r, const double* __restrict__ A,
                                                   int64_t lda, const double* __restrict__ Vr,
                                                   int64_t ldv, double* __restrict__ sv,
                                                   double* __restrict__ Uo, int64_t ldu,
                                                   double* __restrict__ Vo, int64_t ldvo,
                                                   double* __restrict__ sout) {
  const int j = blockIdx.x;
  __shared__ double red[NT / 64];
  __shared__ int rk;
  double a = 0.0;
  for (int i = threadIdx.x; i < r; i += NT) {
    const double x = A[(int64_t)j * lda + i];
    a += x * x;
  }
  a = wsum64(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  const double nrm = sqrt(red[0] + red[1] + red[2] + red[3]);
  if (threadIdx.x == 0) {
    // rank among the column norms, computed from the same sums (sv holds
    // every column's squared norm from the previous pass)
    int k = 0;
    const double mine = sv[j];
    for (int q = 0; q < r; ++q) {
      const double o = sv[q];
      if (o > mine || (o == mine && q < j)) ++k;
    }
    rk = k;
    sout[k] = nrm;
  }
  __syncthreads();
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int i = threadIdx.x; i < r; i += NT) {
    Uo[(int64_t)rk * ldu + i] = A[(int64_t)j * lda + i] * inv;
    Vo[(int64_t)rk * ldvo + i] = Vr[(int64_t)j * ldv + i];
  }
}

__global__ __launch_bounds__(NT) void k_colsq(int r, const double* __restrict__ A, int64_t lda,
                                              double* __restrict__ sv) {
  const int j = blockIdx.x;
  __shared__ double red[NT / 64];
  double a = 0.0;
  for (int i = threadIdx.x; i < r; i += NT) {
    const double x = A[(int64_t)j * lda + i];
    a += x * x;
  }
  a = wsum64(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) sv[j] = red[0] + red[1] + red[2] + red[3];
}

// SVD of the r x r matrix in A (overwritten): A_in = Uo diag(s) Vo^T, s
// descending.  work: r*r (Vr) + r doubles; info: 2 doubles (sweeps, converged).
cr_status small_svd(int r, double* A, int64_t lda, double* Uo, int64_t ldu, double* s, double* Vo,
                    int64_t ldvo, double* work, double* info, hipStream_t st) {
  if (r <= 0) return CR_OK;
  double* Vr = work;
  double* sv = work + (int64_t)r * r;
  // rotation threshold: a few units of roundoff of an r-term dot product
  const double tol = std::max(1e-15, (double)r * 1.2e-16);
  hipLaunchKernelGGL(k_jacobi_svd, dim3(1), dim3(SVD_NT), 0, st, r, A, lda, Vr, (int64_t)r, 60,
                     tol, info);
  CR_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_colsq, dim3((unsigned)r), dim3(NT), 0, st, r, A, lda, sv);
  CR_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_svd_finish, dim3((unsigned)r), dim3(NT), 0, st, r, A, lda, Vr, (int64_t)r,
                     sv, Uo, ldu, Vo, ldvo, s);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// ============================================================== sums
// part[b] = sum of x[i]^2 over workgroup b's grid-stride share (n elements
// of a column-major n_rows x ncols block with leading dimension ld)
__global__ __launch_bounds__(NT) void k_sumsq_part(int64_t rows, int64_t cols,
                                                   const double* __restrict__ x, int64_t ld,
                                                   double* __restrict__ part) {
  __shared__ double red[NT / 64];
  const int64_t n = rows * cols;
  double a = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const double v = x[(e / rows) * ld + e % rows];
    a += v * v;
  }
  a = wsum64(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// out[0] = scale * sum_b part[b] (fixed order)
__global__ __launch_bounds__(64) void k_sum_final(int nb, const double* __restrict__ part,
                                                  double scale, double* __restrict__ out) {
  double a = 0.0;
  for (int b = threadIdx.x; b < nb; b += 64) a += part[b];
  a = wsum64(a);
  if (threadIdx.x == 0) out[0] = scale * a;
}

constexpr int SUMSQ_WG = 512;

// out[0] = scale * ||X||_F^2 (X rows x cols, ld); part: SUMSQ_WG doubles
cr_status sumsq(int64_t rows, int64_t cols, const double* x, int64_t ld, double scale,
                double* part, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sumsq_part, dim3(SUMSQ_WG), dim3(NT), 0, st, rows, cols, x, ld, part);
  CR_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(64), 0, st, SUMSQ_WG, part, scale, out);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// out[0] = scale * trace(P Q) = scale * sum_{i,j} P[i,j] Q[j,i] (m x m)
__global__ __launch_bounds__(NT) void k_trace_prod(int m, const double* __restrict__ P,
                                                   int64_t ldp, const double* __restrict__ Q,
                                                   int64_t ldq, double scale,
                                                   double* __restrict__ out) {
  __shared__ double red[NT / 64];
  double a = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += NT) {
    const int i = (int)(e % m), j = (int)(e / m);
    a += P[(int64_t)j * ldp + i] * Q[(int64_t)i * ldq + j];
  }
  a = wsum64(a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = scale * (red[0] + red[1] + red[2] + red[3]);
}

cr_status trace_prod(int m, const double* P, int64_t ldp, const double* Q, int64_t ldq,
                     double scale, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_trace_prod, dim3(1), dim3(NT), 0, st, m, P, ldp, Q, ldq, scale, out);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// ============================================================== entry statistics
// Statistics over every entry of W = A B^T (A na x k, B nb x k, FP64),
// without storing W.  Workgroup: 4 waves, output tiles of 64 x 64 entries
// (wave w owns the 32 x 32 quadrant (w % 2, w / 2): 2 x 2 blocks of the
// 16 x 16 x 4 FP64 MFMA), walking its row tile's column tiles with a grid
// stride.  A and B fragments come straight from global memory (each is
// reused by the other waves of the workgroup through L1/L2).  Per entry:
// negative count, min, max, max |w|, w^2 and w^2 of negative entries,
// reduced per workgroup into part[wg][ES_N] and then in a fixed order.
typedef double dbl4v __attribute__((ext_vector_type(4)));
constexpr int ES_N = 6, ES_T = 64;

__global__ __launch_bounds__(NT) void k_entry_stats(int64_t na, int64_t nb, int k,
                                                    const double* __restrict__ A, int64_t lda,
                                                    const double* __restrict__ B, int64_t ldb,
                                                    double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int fr = lane & 15, fk = lane >> 4;
  const int64_t rt = blockIdx.x;                      // row tile
  const int64_t nct = (nb + ES_T - 1) / ES_T;          // column tiles
  const int64_t r0 = rt * ES_T + 32 * (wv & 1);
  double cneg = 0.0, mn = INFINITY, mx = -INFINITY, mabs = 0.0, ss = 0.0, ssn = 0.0;
  for (int64_t ct = blockIdx.y; ct < nct; ct += gridDim.y) {
    const int64_t c0 = ct * ES_T + 32 * (wv >> 1);
    dbl4v acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = dbl4v{0.0, 0.0, 0.0, 0.0};
    for (int kk = 0; kk < k; kk += 4) {
      const int kq = kk + fk;
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int64_t row = r0 + 16 * a + fr;
        av[a] = (row < na && kq < k) ? A[(int64_t)kq * lda + row] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int64_t col = c0 + 16 * b + fr;
        bv[b] = (col < nb && kq < k) ? B[(int64_t)kq * ldb + col] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    // element e of lane l in block (a, b): row r0 + 16a + fk + 4e, column c0 + 16b + fr
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = r0 + 16 * a + fk + 4 * e;
          const int64_t col = c0 + 16 * b + fr;
          if (row < na && col < nb) {
            const double w = acc[a][b][e];
            const double w2 = w * w;
            ss += w2;
            mn = fmin(mn, w);
            mx = fmax(mx, w);
            mabs = fmax(mabs, fabs(w));
            if (w < 0.0) {
              cneg += 1.0;
              ssn += w2;
            }
          }
        }
  }
  // wave then workgroup reduction (fixed order)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    cneg += __shfl_xor(cneg, o, WAVE);
    ss += __shfl_xor(ss, o, WAVE);
    ssn += __shfl_xor(ssn, o, WAVE);
    mn = fmin(mn, __shfl_xor(mn, o, WAVE));
    mx = fmax(mx, __shfl_xor(mx, o, WAVE));
    mabs = fmax(mabs, __shfl_xor(mabs, o, WAVE));
  }
  __shared__ double red[4][ES_N];
  if (lane == 0) {
    red[wv][0] = cneg;
    red[wv][1] = mn;
    red[wv][2] = mx;
    red[wv][3] = mabs;
    red[wv][4] = ss;
    red[wv][5] = ssn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * ES_N;
    o[0] = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    o[1] = fmin(fmin(red[0][1], red[1][1]), fmin(red[2][1], red[3][1]));
    o[2] = fmax(fmax(red[0][2], red[1][2]), fmax(red[2][2], red[3][2]));
    o[3] = fmax(fmax(red[0][3], red[1][3]), fmax(red[2][3], red[3][3]));
    o[4] = red[0][4] + red[1][4] + red[2][4] + red[3][4];
    o[5] = red[0][5] + red[1][5] + red[2][5] + red[3][5];
  }
}

__global__ __launch_bounds__(64) void k_entry_stats_final(int64_t nwg,
                                                          const double* __restrict__ part,
                                                          double* __restrict__ out) {
  double cneg = 0.0, mn = INFINITY, mx = -INFINITY, mabs = 0.0, ss = 0.0, ssn = 0.0;
  for (int64_t b = threadIdx.x; b < nwg; b += 64) {
    const double* p = part + b * ES_N;
    cneg += p[0];
    mn = fmin(mn, p[1]);
    mx = fmax(mx, p[2]);
    mabs = fmax(mabs, p[3]);
    ss += p[4];
    ssn += p[5];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    cneg += __shfl_xor(cneg, o, WAVE);
    ss += __shfl_xor(ss, o, WAVE);
    ssn += __shfl_xor(ssn, o, WAVE);
    mn = fmin(mn, __shfl_xor(mn, o, WAVE));
    mx = fmax(mx, __shfl_xor(mx, o, WAVE));
    mabs = fmax(mabs, __shfl_xor(mabs, o, WAVE));
  }
  if (threadIdx.x == 0) {
    out[0] = cneg;
    out[1] = mn;
    out[2] = mx;
    out[3] = mabs;
    out[4] = ss;
    out[5] = ssn;
  }
}

int64_t entry_stats_part_size(int64_t na, int64_t nb) {
  const int64_t rt = (na + ES_T - 1) / ES_T, ct = (nb + ES_T - 1) / ES_T;
  return rt * std::min<int64_t>(ct, 16) * ES_N;
}

cr_status entry_stats(int64_t na, int64_t nb, int k, const double* A, int64_t lda,
                      const double* B, int64_t ldb, double* part, double* out, hipStream_t st) {
  const int64_t rt = (na + ES_T - 1) / ES_T, ct = (nb + ES_T - 1) / ES_T;
  if (rt == 0 || ct == 0) return CR_OK;
  if (rt > 0x7fffffff) {
    set_error("entry_stats: too many row tiles");
    return CR_EINVAL;
  }
  const unsigned gy = (unsigned)std::min<int64_t>(ct, 16);
  hipLaunchKernelGGL(k_entry_stats, dim3((unsigned)rt, gy), dim3(NT), 0, st, na, nb, k, A, lda, B,
                     ldb, part);
  CR_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_entry_stats_final, dim3(1), dim3(64), 0, st, rt * (int64_t)gy, part, out);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

}  // namespace cr

namespace cr {

// ============================================================== residual Grams in a capacity layout
// The Grams of the residual factors F = [N | U | L_y U | L_y^2 U] and
// G = [X | L_x^2 V | L_x V | V] keep block b (b = 0: n_inj columns, b = 1..3:
// r columns each) at a fixed offset ninj + (b - 1) rmax, so a new basis
// column only adds rows and columns instead of shifting the others.
__device__ __forceinline__ int cap_index(int c, int ninj, int r, int rmax) {
  if (c < ninj) return c;
  const int b = (c - ninj) / r, o = (c - ninj) % r;
  return ninj + b * rmax + o;
}

// C (m x n, ldc): row i is compact index row0 + i; column jj is compact
// index col0 + jj (newcol < 0), or the new column `newcol` of block jj + 1
// (newcol >= 0, n = 3).  Writes both (row, col) and (col, row) of Gc.
__global__ __launch_bounds__(NT) void k_gram_scatter(int m, int n, const double* __restrict__ C,
                                                     int64_t ldc, int row0, int col0, int newcol,
                                                     int ninj, int r, int rmax,
                                                     double* __restrict__ Gc, int64_t ldg) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)m * n) return;
  const int i = (int)(e % m), jj = (int)(e / m);
  const int ci = cap_index(row0 + i, ninj, r, rmax);
  const int cj = newcol >= 0 ? ninj + jj * rmax + newcol : cap_index(col0 + jj, ninj, r, rmax);
  const double v = C[(int64_t)jj * ldc + i];
  Gc[(int64_t)cj * ldg + ci] = v;
  Gc[(int64_t)ci * ldg + cj] = v;
}

// out (k x k compact, ld k) = Gc at the capacity positions
__global__ __launch_bounds__(NT) void k_gram_gather(int k, int ninj, int r, int rmax,
                                                    const double* __restrict__ Gc, int64_t ldg,
                                                    double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)k * k) return;
  const int i = (int)(e % k), j = (int)(e / k);
  out[e] = Gc[(int64_t)cap_index(j, ninj, r, rmax) * ldg + cap_index(i, ninj, r, rmax)];
}

cr_status gram_scatter(int m, int n, const double* C, int64_t ldc, int row0, int col0, int newcol,
                       int ninj, int r, int rmax, double* Gc, int64_t ldg, hipStream_t st) {
  const int64_t mn = (int64_t)m * n;
  if (mn == 0) return CR_OK;
  hipLaunchKernelGGL(k_gram_scatter, dim3((unsigned)((mn + NT - 1) / NT)), dim3(NT), 0, st, m, n,
                     C, ldc, row0, col0, newcol, ninj, r, rmax, Gc, ldg);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

cr_status gram_gather(int k, int ninj, int r, int rmax, const double* Gc, int64_t ldg, double* out,
                      hipStream_t st) {
  const int64_t kk = (int64_t)k * k;
  hipLaunchKernelGGL(k_gram_gather, dim3((unsigned)((kk + NT - 1) / NT)), dim3(NT), 0, st, k, ninj,
                     r, rmax, Gc, ldg, out);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// ============================================================== CholQR2 pieces
// s[i] = 1 / sqrt(A_ii) (0 for a zero column)
__global__ __launch_bounds__(NT) void k_diag_rsqrt(int k, const double* __restrict__ A, int64_t lda,
                                                   double* __restrict__ s) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= k) return;
  const double d = A[(int64_t)i * lda + i];
  s[i] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
}

// A <- diag(s) A diag(s); the diagonal entry of a zero column becomes 1 so
// that the Cholesky factor exists (s computed beforehand: no entry of A is
// read after another thread may have rescaled it)
__global__ __launch_bounds__(NT) void k_diag_apply(int k, double* __restrict__ A, int64_t lda,
                                                   const double* __restrict__ s) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)k * k) return;
  const int i = (int)(e % k), j = (int)(e / k);
  double* a = A + (int64_t)j * lda + i;
  *a = (i == j && s[i] == 0.0) ? 1.0 : *a * s[i] * s[j];
}

// In-place Cholesky A = L L^T (lower triangle of A, k <= a few thousand),
// right-looking, one workgroup; info[0] = 0 on success, j + 1 when pivot j
// is not positive.
constexpr int CH_NT = 1024;
__global__ __launch_bounds__(CH_NT) void k_chol(int k, double* __restrict__ A, int64_t lda,
                                                double* __restrict__ info) {
  __shared__ double dj;
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      const double p = A[(int64_t)j * lda + j];
      bad = !(p > 0.0) || !isfinite(p);
      dj = bad ? 1.0 : sqrt(p);
      A[(int64_t)j * lda + j] = dj;
    }
    __syncthreads();
    if (bad) {
      if (tid == 0) info[0] = (double)(j + 1);
      return;
    }
    const double inv = 1.0 / dj;
    for (int i = j + 1 + tid; i < k; i += CH_NT) A[(int64_t)j * lda + i] *= inv;
    __syncthreads();
    // trailing lower triangle: A[i, l] -= A[i, j] A[l, j], j < l <= i
    const int m = k - j - 1;
    const int64_t tri = (int64_t)m * (m + 1) / 2;
    for (int64_t e = tid; e < tri; e += CH_NT) {
      int row = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
      while ((int64_t)row * (row + 1) / 2 > e) --row;
      while ((int64_t)(row + 1) * (row + 2) / 2 <= e) ++row;
      const int col = (int)(e - (int64_t)row * (row + 1) / 2);
      const int i = j + 1 + row, l = j + 1 + col;
      A[(int64_t)l * lda + i] -= A[(int64_t)j * lda + i] * A[(int64_t)j * lda + l];
    }
    __syncthreads();
  }
  if (tid == 0) info[0] = 0.0;
}

// X = L^{-1} (lower triangular, k x k): thread j forms column j by forward
// substitution.  Entries above the diagonal of X are set to 0.
__global__ __launch_bounds__(NT) void k_trinv_lower(int k, const double* __restrict__ L,
                                                    int64_t ldl, double* __restrict__ X,
                                                    int64_t ldx) {
  const int j = blockIdx.x * NT + threadIdx.x;
  if (j >= k) return;
  double* x = X + (int64_t)j * ldx;
  for (int i = 0; i < j; ++i) x[i] = 0.0;
  x[j] = 1.0 / L[(int64_t)j * ldl + j];
  for (int i = j + 1; i < k; ++i) {
    double s = 0.0;
    for (int m = j; m < i; ++m) s += L[(int64_t)m * ldl + i] * x[m];
    x[i] = -s / L[(int64_t)i * ldl + i];
  }
}

// B[c, m] = X[c, m] * s[m] for an upper copy: out = diag? (here: scale
// column m of X by s[m]); and the upper factor R = L^T with column m scaled
// by 1 / s[m] (R1 S^-1).  mode 0: out = X diag(s); mode 1: out = L^T diag(1/s)
__global__ __launch_bounds__(NT) void k_tri_scale(int k, int mode, const double* __restrict__ X,
                                                  int64_t ldx, const double* __restrict__ s,
                                                  double* __restrict__ out, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)k * k) return;
  const int i = (int)(e % k), m = (int)(e / k);
  double v;
  if (mode == 0) {
    v = X[(int64_t)m * ldx + i] * s[m];
  } else {
    // (L^T)[i, m] = L[m, i] for m >= i (upper), zero below
    v = m >= i ? X[(int64_t)i * ldx + m] : 0.0;
    v = s[m] > 0.0 ? v / s[m] : 0.0;
  }
  out[(int64_t)m * ldo + i] = v;
}

cr_status chol_lower(int k, double* A, int64_t lda, double* info, hipStream_t st) {
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(CH_NT), 0, st, k, A, lda, info);
  CR_HIP(hipGetLastError());
  return CR_OK;
}
cr_status trinv_lower(int k, const double* L, int64_t ldl, double* X, int64_t ldx, hipStream_t st) {
  hipLaunchKernelGGL(k_trinv_lower, dim3((unsigned)((k + NT - 1) / NT)), dim3(NT), 0, st, k, L, ldl,
                     X, ldx);
  CR_HIP(hipGetLastError());
  return CR_OK;
}
cr_status diag_scale(int k, double* A, int64_t lda, double* s, hipStream_t st) {
  const int64_t kk = (int64_t)k * k;
  hipLaunchKernelGGL(k_diag_rsqrt, dim3((unsigned)((k + NT - 1) / NT)), dim3(NT), 0, st, k, A, lda,
                     s);
  CR_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_diag_apply, dim3((unsigned)((kk + NT - 1) / NT)), dim3(NT), 0, st, k, A, lda,
                     s);
  CR_HIP(hipGetLastError());
  return CR_OK;
}
cr_status tri_scale(int k, int mode, const double* X, int64_t ldx, const double* s, double* out,
                    int64_t ldo, hipStream_t st) {
  const int64_t kk = (int64_t)k * k;
  hipLaunchKernelGGL(k_tri_scale, dim3((unsigned)((kk + NT - 1) / NT)), dim3(NT), 0, st, k, mode, X,
                     ldx, s, out, ldo);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

}  // namespace cr

namespace cr {

// ============================================================== two-level coarse operator
// A = lam (C2 + c1 C1 + c0 I) + Y diag(gw) Y^T  (m x m, all column-major, Y m x ninj)
__global__ __launch_bounds__(NT) void k_coarse_assemble(int m, double lam,
                                                        const double* __restrict__ coef,
                                                        const double* __restrict__ C1,
                                                        const double* __restrict__ C2,
                                                        const double* __restrict__ Y, int ninj,
                                                        const double* __restrict__ gw,
                                                        double* __restrict__ A) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  const int i = (int)(e % m), j = (int)(e / m);
  double v = lam * (C2[e] + coef[0] * C1[e] + (i == j ? coef[1] : 0.0));
  if (Y)
    for (int al = 0; al < ninj; ++al) v += Y[(int64_t)al * m + i] * gw[al] * Y[(int64_t)al * m + j];
  A[e] = v;
}

// X = L^-1 for the lower triangle L of A (k x k), one workgroup, row by row:
// X[i, i] = 1 / L_ii, X[i, j] = -(1 / L_ii) sum_{j <= q < i} L[i, q] X[q, j].
// Skipped (X left zero) when info[0] reports a failed factorisation.
__global__ __launch_bounds__(CH_NT) void k_trinv_rows(int k, const double* __restrict__ L,
                                                      int64_t ldl, double* __restrict__ X,
                                                      int64_t ldx,
                                                      const double* __restrict__ info) {
  const int tid = threadIdx.x;
  for (int64_t e = tid; e < (int64_t)k * k; e += CH_NT) X[(e / k) * ldx + e % k] = 0.0;
  __syncthreads();
  if (info[0] != 0.0) return;
  for (int i = 0; i < k; ++i) {
    const double inv = 1.0 / L[(int64_t)i * ldl + i];
    for (int j = tid; j < i; j += CH_NT) {
      double s = 0.0;
      for (int q = j; q < i; ++q) s += L[(int64_t)q * ldl + i] * X[(int64_t)j * ldx + q];
      X[(int64_t)j * ldx + i] = -inv * s;
    }
    if (tid == 0) X[(int64_t)i * ldx + i] = inv;
    __syncthreads();
  }
}

cr_status coarse_assemble(int m, double lam, const double* coef, const double* C1,
                          const double* C2, const double* Y, int ninj, const double* gw, double* A,
                          hipStream_t st) {
  const int64_t mm = (int64_t)m * m;
  hipLaunchKernelGGL(k_coarse_assemble, dim3((unsigned)((mm + NT - 1) / NT)), dim3(NT), 0, st, m,
                     lam, coef, C1, C2, Y, ninj, gw, A);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

cr_status trinv_rows(int k, const double* L, int64_t ldl, double* X, int64_t ldx,
                     const double* info, hipStream_t st) {
  hipLaunchKernelGGL(k_trinv_rows, dim3(1), dim3(CH_NT), 0, st, k, L, ldl, X, ldx, info);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

}  // namespace cr
