// Streaming kernels of the greedy low-rank solver (gfx950, wave64):
// graph-Laplacian stencils, tall-skinny products over voxel-length columns,
// the masked products of the data term, and small helpers.
#include <hip/hip_runtime.h>

#include "cr_internal.hpp"

namespace cr {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// ============================================================== stencil
// (L w)_i = K w_i - sum_k w[nbr_k(i)] : with self-padded absent neighbours
// this equals deg_i w_i - sum_{j adjacent} w_j, the graph Laplacian row.
// Workgroups are dispatched round-robin over the 8 XCDs (physical block b
// runs on XCD b % 8); the logical voxel block is remapped so that each XCD
// sweeps one contiguous eighth of the voxels and finds neighbouring planes
// in its own L2.  Each thread handles SCOL columns with independent loads.
constexpr int NXCD = 8;
constexpr int SCOL = 8;

__device__ __forceinline__ int64_t xcd_block(unsigned b, unsigned nb_log) {
  const unsigned per = (nb_log + NXCD - 1) / NXCD;
  return (int64_t)(b % NXCD) * per + b / NXCD;
}

template <typename T, int K>
__global__ __launch_bounds__(NT) void k_stencil(int64_t n, const int32_t* __restrict__ nbr,
                                                int ncols, const T* __restrict__ w, int64_t ldw,
                                                T* __restrict__ out, int64_t ldo,
                                                unsigned nb_log) {
  const int64_t lb = xcd_block(blockIdx.x, nb_log);
  if (lb >= nb_log) return;
  const int64_t i = lb * NT + threadIdx.x;
  if (i >= n) return;
  int32_t nb[K];
#pragma unroll
  for (int k = 0; k < K; ++k) nb[k] = nbr[(int64_t)k * n + i];
  const int c0 = blockIdx.y * SCOL;
  if (c0 + SCOL <= ncols) {
    T s[SCOL];
#pragma unroll
    for (int c = 0; c < SCOL; ++c) {
      const T* wc = w + (int64_t)(c0 + c) * ldw;
      T v = (T)K * wc[i];
#pragma unroll
      for (int k = 0; k < K; ++k) v -= wc[nb[k]];
      s[c] = v;
    }
#pragma unroll
    for (int c = 0; c < SCOL; ++c) out[(int64_t)(c0 + c) * ldo + i] = s[c];
  } else {
    for (int c = c0; c < ncols; ++c) {
      const T* wc = w + (int64_t)c * ldw;
      T v = (T)K * wc[i];
#pragma unroll
      for (int k = 0; k < K; ++k) v -= wc[nb[k]];
      out[(int64_t)c * ldo + i] = v;
    }
  }
}

// Window form (many columns): workgroup = one tile of NT voxels x a chunk of
// columns.  Per column, the tile's window (the voxels its rows read, as index
// intervals) is staged into LDS with coalesced loads, double-buffered so the
// next column's loads are in flight while the current one is computed from
// LDS; each row then reads itself and its neighbours at precomputed window
// positions.  Measured 10-20% faster than the gather form on the shell
// geometry (FP32 data), whose neighbour planes are a few thousand voxels
// apart.
constexpr int WIN_EPT = WIN_MAX / NT;  // window elements staged per thread

template <typename T, int K>
__global__ __launch_bounds__(NT) void k_stencil_win(int64_t n, unsigned nt_log,
                                                    const int32_t* __restrict__ itab,
                                                    const uint16_t* __restrict__ wpos, int ncols,
                                                    int cchunk, const T* __restrict__ w,
                                                    int64_t ldw, T* __restrict__ out,
                                                    int64_t ldo) {
  __shared__ T buf[2][WIN_MAX];
  const int64_t tile = xcd_block(blockIdx.x, nt_log);
  if (tile >= nt_log) return;  // uniform per workgroup
  const int cb = blockIdx.y * cchunk;
  const int ce = min(ncols, cb + cchunk);
  if (cb >= ce) return;  // uniform per workgroup
  const int tid = threadIdx.x;
  const int32_t* it = itab + tile * WIN_TAB;
  const int nint = it[0], tot = it[1];
  int src[WIN_EPT];
#pragma unroll
  for (int m = 0; m < WIN_EPT; ++m) {
    const int e = tid + NT * m;
    int sv = -1;
    if (e < tot) {
      int q = 0;
      for (int k = 1; k < nint; ++k)
        if (it[2 + WIN_NI + k] <= e) q = k;
      sv = it[2 + q] + (e - it[2 + WIN_NI + q]);
    }
    src[m] = sv;
  }
  const int64_t i = tile * NT + tid;
  const bool valid = i < n;
  int q0 = 0, q1[K];
#pragma unroll
  for (int k = 0; k < K; ++k) q1[k] = 0;
  if (valid) {
    q0 = wpos[i];
#pragma unroll
    for (int k = 0; k < K; ++k) q1[k] = wpos[(int64_t)(k + 1) * n + i];
  }
  T rg[WIN_EPT];
  auto load = [&](int c) {
    const T* wc = w + (int64_t)c * ldw;
#pragma unroll
    for (int m = 0; m < WIN_EPT; ++m) rg[m] = src[m] >= 0 ? wc[src[m]] : (T)0;
  };
  auto stage = [&](int b) {
#pragma unroll
    for (int m = 0; m < WIN_EPT; ++m)
      if (tid + NT * m < tot) buf[b][tid + NT * m] = rg[m];
  };
  load(cb);
  stage(0);
  __syncthreads();
  for (int c = cb; c < ce; ++c) {
    const int b = (c - cb) & 1;
    if (c + 1 < ce) load(c + 1);
    if (valid) {
      const T* B = buf[b];
      T v = (T)K * B[q0];
#pragma unroll
      for (int k = 0; k < K; ++k) v -= B[q1[k]];
      out[(int64_t)c * ldo + i] = v;
    }
    if (c + 1 < ce) stage(b ^ 1);
    __syncthreads();
  }
}

template <typename T>
cr_status stencil(const Geom& g, int ncols, const T* w, int64_t ldw, T* out, int64_t ldo,
                  hipStream_t st) {
  if (ncols <= 0 || g.n == 0) return CR_OK;
  const unsigned nb_log = (unsigned)((g.n + NT - 1) / NT);
  const unsigned nb_phys = (nb_log + NXCD - 1) / NXCD * NXCD;
  // FP32 data only: for FP64 the window form is faster alone (153 against
  // 163 us on the shell target side, r = 100) but slower inside the forked
  // operator application (806 against 769 us), where its LDS and register
  // needs compete with the concurrent masked product
  if (sizeof(T) == 4 && g.witab && ncols >= SCOL) {
    // column chunks so that the launch has about 2048 workgroups
    const int nsplit = std::max(1, std::min({4, ncols / 2, (int)(2048 / nb_log)}));
    const int cchunk = (ncols + nsplit - 1) / nsplit;
    dim3 wg(nb_phys, (unsigned)((ncols + cchunk - 1) / cchunk));
    switch (g.K) {
#define WCASE(KK)                                                                          \
  case KK:                                                                                 \
    hipLaunchKernelGGL((k_stencil_win<T, KK>), wg, dim3(NT), 0, st, g.n, nb_log, g.witab, \
                       g.wpos, ncols, cchunk, w, ldw, out, ldo);                           \
    break;
      WCASE(2) WCASE(4) WCASE(6) WCASE(8)
#undef WCASE
      default:
        set_error("stencil width out of range");
        return CR_EINVAL;
    }
    CR_HIP(hipGetLastError());
    return CR_OK;
  }
  dim3 grid(nb_phys, (unsigned)((ncols + SCOL - 1) / SCOL));
  switch (g.K) {
#define CASE(KK)                                                                         \
  case KK:                                                                               \
    hipLaunchKernelGGL((k_stencil<T, KK>), grid, dim3(NT), 0, st, g.n, g.nbr, ncols, w, \
                       ldw, out, ldo, nb_log);                                           \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default:
      set_error("stencil width out of range");
      return CR_EINVAL;
  }
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// ============================================================== gemv_t
// y = A^T x.  Workgroup b owns rows [b*RB, (b+1)*RB), RB = 64*RPL; wave w of
// the 4 handles columns w, w+4, ...; lane l owns rows b*RB + l + 64 m, so
// every column read is a coalesced 64-wide load.  Partial sums per
// (column, workgroup) go to `part`; a second kernel sums them in a fixed
// order (deterministic).
constexpr int GT_RPL = 8;
constexpr int GT_RB = 64 * GT_RPL;

template <typename T, typename TX>
__global__ __launch_bounds__(NT) void k_gemv_t(int64_t n, Blocks<T> A, const TX* __restrict__ x,
                                               double* __restrict__ part, int nrb) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int64_t r0 = (int64_t)blockIdx.x * GT_RB + lane;
  double xv[GT_RPL];
#pragma unroll
  for (int m = 0; m < GT_RPL; ++m) {
    int64_t row = r0 + 64 * m;
    xv[m] = row < n ? (double)x[row] : 0.0;
  }
  const int nc = A.ncols();
  const bool full = (int64_t)(blockIdx.x + 1) * GT_RB <= n;
  // grid.y splits the columns in groups of 16 (4 per wave): a tall product
  // of a few hundred columns then launches nrb x ncols/16 workgroups instead
  // of nrb (125 at 64,000 rows), enough loads in flight to reach HBM speed
  for (int c0 = (int)blockIdx.y * 16 + wv; c0 < nc; c0 += 16 * (int)gridDim.y) {
    double acc[4] = {0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int c = c0 + 4 * u;
      if (c < nc) {
        const T* col = A.col(c);
        if (full) {
#pragma unroll
          for (int m = 0; m < GT_RPL; ++m) acc[u] += (double)col[r0 + 64 * m] * xv[m];
        } else {
#pragma unroll
          for (int m = 0; m < GT_RPL; ++m) {
            int64_t row = r0 + 64 * m;
            if (row < n) acc[u] += (double)col[row] * xv[m];
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int c = c0 + 4 * u;
      double s = wave_sum(acc[u]);
      if (lane == 0 && c < nc) part[(int64_t)c * nrb + blockIdx.x] = s;
    }
  }
}

// y[c] = sum_b part[c*nrb + b], one wave per column, fixed order.
__global__ __launch_bounds__(NT) void k_reduce_part(int ncols, int nrb,
                                                    const double* __restrict__ part,
                                                    double* __restrict__ y) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int c = blockIdx.x * (NT / WAVE) + threadIdx.x / WAVE;
  if (c >= ncols) return;
  double s = 0.0;
  for (int b = lane; b < nrb; b += WAVE) s += part[(int64_t)c * nrb + b];
  s = wave_sum(s);
  if (lane == 0) y[c] = s;
}

int64_t gemv_t_part_size(int64_t n, int ncols) {
  return ((n + GT_RB - 1) / GT_RB) * (int64_t)ncols;
}

template <typename T, typename TX>
cr_status gemv_tx(int64_t n, const Blocks<T>& A, const TX* x, double* y, double* part,
                  hipStream_t st) {
  const int nc = A.ncols();
  if (nc == 0) return CR_OK;
  const int nrb = (int)std::max<int64_t>(1, (n + GT_RB - 1) / GT_RB);
  if (n == 0) {
    CR_HIP(hipMemsetAsync(y, 0, sizeof(double) * nc, st));
    return CR_OK;
  }
  hipLaunchKernelGGL((k_gemv_t<T, TX>), dim3(nrb, (unsigned)((nc + 15) / 16)), dim3(NT), 0, st, n,
                     A, x, part, nrb);
  CR_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_part, dim3((nc + 3) / 4), dim3(NT), 0, st, nc, nrb, part, y);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

template <typename T>
cr_status gemv_t(int64_t n, const Blocks<T>& A, const T* x, double* y, double* part,
                 hipStream_t st) {
  return gemv_tx<T, T>(n, A, x, y, part, st);
}

// ============================================================== gemv_n
// y = beta*y + sum_c A[:,c] coef[c]; one thread per row, coefficients in LDS.
template <typename T>
__global__ __launch_bounds__(NT) void k_gemv_n(int64_t n, Blocks<T> A,
                                               const double* __restrict__ coef, double beta,
                                               T* __restrict__ y) {
  extern __shared__ double cs[];
  const int nc = A.ncols();
  for (int c = threadIdx.x; c < nc; c += NT) cs[c] = coef[c];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int b = 0; b < A.nb; ++b) {
    const T* p = A.p[b] + i;
    const int64_t ld = A.ld[b];
    const int cb = A.col0[b], ce = A.col0[b + 1];
    int c = cb;
    for (; c + 4 <= ce; c += 4) {
      double a0 = (double)p[(int64_t)(c - cb) * ld];
      double a1 = (double)p[(int64_t)(c - cb + 1) * ld];
      double a2 = (double)p[(int64_t)(c - cb + 2) * ld];
      double a3 = (double)p[(int64_t)(c - cb + 3) * ld];
      acc += a0 * cs[c] + a1 * cs[c + 1] + a2 * cs[c + 2] + a3 * cs[c + 3];
    }
    for (; c < ce; ++c) acc += (double)p[(int64_t)(c - cb) * ld] * cs[c];
  }
  y[i] = (T)(beta == 0.0 ? acc : beta * (double)y[i] + acc);
}

template <typename T>
cr_status gemv_n(int64_t n, const Blocks<T>& A, const double* coef, double beta, T* y,
                 hipStream_t st) {
  if (n == 0) return CR_OK;
  const int nc = A.ncols();
  hipLaunchKernelGGL((k_gemv_n<T>), dim3((unsigned)((n + NT - 1) / NT)), dim3(NT),
                     sizeof(double) * std::max(nc, 1), st, n, A, coef, beta, y);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// ============================================================== gemm_tn
// C = A^T B over n rows (split over gridDim.z), 64x64 output tiles, 256
// threads with 4x4 register tiles, K staged through LDS in chunks of 32 rows.
constexpr int TM = 64, KC = 32;

typedef double dbl4 __attribute__((ext_vector_type(4)));

// FP64 MFMA 16x16x4 on gfx950 (layouts checked on the device): lane l
// supplies A(row l%16, k l/16) and B(k l/16, col l%16); result element i of
// lane l is D(row l/16 + 4 i, col l%16).
__device__ __forceinline__ dbl4 mfma64(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T, bool MASK>
__global__ __launch_bounds__(NT) void k_gemm_tn(int64_t n, Blocks<T> A, Blocks<T> B,
                                                const uint32_t* __restrict__ bits,
                                                const T* __restrict__ w, int p, int q,
                                                int64_t kchunk, double* __restrict__ part,
                                                int ptiles, int ntiles, unsigned total) {
  __shared__ double As[KC][TM + 1];
  __shared__ double Bs[KC][TM + 1];
  // one-dimensional grid, remapped so that the output tiles of one row slab
  // are consecutive workgroups of one XCD (physical block b runs on XCD b % 8):
  // they run together and read the slab's rows of A and B from that XCD's L2
  const unsigned per = (total + NXCD - 1) / NXCD;
  const unsigned lin = (blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
  if (lin >= total) return;  // uniform per workgroup
  const int tile = (int)(lin % (unsigned)ntiles);
  const unsigned zb = lin / (unsigned)ntiles;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int tp = (tile % ptiles) * TM, tq = (tile / ptiles) * TM;
  const int64_t k0 = (int64_t)zb * kchunk;
  const int64_t k1 = std::min<int64_t>(n, k0 + kchunk);
  // wave wv computes the 32 x 32 sub-tile (rows 32*(wv%2), cols 32*(wv/2))
  const int wp = 32 * (wv & 1), wq = 32 * (wv >> 1);
  dbl4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
  // loader mapping: element e = tid + 256*m, row = e % KC, col = e / KC
  const int lrow = tid % KC;
  const int lcol = tid / KC;  // 0..7
  const T* acol[8];
  const T* bcol[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    int c = lcol + 8 * m;
    acol[m] = (tp + c < p) ? A.col(tp + c) : nullptr;
    bcol[m] = (!MASK && tq + c < q) ? B.col(tq + c) : nullptr;
  }
  const int fr = lane & 15, fk = lane >> 4;
  // register double buffer: the next chunk's loads are in flight while the
  // MFMAs consume the current chunk from LDS
  double ra[8], rb[8];
  auto load_chunk = [&](int64_t kb) {
    const int64_t row = kb + lrow;
    const bool rin = row < k1;
    double wv_ = 0.0;
    if (MASK && rin) wv_ = (double)w[row];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const int c = lcol + 8 * m;
      ra[m] = (rin && acol[m]) ? (double)acol[m][row] : 0.0;
      if (MASK) {
        const int al = tq + c;
        double v = 0.0;
        if (rin && al < q) {
          uint32_t word = bits[(int64_t)(al >> 5) * n + row];
          v = ((word >> (al & 31)) & 1u) ? wv_ : 0.0;
        }
        rb[m] = v;
      } else {
        rb[m] = (rin && bcol[m]) ? (double)bcol[m][row] : 0.0;
      }
    }
  };
  if (k0 < k1) load_chunk(k0);
  for (int64_t kb = k0; kb < k1; kb += KC) {
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      As[lrow][lcol + 8 * m] = ra[m];
      Bs[lrow][lcol + 8 * m] = rb[m];
    }
    __syncthreads();
    if (kb + KC < k1) load_chunk(kb + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[kk + fk][wp + 16 * a + fr];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kk + fk][wq + 16 * b + fr];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma64(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  double* out = part + (int64_t)zb * p * q;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = tp + wp + 16 * a + fk + 4 * e;
        const int j = tq + wq + 16 * b + fr;
        if (i < p && j < q) out[(int64_t)j * p + i] = acc[a][b][e];
      }
}

// C = A^T B for p, q <= 128 (e.g. H^T = X^T V): every workgroup computes the
// whole p x q product over its slab of rows, so A and B are each read once
// (a grid of 64 x 64 tiles would read every A tile once per B tile).  Rows are
// staged through LDS in chunks of 16 with the next chunk's loads in flight;
// wave wv owns output rows 32 wv .. 32 wv + 31 against all column tiles
// (16 FP64 MFMA accumulators).  Split-K partials go to `part` as in k_gemm_tn.
constexpr int GW_KC = 32, GW_LD = 144, GW_NT = 512;

template <typename T>
__global__ __launch_bounds__(GW_NT) void k_gemm_tn_wide(int64_t n, Blocks<T> A, Blocks<T> B, int p,
                                                        int q, int64_t kchunk,
                                                        double* __restrict__ part) {
  __shared__ double As[GW_KC][GW_LD];
  __shared__ double Bs[GW_KC][GW_LD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;  // 8 waves
  const int fr = lane & 15, fk = lane >> 4;
  const int64_t k0 = (int64_t)blockIdx.x * kchunk;
  const int64_t k1 = min(n, k0 + kchunk);
  // loader: element e = tid + 512 m (m < 16): row e % 32, column e / 32 of the
  // concatenation [A (128 columns) | B (128 columns)]; a column's 32 rows are
  // one 256-byte segment
  const int lrow = tid % GW_KC;
  const int lc0 = tid / GW_KC;  // 0..15
  const T* src[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    const int c = lc0 + 16 * m;  // 0..255
    src[m] = c < 128 ? (c < p ? A.col(c) : nullptr) : (c - 128 < q ? B.col(c - 128) : nullptr);
  }
  T rg[16];
  auto load = [&](int64_t kb) {
    const int64_t row = kb + lrow;
    const bool in = row < k1;
#pragma unroll
    for (int m = 0; m < 16; ++m) rg[m] = (in && src[m]) ? src[m][row] : (T)0;
  };
  dbl4 acc[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) acc[b] = dbl4{0.0, 0.0, 0.0, 0.0};
  const int ntq = (q + 15) / 16;
  const bool rows_live = 16 * wv < p;
  if (k0 < k1) load(k0);
  for (int64_t kb = k0; kb < k1; kb += GW_KC) {
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int c = lc0 + 16 * m;
      if (c < 128)
        As[lrow][c] = (double)rg[m];
      else
        Bs[lrow][c - 128] = (double)rg[m];
    }
    __syncthreads();
    if (kb + GW_KC < k1) load(kb + GW_KC);
    if (rows_live) {
#pragma unroll
      for (int kk = 0; kk < GW_KC; kk += 4) {
        const double av = As[kk + fk][16 * wv + fr];
#pragma unroll
        for (int b = 0; b < 8; ++b)
          if (b < ntq) acc[b] = mfma64(av, Bs[kk + fk][16 * b + fr], acc[b]);
      }
    }
    __syncthreads();
  }
  double* out = part + (int64_t)blockIdx.x * p * q;
#pragma unroll
  for (int b = 0; b < 8; ++b)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 16 * wv + fk + 4 * e;
      const int j = 16 * b + fr;
      if (i < p && j < q) out[(int64_t)j * p + i] = acc[b][e];
    }
}

// C = sum over the ks split partials; 64 outputs per workgroup, the four
// waves sum interleaved quarters of the splits, then combine in a fixed order.
__global__ __launch_bounds__(NT) void k_reduce_split(int p, int q, int ks,
                                                     const double* __restrict__ part,
                                                     double* __restrict__ C, int64_t ldc) {
  __shared__ double red[NT / WAVE][WAVE];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t pq = (int64_t)p * q;
  const int64_t e = (int64_t)blockIdx.x * WAVE + lane;
  double s0 = 0.0, s1 = 0.0;
  if (e < pq) {
    int z = wv;
    for (; z + 4 < ks; z += 8) {
      s0 += part[(int64_t)z * pq + e];
      s1 += part[(int64_t)(z + 4) * pq + e];
    }
    for (; z < ks; z += 4) s0 += part[(int64_t)z * pq + e];
  }
  red[wv][lane] = s0 + s1;
  __syncthreads();
  if (wv == 0 && e < pq) {
    const double s = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
    C[(e / p) * ldc + e % p] = s;
  }
}

template <typename T>
cr_status gemm_tn(int64_t n, const Blocks<T>& A, const Blocks<T>& B, const uint32_t* mask_bits,
                  const T* w, int q_mask, double* C, int64_t ldc, double* part,
                  int64_t part_cap, hipStream_t st, int* ks_out) {
  const int p = A.ncols();
  const int q = mask_bits ? q_mask : B.ncols();
  if (p == 0 || q == 0) return CR_OK;
  if (n == 0) {
    if (ks_out) {
      CR_HIP(hipMemsetAsync(part, 0, (size_t)p * q * sizeof(double), st));
      *ks_out = 1;
      return CR_OK;
    }
    CR_HIP(hipMemset2DAsync(C, ldc * sizeof(double), 0, p * sizeof(double), q, st));
    return CR_OK;
  }
  if (sizeof(T) == 4 && !mask_bits && p <= 128 && q <= 128) {
    // FP32 operands: one slab of at least 512 rows per workgroup, at most about
    // 512 slabs (measured faster than the 64 x 64 tiles below for FP32 data,
    // slower for FP64 data, whose tiled form keeps more loads in flight; in
    // the forked operator application its few workgroups also leave the CUs
    // to the concurrent stencil sweeps: 533 us against 581 us tiled)
    int64_t ks = std::max<int64_t>(1, std::min<int64_t>(512, n / 512));
    while (ks > 1 && ks * (int64_t)p * q > part_cap) --ks;
    if (ks * (int64_t)p * q > part_cap) {
      set_error("gemm_tn workspace too small");
      return CR_EINVAL;
    }
    int64_t kchunk = (n + ks - 1) / ks;
    kchunk = (kchunk + GW_KC - 1) / GW_KC * GW_KC;
    ks = std::max<int64_t>(1, (n + kchunk - 1) / kchunk);
    hipLaunchKernelGGL((k_gemm_tn_wide<T>), dim3((unsigned)ks), dim3(GW_NT), 0, st, n, A, B, p, q,
                       kchunk, part);
    CR_HIP(hipGetLastError());
    if (ks_out) {
      *ks_out = (int)ks;
      return CR_OK;
    }
    const int64_t pq = (int64_t)p * q;
    hipLaunchKernelGGL(k_reduce_split, dim3((unsigned)((pq + WAVE - 1) / WAVE)), dim3(NT), 0, st,
                       p, q, (int)ks, part, C, ldc);
    CR_HIP(hipGetLastError());
    return CR_OK;
  }
  const int tiles = ((p + TM - 1) / TM) * ((q + TM - 1) / TM);
  // about 512 workgroups, each at least 16 LDS chunks deep
  int64_t ks = std::max<int64_t>(1, 512 / tiles);
  ks = std::min<int64_t>(ks, std::max<int64_t>(1, (n + 16 * KC - 1) / (16 * KC)));
  while (ks > 1 && ks * (int64_t)p * q > part_cap) --ks;
  if (ks * (int64_t)p * q > part_cap) {
    set_error("gemm_tn workspace too small");
    return CR_EINVAL;
  }
  int64_t kchunk = (n + ks - 1) / ks;
  kchunk = (kchunk + KC - 1) / KC * KC;
  ks = std::max<int64_t>(1, (n + kchunk - 1) / kchunk);
  const int ptiles = (p + TM - 1) / TM;
  const int ntiles = ptiles * ((q + TM - 1) / TM);
  const unsigned total = (unsigned)(ntiles * ks);
  dim3 grid((total + NXCD - 1) / NXCD * NXCD);
  if (mask_bits)
    hipLaunchKernelGGL((k_gemm_tn<T, true>), grid, dim3(NT), 0, st, n, A, B, mask_bits, w, p, q,
                       kchunk, part, ptiles, ntiles, total);
  else
    hipLaunchKernelGGL((k_gemm_tn<T, false>), grid, dim3(NT), 0, st, n, A, B, mask_bits, w, p,
                       q, kchunk, part, ptiles, ntiles, total);
  CR_HIP(hipGetLastError());
  const int64_t pq = (int64_t)p * q;
  if (ks_out) {
    *ks_out = (int)ks;
    return CR_OK;
  }
  hipLaunchKernelGGL(k_reduce_split, dim3((unsigned)((pq + WAVE - 1) / WAVE)), dim3(NT), 0, st,
                     p, q, (int)ks, part, C, ldc);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// ============================================================== T = Z H from partials
// H = V^T X arrives as split-K partials part[z r n_inj + j + a r] (V^T X
// computed with V as the left operand, so a column of H is contiguous).
// Workgroup a (1024 threads = 8 groups of 128): group g sums partials z = g,
// g + 8, ... for 128 rows j at a time, coalesced, and the 8 group sums are
// added in a fixed order in LDS; then T[:, a] = Z h, with group g taking
// columns j = g, g + 8, ... of Z for 128 rows of T at a time (coalesced column
// reads of Z, which stays in L2 across workgroups), again summed over the
// groups in a fixed order.  Replaces a reduce, a copy of Z and a small GEMM:
// three latency-bound launches in front of the masked product.
constexpr int ZH_NT = 1024, ZH_G = ZH_NT / 128;

template <typename T>
__global__ __launch_bounds__(ZH_NT) void k_zh_part(int p, int r, int ks,
                                                   const double* __restrict__ part,
                                                   const T* __restrict__ Z, int64_t ldz,
                                                   double* __restrict__ Tm, int64_t ldt) {
  extern __shared__ double hs[];  // r doubles of h
  __shared__ double red[ZH_G][128];
  const int a = blockIdx.x;
  const int t = threadIdx.x;
  const int li = t & 127, g = t >> 7;
  const int64_t pq = (int64_t)p * r;
  for (int j0 = 0; j0 < r; j0 += 128) {
    const int j = j0 + li;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (j < r) {
      const double* pj = part + (int64_t)a * r + j;
      int z = g;
      for (; z + 3 * ZH_G < ks; z += 4 * ZH_G) {
        s0 += pj[(int64_t)z * pq];
        s1 += pj[(int64_t)(z + ZH_G) * pq];
        s2 += pj[(int64_t)(z + 2 * ZH_G) * pq];
        s3 += pj[(int64_t)(z + 3 * ZH_G) * pq];
      }
      for (; z < ks; z += ZH_G) s0 += pj[(int64_t)z * pq];
    }
    red[g][li] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (g == 0 && j < r) {
      double h = 0.0;
#pragma unroll
      for (int q = 0; q < ZH_G; ++q) h += red[q][li];
      hs[j] = h;
    }
    __syncthreads();
  }
  for (int k0 = 0; k0 < r; k0 += 128) {
    const int k = k0 + li;
    double s0 = 0.0, s1 = 0.0;
    if (k < r) {
      int j = g;
      for (; j + ZH_G < r; j += 2 * ZH_G) {
        s0 += (double)Z[k + (int64_t)j * ldz] * hs[j];
        s1 += (double)Z[k + (int64_t)(j + ZH_G) * ldz] * hs[j + ZH_G];
      }
      for (; j < r; j += ZH_G) s0 += (double)Z[k + (int64_t)j * ldz] * hs[j];
    }
    red[g][li] = s0 + s1;
    __syncthreads();
    if (g == 0 && k < r) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < ZH_G; ++q) v += red[q][li];
      Tm[k + (int64_t)a * ldt] = v;
    }
    __syncthreads();
  }
}

template <typename T>
cr_status zh_from_partials(int p, int r, int ks, const double* part, const T* Z, int64_t ldz,
                           double* Tm, int64_t ldt, hipStream_t st) {
  if (p <= 0 || r <= 0) return CR_OK;
  if (r > ZH_RMAX || ks < 1) {
    set_error("zh_from_partials: rank out of range");
    return CR_EINVAL;
  }
  hipLaunchKernelGGL((k_zh_part<T>), dim3((unsigned)p), dim3(ZH_NT), r * sizeof(double), st, p, r,
                     ks, part, Z, ldz, Tm, ldt);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// ============================================================== masked tall GEMM
// N[i,a] = OY[i,a] - omega_ia (U T)[i,a]   (or + omega (U T) when OY is null)
// computed transposed on the matrix cores, N^T = T^T U^T, with injections as
// MFMA rows and voxels as MFMA columns: each group of 16 lanes then holds 16
// consecutive voxels of one injection, so the mask, OY reads and N writes are
// coalesced.  Workgroup: 128 voxels x up to 128 injections (every injection
// tile in one pass, so U is read once); wave wv owns voxels 32 wv .. 32 wv + 31
// (two 16-wide column tiles) and all injection tiles.  T^T is staged through
// LDS in chunks of 32 k; the U fragments of the next chunk are in flight while
// the current chunk's MFMAs run.  FP64 operands use v_mfma_f64_16x16x4f64,
// FP32 operands v_mfma_f32_16x16x4f32 (FP32 accumulation).  Voxel blocks are
// remapped per XCD.
typedef float flt4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma16;
template <>
struct Mfma16<double> {
  typedef dbl4 acc_t;
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // result element e of a lane in lane group fk (= lane / 16) sits in row:
  __device__ static int row(int fk, int e) { return fk + 4 * e; }
};
template <>
struct Mfma16<float> {
  typedef flt4v acc_t;
  __device__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int fk, int e) { return 4 * fk + e; }
};

constexpr int MG_ROWS = 64, MG_COLS = 128, MG_KC = 32, MG_LD = 144;

// NTA = injection tiles of 16 per workgroup (1, 2, 4 or 8): the smallest that
// covers min(n_inj, 128), so that no MFMA sits behind a run-time condition.
template <typename T, int NTA>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_masked_tall_gemm(
    int64_t n, int r, int ninj, const T* __restrict__ U, int64_t ldu, const double* __restrict__ Tm,
    int64_t ldt, const uint32_t* __restrict__ bits, const T* __restrict__ OY, int64_t ldoy,
    T* __restrict__ N, int64_t ldn, unsigned nb_log) {
  typedef typename Mfma16<T>::acc_t acc_t;
  constexpr int NC = 16 * NTA;    // injection columns staged per chunk
  __shared__ T Ts[MG_KC][MG_LD];  // Ts[k][a] = T[k0 + k, a0 + a]; row stride 16 mod 64 banks
  const int64_t lb = xcd_block(blockIdx.x, nb_log);
  if (lb >= nb_log) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int fr = lane & 15, fk = lane >> 4;
  const int a0 = blockIdx.y * MG_COLS;
  const int na = min(NC, ninj - a0);
  const int64_t v0 = lb * MG_ROWS + 16 * wv;  // the 16 voxels of this wave
  acc_t acc[NTA];
#pragma unroll
  for (int ta = 0; ta < NTA; ++ta) acc[ta] = acc_t{0, 0, 0, 0};
  const int64_t vrow = v0 + fr;
  const bool ok = vrow < n;
  const int64_t vcl = ok ? vrow : n - 1;  // clamped, so every load below is in bounds
  T b0[MG_KC / 4], n0[MG_KC / 4];
  auto loadB = [&](int k0, T* x0) {
#pragma unroll
    for (int s4 = 0; s4 < MG_KC / 4; ++s4) {
      const int k = k0 + 4 * s4 + fk;
      const T v = U[(int64_t)min(k, r - 1) * ldu + vcl];
      x0[s4] = (k < r && ok) ? v : (T)0;
    }
  };
  if (r > 0) loadB(0, b0);
  for (int k0 = 0; k0 < r; k0 += MG_KC) {
    __syncthreads();
    for (int e = threadIdx.x; e < MG_KC * NC; e += NT) {
      const int kk = e % MG_KC, cc = e / MG_KC;
      const int k = k0 + kk, al = a0 + cc;
      Ts[kk][cc] = (k < r && al < ninj) ? (T)Tm[(int64_t)al * ldt + k] : (T)0;
    }
    __syncthreads();
    const bool more = k0 + MG_KC < r;
    if (more) loadB(k0 + MG_KC, n0);
#pragma unroll
    for (int s4 = 0; s4 < MG_KC / 4; ++s4) {
#pragma unroll
      for (int ta = 0; ta < NTA; ++ta)
        acc[ta] = Mfma16<T>::mma(Ts[4 * s4 + fk][16 * ta + fr], b0[s4], acc[ta]);
    }
    if (more) {
#pragma unroll
      for (int s4 = 0; s4 < MG_KC / 4; ++s4) b0[s4] = n0[s4];
    }
  }
  // epilogue: element e of lane l is (injection 16 ta + row(fk, e), voxel fr)
  if (!ok) return;
  uint32_t wd[(NC + 31) / 32];
#pragma unroll
  for (int q = 0; q < (NC + 31) / 32; ++q)
    wd[q] = (32 * q < na) ? bits[(int64_t)((a0 >> 5) + q) * n + vrow] : 0u;
#pragma unroll
  for (int ta = 0; ta < NTA; ++ta) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int al_loc = 16 * ta + Mfma16<T>::row(fk, e);
      if (al_loc < na) {
        const int64_t al = a0 + al_loc;
        // 16 ta <= al_loc < 16 ta + 16, so the mask word is wd[ta / 2]
        const T om = (T)((wd[ta >> 1] >> (al_loc & 31)) & 1u);
        const T v = om * acc[ta][e];
        N[al * ldn + vrow] = OY ? OY[al * ldoy + vrow] - v : v;
      }
    }
  }
}

// Register-resident variant for r <= 112: wave w of a workgroup owns
// injection tiles 2w, 2w + 1 (32 injections) and keeps their T^T fragments for
// every k in registers, loaded once; the workgroup then walks 16-voxel tiles
// (grid-stride), each wave streaming the tile's U fragments (the next tile's
// are in flight while the current tile's MFMAs run).  No LDS: T is read once
// per workgroup instead of once per voxel tile, and the MFMA chain of a tile
// is 2 KS back-to-back instructions.  KS = k steps of 4 (r <= 4 KS; exact
// for KS > 16); the mask word of a wave's 32 injections is a single bits
// word.  The register budget decides the overlap of MFMAs with memory: at
// r = 100 the FP64 variant holds 224 VGPRs, two waves per SIMD.  SYNC adds a
// workgroup barrier per tile (the four waves then read each U tile together).
// HAS_OY selects N = OY - Omega o (U T) over N = Omega o (U T).
template <typename T, int KS, bool HAS_OY, bool SYNC>
__global__ __launch_bounds__(NT) void k_masked_gemm_rt(
    int64_t n, int r, int ninj, const T* __restrict__ U, int64_t ldu, const double* __restrict__ Tm,
    int64_t ldt, const uint32_t* __restrict__ bits, const T* __restrict__ OY, int64_t ldoy,
    T* __restrict__ N, int64_t ldn) {
  typedef typename Mfma16<T>::acc_t acc_t;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int fr = lane & 15, fk = lane >> 4;
  const int a0 = blockIdx.y * MG_COLS + 32 * wv;  // first injection of this wave
  const int64_t ntile = (n + 15) / 16;
  const int64_t stride = gridDim.x;
  int64_t tile = blockIdx.x;
  if (tile >= ntile) return;  // uniform per workgroup
  if (a0 >= ninj) {
    // whole wave idle: with SYNC it still takes the per-tile barrier
    if (SYNC)
      for (; tile < ntile; tile += stride) __syncthreads();
    return;
  }
  T a[2][KS];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int al = a0 + 16 * t + fr;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + fk;
      a[t][ks] = (k < r && al < ninj) ? (T)Tm[(int64_t)al * ldt + k] : (T)0;
    }
  }
  const bool full = a0 + 32 <= ninj;
  // FP64 at large KS: no second fragment buffer (register budget of two waves
  // per SIMD); the other wave on the SIMD covers the load latency instead
  constexpr bool PF = sizeof(T) == 4 || KS <= 16;
  T b[KS], bn[PF ? KS : 1];
  // the k part of an address is uniform (scalar); the lane part is one 32-bit
  // offset fk ldu + voxel (the host checks that it fits).  Columns k >= r are
  // clamped to r - 1: their T^T fragments are zero, so any finite value works.
  // Full k steps address as a uniform column base (scalar registers) plus one
  // 32-bit lane byte offset (the host checks that it fits), so the loads use
  // the scalar-base form and no per-step 64-bit lane addresses are kept.
  auto loadB = [&](int64_t tl, T* x) {
    const int64_t v = tl * 16 + fr;
    const int32_t vc = (int32_t)(v < n ? v : n - 1);
    const int32_t off = fk * (int32_t)ldu + vc;
    const uint32_t offb = (uint32_t)off * (uint32_t)sizeof(T);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      // KS > 16 is launched only with KS = ceil(r / 4): every step but the
      // last is then full, known at compile time (no clamped alternative
      // address is formed for them)
      if ((KS > 16 && ks < KS - 1) || 4 * ks + 3 < r) {
        const char* base = reinterpret_cast<const char*>(U + (int64_t)(4 * ks) * ldu);
        x[ks] = *reinterpret_cast<const T*>(base + offb);
      } else {
        const int k = min(4 * ks + fk, r - 1);
        x[ks] = U[(int64_t)k * ldu + vc];
      }
    }
  };
  const uint32_t* wbits = bits + (int64_t)(a0 >> 5) * n;
  // mask word of a tile's voxel (clamped: always in bounds)
  auto loadW = [&](int64_t tl) {
    const int64_t v = tl * 16 + fr;
    return wbits[v < n ? v : n - 1];
  };
  loadB(tile, b);
  uint32_t wd = loadW(tile), wdn = 0u;
  for (; tile < ntile; tile += stride) {
    // SYNC: the workgroup's waves (one per SIMD) read the same U tile; a
    // barrier per tile keeps them together, so the lines one wave brings
    // into L2 are still there for the others
    if (SYNC) __syncthreads();
    const bool more = tile + stride < ntile;
    if (more) wdn = loadW(tile + stride);
    if (PF && more) loadB(tile + stride, bn);
    acc_t acc0 = acc_t{0, 0, 0, 0}, acc1 = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      acc0 = Mfma16<T>::mma(a[0][ks], b[ks], acc0);
      acc1 = Mfma16<T>::mma(a[1][ks], b[ks], acc1);
    }
    // without a second buffer, the next tile's fragments are requested as
    // soon as the MFMAs have been issued, so they load during the stores
    if (!PF && more) loadB(tile + stride, b);
    const int64_t v = tile * 16 + fr;
    if (v < n) {
      if (full) {
        // all 32 injections of the wave exist: unconditional stores
#pragma unroll
        for (int t = 0; t < 2; ++t) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int al_loc = 16 * t + Mfma16<T>::row(fk, e);
            const int64_t al = a0 + al_loc;
            const T om = (T)((wd >> al_loc) & 1u);
            const T val = om * (t ? acc1[e] : acc0[e]);
            if (HAS_OY)
              N[al * ldn + v] = OY[al * ldoy + v] - val;
            else
              N[al * ldn + v] = val;
          }
        }
      } else {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int al_loc = 16 * t + Mfma16<T>::row(fk, e);  // < 32
            const int64_t al = a0 + al_loc;
            if (al < ninj) {
              const T om = (T)((wd >> al_loc) & 1u);
              const T val = om * (t ? acc1[e] : acc0[e]);
              N[al * ldn + v] = HAS_OY ? OY[al * ldoy + v] - val : val;
            }
          }
        }
      }
    }
    if (more) {
      wd = wdn;
      if (PF) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) b[ks] = bn[ks];
      }
    }
  }
}

template <typename T>
cr_status masked_tall_gemm(int64_t n, int r, int ninj, const T* U, int64_t ldu, const double* Tm,
                           int64_t ldt, const uint32_t* bits, const T* OY, int64_t ldoy, T* N,
                           int64_t ldn, hipStream_t st) {
  if (n == 0 || ninj == 0) return CR_OK;
  if (r >= 1 && r <= 112 && (4 * ldu + n) * (int64_t)sizeof(T) <= (int64_t)UINT32_MAX) {
    // one wave per 32 injections of a 128-injection block; as many workgroups
    // as fit on the device at once (two per CU for FP64 at r = 100)
    const int na = std::min(ninj, MG_COLS);
    const int waves = (na + 31) / 32;
    const int64_t ntile = (n + 15) / 16;
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    // the grid-stride loop wants exactly one round of resident workgroups:
    // a partial second round runs at a fraction of the occupancy
    const int ks = (r + 3) / 4;
    // a barrier per tile keeps a workgroup's waves on the same U tile: for
    // FP32 data 114 against 140 us alone and 499 against 524 us for the forked
    // operator call; FP64 fetches less U with it (318 against 441 MB) but runs
    // slower (218 against 211 us alone, 786 against 770 us forked)
    constexpr bool mg_sync = sizeof(T) == 4;
#define RT_CASE(K)                                                                             \
  if (ks <= K) {                                                                               \
    int per_cu = 0;                                                                            \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(                                          \
            &per_cu, k_masked_gemm_rt<T, K, false, false>, 64 * waves, 0) != hipSuccess ||     \
        per_cu < 1)                                                                            \
      per_cu = 1;                                                                              \
    const int gy = (ninj + MG_COLS - 1) / MG_COLS;                                             \
    const int64_t want = (int64_t)ncu * per_cu / gy;                                           \
    dim3 grid((unsigned)std::max<int64_t>(1, std::min(ntile, want)), gy);                      \
    if constexpr (mg_sync) {                                                                   \
      if (OY)                                                                                  \
        hipLaunchKernelGGL((k_masked_gemm_rt<T, K, true, true>), grid, dim3(64 * waves), 0,    \
                           st, n, r, ninj, U, ldu, Tm, ldt, bits, OY, ldoy, N, ldn);           \
      else                                                                                     \
        hipLaunchKernelGGL((k_masked_gemm_rt<T, K, false, true>), grid, dim3(64 * waves), 0,   \
                           st, n, r, ninj, U, ldu, Tm, ldt, bits, OY, ldoy, N, ldn);           \
    } else {                                                                                   \
      if (OY)                                                                                  \
        hipLaunchKernelGGL((k_masked_gemm_rt<T, K, true, false>), grid, dim3(64 * waves), 0,   \
                           st, n, r, ninj, U, ldu, Tm, ldt, bits, OY, ldoy, N, ldn);           \
      else                                                                                     \
        hipLaunchKernelGGL((k_masked_gemm_rt<T, K, false, false>), grid, dim3(64 * waves), 0,  \
                           st, n, r, ninj, U, ldu, Tm, ldt, bits, OY, ldoy, N, ldn);           \
    }                                                                                          \
    CR_HIP(hipGetLastError());                                                                 \
    return CR_OK;                                                                              \
  }
    // k steps in fours up to 16, then exact: at r > 64 the FP64 MFMA work is
    // the kernel's floor, and a padded step costs a full MFMA pair per tile
    RT_CASE(4) RT_CASE(8) RT_CASE(12) RT_CASE(16) RT_CASE(17) RT_CASE(18) RT_CASE(19)
    RT_CASE(20) RT_CASE(21) RT_CASE(22) RT_CASE(23) RT_CASE(24) RT_CASE(25) RT_CASE(26)
    RT_CASE(27) RT_CASE(28)
#undef RT_CASE
  }
  const unsigned nb_log = (unsigned)((n + MG_ROWS - 1) / MG_ROWS);
  const unsigned nb_phys = (nb_log + NXCD - 1) / NXCD * NXCD;
  dim3 grid(nb_phys, (ninj + MG_COLS - 1) / MG_COLS);
  const int na = std::min(ninj, MG_COLS);
  const int nta = na <= 16 ? 1 : na <= 32 ? 2 : na <= 64 ? 4 : 8;
#define MG_CASE(K)                                                                               \
  case K:                                                                                        \
    hipLaunchKernelGGL((k_masked_tall_gemm<T, K>), grid, dim3(NT), 0, st, n, r, ninj, U, ldu, Tm, \
                       ldt, bits, OY, ldoy, N, ldn, nb_log);                                     \
    break;
  switch (nta) {
    MG_CASE(1) MG_CASE(2) MG_CASE(4) MG_CASE(8)
  }
#undef MG_CASE
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// ============================================================== fused operator sweep
// One pass over a tile of W2_TILE consecutive voxels that writes L w and
// L^2 w for every column of w and, with DATA, N = Omega o (w T) (the masked
// data term of eq. multitermSylv) from the same staged values.  Columns go in
// groups of four: the tile's ring-2 window of the group (the voxels its rows
// of L^2 read) is staged into LDS with coalesced loads, double-buffered so
// that the next group's loads are in flight while the current group is
// computed.  Stencil role: thread (wave c, lane v) forms rows v of L and L^2
// for column c of the group from 25 packed entries held in registers.
// Product role: wave q owns injections 32q .. 32q + 31 and accumulates
// (w T)^T over the groups on FP64 (or FP32) MFMA tiles, reading the w
// fragments from the same LDS window (the tile's own voxels); the masked
// result is stored once at the end.  L w is never written and re-read, and
// the product reads no w of its own; but the windows of neighbouring tiles
// overlap, and what of them has left L2 is fetched again (on the cortex
// shells the target pass fetched 4.2 times w and ran slower than the two
// stencil passes and the product it replaces, so the form is opt-in).
constexpr int W2_EPT = W2_MAX / NT;  // window elements staged per thread

template <typename T, bool DATA>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_op_win2(
    int64_t n, unsigned nt_log, const int32_t* __restrict__ itab,
    const uint32_t* __restrict__ ent, int r, const T* __restrict__ w, int64_t ldw,
    T* __restrict__ out1, T* __restrict__ out2, int64_t ldo, int ninj,
    const double* __restrict__ Tm, int64_t ldt, const uint32_t* __restrict__ bits,
    T* __restrict__ N, int64_t ldn) {
  typedef typename Mfma16<T>::acc_t acc_t;
  __shared__ T buf[2][4][W2_MAX];
  const int64_t tile = xcd_block(blockIdx.x, nt_log);
  if (tile >= nt_log) return;  // uniform per workgroup
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int fr = lane & 15, fk = lane >> 4;
  const int32_t* it = itab + tile * W2_TAB;
  const int nint = it[0], tot = it[1];
  // staging map: window element e = tid + NT m comes from voxel src[m]
  int src[W2_EPT];
#pragma unroll
  for (int m = 0; m < W2_EPT; ++m) {
    const int e = tid + NT * m;
    int sv = -1;
    if (e < tot) {
      int q = 0;
      for (int k = 1; k < nint; ++k)
        if (it[2 + W2_NI + k] <= e) q = k;
      sv = it[2 + q] + (e - it[2 + W2_NI + q]);
    }
    src[m] = sv;
  }
  const int64_t v0 = tile * W2_TILE;
  const int64_t i = v0 + lane;  // stencil row of this thread
  const bool valid = i < n;
  uint32_t en[W2_NE];
#pragma unroll
  for (int e = 0; e < W2_NE; ++e) en[e] = valid ? ent[(int64_t)e * n + i] : 0u;
  const int ngr = (r + 3) / 4;
  T rg[4][W2_EPT];
  auto load = [&](int g) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = 4 * g + q;
      const T* wc = w + (int64_t)min(c, r - 1) * ldw;
#pragma unroll
      for (int m = 0; m < W2_EPT; ++m) rg[q][m] = (src[m] >= 0 && c < r) ? wc[src[m]] : (T)0;
    }
  };
  auto stage = [&](int b) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int m = 0; m < W2_EPT; ++m)
        if (tid + NT * m < tot) buf[b][q][tid + NT * m] = rg[q][m];
  };
  // product role: window positions of the tile's voxels 16 vb + fr, the
  // wave's first injection, and its accumulators (injection x voxel tiles)
  const int a0 = 32 * wv;
  const bool prod = DATA && a0 < ninj;  // uniform per wave
  int cpos[4];
  acc_t acc[4][2];
#pragma unroll
  for (int vb = 0; vb < 4; ++vb) {
    const int64_t v = v0 + 16 * vb + fr;
    cpos[vb] = (prod && v < n) ? (int)(ent[v] & 0xffffu) : 0;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) acc[vb][cb] = acc_t{0, 0, 0, 0};
  }
  // T^T fragments of a group (rows: the wave's injections; k: the group's
  // columns), fetched one group ahead like the window
  T ta[2], tn[2];
  auto loadT = [&](int g, T* x) {
    const int k = 4 * g + fk;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int al = a0 + 16 * cb + fr;
      x[cb] = (k < r && al < ninj) ? (T)Tm[(int64_t)al * ldt + k] : (T)0;
    }
  };
  if (prod) loadT(0, tn);
  load(0);
  stage(0);
  __syncthreads();
  for (int g = 0; g < ngr; ++g) {
    const int b = g & 1;
    if (prod) {
      ta[0] = tn[0];
      ta[1] = tn[1];
      if (g + 1 < ngr) loadT(g + 1, tn);
    }
    if (g + 1 < ngr) load(g + 1);
    const int c = 4 * g + wv;
    if (valid && c < r) {
      const T* B = buf[b][wv];
      T s1 = (T)0, s2 = (T)0;
#pragma unroll
      for (int e = 0; e < W2_NL; ++e) {
        const T x = B[en[e] & 0xffffu];
        s1 += (T)((int32_t)en[e] >> 24) * x;
        s2 += (T)((int32_t)(en[e] << 8) >> 24) * x;
      }
#pragma unroll
      for (int e = W2_NL; e < W2_NE; ++e)
        s2 += (T)((int32_t)(en[e] << 8) >> 24) * B[en[e] & 0xffffu];
      out1[(int64_t)c * ldo + i] = s1;
      out2[(int64_t)c * ldo + i] = s2;
    }
    if (prod) {
      const T* B = buf[b][fk];
#pragma unroll
      for (int vb = 0; vb < 4; ++vb) {
        const T x = B[cpos[vb]];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[vb][cb] = Mfma16<T>::mma(ta[cb], x, acc[vb][cb]);
      }
    }
    if (g + 1 < ngr) stage(b ^ 1);
    __syncthreads();
  }
  if (prod) {
    const uint32_t* wb = bits + (int64_t)(a0 >> 5) * n;
#pragma unroll
    for (int vb = 0; vb < 4; ++vb) {
      const int64_t v = v0 + 16 * vb + fr;
      if (v < n) {
        const uint32_t wd = wb[v];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int al_loc = 16 * cb + Mfma16<T>::row(fk, e);  // < 32
            const int al = a0 + al_loc;
            if (al < ninj) N[(int64_t)al * ldn + v] = (T)((wd >> al_loc) & 1u) * acc[vb][cb][e];
          }
        }
      }
    }
  }
}

template <typename T>
bool op_win2_ok(const Geom& g, int r, int ninj) {
  return g.w2tab && g.w2ent && r >= 1 && ninj <= 4 * 32 && g.n <= INT32_MAX;
}

template <typename T>
cr_status op_win2(const Geom& g, int r, const T* w, int64_t ldw, T* out1, T* out2, int64_t ldo,
                  int ninj, const double* Tm, int64_t ldt, const uint32_t* bits, T* N,
                  int64_t ldn, hipStream_t st) {
  if (g.n == 0 || r <= 0) return CR_OK;
  if (!op_win2_ok<T>(g, r, N ? ninj : 0)) {
    set_error("fused operator sweep: no ring-2 tables for this geometry or sizes out of range");
    return CR_EINVAL;
  }
  const unsigned nt_log = (unsigned)((g.n + W2_TILE - 1) / W2_TILE);
  const unsigned nb_phys = (nt_log + NXCD - 1) / NXCD * NXCD;
  if (N)
    hipLaunchKernelGGL((k_op_win2<T, true>), dim3(nb_phys), dim3(NT), 0, st, g.n, nt_log,
                       g.w2tab, g.w2ent, r, w, ldw, out1, out2, ldo, ninj, Tm, ldt, bits, N,
                       ldn);
  else
    hipLaunchKernelGGL((k_op_win2<T, false>), dim3(nb_phys), dim3(NT), 0, st, g.n, nt_log,
                       g.w2tab, g.w2ent, r, w, ldw, out1, out2, ldo, 0, (const double*)nullptr,
                       0, (const uint32_t*)nullptr, (T*)nullptr, 0);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// ============================================================== masked reductions
// d_i = sum_a omega_ia h_a^2 = sum_a h_a^2 - sum_{a: omega_ia = 0} h_a^2
__global__ __launch_bounds__(NT) void k_hsq(int ninj, const double* __restrict__ h,
                                            double* __restrict__ out) {
  __shared__ double red[NT / WAVE];
  double s = 0.0;
  for (int a = threadIdx.x; a < ninj; a += NT) s += h[a] * h[a];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = red[0] + red[1] + red[2] + red[3];
}

template <typename T>
__global__ __launch_bounds__(NT) void k_masked_quad(int64_t n, int ninj,
                                                    const uint32_t* __restrict__ bits,
                                                    const double* __restrict__ h,
                                                    const double* __restrict__ hsq_total,
                                                    T* __restrict__ d) {
  extern __shared__ double h2[];
  for (int a = threadIdx.x; a < ninj; a += NT) h2[a] = h[a] * h[a];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  double s = hsq_total[0];
  const int nw = (ninj + 31) / 32;
  for (int wdx = 0; wdx < nw; ++wdx) {
    uint32_t zero = ~bits[(int64_t)wdx * n + i];
    const int valid = ninj - 32 * wdx;
    if (valid < 32) zero &= (1u << valid) - 1u;
    while (zero) {
      const int b = __ffs(zero) - 1;
      s -= h2[32 * wdx + b];
      zero &= zero - 1u;
    }
  }
  d[i] = (T)s;
}

template <typename T>
cr_status masked_quad_ws(int64_t n, int ninj, const uint32_t* bits, const double* h, T* d,
                         double* tmp, hipStream_t st) {
  if (n == 0) return CR_OK;
  hipLaunchKernelGGL(k_hsq, dim3(1), dim3(NT), 0, st, ninj, h, tmp);
  CR_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_masked_quad<T>), dim3((unsigned)((n + NT - 1) / NT)), dim3(NT),
                     sizeof(double) * std::max(ninj, 1), st, n, ninj, bits, h, tmp, d);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// g_a = sum_i omega_ia w_i^2: structure of k_gemv_t with the mask as matrix.
template <typename T>
__global__ __launch_bounds__(NT) void k_masked_colsq(int64_t n, int ninj,
                                                     const uint32_t* __restrict__ bits,
                                                     const T* __restrict__ w,
                                                     double* __restrict__ part, int nrb) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int wv = threadIdx.x / WAVE;
  const int64_t r0 = (int64_t)blockIdx.x * GT_RB + lane;
  double xv[GT_RPL];
#pragma unroll
  for (int m = 0; m < GT_RPL; ++m) {
    int64_t row = r0 + 64 * m;
    double t = row < n ? (double)w[row] : 0.0;
    xv[m] = t * t;
  }
  const int nw = (ninj + 31) / 32;
  for (int wdx = 0; wdx < nw; ++wdx) {
    uint32_t word[GT_RPL];
#pragma unroll
    for (int m = 0; m < GT_RPL; ++m) {
      int64_t row = r0 + 64 * m;
      word[m] = row < n ? bits[(int64_t)wdx * n + row] : 0u;
    }
    for (int b = wv; b < 32 && 32 * wdx + b < ninj; b += 4) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < GT_RPL; ++m) acc += ((word[m] >> b) & 1u) ? xv[m] : 0.0;
      acc = wave_sum(acc);
      if (lane == 0) part[(int64_t)(32 * wdx + b) * nrb + blockIdx.x] = acc;
    }
  }
}

template <typename T>
cr_status masked_colsq(int64_t n, int ninj, const uint32_t* bits, const T* w, double* g,
                       double* part, hipStream_t st) {
  if (ninj == 0) return CR_OK;
  const int nrb = (int)std::max<int64_t>(1, (n + GT_RB - 1) / GT_RB);
  if (n == 0) {
    CR_HIP(hipMemsetAsync(g, 0, sizeof(double) * ninj, st));
    return CR_OK;
  }
  hipLaunchKernelGGL((k_masked_colsq<T>), dim3(nrb), dim3(NT), 0, st, n, ninj, bits, w, part,
                     nrb);
  CR_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_part, dim3((ninj + 3) / 4), dim3(NT), 0, st, ninj, nrb, part, g);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// ============================================================== elementwise / small
template <typename Td, typename Ts>
__global__ __launch_bounds__(NT) void k_convert2d(int64_t rows, int64_t cols,
                                                  const Ts* __restrict__ src, int64_t lds,
                                                  Td* __restrict__ dst, int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= rows) return;
  for (int64_t c = blockIdx.y; c < cols; c += gridDim.y) dst[c * ldd + i] = (Td)src[c * lds + i];
}

template <typename Td, typename Ts>
cr_status convert2d(int64_t rows, int64_t cols, const Ts* src, int64_t lds, Td* dst, int64_t ldd,
                    hipStream_t st) {
  if (rows == 0 || cols == 0) return CR_OK;
  dim3 grid((unsigned)((rows + NT - 1) / NT), (unsigned)std::min<int64_t>(cols, 64));
  hipLaunchKernelGGL((k_convert2d<Td, Ts>), grid, dim3(NT), 0, st, rows, cols, src, lds, dst, ldd);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

template <typename Td, typename Ts>
cr_status convert(int64_t n, const Ts* src, Td* dst, hipStream_t st) {
  return convert2d<Td, Ts>(n, 1, src, n, dst, n, st);
}

// out[i] = alpha * sum_k op(M)[i,k] v[k]; one workgroup (small sizes only)
__global__ __launch_bounds__(NT) void k_small_gemv(int m, int kk, const double* __restrict__ M,
                                                   int64_t ldm, int trans,
                                                   const double* __restrict__ v, double alpha,
                                                   double* __restrict__ out) {
  for (int i = threadIdx.x + blockIdx.x * NT; i < m; i += NT * gridDim.x) {
    double s = 0.0;
    if (trans)
      for (int k = 0; k < kk; ++k) s += M[(int64_t)i * ldm + k] * v[k];
    else
      for (int k = 0; k < kk; ++k) s += M[(int64_t)k * ldm + i] * v[k];
    out[i] = alpha * s;
  }
}

cr_status small_gemv(int m, int kk, const double* M, int64_t ldm, bool trans, const double* v,
                     double alpha, double* out, hipStream_t st) {
  if (m <= 0) return CR_OK;
  hipLaunchKernelGGL(k_small_gemv, dim3((m + NT - 1) / NT), dim3(NT), 0, st, m, kk, M, ldm,
                     trans ? 1 : 0, v, alpha, out);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// C = alpha op(A) op(B) on FP64 MFMA: a workgroup per 64 x 64 tile of C,
// wave w the 32 x 32 quadrant (w % 2, w / 2) as 2 x 2 blocks of 16 x 16 x 4;
// fragments straight from memory (the operands are small enough for L2),
// four k-steps of loads in flight ahead of their MFMAs.  A(i, t) =
// A[i sa_i + t sa_t], B(t, j) = B[t sb_t + j sb_j].
__global__ __launch_bounds__(NT) void k_small_gemm(int m, int n, int k, const double* __restrict__ A,
                                                   int64_t sa_i, int64_t sa_t,
                                                   const double* __restrict__ B, int64_t sb_t,
                                                   int64_t sb_j, double alpha,
                                                   double* __restrict__ C, int64_t ldc) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int fr = lane & 15, fk = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * 64 + 32 * (wv & 1);
  const int64_t c0 = (int64_t)blockIdx.y * 64 + 32 * (wv >> 1);
  int64_t ia[2], jb[2];
  bool aok[2], bok[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    ia[t] = r0 + 16 * t + fr;
    jb[t] = c0 + 16 * t + fr;
    aok[t] = ia[t] < m;
    bok[t] = jb[t] < n;
  }
  dbl4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
  constexpr int UNR = 4;
  for (int kk = 0; kk < k; kk += 4 * UNR) {
    double av[UNR][2], bv[UNR][2];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int64_t t = kk + 4 * u + fk;
      const bool tok = t < k;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        av[u][q] = (tok && aok[q]) ? A[ia[q] * sa_i + t * sa_t] : 0.0;
        bv[u][q] = (tok && bok[q]) ? B[t * sb_t + jb[q] * sb_j] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma64(av[u][a], bv[u][b], acc[a][b]);
  }
  // element e of lane l in block (a, b): row r0 + 16 a + fk + 4 e, column c0 + 16 b + fr
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = r0 + 16 * a + fk + 4 * e, col = c0 + 16 * b + fr;
        if (row < m && col < n) C[col * ldc + row] = alpha * acc[a][b][e];
      }
}

cr_status small_gemm(int m, int n, int k, const double* A, int64_t lda, bool ta, const double* B,
                     int64_t ldb, bool tb, double alpha, double* C, int64_t ldc, hipStream_t st) {
  if (m <= 0 || n <= 0) return CR_OK;
  const int64_t sa_i = ta ? lda : 1, sa_t = ta ? 1 : lda;
  const int64_t sb_t = tb ? ldb : 1, sb_j = tb ? 1 : ldb;
  const dim3 grid((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64));
  hipLaunchKernelGGL(k_small_gemm, grid, dim3(NT), 0, st, m, n, k, A, sa_i, sa_t, B, sb_t, sb_j,
                     alpha, C, ldc);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_scale_inv_sqrt(int64_t n, T* __restrict__ x,
                                                       const double* __restrict__ nrm2) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const double s = 1.0 / sqrt(nrm2[0]);
  x[i] = (T)((double)x[i] * s);
}

template <typename T>
cr_status scale_inv_sqrt(int64_t n, T* x, const double* nrm2, hipStream_t st) {
  if (n == 0) return CR_OK;
  hipLaunchKernelGGL((k_scale_inv_sqrt<T>), dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st,
                     n, x, nrm2);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// SplitMix64 (Steele, Lea & Flood 2014): output k >= 1 of the generator whose
// state starts at seed ^ (stream * 0xD1B54A32D192ED03), top 53 bits mapped to
// [-1, 1).
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_splitmix(int64_t n, uint64_t state, T* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const uint64_t z = sm64_mix(state + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull);
  q[i] = (T)((double)(z >> 11) * 0x1.0p-52 - 1.0);
}

template <typename T>
cr_status splitmix_fill(int64_t n, uint64_t seed, uint64_t stream, T* q, hipStream_t st) {
  if (n == 0) return CR_OK;
  const uint64_t state = seed ^ (stream * 0xD1B54A32D192ED03ull);
  hipLaunchKernelGGL((k_splitmix<T>), dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, st, n,
                     state, q);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// out[c + a*ldo] -= sum_{i in hole_a} U[i,c] w[i]   (one workgroup per a)
template <typename T>
__global__ __launch_bounds__(NT) void k_hole_gram_col(const int32_t* __restrict__ hptr,
                                                      const int32_t* __restrict__ hidx, int r,
                                                      const T* __restrict__ U, int64_t ldu,
                                                      const T* __restrict__ w,
                                                      double* __restrict__ out, int64_t ldo) {
  __shared__ double red[NT / WAVE];
  const int a = blockIdx.x;
  const int b = hptr[a], e = hptr[a + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int c = 0; c < r; ++c) {
    double s = 0.0;
    for (int k = b + threadIdx.x; k < e; k += NT) {
      const int64_t i = hidx[k];
      s += (double)U[(int64_t)c * ldu + i] * (double)w[i];
    }
    s = wave_sum(s);
    if (lane == 0) red[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[(int64_t)a * ldo + c] -= red[0] + red[1] + red[2] + red[3];
    __syncthreads();
  }
}

template <typename T>
cr_status hole_gram_col(int ninj, const int32_t* hptr, const int32_t* hidx, int r, const T* U,
                        int64_t ldu, const T* w, double* out, int64_t ldo, hipStream_t st) {
  if (ninj == 0 || r == 0) return CR_OK;
  hipLaunchKernelGGL((k_hole_gram_col<T>), dim3(ninj), dim3(NT), 0, st, hptr, hidx, r, U, ldu, w,
                     out, ldo);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// ============================================================== instantiations
#define INST(T)                                                                                  \
  template cr_status stencil<T>(const Geom&, int, const T*, int64_t, T*, int64_t, hipStream_t); \
  template cr_status gemv_t<T>(int64_t, const Blocks<T>&, const T*, double*, double*,           \
                               hipStream_t);                                                    \
  template cr_status gemv_n<T>(int64_t, const Blocks<T>&, const double*, double, T*,            \
                               hipStream_t);                                                    \
  template cr_status gemm_tn<T>(int64_t, const Blocks<T>&, const Blocks<T>&, const uint32_t*,   \
                                const T*, int, double*, int64_t, double*, int64_t,             \
                                hipStream_t, int*);                                             \
  template cr_status zh_from_partials<T>(int, int, int, const double*, const T*, int64_t,       \
                                         double*, int64_t, hipStream_t);                        \
  template cr_status masked_tall_gemm<T>(int64_t, int, int, const T*, int64_t, const double*,   \
                                         int64_t, const uint32_t*, const T*, int64_t, T*,       \
                                         int64_t, hipStream_t);                                 \
  template bool op_win2_ok<T>(const Geom&, int, int);                                           \
  template cr_status op_win2<T>(const Geom&, int, const T*, int64_t, T*, T*, int64_t, int,      \
                                const double*, int64_t, const uint32_t*, T*, int64_t,          \
                                hipStream_t);                                                   \
  template cr_status masked_quad_ws<T>(int64_t, int, const uint32_t*, const double*, T*,        \
                                       double*, hipStream_t);                                   \
  template cr_status masked_colsq<T>(int64_t, int, const uint32_t*, const T*, double*,          \
                                     double*, hipStream_t);                                     \
  template cr_status scale_inv_sqrt<T>(int64_t, T*, const double*, hipStream_t);                \
  template cr_status splitmix_fill<T>(int64_t, uint64_t, uint64_t, T*, hipStream_t);            \
  template cr_status hole_gram_col<T>(int, const int32_t*, const int32_t*, int, const T*,       \
                                      int64_t, const T*, double*, int64_t, hipStream_t);
INST(double)
INST(float)
#undef INST
template cr_status gemv_tx<float, double>(int64_t, const Blocks<float>&, const double*, double*,
                                          double*, hipStream_t);
template cr_status convert2d<float, double>(int64_t, int64_t, const double*, int64_t, float*,
                                            int64_t, hipStream_t);
template cr_status convert2d<double, float>(int64_t, int64_t, const float*, int64_t, double*,
                                            int64_t, hipStream_t);
template cr_status convert2d<double, double>(int64_t, int64_t, const double*, int64_t, double*,
                                             int64_t, hipStream_t);
template cr_status convert2d<float, float>(int64_t, int64_t, const float*, int64_t, float*,
                                           int64_t, hipStream_t);
template cr_status convert<float, double>(int64_t, const double*, float*, hipStream_t);
template cr_status convert<double, float>(int64_t, const float*, double*, hipStream_t);

}  // namespace cr
