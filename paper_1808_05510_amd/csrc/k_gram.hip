// Batched masked Grams G_a = U^T diag(Omega_a) U for all injections a at once
// (the data term of eq. Proj_Sylv), in Khatri-Rao form: with one row per
// column pair (a <= b),
//   C[(a,b), alpha] = sum_i U_ia U_ib omega_{i,alpha},
// a GEMM of M = r(r+1)/2, N = n_inj, K = n_y on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  Omega is 0/1, exact in
// BF16; the products U_ia U_ib are rounded to BF16, so each entry carries an
// error below 2^-8 ||U_a|| ||U_b|| (relative 2^-9 per product, summed with
// nonnegative weights) plus the FP32 accumulation error.
#include <hip/hip_runtime.h>

#include "cr_internal.hpp"

namespace cr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float flt4 __attribute__((ext_vector_type(4)));

constexpr int KG_PAIRS = 128;  // pairs per workgroup (8 MFMA row tiles)
constexpr int KG_ALPHA = 128;  // injections per workgroup (8 MFMA column tiles)
constexpr int KG_K = 32;       // voxels per MFMA step
constexpr int KG_RMAX = 256;   // rank limit of the staged U rows

// pair index p = b (b + 1) / 2 + a  (a <= b, column-major upper triangle)
__host__ __device__ inline void pair_of(int p, int& a, int& b) {
  int bb = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while ((bb + 1) * (bb + 2) / 2 <= p) ++bb;
  while (bb * (bb + 1) / 2 > p) --bb;
  b = bb;
  a = p - bb * (bb + 1) / 2;
}

template <typename TU>
__global__ __launch_bounds__(NT) void k_kr_gram_bf16(int64_t n, int r, int ninj,
                                                     const TU* __restrict__ U, int64_t ldu,
                                                     const uint32_t* __restrict__ bits,
                                                     int npairs, int64_t kchunk,
                                                     float* __restrict__ part) {
  __shared__ float Us[KG_K][KG_RMAX + 1];
  __shared__ __attribute__((aligned(16))) __bf16 KR[KG_PAIRS][KG_K];
  __shared__ __attribute__((aligned(16))) __bf16 Bm[KG_ALPHA][KG_K];
  __shared__ int2 pab[KG_PAIRS];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int p0 = blockIdx.x * KG_PAIRS;
  const int al0 = blockIdx.z * KG_ALPHA;
  const int64_t k0 = (int64_t)blockIdx.y * kchunk;
  const int64_t k1 = min(n, k0 + kchunk);
  for (int q = tid; q < KG_PAIRS; q += NT) {
    int a = 0, b = 0;
    if (p0 + q < npairs) pair_of(p0 + q, a, b);
    pab[q] = make_int2(a, b);
  }
  flt4 acc[2][8];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[t][u] = flt4{0.f, 0.f, 0.f, 0.f};
  const int fr = lane & 15, fk = lane >> 4;
  for (int64_t kb = k0; kb < k1; kb += KG_K) {
    __syncthreads();
    // U rows of this voxel chunk
    for (int e = tid; e < KG_K * r; e += NT) {
      const int kk = e % KG_K, c = e / KG_K;
      const int64_t i = kb + kk;
      Us[kk][c] = i < k1 ? (float)U[(int64_t)c * ldu + i] : 0.f;
    }
    // Omega as BF16 0/1, [alpha][k]
    for (int e = tid; e < KG_ALPHA * KG_K; e += NT) {
      const int kk = e % KG_K, aa = e / KG_K;
      const int64_t i = kb + kk;
      const int al = al0 + aa;
      float v = 0.f;
      if (i < k1 && al < ninj) v = (float)((bits[(int64_t)(al >> 5) * n + i] >> (al & 31)) & 1u);
      Bm[aa][kk] = (__bf16)v;
    }
    __syncthreads();
    // Khatri-Rao rows U_ia U_ib for the block's pairs, [pair][k]
    for (int e = tid; e < KG_PAIRS * KG_K; e += NT) {
      const int kk = e % KG_K, q = e / KG_K;
      const int2 ab = pab[q];
      KR[q][kk] = (__bf16)(Us[kk][ab.x] * Us[kk][ab.y]);
    }
    __syncthreads();
    bf16x8 bfr[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) bfr[u] = *(const bf16x8*)&Bm[16 * u + fr][8 * fk];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const bf16x8 afr = *(const bf16x8*)&KR[32 * wv + 16 * t + fr][8 * fk];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[u], acc[t][u], 0, 0, 0);
    }
  }
  // result element e of lane l: row (pair) 16 t + 4 fk + e, column (alpha) 16 u + fr
  float* out = part + (int64_t)blockIdx.y * npairs * ninj;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int p = p0 + 32 * wv + 16 * t + 4 * fk + e;
        const int al = al0 + 16 * u + fr;
        if (p < npairs && al < ninj) out[(int64_t)al * npairs + p] = acc[t][u][e];
      }
}

// G[al](a, b) = G[al](b, a) = sum_z part[z][al][p]  (FP64 output, ld ldr)
__global__ __launch_bounds__(NT) void k_kr_scatter(int npairs, int ninj, int ks,
                                                   const float* __restrict__ part,
                                                   double* __restrict__ G, int64_t ldr) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= (int64_t)npairs * ninj) return;
  const int p = (int)(e % npairs), al = (int)(e / npairs);
  double s = 0.0;
  for (int z = 0; z < ks; ++z) s += (double)part[(int64_t)z * npairs * ninj + e];
  int a, b;
  pair_of(p, a, b);
  double* Ga = G + (int64_t)al * ldr * ldr;
  Ga[(int64_t)b * ldr + a] = s;
  Ga[(int64_t)a * ldr + b] = s;
}

int64_t kr_gram_part_size(int64_t n, int r, int ninj) {
  const int64_t npairs = (int64_t)r * (r + 1) / 2;
  const int64_t ks = std::max<int64_t>(1, std::min<int64_t>(32, (n + 4095) / 4096));
  return ks * npairs * ninj;
}

template <typename TU>
cr_status kr_gram_bf16(int64_t n, int r, int ninj, const TU* U, int64_t ldu, const uint32_t* bits,
                       double* G, int64_t ldr, float* part, hipStream_t st) {
  if (r <= 0 || ninj <= 0) return CR_OK;
  if (r > KG_RMAX) {
    set_error("BF16 masked Gram: rank above 256");
    return CR_EINVAL;
  }
  const int npairs = r * (r + 1) / 2;
  int64_t ks = std::max<int64_t>(1, std::min<int64_t>(32, (n + 4095) / 4096));
  int64_t kchunk = (n + ks - 1) / ks;
  kchunk = (kchunk + KG_K - 1) / KG_K * KG_K;
  ks = std::max<int64_t>(1, (n + kchunk - 1) / kchunk);
  dim3 grid((npairs + KG_PAIRS - 1) / KG_PAIRS, (unsigned)ks, (ninj + KG_ALPHA - 1) / KG_ALPHA);
  hipLaunchKernelGGL((k_kr_gram_bf16<TU>), grid, dim3(NT), 0, st, n, r, ninj, U, ldu, bits, npairs,
                     kchunk, part);
  CR_HIP(hipGetLastError());
  const int64_t m = (int64_t)npairs * ninj;
  hipLaunchKernelGGL(k_kr_scatter, dim3((unsigned)((m + NT - 1) / NT)), dim3(NT), 0, st, npairs,
                     ninj, (int)ks, part, G, ldr);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

template cr_status kr_gram_bf16<double>(int64_t, int, int, const double*, int64_t, const uint32_t*,
                                        double*, int64_t, float*, hipStream_t);
template cr_status kr_gram_bf16<float>(int64_t, int, int, const float*, int64_t, const uint32_t*,
                                       double*, int64_t, float*, hipStream_t);

}  // namespace cr
