// Batched masked Grams G_a = U^T diag(Omega_a) U for all injections a at once
// (the data term of eq. Proj_Sylv), in Khatri-Rao form: with one row per
// column pair (a <= b),
//   C[(a,b), alpha] = sum_i U_ia U_ib omega_{i,alpha},
// a GEMM of M = r(r+1)/2, N = n_inj, K = n_y on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  Omega is 0/1, exact in
// BF16; the products U_ia U_ib are rounded to BF16, so each entry carries an
// error below 2^-8 ||U_a|| ||U_b|| (relative 2^-9 per product, summed with
// nonnegative weights) plus the FP32 accumulation error.
// Pairs are taken in 16 x 16 column blocks (a-block <= b-block), so a
// workgroup stages only 32 columns of U per step and forms the 256 products
// per voxel in registers; Omega is converted once to a BF16 matrix and
// staged as the shared B tile.  Diagonal blocks compute their lower half
// too (discarded), and r is padded to a multiple of 16.
#include <hip/hip_runtime.h>

#include "cr_internal.hpp"

#include <vector>

namespace cr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float flt4 __attribute__((ext_vector_type(4)));

constexpr int KG_BLK = 16;    // columns per a-block and per b-block (256 pairs per workgroup)
constexpr int KG_INJ = 128;   // injections per workgroup (8 MFMA column tiles)
constexpr int KG_K = 32;      // voxels per MFMA step
constexpr int KG_ULD = KG_K + 1;   // LDS row of one staged U column (floats)
constexpr int KG_OLD = KG_K + 8;   // LDS row of one staged Omega column (bf16)

// Omega as BF16 0/1, column-major n x ninj (ld n): the B operand of the GEMM,
// read as 16-byte fragments (8 consecutive voxels of one injection)
__global__ __launch_bounds__(NT) void k_omega_bf16(int64_t n, int ninj,
                                                   const uint32_t* __restrict__ bits,
                                                   __bf16* __restrict__ ob) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int al = blockIdx.y;
  if (i >= n) return;
  const uint32_t w = bits[(int64_t)(al >> 5) * n + i];
  ob[(int64_t)al * n + i] = (__bf16)(float)((w >> (al & 31)) & 1u);
}

// Workgroup (blk, z, ib): column block pair (ablk <= bblk) from the upper
// triangle list, voxel slab z, injection block ib.  Wave wv owns the pair
// tiles b = bblk*16 + 4 wv + tt (tt < 4), each tile being the 16 pairs
// (a = ablk*16 + 0..15, b) -- 32 MFMA tiles with the 8 injection tiles.
// Per 32-voxel step: U columns of both blocks (32 x 32, FP32) and the Omega
// tile (128 injections x 32 voxels, BF16) are staged in LDS (double
// buffered, loads for the next step in flight); each wave forms its A
// fragments U_ia U_ib in registers and issues 32 MFMAs.
template <typename TU>
__global__ __launch_bounds__(NT) void k_kr_gram_bf16(int64_t n, int r, int ninj,
                                                     const TU* __restrict__ U, int64_t ldu,
                                                     const __bf16* __restrict__ ob,
                                                     const int2* __restrict__ blocks,
                                                     int64_t kchunk, float* __restrict__ part) {
  __shared__ float Us[2][2 * KG_BLK][KG_ULD];
  __shared__ __attribute__((aligned(16))) __bf16 Os[2][KG_INJ][KG_OLD];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int2 bp = blocks[blockIdx.x];
  const int a0 = bp.x * KG_BLK, b0 = bp.y * KG_BLK;
  const int al0 = blockIdx.z * KG_INJ;
  const int64_t k0 = (int64_t)blockIdx.y * kchunk;
  const int64_t k1 = min(n, k0 + kchunk);
  // loaders: U element (column uc, voxels 4 uq .. 4 uq + 3); Omega 16-byte
  // pieces (injection oc + 64 m, voxels 8 oq .. 8 oq + 7)
  const int uc = tid >> 3, uq = tid & 7;
  const int ucol = uc < KG_BLK ? a0 + uc : b0 + uc - KG_BLK;
  const TU* ubase = ucol < r ? U + (int64_t)ucol * ldu : nullptr;
  const int oc = tid >> 2, oq = tid & 3;
  float ur[4];
  uint4 orr[2];
  auto load = [&](int64_t kb) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t v = kb + 4 * uq + j;
      ur[j] = (ubase && v < k1) ? (float)ubase[v] : 0.f;
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int al = al0 + oc + 64 * m;
      const int64_t v = kb + 8 * oq;
      uint4 val = make_uint4(0u, 0u, 0u, 0u);
      if (al < ninj) {
        if (v + 8 <= k1 && ((n & 7) == 0)) {
          val = *(const uint4*)(ob + (int64_t)al * n + v);
        } else {
          __bf16 tmp[8];
#pragma unroll
          for (int j = 0; j < 8; ++j)
            tmp[j] = (v + j < k1) ? ob[(int64_t)al * n + v + j] : (__bf16)0.f;
          val = *(const uint4*)tmp;
        }
      }
      orr[m] = val;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 4; ++j) Us[buf][uc][4 * uq + j] = ur[j];
#pragma unroll
    for (int m = 0; m < 2; ++m) *(uint4*)&Os[buf][oc + 64 * m][8 * oq] = orr[m];
  };
  flt4 acc[4][8];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[t][u] = flt4{0.f, 0.f, 0.f, 0.f};
  const int fr = lane & 15, fk = lane >> 4;
  int buf = 0;
  if (k0 < k1) {
    load(k0);
    store(0);
  }
  __syncthreads();
  for (int64_t kb = k0; kb < k1; kb += KG_K) {
    const bool more = kb + KG_K < k1;
    if (more) load(kb + KG_K);
    // A fragments: lane (fr, fk) holds pair (a0 + fr, b) at voxels 8 fk .. 8 fk + 7
    float av[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) av[j] = Us[buf][fr][8 * fk + j];
    bf16x8 afr[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int bc = KG_BLK + 4 * wv + t;
#pragma unroll
      for (int j = 0; j < 8; ++j) afr[t][j] = (__bf16)(av[j] * Us[buf][bc][8 * fk + j]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bf16x8 bfr = *(const bf16x8*)&Os[buf][16 * u + fr][8 * fk];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[t], bfr, acc[t][u], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // result element e of lane l: row (a offset) 4 fk + e, column (injection) 16 u + fr
  // partial layout: part[z][blk][b_local][a_local][injection]
  const int nib = gridDim.z;
  float* out = part + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * (KG_BLK * KG_BLK) *
                          (int64_t)(KG_INJ * nib);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int al = al0 + 16 * u + fr;
        const int pl = (4 * wv + t) * KG_BLK + 4 * fk + e;
        out[(int64_t)pl * (KG_INJ * nib) + al] = acc[t][u][e];
      }
}

// G[al](a, b) = G[al](b, a) = sum_z part[z][blk][b_local][a_local][al]
__global__ __launch_bounds__(NT) void k_kr_scatter(int nblk, int ks, int r, int ninj, int ninjp,
                                                   const int2* __restrict__ blocks,
                                                   const float* __restrict__ part,
                                                   double* __restrict__ G, int64_t ldr) {
  const int64_t per = (int64_t)KG_BLK * KG_BLK * ninjp;
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= per * nblk) return;
  const int blk = (int)(e / per);
  const int64_t w = e % per;
  const int al = (int)(w % ninjp);
  const int pl = (int)(w / ninjp);
  const int a = blocks[blk].x * KG_BLK + pl % KG_BLK;
  const int b = blocks[blk].y * KG_BLK + pl / KG_BLK;
  if (al >= ninj || a >= r || b >= r || a > b) return;
  double s = 0.0;
  for (int z = 0; z < ks; ++z) s += (double)part[((int64_t)z * nblk + blk) * per + w];
  double* Ga = G + (int64_t)al * ldr * ldr;
  Ga[(int64_t)b * ldr + a] = s;
  Ga[(int64_t)a * ldr + b] = s;
}

static int kr_nblocks(int r) {
  const int nb = (r + KG_BLK - 1) / KG_BLK;
  return nb * (nb + 1) / 2;
}

static int64_t kr_splits(int64_t n, int r, int ninj) {
  const int64_t wgs = (int64_t)kr_nblocks(r) * ((ninj + KG_INJ - 1) / KG_INJ);
  // about 1024 workgroups, each at least 64 steps of 32 voxels deep
  int64_t ks = std::max<int64_t>(1, 1024 / std::max<int64_t>(wgs, 1));
  ks = std::min<int64_t>(ks, std::max<int64_t>(1, n / (64 * KG_K)));
  return ks;
}

int64_t kr_gram_part_size(int64_t n, int r, int ninj) {
  const int ninjp = (ninj + KG_INJ - 1) / KG_INJ * KG_INJ;
  return kr_splits(n, r, ninj) * kr_nblocks(r) * (int64_t)KG_BLK * KG_BLK * ninjp;
}

int64_t kr_gram_aux_size(int64_t n, int r, int ninj) {
  // bytes: BF16 Omega (n x ninj) + block list
  return (int64_t)n * ninj * 2 + 16 * (int64_t)kr_nblocks(r) + 256;
}

template <typename TU>
cr_status kr_gram_bf16(int64_t n, int r, int ninj, const TU* U, int64_t ldu, const uint32_t* bits,
                       double* G, int64_t ldr, float* part, void* aux, bool omega_ready,
                       hipStream_t st) {
  if (r <= 0 || ninj <= 0) return CR_OK;
  __bf16* ob = (__bf16*)aux;
  int2* blocks = (int2*)((char*)aux + ((int64_t)n * ninj * 2 + 255) / 256 * 256);
  const int nb = (r + KG_BLK - 1) / KG_BLK;
  const int nblk = kr_nblocks(r);
  std::vector<int2> hb;
  for (int bb = 0; bb < nb; ++bb)
    for (int ab = 0; ab <= bb; ++ab) hb.push_back(make_int2(ab, bb));
  CR_HIP(hipMemcpyAsync(blocks, hb.data(), sizeof(int2) * hb.size(), hipMemcpyHostToDevice, st));
  if (!omega_ready) {
    hipLaunchKernelGGL(k_omega_bf16, dim3((unsigned)((n + NT - 1) / NT), (unsigned)ninj), dim3(NT),
                       0, st, n, ninj, bits, ob);
    CR_HIP(hipGetLastError());
  }
  int64_t ks = kr_splits(n, r, ninj);
  int64_t kchunk = (n + ks - 1) / ks;
  kchunk = (kchunk + KG_K - 1) / KG_K * KG_K;
  ks = std::max<int64_t>(1, (n + kchunk - 1) / kchunk);
  const int nib = (ninj + KG_INJ - 1) / KG_INJ;
  dim3 grid((unsigned)nblk, (unsigned)ks, (unsigned)nib);
  hipLaunchKernelGGL((k_kr_gram_bf16<TU>), grid, dim3(NT), 0, st, n, r, ninj, U, ldu, ob, blocks,
                     kchunk, part);
  CR_HIP(hipGetLastError());
  const int ninjp = nib * KG_INJ;
  const int64_t m = (int64_t)nblk * KG_BLK * KG_BLK * ninjp;
  hipLaunchKernelGGL(k_kr_scatter, dim3((unsigned)((m + NT - 1) / NT)), dim3(NT), 0, st, nblk,
                     (int)ks, r, ninj, ninjp, blocks, part, G, ldr);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

template cr_status kr_gram_bf16<double>(int64_t, int, int, const double*, int64_t, const uint32_t*,
                                        double*, int64_t, float*, void*, bool, hipStream_t);
template cr_status kr_gram_bf16<float>(int64_t, int, int, const float*, int64_t, const uint32_t*,
                                       double*, int64_t, float*, void*, bool, hipStream_t);

}  // namespace cr
