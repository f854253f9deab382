// Learned preconditioner for the ALS u-system (eq. ALS_linsys) on a box
// grid: a small two-level 3-D convolutional network trained on the GPU by
// the kernels below (forward, data gradient, weight gradient, pooling,
// loss, Adam), applied inside flexible CG with the base step as fallback and
// Jacobi-PCG as the last resort.
//
// Grid: nx * ny * nz voxels, index v = x + nx (y + ny z), the numbering of
// the box generator.  Activations are channel-major [C][N] float.
// Network (C hidden channels, 3x3x3 convolutions with zero padding):
//   a0 = relu(conv(in, 4 -> C))         full resolution
//   a1 = relu(conv(a0, C -> C))         full
//   p  = avgpool2(a1)                   half
//   a2 = relu(conv(p, C -> C))          half
//   a3 = relu(conv(a2, C -> C))         half
//   s  = upsample2(a3) + a1             full (nearest, skip connection)
//   y  = conv(s, C -> 1)                full
// The network refines the base step w = M^-1 r of the flexible CG (the
// spectral solve of the box when the target is declared a full box, else the
// Jacobi step D^-1 r, D the Jacobi diagonal of the u-system).  Its inputs are
//   [ sqrt(N) w / ||w||,  d / D,  lambda c0 / D,  lambda c1 deg / D ]
// (the last three are the data, mass and first-order fractions of the
// diagonal, all in [0, 1]) and the preconditioned residual is
//   z = sqrt(N) w / ||w|| + y,
// so an untrained network (zero last layer) returns the base step.  FCG is
// invariant to the scale of z; training minimises 1 - cos^2(z, x*) with x*
// the exact solution for right-hand side r.
#include <hip/hip_runtime.h>

#include "cr_internal.hpp"

namespace cr {

__device__ __forceinline__ float wsumf(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

struct Dims {
  int nx, ny, nz;
};

__device__ __forceinline__ void coords(const Dims& d, int64_t v, int& x, int& y, int& z) {
  x = (int)(v % d.nx);
  const int64_t t = v / d.nx;
  y = (int)(t % d.ny);
  z = (int)(t / d.ny);
}

// ---------------------------------------------------------------- conv forward
// out[co][v] = bias[co] + sum_{ci,k} W[co][ci][k] in[ci][v + off_k], relu optional
__global__ __launch_bounds__(NT) void k_conv_fwd(Dims d, int CI, int CO, const float* __restrict__ in,
                                                 const float* __restrict__ W,
                                                 const float* __restrict__ bias,
                                                 float* __restrict__ out, int relu) {
  __shared__ float ws[LPC_MAXC * LPC_MAXC * 27];
  const int nw = CO * CI * 27;
  for (int e = threadIdx.x; e < nw; e += NT) ws[e] = W[e];
  __syncthreads();
  const int64_t N = (int64_t)d.nx * d.ny * d.nz;
  const int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (v >= N) return;
  int x, y, z;
  coords(d, v, x, y, z);
  float acc[LPC_MAXC];
#pragma unroll
  for (int co = 0; co < LPC_MAXC; ++co) acc[co] = co < CO ? bias[co] : 0.f;
  for (int k = 0; k < 27; ++k) {
    const int dz = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
    const int xx = x + dx, yy = y + dy, zz = z + dz;
    if (xx < 0 || yy < 0 || zz < 0 || xx >= d.nx || yy >= d.ny || zz >= d.nz) continue;
    const int64_t u = xx + (int64_t)d.nx * (yy + (int64_t)d.ny * zz);
    for (int ci = 0; ci < CI; ++ci) {
      const float val = in[(int64_t)ci * N + u];
#pragma unroll
      for (int co = 0; co < LPC_MAXC; ++co)
        if (co < CO) acc[co] += ws[(co * CI + ci) * 27 + k] * val;
    }
  }
  for (int co = 0; co < CO; ++co) {
    const float a = acc[co];
    out[(int64_t)co * N + v] = relu ? fmaxf(a, 0.f) : a;
  }
}

// Inference form of the same convolution: one thread per (voxel, group of G
// output channels), the group on grid.y.  Taps and input channels are
// unrolled at compile time (one z-plane of taps at a time), out-of-box taps
// read the voxel itself with a zero factor, so the 9 * CI loads of a plane
// are independent and in flight together.  At 40^3 the one-output-set-per-thread form had one wave per SIMD
// and paid each load's latency in turn; splitting the outputs over G-groups
// multiplies the waves.
//
// BWD: the data gradient din[c][v] = sum_{o,k} W[o][c][k] dout[o][v - off_k]
// of a layer with nout = its input count, in the same form: off_{26-k} =
// -off_k, so the staged weights are ws[g][o][k] = W[o][co0 + g][26 - k]
// (flipped and transposed), CI is the layer's output count and no bias.
template <int CI, int G, bool BWD>
__global__ __launch_bounds__(NT) void k_conv_fwd_g(Dims d, const float* __restrict__ in,
                                                   const float* __restrict__ W,
                                                   const float* __restrict__ bias,
                                                   float* __restrict__ out, int relu, int nout) {
  __shared__ float ws[G * CI * 27];
  const int co0 = blockIdx.y * G;
  for (int e = threadIdx.x; e < G * CI * 27; e += NT) {
    if constexpr (BWD) {
      const int g = e / (CI * 27), c = (e / 27) % CI, k = e % 27;
      ws[e] = W[(c * nout + co0 + g) * 27 + 26 - k];
    } else {
      ws[e] = W[co0 * CI * 27 + e];
    }
  }
  __syncthreads();
  const int N = d.nx * d.ny * d.nz;
  const int v = blockIdx.x * NT + threadIdx.x;
  if (v >= N) return;
  const int x = v % d.nx;
  const int t = v / d.nx;
  const int y = t % d.ny;
  const int z = t / d.ny;
  float acc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) acc[g] = BWD ? 0.f : bias[co0 + g];
  // one z-plane of taps (9 x CI loads) unrolled at a time: all taps at once
  // held 216 loads in flight and 454+ VGPRs (one wave per SIMD, spills at G 2)
#pragma unroll 1
  for (int kz = 0; kz < 3; ++kz) {
    const int zz = z + kz - 1;
#pragma unroll
    for (int kk = 0; kk < 9; ++kk) {
      const int k = 9 * kz + kk;
      const int dy = kk / 3 - 1, dx = kk % 3 - 1;
      const int xx = x + dx, yy = y + dy;
      const bool inside =
          xx >= 0 && yy >= 0 && zz >= 0 && xx < d.nx && yy < d.ny && zz < d.nz;
      const int u = inside ? xx + d.nx * (yy + d.ny * zz) : v;
      const float f = inside ? 1.f : 0.f;
#pragma unroll
      for (int ci = 0; ci < CI; ++ci) {
        const float val = f * in[ci * N + u];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] += ws[(g * CI + ci) * 27 + k] * val;
      }
    }
  }
#pragma unroll
  for (int g = 0; g < G; ++g) out[(co0 + g) * N + v] = relu ? fmaxf(acc[g], 0.f) : acc[g];
}

// ---------------------------------------------------------------- conv data gradient
// din[ci][v] = sum_{co,k} W[co][ci][k] dout[co][v - off_k]
__global__ __launch_bounds__(NT) void k_conv_dgrad(Dims d, int CI, int CO,
                                                   const float* __restrict__ dout,
                                                   const float* __restrict__ W,
                                                   float* __restrict__ din) {
  __shared__ float ws[LPC_MAXC * LPC_MAXC * 27];
  const int nw = CO * CI * 27;
  for (int e = threadIdx.x; e < nw; e += NT) ws[e] = W[e];
  __syncthreads();
  const int64_t N = (int64_t)d.nx * d.ny * d.nz;
  const int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (v >= N) return;
  int x, y, z;
  coords(d, v, x, y, z);
  float acc[LPC_MAXC];
#pragma unroll
  for (int ci = 0; ci < LPC_MAXC; ++ci) acc[ci] = 0.f;
  for (int k = 0; k < 27; ++k) {
    const int dz = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
    const int xx = x - dx, yy = y - dy, zz = z - dz;
    if (xx < 0 || yy < 0 || zz < 0 || xx >= d.nx || yy >= d.ny || zz >= d.nz) continue;
    const int64_t u = xx + (int64_t)d.nx * (yy + (int64_t)d.ny * zz);
    for (int co = 0; co < CO; ++co) {
      const float g = dout[(int64_t)co * N + u];
#pragma unroll
      for (int ci = 0; ci < LPC_MAXC; ++ci)
        if (ci < CI) acc[ci] += ws[(co * CI + ci) * 27 + k] * g;
    }
  }
  for (int ci = 0; ci < CI; ++ci) din[(int64_t)ci * N + v] = acc[ci];
}

// ---------------------------------------------------------------- conv weight gradient
// partial[b][(co*CI+ci)*27+k] = sum_{v in block b} dout[co][v] in[ci][v + off_k];
// partial[b][CO*CI*27 + co] = sum_{v in block b} dout[co][v] (bias).
// Wave sums of each product, accumulated per workgroup in LDS.
__global__ __launch_bounds__(NT) void k_conv_wgrad(Dims d, int CI, int CO,
                                                   const float* __restrict__ in,
                                                   const float* __restrict__ dout,
                                                   float* __restrict__ partial) {
  __shared__ float acc[LPC_MAXC * LPC_MAXC * 27 + LPC_MAXC];
  const int nw = CO * CI * 27;
  for (int e = threadIdx.x; e < nw + CO; e += NT) acc[e] = 0.f;
  __syncthreads();
  const int64_t N = (int64_t)d.nx * d.ny * d.nz;
  const int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const bool ok = v < N;
  int x = 0, y = 0, z = 0;
  if (ok) coords(d, v, x, y, z);
  float g[LPC_MAXC];
#pragma unroll
  for (int co = 0; co < LPC_MAXC; ++co) g[co] = (ok && co < CO) ? dout[(int64_t)co * N + v] : 0.f;
  for (int co = 0; co < CO; ++co) {
    const float s = wsumf(g[co]);
    if (lane == 0) atomicAdd(&acc[nw + co], s);
  }
  for (int k = 0; k < 27; ++k) {
    const int dz = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
    const int xx = x + dx, yy = y + dy, zz = z + dz;
    const bool in_range =
        ok && !(xx < 0 || yy < 0 || zz < 0 || xx >= d.nx || yy >= d.ny || zz >= d.nz);
    const int64_t u = in_range ? xx + (int64_t)d.nx * (yy + (int64_t)d.ny * zz) : 0;
    for (int ci = 0; ci < CI; ++ci) {
      const float val = in_range ? in[(int64_t)ci * N + u] : 0.f;
      for (int co = 0; co < CO; ++co) {
        const float s = wsumf(g[co] * val);
        if (lane == 0) atomicAdd(&acc[(co * CI + ci) * 27 + k], s);
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nw + CO; e += NT)
    partial[(int64_t)blockIdx.x * (nw + CO) + e] = acc[e];
}

// Register form of the weight gradient.  Grid (xb, 27): block (b, k) takes
// tap k over the voxels v = b NT + t + j S (S = NT xb, j = 0, 1, ...); each
// thread keeps the CO x CI products dout[co][v] in[ci][v + off_k] and the
// CO bias terms of its voxels in registers, and the block sums them once at
// the end (wave shuffles, then the waves through LDS) into
// partial[b][(co CI + ci) 27 + k], the k = 0 blocks also into the bias slots
// partial[b][CO CI 27 + co].  The generic kernel above reduced over the wave
// for every product of every voxel.
template <int CI, int CO>
__global__ __launch_bounds__(NT) void k_conv_wgrad_t(Dims d, const float* __restrict__ in,
                                                     const float* __restrict__ dout,
                                                     float* __restrict__ partial) {
  constexpr int NA = CO * CI + CO;
  constexpr int NWV = NT / WAVE;
  __shared__ float red[NWV][NA];
  const int k = blockIdx.y;
  const int N = d.nx * d.ny * d.nz;
  const int dz = k / 9 - 1, dy = (k / 3) % 3 - 1, dx = k % 3 - 1;
  const int off = dx + d.nx * (dy + d.ny * dz);
  const int S = NT * gridDim.x;
  // coordinates of the first voxel and of the stride S; the loop advances
  // them digit by digit (x, y < their extents, so one carry each)
  int v = blockIdx.x * NT + threadIdx.x;
  int x = v % d.nx, t = v / d.nx;
  int y = t % d.ny, z = t / d.ny;
  const int sx = S % d.nx, st = S / d.nx;
  const int sy = st % d.ny, sz = st / d.ny;
  float acc[NA];
#pragma unroll
  for (int e = 0; e < NA; ++e) acc[e] = 0.f;
  for (; v < N; v += S) {
    const int xx = x + dx, yy = y + dy, zz = z + dz;
    const bool inside =
        xx >= 0 && yy >= 0 && zz >= 0 && xx < d.nx && yy < d.ny && zz < d.nz;
    const int u = inside ? v + off : v;
    const float f = inside ? 1.f : 0.f;
    float a[CI], g[CO];
#pragma unroll
    for (int ci = 0; ci < CI; ++ci) a[ci] = f * in[ci * N + u];
#pragma unroll
    for (int co = 0; co < CO; ++co) g[co] = dout[co * N + v];
#pragma unroll
    for (int co = 0; co < CO; ++co) {
#pragma unroll
      for (int ci = 0; ci < CI; ++ci) acc[co * CI + ci] += g[co] * a[ci];
      acc[CO * CI + co] += g[co];
    }
    x += sx;
    const int cy = x >= d.nx;
    x -= cy ? d.nx : 0;
    y += sy + cy;
    const int cz = y >= d.ny;
    y -= cz ? d.ny : 0;
    z += sz + cz;
  }
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
  for (int e = 0; e < NA; ++e) {
    const float s = wsumf(acc[e]);
    if (lane == 0) red[w][e] = s;
  }
  __syncthreads();
  float* p = partial + (int64_t)blockIdx.x * (CO * CI * 27 + CO);
  for (int e = threadIdx.x; e < NA; e += NT) {
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < NWV; ++i) s += red[i][e];
    if (e < CO * CI)
      p[e * 27 + k] = s;
    else if (k == 0)
      p[CO * CI * 27 + (e - CO * CI)] = s;
  }
}

// gW[e] += sum_b partial[b][e]  (fixed order)
__global__ __launch_bounds__(NT) void k_sum_partials(int nb, int m, const float* __restrict__ partial,
                                                     float* __restrict__ gW, float* __restrict__ gB,
                                                     int nw) {
  const int e = blockIdx.x * NT + threadIdx.x;
  if (e >= m) return;
  float s = 0.f;
  for (int b = 0; b < nb; ++b) s += partial[(int64_t)b * m + e];
  if (e < nw)
    gW[e] += s;
  else
    gB[e - nw] += s;
}

// ---------------------------------------------------------------- pooling / upsampling
// coarse dims: ceil(n/2) per axis; coarse voxel averages its (up to 8) children
__host__ __device__ __forceinline__ Dims coarse(const Dims& d) {
  return Dims{(d.nx + 1) / 2, (d.ny + 1) / 2, (d.nz + 1) / 2};
}

__global__ __launch_bounds__(NT) void k_pool_fwd(Dims d, int C, const float* __restrict__ in,
                                                 float* __restrict__ out) {
  const Dims c = coarse(d);
  const int64_t Nc = (int64_t)c.nx * c.ny * c.nz, N = (int64_t)d.nx * d.ny * d.nz;
  const int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (q >= Nc) return;
  int X, Y, Z;
  coords(c, q, X, Y, Z);
  for (int ch = 0; ch < C; ++ch) {
    float s = 0.f;
    for (int t = 0; t < 8; ++t) {
      const int x = 2 * X + (t & 1), y = 2 * Y + ((t >> 1) & 1), z = 2 * Z + (t >> 2);
      if (x < d.nx && y < d.ny && z < d.nz) s += in[(int64_t)ch * N + x + (int64_t)d.nx * (y + (int64_t)d.ny * z)];
    }
    out[(int64_t)ch * Nc + q] = 0.125f * s;
  }
}

// din[child] += dout[parent] / 8
__global__ __launch_bounds__(NT) void k_pool_bwd(Dims d, int C, const float* __restrict__ dout,
                                                 float* __restrict__ din) {
  const Dims c = coarse(d);
  const int64_t Nc = (int64_t)c.nx * c.ny * c.nz, N = (int64_t)d.nx * d.ny * d.nz;
  const int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (v >= N) return;
  int x, y, z;
  coords(d, v, x, y, z);
  const int64_t q = (x / 2) + (int64_t)c.nx * ((y / 2) + (int64_t)c.ny * (z / 2));
  for (int ch = 0; ch < C; ++ch) din[(int64_t)ch * N + v] += 0.125f * dout[(int64_t)ch * Nc + q];
}

// out[v] = in[parent(v)] + skip[v]
__global__ __launch_bounds__(NT) void k_up_add(Dims d, int C, const float* __restrict__ inc,
                                               const float* __restrict__ skip,
                                               float* __restrict__ out) {
  const Dims c = coarse(d);
  const int64_t Nc = (int64_t)c.nx * c.ny * c.nz, N = (int64_t)d.nx * d.ny * d.nz;
  const int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (v >= N) return;
  int x, y, z;
  coords(d, v, x, y, z);
  const int64_t q = (x / 2) + (int64_t)c.nx * ((y / 2) + (int64_t)c.ny * (z / 2));
  for (int ch = 0; ch < C; ++ch)
    out[(int64_t)ch * N + v] = inc[(int64_t)ch * Nc + q] + skip[(int64_t)ch * N + v];
}

// dinc[parent] = sum of dout over its children
__global__ __launch_bounds__(NT) void k_up_bwd(Dims d, int C, const float* __restrict__ dout,
                                               float* __restrict__ dinc) {
  const Dims c = coarse(d);
  const int64_t Nc = (int64_t)c.nx * c.ny * c.nz, N = (int64_t)d.nx * d.ny * d.nz;
  const int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (q >= Nc) return;
  int X, Y, Z;
  coords(c, q, X, Y, Z);
  for (int ch = 0; ch < C; ++ch) {
    float s = 0.f;
    for (int t = 0; t < 8; ++t) {
      const int x = 2 * X + (t & 1), y = 2 * Y + ((t >> 1) & 1), z = 2 * Z + (t >> 2);
      if (x < d.nx && y < d.ny && z < d.nz) s += dout[(int64_t)ch * N + x + (int64_t)d.nx * (y + (int64_t)d.ny * z)];
    }
    dinc[(int64_t)ch * Nc + q] = s;
  }
}

// g[i] *= (a[i] > 0)
__global__ __launch_bounds__(NT) void k_relu_bwd(int64_t n, const float* __restrict__ a,
                                                 float* __restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < n && !(a[i] > 0.f)) g[i] = 0.f;
}

// ---------------------------------------------------------------- inputs, loss, Adam
// in = [sqrt(N) w/||w||, d minv, lam c0 minv, lam c1 deg minv], w = minv o r
__global__ __launch_bounds__(NT) void k_lpc_input(int64_t N, const double* __restrict__ w,
                                                  const double* __restrict__ w2,
                                                  const double* __restrict__ minv,
                                                  const double* __restrict__ dvec,
                                                  const uint8_t* __restrict__ deg,
                                                  const double* __restrict__ coef, double lam,
                                                  float* __restrict__ in) {
  const int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (v >= N) return;
  const double s = w2[0] > 0.0 ? sqrt((double)N / w2[0]) : 0.0;
  const double mi = minv[v];
  in[v] = (float)(w[v] * s);
  in[N + v] = (float)(dvec[v] * mi);
  in[2 * N + v] = (float)(lam * coef[1] * mi);
  in[3 * N + v] = (float)(lam * coef[0] * (double)deg[v] * mi);
}

// z = in0 + y
__global__ __launch_bounds__(NT) void k_lpc_output(int64_t N, const float* __restrict__ in0,
                                                   const float* __restrict__ y,
                                                   double* __restrict__ z) {
  const int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (v >= N) return;
  z[v] = (double)in0[v] + (double)y[v];
}

// partial dots of z = in0 + y with the target: [z.x, z.z, x.x] per workgroup
__global__ __launch_bounds__(NT) void k_lpc_dots(int64_t N, const float* __restrict__ in0,
                                                 const float* __restrict__ y,
                                                 const double* __restrict__ xs,
                                                 double* __restrict__ part, int nb) {
  __shared__ double red[3][NT / WAVE];
  const int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x;
  double zx = 0.0, zz = 0.0, xx = 0.0;
  if (v < N) {
    const double z = (double)in0[v] + (double)y[v], x = xs[v];
    zx = z * x;
    zz = z * z;
    xx = x * x;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    zx += __shfl_xor(zx, o, WAVE);
    zz += __shfl_xor(zz, o, WAVE);
    xx += __shfl_xor(xx, o, WAVE);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = zx;
    red[1][threadIdx.x >> 6] = zz;
    red[2][threadIdx.x >> 6] = xx;
  }
  __syncthreads();
  if (threadIdx.x < 3)
    part[(int64_t)threadIdx.x * nb + blockIdx.x] =
        red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
}

// tot[0..2] = sums of the partials; tot[3] = loss 1 - cos^2
__global__ __launch_bounds__(NT) void k_lpc_dots_total(int nb, const double* __restrict__ part,
                                                       double* __restrict__ tot) {
  __shared__ double red[NT / WAVE];
  for (int c = 0; c < 3; ++c) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += NT) s += part[(int64_t)c * nb + b];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, WAVE);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) tot[c] = red[0] + red[1] + red[2] + red[3];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double den = tot[1] * tot[2];
    tot[3] = den > 0.0 ? 1.0 - tot[0] * tot[0] / den : 1.0;
  }
}

// dy = dL/dz for L = 1 - (z.x)^2 / (z.z x.x)
__global__ __launch_bounds__(NT) void k_lpc_cos_grad(int64_t N, const float* __restrict__ in0,
                                                     const float* __restrict__ y,
                                                     const double* __restrict__ xs,
                                                     const double* __restrict__ tot,
                                                     float* __restrict__ dy) {
  const int64_t v = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (v >= N) return;
  const double zx = tot[0], zz = tot[1], xx = tot[2];
  const double den = zz * xx;
  if (!(den > 0.0)) {
    dy[v] = 0.f;
    return;
  }
  const double z = (double)in0[v] + (double)y[v];
  dy[v] = (float)(-2.0 * zx / den * xs[v] + 2.0 * zx * zx / (den * zz) * z);
}

__global__ __launch_bounds__(NT) void k_adam(int n, float* __restrict__ w, float* __restrict__ g,
                                             float* __restrict__ m1, float* __restrict__ m2,
                                             float lr, float b1, float b2, float eps, float c1,
                                             float c2, float scale) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i] * scale;
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  w[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
  g[i] = 0.f;
}

// ================================================================ host side
static inline unsigned nb(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

// one convolution layer: the unrolled form when CI is 4 or 8 and the output
// count splits into groups of G (2 at full resolution, 1 on the coarse grid
// and for the single output channel), else the general form
static void conv(const Dims& d, int CI, int CO, bool fine, const float* in, const float* W,
                 const float* B, float* out, int relu, hipStream_t st) {
  const int64_t N = (int64_t)d.nx * d.ny * d.nz;
  const int G = (fine && CO % 2 == 0) ? 2 : 1;
  const dim3 grid(nb(N), (unsigned)(CO / G));
#define CV(CC, GG)                                                                          \
  if (CI == CC && G == GG && N * LPC_MAXC <= INT32_MAX) {                                \
    hipLaunchKernelGGL((k_conv_fwd_g<CC, GG, false>), grid, dim3(NT), 0, st, d, in, W, B, out, \
                       relu, CI);                                                             \
    return;                                                                                 \
  }
  CV(4, 1) CV(4, 2) CV(8, 1) CV(8, 2)
#undef CV
  hipLaunchKernelGGL(k_conv_fwd, dim3(nb(N)), dim3(NT), 0, st, d, CI, CO, in, W, B, out, relu);
}

cr_status lpc_forward(const LpcNet& net, const float* in, LpcActs& a, hipStream_t st) {
  const Dims d{net.nx, net.ny, net.nz};
  const Dims c = coarse(d);
  const int64_t N = (int64_t)d.nx * d.ny * d.nz, Nc = (int64_t)c.nx * c.ny * c.nz;
  const int C = net.C;
  conv(d, 4, C, true, in, net.W[0], net.B[0], a.a0, 1, st);
  conv(d, C, C, true, a.a0, net.W[1], net.B[1], a.a1, 1, st);
  hipLaunchKernelGGL(k_pool_fwd, dim3(nb(Nc)), dim3(NT), 0, st, d, C, a.a1, a.p);
  conv(c, C, C, false, a.p, net.W[2], net.B[2], a.a2, 1, st);
  conv(c, C, C, false, a.a2, net.W[3], net.B[3], a.a3, 1, st);
  hipLaunchKernelGGL(k_up_add, dim3(nb(N)), dim3(NT), 0, st, d, C, a.a3, a.a1, a.s);
  conv(d, C, 1, true, a.s, net.W[4], net.B[4], a.y, 0, st);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// voxels per thread of the register form of the weight gradient
constexpr int WG_VPT = 8;

// weight and bias gradients of one layer, accumulated into gW / gB: the
// register form for the channel counts of the network at 4 and 8 channels,
// else the generic kernel; partial needs nb(N) * (CO CI 27 + CO) floats
static cr_status wgrad(const Dims& d, int CI, int CO, const float* in, const float* dout,
                       float* gW, float* gB, float* partial, hipStream_t st) {
  const int64_t N = (int64_t)d.nx * d.ny * d.nz;
  const int m = CO * CI * 27 + CO;
  unsigned blocks = nb(N);
  bool done = false;
  if (N * LPC_MAXC <= INT32_MAX) {
    const unsigned xb = (unsigned)std::max<int64_t>(1, (N + NT * WG_VPT - 1) / (NT * WG_VPT));
#define WG(A, B)                                                                          \
  if (!done && CI == A && CO == B) {                                                       \
    hipLaunchKernelGGL((k_conv_wgrad_t<A, B>), dim3(xb, 27), dim3(NT), 0, st, d, in, dout, \
                       partial);                                                          \
    blocks = xb;                                                                          \
    done = true;                                                                          \
  }
    WG(4, 8) WG(8, 8) WG(8, 1) WG(4, 4) WG(4, 1)
#undef WG
  }
  if (!done)
    hipLaunchKernelGGL(k_conv_wgrad, dim3(blocks), dim3(NT), 0, st, d, CI, CO, in, dout, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3((m + NT - 1) / NT), dim3(NT), 0, st, (int)blocks, m,
                     partial, gW, gB, CO * CI * 27);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

// data gradient din = conv^T(dout) of a layer with CI inputs and CO outputs:
// the unrolled forward form with flipped, transposed weights when CO is 1, 4
// or 8, else the generic kernel; din is overwritten
static void dgrad(const Dims& d, int CI, int CO, bool fine, const float* dout, const float* W,
                  float* din, hipStream_t st) {
  const int64_t N = (int64_t)d.nx * d.ny * d.nz;
  const int G = (fine && CI % 2 == 0) ? 2 : 1;
  const dim3 grid(nb(N), (unsigned)(CI / G));
#define DG(CC, GG)                                                                          \
  if (CO == CC && G == GG && N * LPC_MAXC <= INT32_MAX) {                                \
    hipLaunchKernelGGL((k_conv_fwd_g<CC, GG, true>), grid, dim3(NT), 0, st, d, dout, W,      \
                       (const float*)nullptr, din, 0, CI);                                  \
    return;                                                                                 \
  }
  DG(1, 1) DG(1, 2) DG(4, 1) DG(4, 2) DG(8, 1) DG(8, 2)
#undef DG
  hipLaunchKernelGGL(k_conv_dgrad, dim3(nb(N)), dim3(NT), 0, st, d, CI, CO, dout, W, din);
}

// backward from dy; gradients accumulated into net.gW / net.gB
cr_status lpc_backward(LpcNet& net, const float* in, LpcActs& a, hipStream_t st) {
  const Dims d{net.nx, net.ny, net.nz};
  const Dims c = coarse(d);
  const int64_t N = (int64_t)d.nx * d.ny * d.nz, Nc = (int64_t)c.nx * c.ny * c.nz;
  const int C = net.C;
  float* P = a.partial;
  // L4: y = conv(s)
  CR_TRY(wgrad(d, C, 1, a.s, a.dy, net.gW[4], net.gB[4], P, st));
  dgrad(d, C, 1, true, a.dy, net.W[4], a.ds, st);
  // s = up(a3) + a1 : da1 = ds (skip), da3 = up^T ds
  hipLaunchKernelGGL(k_up_bwd, dim3(nb(Nc)), dim3(NT), 0, st, d, C, a.ds, a.da3);
  // L3
  hipLaunchKernelGGL(k_relu_bwd, dim3(nb(C * Nc)), dim3(NT), 0, st, (int64_t)C * Nc, a.a3, a.da3);
  CR_TRY(wgrad(c, C, C, a.a2, a.da3, net.gW[3], net.gB[3], P, st));
  dgrad(c, C, C, false, a.da3, net.W[3], a.da2, st);
  // L2
  hipLaunchKernelGGL(k_relu_bwd, dim3(nb(C * Nc)), dim3(NT), 0, st, (int64_t)C * Nc, a.a2, a.da2);
  CR_TRY(wgrad(c, C, C, a.p, a.da2, net.gW[2], net.gB[2], P, st));
  dgrad(c, C, C, false, a.da2, net.W[2], a.dp, st);
  // pool: da1 = ds + pool^T dp
  hipLaunchKernelGGL(k_pool_bwd, dim3(nb(N)), dim3(NT), 0, st, d, C, a.dp, a.ds);
  // L1 (a.ds now holds da1)
  hipLaunchKernelGGL(k_relu_bwd, dim3(nb(C * N)), dim3(NT), 0, st, (int64_t)C * N, a.a1, a.ds);
  CR_TRY(wgrad(d, C, C, a.a0, a.ds, net.gW[1], net.gB[1], P, st));
  dgrad(d, C, C, true, a.ds, net.W[1], a.da0, st);
  // L0
  hipLaunchKernelGGL(k_relu_bwd, dim3(nb(C * N)), dim3(NT), 0, st, (int64_t)C * N, a.a0, a.da0);
  CR_TRY(wgrad(d, 4, C, in, a.da0, net.gW[0], net.gB[0], P, st));
  CR_HIP(hipGetLastError());
  return CR_OK;
}

cr_status lpc_input(const LpcNet& net, const double* w, const double* w2, const double* minv,
                    const double* dvec, const uint8_t* deg, const double* coef, double lam,
                    float* in, hipStream_t st) {
  const int64_t N = (int64_t)net.nx * net.ny * net.nz;
  hipLaunchKernelGGL(k_lpc_input, dim3(nb(N)), dim3(NT), 0, st, N, w, w2, minv, dvec, deg, coef,
                     lam, in);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

cr_status lpc_output(const LpcNet& net, const float* in0, const float* y, double* z,
                     hipStream_t st) {
  const int64_t N = (int64_t)net.nx * net.ny * net.nz;
  hipLaunchKernelGGL(k_lpc_output, dim3(nb(N)), dim3(NT), 0, st, N, in0, y, z);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

int64_t lpc_loss_scratch(const LpcNet& net) {
  const int64_t N = (int64_t)net.nx * net.ny * net.nz;
  return 3 * (int64_t)nb(N) + 4;
}

cr_status lpc_loss(const LpcNet& net, const float* in0, const float* y, const double* xs,
                   float* dy, double* scratch, hipStream_t st) {
  const int64_t N = (int64_t)net.nx * net.ny * net.nz;
  const int blocks = (int)nb(N);
  double* tot = scratch + 3 * (int64_t)blocks;
  hipLaunchKernelGGL(k_lpc_dots, dim3(blocks), dim3(NT), 0, st, N, in0, y, xs, scratch, blocks);
  hipLaunchKernelGGL(k_lpc_dots_total, dim3(1), dim3(NT), 0, st, blocks, scratch, tot);
  hipLaunchKernelGGL(k_lpc_cos_grad, dim3(nb(N)), dim3(NT), 0, st, N, in0, y, xs, tot, dy);
  CR_HIP(hipGetLastError());
  return CR_OK;
}

cr_status lpc_adam(LpcNet& net, float lr, float scale, hipStream_t st) {
  net.step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)net.step), c2 = 1.f - powf(b2, (float)net.step);
  for (int l = 0; l < LPC_LAYERS; ++l) {
    const int nw = net.co[l] * net.ci[l] * 27, nbias = net.co[l];
    hipLaunchKernelGGL(k_adam, dim3((nw + NT - 1) / NT), dim3(NT), 0, st, nw, net.W[l], net.gW[l],
                       net.mW[l], net.vW[l], lr, b1, b2, eps, c1, c2, scale);
    hipLaunchKernelGGL(k_adam, dim3((nbias + NT - 1) / NT), dim3(NT), 0, st, nbias, net.B[l],
                       net.gB[l], net.mB[l], net.vB[l], lr, b1, b2, eps, c1, c2, scale);
  }
  CR_HIP(hipGetLastError());
  return CR_OK;
}

}  // namespace cr
