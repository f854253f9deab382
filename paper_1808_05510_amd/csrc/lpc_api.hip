// C ABI of the learned preconditioner network: creation, parameters,
// forward and vector-Jacobian product (the training step and the FCG solve
// live in api.hip next to the problem handle).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "cr_internal.hpp"

using namespace cr;

// SplitMix64 output for counter k of a state (Steele, Lea & Flood 2014)
static inline uint64_t sm64(uint64_t state, uint64_t k) {
  uint64_t z = state + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static cr_status alloc_acts(cr_pc* pc) {
  LpcNet& n = pc->net;
  const int64_t N = (int64_t)n.nx * n.ny * n.nz;
  const int64_t Nc = (int64_t)((n.nx + 1) / 2) * ((n.ny + 1) / 2) * ((n.nz + 1) / 2);
  const int64_t C = n.C;
  const int64_t nb = (N + NT - 1) / NT;
  const int64_t part = nb * (LPC_MAXC * LPC_MAXC * 27 + LPC_MAXC);
  const int64_t total = 4 * N + 5 * C * N + 2 * N + 6 * C * Nc + part;
  float* m = nullptr;
  if (hipMalloc(&m, sizeof(float) * total) != hipSuccess) {
    set_error("allocation of network activations failed");
    return CR_ENOMEM;
  }
  LpcActs& a = pc->acts;
  a.mem = m;
  a.in = m; m += 4 * N;
  a.a0 = m; m += C * N;
  a.a1 = m; m += C * N;
  a.s = m; m += C * N;
  a.ds = m; m += C * N;
  a.da0 = m; m += C * N;
  a.y = m; m += N;
  a.dy = m; m += N;
  a.p = m; m += C * Nc;
  a.a2 = m; m += C * Nc;
  a.a3 = m; m += C * Nc;
  a.da3 = m; m += C * Nc;
  a.da2 = m; m += C * Nc;
  a.dp = m; m += C * Nc;
  a.partial = m;  // wgrad per-workgroup partial sums (nb x (C*C*27 + C))
  return CR_OK;
}

extern "C" cr_status cr_pc_create(int32_t nx, int32_t ny, int32_t nz, int32_t channels,
                                  uint64_t seed, void* hip_stream, cr_pc** out) {
  if (!out || nx < 2 || ny < 2 || nz < 2 || channels < 1 || channels > LPC_MAXC) {
    set_error("cr_pc_create: dims must be >= 2 and channels in [1, 8]");
    return CR_EINVAL;
  }
  *out = nullptr;
  cr_pc* pc = new cr_pc();
  pc->st = (hipStream_t)hip_stream;
  LpcNet& n = pc->net;
  n.nx = nx;
  n.ny = ny;
  n.nz = nz;
  n.C = channels;
  const int ci[LPC_LAYERS] = {4, channels, channels, channels, channels};
  const int co[LPC_LAYERS] = {channels, channels, channels, channels, 1};
  int64_t np = 0;
  for (int l = 0; l < LPC_LAYERS; ++l) {
    n.ci[l] = ci[l];
    n.co[l] = co[l];
    np += (int64_t)co[l] * ci[l] * 27 + co[l];
  }
  n.nparam = np;
  if (hipMalloc(&n.mem, sizeof(float) * 4 * np) != hipSuccess) {
    delete pc;
    set_error("allocation of network parameters failed");
    return CR_ENOMEM;
  }
  float* base[4] = {n.mem, n.mem + np, n.mem + 2 * np, n.mem + 3 * np};  // param, grad, m, v
  int64_t off = 0;
  for (int l = 0; l < LPC_LAYERS; ++l) {
    const int64_t nw = (int64_t)co[l] * ci[l] * 27;
    n.W[l] = base[0] + off;
    n.gW[l] = base[1] + off;
    n.mW[l] = base[2] + off;
    n.vW[l] = base[3] + off;
    off += nw;
    n.B[l] = base[0] + off;
    n.gB[l] = base[1] + off;
    n.mB[l] = base[2] + off;
    n.vB[l] = base[3] + off;
    off += co[l];
  }
  // He-uniform weights from SplitMix64(seed), zero biases; the last layer
  // starts at zero, so an untrained network returns its input's base step
  // unchanged (z = w) and training moves it only as far as the loss asks
  std::vector<float> h(np, 0.f);
  int64_t k = 0;
  for (int l = 0; l < LPC_LAYERS; ++l) {
    const int64_t nw = (int64_t)co[l] * ci[l] * 27;
    const double lim = l == LPC_LAYERS - 1 ? 0.0 : std::sqrt(6.0 / (ci[l] * 27.0));
    for (int64_t e = 0; e < nw; ++e, ++k) {
      const double u = (double)(sm64(seed, (uint64_t)k + 1) >> 11) * 0x1.0p-52 - 1.0;
      h[k] = (float)(lim * u);
    }
    k += co[l];
  }
  std::vector<float> z(3 * np, 0.f);
  if (stage_to_device(n.mem, h.data(), sizeof(float) * np, pc->st) != hipSuccess ||
      stage_to_device(n.mem + np, z.data(), sizeof(float) * 3 * np, pc->st) != hipSuccess) {
    (void)hipFree(n.mem);
    delete pc;
    set_error("upload of network parameters failed");
    return CR_EHIP;
  }
  cr_status s = alloc_acts(pc);
  if (s != CR_OK) {
    (void)hipFree(n.mem);
    delete pc;
    return s;
  }
  *out = pc;
  return CR_OK;
}

extern "C" void cr_pc_destroy(cr_pc* pc) {
  if (!pc) return;
  (void)hipStreamSynchronize(pc->st);
  if (pc->net.mem) (void)hipFree(pc->net.mem);
  if (pc->acts.mem) (void)hipFree(pc->acts.mem);
  if (pc->dwork) (void)hipFree(pc->dwork);
  delete pc;
}

extern "C" int64_t cr_pc_num_params(const cr_pc* pc) { return pc ? pc->net.nparam : 0; }

extern "C" cr_status cr_pc_get_params(cr_pc* pc, float* host_out) {
  if (!pc || !host_out) {
    set_error("null argument");
    return CR_EINVAL;
  }
  CR_HIP(hipStreamSynchronize(pc->st));
  CR_HIP(stage_to_host(host_out, pc->net.mem, sizeof(float) * pc->net.nparam, 1, 0, pc->st));
  return CR_OK;
}

extern "C" cr_status cr_pc_set_params(cr_pc* pc, const float* host_in) {
  if (!pc || !host_in) {
    set_error("null argument");
    return CR_EINVAL;
  }
  CR_HIP(hipStreamSynchronize(pc->st));
  CR_HIP(stage_to_device(pc->net.mem, host_in, sizeof(float) * pc->net.nparam, pc->st));
  pc->net.step = 0;
  CR_HIP(hipMemsetAsync(pc->net.mem + pc->net.nparam, 0, sizeof(float) * 3 * pc->net.nparam,
                        pc->st));
  CR_HIP(hipStreamSynchronize(pc->st));
  return CR_OK;
}

extern "C" cr_status cr_pc_forward(cr_pc* pc, const float* in, float* y) {
  if (!pc || !in || !y) {
    set_error("null argument");
    return CR_EINVAL;
  }
  const int64_t N = (int64_t)pc->net.nx * pc->net.ny * pc->net.nz;
  CR_TRY(lpc_forward(pc->net, in, pc->acts, pc->st));
  CR_HIP(hipMemcpyAsync(y, pc->acts.y, sizeof(float) * N, hipMemcpyDeviceToDevice, pc->st));
  CR_HIP(hipStreamSynchronize(pc->st));
  return CR_OK;
}

extern "C" cr_status cr_pc_vjp(cr_pc* pc, const float* in, const float* dy, float* grad_host) {
  if (!pc || !in || !dy || !grad_host) {
    set_error("null argument");
    return CR_EINVAL;
  }
  const int64_t N = (int64_t)pc->net.nx * pc->net.ny * pc->net.nz;
  const int64_t np = pc->net.nparam;
  CR_HIP(hipMemsetAsync(pc->net.mem + np, 0, sizeof(float) * np, pc->st));
  CR_TRY(lpc_forward(pc->net, in, pc->acts, pc->st));
  CR_HIP(hipMemcpyAsync(pc->acts.dy, dy, sizeof(float) * N, hipMemcpyDeviceToDevice, pc->st));
  CR_TRY(lpc_backward(pc->net, in, pc->acts, pc->st));
  CR_HIP(hipStreamSynchronize(pc->st));
  CR_HIP(stage_to_host(grad_host, pc->net.mem + np, sizeof(float) * np, 1, 0, pc->st));
  CR_HIP(hipMemsetAsync(pc->net.mem + np, 0, sizeof(float) * np, pc->st));
  CR_HIP(hipStreamSynchronize(pc->st));
  return CR_OK;
}
